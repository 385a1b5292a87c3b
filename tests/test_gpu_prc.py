"""GPU partial rejection control against the oracle: ancestors bit for bit
(the oracle clips the weights explicitly, the GPU runs the rejection test on
the raw weights with bound v_max), importance weights bit for bit (binary64
quotients rounded to the weight type on both sides)."""
import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pfr():
    import paper_1301_4019_amd as m
    return m


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [1000, 1 << 16, 1 << 20])
@pytest.mark.parametrize("q", [0.5, 0.95, None])
def test_single_vector(n, q, dtype):
    w = inputs.weights(n, 2.0, seed=n).astype(dtype)
    vmax = float(np.quantile(w, q)) if q is not None else 1.0
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    a, wo = pfr().resample_partial_rejection(torch.from_numpy(w).cuda(), vmax, seed=4, offset=2,
                                             flags=fl)
    a_ref, wo_ref, fl_ref = oracle.partial_rejection(w, vmax, seed=4, offset=2)
    assert int(host(fl)[0]) == fl_ref == 0
    assert np.array_equal(host(a), a_ref)
    assert np.array_equal(host(wo), wo_ref.astype(dtype))


def test_ragged_batch_with_per_segment_bounds():
    w, off, ys = inputs.ragged_batch(n_filters=48, seed=5)
    sizes = np.diff(off)
    vm = np.array([np.quantile(w[off[f]:off[f + 1]], 0.7) for f in range(48)], dtype=np.float64)
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    a, wo = pfr().resample_partial_rejection(
        torch.from_numpy(w).cuda(), 1.0, seed=9, filter_base=3,
        v_max_per_filter=torch.from_numpy(vm).cuda(), offsets=torch.from_numpy(off).cuda(),
        max_len=int(sizes.max()), flags=fl)
    a, wo = host(a), host(wo)
    assert int(host(fl)[0]) == 0
    for f in range(48):
        sl = slice(off[f], off[f + 1])
        a_ref, wo_ref, _ = oracle.partial_rejection(w[sl], vm[f], seed=9, filt=3 + f)
        assert np.array_equal(a[sl], a_ref), f
        assert np.array_equal(wo[sl], wo_ref.astype(np.float32)), f


def test_trial_cap_keeps_zero_weight_particle():
    w = np.zeros(300, dtype=np.float32)
    w[7] = 1.0
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    a, wo = pfr().resample_partial_rejection(torch.from_numpy(w).cuda(), 0.5, seed=1,
                                             max_trials=3, flags=fl)
    a_ref, wo_ref, fl_ref = oracle.partial_rejection(w, 0.5, seed=1, max_trials=3)
    assert int(host(fl)[0]) == fl_ref == pfr().FLAG_TRIAL_CAP
    assert np.array_equal(host(a), a_ref)
    assert np.array_equal(host(wo), wo_ref.astype(np.float32))


def test_per_segment_arrays_of_the_wrong_type_are_refused():
    w = torch.ones(100, device="cuda")
    off = torch.tensor([0, 50, 100], dtype=torch.int64, device="cuda")
    with pytest.raises(TypeError):
        pfr().resample_partial_rejection(w, 1.0, offsets=off,
                                         v_max_per_filter=torch.ones(2, device="cuda"))
    with pytest.raises(TypeError):
        pfr().resample_rejection(w, 1.0, offsets=off,
                                 w_max_per_filter=torch.ones(1, dtype=torch.float64,
                                                             device="cuda"))
    with pytest.raises(TypeError):
        pfr().resample_metropolis(w, 4, offsets=off,
                                  B_per_filter=torch.ones(2, dtype=torch.int64, device="cuda"))
