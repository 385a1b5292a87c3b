"""GPU Code 5 with independent uniforms against the oracle: the points p_i
are the same binary64 values on both sides, so ancestors agree except where
a point lies within the GPU prefix's error bound of a bin edge (tie rule)."""
import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import inputs
from tiecheck import check_ties, gpu_r_error_bound

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pfr():
    import paper_1301_4019_amd as m
    return m


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [1, 7, 1000, 4097, (1 << 16) + 3, 1 << 20, 1 << 22])
@pytest.mark.parametrize("y", [0.0, 3.0])
def test_matches_oracle(n, y, dtype):
    w = inputs.weights(n, y, seed=n + 1).astype(dtype)
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    a = host(pfr().resample_multinomial_iid(torch.from_numpy(w).cuda(), seed=6, offset=1,
                                            filter_base=2, flags=fl))
    a_or, fl_or, r, p = oracle.multinomial_iid(w, seed=6, filt=2, offset=1, return_rp=True)
    assert int(host(fl)[0]) == fl_or == 0
    delta = gpu_r_error_bound(w.astype(np.float64), n)
    check_ties(a, a_or, r, p, delta, max_ties=5 + int(20 * delta * n))


def test_zero_and_bad_weights_give_the_identity():
    for w, flag in ((np.zeros(5000, dtype=np.float32), 1), (np.r_[np.ones(10), -1.0], 8)):
        fl = torch.zeros(1, dtype=torch.int32, device="cuda")
        a = host(pfr().resample_multinomial_iid(torch.from_numpy(w).cuda(), flags=fl))
        assert int(host(fl)[0]) == flag
        assert np.array_equal(a, np.arange(w.size))


def test_offspring_match_sorted_multinomial_in_law():
    """Both multinomial forms give offspring with mean n w / W: over 64 seeds
    the per-particle mean offspring of the two agree within the noise."""
    n = 4096
    w = inputs.weights(n, 2.0, seed=3)
    wd = torch.from_numpy(w).cuda()
    s_iid = np.zeros(n)
    s_srt = np.zeros(n)
    for k in range(64):
        s_iid += np.bincount(host(pfr().resample_multinomial_iid(wd, seed=k)), minlength=n)
        s_srt += np.bincount(host(pfr().resample_multinomial(wd, seed=k)), minlength=n)
    e = n * w.astype(np.float64) / w.astype(np.float64).sum()
    z_iid = (s_iid / 64 - e) / np.sqrt(e * (1 - w / w.sum()) / 64 + 1e-300)
    z_srt = (s_srt / 64 - e) / np.sqrt(e * (1 - w / w.sum()) / 64 + 1e-300)
    live = e > 0.5
    assert abs(np.mean(z_iid[live] ** 2) - 1.0) < 0.15
    assert abs(np.mean(z_srt[live] ** 2) - 1.0) < 0.15
