"""GPU parity of the floating-point prefix modes (F64, COMP_F32, NAIVE_F32) of
the collective resamplers against the exact CPU oracle.

The modes round their prefix sums, so a GPU ancestor may differ from the
oracle's only where the point lies within the mode's error bound of a bin
boundary (tiecheck.float_r_error_bound); outputs stay sorted and in range, and
the batched and single-vector paths run the same arithmetic, so they agree
bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import inputs
from tiecheck import check_ties, float_r_error_bound, strata_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCHEMES = ["stratified", "systematic", "multinomial"]
MODES = {"f64": "SCAN_F64", "comp_f32": "SCAN_COMP_F32", "naive_f32": "SCAN_NAIVE_F32"}


def pfr():
    import paper_1301_4019_amd as m
    return m


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def prec(mode):
    return getattr(pfr(), MODES[mode])


def oracle_run(scheme, w, seed, filt=0, offset=0):
    n = w.size
    if scheme == "multinomial":
        a, fl, r, p = oracle.multinomial(w, seed=seed, filt=filt, offset=offset, return_rp=True)
        return a, fl, r, p
    if scheme == "stratified":
        a, fl, r = oracle.stratified(w, seed=seed, filt=filt, offset=offset, return_r=True)
        u = oracle.stratum_offsets(n, seed=seed, filt=filt, offset=offset)
    else:
        a, fl, r = oracle.systematic(w, seed=seed, filt=filt, offset=offset, return_r=True)
        u = np.full(n, oracle.systematic_offset(seed=seed, filt=filt, offset=offset))
    return a, fl, r, strata_points(u)


def check_mode(scheme, mode, w, a_gpu, seed, filt=0, offset=0):
    n = w.size
    a_or, fl, r, pts = oracle_run(scheme, w, seed, filt, offset)
    assert fl == 0
    assert a_gpu.min() >= 0 and a_gpu.max() < n
    assert np.all(np.diff(a_gpu) >= 0)
    delta = float_r_error_bound(n, mode)
    if scheme == "multinomial":
        delta += n * 2.0**-44  # exponential spacings quantised at 2^-48, logs to ~1 ulp
    return check_ties(a_gpu, a_or, r, pts, delta, max_ties=5 + int(20 * delta * n))


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("dtype,n,y", [(np.float32, 1000, 3.0), (np.float32, 4096, 2.0),
                                       (np.float32, 4097, 0.0), (np.float32, 100003, 4.0),
                                       (np.float64, 3, 1.0), (np.float64, 50001, 2.0)])
def test_mode_parity(scheme, mode, dtype, n, y):
    w = inputs.weights(n, y, seed=n + 31, dtype=dtype)
    fn = getattr(pfr(), "resample_" + scheme)
    a = host(fn(dev(w), seed=21, offset=4, filter_base=1, precision=prec(mode)))
    check_mode(scheme, mode, w, a, seed=21, filt=1, offset=4)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("mode", ["f64", "comp_f32"])
def test_mode_parity_full_size(scheme, mode):
    n = 1 << 20
    w = inputs.weights(n, 3.0, seed=2)
    fn = getattr(pfr(), "resample_" + scheme)
    a = host(fn(dev(w), seed=8, precision=prec(mode)))
    ties = check_mode(scheme, mode, w, a, seed=8)
    assert ties <= 2


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("mode", list(MODES))
def test_mode_zero_and_bad_weights(scheme, mode):
    fn = getattr(pfr(), "resample_" + scheme)
    n = 5000
    w = np.zeros(n, dtype=np.float32)
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    a = host(fn(dev(w), seed=1, precision=prec(mode), flags=fl))
    assert np.array_equal(a, np.arange(n))
    assert int(host(fl)[0]) == pfr().FLAG_ZERO_TOTAL
    w = inputs.weights(n, 1.0, seed=3)
    w[1234] = np.nan
    fl.zero_()
    a = host(fn(dev(w), seed=1, precision=prec(mode), flags=fl))
    assert np.array_equal(a, np.arange(n))
    assert int(host(fl)[0]) == pfr().FLAG_BAD_WEIGHTS


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("mode", list(MODES))
def test_mode_batched_equals_single(scheme, mode):
    lens = [4097, 1, 30000, 0, 8192, 777]
    rng = np.random.default_rng(5)
    ws = [inputs.weights(m, float(rng.uniform(0, 4)), seed=100 + i) for i, m in enumerate(lens)]
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w_all = np.concatenate(ws).astype(np.float32)
    fn = getattr(pfr(), "resample_" + scheme)
    a_all = host(fn(dev(w_all), seed=6, offset=2, filter_base=10, precision=prec(mode),
                    offsets=dev(offsets), max_len=max(lens)))
    for f, w in enumerate(ws):
        if w.size == 0:
            continue
        a = host(fn(dev(w), seed=6, offset=2, filter_base=10 + f, precision=prec(mode)))
        assert np.array_equal(a_all[offsets[f]:offsets[f + 1]], a), f


def test_mode_deterministic():
    w = dev(inputs.weights(300000, 2.0, seed=9))
    for mode in MODES:
        outs = [host(pfr().resample_stratified(w, seed=3, precision=prec(mode))) for _ in range(3)]
        assert all(np.array_equal(outs[0], o) for o in outs[1:]), mode
