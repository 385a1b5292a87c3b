"""GPU parity: every entry point of libpfresample against the CPU oracle on the
same seeded inputs and the same Philox counters.

Bit-exact: Metropolis, rejection, offspring_to_ancestors, permute_ancestors.
Collective schemes: equal except at stated bin-boundary ties (tiecheck.py),
with sorted output, sum-to-n and zero weights never selected.
"""
import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import inputs
from tiecheck import check_ties, gpu_r_error_bound, strata_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pfr():
    import paper_1301_4019_amd as m
    return m


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def new_flags():
    return torch.zeros(1, dtype=torch.int32, device="cuda")


# ----------------------------------------------------------------- alternatives
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,y,B", [(1024, 2.0, 64), (1, 2.0, 5), (3, 0.0, 7), (4097, 3.0, 11),
                                   (100003, 4.0, 9), (16385, 4.0, 300), (20000, 3.0, 61),
                                   (32768, 4.0, 357), (32769, 1.0, 8), (12000, 3.0, 60)])
def test_metropolis_bit_exact(dtype, n, y, B):
    w = inputs.weights(n, y, seed=n, dtype=dtype)
    a = host(pfr().resample_metropolis(dev(w), B, seed=12345, offset=3, filter_base=7))
    ref = oracle.metropolis(w, B, seed=12345, filt=7, offset=3)
    assert np.array_equal(a, ref)


def test_metropolis_full_size_config():
    n = 1 << 20
    for y, B in ((0.0, 4), (3.0, 60)):
        w = inputs.weights(n, y, seed=1)
        a = host(pfr().resample_metropolis(dev(w), B, seed=2))
        ref = oracle.metropolis(w, B, seed=2)
        assert np.array_equal(a, ref), y


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,y", [(1024, 2.0), (1, 0.0), (2, 4.0), (5000, 3.0), (65537, 1.0),
                                 (4096, 4.0), (16384, 4.0), (16385, 4.0), (40000, 2.0),
                                 (131071, 4.0)])
def test_rejection_bit_exact(dtype, n, y):
    w = inputs.weights(n, y, seed=n + 1, dtype=dtype)
    fl = new_flags()
    a = host(pfr().resample_rejection(dev(w), 1.0, seed=99, offset=1, flags=fl))
    ref, rfl = oracle.rejection(w, 1.0, seed=99, offset=1)
    assert np.array_equal(a, ref)
    assert int(host(fl)[0]) == rfl == 0


def test_rejection_full_size_and_trial_cap():
    n = 1 << 20
    w = inputs.weights(n, 3.0, seed=5)
    a = host(pfr().resample_rejection(dev(w), 1.0, seed=11))
    ref, _ = oracle.rejection(w, 1.0, seed=11)
    assert np.array_equal(a, ref)
    # a bound far above the weights with a small cap: capped lanes keep a_i = i
    w = inputs.weights(4096, 4.0, seed=6)
    fl = new_flags()
    a = host(pfr().resample_rejection(dev(w), 64.0, seed=3, max_trials=8, flags=fl))
    ref, rfl = oracle.rejection(w, 64.0, seed=3, max_trials=8)
    assert np.array_equal(a, ref)
    assert rfl & oracle.FLAG_TRIAL_CAP and int(host(fl)[0]) & oracle.FLAG_TRIAL_CAP


def test_rejection_repeat_calls_identical():
    w = inputs.weights(300000, 2.0, seed=8)
    wd = dev(w)
    outs = [host(pfr().resample_rejection(wd, 1.0, seed=4)) for _ in range(3)]
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    assert np.array_equal(outs[0], oracle.rejection(w, 1.0, seed=4)[0])


# ----------------------------------------------------------------- collective
SCHEMES = ["stratified", "systematic", "multinomial"]


def gpu_collective(scheme, w, **kw):
    fn = getattr(pfr(), "resample_" + scheme)
    return fn(dev(w), **kw)


def oracle_collective(scheme, w, seed, filt=0, offset=0):
    """(a, flags, r, points) from the oracle."""
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


def check_collective(scheme, w, a_gpu, seed, filt=0, offset=0):
    n = w.size
    a_or, fl, r, pts = oracle_collective(scheme, w, seed, filt, offset)
    assert fl == 0
    assert a_gpu.min() >= 0 and a_gpu.max() < n
    assert np.all(np.diff(a_gpu) >= 0)
    w64 = w.astype(np.float64)
    assert not np.any(w64[a_gpu] == 0.0)
    delta = gpu_r_error_bound(w64, n)
    if scheme == "multinomial":
        delta += n * 2.0**-44  # exponential spacings quantised at 2^-48, logs to ~1 ulp
    return check_ties(a_gpu, a_or, r, pts, delta, max_ties=5 + int(20 * delta * n))


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("n,y", [(1024, 2.0), (1, 1.0), (2, 0.0), (3, 4.0), (1000, 3.0),
                                 (4096, 2.0), (4097, 2.0), (16385, 2.0), (100003, 4.0)])
def test_collective_parity(scheme, dtype, n, y):
    w = inputs.weights(n, y, seed=n + 17, dtype=dtype)
    a = host(gpu_collective(scheme, w, seed=77, offset=5, filter_base=2))
    check_collective(scheme, w, a, seed=77, filt=2, offset=5)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("y", [0.0, 2.0, 4.0])
def test_collective_full_size(scheme, y):
    n = 1 << 20
    w = inputs.weights(n, y, seed=3)
    a = host(gpu_collective(scheme, w, seed=1))
    check_collective(scheme, w, a, seed=1)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_collective_zero_weights_and_degenerate(scheme):
    g = np.random.default_rng(4)
    for n in (5000, 70000):
        w = inputs.weights(n, 2.0, seed=n)
        w[g.random(n) < 0.3] = 0.0
        w[-100:] = 0.0
        w[:50] = 0.0
        a = host(gpu_collective(scheme, w, seed=9))
        check_collective(scheme, w, a, seed=9)
    for n in (10, 50000):
        fl = new_flags()
        a = host(gpu_collective(scheme, np.zeros(n, np.float32), seed=1, flags=fl))
        assert np.array_equal(a, np.arange(n)) and int(host(fl)[0]) & oracle.FLAG_ZERO_TOTAL
        w = inputs.weights(n, 1.0, seed=2)
        w[n // 2] = np.nan
        fl = new_flags()
        a = host(gpu_collective(scheme, w, seed=1, flags=fl))
        assert np.array_equal(a, np.arange(n)) and int(host(fl)[0]) & oracle.FLAG_BAD_WEIGHTS
        w[n // 2] = -1.0
        fl = new_flags()
        a = host(gpu_collective(scheme, w, seed=1, flags=fl))
        assert int(host(fl)[0]) & oracle.FLAG_BAD_WEIGHTS
    # a single heavy particle takes every output
    w = np.full(30000, 1e-30, np.float32)
    w[12345] = 1.0
    a = host(gpu_collective(scheme, w, seed=5))
    check_collective(scheme, w, a, seed=5)


def test_systematic_offspring_floor_ceil_full_size():
    n = 1 << 20
    w = inputs.weights(n, 4.0, seed=21)
    a = host(gpu_collective("systematic", w, seed=8))
    o = np.bincount(a, minlength=n)
    e = n * w.astype(np.float64) / w.astype(np.float64).sum()
    assert o.sum() == n
    assert np.all((o >= np.floor(e) - 0) & (o <= np.ceil(e)))


def test_collective_deterministic():
    w = inputs.weights(300000, 3.0, seed=4)
    wd = dev(w)
    for scheme in SCHEMES:
        fn = getattr(pfr(), "resample_" + scheme)
        outs = [host(fn(wd, seed=6)) for _ in range(3)]
        assert all(np.array_equal(outs[0], o) for o in outs[1:]), scheme


# ----------------------------------------------------------------- batched
def ragged(nf=48, seed=3):
    w, off, ys = inputs.ragged_batch(n_filters=nf, seed=seed)
    return w, off, ys


@pytest.mark.parametrize("scheme", SCHEMES)
def test_collective_batched_matches_single_calls(scheme):
    w, off, _ = ragged()
    fn = getattr(pfr(), "resample_" + scheme)
    a = host(fn(dev(w), seed=13, offset=2, filter_base=100, offsets=dev(off),
                max_len=int(np.diff(off).max())))
    for f in range(off.size - 1):
        seg = w[off[f]:off[f + 1]]
        check_collective(scheme, seg, a[off[f]:off[f + 1]], seed=13, filt=100 + f, offset=2)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_collective_batched_block_parallel_equals_one_workgroup(scheme, dtype):
    """With a workspace a batch runs block-parallel; without one, one workgroup
    per segment.  Both use the same blocks and exact sums: identical bits."""
    lens = [1, 1023, 1024, 1025, 0, 5000, 65536, 3, 100003, 2048]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w = np.concatenate([inputs.weights(m, 0.5 + (f % 4), seed=300 + f, dtype=dtype)
                        for f, m in enumerate(lens)])
    w[off[5] + 17] = 0.0
    fn = getattr(pfr(), "resample_" + scheme)
    kw = dict(seed=21, offset=3, filter_base=7, offsets=dev(off), max_len=max(lens))
    a_seg = host(fn(dev(w), **kw))
    none = torch.empty(0, dtype=torch.uint8, device="cuda")
    a_one = host(fn(dev(w), workspace=none, **kw))
    assert np.array_equal(a_seg, a_one)
    for f in (0, 3, 6, 8):
        seg = w[off[f]:off[f + 1]]
        check_collective(scheme, seg, a_seg[off[f]:off[f + 1]], seed=21, filt=7 + f, offset=3)


def test_collective_batched_bad_and_zero_segments():
    lens = [3000, 2000, 70000, 10]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w = np.concatenate([inputs.weights(m, 1.0, seed=f) for f, m in enumerate(lens)])
    w[off[1]:off[2]] = 0.0            # all-zero segment: identity
    w[off[2] + 40000] = -1.0          # invalid weight: identity
    fl = new_flags()
    a = host(pfr().resample_systematic(dev(w), seed=2, offsets=dev(off), max_len=max(lens),
                                       flags=fl))
    assert np.array_equal(a[off[1]:off[2]], np.arange(lens[1]))
    assert np.array_equal(a[off[2]:off[3]], np.arange(lens[2]))
    assert int(host(fl)[0]) == pfr().FLAG_ZERO_TOTAL | pfr().FLAG_BAD_WEIGHTS
    for f in (0, 3):
        check_collective("systematic", w[off[f]:off[f + 1]], a[off[f]:off[f + 1]], seed=2,
                         filt=f)


def test_alternatives_batched_match_single_calls():
    w, off, ys = ragged(nf=40, seed=5)
    nf = off.size - 1
    B = np.array([4 + (f % 7) for f in range(nf)], dtype=np.int32)
    wm = np.ones(nf)
    am = host(pfr().resample_metropolis(dev(w), 0, seed=3, filter_base=10, B_per_filter=dev(B),
                                        offsets=dev(off)))
    ar = host(pfr().resample_rejection(dev(w), 1.0, seed=3, filter_base=10,
                                       w_max_per_filter=dev(wm), offsets=dev(off)))
    for f in range(nf):
        seg = w[off[f]:off[f + 1]]
        assert np.array_equal(am[off[f]:off[f + 1]],
                              oracle.metropolis(seg, int(B[f]), seed=3, filt=10 + f))
        assert np.array_equal(ar[off[f]:off[f + 1]],
                              oracle.rejection(seg, 1.0, seed=3, filt=10 + f)[0])


# segment lengths that land in every LDS capacity tier (16, 64, 128 KB of
# weights) and beyond it, with empty segments in between
TIER_LENGTHS = [5, 0, 300, 4096, 4097, 1, 16384, 0, 16385, 32768, 32769, 70000, 2, 999]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("max_len", ["exact", "unknown", "small_cap"])
def test_alternatives_batched_all_capacity_tiers(dtype, max_len):
    lens = TIER_LENGTHS
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    w = np.concatenate([inputs.weights(m, 1.0 + (f % 4), seed=200 + f, dtype=dtype)
                        for f, m in enumerate(lens)])
    nf = len(lens)
    ml = {"exact": max(lens), "unknown": None, "small_cap": 3000}[max_len]
    B = np.array([3 + (f % 9) for f in range(nf)], dtype=np.int32)
    am = host(pfr().resample_metropolis(dev(w), 0, seed=8, offset=1, filter_base=4,
                                        B_per_filter=dev(B), offsets=dev(off), max_len=ml))
    ar = host(pfr().resample_rejection(dev(w), 1.0, seed=8, offset=1, filter_base=4,
                                       offsets=dev(off), max_len=ml))
    for f in range(nf):
        if lens[f] == 0:
            continue
        seg = w[off[f]:off[f + 1]]
        assert np.array_equal(am[off[f]:off[f + 1]],
                              oracle.metropolis(seg, int(B[f]), seed=8, filt=4 + f, offset=1)), f
        assert np.array_equal(ar[off[f]:off[f + 1]],
                              oracle.rejection(seg, 1.0, seed=8, filt=4 + f, offset=1)[0]), f


@pytest.mark.parametrize("n", [100, 4096, 16384, 16385, 40000])
def test_alternatives_single_vector_each_tier(n):
    w = inputs.weights(n, 3.0, seed=n + 5)
    a = host(pfr().resample_metropolis(dev(w), 13, seed=2))
    assert np.array_equal(a, oracle.metropolis(w, 13, seed=2))
    a = host(pfr().resample_rejection(dev(w), 1.0, seed=2))
    assert np.array_equal(a, oracle.rejection(w, 1.0, seed=2)[0])


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n,y,B", [(65536, 4.0, 354), (100003, 3.0, 60), (1 << 20, 4.0, 41),
                                   (1 << 20, 0.5, 9), (3 << 20, 2.0, 16), (1 << 19, 4.0, 100),
                                   (300007, 3.0, 60), ((1 << 20) + 5, 4.0, 70)])
def test_alternatives_bound_table(dtype, n, y, B):
    """Long single vectors use the bound table when given a workspace; the
    result is the same as without one, and bit-exact against the oracle."""
    w = inputs.weights(n, y, seed=n + 9, dtype=dtype)
    wd = dev(w)
    am = host(pfr().resample_metropolis(wd, B, seed=6, offset=2))
    ar = host(pfr().resample_rejection(wd, 1.0, seed=6, offset=2))
    torch_ws = torch.empty(256, dtype=torch.uint8, device="cuda")  # too small: no table
    am0 = host(pfr().resample_metropolis(wd, B, seed=6, offset=2, workspace=torch_ws))
    ar0 = host(pfr().resample_rejection(wd, 1.0, seed=6, offset=2, workspace=torch_ws))
    assert np.array_equal(am, am0) and np.array_equal(ar, ar0)
    if n <= (1 << 20):
        assert np.array_equal(am, oracle.metropolis(w, B, seed=6, offset=2))
        assert np.array_equal(ar, oracle.rejection(w, 1.0, seed=6, offset=2)[0])


@pytest.mark.parametrize("n", [5000, 1 << 17])
def test_alternatives_tiny_binary64_weights(n):
    """Binary64 weights scaled by 2^-900 (inside the range where the single
    fused multiply-add accept test is exact) give the oracle's ancestors for
    Metropolis and rejection, on the LDS-staged (n = 5000) and the bound-table
    (n = 2^17) paths."""
    w = inputs.weights(n, 2.0, seed=n + 21).astype(np.float64) * 2.0**-900
    wmax = float(w.max())
    a = host(pfr().resample_metropolis(dev(w), 24, seed=4))
    assert np.array_equal(a, oracle.metropolis(w, 24, seed=4))
    a = host(pfr().resample_rejection(dev(w), wmax, seed=4))
    assert np.array_equal(a, oracle.rejection(w, wmax, seed=4)[0])


@pytest.mark.parametrize("n", [5000, 1 << 17, 1 << 20])
def test_alternatives_subnormal_binary64_weights(n):
    """Binary64 weights k 2^-1074, k = 0..7 (subnormal): a rounded fused
    multiply-add maps many nonzero differences u w_k - w_j to zero here (for
    w_k = 3 2^-1074, w_j = 2^-1074 every u in (1/3, 1/2) does), so the exact
    accept test must decide them on rescaled weights.  Metropolis (staged, global
    and bound-table paths) and rejection must give the oracle's ancestors (Code 2
    and Code 3 with the exact test)."""
    rng = np.random.default_rng(n + 3)
    w = rng.integers(0, 8, size=n).astype(np.float64) * 2.0**-1074
    w[0] = 7 * 2.0**-1074
    assert np.all((w == 0) | (w < 2.0**-1070))
    a = host(pfr().resample_metropolis(dev(w), 24, seed=6))
    assert np.array_equal(a, oracle.metropolis(w, 24, seed=6))
    wmax = float(w.max())
    a = host(pfr().resample_rejection(dev(w), wmax, seed=6))
    assert np.array_equal(a, oracle.rejection(w, wmax, seed=6)[0])


@pytest.mark.parametrize("max_trials", [1, 3, 7, 13])
def test_rejection_table_trial_cap(max_trials):
    """A bound far above the weights on the bound-table path: passes of four
    trials and four-trial tail slots must not use a trial at or beyond the
    cap (odd caps end inside a pass)."""
    n = 1 << 20
    w = inputs.weights(n, 3.0, seed=max_trials)
    fl = new_flags()
    a = host(pfr().resample_rejection(dev(w), 64.0, seed=5, max_trials=max_trials, flags=fl))
    ref, rfl = oracle.rejection(w, 64.0, seed=5, max_trials=max_trials)
    assert np.array_equal(a, ref)
    assert int(host(fl)[0]) == rfl


def test_bound_table_with_zero_and_huge_weights():
    n = 1 << 20
    w = inputs.weights(n, 3.0, seed=1).astype(np.float64)
    w[::7] = 0.0
    w[5] = 1e300  # beyond binary32 codes: the table is switched off for this vector
    a = host(pfr().resample_metropolis(dev(w), 30, seed=3))
    assert np.array_equal(a, oracle.metropolis(w, 30, seed=3))
    w[5] = 1.0
    a = host(pfr().resample_metropolis(dev(w), 30, seed=3))
    assert np.array_equal(a, oracle.metropolis(w, 30, seed=3))
    a = host(pfr().resample_rejection(dev(w), 1.0, seed=3))
    assert np.array_equal(a, oracle.rejection(w, 1.0, seed=3)[0])


# ----------------------------------------------------------------- auxiliaries
@pytest.mark.parametrize("n", [1, 7, 4096, 4097, 50000, 1 << 20])
def test_offspring_to_ancestors_bit_exact(n):
    g = np.random.default_rng(n)
    p = g.random(n) ** 4
    o = g.multinomial(n, p / p.sum()).astype(np.int32)
    a = host(pfr().offspring_to_ancestors(dev(o)))
    ref, fl = oracle.offspring_to_ancestors(o)
    assert fl == 0 and np.array_equal(a, ref)


def test_offspring_to_ancestors_bad_counts():
    for n in (100, 20000):
        g = np.random.default_rng(1)
        cases = [np.zeros(n, np.int32), g.integers(0, 3, n).astype(np.int32),
                 np.full(n, 5, np.int32)]
        neg = g.multinomial(n, np.ones(n) / n).astype(np.int32)
        neg[3] = -4
        cases.append(neg)
        for o in cases:
            fl = new_flags()
            a = host(pfr().offspring_to_ancestors(dev(o), flags=fl))
            ref, rfl = oracle.offspring_to_ancestors(o)
            assert np.array_equal(a, ref)
            assert int(host(fl)[0]) == rfl


def test_offspring_to_ancestors_batched():
    g = np.random.default_rng(2)
    sizes = g.integers(1, 9000, 30)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    o = np.concatenate([g.multinomial(s, np.ones(s) / s) for s in sizes]).astype(np.int32)
    a = host(pfr().offspring_to_ancestors(dev(o), offsets=dev(off)))
    for f in range(sizes.size):
        ref, _ = oracle.offspring_to_ancestors(o[off[f]:off[f + 1]])
        assert np.array_equal(a[off[f]:off[f + 1]], ref)


@pytest.mark.parametrize("n", [1, 2, 5, 1000, 4097, 1 << 20])
def test_permute_sorted_bit_exact(n):
    w = inputs.weights(n, 3.0, seed=n)
    a, _ = oracle.systematic(w, seed=2)
    c = host(pfr().permute_ancestors(dev(a), sorted_hint=True))
    ref, fl = oracle.permute(a)
    assert fl == 0 and np.array_equal(c, ref)


@pytest.mark.parametrize("n", [1, 3, 1000, 65536, 1 << 20])
def test_permute_unsorted_bit_exact(n):
    w = inputs.weights(n, 3.0, seed=n + 1)
    a, _ = oracle.rejection(w, 1.0, seed=4)
    c = host(pfr().permute_ancestors(dev(a), sorted_hint=False))
    ref, fl = oracle.permute(a)
    assert fl == 0 and np.array_equal(c, ref)
    g = np.random.default_rng(n)
    a = g.integers(0, n, n).astype(np.int32)
    c = host(pfr().permute_ancestors(dev(a)))
    assert np.array_equal(c, oracle.permute(a)[0])


@pytest.mark.parametrize("hint", [True, False])
@pytest.mark.parametrize("max_len", [None, "exact"])
def test_permute_batched_lds_and_global_segments(hint, max_len):
    g = np.random.default_rng(7)
    sizes = [5, 20000, 0, 16384, 16385, 700, 1, 40000]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    parts = []
    for s in sizes:
        p = g.random(s) ** 6 if s else np.zeros(0)
        a = g.choice(s, size=s, p=p / p.sum()).astype(np.int32) if s else np.zeros(0, np.int32)
        parts.append(np.sort(a) if hint else a)
    a = np.concatenate(parts).astype(np.int32)
    # out of range: treated as its own index and flagged; at the end of the
    # first segment it keeps a sorted ancestry sorted
    a[4 if hint else 3] = 99
    fl = new_flags()
    c = host(pfr().permute_ancestors(dev(a), sorted_hint=hint, offsets=dev(off),
                                     max_len=max(sizes) if max_len else None, flags=fl))
    for f, s in enumerate(sizes):
        if s == 0:
            continue
        ref, _ = oracle.permute(a[off[f]:off[f + 1]])
        assert np.array_equal(c[off[f]:off[f + 1]], ref), f
    assert int(host(fl)[0]) == pfr().FLAG_BAD_ANCESTOR
    if hint:  # sorted input through the atomic-free claim (segment 0 has the bad value)
        a2 = a.copy()
        a2[3] = 0
        a2[off[0]:off[1]] = np.sort(a2[off[0]:off[1]])
        c2 = host(pfr().permute_ancestors(dev(a2), sorted_hint=True, offsets=dev(off),
                                          max_len=max(sizes) if max_len else None))
        for f, s in enumerate(sizes):
            if s:
                ref, _ = oracle.permute(a2[off[f]:off[f + 1]])
                assert np.array_equal(c2[off[f]:off[f + 1]], ref), f


def test_permute_bad_ancestors_and_batched():
    a = np.array([1, 9, -3, 1, 0], dtype=np.int32)
    fl = new_flags()
    c = host(pfr().permute_ancestors(dev(a), flags=fl))
    ref, rfl = oracle.permute(a)
    assert np.array_equal(c, ref) and int(host(fl)[0]) == rfl
    g = np.random.default_rng(3)
    sizes = g.integers(1, 3000, 25)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    a = np.concatenate([np.sort(g.integers(0, s, s)) for s in sizes]).astype(np.int32)
    for hint in (True, False):
        c = host(pfr().permute_ancestors(dev(a), sorted_hint=hint, offsets=dev(off)))
        for f in range(sizes.size):
            ref, _ = oracle.permute(a[off[f]:off[f + 1]])
            assert np.array_equal(c[off[f]:off[f + 1]], ref)


def test_permute_degenerate_ancestries():
    # many equal claims inside one workgroup, and distinct slots that share a
    # low-bits entry of the per-workgroup claim table (multiples of 256)
    n = 1 << 20
    g = np.random.default_rng(11)
    cases = {
        "one parent": np.full(n, 12345, np.int32),
        "sixteen parents": g.integers(0, 16, n).astype(np.int32) * 4099,
        "colliding slots": g.integers(0, 16, n).astype(np.int32) * 256,
        "two blocks": np.repeat(np.array([n - 1, 0], np.int32), n // 2),
    }
    for name, a in cases.items():
        ref, _ = oracle.permute(a)
        c = host(pfr().permute_ancestors(dev(a), sorted_hint=False))
        assert np.array_equal(c, ref), name
    # the same through the batched global kernels (segments longer than 16384)
    sizes = [100000, 3, 70000, 40000]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    a = np.concatenate([np.full(sizes[0], 7), g.integers(0, 3, 3), g.integers(0, 4, sizes[2]) * 256,
                        np.full(sizes[3], sizes[3] - 1)]).astype(np.int32)
    c = host(pfr().permute_ancestors(dev(a), sorted_hint=False, offsets=dev(off)))
    for f in range(len(sizes)):
        ref, _ = oracle.permute(a[off[f]:off[f + 1]])
        assert np.array_equal(c[off[f]:off[f + 1]], ref), f


@pytest.mark.parametrize("n", [4097, 5000, (1 << 22) + 3, 5 * (1 << 20) + 7])
def test_permute_unsorted_bucketed_and_atomic_claims(n):
    """One unsorted vector beyond the LDS path: the claim by buckets of slots
    (full workspace) and the atomic claim (a workspace of only the claim
    vector and marks) give Code 10's permutation; out-of-range ancestors are
    flagged and count as their own index on both."""
    m = pfr()
    g = np.random.default_rng(n)
    p = g.random(n) ** 8
    a = g.choice(n, size=n, p=p / p.sum()).astype(np.int32)
    a[g.integers(0, n, 5)] = np.array([-1, n, n + 7, -100, 2**31 - 1], dtype=np.int32)
    ref, rfl = oracle.permute(a)
    full = m.workspace_bytes(m._lib.OP_PERMUTE, n)
    small = 2 * ((4 * n + 255) // 256 * 256)
    assert full > small
    for nbytes in (full, small):
        fl = new_flags()
        c = host(m.permute_ancestors(dev(a), flags=fl, workspace=m.new_workspace(nbytes)))
        assert np.array_equal(c, ref), nbytes
        assert int(host(fl)[0]) == rfl == m.FLAG_BAD_ANCESTOR


def test_permute_long_chain():
    # a = [0, 0, 1, 2, ..., n-2]: one chain runs through every slot
    n = 3000
    a = np.concatenate([[0], np.arange(n - 1)]).astype(np.int32)
    ref, _ = oracle.permute(a)
    for hint in (True, False):
        c = host(pfr().permute_ancestors(dev(a), sorted_hint=hint))
        assert np.array_equal(c, ref)
