"""GPU parity of the auxiliary exports against the oracle: offspring counts
(Code 12), the effective sample size (section 3.4) and the in-place copy step
(section 2.3) for states of several dimensions and layouts.

Counts and copies are integer / byte work and must match bit for bit; the
ESS must lie within the documented error bound of the oracle's binary128
value."""
import math

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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def flags():
    return torch.zeros(1, dtype=torch.int32, device="cuda")


def ragged_offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


# ------------------------------------------------------------------ Code 12
def sorted_ancestries(n, rng):
    """Non-decreasing ancestries of several shapes."""
    out = {"systematic": None}
    w = inputs.weights(n, 2.0, seed=int(rng.integers(1 << 30)))
    out["systematic"] = oracle.systematic(w.astype(np.float64), seed=3)[0]
    out["one_parent"] = np.full(n, n // 2, dtype=np.int32)
    out["identity"] = np.arange(n, dtype=np.int32)
    out["random_sorted"] = np.sort(rng.integers(0, n, n)).astype(np.int32)
    # few parents with long runs and wide gaps
    k = max(1, n // 1000)
    out["few_parents"] = np.sort(rng.choice(n, k, replace=True)[rng.integers(0, k, n)]).astype(
        np.int32)
    return out


@pytest.mark.parametrize("n", [1, 2, 100, 4095, 4096, 4097, 70001, (1 << 20) + 123])
def test_a2o_single_vector_sorted_and_unsorted(n):
    rng = np.random.default_rng(n)
    for name, a in sorted_ancestries(n, rng).items():
        ref, fl_ref = oracle.ancestors_to_offspring(a)
        for hint in (True, False):
            fl = flags()
            o = host(pfr().ancestors_to_offspring(dev(a), sorted_hint=hint, flags=fl))
            assert np.array_equal(o, ref), (name, hint)
            assert int(host(fl)[0]) == fl_ref == 0
    a = rng.integers(0, n, n).astype(np.int32)  # unsorted
    o = host(pfr().ancestors_to_offspring(dev(a)))
    assert np.array_equal(o, oracle.ancestors_to_offspring(a)[0])


def test_a2o_metropolis_output():
    n = 1 << 16
    w = inputs.weights(n, 1.0, seed=4)
    a = pfr().resample_metropolis(dev(w), 8, seed=2)
    o = host(pfr().ancestors_to_offspring(a))
    assert np.array_equal(o, oracle.ancestors_to_offspring(host(a))[0])
    assert o.sum() == n


@pytest.mark.parametrize("hint", [True, False])
def test_a2o_out_of_range_ancestors(hint):
    n = 9000
    a = np.sort(np.random.default_rng(1).integers(0, n, n)).astype(np.int32)
    a[:3] = [-5, -1, -1]
    a[-2:] = [n, n + 7]
    ref, fl_ref = oracle.ancestors_to_offspring(a)
    assert fl_ref == oracle.FLAG_BAD_ANCESTOR
    fl = flags()
    o = host(pfr().ancestors_to_offspring(dev(a), sorted_hint=hint, flags=fl))
    assert np.array_equal(o, ref)
    assert int(host(fl)[0]) == pfr().FLAG_BAD_ANCESTOR


@pytest.mark.parametrize("hint", [True, False])
@pytest.mark.parametrize("with_max_len", [True, False])
def test_a2o_ragged_batch(hint, with_max_len):
    rng = np.random.default_rng(7)
    sizes = np.array([0, 1, 5, 300, 4096, 16384, 16385, 0, 20000, 777, 70000, 2, 140001])
    off = ragged_offsets(sizes)
    parts = []
    for f, n in enumerate(sizes):
        if n == 0:
            continue
        a = np.sort(rng.integers(0, n, n)) if hint else rng.integers(0, n, n)
        if f == 5:
            a = np.full(n, n - 1)  # one parent at the end of its segment
        parts.append(a.astype(np.int32))
    a = np.concatenate(parts)
    fl = flags()
    o = host(pfr().ancestors_to_offspring(dev(a), sorted_hint=hint, offsets=dev(off),
                                          max_len=int(sizes.max()) if with_max_len else None,
                                          flags=fl))
    assert int(host(fl)[0]) == 0
    for f in range(sizes.size):
        sl = slice(off[f], off[f + 1])
        assert np.array_equal(o[sl], oracle.ancestors_to_offspring(a[sl])[0]), f


def test_a2o_ragged_batch_of_resampler_outputs():
    w, off, _ = inputs.ragged_batch(n_filters=64, seed=3)
    wd, od = dev(w), dev(off)
    ml = int(np.diff(off).max())
    a = pfr().resample_systematic(wd, seed=1, offsets=od, max_len=ml)
    o = host(pfr().ancestors_to_offspring(a, sorted_hint=True, offsets=od, max_len=ml))
    ah = host(a)
    for f in range(64):
        sl = slice(off[f], off[f + 1])
        assert np.array_equal(o[sl], oracle.ancestors_to_offspring(ah[sl])[0]), f


# ------------------------------------------------------------------ ESS
def ess_bound(n):
    """Relative error bound of the GPU ESS (header): (3d + 8) 2^-53 with
    d = 31 + ceil(P / 64), P = ceil(n / 4096); plus half an ulp for the
    oracle's final rounding."""
    P = -(-n // 4096)
    d = 31 + -(-P // 64)
    return (3 * d + 8) * 2.0**-53 + 2.0**-53


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [1, 3, 4095, 4096, 4097, 100000, 1 << 22])
def test_ess_single_vector(n, dtype):
    w = inputs.weights(n, 2.0, seed=n).astype(dtype)
    ref, fl_ref = oracle.ess(w)
    fl = flags()
    e = float(host(pfr().effective_sample_size(dev(w), flags=fl))[0])
    assert fl_ref == 0 and int(host(fl)[0]) == 0
    assert abs(e - ref) <= ess_bound(n) * ref, (e, ref)


def test_ess_ragged_batch_and_edge_segments():
    rng = np.random.default_rng(5)
    sizes = np.array([0, 1, 4096, 9000, 5, 70000, 3, 4, 2])
    off = ragged_offsets(sizes)
    segs = []
    for n in sizes:
        segs.append(rng.exponential(size=n))
    segs[4][:] = 0.0          # all zero
    segs[6][1] = -1.0         # negative weight
    segs[7][2] = np.nan       # NaN
    segs[8][:] = [1e300, 3e299]  # squares overflow binary64
    w = np.concatenate(segs)
    fl = flags()
    e = host(pfr().effective_sample_size(dev(w), offsets=dev(off), flags=fl))
    assert int(host(fl)[0]) == pfr().FLAG_ZERO_TOTAL | pfr().FLAG_BAD_WEIGHTS
    for f, n in enumerate(sizes):
        ref, _ = oracle.ess(segs[f])
        if math.isnan(ref):
            assert math.isnan(e[f]), f
        else:
            assert abs(e[f] - ref) <= ess_bound(max(n, 1)) * max(ref, 1e-300), (f, e[f], ref)
    assert e[0] == 0.0 and e[4] == 0.0 and e[1] == 1.0


def test_ess_exact_properties():
    """Equal weights with a short significand (exact sums) give n exactly; a
    power-of-two scaling that keeps every weight normal, and the position of
    a segment in a batch, leave every bit unchanged."""
    n = 300000
    assert float(host(pfr().effective_sample_size(dev(np.full(n, 0.375))))[0]) == n
    w = inputs.weights(n, 1.0, seed=9).astype(np.float64)
    e0 = host(pfr().effective_sample_size(dev(w)))[0]
    e1 = host(pfr().effective_sample_size(dev(w * 2.0**600)))[0]
    e2 = host(pfr().effective_sample_size(dev(w * 2.0**-700)))[0]
    assert e0 == e1 == e2
    batch = np.concatenate([np.ones(12345), w, w[:777]])
    off = ragged_offsets([12345, n, 777])
    eb = host(pfr().effective_sample_size(dev(batch), offsets=dev(off)))
    assert eb[1] == e0 and eb[0] == 12345.0


# ------------------------------------------------------------------ copy
def element_sources(c, dim):
    """Which source element each element of an (n, dim) state receives, from
    the oracle's out-of-place copy applied to element ids."""
    n = c.size
    ids = np.arange(n * dim, dtype=np.float64).reshape(n, dim)
    out, fl = oracle.copy_rows(c, ids)
    return out.astype(np.int64), fl


def permuted_ancestry(n, rng):
    w = inputs.weights(n, 2.0, seed=int(rng.integers(1 << 30)))
    a = oracle.stratified(w.astype(np.float64), seed=1)[0]
    return oracle.permute(a)[0]


@pytest.mark.parametrize("dtype,dim", [(torch.float32, 1), (torch.float32, 3), (torch.float64, 5),
                                       (torch.int16, 7), (torch.uint8, 2),
                                       (torch.complex128, 2)])
@pytest.mark.parametrize("layout", ["rows", "columns"])
def test_copy_single_vector(dtype, dim, layout):
    n = 50000
    rng = np.random.default_rng(dim)
    c = permuted_ancestry(n, rng)
    src, fl_ref = element_sources(c, dim)
    assert fl_ref == 0
    vals = torch.arange(n * dim, device="cuda") % 251
    if layout == "rows":
        x = vals.reshape(n, dim).to(dtype)                 # strides (dim, 1)
    else:
        x = vals.reshape(n, dim).t().contiguous().to(dtype).t()  # strides (1, n)
    before = host(x).reshape(-1)
    fl = flags()
    pfr().copy_particles(dev(c), x, flags=fl)
    assert int(host(fl)[0]) == 0
    assert np.array_equal(host(x), before[src].reshape(n, dim))


def test_copy_ragged_batch_with_bad_entries():
    rng = np.random.default_rng(11)
    sizes = np.array([3, 0, 4096, 1, 20000, 17])
    off = ragged_offsets(sizes)
    cs = [permuted_ancestry(n, rng) if n > 1 else np.zeros(n, dtype=np.int32) for n in sizes]
    cs[2] = cs[2].copy()
    cs[2][10] = 5000          # outside its segment
    cs[5] = np.array([1, 2, 2] + list(range(3, 17)), dtype=np.int32)  # source overwritten
    c = np.concatenate(cs).astype(np.int32)
    dim = 4
    x0 = rng.normal(size=(c.size, dim))
    x = dev(x0)
    fl = flags()
    pfr().copy_particles(dev(c), x, offsets=dev(off), flags=fl)
    got = host(x)
    assert int(host(fl)[0]) == pfr().FLAG_BAD_ANCESTOR
    for f in range(sizes.size):
        sl = slice(off[f], off[f + 1])
        ref, _ = oracle.copy_rows(cs[f], x0[sl])
        assert np.array_equal(got[sl], ref), f


def test_copy_after_resampling_equals_gather():
    """Resample, permute and copy on the GPU: the state equals x[c] taken
    out of place, and its rows are those of x[a] rearranged."""
    n = 1 << 18
    w = inputs.weights(n, 3.0, seed=2)
    a = pfr().resample_systematic(dev(w), seed=8)
    c = pfr().permute_ancestors(a, sorted_hint=True)
    x0 = np.random.default_rng(0).normal(size=(n, 2)).astype(np.float32)
    x = dev(x0)
    pfr().copy_particles(c, x)
    ch, ah = host(c), host(a)
    got = host(x)
    assert np.array_equal(got, x0[ch])
    assert np.array_equal(np.sort(got[:, 0]), np.sort(x0[ah, 0]))
