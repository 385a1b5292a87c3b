"""Parity of the benchmark's own cells, in the benchmark's launch configuration.

One step of the timed workload -- n = 2^20 float32 weights for y = 0..4 (data
seed 100 + y), all five resamplers with Philox seed 1 (Metropolis with
B = 4, 6, 16, 60, 354 from eq. (B), rejection with w_max = 1), and the
permutation of every ancestry (the fused claim of resample_permuted for
the three collective schemes) -- is run through the benchmark's own StepWorkload
and every output is compared with the oracle: bit for bit for Metropolis
(Code 2), rejection (Code 3) and the permutation (Code 10), by the tie rule
for the collective schemes (Codes 5, 7, 8).  The oracle's Metropolis and
rejection run on all host cores (bit-identical to the serial oracle).

The ragged 4096-vector batch runs whole in the benchmark's calls; the
collective schemes and rejection are checked on every vector, Metropolis on
every fourth vector by length (1024 vectors over the whole length range).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import inputs
from tiecheck import check_ties, gpu_r_error_bound, strata_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

YS = (0.0, 1.0, 2.0, 3.0, 4.0)


def pfr():
    import paper_1301_4019_amd as m
    return m


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def b_star(y):
    return math.ceil(math.log(0.01) / math.log(1.0 - inputs.expected_weight(y)))


def oracle_collective(scheme, w, seed, filt=0):
    """Oracle ancestry, flags, r, the points and the tie tolerance."""
    n = w.size
    if scheme == "multinomial":
        a_or, fl, r, pts = oracle.multinomial(w, seed=seed, filt=filt, return_rp=True)
        delta = gpu_r_error_bound(w, n) + n * 2.0**-44
    else:
        a_or, fl, r = getattr(oracle, scheme)(w, seed=seed, filt=filt, return_r=True)
        if scheme == "stratified":
            u = oracle.stratum_offsets(n, seed=seed, filt=filt)
        else:
            u = np.full(n, oracle.systematic_offset(seed=seed, filt=filt))
        pts = strata_points(u)
        delta = gpu_r_error_bound(w, n)
    return a_or, fl, r, pts, delta


@pytest.fixture(scope="module")
def step_outputs():
    import bench
    wl = bench.StepWorkload(torch, pfr(), torch.device("cuda:0"), n_streams=1)
    assert tuple(wl.Bs) == (4, 6, 16, 60, 354)
    wl.step(record=False, n_st=1)
    torch.cuda.synchronize()
    assert int(host(wl.flags)[0]) == 0
    outs = {k: host(v) for k, v in wl.out.items()}
    perms = {k: host(v) for k, v in wl.perm.items()}
    ws = [host(w) for w in wl.w]
    return ws, outs, perms


@pytest.mark.parametrize("yi", range(5))
def test_bench_metropolis_bit_exact(step_outputs, yi):
    ws, outs, perms = step_outputs
    y = YS[yi]
    w = ws[yi]
    assert np.array_equal(w, inputs.weights(1 << 20, y, seed=100 + int(y)))
    a = outs[(y, "metropolis")]
    assert np.array_equal(a, oracle.metropolis_mt(w, b_star(y), seed=1)), y
    assert np.array_equal(perms[(y, "metropolis")], oracle.permute(a)[0])


@pytest.mark.parametrize("yi", range(5))
def test_bench_rejection_bit_exact(step_outputs, yi):
    ws, outs, perms = step_outputs
    y = YS[yi]
    a = outs[(y, "rejection")]
    ref, fl = oracle.rejection_mt(ws[yi], 1.0, seed=1)
    assert fl == 0
    assert np.array_equal(a, ref), y
    assert np.array_equal(perms[(y, "rejection")], oracle.permute(a)[0])


@pytest.mark.parametrize("scheme", ["multinomial", "stratified", "systematic"])
@pytest.mark.parametrize("yi", range(5))
def test_bench_collective_tie_rule(step_outputs, scheme, yi):
    ws, outs, perms = step_outputs
    y = YS[yi]
    w = ws[yi].astype(np.float64)
    a = outs[(y, scheme)]
    a_or, fl, r, pts, delta = oracle_collective(scheme, w, seed=1)
    assert fl == 0
    assert np.all(np.diff(a) >= 0) and a[0] >= 0 and a[-1] < w.size
    assert np.all(w[a] > 0)
    check_ties(a, a_or, r, pts, delta, max_ties=5 + int(20 * delta * w.size))
    # the permutation (fused claim for the collective schemes) of the GPU's ancestry
    assert np.array_equal(perms[(y, scheme)], oracle.permute(a)[0])


def test_bench_metropolis_table_float64_b354():
    """The bound-table Metropolis kernel on binary64 weights at the dominant cell."""
    n, y = 1 << 20, 4.0
    w = inputs.weights(n, y, seed=104, dtype=np.float64)
    a = host(pfr().resample_metropolis(torch.from_numpy(w).cuda(), 354, seed=1))
    assert np.array_equal(a, oracle.metropolis_mt(w, 354, seed=1))


@pytest.fixture(scope="module")
def batch_outputs():
    import bench
    w_np, off_np, ys = inputs.ragged_batch(n_filters=4096, seed=0)
    w = torch.from_numpy(w_np).cuda()
    off = torch.from_numpy(off_np).cuda()
    max_len = int(np.diff(off_np).max())
    B_np = np.array([b_star(float(v)) for v in ys], dtype=np.int32)
    B = torch.from_numpy(B_np).cuda()
    a = torch.empty(w_np.size, dtype=torch.int32, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    outs = {}
    for name, fn in bench.batch_calls(pfr(), w, off, max_len, B, a, flags).items():
        if name.endswith("comp_f32"):
            continue
        fn()
        outs[name.replace("_exact", "")] = host(a).copy()
    assert int(host(flags)[0]) == 0
    return w_np.astype(np.float64), off_np, B_np, outs


@pytest.mark.parametrize("scheme", ["multinomial", "stratified", "systematic"])
def test_batch_every_vector_collective(batch_outputs, scheme):
    w, off, _, outs = batch_outputs
    a = outs[scheme]
    a_or, fl, r, p = oracle.batch_mt(scheme, w, off, seed=1, return_rp=True)
    assert fl == 0
    for f in range(off.size - 1):
        sl = slice(off[f], off[f + 1])
        seg, ag = w[sl], a[sl]
        if np.array_equal(ag, a_or[sl]):
            continue
        n = seg.size
        if scheme == "multinomial":
            pts, delta = p[sl], gpu_r_error_bound(seg, n) + n * 2.0**-44
        else:
            u = (oracle.stratum_offsets(n, seed=1, filt=f) if scheme == "stratified"
                 else np.full(n, oracle.systematic_offset(seed=1, filt=f)))
            pts, delta = strata_points(u), gpu_r_error_bound(seg, n)
        assert np.all(np.diff(ag) >= 0)
        check_ties(ag, a_or[sl], r[sl], pts, delta, max_ties=5 + int(20 * delta * n))


def test_batch_every_vector_rejection(batch_outputs):
    w, off, _, outs = batch_outputs
    a_or, fl = oracle.batch_mt("rejection", w, off, w_max=1.0, seed=1)
    assert fl == 0
    assert np.array_equal(outs["rejection"], a_or)


def test_batch_metropolis_quarter_of_vectors(batch_outputs):
    w, off, B, outs = batch_outputs
    by_len = np.argsort(np.diff(off), kind="stable")
    segs = np.sort(by_len[::4]).astype(np.int32)
    segs = np.union1d(segs, [0, by_len[-1], off.size - 2]).astype(np.int32)
    a_or, _ = oracle.batch_mt("metropolis", w, off, segs=segs, B=B, seed=1)
    a = outs["metropolis"]
    for f in segs:
        sl = slice(off[f], off[f + 1])
        assert np.array_equal(a[sl], a_or[sl]), f
