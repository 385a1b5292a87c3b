"""The tuning parameters only change how work is split: every setting gives
the same bits (and the oracle's, where the parity tests already pin them)."""
import numpy as np
import pytest

from paper_1301_4019_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SETTINGS = [
    {"single_wg_max": 0, "direct_max_blocks": 0, "metropolis_table_min_B": 0,
     "rejection_table": 0, "rejection_per_wave": 64, "metropolis_chunk": 256,
     "batch_scan_wg_max_len": 0, "batch_stage_max_kb": 16, "batch_metropolis_chunk": 1024,
     "batch_rejection_per_wave": 64, "batch_permute_lds_max": 4096},
    {"single_wg_max": 65536, "direct_max_blocks": 2048, "metropolis_table_min_B": 1,
     "rejection_table": 1, "rejection_per_wave": 4096, "metropolis_chunk": 8192,
     "batch_scan_wg_max_len": 65536, "batch_stage_max_kb": 128, "batch_metropolis_chunk": 65536,
     "batch_rejection_per_wave": 4096, "batch_permute_lds_max": 16384},
    {"single_wg_max": 1000, "direct_max_blocks": 7, "metropolis_table_min_B": 20,
     "rejection_table": 1, "rejection_per_wave": 192, "metropolis_chunk": 768,
     "batch_scan_wg_max_len": 4096, "batch_stage_max_kb": 64, "batch_metropolis_chunk": 3072,
     "batch_rejection_per_wave": 192, "batch_permute_lds_max": 8192},
]


def pfr():
    import paper_1301_4019_amd as m
    return m


def run_all(w, off=None, max_len=None):
    m = pfr()
    outs = []
    for s in ("stratified", "systematic", "multinomial"):
        outs.append(getattr(m, "resample_" + s)(w, seed=5, offsets=off, max_len=max_len))
    outs.append(m.resample_metropolis(w, 37, seed=5, offsets=off, max_len=max_len))
    outs.append(m.resample_rejection(w, 1.0, seed=5, offsets=off, max_len=max_len))
    # the permutation of an unsorted (Metropolis) and a sorted (systematic) vector
    outs.append(m.permute_ancestors(outs[3], offsets=off, max_len=max_len))
    outs.append(m.permute_ancestors(outs[1], sorted_hint=True, offsets=off, max_len=max_len))
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("n", [3000, 5000, 70000, 1 << 20])
def test_results_do_not_depend_on_tuning(n):
    m = pfr()
    saved = m.get_tuning()
    w = torch.from_numpy(inputs.weights(n, 3.0, seed=n)).cuda()
    try:
        ref = run_all(w)
        for st in SETTINGS:
            m.set_tuning(**st)
            got = run_all(w)
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), st
    finally:
        m.set_tuning(**saved)


def test_batched_results_do_not_depend_on_tuning():
    m = pfr()
    saved = m.get_tuning()
    lens = [300, 5000, 17000, 1, 0, 40000, 4096, 8193, 1024]
    off = torch.tensor(np.concatenate([[0], np.cumsum(lens)]), dtype=torch.int64).cuda()
    w = torch.from_numpy(np.concatenate([inputs.weights(k, 2.5, seed=k + 1) for k in lens])).cuda()
    try:
        ref = run_all(w, off, max(lens))
        for st in SETTINGS:
            m.set_tuning(**st)
            got = run_all(w, off, max(lens))
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), st
    finally:
        m.set_tuning(**saved)


@pytest.mark.parametrize("case", ["invalid_weights", "loose_bound", "tight_bound", "float64"])
def test_rejection_table_equals_plain_kernel(case):
    """The rejection bound table (distances from the code of w_max) against the
    plain kernel, the table switched off: the same bits, with invalid weights
    (their buckets are never skipped), a bound 16 times the largest weight
    (distances saturate four octaves earlier), one equal to the largest weight
    and binary64 weights near 2^-100."""
    m = pfr()
    saved = m.get_tuning()
    n = 1 << 20
    x = inputs.weights(n, 2.0, seed=11)
    w_max = 1.0
    if case == "invalid_weights":
        x[[7, n // 3]] = np.nan
        x[n // 2] = -0.5
        x[n - 5] = np.inf
    elif case == "loose_bound":
        w_max = 16.0
    elif case == "tight_bound":
        w_max = float(x.max())
    elif case == "float64":
        x = x.astype(np.float64) * 2.0**-100
        w_max = 2.0**-100
    w = torch.from_numpy(x).cuda()
    kw = dict(seed=5)
    try:
        m.set_tuning(**{**saved, "rejection_table": 1})
        fa = torch.zeros(1, dtype=torch.int32, device="cuda")
        a = m.resample_rejection(w, w_max, flags=fa, **kw).cpu().numpy()
        m.set_tuning(**{**saved, "rejection_table": 0})
        fb = torch.zeros(1, dtype=torch.int32, device="cuda")
        b = m.resample_rejection(w, w_max, flags=fb, **kw).cpu().numpy()
    finally:
        m.set_tuning(**saved)
    assert np.array_equal(a, b)
    assert int(fa.cpu()[0]) == int(fb.cpu()[0])
