"""The exported scaled prefix r_i = n W_i / W_n (pfr_scaled_prefix) against
the oracle's r (binary128 sums rounded once), in every precision mode.

The exact mode stays within the GPU's error bound of the exact value
(tiecheck.gpu_r_error_bound), the floating-point modes within theirs
(tiecheck.float_r_error_bound); r is non-decreasing, ends at n exactly, and
is what the resamplers use: the systematic ancestors recomputed on the host
from the exported r and the Philox offset (Code 8 with the exact floor/frac
test) equal the GPU's, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1301_4019_amd import inputs
from tiecheck import float_r_error_bound, gpu_r_error_bound

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pfr():
    import paper_1301_4019_amd as m
    return m


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


MODES = [("exact", "SCAN_EXACT"), ("f64", "SCAN_F64"), ("comp_f32", "SCAN_COMP_F32"),
         ("naive_f32", "SCAN_NAIVE_F32")]


def systematic_from_r(r, u):
    """Code 8 on a given r: a[s] = #{i : r_i < s + 1 - u} (exact comparison)."""
    n = r.size
    m = np.floor(r)
    f = r - m
    O = np.minimum(m + (f >= 1.0 - u), n).astype(np.int64)
    O[m >= n] = n
    o = np.diff(np.concatenate([[0], O]))
    return np.repeat(np.arange(n, dtype=np.int32), o)


@pytest.mark.parametrize("mode,attr", MODES)
@pytest.mark.parametrize("n,y,dt", [(5000, 2.0, np.float64), (1 << 20, 3.0, np.float32),
                                    ((1 << 22) + 7, 4.0, np.float32)])
def test_scaled_prefix_against_oracle(mode, attr, n, y, dt):
    w = inputs.weights(n, y, seed=n % 97, dtype=dt)
    wd = torch.from_numpy(w).cuda()
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    r = host(pfr().scaled_prefix(wd, precision=getattr(pfr(), attr), flags=fl))
    assert int(host(fl)[0]) == 0
    w64 = w.astype(np.float64)
    _, _, r_or = oracle.systematic(w64, seed=1, return_r=True)
    bound = (gpu_r_error_bound(w64, n) if mode == "exact" else float_r_error_bound(n, mode))
    err = np.abs(r - r_or)
    assert err.max() <= bound, (err.max(), bound)
    assert np.all(np.diff(r) >= 0)
    assert r[-1] == n
    if mode == "exact" and dt == np.float32:
        # the systematic resampler compares against exactly this r
        a = host(pfr().resample_systematic(wd, seed=1))
        u = oracle.systematic_offset(seed=1)
        assert np.array_equal(a, systematic_from_r(r, u))


def test_scaled_prefix_flags_zero_total():
    w = torch.zeros(10000, dtype=torch.float32, device="cuda")
    fl = torch.zeros(1, dtype=torch.int32, device="cuda")
    pfr().scaled_prefix(w, flags=fl)
    assert int(host(fl)[0]) == pfr().FLAG_ZERO_TOTAL
