"""Parity rule for the collective resamplers.

The oracle resolves every point against an r computed in binary128; the GPU
rounds its r (and, for the multinomial scheme, its points) to binary64 after
an exact fixed-point prefix sum.  The two may therefore disagree only where a
point lies within the stated tolerance of a bin boundary.  A disagreement at
output s is accepted only if every boundary r_j between the two answers lies
within delta of the point; the number of such ties is reported and bounded.
"""
import numpy as np


def gpu_r_error_bound(w, n):
    """Bound on |r_gpu - r_exact| (in offspring units) for n weights w.

    Each weight is quantised with absolute error below max(w) 2^-52 (it is
    truncated at 2^-s of its block, s set by the block maximum), so a prefix of
    i weights is off by at most i max(w) 2^-52, i.e. n^2 max(w) 2^-52 / W in r
    units.  The block's first value r(C_b) = n (C_b / Q) costs at most seven
    roundings relative to r <= n (the two 128-bit conversions, the reciprocal
    and the two products); inside a block r = fl(L c + r(C_b)) adds the
    rounding of L, four in c = n 2^k / Q and the final one, at most six more:
    13 n 2^-53 in all, taken as 16 n 2^-53.
    """
    w = np.asarray(w, dtype=np.float64)
    W = w.sum()
    if n == 0 or W == 0:
        return 0.0
    return n * n * w.max() * 2.0**-52 / W + 16.0 * n * 2.0**-53


def check_ties(a_gpu, a_or, r, points, delta, max_ties):
    a_gpu = np.asarray(a_gpu)
    a_or = np.asarray(a_or)
    mism = np.nonzero(a_gpu != a_or)[0]
    for s in mism:
        lo, hi = sorted((int(a_gpu[s]), int(a_or[s])))
        gap = np.abs(r[lo:hi] - points[s])
        assert np.all(gap <= delta), (
            f"output {s}: gpu {a_gpu[s]} oracle {a_or[s]} point {points[s]!r} "
            f"max distance to boundaries {gap.max():.3e} > delta {delta:.3e}")
    assert mism.size <= max_ties, f"{mism.size} ties exceed the bound {max_ties}"
    return int(mism.size)


def strata_points(u):
    """q_s = s + 1 - u_s (binary64; exact enough for a distance test)."""
    u = np.asarray(u, dtype=np.float64)
    s = np.arange(u.size, dtype=np.float64)
    return (s + 1.0) - u


def float_r_error_bound(n, mode):
    """Bound on |r_gpu - r_exact| for the floating-point prefix modes.

    Every prefix value passes through at most k = 42 + n / 2^20 roundings (3
    in a thread's serial sum, 9 in the workgroup scan tree, 3 across waves and
    within the carries, one per chunk of 2^20 weights in the carry chain, ...),
    so |W_i' - W_i| <= k eps W and r = n W_i / W is off by at most
    n (2k + 6) eps, the 6 covering the reciprocal, the two products, the
    binary32 rounding of float64 weights and, for NAIVE_F32, the binary32 sum
    r + u and the 24-bit offsets.  eps is the unit roundoff of one addition:
    2^-53 (F64), 4 * 2^-48 for a double-float addition of non-negative pairs
    (COMP_F32, Joldes, Muller & Popescu 2017), 2^-24 (NAIVE_F32).  Clamping and
    the max-scan only replace a value by a neighbour within the same bound.
    """
    k = 42.0 + n / float(1 << 20)
    eps = {"f64": 2.0**-53, "comp_f32": 4.0 * 2.0**-48, "naive_f32": 2.0**-24}[mode]
    return n * (2.0 * k + 6.0) * eps + 8.0 * n * 2.0**-53
