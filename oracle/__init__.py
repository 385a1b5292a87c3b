"""CPU oracle for the resampling step -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around ``liboracle.so`` (``pfr_oracle.c``): a plain, slow,
single-threaded reference of Murray, Lee & Jacob, "Parallel resampling in the
particle filter" (arXiv:1301.4019), used by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports this
package; it shares no code with the HIP library.

All functions take and return numpy arrays.  Weights are converted to float64
(an exact widening for float32 input).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pfr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FLAG_ZERO_TOTAL = 1
FLAG_TRIAL_CAP = 2
FLAG_BAD_COUNTS = 4
FLAG_BAD_WEIGHTS = 8
FLAG_BAD_ANCESTOR = 16

DOM_STRATA, DOM_EXP, DOM_TRIAL, DOM_NOISE, DOM_INIT, DOM_UNIFORM = 0, 1, 2, 3, 4, 5


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no fast-math, no FP contraction)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u32, i32, i64, u64, dbl = (ctypes.c_uint32, ctypes.c_int32, ctypes.c_int64,
                               ctypes.c_uint64, ctypes.c_double)
    P = ctypes.c_void_p
    sig = {
        "orc_philox4x32_10": (None, [P, P, P]),
        "orc_philox4x32_r": (None, [P, P, ctypes.c_int, P]),
        "orc_set_philox_rounds": (ctypes.c_int, [ctypes.c_int]),
        "orc_u_accept": (dbl, [u32]),
        "orc_index": (i64, [u32, u32, i64]),
        "orc_accept": (ctypes.c_int, [dbl, dbl, dbl]),
        "orc_resample_metropolis": (ctypes.c_int, [P, i64, i32, u64, u32, u32, P]),
        "orc_resample_rejection": (ctypes.c_int, [P, i64, dbl, u32, u64, u32, u32, P, P, P]),
        "orc_stratified_u": (ctypes.c_int, [P, i64, P, P, P, P]),
        "orc_resample_partial_rejection": (ctypes.c_int, [P, i64, dbl, u32, u64, u32, u32, P, P,
                                                          P]),
        "orc_resample_stratified": (ctypes.c_int, [P, i64, u64, u32, u32, P, P, P]),
        "orc_resample_systematic": (ctypes.c_int, [P, i64, u64, u32, u32, P, P, P]),
        "orc_systematic_offset": (dbl, [u64, u32, u32]),
        "orc_stratum_offsets": (None, [i64, u64, u32, u32, P]),
        "orc_resample_multinomial": (ctypes.c_int, [P, i64, u64, u32, u32, P, P, P, P]),
        "orc_multinomial_points": (ctypes.c_int, [P, i64, P, P, P]),
        "orc_resample_multinomial_iid": (ctypes.c_int, [P, i64, u64, u32, u32, P, P, P, P]),
        "orc_offspring_to_ancestors": (ctypes.c_int, [P, i64, P, P]),
        "orc_ancestors_to_offspring": (ctypes.c_int, [P, i64, P, P]),
        "orc_permute": (ctypes.c_int, [P, i64, P, P, P]),
        "orc_ess": (ctypes.c_int, [P, i64, P, P]),
        "orc_copy_rows": (ctypes.c_int, [P, i64, i64, P, P, P]),
        "orc_permute_serial": (ctypes.c_int, [P, i64]),
        "orc_normal": (dbl, [u64, u32, u32, u32, u32, u32]),
        "orc_lgssm_init": (None, [i32, i32, dbl, u64, u32, u32, P]),
        "orc_lgssm_move": (None, [i32, i32, dbl, dbl, dbl, u32, dbl, u64, u32, u32, P, P, P, P,
                                  P]),
        "orc_kalman_loglik": (dbl, [P, i64, dbl, dbl, dbl, dbl]),
        "orc_threads": (ctypes.c_int, [ctypes.c_int]),
        "orc_resample_metropolis_mt": (ctypes.c_int, [P, i64, i32, u64, u32, u32, P,
                                                      ctypes.c_int]),
        "orc_resample_rejection_mt": (ctypes.c_int, [P, i64, dbl, u32, u64, u32, u32, P, P, P,
                                                     ctypes.c_int]),
        "orc_batch_mt": (ctypes.c_int, [ctypes.c_int, P, P, P, i32, P, dbl, u64, u32, u32, P, P,
                                        P, P, ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(x):
    return None if x is None else x.ctypes.data_as(ctypes.c_void_p)


def _w(w):
    return np.ascontiguousarray(np.asarray(w), dtype=np.float64)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"oracle {name} rejected its arguments")


# ------------------------------------------------------------------ Philox
def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: ctr = 4 uint32, key = 2 uint32 -> 4 uint32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox4x32_r(ctr, key, rounds):
    """One Philox4x32 block with the given round count."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_r(_ptr(c), _ptr(k), int(rounds), _ptr(out))
    return out


_ROUNDS = 10  # round count of draw(), kept equal to the C side's


class philox_rounds:
    """Context manager: every draw of the oracle uses this many Philox rounds
    (the round-count study), 10 again on exit."""

    def __init__(self, rounds):
        self.rounds = int(rounds)

    def __enter__(self):
        global _ROUNDS
        _check(_load().orc_set_philox_rounds(self.rounds), "philox_rounds")
        _ROUNDS = self.rounds
        return self

    def __exit__(self, *exc):
        global _ROUNDS
        _load().orc_set_philox_rounds(10)
        _ROUNDS = 10
        return False


def draw(seed, index, domain, step, filt=0, offset=0):
    """The canonical Philox call for (index, domain, step, filter, offset)."""
    ctr = [index & 0xFFFFFFFF, ((domain << 28) | (step & 0x0FFFFFFF)) & 0xFFFFFFFF,
           filt & 0xFFFFFFFF, offset & 0xFFFFFFFF]
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    return philox4x32_r(ctr, key, _ROUNDS)


def u_accept(x):
    return _load().orc_u_accept(int(x))


def index(x0, x1, n):
    return _load().orc_index(int(x0), int(x1), int(n))


def accept(u, w_k, w_j):
    return bool(_load().orc_accept(float(u), float(w_k), float(w_j)))


# ------------------------------------------------------------------ resamplers
def metropolis(w, B, seed=0, filt=0, offset=0):
    w = _w(w)
    a = np.empty(w.size, dtype=np.int32)
    _check(_load().orc_resample_metropolis(_ptr(w), w.size, int(B), seed, filt, offset,
                                           _ptr(a)), "metropolis")
    return a


def rejection(w, w_max, seed=0, filt=0, offset=0, max_trials=1 << 20, return_trials=False):
    w = _w(w)
    a = np.empty(w.size, dtype=np.int32)
    t = np.empty(w.size, dtype=np.uint32)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_resample_rejection(_ptr(w), w.size, float(w_max), int(max_trials),
                                          seed, filt, offset, _ptr(a), _ptr(t), _ptr(fl)),
           "rejection")
    if return_trials:
        return a, int(fl[0]), t
    return a, int(fl[0])


def stratified_u(w, u, return_r=False):
    w = _w(w)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.size >= w.size
    a = np.empty(w.size, dtype=np.int32)
    r = np.empty(w.size, dtype=np.float64)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_stratified_u(_ptr(w), w.size, _ptr(u), _ptr(a), _ptr(r), _ptr(fl)),
           "stratified_u")
    return (a, int(fl[0]), r) if return_r else (a, int(fl[0]))


def stratified(w, seed=0, filt=0, offset=0, return_r=False):
    w = _w(w)
    a = np.empty(w.size, dtype=np.int32)
    r = np.empty(w.size, dtype=np.float64)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_resample_stratified(_ptr(w), w.size, seed, filt, offset, _ptr(a),
                                           _ptr(r), _ptr(fl)), "stratified")
    return (a, int(fl[0]), r) if return_r else (a, int(fl[0]))


def systematic(w, seed=0, filt=0, offset=0, return_r=False):
    w = _w(w)
    a = np.empty(w.size, dtype=np.int32)
    r = np.empty(w.size, dtype=np.float64)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_resample_systematic(_ptr(w), w.size, seed, filt, offset, _ptr(a),
                                           _ptr(r), _ptr(fl)), "systematic")
    return (a, int(fl[0]), r) if return_r else (a, int(fl[0]))


def systematic_offset(seed=0, filt=0, offset=0):
    return _load().orc_systematic_offset(seed, filt, offset)


def stratum_offsets(n, seed=0, filt=0, offset=0):
    u = np.empty(n, dtype=np.float64)
    _load().orc_stratum_offsets(n, seed, filt, offset, _ptr(u))
    return u


def multinomial(w, seed=0, filt=0, offset=0, return_rp=False):
    w = _w(w)
    a = np.empty(w.size, dtype=np.int32)
    r = np.empty(w.size, dtype=np.float64)
    p = np.empty(w.size, dtype=np.float64)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_resample_multinomial(_ptr(w), w.size, seed, filt, offset, _ptr(a),
                                            _ptr(r), _ptr(p), _ptr(fl)), "multinomial")
    return (a, int(fl[0]), r, p) if return_rp else (a, int(fl[0]))


def partial_rejection(w, v_max, seed=0, filt=0, offset=0, max_trials=1 << 20):
    """Partial rejection control -> (ancestors, importance weights (float64), flags)."""
    w = _w(w)
    a = np.empty(w.size, dtype=np.int32)
    wo = np.empty(w.size, dtype=np.float64)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_resample_partial_rejection(_ptr(w), w.size, float(v_max), max_trials,
                                                  int(seed) & (2**64 - 1), filt, offset, _ptr(a),
                                                  _ptr(wo), _ptr(fl)), "partial_rejection")
    return a, wo, int(fl[0])


def multinomial_iid(w, seed=0, filt=0, offset=0, return_rp=False):
    """Code 5 with one independent uniform per particle (unsorted output)."""
    w = _w(w)
    a = np.empty(w.size, dtype=np.int32)
    r = np.empty(w.size, dtype=np.float64)
    p = np.empty(w.size, dtype=np.float64)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_resample_multinomial_iid(_ptr(w), w.size, int(seed) & (2**64 - 1), filt,
                                                offset, _ptr(a), _ptr(r), _ptr(p), _ptr(fl)),
           "multinomial_iid")
    return (a, int(fl[0]), r, p) if return_rp else (a, int(fl[0]))


def multinomial_points(w, p):
    w = _w(w)
    p = np.ascontiguousarray(p, dtype=np.float64)
    a = np.empty(w.size, dtype=np.int32)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_multinomial_points(_ptr(w), w.size, _ptr(p), _ptr(a), _ptr(fl)),
           "multinomial_points")
    return a, int(fl[0])


# ------------------------------------------------------------------ all-cores legs
def default_threads():
    """Host threads for the all-cores legs: every core, at most 16."""
    return max(1, min(16, os.cpu_count() or 1))


def threads(requested=0):
    """The number of host threads a call with `requested` threads uses."""
    return int(_load().orc_threads(int(requested)))


def metropolis_mt(w, B, seed=0, filt=0, offset=0, nthreads=None):
    """metropolis() over disjoint lane ranges on several host threads (same bits)."""
    w = _w(w)
    a = np.empty(w.size, dtype=np.int32)
    nt = default_threads() if nthreads is None else int(nthreads)
    _check(_load().orc_resample_metropolis_mt(_ptr(w), w.size, int(B), seed, filt, offset,
                                              _ptr(a), nt), "metropolis_mt")
    return a


def rejection_mt(w, w_max, seed=0, filt=0, offset=0, max_trials=1 << 20, nthreads=None):
    """rejection() over disjoint lane ranges on several host threads (same bits)."""
    w = _w(w)
    a = np.empty(w.size, dtype=np.int32)
    fl = np.zeros(1, dtype=np.uint32)
    nt = default_threads() if nthreads is None else int(nthreads)
    _check(_load().orc_resample_rejection_mt(_ptr(w), w.size, float(w_max), int(max_trials),
                                             seed, filt, offset, _ptr(a), None, _ptr(fl), nt),
           "rejection_mt")
    return a, int(fl[0])


BATCH_OPS = {"multinomial": 0, "stratified": 1, "systematic": 2, "metropolis": 3, "rejection": 4}


def batch_mt(scheme, w, offsets, segs=None, B=None, w_max=1.0, seed=0, filter_base=0, offset=0,
             return_rp=False, nthreads=None):
    """One call per listed vector of a ragged batch, vectors spread over host
    threads.  Returns (a, flags) or, with return_rp, (a, flags, r, p); entries
    outside the listed vectors are left unset."""
    w = _w(w)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    F = off.size - 1
    segs = np.arange(F, dtype=np.int32) if segs is None else np.ascontiguousarray(segs,
                                                                               dtype=np.int32)
    Bv = None if B is None else np.ascontiguousarray(B, dtype=np.int32)
    a = np.full(w.size, -1, dtype=np.int32)
    r = np.full(w.size, np.nan) if return_rp else None
    p = np.full(w.size, np.nan) if (return_rp and scheme == "multinomial") else None
    fl = np.zeros(1, dtype=np.uint32)
    nt = default_threads() if nthreads is None else int(nthreads)
    _check(_load().orc_batch_mt(BATCH_OPS[scheme], _ptr(w), _ptr(off), _ptr(segs), segs.size,
                                _ptr(Bv), float(w_max), int(seed) & (2**64 - 1), filter_base,
                                offset, _ptr(a), _ptr(r), _ptr(p), _ptr(fl), nt), "batch_mt")
    return (a, int(fl[0]), r, p) if return_rp else (a, int(fl[0]))


# ------------------------------------------------------------------ auxiliaries
def offspring_to_ancestors(o):
    o = np.ascontiguousarray(o, dtype=np.int32)
    a = np.empty(o.size, dtype=np.int32)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_offspring_to_ancestors(_ptr(o), o.size, _ptr(a), _ptr(fl)),
           "offspring_to_ancestors")
    return a, int(fl[0])


def ancestors_to_offspring(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    o = np.empty(a.size, dtype=np.int32)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_ancestors_to_offspring(_ptr(a), a.size, _ptr(o), _ptr(fl)),
           "ancestors_to_offspring")
    return o, int(fl[0])


def ess(w):
    """Effective sample size Sum(w)^2 / w^T w -> (ess, flags)."""
    w = _w(w)
    out = np.zeros(1, dtype=np.float64)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_ess(_ptr(w), w.size, _ptr(out), _ptr(fl)), "ess")
    return float(out[0]), int(fl[0])


def copy_rows(c, x):
    """Copy step of section 2.3 out of place: x (n, dim) float64 -> (x', flags)."""
    c = np.ascontiguousarray(c, dtype=np.int32)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x.reshape(-1, 1)
    assert x.shape[0] == c.size
    out = np.empty_like(x)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_copy_rows(_ptr(c), c.size, x.shape[1], _ptr(x), _ptr(out), _ptr(fl)),
           "copy_rows")
    return out, int(fl[0])


def permute(a, return_d=False):
    a = np.ascontiguousarray(a, dtype=np.int32)
    c = np.empty(a.size, dtype=np.int32)
    d = np.empty(a.size, dtype=np.int32)
    fl = np.zeros(1, dtype=np.uint32)
    _check(_load().orc_permute(_ptr(a), a.size, _ptr(c), _ptr(d), _ptr(fl)), "permute")
    return (c, int(fl[0]), d) if return_d else (c, int(fl[0]))


def permute_serial(a):
    a = np.array(a, dtype=np.int32, copy=True)
    _check(_load().orc_permute_serial(_ptr(a), a.size), "permute_serial")
    return a


# ------------------------------------------------------------------ filter
def normal(seed, index, domain, step, filt=0, offset=0):
    """Box-Muller standard normal of one canonical Philox draw."""
    return float(_load().orc_normal(int(seed) & (2**64 - 1), index, domain, step, filt, offset))


def lgssm_init(n_filters, n, s0, seed=0, offset=0, filter_base=0):
    """x_0 (float32, n_filters * n) of the bootstrap filter."""
    x = np.empty(n_filters * n, dtype=np.float32)
    _load().orc_lgssm_init(n_filters, n, float(s0), int(seed) & (2**64 - 1), offset, filter_base,
                           _ptr(x))
    return x


def lgssm_move(c, x, log_z, n_filters, n, phi, q, r, t, y_t, seed=0, offset=0, filter_base=0):
    """Copy, propagate and weight after resampling (one step of Code 1).

    Returns (x, w, log_z, B) as new arrays; the inputs are not modified."""
    c = np.ascontiguousarray(c, dtype=np.int32)
    x = np.array(x, dtype=np.float32, copy=True)
    lz = np.array(log_z, dtype=np.float64, copy=True)
    w = np.empty(n_filters * n, dtype=np.float32)
    B = np.empty(n_filters, dtype=np.int32)
    _load().orc_lgssm_move(n_filters, n, float(phi), float(q), float(r), int(t), float(y_t),
                           int(seed) & (2**64 - 1), offset, filter_base, _ptr(c), _ptr(x),
                           _ptr(w), _ptr(lz), _ptr(B))
    return x, w, lz, B


def kalman_loglik(y, phi, q, r, s0):
    """Exact log p(y_1..y_T) of the linear-Gaussian model (Kalman filter)."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    return float(_load().orc_kalman_loglik(_ptr(y), y.size, float(phi), float(q), float(r),
                                           float(s0)))
