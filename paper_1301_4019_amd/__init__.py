"""Particle-filter resampling on AMD Instinct MI355X (gfx950).

Python face of libpfresample (include/pfresample.h): the resamplers of Murray,
Lee & Jacob, "Parallel resampling in the particle filter" (arXiv:1301.4019),
the conversion of offspring counts to ancestors and the ancestor permutation
for in-place propagation.  Functions take torch tensors that live on the GPU
and enqueue the library's HIP kernels on the current torch stream; torch only
provides memory and streams.  Nothing here computes on the CPU.

    import paper_1301_4019_amd as pfr
    a = pfr.resample_systematic(w, seed=1)              # w: float32/float64 on cuda
    c = pfr.permute_ancestors(a, sorted_hint=True)
"""
from __future__ import annotations

import collections
import ctypes
import os

from . import _lib
from ._lib import (FLAG_BAD_ANCESTOR, FLAG_BAD_COUNTS, FLAG_BAD_STEP, FLAG_BAD_WEIGHTS,
                   FLAG_NOT_SORTED, FLAG_TRIAL_CAP, FLAG_WMAX_BELOW,
                   FLAG_ZERO_TOTAL, MAX_BATCH_SEGMENT, SCAN_COMP_F32, SCAN_EXACT, SCAN_F64,
                   SCAN_NAIVE_F32, PfrError)

__all__ = [
    "resample_multinomial", "resample_stratified", "resample_systematic",
    "resample_metropolis", "resample_rejection", "offspring_to_ancestors",
    "permute_ancestors", "workspace_bytes", "new_workspace", "version", "PfrError",
    "LGSSMFilter", "get_tuning", "set_tuning", "default_tuning",
    "SCAN_EXACT", "SCAN_F64", "SCAN_COMP_F32", "SCAN_NAIVE_F32",
    "FLAG_ZERO_TOTAL", "FLAG_TRIAL_CAP", "FLAG_BAD_COUNTS", "FLAG_BAD_WEIGHTS",
    "FLAG_BAD_ANCESTOR", "FLAG_BAD_STEP", "FLAG_WMAX_BELOW", "FLAG_NOT_SORTED",
    "MAX_BATCH_SEGMENT", "set_checks", "get_checks", "take_check_flags",
]


def _torch():
    import torch
    return torch


def version() -> str:
    return _lib.load().pfr_version().decode()


def set_checks(on: bool) -> None:
    """Turn the library's precondition checks on or off (process-wide)."""
    _lib.check(_lib.load().pfr_set_checks(1 if on else 0), "set_checks")


def get_checks() -> bool:
    return bool(_lib.load().pfr_get_checks())


def take_check_flags() -> int:
    """Wait for the current stream; return and clear the FLAG_* bits that the
    checks recorded on the current GPU."""
    out = ctypes.c_uint32(0)
    _lib.check(_lib.load().pfr_take_check_flags(_stream(), ctypes.byref(out)),
               "take_check_flags")
    return int(out.value)


def get_tuning() -> dict:
    """The library's launch parameters (pfr_tuning in the C header)."""
    t = _lib.Tuning()
    _lib.check(_lib.load().pfr_get_tuning(ctypes.byref(t)), "get_tuning")
    return {name: int(getattr(t, name)) for name, _ in _lib.Tuning._fields_ if name != "version"}


def set_tuning(**fields) -> None:
    """Change launch parameters (results do not depend on them)."""
    t = _lib.Tuning()
    _lib.check(_lib.load().pfr_get_tuning(ctypes.byref(t)), "get_tuning")
    for k, v in fields.items():
        if k not in dict(_lib.Tuning._fields_) or k == "version":
            raise KeyError(k)
        setattr(t, k, int(v))
    _lib.check(_lib.load().pfr_set_tuning(ctypes.byref(t)), "set_tuning")


def default_tuning() -> dict:
    t = _lib.Tuning()
    _lib.load().pfr_tuning_defaults(ctypes.byref(t))
    return {name: int(getattr(t, name)) for name, _ in _lib.Tuning._fields_ if name != "version"}


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dtype_code(w):
    torch = _torch()
    if w.dtype == torch.float32:
        return _lib.PFR_F32
    if w.dtype == torch.float64:
        return _lib.PFR_F64
    raise TypeError("weights must be float32 or float64")


def _require_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("tensors must be contiguous GPU tensors")


def _segments(n_total, offsets=None, max_len=None):
    if offsets is None:
        return _lib.Segments(int(n_total), 1, None, int(n_total))
    _require_cuda(offsets)
    torch = _torch()
    if offsets.dtype != torch.int64:
        raise TypeError("offsets must be int64")
    nf = offsets.numel() - 1
    return _lib.Segments(int(n_total), int(nf), offsets.data_ptr(),
                         int(max_len) if max_len is not None else 0)


def _per_segment(t, dtype, seg, what):
    """A per-segment device array must have the C type the library reads and
    one entry per segment."""
    if t is None:
        return
    torch = _torch()
    want = {"int32": torch.int32, "float64": torch.float64}[dtype]
    if t.dtype != want or t.numel() < seg.n_filters:
        raise TypeError(f"{what} must be a {dtype} tensor with one entry per segment")


def _rng(seed, offset, filter_base, offset_dev=None):
    return _lib.Rng(int(seed) & (2**64 - 1), int(offset) & 0xFFFFFFFF,
                    int(filter_base) & 0xFFFFFFFF,
                    None if offset_dev is None else offset_dev.data_ptr())


class _WorkspaceCache:
    """Workspaces are zeroed once and reused; calls sharing one must be
    ordered, so there is one per (device, stream, op, size): calls on
    different streams never share a cached workspace.  The least recently
    used ones are dropped once the cached bytes exceed the budget
    ($PFR_WS_CACHE_BYTES, default 4 GiB); a dropped workspace goes back to
    torch's stream-ordered allocator, so work already enqueued on its stream
    still finds it intact."""

    def __init__(self, budget):
        self.budget = int(budget)
        self.items = collections.OrderedDict()
        self.bytes = 0

    def get(self, key):
        ws = self.items.get(key)
        if ws is not None:
            self.items.move_to_end(key)
        return ws

    def put(self, key, ws):
        self.items[key] = ws
        self.bytes += ws.numel()
        while self.bytes > self.budget and len(self.items) > 1:
            _, old = self.items.popitem(last=False)
            self.bytes -= old.numel()

    def clear(self):
        self.items.clear()
        self.bytes = 0


_WS_CACHE = _WorkspaceCache(int(os.environ.get("PFR_WS_CACHE_BYTES", 4 << 30)))


def _stream_key():
    return _torch().cuda.current_stream().cuda_stream


def workspace_bytes(op: int, n_total: int, offsets=None, max_len=None, dtype_code=0) -> int:
    seg = _segments(n_total, offsets, max_len)
    return int(_lib.load().pfr_workspace_bytes(op, ctypes.byref(seg), dtype_code))


def new_workspace(nbytes: int, device=None):
    """A zero-initialised workspace of at least nbytes (256-byte aligned)."""
    torch = _torch()
    nbytes = max(256, (int(nbytes) + 255) // 256 * 256)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")
    _lib.check(_lib.load().pfr_workspace_init(_ptr(ws), nbytes, _stream()), "workspace_init")
    return ws


def _workspace(op, seg, dtype_code, device, ws):
    need = int(_lib.load().pfr_workspace_bytes(op, ctypes.byref(seg), dtype_code))
    if ws is not None:
        return ws, need
    if need == 0:
        return None, 0
    key = (str(device), _stream_key(), op, need)
    cached = _WS_CACHE.get(key)
    if cached is None:
        cached = new_workspace(need, device)
        _WS_CACHE.put(key, cached)
    return cached, need


def _out_like(n, device, out):
    torch = _torch()
    if out is None:
        return torch.empty(n, dtype=torch.int32, device=device)
    if out.dtype != torch.int32 or out.numel() != n:
        raise ValueError("out must be an int32 tensor with one entry per particle")
    _require_cuda(out)
    return out


def _collective(fn_name, op, w, seed, offset, filter_base, precision, offsets, max_len, out,
                flags, workspace):
    _require_cuda(w, flags)
    dt = _dtype_code(w)
    seg = _segments(w.numel(), offsets, max_len)
    a = _out_like(w.numel(), w.device, out)
    ws, _ = _workspace(op, seg, dt, w.device, workspace)
    fn = getattr(_lib.load(), fn_name)
    rc = fn(_ptr(w), dt, ctypes.byref(seg), int(precision), _rng(seed, offset, filter_base),
            _ptr(a), _ptr(ws), 0 if ws is None else ws.numel(), _ptr(flags), _stream())
    _lib.check(rc, fn_name)
    return a


def resample_multinomial(w, seed=0, offset=0, filter_base=0, precision=SCAN_EXACT, offsets=None,
                         max_len=None, out=None, flags=None, workspace=None):
    """Multinomial ancestry (Code 5, sorted uniforms); see resample_multinomial in the C header."""
    return _collective("resample_multinomial", _lib.OP_MULTINOMIAL, w, seed, offset, filter_base,
                       precision, offsets, max_len, out, flags, workspace)


def resample_multinomial_iid(w, seed=0, offset=0, filter_base=0, out=None, flags=None,
                             workspace=None):
    """Multinomial ancestry as Code 5 prints it: one independent uniform and
    one search per particle (unsorted output; single vectors)."""
    _require_cuda(w, flags)
    dt = _dtype_code(w)
    seg = _segments(w.numel())
    a = _out_like(w.numel(), w.device, out)
    ws, _ = _workspace(_lib.OP_MULTINOMIAL_IID, seg, dt, w.device, workspace)
    rc = _lib.load().resample_multinomial_iid(_ptr(w), dt, ctypes.byref(seg),
                                              _rng(seed, offset, filter_base), _ptr(a), _ptr(ws),
                                              0 if ws is None else ws.numel(), _ptr(flags),
                                              _stream())
    _lib.check(rc, "resample_multinomial_iid")
    return a


def resample_stratified(w, seed=0, offset=0, filter_base=0, precision=SCAN_EXACT, offsets=None,
                        max_len=None, out=None, flags=None, workspace=None):
    """Stratified ancestry (Code 7 + Code 11)."""
    return _collective("resample_stratified", _lib.OP_STRATIFIED, w, seed, offset, filter_base,
                       precision, offsets, max_len, out, flags, workspace)


def resample_systematic(w, seed=0, offset=0, filter_base=0, precision=SCAN_EXACT, offsets=None,
                        max_len=None, out=None, flags=None, workspace=None):
    """Systematic ancestry (Code 8 + Code 11)."""
    return _collective("resample_systematic", _lib.OP_SYSTEMATIC, w, seed, offset, filter_base,
                       precision, offsets, max_len, out, flags, workspace)


def resample_metropolis(w, B, seed=0, offset=0, filter_base=0, B_per_filter=None, offsets=None,
                        max_len=None, out=None, workspace=None):
    """Metropolis ancestry (Code 2), B steps per lane (or B_per_filter[f])."""
    _require_cuda(w, B_per_filter)
    dt = _dtype_code(w)
    seg = _segments(w.numel(), offsets, max_len)
    _per_segment(B_per_filter, "int32", seg, "B_per_filter")
    a = _out_like(w.numel(), w.device, out)
    ws, _ = _workspace(_lib.OP_METROPOLIS, seg, dt, w.device, workspace)
    rc = _lib.load().resample_metropolis(_ptr(w), dt, ctypes.byref(seg), int(B),
                                         _ptr(B_per_filter), _rng(seed, offset, filter_base),
                                         _ptr(a), _ptr(ws), 0 if ws is None else ws.numel(),
                                         _stream())
    _lib.check(rc, "resample_metropolis")
    return a


def resample_rejection(w, w_max, seed=0, offset=0, filter_base=0, max_trials=1 << 20,
                       w_max_per_filter=None, offsets=None, max_len=None, out=None, flags=None,
                       workspace=None):
    """Rejection ancestry (Code 3) with first proposal j = i and bound w_max."""
    _require_cuda(w, w_max_per_filter, flags)
    dt = _dtype_code(w)
    seg = _segments(w.numel(), offsets, max_len)
    _per_segment(w_max_per_filter, "float64", seg, "w_max_per_filter")
    a = _out_like(w.numel(), w.device, out)
    ws, _ = _workspace(_lib.OP_REJECTION, seg, dt, w.device, workspace)
    rc = _lib.load().resample_rejection(_ptr(w), dt, ctypes.byref(seg), float(w_max),
                                        _ptr(w_max_per_filter), int(max_trials),
                                        _rng(seed, offset, filter_base), _ptr(a), _ptr(ws),
                                        0 if ws is None else ws.numel(), _ptr(flags),
                                        _stream())
    _lib.check(rc, "resample_rejection")
    return a


def resample_partial_rejection(w, v_max, seed=0, offset=0, filter_base=0, max_trials=1 << 20,
                               v_max_per_filter=None, offsets=None, max_len=None, out=None,
                               weights_out=None, flags=None, workspace=None):
    """Partial rejection control: rejection ancestry on min(w, v_max) with
    bound v_max and the importance weights w_{a_i} / min(w_{a_i}, v_max).
    Returns (ancestors, weights)."""
    torch = _torch()
    _require_cuda(w, v_max_per_filter, flags, weights_out)
    dt = _dtype_code(w)
    seg = _segments(w.numel(), offsets, max_len)
    _per_segment(v_max_per_filter, "float64", seg, "v_max_per_filter")
    a = _out_like(w.numel(), w.device, out)
    if weights_out is None:
        weights_out = torch.empty_like(w)
    elif weights_out.dtype != w.dtype or weights_out.numel() != w.numel():
        raise ValueError("weights_out must match the weights' type and size")
    ws, _ = _workspace(_lib.OP_REJECTION, seg, dt, w.device, workspace)
    rc = _lib.load().resample_partial_rejection(_ptr(w), dt, ctypes.byref(seg), float(v_max),
                                                _ptr(v_max_per_filter), int(max_trials),
                                                _rng(seed, offset, filter_base), _ptr(a),
                                                _ptr(weights_out), _ptr(ws),
                                                0 if ws is None else ws.numel(), _ptr(flags),
                                                _stream())
    _lib.check(rc, "resample_partial_rejection")
    return a, weights_out


def resample_permuted(scheme, w, seed=0, offset=0, filter_base=0, precision=SCAN_EXACT, B=0,
                      B_per_filter=None, w_max=1.0, w_max_per_filter=None, max_trials=1 << 20,
                      offsets=None, max_len=None, out=None, permuted=None, flags=None,
                      workspace=None):
    """Resample and permute in one call (Prepermute fused into the resampler
    for long single vectors).  scheme: "multinomial", "stratified",
    "systematic", "metropolis" or "rejection".  Returns (ancestors, permuted),
    the same bits as resample_<scheme> followed by permute_ancestors."""
    _require_cuda(w, B_per_filter, w_max_per_filter, flags)
    op = _SCHEME_OPS[scheme]
    dt = _dtype_code(w)
    seg = _segments(w.numel(), offsets, max_len)
    _per_segment(B_per_filter, "int32", seg, "B_per_filter")
    _per_segment(w_max_per_filter, "float64", seg, "w_max_per_filter")
    a = _out_like(w.numel(), w.device, out)
    c = _out_like(w.numel(), w.device, permuted)
    lib = _lib.load()
    need = int(lib.pfr_resample_permuted_workspace_bytes(op, ctypes.byref(seg), dt))
    if workspace is None:
        key = (str(w.device), _stream_key(), "permuted", op, need)
        workspace = _WS_CACHE.get(key)
        if workspace is None:
            workspace = new_workspace(need, w.device)
            _WS_CACHE.put(key, workspace)
    params = _lib.SchemeParams(int(precision), int(B), None if B_per_filter is None
                               else B_per_filter.data_ptr(), float(w_max),
                               None if w_max_per_filter is None else w_max_per_filter.data_ptr(),
                               int(max_trials))
    rc = lib.resample_permuted(op, _ptr(w), dt, ctypes.byref(seg), ctypes.byref(params),
                               _rng(seed, offset, filter_base), _ptr(a), _ptr(c), _ptr(workspace),
                               workspace.numel(), _ptr(flags), _stream())
    _lib.check(rc, "resample_permuted")
    return a, c


def offspring_to_ancestors(o, offsets=None, max_len=None, out=None, flags=None, workspace=None):
    """Ancestors from int32 offspring counts (Code 11 after a prefix sum)."""
    torch = _torch()
    _require_cuda(o, flags)
    if o.dtype != torch.int32:
        raise TypeError("offspring must be int32")
    seg = _segments(o.numel(), offsets, max_len)
    a = _out_like(o.numel(), o.device, out)
    ws, _ = _workspace(_lib.OP_OFFSPRING_TO_ANCESTORS, seg, 0, o.device, workspace)
    rc = _lib.load().offspring_to_ancestors(_ptr(o), ctypes.byref(seg), _ptr(a), _ptr(ws),
                                            0 if ws is None else ws.numel(), _ptr(flags),
                                            _stream())
    _lib.check(rc, "offspring_to_ancestors")
    return a


def permute_ancestors(a, sorted_hint=False, offsets=None, max_len=None, out=None, flags=None,
                      workspace=None):
    """Permutation of an ancestry for in-place propagation (Code 10)."""
    torch = _torch()
    _require_cuda(a, flags)
    if a.dtype != torch.int32:
        raise TypeError("ancestors must be int32")
    seg = _segments(a.numel(), offsets, max_len)
    c = _out_like(a.numel(), a.device, out)
    ws, _ = _workspace(_lib.OP_PERMUTE, seg, 0, a.device, workspace)
    rc = _lib.load().permute_ancestors(_ptr(a), ctypes.byref(seg), 1 if sorted_hint else 0,
                                       _ptr(c), _ptr(ws), 0 if ws is None else ws.numel(),
                                       _ptr(flags), _stream())
    _lib.check(rc, "permute_ancestors")
    return c


def permute_ancestors_noalloc(a, sorted_hint=False, offsets=None, max_len=None, out=None,
                              flags=None):
    """permute_ancestors with the library's static device scratch instead of a
    workspace (at most NOALLOC_MAX_N particles).  The call itself allocates
    nothing on the device when `out` is given."""
    torch = _torch()
    _require_cuda(a, flags)
    if a.dtype != torch.int32:
        raise TypeError("ancestors must be int32")
    seg = _segments(a.numel(), offsets, max_len)
    c = _out_like(a.numel(), a.device, out)
    rc = _lib.load().permute_ancestors_noalloc(_ptr(a), ctypes.byref(seg),
                                               1 if sorted_hint else 0, _ptr(c), _ptr(flags),
                                               _stream())
    _lib.check(rc, "permute_ancestors_noalloc")
    return c


def scaled_prefix(w, precision=SCAN_EXACT, out=None, flags=None, workspace=None):
    """The scaled prefix r_i = n W_i / W_n (float64) a collective resampler
    of this single vector compares against in the given precision mode."""
    torch = _torch()
    _require_cuda(w, flags)
    dt = _dtype_code(w)
    seg = _segments(w.numel())
    r = out if out is not None else torch.empty(w.numel(), dtype=torch.float64, device=w.device)
    if r.dtype != torch.float64 or r.numel() != w.numel():
        raise ValueError("out must be a float64 tensor with one entry per particle")
    _require_cuda(r)
    ws, _ = _workspace(_lib.OP_SCALED_PREFIX, seg, dt, w.device, workspace)
    rc = _lib.load().pfr_scaled_prefix(_ptr(w), dt, ctypes.byref(seg), int(precision), _ptr(r),
                                       _ptr(ws), 0 if ws is None else ws.numel(), _ptr(flags),
                                       _stream())
    _lib.check(rc, "pfr_scaled_prefix")
    return r


def ancestors_to_offspring(a, sorted_hint=False, offsets=None, max_len=None, out=None,
                           flags=None):
    """Offspring counts o_j = #{i : a_i = j} (Code 12); atomic-free when
    sorted_hint says the ancestry is non-decreasing."""
    torch = _torch()
    _require_cuda(a, flags)
    if a.dtype != torch.int32:
        raise TypeError("ancestors must be int32")
    seg = _segments(a.numel(), offsets, max_len)
    o = _out_like(a.numel(), a.device, out)
    rc = _lib.load().ancestors_to_offspring(_ptr(a), ctypes.byref(seg), 1 if sorted_hint else 0,
                                            _ptr(o), _ptr(flags), _stream())
    _lib.check(rc, "ancestors_to_offspring")
    return o


def effective_sample_size(w, offsets=None, max_len=None, out=None, flags=None, workspace=None):
    """ESS (sum w)^2 / w^T w per segment (section 3.4) -> float64 [n_filters]."""
    torch = _torch()
    _require_cuda(w, flags, out)
    dt = _dtype_code(w)
    seg = _segments(w.numel(), offsets, max_len)
    nf = seg.n_filters
    if out is None:
        out = torch.empty(nf, dtype=torch.float64, device=w.device)
    elif out.dtype != torch.float64 or out.numel() != nf:
        raise ValueError("out must be a float64 tensor with one entry per segment")
    ws, _ = _workspace(_lib.OP_ESS, seg, dt, w.device, workspace)
    rc = _lib.load().effective_sample_size(_ptr(w), dt, ctypes.byref(seg), _ptr(out), _ptr(ws),
                                           0 if ws is None else ws.numel(), _ptr(flags),
                                           _stream())
    _lib.check(rc, "effective_sample_size")
    return out


def copy_particles(c, x, offsets=None, max_len=None, flags=None):
    """In-place copy step x_i <- x_{c_i} for c_i != i (section 2.3).

    x has one row per particle, shape (n,) or (n, D), with any strides that
    keep either the rows or the columns contiguous (an (n, D) tensor, or the
    transpose of a (D, n) one)."""
    torch = _torch()
    _require_cuda(c, flags)
    if c.dtype != torch.int32:
        raise TypeError("permuted ancestors must be int32")
    if not x.is_cuda or x.dim() not in (1, 2) or x.shape[0] != c.numel():
        raise ValueError("x must be a GPU tensor with one row per particle")
    dim = 1 if x.dim() == 1 else x.shape[1]
    ps = x.stride(0)
    cs = 1 if x.dim() == 1 else x.stride(1)
    seg = _segments(c.numel(), offsets, max_len)
    rc = _lib.load().copy_particles(_ptr(c), ctypes.byref(seg), _ptr(x), x.element_size(),
                                    int(dim), int(ps), int(cs), _ptr(flags), _stream())
    _lib.check(rc, "copy_particles")
    return x


_SCHEME_OPS = {"multinomial": _lib.OP_MULTINOMIAL, "stratified": _lib.OP_STRATIFIED,
               "systematic": _lib.OP_SYSTEMATIC, "metropolis": _lib.OP_METROPOLIS,
               "rejection": _lib.OP_REJECTION}


class LGSSMFilter:
    """Batched bootstrap particle filter on the 1-D linear-Gaussian model
    x_t = phi x_{t-1} + q e_t, y_t = x_t + r v_t (lgssm_* in the C header).

    Holds the device state of n_filters filters of n particles: x, w (float32),
    log_z (float64 per filter), the Metropolis step counts B and the device
    step counter t.  `run` initialises and then advances T steps, replaying one
    captured graph of a step by default.
    """

    def __init__(self, y, n_filters, n, phi=0.9, q=1.0, r=0.5, s0=None, scheme="systematic",
                 precision=SCAN_EXACT, seed=0, offset=0, filter_base=0, device="cuda"):
        import math
        torch = _torch()
        if s0 is None:  # stationary prior of the state
            s0 = q / math.sqrt(1.0 - phi * phi)
        self.model = _lib.LGSSM(float(phi), float(q), float(r), float(s0))
        self.y = torch.as_tensor(y, dtype=torch.float64).to(device).contiguous()
        self.T = int(self.y.numel())
        self.F, self.n = int(n_filters), int(n)
        total = self.F * self.n
        self.x = torch.empty(total, dtype=torch.float32, device=device)
        self.w = torch.empty(total, dtype=torch.float32, device=device)
        self.log_z = torch.zeros(self.F, dtype=torch.float64, device=device)
        self.B = torch.zeros(self.F, dtype=torch.int32, device=device)
        self.t = torch.zeros(1, dtype=torch.int32, device=device)
        self.ancestors = torch.empty(total, dtype=torch.int32, device=device)
        self.permuted = torch.empty(total, dtype=torch.int32, device=device)
        self.flags = torch.zeros(1, dtype=torch.int32, device=device)
        nbytes = int(_lib.load().lgssm_workspace_bytes(self.F, self.n))
        if nbytes == 0:
            raise ValueError("invalid filter size")
        self.ws = new_workspace(nbytes, device)
        self.scheme = _SCHEME_OPS[scheme]
        self.precision = int(precision)
        self.rng = _rng(seed, offset, filter_base)
        self.graph = None

    def reset(self):
        rc = _lib.load().lgssm_init(ctypes.byref(self.model), self.F, self.n, self.rng,
                                    _ptr(self.x), _ptr(self.w), _ptr(self.log_z), _ptr(self.B),
                                    _ptr(self.t), _ptr(self.ws), self.ws.numel(), _stream())
        _lib.check(rc, "lgssm_init")

    def step(self):
        rc = _lib.load().lgssm_step(ctypes.byref(self.model), self.scheme, self.precision, self.F,
                                    self.n, _ptr(self.y), self.T, _ptr(self.t), self.rng,
                                    _ptr(self.x), _ptr(self.w), _ptr(self.log_z), _ptr(self.B),
                                    _ptr(self.ancestors), _ptr(self.permuted), _ptr(self.ws),
                                    self.ws.numel(), _ptr(self.flags), _stream())
        _lib.check(rc, "lgssm_step")

    def capture(self):
        """Capture one step in a HIP graph (every step argument is read on the device)."""
        torch = _torch()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g

    def run(self, T=None, graph=True):
        """reset() and T steps (default: all observations); returns log_z."""
        T = self.T if T is None else int(T)
        self.reset()
        if graph:
            if self.graph is None:
                _torch().cuda.synchronize()
                self.capture()
            for _ in range(T):
                self.graph.replay()
        else:
            for _ in range(T):
                self.step()
        return self.log_z
