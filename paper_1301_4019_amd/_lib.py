"""ctypes binding of libpfresample.so (argument marshalling only).

Every entry point mirrors a C function of include/pfresample.h; tensors are
torch device tensors, passed as raw device pointers together with the current
HIP stream.  All arithmetic runs in the library's HIP kernels: if the shared
library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfresample.so")

PFR_OK, PFR_EINVAL, PFR_EWORKSPACE, PFR_ELAUNCH, PFR_ENOTSUP, PFR_ETOOBIG = range(6)
PFR_F32, PFR_F64 = 0, 1
SCAN_EXACT, SCAN_F64, SCAN_COMP_F32, SCAN_NAIVE_F32 = 0, 1, 2, 3
(OP_MULTINOMIAL, OP_STRATIFIED, OP_SYSTEMATIC, OP_METROPOLIS, OP_REJECTION,
 OP_OFFSPRING_TO_ANCESTORS, OP_PERMUTE, OP_ANCESTORS_TO_OFFSPRING, OP_ESS,
 OP_MULTINOMIAL_IID, OP_SCALED_PREFIX) = range(11)

FLAG_ZERO_TOTAL = 1
FLAG_TRIAL_CAP = 2
FLAG_BAD_COUNTS = 4
FLAG_BAD_WEIGHTS = 8
FLAG_BAD_ANCESTOR = 16
FLAG_BAD_STEP = 32
FLAG_WMAX_BELOW = 64
FLAG_NOT_SORTED = 128
MAX_BATCH_SEGMENT = 256 * 1024 - 1
NOALLOC_MAX_N = 1 << 22

EXPORTS = (
    "pfr_workspace_bytes", "pfr_workspace_init", "pfr_scaled_prefix", "resample_multinomial",
    "resample_multinomial_iid", "resample_stratified",
    "resample_systematic", "resample_metropolis", "resample_rejection",
    "resample_partial_rejection", "offspring_to_ancestors",
    "permute_ancestors", "permute_ancestors_noalloc", "ancestors_to_offspring", "effective_sample_size", "copy_particles",
    "pfr_resample_permuted_workspace_bytes", "resample_permuted",
    "lgssm_workspace_bytes", "lgssm_init", "lgssm_step",
    "pfr_tuning_defaults", "pfr_get_tuning", "pfr_set_tuning", "pfr_load_tuning",
    "pfr_status_string", "pfr_version", "pfr_philox_rounds",
    "pfr_set_checks", "pfr_get_checks", "pfr_take_check_flags",
)

TUNING_VERSION = 2
# tuning chosen for this machine by autotune.py; PFR_TUNING overrides the path
TUNING_PATH = os.environ.get("PFR_TUNING", os.path.join(HERE, "tuning.json"))


class SchemeParams(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("B", ctypes.c_int32),
                ("B_dev", ctypes.c_void_p), ("w_max", ctypes.c_double),
                ("w_max_dev", ctypes.c_void_p), ("max_trials", ctypes.c_uint32)]


class Segments(ctypes.Structure):
    _fields_ = [("n_total", ctypes.c_int64), ("n_filters", ctypes.c_int32),
                ("offsets", ctypes.c_void_p), ("max_len", ctypes.c_int64)]


class Rng(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("offset", ctypes.c_uint32),
                ("filter_base", ctypes.c_uint32), ("offset_dev", ctypes.c_void_p)]


class LGSSM(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_double), ("q", ctypes.c_double), ("r", ctypes.c_double),
                ("s0", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("single_wg_max", ctypes.c_int32),
                ("direct_max_blocks", ctypes.c_int32),
                ("metropolis_table_min_B", ctypes.c_int32),
                ("rejection_table", ctypes.c_int32), ("rejection_per_wave", ctypes.c_int32),
                ("metropolis_chunk", ctypes.c_int32),
                ("batch_scan_wg_max_len", ctypes.c_int32), ("batch_stage_max_kb", ctypes.c_int32),
                ("batch_metropolis_chunk", ctypes.c_int32),
                ("batch_rejection_per_wave", ctypes.c_int32),
                ("batch_permute_lds_max", ctypes.c_int32)]


class PfrError(RuntimeError):
    pass


_lib = None


def open_library(path: str) -> ctypes.CDLL:
    """Open a build of the library, declare every signature and load the
    tuning file into it."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1301_4019_amd.build`")
    lib = ctypes.CDLL(path)
    P, I, U32, I32, D, SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_int32,
                             ctypes.c_double, ctypes.c_size_t)
    SEG = ctypes.POINTER(Segments)
    MODEL = ctypes.POINTER(LGSSM)
    sigs = {
        "pfr_workspace_bytes": (SZ, [I, SEG, I]),
        "pfr_workspace_init": (I, [P, SZ, P]),
        "pfr_scaled_prefix": (I, [P, I, SEG, I, P, P, SZ, P, P]),
        "resample_multinomial": (I, [P, I, SEG, I, Rng, P, P, SZ, P, P]),
        "resample_multinomial_iid": (I, [P, I, SEG, Rng, P, P, SZ, P, P]),
        "resample_stratified": (I, [P, I, SEG, I, Rng, P, P, SZ, P, P]),
        "resample_systematic": (I, [P, I, SEG, I, Rng, P, P, SZ, P, P]),
        "resample_metropolis": (I, [P, I, SEG, I32, P, Rng, P, P, SZ, P]),
        "resample_rejection": (I, [P, I, SEG, D, P, U32, Rng, P, P, SZ, P, P]),
        "resample_partial_rejection": (I, [P, I, SEG, D, P, U32, Rng, P, P, P, SZ, P, P]),
        "offspring_to_ancestors": (I, [P, SEG, P, P, SZ, P, P]),
        "permute_ancestors": (I, [P, SEG, I32, P, P, SZ, P, P]),
        "permute_ancestors_noalloc": (I, [P, SEG, I32, P, P, P]),
        "pfr_resample_permuted_workspace_bytes": (SZ, [I, SEG, I]),
        "resample_permuted": (I, [I, P, I, SEG, ctypes.POINTER(SchemeParams), Rng, P, P, P, SZ,
                                  P, P]),
        "ancestors_to_offspring": (I, [P, SEG, I32, P, P, P]),
        "effective_sample_size": (I, [P, I, SEG, P, P, SZ, P, P]),
        "copy_particles": (I, [P, SEG, P, SZ, I32, ctypes.c_int64, ctypes.c_int64, P, P]),
        "lgssm_workspace_bytes": (SZ, [I32, I32]),
        "lgssm_init": (I, [MODEL, I32, I32, Rng, P, P, P, P, P, P, SZ, P]),
        "lgssm_step": (I, [MODEL, I, I, I32, I32, P, I32, P, Rng, P, P, P, P, P, P, P, SZ, P,
                           P]),
        "pfr_tuning_defaults": (None, [ctypes.POINTER(Tuning)]),
        "pfr_get_tuning": (I, [ctypes.POINTER(Tuning)]),
        "pfr_set_tuning": (I, [ctypes.POINTER(Tuning)]),
        "pfr_load_tuning": (I, [ctypes.c_char_p]),
        "pfr_status_string": (ctypes.c_char_p, [I]),
        "pfr_version": (ctypes.c_char_p, []),
        "pfr_philox_rounds": (I, []),
        "pfr_set_checks": (I, [I32]),
        "pfr_get_checks": (I32, []),
        "pfr_take_check_flags": (I, [P, ctypes.POINTER(ctypes.c_uint32)]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    load_tuning_file(lib, TUNING_PATH)
    return lib


def _device_arch():
    """ISA name of GPU 0 (e.g. gfx950), or None without a GPU."""
    try:
        import torch
        if not torch.cuda.is_available():
            return None
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return None


def load_tuning_file(lib, path):
    """Apply the tuning file written by autotune.py if it was tuned for this
    GPU's architecture and this library's tuning version; otherwise keep the
    library's defaults (a file for another GPU would only mislead)."""
    import json
    import sys
    if not os.path.exists(path):
        return False
    with open(path) as f:
        doc = json.load(f)
    arch = _device_arch()
    if doc.get("version") != TUNING_VERSION or (arch and doc.get("arch") not in (None, arch)):
        print(f"libpfresample: {path} was tuned for {doc.get('arch')} (version "
              f"{doc.get('version')}); keeping the defaults", file=sys.stderr)
        return False
    t = Tuning()
    lib.pfr_get_tuning(ctypes.byref(t))
    for name, _ in Tuning._fields_:
        if name in doc and name != "version":
            setattr(t, name, int(doc[name]))
    t.version = TUNING_VERSION
    rc = lib.pfr_set_tuning(ctypes.byref(t))
    if rc != PFR_OK:
        raise PfrError(f"invalid tuning file {path} (status {rc})")
    return True


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """The library every binding call goes through (opened once)."""
    global _lib
    if _lib is None:
        _lib = open_library(path)
    return _lib


class use_library:
    """Context manager: route the binding through another build of the
    library (the Philox round-count study's variant), then back."""

    def __init__(self, path: str):
        self.path = path
        self.saved = None

    def __enter__(self):
        global _lib
        self.saved = load()
        _lib = open_library(self.path)
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def check(rc: int, what: str) -> None:
    if rc != PFR_OK:
        msg = load().pfr_status_string(rc).decode()
        raise PfrError(f"{what}: {msg} (status {rc})")
