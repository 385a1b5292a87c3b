"""Host-side checks of libpfresample: it loads without a GPU, exports every
entry point include/pfresample.h declares, and rejects invalid arguments
before enqueuing any work (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_1301_4019_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfresample.h")


def declared_functions():
    src = open(HEADER).read()
    return re.findall(r"PFR_API\s+[\w\s\*]+?\b(\w+)\s*\(", src)


def test_header_declares_the_entry_points():
    names = set(declared_functions())
    assert names == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.pfr_version().decode().count(".") == 2
    assert lib.pfr_status_string(_lib.PFR_EINVAL).decode() == "invalid argument"


def seg(n, nf=1, offsets=None, max_len=0):
    return _lib.Segments(n, nf, offsets, max_len)


def test_workspace_sizes():
    lib = _lib.load()
    s_small = seg(1024)
    s_big = seg(1 << 20)
    # small single vectors run in one workgroup without workspace
    assert lib.pfr_workspace_bytes(_lib.OP_STRATIFIED, ctypes.byref(s_small), 0) == 0
    big = lib.pfr_workspace_bytes(_lib.OP_STRATIFIED, ctypes.byref(s_big), 0)
    multi = lib.pfr_workspace_bytes(_lib.OP_MULTINOMIAL, ctypes.byref(s_big), 0)
    assert big > 0 and multi > big and big % 256 == 0
    # a 16-byte record per 1024-weight block and a 32-byte prefix per 4096-particle tile
    assert big >= 256 + 1024 * 16 + 256 * 32
    # Metropolis / rejection: optional bound table for a long single vector
    # (2^18 buckets of 4 particles: one code byte each plus per-workgroup maxima)
    tab = lib.pfr_workspace_bytes(_lib.OP_METROPOLIS, ctypes.byref(s_big), 0)
    assert tab >= (1 << 18) and tab % 256 == 0
    assert lib.pfr_workspace_bytes(_lib.OP_METROPOLIS, ctypes.byref(s_small), 0) == 0
    assert lib.pfr_workspace_bytes(_lib.OP_PERMUTE, ctypes.byref(s_big), 0) >= 4 << 20
    assert lib.pfr_workspace_bytes(_lib.OP_OFFSPRING_TO_ANCESTORS, ctypes.byref(s_big), 0) >= 256 + 256 * 8
    assert lib.pfr_workspace_bytes(_lib.OP_REJECTION, ctypes.byref(s_big), 0) == tab
    # ESS: a 32-byte partial per 4096-weight chunk (plus one per segment)
    ess_big = lib.pfr_workspace_bytes(_lib.OP_ESS, ctypes.byref(s_big), 0)
    assert ess_big >= 256 * 32 and ess_big % 256 == 0
    assert lib.pfr_workspace_bytes(_lib.OP_ESS, ctypes.byref(seg(0)), 0) > 0
    assert lib.pfr_workspace_bytes(_lib.OP_ANCESTORS_TO_OFFSPRING, ctypes.byref(s_big), 0) == 0


def test_auxiliary_arguments_rejected_on_host():
    lib = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    out = ctypes.c_void_p(0x10000 + (1 << 30))
    ws = ctypes.c_void_p(0x10000 + (2 << 30))
    # Code 12: output aliases input, null pointers, batch without offsets
    assert lib.ancestors_to_offspring(fake, ctypes.byref(seg(10)), 1, fake, None,
                                      None) == _lib.PFR_EINVAL
    assert lib.ancestors_to_offspring(None, ctypes.byref(seg(10)), 0, out, None,
                                      None) == _lib.PFR_EINVAL
    assert lib.ancestors_to_offspring(fake, ctypes.byref(seg(10, 3, None)), 0, out, None,
                                      None) == _lib.PFR_EINVAL
    # ESS: workspace missing or small, null output, unknown dtype
    assert lib.effective_sample_size(fake, 0, ctypes.byref(seg(10)), out, None, 0, None,
                                     None) == _lib.PFR_EWORKSPACE
    assert lib.effective_sample_size(fake, 0, ctypes.byref(seg(1 << 20)), out, ws, 256, None,
                                     None) == _lib.PFR_EWORKSPACE
    assert lib.effective_sample_size(fake, 0, ctypes.byref(seg(10)), None, ws, 1 << 20, None,
                                     None) == _lib.PFR_EINVAL
    assert lib.effective_sample_size(fake, 5, ctypes.byref(seg(10)), out, ws, 1 << 20, None,
                                     None) == _lib.PFR_EINVAL
    # copy: element size, strides that alias elements, misaligned state
    I64 = ctypes.c_int64
    assert lib.copy_particles(fake, ctypes.byref(seg(10)), out, 3, 1, I64(1), I64(1), None,
                              None) == _lib.PFR_EINVAL
    assert lib.copy_particles(fake, ctypes.byref(seg(10)), out, 4, 4, I64(2), I64(1), None,
                              None) == _lib.PFR_EINVAL
    assert lib.copy_particles(fake, ctypes.byref(seg(10)), out, 4, 2, I64(1), I64(5), None,
                              None) == _lib.PFR_EINVAL
    assert lib.copy_particles(fake, ctypes.byref(seg(10)), out, 4, 0, I64(1), I64(1), None,
                              None) == _lib.PFR_EINVAL
    assert lib.copy_particles(fake, ctypes.byref(seg(10)), ctypes.c_void_p(0x10000 + (1 << 30) + 2),
                              4, 1, I64(1), I64(1), None, None) == _lib.PFR_EINVAL
    # the state overlaps the permutation
    assert lib.copy_particles(fake, ctypes.byref(seg(10)), fake, 4, 1, I64(1), I64(1), None,
                              None) == _lib.PFR_EINVAL
    # partial rejection control: no weight output, weight output aliasing the ancestry
    rng = _lib.Rng(0, 0, 0)
    assert lib.resample_partial_rejection(fake, 0, ctypes.byref(seg(10)), 1.0, None, 16, rng, out,
                                          None, None, 0, None, None) == _lib.PFR_EINVAL
    assert lib.resample_partial_rejection(fake, 0, ctypes.byref(seg(10)), 1.0, None, 16, rng, out,
                                          out, None, 0, None, None) == _lib.PFR_EINVAL
    assert lib.resample_partial_rejection(fake, 0, ctypes.byref(seg(10)), 0.0, None, 16, rng, out,
                                          ws, None, 0, None, None) == _lib.PFR_EINVAL
    # Code 5 with independent uniforms: single vectors only, workspace required
    assert lib.resample_multinomial_iid(fake, 0, ctypes.byref(seg(100, 3, fake)), rng, out, ws,
                                        1 << 20, None, None) == _lib.PFR_ENOTSUP
    assert lib.resample_multinomial_iid(fake, 0, ctypes.byref(seg(100)), rng, out, None, 0, None,
                                        None) == _lib.PFR_EWORKSPACE
    small = lib.pfr_workspace_bytes(_lib.OP_MULTINOMIAL_IID, ctypes.byref(seg(1 << 20)), 0)
    assert small >= 8 << 20
    assert lib.resample_multinomial_iid(fake, 0, ctypes.byref(seg(1 << 20)), rng, out, ws,
                                        small - 256, None, None) == _lib.PFR_EWORKSPACE
    # resample_permuted: no parameters, unknown scheme, no workspace, outputs aliasing
    prm = _lib.SchemeParams(0, 4, None, 1.0, None, 16)
    assert lib.resample_permuted(_lib.OP_SYSTEMATIC, fake, 0, ctypes.byref(seg(10)), None, rng,
                                 out, ws, ws, 1 << 20, None, None) == _lib.PFR_EINVAL
    assert lib.resample_permuted(_lib.OP_PERMUTE, fake, 0, ctypes.byref(seg(10)),
                                 ctypes.byref(prm), rng, out, ws, ws, 1 << 20, None,
                                 None) == _lib.PFR_EINVAL
    perm_out = ctypes.c_void_p(0x10000 + (3 << 30))
    assert lib.resample_permuted(_lib.OP_SYSTEMATIC, fake, 0, ctypes.byref(seg(1 << 20)),
                                 ctypes.byref(prm), rng, out, perm_out, None, 0, None,
                                 None) == _lib.PFR_EWORKSPACE
    assert lib.resample_permuted(_lib.OP_METROPOLIS, fake, 0, ctypes.byref(seg(10)),
                                 ctypes.byref(prm), rng, out, out, ws, 1 << 20, None,
                                 None) == _lib.PFR_EINVAL
    need = lib.pfr_resample_permuted_workspace_bytes(_lib.OP_SYSTEMATIC, ctypes.byref(seg(1 << 20)), 0)
    assert need >= lib.pfr_workspace_bytes(_lib.OP_PERMUTE, ctypes.byref(seg(1 << 20)), 0) + \
        lib.pfr_workspace_bytes(_lib.OP_SYSTEMATIC, ctypes.byref(seg(1 << 20)), 0)
    assert ctypes.sizeof(_lib.SchemeParams) == 40
    # the no-allocation permutation: aliasing, null output, input beyond its
    # static scratch (rejected before any GPU call)
    assert lib.permute_ancestors_noalloc(fake, ctypes.byref(seg(10)), 1, fake, None,
                                         None) == _lib.PFR_EINVAL
    assert lib.permute_ancestors_noalloc(fake, ctypes.byref(seg(10)), 0, None, None,
                                         None) == _lib.PFR_EINVAL
    assert lib.permute_ancestors_noalloc(fake, ctypes.byref(seg(_lib.NOALLOC_MAX_N + 1)), 0, out,
                                         None, None) == _lib.PFR_ETOOBIG
    assert lib.permute_ancestors_noalloc(None, ctypes.byref(seg(0)), 0, None, None,
                                         None) == _lib.PFR_OK
    assert b"static scratch" in lib.pfr_status_string(_lib.PFR_ETOOBIG)
    # empty input is a no-op
    assert lib.copy_particles(None, ctypes.byref(seg(0)), None, 4, 3, I64(3), I64(1), None,
                              None) == _lib.PFR_OK
    assert lib.ancestors_to_offspring(None, ctypes.byref(seg(0)), 1, None, None,
                                      None) == _lib.PFR_OK


def test_invalid_arguments_rejected_on_host():
    lib = _lib.load()
    rng = _lib.Rng(0, 0, 0)
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: every call below fails validation
    # negative size
    assert lib.resample_stratified(fake, 0, ctypes.byref(seg(-1)), 0, rng, fake, None, 0, None,
                                   None) == _lib.PFR_EINVAL
    # too large
    assert lib.resample_systematic(fake, 0, ctypes.byref(seg(1 << 31)), 0, rng, fake, None, 0,
                                   None, None) == _lib.PFR_EINVAL
    # unknown dtype
    assert lib.resample_multinomial(fake, 7, ctypes.byref(seg(10)), 0, rng, fake, None, 0, None,
                                    None) == _lib.PFR_EINVAL
    # null weights
    assert lib.resample_stratified(None, 0, ctypes.byref(seg(10)), 0, rng, fake, None, 0, None,
                                   None) == _lib.PFR_EINVAL
    # output aliases input
    assert lib.resample_stratified(fake, 0, ctypes.byref(seg(10)), 0, rng, fake, None, 0, None,
                                   None) == _lib.PFR_EINVAL
    # a large single vector needs a workspace
    out = ctypes.c_void_p(0x10000 + (1 << 30))
    assert lib.resample_stratified(fake, 0, ctypes.byref(seg(1 << 20)), 0, rng, out, None, 0,
                                   None, None) == _lib.PFR_EWORKSPACE
    # batched without offsets
    assert lib.resample_stratified(fake, 0, ctypes.byref(seg(100, 4, None)), 0, rng, out, None,
                                   0, None, None) == _lib.PFR_EINVAL
    # Metropolis step count out of range
    assert lib.resample_metropolis(fake, 0, ctypes.byref(seg(10)), -1, None, rng, out, None, 0,
                                   None) == _lib.PFR_EINVAL
    # rejection: bad bound, zero trials
    assert lib.resample_rejection(fake, 0, ctypes.byref(seg(10)), 0.0, None, 16, rng, out, None,
                                  0, None, None) == _lib.PFR_EINVAL
    assert lib.resample_rejection(fake, 0, ctypes.byref(seg(10)), 1.0, None, 0, rng, out, None,
                                  0, None, None) == _lib.PFR_EINVAL
    # misaligned optional workspace
    assert lib.resample_metropolis(fake, 0, ctypes.byref(seg(1 << 20)), 4, None, rng, out,
                                   ctypes.c_void_p(0x10008), 1 << 20, None) == _lib.PFR_EWORKSPACE
    # permute: output aliases input; workspace missing
    assert lib.permute_ancestors(fake, ctypes.byref(seg(10)), 1, fake, out, 1 << 20, None,
                                 None) == _lib.PFR_EINVAL
    assert lib.permute_ancestors(fake, ctypes.byref(seg(10)), 1, out, None, 0, None,
                                 None) == _lib.PFR_EWORKSPACE
    # empty input is a no-op
    assert lib.resample_stratified(None, 0, ctypes.byref(seg(0)), 0, rng, None, None, 0, None,
                                   None) == _lib.PFR_OK
    # unknown precision mode
    assert lib.resample_stratified(fake, 0, ctypes.byref(seg(10)), 4, rng, out, None, 0, None,
                                   None) == _lib.PFR_EINVAL
    assert lib.resample_stratified(fake, 0, ctypes.byref(seg(10)), -1, rng, out, None, 0, None,
                                   None) == _lib.PFR_EINVAL


def test_tuning_set_get_load_roundtrip(tmp_path):
    import paper_1301_4019_amd as pfr
    saved = pfr.get_tuning()
    try:
        d = pfr.default_tuning()
        assert d["single_wg_max"] > 0 and d["rejection_per_wave"] >= 64
        pfr.set_tuning(rejection_per_wave=512, metropolis_chunk=1024, direct_max_blocks=0)
        t = pfr.get_tuning()
        assert (t["rejection_per_wave"], t["metropolis_chunk"], t["direct_max_blocks"]) == (512, 1024, 0)
        # out-of-range values leave everything unchanged
        for bad in ({"rejection_per_wave": 32}, {"metropolis_chunk": 300},
                    {"direct_max_blocks": 4096}, {"rejection_table": 2},
                    {"single_wg_max": -1}):
            with pytest.raises(pfr.PfrError):
                pfr.set_tuning(**bad)
            assert pfr.get_tuning() == t
        # JSON file: top-level integers, unknown keys ignored, absent keys kept
        f = tmp_path / "tuning.json"
        f.write_text('{"version": 2, "rejection_per_wave": 128, "device": "x", '
                     '"measured_ms": {"metropolis_chunk": 7}}')
        lib = _lib.load()
        assert lib.pfr_load_tuning(str(f).encode()) == _lib.PFR_OK
        t2 = pfr.get_tuning()
        assert t2["rejection_per_wave"] == 128 and t2["metropolis_chunk"] == 1024
        f.write_text('{"version": 1, "rejection_per_wave": 128}')
        assert lib.pfr_load_tuning(str(f).encode()) == _lib.PFR_EINVAL
        f.write_text('{"version": 2, "batch_stage_max_kb": 32}')
        assert lib.pfr_load_tuning(str(f).encode()) == _lib.PFR_EINVAL
        f.write_text('{"version": 2, "batch_permute_lds_max": 8192, "batch_metropolis_chunk": 2048}')
        assert lib.pfr_load_tuning(str(f).encode()) == _lib.PFR_OK
        t3 = pfr.get_tuning()
        assert (t3["batch_permute_lds_max"], t3["batch_metropolis_chunk"]) == (8192, 2048)
        assert lib.pfr_load_tuning(str(tmp_path / "missing.json").encode()) == _lib.PFR_EINVAL
    finally:
        pfr.set_tuning(**saved)
