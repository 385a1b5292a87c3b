// pfr_api.hip -- the C ABI of libpfresample (declared in include/pfresample.h):
// argument checks, workspace sizing and kernel launches.  Nothing here
// allocates or frees, and only pfr_take_check_flags synchronises.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "pfresample.h"
#include "pfr_kernels.h"

namespace pfr {

namespace {
// Set by pfr_set_tuning, read by the launchers of any host thread: every
// access holds the lock, and readers get a copy.
std::mutex g_tuning_mu;
// the values the autotuner chose on MI355X (gfx950), also in tuning.json
Tuning g_tuning = {4096, 256, 60, 1, 256, 2048, 0, 128, 8192, 1024, 16384};
}  // namespace

Tuning tuning() {
  std::lock_guard<std::mutex> lock(g_tuning_mu);
  return g_tuning;
}

}  // namespace pfr

namespace {

using namespace pfr;

constexpr int64_t kMaxN = (int64_t)1 << 31;

struct SegInfo {
  int64_t n_total;
  uint32_t n_filters;
  const int64_t* offsets;  // NULL for one segment
  int64_t max_len;
};

// Validates the segment description; returns PFR_OK and fills info.
int check_segments(const pfr_segments* seg, SegInfo* info) {
  if (!seg) return PFR_EINVAL;
  if (seg->n_total < 0 || seg->n_total >= kMaxN) return PFR_EINVAL;
  if (seg->n_filters < 1) return PFR_EINVAL;
  if (seg->n_filters > 1 && !seg->offsets) return PFR_EINVAL;
  info->n_total = seg->n_total;
  info->n_filters = (uint32_t)seg->n_filters;
  info->offsets = seg->n_filters > 1 ? seg->offsets : seg->offsets;
  info->max_len = seg->max_len;
  if (seg->n_filters == 1) {
    info->offsets = nullptr;  // one segment covers [0, n_total)
    info->max_len = seg->n_total;
  }
  return PFR_OK;
}

Key make_key(const pfr_rng& rng) {
  Key k;
  k.k0 = (uint32_t)rng.seed;
  k.k1 = (uint32_t)(rng.seed >> 32);
  k.offset_dev = rng.offset_dev;
  return k;
}

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

int launch_result(hipError_t e) { return e == hipSuccess ? PFR_OK : PFR_ELAUNCH; }

// pfr_set_checks: the precondition checks run before the calls they cover.
std::atomic<int> g_checks{0};
bool checks_on() { return g_checks.load(std::memory_order_relaxed) != 0; }

// With the checks on, a sorted_hint is tested and then not relied on: the
// call takes the path for any ancestry, whose result is the same for sorted
// input and the defined one for any other.
int check_hint(const int32_t* a, const SegInfo& s, int32_t* sorted_hint, uint32_t* dev_flags,
               void* stream) {
  if (!checks_on() || !*sorted_hint) return PFR_OK;
  *sorted_hint = 0;
  return launch_result(
      launch_check_sorted(a, s.n_total, s.offsets, s.n_filters, dev_flags, (hipStream_t)stream));
}

size_t lgssm_offsets_bytes(int32_t n_filters) {
  return (((size_t)n_filters + 1) * sizeof(int64_t) + 255) & ~(size_t)255;
}

size_t dtype_size(pfr_dtype dt) { return dt == PFR_F64 ? 8 : 4; }

bool uses_scan_workspace(const SegInfo& s) {
  return s.n_filters == 1 && s.n_total > tuning().single_wg_max;
}

int collective(int scheme, const void* w, pfr_dtype dtype, const pfr_segments* seg,
               pfr_precision precision, pfr_rng rng, int32_t* a, void* ws, size_t ws_bytes,
               uint32_t* dev_flags, void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (dtype != PFR_F32 && dtype != PFR_F64) return PFR_EINVAL;
  if (precision < PFR_SCAN_EXACT || precision > PFR_SCAN_NAIVE_F32) return PFR_EINVAL;
  if (s.n_total == 0) return PFR_OK;
  if (!w || !a) return PFR_EINVAL;
  if (overlaps(w, (size_t)s.n_total * dtype_size(dtype), a, (size_t)s.n_total * 4))
    return PFR_EINVAL;
  const hipStream_t st = (hipStream_t)stream;
  const Key key = make_key(rng);
  if (!uses_scan_workspace(s)) {
    if (s.n_filters > 1 && s.max_len > PFR_MAX_BATCH_SEGMENT) return PFR_ENOTSUP;
    if (precision != PFR_SCAN_EXACT)
      return launch_result(launch_fscan_batched(scheme, (int)precision, dtype == PFR_F64, w,
                                                s.n_total, s.offsets, s.n_filters, key,
                                                rng.offset, rng.filter_base, a, dev_flags, st));
    // a batch with a workspace runs block-parallel, without one (or when
    // its longest segment is short) in one workgroup per segment; the
    // results are the same
    if (s.n_filters > 1 && ws &&
        !(s.max_len > 0 && s.max_len <= tuning().batch_scan_wg_max_len)) {
      const SegLayout SL = seg_layout(s.n_total, s.n_filters, scheme == SCHEME_MULTINOMIAL);
      if (ws_bytes < SL.total || !aligned256(ws)) return PFR_EWORKSPACE;
      if (overlaps(ws, SL.total, a, (size_t)s.n_total * 4)) return PFR_EINVAL;
      return launch_result(launch_scan_segmented(scheme, dtype == PFR_F64, w, s.n_total,
                                                 s.offsets, s.n_filters, key, rng.offset,
                                                 rng.filter_base, a, ws, dev_flags, st));
    }
    return launch_result(launch_scan_batched(scheme, dtype == PFR_F64, w, s.n_total, s.offsets,
                                             s.n_filters, key, rng.offset, rng.filter_base, a,
                                             dev_flags, st));
  }
  const ScanLayout L = scan_layout(s.n_total, scheme == SCHEME_MULTINOMIAL);
  if (!ws || ws_bytes < L.total) return PFR_EWORKSPACE;
  if (!aligned256(ws)) return PFR_EWORKSPACE;
  if (overlaps(ws, L.total, a, (size_t)s.n_total * 4)) return PFR_EINVAL;
  if (precision != PFR_SCAN_EXACT)
    return launch_result(launch_fscan(scheme, (int)precision, dtype == PFR_F64, w, s.n_total, key,
                                      rng.offset, rng.filter_base, a, ws, dev_flags, st));
  return launch_result(launch_scan(scheme, dtype == PFR_F64, w, s.n_total, key, rng.offset,
                                   rng.filter_base, a, ws, dev_flags, st));
}

}  // namespace

extern "C" {

size_t pfr_workspace_bytes(pfr_op op, const pfr_segments* seg, pfr_dtype dtype) {
  SegInfo s;
  if (check_segments(seg, &s)) return 0;
  switch (op) {
    case PFR_OP_MULTINOMIAL:
    case PFR_OP_STRATIFIED:
    case PFR_OP_SYSTEMATIC:
      if (s.n_filters > 1) return seg_layout(s.n_total, s.n_filters, op == PFR_OP_MULTINOMIAL).total;
      if (!uses_scan_workspace(s)) return 0;
      return scan_layout(s.n_total, op == PFR_OP_MULTINOMIAL).total;
    case PFR_OP_METROPOLIS:
    case PFR_OP_REJECTION:
      return alt_workspace_bytes(dtype == PFR_F64, s.n_total, s.n_filters, s.max_len);
    case PFR_OP_OFFSPRING_TO_ANCESTORS:
      return o2a_workspace_bytes(s.n_total);
    case PFR_OP_PERMUTE:
      return permute_workspace_bytes(s.n_total, s.n_filters);
    case PFR_OP_ANCESTORS_TO_OFFSPRING:
      return 0;
    case PFR_OP_ESS:
      return ess_workspace_bytes(s.n_total, s.n_filters);
    case PFR_OP_MULTINOMIAL_IID:
      return multinomial_iid_workspace_bytes(s.n_total);
    case PFR_OP_SCALED_PREFIX:
      return s.n_filters == 1 && s.n_total > 0 ? scan_layout(s.n_total, false).total : 0;
  }
  return 0;
}

int pfr_scaled_prefix(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                      pfr_precision precision, double* r_out, void* ws, size_t ws_bytes,
                      uint32_t* dev_flags, void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (dtype != PFR_F32 && dtype != PFR_F64) return PFR_EINVAL;
  if (precision < PFR_SCAN_EXACT || precision > PFR_SCAN_NAIVE_F32) return PFR_EINVAL;
  if (s.n_filters > 1) return PFR_ENOTSUP;
  if (s.n_total == 0) return PFR_OK;
  if (!w || !r_out) return PFR_EINVAL;
  const size_t need = scan_layout(s.n_total, false).total;
  if (!ws || ws_bytes < need || !aligned256(ws)) return PFR_EWORKSPACE;
  const size_t rb = (size_t)s.n_total * sizeof(double);
  if (overlaps(w, (size_t)s.n_total * dtype_size(dtype), r_out, rb) || overlaps(ws, need, r_out, rb))
    return PFR_EINVAL;
  const hipStream_t st = (hipStream_t)stream;
  if (precision == PFR_SCAN_EXACT)
    return launch_result(launch_scan_r(dtype == PFR_F64, w, s.n_total, r_out, ws, dev_flags, st));
  return launch_result(launch_fscan_r((int)precision, dtype == PFR_F64, w, s.n_total, r_out, ws,
                                      dev_flags, st));
}

int pfr_workspace_init(void* ws, size_t ws_bytes, void* stream) {
  if (ws_bytes == 0) return PFR_OK;
  if (!ws || !aligned256(ws)) return PFR_EWORKSPACE;
  return launch_result(launch_zero_u32((uint32_t*)ws, ws_bytes / 4, (hipStream_t)stream));
}

int resample_multinomial(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                         pfr_precision precision, pfr_rng rng, int32_t* ancestors, void* ws,
                         size_t ws_bytes, uint32_t* dev_flags, void* stream) {
  return collective(SCHEME_MULTINOMIAL, w, dtype, seg, precision, rng, ancestors, ws, ws_bytes,
                    dev_flags, stream);
}

int resample_multinomial_iid(const void* w, pfr_dtype dtype, const pfr_segments* seg, pfr_rng rng,
                             int32_t* ancestors, void* ws, size_t ws_bytes, uint32_t* dev_flags,
                             void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (dtype != PFR_F32 && dtype != PFR_F64) return PFR_EINVAL;
  if (s.n_filters > 1) return PFR_ENOTSUP;
  if (s.n_total == 0) return PFR_OK;
  if (!w || !ancestors) return PFR_EINVAL;
  if (overlaps(w, (size_t)s.n_total * dtype_size(dtype), ancestors, (size_t)s.n_total * 4))
    return PFR_EINVAL;
  const size_t need = multinomial_iid_workspace_bytes(s.n_total);
  if (!ws || ws_bytes < need || !aligned256(ws)) return PFR_EWORKSPACE;
  if (overlaps(ws, need, ancestors, (size_t)s.n_total * 4) ||
      overlaps(ws, need, w, (size_t)s.n_total * dtype_size(dtype)))
    return PFR_EINVAL;
  return launch_result(launch_multinomial_iid(dtype == PFR_F64, w, s.n_total, make_key(rng),
                                              rng.offset, rng.filter_base, ancestors, ws,
                                              dev_flags, (hipStream_t)stream));
}

int resample_stratified(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                        pfr_precision precision, pfr_rng rng, int32_t* ancestors, void* ws,
                        size_t ws_bytes, uint32_t* dev_flags, void* stream) {
  return collective(SCHEME_STRATIFIED, w, dtype, seg, precision, rng, ancestors, ws, ws_bytes,
                    dev_flags, stream);
}

int resample_systematic(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                        pfr_precision precision, pfr_rng rng, int32_t* ancestors, void* ws,
                        size_t ws_bytes, uint32_t* dev_flags, void* stream) {
  return collective(SCHEME_SYSTEMATIC, w, dtype, seg, precision, rng, ancestors, ws, ws_bytes,
                    dev_flags, stream);
}

int resample_metropolis(const void* w, pfr_dtype dtype, const pfr_segments* seg, int32_t B,
                        const int32_t* B_dev, pfr_rng rng, int32_t* ancestors, void* ws,
                        size_t ws_bytes, void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (dtype != PFR_F32 && dtype != PFR_F64) return PFR_EINVAL;
  if (B < 0 || B >= (1 << 28)) return PFR_EINVAL;
  if (s.n_total == 0) return PFR_OK;
  if (!w || !ancestors) return PFR_EINVAL;
  if (overlaps(w, (size_t)s.n_total * dtype_size(dtype), ancestors, (size_t)s.n_total * 4))
    return PFR_EINVAL;
  if (ws && !aligned256(ws)) return PFR_EWORKSPACE;
  if (checks_on()) {
    rc = launch_result(launch_check_weights(dtype == PFR_F64, w, s.n_total, s.offsets,
                                            s.n_filters, false, 0.0, nullptr, nullptr,
                                            (hipStream_t)stream));
    if (rc) return rc;
  }
  return launch_result(launch_metropolis(dtype == PFR_F64, w, s.n_total, s.offsets, s.n_filters,
                                         s.max_len, B, B_dev, make_key(rng), rng.offset,
                                         rng.filter_base, ancestors, ws, ws ? ws_bytes : 0,
                                         (hipStream_t)stream));
}

}  // extern "C"

namespace {

// resample_rejection, with the bound check of the precondition checks unless
// the bound need not hold (partial rejection control)
int rejection(const void* w, pfr_dtype dtype, const pfr_segments* seg, double w_max,
              const double* w_max_dev, uint32_t max_trials, pfr_rng rng, int32_t* ancestors,
              void* ws, size_t ws_bytes, uint32_t* dev_flags, void* stream, bool bounded) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (dtype != PFR_F32 && dtype != PFR_F64) return PFR_EINVAL;
  if (max_trials < 1 || max_trials >= (1u << 28)) return PFR_EINVAL;
  if (!w_max_dev && !(w_max > 0.0 && w_max < __builtin_huge_val())) return PFR_EINVAL;
  if (s.n_total == 0) return PFR_OK;
  if (!w || !ancestors) return PFR_EINVAL;
  if (overlaps(w, (size_t)s.n_total * dtype_size(dtype), ancestors, (size_t)s.n_total * 4))
    return PFR_EINVAL;
  if (ws && !aligned256(ws)) return PFR_EWORKSPACE;
  if (checks_on()) {
    rc = launch_result(launch_check_weights(dtype == PFR_F64, w, s.n_total, s.offsets,
                                            s.n_filters, bounded, w_max, w_max_dev, dev_flags,
                                            (hipStream_t)stream));
    if (rc) return rc;
  }
  return launch_result(launch_rejection(dtype == PFR_F64, w, s.n_total, s.offsets, s.n_filters,
                                        s.max_len, w_max, w_max_dev, max_trials, make_key(rng),
                                        rng.offset, rng.filter_base, ancestors, dev_flags, ws,
                                        ws ? ws_bytes : 0,
                                        (hipStream_t)stream));
}

}  // namespace

extern "C" {

int resample_rejection(const void* w, pfr_dtype dtype, const pfr_segments* seg, double w_max,
                       const double* w_max_dev, uint32_t max_trials, pfr_rng rng,
                       int32_t* ancestors, void* ws, size_t ws_bytes, uint32_t* dev_flags,
                       void* stream) {
  return rejection(w, dtype, seg, w_max, w_max_dev, max_trials, rng, ancestors, ws, ws_bytes,
                   dev_flags, stream, true);
}

int resample_partial_rejection(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                               double v_max, const double* v_max_dev, uint32_t max_trials,
                               pfr_rng rng, int32_t* ancestors, void* weights_out, void* ws,
                               size_t ws_bytes, uint32_t* dev_flags, void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (dtype != PFR_F32 && dtype != PFR_F64) return PFR_EINVAL;
  if (s.n_total > 0 && !weights_out) return PFR_EINVAL;
  if (s.n_total > 0) {
    const size_t wb = (size_t)s.n_total * dtype_size(dtype);
    if (overlaps(weights_out, wb, ancestors, (size_t)s.n_total * 4) ||
        (w && overlaps(weights_out, wb, w, wb)))
      return PFR_EINVAL;
  }
  rc = rejection(w, dtype, seg, v_max, v_max_dev, max_trials, rng, ancestors, ws, ws_bytes,
                 dev_flags, stream, false);
  if (rc || s.n_total == 0) return rc;
  return launch_result(launch_prc_weights(dtype == PFR_F64, w, s.n_total, s.offsets, s.n_filters,
                                          v_max, v_max_dev, ancestors, weights_out,
                                          (hipStream_t)stream));
}

int offspring_to_ancestors(const int32_t* offspring, const pfr_segments* seg, int32_t* ancestors,
                           void* ws, size_t ws_bytes, uint32_t* dev_flags, void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (s.n_total == 0) return PFR_OK;
  if (!offspring || !ancestors) return PFR_EINVAL;
  if (overlaps(offspring, (size_t)s.n_total * 4, ancestors, (size_t)s.n_total * 4))
    return PFR_EINVAL;
  const size_t need = o2a_workspace_bytes(s.n_total);
  if (!ws || ws_bytes < need || !aligned256(ws)) return PFR_EWORKSPACE;
  return launch_result(launch_offspring_to_ancestors(offspring, s.n_total, s.offsets, s.n_filters,
                                                     ancestors, ws, dev_flags,
                                                     (hipStream_t)stream));
}

int permute_ancestors(const int32_t* ancestors, const pfr_segments* seg, int32_t sorted_hint,
                      int32_t* permuted, void* ws, size_t ws_bytes, uint32_t* dev_flags,
                      void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (s.n_total == 0) return PFR_OK;
  if (!ancestors || !permuted) return PFR_EINVAL;
  if (overlaps(ancestors, (size_t)s.n_total * 4, permuted, (size_t)s.n_total * 4))
    return PFR_EINVAL;
  // the size pfr_workspace_bytes reports; a smaller one of at least the claim
  // vector and marks (8 bytes per particle) runs the atomic claim instead
  const size_t full = permute_workspace_bytes(s.n_total, s.n_filters);
  const size_t need = ws_bytes >= full ? full : permute_workspace_min_bytes(s.n_total);
  if (!ws || ws_bytes < need || !aligned256(ws)) return PFR_EWORKSPACE;
  if (overlaps(ws, need, permuted, (size_t)s.n_total * 4) ||
      overlaps(ws, need, ancestors, (size_t)s.n_total * 4))
    return PFR_EINVAL;
  rc = check_hint(ancestors, s, &sorted_hint, dev_flags, stream);
  if (rc) return rc;
  return launch_result(launch_permute(ancestors, s.n_total, s.offsets, s.n_filters, s.max_len,
                                      sorted_hint != 0, permuted, ws, need, dev_flags,
                                      (hipStream_t)stream));
}

}  // extern "C"

namespace {

// Scratch of permute_ancestors_noalloc: the claim vector and the marked
// ancestry (4 + 4 bytes per particle, each part 256-byte aligned) of up to
// PFR_NOALLOC_MAX_N particles, and the bucketed claim's counts and pairs when
// they fit beside them.  One copy per GPU, at that GPU's own address,
// held until the process ends.  Host code never uses the name `scratch` as an
// address: the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) uint8_t scratch[PFR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices];  // device address of `scratch` on each device (or null)

// The current device's scratch address, looked up on the first call on that
// device.  The permutation writes every claim, mark, count and pair before
// reading it, so the scratch needs no clearing.
int noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PFR_ELAUNCH;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PFR_ELAUNCH;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return PFR_OK;
}

}  // namespace

extern "C" {

int permute_ancestors_noalloc(const int32_t* ancestors, const pfr_segments* seg,
                              int32_t sorted_hint, int32_t* permuted, uint32_t* dev_flags,
                              void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (s.n_total == 0) return PFR_OK;
  if (s.n_total > PFR_NOALLOC_MAX_N) return PFR_ETOOBIG;
  if (!ancestors || !permuted) return PFR_EINVAL;
  if (overlaps(ancestors, (size_t)s.n_total * 4, permuted, (size_t)s.n_total * 4))
    return PFR_EINVAL;
  static_assert(PFR_NOALLOC_SCRATCH_BYTES >= 2 * (size_t)PFR_NOALLOC_MAX_N * sizeof(int32_t),
                "the scratch holds the claim vector and the marks of PFR_NOALLOC_MAX_N particles");
  if (permute_workspace_min_bytes(s.n_total) > PFR_NOALLOC_SCRATCH_BYTES) return PFR_ETOOBIG;
  void* ws = nullptr;
  rc = noalloc_scratch(&ws);
  if (rc) return rc;
  rc = check_hint(ancestors, s, &sorted_hint, dev_flags, stream);
  if (rc) return rc;
  return launch_result(launch_permute(ancestors, s.n_total, s.offsets, s.n_filters, s.max_len,
                                      sorted_hint != 0, permuted, ws, PFR_NOALLOC_SCRATCH_BYTES,
                                      dev_flags, (hipStream_t)stream));
}

int ancestors_to_offspring(const int32_t* ancestors, const pfr_segments* seg, int32_t sorted_hint,
                           int32_t* offspring, uint32_t* dev_flags, void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (s.n_total == 0) return PFR_OK;
  if (!ancestors || !offspring) return PFR_EINVAL;
  if (overlaps(ancestors, (size_t)s.n_total * 4, offspring, (size_t)s.n_total * 4))
    return PFR_EINVAL;
  rc = check_hint(ancestors, s, &sorted_hint, dev_flags, stream);
  if (rc) return rc;
  return launch_result(launch_ancestors_to_offspring(ancestors, s.n_total, s.offsets,
                                                     s.n_filters, s.max_len, sorted_hint != 0,
                                                     offspring, dev_flags,
                                                     (hipStream_t)stream));
}

int effective_sample_size(const void* w, pfr_dtype dtype, const pfr_segments* seg, double* ess,
                          void* ws, size_t ws_bytes, uint32_t* dev_flags, void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (dtype != PFR_F32 && dtype != PFR_F64) return PFR_EINVAL;
  if (!ess || (s.n_total > 0 && !w)) return PFR_EINVAL;
  const size_t need = ess_workspace_bytes(s.n_total, s.n_filters);
  if (!ws || ws_bytes < need || !aligned256(ws)) return PFR_EWORKSPACE;
  const size_t ebytes = (size_t)s.n_filters * sizeof(double);
  if (overlaps(ws, need, ess, ebytes) ||
      (s.n_total > 0 && overlaps(w, (size_t)s.n_total * dtype_size(dtype), ess, ebytes)))
    return PFR_EINVAL;
  return launch_result(launch_ess(dtype == PFR_F64, w, s.n_total, s.offsets, s.n_filters, ess, ws,
                                  dev_flags, (hipStream_t)stream));
}

int copy_particles(const int32_t* permuted, const pfr_segments* seg, void* x, size_t elem_bytes,
                   int32_t dim, int64_t particle_stride, int64_t component_stride,
                   uint32_t* dev_flags, void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (elem_bytes != 1 && elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8 &&
      elem_bytes != 16)
    return PFR_EINVAL;
  if (dim < 1 || particle_stride < 1 || component_stride < 1) return PFR_EINVAL;
  // distinct (particle, component) pairs must address distinct elements
  const bool rows = component_stride == 1 && particle_stride >= dim;
  const bool cols = particle_stride == 1 && component_stride >= s.n_total;
  if (!(dim == 1 || rows || cols)) return PFR_EINVAL;
  if (s.n_total == 0) return PFR_OK;
  if (!permuted || !x) return PFR_EINVAL;
  if ((reinterpret_cast<uintptr_t>(x) & (elem_bytes - 1)) != 0) return PFR_EINVAL;
  const double span = ((double)(s.n_total - 1) * (double)particle_stride +
                       (double)(dim - 1) * (double)component_stride + 1.0) * (double)elem_bytes;
  if (span >= 0x1p62) return PFR_EINVAL;
  if (overlaps(x, (size_t)span, permuted, (size_t)s.n_total * 4)) return PFR_EINVAL;
  return launch_result(launch_copy(permuted, s.n_total, s.offsets, s.n_filters, x, elem_bytes, dim,
                                   particle_stride, dim == 1 ? 1 : component_stride, dev_flags,
                                   (hipStream_t)stream));
}

size_t pfr_resample_permuted_workspace_bytes(pfr_op scheme, const pfr_segments* seg,
                                             pfr_dtype dtype) {
  SegInfo s;
  if (check_segments(seg, &s)) return 0;
  if (scheme < PFR_OP_MULTINOMIAL || scheme > PFR_OP_REJECTION) return 0;
  const size_t perm = permute_workspace_bytes(s.n_total, s.n_filters);
  return perm + pfr_workspace_bytes(scheme, seg, dtype);
}

int resample_permuted(pfr_op scheme, const void* w, pfr_dtype dtype, const pfr_segments* seg,
                      const pfr_scheme_params* params, pfr_rng rng, int32_t* ancestors,
                      int32_t* permuted, void* ws, size_t ws_bytes, uint32_t* dev_flags,
                      void* stream) {
  SegInfo s;
  int rc = check_segments(seg, &s);
  if (rc) return rc;
  if (!params || scheme < PFR_OP_MULTINOMIAL || scheme > PFR_OP_REJECTION) return PFR_EINVAL;
  if (dtype != PFR_F32 && dtype != PFR_F64) return PFR_EINVAL;
  if (s.n_total == 0) return PFR_OK;
  if (!w || !ancestors || !permuted) return PFR_EINVAL;
  const size_t abytes = (size_t)s.n_total * 4;
  if (overlaps(ancestors, abytes, permuted, abytes) ||
      overlaps(w, (size_t)s.n_total * dtype_size(dtype), permuted, abytes))
    return PFR_EINVAL;
  const size_t perm = permute_workspace_bytes(s.n_total, s.n_filters);
  const size_t need = perm + pfr_workspace_bytes(scheme, seg, dtype);
  if (!ws || ws_bytes < need || !aligned256(ws)) return PFR_EWORKSPACE;
  if (overlaps(ws, need, ancestors, abytes) || overlaps(ws, need, permuted, abytes))
    return PFR_EINVAL;
  void* rws = (char*)ws + perm;  // the resampler's own workspace
  const size_t rbytes = ws_bytes - perm;
  const bool sorted_out = scheme <= PFR_OP_SYSTEMATIC;  // collective schemes
  const hipStream_t st = (hipStream_t)stream;
  // the claim fused into the emission: long single vectors of the exact
  // collective schemes, whose ancestries are sorted (shorter ones are
  // permuted in LDS)
  if (s.n_filters == 1 && sorted_out && params->precision == PFR_SCAN_EXACT &&
      uses_scan_workspace(s) && s.n_total > 1024) {
    rc = launch_result(launch_scan_claimed(scheme == PFR_OP_MULTINOMIAL   ? SCHEME_MULTINOMIAL
                                           : scheme == PFR_OP_STRATIFIED ? SCHEME_STRATIFIED
                                                                         : SCHEME_SYSTEMATIC,
                                           dtype == PFR_F64, w, s.n_total, make_key(rng),
                                           rng.offset, rng.filter_base, ancestors, rws, dev_flags,
                                           permute_claims(ws), permute_marks(ws, s.n_total), st));
    if (rc) return rc;
    return launch_result(launch_resolve(s.n_total, permuted, ws, dev_flags, st));
  }
  // the two steps one after the other
  switch (scheme) {
    case PFR_OP_MULTINOMIAL:
    case PFR_OP_STRATIFIED:
    case PFR_OP_SYSTEMATIC:
      rc = collective(scheme == PFR_OP_MULTINOMIAL   ? SCHEME_MULTINOMIAL
                      : scheme == PFR_OP_STRATIFIED ? SCHEME_STRATIFIED
                                                    : SCHEME_SYSTEMATIC,
                      w, dtype, seg, params->precision, rng, ancestors, rws, rbytes, dev_flags,
                      stream);
      break;
    case PFR_OP_METROPOLIS:
      rc = resample_metropolis(w, dtype, seg, params->B, params->B_dev, rng, ancestors, rws,
                               rbytes, stream);
      break;
    default:
      rc = resample_rejection(w, dtype, seg, params->w_max, params->w_max_dev, params->max_trials,
                              rng, ancestors, rws, rbytes, dev_flags, stream);
      break;
  }
  if (rc) return rc;
  return permute_ancestors(ancestors, seg, sorted_out ? 1 : 0, permuted, ws, perm, dev_flags,
                           stream);
}

size_t lgssm_workspace_bytes(int32_t n_filters, int32_t n) {
  if (n_filters < 1 || n < 1 || (int64_t)n_filters * n >= kMaxN) return 0;
  const int64_t total = (int64_t)n_filters * n;
  const size_t perm = permute_workspace_bytes(total, (uint32_t)n_filters);
  const size_t seg = seg_layout(total, (uint32_t)n_filters, true).total;
  return lgssm_offsets_bytes(n_filters) + (perm > seg ? perm : seg);
}

int lgssm_init(const pfr_lgssm* model, int32_t n_filters, int32_t n, pfr_rng rng, float* x,
               float* w, double* log_z, int32_t* B_dev, uint32_t* t_dev, void* ws,
               size_t ws_bytes, void* stream) {
  if (!model || n_filters < 1 || n < 1 || (int64_t)n_filters * n >= kMaxN) return PFR_EINVAL;
  if (!x || !w || !log_z || !B_dev || !t_dev) return PFR_EINVAL;
  if (!(model->s0 >= 0.0)) return PFR_EINVAL;
  if (!ws || !aligned256(ws) || ws_bytes < lgssm_workspace_bytes(n_filters, n))
    return PFR_EWORKSPACE;
  Key key = make_key(rng);
  key.offset_dev = nullptr;
  return launch_result(launch_lgssm_init(n_filters, n, model->s0, key, rng.offset,
                                         rng.filter_base, x, w, log_z, B_dev, t_dev,
                                         (int64_t*)ws, (hipStream_t)stream));
}

int lgssm_step(const pfr_lgssm* model, pfr_op scheme, pfr_precision precision, int32_t n_filters,
               int32_t n, const double* y, int32_t T, uint32_t* t_dev, pfr_rng rng, float* x, float* w,
               double* log_z, int32_t* B_dev, int32_t* ancestors, int32_t* permuted, void* ws,
               size_t ws_bytes, uint32_t* dev_flags, void* stream) {
  if (!model || n_filters < 1 || n < 1 || (int64_t)n_filters * n >= kMaxN) return PFR_EINVAL;
  if (!y || T < 1 || !t_dev || !x || !w || !log_z || !B_dev || !ancestors || !permuted)
    return PFR_EINVAL;
  if (!(model->r > 0.0) || !(model->q >= 0.0)) return PFR_EINVAL;
  if (precision < PFR_SCAN_EXACT || precision > PFR_SCAN_NAIVE_F32) return PFR_EINVAL;
  if (scheme > PFR_OP_REJECTION || scheme < PFR_OP_MULTINOMIAL) return PFR_EINVAL;
  const bool collective_scheme = scheme <= PFR_OP_SYSTEMATIC;
  if (collective_scheme && n > PFR_MAX_BATCH_SEGMENT) return PFR_ENOTSUP;
  if (!ws || !aligned256(ws) || ws_bytes < lgssm_workspace_bytes(n_filters, n))
    return PFR_EWORKSPACE;
  const int64_t total = (int64_t)n_filters * n;
  if (overlaps(ancestors, (size_t)total * 4, permuted, (size_t)total * 4)) return PFR_EINVAL;
  const hipStream_t st = (hipStream_t)stream;
  const int64_t* offsets = (const int64_t*)ws;
  void* perm_ws = (char*)ws + lgssm_offsets_bytes(n_filters);
  // the resampler at step t uses counter offset t
  Key rkey = make_key(rng);
  rkey.offset_dev = t_dev;
  const uint32_t nf = (uint32_t)n_filters;
  hipError_t e;
  switch (scheme) {
    case PFR_OP_METROPOLIS:
      e = launch_metropolis(false, w, total, offsets, nf, n, 0, B_dev, rkey, 0u, rng.filter_base,
                            ancestors, nullptr, 0, st);
      break;
    case PFR_OP_REJECTION:
      e = launch_rejection(false, w, total, offsets, nf, n, 1.0, nullptr, 1u << 20, rkey, 0u,
                           rng.filter_base, ancestors, dev_flags, nullptr, 0, st);
      break;
    default: {
      const int sch = scheme == PFR_OP_MULTINOMIAL   ? SCHEME_MULTINOMIAL
                      : scheme == PFR_OP_STRATIFIED ? SCHEME_STRATIFIED
                                                    : SCHEME_SYSTEMATIC;
      // the resampler's workspace is free again before the permutation uses it
      e = precision == PFR_SCAN_EXACT
              ? launch_scan_segmented(sch, false, w, total, offsets, nf, rkey, 0u,
                                      rng.filter_base, ancestors, perm_ws, dev_flags, st)
              : launch_fscan_batched(sch, (int)precision, false, w, total, offsets, nf, rkey, 0u,
                                     rng.filter_base, ancestors, dev_flags, st);
    }
  }
  if (e != hipSuccess) return PFR_ELAUNCH;
  e = launch_permute(ancestors, total, offsets, nf, n, collective_scheme, permuted, perm_ws,
                     permute_workspace_bytes(total, nf), dev_flags, st);
  if (e != hipSuccess) return PFR_ELAUNCH;
  Key nkey = make_key(rng);
  nkey.offset_dev = nullptr;
  return launch_result(launch_lgssm_move(n_filters, n, model->phi, model->q, model->r,
                                         log(0.01), y, T, t_dev, nkey, rng.offset,
                                         rng.filter_base, permuted, x, w, log_z, B_dev, dev_flags,
                                         st));
}

void pfr_tuning_defaults(pfr_tuning* t) {
  if (!t) return;
  t->version = PFR_TUNING_VERSION;
  t->single_wg_max = 4096;
  t->direct_max_blocks = 256;
  t->metropolis_table_min_B = 60;
  t->rejection_table = 1;
  t->rejection_per_wave = 256;
  t->metropolis_chunk = 2048;
  t->batch_scan_wg_max_len = 0;
  t->batch_stage_max_kb = 128;
  t->batch_metropolis_chunk = 8192;
  t->batch_rejection_per_wave = 1024;
  t->batch_permute_lds_max = 16384;
}

int pfr_get_tuning(pfr_tuning* t) {
  if (!t) return PFR_EINVAL;
  const Tuning g = tuning();
  t->version = PFR_TUNING_VERSION;
  t->single_wg_max = g.single_wg_max;
  t->direct_max_blocks = g.direct_max_blocks;
  t->metropolis_table_min_B = g.metropolis_table_min_B;
  t->rejection_table = g.rejection_table;
  t->rejection_per_wave = g.rejection_per_wave;
  t->metropolis_chunk = g.metropolis_chunk;
  t->batch_scan_wg_max_len = g.batch_scan_wg_max_len;
  t->batch_stage_max_kb = g.batch_stage_max_kb;
  t->batch_metropolis_chunk = g.batch_metropolis_chunk;
  t->batch_rejection_per_wave = g.batch_rejection_per_wave;
  t->batch_permute_lds_max = g.batch_permute_lds_max;
  return PFR_OK;
}

int pfr_set_tuning(const pfr_tuning* t) {
  if (!t || t->version != PFR_TUNING_VERSION) return PFR_EINVAL;
  if (t->single_wg_max < 0 || t->single_wg_max > PFR_MAX_BATCH_SEGMENT) return PFR_EINVAL;
  if (t->direct_max_blocks < 0 || t->direct_max_blocks > 2048) return PFR_EINVAL;
  if (t->metropolis_table_min_B < 0) return PFR_EINVAL;
  if (t->rejection_table != 0 && t->rejection_table != 1) return PFR_EINVAL;
  if (t->rejection_per_wave < 64 || t->rejection_per_wave > 4096) return PFR_EINVAL;
  if (t->metropolis_chunk < 256 || t->metropolis_chunk > 8192 || t->metropolis_chunk % 256)
    return PFR_EINVAL;
  if (t->batch_scan_wg_max_len < 0 || t->batch_scan_wg_max_len > PFR_MAX_BATCH_SEGMENT)
    return PFR_EINVAL;
  if (t->batch_stage_max_kb != 16 && t->batch_stage_max_kb != 64 && t->batch_stage_max_kb != 128)
    return PFR_EINVAL;
  if (t->batch_metropolis_chunk < 1024 || t->batch_metropolis_chunk > 65536 ||
      t->batch_metropolis_chunk % 1024)
    return PFR_EINVAL;
  if (t->batch_rejection_per_wave < 64 || t->batch_rejection_per_wave > 4096) return PFR_EINVAL;
  if (t->batch_permute_lds_max != 4096 && t->batch_permute_lds_max != 8192 &&
      t->batch_permute_lds_max != 16384)
    return PFR_EINVAL;
  std::lock_guard<std::mutex> lock(g_tuning_mu);
  g_tuning.single_wg_max = t->single_wg_max;
  g_tuning.direct_max_blocks = t->direct_max_blocks;
  g_tuning.metropolis_table_min_B = t->metropolis_table_min_B;
  g_tuning.rejection_table = t->rejection_table;
  g_tuning.rejection_per_wave = t->rejection_per_wave;
  g_tuning.metropolis_chunk = t->metropolis_chunk;
  g_tuning.batch_scan_wg_max_len = t->batch_scan_wg_max_len;
  g_tuning.batch_stage_max_kb = t->batch_stage_max_kb;
  g_tuning.batch_metropolis_chunk = t->batch_metropolis_chunk;
  g_tuning.batch_rejection_per_wave = t->batch_rejection_per_wave;
  g_tuning.batch_permute_lds_max = t->batch_permute_lds_max;
  return PFR_OK;
}

// Reads the integer fields named like pfr_tuning's from the top level of a
// JSON object (nested objects and other fields are skipped); fields that are
// absent keep their current value.
int pfr_load_tuning(const char* path) {
  if (!path) return PFR_EINVAL;
  FILE* f = fopen(path, "rb");
  if (!f) return PFR_EINVAL;
  static char buf[1 << 16];
  const size_t len = fread(buf, 1, sizeof(buf) - 1, f);
  fclose(f);
  buf[len] = 0;
  pfr_tuning t;
  pfr_get_tuning(&t);
  struct Field {
    const char* name;
    int32_t* slot;
  } fields[] = {{"version", &t.version},
                {"single_wg_max", &t.single_wg_max},
                {"direct_max_blocks", &t.direct_max_blocks},
                {"metropolis_table_min_B", &t.metropolis_table_min_B},
                {"rejection_table", &t.rejection_table},
                {"rejection_per_wave", &t.rejection_per_wave},
                {"metropolis_chunk", &t.metropolis_chunk},
                {"batch_scan_wg_max_len", &t.batch_scan_wg_max_len},
                {"batch_stage_max_kb", &t.batch_stage_max_kb},
                {"batch_metropolis_chunk", &t.batch_metropolis_chunk},
                {"batch_rejection_per_wave", &t.batch_rejection_per_wave},
                {"batch_permute_lds_max", &t.batch_permute_lds_max}};
  int depth = 0;
  const char* key = nullptr;  // last string seen at depth 1
  size_t key_len = 0;
  for (const char* p = buf; *p; ++p) {
    const char ch = *p;
    if (ch == '"') {  // a string: find its end (backslash escapes skipped)
      const char* q = p + 1;
      while (*q && *q != '"') q += (*q == '\\' && q[1]) ? 2 : 1;
      if (!*q) return PFR_EINVAL;
      if (depth == 1) {
        key = p + 1;
        key_len = (size_t)(q - p - 1);
      }
      p = q;
    } else if (ch == '{' || ch == '[') {
      ++depth;
      key = nullptr;
    } else if (ch == '}' || ch == ']') {
      --depth;
      key = nullptr;
    } else if (ch == ':' && depth == 1 && key) {
      for (const Field& fd : fields) {
        if (strlen(fd.name) == key_len && strncmp(fd.name, key, key_len) == 0) {
          char* end = nullptr;
          const long v = strtol(p + 1, &end, 10);
          if (end == p + 1) return PFR_EINVAL;
          *fd.slot = (int32_t)v;
        }
      }
      key = nullptr;
    }
  }
  if (depth != 0) return PFR_EINVAL;
  return pfr_set_tuning(&t);
}

const char* pfr_status_string(int status) {
  switch (status) {
    case PFR_OK: return "ok";
    case PFR_EINVAL: return "invalid argument";
    case PFR_EWORKSPACE: return "workspace missing, too small or misaligned";
    case PFR_ELAUNCH: return "kernel launch failed";
    case PFR_ENOTSUP: return "not supported";
    case PFR_ETOOBIG:
      return "input longer than the static scratch of the no-allocation entry point allows";
  }
  return "unknown status";
}

const char* pfr_version(void) { return "0.1.0"; }

int pfr_set_checks(int32_t on) {
  g_checks.store(on ? 1 : 0, std::memory_order_relaxed);
  return PFR_OK;
}

int32_t pfr_get_checks(void) { return checks_on() ? 1 : 0; }

int pfr_take_check_flags(void* stream, uint32_t* flags) {
  if (!flags) return PFR_EINVAL;
  return launch_result(take_check_word((hipStream_t)stream, flags));
}

int pfr_philox_rounds(void) { return kPhiloxRounds; }

}  // extern "C"
