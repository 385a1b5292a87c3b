// pfr_api.hip -- the C ABI of libpfresample (declared in include/pfresample.h):
// argument checks, workspace sizing and kernel launches.  Nothing here
// allocates, frees or synchronises.
#include "pfresample.h"
#include "pfr_kernels.h"

namespace {

using namespace pfr;

constexpr int64_t kMaxN = (int64_t)1 << 31;
constexpr int64_t kSingleWGMax = 4096;  // single vectors up to this run in one workgroup

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

size_t lgssm_offsets_bytes(int32_t n_filters) {
  return (((size_t)n_filters + 1) * sizeof(int64_t) + 255) & ~(size_t)255;
}

size_t dtype_size(pfr_dtype dt) { return dt == PFR_F64 ? 8 : 4; }

bool uses_scan_workspace(const SegInfo& s) {
  return s.n_filters == 1 && s.n_total > kSingleWGMax;
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
      if (!uses_scan_workspace(s)) return 0;
      return scan_layout(s.n_total, op == PFR_OP_MULTINOMIAL).total;
    case PFR_OP_METROPOLIS:
    case PFR_OP_REJECTION:
      return alt_workspace_bytes(dtype == PFR_F64, s.n_total, s.n_filters, s.max_len);
    case PFR_OP_OFFSPRING_TO_ANCESTORS:
      return o2a_workspace_bytes(s.n_total);
    case PFR_OP_PERMUTE:
      return permute_workspace_bytes(s.n_total);
  }
  return 0;
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
  return launch_result(launch_metropolis(dtype == PFR_F64, w, s.n_total, s.offsets, s.n_filters,
                                         s.max_len, B, B_dev, make_key(rng), rng.offset,
                                         rng.filter_base, ancestors, ws, ws ? ws_bytes : 0,
                                         (hipStream_t)stream));
}

int resample_rejection(const void* w, pfr_dtype dtype, const pfr_segments* seg, double w_max,
                       const double* w_max_dev, uint32_t max_trials, pfr_rng rng,
                       int32_t* ancestors, void* ws, size_t ws_bytes, uint32_t* dev_flags,
                       void* stream) {
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
  return launch_result(launch_rejection(dtype == PFR_F64, w, s.n_total, s.offsets, s.n_filters,
                                        s.max_len, w_max, w_max_dev, max_trials, make_key(rng),
                                        rng.offset, rng.filter_base, ancestors, dev_flags, ws,
                                        ws ? ws_bytes : 0,
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
  const size_t need = permute_workspace_bytes(s.n_total);
  if (!ws || ws_bytes < need || !aligned256(ws)) return PFR_EWORKSPACE;
  if (overlaps(ws, need, permuted, (size_t)s.n_total * 4) ||
      overlaps(ws, need, ancestors, (size_t)s.n_total * 4))
    return PFR_EINVAL;
  return launch_result(launch_permute(ancestors, s.n_total, s.offsets, s.n_filters, s.max_len,
                                      sorted_hint != 0, permuted, ws, dev_flags,
                                      (hipStream_t)stream));
}

size_t lgssm_workspace_bytes(int32_t n_filters, int32_t n) {
  if (n_filters < 1 || n < 1 || (int64_t)n_filters * n >= kMaxN) return 0;
  return lgssm_offsets_bytes(n_filters) + permute_workspace_bytes((int64_t)n_filters * n);
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
      e = precision == PFR_SCAN_EXACT
              ? launch_scan_batched(sch, false, w, total, offsets, nf, rkey, 0u, rng.filter_base,
                                    ancestors, dev_flags, st)
              : launch_fscan_batched(sch, (int)precision, false, w, total, offsets, nf, rkey, 0u,
                                     rng.filter_base, ancestors, dev_flags, st);
    }
  }
  if (e != hipSuccess) return PFR_ELAUNCH;
  e = launch_permute(ancestors, total, offsets, nf, n, collective_scheme, permuted, perm_ws,
                     dev_flags, st);
  if (e != hipSuccess) return PFR_ELAUNCH;
  Key nkey = make_key(rng);
  nkey.offset_dev = nullptr;
  return launch_result(launch_lgssm_move(n_filters, n, model->phi, model->q, model->r,
                                         log(0.01), y, T, t_dev, nkey, rng.offset,
                                         rng.filter_base, permuted, x, w, log_z, B_dev, dev_flags,
                                         st));
}

const char* pfr_status_string(int status) {
  switch (status) {
    case PFR_OK: return "ok";
    case PFR_EINVAL: return "invalid argument";
    case PFR_EWORKSPACE: return "workspace missing, too small or misaligned";
    case PFR_ELAUNCH: return "kernel launch failed";
    case PFR_ENOTSUP: return "not supported";
  }
  return "unknown status";
}

const char* pfr_version(void) { return "0.1.0"; }

}  // extern "C"
