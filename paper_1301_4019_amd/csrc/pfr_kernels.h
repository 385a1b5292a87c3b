// pfr_kernels.h -- launchers shared between the kernel files and the C-ABI
// layer of libpfresample.  Host-side declarations only; no torch types.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "pfr_device.h"

namespace pfr {

// Launch parameters chosen by the autotuner.  None of them changes a result:
// every kernel draws its random numbers by particle, and the exact prefix
// sums do not depend on how they are split.
struct Tuning {
  int32_t single_wg_max;           // collective: single vectors up to this length in one workgroup
  int32_t direct_max_blocks;       // exact collective: emit forms its own carries up to this many blocks
  int32_t metropolis_table_min_B;  // long vectors: bound-table Metropolis from this many steps (0 = never)
  int32_t rejection_table;         // long vectors: rejection with the bound table (0 / 1)
  int32_t rejection_per_wave;      // particles per wave of the rejection schedule
  int32_t metropolis_chunk;        // particles per workgroup of the global-memory Metropolis kernel
  int32_t batch_scan_wg_max_len;   // batches: one workgroup per segment up to this longest segment
  int32_t batch_stage_max_kb;      // batches: largest LDS staging tier of Metropolis / rejection
  int32_t batch_metropolis_chunk;  // batches: particles per workgroup of staged Metropolis
  int32_t batch_rejection_per_wave;  // batches: particles per wave of staged rejection
  int32_t batch_permute_lds_max;   // batches: segments permuted in LDS up to this length
};
Tuning tuning();  // a copy of the current settings (thread-safe)

// Collective schemes handled by the scan kernels.
enum Scheme : int { SCHEME_MULTINOMIAL = 0, SCHEME_STRATIFIED = 1, SCHEME_SYSTEMATIC = 2 };

// Canonical quantisation block of the exact prefix sums: 1024 weights.  The
// single-vector kernels give a block to one wave (16 consecutive weights per
// lane); the one-workgroup-per-segment and floating-point kernels to one
// workgroup of kWGThreads = 256 threads, 4 consecutive weights each.
constexpr int kBlock = 1024;
constexpr int kBlocksPerWG = 4;
constexpr int kWGThreads = kWave * kBlocksPerWG;

// Per-block record written by the reduce pass.
struct BlockRec {
  uint64_t sum;    // sum of the block's quantised values
  int32_t scale;   // q = floor(w * 2^scale) inside the block
  uint32_t bad;    // FLAG_BAD_WEIGHTS if a weight is negative or not finite
};

// Header at the start of a collective-scheme workspace.
struct ScanHeader {
  uint32_t status;       // FLAG_* bits of this call
  int32_t gscale;        // global fixed-point scale of the carries
  uint32_t groups_done;  // carry groups finished (zeroed by the records pass)
  uint32_t pad0;
  union {
    u128 Q;          // exact total at the global scale
    double W;        // floating-point total (precision modes other than exact)
  };
  uint32_t pad[56];  // header padded to 256 bytes
};
static_assert(sizeof(ScanHeader) == 256, "scan header is 256 bytes");

struct ScanLayout {
  size_t recs, carries, erecs, ecarries, groups, egroups, evals, total;
};
ScanLayout scan_layout(int64_t n, bool multinomial);

// Workspace of a block-parallel batch (exact prefix): block prefixes per
// segment, one record per weight block, one sum per exponential block and
// (multinomial) the quantised spacings of every exponential block.
struct SegLayout {
  uint32_t grid_b, grid_e;  // launch bounds on the block counts
  size_t bstart, estart, recs, esums, carries, ecarries, hdr, evals, total;
};
SegLayout seg_layout(int64_t n_total, uint32_t n_filters, bool multinomial);
hipError_t launch_scan_segmented(int scheme, bool f64, const void* w, int64_t n_total,
                                 const int64_t* offsets, uint32_t n_filters, Key key,
                                 uint32_t offset, uint32_t filter_base, int32_t* a, void* ws,
                                 uint32_t* flags, hipStream_t stream);
size_t batch_scan_lds_bytes();

hipError_t launch_scan(int scheme, bool f64, const void* w, int64_t n, Key key, uint32_t offset,
                       uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                       hipStream_t stream);
hipError_t launch_scan_batched(int scheme, bool f64, const void* w, int64_t n_total,
                               const int64_t* offsets, uint32_t n_filters, Key key,
                               uint32_t offset, uint32_t filter_base, int32_t* a, uint32_t* flags,
                               hipStream_t stream);

// Code 5 with independent uniforms (single vectors, exact prefix).
size_t multinomial_iid_workspace_bytes(int64_t n);
hipError_t launch_multinomial_iid(bool f64, const void* w, int64_t n, Key key, uint32_t offset,
                                  uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                                  hipStream_t stream);

// The scaled prefix r = n W_i / W (binary64) of a single vector, exact mode /
// floating-point modes; workspace as scan_layout(n, false).
hipError_t launch_scan_r(bool f64, const void* w, int64_t n, double* r, void* ws, uint32_t* flags,
                         hipStream_t stream);

// Floating-point prefix modes (pfr_precision values 1..3).
enum Prec : int { PREC_F64 = 1, PREC_COMP_F32 = 2, PREC_NAIVE_F32 = 3 };
hipError_t launch_fscan(int scheme, int prec, bool f64, const void* w, int64_t n, Key key,
                        uint32_t offset, uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                        hipStream_t stream);
hipError_t launch_fscan_r(int prec, bool f64, const void* w, int64_t n, double* r, void* ws,
                          uint32_t* flags, hipStream_t stream);
hipError_t launch_fscan_batched(int scheme, int prec, bool f64, const void* w, int64_t n_total,
                                const int64_t* offsets, uint32_t n_filters, Key key,
                                uint32_t offset, uint32_t filter_base, int32_t* a,
                                uint32_t* flags, hipStream_t stream);

// max_len: longest segment (0 = unknown); segments that fit in LDS are staged.
// ws (may be NULL) holds the weight-bound table of a long single vector.
size_t alt_workspace_bytes(bool f64, int64_t n_total, uint32_t n_filters, int64_t max_len);
hipError_t launch_metropolis(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                             uint32_t n_filters, int64_t max_len, int32_t B, const int32_t* B_dev,
                             Key key, uint32_t offset, uint32_t filter_base, int32_t* a, void* ws,
                             size_t ws_bytes, hipStream_t stream);
hipError_t launch_rejection(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                            uint32_t n_filters, int64_t max_len, double w_max,
                            const double* w_max_dev, uint32_t max_trials, Key key,
                            uint32_t offset, uint32_t filter_base, int32_t* a, uint32_t* flags,
                            void* ws, size_t ws_bytes, hipStream_t stream);

size_t o2a_workspace_bytes(int64_t n_total);
hipError_t launch_offspring_to_ancestors(const int32_t* o, int64_t n_total, const int64_t* offsets,
                                         uint32_t n_filters, int32_t* a, void* ws,
                                         uint32_t* flags, hipStream_t stream);
size_t permute_workspace_bytes(int64_t n_total, uint32_t n_filters);
size_t permute_workspace_min_bytes(int64_t n_total);
// The rest of Code 10 after an emission that wrote the claim vector and the
// marked ancestry itself (launch_scan_claimed): the resolve pass over a
// single vector.  permute_claims / permute_marks locate d and e in a
// permutation workspace.
int32_t* permute_claims(void* ws);
int32_t* permute_marks(void* ws, int64_t n_total);
hipError_t launch_resolve(int64_t n_total, int32_t* c, void* ws, uint32_t* flags,
                          hipStream_t stream);
hipError_t launch_scan_claimed(int scheme, bool f64, const void* w, int64_t n, Key key,
                               uint32_t offset, uint32_t filter, int32_t* a, void* ws,
                               uint32_t* flags, int32_t* d, int32_t* e, hipStream_t stream);
// Precondition checks (pfr_check.hip): OR violations into flags (may be null)
// and into the library's per-GPU check word; take_check_word waits for the
// stream, returns the word and clears it.
hipError_t launch_check_weights(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                                uint32_t n_filters, bool use_bound, double bound,
                                const double* bound_dev, uint32_t* flags, hipStream_t stream);
hipError_t launch_check_sorted(const int32_t* a, int64_t n_total, const int64_t* offsets,
                               uint32_t n_filters, uint32_t* flags, hipStream_t stream);
hipError_t take_check_word(hipStream_t stream, uint32_t* out);

hipError_t launch_permute(const int32_t* a, int64_t n_total, const int64_t* offsets,
                          uint32_t n_filters, int64_t max_len, bool sorted, int32_t* c, void* ws,
                          size_t ws_bytes, uint32_t* flags, hipStream_t stream);

// Code 12; max_len as for launch_permute.
hipError_t launch_ancestors_to_offspring(const int32_t* a, int64_t n_total, const int64_t* offsets,
                                         uint32_t n_filters, int64_t max_len, bool sorted,
                                         int32_t* o, uint32_t* flags, hipStream_t stream);
size_t ess_workspace_bytes(int64_t n_total, uint32_t n_filters);
hipError_t launch_ess(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                      uint32_t n_filters, double* ess, void* ws, uint32_t* flags,
                      hipStream_t stream);
hipError_t launch_copy(const int32_t* c, int64_t n_total, const int64_t* offsets,
                       uint32_t n_filters, void* x, size_t elem_bytes, int32_t dim, int64_t ps,
                       int64_t cs, uint32_t* flags, hipStream_t stream);

// Importance weights of partial rejection control (after a rejection launch
// with bound v_max).
hipError_t launch_prc_weights(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                              uint32_t n_filters, double v_max, const double* v_max_dev,
                              const int32_t* a, void* w_out, hipStream_t stream);

hipError_t launch_lgssm_init(int32_t n_filters, int32_t n, double s0, Key key, uint32_t offset,
                             uint32_t filter_base, float* x, float* w, double* logz,
                             int32_t* B_dev, uint32_t* t_dev, int64_t* offsets,
                             hipStream_t stream);
hipError_t launch_lgssm_move(int32_t n_filters, int32_t n, double phi, double q, double r,
                             double log_eps, const double* y, int32_t T, uint32_t* t_dev,
                             Key key, uint32_t offset, uint32_t filter_base, const int32_t* c,
                             float* x, float* w, double* logz, int32_t* B_dev, uint32_t* flags,
                             hipStream_t stream);

hipError_t launch_zero_u32(uint32_t* p, size_t count, hipStream_t stream);

}  // namespace pfr
