// pfr_scan.hip -- the collective resamplers: multinomial (Code 5 of the
// paper), stratified (Code 7) and systematic (Code 8).
//
// All three compute the scaled prefix r_i = n W_i / W_n of the weights and map
// sorted points onto it:
//   stratified   point q_s = s + 1 - u_s in (s, s+1], ancestor = min{i : r_i >= q_s}
//   systematic   the same with one offset u for all strata
//   multinomial  p_k = n S_k / S_n from exponential spacings (sorted uniforms),
//                ancestor = #{i < n-1 : r_i <= p_k}
// which is Code 7/8 followed by Code 11 (and Code 5 with an upper-bound
// search), written point by point so that each output is computed once.
//
// Exact prefix sums.  The paper shows that a float32 prefix sum biases these
// schemes for large n.  Here each block of 1024 weights is quantised to
// integers q = floor(w * 2^s_b) < 2^53 relative to the block maximum (every
// float32 weight within 2^29 of the block maximum is represented exactly),
// block sums are exact 64-bit integers, and the carries between blocks are
// exact 128-bit integers at one global scale.  Integer sums do not depend on
// the order of addition, so the prefix is deterministic, monotone, exactly
// flat across zero weights, and consistent at every block boundary; the only
// rounding is the final conversion r = n * (I / I_total) to binary64.
//
// Passes (single vector): a reduce kernel writes one record per block, and
// its last workgroup (ticket counter) scans the records into carries; the emit
// kernel re-reads the weights, rebuilds r for a tile of 4096 particles in LDS
// and writes every point whose value falls in the tile's r-range, so that
// outputs are written once and coalesced.  Ragged batches run the same steps
// inside one workgroup per filter.
#include "pfr_kernels.h"

namespace pfr {

namespace {

constexpr int kTile = kBlock * kBlocksPerWG;  // particles per emit workgroup
constexpr int kCarryBits = 100;               // carries stay below 2^100

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename T>
struct Blk {
  static constexpr int V = 16 / (int)sizeof(T);  // values per vector load
  static constexpr int G = kBlock / (kWave * V);  // vector loads per lane
};

// ---------------------------------------------------------------- block loads
// Lane l holds, for g = 0..G-1 and v = 0..V-1, element g*64*V + l*V + v of the
// block: every vector load of the wave reads one contiguous kilobyte.
template <typename T>
__device__ __forceinline__ void load_block(const T* __restrict__ w, int64_t n, int64_t base,
                                           T (&x)[16]) {
  constexpr int V = Blk<T>::V, G = Blk<T>::G;
  const int lane = (int)lane_id();
  const bool aligned = ((reinterpret_cast<uintptr_t>(w + base) & 15u) == 0);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int64_t idx = base + (int64_t)g * kWave * V + (int64_t)lane * V;
    if (aligned && idx + V <= n) {
      if constexpr (V == 4) {
        const float4 t = *reinterpret_cast<const float4*>(w + idx);
        x[g * V + 0] = t.x;
        x[g * V + 1] = t.y;
        x[g * V + 2] = t.z;
        x[g * V + 3] = t.w;
      } else {
        const double2 t = *reinterpret_cast<const double2*>(w + idx);
        x[g * V + 0] = t.x;
        x[g * V + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) x[g * V + v] = (idx + v < n) ? w[idx + v] : (T)0;
    }
  }
}

// In-place inclusive prefix of 16 per-lane values in (g, lane, v) order.
template <int G, int V, typename U>
__device__ __forceinline__ U block_inclusive_scan(U (&q)[16]) {
  U run = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    U s = 0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      s += q[g * V + v];
      q[g * V + v] = s;
    }
    const U incl = wave_inclusive_scan(s, OpAdd());
    const U add = run + (incl - s);
#pragma unroll
    for (int v = 0; v < V; ++v) q[g * V + v] += add;
    run += readlane(incl, kWave - 1);
  }
  return run;
}

// ---------------------------------------------------------------- reduce step
// One weight block: validity, reference exponent (block maximum), quantised
// sum.  Returns the record (identical in every lane).
template <typename T>
__device__ BlockRec weight_block_record(const T* __restrict__ w, int64_t n, int64_t base) {
  T x[16];
  load_block(w, n, base, x);
  uint32_t bad = 0;
  int emax = 1;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (!weight_ok(x[i])) bad = FLAG_BAD_WEIGHTS;
    else emax = max(emax, exp_field(x[i]));
  }
  bad = wave_reduce(bad, OpOr());
  emax = (int)wave_reduce((uint32_t)emax, OpMax());
  uint64_t s = 0;
  if (!bad) {
#pragma unroll
    for (int i = 0; i < 16; ++i) s += quantize(x[i], emax);
  }
  s = wave_reduce(s, OpAdd());
  BlockRec r;
  r.sum = s;
  r.scale = scale_of<T>(emax);
  r.bad = bad;
  return r;
}

// Exponential spacing E_k = -log((x + 1/2) 2^-32) for k = 0..n (word k&3 of
// Philox call k>>2 in the exponential domain), quantised to floor(E 2^48).
// Block layout (g, lane, v) with V = 4: Philox call b*256 + g*64 + lane
// supplies the lane's 4 values of group g.
__device__ __forceinline__ void exp_block_values(Key key, uint32_t filter, uint32_t offset,
                                                 int64_t n, uint32_t blk, uint64_t (&q)[16]) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const uint32_t call = blk * 256u + (uint32_t)g * 64u + lane;
    const uint4 x = draw(key, call, DOM_EXP, 0, filter, offset);
    const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t k = (int64_t)call * 4 + v;
      const double e = -log(((double)xs[v] + 0.5) * 0x1p-32);
      q[g * 4 + v] = (k <= n) ? (uint64_t)(e * 0x1p48) : 0ull;
    }
  }
}

__device__ __forceinline__ uint64_t exp_block_sum(Key key, uint32_t filter, uint32_t offset,
                                                  int64_t n, uint32_t blk) {
  uint64_t q[16];
  exp_block_values(key, filter, offset, n, blk, q);
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += q[i];
  return wave_reduce(s, OpAdd());
}

// ---------------------------------------------------------------- carry scan
// Exclusive scan of nb records into C[0..nb] (C[nb] = total) by one
// workgroup of kWGThreads threads.  Weight records are first moved to the
// global scale gscale; exponential records (scale fixed) are used as is.
// Returns the OR of the bad bits and writes gscale.
__device__ __forceinline__ int ceil_log2(uint32_t x) {
  return x <= 1 ? 0 : 32 - __clz(x - 1);
}

template <typename RecLoad>
__device__ void wg_exclusive_scan_u128(uint32_t count, RecLoad load, u128* __restrict__ C,
                                       u128* lds_wave) {
  const int tid = (int)threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const uint32_t per = (count + kWGThreads - 1) / kWGThreads;
  const uint32_t b0 = (uint32_t)tid * per;
  const uint32_t b1 = min(b0 + per, count);
  u128 mine = 0;
  for (uint32_t b = b0; b < b1; ++b) mine += load(b);
  const u128 incl = wave_inclusive_scan(mine, OpAdd());
  if (lane == kWave - 1) lds_wave[wave] = incl;
  __syncthreads();
  u128 run = incl - mine;
  for (int w2 = 0; w2 < wave; ++w2) run += lds_wave[w2];
  for (uint32_t b = b0; b < b1; ++b) {
    C[b] = run;
    run += load(b);
  }
  if (tid == kWGThreads - 1) C[count] = run;
  __syncthreads();
}

template <typename RecArr>
__device__ void scan_weight_records(uint32_t nb, const RecArr recs, u128* __restrict__ C,
                                    u128* lds_wave, int32_t* lds_misc, uint32_t* status_out,
                                    int32_t* gscale_out) {
  const int tid = (int)threadIdx.x;
  // global status and the scale of the largest block
  uint32_t bad = 0;
  int32_t smin = 0x7fffffff;
  for (uint32_t b = tid; b < nb; b += kWGThreads) {
    const BlockRec r = recs[b];
    bad |= r.bad;
    if (r.sum) smin = min(smin, r.scale);
  }
  bad = wave_reduce(bad, OpOr());
  smin = (int32_t)wave_reduce((uint32_t)(smin ^ 0x80000000u), OpMin()) ^ 0x80000000;
  if (tid == 0) {
    lds_misc[0] = 0;
    lds_misc[1] = 0x7fffffff;
  }
  __syncthreads();
  if ((tid % kWave) == 0) {
    atomicOr((uint32_t*)&lds_misc[0], bad);
    atomicMin(&lds_misc[1], smin);
  }
  __syncthreads();
  bad = (uint32_t)lds_misc[0];
  smin = lds_misc[1];
  __syncthreads();
  // every converted block sum is below 2^(63 + gscale - smin); nb of them stay
  // below 2^kCarryBits
  const int32_t gscale = (smin == 0x7fffffff) ? 0 : smin + (kCarryBits - 63) - ceil_log2(nb);
  wg_exclusive_scan_u128(
      nb,
      [&](uint32_t b) -> u128 {
        const BlockRec r = recs[b];
        return shift_u128((u128)r.sum, gscale - r.scale);
      },
      C, lds_wave);
  uint32_t st = bad;
  if (!bad && C[nb] == 0) st |= FLAG_ZERO_TOTAL;
  *status_out = st;
  *gscale_out = gscale;
}

// ---------------------------------------------------------------- r of a block
// r values (binary64) of one weight block, written to r_out[e] in particle
// order, given the block's carry and record.
template <typename T>
__device__ void weight_block_r(const T* __restrict__ w, int64_t n, int64_t base, const BlockRec rec,
                               u128 carry, int32_t gscale, double fQ, double Nd,
                               double* __restrict__ r_out) {
  constexpr int V = Blk<T>::V, G = Blk<T>::G;
  T x[16];
  load_block(w, n, base, x);
  const int emax = 52 + WTraits<T>::BIAS - rec.scale;
  uint64_t q[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) q[i] = quantize(x[i], emax);
  block_inclusive_scan<G, V>(q);
  const int lane = (int)lane_id();
  const int sh = gscale - rec.scale;
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const u128 I = carry + shift_u128((u128)q[g * V + v], sh);
      r_out[g * kWave * V + lane * V + v] = Nd * (u128_to_double(I) / fQ);
    }
  }
}

// ---------------------------------------------------------------- emission
// r >= s + 1 - u, decided exactly: with m = floor(r), true iff m > s, or
// m == s and frac(r) >= 1 - u (both sides exact in binary64).
__device__ __forceinline__ bool reaches(double r, int64_t s, double u) {
  const double mf = floor(r);
  const int64_t m = (int64_t)mf;
  if (m != s) return m > s;
  return (r - mf) >= (1.0 - u);
}

// First i in [0, cnt) with reaches(r[i], s, u) (r non-decreasing); cnt if none.
__device__ __forceinline__ int first_reaching(const double* __restrict__ r, int cnt, int64_t s,
                                              double u) {
  int lo = 0, hi = cnt;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (reaches(r[mid], s, u)) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}
// #{i in [0, cnt) : r[i] <= p}.
__device__ __forceinline__ int count_le(const double* __restrict__ r, int cnt, double p) {
  int lo = 0, hi = cnt;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (r[mid] <= p) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Strata points for a tile whose particles [0, cnt) (local) have r in LDS and
// whose r-range is (r_lo, r_hi]; the last tile of a vector also takes points
// above r_hi (none exist: r_hi = n there).  Outputs a_out[s] = P0 + i.
template <bool SYSTEMATIC>
__device__ void emit_strata(const double* __restrict__ r_lds, int cnt, double r_lo, double r_hi,
                            int64_t n, int64_t P0, Key key, uint32_t filter, uint32_t offset,
                            double u_sys, int32_t* __restrict__ a_out, int tid, int nthreads) {
  if (cnt <= 0 || !(r_hi > r_lo)) return;
  const int64_t s_lo = max((int64_t)0, (int64_t)floor(r_lo) - 1);
  const int64_t s_hi = min(n - 1, (int64_t)floor(r_hi));
  const int64_t c_lo = s_lo >> 2, c_hi = s_hi >> 2;
  for (int64_t c = c_lo + tid; c <= c_hi; c += nthreads) {
    uint32_t xs[4];
    if (!SYSTEMATIC) {
      const uint4 x = draw(key, (uint32_t)c, DOM_STRATA, 0, filter, offset);
      xs[0] = x.x; xs[1] = x.y; xs[2] = x.z; xs[3] = x.w;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t s = c * 4 + v;
      if (s < s_lo || s > s_hi) continue;
      const double u = SYSTEMATIC ? u_sys : u_offset(xs[v]);
      if (reaches(r_lo, s, u)) continue;   // point at or below r_lo: earlier tile
      if (!reaches(r_hi, s, u)) continue;  // point above r_hi: later tile
      a_out[s] = (int32_t)(P0 + first_reaching(r_lds, cnt, s, u));
    }
  }
}

// Multinomial points for a tile with r-range [r_lo, r_hi) (the last tile:
// [r_lo, inf)).  The points p_k = n S_k / S_n come from exponential blocks
// [b_first, b_last], each rebuilt by one wave from its Philox calls and its
// exact carry CE[b].
__device__ void emit_multinomial(const double* __restrict__ r_lds, int cnt, double r_lo,
                                 double r_hi, bool last_tile, int64_t n, int64_t P0, Key key,
                                 uint32_t filter, uint32_t offset, const u128* __restrict__ CE,
                                 uint32_t nbe, int32_t* __restrict__ a_out, int wave, int nwaves) {
  if (cnt <= 0 || !(last_tile || r_hi > r_lo)) return;
  const double Nd = (double)n;
  const double fQE = u128_to_double(CE[nbe]);
  // P(b) = value of the last point of block b-1, b = 1..nbe-1
  auto boundary = [&](uint32_t b) -> double { return Nd * (u128_to_double(CE[b]) / fQE); };
  auto count_below = [&](double x) -> uint32_t {  // #{b in [1, nbe-1] : P(b) < x}
    uint32_t lo = 1, hi = nbe;                    // search in [1, nbe)
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (boundary(mid) < x) lo = mid + 1;
      else hi = mid;
    }
    return lo - 1;
  };
  const uint32_t b_first = count_below(r_lo);
  const uint32_t b_last = last_tile ? nbe - 1 : count_below(r_hi);
  const int lane = (int)lane_id();
  for (uint32_t b = b_first + (uint32_t)wave; b <= b_last; b += (uint32_t)nwaves) {
    uint64_t q[16];
    exp_block_values(key, filter, offset, n, b, q);
    block_inclusive_scan<4, 4>(q);
    const u128 carry = CE[b];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t k = (int64_t)b * kBlock + g * 256 + lane * 4 + v;
        if (k >= n) continue;
        const double p = Nd * (u128_to_double(carry + (u128)q[g * 4 + v]) / fQE);
        if (p < r_lo) continue;
        if (!last_tile && !(p < r_hi)) continue;
        int64_t anc = P0 + count_le(r_lds, cnt, p);
        if (anc > n - 1) anc = n - 1;
        a_out[k] = (int32_t)anc;
      }
    }
  }
}

// ---------------------------------------------------------------- kernels
template <typename T, bool MULTI>
__global__ __launch_bounds__(kWGThreads) void k_scan_reduce(const T* __restrict__ w, int64_t n,
                                                            uint32_t nb, uint32_t nbe,
                                                            uint32_t wg_weights, Key key,
                                                            uint32_t offset, uint32_t filter,
                                                            ScanHeader* __restrict__ hdr,
                                                            BlockRec* __restrict__ recs,
                                                            uint64_t* __restrict__ erecs,
                                                            u128* __restrict__ C,
                                                            u128* __restrict__ CE) {
  __shared__ u128 lds_wave[kBlocksPerWG];
  __shared__ int32_t lds_misc[4];
  const int wave = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  if (blockIdx.x < wg_weights) {
    const uint32_t blk = blockIdx.x * kBlocksPerWG + wave;
    if (blk < nb) {
      const BlockRec r = weight_block_record(w, n, (int64_t)blk * kBlock);
      if (lane == 0) recs[blk] = r;
    }
  } else if (MULTI) {
    const uint32_t blk = (blockIdx.x - wg_weights) * kBlocksPerWG + wave;
    if (blk < nbe) {
      const uint64_t s = exp_block_sum(key, filter, offset, n, blk);
      if (lane == 0) erecs[blk] = s;
    }
  }
  // the last workgroup to finish scans every record into carries
  __shared__ uint32_t is_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t prev = atomicAdd(&hdr->ticket, 1u);
    is_last = (prev == gridDim.x - 1) ? 1u : 0u;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  uint32_t status = 0;
  int32_t gscale = 0;
  scan_weight_records(nb, recs, C, lds_wave, lds_misc, &status, &gscale);
  if (MULTI) {
    wg_exclusive_scan_u128(
        nbe, [&](uint32_t b) -> u128 { return (u128)erecs[b]; }, CE, lds_wave);
  }
  if (threadIdx.x == 0) {
    hdr->status = status;
    hdr->gscale = gscale;
    hdr->nb = nb;
    hdr->nbe = nbe;
    hdr->ticket = 0;
  }
}

template <typename T, int SCHEME>
__global__ __launch_bounds__(kWGThreads) void k_scan_emit(const T* __restrict__ w, int64_t n,
                                                          uint32_t nb, uint32_t nbe, Key key,
                                                          uint32_t offset, uint32_t filter,
                                                          const ScanHeader* __restrict__ hdr,
                                                          const BlockRec* __restrict__ recs,
                                                          const u128* __restrict__ C,
                                                          const u128* __restrict__ CE,
                                                          int32_t* __restrict__ a,
                                                          uint32_t* __restrict__ flags) {
  __shared__ double r_lds[kTile];
  const int tid = (int)threadIdx.x, wave = tid / kWave;
  const uint32_t status = hdr->status;
  const int64_t P0 = (int64_t)blockIdx.x * kTile;
  const int64_t P1 = min(P0 + kTile, n);
  if (flags && blockIdx.x == 0 && tid == 0 && status) atomicOr(flags, status);
  if (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    for (int64_t i = P0 + tid; i < P1; i += kWGThreads) a[i] = (int32_t)i;
    return;
  }
  const int32_t gscale = hdr->gscale;
  const double fQ = u128_to_double(C[nb]);
  const double Nd = (double)n;
  const uint32_t blk = blockIdx.x * kBlocksPerWG + wave;
  if (blk < nb)
    weight_block_r(w, n, (int64_t)blk * kBlock, recs[blk], C[blk], gscale, fQ, Nd,
                   r_lds + wave * kBlock);
  __syncthreads();
  const uint32_t b0 = blockIdx.x * kBlocksPerWG;
  const uint32_t b_end = min(b0 + kBlocksPerWG, nb);
  const double r_lo = Nd * (u128_to_double(C[b0]) / fQ);
  const double r_hi = Nd * (u128_to_double(C[b_end]) / fQ);
  const int cnt = (int)(P1 - P0);
  if (SCHEME == SCHEME_MULTINOMIAL) {
    emit_multinomial(r_lds, cnt, r_lo, r_hi, P1 == n, n, P0, key, filter, offset, CE, nbe, a,
                     wave, kBlocksPerWG);
  } else {
    double u_sys = 0.0;
    if (SCHEME == SCHEME_SYSTEMATIC) u_sys = u_offset(draw(key, 0, DOM_STRATA, 0, filter, offset).x);
    emit_strata<SCHEME == SCHEME_SYSTEMATIC>(r_lds, cnt, r_lo, r_hi, n, P0, key, filter, offset,
                                             u_sys, a, tid, kWGThreads);
  }
}

// Ragged batch: one workgroup per filter runs the reduce, the carry scan and
// the emission for its own segment, with the records in LDS.
constexpr int kBatchMaxBlocks = 256;  // filters up to 2^18 particles

struct BatchLds {
  double r[kTile];
  BlockRec recs[kBatchMaxBlocks];
  u128 C[kBatchMaxBlocks + 1];
  uint64_t erecs[kBatchMaxBlocks + 1];
  u128 CE[kBatchMaxBlocks + 2];
  u128 wave_tot[kBlocksPerWG];
  int32_t misc[4];
  uint32_t status;
  int32_t gscale;
};

template <typename T, int SCHEME>
__global__ __launch_bounds__(kWGThreads) void k_scan_batched(const T* __restrict__ w,
                                                             int64_t n_total,
                                                             const int64_t* __restrict__ offsets,
                                                             uint32_t n_filters, Key key,
                                                             uint32_t offset, uint32_t filter_base,
                                                             int32_t* __restrict__ a,
                                                             uint32_t* __restrict__ flags) {
  __shared__ BatchLds L;
  const uint32_t f = blockIdx.x;
  if (f >= n_filters) return;
  const int tid = (int)threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int64_t base = offsets ? offsets[f] : 0;
  const int64_t n = offsets ? offsets[f + 1] - base : n_total;
  if (n <= 0) return;
  const T* __restrict__ ws = w + base;
  int32_t* __restrict__ as = a + base;
  const uint32_t filt = filter_base + f;
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  const uint32_t nbe = (uint32_t)((n + 1 + kBlock - 1) / kBlock);
  if (nbe > kBatchMaxBlocks) {  // segment too long for this path: identity + flag
    for (int64_t i = tid; i < n; i += kWGThreads) as[i] = (int32_t)i;
    if (tid == 0 && flags) atomicOr(flags, FLAG_BAD_COUNTS);
    return;
  }
  for (uint32_t b = wave; b < nb; b += kBlocksPerWG) {
    const BlockRec r = weight_block_record(ws, n, (int64_t)b * kBlock);
    if (lane == 0) L.recs[b] = r;
  }
  if (SCHEME == SCHEME_MULTINOMIAL) {
    for (uint32_t b = wave; b < nbe; b += kBlocksPerWG) {
      const uint64_t s = exp_block_sum(key, filt, offset, n, b);
      if (lane == 0) L.erecs[b] = s;
    }
  }
  __syncthreads();
  uint32_t status = 0;
  int32_t gscale = 0;
  scan_weight_records(nb, L.recs, L.C, L.wave_tot, L.misc, &status, &gscale);
  if (SCHEME == SCHEME_MULTINOMIAL)
    wg_exclusive_scan_u128(
        nbe, [&](uint32_t b) -> u128 { return (u128)L.erecs[b]; }, L.CE, L.wave_tot);
  __syncthreads();
  if (flags && tid == 0 && status) atomicOr(flags, status);
  if (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    for (int64_t i = tid; i < n; i += kWGThreads) as[i] = (int32_t)i;
    return;
  }
  const double fQ = u128_to_double(L.C[nb]);
  const double Nd = (double)n;
  double u_sys = 0.0;
  if (SCHEME == SCHEME_SYSTEMATIC) u_sys = u_offset(draw(key, 0, DOM_STRATA, 0, filt, offset).x);
  const uint32_t ntiles = (uint32_t)((n + kTile - 1) / kTile);
  for (uint32_t t = 0; t < ntiles; ++t) {
    const uint32_t blk = t * kBlocksPerWG + wave;
    if (blk < nb)
      weight_block_r(ws, n, (int64_t)blk * kBlock, L.recs[blk], L.C[blk], gscale, fQ, Nd,
                     L.r + wave * kBlock);
    __syncthreads();
    const int64_t P0 = (int64_t)t * kTile;
    const int64_t P1 = min(P0 + kTile, n);
    const uint32_t b0 = t * kBlocksPerWG;
    const uint32_t b_end = min(b0 + kBlocksPerWG, nb);
    const double r_lo = Nd * (u128_to_double(L.C[b0]) / fQ);
    const double r_hi = Nd * (u128_to_double(L.C[b_end]) / fQ);
    const int cnt = (int)(P1 - P0);
    if (SCHEME == SCHEME_MULTINOMIAL) {
      emit_multinomial(L.r, cnt, r_lo, r_hi, P1 == n, n, P0, key, filt, offset, L.CE, nbe, as,
                       wave, kBlocksPerWG);
    } else {
      emit_strata<SCHEME == SCHEME_SYSTEMATIC>(L.r, cnt, r_lo, r_hi, n, P0, key, filt, offset,
                                               u_sys, as, tid, kWGThreads);
    }
    __syncthreads();
  }
}

template <typename T, int SCHEME>
hipError_t launch_scan_t(const void* wv, int64_t n, Key key, uint32_t offset, uint32_t filter,
                         int32_t* a, void* ws, uint32_t* flags, hipStream_t stream) {
  const T* w = (const T*)wv;
  const bool multi = SCHEME == SCHEME_MULTINOMIAL;
  const ScanLayout L = scan_layout(n, multi);
  char* base = (char*)ws;
  ScanHeader* hdr = (ScanHeader*)base;
  BlockRec* recs = (BlockRec*)(base + L.recs);
  u128* C = (u128*)(base + L.carries);
  uint64_t* erecs = (uint64_t*)(base + L.erecs);
  u128* CE = (u128*)(base + L.ecarries);
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  const uint32_t nbe = multi ? (uint32_t)((n + 1 + kBlock - 1) / kBlock) : 0u;
  const uint32_t wg_w = (nb + kBlocksPerWG - 1) / kBlocksPerWG;
  const uint32_t wg_e = (nbe + kBlocksPerWG - 1) / kBlocksPerWG;
  if (multi)
    hipLaunchKernelGGL((k_scan_reduce<T, true>), dim3(wg_w + wg_e), dim3(kWGThreads), 0, stream, w,
                       n, nb, nbe, wg_w, key, offset, filter, hdr, recs, erecs, C, CE);
  else
    hipLaunchKernelGGL((k_scan_reduce<T, false>), dim3(wg_w), dim3(kWGThreads), 0, stream, w, n,
                       nb, nbe, wg_w, key, offset, filter, hdr, recs, erecs, C, CE);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t tiles = (uint32_t)((n + kTile - 1) / kTile);
  hipLaunchKernelGGL((k_scan_emit<T, SCHEME>), dim3(tiles), dim3(kWGThreads), 0, stream, w, n, nb,
                     nbe, key, offset, filter, hdr, recs, C, CE, a, flags);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scan_scheme(int scheme, const void* w, int64_t n, Key key, uint32_t offset,
                              uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                              hipStream_t stream) {
  switch (scheme) {
    case SCHEME_MULTINOMIAL:
      return launch_scan_t<T, SCHEME_MULTINOMIAL>(w, n, key, offset, filter, a, ws, flags, stream);
    case SCHEME_STRATIFIED:
      return launch_scan_t<T, SCHEME_STRATIFIED>(w, n, key, offset, filter, a, ws, flags, stream);
    default:
      return launch_scan_t<T, SCHEME_SYSTEMATIC>(w, n, key, offset, filter, a, ws, flags, stream);
  }
}

template <typename T>
hipError_t launch_batched_scheme(int scheme, const void* w, int64_t n_total, const int64_t* offsets,
                                 uint32_t n_filters, Key key, uint32_t offset,
                                 uint32_t filter_base, int32_t* a, uint32_t* flags,
                                 hipStream_t stream) {
  const T* wt = (const T*)w;
  switch (scheme) {
    case SCHEME_MULTINOMIAL:
      hipLaunchKernelGGL((k_scan_batched<T, SCHEME_MULTINOMIAL>), dim3(n_filters),
                         dim3(kWGThreads), 0, stream, wt, n_total, offsets, n_filters, key, offset,
                         filter_base, a, flags);
      break;
    case SCHEME_STRATIFIED:
      hipLaunchKernelGGL((k_scan_batched<T, SCHEME_STRATIFIED>), dim3(n_filters),
                         dim3(kWGThreads), 0, stream, wt, n_total, offsets, n_filters, key, offset,
                         filter_base, a, flags);
      break;
    default:
      hipLaunchKernelGGL((k_scan_batched<T, SCHEME_SYSTEMATIC>), dim3(n_filters),
                         dim3(kWGThreads), 0, stream, wt, n_total, offsets, n_filters, key, offset,
                         filter_base, a, flags);
      break;
  }
  return hipGetLastError();
}

}  // namespace

ScanLayout scan_layout(int64_t n, bool multinomial) {
  const size_t nb = (size_t)((n + kBlock - 1) / kBlock);
  const size_t nbe = multinomial ? (size_t)((n + 1 + kBlock - 1) / kBlock) : 0;
  ScanLayout L;
  L.recs = 256;
  L.carries = L.recs + align256(nb * sizeof(BlockRec));
  L.erecs = L.carries + align256((nb + 1) * sizeof(u128));
  L.ecarries = L.erecs + align256(nbe * sizeof(uint64_t));
  L.total = L.ecarries + align256((nbe + 1) * sizeof(u128));
  return L;
}

size_t batch_scan_lds_bytes() { return sizeof(BatchLds); }

hipError_t launch_scan(int scheme, bool f64, const void* w, int64_t n, Key key, uint32_t offset,
                       uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                       hipStream_t stream) {
  return f64 ? launch_scan_scheme<double>(scheme, w, n, key, offset, filter, a, ws, flags, stream)
             : launch_scan_scheme<float>(scheme, w, n, key, offset, filter, a, ws, flags, stream);
}

hipError_t launch_scan_batched(int scheme, bool f64, const void* w, int64_t n_total,
                               const int64_t* offsets, uint32_t n_filters, Key key,
                               uint32_t offset, uint32_t filter_base, int32_t* a, uint32_t* flags,
                               hipStream_t stream) {
  return f64 ? launch_batched_scheme<double>(scheme, w, n_total, offsets, n_filters, key, offset,
                                             filter_base, a, flags, stream)
             : launch_batched_scheme<float>(scheme, w, n_total, offsets, n_filters, key, offset,
                                            filter_base, a, flags, stream);
}

}  // namespace pfr
