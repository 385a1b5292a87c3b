// pfr_alt.hip -- the collective-free resamplers: Metropolis (Code 2 of the
// paper) and rejection (Code 3), one lane per particle on a counter-based
// Philox stream.
//
// Lane results depend only on (particle, step/trial, filter, offset) through
// the Philox counter, never on which lane or wave did the work, so every
// launch shape gives the same bits.
#include "pfr_kernels.h"
#include <cstring>

namespace pfr {

// Per-particle context for ragged batches: where the particle's segment starts
// and how long it is.  A single vector is one segment.
struct SegCtx {
  int64_t base;
  uint32_t n;
  uint32_t f;
};

__device__ __forceinline__ SegCtx seg_of(const int64_t* __restrict__ offsets, uint32_t n_filters,
                                         int64_t n_total, int64_t g) {
  SegCtx c;
  if (!offsets) {
    c.base = 0;
    c.n = (uint32_t)n_total;
    c.f = 0;
  } else {
    c.f = find_segment(offsets, n_filters, g);
    c.base = offsets[c.f];
    c.n = (uint32_t)(offsets[c.f + 1] - c.base);
  }
  return c;
}

// ------------------------------------------------------------------ Metropolis
// Lane i runs B steps of an independent Metropolis chain started at k = i.
// Step s takes (j, u) from words 3s, 3s+1, 3s+2 of the lane's Philox stream
// (word m = word m&3 of counter (i, TRIAL<<28 | m>>2, filter, offset)) and
// moves to j when u * w_k <= w_j.  The proposals and their weight loads do not
// depend on the chain state: a group of 4 steps takes 3 Philox calls and
// issues its 4 gathers at once, and the gathers of group m+1 are in flight
// while the accept decisions of group m run in order (two register sets, used
// alternately, so that no load has to complete before it is consumed).
struct MGroup {
  uint32_t j[4];
  uint32_t u[4];
  double wj[4];
  int nq;
};

// pl: the lane's Philox parts for particle i (philox_lane); the step number,
// filter and offset are the same on every lane of the wave.
template <typename T>
__device__ __forceinline__ void metropolis_fetch(const T* __restrict__ ws, Key key, uint32_t i,
                                                 const PhiloxLane& pl, uint32_t filt,
                                                 uint32_t offset, uint32_t n, int32_t steps,
                                                 int32_t m, MGroup& g) {
  uint32_t x[12];
  const int32_t left = steps - 4 * m;
  const int ncall = left >= 4 ? 3 : (3 * left + 3) / 4;
#pragma unroll
  for (int c3 = 0; c3 < 3; ++c3) {
    if (c3 < ncall) {
      const uint4 v = philox_lane_call(pl, key, DOM_TRIAL, (uint32_t)(3 * m + c3), filt, offset);
      x[4 * c3 + 0] = v.x;
      x[4 * c3 + 1] = v.y;
      x[4 * c3 + 2] = v.z;
      x[4 * c3 + 3] = v.w;
    }
  }
  g.nq = left >= 4 ? 4 : left;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    g.j[q] = q < g.nq ? index_draw(x[3 * q], x[3 * q + 1], n) : i;
    g.u[q] = x[3 * q + 2];
    g.wj[q] = (double)ws[g.j[q]];
  }
}

template <typename T>
__device__ __forceinline__ void metropolis_accept(const MGroup& g, uint32_t& k, double& wk) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < g.nq && accept_exact<T>(u_accept(g.u[q]), wk, g.wj[q])) {
      k = g.j[q];
      wk = g.wj[q];
    }
  }
}

// A workgroup takes the particles [p0, p1) of the global array (chunk per
// workgroup) and walks the segments that overlap them; a segment of at most
// CAP weights is first copied into LDS, so that every random weight load of
// its chains is an LDS read.  Longer segments load from global memory, with
// the gathers of the next group of steps in flight while the current group
// is decided.  The chains do not depend on the launch shape.
template <typename T>
__device__ __forceinline__ void stage_weights(const T* __restrict__ w, uint32_t n, T* sw) {
  for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) sw[k] = w[k];
}

template <typename T>
__device__ __forceinline__ uint32_t metropolis_chain(const T* ws, Key key, uint32_t i,
                                                     uint32_t filt, uint32_t offset, uint32_t n,
                                                     int32_t steps) {
  uint32_t k = i;
  double wk = (double)ws[i];
  const PhiloxLane pl = philox_lane(key, i, filt, offset);
  const int32_t groups = (steps + 3) / 4;
  for (int32_t m = 0; m < groups; ++m) {
    MGroup g;
    metropolis_fetch(ws, key, i, pl, filt, offset, n, steps, m, g);
    metropolis_accept<T>(g, k, wk);
  }
  return k;
}

template <typename T, int CAP, int THREADS>
__global__ __launch_bounds__(THREADS) void k_metropolis_staged(
    const T* __restrict__ w, int64_t n_total, const int64_t* __restrict__ offsets,
    uint32_t n_filters, int32_t B, const int32_t* __restrict__ B_dev, Key key, uint32_t offset,
    uint32_t filter_base, int32_t* __restrict__ a, int64_t chunk, int64_t min_len,
    int64_t max_len) {
  __shared__ T sw[CAP > 0 ? CAP : 1];
  offset = counter_offset(key, offset);
  const int64_t p0 = (int64_t)blockIdx.x * chunk;
  const int64_t p1 = p0 + chunk < n_total ? p0 + chunk : n_total;
  uint32_t f = offsets ? find_segment(offsets, n_filters, p0) : 0u;
  for (int64_t g0 = p0; g0 < p1; ++f) {
    const int64_t base = offsets ? offsets[f] : 0;
    const int64_t end = offsets ? offsets[f + 1] : n_total;
    const int64_t q1 = end < p1 ? end : p1;
    if (q1 <= g0) continue;  // empty segment
    const uint32_t n = (uint32_t)(end - base);
    if (end - base < min_len || end - base > max_len) {  // another launch runs this segment
      g0 = q1;
      continue;
    }
    const int32_t steps = B_dev ? B_dev[f] : B;
    const uint32_t filt = filter_base + f;
    if (CAP > 0 && n <= (uint32_t)CAP) {
      __syncthreads();  // the previous segment's chains are done with sw
      stage_weights(w + base, n, sw);
      __syncthreads();
      for (int64_t g = g0 + threadIdx.x; g < q1; g += THREADS)
        a[g] = (int32_t)metropolis_chain(sw, key, (uint32_t)(g - base), filt, offset, n, steps);
    } else if (CAP > 0) {  // a long segment in a staged launch: plain chains
      for (int64_t g = g0 + threadIdx.x; g < q1; g += THREADS)
        a[g] = (int32_t)metropolis_chain(w + base, key, (uint32_t)(g - base), filt, offset, n,
                                         steps);
    } else {
      for (int64_t g = g0 + threadIdx.x; g < q1; g += THREADS) {
        const uint32_t i = (uint32_t)(g - base);
        const T* __restrict__ ws = w + base;
        uint32_t k = i;
        double wk = (double)ws[i];
        const int32_t groups = (steps + 3) / 4;
        const PhiloxLane pl = philox_lane(key, i, filt, offset);
        MGroup ga, gb;
        if (groups > 0) metropolis_fetch(ws, key, i, pl, filt, offset, n, steps, 0, ga);
        for (int32_t m = 0; m < groups; m += 2) {
          if (m + 1 < groups)
            metropolis_fetch(ws, key, i, pl, filt, offset, n, steps, m + 1, gb);
          metropolis_accept<T>(ga, k, wk);
          if (m + 2 < groups)
            metropolis_fetch(ws, key, i, pl, filt, offset, n, steps, m + 2, ga);
          if (m + 1 < groups) metropolis_accept<T>(gb, k, wk);
        }
        a[g] = (int32_t)k;
      }
    }
    g0 = q1;
  }
}

// ------------------------------------------------------------------ bound table
// For a vector too long for LDS, an upper bound of the weights, one per bucket
// of S = 2^shift consecutive particles, lets most proposals be rejected
// without loading w_j: if u * w_k > ub >= w_j the step (or trial) rejects.
// The bound is a power of two, 2^(cM - 127 - c4): cM is the largest bucket
// code of the vector and c4 = min(15, cM - c) the 4-bit distance of the
// bucket's code c, where 2^(c - 127) >= the bucket maximum.  Two buckets per
// LDS byte: 128 KB cover 2^18 buckets.  The skip test compares the rounded
// product u * (a lower bound of w_k) with ub with a margin of 2^-20 relative,
// far above the product's rounding, so a skipped step is one that the exact
// test rejects; the output is the same.
constexpr int kTableBuckets = 1 << 18;  // nibbles in LDS (128 KB)
constexpr int kTableThreads = 1024;
constexpr int kCodeThreads = 256;

__device__ __forceinline__ uint32_t bound_code(float v) {
  const uint32_t b = __float_as_uint(v);
  return (b >> 23) + ((b & 0x7FFFFFu) != 0u);  // 0 .. 255 for finite v >= 0
}
__device__ __forceinline__ uint32_t bound_code(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const int e = (int)((b >> 52) & 0x7FF);
  if (e == 0) return 0u;  // zero or below 2^-1022
  const int c = e - 1023 + 127 + (((b & 0xFFFFFFFFFFFFFull) != 0ull) ? 1 : 0);
  return c < 0 ? 0u : (c > 255 ? 255u : (uint32_t)c);
}

// One thread per bucket: its 8-bit code; per workgroup the largest code.
// Invalid weights (negative, non-finite) give code 255, which disables the
// skips of the vector (the kernels then load every weight).
template <typename T>
__global__ __launch_bounds__(kCodeThreads) void k_bound_codes(const T* __restrict__ w, int64_t n,
                                                              int shift,
                                                              uint8_t* __restrict__ codes,
                                                              uint32_t* __restrict__ wg_max) {
  __shared__ uint32_t slot[kCodeThreads / kWave];
  const int64_t b = (int64_t)blockIdx.x * kCodeThreads + threadIdx.x;
  const int64_t S = (int64_t)1 << shift;
  uint32_t c = 0;
  if ((b << shift) < n) {
    const int64_t e = ((b + 1) << shift) < n ? ((b + 1) << shift) : n;
    for (int64_t k = b << shift; k < e; ++k) {
      const T v = w[k];
      const uint32_t ck = weight_ok(v) ? bound_code(v) : 255u;
      c = ck > c ? ck : c;
    }
    codes[b] = (uint8_t)c;
  }
  (void)S;
  c = wave_reduce(c, OpMax());
  if (lane_id() == 0) slot[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = slot[0];
    for (int k = 1; k < kCodeThreads / kWave; ++k) m = slot[k] > m ? slot[k] : m;
    wg_max[blockIdx.x] = m;
  }
}

struct BoundTable {
  const uint8_t* nib;  // LDS, two 4-bit codes per byte
  int shift;
  // high word of the binary64 bound 2^(cM - 127) of the largest bucket, or
  // 0xFFFFFFFF when the table is unusable (no product exceeds it)
  uint32_t hi_top;
  // bucket b = j >> shift sits in byte b >> 1, low nibble for even b; the
  // nibble's bit offset 4 (b & 1) is bit `shift` of j moved to bit 2
  // (shift >= 2)
  __device__ __forceinline__ uint32_t c4(uint32_t j) const {
    return __builtin_amdgcn_ubfe((uint32_t)nib[j >> (shift + 1)], (j >> (shift - 2)) & 4u, 4u);
  }
  // true when u * lb > ub(j) = 2^(cM - 127 - c4), i.e. u * w_k > w_j for every
  // w_k >= lb.  The test reads only the high word of p = fl(u * lb) (the same
  // product the exact accept test forms): high(p) > high(ub) means
  // p >= ub (1 + 2^-20), and since p exceeds u * lb by at most a factor
  // 1 + 2^-53, u * lb > ub follows.  Adding c4 << 20 to high(p) instead of
  // subtracting it from the exponent of ub keeps the test to two integer
  // instructions; neither side wraps (high(p) < 2^31).
  __device__ __forceinline__ bool rejects(double u, double lb, uint32_t j) const {
    const uint32_t hp = (uint32_t)((uint64_t)__double_as_longlong(u * lb) >> 32);
    return hp + (c4(j) << 20) > hi_top;
  }
};

// The 4-bit table, packed once per call: every workgroup takes the largest
// code from the per-workgroup maxima of k_bound_codes, each thread packs 8
// codes into one word (the code array is padded to a multiple of 8; the
// padding is never looked up), and workgroup 0 stores the largest code.
constexpr int kPackThreads = 256;

__global__ __launch_bounds__(kPackThreads) void k_pack_table(const uint8_t* __restrict__ codes,
                                                             const uint32_t* __restrict__ wg_max,
                                                             uint32_t n_wg, uint32_t nb,
                                                             uint32_t* __restrict__ nib,
                                                             uint32_t* __restrict__ cm_out) {
  __shared__ uint32_t slot[kPackThreads / kWave];
  uint32_t m = 0;
  for (uint32_t k = threadIdx.x; k < n_wg; k += kPackThreads) m = wg_max[k] > m ? wg_max[k] : m;
  m = wave_reduce(m, OpMax());
  if (lane_id() == 0) slot[threadIdx.x / kWave] = m;
  __syncthreads();
  uint32_t cM = slot[0];
  for (int k = 1; k < kPackThreads / kWave; ++k) cM = slot[k] > cM ? slot[k] : cM;
  const uint32_t p = blockIdx.x * kPackThreads + threadIdx.x;
  if (8 * p < nb) {
    const uint2 v = reinterpret_cast<const uint2*>(codes)[p];
    uint32_t packed = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint32_t c = ((q < 4 ? v.x : v.y) >> (8 * (q & 3))) & 0xFFu;
      const uint32_t d = c > cM ? 15u : (cM - c > 15u ? 15u : cM - c);
      packed |= d << (4 * q);
    }
    nib[p] = packed;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *cm_out = cM;
}

// The rejection table in one pass, without the vector's largest code: the
// distances are taken from c_ref, the code of the caller's w_max, which
// bounds every valid weight.  A bucket whose code reaches c_ref (or whose
// weights are invalid, code 255) gets distance 0, i.e. the bound
// 2^(c_ref - 127) >= w_max, which no trial's u * w_max exceeds: it is never
// skipped, and the exact test decides as without the table.  One thread per
// bucket; eight lanes OR their nibbles into one word, stored by the first.
template <typename T>
__global__ __launch_bounds__(kCodeThreads) void k_bound_nibbles(const T* __restrict__ w,
                                                                int64_t n, int shift, uint32_t nb,
                                                                uint32_t c_ref,
                                                                uint32_t* __restrict__ nib,
                                                                uint32_t* __restrict__ cm_out) {
  const int64_t b = (int64_t)blockIdx.x * kCodeThreads + threadIdx.x;
  uint32_t d = 0;
  if (b < (int64_t)nb) {
    const int64_t e = ((b + 1) << shift) < n ? ((b + 1) << shift) : n;
    uint32_t c = 0;
    for (int64_t k = b << shift; k < e; ++k) {
      const T v = w[k];
      const uint32_t ck = weight_ok(v) ? bound_code(v) : 255u;
      c = ck > c ? ck : c;
    }
    d = c >= c_ref ? 0u : (c_ref - c > 15u ? 15u : c_ref - c);
  }
  uint32_t word = d << (4 * (threadIdx.x & 7u));
  word |= __shfl_xor(word, 1);
  word |= __shfl_xor(word, 2);
  word |= __shfl_xor(word, 4);
  if ((threadIdx.x & 7u) == 0 && b < (int64_t)nb) nib[b >> 3] = word;
  if (blockIdx.x == 0 && threadIdx.x == 0) *cm_out = c_ref;
}

// Workgroup prologue: the packed table copied into LDS with 16-byte loads (the
// packed array is padded to a multiple of 16 bytes).
__device__ BoundTable load_bound_table(const uint32_t* __restrict__ nib_g,
                                       const uint32_t* __restrict__ cm, uint32_t nb, int shift,
                                       uint8_t* nib) {
  const uint32_t n4 = (nb + 31) / 32;  // 16-byte pieces (32 nibbles each)
  const uint4* __restrict__ src = reinterpret_cast<const uint4*>(nib_g);
  uint4* dst = reinterpret_cast<uint4*>(nib);
  for (uint32_t p = threadIdx.x; p < n4; p += blockDim.x) dst[p] = src[p];
  const uint32_t cM = *cm;
  __syncthreads();
  BoundTable t;
  t.nib = nib;
  t.shift = shift;
  // 2^(cM - 127) has binary64 exponent field cM - 127 + 1023 = cM + 896
  t.hi_top = cM < 255u ? (cM + 896u) << 20 : 0xFFFFFFFFu;
  return t;
}

// Metropolis with the bound table.  A skip needs the exact current w_k, so
// the gathers cannot be issued ahead of the decisions of earlier steps;
// instead each lane runs K independent chains in lockstep: at every step the
// chains whose proposal the table cannot reject issue their loads together
// and the K decisions follow.  Particles of the chunk: lane l runs
// p0 + l + c * kTableThreads for c < K.
template <typename T, int K>
__global__ __launch_bounds__(kTableThreads) void k_metropolis_table(
    const T* __restrict__ w, int64_t n, int32_t B, Key key, uint32_t offset, uint32_t filter,
    int32_t* __restrict__ a, int64_t chunk, const uint32_t* __restrict__ nib_g,
    const uint32_t* __restrict__ cm, uint32_t nb, int shift) {
  __shared__ __align__(16) uint8_t nib[kTableBuckets / 2];
  offset = counter_offset(key, offset);
  const BoundTable tab = load_bound_table(nib_g, cm, nb, shift, nib);
  // n * sizeof(T) < 2^31 (checked by the launcher)
  const __amdgpu_buffer_rsrc_t wv = buffer_view(w, (uint32_t)(n * (int64_t)sizeof(T)));
  const int64_t p0 = (int64_t)blockIdx.x * chunk;
  const int64_t p1 = p0 + chunk < n ? p0 + chunk : n;
  for (int64_t gb = p0 + threadIdx.x; gb < p1; gb += (int64_t)K * kTableThreads) {
    uint32_t idx[K], k[K];
    double wk[K];
    bool live[K];
    PhiloxLane pl[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const int64_t g = gb + (int64_t)c * kTableThreads;
      live[c] = g < p1;
      idx[c] = (uint32_t)(live[c] ? g : gb);
      k[c] = idx[c];
      wk[c] = (double)w[idx[c]];
      pl[c] = philox_lane(key, idx[c], filter, offset);
    }
    for (int32_t m = 0; 4 * m < B; ++m) {
      const int32_t left = B - 4 * m;
      const int ncall = left >= 4 ? 3 : (3 * left + 3) / 4;
      const int nq = left >= 4 ? 4 : left;
      uint32_t x[K][12];
#pragma unroll
      for (int c = 0; c < K; ++c) {
#pragma unroll
        for (int c3 = 0; c3 < 3; ++c3) {
          if (c3 < ncall) {
            // step, filter and offset are the same on every lane (one vector)
            const uint4 v =
                philox_lane_call(pl[c], key, DOM_TRIAL, (uint32_t)(3 * m + c3), filter, offset);
            x[c][4 * c3 + 0] = v.x;
            x[c][4 * c3 + 1] = v.y;
            x[c][4 * c3 + 2] = v.z;
            x[c][4 * c3 + 3] = v.w;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < nq) {
          uint32_t j[K];
          double u[K], v[K];
          bool need[K];
#pragma unroll
          for (int c = 0; c < K; ++c) {
            j[c] = index_draw(x[c][3 * q], x[c][3 * q + 1], (uint32_t)n);
            u[c] = u_accept(x[c][3 * q + 2]);
            // a dead chain (past the chunk end) runs a copy of chain gb and is not stored
            need[c] = !tab.rejects(u[c], wk[c], j[c]);
          }
          // the K gathers go out together; lanes with nothing to load read zero
#pragma unroll
          for (int c = 0; c < K; ++c)
            v[c] = (double)buffer_gather<T>(wv, need[c] ? j[c] * (uint32_t)sizeof(T) : kNoLoad);
#pragma unroll
          for (int c = 0; c < K; ++c) {
            // selects, not a branch: the gathered value is used on every lane,
            // so the gathers cannot be sunk into per-chain branches
            const bool acc = need[c] & accept_exact<T>(u[c], wk[c], v[c]);
            k[c] = acc ? j[c] : k[c];
            wk[c] = acc ? v[c] : wk[c];
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < K; ++c)
      if (live[c]) a[gb + (int64_t)c * kTableThreads] = (int32_t)k[c];
  }
}

// ------------------------------------------------------------------ rejection
// Particle i: trial 0 proposes j = i; trial t >= 1 proposes j from Philox
// counter (i, TRIAL<<28 | t, filter, offset); every trial takes its u from the
// same block.  The first trial with u * w_max <= w_j wins.  After max_trials
// rejections the particle keeps a_i = i and FLAG_TRIAL_CAP is raised.
//
// Scheduling (the variable task-length problem of the paper's section 2.2):
// every wave owns a contiguous range of particles.  While the range lasts, a
// lane that finishes takes the next particle of the range (ballot + prefix
// count, no atomics).  When the range is used up, the particles still running
// share all 64 lanes: each gets 64/m lanes (m = particles left) that try
// consecutive trials of it at once, and the lowest accepting trial wins.
// That is the same answer as trying the trials one by one, so the output does
// not depend on the schedule, and the slowest particle of a wave no longer
// runs alone on one lane.

// position of the q-th set bit (0-based) of mask, which has more than q bits
__device__ __forceinline__ int nth_set_bit(uint64_t mask, int q) {
  int pos = 0;
#pragma unroll
  for (int width = 32; width >= 1; width >>= 1) {
    const uint64_t low = mask & ((1ull << width) - 1ull);
    const int cnt = __popcll(low);
    if (q >= cnt) {
      q -= cnt;
      mask >>= width;
      pos += width;
    }
  }
  return pos;
}

// One wave works through the particles [r0, r1) (global indices) of one
// segment (weights ws, length n, filter id filt).  With a queue (an LDS
// counter shared by the workgroup's waves, starting at 0) the waves hand out
// the particles of [r0, r1) among themselves, so that none runs out of work
// while another still holds a long range: a wave takes as many particles as
// it has free lanes.  (Pieces of about four passes' worth, to wait on the
// counter less often, were slower: the waves then ran out unevenly.)
// With TABLE, a trial whose u * w_max exceeds the bucket bound of j is
// rejected without loading w_j.
constexpr int kRejBatch = 4;  // trials per lane and pass (past the first pass)
template <bool TABLE, typename T>
__device__ void rejection_wave_range(const T* ws, int64_t base, uint32_t n, uint32_t filt,
                                     double wmax, int64_t r0, int64_t r1, uint32_t max_trials,
                                     Key key, uint32_t offset, int32_t* __restrict__ a,
                                     uint32_t& my_flags, const BoundTable& tab,
                                     uint32_t* queue = nullptr) {
  const uint32_t lane = lane_id();
  // table kernels: ws is a global vector of n * sizeof(T) < 2^31 bytes
  const __amdgpu_buffer_rsrc_t wv = buffer_view(ws, TABLE ? n * (uint32_t)sizeof(T) : 0u);
  int64_t next = r0;  // wave-uniform: next particle of the range to hand out
  int64_t cur = -1;   // particle (global index) this lane works on
  uint32_t t = 0;     // its next trial

  // main phase: each pass tries trials t .. t + nq - 1 of every lane's
  // particle, of which the lowest accepting one counts (as if they ran one by
  // one).  nq is the same on every lane, so the wave never runs two code
  // paths in one pass (a particle's trial 0 proposes j = i): 4 while the
  // wave's acceptance rate so far is below 1/2 (long runs of rejections,
  // where four trials share one pass's overhead), else 1 (acceptance is
  // likely and further trials would be wasted draws and loads).
  uint64_t tried = 0, accepted = 0;  // wave-uniform counts of this range
  while (true) {
    const uint64_t freem = ballot(cur < 0);
    if (freem != 0 && next < r1) {
      const int64_t nfree = __popcll(freem);
      if (queue) {  // the next nfree particles of the workgroup's range
        uint32_t old = 0;
        if (lane == 0) old = atomicAdd(queue, (uint32_t)nfree);
        next = r0 + (int64_t)shfl(old, 0);
      }
      const int64_t avail = r1 - next > 0 ? r1 - next : 0;
      const int64_t take = nfree < avail ? nfree : avail;
      const int64_t rank = __popcll(freem & lanemask_lt());
      if (cur < 0 && rank < take) {
        cur = next + rank;
        t = 0;
      }
      // past the range: the queue is used up for every wave
      next += queue ? nfree : take;
    }
    if (next >= r1) break;
    const int nq = accepted * 2u < tried ? kRejBatch : 1;  // (results do not depend on nq)
    const uint64_t busy = ballot(cur >= 0);
    bool won = false;
    if (cur >= 0) {
      const uint32_t i = (uint32_t)(cur - base);
      // the trials' draws, then their table checks, then their weight loads
      // issued together, then the decisions: one wait per pass instead of one
      // per trial.  A trial that needs no load reads nothing (table kernel: an
      // out-of-range buffer offset) or re-reads the particle's own weight
      // (staged kernels: an LDS read)
      uint32_t jq[kRejBatch];
      double uq[kRejBatch];
      bool live[kRejBatch];
#pragma unroll
      for (int q = 0; q < kRejBatch; ++q) {
        live[q] = false;
        jq[q] = i;
        uq[q] = 1.0;
        if (q < nq) {
          const uint4 x = draw(key, i, DOM_TRIAL, t + (uint32_t)q, filt, offset);
          jq[q] = (q == 0 && t == 0) ? i : index_draw(x.x, x.y, n);
          uq[q] = u_accept(x.z);
          live[q] = (t + (uint32_t)q < max_trials) & !(TABLE && tab.rejects(uq[q], wmax, jq[q]));
        }
      }
      double vq[kRejBatch];
#pragma unroll
      for (int q = 0; q < kRejBatch; ++q) {
        if constexpr (TABLE)
          vq[q] = (double)buffer_gather<T>(wv, live[q] ? jq[q] * (uint32_t)sizeof(T) : kNoLoad);
        else
          vq[q] = (double)ws[live[q] ? jq[q] : i];
      }
      bool accq[kRejBatch];
#pragma unroll
      for (int q = 0; q < kRejBatch; ++q) accq[q] = live[q] & accept_exact<double>(uq[q], wmax, vq[q]);
      int first = -1;
#pragma unroll
      for (int q = kRejBatch - 1; q >= 0; --q)
        if (accq[q]) first = q;
      if (first >= 0) {
        uint32_t jsel = jq[0];
#pragma unroll
        for (int q = 1; q < kRejBatch; ++q)
          if (q == first) jsel = jq[q];
        a[cur] = (int32_t)jsel;
        cur = -1;
        won = true;
      } else {
        t += (uint32_t)nq;
        if (t >= max_trials) {
          a[cur] = (int32_t)i;
          my_flags |= FLAG_TRIAL_CAP;
          cur = -1;
        }
      }
    }
    tried += (uint64_t)nq * (uint64_t)__popcll(busy);
    accepted += (uint64_t)__popcll(ballot(won));
  }

  // tail phase: the remaining particles share the wave's lanes.  Each gets
  // slot = 64 / m lanes (m = particles left); lane r of a particle's group
  // tries its trials t + tb r .. t + tb r + tb - 1, so a pass covers trials
  // t .. t + slot tb - 1 of every particle, and the lowest accepting one wins
  // (the lowest lane of the group with an acceptance, and its lowest trial).
  // tb follows the wave's acceptance rate as nq does (the counts go on in
  // the tail, which is all there is when the range is shorter than a wave).
  while (true) {
    const uint64_t act = ballot(cur >= 0);
    if (act == 0) break;
    const int tb = accepted * 2u < tried ? kRejBatch : 1;
    const int m = __popcll(act);
    const int slot = kWave / m;  // lanes per particle
    const int grp = (int)lane / slot;
    const bool helper = grp < m;
    const int owner = helper ? nth_set_bit(act, grp) : (int)lane;
    const int64_t o_cur = shfl(cur, owner);
    const uint32_t o_t = shfl(t, owner);
    const uint32_t t0 = o_t + (uint32_t)tb * (lane - (uint32_t)(grp * slot));
    bool acc = false;
    uint32_t jj = 0;
    if (helper) {
      const uint32_t i = (uint32_t)(o_cur - base);
      uint32_t jb[kRejBatch];
      double ub[kRejBatch];
      bool live[kRejBatch];
#pragma unroll
      for (int b = 0; b < kRejBatch; ++b) {
        live[b] = false;
        jb[b] = i;
        ub[b] = 1.0;
        if (b < tb) {
          const uint32_t tt = t0 + (uint32_t)b;  // < 2^28 + 256: no wrap
          const uint4 x = draw(key, i, DOM_TRIAL, tt, filt, offset);
          jb[b] = (tt == 0) ? i : index_draw(x.x, x.y, n);
          ub[b] = u_accept(x.z);
          live[b] = (tt < max_trials) & !(TABLE && tab.rejects(ub[b], wmax, jb[b]));
        }
      }
      double vb[kRejBatch];
#pragma unroll
      for (int b = 0; b < kRejBatch; ++b) {
        if constexpr (TABLE)
          vb[b] = (double)buffer_gather<T>(wv, live[b] ? jb[b] * (uint32_t)sizeof(T) : kNoLoad);
        else
          vb[b] = (double)ws[live[b] ? jb[b] : i];
      }
#pragma unroll
      for (int b = kRejBatch - 1; b >= 0; --b) {
        if (live[b] & accept_exact<double>(ub[b], wmax, vb[b])) {
          acc = true;
          jj = jb[b];
        }
      }
    }
    const uint64_t accm = ballot(acc);
    int src = (int)lane;
    uint64_t g = 0;
    if (cur >= 0) {
      const int rank = __popcll(act & lanemask_lt());
      const uint64_t gm = (slot >= kWave ? ~0ull : ((1ull << slot) - 1ull)) << (rank * slot);
      g = accm & gm;
      if (g) src = __ffsll((long long)g) - 1;
    }
    const uint32_t jsel = shfl(jj, src);
    bool won = false;
    if (cur >= 0) {
      if (g) {
        a[cur] = (int32_t)jsel;
        cur = -1;
        won = true;
      } else {
        t += (uint32_t)(slot * tb);
        if (t >= max_trials) {
          a[cur] = (int32_t)(cur - base);
          my_flags |= FLAG_TRIAL_CAP;
          cur = -1;
        }
      }
    }
    tried += (uint64_t)(m * slot * tb);
    accepted += (uint64_t)__popcll(ballot(won));
  }
}

// A workgroup takes the particles [p0, p1) and walks the segments that overlap
// them; the waves hand out each segment part among themselves (an LDS
// counter reset between the part's barriers).  A segment of at most CAP
// weights is first copied into LDS.
template <typename T, int CAP, int THREADS>
__global__ __launch_bounds__(THREADS) void k_rejection(
    const T* __restrict__ w, int64_t n_total, const int64_t* __restrict__ offsets,
    uint32_t n_filters, double w_max, const double* __restrict__ w_max_dev, uint32_t max_trials,
    Key key, uint32_t offset, uint32_t filter_base, int32_t* __restrict__ a,
    uint32_t* __restrict__ flags, int64_t chunk) {
  __shared__ T sw[CAP > 0 ? CAP : 1];
  __shared__ uint32_t queue;  // particles of the segment part handed out so far
  offset = counter_offset(key, offset);
  const int64_t p0 = (int64_t)blockIdx.x * chunk;
  const int64_t p1 = p0 + chunk < n_total ? p0 + chunk : n_total;
  uint32_t my_flags = 0;
  uint32_t f = offsets ? find_segment(offsets, n_filters, p0) : 0u;
  for (int64_t g0 = p0; g0 < p1; ++f) {
    const int64_t base = offsets ? offsets[f] : 0;
    const int64_t end = offsets ? offsets[f + 1] : n_total;
    const int64_t q1 = end < p1 ? end : p1;
    if (q1 <= g0) continue;  // empty segment
    const uint32_t n = (uint32_t)(end - base);
    const double wmax = w_max_dev ? w_max_dev[f] : w_max;
    const bool staged = CAP > 0 && n <= (uint32_t)CAP;
    __syncthreads();  // the previous part's trials are done with sw and the queue
    if (threadIdx.x == 0) queue = 0;
    if (staged) stage_weights(w + base, n, sw);
    __syncthreads();
    if (staged)
      rejection_wave_range<false>(sw, base, n, filter_base + f, wmax, g0, q1, max_trials, key,
                                  offset, a, my_flags, BoundTable{}, &queue);
    else
      rejection_wave_range<false>(w + base, base, n, filter_base + f, wmax, g0, q1, max_trials,
                                  key, offset, a, my_flags, BoundTable{}, &queue);
    g0 = q1;
  }
  if (flags) {
    const uint32_t wf = wave_reduce(my_flags, OpOr());
    if (lane_id() == 0 && wf) atomicOr(flags, wf);
  }
}

// One vector with the LDS bound table; the workgroup's waves hand out its
// chunk among themselves.
template <typename T>
__global__ __launch_bounds__(kTableThreads) void k_rejection_table(
    const T* __restrict__ w, int64_t n, double w_max, uint32_t max_trials, Key key,
    uint32_t offset, uint32_t filter, int32_t* __restrict__ a, uint32_t* __restrict__ flags,
    int64_t chunk, const uint32_t* __restrict__ nib_g, const uint32_t* __restrict__ cm,
    uint32_t nb, int shift) {
  __shared__ __align__(16) uint8_t nib[kTableBuckets / 2];
  __shared__ uint32_t queue;  // particles of the chunk handed out so far
  offset = counter_offset(key, offset);
  if (threadIdx.x == 0) queue = 0;  // before the barrier of the table's load
  const BoundTable tab = load_bound_table(nib_g, cm, nb, shift, nib);
  const int64_t p0 = (int64_t)blockIdx.x * chunk;
  const int64_t p1 = p0 + chunk < n ? p0 + chunk : n;
  uint32_t my_flags = 0;
  if (p0 < p1)
    rejection_wave_range<true>(w, 0, (uint32_t)n, filter, w_max, p0, p1, max_trials, key,
                               offset, a, my_flags, tab, &queue);
  if (flags) {
    const uint32_t wf = wave_reduce(my_flags, OpOr());
    if (lane_id() == 0 && wf) atomicOr(flags, wf);
  }
}

// ------------------------------------------------------------------ launchers
// LDS capacity (weights) for the longest segment: 16, 64 or 128 KB, or none
// when some segment is longer (or the lengths are unknown and the vector is
// long) -- then every weight load goes to global memory.
template <typename T>
int staged_capacity(int64_t max_len, int64_t n_total, uint32_t n_filters) {
  constexpr int64_t per_kb = 1024 / (int64_t)sizeof(T);
  if (n_filters == 1) {
    if (n_total <= 16 * per_kb) return (int)(16 * per_kb);
    if (n_total <= 64 * per_kb) return (int)(64 * per_kb);
    return 0;
  }
  // batches: up to the tuned largest tier; longer segments run in the same
  // launch from global memory
  if (max_len <= 0) max_len = (int64_t)128 * per_kb;
  const int64_t top = (int64_t)tuning().batch_stage_max_kb;
  if (max_len <= 16 * per_kb || top == 16) return (int)(16 * per_kb);
  if (max_len <= 64 * per_kb || top == 64) return (int)(64 * per_kb);
  return (int)(128 * per_kb);
}

template <typename T>
hipError_t launch_metropolis_t(const void* wv, int64_t n_total, const int64_t* offsets,
                               uint32_t n_filters, int64_t max_len, int32_t B,
                               const int32_t* B_dev, Key key, uint32_t offset,
                               uint32_t filter_base, int32_t* a, hipStream_t stream) {
  const T* w = (const T*)wv;
  constexpr int per_kb = 1024 / (int)sizeof(T);
  const int cap = staged_capacity<T>(max_len, n_total, n_filters);
  constexpr int64_t kAll = INT64_MAX;
  auto global_launch = [&](int64_t min_len) {
    const int64_t chunk = tuning().metropolis_chunk;
    hipLaunchKernelGGL((k_metropolis_staged<T, 0, 256>), dim3((unsigned)((n_total + chunk - 1) / chunk)),
                       dim3(256), 0, stream, w, n_total, offsets, n_filters, B, B_dev, key, offset,
                       filter_base, a, chunk, min_len, kAll);
    return hipGetLastError();
  };
  if (cap == 0) {
    // one vector of up to 128 KB of weights: staged as below (one workgroup
    // per CU for the LDS), otherwise chains gather from global memory
    if ((!offsets || n_filters <= 1) && n_total <= 128 * per_kb) {
      const int64_t chunk1 = 256;
      hipLaunchKernelGGL((k_metropolis_staged<T, 128 * per_kb, 256>),
                         dim3((unsigned)((n_total + chunk1 - 1) / chunk1)), dim3(256), 0, stream,
                         w, n_total, offsets, n_filters, B, B_dev, key, offset, filter_base, a,
                         chunk1, (int64_t)0, kAll);
      return hipGetLastError();
    }
    return global_launch(0);
  }
  // segments longer than the LDS tier run in the same launch, from global
  // memory (a second, pipelined launch for them measured slower on ragged
  // batches: its chunks hold several long chains per lane)
  const int64_t hi = kAll;
  if (!offsets || n_filters <= 1) {
    // one short vector: every workgroup stages all of it and runs 256 of its
    // chains, one per lane, so that long chains (large B) spread over many CUs
    // instead of running four to a lane on one to four of them
    const int64_t chunk1 = 256;
    const dim3 grid1((unsigned)((n_total + chunk1 - 1) / chunk1));
    if (cap == 16 * per_kb)
      hipLaunchKernelGGL((k_metropolis_staged<T, 16 * per_kb, 256>), grid1, dim3(256), 0, stream,
                         w, n_total, offsets, n_filters, B, B_dev, key, offset, filter_base, a,
                         chunk1, (int64_t)0, hi);
    else
      hipLaunchKernelGGL((k_metropolis_staged<T, 64 * per_kb, 256>), grid1, dim3(256), 0, stream,
                         w, n_total, offsets, n_filters, B, B_dev, key, offset, filter_base, a,
                         chunk1, (int64_t)0, hi);
    return hipGetLastError();
  }
  const int64_t chunk = tuning().batch_metropolis_chunk;
  const dim3 grid((unsigned)((n_total + chunk - 1) / chunk));
  if (cap == 16 * per_kb)
    hipLaunchKernelGGL((k_metropolis_staged<T, 16 * per_kb, 1024>), grid, dim3(1024), 0, stream, w,
                       n_total, offsets, n_filters, B, B_dev, key, offset, filter_base, a, chunk,
                       (int64_t)0, hi);
  else if (cap == 64 * per_kb)
    hipLaunchKernelGGL((k_metropolis_staged<T, 64 * per_kb, 1024>), grid, dim3(1024), 0, stream, w,
                       n_total, offsets, n_filters, B, B_dev, key, offset, filter_base, a, chunk,
                       (int64_t)0, hi);
  else
    hipLaunchKernelGGL((k_metropolis_staged<T, 128 * per_kb, 1024>), grid, dim3(1024), 0, stream,
                       w, n_total, offsets, n_filters, B, B_dev, key, offset, filter_base, a,
                       chunk, (int64_t)0, hi);
  return hipGetLastError();
}

// Bound-table geometry for one vector of n weights: buckets of 2^shift
// particles, at most kTableBuckets of them.
struct TableGeom {
  int shift;
  uint32_t nb, n_wg;
  size_t wg_off, codes_off, nib_off, cm_off, bytes;
};

TableGeom table_geom(int64_t n) {
  TableGeom g;
  g.shift = 2;  // at least 4 particles per bucket (BoundTable::c4 needs shift >= 2)
  while ((((n - 1) >> g.shift) + 1) > kTableBuckets) ++g.shift;
  g.nb = (uint32_t)(((n - 1) >> g.shift) + 1);
  g.n_wg = (g.nb + kCodeThreads - 1) / kCodeThreads;
  g.wg_off = 0;
  g.codes_off = ((size_t)g.n_wg * 4 + 255) & ~(size_t)255;
  g.nib_off = g.codes_off + (((size_t)g.nb + 7) / 8 * 8 + 255) / 256 * 256;
  // packed nibbles, padded to 16-byte pieces; then the largest code
  g.cm_off = g.nib_off + (((size_t)g.nb + 31) / 32 * 16 + 255) / 256 * 256;
  g.bytes = g.cm_off + 256;
  return g;
}

// A vector long enough for the table path: not staged in LDS, and long enough
// that the table prologue pays off.
template <typename T>
bool use_table(int64_t n_total, uint32_t n_filters, int64_t max_len) {
  // the table kernels gather through a buffer resource, whose byte range
  // must stay below 2^31
  return n_filters == 1 && n_total >= (1 << 16) &&
         n_total * (int64_t)sizeof(T) < ((int64_t)1 << 31) &&
         staged_capacity<T>(max_len, n_total, n_filters) == 0;
}

size_t alt_workspace_bytes(bool f64, int64_t n_total, uint32_t n_filters, int64_t max_len) {
  const bool t = f64 ? use_table<double>(n_total, n_filters, max_len)
                     : use_table<float>(n_total, n_filters, max_len);
  return t ? table_geom(n_total).bytes : 0;
}

template <typename T>
hipError_t launch_bound_codes(const T* w, int64_t n, const TableGeom& g, void* ws,
                              hipStream_t stream) {
  char* base = (char*)ws;
  hipLaunchKernelGGL(k_bound_codes<T>, dim3(g.n_wg), dim3(kCodeThreads), 0, stream, w, n, g.shift,
                     (uint8_t*)(base + g.codes_off), (uint32_t*)(base + g.wg_off));
  const uint32_t words = (g.nb + 7) / 8;
  hipLaunchKernelGGL(k_pack_table, dim3((words + kPackThreads - 1) / kPackThreads),
                     dim3(kPackThreads), 0, stream, (const uint8_t*)(base + g.codes_off),
                     (const uint32_t*)(base + g.wg_off), g.n_wg, g.nb,
                     (uint32_t*)(base + g.nib_off), (uint32_t*)(base + g.cm_off));
  return hipGetLastError();
}

// bound_code of a finite positive binary64 on the host: 2^(c - 127) >= v
uint32_t ref_code(double v) {
  uint64_t bits;
  memcpy(&bits, &v, sizeof bits);
  const int e = (int)((bits >> 52) & 0x7FF);
  if (e == 0) return 0u;  // below 2^-1022: every code reaches it
  const int c = e - 1023 + 127 + ((bits & 0xFFFFFFFFFFFFFull) != 0ull ? 1 : 0);
  return c < 0 ? 0u : (c > 255 ? 255u : (uint32_t)c);
}

// Workgroups of the table kernels: one per CU, each with a chunk of particles.
constexpr int64_t kTableGrid = 256;

template <typename T>
hipError_t launch_metropolis_table(const T* w, int64_t n, int32_t B, Key key, uint32_t offset,
                                   uint32_t filter, int32_t* a, void* ws, hipStream_t stream) {
  const TableGeom g = table_geom(n);
  hipError_t e = launch_bound_codes(w, n, g, ws, stream);
  if (e != hipSuccess) return e;
  const int64_t chunk = (n + kTableGrid - 1) / kTableGrid;
  char* base = (char*)ws;
  const dim3 grid((unsigned)((n + chunk - 1) / chunk));
  const uint32_t* nib = (const uint32_t*)(base + g.nib_off);
  const uint32_t* cm = (const uint32_t*)(base + g.cm_off);
  // chains per lane: as many as the chunk fills (four from 2^20 particles up);
  // more than that would run copies of dead chains on every lane
  if (chunk <= kTableThreads)
    hipLaunchKernelGGL((k_metropolis_table<T, 1>), grid, dim3(kTableThreads), 0, stream, w, n, B,
                       key, offset, filter, a, chunk, nib, cm, g.nb, g.shift);
  else if (chunk <= 2 * kTableThreads)
    hipLaunchKernelGGL((k_metropolis_table<T, 2>), grid, dim3(kTableThreads), 0, stream, w, n, B,
                       key, offset, filter, a, chunk, nib, cm, g.nb, g.shift);
  else
    hipLaunchKernelGGL((k_metropolis_table<T, 4>), grid, dim3(kTableThreads), 0, stream, w, n, B,
                       key, offset, filter, a, chunk, nib, cm, g.nb, g.shift);
  return hipGetLastError();
}

hipError_t launch_metropolis(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                             uint32_t n_filters, int64_t max_len, int32_t B, const int32_t* B_dev,
                             Key key, uint32_t offset, uint32_t filter_base, int32_t* a, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
  // the table pays off once chains are long (small beta, most proposals rejected)
  const int32_t min_B = tuning().metropolis_table_min_B;
  if (ws && !B_dev && min_B > 0 && B >= min_B &&
      ws_bytes >= alt_workspace_bytes(f64, n_total, n_filters, max_len) &&
      (f64 ? use_table<double>(n_total, n_filters, max_len)
           : use_table<float>(n_total, n_filters, max_len)))
    return f64 ? launch_metropolis_table((const double*)w, n_total, B, key, offset, filter_base,
                                         a, ws, stream)
               : launch_metropolis_table((const float*)w, n_total, B, key, offset, filter_base, a,
                                         ws, stream);
  return f64 ? launch_metropolis_t<double>(w, n_total, offsets, n_filters, max_len, B, B_dev, key,
                                           offset, filter_base, a, stream)
             : launch_metropolis_t<float>(w, n_total, offsets, n_filters, max_len, B, B_dev, key,
                                          offset, filter_base, a, stream);
}


template <typename T>
hipError_t launch_rejection_t(const void* wv, int64_t n_total, const int64_t* offsets,
                              uint32_t n_filters, int64_t max_len, double w_max,
                              const double* w_max_dev, uint32_t max_trials, Key key,
                              uint32_t offset, uint32_t filter_base, int32_t* a, uint32_t* flags,
                              hipStream_t stream) {
  const T* w = (const T*)wv;
  constexpr int per_kb = 1024 / (int)sizeof(T);
  const int cap = staged_capacity<T>(max_len, n_total, n_filters);
  const bool single = !offsets || n_filters <= 1;
  if (cap == 0) {
    // a short single vector: 256 particles per workgroup, so that its long
    // trial sequences spread over more CUs
    const int64_t chunk = single && n_total < (1 << 19) ? 256
                                                          : (int64_t)tuning().rejection_per_wave * 4;
    hipLaunchKernelGGL((k_rejection<T, 0, 256>), dim3((unsigned)((n_total + chunk - 1) / chunk)),
                       dim3(256), 0, stream, w, n_total, offsets, n_filters, w_max, w_max_dev,
                       max_trials, key, offset, filter_base, a, flags, chunk);
    return hipGetLastError();
  }
  if (single) {
    // one vector in LDS: every 256-thread workgroup stages all of it and takes
    // 256 of its particles (one per lane on average)
    const int64_t chunk1 = 256;
    const dim3 grid1((unsigned)((n_total + chunk1 - 1) / chunk1));
    if (cap == 16 * per_kb)
      hipLaunchKernelGGL((k_rejection<T, 16 * per_kb, 256>), grid1, dim3(256), 0, stream, w,
                         n_total, offsets, n_filters, w_max, w_max_dev, max_trials, key, offset,
                         filter_base, a, flags, chunk1);
    else
      hipLaunchKernelGGL((k_rejection<T, 64 * per_kb, 256>), grid1, dim3(256), 0, stream, w,
                         n_total, offsets, n_filters, w_max, w_max_dev, max_trials, key, offset,
                         filter_base, a, flags, chunk1);
    return hipGetLastError();
  }
  const int64_t chunk = (int64_t)tuning().batch_rejection_per_wave * 16;
  const dim3 grid((unsigned)((n_total + chunk - 1) / chunk));
  if (cap == 16 * per_kb)
    hipLaunchKernelGGL((k_rejection<T, 16 * per_kb, 1024>), grid, dim3(1024), 0, stream, w,
                       n_total, offsets, n_filters, w_max, w_max_dev, max_trials, key, offset,
                       filter_base, a, flags, chunk);
  else if (cap == 64 * per_kb)
    hipLaunchKernelGGL((k_rejection<T, 64 * per_kb, 1024>), grid, dim3(1024), 0, stream, w,
                       n_total, offsets, n_filters, w_max, w_max_dev, max_trials, key, offset,
                       filter_base, a, flags, chunk);
  else
    hipLaunchKernelGGL((k_rejection<T, 128 * per_kb, 1024>), grid, dim3(1024), 0, stream, w,
                       n_total, offsets, n_filters, w_max, w_max_dev, max_trials, key, offset,
                       filter_base, a, flags, chunk);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rejection_table(const T* w, int64_t n, double w_max, uint32_t max_trials,
                                  Key key, uint32_t offset, uint32_t filter, int32_t* a,
                                  uint32_t* flags, void* ws, hipStream_t stream) {
  const TableGeom g = table_geom(n);
  char* base = (char*)ws;
  hipLaunchKernelGGL(k_bound_nibbles<T>, dim3((g.nb + kCodeThreads - 1) / kCodeThreads),
                     dim3(kCodeThreads), 0, stream, w, n, g.shift, g.nb, ref_code(w_max),
                     (uint32_t*)(base + g.nib_off), (uint32_t*)(base + g.cm_off));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // chunks of 16 waves x rejection_per_wave particles, several per CU
  const int64_t chunk = (int64_t)tuning().rejection_per_wave * (kTableThreads / kWave);
  hipLaunchKernelGGL(k_rejection_table<T>, dim3((unsigned)((n + chunk - 1) / chunk)),
                     dim3(kTableThreads), 0, stream, w, n, w_max, max_trials, key, offset, filter,
                     a, flags, chunk, (const uint32_t*)(base + g.nib_off),
                     (const uint32_t*)(base + g.cm_off), g.nb, g.shift);
  return hipGetLastError();
}

hipError_t launch_rejection(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                            uint32_t n_filters, int64_t max_len, double w_max,
                            const double* w_max_dev, uint32_t max_trials, Key key,
                            uint32_t offset, uint32_t filter_base, int32_t* a, uint32_t* flags,
                            void* ws, size_t ws_bytes, hipStream_t stream) {
  // below 2^20 particles the plain kernel was faster at every y measured (0..4)
  if (ws && !w_max_dev && tuning().rejection_table && n_total >= (1 << 20) &&
      ws_bytes >= alt_workspace_bytes(f64, n_total, n_filters, max_len) &&
      (f64 ? use_table<double>(n_total, n_filters, max_len)
           : use_table<float>(n_total, n_filters, max_len)))
    return f64 ? launch_rejection_table((const double*)w, n_total, w_max, max_trials, key, offset,
                                        filter_base, a, flags, ws, stream)
               : launch_rejection_table((const float*)w, n_total, w_max, max_trials, key, offset,
                                        filter_base, a, flags, ws, stream);
  return f64 ? launch_rejection_t<double>(w, n_total, offsets, n_filters, max_len, w_max,
                                          w_max_dev, max_trials, key, offset, filter_base, a,
                                          flags, stream)
             : launch_rejection_t<float>(w, n_total, offsets, n_filters, max_len, w_max,
                                         w_max_dev, max_trials, key, offset, filter_base, a,
                                         flags, stream);
}

}  // namespace pfr
