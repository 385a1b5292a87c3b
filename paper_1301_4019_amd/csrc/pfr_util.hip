// pfr_util.hip -- auxiliaries around the resampling step:
//   ancestors_to_offspring  (Code 12 of the paper)
//   effective_sample_size   (the ESS of section 3.4)
//   copy_particles          (the in-place copy step of section 2.3, for
//                            particle states of any dimension)
#include "pfr_kernels.h"

namespace pfr {

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Segment of a workgroup slot.  Work items of kChunk elements are numbered so
// that segment f owns slots [f + floor(offsets[f] / kChunk), + ceil(n_f / kChunk)):
// since floor(x + y) >= floor(x) + floor(y), consecutive segments never share
// a slot, and every slot lies below n_filters + n_total / kChunk + 1.  Returns
// false for a slot no segment owns.
struct SlotSeg {
  int64_t base, n, p;  // segment start, length, chunk index inside it
  uint32_t f;
};

template <int kChunk>
__device__ __forceinline__ bool slot_segment(const int64_t* __restrict__ offsets,
                                             uint32_t n_filters, int64_t n_total, int64_t slot,
                                             SlotSeg& s) {
  if (!offsets) {
    s.f = 0;
    s.base = 0;
    s.n = n_total;
    s.p = slot;
  } else {
    uint32_t lo = 0, hi = n_filters;  // largest f with f + offsets[f] / kChunk <= slot
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if ((int64_t)mid + offsets[mid] / kChunk <= slot) lo = mid;
      else hi = mid;
    }
    s.f = lo;
    s.base = offsets[lo];
    s.n = offsets[lo + 1] - s.base;
    s.p = slot - ((int64_t)lo + s.base / kChunk);
  }
  return s.p * kChunk < s.n;
}

template <int kChunk>
uint32_t slot_count(int64_t n_total, uint32_t n_filters) {
  return n_filters + (uint32_t)(n_total / kChunk) + 1;
}

// ================================================================ Code 12
// o_j = #{i : a_i = j}.  For a non-decreasing ancestry the count of value j
// is the length of its run, (last position + 1) - first position, so o is
// formed without atomics in two ordered phases over a zeroed count array:
// the position that ends a run stores last + 1 into its value's slot, then
// the position that starts it subtracts its own index.  Each slot has one
// writer per phase; values that appear in no run keep their zero.
//
// Segments of at most kA2oCap particles (batches) are converted in LDS by one
// workgroup each.  Longer segments are cut into tiles of kA2oTile offspring
// slots: a tile finds the range of positions holding its values with two
// wave-wide 64-ary searches, runs the two phases over that range into an LDS
// count array and writes its slots once.  An unsorted ancestry goes through
// counting: LDS histograms over windows of values for segments of up to
// kA2oWinMax particles, a zero pass then atomic additions in global memory,
// as in Code 12, for longer ones.
constexpr int kA2oCap = 16384;
constexpr int kA2oStagedThreads = 1024;
constexpr int kA2oTile = 4096;
constexpr int kA2oThreads = 256;

__global__ __launch_bounds__(kA2oStagedThreads) void k_a2o_staged(
    const int32_t* __restrict__ a, const int64_t* __restrict__ offsets, uint32_t n_filters,
    int32_t* __restrict__ o, uint32_t* __restrict__ flags) {
  __shared__ int32_t cnt[kA2oCap];
  __shared__ int32_t as[kA2oCap];
  __shared__ uint32_t s_bad;
  const uint32_t f = blockIdx.x;
  if (f >= n_filters) return;
  const int64_t base = offsets[f];
  const int64_t n64 = offsets[f + 1] - base;
  if (n64 > kA2oCap || n64 <= 0) return;  // long segments: tiled kernels
  const int n = (int)n64;
  const int tid = (int)threadIdx.x;
  if (tid == 0) s_bad = 0;
  bool bad = false;
  for (int j = tid; j < n; j += kA2oStagedThreads) cnt[j] = 0;
  for (int i = tid; i < n; i += kA2oStagedThreads) as[i] = a[base + i];
  __syncthreads();
  // phase 1: run ends
  for (int i = tid; i < n; i += kA2oStagedThreads) {
    const int v = as[i];
    if (v < 0 || v >= n) {
      bad = true;
      continue;
    }
    if (i == n - 1 || as[i + 1] != v) cnt[v] = i + 1;
  }
  __syncthreads();
  // phase 2: run starts
  for (int i = tid; i < n; i += kA2oStagedThreads) {
    const int v = as[i];
    if (v < 0 || v >= n) continue;
    if (i == 0 || as[i - 1] != v) cnt[v] -= i;
  }
  __syncthreads();
  for (int j = tid; j < n; j += kA2oStagedThreads) o[base + j] = cnt[j];
  if (ballot(bad) != 0 && lane_id() == 0) atomicOr(&s_bad, 1u);
  __syncthreads();
  if (tid == 0 && s_bad && flags) atomicOr(flags, FLAG_BAD_ANCESTOR);
}

// Unsorted segments of up to kA2oWinMax particles: the workgroup of slot
// (f, p) counts values [p W, (p + 1) W) of segment f in an LDS histogram
// (W = kA2oWin), reading the whole segment; a segment is read
// ceil(n_f / W) times, which for these lengths costs less than atomics in
// global memory.
constexpr int kA2oWin = 32768;
constexpr int kA2oWinMax = 4 * kA2oWin;

__global__ __launch_bounds__(kA2oStagedThreads) void k_a2o_window(
    const int32_t* __restrict__ a, int64_t n_total, const int64_t* __restrict__ offsets,
    uint32_t n_filters, int32_t* __restrict__ o, uint32_t* __restrict__ flags) {
  __shared__ int32_t cnt[kA2oWin];
  SlotSeg s;
  if (!slot_segment<kA2oWin>(offsets, n_filters, n_total, blockIdx.x, s)) return;
  if (s.n > kA2oWinMax) return;  // global atomics
  const int tid = (int)threadIdx.x;
  const int64_t j0 = s.p * kA2oWin;
  const int win = (int)min((int64_t)kA2oWin, s.n - j0);
  for (int j = tid; j < win; j += kA2oStagedThreads) cnt[j] = 0;
  __syncthreads();
  bool bad = false;
  const int32_t* __restrict__ as = a + s.base;
  for (int64_t i = tid; i < s.n; i += kA2oStagedThreads) {
    const int64_t v = as[i];
    if (v < 0 || v >= s.n) {
      bad = true;
      continue;
    }
    const int64_t r = v - j0;
    if (r >= 0 && r < win) atomicAdd(&cnt[r], 1);
  }
  __syncthreads();
  for (int j = tid; j < win; j += kA2oStagedThreads) o[s.base + j0 + j] = cnt[j];
  // every window sees every out-of-range value; the first one reports it
  if (flags && s.p == 0 && ballot(bad) != 0 && lane_id() == 0) atomicOr(flags, FLAG_BAD_ANCESTOR);
}

// First position p in [0, n) with a[p] >= v (n if none), for a non-decreasing
// a, by the whole wave: each round reads 64 evenly spaced pivots of the
// remaining interval and keeps the gap where the predicate a[p] < v turns
// false.  Three rounds cover 2^18 positions.  On an unsorted a the result is
// some position in [0, n].
__device__ __forceinline__ int64_t wave_lower_bound(const int32_t* __restrict__ a, int64_t n,
                                                    int64_t v) {
  const int lane = (int)lane_id();
  int64_t lo = 0, hi = n;  // answer in [lo, hi]
  while (hi - lo > kWave) {
    const int64_t span = hi - lo;
    const int64_t p = lo + (span * (lane + 1)) / (kWave + 1);  // lo <= p < hi
    const int k = __popcll(ballot((int64_t)a[p] < v));
    const int64_t plo = shfl(p, k > 0 ? k - 1 : 0);
    const int64_t phi = shfl(p, k < kWave ? k : kWave - 1);
    const int64_t nlo = k > 0 ? plo + 1 : lo;
    const int64_t nhi = k < kWave ? phi : hi;
    lo = nlo;
    hi = nhi;
  }
  const int64_t p = lo + lane;
  return lo + __popcll(ballot(p < hi && (int64_t)a[p] < v));
}

__global__ __launch_bounds__(kA2oThreads) void k_a2o_sorted_tiles(
    const int32_t* __restrict__ a, int64_t n_total, const int64_t* __restrict__ offsets,
    uint32_t n_filters, int64_t min_len, int32_t* __restrict__ o,
    uint32_t* __restrict__ flags) {
  __shared__ int32_t cnt[kA2oTile];
  __shared__ int64_t s_range[2];
  SlotSeg s;
  if (!slot_segment<kA2oTile>(offsets, n_filters, n_total, blockIdx.x, s)) return;
  if (s.n < min_len) return;  // converted in LDS by k_a2o_staged
  const int tid = (int)threadIdx.x, wave = tid / kWave;
  const int32_t* __restrict__ as = a + s.base;
  const int64_t j0 = s.p * kA2oTile;
  const int tile = (int)min((int64_t)kA2oTile, s.n - j0);
  for (int j = tid; j < tile; j += kA2oThreads) cnt[j] = 0;
  if (wave < 2) {
    const int64_t r = wave_lower_bound(as, s.n, wave == 0 ? j0 : j0 + tile);
    if (lane_id() == 0) s_range[wave] = r;
  }
  __syncthreads();
  const int64_t lo = s_range[0], hi = s_range[1];
  // values below 0 sort before every tile, values >= n after the last one
  if (tid == 0 && flags && ((j0 == 0 && lo > 0) || (j0 + tile == s.n && hi < s.n)))
    atomicOr(flags, FLAG_BAD_ANCESTOR);
  for (int64_t i = lo + tid; i < hi; i += kA2oThreads) {
    const int64_t v = (int64_t)as[i] - j0;
    if (v < 0 || v >= tile) continue;  // only an unsorted input gets here
    if (i == s.n - 1 || as[i + 1] != as[i]) cnt[v] = (int32_t)(i + 1 - lo);
  }
  __syncthreads();
  for (int64_t i = lo + tid; i < hi; i += kA2oThreads) {
    const int64_t v = (int64_t)as[i] - j0;
    if (v < 0 || v >= tile) continue;
    if (i == 0 || as[i - 1] != as[i]) cnt[v] -= (int32_t)(i - lo);
  }
  __syncthreads();
  for (int j = tid; j < tile; j += kA2oThreads) o[s.base + j0 + j] = cnt[j];
}

// Unsorted segments longer than kA2oWinMax: zero pass, then one atomic
// addition per ancestor, both over tiles of kA2oTile positions per workgroup.
__global__ __launch_bounds__(kA2oThreads) void k_a2o_zero(int64_t n_total,
                                                          const int64_t* __restrict__ offsets,
                                                          uint32_t n_filters, int64_t min_len,
                                                          int32_t* __restrict__ o) {
  SlotSeg s;
  if (!slot_segment<kA2oTile>(offsets, n_filters, n_total, blockIdx.x, s)) return;
  if (s.n < min_len) return;
  const int64_t j0 = s.p * kA2oTile;
  const int tile = (int)min((int64_t)kA2oTile, s.n - j0);
  for (int j = (int)threadIdx.x; j < tile; j += kA2oThreads) o[s.base + j0 + j] = 0;
}

__global__ __launch_bounds__(kA2oThreads) void k_a2o_atomic(const int32_t* __restrict__ a,
                                                            int64_t n_total,
                                                            const int64_t* __restrict__ offsets,
                                                            uint32_t n_filters, int64_t min_len,
                                                            int32_t* __restrict__ o,
                                                            uint32_t* __restrict__ flags) {
  SlotSeg s;
  if (!slot_segment<kA2oTile>(offsets, n_filters, n_total, blockIdx.x, s)) return;
  if (s.n < min_len) return;
  const int64_t i0 = s.p * kA2oTile;
  const int tile = (int)min((int64_t)kA2oTile, s.n - i0);
  bool bad = false;
  for (int i = (int)threadIdx.x; i < tile; i += kA2oThreads) {
    const int64_t v = a[s.base + i0 + i];
    if (v < 0 || v >= s.n) {
      bad = true;
      continue;
    }
    atomicAdd(&o[s.base + v], 1);
  }
  if (flags && ballot(bad) != 0 && lane_id() == 0) atomicOr(flags, FLAG_BAD_ANCESTOR);
}

// ================================================================ ESS
// ESS = (sum w)^2 / sum w^2 per segment.  Each chunk of kEssChunk weights is
// scaled by the power of two 2^-e, e the exponent of its largest weight (an
// exact scaling, so squares neither overflow nor lose the small weights'
// bits), and summed in binary64 in a fixed order; a wave per segment then
// rescales the chunk sums to the largest exponent and adds them, again in a
// fixed order.  The order depends only on the segment's length, so a result
// is reproducible bit for bit.  Summation depth: 16 sequential terms per
// thread, 6 butterfly levels, 3 wave additions, ceil(P / 64) sequential
// chunk sums per lane and 6 butterfly levels (P chunks).
constexpr int kEssChunk = 4096;
constexpr int kEssThreads = 256;
constexpr int kEssPer = kEssChunk / kEssThreads;
constexpr int kEssZero = -100000;  // exponent of an all-zero chunk

struct EssPart {
  double s1, s2;
  int32_t e;
  uint32_t bad;
  uint64_t pad;
};

template <typename T>
__global__ __launch_bounds__(kEssThreads) void k_ess_partials(
    const T* __restrict__ w, int64_t n_total, const int64_t* __restrict__ offsets,
    uint32_t n_filters, EssPart* __restrict__ parts) {
  __shared__ double s_max[4], s_s1[4], s_s2[4];
  __shared__ uint32_t s_bad[4];
  SlotSeg s;
  if (!slot_segment<kEssChunk>(offsets, n_filters, n_total, blockIdx.x, s)) return;
  const int tid = (int)threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int64_t i0 = s.p * kEssChunk;
  const T* __restrict__ ws = w + s.base;
  double v[kEssPer];
  double m = 0.0;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < kEssPer; ++k) {
    const int64_t idx = i0 + k * kEssThreads + tid;
    const T x = idx < s.n ? ws[idx] : (T)0;
    if (!weight_ok(x)) bad = true;
    v[k] = (double)x;
    if (v[k] > m) m = v[k];
  }
  m = wave_reduce(m, OpMax());
  const uint32_t wbad = ballot(bad) != 0 ? 1u : 0u;
  if (lane == 0) {
    s_max[wave] = m;
    s_bad[wave] = wbad;
  }
  __syncthreads();
  const double mx = fmax(fmax(s_max[0], s_max[1]), fmax(s_max[2], s_max[3]));
  const uint32_t anybad = s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3];
  const int64_t slot = blockIdx.x;
  if (anybad || mx == 0.0) {
    if (tid == 0) {
      EssPart p;
      p.s1 = 0.0;
      p.s2 = 0.0;
      p.e = kEssZero;
      p.bad = anybad;
      p.pad = 0;
      parts[slot] = p;
    }
    return;
  }
  const int e = ilogb(mx);
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int k = 0; k < kEssPer; ++k) {
    const double x = ldexp(v[k], -e);
    s1 += x;
    s2 += x * x;
  }
  s1 = wave_reduce(s1, OpAdd());
  s2 = wave_reduce(s2, OpAdd());
  if (lane == 0) {
    s_s1[wave] = s1;
    s_s2[wave] = s2;
  }
  __syncthreads();
  if (tid == 0) {
    EssPart p;
    p.s1 = ((s_s1[0] + s_s1[1]) + s_s1[2]) + s_s1[3];
    p.s2 = ((s_s2[0] + s_s2[1]) + s_s2[2]) + s_s2[3];
    p.e = e;
    p.bad = 0;
    p.pad = 0;
    parts[slot] = p;
  }
}

__global__ __launch_bounds__(256) void k_ess_finish(int64_t n_total,
                                                    const int64_t* __restrict__ offsets,
                                                    uint32_t n_filters,
                                                    const EssPart* __restrict__ parts,
                                                    double* __restrict__ ess,
                                                    uint32_t* __restrict__ flags) {
  const uint32_t f = blockIdx.x * 4 + threadIdx.x / kWave;
  if (f >= n_filters) return;
  const int lane = (int)lane_id();
  const int64_t base = offsets ? offsets[f] : 0;
  const int64_t n = offsets ? offsets[f + 1] - base : n_total;
  const int64_t first = (int64_t)f + base / kEssChunk;
  const int64_t P = (n + kEssChunk - 1) / kEssChunk;
  int emax = kEssZero;
  uint32_t bad = 0;
  for (int64_t p = lane; p < P; p += kWave) {
    const EssPart q = parts[first + p];
    bad |= q.bad;
    if (q.e > emax) emax = q.e;
  }
  emax = wave_reduce(emax, OpMax());
  bad = wave_reduce(bad, OpOr());
  double result;
  uint32_t fl = 0;
  if (bad) {
    result = __builtin_nan("");
    fl = FLAG_BAD_WEIGHTS;
  } else if (emax == kEssZero) {
    result = 0.0;
    if (n > 0) fl = FLAG_ZERO_TOTAL;
  } else {
    double s1 = 0.0, s2 = 0.0;
    for (int64_t p = lane; p < P; p += kWave) {
      const EssPart q = parts[first + p];
      if (q.e == kEssZero) continue;
      const int d = q.e - emax;  // <= 0
      s1 += ldexp(q.s1, d);
      s2 += ldexp(q.s2, 2 * d);
    }
    s1 = wave_reduce(s1, OpAdd());
    s2 = wave_reduce(s2, OpAdd());
    result = s1 * s1 / s2;
  }
  if (lane == 0) {
    ess[f] = result;
    if (fl && flags) atomicOr(flags, fl);
  }
}

// ================================================================ copy
// x_i <- x_{c_i} for every particle with c_i != i, on one buffer.  The copy
// is race-free when c satisfies the in-place predicate (a slot that is read
// is never written); a particle whose source is out of range or is itself
// overwritten (c_{c_i} != c_i) is left alone and flagged, which keeps the
// step race-free for any input.  Element (g, k) of the state (particle g,
// component k) sits at x[g * ps + k * cs].  A workgroup takes a tile of
// kCopyTile particles of one segment: with contiguous rows (cs == 1)
// consecutive threads take consecutive elements of the tile's rows; with
// contiguous columns a thread takes one particle and walks its components,
// consecutive threads taking consecutive particles.  Either way the stores
// are coalesced and the ancestry is read once per particle.
constexpr int kCopyTile = 1024;

template <typename E>
__device__ __forceinline__ bool copy_source(const int32_t* __restrict__ cs_, int64_t i, int64_t n,
                                            int64_t& ci, bool& bad) {
  ci = cs_[i];
  if (ci == i) return false;
  if (ci < 0 || ci >= n || cs_[ci] != ci) {
    bad = true;
    return false;
  }
  return true;
}

template <typename E>
__global__ __launch_bounds__(256) void k_copy(const int32_t* __restrict__ c, int64_t n_total,
                                              const int64_t* __restrict__ offsets,
                                              uint32_t n_filters, E* __restrict__ x, int32_t dim,
                                              int64_t ps, int64_t cs, bool rows,
                                              uint32_t* __restrict__ flags) {
  SlotSeg s;
  if (!slot_segment<kCopyTile>(offsets, n_filters, n_total, blockIdx.x, s)) return;
  const int64_t p0 = s.p * kCopyTile;
  const int tile = (int)min((int64_t)kCopyTile, s.n - p0);
  const int32_t* __restrict__ cseg = c + s.base;
  E* __restrict__ xs = x + s.base * ps;
  bool bad = false;
  if (rows) {
    const int64_t total = (int64_t)tile * dim;
    for (int64_t t = threadIdx.x; t < total; t += 256) {
      const int64_t il = t / dim;
      const int64_t k = t - il * dim;
      const int64_t i = p0 + il;
      int64_t ci;
      bool b = false;
      if (copy_source<E>(cseg, i, s.n, ci, b)) xs[i * ps + k] = xs[ci * ps + k];
      bad |= b && k == 0;
    }
  } else {
    for (int il = (int)threadIdx.x; il < tile; il += 256) {
      const int64_t i = p0 + il;
      int64_t ci;
      if (!copy_source<E>(cseg, i, s.n, ci, bad)) continue;
      for (int k = 0; k < dim; ++k) xs[i * ps + k * cs] = xs[ci * ps + k * cs];
    }
  }
  if (flags && ballot(bad) != 0 && lane_id() == 0) atomicOr(flags, FLAG_BAD_ANCESTOR);
}

// ================================================================ PRC weights
// Importance weight of each particle after partial rejection control:
// w_{a_i} / min(w_{a_i}, v_max), i.e. w_{a_i} / v_max above the bound, 1 at
// or below it, and 0 where the ancestor's weight is not positive (only a
// lane that hit the trial cap keeps such an ancestor).  The quotient is a
// binary64 division rounded to the weight type.
template <typename T>
__global__ __launch_bounds__(256) void k_prc_weights(const T* __restrict__ w, int64_t n_total,
                                                     const int64_t* __restrict__ offsets,
                                                     uint32_t n_filters, double v_max,
                                                     const double* __restrict__ v_max_dev,
                                                     const int32_t* __restrict__ a,
                                                     T* __restrict__ w_out) {
  SlotSeg s;
  if (!slot_segment<kCopyTile>(offsets, n_filters, n_total, blockIdx.x, s)) return;
  const double vm = v_max_dev ? v_max_dev[s.f] : v_max;
  const int64_t p0 = s.p * kCopyTile;
  const int tile = (int)min((int64_t)kCopyTile, s.n - p0);
  for (int il = (int)threadIdx.x; il < tile; il += 256) {
    const int64_t g = s.base + p0 + il;
    const int64_t ai = a[g];
    const double wa = (ai >= 0 && ai < s.n) ? (double)w[s.base + ai] : 0.0;
    double r = 0.0;
    if (wa > vm) r = wa / vm;
    else if (wa > 0.0) r = 1.0;
    w_out[g] = (T)r;
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_ancestors_to_offspring(const int32_t* a, int64_t n_total, const int64_t* offsets,
                                         uint32_t n_filters, int64_t max_len, bool sorted,
                                         int32_t* o, uint32_t* flags, hipStream_t stream) {
  if (!(offsets && n_filters > 1)) {
    offsets = nullptr;  // one segment covers [0, n_total)
    n_filters = 1;
    max_len = n_total;
  }
  if (sorted) {
    int64_t min_len = 0;  // shorter segments are converted in LDS
    if (offsets) {
      hipLaunchKernelGGL(k_a2o_staged, dim3(n_filters), dim3(kA2oStagedThreads), 0, stream, a,
                         offsets, n_filters, o, flags);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      if (max_len > 0 && max_len <= kA2oCap) return hipSuccess;
      min_len = kA2oCap + 1;
    }
    const uint32_t slots = slot_count<kA2oTile>(n_total, n_filters);
    hipLaunchKernelGGL(k_a2o_sorted_tiles, dim3(slots), dim3(kA2oThreads), 0, stream, a, n_total,
                       offsets, n_filters, min_len, o, flags);
    return hipGetLastError();
  }
  // a batch may hold both kinds of segment; each kernel skips the other kind
  const bool any_short = offsets ? true : n_total <= kA2oWinMax;
  const bool any_long = offsets ? (max_len <= 0 || max_len > kA2oWinMax) : n_total > kA2oWinMax;
  if (any_short) {
    const uint32_t slots = slot_count<kA2oWin>(n_total, n_filters);
    hipLaunchKernelGGL(k_a2o_window, dim3(slots), dim3(kA2oStagedThreads), 0, stream, a, n_total,
                       offsets, n_filters, o, flags);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (!any_long) return hipSuccess;
  const int64_t min_len = kA2oWinMax + 1;
  const uint32_t slots = slot_count<kA2oTile>(n_total, n_filters);
  hipLaunchKernelGGL(k_a2o_zero, dim3(slots), dim3(kA2oThreads), 0, stream, n_total, offsets,
                     n_filters, min_len, o);
  hipLaunchKernelGGL(k_a2o_atomic, dim3(slots), dim3(kA2oThreads), 0, stream, a, n_total,
                     offsets, n_filters, min_len, o, flags);
  return hipGetLastError();
}

size_t ess_workspace_bytes(int64_t n_total, uint32_t n_filters) {
  return align256((size_t)slot_count<kEssChunk>(n_total, n_filters) * sizeof(EssPart));
}

hipError_t launch_ess(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                      uint32_t n_filters, double* ess, void* ws, uint32_t* flags,
                      hipStream_t stream) {
  if (n_filters == 1) offsets = nullptr;
  EssPart* parts = (EssPart*)ws;
  const uint32_t slots = slot_count<kEssChunk>(n_total, n_filters);
  if (n_total > 0) {
    if (f64)
      hipLaunchKernelGGL(k_ess_partials<double>, dim3(slots), dim3(kEssThreads), 0, stream,
                         (const double*)w, n_total, offsets, n_filters, parts);
    else
      hipLaunchKernelGGL(k_ess_partials<float>, dim3(slots), dim3(kEssThreads), 0, stream,
                         (const float*)w, n_total, offsets, n_filters, parts);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ess_finish, dim3((n_filters + 3) / 4), dim3(256), 0, stream, n_total,
                     offsets, n_filters, parts, ess, flags);
  return hipGetLastError();
}

hipError_t launch_copy(const int32_t* c, int64_t n_total, const int64_t* offsets,
                       uint32_t n_filters, void* x, size_t elem_bytes, int32_t dim, int64_t ps,
                       int64_t cs, uint32_t* flags, hipStream_t stream) {
  if (n_filters == 1) offsets = nullptr;
  const bool rows = (cs == 1);
  const uint32_t grid = slot_count<kCopyTile>(n_total, n_filters);
  switch (elem_bytes) {
    case 1:
      hipLaunchKernelGGL(k_copy<uint8_t>, dim3(grid), dim3(256), 0, stream, c, n_total, offsets,
                         n_filters, (uint8_t*)x, dim, ps, cs, rows, flags);
      break;
    case 2:
      hipLaunchKernelGGL(k_copy<uint16_t>, dim3(grid), dim3(256), 0, stream, c, n_total, offsets,
                         n_filters, (uint16_t*)x, dim, ps, cs, rows, flags);
      break;
    case 4:
      hipLaunchKernelGGL(k_copy<uint32_t>, dim3(grid), dim3(256), 0, stream, c, n_total, offsets,
                         n_filters, (uint32_t*)x, dim, ps, cs, rows, flags);
      break;
    case 8:
      hipLaunchKernelGGL(k_copy<uint64_t>, dim3(grid), dim3(256), 0, stream, c, n_total, offsets,
                         n_filters, (uint64_t*)x, dim, ps, cs, rows, flags);
      break;
    case 16:
      hipLaunchKernelGGL(k_copy<uint4>, dim3(grid), dim3(256), 0, stream, c, n_total, offsets,
                         n_filters, (uint4*)x, dim, ps, cs, rows, flags);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_prc_weights(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                              uint32_t n_filters, double v_max, const double* v_max_dev,
                              const int32_t* a, void* w_out, hipStream_t stream) {
  if (n_filters == 1) offsets = nullptr;
  const uint32_t grid = slot_count<kCopyTile>(n_total, n_filters);
  if (f64)
    hipLaunchKernelGGL(k_prc_weights<double>, dim3(grid), dim3(256), 0, stream, (const double*)w,
                       n_total, offsets, n_filters, v_max, v_max_dev, a, (double*)w_out);
  else
    hipLaunchKernelGGL(k_prc_weights<float>, dim3(grid), dim3(256), 0, stream, (const float*)w,
                       n_total, offsets, n_filters, v_max, v_max_dev, a, (float*)w_out);
  return hipGetLastError();
}

}  // namespace pfr
