// pfr_aux.hip -- auxiliaries of the resampling step:
//   offspring_to_ancestors  (Code 11 of the paper after an exclusive scan of
//                            the offspring counts)
//   permute_ancestors       (Code 10: Prepermute, chain walk, gather)
#include "pfr_kernels.h"

namespace pfr {

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ================================================================ o2a
// Single pass with a decoupled look-back (Merrill & Garland, 2016) over tiles
// of 4096 counts.  Counts are exact integers, so the carry a tile obtains does
// not depend on how far it had to look back.  Tile ids come from a ticket so
// that every tile's predecessors are already running.
//
// Status word of a tile (64 bits):  [63:35] epoch  [34:33] kind  [32:0] value
// kind 1 = aggregate of the tile, 2 = inclusive prefix; a word whose epoch is
// not the current call's is treated as not yet written.  The epoch advances
// when the last tile of a call finishes, so the status array never needs to
// be cleared between calls (a zeroed workspace is a valid initial state).
constexpr int kO2aTile = 4096;
constexpr uint64_t kKindAgg = 1, kKindInc = 2;
constexpr uint64_t kValMask = (1ull << 33) - 1;

struct O2aHeader {
  uint32_t epoch;
  uint32_t tile_ticket;
  uint32_t done;
  uint32_t pad[61];
};

__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint64_t kind, uint64_t value) {
  return ((uint64_t)(epoch & 0x1FFFFFFFu) << 35) | (kind << 33) | (value & kValMask);
}
__device__ __forceinline__ uint64_t status_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Offspring values of a tile in (g, lane, v) order per wave; negative counts
// count as 0 and counts above n as n + 1 (both raise FLAG_BAD_COUNTS), so sums
// stay far below 2^33 per tile.
__device__ __forceinline__ void load_counts(const int32_t* __restrict__ o, int64_t n, int64_t base,
                                            uint64_t (&q)[16], uint32_t& bad) {
  const int lane = (int)lane_id();
  const bool aligned = ((reinterpret_cast<uintptr_t>(o + base) & 15u) == 0);
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int64_t idx = base + (int64_t)g * 256 + lane * 4;
    int32_t v4[4];
    if (aligned && idx + 4 <= n) {
      const int4 t = *reinterpret_cast<const int4*>(o + idx);
      v4[0] = t.x; v4[1] = t.y; v4[2] = t.z; v4[3] = t.w;
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) v4[v] = (idx + v < n) ? o[idx + v] : 0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int64_t x = v4[v];
      if (x < 0) { bad = FLAG_BAD_COUNTS; x = 0; }
      if (x > n) { bad = FLAG_BAD_COUNTS; x = n + 1; }
      q[g * 4 + v] = (uint64_t)x;
    }
  }
}

template <int G, int V>
__device__ __forceinline__ uint64_t inclusive_scan16(uint64_t (&q)[16]) {
  uint64_t run = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    uint64_t s = 0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      s += q[g * V + v];
      q[g * V + v] = s;
    }
    const uint64_t incl = wave_inclusive_scan(s, OpAdd());
    const uint64_t add = run + (incl - s);
#pragma unroll
    for (int v = 0; v < V; ++v) q[g * V + v] += add;
    run += readlane(incl, kWave - 1);
  }
  return run;
}

// Expansion of one tile: positions s in [lo, hi) get P0 + #{i : O_i <= s},
// where O (inclusive cumulative counts, saturated at n + 1) sits in LDS.
__device__ __forceinline__ void expand_tile(const uint32_t* __restrict__ O_lds, int cnt,
                                            int64_t lo, int64_t hi, int64_t P0,
                                            int32_t* __restrict__ a, int tid, int nthreads) {
  for (int64_t s = lo + tid; s < hi; s += nthreads) {
    int l = 0, h = cnt;
    while (l < h) {
      const int m = (l + h) >> 1;
      if ((int64_t)O_lds[m] <= s) l = m + 1;
      else h = m;
    }
    a[s] = (int32_t)(P0 + l);
  }
}

// Builds the tile's cumulative counts in LDS (4 waves x 1024) given its carry
// and returns through the arguments the tile total.
__device__ __forceinline__ void tile_counts_to_lds(uint64_t (&q)[16], uint64_t carry, int64_t n,
                                                   uint32_t* __restrict__ O_lds, int wave,
                                                   const uint64_t* wave_prefix) {
  const int lane = (int)lane_id();
#pragma unroll
  for (int g = 0; g < 4; ++g) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      uint64_t O = carry + wave_prefix[wave] + q[g * 4 + v];
      if (O > (uint64_t)n + 1) O = (uint64_t)n + 1;
      O_lds[wave * 1024 + g * 256 + lane * 4 + v] = (uint32_t)O;
    }
  }
}

__global__ __launch_bounds__(256) void k_o2a(const int32_t* __restrict__ o, int64_t n,
                                             int32_t* __restrict__ a, O2aHeader* __restrict__ hdr,
                                             uint64_t* __restrict__ status,
                                             uint32_t* __restrict__ flags, uint32_t ntiles) {
  __shared__ uint32_t O_lds[kO2aTile];
  __shared__ uint64_t wave_tot[4], wave_prefix[4];
  __shared__ uint32_t s_tile, s_epoch, s_bad;
  __shared__ uint64_t s_carry;
  const int tid = (int)threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  if (tid == 0) {
    s_tile = atomicAdd(&hdr->tile_ticket, 1u);
    s_epoch = __hip_atomic_load(&hdr->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_bad = 0;
  }
  __syncthreads();
  const uint32_t t = s_tile, epoch = s_epoch;
  const int64_t P0 = (int64_t)t * kO2aTile;
  uint64_t q[16];
  uint32_t bad = 0;
  load_counts(o, n, P0 + wave * 1024, q, bad);
  const uint64_t wsum = inclusive_scan16<4, 4>(q);
  if (lane == 0) wave_tot[wave] = wsum;
  bad = wave_reduce(bad, OpOr());
  if (lane == 0 && bad) atomicOr(&s_bad, bad);
  __syncthreads();
  if (tid == 0) {
    uint64_t run = 0;
    for (int w2 = 0; w2 < 4; ++w2) {
      wave_prefix[w2] = run;
      run += wave_tot[w2];
    }
    const uint64_t agg = run > (uint64_t)n + 1 ? (uint64_t)n + 1 : run;
    if (t == 0) {
      s_carry = 0;
      status_store(&status[0], pack_status(epoch, kKindInc, agg));
    } else {
      status_store(&status[t], pack_status(epoch, kKindAgg, agg));
    }
  }
  __syncthreads();
  // look-back by wave 0: lane l inspects tile t-1-l
  if (t > 0 && wave == 0) {
    uint64_t carry = 0;
    int64_t pos = (int64_t)t - 1;  // highest tile not yet accounted for
    while (true) {
      const int64_t j = pos - lane;
      uint64_t st = 0, kind = 0;
      bool ready = true;
      if (j >= 0) {
        st = status_load(&status[j]);
        kind = ((uint32_t)(st >> 35) == (epoch & 0x1FFFFFFFu)) ? ((st >> 33) & 3u) : 0u;
        ready = kind != 0;
      }
      // lanes up to (and including) the nearest inclusive tile must be ready
      const uint64_t inc_mask = ballot(j >= 0 && kind == kKindInc);
      const uint64_t end_mask = inc_mask | ballot(j < 0);
      const int stop = end_mask ? (__ffsll((long long)end_mask) - 1) : kWave;  // first lane that ends the walk
      const uint64_t need = (stop >= kWave - 1) ? ~0ull : ((2ull << stop) - 1);
      if ((ballot(!ready) & need) != 0) {
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      const uint64_t val = (j >= 0 && lane <= stop) ? (st & kValMask) : 0;
      carry += wave_reduce(val, OpAdd());
      if (stop < kWave) break;
      pos -= kWave;
    }
    if (carry > (uint64_t)n + 1) carry = (uint64_t)n + 1;
    if (lane == 0) {
      s_carry = carry;
      uint64_t inc = carry + wave_prefix[3] + wave_tot[3];
      if (inc > (uint64_t)n + 1) inc = (uint64_t)n + 1;
      status_store(&status[t], pack_status(epoch, kKindInc, inc));
    }
  }
  __syncthreads();
  const uint64_t carry = s_carry;
  tile_counts_to_lds(q, carry, n, O_lds, wave, wave_prefix);
  __syncthreads();
  uint64_t total = carry + wave_prefix[3] + wave_tot[3];
  if (total > (uint64_t)n + 1) total = (uint64_t)n + 1;
  const int cnt = (int)min((int64_t)kO2aTile, n - P0);
  const int64_t lo = min((int64_t)carry, n), hi = min((int64_t)total, n);
  expand_tile(O_lds, cnt, lo, hi, P0, a, tid, 256);
  uint32_t fl = s_bad;
  if (t == ntiles - 1) {
    // positions beyond the last offspring keep the identity
    for (int64_t s = hi + tid; s < n; s += 256) a[s] = (int32_t)s;
    if (total != (uint64_t)n) fl |= FLAG_BAD_COUNTS;
  }
  if (tid == 0) {
    if (fl && flags) atomicOr(flags, fl);
    __threadfence();
    const uint32_t prev = atomicAdd(&hdr->done, 1u);
    if (prev == ntiles - 1) {  // last tile out: next call gets a new epoch
      hdr->tile_ticket = 0;
      hdr->done = 0;
      __hip_atomic_store(&hdr->epoch, (epoch + 1) & 0x1FFFFFFFu, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
    }
  }
}

// Ragged batch: one workgroup per segment walks its tiles in order and keeps
// the carry in a register.
__global__ __launch_bounds__(256) void k_o2a_batched(const int32_t* __restrict__ o,
                                                     int64_t n_total,
                                                     const int64_t* __restrict__ offsets,
                                                     uint32_t n_filters, int32_t* __restrict__ a,
                                                     uint32_t* __restrict__ flags) {
  __shared__ uint32_t O_lds[kO2aTile];
  __shared__ uint64_t wave_tot[4], wave_prefix[4];
  __shared__ uint32_t s_bad;
  const uint32_t f = blockIdx.x;
  if (f >= n_filters) return;
  const int tid = (int)threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int64_t base = offsets ? offsets[f] : 0;
  const int64_t n = offsets ? offsets[f + 1] - base : n_total;
  const int32_t* __restrict__ os = o + base;
  int32_t* __restrict__ as = a + base;
  if (tid == 0) s_bad = 0;
  uint64_t carry = 0;
  for (int64_t P0 = 0; P0 < n; P0 += kO2aTile) {
    uint64_t q[16];
    uint32_t bad = 0;
    load_counts(os, n, P0 + wave * 1024, q, bad);
    const uint64_t wsum = inclusive_scan16<4, 4>(q);
    if (lane == 0) wave_tot[wave] = wsum;
    bad = wave_reduce(bad, OpOr());
    __syncthreads();
    if (lane == 0 && bad) atomicOr(&s_bad, bad);
    if (tid == 0) {
      uint64_t run = 0;
      for (int w2 = 0; w2 < 4; ++w2) {
        wave_prefix[w2] = run;
        run += wave_tot[w2];
      }
    }
    __syncthreads();
    tile_counts_to_lds(q, carry, n, O_lds, wave, wave_prefix);
    __syncthreads();
    uint64_t total = carry + wave_prefix[3] + wave_tot[3];
    if (total > (uint64_t)n + 1) total = (uint64_t)n + 1;
    const int cnt = (int)min((int64_t)kO2aTile, n - P0);
    expand_tile(O_lds, cnt, min((int64_t)carry, n), min((int64_t)total, n), P0, as, tid, 256);
    carry = total;
    __syncthreads();
  }
  const int64_t hi = min((int64_t)carry, n);
  for (int64_t s = hi + tid; s < n; s += 256) as[s] = (int32_t)s;
  __syncthreads();
  if (tid == 0 && flags) {
    uint32_t fl = s_bad;
    if (carry != (uint64_t)n) fl |= FLAG_BAD_COUNTS;
    if (fl) atomicOr(flags, fl);
  }
}

// ================================================================ permute
// Code 10.  d[j] holds the particle index that claims slot j, or n (unclaimed).
// Prepermute keeps the lowest claimer of every slot.  For a sorted ancestry
// (the output of the collective resamplers) the lowest claimer of slot a_i is
// the first i of its run, so the claim vector is written with plain stores in
// one pass: position i writes slot a_i when it starts a run, and n into every
// slot strictly between a_{i-1} and a_i, which no position claims.  For an
// unsorted ancestry the claim vector is filled with n and the lowest claimer
// found with an atomic minimum (a relaxed load first skips the atomic once a
// lower claimer is in place).
//
// Permute then lets every failed claimer i follow x <- d_x from x = i to an
// unclaimed slot and take it; finally c_j = a_{d_j}.  The chains are disjoint
// paths (the paper's termination argument), one per failed claimer, each
// ending in its own unclaimed slot.  The resolve kernel walks them backwards
// instead: a claimed slot j keeps c_j = j; from an unclaimed slot j it steps
// y <- a_y for as long as position y is the winning claimer of slot a_y
// (d[a_y] == y), which retraces the one chain that ends at j back to its
// failed claimer y, and sets c_j = a_y.  This is the same c as Code 10, reads
// only a and d, and needs no second pass over d.
struct SegIdx {
  int64_t base, n, i;
};

__device__ __forceinline__ SegIdx seg_index(const int64_t* __restrict__ offsets, uint32_t n_filters,
                                            int64_t n_total, int64_t g) {
  SegIdx s;
  if (!offsets) {
    s.base = 0;
    s.n = n_total;
  } else {
    const uint32_t f = find_segment(offsets, n_filters, g);
    s.base = offsets[f];
    s.n = offsets[f + 1] - s.base;
  }
  s.i = g - s.base;
  return s;
}

// ancestor of local position i, with out-of-range values replaced by i
__device__ __forceinline__ int64_t anc_at(const int32_t* __restrict__ a, const SegIdx& s, int64_t i,
                                          bool& bad) {
  const int64_t v = a[s.base + i];
  if (v < 0 || v >= s.n) {
    bad = true;
    return i;
  }
  return v;
}

__global__ __launch_bounds__(256) void k_claim_sorted(const int32_t* __restrict__ a,
                                                      int64_t n_total,
                                                      const int64_t* __restrict__ offsets,
                                                      uint32_t n_filters, int64_t min_len,
                                                      int32_t* __restrict__ d,
                                                      int32_t* __restrict__ e,
                                                      uint32_t* __restrict__ flags) {
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_total; g += stride) {
    const SegIdx s = seg_index(offsets, n_filters, n_total, g);
    if (s.n < min_len) continue;  // permuted in LDS by k_permute_staged
    const int64_t ai = anc_at(a, s, s.i, bad);
    const int64_t prev = (s.i == 0) ? -1 : anc_at(a, s, s.i - 1, bad);
    int32_t* ds = d + s.base;
    e[g] = ai > prev ? (int32_t)ai : (int32_t)(-1 - ai);
    if (ai > prev) {
      ds[ai] = (int32_t)s.i;  // first of its run
      for (int64_t j = prev + 1; j < ai; ++j) ds[j] = (int32_t)s.n;
    }
    if (s.i == s.n - 1) {
      const int64_t top = ai > prev ? ai : prev;
      for (int64_t j = top + 1; j < s.n; ++j) ds[j] = (int32_t)s.n;
    }
  }
  if (flags) {
    const uint32_t b = (uint32_t)wave_reduce((uint32_t)bad, OpOr());
    if (b && lane_id() == 0) atomicOr(flags, FLAG_BAD_ANCESTOR);
  }
}

__global__ __launch_bounds__(256) void k_fill_unclaimed(int32_t* __restrict__ d, int64_t n_total,
                                                        const int64_t* __restrict__ offsets,
                                                        uint32_t n_filters, int64_t min_len) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_total; g += stride) {
    const SegIdx s = seg_index(offsets, n_filters, n_total, g);
    if (s.n < min_len) continue;
    d[g] = (int32_t)s.n;
  }
}

// Claims of one workgroup are first merged in LDS: a 256-entry table keyed
// by the slot's low bits keeps the smallest (slot, position) pair per entry,
// and a position whose entry holds the same slot with a smaller position
// cannot win, so it issues no global atomic.  Equal ancestors inside a
// workgroup (degenerate weights: every particle descends from one) then cost
// one atomic per workgroup instead of one per particle, all on one address.
// Positions whose entry holds another slot still claim, so the result is the
// same minimum as without the table.  Slots are global indices (< 2^31).
__global__ __launch_bounds__(256) void k_claim_min(const int32_t* __restrict__ a, int64_t n_total,
                                                   const int64_t* __restrict__ offsets,
                                                   uint32_t n_filters, int64_t min_len,
                                                   int32_t* __restrict__ d,
                                                   uint32_t* __restrict__ flags) {
  __shared__ unsigned long long tab[256];
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g0 = (int64_t)blockIdx.x * blockDim.x; g0 < n_total; g0 += stride) {
    const int64_t g = g0 + threadIdx.x;
    bool valid = false;
    uint32_t slot = 0, pos = 0;
    if (g < n_total) {
      const SegIdx s = seg_index(offsets, n_filters, n_total, g);
      if (s.n >= min_len) {
        valid = true;
        slot = (uint32_t)(s.base + anc_at(a, s, s.i, bad));
        pos = (uint32_t)s.i;
      }
    }
    const unsigned long long key = ((unsigned long long)slot << 32) | pos;
    tab[threadIdx.x] = ~0ull;
    __syncthreads();
    if (valid) atomicMin(&tab[slot & 255u], key);
    __syncthreads();
    if (valid) {
      const unsigned long long best = tab[slot & 255u];
      const bool beaten = (uint32_t)(best >> 32) == slot && (uint32_t)best < pos;
      int32_t* dst = &d[slot];
      // d only decreases, so a stale (cached) value that is already <= pos
      // proves the claim lost; only a larger one needs the atomic
      if (!beaten &&
          __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) > (int32_t)pos)
        atomicMin(dst, (int32_t)pos);
    }
    __syncthreads();  // the table is reset by the next iteration
  }
  if (flags) {
    const uint32_t b = (uint32_t)wave_reduce((uint32_t)bad, OpOr());
    if (b && lane_id() == 0) atomicOr(flags, FLAG_BAD_ANCESTOR);
  }
}

// e[i] = a_i if position i won its claim (d[a_i] == i), else -1 - a_i.
__global__ __launch_bounds__(256) void k_mark(const int32_t* __restrict__ a, int64_t n_total,
                                              const int64_t* __restrict__ offsets,
                                              uint32_t n_filters, int64_t min_len,
                                              const int32_t* __restrict__ d,
                                              int32_t* __restrict__ e) {
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_total; g += stride) {
    const SegIdx s = seg_index(offsets, n_filters, n_total, g);
    if (s.n < min_len) continue;
    const int64_t ai = anc_at(a, s, s.i, bad);
    e[g] = d[s.base + ai] == s.i ? (int32_t)ai : (int32_t)(-1 - ai);
  }
}

// Backward walk on the ancestry itself (unsorted input, no marked ancestry):
// from an unclaimed slot j, y = j; while position y won its claim
// (d[a_y] == y) step to y = a_y; then c_j = a_y.  The same walk as k_resolve
// on e = marks(a, d), with the mark of each visited position formed on the
// way (two dependent loads per step instead of one), which saves the pass
// that writes e.  d[j] and a[j] are loaded together.
__global__ __launch_bounds__(256) void k_resolve_ad(const int32_t* __restrict__ a,
                                                    int64_t n_total,
                                                    const int64_t* __restrict__ offsets,
                                                    uint32_t n_filters, int64_t min_len,
                                                    const int32_t* __restrict__ d,
                                                    int32_t* __restrict__ c,
                                                    uint32_t* __restrict__ flags) {
  bool broken = false, bad = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_total; g += stride) {
    const SegIdx s = seg_index(offsets, n_filters, n_total, g);
    if (s.n < min_len) continue;
    const int64_t j = s.i;
    const int64_t dj = d[g];
    int64_t ay = anc_at(a, s, j, bad);
    if (dj >= 0 && dj < s.n) {  // claimed: its winner's ancestor is j
      c[g] = (int32_t)j;
      continue;
    }
    // unclaimed: retrace the chain that ends here back to its failed claimer
    const int32_t* ds = d + s.base;
    int64_t y = j;
    int64_t steps = 0;
    bool br = false;
    while (ds[ay] == y) {  // position y won slot a_y: the chain came through it
      y = ay;
      ay = anc_at(a, s, y, bad);
      if (++steps > s.n) {  // a chain visits distinct slots; only bad input gets here
        br = true;
        break;
      }
    }
    broken |= br;
    c[g] = br ? (int32_t)j : (int32_t)ay;
  }
  if (flags) {
    const uint32_t b = (uint32_t)wave_reduce((uint32_t)(broken ? FLAG_BAD_ANCESTOR : 0u), OpOr());
    if (b && lane_id() == 0) atomicOr(flags, b);
  }
}

// Backward walk on e: one dependent load per chain step.
__global__ __launch_bounds__(256) void k_resolve(int64_t n_total,
                                                 const int64_t* __restrict__ offsets,
                                                 uint32_t n_filters, int64_t min_len,
                                                 const int32_t* __restrict__ d,
                                                 const int32_t* __restrict__ e,
                                                 int32_t* __restrict__ c,
                                                 uint32_t* __restrict__ flags) {
  bool broken = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_total; g += stride) {
    const SegIdx s = seg_index(offsets, n_filters, n_total, g);
    if (s.n < min_len) continue;
    const int64_t j = s.i;
    const int64_t dj = d[g];
    const int32_t* es = e + s.base;
    int64_t ey = es[j];  // loaded with d[g]: the two loads are in flight together
    if (dj >= 0 && dj < s.n) {  // claimed: its winner's ancestor is j
      c[g] = (int32_t)j;
      continue;
    }
    // unclaimed: retrace the chain that ends here back to its failed claimer
    int64_t steps = 0;
    while (ey >= 0) {
      ey = es[ey];
      if (++steps > s.n) {  // a chain visits distinct slots; only bad input gets here
        broken = true;
        break;
      }
    }
    c[g] = broken ? (int32_t)j : (int32_t)(-1 - ey);
  }
  if (flags) {
    const uint32_t b = (uint32_t)wave_reduce((uint32_t)(broken ? FLAG_BAD_ANCESTOR : 0u), OpOr());
    if (b && lane_id() == 0) atomicOr(flags, b);
  }
}

// Segments of at most CAP particles, one workgroup each, entirely in LDS: the
// claim vector d (minimum claimer per slot, by LDS atomic minimum), then the
// marked ancestry e overwrites d (a claimed-slot bitmap keeps what resolve
// needs of d), then every slot resolves as in k_resolve.  Global traffic is
// the ancestry read and the permutation written.
constexpr int kPermThreads = 1024;
// Single vectors up to these lengths are permuted in LDS by one workgroup
// (one launch instead of two to four); beyond them the multi-workgroup
// kernels are faster (measured on MI355X: the crossover lies near 2^10
// particles for a sorted ancestry and 2^12 for an unsorted one).
constexpr int kPermSingleMax = 4096;
constexpr int kPermSingleMaxSorted = 1024;

template <int CAP>
__global__ __launch_bounds__(kPermThreads) void k_permute_staged(
    const int32_t* __restrict__ a, int64_t n_total, const int64_t* __restrict__ offsets,
    uint32_t n_filters, int32_t* __restrict__ c, uint32_t* __restrict__ flags) {
  __shared__ int32_t de[CAP];
  __shared__ uint32_t claimed[CAP / 32];
  constexpr int kPer = CAP / kPermThreads;  // particles per thread
  const uint32_t f = blockIdx.x;
  const int64_t base = offsets ? offsets[f] : 0;
  const int64_t n64 = offsets ? offsets[f + 1] - base : n_total;
  if (n64 <= 0 || n64 > CAP) return;  // long segments: global kernels
  const int32_t n = (int32_t)n64;
  const int tid = (int)threadIdx.x;
  bool bad = false;
  // ancestor of local position i; out-of-range values count as i
  auto anc = [&](int32_t i) -> int32_t {
    const int32_t v = a[base + i];
    return (v < 0 || v >= n) ? i : v;
  };
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int32_t i = tid + q * kPermThreads;
    de[i] = n;
    if (q * kPermThreads < CAP / 32 && i < CAP / 32) claimed[i] = 0u;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int32_t i = tid + q * kPermThreads;
    if (i < n) {
      const int32_t v = a[base + i];
      if (v < 0 || v >= n) bad = true;
      atomicMin(&de[(v < 0 || v >= n) ? i : v], i);
    }
  }
  __syncthreads();
  int32_t ev[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int32_t i = tid + q * kPermThreads;
    ev[q] = 0;
    if (i < n) {
      const int32_t ai = anc(i);
      ev[q] = de[ai] == i ? ai : -1 - ai;
      if (de[i] < n) atomicOr(&claimed[i >> 5], 1u << (i & 31));
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int32_t i = tid + q * kPermThreads;
    if (i < n) de[i] = ev[q];
  }
  __syncthreads();
  bool broken = false;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int32_t j = tid + q * kPermThreads;
    if (j >= n) continue;
    if ((claimed[j >> 5] >> (j & 31)) & 1u) {
      c[base + j] = j;
      continue;
    }
    int32_t ey = de[j];
    int32_t steps = 0;
    bool br = false;
    while (ey >= 0) {
      ey = de[ey];
      if (++steps > n) {
        br = true;
        break;
      }
    }
    broken |= br;
    c[base + j] = br ? j : -1 - ey;
  }
  if (flags) {
    const uint32_t fl = (bad || broken) ? FLAG_BAD_ANCESTOR : 0u;
    const uint32_t b = wave_reduce(fl, OpOr());
    if (b && lane_id() == 0) atomicOr(flags, b);
  }
}

// ---------------------------------------------------------------- bucketed claim
// The claim vector of one unsorted vector without global atomics.  The slots
// fall into B buckets of S consecutive slots and the positions into W chunks
// of C; (1) every chunk counts its claims per bucket, (2) one workgroup per
// bucket scans its chunks' counts (the bucket totals give the buckets' bases),
// (3) every chunk writes its (position, slot) pairs to those places (the
// order inside a bucket does not matter), and (4) one workgroup per bucket
// takes the minimum claimer of each of its slots in LDS, writes that part of
// d (unclaimed: n) and the mark e_i = a_i of every winner; (3) has marked
// every position as a loser (-1 - a_i) before.  Claims that lose inside their
// own chunk get no pair.  k_resolve then walks e.  The minimum does not depend
// on the order, so d and e are those of the atomic claim.  Traffic: a read
// four times (8 + 8 bytes, half from the L2), 4 + 8 + 8 bytes of marks and
// pairs, 4 of d, and one scattered 4-byte write per claimed slot.
struct BucketGeom {
  int64_t n;
  uint32_t S, C, B, W;  // slots per bucket, positions per chunk, buckets, chunks
  int log2S;
  size_t cnt_off, tot_off, pairs_off, bytes;  // workspace parts after d and e
};

constexpr int kBucketMax = 4096;  // buckets (LDS counters of the chunk kernels)
constexpr int kBucketSlotsMax = 32768;
constexpr int kBucketThreads = 1024;
constexpr int kClaimThreads = 1024;

__host__ __device__ inline uint32_t pow2_at_least(int64_t x) {
  uint32_t p = 1;
  while ((int64_t)p < x && p < (1u << 30)) p <<= 1;
  return p;
}

BucketGeom bucket_geom(int64_t n) {
  BucketGeom g;
  g.n = n;
  // about 256 buckets and 1024 chunks: S and C powers of two, S from 4096 to
  // kBucketSlotsMax (the claim kernel's LDS table), C from 4096
  const uint32_t t = pow2_at_least((n + 255) / 256), tc = pow2_at_least((n + 1023) / 1024);
  g.S = t < 4096 ? 4096 : (t > (uint32_t)kBucketSlotsMax ? (uint32_t)kBucketSlotsMax : t);
  g.C = tc < 4096 ? 4096 : tc;
  g.log2S = 0;
  while ((1u << g.log2S) < g.S) ++g.log2S;
  g.B = (uint32_t)((n + g.S - 1) / g.S);
  g.W = (uint32_t)((n + g.C - 1) / g.C);
  const size_t base = 2 * align256((size_t)n * sizeof(int32_t));  // d, e
  const size_t pairs = (size_t)g.B * g.W;
  g.cnt_off = base;
  g.tot_off = g.cnt_off + align256(pairs * sizeof(uint32_t));
  g.pairs_off = g.tot_off + align256((size_t)g.B * sizeof(uint32_t));
  g.bytes = g.pairs_off + align256((size_t)n * sizeof(uint64_t));
  return g;
}

// the bucketed claim applies to single vectors of up to 2^31 - 1 particles
// whose bucket count fits the chunk kernels' LDS counters
bool bucket_claim_fits(int64_t n) {
  return n > 0 && n < ((int64_t)1 << 31) && bucket_geom(n).B <= (uint32_t)kBucketMax;
}

// slot claimed by position i (out-of-range ancestors claim their own index)
__device__ __forceinline__ uint32_t claim_slot(int32_t v, uint32_t i, uint32_t n, bool& bad) {
  if (v < 0 || (uint32_t)v >= n) {
    bad = true;
    return i;
  }
  return (uint32_t)v;
}

// Positions of chunk w, four per thread and round, their loads issued together
// (clamped to the chunk; f(i, slot) is called for the positions inside it).
template <typename F>
__device__ __forceinline__ void chunk_claims(const int32_t* __restrict__ a, uint32_t n,
                                             uint32_t p0, uint32_t p1, bool& bad, F f) {
  for (uint32_t i0 = p0; i0 < p1; i0 += 4 * kBucketThreads) {
    int32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      v[k] = a[min(i0 + (uint32_t)(k * kBucketThreads) + threadIdx.x, p1 - 1)];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = i0 + (uint32_t)(k * kBucketThreads) + threadIdx.x;
      if (i < p1) f(i, claim_slot(v[k], i, n, bad));
    }
  }
}

// Equal claims inside a chunk are merged first: an LDS table keyed by the
// slot's low bits keeps the smallest (slot, position) per entry, and a
// position whose entry holds its slot with a smaller position has lost (it is
// not the minimum claimer), so it needs no pair.  Distinct slots sharing an
// entry all keep their pairs.  An ancestry with one parent then gives one
// pair per chunk instead of one per particle.
constexpr int kDedup = 4096;
__device__ __forceinline__ void dedup_fill(const int32_t* __restrict__ a, uint32_t n, uint32_t p0,
                                           uint32_t p1, unsigned long long* tab, bool& bad) {
  for (uint32_t k = threadIdx.x; k < kDedup; k += kBucketThreads) tab[k] = ~0ull;
  __syncthreads();
  chunk_claims(a, n, p0, p1, bad, [&](uint32_t i, uint32_t slot) {
    atomicMin(&tab[slot & (kDedup - 1)], ((unsigned long long)slot << 32) | i);
  });
  __syncthreads();
}
__device__ __forceinline__ bool dedup_lost(const unsigned long long* tab, uint32_t slot,
                                           uint32_t i) {
  const unsigned long long best = tab[slot & (kDedup - 1)];
  return (uint32_t)(best >> 32) == slot && (uint32_t)best < i;
}

__global__ __launch_bounds__(kBucketThreads) void k_bucket_count(
    const int32_t* __restrict__ a, uint32_t n, int log2S, uint32_t C, uint32_t B, uint32_t W,
    uint32_t* __restrict__ cnt, uint32_t* __restrict__ flags) {
  __shared__ uint32_t hist[kBucketMax];
  __shared__ unsigned long long tab[kDedup];
  const uint32_t w = blockIdx.x;
  for (uint32_t b = threadIdx.x; b < B; b += kBucketThreads) hist[b] = 0;
  bool bad = false;
  const uint32_t p0 = w * C, p1 = min(n, p0 + C);
  dedup_fill(a, n, p0, p1, tab, bad);
  chunk_claims(a, n, p0, p1, bad, [&](uint32_t i, uint32_t slot) {
    if (!dedup_lost(tab, slot, i)) atomicAdd(&hist[slot >> log2S], 1u);
  });
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < B; b += kBucketThreads) cnt[(size_t)b * W + w] = hist[b];
  if (flags) {
    const uint32_t f = (uint32_t)wave_reduce((uint32_t)bad, OpOr());
    if (f && lane_id() == 0) atomicOr(flags, FLAG_BAD_ANCESTOR);
  }
}

// Exclusive scan in place of each bucket's W chunk counts (row b of the
// bucket-major count matrix), one workgroup per bucket; the row total goes to
// tot[b].  The bucket's first pair, the sum of the totals of the buckets
// before it, is formed by its readers (bucket_bases).
__global__ __launch_bounds__(kBucketThreads) void k_bucket_rows(uint32_t* __restrict__ cnt,
                                                                uint32_t W,
                                                                uint32_t* __restrict__ tot) {
  __shared__ uint32_t s_w[kBucketThreads / kWave];
  const int tid = (int)threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  uint32_t* row = cnt + (size_t)blockIdx.x * W;
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < W; c0 += kBucketThreads) {
    const uint32_t j = c0 + (uint32_t)tid;
    const uint32_t x = j < W ? row[j] : 0u;
    const uint32_t inc = wave_incl_add_u32(x);
    if (lane == kWave - 1) s_w[wave] = inc;
    __syncthreads();
    uint32_t before = carry + inc - x, t = 0;
    for (int w2 = 0; w2 < kBucketThreads / kWave; ++w2) {
      before += w2 < wave ? s_w[w2] : 0u;
      t += s_w[w2];
    }
    if (j < W) row[j] = before;
    carry += t;
    __syncthreads();
  }
  if (tid == 0) tot[blockIdx.x] = carry;
}

// base[b] = sum of tot[b'] for b' < b, for b <= B, by the calling workgroup
// (kBucketThreads threads, B <= kBucketMax; s_w holds kBucketThreads / 64).
__device__ void bucket_bases(const uint32_t* __restrict__ tot, uint32_t B, uint32_t* base,
                             uint32_t* s_w) {
  const int tid = (int)threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  constexpr int kPerT = kBucketMax / kBucketThreads;  // 4 consecutive buckets per thread
  uint32_t x[kPerT], run = 0;
#pragma unroll
  for (int k = 0; k < kPerT; ++k) {
    const uint32_t b = (uint32_t)tid * kPerT + k;
    const uint32_t v = b < B ? tot[b] : 0u;
    x[k] = run;
    run += v;
  }
  const uint32_t inc = wave_incl_add_u32(run);
  if (lane == kWave - 1) s_w[wave] = inc;
  __syncthreads();
  uint32_t before = inc - run;
  for (int w2 = 0; w2 < wave; ++w2) before += s_w[w2];
#pragma unroll
  for (int k = 0; k < kPerT; ++k) {
    const uint32_t b = (uint32_t)tid * kPerT + k;
    if (b <= B) base[b] = before + x[k];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kBucketThreads) void k_bucket_scatter(
    const int32_t* __restrict__ a, uint32_t n, int log2S, uint32_t C, uint32_t B, uint32_t W,
    const uint32_t* __restrict__ off, const uint32_t* __restrict__ tot,
    uint64_t* __restrict__ pairs, int32_t* __restrict__ e) {
  __shared__ uint32_t cur[kBucketMax + 1];
  __shared__ uint32_t s_w[kBucketThreads / kWave];
  __shared__ unsigned long long tab[kDedup];
  const uint32_t w = blockIdx.x;
  bucket_bases(tot, B, cur, s_w);
  for (uint32_t b = threadIdx.x; b < B; b += kBucketThreads) cur[b] += off[(size_t)b * W + w];
  bool bad = false;
  const uint32_t p0 = w * C, p1 = min(n, p0 + C);
  dedup_fill(a, n, p0, p1, tab, bad);
  // every position is marked as a loser here (in order, coalesced); the
  // claim kernel then marks the winners, one per claimed slot
  chunk_claims(a, n, p0, p1, bad, [&](uint32_t i, uint32_t slot) {
    e[i] = -1 - (int32_t)slot;
    if (!dedup_lost(tab, slot, i)) {  // (a loser here: a smaller position of the chunk claims it)
      const uint32_t r = atomicAdd(&cur[slot >> log2S], 1u);
      pairs[r] = ((uint64_t)i << 32) | slot;
    }
  });
}

// The pairs [q0, q1) of a bucket, four per thread and round, loads together.
template <typename F>
__device__ __forceinline__ void bucket_pairs(const uint64_t* __restrict__ pairs, uint32_t q0,
                                             uint32_t q1, F f) {
  for (uint32_t b0 = q0; b0 < q1; b0 += 4 * kClaimThreads) {
    uint64_t p[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      p[k] = pairs[min(b0 + (uint32_t)(k * kClaimThreads) + threadIdx.x, q1 - 1)];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (b0 + (uint32_t)(k * kClaimThreads) + threadIdx.x < q1)
        f((uint32_t)(p[k] >> 32), (uint32_t)p[k]);
  }
}

__global__ __launch_bounds__(kClaimThreads) void k_bucket_claim(
    uint32_t n, uint32_t S, const uint32_t* __restrict__ tot,
    const uint64_t* __restrict__ pairs, int32_t* __restrict__ d, int32_t* __restrict__ e) {
  __shared__ uint32_t tab[kBucketSlotsMax];
  __shared__ uint32_t s_q[kClaimThreads / kWave];
  const uint32_t b = blockIdx.x;
  const uint32_t s0 = b * S, ns = min(S, n - s0);
  for (uint32_t k = threadIdx.x; k < ns; k += kClaimThreads) tab[k] = n;
  // the bucket's first pair: the pairs of the buckets before it
  uint32_t q = 0;
  for (uint32_t k = threadIdx.x; k < b; k += kClaimThreads) q += tot[k];
  q = wave_reduce(q, OpAdd());
  if (lane_id() == 0) s_q[threadIdx.x / kWave] = q;
  __syncthreads();
  uint32_t q0 = 0;
  for (int w2 = 0; w2 < kClaimThreads / kWave; ++w2) q0 += s_q[w2];
  const uint32_t q1 = q0 + tot[b];
  bucket_pairs(pairs, q0, q1, [&](uint32_t i, uint32_t slot) { atomicMin(&tab[slot - s0], i); });
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < ns; k += kClaimThreads) {
    const uint32_t i = tab[k];
    d[s0 + k] = (int32_t)i;
    if (i < n) e[i] = (int32_t)(s0 + k);  // the winner of slot s0 + k
  }
}

int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

size_t o2a_workspace_bytes(int64_t n_total) {
  const size_t tiles = (size_t)((n_total + kO2aTile - 1) / kO2aTile);
  return 256 + align256(tiles * sizeof(uint64_t));
}

hipError_t launch_offspring_to_ancestors(const int32_t* o, int64_t n_total, const int64_t* offsets,
                                         uint32_t n_filters, int32_t* a, void* ws,
                                         uint32_t* flags, hipStream_t stream) {
  if (offsets || n_filters > 1 || n_total <= kO2aTile) {
    hipLaunchKernelGGL(k_o2a_batched, dim3(offsets ? n_filters : 1u), dim3(256), 0, stream, o,
                       n_total, offsets, offsets ? n_filters : 1u, a, flags);
    return hipGetLastError();
  }
  const uint32_t ntiles = (uint32_t)((n_total + kO2aTile - 1) / kO2aTile);
  O2aHeader* hdr = (O2aHeader*)ws;
  uint64_t* status = (uint64_t*)((char*)ws + 256);
  hipLaunchKernelGGL(k_o2a, dim3(ntiles), dim3(256), 0, stream, o, n_total, a, hdr, status, flags,
                     ntiles);
  return hipGetLastError();
}

// Workspace: the claim vector d and the marked ancestry e, n int32 each; a
// single unsorted vector beyond the LDS path also gets the bucketed claim's
// counts and pairs (8 more bytes per particle), without which it takes the
// atomic claim.
size_t permute_workspace_min_bytes(int64_t n_total) {
  return 2 * align256((size_t)n_total * sizeof(int32_t));
}
size_t permute_workspace_bytes(int64_t n_total, uint32_t n_filters) {
  if (n_filters <= 1 && n_total > kPermSingleMax && bucket_claim_fits(n_total))
    return bucket_geom(n_total).bytes;
  return permute_workspace_min_bytes(n_total);
}

// Batches whose segments fit in LDS, and short single vectors, are permuted
// there (k_permute_staged, one workgroup per segment); longer segments go
// through the global kernels.  max_len: longest segment (0 = unknown).
hipError_t launch_permute(const int32_t* a, int64_t n_total, const int64_t* offsets,
                          uint32_t n_filters, int64_t max_len, bool sorted, int32_t* c, void* ws,
                          size_t ws_bytes, uint32_t* flags, hipStream_t stream) {
  int32_t* d = (int32_t*)ws;
  int32_t* e = (int32_t*)((char*)ws + align256((size_t)n_total * sizeof(int32_t)));
  const int grid = grid_for(n_total);
  int64_t min_len = 0;  // shorter segments are done in LDS
  if (!(offsets && n_filters > 1) && n_total <= (sorted ? kPermSingleMaxSorted : kPermSingleMax)) {
    // a short single vector: one workgroup, one launch
    hipLaunchKernelGGL(k_permute_staged<kPermSingleMax>, dim3(1), dim3(kPermThreads), 0, stream,
                       a, n_total, nullptr, 1u, c, flags);
    return hipGetLastError();
  }
  if (offsets && n_filters > 1) {
    // segments up to the tuned length in LDS, the longer ones below
    const int cap = tuning().batch_permute_lds_max;
    if (cap == 4096)
      hipLaunchKernelGGL(k_permute_staged<4096>, dim3(n_filters), dim3(kPermThreads), 0, stream,
                         a, n_total, offsets, n_filters, c, flags);
    else if (cap == 8192)
      hipLaunchKernelGGL(k_permute_staged<8192>, dim3(n_filters), dim3(kPermThreads), 0, stream,
                         a, n_total, offsets, n_filters, c, flags);
    else
      hipLaunchKernelGGL(k_permute_staged<16384>, dim3(n_filters), dim3(kPermThreads), 0, stream,
                         a, n_total, offsets, n_filters, c, flags);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
    if (max_len > 0 && max_len <= cap) return hipSuccess;
    min_len = cap + 1;
  }
  if (sorted) {
    hipLaunchKernelGGL(k_claim_sorted, dim3(grid), dim3(256), 0, stream, a, n_total, offsets,
                       n_filters, min_len, d, e, flags);
    hipLaunchKernelGGL(k_resolve, dim3(grid), dim3(256), 0, stream, n_total, offsets, n_filters,
                       min_len, d, e, c, flags);
    return hipGetLastError();
  }
  if (!(offsets && n_filters > 1) && bucket_claim_fits(n_total) &&
      ws_bytes >= bucket_geom(n_total).bytes) {
    // one vector: the bucketed claim writes d and e, then the walk on e
    const BucketGeom g = bucket_geom(n_total);
    char* base = (char*)ws;
    uint32_t* cnt = (uint32_t*)(base + g.cnt_off);
    uint32_t* tot = (uint32_t*)(base + g.tot_off);
    uint64_t* pairs = (uint64_t*)(base + g.pairs_off);
    const uint32_t n = (uint32_t)n_total;
    hipLaunchKernelGGL(k_bucket_count, dim3(g.W), dim3(kBucketThreads), 0, stream, a, n, g.log2S,
                       g.C, g.B, g.W, cnt, flags);
    hipLaunchKernelGGL(k_bucket_rows, dim3(g.B), dim3(kBucketThreads), 0, stream, cnt, g.W, tot);
    hipLaunchKernelGGL(k_bucket_scatter, dim3(g.W), dim3(kBucketThreads), 0, stream, a, n,
                       g.log2S, g.C, g.B, g.W, (const uint32_t*)cnt, (const uint32_t*)tot, pairs,
                       e);
    hipLaunchKernelGGL(k_bucket_claim, dim3(g.B), dim3(kClaimThreads), 0, stream, n, g.S,
                       (const uint32_t*)tot, (const uint64_t*)pairs, d, e);
    hipLaunchKernelGGL(k_resolve, dim3(grid), dim3(256), 0, stream, n_total, offsets, n_filters,
                       min_len, d, e, c, flags);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_fill_unclaimed, dim3(grid), dim3(256), 0, stream, d, n_total, offsets,
                     n_filters, min_len);
  hipLaunchKernelGGL(k_claim_min, dim3(grid), dim3(256), 0, stream, a, n_total, offsets,
                     n_filters, min_len, d, flags);
  hipLaunchKernelGGL(k_resolve_ad, dim3(grid), dim3(256), 0, stream, a, n_total, offsets,
                     n_filters, min_len, d, c, flags);
  return hipGetLastError();
}

int32_t* permute_claims(void* ws) { return (int32_t*)ws; }
int32_t* permute_marks(void* ws, int64_t n_total) {
  return (int32_t*)((char*)ws + align256((size_t)n_total * sizeof(int32_t)));
}

hipError_t launch_resolve(int64_t n_total, int32_t* c, void* ws, uint32_t* flags,
                          hipStream_t stream) {
  hipLaunchKernelGGL(k_resolve, dim3(grid_for(n_total)), dim3(256), 0, stream, n_total,
                     (const int64_t*)nullptr, 1u, (int64_t)0, permute_claims(ws),
                     permute_marks(ws, n_total), c, flags);
  return hipGetLastError();
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, size_t count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0;
}

hipError_t launch_zero_u32(uint32_t* p, size_t count, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)blocks), dim3(256), 0, stream, p, count);
  return hipGetLastError();
}

}  // namespace pfr
