// pfr_scan.hip -- the collective resamplers: multinomial (Code 5 of the
// paper), stratified (Code 7) and systematic (Code 8).
//
// All three compute the scaled prefix r_i = n W_i / W_n of the weights and map
// sorted points onto it:
//   stratified   point q_s = s + 1 - u_s in (s, s+1], ancestor = min{i : r_i >= q_s}
//   systematic   the same with one offset u for all strata
//   multinomial  p_k = n S_k / S_n from exponential spacings (sorted uniforms),
//                ancestor = #{i < n-1 : r_i <= p_k}
// i.e. Code 7/8 followed by Code 11, and Code 5 with an upper-bound search.
//
// Exact prefix sums.  The paper shows that a float32 prefix sum biases these
// schemes for large n.  Here each block of 1024 weights is quantised to
// integers q = floor(w * 2^s_b) < 2^53 relative to the block maximum (every
// float32 weight within 2^29 of the block maximum is represented exactly),
// block sums are exact 64-bit integers, and the carries between blocks are
// exact 128-bit integers at one global scale.  Integer sums do not depend on
// the order of addition, so the prefix is deterministic, monotone, exactly
// flat across zero weights and consistent at every block boundary; the only
// rounding is the final map r = n * I / I_total to binary64, itself monotone
// with r = n at the end.
//
// One vector: one wave handles one block, 16 consecutive weights per lane
// (four 16-byte loads for float32), four waves per workgroup.  Passes:
//   records one record per block (validity, block scale, quantised sum), and
//           one sum per exponential-spacing block of the multinomial scheme
//           (whose points are kept for the emission).
//   carries one workgroup of 1024 threads turns the records into the global
//           scale, the exact carries C_b and the total, and scans the
//           exponential-block sums.  With at most direct_max_blocks blocks
//           and no exponential blocks this step is folded into the emission:
//           every emit workgroup reduces all records itself, which costs less
//           than one more launch.
//   emit    each block rebuilds its exact prefix, I = C_b + local prefix, and
//           r = n I / Q (a wave scan through DPP).  Stratified / systematic:
//           every particle computes its cumulative offspring
//           O_i = #{s : q_s <= r_i} in O(1), and the block's output range
//           [O(C_b), O(C_b+1)) is filled through LDS markers and a wave
//           max-scan, then written coalesced.  Multinomial: each block reads
//           the exponential blocks whose points fall in its r-range and
//           settles its particles with interleaved binary searches in LDS.
// The workgroup-per-block variants (256 threads, 4 weights per thread) serve
// the single-workgroup path of short vectors and the batch kernels.
// Ragged batches run the same steps inside one workgroup per filter.
#include "pfr_kernels.h"

namespace pfr {

namespace {
#include "pfr_scan_common.h"


// ---------------------------------------------------------------- records
// Record of the block at base: validity, reference exponent (block maximum),
// quantised sum.  Same value in every thread.
template <typename T>
__device__ BlockRec block_record(const T* __restrict__ w, int64_t n, int64_t base, WgScratch* s) {
  T x[kPer];
  load4(w, n, base, x);
  uint32_t bad = 0;
  uint32_t emax = 1;
#pragma unroll
  for (int v = 0; v < kPer; ++v) {
    if (!weight_ok(x[v])) bad = FLAG_BAD_WEIGHTS;
    else emax = max(emax, (uint32_t)exp_field(x[v]));
  }
  // pack (bad, emax) into one max-reduction: bad dominates
  const uint32_t key = (bad << 16) | emax;
  const uint32_t red = wg_reduce(key, OpMax(), (uint32_t*)s->i);
  BlockRec r;
  r.bad = red >> 16;
  const int e_ref = (int)(red & 0xFFFFu);
  uint64_t sum = 0;
  if (!r.bad) {
#pragma unroll
    for (int v = 0; v < kPer; ++v) sum += quantize(x[v], e_ref);
  }
  r.sum = wg_reduce(sum, OpAdd(), s->u);
  r.scale = scale_of<T>(e_ref);
  return r;
}


__device__ __forceinline__ u128 conv_rec(const BlockRec& r, int32_t gscale) {
  return shift_u128((u128)r.sum, gscale - r.scale);
}

// ---------------------------------------------------------------- carries
// From nb records: global scale, exact exclusive carries C[0..nb] (C[nb] is
// the total) and status.  Whole workgroup; records are read in chunks of
// kBlock, 4 consecutive per thread, all loads of a chunk issued together.
struct Totals {
  u128 Q;
  int32_t gscale;
  uint32_t status;
};

template <typename RecPtr, typename CPtr>
__device__ Totals carries_from_records(uint32_t nb, RecPtr recs, CPtr C, WgScratch* s) {
  const int tid = (int)threadIdx.x;
  uint32_t bad = 0;
  uint32_t smin_key = 0xFFFFFFFFu;  // scale + 2^31, min over non-empty blocks
  for (uint32_t base = 0; base < nb; base += kBlock) {
    BlockRec r[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t b = base + (uint32_t)tid * kPer + k;
      if (b < nb) r[k] = recs[b];
      else r[k].sum = 0, r[k].scale = 0, r[k].bad = 0;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      bad |= r[k].bad;
      if (r[k].sum) smin_key = min(smin_key, (uint32_t)r[k].scale ^ 0x80000000u);
    }
  }
  bad = wg_reduce(bad, OpOr(), (uint32_t*)s->i);
  smin_key = wg_reduce(smin_key, OpMin(), (uint32_t*)s->i);
  Totals t;
  // every converted block sum is below 2^(63 + gscale - smin); nb of them stay
  // below 2^kCarryBits
  t.gscale = (smin_key == 0xFFFFFFFFu)
                 ? 0
                 : (int32_t)(smin_key ^ 0x80000000u) + (kCarryBits - 63) - ceil_log2(nb);
  u128 carry = 0;
  for (uint32_t base = 0; base < nb; base += kBlock) {
    u128 v[kPer];
    u128 mine = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t b = base + (uint32_t)tid * kPer + k;
      v[k] = (b < nb) ? conv_rec(recs[b], t.gscale) : (u128)0;
      mine += v[k];
    }
    u128 tot;
    u128 run = carry + wg_exclusive(mine, s->v, &tot);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t b = base + (uint32_t)tid * kPer + k;
      if (b < nb) C[b] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (tid == 0) C[nb] = carry;
  __syncthreads();
  t.Q = carry;
  t.status = bad;
  if (!bad && carry == 0) t.status |= FLAG_ZERO_TOTAL;
  return t;
}

// ---------------------------------------------------------------- kernels
// ---------------------------------------------------------------- carries
// Two levels.  The records fall into groups of kGrp = 1024 consecutive
// blocks.  k_carry_groups (one 256-thread workgroup per group, all in
// parallel) fixes the group's own scale gs_g from its largest block, exactly
// as the global scale is fixed from the largest block overall (with the
// group's 2^10 blocks in place of nb, so group sums stay below 2^100), and
// writes every block's exclusive prefix P_b inside the group at that scale
// and the group total T_g.  The group workgroup that finishes last (a count
// in the header, zeroed by the records pass) takes the global scale from the
// group keys, converts each T_g to it (a shift: truncation when gs_g is
// finer) and scans them into Tx_g; the total Q is Tx_G.  The
// carry of block b in group g is then
//   C_b = Tx_g + floor(P_b 2^(gscale - gs_g)),  C_nb = Q,
// an integer function of the records alone, monotone in b and continuous at
// group ends (P at a group's end is T_g).  It differs from converting every
// block to the global scale by truncation only (one unit of the global scale
// per group), within the bound of the per-block quantisation.  The
// exponential-block sums of the multinomial scheme are plain integers and
// take the same two levels without scales.
constexpr int kGrpLog = 10;
constexpr uint32_t kGrp = 1u << kGrpLog;
constexpr int kGPer = (int)kGrp / kT;  // blocks per thread of a group workgroup (4)

struct CarryGroup {
  u128 T;        // group total at the group's scale (exponential groups: plain sum)
  int32_t gs;    // the group's scale
  uint32_t key;  // min over non-empty blocks of scale ^ 2^31, ~0u if none
  uint32_t bad;
  uint32_t pad;
};

// conv_rec with 64-bit shifts only.  A non-empty block's shift is at most
// kCarryBits - 63 (a group's or the global scale exceeds no non-empty block's
// scale by more), and an empty block converts to zero under any shift, so
// clamping the left shift to 63 changes nothing.
static_assert(kCarryBits - 63 < 64, "left shifts of block sums stay below 64");
__device__ __forceinline__ u128 conv_rec_fast(const BlockRec& r, int32_t scale) {
  const int sh = scale - r.scale;
  const uint64_t s = r.sum;
  const uint32_t l = (uint32_t)min(max(sh, 0), 63), d = (uint32_t)min(-sh, 64);
  const uint64_t lo = sh >= 0 ? s << l : (d >= 64 ? 0ull : s >> d);
  const uint64_t hi = l > 0 ? s >> (64 - l) : 0ull;
  return ((u128)hi << 64) | lo;
}

// Exclusive scan of the kGrp values x (kGPer consecutive per thread) of one
// workgroup; returns the thread's exclusive base and the workgroup total.
__device__ __forceinline__ u128 group_scan(u128 (&x)[kGPer], u128* s_w, u128* total) {
  const int wave = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  u128 run = 0;
#pragma unroll
  for (int k = 0; k < kGPer; ++k) {
    const u128 v = x[k];
    x[k] = run;
    run += v;
  }
  const u128 inc = wave_incl_add_u128(run);
  if (lane == kWave - 1) s_w[wave] = inc;
  __syncthreads();
  u128 before = inc - run, tot = 0;
#pragma unroll
  for (int w2 = 0; w2 < kNW; ++w2) {
    const u128 t = s_w[w2];
    before += w2 < wave ? t : (u128)0;
    tot += t;
  }
  *total = tot;
  return before;
}

// Exclusive scan, in index order, of val(j) for j < m by a workgroup of NT
// threads (CK consecutive values per thread per chunk); put(j, prefix) gets
// each result.  Returns the total; s_w holds NT / 64 values.
template <int NT, int CK, typename Val, typename Put>
__device__ u128 wg_scan_blocked(uint32_t m, Val val, Put put, u128* s_w) {
  constexpr int NW = NT / kWave;
  constexpr uint32_t chunk = (uint32_t)NT * CK;
  const int tid = (int)threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  u128 carry = 0;
  for (uint32_t c0 = 0; c0 < m; c0 += chunk) {
    const uint32_t j0 = c0 + (uint32_t)tid * CK;
    u128 x[CK];
#pragma unroll
    for (int k = 0; k < CK; ++k) x[k] = j0 + (uint32_t)k < m ? val(j0 + (uint32_t)k) : (u128)0;
    u128 run = 0;
#pragma unroll
    for (int k = 0; k < CK; ++k) {
      const u128 v = x[k];
      x[k] = run;
      run += v;
    }
    const u128 inc = wave_incl_add_u128(run);
    if (lane == kWave - 1) s_w[wave] = inc;
    __syncthreads();
    u128 before = carry + (inc - run), tot = 0;
#pragma unroll 2
    for (int w2 = 0; w2 < NW; ++w2) {
      const u128 t = s_w[w2];
      before += w2 < wave ? t : (u128)0;
      tot += t;
    }
#pragma unroll
    for (int k = 0; k < CK; ++k)
      if (j0 + (uint32_t)k < m) put(j0 + (uint32_t)k, before + x[k]);
    carry += tot;
    __syncthreads();
  }
  return carry;
}

// The top level over the G group records (and the Ge exponential ones): global
// scale, status, Tx[0..G] and TEx[0..Ge].  Run by the group workgroup that
// finishes last (kT threads; G <= 2048 for n < 2^31, one chunk).
template <bool MULTI>
__device__ void carry_top(uint32_t nb, uint32_t G, uint32_t Ge,
                          const CarryGroup* __restrict__ groups,
                          const CarryGroup* __restrict__ egroups, u128* __restrict__ Tx,
                          u128* __restrict__ TEx, ScanHeader* __restrict__ hdr, uint32_t* s_u,
                          u128* s_w) {
  const int tid = (int)threadIdx.x;
  uint32_t bad = 0, key = 0xFFFFFFFFu;
  for (uint32_t g = (uint32_t)tid; g < G; g += kT) {
    bad |= groups[g].bad;
    key = min(key, groups[g].key);
  }
  key = wg_reduce(key, OpMin(), s_u);
  bad = wg_reduce(bad, OpOr(), s_u + kNW);
  const int32_t gscale =
      key == 0xFFFFFFFFu ? 0 : (int32_t)(key ^ 0x80000000u) + (kCarryBits - 63) - ceil_log2(nb);
  const u128 Q = wg_scan_blocked<kT, 8>(
      G, [&](uint32_t g) { return shift_u128(groups[g].T, gscale - groups[g].gs); },
      [&](uint32_t g, u128 c) { Tx[g] = c; }, s_w);
  if (MULTI) {
    const u128 S = wg_scan_blocked<kT, 8>(
        Ge, [&](uint32_t g) { return egroups[g].T; }, [&](uint32_t g, u128 c) { TEx[g] = c; },
        s_w);
    if (tid == 0) TEx[Ge] = S;
  }
  if (tid == 0) {
    Tx[G] = Q;
    uint32_t status = bad;
    if (!bad && Q == 0) status |= FLAG_ZERO_TOTAL;
    hdr->status = status;
    hdr->gscale = gscale;
    hdr->Q = Q;
  }
}

// The group step: group g of the weight blocks (weights) or of the
// exponential blocks; its scale, every block's prefix inside it and its
// record.  All kT threads call it.
__device__ void carry_group(bool weights, uint32_t g, uint32_t m,
                            const BlockRec* __restrict__ recs,
                            const uint64_t* __restrict__ esums, u128* __restrict__ out,
                            CarryGroup* __restrict__ rec_out, u128* s_w, uint32_t* s_u) {
  const int tid = (int)threadIdx.x;
  const uint32_t j0 = g * kGrp + (uint32_t)tid * kGPer;
  u128 x[kGPer];
  uint32_t key = 0xFFFFFFFFu, bad = 0;
  int32_t gs = 0;
  if (weights) {
    BlockRec r[kGPer];
#pragma unroll
    for (int k = 0; k < kGPer; ++k) {
      if (j0 + k < m) r[k] = recs[j0 + k];
      else r[k].sum = 0, r[k].scale = 0, r[k].bad = 0;
    }
#pragma unroll
    for (int k = 0; k < kGPer; ++k) {
      bad |= r[k].bad;
      if (r[k].sum) key = min(key, (uint32_t)r[k].scale ^ 0x80000000u);
    }
    key = wg_reduce(key, OpMin(), s_u);
    bad = wg_reduce(bad, OpOr(), s_u + kNW);
    gs = key == 0xFFFFFFFFu ? 0 : (int32_t)(key ^ 0x80000000u) + (kCarryBits - 63) - kGrpLog;
#pragma unroll
    for (int k = 0; k < kGPer; ++k) x[k] = conv_rec_fast(r[k], gs);
  } else {
#pragma unroll
    for (int k = 0; k < kGPer; ++k) x[k] = j0 + k < m ? (u128)esums[j0 + k] : (u128)0;
  }
  u128 total;
  const u128 before = group_scan(x, s_w, &total);
#pragma unroll
  for (int k = 0; k < kGPer; ++k)
    if (j0 + k < m) out[j0 + k] = before + x[k];
  if (tid == 0) {
    CarryGroup c;
    c.T = total;
    c.gs = gs;
    c.key = key;
    c.bad = bad;
    c.pad = 0;
    rec_out[g] = c;
  }
}

// With a single group in all (strata schemes up to 2^20 particles) its
// workgroup goes on to the top level: no count and no fences.  Otherwise one
// workgroup per group, and the last to finish runs the top level (measured:
// one workgroup taking the three groups of a 2^20 multinomial call in turn,
// 9.7 us, is slower than three in parallel with the count, 8.8 us).
constexpr uint32_t kFewGroups = 1;

template <bool MULTI>
__global__ __launch_bounds__(kT) void k_carry_groups(uint32_t nb, uint32_t nbe, uint32_t G,
                                                     const BlockRec* __restrict__ recs,
                                                     const uint64_t* __restrict__ esums,
                                                     u128* __restrict__ P, u128* __restrict__ PE,
                                                     CarryGroup* __restrict__ groups,
                                                     CarryGroup* __restrict__ egroups,
                                                     uint32_t Ge, u128* __restrict__ Tx,
                                                     u128* __restrict__ TEx,
                                                     ScanHeader* __restrict__ hdr) {
  __shared__ u128 s_w[kNW];
  __shared__ uint32_t s_u[2 * kNW];
  __shared__ uint32_t s_last;
  if (G + (MULTI ? Ge : 0u) <= kFewGroups) {
    for (uint32_t g = 0; g < G; ++g) {
      carry_group(true, g, nb, recs, esums, P, groups, s_w, s_u);
      __syncthreads();  // the scratch is reused; the group records are read by all
    }
    if (MULTI) {
      for (uint32_t g = 0; g < Ge; ++g) {
        carry_group(false, g, nbe, recs, esums, PE, egroups, s_w, s_u);
        __syncthreads();
      }
    }
    carry_top<MULTI>(nb, G, Ge, groups, egroups, Tx, TEx, hdr, s_u, s_w);
    return;
  }
  const bool weights = blockIdx.x < G;
  if (!MULTI && !weights) return;  // (never: the grid has G workgroups then)
  const uint32_t g = weights ? blockIdx.x : blockIdx.x - G;
  carry_group(weights, g, weights ? nb : nbe, recs, esums, weights ? P : PE,
              weights ? groups : egroups, s_w, s_u);
  if (threadIdx.x == 0) {
    // the last group to finish (the records pass zeroed the count) runs the
    // top level: release this group's record, count it, acquire the others
    __threadfence();
    s_last = atomicAdd(&hdr->groups_done, 1u) == G + (MULTI ? Ge : 0u) - 1u ? 1u : 0u;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  carry_top<MULTI>(nb, G, Ge, groups, egroups, Tx, TEx, hdr, s_u, s_w);
}

// The exact carry C_b of block b (0 <= b <= nb) from the two levels.
struct Carries {
  const u128* __restrict__ P;
  const u128* __restrict__ Tx;
  const CarryGroup* __restrict__ grp;
  uint32_t nb, G;
  int32_t gscale;
  __device__ __forceinline__ u128 operator[](uint32_t b) const {
    if (b >= nb) return Tx[G];
    const uint32_t g = b >> kGrpLog;
    return Tx[g] + shift_u128(P[b], gscale - grp[g].gs);
  }
};

// The exponential-block carries CE[e] (0 <= e <= nbe) from the two levels.
struct ECarries {
  const u128* __restrict__ PE;
  const u128* __restrict__ TEx;
  uint32_t nbe, Ge;
  __device__ __forceinline__ u128 operator[](uint32_t e) const {
    if (e >= nbe) return TEx[Ge];
    return TEx[e >> kGrpLog] + PE[e];
  }
};

__host__ __device__ constexpr uint32_t carry_groups(uint32_t nblocks) {
  return (nblocks + kGrp - 1) / kGrp;
}

// Direct carries: with at most kDirectMax blocks every emit workgroup derives
// the global scale, its own exact carry and the total from all records itself,
// which saves the carry kernel.
constexpr uint32_t kDirectMax = kT * 8;

// ---------------------------------------------------------------- one block per wave
// The stratified and systematic emission and the records pass run one
// 1024-weight block per wave, lane l holding particles 16 l .. 16 l + 15 of
// the block, four waves (four consecutive blocks) per workgroup.  A block's
// prefix then needs no workgroup barrier: the lane sums its 16 quantised
// weights and one DPP scan over the wave gives the lane's offset.  r is formed
// from the exact block carry by an affine map in binary64,
//   r_i = min(fl(L_i c + r(C_b)), r(C_{b+1})),  c = n 2^(gscale - scale_b) / Q,
// with L_i the block's exact integer prefix (below 2^63) rounded once: the map
// is monotone in L_i, flat over zero weights and clamped to the block's range,
// so O_i is monotone across blocks as well; it adds at most five roundings of
// n 2^-53 to the error of r against the exact value.
constexpr int kWPer = kBlock / kWave;  // particles per lane (16)
constexpr int kWavesPerWG = kT / kWave;
constexpr int kUTabW = 2048;           // stratum offset words cached per wave

template <typename T>
__device__ __forceinline__ void wave_load(const T* __restrict__ w, int64_t n, int64_t base,
                                          T (&x)[kWPer]) {
  const int64_t idx = base + (int64_t)lane_id() * kWPer;
  const bool aligned = ((reinterpret_cast<uintptr_t>(w + idx) & 15u) == 0);
  if (aligned && idx + kWPer <= n) {
    if constexpr (sizeof(T) == 4) {
      const float4* p = reinterpret_cast<const float4*>(w + idx);
#pragma unroll
      for (int k = 0; k < kWPer / 4; ++k) {
        const float4 t = p[k];
        x[4 * k] = t.x; x[4 * k + 1] = t.y; x[4 * k + 2] = t.z; x[4 * k + 3] = t.w;
      }
    } else {
      const double2* p = reinterpret_cast<const double2*>(w + idx);
#pragma unroll
      for (int k = 0; k < kWPer / 2; ++k) {
        const double2 t = p[k];
        x[2 * k] = t.x; x[2 * k + 1] = t.y;
      }
    }
  } else {
#pragma unroll
    for (int v = 0; v < kWPer; ++v) x[v] = (idx + v < n) ? w[idx + v] : (T)0;
  }
}

// The block's weights in an order in which every load instruction is
// coalesced (lane l takes the 16-byte pieces l, l + 64, ... of the block), for
// the record, whose maximum and sum do not depend on the order.  Values past
// the vector's end are zero.
template <typename T>
__device__ __forceinline__ void wave_load_unordered(const T* __restrict__ w, int64_t n,
                                                    int64_t base, T (&x)[kWPer]) {
  constexpr int kV = 16 / (int)sizeof(T);  // values per 16-byte piece
  const int lane = (int)lane_id();
  const bool aligned = ((reinterpret_cast<uintptr_t>(w + base) & 15u) == 0);
  if (aligned && base + kBlock <= n) {
#pragma unroll
    for (int k = 0; k < kWPer / kV; ++k) {
      const int64_t idx = base + (int64_t)(k * kWave + lane) * kV;
      if constexpr (sizeof(T) == 4) {
        const float4 t = *reinterpret_cast<const float4*>(w + idx);
        x[4 * k] = t.x; x[4 * k + 1] = t.y; x[4 * k + 2] = t.z; x[4 * k + 3] = t.w;
      } else {
        const double2 t = *reinterpret_cast<const double2*>(w + idx);
        x[2 * k] = t.x; x[2 * k + 1] = t.y;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < kWPer / kV; ++k)
#pragma unroll
      for (int v = 0; v < kV; ++v) {
        const int64_t idx = base + (int64_t)(k * kWave + lane) * kV + v;
        x[kV * k + v] = idx < n ? w[idx] : (T)0;
      }
  }
}

// wave_load of a whole, 16-byte aligned float32 block through 4 KB of the
// wave's LDS: the global loads are coalesced (lane l takes the 16-byte pieces
// l, l + 64, ...) and the lanes read their 16 consecutive weights back.  Piece
// u sits at u ^ ((u >> 4) & 3), so that 16 lanes reading pieces 4l + k touch
// 16 different bank groups.  Other blocks and binary64 load directly.
template <typename T>
__device__ __forceinline__ void wave_load_staged(const T* __restrict__ w, int64_t n, int64_t base,
                                                 T (&x)[kWPer], int32_t* stage) {
  if constexpr (sizeof(T) == 4) {
    const bool aligned = ((reinterpret_cast<uintptr_t>(w + base) & 15u) == 0);
    if (stage && aligned && base + kBlock <= n) {
      const int lane = (int)lane_id();
      const float4* g = reinterpret_cast<const float4*>(w + base);
      float4* S = reinterpret_cast<float4*>(stage);
      float4 t[kWPer / 4];
#pragma unroll
      for (int k = 0; k < kWPer / 4; ++k) t[k] = g[k * kWave + lane];
#pragma unroll
      for (int k = 0; k < kWPer / 4; ++k) {
        const int u = k * kWave + lane;
        S[u ^ ((u >> 4) & 3)] = t[k];
      }
      wave_lds_sync();
#pragma unroll
      for (int k = 0; k < kWPer / 4; ++k) {
        const int u = lane * (kWPer / 4) + k;
        const float4 v = S[u ^ ((u >> 4) & 3)];
        x[4 * k] = v.x; x[4 * k + 1] = v.y; x[4 * k + 2] = v.z; x[4 * k + 3] = v.w;
      }
      wave_lds_sync();
      return;
    }
  }
  wave_load(w, n, base, x);
}

// quantize() without branches: q = floor(v 2^scale) for every finite v >= 0
// of a block whose scale keeps q below 2^53.  binary32: scaling by a power of
// two is exact (a result below 2^-126 may round, but it floors to zero
// anyway), the floor is exact, and q splits exactly into two 32-bit halves
// (t - hi 2^32 keeps at most t's 24 significant bits).  binary64: the
// significand shifted by scale + exponent - 1075, truncated.
template <typename T>
__device__ __forceinline__ uint64_t quantize_nb(T v, int scale) {
  if constexpr (sizeof(T) == 4) {
    const float t = floorf(ldexpf(v, scale));
    const float hi = floorf(t * 0x1p-32f);
    const float lo = __builtin_fmaf(hi, -0x1p32f, t);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
  } else {
    typedef WTraits<T> Tr;
    const uint64_t b = Tr::bits(v);
    const uint32_t ef = (uint32_t)((b >> 52) & 0x7FFu);
    const uint64_t m = (b & 0xFFFFFFFFFFFFFull) | (ef ? (1ull << 52) : 0ull);
    const int sh = (int)(ef < 1u ? 1u : ef) - 1075 + scale;
    const uint64_t up = m << (sh & 63);
    const uint64_t dn = m >> (uint32_t)min(-sh, 63);
    return sh >= 0 ? up : dn;
  }
}

// u64 -> binary64, rounded once (the high half converts exactly).
__device__ __forceinline__ double u64_to_f64(uint64_t x) { return (double)x; }

// Record of the block at base (one wave): validity, reference exponent, sum.
template <typename T>
__device__ __forceinline__ BlockRec wave_block_record(const T* __restrict__ w, int64_t n, int64_t base) {
  T x[kWPer];
  wave_load_unordered(w, n, base, x);
  uint32_t bad = 0, emax = 1;
#pragma unroll
  for (int v = 0; v < kWPer; ++v) {
    if (!weight_ok(x[v])) bad = FLAG_BAD_WEIGHTS;
    else emax = max(emax, (uint32_t)exp_field(x[v]));
  }
  const uint32_t key = wave_reduce((bad << 16) | emax, OpMax());
  BlockRec r;
  r.bad = key >> 16;
  const int e_ref = (int)(key & 0xFFFFu);
  r.scale = scale_of<T>(e_ref);
  uint64_t sum = 0;
  if (!r.bad) {
#pragma unroll
    for (int v = 0; v < kWPer; ++v) sum += quantize_nb(x[v], r.scale);
  }
  r.sum = readlane(wave_incl_add_u64(sum), kWave - 1);
  return r;
}

// r of the wave's block: lane l gets r_i of particles P0 + 16 l + v (values
// past the vector's end repeat the last one), and the block's range
// [r(C_b), r(C_{b+1})].
struct BlockR {
  double r[kWPer];
  double lo, hi;
};

template <typename T>
__device__ __forceinline__ void block_r_wave(const T* __restrict__ w, int64_t n, int64_t P0,
                                             const BlockRec rec, u128 Cb, u128 Cb1,
                                             int32_t gscale, u128 Q, BlockR& R,
                                             int32_t* stage = nullptr) {
  const RMap rm = make_rmap(Q, n);
  R.lo = rm(Cb);
  R.hi = rm(Cb1);
  const int32_t scale = (int32_t)__builtin_amdgcn_readfirstlane(rec.scale);
  const int sh = (int32_t)__builtin_amdgcn_readfirstlane(gscale) - scale;
  const double c = ldexp(rm.Nd * rm.invQ, sh);
  T x[kWPer];
  wave_load_staged(w, n, P0, x, stage);
  uint64_t q[kWPer];
  uint64_t acc = 0;
#pragma unroll
  for (int v = 0; v < kWPer; ++v) {
    acc += quantize_nb(x[v], scale);
    q[v] = acc;
  }
  const uint64_t incl = wave_incl_add_u64(acc);
  const uint64_t off = incl - acc;
  const uint64_t total = readlane(incl, kWave - 1);
  // every particle from the block's last positive weight on has the whole
  // block sum, i.e. r = r(C_{b+1}) exactly: that particle then ends the
  // block's range, as in exact arithmetic
#pragma unroll
  for (int v = 0; v < kWPer; ++v) {
    const uint64_t Lv = off + q[v];
    const double rv = __fma_rn(u64_to_f64(Lv), c, R.lo);
    R.r[v] = (Lv == total || rv > R.hi) ? R.hi : rv;
  }
}

// Expansion of cumulative offspring into ancestors, 1024 outputs at a time:
// the block's outputs are [O_lo, O_hi) and particle P0 + 16 lane + v takes
// [Op[v], O[v]).  A marker at the first output of every run, a max-scan (16
// values per lane in registers, then over the wave), the result written back
// to LDS and stored row by row (coalesced).  With e_out also the marked
// ancestry of Code 10's Prepermute (run starts keep i, the others -1 - i).
__device__ __forceinline__ void expand_wave(const uint32_t (&O)[kWPer], const uint32_t (&Op)[kWPer],
                                            uint32_t O_lo, uint32_t O_hi, int64_t P0, int64_t n,
                                            int32_t* __restrict__ a_out, int32_t* M,
                                            int32_t* __restrict__ e_out) {
  const int lane = (int)lane_id();
  O_hi = min(O_hi, (uint32_t)n);  // (never binds: every O is at most n)
  int32_t carry = -1;  // particle covering the first output of the chunk
  int4* M4 = reinterpret_cast<int4*>(M) + lane * (kWPer / 4);
  const int32_t P0_32 = (int32_t)P0;
  for (uint32_t cs = O_lo; cs < O_hi; cs += kBlock) {
    const uint32_t len = min((uint32_t)kBlock, O_hi - cs);
#pragma unroll
    for (int k = 0; k < kWPer / 4; ++k) M4[k] = make_int4(-1, -1, -1, -1);
    wave_lds_sync();
    // (a particle that starts no run in this chunk writes the spare slot)
#pragma unroll
    for (int v = 0; v < kWPer; ++v) {
      const uint32_t pos = Op[v] - cs;
      M[(O[v] > Op[v] && pos < len) ? pos : (uint32_t)kBlock] = lane * kWPer + v;
    }
    wave_lds_sync();
    int32_t m[kWPer];
    uint32_t marked = 0;  // bit k: position 16 lane + k starts a run
#pragma unroll
    for (int k = 0; k < kWPer / 4; ++k) {
      const int4 t = M4[k];
      m[4 * k] = t.x; m[4 * k + 1] = t.y; m[4 * k + 2] = t.z; m[4 * k + 3] = t.w;
    }
#pragma unroll
    for (int k = 0; k < kWPer; ++k) {
      marked |= (m[k] >= 0 ? 1u : 0u) << k;
      if (k > 0) m[k] = max(m[k], m[k - 1]);
    }
    const int32_t incl = wave_incl_max_i32(m[kWPer - 1]);
    const int32_t before = max(carry, (int32_t)wave_shift_up_u32((uint32_t)incl, 0xFFFFFFFFu));
#pragma unroll
    for (int k = 0; k < kWPer; ++k) m[k] = max(m[k], before);
    carry = (int32_t)__builtin_amdgcn_readlane(m[kWPer - 1], kWave - 1);
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < kWPer / 4; ++k) {
      int4 t;
      if (e_out) {
        t = make_int4(2 * m[4 * k] + (int)((marked >> (4 * k)) & 1u),
                      2 * m[4 * k + 1] + (int)((marked >> (4 * k + 1)) & 1u),
                      2 * m[4 * k + 2] + (int)((marked >> (4 * k + 2)) & 1u),
                      2 * m[4 * k + 3] + (int)((marked >> (4 * k + 3)) & 1u));
      } else {
        t = make_int4(m[4 * k], m[4 * k + 1], m[4 * k + 2], m[4 * k + 3]);
      }
      M4[k] = t;
    }
    wave_lds_sync();
    int32_t* __restrict__ a_chunk = a_out + cs;  // the same on every lane
#pragma unroll
    for (int j = 0; j < kWPer; ++j) {
      const uint32_t p = (uint32_t)lane + (uint32_t)j * kWave;
      if (p < len) {
        const int32_t v = M[p];
        if (e_out) {
          const int32_t i = P0_32 + (v >> 1);
          a_chunk[p] = i;
          e_out[cs + p] = (v & 1) ? i : -1 - i;
        } else {
          a_chunk[p] = P0_32 + v;
        }
      }
    }
    wave_lds_sync();
  }
}

template <bool SYSTEMATIC>
struct StrataWaveLds {
  alignas(16) int32_t M[kBlock + 4];                   // expansion markers, then the expanded chunk; M[kBlock] spare
  uint32_t u[SYSTEMATIC ? 1 : kUTabW];     // raw offset words of strata [m_lo, m_lo + kUTabW)
};

// Stratified / systematic emission of one block by one wave: the block's
// particles are P0 .. P0 + cnt - 1 of a vector of n, with exclusive exact
// carry Cb and inclusive Cb1 at global scale gscale, total Q.  Writes a_out[s]
// = P0 + i for every s in [O_{i-1}, O_i); with d_out and e_out also the claim
// vector and the marked ancestry of Code 10's Prepermute (as emit_strata).
template <typename T, bool SYSTEMATIC>
__device__ __forceinline__ void emit_block_wave(const T* __restrict__ w, int64_t n, int64_t P0,
                                                const BlockRec rec, u128 Cb, u128 Cb1,
                                                int32_t gscale, u128 Q, Key key, uint32_t filter,
                                                uint32_t offset, int32_t* __restrict__ a_out,
                                                StrataWaveLds<SYSTEMATIC>* L,
                                                int32_t* __restrict__ d_out,
                                                int32_t* __restrict__ e_out) {
  const int lane = (int)lane_id();
  const int cnt = (int)min((int64_t)kBlock, n - P0);
  BlockR R;
  block_r_wave(w, n, P0, rec, Cb, Cb1, gscale, Q, R, L->M);
  if (!(R.hi > R.lo) && !d_out) return;  // an empty range has no outputs

  // stratum offsets of the strata the block's range touches
  const int64_t m_lo = (int64_t)floor(R.lo);
  const int64_t m_hi = min(n - 1, (int64_t)floor(R.hi));
  const bool table = !SYSTEMATIC && (m_hi - m_lo + 1 <= kUTabW);
  const double t_sys =
      SYSTEMATIC ? 1.0 - u_offset(draw_uniform(key, 0, DOM_STRATA, 0, filter, offset).x) : 0.0;
  if (table && m_hi >= m_lo) {
    for (int64_t cc = (m_lo >> 2) + lane; cc <= (m_hi >> 2); cc += kWave) {
      const uint4 xw = draw(key, (uint32_t)cc, DOM_STRATA, 0, filter, offset);
      const uint32_t xs[4] = {xw.x, xw.y, xw.z, xw.w};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = cc * 4 + v;
        if (m >= m_lo && m <= m_hi) L->u[m - m_lo] = xs[v];
      }
    }
    wave_lds_sync();
  }
  // O(r) = #{s : s + 1 - u_s <= r}, exactly: m = floor(r), frac(r) >= 1 - u_m
  // (0 <= r <= n < 2^31, so m converts exactly to 32 bits)
  const int32_t n32 = (int32_t)n, mlo32 = (int32_t)m_lo;
  auto cum_sys = [&](double rv) -> uint32_t {
    const double mf = floor(rv);
    const int32_t m = (int32_t)mf;
    return m >= n32 ? (uint32_t)n32 : (uint32_t)m + ((rv - mf) >= t_sys ? 1u : 0u);
  };
  auto cum_tab = [&](double rv) -> uint32_t {
    const double mf = floor(rv);
    const int32_t m = (int32_t)mf;
    const double t = 1.0 - u_offset(L->u[m >= n32 ? 0 : m - mlo32]);
    return m >= n32 ? (uint32_t)n32 : (uint32_t)m + ((rv - mf) >= t ? 1u : 0u);
  };
  auto cum_draw = [&](double rv) -> uint32_t {
    const double mf = floor(rv);
    const int32_t m = (int32_t)mf;
    if (m >= n32) return (uint32_t)n32;
    const double t = 1.0 - u_offset(stratum_word(key, filter, offset, m));
    return (uint32_t)m + ((rv - mf) >= t ? 1u : 0u);
  };
  uint32_t O[kWPer];
  uint32_t O_lo, O_hi;
  if (SYSTEMATIC) {
#pragma unroll
    for (int v = 0; v < kWPer; ++v) O[v] = cum_sys(R.r[v]);
    O_lo = cum_sys(R.lo);
    O_hi = cum_sys(R.hi);
  } else if (table) {
#pragma unroll
    for (int v = 0; v < kWPer; ++v) O[v] = cum_tab(R.r[v]);
    O_lo = cum_tab(R.lo);
    O_hi = cum_tab(R.hi);
  } else {
#pragma unroll
    for (int v = 0; v < kWPer; ++v) O[v] = cum_draw(R.r[v]);
    O_lo = cum_draw(R.lo);
    O_hi = cum_draw(R.hi);
  }
  O_lo = (uint32_t)__builtin_amdgcn_readfirstlane(O_lo);
  O_hi = (uint32_t)__builtin_amdgcn_readfirstlane(O_hi);
  uint32_t Op[kWPer];
  Op[0] = wave_shift_up_u32(O[kWPer - 1], O_lo);
#pragma unroll
  for (int v = 1; v < kWPer; ++v) Op[v] = O[v - 1];

  if (d_out) {
#pragma unroll
    for (int v = 0; v < kWPer; ++v) {
      const int i = lane * kWPer + v;
      if (i < cnt) d_out[P0 + i] = O[v] > Op[v] ? (int32_t)Op[v] : (int32_t)n;
    }
  }
  expand_wave(O, Op, O_lo, O_hi, P0, n, a_out, L->M, e_out);
}

// ---------------------------------------------------------------- multinomial, one block per wave
// The points p_k = n S_k / S_n of the exponential spacings are formed per
// exponential block as r is per weight block: the block's exact carry CE[e]
// plus the lane's quantised spacings, by the affine map (p of the block's
// last spacing pinned to r(CE[e+1]), so blocks meet exactly).  A weight
// block's particles need O_i = #{k : p_k < r_i}, the cumulative offspring:
// particle i is then the ancestor of outputs [O_{i-1}, O_i), which is
// a_k = #{i : r_i <= p_k}, the upper-bound search of Code 5 (below n - 1, as
// i < cnt).  O_i comes from a binary search over the 1024 points of the one
// exponential block whose range holds r_i, in LDS; the wave walks the
// exponential blocks from the one holding the first point at or above
// r(C_b) to the one holding the first at or above r(C_{b+1}) (usually one or
// two), and the expansion is the one of the stratified scheme.
struct MultiWaveLds {
  double P[kBlock];                   // the points of one exponential block
  alignas(16) int32_t M[kBlock + 4];  // expansion markers; M[kBlock] spare
};

// The lane's 16 quantised spacings of exponential block e (indices
// 1024 e + 16 lane + v): as the records pass stored them (STORED), or drawn
// again (the one-workgroup batch path, which keeps no spacings).
template <bool STORED>
__device__ __forceinline__ void exp_values_wave(Key key, uint32_t filter, uint32_t offset,
                                                int64_t n, uint32_t e,
                                                const uint64_t* __restrict__ evals,
                                                uint64_t (&q)[kWPer]) {
  const int lane = (int)lane_id();
  if constexpr (STORED) {
    const ulonglong2* p =
        reinterpret_cast<const ulonglong2*>(evals + (size_t)e * kBlock + lane * kWPer);
#pragma unroll
    for (int k = 0; k < kWPer / 2; ++k) {
      const ulonglong2 t = p[k];
      q[2 * k] = t.x;
      q[2 * k + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int c = 0; c < kWPer / 4; ++c) {
      const uint32_t call = e * (uint32_t)(kBlock / 4) + (uint32_t)lane * (kWPer / 4) + c;
      const uint4 x = draw(key, call, DOM_EXP, 0, filter, offset);
      const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t k = (int64_t)call * 4 + v;
        const double ev = neg_log_spacing(xs[v]);
        q[4 * c + v] = (k <= n) ? (uint64_t)(ev * 0x1p48) : 0ull;
      }
    }
  }
}

// Exponential block holding the first point at or above x: the number of
// blocks whose last point P(b + 1) = em(CE[b + 1]) lies below x.  The last
// points sit within a few blocks of (b + 1) 1024 n / (n + 1), so one probe of
// 256 consecutive boundaries (four per lane) around the guess settles it; a
// bisection is the fallback.
template <typename CEPtr>
__device__ __forceinline__ uint32_t exp_block_of(double x, int64_t n, CEPtr CE, uint32_t nbe,
                                                 const RMap& em) {
  const double per_block = (double)kBlock * (double)n / (double)(n + 1);
  int64_t w0 = (int64_t)(x / per_block) - 128;  // first probed boundary index b + 1
  if (w0 < 1) w0 = 1;
  const int64_t last = (int64_t)nbe - 1;  // boundaries 1 .. nbe - 1
  const int lane = (int)lane_id();
  uint32_t below = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t b = w0 + lane * 4 + k;
    below += (b <= last && em(CE[b]) < x) ? 1u : 0u;
  }
  below = wave_reduce(below, OpAdd());
  const int64_t w1 = min(w0 + 255, last);
  const int64_t span = w1 - w0 + 1;
  const bool ok = w0 > last || ((w0 == 1 || below > 0) && (w1 == last || (int64_t)below < span));
  if (ok) return (uint32_t)(w0 > last ? last : w0 - 1 + below);
  uint32_t lo = 1, hi = nbe;  // #{b in [1, nbe - 1] : P(b) < x}
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (em(CE[mid]) < x) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

template <typename T, bool STORED, typename CEPtr>
__device__ __forceinline__ void emit_multi_wave(const T* __restrict__ w, int64_t n, int64_t P0,
                                                const BlockRec rec, u128 Cb, u128 Cb1,
                                                int32_t gscale, u128 Q, Key key, uint32_t filter,
                                                uint32_t offset, CEPtr CE, uint32_t nbe,
                                                const uint64_t* __restrict__ evals,
                                                int32_t* __restrict__ a_out, MultiWaveLds* L,
                                                int32_t* __restrict__ d_out = nullptr,
                                                int32_t* __restrict__ e_out = nullptr) {
  const int lane = (int)lane_id();
  const int cnt = (int)min((int64_t)kBlock, n - P0);
  BlockR R;
  block_r_wave(w, n, P0, rec, Cb, Cb1, gscale, Q, R, L->M);
  if (!(R.hi > R.lo) && !d_out) return;  // an empty range has no outputs
  const RMap em = make_rmap(CE[nbe], n);
  const double ce = em.Nd * em.invQ;
  const uint32_t e_first = (uint32_t)__builtin_amdgcn_readfirstlane(exp_block_of(R.lo, n, CE, nbe, em));
  const uint32_t e_last = (uint32_t)__builtin_amdgcn_readfirstlane(exp_block_of(R.hi, n, CE, nbe, em));
  uint32_t O[kWPer];
#pragma unroll
  for (int v = 0; v < kWPer; ++v) O[v] = 0;
  uint32_t det = 0;  // bit v: O[v] is known
  uint32_t O_lo = 0, O_hi = 0;
  bool lo_det = false, hi_det = false;
  double2* P2 = reinterpret_cast<double2*>(L->P) + lane * (kWPer / 2);
  // lower bound in the block's points (x at most its last point)
  auto lb = [&](double x) -> uint32_t {
    uint32_t pos = (L->P[kBlock / 2 - 1] < x) ? (uint32_t)(kBlock / 2) : 0u;
#pragma unroll
    for (uint32_t st = kBlock / 4; st > 0; st >>= 1) pos += (L->P[pos + st - 1] < x) ? st : 0u;
    return pos;
  };
  for (uint32_t e = e_first; e <= e_last; ++e) {
    uint64_t q[kWPer];
    exp_values_wave<STORED>(key, filter, offset, n, e, evals, q);
    uint64_t acc = 0;
#pragma unroll
    for (int v = 0; v < kWPer; ++v) {
      acc += q[v];
      q[v] = acc;
    }
    const uint64_t incl = wave_incl_add_u64(acc);
    const uint64_t off = incl - acc;
    const uint64_t total = readlane(incl, kWave - 1);
    const double p_base = em(CE[e]), p_top = em(CE[e + 1]);
#pragma unroll
    for (int k = 0; k < kWPer / 2; ++k) {
      double pv[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint64_t Lv = off + q[2 * k + h];
        const double v = __fma_rn(u64_to_f64(Lv), ce, p_base);
        pv[h] = (Lv == total || v > p_top) ? p_top : v;
      }
      P2[k] = make_double2(pv[0], pv[1]);
    }
    wave_lds_sync();
    const uint32_t base = e * (uint32_t)kBlock;
    // the particles this block settles: not settled yet and r <= its last
    // point; eight of the lane's searches run step by step together, so that
    // their LDS reads are in flight at the same time (eight, not sixteen,
    // bounds the registers the reads hold: three waves per SIMD instead of one)
    uint32_t need = 0;
#pragma unroll
    for (int v = 0; v < kWPer; ++v)
      need |= (!((det >> v) & 1u) && R.r[v] <= p_top) ? (1u << v) : 0u;
#pragma unroll
    for (int h = 0; h < kWPer; h += kWPer / 2) {
      const uint32_t need_h = need & (((1u << (kWPer / 2)) - 1u) << h);
      if (ballot(need_h != 0)) {
        uint32_t pos[kWPer / 2];
#pragma unroll
        for (int v = 0; v < kWPer / 2; ++v)
          pos[v] = (L->P[kBlock / 2 - 1] < R.r[h + v]) ? (uint32_t)(kBlock / 2) : 0u;
#pragma unroll
        for (uint32_t st = kBlock / 4; st > 0; st >>= 1) {
#pragma unroll
          for (int v = 0; v < kWPer / 2; ++v)
            pos[v] += (L->P[pos[v] + st - 1] < R.r[h + v]) ? st : 0u;
        }
#pragma unroll
        for (int v = 0; v < kWPer / 2; ++v)
          if ((need_h >> (h + v)) & 1u) O[h + v] = base + pos[v];
      }
    }
    det |= need;
    if (!lo_det && R.lo <= p_top) {
      O_lo = base + lb(R.lo);
      lo_det = true;
    }
    if (!hi_det && R.hi <= p_top) {
      O_hi = base + lb(R.hi);
      hi_det = true;
    }
    wave_lds_sync();
  }
  O_lo = (uint32_t)__builtin_amdgcn_readfirstlane(O_lo);
  O_hi = (uint32_t)__builtin_amdgcn_readfirstlane(O_hi);
  uint32_t Op[kWPer];
  Op[0] = wave_shift_up_u32(O[kWPer - 1], O_lo);
#pragma unroll
  for (int v = 1; v < kWPer; ++v) Op[v] = O[v - 1];
  if (d_out) {  // the ancestry is sorted: the sorted claim, as the strata schemes form it
#pragma unroll
    for (int v = 0; v < kWPer; ++v) {
      const int i = lane * kWPer + v;
      if (i < cnt) d_out[P0 + i] = O[v] > Op[v] ? (int32_t)Op[v] : (int32_t)n;
    }
  }
  expand_wave(O, Op, O_lo, O_hi, P0, n, a_out, L->M, e_out);
}

// Weight records, one block per wave (blockIdx.x < wgs_b), and for the
// multinomial scheme the exponential blocks (one per workgroup beyond them).
template <typename T, bool MULTI>
__global__ __launch_bounds__(kT) void k_scan_records_w(const T* __restrict__ w, int64_t n,
                                                       uint32_t nb, uint32_t wgs_b, Key key,
                                                       uint32_t offset, uint32_t filter,
                                                       BlockRec* __restrict__ recs,
                                                       uint64_t* __restrict__ esums,
                                                       uint64_t* __restrict__ evals,
                                                       ScanHeader* __restrict__ hdr) {
  offset = counter_offset(key, offset);
  if (blockIdx.x == 0 && threadIdx.x == 0) hdr->groups_done = 0;  // for the carries pass
  if (blockIdx.x < wgs_b) {
    const uint32_t b = blockIdx.x * kWavesPerWG +
                       (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (b >= nb) return;
    const BlockRec r = wave_block_record(w, n, (int64_t)b * kBlock);
    if (lane_id() == 0) recs[b] = r;
  } else if (MULTI) {
    __shared__ WgScratch s;
    const uint32_t b = blockIdx.x - wgs_b;
    uint64_t q[kPer];
    exp_values(key, filter, offset, n, b, q);
    store_exp_values(evals, b, q);
    const uint64_t sum = wg_reduce(q[0] + q[1] + q[2] + q[3], OpAdd(), s.u);
    if (threadIdx.x == 0) esums[b] = sum;
  }
}

// Direct carries of block b by its own wave: the global scale, the block's
// exact carry and the total from all nb records, read by the wave in two
// lane-strided passes and summed by DPP scans, with no workgroup barrier and
// no LDS.  Every record is converted straight to the global scale (the
// carries pass converts a group's sums to the group's scale first, which
// gives the same values when there is one group of 1024 blocks).
struct DirectW {
  u128 Cb, Cb1, Q;
  int32_t gscale;
  uint32_t status;
};

__device__ DirectW wave_direct_carries(uint32_t nb, uint32_t b,
                                       const BlockRec* __restrict__ recs) {
  const uint32_t lane = lane_id();
  uint32_t bad = 0, key = 0xFFFFFFFFu;
  for (uint32_t j = lane; j < nb; j += kWave) {
    const BlockRec r = recs[j];
    bad |= r.bad;
    if (r.sum) key = min(key, (uint32_t)r.scale ^ 0x80000000u);
  }
  bad = wave_reduce(bad, OpOr());
  key = wave_reduce(key, OpMin());
  DirectW d;
  d.gscale = key == 0xFFFFFFFFu
                 ? 0
                 : (int32_t)(key ^ 0x80000000u) + (kCarryBits - 63) - ceil_log2(nb);
  u128 before = 0, all = 0, own = 0;
  for (uint32_t j = lane; j < nb; j += kWave) {
    const u128 v = conv_rec(recs[j], d.gscale);
    all += v;
    before += j < b ? v : (u128)0;
    own += j == b ? v : (u128)0;
  }
  d.Q = readlane(wave_incl_add_u128(all), kWave - 1);
  d.Cb = readlane(wave_incl_add_u128(before), kWave - 1);
  d.Cb1 = d.Cb + readlane(wave_incl_add_u128(own), kWave - 1);
  d.status = bad;
  if (!bad && d.Q == 0) d.status |= FLAG_ZERO_TOTAL;
  return d;
}

template <typename T, int SCHEME, bool DIRECT>
__global__ __launch_bounds__(kT) void k_scan_emit_w(const T* __restrict__ w, int64_t n,
                                                    uint32_t nb, Key key, uint32_t offset,
                                                    uint32_t filter,
                                                    const ScanHeader* __restrict__ hdr,
                                                    const BlockRec* __restrict__ recs,
                                                    Carries C, int32_t* __restrict__ a,
                                                    uint32_t* __restrict__ flags,
                                                    int32_t* __restrict__ d_out,
                                                    int32_t* __restrict__ e_out) {
  static_assert(SCHEME != SCHEME_MULTINOMIAL, "strata schemes only");
  offset = counter_offset(key, offset);
  __shared__ StrataWaveLds<SCHEME == SCHEME_SYSTEMATIC> L[kWavesPerWG];
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t b = blockIdx.x * kWavesPerWG + wave;
  uint32_t status;
  u128 Cb, Cb1, Q;
  int32_t gscale;
  if (DIRECT) {
    if (b >= nb) return;
    const DirectW d = wave_direct_carries(nb, b, recs);
    status = d.status;
    Cb = d.Cb;
    Cb1 = d.Cb1;
    Q = d.Q;
    gscale = d.gscale;
  } else {
    if (b >= nb) return;
    status = hdr->status;
    gscale = hdr->gscale;
    C.gscale = gscale;
    Cb = C[b];
    Cb1 = C[b + 1];
    Q = hdr->Q;
  }
  if (b >= nb) return;
  if (flags && b == 0 && threadIdx.x == 0 && status) atomicOr(flags, status);
  const int64_t P0 = (int64_t)b * kBlock;
  if (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    // identity: every position claims its own slot
    for (int64_t i = P0 + lane_id(); i < min(P0 + kBlock, n); i += kWave) {
      a[i] = (int32_t)i;
      if (d_out) {
        d_out[i] = (int32_t)i;
        e_out[i] = (int32_t)i;
      }
    }
    return;
  }
  emit_block_wave<T, SCHEME == SCHEME_SYSTEMATIC>(w, n, P0, recs[b], Cb, Cb1, gscale, Q, key,
                                                   filter, offset, a, &L[wave], d_out, e_out);
}

// Multinomial emission, one weight block per wave (after the carries); with
// d_out and e_out also the claim vector and the marked ancestry of Code 10's
// Prepermute (the multinomial ancestry is sorted, as the strata schemes' is).
template <typename T>
__global__ __launch_bounds__(kT) void k_scan_emit_mw(const T* __restrict__ w, int64_t n,
                                                     uint32_t nb, uint32_t nbe, Key key,
                                                     uint32_t offset, uint32_t filter,
                                                     const ScanHeader* __restrict__ hdr,
                                                     const BlockRec* __restrict__ recs,
                                                     Carries C, ECarries CE,
                                                     const uint64_t* __restrict__ evals,
                                                     int32_t* __restrict__ a,
                                                     uint32_t* __restrict__ flags,
                                                     int32_t* __restrict__ d_out,
                                                     int32_t* __restrict__ e_out) {
  offset = counter_offset(key, offset);
  __shared__ MultiWaveLds L[kWavesPerWG];
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t b = blockIdx.x * kWavesPerWG + wave;
  if (b >= nb) return;
  const uint32_t status = hdr->status;
  if (flags && b == 0 && threadIdx.x == 0 && status) atomicOr(flags, status);
  const int64_t P0 = (int64_t)b * kBlock;
  if (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    for (int64_t i = P0 + lane_id(); i < min(P0 + kBlock, n); i += kWave) {
      a[i] = (int32_t)i;
      if (d_out) {
        d_out[i] = (int32_t)i;
        e_out[i] = (int32_t)i;
      }
    }
    return;
  }
  C.gscale = hdr->gscale;
  emit_multi_wave<T, true>(w, n, P0, recs[b], C[b], C[b + 1], C.gscale, hdr->Q, key, filter,
                           offset, CE, nbe, evals, a, &L[wave], d_out, e_out);
}

// ---------------------------------------------------------------- Code 5
// Multinomial resampling with one independent uniform per particle, as Code 5
// prints it: the scaled prefix r_k = n W_k / W_n of the exact sums is written
// out (binary64, the same values the other schemes compare against), then
// particle i draws u_i = m 2^-53 (m: 21 bits of word 0 and 32 of word 1 of its
// uniform-domain Philox call), p_i = n u_i, and takes #{k < n-1 : r_k <= p_i}.
// The search is two-level: every workgroup holds up to kSplit splitters
// r_{(j+1) S - 1} (S a power of two) in LDS, which narrow each point to S
// candidates, and a bisection over those in global memory finishes it.
template <typename T>
__global__ __launch_bounds__(kT) void k_scan_r(const T* __restrict__ w, int64_t n, uint32_t nb,
                                               const ScanHeader* __restrict__ hdr,
                                               const BlockRec* __restrict__ recs, Carries C,
                                               double* __restrict__ r_out) {
  if (hdr->status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) return;
  const uint32_t b = blockIdx.x * kWavesPerWG +
                     (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (b >= nb) return;
  const int64_t P0 = (int64_t)b * kBlock;
  BlockR R;
  C.gscale = hdr->gscale;
  block_r_wave(w, n, P0, recs[b], C[b], C[b + 1], C.gscale, hdr->Q, R);
  const int64_t i0 = P0 + (int64_t)lane_id() * kWPer;
#pragma unroll
  for (int v = 0; v < kWPer; ++v)
    if (i0 + v < n) r_out[i0 + v] = R.r[v];
}

__global__ void k_scan_status(const ScanHeader* __restrict__ hdr, uint32_t* __restrict__ flags) {
  if (hdr->status) atomicOr(flags, hdr->status);
}

constexpr int kSplit = 4096;

__global__ __launch_bounds__(kT) void k_multinomial_iid(int64_t n,
                                                        const ScanHeader* __restrict__ hdr,
                                                        const double* __restrict__ r,
                                                        int stride_log2, Key key,
                                                        uint32_t offset, uint32_t filter,
                                                        int32_t* __restrict__ a,
                                                        uint32_t* __restrict__ flags) {
  __shared__ double sp[kSplit];
  offset = counter_offset(key, offset);
  const uint32_t status = hdr->status;
  if (flags && blockIdx.x == 0 && threadIdx.x == 0 && status) atomicOr(flags, status);
  const bool identity = (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) != 0;
  const int64_t m = n - 1;                  // candidates r_0 .. r_{m-1}
  const int64_t S = (int64_t)1 << stride_log2;
  const int J = (int)(m >> stride_log2);  // splitters inside [0, m), J <= kSplit
  if (!identity)
    for (int j = (int)threadIdx.x; j < J; j += kT) sp[j] = r[((int64_t)(j + 1) << stride_log2) - 1];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kT;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += stride) {
    if (identity) {
      a[i] = (int32_t)i;
      continue;
    }
    const uint4 x = draw(key, (uint32_t)i, DOM_UNIFORM, 0, filter, offset);
    const uint64_t mb = ((uint64_t)(x.x >> 11) << 32) | (uint64_t)x.y;
    const double p = (double)n * ((double)mb * 0x1p-53);
    // splitters: every r_k with k < lo S is <= p; r_{(lo+1) S - 1} > p if lo < J
    int lo = 0, hi = J;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sp[mid] <= p) lo = mid + 1;
      else hi = mid;
    }
    int64_t L = (int64_t)lo << stride_log2;
    int64_t H = lo < J ? L + S - 1 : m;  // the answer lies in [L, H]
    while (L < H) {
      const int64_t mid = (L + H) >> 1;
      if (r[mid] <= p) L = mid + 1;
      else H = mid;
    }
    a[i] = (int32_t)L;
  }
}

// Ragged batch: one workgroup per filter runs the reduce, the carries and the
// emission of its own segment, with the records and carries in LDS.
constexpr int kBatchMaxBlocks = 256;  // segments up to 2^18 particles

struct BatchLds {
  BlockRec recs[kBatchMaxBlocks];
  u128 C[kBatchMaxBlocks + 1];
  uint64_t esums[kBatchMaxBlocks];
  u128 CE[kBatchMaxBlocks + 1];
};

template <typename T, int SCHEME>
__global__ __launch_bounds__(kT) void k_scan_batched(const T* __restrict__ w, int64_t n_total,
                                                     const int64_t* __restrict__ offsets,
                                                     uint32_t n_filters, Key key, uint32_t offset,
                                                     uint32_t filter_base, int32_t* __restrict__ a,
                                                     uint32_t* __restrict__ flags) {
  offset = counter_offset(key, offset);
  __shared__ BatchLds B;
  __shared__ WgScratch s;
  const uint32_t f = blockIdx.x;
  if (f >= n_filters) return;
  const int tid = (int)threadIdx.x;
  const int64_t base = offsets ? offsets[f] : 0;
  const int64_t n = offsets ? offsets[f + 1] - base : n_total;
  if (n <= 0) return;
  const T* __restrict__ ws = w + base;
  int32_t* __restrict__ as = a + base;
  const uint32_t filt = filter_base + f;
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  const uint32_t nbe = (uint32_t)((n + 1 + kBlock - 1) / kBlock);
  if (nbe > kBatchMaxBlocks) {  // segment too long for this path: identity + flag
    for (int64_t i = tid; i < n; i += kT) as[i] = (int32_t)i;
    if (tid == 0 && flags) atomicOr(flags, FLAG_BAD_COUNTS);
    return;
  }
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (uint32_t b = wave; b < nb; b += kWavesPerWG) {
    const BlockRec r = wave_block_record(ws, n, (int64_t)b * kBlock);
    if (lane_id() == 0) B.recs[b] = r;
  }
  if (SCHEME == SCHEME_MULTINOMIAL) {
    for (uint32_t b = 0; b < nbe; ++b) {
      uint64_t q[kPer];
      exp_values(key, filt, offset, n, b, q);
      const uint64_t sum = wg_reduce(q[0] + q[1] + q[2] + q[3], OpAdd(), s.u);
      if (tid == 0) B.esums[b] = sum;
    }
  }
  __syncthreads();
  const Totals t = carries_from_records(nb, (const BlockRec*)B.recs, (u128*)B.C, &s);
  if (SCHEME == SCHEME_MULTINOMIAL) exp_carries(nbe, (const uint64_t*)B.esums, (u128*)B.CE, &s);
  if (flags && tid == 0 && t.status) atomicOr(flags, t.status);
  if (t.status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    for (int64_t i = tid; i < n; i += kT) as[i] = (int32_t)i;
    return;
  }
  if constexpr (SCHEME == SCHEME_MULTINOMIAL) {
    __shared__ MultiWaveLds L[kWavesPerWG];
    for (uint32_t b = wave; b < nb; b += kWavesPerWG)
      emit_multi_wave<T, false>(ws, n, (int64_t)b * kBlock, B.recs[b], B.C[b], B.C[b + 1],
                                t.gscale, t.Q, key, filt, offset, (const u128*)B.CE, nbe,
                                (const uint64_t*)nullptr, as, &L[wave]);
  } else {
    __shared__ StrataWaveLds<SCHEME == SCHEME_SYSTEMATIC> L[kWavesPerWG];
    for (uint32_t b = wave; b < nb; b += kWavesPerWG)
      emit_block_wave<T, SCHEME == SCHEME_SYSTEMATIC>(ws, n, (int64_t)b * kBlock, B.recs[b],
                                                       B.C[b], B.C[b + 1], t.gscale, t.Q, key,
                                                       filt, offset, as, &L[wave], nullptr,
                                                       nullptr);
  }
}

// ---------------------------------------------------------------- segmented batches
// A batch with a workspace runs block-parallel: every 1024-weight block of
// every segment is one workgroup of the records and of the emit kernel, so a
// long segment no longer runs through one workgroup.  Blocks start at each
// segment's first weight (the same blocks as a single call on the segment),
// and one workgroup per segment forms the segment's exact carries, so the
// result is that of one call per segment.

// Exclusive block prefixes over the segments: bstart[f] (weight blocks) and,
// for the multinomial scheme, estart[f] (exponential blocks).  One workgroup.
__global__ __launch_bounds__(kT) void k_seg_prefix(const int64_t* __restrict__ offsets,
                                                   uint32_t n_filters,
                                                   uint32_t* __restrict__ bstart,
                                                   uint32_t* __restrict__ estart) {
  __shared__ WgScratch s;
  uint64_t carry_b = 0, carry_e = 0;
  for (uint32_t base = 0; base < n_filters; base += kT) {
    const uint32_t f = base + threadIdx.x;
    uint64_t nb = 0, ne = 0;
    if (f < n_filters) {
      const int64_t n = offsets[f + 1] - offsets[f];
      nb = n > 0 ? (uint64_t)((n + kBlock - 1) / kBlock) : 0;
      ne = n > 0 ? (uint64_t)((n + 1 + kBlock - 1) / kBlock) : 0;
    }
    uint64_t tb, te;
    const uint64_t xb = wg_exclusive(nb, s.u, &tb);
    const uint64_t xe = wg_exclusive(ne, s.u, &te);
    if (f < n_filters) {
      bstart[f] = (uint32_t)(carry_b + xb);
      if (estart) estart[f] = (uint32_t)(carry_e + xe);
    }
    carry_b += tb;
    carry_e += te;
  }
  if (threadIdx.x == 0) {
    bstart[n_filters] = (uint32_t)carry_b;
    if (estart) estart[n_filters] = (uint32_t)carry_e;
  }
}

// segment f of global block g: the last f with start[f] <= g (start non-decreasing)
__device__ __forceinline__ uint32_t seg_of_block(const uint32_t* __restrict__ start,
                                                 uint32_t n_filters, uint32_t g) {
  uint32_t lo = 0, hi = n_filters;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (start[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename T, bool MULTI>
__global__ __launch_bounds__(kT) void k_seg_records(
    const T* __restrict__ w, const int64_t* __restrict__ offsets, uint32_t n_filters,
    uint32_t grid_b, Key key, uint32_t offset, uint32_t filter_base,
    const uint32_t* __restrict__ bstart, const uint32_t* __restrict__ estart,
    BlockRec* __restrict__ recs, uint64_t* __restrict__ esums, uint64_t* __restrict__ evals) {
  __shared__ WgScratch s;
  offset = counter_offset(key, offset);
  if (blockIdx.x < grid_b) {
    const uint32_t g = blockIdx.x;
    if (g >= bstart[n_filters]) return;
    const uint32_t f = seg_of_block(bstart, n_filters, g);
    const int64_t base = offsets[f];
    const int64_t n = offsets[f + 1] - base;
    const BlockRec r = block_record(w + base, n, (int64_t)(g - bstart[f]) * kBlock, &s);
    if (threadIdx.x == 0) recs[g] = r;
  } else if (MULTI) {
    const uint32_t g = blockIdx.x - grid_b;
    if (g >= estart[n_filters]) return;
    const uint32_t f = seg_of_block(estart, n_filters, g);
    const int64_t n = offsets[f + 1] - offsets[f];
    uint64_t q[kPer];
    exp_values(key, filter_base + f, offset, n, g - estart[f], q);
    store_exp_values(evals, g, q);  // global block g = segment block g - estart[f]
    const uint64_t sum = wg_reduce(q[0] + q[1] + q[2] + q[3], OpAdd(), s.u);
    if (threadIdx.x == 0) esums[g] = sum;
  }
}

// Weight records of the segmented batch, one block per wave (strata schemes;
// the multinomial scheme keeps k_seg_records for its exponential blocks).
template <typename T>
__global__ __launch_bounds__(kT) void k_seg_records_w(const T* __restrict__ w,
                                                      const int64_t* __restrict__ offsets,
                                                      uint32_t n_filters,
                                                      const uint32_t* __restrict__ bstart,
                                                      BlockRec* __restrict__ recs) {
  const uint32_t g = blockIdx.x * kWavesPerWG +
                     (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (g >= bstart[n_filters]) return;
  const uint32_t f = seg_of_block(bstart, n_filters, g);
  const int64_t base = offsets[f];
  const int64_t n = offsets[f + 1] - base;
  const BlockRec r = wave_block_record(w + base, n, (int64_t)(g - bstart[f]) * kBlock);
  if (lane_id() == 0) recs[g] = r;
}

// Per segment (one workgroup each): global scale, exact carries C (nb + 1 per
// segment, at cstart = bstart[f] + f), total and status, and the
// exponential-block carries of the multinomial scheme (at estart[f] + f).
struct SegHdr {
  u128 Q;
  int32_t gscale;
  uint32_t status;
  uint64_t pad;
};

template <bool MULTI>
__global__ __launch_bounds__(kT) void k_seg_carries(uint32_t n_filters,
                                                    const uint32_t* __restrict__ bstart,
                                                    const uint32_t* __restrict__ estart,
                                                    const BlockRec* __restrict__ recs,
                                                    const uint64_t* __restrict__ esums,
                                                    u128* __restrict__ C, u128* __restrict__ CE,
                                                    SegHdr* __restrict__ hdr) {
  __shared__ WgScratch s;
  const uint32_t f = blockIdx.x;
  if (f >= n_filters) return;
  const uint32_t b0 = bstart[f], nb = bstart[f + 1] - b0;
  if (nb == 0) return;
  const Totals t = carries_from_records(nb, recs + b0, C + b0 + f, &s);
  if (MULTI) {
    const uint32_t e0 = estart[f];
    exp_carries(estart[f + 1] - e0, esums + e0, CE + e0 + f, &s);
  }
  if (threadIdx.x == 0) {
    hdr[f].Q = t.Q;
    hdr[f].gscale = t.gscale;
    hdr[f].status = t.status;
  }
}

// Emission of the segmented batch, one block per wave (strata schemes).
template <typename T, int SCHEME>
__global__ __launch_bounds__(kT) void k_seg_emit_w(
    const T* __restrict__ w, const int64_t* __restrict__ offsets, uint32_t n_filters, Key key,
    uint32_t offset, uint32_t filter_base, const uint32_t* __restrict__ bstart,
    const BlockRec* __restrict__ recs, const u128* __restrict__ C,
    const SegHdr* __restrict__ hdr, int32_t* __restrict__ a, uint32_t* __restrict__ flags) {
  static_assert(SCHEME != SCHEME_MULTINOMIAL, "strata schemes only");
  __shared__ StrataWaveLds<SCHEME == SCHEME_SYSTEMATIC> L[kWavesPerWG];
  offset = counter_offset(key, offset);
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t g = blockIdx.x * kWavesPerWG + wave;
  if (g >= bstart[n_filters]) return;
  const uint32_t f = seg_of_block(bstart, n_filters, g);
  const int64_t base = offsets[f];
  const int64_t n = offsets[f + 1] - base;
  const uint32_t b = g - bstart[f];
  int32_t* __restrict__ as = a + base;
  const uint32_t status = hdr[f].status;
  if (flags && b == 0 && lane_id() == 0 && status) atomicOr(flags, status);
  const int64_t P0 = (int64_t)b * kBlock;
  if (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    for (int64_t i = P0 + lane_id(); i < min(P0 + kBlock, n); i += kWave) as[i] = (int32_t)i;
    return;
  }
  const u128* Cs = C + bstart[f] + f;
  emit_block_wave<T, SCHEME == SCHEME_SYSTEMATIC>(w + base, n, P0, recs[g], Cs[b], Cs[b + 1],
                                                   hdr[f].gscale, hdr[f].Q, key, filter_base + f,
                                                   offset, as, &L[wave], nullptr, nullptr);
}

// Multinomial emission of the segmented batch, one block per wave.
template <typename T>
__global__ __launch_bounds__(kT) void k_seg_emit_mw(
    const T* __restrict__ w, const int64_t* __restrict__ offsets, uint32_t n_filters, Key key,
    uint32_t offset, uint32_t filter_base, const uint32_t* __restrict__ bstart,
    const uint32_t* __restrict__ estart, const BlockRec* __restrict__ recs,
    const u128* __restrict__ C, const u128* __restrict__ CE, const SegHdr* __restrict__ hdr,
    int32_t* __restrict__ a, uint32_t* __restrict__ flags, const uint64_t* __restrict__ evals) {
  __shared__ MultiWaveLds L[kWavesPerWG];
  offset = counter_offset(key, offset);
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t g = blockIdx.x * kWavesPerWG + wave;
  if (g >= bstart[n_filters]) return;
  const uint32_t f = seg_of_block(bstart, n_filters, g);
  const int64_t base = offsets[f];
  const int64_t n = offsets[f + 1] - base;
  const uint32_t b = g - bstart[f];
  int32_t* __restrict__ as = a + base;
  const uint32_t status = hdr[f].status;
  if (flags && b == 0 && lane_id() == 0 && status) atomicOr(flags, status);
  const int64_t P0 = (int64_t)b * kBlock;
  if (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    for (int64_t i = P0 + lane_id(); i < min(P0 + kBlock, n); i += kWave) as[i] = (int32_t)i;
    return;
  }
  const u128* Cs = C + bstart[f] + f;
  const uint32_t nbe = estart[f + 1] - estart[f];
  emit_multi_wave<T, true>(w + base, n, P0, recs[g], Cs[b], Cs[b + 1], hdr[f].gscale, hdr[f].Q,
                           key, filter_base + f, offset, CE + estart[f] + f, nbe,
                           evals + (size_t)estart[f] * kBlock, as, &L[wave]);
}

// The two-level carries of a single vector in its workspace.
struct CarrySet {
  Carries C;
  ECarries CE;
  CarryGroup* groups;
  CarryGroup* egroups;
};

CarrySet carry_set(const ScanLayout& L, char* base, uint32_t nb, uint32_t nbe) {
  CarrySet c;
  const uint32_t G = carry_groups(nb), Ge = carry_groups(nbe);
  c.groups = (CarryGroup*)(base + L.groups);
  c.egroups = (CarryGroup*)(base + L.egroups);
  c.C = Carries{(const u128*)(base + L.carries), (const u128*)(c.groups + G), c.groups, nb, G, 0};
  c.CE = ECarries{(const u128*)(base + L.ecarries), (const u128*)(c.egroups + Ge), nbe, Ge};
  return c;
}

template <bool MULTI>
hipError_t launch_carries(const CarrySet& c, ScanHeader* hdr, const BlockRec* recs,
                          const uint64_t* esums, hipStream_t stream) {
  const uint32_t G = c.C.G, Ge = MULTI ? c.CE.Ge : 0u;
  // one workgroup for all groups when there are few
  const uint32_t grid = G + Ge <= kFewGroups ? 1u : G + Ge;
  hipLaunchKernelGGL((k_carry_groups<MULTI>), dim3(grid), dim3(kT), 0, stream, c.C.nb,
                     c.CE.nbe, G, recs, esums, (u128*)c.C.P, (u128*)c.CE.PE, c.groups,
                     c.egroups, Ge, (u128*)c.C.Tx, (u128*)c.CE.TEx, hdr);
  return hipGetLastError();
}

template <typename T, int SCHEME>
hipError_t launch_scan_t(const void* wv, int64_t n, Key key, uint32_t offset, uint32_t filter,
                         int32_t* a, void* ws, uint32_t* flags, hipStream_t stream,
                         int32_t* d_out = nullptr, int32_t* e_out = nullptr) {
  const T* w = (const T*)wv;
  constexpr bool multi = SCHEME == SCHEME_MULTINOMIAL;
  const ScanLayout L = scan_layout(n, multi);
  char* base = (char*)ws;
  ScanHeader* hdr = (ScanHeader*)base;
  BlockRec* recs = (BlockRec*)(base + L.recs);
  uint64_t* esums = (uint64_t*)(base + L.erecs);
  uint64_t* evals = multi ? (uint64_t*)(base + L.evals) : nullptr;
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  const uint32_t nbe = multi ? (uint32_t)((n + 1 + kBlock - 1) / kBlock) : 0u;
  const uint32_t wgs_b = (nb + kWavesPerWG - 1) / kWavesPerWG;
  const CarrySet cs = carry_set(L, base, nb, nbe);
  hipLaunchKernelGGL((k_scan_records_w<T, multi>), dim3(wgs_b + nbe), dim3(kT), 0, stream, w, n,
                     nb, wgs_b, key, offset, filter, recs, esums, evals, hdr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if constexpr (!multi) {
    if (nb <= (uint32_t)tuning().direct_max_blocks && nb <= kDirectMax) {
      hipLaunchKernelGGL((k_scan_emit_w<T, SCHEME, true>), dim3(wgs_b), dim3(kT), 0, stream, w,
                         n, nb, key, offset, filter, hdr, recs, cs.C, a, flags, d_out, e_out);
      return hipGetLastError();
    }
  }
  e = launch_carries<multi>(cs, hdr, recs, esums, stream);
  if (e != hipSuccess) return e;
  if constexpr (multi) {
    hipLaunchKernelGGL((k_scan_emit_mw<T>), dim3(wgs_b), dim3(kT), 0, stream, w, n, nb, nbe, key,
                       offset, filter, hdr, recs, cs.C, cs.CE, (const uint64_t*)evals, a, flags,
                       d_out, e_out);
  } else {
    hipLaunchKernelGGL((k_scan_emit_w<T, SCHEME, false>), dim3(wgs_b), dim3(kT), 0, stream, w,
                       n, nb, key, offset, filter, hdr, recs, cs.C, a, flags, d_out, e_out);
  }
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
hipError_t launch_batched_scheme(int scheme, const void* w, int64_t n_total,
                                 const int64_t* offsets, uint32_t n_filters, Key key,
                                 uint32_t offset, uint32_t filter_base, int32_t* a,
                                 uint32_t* flags, hipStream_t stream) {
  const T* wt = (const T*)w;
  switch (scheme) {
    case SCHEME_MULTINOMIAL:
      hipLaunchKernelGGL((k_scan_batched<T, SCHEME_MULTINOMIAL>), dim3(n_filters), dim3(kT), 0,
                         stream, wt, n_total, offsets, n_filters, key, offset, filter_base, a,
                         flags);
      break;
    case SCHEME_STRATIFIED:
      hipLaunchKernelGGL((k_scan_batched<T, SCHEME_STRATIFIED>), dim3(n_filters), dim3(kT), 0,
                         stream, wt, n_total, offsets, n_filters, key, offset, filter_base, a,
                         flags);
      break;
    default:
      hipLaunchKernelGGL((k_scan_batched<T, SCHEME_SYSTEMATIC>), dim3(n_filters), dim3(kT), 0,
                         stream, wt, n_total, offsets, n_filters, key, offset, filter_base, a,
                         flags);
      break;
  }
  return hipGetLastError();
}

template <typename T, int SCHEME>
hipError_t launch_segmented_t(const T* w, int64_t n_total, const int64_t* offsets,
                              uint32_t n_filters, Key key, uint32_t offset, uint32_t filter_base,
                              int32_t* a, void* ws, uint32_t* flags, hipStream_t stream) {
  constexpr bool multi = SCHEME == SCHEME_MULTINOMIAL;
  const SegLayout L = seg_layout(n_total, n_filters, multi);
  char* base = (char*)ws;
  uint32_t* bstart = (uint32_t*)(base + L.bstart);
  uint32_t* estart = multi ? (uint32_t*)(base + L.estart) : nullptr;
  BlockRec* recs = (BlockRec*)(base + L.recs);
  uint64_t* esums = (uint64_t*)(base + L.esums);
  uint64_t* evals = multi ? (uint64_t*)(base + L.evals) : nullptr;
  hipLaunchKernelGGL(k_seg_prefix, dim3(1), dim3(kT), 0, stream, offsets, n_filters, bstart,
                     estart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t wgs_b = (L.grid_b + kWavesPerWG - 1) / kWavesPerWG;
  if constexpr (multi)
    hipLaunchKernelGGL((k_seg_records<T, multi>), dim3(L.grid_b + L.grid_e), dim3(kT), 0, stream,
                       w, offsets, n_filters, L.grid_b, key, offset, filter_base, bstart, estart,
                       recs, esums, evals);
  else
    hipLaunchKernelGGL((k_seg_records_w<T>), dim3(wgs_b), dim3(kT), 0, stream, w, offsets,
                       n_filters, bstart, recs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  u128* C = (u128*)(base + L.carries);
  u128* CE = (u128*)(base + L.ecarries);
  SegHdr* hdr = (SegHdr*)(base + L.hdr);
  hipLaunchKernelGGL((k_seg_carries<multi>), dim3(n_filters), dim3(kT), 0, stream, n_filters,
                     bstart, estart, recs, esums, C, CE, hdr);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if constexpr (multi)
    hipLaunchKernelGGL((k_seg_emit_mw<T>), dim3(wgs_b), dim3(kT), 0, stream, w, offsets,
                       n_filters, key, offset, filter_base, bstart, estart, recs, C, CE, hdr, a,
                       flags, (const uint64_t*)evals);
  else
    hipLaunchKernelGGL((k_seg_emit_w<T, SCHEME>), dim3(wgs_b), dim3(kT), 0, stream, w, offsets,
                       n_filters, key, offset, filter_base, bstart, recs, C, hdr, a, flags);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_segmented_scheme(int scheme, const void* w, int64_t n_total,
                                   const int64_t* offsets, uint32_t n_filters, Key key,
                                   uint32_t offset, uint32_t filter_base, int32_t* a, void* ws,
                                   uint32_t* flags, hipStream_t stream) {
  const T* wt = (const T*)w;
  switch (scheme) {
    case SCHEME_MULTINOMIAL:
      return launch_segmented_t<T, SCHEME_MULTINOMIAL>(wt, n_total, offsets, n_filters, key,
                                                       offset, filter_base, a, ws, flags, stream);
    case SCHEME_STRATIFIED:
      return launch_segmented_t<T, SCHEME_STRATIFIED>(wt, n_total, offsets, n_filters, key,
                                                      offset, filter_base, a, ws, flags, stream);
    default:
      return launch_segmented_t<T, SCHEME_SYSTEMATIC>(wt, n_total, offsets, n_filters, key,
                                                      offset, filter_base, a, ws, flags, stream);
  }
}

}  // namespace

SegLayout seg_layout(int64_t n_total, uint32_t n_filters, bool multinomial) {
  SegLayout L;
  // upper bounds of the block counts: each segment adds at most one partial block
  L.grid_b = (uint32_t)(n_total / kBlock + n_filters);
  L.grid_e = multinomial ? (uint32_t)((n_total + n_filters) / kBlock + n_filters) : 0u;
  L.bstart = 0;
  L.estart = align256(((size_t)n_filters + 1) * sizeof(uint32_t));
  L.recs = L.estart + (multinomial ? align256(((size_t)n_filters + 1) * sizeof(uint32_t)) : 0);
  L.esums = L.recs + align256((size_t)L.grid_b * sizeof(BlockRec));
  L.carries = L.esums + align256((size_t)L.grid_e * sizeof(uint64_t));
  L.ecarries = L.carries + align256(((size_t)L.grid_b + n_filters) * sizeof(u128));
  L.hdr = L.ecarries +
          (multinomial ? align256(((size_t)L.grid_e + n_filters) * sizeof(u128)) : 0);
  L.evals = L.hdr + align256((size_t)n_filters * sizeof(SegHdr));
  L.total = L.evals + (multinomial ? align256((size_t)L.grid_e * kBlock * sizeof(uint64_t)) : 0);
  return L;
}

hipError_t launch_scan_segmented(int scheme, bool f64, const void* w, int64_t n_total,
                                 const int64_t* offsets, uint32_t n_filters, Key key,
                                 uint32_t offset, uint32_t filter_base, int32_t* a, void* ws,
                                 uint32_t* flags, hipStream_t stream) {
  return f64 ? launch_segmented_scheme<double>(scheme, w, n_total, offsets, n_filters, key,
                                               offset, filter_base, a, ws, flags, stream)
             : launch_segmented_scheme<float>(scheme, w, n_total, offsets, n_filters, key,
                                              offset, filter_base, a, ws, flags, stream);
}

ScanLayout scan_layout(int64_t n, bool multinomial) {
  const size_t nb = (size_t)((n + kBlock - 1) / kBlock);
  const size_t nbe = multinomial ? (size_t)((n + 1 + kBlock - 1) / kBlock) : 0;
  ScanLayout L;
  L.recs = 256;
  L.carries = L.recs + align256(nb * sizeof(BlockRec));
  L.erecs = L.carries + align256((nb + 1) * sizeof(u128));
  L.ecarries = L.erecs + align256(nbe * sizeof(uint64_t));
  L.groups = L.ecarries + align256((nbe + 1) * sizeof(u128));
  const size_t G = carry_groups((uint32_t)nb), Ge = carry_groups((uint32_t)nbe);
  L.egroups = L.groups + align256(G * sizeof(CarryGroup) + (G + 1) * sizeof(u128));
  L.evals = L.egroups + align256(Ge * sizeof(CarryGroup) + (Ge + 1) * sizeof(u128));
  L.total = L.evals + align256(nbe * kBlock * sizeof(uint64_t));
  return L;
}

size_t batch_scan_lds_bytes() { return sizeof(BatchLds) + sizeof(EmitLds); }

hipError_t launch_scan(int scheme, bool f64, const void* w, int64_t n, Key key, uint32_t offset,
                       uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                       hipStream_t stream) {
  return f64 ? launch_scan_scheme<double>(scheme, w, n, key, offset, filter, a, ws, flags, stream)
             : launch_scan_scheme<float>(scheme, w, n, key, offset, filter, a, ws, flags, stream);
}

size_t multinomial_iid_workspace_bytes(int64_t n) {
  return scan_layout(n, false).total + align256((size_t)n * sizeof(double));
}

template <typename T>
hipError_t launch_multinomial_iid_t(const T* w, int64_t n, Key key, uint32_t offset,
                                    uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                                    hipStream_t stream) {
  const ScanLayout L = scan_layout(n, false);
  char* base = (char*)ws;
  ScanHeader* hdr = (ScanHeader*)base;
  BlockRec* recs = (BlockRec*)(base + L.recs);
  double* r = (double*)(base + L.total);
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  const uint32_t wgs_b = (nb + kWavesPerWG - 1) / kWavesPerWG;
  const CarrySet cs = carry_set(L, base, nb, 0u);
  hipLaunchKernelGGL((k_scan_records_w<T, false>), dim3(wgs_b), dim3(kT), 0, stream, w, n, nb,
                     wgs_b, key, offset, filter, recs, (uint64_t*)nullptr, (uint64_t*)nullptr, hdr);
  launch_carries<false>(cs, hdr, recs, nullptr, stream);
  hipLaunchKernelGGL((k_scan_r<T>), dim3(wgs_b), dim3(kT), 0, stream, w, n, nb, hdr, recs, cs.C,
                     r);
  // splitter stride: the smallest power of two leaving at most kSplit splitters
  int sl = 0;
  while (((n - 1) >> sl) > kSplit) ++sl;
  int64_t grid = (n + kT - 1) / kT;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(k_multinomial_iid, dim3((unsigned)grid), dim3(kT), 0, stream, n, hdr, r, sl,
                     key, offset, filter, a, flags);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scan_r_t(const T* w, int64_t n, double* r, void* ws, uint32_t* flags,
                           hipStream_t stream) {
  const ScanLayout L = scan_layout(n, false);
  char* base = (char*)ws;
  ScanHeader* hdr = (ScanHeader*)base;
  BlockRec* recs = (BlockRec*)(base + L.recs);
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  const uint32_t wgs_b = (nb + kWavesPerWG - 1) / kWavesPerWG;
  const CarrySet cs = carry_set(L, base, nb, 0u);
  hipLaunchKernelGGL((k_scan_records_w<T, false>), dim3(wgs_b), dim3(kT), 0, stream, w, n, nb,
                     wgs_b, Key{0, 0, nullptr}, 0u, 0u, recs, (uint64_t*)nullptr,
                     (uint64_t*)nullptr, hdr);
  launch_carries<false>(cs, hdr, recs, nullptr, stream);
  hipLaunchKernelGGL((k_scan_r<T>), dim3(wgs_b), dim3(kT), 0, stream, w, n, nb, hdr, recs, cs.C,
                     r);
  if (flags) hipLaunchKernelGGL(k_scan_status, dim3(1), dim3(1), 0, stream, hdr, flags);
  return hipGetLastError();
}

hipError_t launch_scan_r(bool f64, const void* w, int64_t n, double* r, void* ws, uint32_t* flags,
                         hipStream_t stream) {
  return f64 ? launch_scan_r_t((const double*)w, n, r, ws, flags, stream)
             : launch_scan_r_t((const float*)w, n, r, ws, flags, stream);
}

hipError_t launch_multinomial_iid(bool f64, const void* w, int64_t n, Key key, uint32_t offset,
                                  uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                                  hipStream_t stream) {
  return f64 ? launch_multinomial_iid_t((const double*)w, n, key, offset, filter, a, ws, flags,
                                        stream)
             : launch_multinomial_iid_t((const float*)w, n, key, offset, filter, a, ws, flags,
                                        stream);
}

hipError_t launch_scan_claimed(int scheme, bool f64, const void* w, int64_t n, Key key,
                               uint32_t offset, uint32_t filter, int32_t* a, void* ws,
                               uint32_t* flags, int32_t* d, int32_t* e, hipStream_t stream) {
  if (scheme == SCHEME_MULTINOMIAL)
    return f64 ? launch_scan_t<double, SCHEME_MULTINOMIAL>(w, n, key, offset, filter, a, ws,
                                                           flags, stream, d, e)
               : launch_scan_t<float, SCHEME_MULTINOMIAL>(w, n, key, offset, filter, a, ws, flags,
                                                          stream, d, e);
  if (scheme == SCHEME_STRATIFIED)
    return f64 ? launch_scan_t<double, SCHEME_STRATIFIED>(w, n, key, offset, filter, a, ws, flags,
                                                          stream, d, e)
               : launch_scan_t<float, SCHEME_STRATIFIED>(w, n, key, offset, filter, a, ws, flags,
                                                         stream, d, e);
  if (scheme == SCHEME_SYSTEMATIC)
    return f64 ? launch_scan_t<double, SCHEME_SYSTEMATIC>(w, n, key, offset, filter, a, ws, flags,
                                                          stream, d, e)
               : launch_scan_t<float, SCHEME_SYSTEMATIC>(w, n, key, offset, filter, a, ws, flags,
                                                         stream, d, e);
  return hipErrorInvalidValue;
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
