// pfr_device.h -- device-side building blocks of libpfresample (gfx950).
//
// Philox4x32-10 counter-based random numbers, the canonical draws every kernel
// takes from it, the exact accept test of the Metropolis and rejection
// resamplers, wave64 primitives (shuffle, ballot, scans) and the 128-bit
// integer helpers of the exact prefix sums.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfr {

constexpr int kWave = 64;

// Philox counter word 1 is (domain << 28) | step.
constexpr uint32_t DOM_STRATA = 0u;  // stratified / systematic offsets
constexpr uint32_t DOM_EXP = 1u;     // exponential spacings (multinomial)
constexpr uint32_t DOM_TRIAL = 2u;   // Metropolis steps, rejection trials
constexpr uint32_t DOM_NOISE = 3u;   // state-space propagation noise
constexpr uint32_t DOM_INIT = 4u;    // state-space initial state
constexpr uint32_t DOM_UNIFORM = 5u; // independent uniforms (multinomial, Code 5)

// Result bits OR-ed into the caller's device flag word.
constexpr uint32_t FLAG_ZERO_TOTAL = 1u;
constexpr uint32_t FLAG_TRIAL_CAP = 2u;
constexpr uint32_t FLAG_BAD_COUNTS = 4u;
constexpr uint32_t FLAG_BAD_WEIGHTS = 8u;
constexpr uint32_t FLAG_BAD_ANCESTOR = 16u;
constexpr uint32_t FLAG_BAD_STEP = 32u;
constexpr uint32_t FLAG_WMAX_BELOW = 64u;   // precondition checks only
constexpr uint32_t FLAG_NOT_SORTED = 128u;  // precondition checks only

// Philox key, and optionally the device word that holds the counter offset
// (read when the kernel runs, so that a captured graph can advance it).
struct Key {
  uint32_t k0, k1;
  const uint32_t* offset_dev;
};

__device__ __forceinline__ uint32_t counter_offset(const Key& key, uint32_t offset) {
  // the same value on every lane: kept in a scalar register, so that the
  // uniform parts of the Philox calls that use it stay on the scalar unit
  return key.offset_dev ? (uint32_t)__builtin_amdgcn_readfirstlane(*key.offset_dev) : offset;
}

// Philox4x32 (Salmon, Moraes, Dror & Shaw, SC'11).  Each round
// forms the 64-bit products of counter words 0 and 2 with two odd multipliers
// and mixes their high halves with words 1 and 3 and the round key; the key
// advances by two Weyl increments per round.  The key is uniform across the
// wave in every kernel, so its schedule stays in scalar registers.
// a ^ b ^ k in one VALU instruction (gfx950 three-input bit operation, truth
// table 0x96 = xor of the three inputs).
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k) {
  return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

// The round count is 10 (Philox4x32-10); a study build may set another with
// -DPFR_PHILOX_ROUNDS (Salmon et al. report 7 rounds as the least that passes
// their statistical test batteries, 10 as the default with a safety margin).
#ifndef PFR_PHILOX_ROUNDS
#define PFR_PHILOX_ROUNDS 10
#endif
static_assert(PFR_PHILOX_ROUNDS >= 1 && PFR_PHILOX_ROUNDS <= 16, "Philox round count");
constexpr int kPhiloxRounds = PFR_PHILOX_ROUNDS;

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        Key key) {
  uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
  for (int r = 0; r < kPhiloxRounds; ++r) {
    // one v_mad_u64_u32 per product (instead of separate mul_hi / mul_lo)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    c0 = xor3_key((uint32_t)(p1 >> 32), c1, k0);
    c1 = (uint32_t)p1;
    c2 = xor3_key((uint32_t)(p0 >> 32), c3, k1);
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint4 draw(Key key, uint32_t index, uint32_t domain, uint32_t step,
                                      uint32_t filter, uint32_t offset) {
  return philox(index, (domain << 28) | (step & 0x0FFFFFFFu), filter, offset, key);
}

// The same call for arguments that are the same on every lane of the wave:
// plain two-input xors, which the compiler keeps on the scalar unit (the
// three-input form above exists only as a vector instruction).  Same bits.
__device__ __forceinline__ uint4 draw_uniform(Key key, uint32_t index, uint32_t domain,
                                              uint32_t step, uint32_t filter, uint32_t offset) {
  uint32_t c0 = index, c1 = (domain << 28) | (step & 0x0FFFFFFFu), c2 = filter, c3 = offset;
  uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
  for (int r = 0; r < kPhiloxRounds; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    c0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    c1 = (uint32_t)p1;
    c2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}


// u in (0, 1] on the 2^-32 lattice (accept tests).
__device__ __forceinline__ double u_accept(uint32_t x) { return ((double)x + 1.0) * 0x1p-32; }
// u in [0, 1) on the 2^-32 lattice (stratum offsets).
__device__ __forceinline__ double u_offset(uint32_t x) { return (double)x * 0x1p-32; }
// j uniform on [0, n): high 64 bits of the 64x64-bit product.
__device__ __forceinline__ uint32_t index_draw(uint32_t x0, uint32_t x1, uint32_t n) {
  const uint64_t r = ((uint64_t)x1 << 32) | x0;
  return (uint32_t)__umul64hi(r, (uint64_t)n);
}

// Exact u * wk <= wj for weights of type T (u on the 2^-32 lattice).  One
// fused multiply-add forms u wk - wj exactly and rounds it once; rounding to
// nearest keeps the sign and maps only zero to zero as long as a nonzero
// difference exceeds 2^-1075.  It does whenever wk and wj lie on the 2^-1042
// lattice (u wk then lies on the 2^-1074 lattice): every float32 weight, and
// binary64 weights from 2^-990 up (zero included).  Below that a nonzero
// difference of binary64 weights can round to zero; then both weights are
// below 2^-900 (they differ by less than 2^-1075), so the test is repeated on
// both scaled by 2^200, which is exact and puts them back on the lattice.
template <typename T>
__device__ __forceinline__ bool accept_exact(double u, double wk, double wj) {
  double d = __fma_rn(u, wk, -wj);
  if constexpr (sizeof(T) == 8) {
    if (d == 0.0 && wk < 0x1p-900) d = __fma_rn(u, wk * 0x1p200, -(wj * 0x1p200));
  }
  return d <= 0.0;
}

// ------------------------------------------------------------------ buffer gathers
// A raw buffer resource over [base, base + bytes) (bytes below 2^31).  A load
// at a byte offset at or beyond `bytes` is dropped by the range check and
// returns zero without touching memory, so a wave can issue one gather for
// all lanes, without a branch, while only the lanes that need a value read
// one: the others pass kNoLoad.  Several such gathers are then in flight at
// once and a single wait covers them.
constexpr uint32_t kNoLoad = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_view(const void* base, uint32_t bytes) {
  // 0x00020000: 32-bit data format, the setting for untyped loads on gfx9
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buffer_gather(__amdgpu_buffer_rsrc_t r, uint32_t byte_off);
template <>
__device__ __forceinline__ float buffer_gather<float>(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
}
template <>
__device__ __forceinline__ double buffer_gather<double>(__amdgpu_buffer_rsrc_t r,
                                                        uint32_t byte_off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0);
  return __builtin_bit_cast(double, ((uint64_t)v[1] << 32) | v[0]);
}

// ------------------------------------------------------------------ wave64
__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}
__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// Philox calls of one lane whose counter words 1..3 are the same on every lane
// of the wave (word 1 changing from call to call) and whose word 0 is the
// lane's particle index.  Everything that depends only on (word 0, word 2,
// word 3) -- the first round's product of word 0 and the second round's
// product of word 2 -- is formed once per lane (PhiloxLane); what depends on
// word 1 alone -- the first round's product of word 2 and the second round's
// product of word 0 -- runs on the scalar unit.  Each call then costs one
// VALU instruction for rounds 1-2 instead of eight.  The bits are those of
// draw() for any arguments; only the cost depends on the uniformity (word 1
// from a loop counter, filter and offset from kernel arguments).
struct PhiloxLane {
  uint32_t index, e0, e1, d3;
};
__device__ __forceinline__ PhiloxLane philox_lane(Key key, uint32_t index, uint32_t filter,
                                                  uint32_t offset) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * index;             // round 1, word 0
  const uint32_t d2 = (uint32_t)(p0 >> 32) ^ offset ^ key.k1;
  const uint32_t d1 = 0xCD9E8D57u * filter;                       // round 1, word 2 (low)
  const uint64_t q1 = (uint64_t)0xCD9E8D57u * d2;                 // round 2, word 2
  PhiloxLane L;
  L.index = index;
  L.e0 = (uint32_t)(q1 >> 32) ^ d1 ^ (key.k0 + 0x9E3779B9u);
  L.e1 = (uint32_t)q1;
  L.d3 = (uint32_t)p0;
  return L;
}
__device__ __forceinline__ uint4 philox_lane_call(const PhiloxLane& L, Key key, uint32_t domain,
                                                  uint32_t step, uint32_t filter,
                                                  uint32_t offset) {
  if (kPhiloxRounds < 3) return draw(key, L.index, domain, step, filter, offset);
  // (the arguments other than L are kernel arguments and loop counters, which
  // the compiler keeps in scalar registers; so are the values below)
  const uint32_t c1 = (domain << 28) | (step & 0x0FFFFFFFu);
  const uint32_t k0 = key.k0, k1 = key.k1;
  // round 1, word 2 (high): scalar
  const uint32_t d0 = __umulhi(0xCD9E8D57u, filter) ^ c1 ^ k0;
  // round 2, word 0: scalar product; its high word meets the lane's d3
  const uint64_t q0 = (uint64_t)0xD2511F53u * d0;
  const uint32_t q0hi = (uint32_t)(q0 >> 32), q0lo = (uint32_t)q0;
  const uint32_t e2 = L.d3 ^ (q0hi ^ (k1 + 0xBB67AE85u));
  // round 3: word 3 (q0lo) is still uniform
  uint32_t kk0 = k0 + 2u * 0x9E3779B9u, kk1 = k1 + 2u * 0xBB67AE85u;
  const uint64_t a0 = (uint64_t)0xD2511F53u * L.e0;
  const uint64_t a1 = (uint64_t)0xCD9E8D57u * e2;
  uint32_t c[4] = {xor3_key((uint32_t)(a1 >> 32), L.e1, kk0), (uint32_t)a1,
                   (uint32_t)(a0 >> 32) ^ (q0lo ^ kk1), (uint32_t)a0};
  kk0 += 0x9E3779B9u;
  kk1 += 0xBB67AE85u;
#pragma unroll
  for (int r = 3; r < kPhiloxRounds; ++r) {
    const uint64_t b0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t b1 = (uint64_t)0xCD9E8D57u * c[2];
    c[0] = xor3_key((uint32_t)(b1 >> 32), c[1], kk0);
    c[1] = (uint32_t)b1;
    c[2] = xor3_key((uint32_t)(b0 >> 32), c[3], kk1);
    c[3] = (uint32_t)b0;
    kk0 += 0x9E3779B9u;
    kk1 += 0xBB67AE85u;
  }
  return make_uint4(c[0], c[1], c[2], c[3]);
}

template <typename T>
__device__ __forceinline__ T shfl(T v, int src) {
  static_assert(sizeof(T) % 4 == 0, "shfl needs 32-bit words");
  union U {
    T t;
    uint32_t w[sizeof(T) / 4];
  } a, b;
  a.t = v;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) b.w[i] = shfl_u32(a.w[i], src);
  return b.t;
}
template <typename T>
__device__ __forceinline__ T readlane(T v, int lane) {
  union U {
    T t;
    uint32_t w[sizeof(T) / 4];
  } a, b;
  a.t = v;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) b.w[i] = readlane_u32(a.w[i], lane);
  return b.t;
}

// Inclusive wave scan (Hillis-Steele over 64 lanes) with a binary operator.
template <typename T, typename Op>
__device__ __forceinline__ T wave_inclusive_scan(T v, Op op) {
  const int l = (int)lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const T t = shfl(v, l >= d ? l - d : l);
    if (l >= d) v = op(t, v);
  }
  return v;
}
template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
  const int l = (int)lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) v = op(v, shfl(v, l ^ d));
  return v;
}

// ------------------------------------------------------------------ DPP scans
// Cross-lane moves of the GFX9 data-parallel primitives: shifts by 1, 2, 4, 8
// inside rows of 16 lanes, broadcasts of lane 15 (to the next row) and lane 31
// (to rows 2 and 3), and a shift of the whole wave by one lane.  A lane whose
// source lies outside its row, or whose row ROW_MASK leaves out, gets `old`.
constexpr int kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr4 = 0x114, kDppShr8 = 0x118;
constexpr int kDppBcast15 = 0x142, kDppBcast31 = 0x143, kDppWaveShr1 = 0x138;

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xF, false);
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t old, uint64_t v) {
  const uint32_t lo = dpp_u32<CTRL, ROW_MASK>((uint32_t)old, (uint32_t)v);
  const uint32_t hi = dpp_u32<CTRL, ROW_MASK>((uint32_t)(old >> 32), (uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Inclusive scans over the 64 lanes in six DPP steps: within rows, then row 0
// into row 1 and row 2 into row 3, then rows 0-1 into rows 2-3.
__device__ __forceinline__ uint64_t wave_incl_add_u64(uint64_t x) {
  x += dpp_u64<kDppShr1>(0ull, x);
  x += dpp_u64<kDppShr2>(0ull, x);
  x += dpp_u64<kDppShr4>(0ull, x);
  x += dpp_u64<kDppShr8>(0ull, x);
  x += dpp_u64<kDppBcast15, 0xA>(0ull, x);
  x += dpp_u64<kDppBcast31, 0xC>(0ull, x);
  return x;
}
// Inclusive max-scan of values >= -1.
__device__ __forceinline__ uint32_t wave_incl_add_u32(uint32_t x) {
  x += dpp_u32<kDppShr1>(0u, x);
  x += dpp_u32<kDppShr2>(0u, x);
  x += dpp_u32<kDppShr4>(0u, x);
  x += dpp_u32<kDppShr8>(0u, x);
  x += dpp_u32<kDppBcast15, 0xA>(0u, x);
  x += dpp_u32<kDppBcast31, 0xC>(0u, x);
  return x;
}
__device__ __forceinline__ int32_t wave_incl_max_i32(int32_t x) {
  const uint32_t m1 = 0xFFFFFFFFu;
  x = max(x, (int32_t)dpp_u32<kDppShr1>(m1, (uint32_t)x));
  x = max(x, (int32_t)dpp_u32<kDppShr2>(m1, (uint32_t)x));
  x = max(x, (int32_t)dpp_u32<kDppShr4>(m1, (uint32_t)x));
  x = max(x, (int32_t)dpp_u32<kDppShr8>(m1, (uint32_t)x));
  x = max(x, (int32_t)dpp_u32<kDppBcast15, 0xA>(m1, (uint32_t)x));
  x = max(x, (int32_t)dpp_u32<kDppBcast31, 0xC>(m1, (uint32_t)x));
  return x;
}
// The value of the previous lane (lane 0 gets `first`).
__device__ __forceinline__ uint32_t wave_shift_up_u32(uint32_t v, uint32_t first) {
  return dpp_u32<kDppWaveShr1>(first, v);
}
// Orders the LDS accesses of the lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

struct OpAdd {
  template <typename T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
  template <typename T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a > b ? a : b; }
};
struct OpMin {
  template <typename T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a < b ? a : b; }
};
struct OpOr {
  template <typename T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a | b; }
};

// ------------------------------------------------------------------ u128
typedef unsigned __int128 u128;

// x * 2^sh for a signed shift; bits shifted out to the right are dropped
// (floor), which is monotone in x.
__device__ __forceinline__ u128 shift_u128(u128 x, int sh) {
  if (sh >= 0) return sh >= 128 ? (u128)0 : (x << sh);
  const int r = -sh;
  return r >= 128 ? (u128)0 : (x >> r);
}
// u128 -> double for values below 2^116: the high word converts exactly, so
// fl(hi * 2^64 + fl(lo)) is monotone in x and deterministic.
__device__ __forceinline__ double u128_to_double(u128 x) {
  const uint64_t hi = (uint64_t)(x >> 64), lo = (uint64_t)x;
  return (double)hi * 0x1p64 + (double)lo;
}

// Inclusive wave scan of a 128-bit sum (six DPP steps on the four words).
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ u128 dpp_u128(u128 v) {
  const uint64_t lo = dpp_u64<CTRL, ROW_MASK>(0ull, (uint64_t)v);
  const uint64_t hi = dpp_u64<CTRL, ROW_MASK>(0ull, (uint64_t)(v >> 64));
  return ((u128)hi << 64) | (u128)lo;
}
__device__ __forceinline__ u128 wave_incl_add_u128(u128 x) {
  x += dpp_u128<kDppShr1>(x);
  x += dpp_u128<kDppShr2>(x);
  x += dpp_u128<kDppShr4>(x);
  x += dpp_u128<kDppShr8>(x);
  x += dpp_u128<kDppBcast15, 0xA>(x);
  x += dpp_u128<kDppBcast31, 0xC>(x);
  return x;
}

// ------------------------------------------------------------------ segments
// Segment f holds global indices [offsets[f], offsets[f+1]); returns the f
// with offsets[f] <= g < offsets[f+1] (offsets non-decreasing, g < offsets[F]).
__device__ __forceinline__ uint32_t find_segment(const int64_t* __restrict__ offsets,
                                                 uint32_t n_filters, int64_t g) {
  uint32_t lo = 0, hi = n_filters;  // answer in [lo, hi)
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (offsets[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------------ weights
// Weight element traits: P = significand bits (with the implicit bit), bias.
template <typename T>
struct WTraits;
template <>
struct WTraits<float> {
  typedef uint32_t Bits;
  static constexpr int P = 24, BIAS = 127, EXP_BITS = 8;
  __device__ static Bits bits(float v) { return __float_as_uint(v); }
};
template <>
struct WTraits<double> {
  typedef uint64_t Bits;
  static constexpr int P = 53, BIAS = 1023, EXP_BITS = 11;
  __device__ static Bits bits(double v) { return (Bits)__double_as_longlong(v); }
};

// A weight is usable when it is finite and >= 0 (-0 counts as 0).
template <typename T>
__device__ __forceinline__ bool weight_ok(T v) {
  return v >= (T)0 && v < (T)__builtin_huge_val();
}

// Biased exponent field of a non-negative finite weight, at least 1 (zero and
// subnormal weights share the exponent of the smallest normal).
template <typename T>
__device__ __forceinline__ int exp_field(T v) {
  typedef WTraits<T> Tr;
  const int e = (int)((Tr::bits(v) >> (Tr::P - 1)) & ((1u << Tr::EXP_BITS) - 1));
  return e < 1 ? 1 : e;
}

// Fixed-point quantisation of a weight relative to a block's reference
// exponent e_ref (the exponent field of the block maximum):
//   q = floor(v * 2^s),  s = 52 + BIAS - e_ref,
// so that q < 2^53 for every v in the block.  Computed from the bits: the
// significand (with its implicit bit) shifted by (53 - P) + e - e_ref.
template <typename T>
__device__ __forceinline__ uint64_t quantize(T v, int e_ref) {
  typedef WTraits<T> Tr;
  const typename Tr::Bits b = Tr::bits(v);
  const int ef = (int)((b >> (Tr::P - 1)) & ((1u << Tr::EXP_BITS) - 1));
  const uint64_t frac = (uint64_t)(b & (((typename Tr::Bits)1 << (Tr::P - 1)) - 1));
  const uint64_t m = ef ? (frac | ((uint64_t)1 << (Tr::P - 1))) : frac;
  const int sh = (53 - Tr::P) + (ef < 1 ? 1 : ef) - e_ref;
  if (sh >= 0) return m << sh;  // sh <= 53 - P
  return sh <= -64 ? 0ull : (m >> (-sh));
}
template <typename T>
__device__ __forceinline__ int scale_of(int e_ref) {
  return 52 + WTraits<T>::BIAS - e_ref;
}

}  // namespace pfr
