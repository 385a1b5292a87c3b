// pfr_scan_common.h -- device code shared by the exact and the floating-point
// prefix paths of the collective resamplers: workgroup scans, block loads,
// the exponential spacings of the multinomial scheme, and the emission of
// ancestors from a monotone scaled prefix r (stratified / systematic strata
// and multinomial points).  Included inside namespace pfr { namespace { } }.
#pragma once


constexpr int kT = kWGThreads;   // threads per workgroup
constexpr int kPer = kBlock / kT;  // consecutive values per thread (4)
constexpr int kNW = kT / kWave;    // waves per workgroup
constexpr int kCarryBits = 100;    // carries stay below 2^100
constexpr int kChunk = 2048;       // output positions per LDS marker pass
constexpr int kUTab = 2048;        // stratum offsets cached per block

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------- workgroup
struct WgScratch {
  u128 v[kNW];
  uint64_t u[kNW];
  int32_t i[2 * kNW];
};

template <typename U, typename Op>
__device__ U wg_reduce(U x, Op op, U* slot) {
  const int wave = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  x = wave_reduce(x, op);
  __syncthreads();
  if (lane == 0) slot[wave] = x;
  __syncthreads();
  U t = slot[0];
#pragma unroll
  for (int w2 = 1; w2 < kNW; ++w2) t = op(t, slot[w2]);
  __syncthreads();
  return t;
}

// Exclusive prefix (across the workgroup, in thread order) of x; *total gets
// the workgroup sum.
template <typename U>
__device__ U wg_exclusive(U x, U* slot, U* total) {
  const int wave = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  const U incl = wave_inclusive_scan(x, OpAdd());
  __syncthreads();
  if (lane == kWave - 1) slot[wave] = incl;
  __syncthreads();
  U run = incl - x, tot = 0;
#pragma unroll
  for (int w2 = 0; w2 < kNW; ++w2) {
    if (w2 < wave) run += slot[w2];
    tot += slot[w2];
  }
  __syncthreads();
  *total = tot;
  return run;
}

// ---------------------------------------------------------------- block loads
// Thread t holds elements 4t .. 4t+3 of the block.
template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ w, int64_t n, int64_t base,
                                      T (&x)[kPer]) {
  const int64_t idx = base + (int64_t)threadIdx.x * kPer;
  const bool aligned = ((reinterpret_cast<uintptr_t>(w + idx) & 15u) == 0);
  if (aligned && idx + kPer <= n) {
    if constexpr (sizeof(T) == 4) {
      const float4 t = *reinterpret_cast<const float4*>(w + idx);
      x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
    } else {
      const double2 t0 = *reinterpret_cast<const double2*>(w + idx);
      const double2 t1 = *reinterpret_cast<const double2*>(w + idx + 2);
      x[0] = t0.x; x[1] = t0.y; x[2] = t1.x; x[3] = t1.y;
    }
  } else {
#pragma unroll
    for (int v = 0; v < kPer; ++v) x[v] = (idx + v < n) ? w[idx + v] : (T)0;
  }
}
// -log((x + 1/2) 2^-32) for a 32-bit word x, in binary64 within about 2^-48
// of the true value (E is below 23).  y = x + 1/2 = m 2^e with m in
// [sqrt(1/2), sqrt(2)); log m = 2 atanh(s), s = (m - 1) / (m + 1), |s| <= 0.1716,
// by the series s + s^3/3 + ... + s^21/21 (Abramowitz & Stegun 4.1.27; the
// next term is below 2^-62); s comes from a reciprocal refined by two Newton
// steps.  E = (32 - e) ln 2 - log m, with ln 2 split so that (32 - e) times its
// leading part is exact.  About 30 instructions instead of a general log.
__device__ __forceinline__ double neg_log_spacing(uint32_t x) {
  const double y = (double)x + 0.5;
  int e;
  double m = frexp(y, &e);  // y = m 2^e, m in [1/2, 1)
  const bool lo = m < 0x1.6a09e667f3bcdp-1;  // sqrt(1/2)
  m = lo ? 2.0 * m : m;
  e = lo ? e - 1 : e;
  const double num = m - 1.0, den = m + 1.0;
  double rc = __builtin_amdgcn_rcp(den);
  rc = __fma_rn(__fma_rn(-den, rc, 1.0), rc, rc);
  rc = __fma_rn(__fma_rn(-den, rc, 1.0), rc, rc);
  const double sv = num * rc;
  const double s2 = sv * sv;
  double t = 1.0 / 21.0;
  t = __fma_rn(t, s2, 1.0 / 19.0);
  t = __fma_rn(t, s2, 1.0 / 17.0);
  t = __fma_rn(t, s2, 1.0 / 15.0);
  t = __fma_rn(t, s2, 1.0 / 13.0);
  t = __fma_rn(t, s2, 1.0 / 11.0);
  t = __fma_rn(t, s2, 1.0 / 9.0);
  t = __fma_rn(t, s2, 1.0 / 7.0);
  t = __fma_rn(t, s2, 1.0 / 5.0);
  t = __fma_rn(t, s2, 1.0 / 3.0);
  t *= s2;
  const double two_s = 2.0 * sv;
  const double log_m = __fma_rn(two_s, t, two_s);
  const double k = (double)(32 - e);
  constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;  // ln 2 to 42 bits: k * kLn2Hi is exact
  constexpr double kLn2Lo = 0x1.ef35793c76730p-45;  // ln 2 - kLn2Hi
  return k * kLn2Hi + __fma_rn(k, kLn2Lo, -log_m);
}

// Exponential spacing E_k = -log((x + 1/2) 2^-32), k = 0..n: word k&3 of
// Philox call k>>2 (exponential domain), quantised to floor(E 2^48).  Thread t
// of block b holds k = 1024 b + 4t + v, all four from call 256 b + t.
__device__ __forceinline__ void exp_values(Key key, uint32_t filter, uint32_t offset, int64_t n,
                                           uint32_t blk, uint64_t (&q)[kPer]) {
  const uint32_t call = blk * (uint32_t)kT + threadIdx.x;
  const uint4 x = draw(key, call, DOM_EXP, 0, filter, offset);
  const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
  for (int v = 0; v < kPer; ++v) {
    const int64_t k = (int64_t)call * 4 + v;
    const double e = neg_log_spacing(xs[v]);
    q[v] = (k <= n) ? (uint64_t)(e * 0x1p48) : 0ull;
  }
}

// The four quantised spacings of thread t in block b, stored by the records
// pass at evals[b kBlock + 4 t ..] (32-byte aligned).
__device__ __forceinline__ void store_exp_values(uint64_t* __restrict__ evals, uint32_t blk,
                                                 const uint64_t (&q)[kPer]) {
  ulonglong2* p = reinterpret_cast<ulonglong2*>(evals + (size_t)blk * kBlock + threadIdx.x * kPer);
  p[0] = make_ulonglong2(q[0], q[1]);
  p[1] = make_ulonglong2(q[2], q[3]);
}
__device__ __forceinline__ void load_exp_values(const uint64_t* __restrict__ evals, uint32_t blk,
                                                uint64_t (&q)[kPer]) {
  const ulonglong2* p =
      reinterpret_cast<const ulonglong2*>(evals + (size_t)blk * kBlock + threadIdx.x * kPer);
  const ulonglong2 v0 = p[0], v1 = p[1];
  q[0] = v0.x;
  q[1] = v0.y;
  q[2] = v1.x;
  q[3] = v1.y;
}

__device__ __forceinline__ int ceil_log2(uint32_t x) {
  return x <= 1 ? 0 : 32 - __clz(x - 1);
}
// Exclusive scan of the exponential block sums into CE[0..nbe].
template <typename SumPtr, typename CPtr>
__device__ void exp_carries(uint32_t nbe, SumPtr sums, CPtr CE, WgScratch* s) {
  const int tid = (int)threadIdx.x;
  u128 carry = 0;
  for (uint32_t base = 0; base < nbe; base += kBlock) {
    u128 v[kPer];
    u128 mine = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t b = base + (uint32_t)tid * kPer + k;
      v[k] = (b < nbe) ? (u128)sums[b] : (u128)0;
      mine += v[k];
    }
    u128 tot;
    u128 run = carry + wg_exclusive(mine, s->v, &tot);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t b = base + (uint32_t)tid * kPer + k;
      if (b < nbe) CE[b] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (tid == 0) CE[nbe] = carry;
  __syncthreads();
}

// ---------------------------------------------------------------- r map
// r(I) = n * I / Q in binary64, monotone in I, with r(Q) = n exactly.
struct RMap {
  u128 Q;
  double invQ;
  double Nd;
  __device__ double operator()(u128 I) const {
    if (I >= Q) return Nd;
    const double r = Nd * (u128_to_double(I) * invQ);
    return r < Nd ? r : Nd;
  }
};

__device__ __forceinline__ RMap make_rmap(u128 Q, int64_t n) {
  RMap m;
  m.Q = Q;
  m.invQ = 1.0 / u128_to_double(Q);
  m.Nd = (double)n;
  return m;
}

// ---------------------------------------------------------------- strata
// O = #{s : s + 1 - u_s <= r}: all strata below floor(r), plus stratum
// m = floor(r) when frac(r) >= 1 - u_m (both sides exact in binary64).
__device__ __forceinline__ int64_t cum_strata(double r, int64_t n, double u) {
  const double mf = floor(r);
  const int64_t m = (int32_t)mf;  // 0 <= r <= n < 2^31: the 32-bit conversion is exact
  if (m >= n) return n;
  return m + (((r - mf) >= (1.0 - u)) ? 1 : 0);
}

// The literal binary32 form min(n, floor(r + u_m)), m = floor(r), of Codes 7
// and 8, with u_m the 24-bit offset (x >> 8) 2^-24 (r is a binary32 value).
// The sum r + u_m is rounded to binary32, which can move it across an integer:
// this is the numerical defect the paper measures for large n.
__device__ __forceinline__ int64_t cum_strata_naive(double r, int64_t n, uint32_t word) {
  const float rf = (float)r;
  if (floor(r) >= (double)n) return n;
  const float u = (float)(word >> 8) * 0x1p-24f;
  const float t = rf + u;
  const int64_t o = (int64_t)floorf(t);
  return o < n ? o : n;
}

// Cumulative offspring O(r) given the raw offset word of stratum floor(r).
template <bool NAIVE>
__device__ __forceinline__ int64_t cum_of(double r, int64_t n, uint32_t word) {
  if (NAIVE) return cum_strata_naive(r, n, word);
  return cum_strata(r, n, u_offset(word));
}

struct StrataLds {
  uint32_t O[kBlock];  // cumulative offspring of the block's particles
  uint32_t u[kUTab];   // raw stratum-offset words of strata [m_lo, m_lo + kUTab)
  int32_t M[kChunk];   // expansion markers
};

// Raw 32-bit word of stratum m's offset (word m&3 of Philox call m>>2).
__device__ __forceinline__ uint32_t stratum_word(Key key, uint32_t filter, uint32_t offset,
                                                 int64_t m) {
  const uint4 x = draw(key, (uint32_t)(m >> 2), DOM_STRATA, 0, filter, offset);
  const uint32_t k = (uint32_t)(m & 3);
  return k == 0 ? x.x : k == 1 ? x.y : k == 2 ? x.z : x.w;
}

// In-place inclusive max-scan of M[0..len), len <= kChunk, entries >= -1.
__device__ void wg_max_scan(int32_t* M, int len, WgScratch* s) {
  const int tid = (int)threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  constexpr int per = kChunk / kT;
  int32_t run = -1;
  int32_t v[per];
#pragma unroll
  for (int k = 0; k < per; ++k) {
    const int idx = tid * per + k;
    v[k] = idx < len ? M[idx] : -1;
    run = max(run, v[k]);
  }
  // shifted by one so that the scan runs on non-negative values
  const uint32_t incl = wave_inclusive_scan((uint32_t)(run + 1), OpMax());
  __syncthreads();
  if (lane == kWave - 1) s->i[wave] = (int32_t)incl - 1;
  __syncthreads();
  const uint32_t prev = shfl(incl, lane > 0 ? lane - 1 : 0);
  int32_t carry = lane > 0 ? (int32_t)prev - 1 : -1;
  for (int w2 = 0; w2 < wave; ++w2) carry = max(carry, s->i[w2]);
#pragma unroll
  for (int k = 0; k < per; ++k) {
    carry = max(carry, v[k]);
    const int idx = tid * per + k;
    if (idx < len) M[idx] = carry;
  }
  __syncthreads();
}

// Stratified / systematic emission for one block: r[4] are the thread's
// particles (4t .. 4t+3; values past the vector's end equal r_hi).  Writes
// a_out[s] = P0 + i for every stratum s in [O(r_lo), O(r_hi)).  The r must be
// non-decreasing and within [r_lo, r_hi]; u_sys is the raw offset word of the
// systematic scheme.
//
// With d_out and e_out (both or neither), the Prepermute of Code 10 is fused
// in: the output is sorted, so particle i's claim is the first position of its
// run, d_out[i] = O_{i-1} (n when it has no offspring), and the marked
// ancestry is e_out[s] = i at the first position of i's run, -1 - i at the
// others -- what the claim pass of permute_ancestors would write.
template <bool SYSTEMATIC, bool NAIVE>
__device__ void emit_strata(const double (&r)[kPer], int cnt, double r_lo, double r_hi, int64_t n,
                            int64_t P0, Key key, uint32_t filter, uint32_t offset, uint32_t u_sys,
                            int32_t* __restrict__ a_out, StrataLds* L, WgScratch* s,
                            int32_t* __restrict__ d_out = nullptr,
                            int32_t* __restrict__ e_out = nullptr) {
  const int tid = (int)threadIdx.x;
  // stratum offsets of the strata the block's r-range touches
  const int64_t m_lo = (int64_t)floor(r_lo);
  const int64_t m_hi = min(n - 1, (int64_t)floor(r_hi));
  const bool table = SYSTEMATIC || (m_hi - m_lo + 1 <= kUTab);
  if (!SYSTEMATIC && table && m_hi >= m_lo) {
    for (int64_t c = (m_lo >> 2) + tid; c <= (m_hi >> 2); c += kT) {
      const uint4 x = draw(key, (uint32_t)c, DOM_STRATA, 0, filter, offset);
      const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = c * 4 + v;
        if (m >= m_lo && m <= m_hi) L->u[m - m_lo] = xs[v];
      }
    }
  }
  __syncthreads();
  auto u_of = [&](int64_t m) -> uint32_t {
    if (SYSTEMATIC) return u_sys;
    if (m > m_hi) return 0u;  // reached only with m >= n, where u is unused
    return table ? L->u[m - m_lo] : stratum_word(key, filter, offset, m);
  };
#pragma unroll
  for (int v = 0; v < kPer; ++v)
    L->O[tid * kPer + v] = (uint32_t)cum_of<NAIVE>(r[v], n, u_of((int64_t)floor(r[v])));
  const int64_t O_lo = cum_of<NAIVE>(r_lo, n, u_of(m_lo));
  const int64_t O_hi = cum_of<NAIVE>(r_hi, n, u_of((int64_t)floor(r_hi)));
  __syncthreads();
  if (d_out) {
    for (int e = tid; e < cnt; e += kT) {
      const int64_t Oe = L->O[e];
      const int64_t Op = e == 0 ? O_lo : (int64_t)L->O[e - 1];
      d_out[P0 + e] = (int32_t)(Oe > Op ? Op : n);
    }
  }
  // expansion: a marker at the first output of every particle, then a max-scan
  for (int64_t cs = O_lo; cs < O_hi; cs += kChunk) {
    const int64_t ce = min(cs + (int64_t)kChunk, O_hi);
    for (int k = tid; k < kChunk; k += kT) L->M[k] = -1;
    __syncthreads();
    for (int e = tid; e < cnt; e += kT) {
      const int64_t Oe = L->O[e];
      const int64_t Op = e == 0 ? O_lo : (int64_t)L->O[e - 1];
      if (Oe > Op && Oe > cs && Op < ce) L->M[(Op > cs ? Op : cs) - cs] = e;
    }
    __syncthreads();
    const int len = (int)(ce - cs);
    wg_max_scan(L->M, len, s);
    for (int k = tid; k < len; k += kT) a_out[cs + k] = (int32_t)(P0 + L->M[k]);
    if (e_out) {
      for (int k = tid; k < len; k += kT) {
        const int e = L->M[k];
        const int64_t Op = e == 0 ? O_lo : (int64_t)L->O[e - 1];
        e_out[cs + k] = (cs + k == Op) ? (int32_t)(P0 + e) : (int32_t)(-1 - (P0 + e));
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- multinomial
struct MultiLds {
  double r[kBlock];
};

// #{i in [0, cnt) : r[i] <= p} for the 4 points of a thread, searched together
// so that the LDS loads of the 4 searches overlap.
__device__ __forceinline__ void count_le4(const double* __restrict__ r, int cnt,
                                          const double (&p)[kPer], int (&pos)[kPer]) {
#pragma unroll
  for (int q = 0; q < kPer; ++q) pos[q] = 0;
  int step = 1;
  while ((step << 1) <= cnt) step <<= 1;
  for (; step > 0; step >>= 1) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int np = pos[q] + step;
      const double v = r[min(np, cnt) - 1];
      if (np <= cnt && v <= p[q]) pos[q] = np;
    }
  }
}

// Multinomial points for a block with r-range [r_lo, r_hi) (the vector's last
// block: [r_lo, inf)).  The points p_k = n S_k / S_n of every exponential
// block whose points can fall in the range are rebuilt from the exact carries
// CE[b] and the quantised spacings of the block: read from `evals` (kBlock
// per block, stored by the records pass) when given, else recomputed from
// their Philox calls.
template <typename CEPtr>
__device__ void emit_multinomial(const double* __restrict__ r_lds, int cnt, double r_lo,
                                 double r_hi, bool last, int64_t n, int64_t P0, Key key,
                                 uint32_t filter, uint32_t offset, CEPtr CE, uint32_t nbe,
                                 int32_t* __restrict__ a_out, WgScratch* s,
                                 const uint64_t* __restrict__ evals = nullptr) {
  if (cnt <= 0 || !(last || r_hi > r_lo)) return;
  const RMap em = make_rmap(CE[nbe], n);
  // P(b) = value of the last point of exponential block b-1, b = 1..nbe-1
  auto count_below = [&](double x) -> uint32_t {  // #{b in [1, nbe-1] : P(b) < x}
    uint32_t lo = 1, hi = nbe;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (em(CE[mid]) < x) lo = mid + 1;
      else hi = mid;
    }
    return lo - 1;
  };
  // The boundaries lie within a few blocks of b * 1024 (the spacings have
  // mean 1), so one coalesced probe of a 256-block window around the guess
  // settles both counts; the bisection above is the fallback.
  uint32_t b_first, b_last;
  {
    const double per_block = (double)kBlock * (double)n / (double)(n + 1);
    const int64_t guess = (int64_t)(r_lo / per_block);
    int64_t w0 = guess - kT / 2;
    if (w0 < 1) w0 = 1;
    const int64_t b = w0 + threadIdx.x;
    const bool in = b <= (int64_t)nbe - 1;
    const double P = in ? em(CE[b]) : 0.0;
    const uint32_t below_lo = wg_reduce((uint32_t)(in && P < r_lo), OpAdd(), (uint32_t*)s->i);
    const uint32_t below_hi = wg_reduce((uint32_t)(in && P < r_hi), OpAdd(), (uint32_t*)s->i);
    const int64_t w1 = min(w0 + (int64_t)kT - 1, (int64_t)nbe - 1);  // last probed boundary
    // every boundary before w0 must be below r_lo, every one after w1 at or above
    // the value counted (checked on the probed end points)
    const int64_t span = w1 - w0 + 1;
    const bool lo_ok = (w0 == 1 || below_lo > 0) && (w1 == (int64_t)nbe - 1 || below_lo < span);
    const bool hi_ok = (w0 == 1 || below_hi > 0) && (w1 == (int64_t)nbe - 1 || below_hi < span);
    b_first = lo_ok ? (uint32_t)(w0 - 1 + below_lo) : count_below(r_lo);
    b_last = last ? nbe - 1 : (hi_ok ? (uint32_t)(w0 - 1 + below_hi) : count_below(r_hi));
  }
  for (uint32_t b = b_first; b <= b_last; ++b) {
    uint64_t q[kPer];
    if (evals) load_exp_values(evals, b, q);
    else exp_values(key, filter, offset, n, b, q);
    uint64_t acc = 0;
#pragma unroll
    for (int v = 0; v < kPer; ++v) {
      acc += q[v];
      q[v] = acc;
    }
    uint64_t tot;
    const uint64_t off = wg_exclusive(acc, s->u, &tot);
    const u128 base = CE[b] + (u128)off;
    double p[kPer];
#pragma unroll
    for (int v = 0; v < kPer; ++v) p[v] = em(base + (u128)q[v]);
    int pos[kPer];
    count_le4(r_lds, cnt, p, pos);
#pragma unroll
    for (int v = 0; v < kPer; ++v) {
      const int64_t k = (int64_t)b * kBlock + threadIdx.x * kPer + v;
      if (k >= n) continue;
      if (p[v] < r_lo) continue;
      if (!last && !(p[v] < r_hi)) continue;
      int64_t anc = P0 + pos[v];
      if (anc > n - 1) anc = n - 1;
      a_out[k] = (int32_t)anc;
    }
  }
}

// ---------------------------------------------------------------- block emit
union EmitLds {
  StrataLds st;
  MultiLds mu;
};

