// pfr_fscan.hip -- floating-point prefix sums for the collective resamplers.
//
// Section 3.2 of the paper traces the bias its multinomial, stratified and
// systematic resamplers show from a few hundred thousand particles on to the
// rounding of the single-precision prefix sum, and reports that double
// precision removes it.  These modes run the same schemes with that
// arithmetic, so that the effect can be measured on this hardware:
//   F64        weights widened to binary64; binary64 sums and scaling
//   COMP_F32   double-float binary32 pairs (hi, lo) added with Knuth's
//              error-free TwoSum and a Fast2Sum renormalisation (Dekker);
//              binary64 scaling
//   NAIVE_F32  binary32 weights, sums and scaling r = n (W_i / W), and the
//              literal binary32 floor(r + u) of Codes 7 and 8
// Only the weight prefix changes: the multinomial points (exponential
// spacings) are the exact ones of the default mode.
//
// Passes for one vector:
//   records  one floating block sum per 1024 weights (and the exact sums of
//            the exponential blocks of the multinomial scheme)
//   carries  one workgroup scans the block sums in the mode's arithmetic into
//            carries C_b, stored as binary64 values (exact for F64 and
//            NAIVE_F32, rounded at 2^-53 for the pairs of COMP_F32) and made
//            non-decreasing by a max-scan
//   emit     each block rebuilds its local prefix, adds C_b, maps to
//            r = n W_i / W, clamps into [r(C_b), r(C_{b+1})] and makes it
//            non-decreasing, and gives its last particle r(C_{b+1}); blocks
//            therefore agree at their boundaries although the block sum of
//            the records pass and the local scan round differently.  The
//            ancestors are then emitted by the code of the exact path.
// Ragged batches run all three steps in one workgroup per filter.
#include "pfr_kernels.h"

namespace pfr {

namespace {
#include "pfr_scan_common.h"

// ---------------------------------------------------------------- arithmetic
struct FF {  // double-float value hi + lo, |lo| <= ulp(hi) / 2
  float hi, lo;
};

template <int P>
struct FA;

template <>
struct FA<PREC_F64> {
  typedef double V;
  template <typename T>
  __device__ static V from(T w) { return (double)w; }
  __device__ static V from_value(double d) { return d; }
  __device__ static V zero() { return 0.0; }
  __device__ static V add(V a, V b) { return a + b; }
  __device__ static double value(V a) { return a; }
};

template <>
struct FA<PREC_NAIVE_F32> {
  typedef float V;
  template <typename T>
  __device__ static V from(T w) { return (float)w; }
  __device__ static V from_value(double d) { return (float)d; }  // exact: d came from a float
  __device__ static V zero() { return 0.0f; }
  __device__ static V add(V a, V b) { return a + b; }
  __device__ static double value(V a) { return (double)a; }
};

template <>
struct FA<PREC_COMP_F32> {
  typedef FF V;
  __device__ static V from(float w) { return FF{w, 0.0f}; }
  __device__ static V from(double w) {
    const float h = (float)w;
    return FF{h, (float)(w - (double)h)};
  }
  // splits a binary64 value (a pair rounded by value()) with relative error
  // below 2^-48
  __device__ static V from_value(double d) { return from(d); }
  __device__ static V zero() { return FF{0.0f, 0.0f}; }
  __device__ static V add(V a, V b) {
    const float s = a.hi + b.hi;
    const float bb = s - a.hi;
    float e = (a.hi - (s - bb)) + (b.hi - bb);  // s + e = a.hi + b.hi exactly
    e += a.lo + b.lo;
    const float h = s + e;
    return FF{h, e - (h - s)};
  }
  // hi + lo rounded once to binary64 (relative error 2^-53)
  __device__ static double value(V a) { return (double)a.hi + (double)a.lo; }
};

template <int P>
struct FAdd {
  template <typename V>
  __device__ __forceinline__ V operator()(V a, V b) const { return FA<P>::add(a, b); }
};

// r = n W_i / W in the mode's arithmetic, monotone in I, r(W) = n.
template <int P>
struct FRMap {
  double Wd, invW, Nd;
  __device__ double operator()(typename FA<P>::V I) const {
    if constexpr (P == PREC_NAIVE_F32) {
      const float Wf = (float)Wd;
      if (I >= Wf) return Nd;
      const float q = I / Wf;
      const float r = (float)Nd * q;
      const double rd = (double)r;
      return rd < Nd ? rd : Nd;
    } else {
      const double Id = FA<P>::value(I);
      if (Id >= Wd) return Nd;
      const double r = Nd * (Id * invW);
      return r < Nd ? r : Nd;
    }
  }
};

template <int P>
__device__ __forceinline__ FRMap<P> make_frmap(double W, int64_t n) {
  FRMap<P> m;
  m.Wd = W;
  m.invW = 1.0 / W;
  m.Nd = (double)n;
  return m;
}

// ---------------------------------------------------------------- workgroup
// Exclusive scan (thread order) of x with op; *total gets the reduction.
// Slot holds at least kNW values of V.
template <typename V, typename Op>
__device__ V wg_exclusive_op(V x, Op op, V zero, V* slot, V* total) {
  const int wave = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  const V incl = wave_inclusive_scan(x, op);
  V excl = shfl(incl, lane > 0 ? lane - 1 : 0);
  __syncthreads();
  if (lane == kWave - 1) slot[wave] = incl;
  __syncthreads();
  V before = slot[0];
  for (int w2 = 1; w2 < wave; ++w2) before = op(before, slot[w2]);
  V tot = slot[0];
#pragma unroll
  for (int w2 = 1; w2 < kNW; ++w2) tot = op(tot, slot[w2]);
  __syncthreads();
  *total = tot;
  if (wave == 0) return lane == 0 ? zero : excl;
  return lane == 0 ? before : op(before, excl);
}

// Exclusive max-scan of non-negative binary64 values (0 for thread 0); the
// bit patterns of non-negative doubles are ordered like the values.
__device__ double wg_exclusive_max(double x, WgScratch* s) {
  const int wave = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  const uint64_t incl = wave_inclusive_scan((uint64_t)__double_as_longlong(x), OpMax());
  uint64_t excl = shfl(incl, lane > 0 ? lane - 1 : 0);
  if (lane == 0) excl = 0;
  __syncthreads();
  if (lane == kWave - 1) s->u[wave] = incl;
  __syncthreads();
  for (int w2 = 0; w2 < wave; ++w2) excl = excl > s->u[w2] ? excl : s->u[w2];
  __syncthreads();
  return __longlong_as_double((long long)excl);
}

// ---------------------------------------------------------------- records
// Block sum in the mode's arithmetic as a binary64 value; -1 marks a block
// holding a negative or non-finite weight.
template <typename T, int P>
__device__ double fblock_sum(const T* __restrict__ w, int64_t n, int64_t base, WgScratch* s) {
  typedef typename FA<P>::V V;
  T x[kPer];
  load4(w, n, base, x);
  uint32_t bad = 0;
  V acc = FA<P>::zero();
#pragma unroll
  for (int v = 0; v < kPer; ++v) {
    if (!weight_ok(x[v])) bad = 1;
    acc = FA<P>::add(acc, FA<P>::from(x[v]));
  }
  bad = wg_reduce(bad, OpOr(), (uint32_t*)s->i);
  const V sum = wg_reduce(acc, FAdd<P>(), (V*)s->v);
  return bad ? -1.0 : FA<P>::value(sum);
}

// ---------------------------------------------------------------- carries
// From nb block sums: carries C[0..nb] (C[nb] = total W), non-decreasing, and
// the status of the call.
template <int P, typename SumPtr, typename CPtr>
__device__ uint32_t fcarries(uint32_t nb, SumPtr sums, CPtr C, WgScratch* s) {
  typedef typename FA<P>::V V;
  const int tid = (int)threadIdx.x;
  uint32_t bad = 0;
  V carry = FA<P>::zero();
  double floor_c = 0.0;  // largest carry written so far
  for (uint32_t base = 0; base < nb; base += kBlock) {
    V v[kPer];
    V mine = FA<P>::zero();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t b = base + (uint32_t)tid * kPer + k;
      const double d = b < nb ? sums[b] : 0.0;
      if (d < 0.0) bad = 1;
      v[k] = FA<P>::from_value(d < 0.0 ? 0.0 : d);
      mine = FA<P>::add(mine, v[k]);
    }
    V tot;
    const V excl = wg_exclusive_op(mine, FAdd<P>(), FA<P>::zero(), (V*)s->v, &tot);
    V run = FA<P>::add(carry, excl);
    double c[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      c[k] = FA<P>::value(run);
      run = FA<P>::add(run, v[k]);
    }
    // non-decreasing across threads and chunks
    const double m = wg_exclusive_max(c[kPer - 1], s);
    double hi = floor_c > m ? floor_c : m;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      hi = c[k] > hi ? c[k] : hi;
      const uint32_t b = base + (uint32_t)tid * kPer + k;
      if (b < nb) C[b] = hi;
    }
    carry = FA<P>::add(carry, tot);
    // the next chunk starts at or above every carry of this one
    const double last = wg_reduce(hi, OpMax(), (double*)s->v);
    floor_c = last;
  }
  bad = wg_reduce(bad, OpOr(), (uint32_t*)s->i);
  double W = FA<P>::value(carry);
  W = W > floor_c ? W : floor_c;
  if (tid == 0) C[nb] = W;
  __syncthreads();
  uint32_t status = bad ? FLAG_BAD_WEIGHTS : 0u;
  if (!bad && W == 0.0) status |= FLAG_ZERO_TOTAL;
  if (!bad && !(W < __builtin_huge_val())) status |= FLAG_BAD_WEIGHTS;  // overflowed total
  return status;
}

// ---------------------------------------------------------------- emit
// r of the thread's 4 particles of block b in the mode's arithmetic: local
// prefix plus C_b, mapped, clamped into [r(C_b), r(C_{b+1})], made
// non-decreasing, and r(C_{b+1}) for the block's last particle.
template <typename T, int P>
__device__ void fblock_r(const T* __restrict__ w, int64_t n, uint32_t b, double Cb, double Cb1,
                         const FRMap<P>& rm, double r_lo, double r_hi, double (&r)[kPer],
                         WgScratch* s) {
  typedef typename FA<P>::V V;
  const int tid = (int)threadIdx.x;
  const int64_t P0 = (int64_t)b * kBlock;
  const int cnt = (int)min((int64_t)kBlock, n - P0);
  T x[kPer];
  load4(w, n, P0, x);
  V acc[kPer];
  V run = FA<P>::zero();
#pragma unroll
  for (int v = 0; v < kPer; ++v) {
    run = FA<P>::add(run, FA<P>::from(x[v]));
    acc[v] = run;
  }
  V tot;
  const V off = wg_exclusive_op(run, FAdd<P>(), FA<P>::zero(), (V*)s->v, &tot);
  const V base = FA<P>::add(FA<P>::from_value(Cb), off);
#pragma unroll
  for (int v = 0; v < kPer; ++v) {
    double t = rm(FA<P>::add(base, acc[v]));
    t = t < r_lo ? r_lo : t;
    r[v] = t > r_hi ? r_hi : t;
  }
  const double ex = wg_exclusive_max(r[kPer - 1], s);
#pragma unroll
  for (int v = 0; v < kPer; ++v) {
    r[v] = r[v] > ex ? r[v] : ex;
    if (tid * kPer + v >= cnt - 1) r[v] = r_hi;  // block end and past the vector's end
  }
}

template <typename T, int P, int SCHEME, typename CEPtr>
__device__ void femit_block(const T* __restrict__ w, int64_t n, uint32_t b, double Cb, double Cb1,
                            const FRMap<P>& rm, Key key, uint32_t filter, uint32_t offset,
                            CEPtr CE, uint32_t nbe, int32_t* __restrict__ a_out, EmitLds* L,
                            WgScratch* s) {
  typedef typename FA<P>::V V;
  const int tid = (int)threadIdx.x;
  const int64_t P0 = (int64_t)b * kBlock;
  const int cnt = (int)min((int64_t)kBlock, n - P0);
  const double r_lo = rm(FA<P>::from_value(Cb));
  const double r_hi = rm(FA<P>::from_value(Cb1));
  double r[kPer];
  fblock_r<T, P>(w, n, b, Cb, Cb1, rm, r_lo, r_hi, r, s);
  if (SCHEME == SCHEME_MULTINOMIAL) {
#pragma unroll
    for (int v = 0; v < kPer; ++v) L->mu.r[tid * kPer + v] = r[v];
    __syncthreads();
    emit_multinomial(L->mu.r, cnt, r_lo, r_hi, P0 + cnt == n, n, P0, key, filter, offset, CE, nbe,
                     a_out, s);
  } else {
    const uint32_t u_sys =
        SCHEME == SCHEME_SYSTEMATIC ? draw(key, 0, DOM_STRATA, 0, filter, offset).x : 0u;
    emit_strata<SCHEME == SCHEME_SYSTEMATIC, P == PREC_NAIVE_F32>(
        r, cnt, r_lo, r_hi, n, P0, key, filter, offset, u_sys, a_out, &L->st, s);
  }
}

// ---------------------------------------------------------------- kernels
template <typename T, int P, bool MULTI>
__global__ __launch_bounds__(kT) void k_fscan_records(const T* __restrict__ w, int64_t n,
                                                      uint32_t nb, Key key, uint32_t offset,
                                                      uint32_t filter, double* __restrict__ sums,
                                                      uint64_t* __restrict__ esums) {
  offset = counter_offset(key, offset);
  __shared__ WgScratch s;
  if (blockIdx.x < nb) {
    const double d = fblock_sum<T, P>(w, n, (int64_t)blockIdx.x * kBlock, &s);
    if (threadIdx.x == 0) sums[blockIdx.x] = d;
  } else if (MULTI) {
    const uint32_t b = blockIdx.x - nb;
    uint64_t q[kPer];
    exp_values(key, filter, offset, n, b, q);
    const uint64_t sum = wg_reduce(q[0] + q[1] + q[2] + q[3], OpAdd(), s.u);
    if (threadIdx.x == 0) esums[b] = sum;
  }
}

template <int P, bool MULTI>
__global__ __launch_bounds__(kT) void k_fscan_carries(uint32_t nb, uint32_t nbe,
                                                      ScanHeader* __restrict__ hdr,
                                                      const double* __restrict__ sums,
                                                      const uint64_t* __restrict__ esums,
                                                      double* __restrict__ C,
                                                      u128* __restrict__ CE) {
  __shared__ WgScratch s;
  const uint32_t status = fcarries<P>(nb, sums, C, &s);
  if (MULTI) exp_carries(nbe, esums, CE, &s);
  if (threadIdx.x == 0) {
    hdr->status = status;
    hdr->W = C[nb];
  }
}

template <typename T, int P, int SCHEME>
__global__ __launch_bounds__(kT) void k_fscan_emit(const T* __restrict__ w, int64_t n,
                                                   uint32_t nbe, Key key, uint32_t offset,
                                                   uint32_t filter,
                                                   const ScanHeader* __restrict__ hdr,
                                                   const double* __restrict__ C,
                                                   const u128* __restrict__ CE,
                                                   int32_t* __restrict__ a,
                                                   uint32_t* __restrict__ flags) {
  offset = counter_offset(key, offset);
  __shared__ EmitLds L;
  __shared__ WgScratch s;
  const uint32_t b = blockIdx.x;
  const uint32_t status = hdr->status;
  if (flags && b == 0 && threadIdx.x == 0 && status) atomicOr(flags, status);
  if (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    const int64_t P0 = (int64_t)b * kBlock;
    for (int64_t i = P0 + threadIdx.x; i < min(P0 + kBlock, n); i += kT) a[i] = (int32_t)i;
    return;
  }
  const FRMap<P> rm = make_frmap<P>(hdr->W, n);
  femit_block<T, P, SCHEME>(w, n, b, C[b], C[b + 1], rm, key, filter, offset, CE, nbe, a, &L,
                            &s);
}

__global__ void k_fscan_status(const ScanHeader* __restrict__ hdr, uint32_t* __restrict__ flags) {
  if (hdr->status) atomicOr(flags, hdr->status);
}

// The scaled prefix r of the mode, written out (binary64) instead of
// resampling: what the emission compares its points against.
template <typename T, int P>
__global__ __launch_bounds__(kT) void k_fscan_r(const T* __restrict__ w, int64_t n,
                                                const ScanHeader* __restrict__ hdr,
                                                const double* __restrict__ C,
                                                double* __restrict__ r_out) {
  __shared__ WgScratch s;
  if (hdr->status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) return;
  const uint32_t b = blockIdx.x;
  const FRMap<P> rm = make_frmap<P>(hdr->W, n);
  const double r_lo = rm(FA<P>::from_value(C[b]));
  const double r_hi = rm(FA<P>::from_value(C[b + 1]));
  double r[kPer];
  fblock_r<T, P>(w, n, b, C[b], C[b + 1], rm, r_lo, r_hi, r, &s);
#pragma unroll
  for (int v = 0; v < kPer; ++v) {
    const int64_t i = (int64_t)b * kBlock + threadIdx.x * kPer + v;
    if (i < n) r_out[i] = r[v];
  }
}

constexpr int kFBatchMaxBlocks = 256;  // segments up to 2^18 particles

struct FBatchLds {
  double sums[kFBatchMaxBlocks];
  double C[kFBatchMaxBlocks + 1];
  uint64_t esums[kFBatchMaxBlocks];
  u128 CE[kFBatchMaxBlocks + 1];
};

template <typename T, int P, int SCHEME>
__global__ __launch_bounds__(kT) void k_fscan_batched(const T* __restrict__ w, int64_t n_total,
                                                      const int64_t* __restrict__ offsets,
                                                      uint32_t n_filters, Key key,
                                                      uint32_t offset, uint32_t filter_base,
                                                      int32_t* __restrict__ a,
                                                      uint32_t* __restrict__ flags) {
  offset = counter_offset(key, offset);
  __shared__ FBatchLds B;
  __shared__ EmitLds L;
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
  if (nbe > kFBatchMaxBlocks) {  // segment too long for this path: identity + flag
    for (int64_t i = tid; i < n; i += kT) as[i] = (int32_t)i;
    if (tid == 0 && flags) atomicOr(flags, FLAG_BAD_COUNTS);
    return;
  }
  for (uint32_t b = 0; b < nb; ++b) {
    const double d = fblock_sum<T, P>(ws, n, (int64_t)b * kBlock, &s);
    if (tid == 0) B.sums[b] = d;
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
  const uint32_t status = fcarries<P>(nb, (const double*)B.sums, (double*)B.C, &s);
  if (SCHEME == SCHEME_MULTINOMIAL) exp_carries(nbe, (const uint64_t*)B.esums, (u128*)B.CE, &s);
  if (flags && tid == 0 && status) atomicOr(flags, status);
  if (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    for (int64_t i = tid; i < n; i += kT) as[i] = (int32_t)i;
    return;
  }
  const FRMap<P> rm = make_frmap<P>(B.C[nb], n);
  for (uint32_t b = 0; b < nb; ++b) {
    femit_block<T, P, SCHEME>(ws, n, b, B.C[b], B.C[b + 1], rm, key, filt, offset,
                              (const u128*)B.CE, nbe, as, &L, &s);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launchers
template <typename T, int P, int SCHEME>
hipError_t launch_fscan_t(const void* wv, int64_t n, Key key, uint32_t offset, uint32_t filter,
                          int32_t* a, void* ws, uint32_t* flags, hipStream_t stream) {
  const T* w = (const T*)wv;
  constexpr bool multi = SCHEME == SCHEME_MULTINOMIAL;
  const ScanLayout L = scan_layout(n, multi);
  char* base = (char*)ws;
  ScanHeader* hdr = (ScanHeader*)base;
  double* sums = (double*)(base + L.recs);
  double* C = (double*)(base + L.carries);
  uint64_t* esums = (uint64_t*)(base + L.erecs);
  u128* CE = (u128*)(base + L.ecarries);
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  const uint32_t nbe = multi ? (uint32_t)((n + 1 + kBlock - 1) / kBlock) : 0u;
  hipLaunchKernelGGL((k_fscan_records<T, P, multi>), dim3(nb + nbe), dim3(kT), 0, stream, w, n,
                     nb, key, offset, filter, sums, esums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fscan_carries<P, multi>), dim3(1), dim3(kT), 0, stream, nb, nbe, hdr, sums,
                     esums, C, CE);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fscan_emit<T, P, SCHEME>), dim3(nb), dim3(kT), 0, stream, w, n, nbe, key,
                     offset, filter, hdr, C, CE, a, flags);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t fscan_scheme(int scheme, const void* w, int64_t n, Key key, uint32_t offset,
                        uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                        hipStream_t stream) {
  switch (scheme) {
    case SCHEME_MULTINOMIAL:
      return launch_fscan_t<T, P, SCHEME_MULTINOMIAL>(w, n, key, offset, filter, a, ws, flags,
                                                      stream);
    case SCHEME_STRATIFIED:
      return launch_fscan_t<T, P, SCHEME_STRATIFIED>(w, n, key, offset, filter, a, ws, flags,
                                                     stream);
    default:
      return launch_fscan_t<T, P, SCHEME_SYSTEMATIC>(w, n, key, offset, filter, a, ws, flags,
                                                     stream);
  }
}

template <typename T>
hipError_t fscan_prec(int scheme, int prec, const void* w, int64_t n, Key key, uint32_t offset,
                      uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                      hipStream_t stream) {
  switch (prec) {
    case PREC_F64:
      return fscan_scheme<T, PREC_F64>(scheme, w, n, key, offset, filter, a, ws, flags, stream);
    case PREC_COMP_F32:
      return fscan_scheme<T, PREC_COMP_F32>(scheme, w, n, key, offset, filter, a, ws, flags,
                                            stream);
    default:
      return fscan_scheme<T, PREC_NAIVE_F32>(scheme, w, n, key, offset, filter, a, ws, flags,
                                             stream);
  }
}

template <typename T, int P>
hipError_t fbatched_scheme(int scheme, const void* w, int64_t n_total, const int64_t* offsets,
                           uint32_t n_filters, Key key, uint32_t offset, uint32_t filter_base,
                           int32_t* a, uint32_t* flags, hipStream_t stream) {
  const T* wt = (const T*)w;
  switch (scheme) {
    case SCHEME_MULTINOMIAL:
      hipLaunchKernelGGL((k_fscan_batched<T, P, SCHEME_MULTINOMIAL>), dim3(n_filters), dim3(kT), 0,
                         stream, wt, n_total, offsets, n_filters, key, offset, filter_base, a,
                         flags);
      break;
    case SCHEME_STRATIFIED:
      hipLaunchKernelGGL((k_fscan_batched<T, P, SCHEME_STRATIFIED>), dim3(n_filters), dim3(kT), 0,
                         stream, wt, n_total, offsets, n_filters, key, offset, filter_base, a,
                         flags);
      break;
    default:
      hipLaunchKernelGGL((k_fscan_batched<T, P, SCHEME_SYSTEMATIC>), dim3(n_filters), dim3(kT), 0,
                         stream, wt, n_total, offsets, n_filters, key, offset, filter_base, a,
                         flags);
      break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t fbatched_prec(int scheme, int prec, const void* w, int64_t n_total,
                         const int64_t* offsets, uint32_t n_filters, Key key, uint32_t offset,
                         uint32_t filter_base, int32_t* a, uint32_t* flags, hipStream_t stream) {
  switch (prec) {
    case PREC_F64:
      return fbatched_scheme<T, PREC_F64>(scheme, w, n_total, offsets, n_filters, key, offset,
                                          filter_base, a, flags, stream);
    case PREC_COMP_F32:
      return fbatched_scheme<T, PREC_COMP_F32>(scheme, w, n_total, offsets, n_filters, key, offset,
                                               filter_base, a, flags, stream);
    default:
      return fbatched_scheme<T, PREC_NAIVE_F32>(scheme, w, n_total, offsets, n_filters, key,
                                                offset, filter_base, a, flags, stream);
  }
}

template <typename T, int P>
hipError_t launch_fscan_r_t(const T* w, int64_t n, double* r, void* ws, uint32_t* flags,
                            hipStream_t stream) {
  const ScanLayout L = scan_layout(n, false);
  char* base = (char*)ws;
  ScanHeader* hdr = (ScanHeader*)base;
  double* sums = (double*)(base + L.recs);
  double* C = (double*)(base + L.carries);
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_fscan_records<T, P, false>), dim3(nb), dim3(kT), 0, stream, w, n, nb,
                     Key{0, 0, nullptr}, 0u, 0u, sums, (uint64_t*)nullptr);
  hipLaunchKernelGGL((k_fscan_carries<P, false>), dim3(1), dim3(kT), 0, stream, nb, 0u, hdr, sums,
                     (const uint64_t*)nullptr, C, (u128*)nullptr);
  hipLaunchKernelGGL((k_fscan_r<T, P>), dim3(nb), dim3(kT), 0, stream, w, n, hdr, C, r);
  if (flags) hipLaunchKernelGGL(k_fscan_status, dim3(1), dim3(1), 0, stream, hdr, flags);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fscan_r_p(int prec, const T* w, int64_t n, double* r, void* ws, uint32_t* flags,
                            hipStream_t stream) {
  switch (prec) {
    case PREC_F64: return launch_fscan_r_t<T, PREC_F64>(w, n, r, ws, flags, stream);
    case PREC_COMP_F32: return launch_fscan_r_t<T, PREC_COMP_F32>(w, n, r, ws, flags, stream);
    default: return launch_fscan_r_t<T, PREC_NAIVE_F32>(w, n, r, ws, flags, stream);
  }
}

}  // namespace

hipError_t launch_fscan_r(int prec, bool f64, const void* w, int64_t n, double* r, void* ws,
                          uint32_t* flags, hipStream_t stream) {
  return f64 ? launch_fscan_r_p<double>(prec, (const double*)w, n, r, ws, flags, stream)
             : launch_fscan_r_p<float>(prec, (const float*)w, n, r, ws, flags, stream);
}

hipError_t launch_fscan(int scheme, int prec, bool f64, const void* w, int64_t n, Key key,
                        uint32_t offset, uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                        hipStream_t stream) {
  return f64 ? fscan_prec<double>(scheme, prec, w, n, key, offset, filter, a, ws, flags, stream)
             : fscan_prec<float>(scheme, prec, w, n, key, offset, filter, a, ws, flags, stream);
}

hipError_t launch_fscan_batched(int scheme, int prec, bool f64, const void* w, int64_t n_total,
                                const int64_t* offsets, uint32_t n_filters, Key key,
                                uint32_t offset, uint32_t filter_base, int32_t* a,
                                uint32_t* flags, hipStream_t stream) {
  return f64 ? fbatched_prec<double>(scheme, prec, w, n_total, offsets, n_filters, key, offset,
                                     filter_base, a, flags, stream)
             : fbatched_prec<float>(scheme, prec, w, n_total, offsets, n_filters, key, offset,
                                    filter_base, a, flags, stream);
}

}  // namespace pfr
