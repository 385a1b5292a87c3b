// pfr_filter.hip -- the bootstrap particle filter of Code 1 for a 1-D
// linear-Gaussian state-space model, batched over F filters of n particles:
//   x_0 ~ N(0, s0^2),   x_t = phi x_{t-1} + q e_t,   y_t = x_t + r v_t.
// The bootstrap choice (section 1) takes the transition density as K_t and
// the observation density as G_t.  Step t of Code 1 runs, for every filter:
// ancestors from the previous weights, the permutation that makes in-place
// propagation safe (section 2.3, eq. predicate), the in-place copy
// x_i <- x_{c_i} for c_i != i, propagation and weighting.  The log-weights are
// shifted by their maximum in binary64 before exponentiation (the
// renormalisation identity of appendix E), the weights handed to the next
// resampling are binary32 values in (0, 1] with maximum exactly 1, and
// log Z accumulates max + log(mean exp(lw - max)) in binary64.
//
// The step index t lives in device memory; the last kernel of a step advances
// it, so one captured graph of a step can be replayed for t = 1..T.
//
// Random numbers: the initial state of particle i of filter f takes Philox
// counter (i, INIT<<28, f, offset), its propagation noise at step t the counter
// (i, NOISE<<28 | t, f, offset); a standard normal is formed from words 0 and
// 1 by the Box-Muller transform with u1 = (x0 + 1) 2^-32 and u2 = x1 2^-32.
#include "pfr_kernels.h"

namespace pfr {

namespace {

constexpr int kFT = 512;  // threads per filter workgroup

__device__ __forceinline__ double normal_bm(uint32_t x0, uint32_t x1) {
  const double u1 = ((double)x0 + 1.0) * 0x1p-32;
  const double u2 = (double)x1 * 0x1p-32;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

__device__ double block_max(double v, double* slot) {
  const int wave = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  v = wave_reduce(v, OpMax());
  __syncthreads();
  if (lane == 0) slot[wave] = v;
  __syncthreads();
  double t = slot[0];
  for (int w2 = 1; w2 < kFT / kWave; ++w2) t = t > slot[w2] ? t : slot[w2];
  __syncthreads();
  return t;
}

__device__ double block_sum(double v, double* slot) {
  const int wave = (int)threadIdx.x / kWave, lane = (int)threadIdx.x % kWave;
  v = wave_reduce(v, OpAdd());
  __syncthreads();
  if (lane == 0) slot[wave] = v;
  __syncthreads();
  double t = slot[0];
  for (int w2 = 1; w2 < kFT / kWave; ++w2) t += slot[w2];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kFT) void k_lg_init(int32_t n_filters, int32_t n, double s0, Key key,
                                                 uint32_t offset, uint32_t filter_base,
                                                 float* __restrict__ x, float* __restrict__ w,
                                                 double* __restrict__ logz,
                                                 int32_t* __restrict__ B_dev,
                                                 uint32_t* __restrict__ t_dev,
                                                 int64_t* __restrict__ offsets) {
  const int64_t total = (int64_t)n_filters * n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += stride) {
    const int32_t f = (int32_t)(g / n), i = (int32_t)(g - (int64_t)f * n);
    const uint4 u = draw(key, (uint32_t)i, DOM_INIT, 0, filter_base + (uint32_t)f, offset);
    x[g] = (float)(s0 * normal_bm(u.x, u.y));
    w[g] = 1.0f;
  }
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= n_filters; g += stride) {
    offsets[g] = g * n;
    if (g < n_filters) {
      logz[g] = 0.0;
      B_dev[g] = 1;
    }
    if (g == 0) *t_dev = 1u;
  }
}

// One workgroup per filter: copy, propagate, weight, log Z and the Metropolis
// step count for the next resampling, B = ceil(log eps / log(1 - beta)) with
// beta = mean(w) (the shifted weights have maximum 1).
// inv_r = 1 / r in binary64: the scaled residual is (y - x) * inv_r, one
// multiply where a division would cost a dozen VALU instructions (it may
// differ from (y - x) / r in the last bit).
__global__ __launch_bounds__(kFT) void k_lg_move(int32_t n, double phi, double q, double inv_r,
                                                 double log_norm, double log_eps,
                                                 const double* __restrict__ y, int32_t T,
                                                 const uint32_t* __restrict__ t_dev, Key key,
                                                 uint32_t offset, uint32_t filter_base,
                                                 const int32_t* __restrict__ c,
                                                 float* __restrict__ x, float* __restrict__ w,
                                                 double* __restrict__ logz,
                                                 int32_t* __restrict__ B_dev,
                                                 uint32_t* __restrict__ flags) {
  __shared__ double slot[kFT / kWave];
  const uint32_t f = blockIdx.x;
  const int64_t base = (int64_t)f * n;
  const uint32_t t = *t_dev;
  if (t < 1u || t > (uint32_t)T) {  // no observation for this step
    if (flags && f == 0 && threadIdx.x == 0) atomicOr(flags, FLAG_BAD_STEP);
    return;
  }
  const double yt = y[t - 1];
  const int tid = (int)threadIdx.x;
  // in-place copy: slots that are read satisfy c_j = j and are never written
  for (int32_t i = tid; i < n; i += kFT) {
    const int32_t ci = c[base + i];
    if (ci != i) x[base + i] = x[base + ci];
  }
  __syncthreads();
  double mx = -__builtin_huge_val();
  for (int32_t i = tid; i < n; i += kFT) {
    const uint4 u = draw(key, (uint32_t)i, DOM_NOISE, t, filter_base + f, offset);
    const float xn = (float)(phi * (double)x[base + i] + q * normal_bm(u.x, u.y));
    x[base + i] = xn;
    const double d = (yt - (double)xn) * inv_r;
    const double lw = -0.5 * d * d + log_norm;
    mx = lw > mx ? lw : mx;
  }
  mx = block_max(mx, slot);
  double sum = 0.0;
  for (int32_t i = tid; i < n; i += kFT) {
    const double d = (yt - (double)x[base + i]) * inv_r;
    const double e = exp((-0.5 * d * d + log_norm) - mx);
    w[base + i] = (float)e;
    sum += e;
  }
  sum = block_sum(sum, slot);
  if (tid == 0) {
    const double beta = sum / (double)n;
    logz[f] += mx + log(beta);
    double B = beta >= 1.0 ? 1.0 : ceil(log_eps / log1p(-beta));
    B = B < 1.0 ? 1.0 : (B > 65536.0 ? 65536.0 : B);
    B_dev[f] = (int32_t)B;
  }
}

__global__ void k_lg_tick(uint32_t* __restrict__ t_dev) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *t_dev += 1u;
}

}  // namespace

hipError_t launch_lgssm_init(int32_t n_filters, int32_t n, double s0, Key key, uint32_t offset,
                             uint32_t filter_base, float* x, float* w, double* logz,
                             int32_t* B_dev, uint32_t* t_dev, int64_t* offsets,
                             hipStream_t stream) {
  const int64_t total = (int64_t)n_filters * n;
  int64_t grid = (total + kFT - 1) / kFT;
  if (grid < 1) grid = 1;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(k_lg_init, dim3((uint32_t)grid), dim3(kFT), 0, stream, n_filters, n, s0, key,
                     offset, filter_base, x, w, logz, B_dev, t_dev, offsets);
  return hipGetLastError();
}

hipError_t launch_lgssm_move(int32_t n_filters, int32_t n, double phi, double q, double r,
                             double log_eps, const double* y, int32_t T, uint32_t* t_dev,
                             Key key, uint32_t offset, uint32_t filter_base, const int32_t* c,
                             float* x, float* w, double* logz, int32_t* B_dev, uint32_t* flags,
                             hipStream_t stream) {
  const double log_norm = -log(r) - 0.5 * log(6.283185307179586);
  hipLaunchKernelGGL(k_lg_move, dim3((uint32_t)n_filters), dim3(kFT), 0, stream, n, phi, q,
                     1.0 / r, log_norm, log_eps, y, T, t_dev, key, offset, filter_base, c, x, w,
                     logz, B_dev, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lg_tick, dim3(1), dim3(64), 0, stream, t_dev);
  return hipGetLastError();
}

}  // namespace pfr
