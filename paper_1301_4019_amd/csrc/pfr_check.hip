// pfr_check.hip -- optional checks of the preconditions the boundary states but
// the hot path does not test: finite, non-negative weights for the resamplers
// without a collective pass (Metropolis and rejection, Codes 2 and 3), a
// w_max that bounds the weights (rejection, section 2.2), and a
// non-decreasing ancestry where the caller passes sorted_hint (Codes 10 and
// 12).  Each check is one pass over the input; a violation is OR-ed into the
// caller's flags and into a word the library keeps per GPU.
#include <mutex>

#include "pfr_kernels.h"

namespace pfr {

namespace {

// Violations recorded while the checks are on, one word per GPU at that GPU's
// own address.  Host code takes the address from hipGetSymbolAddress (once per
// device) and never uses the name as an address.
static __device__ uint32_t check_word;

constexpr int kMaxDevices = 64;
std::mutex g_word_mu;
uint32_t* g_word_dev[kMaxDevices];

hipError_t word_address(uint32_t** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_word_mu);
  if (!g_word_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(check_word));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_word_dev[dev] = (uint32_t*)p;
  }
  *out = g_word_dev[dev];
  return hipSuccess;
}

__device__ __forceinline__ void record(uint32_t f, uint32_t* __restrict__ word,
                                       uint32_t* __restrict__ flags) {
  f = wave_reduce(f, OpOr());
  if (lane_id() == 0 && f) {
    atomicOr(word, f);
    if (flags) atomicOr(flags, f);
  }
}

// Every weight finite and non-negative; with a bound, none above the bound of
// its segment (bound_dev[f] when given, else bound).
template <typename T>
__global__ __launch_bounds__(256) void k_check_weights(const T* __restrict__ w, int64_t n_total,
                                                       const int64_t* __restrict__ offsets,
                                                       uint32_t n_filters, int use_bound,
                                                       double bound,
                                                       const double* __restrict__ bound_dev,
                                                       uint32_t* __restrict__ word,
                                                       uint32_t* __restrict__ flags) {
  uint32_t f = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_total; g += stride) {
    const T v = w[g];
    if (!weight_ok(v)) {
      f |= FLAG_BAD_WEIGHTS;
    } else if (use_bound) {
      const double b =
          bound_dev ? bound_dev[offsets ? find_segment(offsets, n_filters, g) : 0u] : bound;
      if ((double)v > b) f |= FLAG_WMAX_BELOW;
    }
  }
  record(f, word, flags);
}

// a non-decreasing inside every segment (a step down across a segment start
// is allowed).
__global__ __launch_bounds__(256) void k_check_sorted(const int32_t* __restrict__ a,
                                                      int64_t n_total,
                                                      const int64_t* __restrict__ offsets,
                                                      uint32_t n_filters,
                                                      uint32_t* __restrict__ word,
                                                      uint32_t* __restrict__ flags) {
  uint32_t f = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; g < n_total; g += stride) {
    if (a[g] < a[g - 1]) {
      const bool first = offsets && offsets[find_segment(offsets, n_filters, g)] == g;
      if (!first) f |= FLAG_NOT_SORTED;
    }
  }
  record(f, word, flags);
}

unsigned check_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_check_weights(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                                uint32_t n_filters, bool use_bound, double bound,
                                const double* bound_dev, uint32_t* flags, hipStream_t stream) {
  uint32_t* word = nullptr;
  hipError_t e = word_address(&word);
  if (e != hipSuccess) return e;
  if (f64)
    hipLaunchKernelGGL(k_check_weights<double>, dim3(check_grid(n_total)), dim3(256), 0, stream,
                       (const double*)w, n_total, offsets, n_filters, use_bound ? 1 : 0, bound,
                       bound_dev, word, flags);
  else
    hipLaunchKernelGGL(k_check_weights<float>, dim3(check_grid(n_total)), dim3(256), 0, stream,
                       (const float*)w, n_total, offsets, n_filters, use_bound ? 1 : 0, bound,
                       bound_dev, word, flags);
  return hipGetLastError();
}

hipError_t launch_check_sorted(const int32_t* a, int64_t n_total, const int64_t* offsets,
                               uint32_t n_filters, uint32_t* flags, hipStream_t stream) {
  uint32_t* word = nullptr;
  hipError_t e = word_address(&word);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_check_sorted, dim3(check_grid(n_total)), dim3(256), 0, stream, a, n_total,
                     offsets, n_filters, word, flags);
  return hipGetLastError();
}

hipError_t take_check_word(hipStream_t stream, uint32_t* out) {
  uint32_t* word = nullptr;
  hipError_t e = word_address(&word);
  if (e != hipSuccess) return e;
  uint32_t v = 0;
  const uint32_t zero = 0;
  e = hipMemcpyAsync(&v, word, sizeof(v), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(word, &zero, sizeof(zero), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return e;
  *out = v;
  return hipSuccess;
}

}  // namespace pfr
