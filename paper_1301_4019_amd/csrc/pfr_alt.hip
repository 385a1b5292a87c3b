// pfr_alt.hip -- the collective-free resamplers: Metropolis (Code 2 of the
// paper) and rejection (Code 3), one lane per particle on a counter-based
// Philox stream.
//
// Lane results depend only on (particle, step/trial, filter, offset) through
// the Philox counter, never on which lane or wave did the work, so every
// launch shape gives the same bits.
#include "pfr_kernels.h"

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
// Step s draws (j, u) from Philox counter (i, TRIAL<<28 | s, filter, offset)
// and moves to j when u * w_k <= w_j.  The proposals and their weight loads do
// not depend on the chain state, so groups of 4 steps issue their 4 Philox
// blocks and 4 gathers together and only the accept decisions run in order.
template <typename T>
__global__ __launch_bounds__(256) void k_metropolis(const T* __restrict__ w, int64_t n_total,
                                                    const int64_t* __restrict__ offsets,
                                                    uint32_t n_filters, int32_t B,
                                                    const int32_t* __restrict__ B_dev, Key key,
                                                    uint32_t offset, uint32_t filter_base,
                                                    int32_t* __restrict__ a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_total; g += stride) {
    const SegCtx c = seg_of(offsets, n_filters, n_total, g);
    const uint32_t i = (uint32_t)(g - c.base);
    const int32_t steps = B_dev ? B_dev[c.f] : B;
    const uint32_t filt = filter_base + c.f;
    const T* __restrict__ ws = w + c.base;
    uint32_t k = i;
    double wk = (double)ws[i];
    int32_t s = 0;
    for (; s + 4 <= steps; s += 4) {
      uint4 x[4];
      uint32_t j[4];
      double wj[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x[q] = draw(key, i, DOM_TRIAL, (uint32_t)(s + q), filt, offset);
        j[q] = index_draw(x[q].x, x[q].y, c.n);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) wj[q] = (double)ws[j[q]];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (accept_exact(u_accept(x[q].z), wk, wj[q])) {
          k = j[q];
          wk = wj[q];
        }
      }
    }
    for (; s < steps; ++s) {
      const uint4 x = draw(key, i, DOM_TRIAL, (uint32_t)s, filt, offset);
      const uint32_t j = index_draw(x.x, x.y, c.n);
      const double wj = (double)ws[j];
      if (accept_exact(u_accept(x.z), wk, wj)) {
        k = j;
        wk = wj;
      }
    }
    a[g] = (int32_t)k;
  }
}

// ------------------------------------------------------------------ rejection
// Particle i: trial 0 proposes j = i; trial t >= 1 proposes j from Philox
// counter (i, TRIAL<<28 | t, filter, offset); every trial takes its u from the
// same block.  The first trial with u * w_max <= w_j wins.  After max_trials
// rejections the particle keeps a_i = i and FLAG_TRIAL_CAP is raised.
//
// Scheduling (the variable task-length problem): each wave keeps 64 lanes
// busy by handing a finished lane the next particle of the wave's current
// chunk; chunks of kChunk particles come from a global counter (one atomic per
// chunk), so waves that draw short trial sequences take more chunks.  When no
// chunk is left, lanes still working try kSpec trials per pass (speculative:
// the later proposals are used only if the earlier ones reject), which
// shortens the dependent tail of the slowest particles.  The last wave to
// finish resets the two counters for the next launch.
constexpr uint32_t kChunk = 64;
constexpr int kSpec = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_rejection(const T* __restrict__ w, int64_t n_total,
                                                   const int64_t* __restrict__ offsets,
                                                   uint32_t n_filters, double w_max,
                                                   const double* __restrict__ w_max_dev,
                                                   uint32_t max_trials, Key key, uint32_t offset,
                                                   uint32_t filter_base, int32_t* __restrict__ a,
                                                   uint32_t* __restrict__ counters,
                                                   uint32_t* __restrict__ flags) {
  const uint32_t lane = lane_id();
  uint32_t q_next = 0, q_end = 0;  // wave-uniform chunk cursor
  bool exhausted = false;
  int64_t cur = -1;  // particle (global index) this lane works on
  uint32_t t = 0;    // next trial of that particle
  SegCtx c = {0, 0, 0};
  double wmax = w_max;
  uint32_t my_flags = 0;

  while (true) {
    // ---- hand out particles to free lanes
    uint64_t freem = ballot(cur < 0);
    while (freem != 0 && !exhausted) {
      if (q_next >= q_end) {
        uint32_t got = 0;
        if (lane == 0) got = atomicAdd(&counters[0], kChunk);
        got = readlane_u32(got, 0);
        if ((int64_t)got >= n_total) {
          exhausted = true;
          break;
        }
        q_next = got;
        q_end = (uint32_t)(((int64_t)got + kChunk) < n_total ? got + kChunk : n_total);
      }
      const uint32_t nfree = (uint32_t)__popcll(freem);
      const uint32_t avail = q_end - q_next;
      const uint32_t take = nfree < avail ? nfree : avail;
      const uint32_t rank = (uint32_t)__popcll(freem & lanemask_lt());
      if (cur < 0 && rank < take) {
        cur = (int64_t)(q_next + rank);
        t = 0;
        c = seg_of(offsets, n_filters, n_total, cur);
        wmax = w_max_dev ? w_max_dev[c.f] : w_max;
      }
      q_next += take;
      freem = ballot(cur < 0);
    }
    if (ballot(cur >= 0) == 0) break;

    if (cur >= 0) {
      const uint32_t i = (uint32_t)(cur - c.base);
      const uint32_t filt = filter_base + c.f;
      const T* __restrict__ ws = w + c.base;
      // trials [t, t + ntry)
      const uint32_t ntry = (exhausted && t > 0) ? (uint32_t)kSpec : 1u;
      uint4 x[kSpec];
      uint32_t j[kSpec];
      double wj[kSpec];
#pragma unroll
      for (int q = 0; q < kSpec; ++q) {
        if ((uint32_t)q < ntry) {
          x[q] = draw(key, i, DOM_TRIAL, t + q, filt, offset);
          j[q] = (t + q == 0) ? i : index_draw(x[q].x, x[q].y, c.n);
        }
      }
#pragma unroll
      for (int q = 0; q < kSpec; ++q)
        if ((uint32_t)q < ntry) wj[q] = (double)ws[j[q]];
      int done_q = -1;
#pragma unroll
      for (int q = kSpec - 1; q >= 0; --q) {
        if ((uint32_t)q < ntry && t + q < max_trials && accept_exact(u_accept(x[q].z), wmax, wj[q]))
          done_q = q;
      }
      if (done_q >= 0) {
        a[cur] = (int32_t)j[done_q];
        cur = -1;
      } else {
        t += ntry;
        if (t >= max_trials) {
          a[cur] = (int32_t)i;
          my_flags |= FLAG_TRIAL_CAP;
          cur = -1;
        }
      }
    }
  }

  if (flags) {
    const uint32_t wf = wave_reduce(my_flags, OpOr());
    if (lane == 0 && wf) atomicOr(flags, wf);
  }
  // the last wave out resets the counters for the next launch
  if (lane == 0) {
    __threadfence();
    const uint32_t nwaves = gridDim.x * (blockDim.x / kWave);
    const uint32_t prev = atomicAdd(&counters[1], 1u);
    if (prev == nwaves - 1) {
      counters[0] = 0;
      counters[1] = 0;
      __threadfence();
    }
  }
}

// ------------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_metropolis_t(const void* w, int64_t n_total, const int64_t* offsets,
                               uint32_t n_filters, int32_t B, const int32_t* B_dev, Key key,
                               uint32_t offset, uint32_t filter_base, int32_t* a,
                               hipStream_t stream) {
  const int threads = 256;
  int64_t blocks = (n_total + threads - 1) / threads;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  hipLaunchKernelGGL(k_metropolis<T>, dim3((unsigned)blocks), dim3(threads), 0, stream,
                     (const T*)w, n_total, offsets, n_filters, B, B_dev, key, offset, filter_base,
                     a);
  return hipGetLastError();
}

hipError_t launch_metropolis(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                             uint32_t n_filters, int32_t B, const int32_t* B_dev, Key key,
                             uint32_t offset, uint32_t filter_base, int32_t* a,
                             hipStream_t stream) {
  return f64 ? launch_metropolis_t<double>(w, n_total, offsets, n_filters, B, B_dev, key, offset,
                                           filter_base, a, stream)
             : launch_metropolis_t<float>(w, n_total, offsets, n_filters, B, B_dev, key, offset,
                                          filter_base, a, stream);
}

template <typename T>
hipError_t launch_rejection_t(const void* w, int64_t n_total, const int64_t* offsets,
                              uint32_t n_filters, double w_max, const double* w_max_dev,
                              uint32_t max_trials, Key key, uint32_t offset, uint32_t filter_base,
                              int32_t* a, uint32_t* counters, uint32_t* flags, int grid_blocks,
                              hipStream_t stream) {
  const int threads = 256;
  hipLaunchKernelGGL(k_rejection<T>, dim3((unsigned)grid_blocks), dim3(threads), 0, stream,
                     (const T*)w, n_total, offsets, n_filters, w_max, w_max_dev, max_trials, key,
                     offset, filter_base, a, counters, flags);
  return hipGetLastError();
}

hipError_t launch_rejection(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                            uint32_t n_filters, double w_max, const double* w_max_dev,
                            uint32_t max_trials, Key key, uint32_t offset, uint32_t filter_base,
                            int32_t* a, uint32_t* counters, uint32_t* flags, int grid_blocks,
                            hipStream_t stream) {
  return f64 ? launch_rejection_t<double>(w, n_total, offsets, n_filters, w_max, w_max_dev,
                                          max_trials, key, offset, filter_base, a, counters,
                                          flags, grid_blocks, stream)
             : launch_rejection_t<float>(w, n_total, offsets, n_filters, w_max, w_max_dev,
                                         max_trials, key, offset, filter_base, a, counters, flags,
                                         grid_blocks, stream);
}

}  // namespace pfr
