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

template <typename T>
__device__ __forceinline__ void metropolis_fetch(const T* __restrict__ ws, Key key, uint32_t i,
                                                 uint32_t filt, uint32_t offset, uint32_t n,
                                                 int32_t steps, int32_t m, MGroup& g) {
  uint32_t x[12];
  const int32_t left = steps - 4 * m;
  const int ncall = left >= 4 ? 3 : (3 * left + 3) / 4;
#pragma unroll
  for (int c3 = 0; c3 < 3; ++c3) {
    if (c3 < ncall) {
      const uint4 v = draw(key, i, DOM_TRIAL, (uint32_t)(3 * m + c3), filt, offset);
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

__device__ __forceinline__ void metropolis_accept(const MGroup& g, uint32_t& k, double& wk) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q < g.nq && accept_exact(u_accept(g.u[q]), wk, g.wj[q])) {
      k = g.j[q];
      wk = g.wj[q];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_metropolis(const T* __restrict__ w, int64_t n_total,
                                                    const int64_t* __restrict__ offsets,
                                                    uint32_t n_filters, int32_t B,
                                                    const int32_t* __restrict__ B_dev, Key key,
                                                    uint32_t offset, uint32_t filter_base,
                                                    int32_t* __restrict__ a) {
  offset = counter_offset(key, offset);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_total; g += stride) {
    const SegCtx c = seg_of(offsets, n_filters, n_total, g);
    const uint32_t i = (uint32_t)(g - c.base);
    const int32_t steps = B_dev ? B_dev[c.f] : B;
    const uint32_t filt = filter_base + c.f;
    const T* __restrict__ ws = w + c.base;
    uint32_t k = i;
    double wk = (double)ws[i];
    const int32_t groups = (steps + 3) / 4;
    MGroup ga, gb;
    if (groups > 0) metropolis_fetch(ws, key, i, filt, offset, c.n, steps, 0, ga);
    for (int32_t m = 0; m < groups; m += 2) {
      if (m + 1 < groups) metropolis_fetch(ws, key, i, filt, offset, c.n, steps, m + 1, gb);
      metropolis_accept(ga, k, wk);
      if (m + 2 < groups) metropolis_fetch(ws, key, i, filt, offset, c.n, steps, m + 2, ga);
      if (m + 1 < groups) metropolis_accept(gb, k, wk);
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

template <typename T>
__global__ __launch_bounds__(256) void k_rejection(const T* __restrict__ w, int64_t n_total,
                                                   const int64_t* __restrict__ offsets,
                                                   uint32_t n_filters, double w_max,
                                                   const double* __restrict__ w_max_dev,
                                                   uint32_t max_trials, Key key, uint32_t offset,
                                                   uint32_t filter_base, int32_t* __restrict__ a,
                                                   uint32_t* __restrict__ flags,
                                                   int64_t per_wave) {
  offset = counter_offset(key, offset);
  const uint32_t lane = lane_id();
  const int64_t gw = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int64_t r0 = gw * per_wave;
  const int64_t r1 = r0 + per_wave < n_total ? r0 + per_wave : n_total;
  int64_t next = r0;  // wave-uniform: next particle of the range to hand out
  int64_t cur = -1;   // particle (global index) this lane works on
  uint32_t t = 0;     // its next trial
  SegCtx c = {0, 0, 0};
  double wmax = w_max;
  uint32_t my_flags = 0;

  // main phase: one trial per lane per pass
  while (true) {
    const uint64_t freem = ballot(cur < 0);
    if (freem != 0 && next < r1) {
      const int64_t avail = r1 - next;
      const int64_t nfree = __popcll(freem);
      const int64_t take = nfree < avail ? nfree : avail;
      const int64_t rank = __popcll(freem & lanemask_lt());
      if (cur < 0 && rank < take) {
        cur = next + rank;
        t = 0;
        c = seg_of(offsets, n_filters, n_total, cur);
        wmax = w_max_dev ? w_max_dev[c.f] : w_max;
      }
      next += take;
    }
    if (next >= r1) break;
    if (cur >= 0) {
      const uint32_t i = (uint32_t)(cur - c.base);
      const uint4 x = draw(key, i, DOM_TRIAL, t, filter_base + c.f, offset);
      const uint32_t j = (t == 0) ? i : index_draw(x.x, x.y, c.n);
      const double wj = (double)w[c.base + j];
      if (accept_exact(u_accept(x.z), wmax, wj)) {
        a[cur] = (int32_t)j;
        cur = -1;
      } else if (++t >= max_trials) {
        a[cur] = (int32_t)i;
        my_flags |= FLAG_TRIAL_CAP;
        cur = -1;
      }
    }
  }

  // tail phase: the remaining particles share the wave's lanes
  while (true) {
    const uint64_t act = ballot(cur >= 0);
    if (act == 0) break;
    const int m = __popcll(act);
    const int slot = kWave / m;  // lanes per particle
    const int q = (int)lane / slot;
    const bool helper = q < m;
    const int owner = helper ? nth_set_bit(act, q) : (int)lane;
    const int64_t o_cur = shfl(cur, owner);
    const uint32_t o_t = shfl(t, owner);
    const int64_t o_base = shfl(c.base, owner);
    const uint32_t o_n = shfl(c.n, owner);
    const uint32_t o_f = shfl(c.f, owner);
    const double o_wmax = shfl(wmax, owner);
    const uint32_t tt = o_t + (lane - (uint32_t)(q * slot));
    bool acc = false;
    uint32_t jj = 0;
    if (helper && tt < max_trials) {
      const uint32_t i = (uint32_t)(o_cur - o_base);
      const uint4 x = draw(key, i, DOM_TRIAL, tt, filter_base + o_f, offset);
      jj = (tt == 0) ? i : index_draw(x.x, x.y, o_n);
      acc = accept_exact(u_accept(x.z), o_wmax, (double)w[o_base + jj]);
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
    if (cur >= 0) {
      if (g) {
        a[cur] = (int32_t)jsel;
        cur = -1;
      } else {
        t += (uint32_t)slot;
        if (t >= max_trials) {
          a[cur] = (int32_t)(cur - c.base);
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
                              int32_t* a, uint32_t* flags, int64_t per_wave, hipStream_t stream) {
  const int threads = 256;
  const int64_t waves = (n_total + per_wave - 1) / per_wave;
  const int64_t blocks = (waves + (threads / kWave) - 1) / (threads / kWave);
  hipLaunchKernelGGL(k_rejection<T>, dim3((unsigned)blocks), dim3(threads), 0, stream,
                     (const T*)w, n_total, offsets, n_filters, w_max, w_max_dev, max_trials, key,
                     offset, filter_base, a, flags, per_wave);
  return hipGetLastError();
}

// Particles per wave: enough waves to fill the chip (about 16 per CU), at
// least one particle per lane.
int64_t rejection_per_wave(int64_t n_total) {
  const int64_t target_waves = 256 * 16;
  int64_t p = (n_total + target_waves - 1) / target_waves;
  if (p < kWave) p = kWave;
  return p;
}

hipError_t launch_rejection(bool f64, const void* w, int64_t n_total, const int64_t* offsets,
                            uint32_t n_filters, double w_max, const double* w_max_dev,
                            uint32_t max_trials, Key key, uint32_t offset, uint32_t filter_base,
                            int32_t* a, uint32_t* flags, hipStream_t stream) {
  const int64_t pw = rejection_per_wave(n_total);
  return f64 ? launch_rejection_t<double>(w, n_total, offsets, n_filters, w_max, w_max_dev,
                                          max_trials, key, offset, filter_base, a, flags, pw,
                                          stream)
             : launch_rejection_t<float>(w, n_total, offsets, n_filters, w_max, w_max_dev,
                                         max_trials, key, offset, filter_base, a, flags, pw,
                                         stream);
}

}  // namespace pfr
