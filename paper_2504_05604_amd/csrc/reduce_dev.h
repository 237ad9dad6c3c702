// Device-side deterministic block reductions (header-only, included by kernels).
#pragma once

#include "internal.h"

namespace topo {

constexpr int kWave = 64;

template <bool MAX>
__device__ __forceinline__ double red_op(double a, double b) {
  return MAX ? fmax(a, b) : a + b;
}

template <bool MAX>
__device__ __forceinline__ double wave_reduce(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = red_op<MAX>(v, __shfl_down(v, off, kWave));
  return v;
}

// Reduces v[0..N) over the block; block results go to red.partials, and the last
// block to arrive sums them (fixed order) into out[0..N).  Must be called by every
// thread of the block.  blockDim.x <= 1024.
template <int N, bool MAX>
__device__ void block_reduce_finalize(double (&v)[N], const Reducer &red, double *out) {
  __shared__ double sh[N][16];
  __shared__ int is_last;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double t = wave_reduce<MAX>(v[k]);
    if (lane == 0) sh[k][wid] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double t = sh[k][0];
      for (int w = 1; w < nw; ++w) t = red_op<MAX>(t, sh[k][w]);
      red.partials[(size_t)blockIdx.x * kMaxRed + k] = t;
    }
    __threadfence();
    unsigned prev = atomicAdd(red.counter, 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  const volatile double *P = red.partials;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double t = MAX ? -INFINITY : 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x)
      t = red_op<MAX>(t, P[(size_t)b * kMaxRed + k]);
    t = wave_reduce<MAX>(t);
    __syncthreads();
    if (lane == 0) sh[k][wid] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = sh[k][0];
      for (int w = 1; w < nw; ++w) s = red_op<MAX>(s, sh[k][w]);
      out[k] = s;
    }
  }
  if (threadIdx.x == 0) atomicExch(red.counter, 0u);
}

}  // namespace topo
