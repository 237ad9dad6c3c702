// Device-side deterministic reductions (header-only, included by kernels).
//
// A reducing kernel writes one partial per block (fixed-order tree inside the
// block) and a separate one-block finalize kernel sums the partials in block
// order.  No floating-point atomics and no device-scope fences: on a multi-XCD
// part a device-scope release fence in every block would write back the whole
// L2 of that XCD, which costs far more than one extra small launch.
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

// Block-reduces v[0..N) and stores the block's results at
// partials[slot * kMaxRed + k].  Every thread of the block must call it.
template <int N, bool MAX>
__device__ void block_reduce_store(double (&v)[N], double *partials, int slot) {
  __shared__ double sh[N][16];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double t = wave_reduce<MAX>(v[k]);
    if (lane == 0) sh[k][wid] = t;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    const int k = threadIdx.x;
    double t = sh[k][0];
    for (int w = 1; w < nw; ++w) t = red_op<MAX>(t, sh[k][w]);
    partials[(size_t)slot * kMaxRed + k] = t;
  }
}

// The sum a one-block finalize of 256 threads forms from value k of nparts
// partials, in its order (per-thread chains over slots t, t + 256, ..., the
// wave trees, the waves in order), returned to every thread of the calling
// block, which must have 256 threads and call it uniformly.
__device__ __forceinline__ double block_sum_partials(const double *partials, int nparts, int k) {
  __shared__ double sh[16];
  __shared__ double total;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  double t = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) t = t + partials[(size_t)b * kMaxRed + k];
  t = wave_reduce<false>(t);
  if (lane == 0) sh[wid] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = sh[0];
    for (int w = 1; w < nw; ++w) v = v + sh[w];
    total = v;
  }
  __syncthreads();
  return total;
}

__device__ __forceinline__ int linear_block() { return blockIdx.x + gridDim.x * blockIdx.y; }

// CG's stopping test (FIN_CG_CHECK, the iteration already counted) taken by
// every block of a 256-thread kernel from the n block partials of r.r; block 0
// stores r.r and raises cg_done.  Every block reaches the same decision, so a
// block that reads cg_done before block 0 raises it acts as one reading after.
__device__ __forceinline__ bool cg_stop_in_block(const double *parts, int n, Scalars *sc) {
  const double rr = block_sum_partials(parts, n, 0);
  const bool done = !(rr > sc->rtol2 * sc->ff) || sc->cg_iters >= sc->cg_max;
  if (linear_block() == 0 && threadIdx.x == 0) {
    sc->rr = rr;
    if (done) sc->cg_done = 1;
  }
  return done;
}

// The dispatcher hands the workgroups of a launch to the 8 XCDs round-robin by
// linear id, and each XCD has its own L2.  xcd_tile maps a workgroup to the tile
// it processes so that every XCD works through runs of kXcdRun consecutive
// tiles: neighbouring tiles (which read each other's halo) then mostly share
// an L2, while the runs of different XCDs stay interleaved across the domain
// (one contiguous slab per XCD measured slower).  The ragged end keeps the
// plain order.
constexpr int kXcds = 8;
constexpr int kXcdRun = 16;
__device__ __forceinline__ int xcd_tile(int id, int total) {
  constexpr int span = kXcds * kXcdRun;
  const int full = (total / span) * span;
  if (id >= full) return id;
  const int xcd = id % kXcds, q = id / kXcds;
  return ((q / kXcdRun) * kXcds + xcd) * kXcdRun + q % kXcdRun;
}

}  // namespace topo
