// Vector kernels of the conjugate-gradient loop and the Chebyshev smoother.
// All reductions are deterministic (block partials summed in a fixed order).
// Kernels of the CG loop take a `skip` flag (device int, may be NULL): once the
// loop has converged every later kernel of a replayed chunk returns at once.
#include "group_host.h"
#include "internal.h"
#include <algorithm>

#include "reduce_dev.h"

namespace topo {

namespace {
constexpr int kBs = 256;
inline unsigned nblocks(int64_t n, int per_thread = 1) {
  const int64_t m = (n + per_thread - 1) / per_thread;
  return (unsigned)((m + kBs - 1) / kBs);
}
// grid-stride reductions use a bounded grid so partial buffers stay small
inline unsigned red_blocks(int64_t n, const Reducer &red) {
  unsigned nb = nblocks(n, 4);
  if (nb > 1024u) nb = 1024u;
  if (nb < 1u) nb = 1u;
  return nb > (unsigned)red.max_blocks ? (unsigned)red.max_blocks : nb;
}
__device__ __forceinline__ bool skipped(const int *skip) { return skip != nullptr && *skip != 0; }
}  // namespace

__device__ __forceinline__ void zero_fixed_body(int64_t nnodes, const uint8_t *fixed, double *v) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nnodes) return;
  const uint8_t f = fixed[n];
  if (f & 1) v[3 * n + 0] = 0.0;
  if (f & 2) v[3 * n + 1] = 0.0;
  if (f & 4) v[3 * n + 2] = 0.0;
}
__global__ void zero_fixed_kernel(int64_t nnodes, const uint8_t *fixed, double *v) {
  zero_fixed_body(nnodes, fixed, v);
}
__global__ void zero_fixed_group_kernel(int64_t nnodes, GroupTab<const uint8_t *> fixed, GroupTab<double *> v) {
  zero_fixed_body(nnodes, fixed.v[blockIdx.z], v.v[blockIdx.z]);
}

hipError_t launch_zero_fixed(hipStream_t s, int64_t nnodes, const uint8_t *fixed, double *v) {
  zero_fixed_kernel<<<nblocks(nnodes), kBs, 0, s>>>(nnodes, fixed, v);
  return hipGetLastError();
}

__global__ void copy_masked_kernel(int64_t nnodes, const uint8_t *fixed, const double *in,
                                   double *out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nnodes) return;
  const uint8_t f = fixed[n];
#pragma unroll
  for (int c = 0; c < 3; ++c) out[3 * n + c] = ((f >> c) & 1) ? 0.0 : in[3 * n + c];
}

hipError_t launch_copy_masked(hipStream_t s, int64_t nnodes, const uint8_t *fixed, const double *in,
                              double *out) {
  copy_masked_kernel<<<nblocks(nnodes), kBs, 0, s>>>(nnodes, fixed, in, out);
  return hipGetLastError();
}

__global__ void copy_fixed_kernel(int64_t nnodes, const uint8_t *fixed, const double *in,
                                  double *out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nnodes) return;
  const uint8_t f = fixed[n];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if ((f >> c) & 1) out[3 * n + c] = in[3 * n + c];
}

hipError_t launch_copy_fixed(hipStream_t s, int64_t nnodes, const uint8_t *fixed, const double *in,
                             double *out) {
  copy_fixed_kernel<<<nblocks(nnodes), kBs, 0, s>>>(nnodes, fixed, in, out);
  return hipGetLastError();
}

__device__ __forceinline__ void dot_body(int64_t n, const double *a, const double *b, double *partials,
                                         const int *skip) {
  if (skipped(skip)) return;
  double t = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    t = fma(a[i], b[i], t);
  double v[1] = {t};
  block_reduce_store<1, false>(v, partials, blockIdx.x);
}

__global__ void dot_kernel(int64_t n, const double *a, const double *b, double *partials, const int *skip) {
  dot_body(n, a, b, partials, skip);
}
__global__ void dot_group_kernel(int64_t n, GroupTab<DotArgs> t, GroupTab<double *> part) {
  const DotArgs &a = t.v[blockIdx.z];
  dot_body(n, a.a, a.b, part.v[blockIdx.z], a.skip);
}

hipError_t launch_dot(hipStream_t s, int64_t n, const double *a, const double *b, const Reducer &red,
                      const Fin &fin, const int *skip) {
  const unsigned nb = red_blocks(n, red);
  dot_kernel<<<nb, kBs, 0, s>>>(n, a, b, red.partials, skip);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch_finalize(s, red, (int)nb, 1, fin, skip);
}

// nv <= kMaxRed dot products a_k . b in one pass; every value is summed in the
// order of dot_body (the same per-thread chains, block tree and finalize), so
// each equals the separate dot product bit for bit
__device__ __forceinline__ void multi_dot_body(int64_t n, const MultiDotArgs &m, double *partials) {
  double t[kMaxRed] = {};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double bi = m.b[i];
#pragma unroll
    for (int k = 0; k < kMaxRed; ++k)
      if (k < m.nv) t[k] = fma(m.a[k][i], bi, t[k]);
  }
  block_reduce_store<kMaxRed, false>(t, partials, blockIdx.x);
}
__global__ void multi_dot_kernel(int64_t n, MultiDotArgs m, double *partials) { multi_dot_body(n, m, partials); }
__global__ void multi_dot_group_kernel(int64_t n, GroupTab<MultiDotArgs> t, GroupTab<double *> part) {
  multi_dot_body(n, t.v[blockIdx.z], part.v[blockIdx.z]);
}

hipError_t launch_multi_dot(hipStream_t s, int64_t n, const MultiDotArgs &m, const Reducer &red, const Fin &fin) {
  if (m.nv < 1 || m.nv > kMaxRed) return hipErrorInvalidValue;
  const unsigned nb = red_blocks(n, red);
  multi_dot_kernel<<<nb, kBs, 0, s>>>(n, m, red.partials);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch_finalize(s, red, (int)nb, m.nv, fin);
}

// r32 (optional): the new residual rounded to FP32 as well, the right-hand side
// of a single-precision preconditioner
// pq_parts (optional): p.q as npq block partials, summed here by every block
__device__ __forceinline__ void cg_update_xr_body(int64_t n, Scalars *sc, double *x, double *r,
                                                  const double *p, const double *q, float *r32,
                                                  double *partials, const int *skip,
                                                  const double *pq_parts = nullptr, int npq = 0,
                                                  int count_iter = 0) {
  if (skipped(skip)) return;
  double pq;
  if (pq_parts) {
    pq = block_sum_partials(pq_parts, npq, 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->pq = pq;
      sc->rz_old = sc->rz;
      if (count_iter) sc->cg_iters += 1;
    }
  } else {
    pq = sc->pq;
  }
  const double alpha = sc->rz / pq;
  double t = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    x[i] = fma(alpha, p[i], x[i]);
    const double ri = fma(-alpha, q[i], r[i]);
    r[i] = ri;
    if (r32) r32[i] = (float)ri;
    t = fma(ri, ri, t);
  }
  double v[1] = {t};
  block_reduce_store<1, false>(v, partials, blockIdx.x);
}

__global__ void cg_update_xr_kernel(int64_t n, Scalars *sc, double *x, double *r, const double *p,
                                    const double *q, float *r32, double *partials, const int *skip) {
  cg_update_xr_body(n, sc, x, r, p, q, r32, partials, skip);
}
__global__ void cg_update_xr_pq_kernel(int64_t n, Scalars *sc, double *x, double *r, const double *p,
                                       const double *q, float *r32, double *partials, const int *skip,
                                       const double *pq_parts, int npq, int count_iter) {
  cg_update_xr_body(n, sc, x, r, p, q, r32, partials, skip, pq_parts, npq, count_iter);
}
__global__ void cg_update_xr_group_kernel(int64_t n, GroupTab<XrArgs> t, GroupTab<double *> part) {
  const XrArgs &a = t.v[blockIdx.z];
  cg_update_xr_body(n, a.sc, a.x, a.r, a.p, a.q, a.r32, part.v[blockIdx.z], a.skip);
}
// p.q partials at value 0 of the member's slots, r.r to value 1
__global__ void cg_update_xr_group_pq_kernel(int64_t n, GroupTab<XrArgs> t, GroupTab<double *> part, int npq) {
  const XrArgs &a = t.v[blockIdx.z];
  double *pp = part.v[blockIdx.z];
  cg_update_xr_body(n, a.sc, a.x, a.r, a.p, a.q, a.r32, pp + 1, a.skip, pp, npq, 0);
}

hipError_t launch_cg_update_xr(hipStream_t s, int64_t n, Scalars *sc, double *x, double *r,
                               const double *p, const double *q, const Reducer &red, const Fin &fin,
                               const int *skip, float *r32) {
  const unsigned nb = red_blocks(n, red);
  cg_update_xr_kernel<<<nb, kBs, 0, s>>>(n, sc, x, r, p, q, r32, red.partials, skip);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch_finalize(s, red, (int)nb, 1, fin, skip);
}

hipError_t launch_cg_update_xr_pq(hipStream_t s, int64_t n, Scalars *sc, double *x, double *r,
                                  const double *p, const double *q, const Reducer &red, int npq,
                                  const Fin &fin, const int *skip, float *r32, int *defer_rr) {
  static_assert(kBs == 256, "block_sum_partials reproduces the 256-thread finalize");
  if (npq < 1 || npq > red.max_blocks) return hipErrorInvalidValue;
  if (defer_rr && fin.mode != FIN_CG_CHECK) return hipErrorInvalidValue;
  const unsigned nb = red_blocks(n, red);
  // r.r into value 1 of each slot: the p.q partials (value 0) stay intact while
  // other blocks still read them
  Reducer r1 = red;
  r1.partials = red.partials + 1;
  cg_update_xr_pq_kernel<<<nb, kBs, 0, s>>>(n, sc, x, r, p, q, r32, r1.partials, skip, red.partials, npq,
                                            defer_rr ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (defer_rr) return *defer_rr = (int)nb, hipSuccess;
  return launch_finalize(s, r1, (int)nb, 1, fin, skip);
}

__device__ __forceinline__ void cg_start_body(Scalars *sc, double rtol2, int max_iters) {
  sc->cg_iters = 0;
  sc->rtol2 = rtol2;
  sc->cg_max = max_iters;
  sc->nn_fallback = 0;
  sc->rz = 1.0;  // the first r.z finalize forms a beta that is never used: keep it finite
  sc->rr_start = sc->rr;
  sc->cg_done = !(sc->rr > rtol2 * sc->ff) || max_iters <= 0;
}
__global__ void cg_start_kernel(Scalars *sc, double rtol2, int max_iters) { cg_start_body(sc, rtol2, max_iters); }
// one thread per problem
__global__ void cg_start_group_kernel(GroupTab<CgStartArgs> t) {
  const CgStartArgs &a = t.v[threadIdx.x];
  cg_start_body(a.sc, a.rtol2, a.max_iters);
}

hipError_t launch_cg_start(hipStream_t s, Scalars *sc, double rtol2, int max_iters) {
  cg_start_kernel<<<1, 1, 0, s>>>(sc, rtol2, max_iters);
  return hipGetLastError();
}

__global__ void jacobi_kernel(int64_t n, const double *r, const double *dinv, double *z,
                              double *partials, const int *skip) {
  if (skipped(skip)) return;
  double t = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double zi = r[i] * dinv[i];
    z[i] = zi;
    t = fma(r[i], zi, t);
  }
  double v[1] = {t};
  block_reduce_store<1, false>(v, partials, blockIdx.x);
}

hipError_t launch_jacobi(hipStream_t s, int64_t n, const double *r, const double *dinv, double *z,
                         const Reducer &red, const Fin &fin, const int *skip) {
  const unsigned nb = red_blocks(n, red);
  jacobi_kernel<<<nb, kBs, 0, s>>>(n, r, dinv, z, red.partials, skip);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch_finalize(s, red, (int)nb, 1, fin, skip);
}

// p = z + beta p; z in double, or in single precision (the output of a
// single-precision preconditioner, widened exactly)
template <typename Z>
__device__ __forceinline__ void cg_update_p_body(int64_t n, const Scalars *sc, const Z *z, double *p, int first,
                                                 const int *skip) {
  if (skipped(skip)) return;
  const double beta = first ? 0.0 : sc->beta;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double zi = (double)z[i];
    p[i] = first ? zi : fma(beta, p[i], zi);
  }
}

template <typename Z>
__global__ void cg_update_p_kernel(int64_t n, const Scalars *sc, const Z *z, double *p, int first,
                                   const int *skip) {
  cg_update_p_body<Z>(n, sc, z, p, first, skip);
}
__device__ __forceinline__ void cg_update_p_flex_body(int64_t n, Scalars *sc, const float *z, double *p,
                                                      const double *parts, int nrz, const int *skip) {
  if (skipped(skip)) return;
  const double rzn = block_sum_partials(parts, nrz, 0);
  const double rzo = block_sum_partials(parts, nrz, 1);
  const double beta = (rzn - rzo) / sc->rz_old;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->red[0] = rzn;
    sc->red[1] = rzo;
    sc->beta = beta;
    sc->rz = rzn;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = fma(beta, p[i], (double)z[i]);
}
__global__ void cg_update_p_flex_kernel(int64_t n, Scalars *sc, const float *z, double *p, const double *parts,
                                        int nrz, const int *skip) {
  cg_update_p_flex_body(n, sc, z, p, parts, nrz, skip);
}
__global__ void cg_update_p_flex_group_kernel(int64_t n, GroupTab<PArgs> t, GroupTab<double *> part, int nrz) {
  const PArgs &a = t.v[blockIdx.z];
  cg_update_p_flex_body(n, a.sc, static_cast<const float *>(a.z), a.p, part.v[blockIdx.z], nrz, a.skip);
}
template <typename Z>
__global__ void cg_update_p_group_kernel(int64_t n, GroupTab<PArgs> t, int first) {
  const PArgs &a = t.v[blockIdx.z];
  cg_update_p_body<Z>(n, a.sc, static_cast<const Z *>(a.z), a.p, first, a.skip);
}

hipError_t launch_cg_update_p(hipStream_t s, int64_t n, Scalars *sc, const double *z, double *p,
                              int first, const int *skip) {
  cg_update_p_kernel<double><<<nblocks(n, 4), kBs, 0, s>>>(n, sc, z, p, first, skip);
  return hipGetLastError();
}
hipError_t launch_cg_update_p(hipStream_t s, int64_t n, Scalars *sc, const float *z, double *p,
                              int first, const int *skip) {
  cg_update_p_kernel<float><<<nblocks(n, 4), kBs, 0, s>>>(n, sc, z, p, first, skip);
  return hipGetLastError();
}
__global__ void cg_update_p_rz_kernel(int64_t n, Scalars *sc, const double *z, double *p, const double *parts,
                                      int nrz, const int *skip) {
  if (skipped(skip)) return;
  const double rz = block_sum_partials(parts, nrz, 0);
  const double beta = rz / sc->rz_old;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rz_new = rz;
    sc->beta = beta;
    sc->rz = rz;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = fma(beta, p[i], z[i]);
}
hipError_t launch_cg_update_p_rz(hipStream_t s, int64_t n, Scalars *sc, const double *z, double *p,
                                 const Reducer &red, int nrz, const int *skip) {
  if (nrz < 1 || nrz > red.max_blocks) return hipErrorInvalidValue;
  const unsigned nb = std::min(nblocks(n, 4), 1024u);
  cg_update_p_rz_kernel<<<nb, kBs, 0, s>>>(n, sc, z, p, red.partials, nrz, skip);
  return hipGetLastError();
}

__global__ void cheb_last_dot_kernel(int64_t n, const double *res, const double *dinv, double inv_theta, double *x,
                                     const double *r, double *partials, const int *skip) {
  if (skipped(skip)) return;
  double t = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    // x + (res dinv) inv_theta as one fused multiply-add: the form the compiler
    // gives launch_cheb_start's update
    const double xi = fma(res[i] * dinv[i], inv_theta, x[i]);
    x[i] = xi;
    t = fma(r[i], xi, t);
  }
  double v[1] = {t};
  block_reduce_store<1, false>(v, partials, blockIdx.x);
}
hipError_t launch_cheb_last_dot(hipStream_t s, int64_t n, const double *res, const double *dinv, double inv_theta,
                                double *x, const double *r, const Reducer &red, int *nparts, const int *skip) {
  const unsigned nb = red_blocks(n, red);
  cheb_last_dot_kernel<<<nb, kBs, 0, s>>>(n, res, dinv, inv_theta, x, r, red.partials, skip);
  *nparts = (int)nb;
  return hipGetLastError();
}

hipError_t launch_cg_update_p_flex(hipStream_t s, int64_t n, Scalars *sc, const float *z, double *p,
                                   const Reducer &red, int nrz, const int *skip) {
  if (nrz < 1 || nrz > red.max_blocks) return hipErrorInvalidValue;
  // a bounded grid: every block sums the partials first
  const unsigned nb = std::min(nblocks(n, 4), 1024u);
  cg_update_p_flex_kernel<<<nb, kBs, 0, s>>>(n, sc, z, p, red.partials, nrz, skip);
  return hipGetLastError();
}

template <typename T>
__global__ void cheb_first_kernel(int64_t n, const T *r, const T *dinv, T inv_theta, T *d, T *x,
                                  T *res, const int *skip) {
  if (skipped(skip)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T ri = r[i];
  const T di = ri * dinv[i] * inv_theta;
  d[i] = di;
  x[i] = di;
  res[i] = ri;
}

hipError_t launch_cheb_first(hipStream_t s, int64_t n, const double *r, const double *dinv,
                             double inv_theta, double *d, double *x, double *res, const int *skip) {
  cheb_first_kernel<double><<<nblocks(n), kBs, 0, s>>>(n, r, dinv, inv_theta, d, x, res, skip);
  return hipGetLastError();
}
hipError_t launch_cheb_first(hipStream_t s, int64_t n, const float *r, const float *dinv,
                             float inv_theta, float *d, float *x, float *res, const int *skip) {
  cheb_first_kernel<float><<<nblocks(n), kBs, 0, s>>>(n, r, dinv, inv_theta, d, x, res, skip);
  return hipGetLastError();
}

template <typename T>
__device__ __forceinline__ void cheb_start_body(int64_t n, const T *res, const T *dinv, T inv_theta, T *d, T *x,
                                                const int *skip) {
  if (skipped(skip)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T di = res[i] * dinv[i] * inv_theta;
  d[i] = di;
  x[i] += di;
}

template <typename T>
__global__ void cheb_start_kernel(int64_t n, const T *res, const T *dinv, T inv_theta, T *d, T *x,
                                  const int *skip) {
  cheb_start_body<T>(n, res, dinv, inv_theta, d, x, skip);
}
template <typename T>
__global__ void cheb_start_group_kernel(int64_t n, T inv_theta, GroupTab<ChebStartArgs<T>> t) {
  const ChebStartArgs<T> &a = t.v[blockIdx.z];
  cheb_start_body<T>(n, a.res, a.dinv, inv_theta, a.d, a.x, a.skip);
}

hipError_t launch_cheb_start(hipStream_t s, int64_t n, const double *res, const double *dinv,
                             double inv_theta, double *d, double *x, const int *skip) {
  cheb_start_kernel<double><<<nblocks(n), kBs, 0, s>>>(n, res, dinv, inv_theta, d, x, skip);
  return hipGetLastError();
}
hipError_t launch_cheb_start(hipStream_t s, int64_t n, const float *res, const float *dinv,
                             float inv_theta, float *d, float *x, const int *skip) {
  cheb_start_kernel<float><<<nblocks(n), kBs, 0, s>>>(n, res, dinv, inv_theta, d, x, skip);
  return hipGetLastError();
}

// Precision conversions at the boundary of a single-precision preconditioner.
template <typename S, typename D>
__device__ __forceinline__ void convert_body(int64_t n, const S *in, D *out, const int *skip) {
  if (skipped(skip)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (D)in[i];
}
template <typename S, typename D>
__global__ void convert_kernel(int64_t n, const S *in, D *out, const int *skip) {
  convert_body(n, in, out, skip);
}
__global__ void convert_group_kernel(int64_t n, GroupTab<ConvertArgs> t) {
  const ConvertArgs &a = t.v[blockIdx.z];
  convert_body(n, a.in, a.out, a.skip);
}

hipError_t launch_convert(hipStream_t s, int64_t n, const double *in, float *out, const int *skip) {
  convert_kernel<double, float><<<nblocks(n), kBs, 0, s>>>(n, in, out, skip);
  return hipGetLastError();
}
hipError_t launch_convert(hipStream_t s, int64_t n, const float *in, double *out, const int *skip) {
  convert_kernel<float, double><<<nblocks(n), kBs, 0, s>>>(n, in, out, skip);
  return hipGetLastError();
}

// The end of a single-precision preconditioner inside flexible (Polak-Ribiere)
// CG: the new z (kept in single precision; CG widens it exactly where it reads
// it) replaces the previous one in z, and the pass forms r.z_new and r.z_old in
// double.  With res and dinv given, the new z is first the finest level's last
// Chebyshev update x + res dinv / theta (degree-1 smoothing), in the same
// single-precision arithmetic as that update on its own.
__device__ __forceinline__ void flex_dot_body(int64_t n, const float *res, const float *dinv, float inv_theta,
                                              const float *x, const double *r, float *z, double *partials,
                                              const int *skip) {
  if (skipped(skip)) return;
  double tn = 0.0, to = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float zf = x[i];
    if (res) zf += res[i] * dinv[i] * inv_theta;
    const double zo = (double)z[i], zn = (double)zf, ri = r[i];
    z[i] = zf;
    tn = fma(ri, zn, tn);
    to = fma(ri, zo, to);
  }
  double v[2] = {tn, to};
  block_reduce_store<2, false>(v, partials, blockIdx.x);
}

__global__ void flex_dot_kernel(int64_t n, const float *res, const float *dinv, float inv_theta, const float *x,
                                const double *r, float *z, double *partials, const int *skip) {
  flex_dot_body(n, res, dinv, inv_theta, x, r, z, partials, skip);
}
__global__ void flex_dot_group_kernel(int64_t n, float inv_theta, GroupTab<FlexArgs> t, GroupTab<double *> part) {
  const FlexArgs &a = t.v[blockIdx.z];
  flex_dot_body(n, a.res, a.dinv, inv_theta, a.x, a.r, a.z, part.v[blockIdx.z], a.skip);
}

hipError_t launch_flex_dot(hipStream_t s, int64_t n, const float *res, const float *dinv, float inv_theta,
                           const float *x, const double *r, float *z, const Reducer &red, const Fin &fin,
                           const int *skip) {
  const unsigned nb = red_blocks(n, red);
  flex_dot_kernel<<<nb, kBs, 0, s>>>(n, res, dinv, inv_theta, x, r, z, red.partials, skip);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch_finalize(s, red, (int)nb, 2, fin, skip);
}

// linear extrapolation of the solution sequence: u_prev <- u, u <- 2 u - u_prev_old
__device__ __forceinline__ void extrapolate_body(int64_t n, double *u, double *u_prev) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double cur = u[i], old = u_prev[i];
  u_prev[i] = cur;
  u[i] = 2.0 * cur - old;
}
__global__ void extrapolate_kernel(int64_t n, double *u, double *u_prev) { extrapolate_body(n, u, u_prev); }
__global__ void extrapolate_group_kernel(int64_t n, GroupTab<double *> u, GroupTab<double *> u_prev) {
  extrapolate_body(n, u.v[blockIdx.z], u_prev.v[blockIdx.z]);
}

hipError_t launch_extrapolate(hipStream_t s, int64_t n, double *u, double *u_prev) {
  extrapolate_kernel<<<nblocks(n), kBs, 0, s>>>(n, u, u_prev);
  return hipGetLastError();
}

// u = sum_k alpha_k v_k (up to 4 vectors; Combo in internal.h)
__device__ __forceinline__ void combine_body(int64_t n, const Combo &c, double *u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double t = 0.0;
  for (int k = 0; k < c.n; ++k) t = fma(c.alpha[k], c.v[k][i], t);
  u[i] = t;
}
__global__ void combine_kernel(int64_t n, Combo c, double *u) { combine_body(n, c, u); }
__global__ void combine_group_kernel(int64_t n, GroupTab<Combo> c, GroupTab<double *> u) {
  combine_body(n, c.v[blockIdx.z], u.v[blockIdx.z]);
}

hipError_t launch_combine(hipStream_t s, int64_t n, int nv, const double *const *v, const double *alpha, double *u) {
  if (nv < 1 || nv > 4) return hipErrorInvalidValue;
  Combo c{};
  c.n = nv;
  for (int k = 0; k < nv; ++k) {
    c.v[k] = v[k];
    c.alpha[k] = alpha[k];
  }
  combine_kernel<<<nblocks(n), kBs, 0, s>>>(n, c, u);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// grouped launchers (one launch for G problems of equal size; see internal.h)

hipError_t launch_dot_group(hipStream_t s, int G, int64_t n, const DotArgs *a, const Reducer *red, const Fin *fin) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  const unsigned nb = red_blocks(n, red[0]);
  dot_group_kernel<<<dim3(nb, 1, G), kBs, 0, s>>>(n, group_tab(G, a), group_partials(G, red));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const GroupTab<const int *> sk = group_skips(G, a);
  return launch_finalize_group(s, G, red, (int)nb, 1, fin, sk.v);
}

hipError_t launch_cg_update_xr_group(hipStream_t s, int G, int64_t n, const XrArgs *a, const Reducer *red,
                                     const Fin *fin) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  const unsigned nb = red_blocks(n, red[0]);
  cg_update_xr_group_kernel<<<dim3(nb, 1, G), kBs, 0, s>>>(n, group_tab(G, a), group_partials(G, red));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const GroupTab<const int *> sk = group_skips(G, a);
  return launch_finalize_group(s, G, red, (int)nb, 1, fin, sk.v);
}

hipError_t launch_cg_update_xr_group_pq(hipStream_t s, int G, int64_t n, const XrArgs *a, const Reducer *red,
                                        int npq, const Fin *fin) {
  if (!group_ok(G) || npq < 1) return hipErrorInvalidValue;
  Reducer r1[kMaxGroup];
  for (int i = 0; i < G; ++i) {
    if (npq > red[i].max_blocks) return hipErrorInvalidValue;
    r1[i] = red[i];
    r1[i].partials = red[i].partials + 1;
  }
  const unsigned nb = red_blocks(n, red[0]);
  cg_update_xr_group_pq_kernel<<<dim3(nb, 1, G), kBs, 0, s>>>(n, group_tab(G, a), group_partials(G, red), npq);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const GroupTab<const int *> sk = group_skips(G, a);
  return launch_finalize_group(s, G, r1, (int)nb, 1, fin, sk.v);
}

hipError_t launch_cg_update_p_flex_group(hipStream_t s, int G, int64_t n, const PArgs *a, const Reducer *red,
                                         int nrz) {
  if (!group_ok(G) || nrz < 1) return hipErrorInvalidValue;
  for (int i = 0; i < G; ++i)
    if (nrz > red[i].max_blocks) return hipErrorInvalidValue;
  const unsigned nb = std::min(nblocks(n, 4), 1024u);
  cg_update_p_flex_group_kernel<<<dim3(nb, 1, G), kBs, 0, s>>>(n, group_tab(G, a), group_partials(G, red), nrz);
  return hipGetLastError();
}

hipError_t launch_cg_update_p_group(hipStream_t s, int G, int64_t n, bool zsingle, const PArgs *a, int first) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  if (zsingle)
    cg_update_p_group_kernel<float><<<dim3(nblocks(n, 4), 1, G), kBs, 0, s>>>(n, group_tab(G, a), first);
  else
    cg_update_p_group_kernel<double><<<dim3(nblocks(n, 4), 1, G), kBs, 0, s>>>(n, group_tab(G, a), first);
  return hipGetLastError();
}

hipError_t launch_flex_dot_group(hipStream_t s, int G, int64_t n, float inv_theta, const FlexArgs *a,
                                 const Reducer *red, const Fin *fin) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  const unsigned nb = red_blocks(n, red[0]);
  flex_dot_group_kernel<<<dim3(nb, 1, G), kBs, 0, s>>>(n, inv_theta, group_tab(G, a), group_partials(G, red));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const GroupTab<const int *> sk = group_skips(G, a);
  return launch_finalize_group(s, G, red, (int)nb, 2, fin, sk.v);
}

template <typename T>
hipError_t launch_cheb_start_group(hipStream_t s, int G, int64_t n, T inv_theta, const ChebStartArgs<T> *a) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  cheb_start_group_kernel<T><<<dim3(nblocks(n), 1, G), kBs, 0, s>>>(n, inv_theta, group_tab(G, a));
  return hipGetLastError();
}
template hipError_t launch_cheb_start_group<double>(hipStream_t, int, int64_t, double, const ChebStartArgs<double> *);
template hipError_t launch_cheb_start_group<float>(hipStream_t, int, int64_t, float, const ChebStartArgs<float> *);

hipError_t launch_zero_fixed_group(hipStream_t s, int G, int64_t nnodes, const uint8_t *const *fixed,
                                   double *const *v) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  zero_fixed_group_kernel<<<dim3(nblocks(nnodes), 1, G), kBs, 0, s>>>(nnodes, group_tab(G, fixed), group_tab(G, v));
  return hipGetLastError();
}

hipError_t launch_cg_start_group(hipStream_t s, int G, const CgStartArgs *a) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  cg_start_group_kernel<<<1, G, 0, s>>>(group_tab(G, a));
  return hipGetLastError();
}

hipError_t launch_convert_group(hipStream_t s, int G, int64_t n, const ConvertArgs *a) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  convert_group_kernel<<<dim3(nblocks(n), 1, G), kBs, 0, s>>>(n, group_tab(G, a));
  return hipGetLastError();
}

hipError_t launch_extrapolate_group(hipStream_t s, int G, int64_t n, double *const *u, double *const *u_prev) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  extrapolate_group_kernel<<<dim3(nblocks(n), 1, G), kBs, 0, s>>>(n, group_tab(G, u), group_tab(G, u_prev));
  return hipGetLastError();
}

hipError_t launch_combine_group(hipStream_t s, int G, int64_t n, const Combo *c, double *const *u) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  for (int i = 0; i < G; ++i)
    if (c[i].n < 1 || c[i].n > 4) return hipErrorInvalidValue;
  combine_group_kernel<<<dim3(nblocks(n), 1, G), kBs, 0, s>>>(n, group_tab(G, c), group_tab(G, u));
  return hipGetLastError();
}

hipError_t launch_multi_dot_group(hipStream_t s, int G, int64_t n, const MultiDotArgs *m, const Reducer *red,
                                  const Fin *fin) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  for (int i = 0; i < G; ++i)
    if (m[i].nv != m[0].nv || m[i].nv < 1 || m[i].nv > kMaxRed) return hipErrorInvalidValue;
  const unsigned nb = red_blocks(n, red[0]);
  multi_dot_group_kernel<<<dim3(nb, 1, G), kBs, 0, s>>>(n, group_tab(G, m), group_partials(G, red));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int *sk[kMaxGroup] = {};
  return launch_finalize_group(s, G, red, (int)nb, m[0].nv, fin, sk);
}

// plain copies and zero fills of G equally long buffers (32-bit words: every
// buffer here holds doubles or floats)
__global__ void copy_words_group_kernel(int64_t nw, GroupTab<const uint32_t *> src, GroupTab<uint32_t *> dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw) return;
  const uint32_t *sp = src.v[blockIdx.z];
  dst.v[blockIdx.z][i] = sp ? sp[i] : 0u;
}

hipError_t launch_copy_group(hipStream_t s, int G, int64_t bytes, const void *const *src, void *const *dst) {
  if (!group_ok(G) || bytes % 4 != 0) return hipErrorInvalidValue;
  GroupTab<const uint32_t *> a{};
  GroupTab<uint32_t *> b{};
  for (int i = 0; i < G; ++i) {
    a.v[i] = src ? (const uint32_t *)src[i] : nullptr;
    b.v[i] = (uint32_t *)dst[i];
  }
  const int64_t nw = bytes / 4;
  copy_words_group_kernel<<<dim3(nblocks(nw), 1, G), kBs, 0, s>>>(nw, a, b);
  return hipGetLastError();
}

}  // namespace topo
