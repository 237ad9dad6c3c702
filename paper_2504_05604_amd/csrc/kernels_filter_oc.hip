// Cone-weight filter as a 3D stencil, element sensitivities, and the OC update
// with a device-side multisection search for the volume multiplier.
#include "internal.h"
#include "reduce_dev.h"

namespace topo {

namespace {
constexpr int kBs = 256;
inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBs - 1) / kBs); }
constexpr double kSensGamma = 1e-3;
}  // namespace

// ---------------------------------------------------------------------------
// Filter: out_e = sum over stencil offsets o (|o| < rmin) inside the grid of
// w_o * v(e + o) with v chosen by the operation (Sensitivity Filtering section).
enum FiltOp { F_FWD = TOPO_FILTER_FWD, F_ADJ = TOPO_FILTER_ADJ, F_SENS = TOPO_FILTER_SENS,
              F_VOLW = TOPO_FILTER_VOLW, F_HS = 100 };

template <int OP>
__global__ __launch_bounds__(kBs) void filter_kernel(FilterArgs f, const double *__restrict__ in,
                                                     const double *__restrict__ aux,
                                                     double *__restrict__ out) {
  const Grid g = f.g;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.nel()) return;
  const int i = (int)(e % g.nx);
  const int j = (int)((e / g.nx) % g.ny);
  const int k = (int)(e / ((int64_t)g.nx * g.ny));
  double acc = 0.0;
  for (int o = 0; o < f.noff; ++o) {
    const int ii = i + f.off[3 * o], jj = j + f.off[3 * o + 1], kk = k + f.off[3 * o + 2];
    if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny || kk < 0 || kk >= g.nz) continue;
    const int64_t m = ii + (int64_t)g.nx * (jj + (int64_t)g.ny * kk);
    double v;
    if constexpr (OP == F_FWD) v = in[m];
    else if constexpr (OP == F_ADJ) v = in[m] * f.sD[m];
    else if constexpr (OP == F_SENS) v = in[m] * aux[m];
    else if constexpr (OP == F_VOLW) v = f.sD[m];
    else v = 1.0;
    acc = fma(f.w[o], v, acc);
  }
  if constexpr (OP == F_FWD) {
    const int8_t mk = f.mask[e];
    out[e] = mk == 1 ? 0.0 : (mk == 2 ? 1.0 : acc / f.Hs[e]);
  } else if constexpr (OP == F_SENS) {
    out[e] = acc / (f.Hs[e] * fmax(kSensGamma, aux[e]));
  } else {
    out[e] = acc;
  }
}

hipError_t launch_filter_hs(hipStream_t s, const FilterArgs &f, double *Hs) {
  filter_kernel<F_HS><<<nblocks(f.g.nel()), kBs, 0, s>>>(f, nullptr, nullptr, Hs);
  return hipGetLastError();
}

hipError_t launch_filter(hipStream_t s, int op, const FilterArgs &f, const double *in,
                         const double *aux, double *out) {
  const unsigned nb = nblocks(f.g.nel());
  switch (op) {
    case TOPO_FILTER_FWD: filter_kernel<F_FWD><<<nb, kBs, 0, s>>>(f, in, aux, out); break;
    case TOPO_FILTER_ADJ: filter_kernel<F_ADJ><<<nb, kBs, 0, s>>>(f, in, aux, out); break;
    case TOPO_FILTER_SENS: filter_kernel<F_SENS><<<nb, kBs, 0, s>>>(f, in, aux, out); break;
    case TOPO_FILTER_VOLW: filter_kernel<F_VOLW><<<nb, kBs, 0, s>>>(f, in, aux, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ void design_scale_kernel(int64_t nel, const int8_t *mask, const double *Hs, double *sD) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  sD[e] = mask[e] == 0 ? 1.0 / Hs[e] : 0.0;
}

hipError_t launch_design_scale(hipStream_t s, int64_t nel, const int8_t *mask, const double *Hs,
                               double *sD) {
  design_scale_kernel<<<nblocks(nel), kBs, 0, s>>>(nel, mask, Hs, sD);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sensitivities (Optimality Criteria section): ce_e = u_e^T KE u_e and
// dc_e = -p xphys^(p-1) (E0 - Emin) ce_e; thread per element.
__global__ __launch_bounds__(kBs) void sensitivity_kernel(Grid g, const double *__restrict__ KE,
                                                          const double *__restrict__ u,
                                                          const double *__restrict__ xphys,
                                                          double E0, double Emin, double penal,
                                                          double *__restrict__ ce,
                                                          double *__restrict__ dc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.nel()) return;
  const int i = (int)(e % g.nx);
  const int j = (int)((e / g.nx) % g.ny);
  const int k = (int)(e / ((int64_t)g.nx * g.ny));
  double ue[24];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int64_t n = (i + cx(b)) + (int64_t)g.NX() * ((j + cy(b)) + (int64_t)g.NY() * (k + cz(b)));
#pragma unroll
    for (int d = 0; d < 3; ++d) ue[3 * b + d] = u[3 * n + d];
  }
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < 24; ++r) {
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < 24; ++c) t = fma(KE[r * 24 + c], ue[c], t);
    s = fma(ue[r], t, s);
  }
  ce[e] = s;
  const double x = xphys[e];
  const double xp1 = (penal == 3.0) ? x * x : pow(x, penal - 1.0);
  dc[e] = -penal * xp1 * (E0 - Emin) * s;
}

hipError_t launch_sensitivity(hipStream_t s, Grid g, const double *KE, const double *u,
                              const double *xphys, double E0, double Emin, double penal, double *ce,
                              double *dc) {
  sensitivity_kernel<<<nblocks(g.nel()), kBs, 0, s>>>(g, KE, u, xphys, E0, Emin, penal, ce, dc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// OC update.  For design element j: a_j = x_j (max(0,-dc_j)/dv_j)^eta so that the
// candidate is clamp(a_j lambda^-eta, max(0, x_j - move), min(1, x_j + move)).
// The volume V(lambda) = sum_j dv_j x_new_j is non-increasing; every pass
// evaluates it at kOcCand multipliers inside the current bracket (geometric
// spacing while the bracket spans more than a factor 2, linear after) and keeps
// the sub-interval where V crosses the target.

__device__ __forceinline__ double oc_value(double x, double a, double lam_pow, double move) {
  const double lo = fmax(0.0, x - move), hi = fmin(1.0, x + move);
  return fmin(hi, fmax(lo, a * lam_pow));
}

__device__ void oc_make_candidates(Scalars *sc) {
  const double l1 = sc->l1, l2 = sc->l2;
  const bool geo = l1 > 0.0 && l2 > 2.0 * l1;
  for (int c = 0; c < kOcCand; ++c) {
    const double t = (double)(c + 1) / (double)(kOcCand + 1);
    sc->oc_lam[c] = geo ? l1 * pow(l2 / l1, t) : l1 + (l2 - l1) * t;
  }
}

__global__ void oc_prepare_kernel(int64_t nel, const double *__restrict__ x,
                                  const double *__restrict__ dc, const double *__restrict__ dv,
                                  const int8_t *__restrict__ mask, double eta, double target,
                                  double *__restrict__ a, Scalars *sc, Reducer red) {
  double cst = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nel;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (mask[e] == 0) {
      const double B = fmax(0.0, -dc[e]) / dv[e];
      a[e] = x[e] * pow(B, eta);
    } else {
      a[e] = 0.0;
      cst = fma(dv[e], x[e], cst);
    }
  }
  double v[1] = {cst};
  block_reduce_finalize<1, false>(v, red, &sc->vconst);
}

__global__ void oc_init_kernel(Scalars *sc, double target) {
  sc->target = target;
  sc->l1 = 1e-40;   // the multiplier is positive; this stands for the lower end 0
  sc->l2 = 1e40;
  sc->oc_done = 0;
  sc->oc_pass = 0;
  oc_make_candidates(sc);
}

// One multisection pass; the last block picks the new bracket.
__global__ __launch_bounds__(kBs) void oc_pass_kernel(int64_t nel, const double *__restrict__ x,
                                                      const double *__restrict__ a,
                                                      const double *__restrict__ dv,
                                                      const int8_t *__restrict__ mask, double move,
                                                      double eta, double tol, Scalars *sc,
                                                      Reducer red) {
  if (sc->oc_done) return;
  __shared__ double lampow[kOcCand];
  for (int c = threadIdx.x; c < kOcCand; c += blockDim.x) lampow[c] = pow(sc->oc_lam[c], -eta);
  __syncthreads();
  double part[kOcCand];
#pragma unroll
  for (int c = 0; c < kOcCand; ++c) part[c] = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nel;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (mask[e] != 0) continue;
    const double xe = x[e], ae = a[e], we = dv[e];
#pragma unroll
    for (int c = 0; c < kOcCand; ++c) part[c] = fma(we, oc_value(xe, ae, lampow[c], move), part[c]);
  }
  // block reduce all candidates through LDS
  __shared__ double sh[kOcCand][kBs / 64];
  __shared__ int is_last;
  const int lane = threadIdx.x & 63, wid = threadIdx.x / 64;
#pragma unroll
  for (int c = 0; c < kOcCand; ++c) {
    double t = wave_reduce<false>(part[c]);
    if (lane == 0) sh[c][wid] = t;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < kOcCand; c += blockDim.x) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) t += sh[c][w];
    red.partials[(size_t)blockIdx.x * 64 + c] = t;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(red.counter, 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  const volatile double *P = red.partials;
  for (int c = threadIdx.x; c < kOcCand; c += blockDim.x) {
    double t = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) t += P[(size_t)b * 64 + c];
    sc->oc_vol[c] = t + sc->vconst;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicExch(red.counter, 0u);
    const double target = sc->target;
    double l1 = sc->l1, l2 = sc->l2;
    // V non-increasing: the last candidate above the target and the first at/below it
    for (int c = 0; c < kOcCand; ++c) {
      const volatile double *V = sc->oc_vol;
      if (V[c] > target) l1 = sc->oc_lam[c];
      else { l2 = sc->oc_lam[c]; break; }
    }
    sc->l1 = l1;
    sc->l2 = l2;
    sc->oc_pass += 1;
    if ((l2 - l1) / (l1 + l2) < tol || sc->oc_pass >= 64) sc->oc_done = 1;
    else oc_make_candidates(sc);
  }
}

__global__ void oc_final_kernel(int64_t nel, const double *__restrict__ x,
                                const double *__restrict__ a, const double *__restrict__ dv,
                                const int8_t *__restrict__ mask, double move, double eta,
                                double *__restrict__ xnew, Scalars *sc, Reducer red) {
  const double lam = 0.5 * (sc->l1 + sc->l2);
  const double lp = pow(lam, -eta);
  double chg = 0.0, vol = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nel;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double xe = x[e];
    const double xn = mask[e] == 0 ? oc_value(xe, a[e], lp, move) : xe;
    xnew[e] = xn;
    chg = fmax(chg, fabs(xn - xe));
    vol = fma(dv[e], xn, vol);
  }
  double vm[1] = {chg};
  block_reduce_finalize<1, true>(vm, red, &sc->change);
  // second reduction reuses the partial buffer after the first finished; a
  // separate counter slot keeps the two independent
  Reducer red2 = red;
  red2.counter = red.counter + 1;
  red2.partials = red.partials + 1;
  double vs[1] = {vol};
  block_reduce_finalize<1, false>(vs, red2, &sc->volume);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->lambda = lam;
}

hipError_t launch_oc_prepare(hipStream_t s, int64_t nel, const double *x, const double *dc,
                             const double *dv, const int8_t *mask, double eta, double target,
                             double *a, Scalars *sc, const Reducer &red) {
  unsigned nb = nblocks(nel);
  if (nb > (unsigned)red.max_blocks) nb = red.max_blocks;
  oc_prepare_kernel<<<nb, kBs, 0, s>>>(nel, x, dc, dv, mask, eta, target, a, sc, red);
  oc_init_kernel<<<1, 1, 0, s>>>(sc, target);
  return hipGetLastError();
}

hipError_t launch_oc_pass(hipStream_t s, int64_t nel, const double *x, const double *a,
                          const double *dv, const int8_t *mask, double move, double eta,
                          double tol, Scalars *sc, const Reducer &red) {
  unsigned nb = nblocks(nel);
  const unsigned cap = (unsigned)(red.max_blocks * kMaxRed / 64);
  if (nb > cap) nb = cap;
  if (nb > 1024) nb = 1024;
  oc_pass_kernel<<<nb, kBs, 0, s>>>(nel, x, a, dv, mask, move, eta, tol, sc, red);
  return hipGetLastError();
}

hipError_t launch_oc_final(hipStream_t s, int64_t nel, const double *x, const double *a,
                           const double *dv, const int8_t *mask, double move, double eta,
                           double *xnew, Scalars *sc, const Reducer &red) {
  unsigned nb = nblocks(nel);
  if (nb > (unsigned)red.max_blocks) nb = red.max_blocks;
  oc_final_kernel<<<nb, kBs, 0, s>>>(nel, x, a, dv, mask, move, eta, xnew, sc, red);
  return hipGetLastError();
}

}  // namespace topo
