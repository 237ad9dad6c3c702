// Cone-weight filter as a 3D stencil (Sensitivity Filtering section) and the
// element sensitivities (Optimality Criteria section).
#include "internal.h"
#include "ke_code.h"
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
__global__ __launch_bounds__(kBs) void sensitivity_kernel(Grid g, Kappa kap,
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
    for (int c = 0; c < 24; ++c) t = fma(TOPO_KE(kap, r, c), ue[c], t);
    s = fma(ue[r], t, s);
  }
  ce[e] = s;
  const double x = xphys[e];
  const double xp1 = (penal == 3.0) ? x * x : pow(x, penal - 1.0);
  dc[e] = -penal * xp1 * (E0 - Emin) * s;
}

hipError_t launch_sensitivity(hipStream_t s, Grid g, const Kappa &kap, const double *u,
                              const double *xphys, double E0, double Emin, double penal, double *ce,
                              double *dc) {
  sensitivity_kernel<<<nblocks(g.nel()), kBs, 0, s>>>(g, kap, u, xphys, E0, Emin, penal, ce, dc);
  return hipGetLastError();
}

}  // namespace topo
