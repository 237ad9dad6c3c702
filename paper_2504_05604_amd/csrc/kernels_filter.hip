// Cone-weight filter as a 3D stencil (Sensitivity Filtering section) and the
// element sensitivities (Optimality Criteria section).
#include "group_host.h"
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
// filter_kernel: one thread per element over the offset list, for any reach.
enum FiltOp { F_FWD = TOPO_FILTER_FWD, F_ADJ = TOPO_FILTER_ADJ, F_SENS = TOPO_FILTER_SENS,
              F_VOLW = TOPO_FILTER_VOLW, F_HS = 100 };

template <int OP>
__device__ __forceinline__ void filter_body(const FilterArgs &f, const double *__restrict__ in,
                                            const double *__restrict__ aux, double *__restrict__ out) {
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
template <int OP>
__global__ __launch_bounds__(kBs) void filter_kernel(FilterArgs f, const double *__restrict__ in,
                                                     const double *__restrict__ aux,
                                                     double *__restrict__ out) {
  filter_body<OP>(f, in, aux, out);
}
template <int OP>
__global__ __launch_bounds__(kBs) void filter_group_kernel(GroupTab<FilterCall> t) {
  const FilterCall &c = t.v[blockIdx.z];
  filter_body<OP>(c.f, c.in, c.aux, c.out);
}

// ---------------------------------------------------------------------------
// Tiled stencil for reaches R = ceil(rmin) - 1 in 1..3 (rmin in (1, 4]).  A
// block of kFx x kFy threads produces a tile of kFx x kFy x KZ elements: it
// stages the operand v (the operation's pre-scaled input, zero outside the grid,
// which truncates the stencil at the boundary exactly) of the tile plus a halo
// of R elements in LDS, then each thread marches its KZ elements along z with
// KZ accumulators: for every in-plane offset (dj, di) it reads the LDS column
// once (KZ + 2R values, lanes on consecutive x: conflict-free) and applies the
// 2R + 1 weights of the dk offsets, so an element costs 93 multiply-adds but
// only 25 (KZ + 4) / KZ LDS reads at rmin 3.  Weights depend on |d|^2 only: a
// table of (R + 1)^2 entries staged in LDS with the tile (the dj loop stays
// rolled, so its index is not a compile-time constant; unrolled, the compiler
// hoists every column of the stencil into registers and spills).
namespace {
constexpr int kFx = 32, kFy = 8;

template <int OP>
__device__ __forceinline__ double filter_operand(const FilterArgs &f, const double *__restrict__ in,
                                                 const double *__restrict__ aux, int64_t m) {
  if constexpr (OP == F_FWD) return in[m];
  else if constexpr (OP == F_ADJ) return in[m] * f.sD[m];
  else if constexpr (OP == F_SENS) return in[m] * aux[m];
  else if constexpr (OP == F_VOLW) return f.sD[m];
  else return 1.0;
}
}  // namespace

template <int OP, int R, int KZ>
__device__ __forceinline__ void filter_tile_body(const FilterArgs &f, const double *__restrict__ in,
                                                 const double *__restrict__ aux, double *__restrict__ out) {
  constexpr int NTH = kFx * kFy;
  constexpr int LX = kFx + 2 * R, LY = kFy + 2 * R, LZ = KZ + 2 * R, NT = LX * LY * LZ;
  __shared__ double v[LZ][LY][LX];
  __shared__ double wl[16];
  const Grid g = f.g;
  const int tiles_x = (g.nx + kFx - 1) / kFx, tiles_y = (g.ny + kFy - 1) / kFy;
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int x0 = (tile % tiles_x) * kFx, y0 = ((tile / tiles_x) % tiles_y) * kFy;
  const int z0 = (tile / (tiles_x * tiles_y)) * KZ;
  const int tid = threadIdx.x;
  const int tx = tid % kFx, ty = tid / kFx;
  if (tid < 16) wl[tid] = f.wsq[tid];
  // the epilogue's per-element operands, loaded first so their latency hides
  // behind the staging and the stencil
  const int ox = min(x0 + tx, g.nx - 1), oy = min(y0 + ty, g.ny - 1);
  double post[KZ];
  int8_t mk[KZ];
#pragma unroll
  for (int z = 0; z < KZ; ++z) {
    const int64_t e = ox + (int64_t)g.nx * (oy + (int64_t)g.ny * min(z0 + z, g.nz - 1));
    if constexpr (OP == F_FWD) {
      post[z] = f.Hs[e];
      mk[z] = f.mask[e];
    } else if constexpr (OP == F_SENS) {
      post[z] = f.Hs[e] * fmax(kSensGamma, aux[e]);
    }
  }
  // staging: every load of the tile is issued before the first LDS store (the
  // addresses are clamped into the grid, so the loads need no branch; values
  // outside the grid are replaced by zero when stored)
  constexpr int NS = (NT + NTH - 1) / NTH;
  double val[NS];
  bool inside[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int d = min(tid + t * NTH, NT - 1);
    const int lx = d % LX, ly = (d / LX) % LY, lz = d / (LX * LY);
    const int gx = x0 - R + lx, gy = y0 - R + ly, gz = z0 - R + lz;
    inside[t] = gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz;
    const int cx_ = min(max(gx, 0), g.nx - 1), cy_ = min(max(gy, 0), g.ny - 1), cz_ = min(max(gz, 0), g.nz - 1);
    val[t] = filter_operand<OP>(f, in, aux, cx_ + (int64_t)g.nx * (cy_ + (int64_t)g.ny * cz_));
  }
  double *vf = &v[0][0][0];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int d = tid + t * NTH;
    if (d < NT) vf[d] = inside[t] ? val[t] : 0.0;
  }
  __syncthreads();
  const int gx = x0 + tx, gy = y0 + ty;
  if (gx >= g.nx || gy >= g.ny) return;
  double acc[KZ];
#pragma unroll
  for (int z = 0; z < KZ; ++z) acc[z] = 0.0;
#pragma unroll 1
  for (int dj = -R; dj <= R; ++dj) {
#pragma unroll
    for (int di = -R; di <= R; ++di) {
      double col[LZ];
#pragma unroll
      for (int m = 0; m < LZ; ++m) col[m] = v[m][ty + R + dj][tx + R + di];
#pragma unroll
      for (int dk = -R; dk <= R; ++dk) {
        constexpr int lim = (R + 1) * (R + 1);
        const int q = di * di + dj * dj + dk * dk;
        if (q < lim) {
          const double w = wl[q];
#pragma unroll
          for (int z = 0; z < KZ; ++z) acc[z] = fma(w, col[z + R + dk], acc[z]);
        }
      }
    }
  }
#pragma unroll
  for (int z = 0; z < KZ; ++z) {
    const int gz = z0 + z;
    if (gz >= g.nz) break;
    const int64_t e = gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz);
    if constexpr (OP == F_FWD) {
      out[e] = mk[z] == 1 ? 0.0 : (mk[z] == 2 ? 1.0 : acc[z] / post[z]);
    } else if constexpr (OP == F_SENS) {
      out[e] = acc[z] / post[z];
    } else {
      out[e] = acc[z];
    }
  }
}
template <int OP, int R, int KZ>
__global__ __launch_bounds__(kFx *kFy) void filter_tile_kernel(FilterArgs f, const double *__restrict__ in,
                                                               const double *__restrict__ aux,
                                                               double *__restrict__ out) {
  filter_tile_body<OP, R, KZ>(f, in, aux, out);
}
template <int OP, int R, int KZ>
__global__ __launch_bounds__(kFx *kFy) void filter_tile_group_kernel(GroupTab<FilterCall> t) {
  const FilterCall &c = t.v[blockIdx.z];
  filter_tile_body<OP, R, KZ>(c.f, c.in, c.aux, c.out);
}

namespace {
// G == 0: one problem (f, in, aux, out); else the group table t
template <int OP, int R, int KZ>
hipError_t launch_tiled_rk(hipStream_t s, const FilterArgs &f, const double *in, const double *aux, double *out,
                           int64_t tiles, int G = 0, const GroupTab<FilterCall> *t = nullptr) {
  if (G == 0)
    filter_tile_kernel<OP, R, KZ><<<(unsigned)tiles, kFx * kFy, 0, s>>>(f, in, aux, out);
  else
    filter_tile_group_kernel<OP, R, KZ><<<dim3((unsigned)tiles, 1, G), kFx * kFy, 0, s>>>(*t);
  return hipGetLastError();
}

// tiles 8 elements deep where that still gives every CU a tile (measured at
// 160x80x80: 18 / 16 us per FWD / ADJ pass at rmin 3 against 21 / 20 with
// depth 4), else 2 deep for more tiles on small grids (96x48x48: 11 against
// 14 us)
template <int OP, int R>
hipError_t launch_tiled_r(hipStream_t s, const FilterArgs &f, const double *in, const double *aux, double *out,
                          int G = 0, const GroupTab<FilterCall> *t = nullptr) {
  const Grid g = f.g;
  const int64_t txy = (int64_t)((g.nx + kFx - 1) / kFx) * ((g.ny + kFy - 1) / kFy);
  const int64_t t8 = txy * ((g.nz + 7) / 8), t2 = txy * ((g.nz + 1) / 2);
  if (t2 > INT32_MAX) return hipErrorInvalidValue;
  if (t8 >= 256) return launch_tiled_rk<OP, R, 8>(s, f, in, aux, out, t8, G, t);
  return launch_tiled_rk<OP, R, 2>(s, f, in, aux, out, t2, G, t);
}

template <int OP>
hipError_t launch_op(hipStream_t s, const FilterArgs &f, const double *in, const double *aux, double *out,
                     int G = 0, const GroupTab<FilterCall> *t = nullptr) {
  switch (f.R) {
    case 1: return launch_tiled_r<OP, 1>(s, f, in, aux, out, G, t);
    case 2: return launch_tiled_r<OP, 2>(s, f, in, aux, out, G, t);
    case 3: return launch_tiled_r<OP, 3>(s, f, in, aux, out, G, t);
    default:
      if (G == 0)
        filter_kernel<OP><<<nblocks(f.g.nel()), kBs, 0, s>>>(f, in, aux, out);
      else
        filter_group_kernel<OP><<<dim3(nblocks(f.g.nel()), 1, G), kBs, 0, s>>>(*t);
      return hipGetLastError();
  }
}
}  // namespace

hipError_t launch_filter_group(hipStream_t s, int op, int G, const FilterCall *c) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  for (int i = 0; i < G; ++i) {
    const Grid &g = c[i].f.g, &g0 = c[0].f.g;
    if (g.nx != g0.nx || g.ny != g0.ny || g.nz != g0.nz) return hipErrorInvalidValue;
    const bool tiled = c[i].f.R >= 1 && c[i].f.R <= kFilterTiledMaxR;
    const bool tiled0 = c[0].f.R >= 1 && c[0].f.R <= kFilterTiledMaxR;
    if (tiled != tiled0 || (tiled && c[i].f.R != c[0].f.R)) return hipErrorInvalidValue;
  }
  const GroupTab<FilterCall> t = group_tab(G, c);
  const FilterCall &c0 = c[0];
  switch (op) {
    case TOPO_FILTER_FWD: return launch_op<F_FWD>(s, c0.f, c0.in, c0.aux, c0.out, G, &t);
    case TOPO_FILTER_ADJ: return launch_op<F_ADJ>(s, c0.f, c0.in, c0.aux, c0.out, G, &t);
    case TOPO_FILTER_SENS: return launch_op<F_SENS>(s, c0.f, c0.in, c0.aux, c0.out, G, &t);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_filter_hs(hipStream_t s, const FilterArgs &f, double *Hs) {
  return launch_op<F_HS>(s, f, nullptr, nullptr, Hs);
}

hipError_t launch_filter(hipStream_t s, int op, const FilterArgs &f, const double *in,
                         const double *aux, double *out) {
  switch (op) {
    case TOPO_FILTER_FWD: return launch_op<F_FWD>(s, f, in, aux, out);
    case TOPO_FILTER_ADJ: return launch_op<F_ADJ>(s, f, in, aux, out);
    case TOPO_FILTER_SENS: return launch_op<F_SENS>(s, f, in, aux, out);
    case TOPO_FILTER_VOLW: return launch_op<F_VOLW>(s, f, in, aux, out);
    default: return hipErrorInvalidValue;
  }
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
__device__ __forceinline__ void sensitivity_body(Grid g, const Kappa &kap, const double *__restrict__ u,
                                                 const double *__restrict__ xphys, double E0, double Emin,
                                                 double penal, double *__restrict__ ce,
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
__global__ __launch_bounds__(kBs) void sensitivity_kernel(Grid g, Kappa kap,
                                                          const double *__restrict__ u,
                                                          const double *__restrict__ xphys,
                                                          double E0, double Emin, double penal,
                                                          double *__restrict__ ce,
                                                          double *__restrict__ dc) {
  sensitivity_body(g, kap, u, xphys, E0, Emin, penal, ce, dc);
}
__global__ __launch_bounds__(kBs) void sensitivity_group_kernel(Grid g, GroupTab<SensArgs> t) {
  const SensArgs &a = t.v[blockIdx.z];
  sensitivity_body(g, a.kap, a.u, a.xphys, a.E0, a.Emin, a.penal, a.ce, a.dc);
}

hipError_t launch_sensitivity(hipStream_t s, Grid g, const Kappa &kap, const double *u,
                              const double *xphys, double E0, double Emin, double penal, double *ce,
                              double *dc) {
  sensitivity_kernel<<<nblocks(g.nel()), kBs, 0, s>>>(g, kap, u, xphys, E0, Emin, penal, ce, dc);
  return hipGetLastError();
}

hipError_t launch_sensitivity_group(hipStream_t s, int G, Grid g, const SensArgs *a) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  sensitivity_group_kernel<<<dim3(nblocks(g.nel()), 1, G), kBs, 0, s>>>(g, group_tab(G, a));
  return hipGetLastError();
}

}  // namespace topo
