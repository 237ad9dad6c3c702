// Matrix-free element-by-element stiffness operator on the structured hex grid.
//
// y_i = sum over the (up to 8) elements e around node i of E_e (KE u_e)_{local(i)},
// i.e. the product with K = sum_e E_e KE of the Finite Element Analysis section
// without assembling it.
//
// Work decomposition: a thread owns a column of KZ consecutive nodes (i, j, k0..)
// and marches up through the element layers between them.  At layer L it holds
// the 3x3 patches of node planes L and L+1 in registers (18 nodes, 54 values),
// which are exactly the nodes of the 4 elements of that layer around the column;
// it finishes node (i,j,L) with the bottom-face rows of those elements and
// starts node (i,j,L+1) with their top-face rows, then shifts plane L+1 down.
// Each node is written by one thread only (deterministic, no atomics); each
// node value is loaded once per column instead of once per neighbour, and KE
// comes from the compile-time sign/index tables with 10 register values.
//
// The epilogues fuse the vector updates of the conjugate-gradient loop and of
// the Chebyshev smoother into the operator pass, and the first smoothing step
// builds its operand d0 = b dinv / theta on the fly from the right-hand side.
//
// Fixed dofs: inputs are required to be zero there (the solver keeps every
// vector in the subspace of free dofs); outputs get the identity row y = u.
#include <algorithm>
#include <type_traits>

#include "group_host.h"
#include "internal.h"
#include "ke_code.h"
#include "ku_epilogue.h"
#include "reduce_dev.h"

namespace topo {

// Launch shape: KZ nodes per thread column, BS threads per block.  Large grids
// march KZ = 8 nodes (fewer plane reloads); small grids use short columns and
// small blocks so the launch still spreads over the 256 CUs.
template <int EPI, int KZ, int BS, typename T>
__global__ __launch_bounds__(BS) void ku_march_kernel(KuArgsT<T> a, KappaT<T> kap, double *partials) {
  if (a.skip && *a.skip) return;
  const Grid g = a.g;
  const int NX = g.NX(), NY = g.NY(), NZ = g.NZ();
  const int ncol = NX * NY;
  // tiles: BS columns x KZ node planes, x-major; contiguous runs per XCD
  const int tile = xcd_tile(linear_block(), gridDim.x * gridDim.y);
  const int col = (tile % gridDim.x) * BS + threadIdx.x;
  const int k0 = (tile / gridDim.x) * KZ;
  const int k1 = min(k0 + KZ, NZ);
  const bool active = col < ncol;
  const int i = active ? col % NX : 0, j = active ? col / NX : 0;
  const int64_t plane = (int64_t)ncol;
  constexpr bool kScaled = EpiTraits<EPI>::scaled_operand;
  const T *__restrict__ u = kScaled ? a.b : a.u;
  const T *__restrict__ dinv = a.dinv;
  double dotv[2] = {0.0, 0.0};
  if (active) {
    T P0[9][3], P1[9][3];
    auto load_plane = [&](int kp, T(&P)[9][3]) {
      const bool okz = kp >= 0 && kp <= g.nz;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int q = (dx + 1) + 3 * (dy + 1);
          const bool ok = okz && (i + dx >= 0) && (i + dx <= g.nx) && (j + dy >= 0) && (j + dy <= g.ny);
          const int64_t m = (int64_t)kp * plane + (int64_t)(j + dy) * NX + (i + dx);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            if constexpr (kScaled)
              P[q][c] = ok ? u[3 * m + c] * dinv[3 * m + c] * a.s0 : T(0);
            else
              P[q][c] = ok ? u[3 * m + c] : T(0);
          }
        }
    };
    T acc0 = 0, acc1 = 0, acc2 = 0;  // node (i,j,L): top-face part so far
    // element layer L between node planes L (Pb) and L+1 (Pt)
    auto layer = [&](const int L, const T(&Pb)[9][3], const T(&Pt)[9][3]) {
      T nb0 = 0, nb1 = 0, nb2 = 0;  // node (i,j,L+1)
      // bottom-face rows finish node L, top-face rows start node L+1; the first
      // and last layer of a column need only one of the two (uniform per block)
      auto faces = [&](auto bot_tag, auto top_tag) {
        constexpr bool kBot = decltype(bot_tag)::value, kTop = decltype(top_tag)::value;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int ex = e & 1, ey = e >> 1;  // element (i-1+ex, j-1+ey, L)
          const int ei = i - 1 + ex, ej = j - 1 + ey;
          const bool eok = ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny && L >= 0 && L < g.nz;
          const T Ee = eok ? a.E[ei + (int64_t)g.nx * (ej + (int64_t)g.ny * L)] : T(0);
          const int lb = corner_of(1 - ex, 1 - ey, 0), lt = corner_of(1 - ex, 1 - ey, 1);
          T b0 = 0, b1 = 0, b2 = 0, t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
          for (int b = 0; b < 8; ++b) {
            const int q = (ex + cx(b)) + 3 * (ey + cy(b));
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const T v = cz(b) ? Pt[q][d] : Pb[q][d];
              if constexpr (kBot) {
                b0 = fma(TOPO_KE(kap, 3 * lb + 0, 3 * b + d), v, b0);
                b1 = fma(TOPO_KE(kap, 3 * lb + 1, 3 * b + d), v, b1);
                b2 = fma(TOPO_KE(kap, 3 * lb + 2, 3 * b + d), v, b2);
              }
              if constexpr (kTop) {
                t0 = fma(TOPO_KE(kap, 3 * lt + 0, 3 * b + d), v, t0);
                t1 = fma(TOPO_KE(kap, 3 * lt + 1, 3 * b + d), v, t1);
                t2 = fma(TOPO_KE(kap, 3 * lt + 2, 3 * b + d), v, t2);
              }
            }
          }
          if constexpr (kBot) {
            acc0 = fma(Ee, b0, acc0);
            acc1 = fma(Ee, b1, acc1);
            acc2 = fma(Ee, b2, acc2);
          }
          if constexpr (kTop) {
            nb0 = fma(Ee, t0, nb0);
            nb1 = fma(Ee, t1, nb1);
            nb2 = fma(Ee, t2, nb2);
          }
        }
      };
      if constexpr (KZ > 2) {
        // long columns: one shared code path keeps the register count down; the
        // unneeded half of the first/last layer is 1/KZ of the work
        faces(std::true_type{}, std::true_type{});
      } else {
        if (L >= k0 && L + 1 < k1)
          faces(std::true_type{}, std::true_type{});
        else if (L >= k0)
          faces(std::true_type{}, std::false_type{});
        else
          faces(std::false_type{}, std::true_type{});
      }
      if (L >= k0) {  // node (i,j,L) is complete
        const int64_t n = (int64_t)L * plane + col;
        const T self[3] = {Pb[4][0], Pb[4][1], Pb[4][2]};
        const T Au[3] = {acc0, acc1, acc2};
        ku_node_epilogue<EPI>(a, n, self, Au, dinv, dotv);
      }
      acc0 = nb0;
      acc1 = nb1;
      acc2 = nb2;
    };
    load_plane(k0 - 1, P0);
    // fully unrolled over the KZ + 1 layers (the last column of the grid may be
    // shorter): straight-line code lets the compiler rename the plane registers
    // instead of copying them and issue the next plane's loads early
#pragma unroll
    for (int q = 0; q <= KZ; ++q) {
      const int L = k0 - 1 + q;
      if (L >= k1) break;
      load_plane(L + 1, P1);
      layer(L, P0, P1);
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        P0[q][0] = P1[q][0];
        P0[q][1] = P1[q][1];
        P0[q][2] = P1[q][2];
      }
    }
  }
  ku_block_reduce<EPI>(a, dotv, partials);
}

template <int KZ, int BS, typename T>
static hipError_t launch_ku_shape(hipStream_t s, KuEpi epi, const KuArgsT<T> &a, const KappaT<T> &kap,
                                  const Reducer &red, int *nparts_out) {
  const int ncol = a.g.NX() * a.g.NY();
  const dim3 grid((unsigned)((ncol + BS - 1) / BS), (unsigned)((a.g.NZ() + KZ - 1) / KZ));
  const int nparts = (int)(grid.x * grid.y);
  *nparts_out = nparts;
  if (ku_reduces(epi, a) && nparts > red.max_blocks) return hipErrorInvalidValue;
#define TOPO_KU_CASE(E) \
  case E: ku_march_kernel<E, KZ, BS, T><<<grid, BS, 0, s>>>(a, kap, red.partials); break;
  switch (epi) {
    TOPO_KU_CASE(KU_STORE)
    TOPO_KU_CASE(KU_STORE_DOT)
    TOPO_KU_CASE(KU_RESID)
    TOPO_KU_CASE(KU_RES0)
    TOPO_KU_CASE(KU_CHEB0)
    TOPO_KU_CASE(KU_CHEB)
    TOPO_KU_CASE(KU_CHEB_ADD)
    TOPO_KU_CASE(KU_RESUPD)
    TOPO_KU_CASE(KU_RESID_START)
    TOPO_KU_CASE(KU_RESID_FLEX)
    default: return hipErrorInvalidValue;
  }
#undef TOPO_KU_CASE
  return hipGetLastError();
}

// Node-column shapes measured on MI355X: 160x80x80 -> KZ 8 with 256 (smoother
// epilogues) or 128 threads (CG product); 80x40x40 -> KZ 2 x 128; smaller grids ->
// KZ 1 x 64, where a launch is bound by latency rather than arithmetic.
// Element-column shapes measured on MI355X (CG product): 160x80x80 -> 32 x 8
// tiles of 8 planes, 20 us (single-precision smoothing: the same tiles with the
// node planes staged through LDS, about 1 % faster per SIMP iteration); 80x40x40
// -> 8 x 8 tiles of 2 planes with the next plane loaded ahead, 10 us; smaller
// grids -> 8 x 8 tiles of one plane (latency bound, 4-6 us).
int ku_shape_for(const Grid &g, KuEpi epi, int family, bool single) {
  const int64_t nn = g.nnodes();
  if (family == TOPO_KU_NODE) {
    if (nn >= 600000) return epi == KU_STORE_DOT ? 1 : 0;
    if (nn >= 60000) return 2;
    return 3;
  }
  if (nn >= 600000) return single ? kKuShapeHada + 7 : kKuShapeHada + 0;
  if (nn >= 50000) return kKuShapeHada + 3;
  return kKuShapeHada + 4;
}

int64_t ku_max_blocks(const Grid &g) {
  const int64_t ncol = (int64_t)g.NX() * g.NY(), nz = g.NZ();
  // node-column shapes: KZ x BS = 8 x 256, 8 x 128, 2 x 128, 1 x 64
  int64_t m = std::max<int64_t>({(ncol + 255) / 256 * ((nz + 7) / 8), (ncol + 127) / 128 * ((nz + 7) / 8),
                                 (ncol + 127) / 128 * ((nz + 1) / 2), (ncol + 63) / 64 * nz});
  return std::max(m, ku_hada_max_blocks(g));
}

std::vector<int> ku_tunable_shapes(bool single, int family) {
  std::vector<int> v;
  if (family != TOPO_KU_ELEMENT)
    for (int i = 0; i < kKuShapes; ++i) v.push_back(i);
  if (single && family == TOPO_KU_AUTO) v.push_back(kKuShapeMfma);
  if (family != TOPO_KU_NODE)
    for (int i = 0; i < kKuShapesHada; ++i) v.push_back(kKuShapeHada + i);
  return v;
}

template <typename T>
static hipError_t launch_ku_t(hipStream_t s, KuEpi epi, const KuArgsT<T> &a, const KappaT<T> &kap,
                              const Reducer &red, const Fin &fin, int shape, int *defer_parts = nullptr) {
  if (shape < 0) shape = ku_shape_for(a.g, epi, TOPO_KU_AUTO, std::is_same<T, float>::value);
  if constexpr (std::is_same<T, float>::value) {
    if (shape == kKuShapeMfma || shape == kKuShapeMfmaBf16) return launch_ku_mfma(s, epi, a, shape == kKuShapeMfmaBf16);
  }
  int nparts = 0;
  hipError_t e;
  if (shape >= kKuShapeHada && shape < kKuShapeHada + kKuShapesHada) {
    e = launch_ku_hada<T>(s, epi, a, kap, red, shape - kKuShapeHada, &nparts);
    if (e != hipSuccess) return e;
    if (defer_parts) return *defer_parts = nparts, hipSuccess;
    if (ku_reduces(epi, a)) return launch_finalize(s, red, nparts, ku_ndot(epi), fin, a.skip);
    return hipSuccess;
  }
  switch (shape) {
    case 0: e = launch_ku_shape<8, 256>(s, epi, a, kap, red, &nparts); break;
    case 1: e = launch_ku_shape<8, 128>(s, epi, a, kap, red, &nparts); break;
    case 2: e = launch_ku_shape<2, 128>(s, epi, a, kap, red, &nparts); break;
    case 3: e = launch_ku_shape<1, 64>(s, epi, a, kap, red, &nparts); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (defer_parts) return *defer_parts = nparts, hipSuccess;
  if (ku_reduces(epi, a)) return launch_finalize(s, red, nparts, ku_ndot(epi), fin, a.skip);
  return hipSuccess;
}

hipError_t launch_ku(hipStream_t s, KuEpi epi, const KuArgs &a, const Kappa &kap, const Reducer &red,
                     const Fin &fin, int shape, int *defer_parts) {
  if (defer_parts && (epi != KU_STORE_DOT || a.dot_with)) return hipErrorInvalidValue;
  if (a.chk_parts && !(shape >= kKuShapeHada && shape < kKuShapeHada + kKuShapesHada)) return hipErrorInvalidValue;
  return launch_ku_t<double>(s, epi, a, kap, red, fin, shape, defer_parts);
}

hipError_t launch_ku(hipStream_t s, KuEpi epi, const KuArgsT<float> &a, const KappaT<float> &kap,
                     const Reducer &red, const Fin &fin, int shape, int *defer_parts) {
  if (epi == KU_STORE_DOT || epi == KU_RESID || a.dot_with) return hipErrorInvalidValue;
  if (defer_parts && (epi != KU_RESID_FLEX || shape == kKuShapeMfma || shape == kKuShapeMfmaBf16))
    return hipErrorInvalidValue;
  // the stopping test rides on element-column shapes only
  if (a.chk_parts && !(shape >= kKuShapeHada && shape < kKuShapeHada + kKuShapesHada)) return hipErrorInvalidValue;
  return launch_ku_t<float>(s, epi, a, kap, red, fin, shape, defer_parts);
}

// Grouped K.u (element-column shapes only): one launch for G problems of the
// same grid, each reducing into its own partials and finalize.
template <typename T>
hipError_t launch_ku_group(hipStream_t s, KuEpi epi, int G, const KuArgsT<T> *a, const KappaT<T> &kap,
                           const Reducer *red, const Fin *fin, int shape, int *defer_parts) {
  if (G < 1 || G > kMaxGroup) return hipErrorInvalidValue;
  if (shape < kKuShapeHada || shape >= kKuShapeHada + kKuShapesHada) return hipErrorInvalidValue;
  if constexpr (std::is_same<T, float>::value) {
    if (epi == KU_STORE_DOT || epi == KU_RESID) return hipErrorInvalidValue;
  }
  int nparts = 0;
  if (defer_parts && epi != KU_STORE_DOT && epi != KU_RESID_FLEX) return hipErrorInvalidValue;
  hipError_t e = launch_ku_hada_group<T>(s, epi, G, a, kap, red, shape - kKuShapeHada, &nparts);
  if (e != hipSuccess) return e;
  if (defer_parts) return *defer_parts = nparts, hipSuccess;
  if (!ku_reduces(epi, a[0])) return hipSuccess;
  Fin f[kMaxGroup];
  const int *sk[kMaxGroup];
  for (int i = 0; i < G; ++i) {
    f[i] = fin[i];
    sk[i] = a[i].skip;
  }
  return launch_finalize_group(s, G, red, nparts, ku_ndot(epi), f, sk);
}
template hipError_t launch_ku_group<double>(hipStream_t, KuEpi, int, const KuArgsT<double> *, const KappaT<double> &,
                                            const Reducer *, const Fin *, int, int *);
template hipError_t launch_ku_group<float>(hipStream_t, KuEpi, int, const KuArgsT<float> *, const KappaT<float> &,
                                           const Reducer *, const Fin *, int, int *);

// ---------------------------------------------------------------------------
// Sums the block partials in block order.  Besides writing the sum, a finalize
// can run the scalar step of the CG loop that consumes it (FinMode).
__device__ __forceinline__ void finalize_body(const double *partials, int nparts, int n, const Fin &fin,
                                              const int *skip) {
  if (skip && *skip) return;
  __shared__ double sh[kMaxRed][16];
  const bool is_max = fin.mode == FIN_MAX;
  const int lane = threadIdx.x & 63, wid = threadIdx.x / 64, nw = blockDim.x / 64;
  for (int k = 0; k < n; ++k) {
    double t = is_max ? -INFINITY : 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
      const double v = partials[(size_t)b * kMaxRed + k];
      t = is_max ? fmax(t, v) : t + v;
    }
    t = is_max ? wave_reduce<true>(t) : wave_reduce<false>(t);
    if (lane == 0) sh[k][wid] = t;
  }
  __syncthreads();
  if (threadIdx.x < n) {
    const int k = threadIdx.x;
    double t = sh[k][0];
    for (int w = 1; w < nw; ++w) t = is_max ? fmax(t, sh[k][w]) : t + sh[k][w];
    fin.out[k] = t;
    if (k == 0 && fin.mode == FIN_CG_CHECK) {
      Scalars *sc = fin.sc;
      sc->cg_iters += 1;
      if (!(t > sc->rtol2 * sc->ff) || sc->cg_iters >= sc->cg_max) sc->cg_done = 1;
    } else if (k == 0 && fin.mode == FIN_RZ) {
      Scalars *sc = fin.sc;
      sc->beta = t / sc->rz;
      sc->rz = t;
    }
  }
  __syncthreads();
  if ((fin.mode == FIN_RZ_FLEX || fin.mode == FIN_RZ_SAFE) && threadIdx.x == 0) {
    // Polak-Ribiere: beta = r.(z_new - z_old) / rz_old, from the two sums above
    Scalars *sc = fin.sc;
    const double rzn = fin.out[0], rzo = fin.out[1];
    sc->beta = (rzn - rzo) / sc->rz;
    sc->rz = rzn;
    if (fin.mode == FIN_RZ_SAFE) {
      // a preconditioner that is not positive on this residual cannot be used
      const double zz = fin.out[2], bound = kSafeEps * sqrt(sc->rr * zz);
      if (!(rzn > bound) || !isfinite(rzn) || !isfinite(zz) || !isfinite(sc->beta)) {
        sc->nn_fallback = 1;
        sc->cg_done = 1;
      }
    }
  }
}

__global__ void finalize_kernel(const double *partials, int nparts, int n, Fin fin, const int *skip) {
  finalize_body(partials, nparts, n, fin, skip);
}
// one block per problem of a group
__global__ void finalize_group_kernel(int nparts, int n, GroupTab<double *> part, GroupTab<Fin> fin,
                                      GroupTab<const int *> skip) {
  finalize_body(part.v[blockIdx.x], nparts, n, fin.v[blockIdx.x], skip.v[blockIdx.x]);
}

hipError_t launch_finalize_group(hipStream_t s, int G, const Reducer *red, int nparts, int n, const Fin *fin,
                                 const int *const *skip) {
  if (G < 1 || G > kMaxGroup || n > kMaxRed) return hipErrorInvalidValue;
  GroupTab<double *> p{};
  GroupTab<Fin> f{};
  GroupTab<const int *> k{};
  for (int i = 0; i < G; ++i) {
    if (nparts > red[i].max_blocks) return hipErrorInvalidValue;
    p.v[i] = red[i].partials;
    f.v[i] = fin[i];
    k.v[i] = skip[i];
  }
  finalize_group_kernel<<<G, 256, 0, s>>>(nparts, n, p, f, k);
  return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t s, const Reducer &red, int nparts, int n, const Fin &fin,
                           const int *skip) {
  if (n > kMaxRed || nparts > red.max_blocks) return hipErrorInvalidValue;
  finalize_kernel<<<1, 256, 0, s>>>(red.partials, nparts, n, fin, skip);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// E32 (may be NULL): the single-precision copy, rounded from the FP64 value
__device__ __forceinline__ void simp_modulus_body(int64_t nel, const double *xphys, double E0, double Emin,
                                                  double penal, double scale, double *E, float *E32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  const double x = xphys[e];
  const double xp = (penal == 3.0) ? x * x * x : pow(x, penal);
  const double v = scale * (Emin + xp * (E0 - Emin));
  E[e] = v;
  if (E32) E32[e] = (float)v;
}
__global__ void simp_modulus_kernel(int64_t nel, const double *xphys, double E0, double Emin,
                                    double penal, double scale, double *E, float *E32) {
  simp_modulus_body(nel, xphys, E0, Emin, penal, scale, E, E32);
}
__global__ void simp_modulus_group_kernel(int64_t nel, GroupTab<ModulusArgs> t) {
  const ModulusArgs &a = t.v[blockIdx.z];
  simp_modulus_body(nel, a.xphys, a.E0, a.Emin, a.penal, 1.0, a.E, a.E32);
}

hipError_t launch_simp_modulus(hipStream_t s, int64_t nel, const double *xphys, double E0,
                               double Emin, double penal, double scale, double *E, float *E32) {
  const int bs = 256;
  simp_modulus_kernel<<<(unsigned)((nel + bs - 1) / bs), bs, 0, s>>>(nel, xphys, E0, Emin, penal,
                                                                    scale, E, E32);
  return hipGetLastError();
}

// Coarse modulus = 2 * mean of the 8 fine children (missing children are 0):
// the factor 2 is the stiffness scaling of an element of twice the edge length.
__device__ __forceinline__ void coarsen_moduli_body(Grid gf, Grid gc, const double *Ef, double *Ec, float *Ec32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= gc.nel()) return;
  const int I = (int)(e % gc.nx);
  const int J = (int)((e / gc.nx) % gc.ny);
  const int K = (int)(e / ((int64_t)gc.nx * gc.ny));
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), k = 2 * K + (c >> 2);
    if (i < gf.nx && j < gf.ny && k < gf.nz) s += Ef[i + (int64_t)gf.nx * (j + (int64_t)gf.ny * k)];
  }
  Ec[e] = 0.25 * s;
  if (Ec32) Ec32[e] = (float)(0.25 * s);
}
__global__ void coarsen_moduli_kernel(Grid gf, Grid gc, const double *Ef, double *Ec, float *Ec32) {
  coarsen_moduli_body(gf, gc, Ef, Ec, Ec32);
}
__global__ void coarsen_moduli_group_kernel(Grid gf, Grid gc, GroupTab<const double *> Ef, GroupTab<double *> Ec,
                                            GroupTab<float *> Ec32) {
  coarsen_moduli_body(gf, gc, Ef.v[blockIdx.z], Ec.v[blockIdx.z], Ec32.v[blockIdx.z]);
}

hipError_t launch_coarsen_moduli(hipStream_t s, Grid gf, Grid gc, const double *Ef, double *Ec, float *Ec32) {
  const int bs = 256;
  coarsen_moduli_kernel<<<(unsigned)((gc.nel() + bs - 1) / bs), bs, 0, s>>>(gf, gc, Ef, Ec, Ec32);
  return hipGetLastError();
}

// inverse Jacobi diagonal: 1 / sum_{e around i} E_e KE[(3 li + c),(3 li + c)]; 0 on fixed dofs
__device__ __forceinline__ void diag_body(Grid g, const double *E, const Kappa &kap, const uint8_t *fixed,
                                          double *dinv, float *dinv32) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.nnodes()) return;
  const int i = (int)(n % g.NX());
  const int j = (int)((n / g.NX()) % g.NY());
  const int k = (int)(n / ((int64_t)g.NX() * g.NY()));
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
    const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
    if (ei < 0 || ei >= g.nx || ej < 0 || ej >= g.ny || ek < 0 || ek >= g.nz) continue;
    const double Ee = E[ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek)];
    const int li = corner_of(1 - ex, 1 - ey, 1 - ez);
    d0 += Ee * TOPO_KE(kap, 3 * li + 0, 3 * li + 0);
    d1 += Ee * TOPO_KE(kap, 3 * li + 1, 3 * li + 1);
    d2 += Ee * TOPO_KE(kap, 3 * li + 2, 3 * li + 2);
  }
  const uint8_t fx = fixed[n];
  const double v0 = (fx & 1) ? 0.0 : 1.0 / d0, v1 = (fx & 2) ? 0.0 : 1.0 / d1, v2 = (fx & 4) ? 0.0 : 1.0 / d2;
  dinv[3 * n + 0] = v0;
  dinv[3 * n + 1] = v1;
  dinv[3 * n + 2] = v2;
  if (dinv32) {
    dinv32[3 * n + 0] = (float)v0;
    dinv32[3 * n + 1] = (float)v1;
    dinv32[3 * n + 2] = (float)v2;
  }
}
__global__ void diag_kernel(Grid g, const double *E, Kappa kap, const uint8_t *fixed, double *dinv,
                            float *dinv32) {
  diag_body(g, E, kap, fixed, dinv, dinv32);
}
__global__ void diag_group_kernel(Grid g, GroupTab<DiagArgs> t) {
  const DiagArgs &a = t.v[blockIdx.z];
  diag_body(g, a.E, a.kap, a.fixed, a.dinv, a.dinv32);
}

hipError_t launch_diag(hipStream_t s, Grid g, const double *E, const Kappa &kap,
                       const uint8_t *fixed, double *dinv, float *dinv32) {
  const int bs = 256;
  diag_kernel<<<(unsigned)((g.nnodes() + bs - 1) / bs), bs, 0, s>>>(g, E, kap, fixed, dinv, dinv32);
  return hipGetLastError();
}


// grouped operator set-up (problems of equal grids)
hipError_t launch_simp_modulus_group(hipStream_t s, int G, int64_t nel, const ModulusArgs *a) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  const int bs = 256;
  simp_modulus_group_kernel<<<dim3((unsigned)((nel + bs - 1) / bs), 1, G), bs, 0, s>>>(nel, group_tab(G, a));
  return hipGetLastError();
}
hipError_t launch_coarsen_moduli_group(hipStream_t s, int G, Grid gf, Grid gc, const double *const *Ef,
                                       double *const *Ec, float *const *Ec32) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  const int bs = 256;
  coarsen_moduli_group_kernel<<<dim3((unsigned)((gc.nel() + bs - 1) / bs), 1, G), bs, 0, s>>>(
      gf, gc, group_tab(G, Ef), group_tab(G, Ec), group_tab(G, Ec32));
  return hipGetLastError();
}
hipError_t launch_diag_group(hipStream_t s, int G, Grid g, const DiagArgs *a) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  const int bs = 256;
  diag_group_kernel<<<dim3((unsigned)((g.nnodes() + bs - 1) / bs), 1, G), bs, 0, s>>>(g, group_tab(G, a));
  return hipGetLastError();
}

}  // namespace topo
