// Element-column stiffness operator: y = K u with K = sum_e E_e KE (the Finite
// Element Analysis section), computed element by element in the per-axis
// sum/difference basis of the element's corners, where KE splits into eight
// parity blocks with 8 distinct entries (ke_code.h).  Per element that is
//   h = H u_e        (sum/difference passes: additions only),
//   g = E_e M h      (21 multiply-adds with the E-scaled block entries),
//   y_e = H^T g      (sum/difference passes),
// instead of the 576 multiply-adds of the 24 x 24 element mat-vec.
//
// Work decomposition: a block owns a tile of (TX-1) x (TY-1) node columns and a
// slab of KZ node planes.  Its TX x TY threads each own one element column
// (i0-1+tx, j0-1+ty) and march up through its element layers.  A node plane is
// transformed in x and y once, when it is loaded; the z pass then forms the
// element's modes from the planes below and above.  Node plane L collects the
// top face of element layer L-1 and the bottom face of layer L, which are added
// while still in the xy basis and transformed back once per plane.  The four
// element columns around a node column hand their corner contributions over
// through LDS and are summed in a fixed order (deterministic, no atomics); the
// thread whose element has the node as its (+x, +y) corner finishes the node
// with the fused epilogue.  The tile's last row and column of threads compute
// halo elements only.
//
// Fixed dofs: inputs are required to be zero there; see ku_epilogue.h.
#include <algorithm>

#include "internal.h"
#include "ke_code.h"
#include "ku_epilogue.h"
#include "reduce_dev.h"

namespace topo {

// Without the one-layer-ahead loads: at least 3 waves per SIMD (at most 168
// VGPRs), so a 160x80x80 launch runs in one round (3 blocks of 256 threads per
// CU); with them the register budget is left to the compiler.
template <int EPI, int KZ, int TX, int TY, bool PF, typename T>
__device__ __forceinline__ void ku_hada_body(const KuArgsT<T> &a, const HadaW<T> &hw, int tiles_x, int tiles_xy,
                                             double *partials) {
  if (a.skip && *a.skip) return;
  if constexpr (EPI == KU_RES0 && TX * TY == 256) {
    if (a.chk_parts && cg_stop_in_block(a.chk_parts, a.chk_n, a.chk_sc)) return;
  }
  constexpr int NT = TX * TY;
  // corner contributions (0,0), (1,0), (0,1) of every thread's element column,
  // double-buffered over node planes so one barrier per plane suffices
  __shared__ T xch[2][3][3][NT];
  const Grid g = a.g;
  const int NX = g.NX(), NY = g.NY(), NZ = g.NZ();
  const int64_t plane = (int64_t)NX * NY;
  const int tile = xcd_tile(linear_block(), gridDim.x * gridDim.y);
  const int txy = tile % tiles_xy, slab = tile / tiles_xy;
  const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
  const int ie = (txy % tiles_x) * (TX - 1) - 1 + tx;
  const int je = (txy / tiles_x) * (TY - 1) - 1 + ty;
  const int k0 = slab * KZ, k1 = min(k0 + KZ, NZ);
  const bool elem_xy = ie >= 0 && ie < g.nx && je >= 0 && je < g.ny;
  const bool owner = tx < TX - 1 && ty < TY - 1 && ie + 1 <= g.nx && je + 1 <= g.ny;
  constexpr bool kScaled = EpiTraits<EPI>::scaled_operand;
  const T *__restrict__ u = kScaled ? a.b : a.u;
  const T *__restrict__ dinv = a.dinv;

  // Per-lane parts of the addresses, clamped into the grid, so every load is
  // unconditional and in bounds: corner q of the element column sits at node
  // column off[q] of every plane.  A clamped corner or plane only feeds elements
  // outside the grid, whose modulus is taken as 0, so its (finite) values add
  // exact zeros and need no masking.
  uint32_t off[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ci = min(max(ie + (q & 1), 0), g.nx), cj = min(max(je + (q >> 1), 0), g.ny);
    off[q] = 3u * (uint32_t)(cj * NX + ci);
  }
  const uint32_t eoff = (uint32_t)(min(max(je, 0), g.ny - 1) * g.nx + min(max(ie, 0), g.nx - 1));
  const uint32_t own = (uint32_t)((je + 1) * NX + (ie + 1));  // the owned node column (owners only)

  // the operand at the element column's 4 corners on node plane kp; the scaled
  // epilogues also keep b and dinv of corner (1, 1) for their own update
  auto load_raw = [&](int kp, T(&v)[3][4], T(&bd)[2][3]) {
    const int64_t pbase = 3 * (int64_t)min(max(kp, 0), g.nz) * plane;  // uniform
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T *__restrict__ up = u + pbase + off[q];
      const T *__restrict__ dp = dinv + pbase + off[q];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if constexpr (kScaled) {
          const T bv = up[c], dv = dp[c];
          v[c][q] = bv * dv * a.s0;
          if (q == 3) {
            bd[0][c] = bv;
            bd[1][c] = dv;
          }
        } else {
          v[c][q] = up[c];
        }
      }
    }
  };
  // x/y modes of a plane; self gets the operand at corner (1, 1), the node this
  // thread may own
  auto modes = [&](const T(&v)[3][4], T(&m)[3][4], T(&self)[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      self[c] = v[c][3];
      xy_pass(v[c], m[c]);
    }
  };

  // modulus of element layer L of this column, raw; zeroed outside the grid only
  // where it is used (E_at), so a load issued ahead is not waited for at once
  auto load_E = [&](int L) { return a.E[(int64_t)min(max(L, 0), g.nz - 1) * g.nx * g.ny + eoff]; };
  auto E_at = [&](int L, T Eraw) { return (elem_xy && L >= 0 && L < g.nz) ? Eraw : T(0); };

  // Memory order within a layer (vector loads retire in issue order, so a wait
  // for one load waits for every older one): first the epilogue inputs of node
  // plane L, then (PF) the next plane and modulus, which stay in flight through
  // this layer's arithmetic and barrier (the barrier waits for LDS traffic only).
  double dotv[2] = {0.0, 0.0};
  T Pb[3][4], selfb[3];  // node plane L (xy modes) and the operand at the owned node
  T bdb[2][3];           // scaled epilogues: b and dinv at the owned node of plane L
  T ytp[3][4];           // top face of element layer L-1 (xy modes)
  T nxt[3][4];           // PF: node plane L+1 and the modulus of layer L, one layer ahead
  T bdn[2][3];
  T Enxt = T(0);
  {
    T v[3][4];
    load_raw(k0 - 1, v, bdb);
    modes(v, Pb, selfb);
  }
  if constexpr (PF) {
    load_raw(k0, nxt, bdn);
    Enxt = load_E(k0 - 1);
  }
#pragma unroll
  for (int q = 0; q <= KZ; ++q) {
    const int L = k0 - 1 + q;  // element layer between node planes L and L+1
    if (L >= k1) break;
    const int64_t nL = (int64_t)L * plane + own;
    EpiIn<T> in;
    if (q > 0 && owner) {
      ku_epi_load<EPI, kScaled>(a, nL, dinv, in);
      if constexpr (kScaled) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          in.b[c] = bdb[0][c];
          in.d[c] = bdb[1][c];
        }
      }
    }
    T Pt[3][4], selft[3], bdt[2][3];
    T Ee;
    if constexpr (PF) {
      T cur[3][4];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int r = 0; r < 4; ++r) cur[c][r] = nxt[c][r];
        bdt[0][c] = bdn[0][c];
        bdt[1][c] = bdn[1][c];
      }
      Ee = E_at(L, Enxt);
      if (q < KZ && L + 1 < k1) {
        load_raw(L + 2, nxt, bdn);
        Enxt = load_E(L + 1);
      }
      modes(cur, Pt, selft);
    } else {
      T v[3][4];
      load_raw(L + 1, v, bdt);
      Ee = E_at(L, load_E(L));
      modes(v, Pt, selft);
    }
    T w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = Ee * hw.w[k];
    // element modes h[c][s], s = q + 4 z (h[c][0], the rigid translations, is not needed)
    T h[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        h[c][r] = Pb[c][r] + Pt[c][r];
        h[c][r + 4] = Pb[c][r] - Pt[c][r];
      }
    T gm[3][8];
    hada_blocks(w, h, gm);
    // back in z: bottom face (node plane L) and top face (node plane L+1), xy modes
    if (q > 0) {  // node plane L is owned by this slab
      T cn[3][4];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T acc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = ytp[c][r] + (gm[c][r] + gm[c][r + 4]);
        xy_pass(acc, cn[c]);
      }
      T(&buf)[3][3][NT] = xch[q & 1];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        buf[0][c][tid] = cn[c][0];
        buf[1][c][tid] = cn[c][1];
        buf[2][c][tid] = cn[c][2];
      }
      __syncthreads();
      if (owner) {
        // elements (ie, je), (ie+1, je), (ie, je+1), (ie+1, je+1) around node (ie+1, je+1)
        T Au[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
          Au[c] = ((cn[c][3] + buf[2][c][tid + 1]) + buf[1][c][tid + TX]) + buf[0][c][tid + TX + 1];
        ku_epi_finish<EPI>(a, nL, in, selfb, Au, dotv);
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        ytp[c][r] = gm[c][r] - gm[c][r + 4];
        Pb[c][r] = Pt[c][r];
      }
      selfb[c] = selft[c];
      bdb[0][c] = bdt[0][c];
      bdb[1][c] = bdt[1][c];
    }
  }
  ku_block_reduce<EPI>(a, dotv, partials);
}

// Staged variant of the same kernel.  The block loads each node plane of its
// tile once, (TX+1)(TY+1) nodes spread evenly over its threads instead of four
// corners per thread, into registers two planes ahead of use, and hands it to
// the element columns through LDS (double-buffered; the barrier that publishes
// a plane is the one the corner exchange already needs); the moduli are loaded
// two layers and the epilogue inputs one layer ahead as well.  A plane's loads
// thus stay in flight through one layer's arithmetic and barrier, with a third
// of the load instructions.  Same arithmetic in the same order: bit-identical to
// the other shapes.
template <int EPI, int KZ, int TX, int TY, typename T>
__device__ __forceinline__ void ku_hada_lds_body(const KuArgsT<T> &a, const HadaW<T> &hw, int tiles_x,
                                                 int tiles_xy, double *partials) {
  if (a.skip && *a.skip) return;
  if constexpr (EPI == KU_RES0 && TX * TY == 256) {
    if (a.chk_parts && cg_stop_in_block(a.chk_parts, a.chk_n, a.chk_sc)) return;
  }
  constexpr int NT = TX * TY;
  constexpr int NX1 = TX + 1;
  constexpr int NV = NX1 * (TY + 1) * 3;  // values of one node plane of the tile
  constexpr int SL = (NV + NT - 1) / NT;  // of which each thread loads SL
  __shared__ T xch[2][3][3][NT];
  __shared__ T stage[2][NV];
  const Grid g = a.g;
  const int NX = g.NX(), NY = g.NY(), NZ = g.NZ();
  const int64_t plane = (int64_t)NX * NY;
  const int tile = xcd_tile(linear_block(), gridDim.x * gridDim.y);
  const int txy = tile % tiles_xy, slab = tile / tiles_xy;
  const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
  const int i0 = (txy % tiles_x) * (TX - 1) - 1, j0 = (txy / tiles_x) * (TY - 1) - 1;
  const int ie = i0 + tx, je = j0 + ty;
  const int k0 = slab * KZ, k1 = min(k0 + KZ, NZ);
  const bool elem_xy = ie >= 0 && ie < g.nx && je >= 0 && je < g.ny;
  const bool owner = tx < TX - 1 && ty < TY - 1 && ie + 1 <= g.nx && je + 1 <= g.ny;
  constexpr bool kScaled = EpiTraits<EPI>::scaled_operand;
  const T *__restrict__ u = kScaled ? a.b : a.u;
  const T *__restrict__ dinv = a.dinv;

  // value d = tid + s NT of the staged plane: node (d/3 mod NX1, d/3 div NX1) of
  // the tile, component d mod 3; clamped into the grid as in the other shapes
  // (clamped nodes only feed elements of modulus 0)
  uint32_t soff[SL];
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    const int d = min(tid + s * NT, NV - 1), nn = d / 3, c = d - 3 * nn;
    const int ci = min(max(i0 + nn % NX1, 0), g.nx), cj = min(max(j0 + nn / NX1, 0), g.ny);
    soff[s] = 3u * (uint32_t)(cj * NX + ci) + (uint32_t)c;
  }
  auto stage_load = [&](int kp, T(&r)[SL], T(&r2)[SL]) {
    const int64_t pbase = 3 * (int64_t)min(max(kp, 0), g.nz) * plane;  // uniform
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      r[s] = u[pbase + soff[s]];
      if constexpr (kScaled) r2[s] = dinv[pbase + soff[s]];
    }
  };
  auto stage_store = [&](T *buf, const T(&r)[SL], const T(&r2)[SL]) {
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int d = tid + s * NT;
      if (s < SL - 1 || d < NV) buf[d] = kScaled ? r[s] * r2[s] * a.s0 : r[s];
    }
  };
  // x/y modes of the staged plane at this thread's element column, and the
  // operand at corner (1, 1)
  auto modes_lds = [&](const T *buf, T(&m)[3][4], T(&self)[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = buf[3 * ((ty + (q >> 1)) * NX1 + tx + (q & 1)) + c];
      self[c] = v[3];
      xy_pass(v, m[c]);
    }
  };
  const uint32_t eoff = (uint32_t)(min(max(je, 0), g.ny - 1) * g.nx + min(max(ie, 0), g.nx - 1));
  const uint32_t own = (uint32_t)((je + 1) * NX + (ie + 1));
  // modulus of element layer L, loaded ahead of use: the value is taken raw and
  // zeroed outside the grid only where it is used, so no wait for it comes early
  auto load_E = [&](int L) { return a.E[(int64_t)min(max(L, 0), g.nz - 1) * g.nx * g.ny + eoff]; };

  // node plane k0-1+m is staged in stage[m & 1] and loaded into rg[m & 1]
  T rg[2][SL], rd[2][SL];
  double dotv[2] = {0.0, 0.0};
  T Pb[3][4], selfb[3], ytp[3][4];
  T Ecur = load_E(k0 - 1), Enx = load_E(k0);
  EpiIn<T> in_nx;  // epilogue inputs of the next node plane, loaded one layer ahead
  stage_load(k0 - 1, rg[0], rd[0]);
  stage_load(k0, rg[1], rd[1]);
  stage_store(stage[0], rg[0], rd[0]);
  stage_load(k0 + 1, rg[0], rd[0]);
  __syncthreads();
  modes_lds(stage[0], Pb, selfb);
  stage_store(stage[1], rg[1], rd[1]);
  __syncthreads();  // plane k0 staged, and every read of plane k0-1 done
#pragma unroll
  for (int q = 0; q <= KZ; ++q) {
    const int L = k0 - 1 + q;  // element layer between node planes L and L+1
    if (L >= k1) break;
    const int64_t nL = (int64_t)L * plane + own;
    // issue order: modulus two layers ahead, the next plane's epilogue inputs,
    // then the node plane three ahead, so every wait below leaves the loads of
    // this layer in flight
    const T Ee = (elem_xy && L >= 0 && L < g.nz) ? Ecur : T(0);
    Ecur = Enx;
    if (q + 2 <= KZ) Enx = load_E(L + 2);
    const EpiIn<T> in = in_nx;
    if (q + 1 <= KZ && L + 1 < k1 && owner) ku_epi_load<EPI, false>(a, nL + plane, dinv, in_nx);
    if (q + 3 <= KZ + 1) stage_load(L + 3, rg[(q + 1) & 1], rd[(q + 1) & 1]);
    // node plane L+2 (loaded one layer ago) into the buffer whose plane (L) was
    // last read before the previous barrier; published by this layer's barrier
    if (q + 2 <= KZ + 1) stage_store(stage[q & 1], rg[q & 1], rd[q & 1]);
    T Pt[3][4], selft[3];
    modes_lds(stage[(q + 1) & 1], Pt, selft);
    T w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = Ee * hw.w[k];
    T h[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        h[c][r] = Pb[c][r] + Pt[c][r];
        h[c][r + 4] = Pb[c][r] - Pt[c][r];
      }
    T gm[3][8];
    hada_blocks(w, h, gm);
    T cn[3][4];
    if (q > 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T acc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = ytp[c][r] + (gm[c][r] + gm[c][r + 4]);
        xy_pass(acc, cn[c]);
      }
      T(&buf)[3][3][NT] = xch[q & 1];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        buf[0][c][tid] = cn[c][0];
        buf[1][c][tid] = cn[c][1];
        buf[2][c][tid] = cn[c][2];
      }
    }
    __syncthreads();
    if (q > 0 && owner) {
      const T(&buf)[3][3][NT] = xch[q & 1];
      T Au[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        Au[c] = ((cn[c][3] + buf[2][c][tid + 1]) + buf[1][c][tid + TX]) + buf[0][c][tid + TX + 1];
      ku_epi_finish<EPI>(a, nL, in, selfb, Au, dotv);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        ytp[c][r] = gm[c][r] - gm[c][r + 4];
        Pb[c][r] = Pt[c][r];
      }
      selfb[c] = selft[c];
    }
  }
  ku_block_reduce<EPI>(a, dotv, partials);
}

// Kernels: one problem per launch, or a group of problems of the same grid
// (blockIdx.z picks the problem's arguments and partials).
template <int EPI, int KZ, int TX, int TY, bool PF, typename T>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(PF ? 1 : 3))) void ku_hada_kernel(
    KuArgsT<T> a, HadaW<T> hw, int tiles_x, int tiles_xy, double *partials) {
  ku_hada_body<EPI, KZ, TX, TY, PF, T>(a, hw, tiles_x, tiles_xy, partials);
}
template <int EPI, int KZ, int TX, int TY, bool PF, typename T>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(PF ? 1 : 3))) void ku_hada_group_kernel(
    GroupTab<KuArgsT<T>> t, GroupTab<double *> part, HadaW<T> hw, int tiles_x, int tiles_xy) {
  ku_hada_body<EPI, KZ, TX, TY, PF, T>(t.v[blockIdx.z], hw, tiles_x, tiles_xy, part.v[blockIdx.z]);
}
template <int EPI, int KZ, int TX, int TY, typename T>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(3))) void ku_hada_lds_kernel(
    KuArgsT<T> a, HadaW<T> hw, int tiles_x, int tiles_xy, double *partials) {
  ku_hada_lds_body<EPI, KZ, TX, TY, T>(a, hw, tiles_x, tiles_xy, partials);
}
template <int EPI, int KZ, int TX, int TY, typename T>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(3))) void ku_hada_lds_group_kernel(
    GroupTab<KuArgsT<T>> t, GroupTab<double *> part, HadaW<T> hw, int tiles_x, int tiles_xy) {
  ku_hada_lds_body<EPI, KZ, TX, TY, T>(t.v[blockIdx.z], hw, tiles_x, tiles_xy, part.v[blockIdx.z]);
}

template <int KZ, int TX, int TY>
struct HadaShape {
  static int tiles_x(const Grid &g) { return (g.NX() + TX - 2) / (TX - 1); }
  static int tiles_y(const Grid &g) { return (g.NY() + TY - 2) / (TY - 1); }
  static int64_t blocks(const Grid &g) {
    return (int64_t)tiles_x(g) * tiles_y(g) * ((g.NZ() + KZ - 1) / KZ);
  }
};

// VAR: 0 plain, 1 next plane loaded one layer ahead, 2 staged through LDS
template <int KZ, int TX, int TY, int VAR, typename T>
static hipError_t launch_hada_shape(hipStream_t s, KuEpi epi, const KuArgsT<T> &a, const KappaT<T> &kap,
                                    const Reducer &red, int *nparts_out) {
  using S = HadaShape<KZ, TX, TY>;
  const int tx = S::tiles_x(a.g), txy = tx * S::tiles_y(a.g);
  const int64_t nb = S::blocks(a.g);
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  *nparts_out = (int)nb;
  if (ku_reduces(epi, a) && nb > red.max_blocks) return hipErrorInvalidValue;
  const HadaW<T> hw = hada_work(kap);
  const dim3 grid((unsigned)nb);
#define TOPO_KU_CASE(E)                                                                                  \
  case E:                                                                                                \
    if constexpr (VAR == 2)                                                                              \
      ku_hada_lds_kernel<E, KZ, TX, TY, T><<<grid, TX * TY, 0, s>>>(a, hw, tx, txy, red.partials);       \
    else                                                                                                 \
      ku_hada_kernel<E, KZ, TX, TY, VAR == 1, T><<<grid, TX * TY, 0, s>>>(a, hw, tx, txy, red.partials); \
    break;
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

template <int KZ, int TX, int TY, int VAR, typename T>
static hipError_t launch_hada_shape_group(hipStream_t s, KuEpi epi, int G, const KuArgsT<T> *a,
                                          const KappaT<T> &kap, const Reducer *red, int *nparts_out) {
  using S = HadaShape<KZ, TX, TY>;
  const int tx = S::tiles_x(a[0].g), txy = tx * S::tiles_y(a[0].g);
  const int64_t nb = S::blocks(a[0].g);
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  *nparts_out = (int)nb;
  GroupTab<KuArgsT<T>> t{};
  GroupTab<double *> part{};
  for (int i = 0; i < G; ++i) {
    if (a[i].g.nx != a[0].g.nx || a[i].g.ny != a[0].g.ny || a[i].g.nz != a[0].g.nz) return hipErrorInvalidValue;
    if (ku_reduces(epi, a[i]) && nb > red[i].max_blocks) return hipErrorInvalidValue;
    t.v[i] = a[i];
    part.v[i] = red[i].partials;
  }
  const HadaW<T> hw = hada_work(kap);
  const dim3 grid((unsigned)nb, 1, (unsigned)G);
#define TOPO_KU_CASE(E)                                                                             \
  case E:                                                                                           \
    if constexpr (VAR == 2)                                                                         \
      ku_hada_lds_group_kernel<E, KZ, TX, TY, T><<<grid, TX * TY, 0, s>>>(t, part, hw, tx, txy);    \
    else                                                                                            \
      ku_hada_group_kernel<E, KZ, TX, TY, VAR == 1, T><<<grid, TX * TY, 0, s>>>(t, part, hw, tx, txy); \
    break;
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

// element-column shapes (index relative to kKuShapeHada): KZ x TX x TY, and
// how node planes are loaded (VAR above).  Every shape runs the same arithmetic
// in the same order (a node always sums its four element columns in the same
// order), so they give bit-identical results.
#define TOPO_HADA_SHAPES(X) \
  X(0, 8, 32, 8, 0)         \
  X(1, 8, 16, 16, 0)        \
  X(2, 4, 16, 8, 1)         \
  X(3, 2, 8, 8, 1)          \
  X(4, 1, 8, 8, 0)          \
  X(5, 8, 32, 8, 1)         \
  X(6, 8, 16, 16, 1)        \
  X(7, 8, 32, 8, 2)         \
  X(8, 8, 16, 16, 2)

int ku_hada_block_threads(int which) {
  switch (which) {
#define TOPO_HADA_THREADS(I, KZ, TX, TY, VAR) \
  case I: return TX * TY;
    TOPO_HADA_SHAPES(TOPO_HADA_THREADS)
#undef TOPO_HADA_THREADS
    default: return 0;
  }
}

template <typename T>
hipError_t launch_ku_hada(hipStream_t s, KuEpi epi, const KuArgsT<T> &a, const KappaT<T> &kap,
                          const Reducer &red, int which, int *nparts) {
  if (a.chk_parts && (epi != KU_RES0 || ku_hada_block_threads(which) != 256 || a.chk_n < 1 || !a.chk_sc))
    return hipErrorInvalidValue;
  switch (which) {
#define TOPO_HADA_LAUNCH(I, KZ, TX, TY, VAR) \
  case I: return launch_hada_shape<KZ, TX, TY, VAR>(s, epi, a, kap, red, nparts);
    TOPO_HADA_SHAPES(TOPO_HADA_LAUNCH)
#undef TOPO_HADA_LAUNCH
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_ku_hada<double>(hipStream_t, KuEpi, const KuArgsT<double> &,
                                           const KappaT<double> &, const Reducer &, int, int *);
template hipError_t launch_ku_hada<float>(hipStream_t, KuEpi, const KuArgsT<float> &,
                                          const KappaT<float> &, const Reducer &, int, int *);

template <typename T>
hipError_t launch_ku_hada_group(hipStream_t s, KuEpi epi, int G, const KuArgsT<T> *a, const KappaT<T> &kap,
                                const Reducer *red, int which, int *nparts) {
  switch (which) {
#define TOPO_HADA_LAUNCH(I, KZ, TX, TY, VAR) \
  case I: return launch_hada_shape_group<KZ, TX, TY, VAR>(s, epi, G, a, kap, red, nparts);
    TOPO_HADA_SHAPES(TOPO_HADA_LAUNCH)
#undef TOPO_HADA_LAUNCH
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_ku_hada_group<double>(hipStream_t, KuEpi, int, const KuArgsT<double> *,
                                                 const KappaT<double> &, const Reducer *, int, int *);
template hipError_t launch_ku_hada_group<float>(hipStream_t, KuEpi, int, const KuArgsT<float> *,
                                                const KappaT<float> &, const Reducer *, int, int *);

int64_t ku_hada_max_blocks(const Grid &g) {
  int64_t m = 0;
#define TOPO_HADA_BLOCKS(I, KZ, TX, TY, VAR) m = std::max<int64_t>(m, HadaShape<KZ, TX, TY>::blocks(g));
  TOPO_HADA_SHAPES(TOPO_HADA_BLOCKS)
#undef TOPO_HADA_BLOCKS
  return m;
}

}  // namespace topo
