// Matrix-core variant of the single-precision K.u (the smoothing passes of the
// mixed-precision multigrid preconditioner): per element layer, the products
// KE u_e of all elements of a block's tile are one dense contraction
// Y[24][elements] = KE[24][24] U[24][elements] on the gfx950 matrix cores, in
// FP32 (v_mfma_f32_16x16x4_f32) or with BF16 operands (v_mfma_f32_16x16x32_bf16),
// accumulating in FP32.
//
// A block owns a 16 x 16 tile of node columns and marches up KZ node planes.
// The node planes it touches (tile plus a one-node halo) are staged in LDS in a
// ring of three (the next plane is fetched while the current layer computes).
// For element layer L, the 17 x 17 elements around the tile form 19 B-operand
// tiles of 16 columns; each column (element) gathers its 24 dofs from the
// planes L and L+1 in LDS.  The products, scaled by the element moduli, go to
// LDS; then every thread gathers, for its own node column, the bottom-face rows
// of the 4 elements of layer L (finishing node (i, j, L)) and their top-face
// rows (starting node (i, j, L+1)), so each node is summed in a fixed order by
// one thread and the result is deterministic.  The epilogues are those of the
// vector-unit kernel (kernels_ku.hip).
//
// Instruction layouts (one wave), with k the contraction index:
//   16x16x4 f32:  A lane l = row l%16, k = l/16;   B lane l = column l%16, k = l/16
//   16x16x32 bf16: A lane l = row l%16, k = 8(l/16)..+7; B lane l = column l%16, same k
//   D (both):     lane l = column l%16, rows 4(l/16)..+3
#include "internal.h"
#include "reduce_dev.h"

namespace topo {

namespace {
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTile = 16;                  // node columns per block side
constexpr int kPW = kTile + 2;             // LDS plane row length (one halo node each side)
constexpr int kPN = kPW * kPW;             // nodes per LDS plane
constexpr int kEW = kTile + 1;             // elements per tile row
constexpr int kNE = kEW * kEW;             // elements per layer
constexpr int kNT = (kNE + 15) / 16;       // 16-column operand tiles per layer
constexpr int kYP = 25;                    // LDS row pitch of an element's 24 products
constexpr int kLoadsPerThread = (3 * kPN + 255) / 256;
}  // namespace

template <int EPI, bool BF16, int KZ>
__global__ __launch_bounds__(256) void ku_mfma_kernel(KuArgsT<float> a, const float *__restrict__ KEm,
                                                      const __bf16 *__restrict__ KEb) {
  if (a.skip && *a.skip) return;
  __shared__ float Up[3][3 * kPN];
  __shared__ float Y[kNT * 16 * kYP];
  const Grid g = a.g;
  const int NX = g.NX(), NY = g.NY(), NZ = g.NZ();
  const int tilesx = (NX + kTile - 1) / kTile;
  const int tile = xcd_tile(linear_block(), gridDim.x * gridDim.y);
  const int txy = tile % gridDim.x, tz = tile / gridDim.x;
  const int x0 = (txy % tilesx) * kTile, y0 = (txy / tilesx) * kTile;
  const int k0 = tz * KZ, k1 = min(k0 + KZ, NZ);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ti = tid % kTile, tj = tid / kTile;
  const int i = x0 + ti, j = y0 + tj;
  const bool own = i < NX && j < NY;
  constexpr bool kScaled = EPI == KU_RES0 || EPI == KU_CHEB0;
  const float *__restrict__ u = kScaled ? a.b : a.u;
  const int64_t plane = (int64_t)NX * NY;

  // A operand (KE, zero-padded to 32 rows) in registers for the whole launch;
  // the B-operand LDS offsets of this lane's k values
  float Af[2][6];
  bf16x8 Ab[2];
  int boff[8];
  bool bup[8], bok[8];
  if constexpr (!BF16) {
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int s = 0; s < 6; ++s) Af[m][s] = KEm[(16 * m + (lane & 15)) * 24 + (lane >> 4) + 4 * s];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int k = (lane >> 4) + 4 * s, b = k / 3, d = k % 3;
      boff[s] = 3 * (cx(b) + kPW * cy(b)) + d;
      bup[s] = cz(b) != 0;
      bok[s] = true;
    }
  } else {
#pragma unroll
    for (int m = 0; m < 2; ++m) Ab[m] = *reinterpret_cast<const bf16x8 *>(&KEb[(16 * m + (lane & 15)) * 32 + 8 * (lane >> 4)]);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = 8 * (lane >> 4) + q, b = min(k, 23) / 3, d = min(k, 23) % 3;
      boff[q] = 3 * (cx(b) + kPW * cy(b)) + d;
      bup[q] = cz(b) != 0;
      bok[q] = k < 24;
    }
  }

  // plane kp of the operand (tile plus halo, zero outside the grid)
  float pre[kLoadsPerThread];
  auto fetch = [&](int kp) {
#pragma unroll
    for (int r = 0; r < kLoadsPerThread; ++r) {
      const int idx = tid + 256 * r;
      float v = 0.0f;
      if (idx < 3 * kPN && kp >= 0 && kp < NZ) {
        const int nl = idx / 3, c = idx % 3;
        const int gi = x0 - 1 + nl % kPW, gj = y0 - 1 + nl / kPW;
        if (gi >= 0 && gi < NX && gj >= 0 && gj < NY) {
          const int64_t dof = 3 * ((int64_t)kp * plane + (int64_t)gj * NX + gi) + c;
          v = kScaled ? u[dof] * a.dinv[dof] * a.s0 : u[dof];
        }
      }
      pre[r] = v;
    }
  };
  auto store = [&](int slot) {
#pragma unroll
    for (int r = 0; r < kLoadsPerThread; ++r) {
      const int idx = tid + 256 * r;
      if (idx < 3 * kPN) Up[slot][idx] = pre[r];
    }
  };

  fetch(k0 - 1);
  store(0);
  fetch(k0);
  store(1);
  __syncthreads();

  float top0 = 0.0f, top1 = 0.0f, top2 = 0.0f;  // node (i, j, L+1) so far
  double dotv = 0.0;
  int sl = 0;  // ring slot of plane L
  for (int L = k0 - 1; L < k1; ++L) {
    const int sl1 = sl == 2 ? 0 : sl + 1, sl2 = sl1 == 2 ? 0 : sl1 + 1;
    const bool more = L + 2 <= k1;
    if (more) fetch(L + 2);
    // ---- element products of layer L
    const bool layer_ok = L >= 0 && L < g.nz;
    for (int t = wave; t < kNT; t += 4) {
      const int el = 16 * t + (lane & 15);
      const int eli = el % kEW, elj = el / kEW;
      const int ei = x0 - 1 + eli, ej = y0 - 1 + elj;
      const bool eok = layer_ok && el < kNE && ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny;
      const int nb = 3 * (eli + kPW * elj);  // LDS offset of the element's corner 0
      // every lane takes part in the (wave-wide) matrix instructions; padding
      // columns (el >= kNE) feed zeros
      const bool col_ok = el < kNE;
      f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
      if constexpr (!BF16) {
#pragma unroll
        for (int s = 0; s < 6; ++s) {
          const float v = Up[bup[s] ? sl1 : sl][col_ok ? nb + boff[s] : 0];
          const float bv = col_ok ? v : 0.0f;
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Af[0][s], bv, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Af[1][s], bv, acc1, 0, 0, 0);
        }
      } else {
        bf16x8 bv;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float v = Up[bup[q] ? sl1 : sl][col_ok ? nb + boff[q] : 0];
          bv[q] = (__bf16)((col_ok && bok[q]) ? v : 0.0f);
        }
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ab[0], bv, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ab[1], bv, acc1, 0, 0, 0);
      }
      const float Ee = eok ? a.E[ei + (int64_t)g.nx * (ej + (int64_t)g.ny * L)] : 0.0f;
      float *Yr = Y + el * kYP;
      const int r0 = 4 * (lane >> 4);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Yr[r0 + r] = Ee * acc0[r];                      // rows 0..15
        if (r0 + r < 8) Yr[16 + r0 + r] = Ee * acc1[r];  // rows 16..23
      }
    }
    __syncthreads();
    // ---- per node column: bottom faces finish (i,j,L), top faces start (i,j,L+1)
    if (own) {
      float bt0 = 0.f, bt1 = 0.f, bt2 = 0.f, tp0 = 0.f, tp1 = 0.f, tp2 = 0.f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ex = e & 1, ey = e >> 1;
        const float *Yr = Y + ((ti + ex) + kEW * (tj + ey)) * kYP;
        const int ab = corner_of(1 - ex, 1 - ey, 0), at = corner_of(1 - ex, 1 - ey, 1);
        bt0 += Yr[3 * ab];
        bt1 += Yr[3 * ab + 1];
        bt2 += Yr[3 * ab + 2];
        tp0 += Yr[3 * at];
        tp1 += Yr[3 * at + 1];
        tp2 += Yr[3 * at + 2];
      }
      if (L >= k0) {
        const int64_t n = (int64_t)L * plane + (int64_t)j * NX + i;
        const uint8_t fx = a.fixed[n];
        const float *sp = &Up[sl][3 * ((ti + 1) + kPW * (tj + 1))];
        const float self[3] = {sp[0], sp[1], sp[2]};
        const float Au[3] = {top0 + bt0, top1 + bt1, top2 + bt2};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const bool isf = (fx >> c) & 1;
          const int64_t dof = 3 * n + c;
          const float Ac = isf ? 0.0f : Au[c];
          if constexpr (EPI == KU_STORE) {
            a.y[dof] = isf ? self[c] : Au[c];
          } else if constexpr (EPI == KU_RES0) {
            a.res[dof] = a.b[dof] - Ac;
            a.x[dof] = self[c];
          } else if constexpr (EPI == KU_CHEB0) {
            const float r = a.b[dof] - Ac;
            const float dn = a.c1 * self[c] + a.c2 * r * a.dinv[dof];
            a.res[dof] = r;
            a.dout[dof] = dn;
            a.x[dof] = self[c] + dn;
          } else if constexpr (EPI == KU_CHEB || EPI == KU_CHEB_ADD) {
            const float r = a.res[dof] - Ac;
            const float dn = a.c1 * self[c] + a.c2 * r * a.dinv[dof];
            const float xn = a.x[dof] + dn + (EPI == KU_CHEB_ADD ? self[c] : 0.0f);
            if (a.dout) {  // not the last step: its residual and direction are still needed
              a.res[dof] = r;
              a.dout[dof] = dn;
            }
            a.x[dof] = xn;
            if (a.dot_with) dotv = fma((double)a.dot_with[dof], (double)xn, dotv);
          } else if constexpr (EPI == KU_RESUPD) {
            a.res[dof] -= Ac;
          } else if constexpr (EPI == KU_RESID_START) {
            const float r = a.b[dof] - Ac;
            a.res[dof] = r;
            if (a.dout) a.dout[dof] = r * a.dinv[dof] * a.s0;
          }
        }
      }
      top0 = tp0;
      top1 = tp1;
      top2 = tp2;
    }
    if (more) store(sl2);
    __syncthreads();
    sl = sl1;
  }
  (void)dotv;
}

namespace {
template <bool BF16, int KZ>
hipError_t launch_mfma_kz(hipStream_t s, KuEpi epi, const KuArgsT<float> &a, const float *KEm, const __bf16 *KEb) {
  const int tx = (a.g.NX() + kTile - 1) / kTile, ty = (a.g.NY() + kTile - 1) / kTile;
  const dim3 grid((unsigned)(tx * ty), (unsigned)((a.g.NZ() + KZ - 1) / KZ));
#define TOPO_KUM_CASE(E) \
  case E: ku_mfma_kernel<E, BF16, KZ><<<grid, 256, 0, s>>>(a, KEm, KEb); break;
  switch (epi) {
    TOPO_KUM_CASE(KU_STORE)
    TOPO_KUM_CASE(KU_RES0)
    TOPO_KUM_CASE(KU_CHEB0)
    TOPO_KUM_CASE(KU_CHEB)
    TOPO_KUM_CASE(KU_CHEB_ADD)
    TOPO_KUM_CASE(KU_RESUPD)
    TOPO_KUM_CASE(KU_RESID_START)
    default: return hipErrorInvalidValue;
  }
#undef TOPO_KUM_CASE
  return hipGetLastError();
}
}  // namespace

hipError_t launch_ku_mfma(hipStream_t s, KuEpi epi, const KuArgsT<float> &a, bool bf16) {
  const float *KEm = a.ke32;
  const __bf16 *KEb = reinterpret_cast<const __bf16 *>(a.ke16);
  if (a.dot_with) return hipErrorInvalidValue;  // reducing epilogues stay on the vector-unit kernel
  if (!KEm || (bf16 && !KEb)) return hipErrorInvalidValue;
  // short columns on small grids keep enough blocks in flight
  const bool big = a.g.nnodes() >= 200000;
  if (bf16) return big ? launch_mfma_kz<true, 8>(s, epi, a, KEm, KEb) : launch_mfma_kz<true, 2>(s, epi, a, KEm, KEb);
  return big ? launch_mfma_kz<false, 8>(s, epi, a, KEm, KEb) : launch_mfma_kz<false, 2>(s, epi, a, KEm, KEb);
}

}  // namespace topo
