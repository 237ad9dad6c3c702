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
// Fixed dofs: inputs are required to be zero there (the solver keeps every
// vector in the subspace of free dofs); outputs get the identity row y = u.
#include "internal.h"
#include "ke_code.h"
#include "reduce_dev.h"

namespace topo {

constexpr int kKuBlock = 256;
constexpr int kKuKZ = 8;  // nodes per thread column

template <int EPI>
__global__ __launch_bounds__(kKuBlock) void ku_march_kernel(KuArgs a, Kappa kap, double *partials) {
  if (a.skip && *a.skip) return;
  const Grid g = a.g;
  const int NX = g.NX(), NY = g.NY(), NZ = g.NZ();
  const int ncol = NX * NY;
  const int col = blockIdx.x * kKuBlock + threadIdx.x;
  const int k0 = blockIdx.y * kKuKZ;
  const int k1 = min(k0 + kKuKZ, NZ);
  const bool active = col < ncol;
  const int i = active ? col % NX : 0, j = active ? col / NX : 0;
  const int64_t plane = (int64_t)ncol;
  const double *__restrict__ u = a.u;
  double dotv = 0.0;
  if (active) {
    double P0[9][3], P1[9][3];
    auto load_plane = [&](int kp, double(&P)[9][3]) {
      const bool okz = kp >= 0 && kp <= g.nz;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int q = (dx + 1) + 3 * (dy + 1);
          const bool ok = okz && (i + dx >= 0) && (i + dx <= g.nx) && (j + dy >= 0) && (j + dy <= g.ny);
          const int64_t m = (int64_t)kp * plane + (int64_t)(j + dy) * NX + (i + dx);
#pragma unroll
          for (int c = 0; c < 3; ++c) P[q][c] = ok ? u[3 * m + c] : 0.0;
        }
    };
    load_plane(k0 - 1, P0);
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;  // node (i,j,L): top-face part so far
    for (int L = k0 - 1; L < k1; ++L) {
      load_plane(L + 1, P1);
      double nb0 = 0.0, nb1 = 0.0, nb2 = 0.0;  // node (i,j,L+1)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ex = e & 1, ey = e >> 1;  // element (i-1+ex, j-1+ey, L)
        const int ei = i - 1 + ex, ej = j - 1 + ey;
        const bool eok = ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny && L >= 0 && L < g.nz;
        const double Ee = eok ? a.E[ei + (int64_t)g.nx * (ej + (int64_t)g.ny * L)] : 0.0;
        const int lb = corner_of(1 - ex, 1 - ey, 0), lt = corner_of(1 - ex, 1 - ey, 1);
        double b0 = 0.0, b1 = 0.0, b2 = 0.0, t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const int q = (ex + cx(b)) + 3 * (ey + cy(b));
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const double v = cz(b) ? P1[q][d] : P0[q][d];
            b0 = fma(TOPO_KE(kap, 3 * lb + 0, 3 * b + d), v, b0);
            b1 = fma(TOPO_KE(kap, 3 * lb + 1, 3 * b + d), v, b1);
            b2 = fma(TOPO_KE(kap, 3 * lb + 2, 3 * b + d), v, b2);
            t0 = fma(TOPO_KE(kap, 3 * lt + 0, 3 * b + d), v, t0);
            t1 = fma(TOPO_KE(kap, 3 * lt + 1, 3 * b + d), v, t1);
            t2 = fma(TOPO_KE(kap, 3 * lt + 2, 3 * b + d), v, t2);
          }
        }
        acc0 = fma(Ee, b0, acc0);
        acc1 = fma(Ee, b1, acc1);
        acc2 = fma(Ee, b2, acc2);
        nb0 = fma(Ee, t0, nb0);
        nb1 = fma(Ee, t1, nb1);
        nb2 = fma(Ee, t2, nb2);
      }
      if (L >= k0) {  // node (i,j,L) is complete
        const int64_t n = (int64_t)L * plane + col;
        const uint8_t fx = a.fixed[n];
        const double self[3] = {P0[4][0], P0[4][1], P0[4][2]};
        const double Au[3] = {acc0, acc1, acc2};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const bool isf = (fx >> c) & 1;
          const int64_t dof = 3 * n + c;
          if constexpr (EPI == KU_STORE) {
            a.y[dof] = isf ? self[c] : Au[c];
          } else if constexpr (EPI == KU_STORE_DOT) {
            const double yv = isf ? self[c] : Au[c];
            a.y[dof] = yv;
            dotv = fma(self[c], yv, dotv);
          } else if constexpr (EPI == KU_RESID) {
            const double yv = isf ? 0.0 : a.b[dof] - Au[c];
            a.y[dof] = yv;
            dotv = fma(yv, yv, dotv);
          } else if constexpr (EPI == KU_CHEB) {
            if (!isf) {
              const double r = a.res[dof] - Au[c];
              const double dn = a.c1 * self[c] + a.c2 * r / a.diag[dof];
              a.res[dof] = r;
              a.dout[dof] = dn;
              a.x[dof] += dn;
            } else {
              a.dout[dof] = 0.0;
            }
          } else if constexpr (EPI == KU_RESUPD) {
            if (!isf) a.res[dof] -= Au[c];
          }
        }
      }
      acc0 = nb0;
      acc1 = nb1;
      acc2 = nb2;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        P0[q][0] = P1[q][0];
        P0[q][1] = P1[q][1];
        P0[q][2] = P1[q][2];
      }
    }
  }
  if constexpr (EPI == KU_STORE_DOT || EPI == KU_RESID) {
    double v[1] = {dotv};
    block_reduce_store<1, false>(v, partials, linear_block());
  }
}

hipError_t launch_ku(hipStream_t s, KuEpi epi, const KuArgs &a, const Kappa &kap, const Reducer &red,
                     double *out) {
  const int ncol = a.g.NX() * a.g.NY();
  const dim3 grid((unsigned)((ncol + kKuBlock - 1) / kKuBlock), (unsigned)((a.g.NZ() + kKuKZ - 1) / kKuKZ));
  const int nparts = (int)(grid.x * grid.y);
  if ((epi == KU_STORE_DOT || epi == KU_RESID) && nparts > red.max_blocks) return hipErrorInvalidValue;
  switch (epi) {
    case KU_STORE: ku_march_kernel<KU_STORE><<<grid, kKuBlock, 0, s>>>(a, kap, red.partials); break;
    case KU_STORE_DOT: ku_march_kernel<KU_STORE_DOT><<<grid, kKuBlock, 0, s>>>(a, kap, red.partials); break;
    case KU_RESID: ku_march_kernel<KU_RESID><<<grid, kKuBlock, 0, s>>>(a, kap, red.partials); break;
    case KU_CHEB: ku_march_kernel<KU_CHEB><<<grid, kKuBlock, 0, s>>>(a, kap, red.partials); break;
    case KU_RESUPD: ku_march_kernel<KU_RESUPD><<<grid, kKuBlock, 0, s>>>(a, kap, red.partials); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (epi == KU_STORE_DOT || epi == KU_RESID) return launch_finalize(s, red, nparts, 1, false, out, a.skip);
  return hipSuccess;
}

// ---------------------------------------------------------------------------
__global__ void finalize_kernel(const double *partials, int nparts, int n, int is_max, double *out,
                                const int *skip) {
  if (skip && *skip) return;
  __shared__ double sh[kMaxRed][16];
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
    out[k] = t;
  }
}

hipError_t launch_finalize(hipStream_t s, const Reducer &red, int nparts, int n, bool is_max,
                           double *out, const int *skip) {
  if (n > kMaxRed || nparts > red.max_blocks) return hipErrorInvalidValue;
  finalize_kernel<<<1, 256, 0, s>>>(red.partials, nparts, n, is_max ? 1 : 0, out, skip);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void simp_modulus_kernel(int64_t nel, const double *xphys, double E0, double Emin,
                                    double penal, double scale, double *E) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  const double x = xphys[e];
  const double xp = (penal == 3.0) ? x * x * x : pow(x, penal);
  E[e] = scale * (Emin + xp * (E0 - Emin));
}

hipError_t launch_simp_modulus(hipStream_t s, int64_t nel, const double *xphys, double E0,
                               double Emin, double penal, double scale, double *E) {
  const int bs = 256;
  simp_modulus_kernel<<<(unsigned)((nel + bs - 1) / bs), bs, 0, s>>>(nel, xphys, E0, Emin, penal,
                                                                    scale, E);
  return hipGetLastError();
}

// Coarse modulus = 2 * mean of the 8 fine children (missing children are 0):
// the factor 2 is the stiffness scaling of an element of twice the edge length.
__global__ void coarsen_moduli_kernel(Grid gf, Grid gc, const double *Ef, double *Ec) {
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
}

hipError_t launch_coarsen_moduli(hipStream_t s, Grid gf, Grid gc, const double *Ef, double *Ec) {
  const int bs = 256;
  coarsen_moduli_kernel<<<(unsigned)((gc.nel() + bs - 1) / bs), bs, 0, s>>>(gf, gc, Ef, Ec);
  return hipGetLastError();
}

// diag_(i,c) = sum_{e around i} E_e KE[(3 li + c),(3 li + c)]; 1 on fixed dofs
__global__ void diag_kernel(Grid g, const double *E, Kappa kap, const uint8_t *fixed, double *diag) {
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
  diag[3 * n + 0] = (fx & 1) ? 1.0 : d0;
  diag[3 * n + 1] = (fx & 2) ? 1.0 : d1;
  diag[3 * n + 2] = (fx & 4) ? 1.0 : d2;
}

hipError_t launch_diag(hipStream_t s, Grid g, const double *E, const Kappa &kap,
                       const uint8_t *fixed, double *diag) {
  const int bs = 256;
  diag_kernel<<<(unsigned)((g.nnodes() + bs - 1) / bs), bs, 0, s>>>(g, E, kap, fixed, diag);
  return hipGetLastError();
}

}  // namespace topo
