// Matrix-free element-by-element stiffness operator on the structured hex grid.
//
// y_i = sum over the (up to 8) elements e around node i of
//       E_e * (KE u_e)_{local(i)}
// i.e. the product with K = sum_e E_e KE of the Finite Element Analysis section
// without assembling it.  One thread owns one node (3 dofs) and computes its
// rows from the 27 neighbouring nodes and 8 surrounding moduli, so no two
// threads write the same entry: deterministic, no atomics.  KE (24x24) is read
// through a uniform pointer with compile-time indices, i.e. from scalar
// registers, as the second operand of every FMA.
//
// Fixed dofs: inputs are required to be zero there (the solver keeps every
// vector in the subspace of free dofs); outputs get the identity row y = u.
#include "internal.h"
#include "reduce_dev.h"

namespace topo {

template <int EPI>
__global__ __launch_bounds__(256) void ku_node_kernel(KuArgs a, Reducer red, double *out0) {
  const Grid g = a.g;
  const int NX = g.NX(), NY = g.NY();
  const int64_t nn = g.nnodes();
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dotv = 0.0;
  if (n < nn) {
    const int i = (int)(n % NX);
    const int64_t t = n / NX;
    const int j = (int)(t % NY);
    const int k = (int)(t / NY);
    const double *__restrict__ u = a.u;
    const double *__restrict__ KE = a.KE;
    // neighbour displacements, index (dx+1) + 3 (dy+1) + 9 (dz+1)
    double un[27][3];
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int q = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
          const bool ok = (i + dx >= 0) && (i + dx <= g.nx) && (j + dy >= 0) && (j + dy <= g.ny) &&
                          (k + dz >= 0) && (k + dz <= g.nz);
          const int64_t m = n + dx + (int64_t)NX * (dy + (int64_t)NY * dz);
#pragma unroll
          for (int c = 0; c < 3; ++c) un[q][c] = ok ? u[3 * m + c] : 0.0;
        }
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;  // element (i-1+ex, j-1+ey, k-1+ez)
      const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
      const bool eok = ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny && ek >= 0 && ek < g.nz;
      const double Ee = eok ? a.E[ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek)] : 0.0;
      const int li = corner_of(1 - ex, 1 - ey, 1 - ez);  // this node inside element e
      double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int q = (ex + cx(b)) + 3 * (ey + cy(b)) + 9 * (ez + cz(b));
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double v = un[q][d];
          t0 = fma(KE[(3 * li + 0) * 24 + 3 * b + d], v, t0);
          t1 = fma(KE[(3 * li + 1) * 24 + 3 * b + d], v, t1);
          t2 = fma(KE[(3 * li + 2) * 24 + 3 * b + d], v, t2);
        }
      }
      acc0 = fma(Ee, t0, acc0);
      acc1 = fma(Ee, t1, acc1);
      acc2 = fma(Ee, t2, acc2);
    }
    const uint8_t fx = a.fixed[n];
    const double self[3] = {un[13][0], un[13][1], un[13][2]};
    double Au[3] = {acc0, acc1, acc2};
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
  if constexpr (EPI == KU_STORE_DOT || EPI == KU_RESID) {
    double v[1] = {dotv};
    block_reduce_finalize<1, false>(v, red, out0);
  }
}

hipError_t launch_ku(hipStream_t s, KuEpi epi, const KuArgs &a, const Reducer &red, double *out0) {
  const int64_t nn = a.g.nnodes();
  const int bs = 256;
  const unsigned nb = (unsigned)((nn + bs - 1) / bs);
  switch (epi) {
    case KU_STORE: ku_node_kernel<KU_STORE><<<nb, bs, 0, s>>>(a, red, out0); break;
    case KU_STORE_DOT: ku_node_kernel<KU_STORE_DOT><<<nb, bs, 0, s>>>(a, red, out0); break;
    case KU_RESID: ku_node_kernel<KU_RESID><<<nb, bs, 0, s>>>(a, red, out0); break;
    case KU_CHEB: ku_node_kernel<KU_CHEB><<<nb, bs, 0, s>>>(a, red, out0); break;
    case KU_RESUPD: ku_node_kernel<KU_RESUPD><<<nb, bs, 0, s>>>(a, red, out0); break;
  }
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
__global__ void diag_kernel(Grid g, const double *E, const double *KEdiag, const uint8_t *fixed,
                            double *diag) {
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
    d0 += Ee * KEdiag[3 * li + 0];
    d1 += Ee * KEdiag[3 * li + 1];
    d2 += Ee * KEdiag[3 * li + 2];
  }
  const uint8_t fx = fixed[n];
  diag[3 * n + 0] = (fx & 1) ? 1.0 : d0;
  diag[3 * n + 1] = (fx & 2) ? 1.0 : d1;
  diag[3 * n + 2] = (fx & 4) ? 1.0 : d2;
}

hipError_t launch_diag(hipStream_t s, Grid g, const double *E, const double *KEdiag,
                       const uint8_t *fixed, double *diag) {
  const int bs = 256;
  diag_kernel<<<(unsigned)((g.nnodes() + bs - 1) / bs), bs, 0, s>>>(g, E, KEdiag, fixed, diag);
  return hipGetLastError();
}

}  // namespace topo
