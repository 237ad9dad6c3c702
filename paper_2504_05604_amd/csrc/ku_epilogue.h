// Per-node epilogues of the stiffness operator kernels.
//
// Every K.u kernel ends a node with its product (K u) at that node and hands it
// here, where the vector updates of the conjugate-gradient loop and of the
// Chebyshev smoother that consume it are fused into the same pass.  Both the
// node-column kernel and the element-column kernel use these functions, so the
// two run the same per-node arithmetic.
//
// Fixed dofs: inputs are zero there (the solver keeps every vector in the
// subspace of free dofs); STORE/STORE_DOT outputs get the identity row y = u.
#pragma once

#include "internal.h"
#include "reduce_dev.h"

namespace topo {

template <int EPI>
struct EpiTraits {
  // operand built as b * dinv * s0 instead of read from u
  static constexpr bool scaled_operand = EPI == KU_RES0 || EPI == KU_CHEB0;
};

// What an epilogue reads at its node besides the product; loaded ahead of the
// product by kernels that pipeline their memory traffic.  Fields an epilogue does
// not use are never loaded and vanish after inlining.
template <typename T>
struct EpiIn {
  uint8_t fx;  // fixed-dof bits of the node
  T b[3], r[3], d[3], x[3], w[3];  // rhs, residual, inverse diagonal, iterate, dot_with
  double rc[3];                    // RESID_FLEX: the CG residual
  T zo[3];                         // RESID_FLEX: the previous preconditioned residual
};

// HAVE_BD: the caller already holds b and dinv at the node (the scaled
// epilogues read them to form their operand) and fills them in itself.
template <int EPI, bool HAVE_BD = false, typename T>
__device__ __forceinline__ void ku_epi_load(const KuArgsT<T> &a, int64_t n, const T *__restrict__ dinv,
                                            EpiIn<T> &in) {
  in.fx = a.fixed[n];
  constexpr bool kB = !HAVE_BD && (EPI == KU_RESID || EPI == KU_RES0 || EPI == KU_CHEB0 || EPI == KU_RESID_START ||
                                   EPI == KU_RESID_FLEX);
  constexpr bool kR = EPI == KU_CHEB || EPI == KU_CHEB_ADD || EPI == KU_RESUPD;
  constexpr bool kD = !HAVE_BD && (EPI == KU_CHEB0 || EPI == KU_CHEB || EPI == KU_CHEB_ADD || EPI == KU_RESID_START ||
                                   EPI == KU_RESID_FLEX);
  constexpr bool kX = EPI == KU_CHEB || EPI == KU_CHEB_ADD;
  constexpr bool kF = EPI == KU_RESID_FLEX;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t dof = 3 * n + c;
    if constexpr (kB) in.b[c] = a.b[dof];
    if constexpr (kR) in.r[c] = a.res[dof];
    if constexpr (kD) {
      // the residual start reads dinv only for the direction it stores
      if (EPI != KU_RESID_START || a.dout) in.d[c] = dinv[dof];
    }
    if constexpr (kX) in.x[c] = a.x[dof];
    if constexpr (kF) {
      in.rc[c] = a.rflex[dof];
      in.zo[c] = a.zflex[dof];
    }
  }
  if constexpr (kX) {
    if (a.dot_with) {
#pragma unroll
      for (int c = 0; c < 3; ++c) in.w[c] = a.dot_with[3 * n + c];
    }
  }
}

// self: the operand at the node (u, or b dinv s0 for the scaled epilogues);
// Au: the operator's product at the node; dotv accumulates the epilogue's dot
// products (STORE_DOT: u.y, RESID: r.r, CHEB with dot_with: dot_with.x_new;
// RESID_FLEX: r.z_new and r.z_old).
template <int EPI, typename T>
__device__ __forceinline__ void ku_epi_finish(const KuArgsT<T> &a, int64_t n, const EpiIn<T> &in,
                                              const T (&self)[3], const T (&Au)[3], double (&dotv)[2]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const bool isf = (in.fx >> c) & 1;
    const int64_t dof = 3 * n + c;
    const T Ac = isf ? T(0) : Au[c];  // reduced operator: no coupling into fixed rows
    if constexpr (EPI == KU_STORE) {
      a.y[dof] = isf ? self[c] : Au[c];
    } else if constexpr (EPI == KU_STORE_DOT) {
      const T yv = isf ? self[c] : Au[c];
      a.y[dof] = yv;
      dotv[0] = fma((double)self[c], (double)yv, dotv[0]);
    } else if constexpr (EPI == KU_RESID) {
      const T yv = isf ? T(0) : in.b[c] - Au[c];
      a.y[dof] = yv;
      dotv[0] = fma((double)yv, (double)yv, dotv[0]);
    } else if constexpr (EPI == KU_RES0) {  // x = d0, res = b - A d0
      a.res[dof] = in.b[c] - Ac;
      a.x[dof] = self[c];
    } else if constexpr (EPI == KU_CHEB0) {  // res = b - A d0; d1 = c1 d0 + c2 res dinv; x = d0 + d1
      const T r = in.b[c] - Ac;
      const T dn = a.c1 * self[c] + a.c2 * r * in.d[c];
      a.res[dof] = r;
      a.dout[dof] = dn;
      a.x[dof] = self[c] + dn;
    } else if constexpr (EPI == KU_CHEB || EPI == KU_CHEB_ADD) {
      // dinv is 0 on fixed dofs, where res and the operand stay 0
      const T r = in.r[c] - Ac;
      const T dn = a.c1 * self[c] + a.c2 * r * in.d[c];
      const T xn = in.x[c] + dn + (EPI == KU_CHEB_ADD ? self[c] : 0.0);
      if (a.dout) {  // not the last step: its residual and direction are still needed
        a.res[dof] = r;
        a.dout[dof] = dn;
      }
      a.x[dof] = xn;
      if (a.dot_with) dotv[0] = fma((double)in.w[c], (double)xn, dotv[0]);
    } else if constexpr (EPI == KU_RESUPD) {
      a.res[dof] = in.r[c] - Ac;
    } else if constexpr (EPI == KU_RESID_START) {  // res = b - A x; dout = res dinv s0 (unless null)
      const T r = in.b[c] - Ac;
      a.res[dof] = r;
      if (a.dout) a.dout[dof] = r * in.d[c] * a.s0;
    } else if constexpr (EPI == KU_RESID_FLEX) {
      // the last update x + res dinv s0 of the smoothing, as the flexible-CG
      // pass forms it on its own (dinv is 0 on fixed dofs, where x is 0)
      const T r = in.b[c] - Ac;
      const T zf = self[c] + r * in.d[c] * a.s0;
      a.zflex[dof] = zf;
      dotv[0] = fma(in.rc[c], (double)zf, dotv[0]);
      dotv[1] = fma(in.rc[c], (double)in.zo[c], dotv[1]);
    }
  }
}

// load and finish in one go (kernels that do not pipeline)
template <int EPI, typename T>
__device__ __forceinline__ void ku_node_epilogue(const KuArgsT<T> &a, int64_t n, const T (&self)[3],
                                                 const T (&Au)[3], const T *__restrict__ dinv,
                                                 double (&dotv)[2]) {
  EpiIn<T> in;
  ku_epi_load<EPI>(a, n, dinv, in);
  ku_epi_finish<EPI>(a, n, in, self, Au, dotv);
}

// The block's share of the epilogue's dot product (every thread must call it).
template <int EPI, typename T>
__device__ __forceinline__ void ku_block_reduce(const KuArgsT<T> &a, const double (&dotv)[2], double *partials) {
  if constexpr (EPI == KU_STORE_DOT || EPI == KU_RESID) {
    double v[1] = {dotv[0]};
    block_reduce_store<1, false>(v, partials, linear_block());
  } else if constexpr (EPI == KU_CHEB || EPI == KU_CHEB_ADD) {
    if (a.dot_with) {
      double v[1] = {dotv[0]};
      block_reduce_store<1, false>(v, partials, linear_block());
    }
  } else if constexpr (EPI == KU_RESID_FLEX) {
    double v[2] = {dotv[0], dotv[1]};
    block_reduce_store<2, false>(v, partials, linear_block());
  }
}

template <typename T>
inline bool ku_reduces(KuEpi epi, const KuArgsT<T> &a) {
  return epi == KU_STORE_DOT || epi == KU_RESID || epi == KU_RESID_FLEX ||
         ((epi == KU_CHEB || epi == KU_CHEB_ADD) && a.dot_with != nullptr);
}

}  // namespace topo
