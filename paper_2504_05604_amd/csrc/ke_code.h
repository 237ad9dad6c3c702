// Compile-time structure of the 8-node unit-cube stiffness matrix.
//
// With isotropic D(lam, mu), every entry of KE = int B^T D B over the unit cube
// equals (a lam + b mu) / 216 for integers a, b that depend only on the two
// local dofs: each entry is a sum of products of the 1D moments of the linear
// shape factors (int f f = 1/3 or 1/6, int f' f = +-1/2, int f' f' = +-1).  Up to
// sign there are exactly 10 distinct (a, b) pairs, so
//     KE[I][J] = sign(I, J) * kappa[idx(I, J)],
// with both tables known at compile time and only the 10 values
// kappa_t = (a_t lam + b_t mu) / 216 depending on the Poisson ratio.  Kernels
// take kappa by value (kernel arguments live in scalar registers), so every
// multiply-add of the element contraction reads a register, never memory.
#pragma once

#include "internal.h"

namespace topo {

struct KePair {
  int a, b;
};
struct KeTable {
  signed char sign[576];
  unsigned char idx[576];
  KePair pairs[16];
  int npairs;
};

__host__ __device__ constexpr int corner_coord(int a, int d) {
  return d == 0 ? cx(a) : (d == 1 ? cy(a) : cz(a));
}
// 6 x the 1D moments on [0,1] of the factors f_s(t) = t (s = 1) or 1 - t (s = 0)
__host__ __device__ constexpr int m_vv(int s, int r) { return s == r ? 2 : 1; }
__host__ __device__ constexpr int m_dv(int s, int) { return s == 1 ? 3 : -3; }
__host__ __device__ constexpr int m_dd(int s, int r) { return (s == 1 ? 6 : -6) * (r == 1 ? 1 : -1); }

// 216 x int d_p N_a d_q N_b over the unit cube
__host__ __device__ constexpr int g216(int a, int b, int p, int q) {
  int v = 1;
  for (int d = 0; d < 3; ++d) {
    const int s = corner_coord(a, d), r = corner_coord(b, d);
    if (d == p && d == q) v *= m_dd(s, r);
    else if (d == p) v *= m_dv(s, r);
    else if (d == q) v *= m_dv(r, s);
    else v *= m_vv(s, r);
  }
  return v;
}

// K^{ij}_{ab} = lam int d_i N_a d_j N_b + mu (int d_j N_a d_i N_b + delta_ij int grad N_a . grad N_b)
__host__ __device__ constexpr KeTable make_ke_table() {
  KeTable t{};
  t.npairs = 0;
  for (int I = 0; I < 24; ++I)
    for (int J = 0; J < 24; ++J) {
      const int a = I / 3, i = I % 3, b = J / 3, j = J % 3;
      const int lap = g216(a, b, 0, 0) + g216(a, b, 1, 1) + g216(a, b, 2, 2);
      int A = g216(a, b, i, j);
      int B = g216(a, b, j, i) + (i == j ? lap : 0);
      int sg = 1;
      if (A < 0 || (A == 0 && B < 0)) {
        A = -A;
        B = -B;
        sg = -1;
      }
      int k = 0;
      while (k < t.npairs && !(t.pairs[k].a == A && t.pairs[k].b == B)) ++k;
      if (k == t.npairs) {
        t.pairs[k] = KePair{A, B};
        ++t.npairs;
      }
      t.sign[I * 24 + J] = (signed char)sg;
      t.idx[I * 24 + J] = (unsigned char)k;
    }
  return t;
}

constexpr KeTable kKeTable = make_ke_table();
static_assert(kKeTable.npairs == 10, "the H8 stiffness has 10 distinct entries up to sign");

__host__ __device__ constexpr double ke_sign(int I, int J) { return kKeTable.sign[I * 24 + J]; }
__host__ __device__ constexpr int ke_idx(int I, int J) { return kKeTable.idx[I * 24 + J]; }

// KE[I][J] for compile-time I, J, in the precision of kappa (the sign becomes a
// negation modifier on the register operand)
template <typename T>
__host__ __device__ __forceinline__ T ke_value(const KappaT<T> &k, int I, int J) {
  const T v = k.k[ke_idx(I, J)];
  return ke_sign(I, J) > 0 ? v : -v;
}
#define TOPO_KE(kap, I, J) (::topo::ke_value((kap), (I), (J)))

inline Kappa make_kappa(double nu) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  Kappa k{};
  for (int t = 0; t < 10; ++t) k.k[t] = (kKeTable.pairs[t].a * lam + kKeTable.pairs[t].b * mu) / 216.0;
  return k;
}

inline KappaT<float> to_float(const Kappa &k) {
  KappaT<float> f{};
  for (int t = 0; t < 10; ++t) f.k[t] = (float)k.k[t];
  return f;
}

}  // namespace topo
