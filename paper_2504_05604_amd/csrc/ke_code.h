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

// ---------------------------------------------------------------------------
// KE in the per-axis sum/difference (Hadamard) basis of the element's corners.
//
// Mode s (bit 0: x, bit 1: y, bit 2: z) of displacement component c is
//     h(s, c) = sum_a hada_sign(s, a) u(a, c),  hada_sign(s, a) = (-1)^(s . corner(a)),
// i.e. h = H u with H = H8 (x) I3 and H^T H = 8 I.  The unit cube is symmetric
// under the reflection of each axis, which maps u_c to -u_c on its own axis and
// mode s to (-1)^(bit of s) times itself; KE commutes with these reflections, so
// M = H KE H^T / 64 only couples states with the same parity p = s xor 2^c.
// Each parity class holds one state per component, and KE = H^T M H splits into
// eight 3x3 blocks; their entries are integer combinations of the 10 kappa values,
// and the patterns the element-column kernel relies on are checked below at
// compile time:
//   p = 0            (s = 2^c):        alpha on the diagonal, beta off it
//   p = 2^b          (one axis b):     the state c = b is s = 0 (a rigid translation,
//                                      zero row); the other two: gamma / delta
//   p = 2^b + 2^b'   (two axes):       the two states c in {b, b'} couple with eps
//                                      everywhere, the third (s = 7) has zeta alone
//   p = 7:                              eta on the diagonal, theta off it
// With the element's modulus folded into these 8 constants, the element product
// takes 21 multiply-adds plus the sum/difference passes instead of a 24 x 24
// mat-vec.
__host__ __device__ constexpr int hada_sign(int s, int a) {
  return (((s & 1) & cx(a)) ^ (((s >> 1) & 1) & cy(a)) ^ (((s >> 2) & 1) & cz(a))) ? -1 : 1;
}

struct KappaCoef {
  int v[10];
};

// 64 M[(s1,c1),(s2,c2)] as an integer combination of kappa_0..kappa_9
__host__ __device__ constexpr KappaCoef hada_coef(int s1, int c1, int s2, int c2) {
  KappaCoef r{};
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) {
      const int I = 3 * a + c1, J = 3 * b + c2;
      r.v[kKeTable.idx[I * 24 + J]] += hada_sign(s1, a) * hada_sign(s2, b) * kKeTable.sign[I * 24 + J];
    }
  return r;
}

// two entries agree for every Poisson ratio iff their (lam, mu) integer parts agree
__host__ __device__ constexpr bool coef_eq(const KappaCoef &x, const KappaCoef &y) {
  long la = 0, mu = 0;
  for (int t = 0; t < 10; ++t) {
    la += (long)(x.v[t] - y.v[t]) * kKeTable.pairs[t].a;
    mu += (long)(x.v[t] - y.v[t]) * kKeTable.pairs[t].b;
  }
  return la == 0 && mu == 0;
}
__host__ __device__ constexpr bool coef_zero(const KappaCoef &x) { return coef_eq(x, KappaCoef{}); }

// state of component c in parity class p
__host__ __device__ constexpr int hada_state(int p, int c) { return p ^ (1 << c); }

// the 8 constants, in the order alpha, beta, gamma, delta, eps, zeta, eta, theta
enum HadaConst { H_ALPHA, H_BETA, H_GAMMA, H_DELTA, H_EPS, H_ZETA, H_ETA, H_THETA, kHadaConsts };

__host__ __device__ constexpr KappaCoef hada_const_coef(int k) {
  switch (k) {
    case H_ALPHA: return hada_coef(1, 0, 1, 0);
    case H_BETA: return hada_coef(1, 0, 2, 1);
    case H_GAMMA: return hada_coef(3, 1, 3, 1);  // class p = 1, components 1 and 2
    case H_DELTA: return hada_coef(3, 1, 5, 2);
    case H_EPS: return hada_coef(2, 0, 2, 0);  // class p = 3, components 0 and 1
    case H_ZETA: return hada_coef(7, 2, 7, 2);
    case H_ETA: return hada_coef(6, 0, 6, 0);
    default: return hada_coef(6, 0, 5, 1);  // H_THETA
  }
}

__host__ __device__ constexpr bool hada_structure_holds() {
  const KappaCoef al = hada_const_coef(H_ALPHA), be = hada_const_coef(H_BETA);
  const KappaCoef ga = hada_const_coef(H_GAMMA), de = hada_const_coef(H_DELTA);
  const KappaCoef ep = hada_const_coef(H_EPS), ze = hada_const_coef(H_ZETA);
  const KappaCoef et = hada_const_coef(H_ETA), th = hada_const_coef(H_THETA);
  for (int s1 = 0; s1 < 8; ++s1)
    for (int c1 = 0; c1 < 3; ++c1)
      for (int s2 = 0; s2 < 8; ++s2)
        for (int c2 = 0; c2 < 3; ++c2) {
          const KappaCoef m = hada_coef(s1, c1, s2, c2);
          const int p = s1 ^ (1 << c1);
          const int np = (p & 1) + ((p >> 1) & 1) + ((p >> 2) & 1);
          if (p != (s2 ^ (1 << c2))) {  // different classes never couple
            if (!coef_zero(m)) return false;
            continue;
          }
          const bool diag = c1 == c2;
          bool ok = true;
          if (np == 0) {
            ok = coef_eq(m, diag ? al : be);
          } else if (np == 1) {
            const bool tr = s1 == 0 || s2 == 0;  // the rigid translation of this class
            ok = tr ? coef_zero(m) : coef_eq(m, diag ? ga : de);
          } else if (np == 2) {
            const bool in1 = (p >> c1) & 1, in2 = (p >> c2) & 1;
            ok = (in1 && in2) ? coef_eq(m, ep) : (!in1 && !in2) ? coef_eq(m, ze) : coef_zero(m);
          } else {
            ok = coef_eq(m, diag ? et : th);
          }
          if (!ok) return false;
        }
  return true;
}
static_assert(hada_structure_holds(), "KE must split into the 8 parity blocks of the sum/difference basis");

template <typename T>
struct HadaT {
  T k[kHadaConsts];
};

// M's 8 distinct entries for these kappa values (exact integer combinations / 64)
template <typename T>
inline HadaT<T> make_hada(const KappaT<T> &kap) {
  HadaT<T> h{};
  for (int c = 0; c < kHadaConsts; ++c) {
    const KappaCoef cf = hada_const_coef(c);
    double v = 0.0;
    for (int t = 0; t < 10; ++t) v += cf.v[t] * (double)kap.k[t];
    h.k[c] = (T)(v / 64.0);
  }
  return h;
}

// HadaW: the block entries in the form the kernels apply them, before an
// element's modulus is folded in: w[0] = alpha - beta, w[1] = beta, w[2] = gamma - delta,
// w[3] = delta, w[4] = eps, w[5] = zeta, w[6] = eta - theta, w[7] = theta.
template <typename T>
inline HadaW<T> hada_work(const KappaT<T> &kap) {
  KappaT<double> kd{};
  for (int t = 0; t < 10; ++t) kd.k[t] = (double)kap.k[t];
  const HadaT<double> h = make_hada(kd);
  const double w[8] = {h.k[H_ALPHA] - h.k[H_BETA], h.k[H_BETA], h.k[H_GAMMA] - h.k[H_DELTA],
                       h.k[H_DELTA], h.k[H_EPS], h.k[H_ZETA], h.k[H_ETA] - h.k[H_THETA],
                       h.k[H_THETA]};
  HadaW<T> r{};
  for (int i = 0; i < 8; ++i) r.w[i] = (T)w[i];
  return r;
}

// x/y sum-difference pass over a 2 x 2 patch (corner (dx, dy) at index dx + 2 dy):
// out[q] = sum_corner (-1)^(qx dx + qy dy) in[corner].  The matrix is symmetric,
// so the same pass takes modes back to corners (H^T).  No scaling is applied:
// the block entries M = H KE H^T / 64 already carry it (H^T H = 8 I).
template <typename T>
__host__ __device__ __forceinline__ void xy_pass(const T (&in)[4], T (&out)[4]) {
  const T p0 = in[0] + in[1], m0 = in[0] - in[1];
  const T p1 = in[2] + in[3], m1 = in[2] - in[3];
  out[0] = p0 + p1;
  out[1] = m0 + m1;
  out[2] = p0 - p1;
  out[3] = m0 - m1;
}

// g = M h for one element: h[c][s] are the modes (s = q + 4 z; h[c][0], the rigid
// translations, is not read), w the block entries times the element's modulus.
// Class p holds state (p ^ 2^c, c) for c = 0, 1, 2.
template <typename T>
__host__ __device__ __forceinline__ void hada_blocks(const T (&w)[8], const T (&h)[3][8], T (&gm)[3][8]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) gm[c][0] = T(0);
  {  // p = 0
    const T t = w[1] * (h[0][1] + h[1][2] + h[2][4]);
    gm[0][1] = fma(w[0], h[0][1], t);
    gm[1][2] = fma(w[0], h[1][2], t);
    gm[2][4] = fma(w[0], h[2][4], t);
  }
#pragma unroll
  for (int b = 0; b < 3; ++b) {  // p = 2^b: the two components other than b
    const int p = 1 << b, c1 = b == 0 ? 1 : 0, c2 = b == 2 ? 1 : 2;
    const int s1 = p ^ (1 << c1), s2 = p ^ (1 << c2);
    const T t = w[3] * (h[c1][s1] + h[c2][s2]);
    gm[c1][s1] = fma(w[2], h[c1][s1], t);
    gm[c2][s2] = fma(w[2], h[c2][s2], t);
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {  // p = 7 - 2^m: components of the two axes in p, and m
    const int p = 7 ^ (1 << m), c1 = m == 0 ? 1 : 0, c2 = m == 2 ? 1 : 2;
    const int s1 = p ^ (1 << c1), s2 = p ^ (1 << c2);
    const T t = w[4] * (h[c1][s1] + h[c2][s2]);
    gm[c1][s1] = t;
    gm[c2][s2] = t;
    gm[m][7] = w[5] * h[m][7];
  }
  {  // p = 7
    const T t = w[7] * (h[0][6] + h[1][5] + h[2][3]);
    gm[0][6] = fma(w[6], h[0][6], t);
    gm[1][5] = fma(w[6], h[1][5], t);
    gm[2][3] = fma(w[6], h[2][3], t);
  }
}

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
