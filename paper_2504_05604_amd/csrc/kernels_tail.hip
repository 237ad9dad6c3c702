// The coarse end of the multigrid V-cycle in one launch.
//
// Below a thousand or so nodes a level's smoothing pass, transfer or dense solve
// is far too small to fill the device, and launching each of them separately
// costs more than the work.  Here one workgroup walks the whole tail of the
// hierarchy (pre-smoothing and restriction down to the coarsest level, the
// dense solve, prolongation and post-smoothing back up), with a workgroup
// barrier between passes.  An operator pass runs in two phases: one thread per
// element forms the element's product in the sum/difference basis of its
// corners (ke_code.h) into an LDS scratch array, then one thread per node adds
// the products of the up to 8 elements around it in a fixed order and applies
// the pass's vector update.
#include "internal.h"
#include "ke_code.h"

namespace topo {

namespace {

// Phase 1 of an operator pass: every element's product E_e KE u_e, stored per
// corner q = dx + 2 dy + 4 dz and component c at scr[(3 q + c) ne + e].  The
// caller synchronises before phase 2 reads it.
template <typename T>
__device__ void element_products(const Grid &g, const T *__restrict__ E, const HadaW<T> &hw,
                                 const T *__restrict__ u, T *__restrict__ scr) {
  const int ne = (int)g.nel(), NX = g.NX(), NY = g.NY();
  for (int e = threadIdx.x; e < ne; e += blockDim.x) {
    const int i = e % g.nx, j = (e / g.nx) % g.ny, k = e / (g.nx * g.ny);
    const int n0 = i + NX * (j + NY * k);
    T Pb[3][4], Pt[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T vb[4], vt[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = n0 + (q & 1) + NX * (q >> 1);
        vb[q] = u[3 * n + c];
        vt[q] = u[3 * (n + NX * NY) + c];
      }
      xy_pass(vb, Pb[c]);
      xy_pass(vt, Pt[c]);
    }
    T h[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        h[c][r] = Pb[c][r] + Pt[c][r];
        h[c][r + 4] = Pb[c][r] - Pt[c][r];
      }
    const T Ee = E[e];
    T w[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) w[t] = Ee * hw.w[t];
    T gm[3][8];
    hada_blocks(w, h, gm);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T yb[4], yt[4], ob[4], ot[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        yb[r] = gm[c][r] + gm[c][r + 4];
        yt[r] = gm[c][r] - gm[c][r + 4];
      }
      xy_pass(yb, ob);
      xy_pass(yt, ot);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        scr[(3 * q + c) * ne + e] = ob[q];
        scr[(3 * (q + 4) + c) * ne + e] = ot[q];
      }
    }
  }
}

// Phase 2: (A u) at the three dofs of node (i, j, k), free rows only (every
// operand is zero on fixed dofs; callers handle fixed rows), the elements
// around the node added in a fixed order.
template <typename T>
__device__ __forceinline__ void node_product(const Grid &g, const T *__restrict__ scr, int i, int j, int k,
                                             T y[3]) {
  const int ne = (int)g.nel();
  y[0] = y[1] = y[2] = T(0);
#pragma unroll
  for (int e8 = 0; e8 < 8; ++e8) {
    const int ex = e8 & 1, ey = (e8 >> 1) & 1, ez = e8 >> 2;
    const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
    if (ei < 0 || ei >= g.nx || ej < 0 || ej >= g.ny || ek < 0 || ek >= g.nz) continue;
    const int e = ei + g.nx * (ej + g.ny * ek);
    const int q = (1 - ex) + 2 * (1 - ey) + 4 * (1 - ez);  // this node's corner in the element
#pragma unroll
    for (int c = 0; c < 3; ++c) y[c] += scr[(3 * q + c) * ne + e];
  }
}

__device__ __forceinline__ void node_ijk(const Grid &g, int n, int &i, int &j, int &k) {
  i = n % g.NX();
  j = (n / g.NX()) % g.NY();
  k = n / (g.NX() * g.NY());
}

// pre-smoothing from x = 0: on exit x and res = b - A x
template <typename T>
__device__ void pre_smooth(const TailArgs<T> &a, const TailLevel<T> &L, T *scr) {
  const Grid &g = L.g;
  const int nn = (int)g.nnodes();
  for (int d = threadIdx.x; d < 3 * nn; d += blockDim.x) {
    const T v = L.b[d] * L.dinv[d] * a.s0;
    L.d0[d] = v;
    L.x[d] = v;
    L.res[d] = L.b[d];
  }
  __syncthreads();
  T *dc = L.d0, *dn = L.d1;
  for (int s = 1; s <= L.deg; ++s) {
    const bool last = s == L.deg;
    element_products(g, L.E, a.hw, dc, scr);
    __syncthreads();
    for (int n = threadIdx.x; n < nn; n += blockDim.x) {
      int i, j, k;
      node_ijk(g, n, i, j, k);
      T y[3];
      node_product(g, scr, i, j, k, y);
      const uint8_t f = L.fixed[n];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int d = 3 * n + c;
        const T r = ((f >> c) & 1) ? T(0) : L.res[d] - y[c];
        L.res[d] = r;
        if (!last) {
          const T step = a.c1[s] * dc[d] + a.c2[s] * L.dinv[d] * r;
          dn[d] = step;
          L.x[d] += step;
        }
      }
    }
    __syncthreads();
    T *t = dc;
    dc = dn;
    dn = t;
  }
}

// post-smoothing from the current x
template <typename T>
__device__ void post_smooth(const TailArgs<T> &a, const TailLevel<T> &L, T *scr) {
  const Grid &g = L.g;
  const int nn = (int)g.nnodes();
  // res = b - A x; d0 = D^-1 res / theta (added to x together with the next step)
  element_products(g, L.E, a.hw, L.x, scr);
  __syncthreads();
  for (int n = threadIdx.x; n < nn; n += blockDim.x) {
    int i, j, k;
    node_ijk(g, n, i, j, k);
    T y[3];
    node_product(g, scr, i, j, k, y);
    const uint8_t f = L.fixed[n];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int d = 3 * n + c;
      const T r = ((f >> c) & 1) ? T(0) : L.b[d] - y[c];
      L.res[d] = r;
      L.d0[d] = r * L.dinv[d] * a.s0;
    }
  }
  __syncthreads();
  if (L.deg == 1) {
    for (int d = threadIdx.x; d < 3 * nn; d += blockDim.x) L.x[d] += L.d0[d];
    __syncthreads();
    return;
  }
  T *dc = L.d0, *dn = L.d1;
  for (int s = 1; s < L.deg; ++s) {
    element_products(g, L.E, a.hw, dc, scr);
    __syncthreads();
    for (int n = threadIdx.x; n < nn; n += blockDim.x) {
      int i, j, k;
      node_ijk(g, n, i, j, k);
      T y[3];
      node_product(g, scr, i, j, k, y);
      const uint8_t f = L.fixed[n];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int d = 3 * n + c;
        const T r = ((f >> c) & 1) ? T(0) : L.res[d] - y[c];
        L.res[d] = r;
        const T step = a.c1[s] * dc[d] + a.c2[s] * L.dinv[d] * r;
        dn[d] = step;
        L.x[d] += (s == 1) ? dc[d] + step : step;
      }
    }
    __syncthreads();
    T *t = dc;
    dc = dn;
    dn = t;
  }
}

template <typename T>
__device__ void restrict_to(const TailLevel<T> &F, const TailLevel<T> &Cl) {
  const Grid &gf = F.g, &gc = Cl.g;
  const int nc = (int)gc.nnodes();
  for (int m = threadIdx.x; m < nc; m += blockDim.x) {
    int I, J, K;
    node_ijk(gc, m, I, J, K);
    T s0 = 0, s1 = 0, s2 = 0;
    for (int dz = -1; dz <= 1; ++dz) {
      const int k = 2 * K + dz;
      if (k < 0 || k > gf.nz) continue;
      for (int dy = -1; dy <= 1; ++dy) {
        const int j = 2 * J + dy;
        if (j < 0 || j > gf.ny) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          const int i = 2 * I + dx;
          if (i < 0 || i > gf.nx) continue;
          const T w = (T)(dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0);
          const int64_t n = i + (int64_t)gf.NX() * (j + (int64_t)gf.NY() * k);
          s0 = fma(w, F.res[3 * n + 0], s0);
          s1 = fma(w, F.res[3 * n + 1], s1);
          s2 = fma(w, F.res[3 * n + 2], s2);
        }
      }
    }
    const uint8_t f = Cl.fixed[m];
    Cl.b[3 * m + 0] = (f & 1) ? T(0) : s0;
    Cl.b[3 * m + 1] = (f & 2) ? T(0) : s1;
    Cl.b[3 * m + 2] = (f & 4) ? T(0) : s2;
  }
  __syncthreads();
}

template <typename T>
__device__ void prolong_add(const TailLevel<T> &F, const TailLevel<T> &Cl) {
  const Grid &gf = F.g, &gc = Cl.g;
  const int nf = (int)gf.nnodes();
  for (int n = threadIdx.x; n < nf; n += blockDim.x) {
    int i, j, k;
    node_ijk(gf, n, i, j, k);
    const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
    const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (k & 1) ? 2 : 1;
    const T w = ((i & 1) ? T(0.5) : T(1)) * ((j & 1) ? T(0.5) : T(1)) * ((k & 1) ? T(0.5) : T(1));
    T s0 = 0, s1 = 0, s2 = 0;
    for (int c = 0; c < nk; ++c)
      for (int b = 0; b < nj; ++b)
        for (int a = 0; a < ni; ++a) {
          const int64_t m = (I0 + a) + (int64_t)gc.NX() * ((J0 + b) + (int64_t)gc.NY() * (K0 + c));
          s0 += Cl.x[3 * m + 0];
          s1 += Cl.x[3 * m + 1];
          s2 += Cl.x[3 * m + 2];
        }
    const uint8_t f = F.fixed[n];
    if (!(f & 1)) F.x[3 * n + 0] = fma(w, s0, F.x[3 * n + 0]);
    if (!(f & 2)) F.x[3 * n + 1] = fma(w, s1, F.x[3 * n + 1]);
    if (!(f & 4)) F.x[3 * n + 2] = fma(w, s2, F.x[3 * n + 2]);
  }
  __syncthreads();
}

}  // namespace

// Every vector, modulus and flag of the tail lives in LDS for the whole launch
// (layout per level: E | dinv | b | x | res | d0 | d1 | fixed); only the first level's right-hand side comes in from global memory
// and its correction x goes back out.
template <typename T>
__global__ __launch_bounds__(kTailThreads) void vcycle_tail_kernel(TailArgs<T> a) {
  if (a.skip && *a.skip) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char tail_smem[];
  // level l's arrays in LDS, rebuilt from the offsets whenever needed (kept in
  // registers, never stored, so the compiler knows they are LDS addresses)
  auto lev = [&](int l) {
    size_t off = 0;
    for (int q = 0; q < l; ++q) off += tail_level_bytes<T>(a.L[q].g);
    const Grid g = a.L[l].g;
    const int64_t nd = g.ndof(), ne = g.nel();
    T *base = reinterpret_cast<T *>(tail_smem + off);
    TailLevel<T> d;
    d.g = g;
    d.E = base;
    d.dinv = base + ne;
    d.b = base + ne + nd;
    d.x = d.b + nd;
    d.res = d.x + nd;
    d.d0 = d.res + nd;
    d.d1 = d.d0 + nd;
    d.fixed = reinterpret_cast<const uint8_t *>(d.d1 + nd);
    d.deg = a.L[l].deg;
    return d;
  };
  // copy-in as one flat loop over every (level, array) segment, so all the
  // global loads of a thread are independent and in flight together
  {
    int64_t total = 0;
    for (int l = 0; l < a.nlev; ++l) total += a.L[l].g.nel() + a.L[l].g.ndof() + a.L[l].g.nnodes();
    total += a.L[0].g.ndof();  // right-hand side of the first level
    for (int64_t q = threadIdx.x; q < total; q += blockDim.x) {
      int64_t r = q;
      if (r < a.L[0].g.ndof()) {
        lev(0).b[r] = a.L[0].b[r];
        continue;
      }
      r -= a.L[0].g.ndof();
      for (int l = 0; l < a.nlev; ++l) {
        const TailLevel<T> &G = a.L[l];
        const int64_t ne = G.g.nel(), nd = G.g.ndof(), nn = G.g.nnodes();
        if (r < ne) {
          const_cast<T *>(lev(l).E)[r] = G.E[r];
          break;
        }
        r -= ne;
        if (r < nd) {
          const_cast<T *>(lev(l).dinv)[r] = G.dinv[r];
          break;
        }
        r -= nd;
        if (r < nn) {
          const_cast<uint8_t *>(lev(l).fixed)[r] = G.fixed[r];
          break;
        }
        r -= nn;
      }
    }
  }
  __syncthreads();
  // element scratch after the levels and the solve partials
  auto scratch = [&]() {
    size_t ofs = tail_solve_bytes<T>(a.ncoarse);
    for (int q = 0; q < a.nlev; ++q) ofs += tail_level_bytes<T>(a.L[q].g);
    return reinterpret_cast<T *>(tail_smem + ofs);
  };
  const int last = a.nlev - 1;
  for (int l = 0; l < last; ++l) {
    const TailLevel<T> F = lev(l), Cl = lev(l + 1);
    pre_smooth(a, F, scratch());
    restrict_to(F, Cl);
  }
  // coarsest level: x = Ainv b.  Each row is split into kColParts contiguous
  // column chunks, one per thread, so every thread issues all its loads at once;
  // the partial sums meet in LDS (after the levels' arrays) and are added in a
  // fixed order.
  {
    const TailLevel<T> C = lev(last);
    size_t pofs = 0;
    for (int q = 0; q < a.nlev; ++q) pofs += tail_level_bytes<T>(a.L[q].g);
    double *part = reinterpret_cast<double *>(tail_smem + pofs);  // FP64 in every precision
    const int n = a.ncoarse, chunk = (n + kColParts - 1) / kColParts;
    for (int t = threadIdx.x; t < kColParts * n; t += blockDim.x) {
      const int r = t / kColParts, q = t % kColParts;
      const int c0 = q * chunk, c1 = min(n, c0 + chunk);
      const double *row = a.Ainv + (int64_t)r * n;
      double s = 0;
      for (int c = c0; c < c1; ++c) s = fma(row[c], (double)C.b[c], s);
      part[t] = s;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
      double s = 0;
#pragma unroll
      for (int q = 0; q < kColParts; ++q) s += part[kColParts * r + q];
      C.x[r] = (T)s;
    }
    __syncthreads();
  }
  for (int l = last - 1; l >= 0; --l) {
    const TailLevel<T> F = lev(l), Cl = lev(l + 1);
    prolong_add(F, Cl);
    post_smooth(a, F, scratch());
  }
  {
    const TailLevel<T> F = lev(0);
    for (int64_t q = threadIdx.x; q < a.L[0].g.ndof(); q += blockDim.x) a.L[0].x[q] = F.x[q];
  }
}

template <typename T>
hipError_t prepare_vcycle_tail_t(size_t smem_bytes) {
  return hipFuncSetAttribute((const void *)vcycle_tail_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)smem_bytes);
}

template <typename T>
hipError_t launch_vcycle_tail_t(hipStream_t s, const TailArgs<T> &a) {
  if (a.nlev < 1 || a.nlev > kTailMaxLevels || a.deg < 1 || a.deg >= kTailMaxDeg) return hipErrorInvalidValue;
  size_t bytes = tail_solve_bytes<T>(a.ncoarse) + tail_scratch_bytes<T>(a.L[0].g);
  for (int l = 0; l < a.nlev; ++l) bytes += tail_level_bytes<T>(a.L[l].g);
  if (bytes > kTailMaxLds) return hipErrorInvalidValue;
  vcycle_tail_kernel<T><<<1, kTailThreads, bytes, s>>>(a);
  return hipGetLastError();
}

template hipError_t launch_vcycle_tail_t<double>(hipStream_t, const TailArgs<double> &);
template hipError_t launch_vcycle_tail_t<float>(hipStream_t, const TailArgs<float> &);
template hipError_t prepare_vcycle_tail_t<double>(size_t);
template hipError_t prepare_vcycle_tail_t<float>(size_t);

}  // namespace topo
