// Geometric multigrid pieces: trilinear transfers between a grid and the grid of
// half the resolution (odd fine counts round up: the coarse grid extends half a
// coarse element past the fine domain), coarse Dirichlet flags, and the dense
// coarsest-level operator with its explicit inverse.
#include <algorithm>

#include "group_host.h"
#include "internal.h"
#include "ke_code.h"

namespace topo {

namespace {
constexpr int kBs = 256;
inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBs - 1) / kBs); }
}  // namespace

// r_c = P^T r_f: each coarse node gathers the fine nodes within one fine spacing
// of its position 2*(I,J,K), weight prod over axes (1 at distance 0, 1/2 at 1).
// Branch-free: a neighbour outside the fine grid is read at a clamped (valid)
// index with weight 0, which adds an exact zero.
template <typename T>
__device__ __forceinline__ void restrict_node(const Grid &gf, const Grid &gc, const T *__restrict__ rf,
                                              const uint8_t *__restrict__ fixc, int m, T (&out)[3]) {
  const int NXc = gc.NX(), NYc = gc.NY(), NXf = gf.NX(), NYf = gf.NY();
  const int I = m % NXc, J = (m / NXc) % NYc, K = m / (NXc * NYc);
  int xi[3], yj[3], zk[3];
  T wx[3], wy[3], wz[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T wd = d == 1 ? T(1) : T(0.5);
    const int i = 2 * I + d - 1, j = 2 * J + d - 1, k = 2 * K + d - 1;
    xi[d] = min(max(i, 0), gf.nx);
    yj[d] = min(max(j, 0), gf.ny);
    zk[d] = min(max(k, 0), gf.nz);
    wx[d] = (i >= 0 && i <= gf.nx) ? wd : T(0);
    wy[d] = (j >= 0 && j <= gf.ny) ? wd : T(0);
    wz[d] = (k >= 0 && k <= gf.nz) ? wd : T(0);
  }
  T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const T *__restrict__ row = rf + 3 * ((int64_t)(zk[dz] * NYf + yj[dy]) * NXf);
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const T w = wx[dx] * (wy[dy] * wz[dz]);
        const T *__restrict__ v = row + 3 * xi[dx];
        s0 = fma(w, v[0], s0);
        s1 = fma(w, v[1], s1);
        s2 = fma(w, v[2], s2);
      }
    }
  const uint8_t f = fixc[m];
  out[0] = (f & 1) ? T(0) : s0;
  out[1] = (f & 2) ? T(0) : s1;
  out[2] = (f & 4) ? T(0) : s2;
}
template <typename T>
__device__ __forceinline__ void restrict_body(const Grid &gf, const Grid &gc, const T *__restrict__ rf,
                                              const uint8_t *__restrict__ fixc, T *__restrict__ rc,
                                              const int *skip) {
  if (skip && *skip) return;
  const int m = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (m >= (int)gc.nnodes()) return;
  T o[3];
  restrict_node<T>(gf, gc, rf, fixc, m, o);
  rc[3 * (int64_t)m + 0] = o[0];
  rc[3 * (int64_t)m + 1] = o[1];
  rc[3 * (int64_t)m + 2] = o[2];
}

template <typename T>
__global__ void restrict_kernel(Grid gf, Grid gc, const T *__restrict__ rf, const uint8_t *__restrict__ fixc,
                                T *__restrict__ rc, const int *skip) {
  restrict_body<T>(gf, gc, rf, fixc, rc, skip);
}
template <typename T>
__global__ void restrict_group_kernel(Grid gf, Grid gc, GroupTab<TransferArgs<T>> t) {
  const TransferArgs<T> &a = t.v[blockIdx.z];
  restrict_body<T>(gf, gc, a.in, a.fixed, a.out, a.skip);
}

hipError_t launch_restrict(hipStream_t s, Grid gf, Grid gc, const double *rf, const uint8_t *fixc,
                           double *rc, const int *skip) {
  if (gf.nnodes() >= INT32_MAX) return hipErrorInvalidValue;
  restrict_kernel<double><<<nblocks(gc.nnodes()), kBs, 0, s>>>(gf, gc, rf, fixc, rc, skip);
  return hipGetLastError();
}
hipError_t launch_restrict(hipStream_t s, Grid gf, Grid gc, const float *rf, const uint8_t *fixc,
                           float *rc, const int *skip) {
  if (gf.nnodes() >= INT32_MAX) return hipErrorInvalidValue;
  restrict_kernel<float><<<nblocks(gc.nnodes()), kBs, 0, s>>>(gf, gc, rf, fixc, rc, skip);
  return hipGetLastError();
}

// x_f += P e_c on free fine dofs (trilinear interpolation of the coarse values):
// a fine node on an odd index of an axis sits between two coarse nodes (weight
// 1/2 each), on an even one on a coarse node (weight 1).  Branch-free: the 8
// candidate coarse values are always read (clamped), the unused ones with a 0
// multiplier, which adds an exact zero to the sum.
template <typename T>
__device__ __forceinline__ void prolong_add_body(const Grid &gf, const Grid &gc, const T *__restrict__ ec,
                                                 const uint8_t *__restrict__ fixf, T *__restrict__ xf,
                                                 const int *skip) {
  if (skip && *skip) return;
  const int n = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (n >= (int)gf.nnodes()) return;
  const int NXf = gf.NX(), NYf = gf.NY(), NXc = gc.NX(), NYc = gc.NY();
  const int i = n % NXf, j = (n / NXf) % NYf, k = n / (NXf * NYf);
  const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
  const int I1 = min(I0 + 1, gc.nx), J1 = min(J0 + 1, gc.ny), K1 = min(K0 + 1, gc.nz);
  const T ia = (i & 1) ? T(1) : T(0), jb = (j & 1) ? T(1) : T(0), kc = (k & 1) ? T(1) : T(0);
  const T w = ((i & 1) ? T(0.5) : T(1)) * ((j & 1) ? T(0.5) : T(1)) * ((k & 1) ? T(0.5) : T(1));
  T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const T inc_cb = (c ? kc : T(1)) * (b ? jb : T(1));
      const T *__restrict__ row = ec + 3 * ((int64_t)((c ? K1 : K0) * NYc + (b ? J1 : J0)) * NXc);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T inc = inc_cb * (a ? ia : T(1));
        const T *__restrict__ v = row + 3 * (a ? I1 : I0);
        s0 = fma(inc, v[0], s0);
        s1 = fma(inc, v[1], s1);
        s2 = fma(inc, v[2], s2);
      }
    }
  // the node's x read with the other loads and written back whole (a fixed dof
  // keeps its value): no load-wait-store round trip per component at the end
  const uint8_t f = fixf[n];
  T *__restrict__ xn = xf + 3 * (int64_t)n;
  const T x0 = xn[0], x1 = xn[1], x2 = xn[2];
  xn[0] = (f & 1) ? x0 : fma(w, s0, x0);
  xn[1] = (f & 2) ? x1 : fma(w, s1, x1);
  xn[2] = (f & 4) ? x2 : fma(w, s2, x2);
}

// The same prolongation per coarse cell (I, J, K), for large fine grids: the
// up to 8 fine nodes (2I + a, 2J + b, 2K + c) take the sums of prolong_add_body
// (the same 8 terms in the same order, the same weights: bit for bit) from the
// cell's 8 coarse values, read once instead of once per fine node.
constexpr int64_t kProlongCellNodes = 500000;  // fine nodes from which the cell form is used
template <typename T>
__device__ __forceinline__ void prolong_cell_body(const Grid &gf, const Grid &gc, const T *__restrict__ ec,
                                                  const uint8_t *__restrict__ fixf, T *__restrict__ xf,
                                                  const int *skip) {
  if (skip && *skip) return;
  const int NXf = gf.NX(), NYf = gf.NY(), NZf = gf.NZ(), NXc = gc.NX(), NYc = gc.NY();
  const int CX = (NXf + 1) / 2, CY = (NYf + 1) / 2, CZ = (NZf + 1) / 2;
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= CX * CY * CZ) return;
  const int I = t % CX, J = (t / CX) % CY, K = t / (CX * CY);
  const int I1 = min(I + 1, gc.nx), J1 = min(J + 1, gc.ny), K1 = min(K + 1, gc.nz);
  T v[2][2][2][3];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T *__restrict__ p = ec + 3 * ((int64_t)((c ? K1 : K) * NYc + (b ? J1 : J)) * NXc + (a ? I1 : I));
        v[c][b][a][0] = p[0];
        v[c][b][a][1] = p[1];
        v[c][b][a][2] = p[2];
      }
#pragma unroll
  for (int fk = 0; fk < 2; ++fk)
#pragma unroll
    for (int fj = 0; fj < 2; ++fj)
#pragma unroll
      for (int fi = 0; fi < 2; ++fi) {
        const int i = 2 * I + fi, j = 2 * J + fj, k = 2 * K + fk;
        if (i >= NXf || j >= NYf || k >= NZf) continue;
        const T ia = fi ? T(1) : T(0), jb = fj ? T(1) : T(0), kc = fk ? T(1) : T(0);
        const T w = (fi ? T(0.5) : T(1)) * (fj ? T(0.5) : T(1)) * (fk ? T(0.5) : T(1));
        T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const T inc_cb = (c ? kc : T(1)) * (b ? jb : T(1));
#pragma unroll
            for (int a = 0; a < 2; ++a) {
              const T inc = inc_cb * (a ? ia : T(1));
              s0 = fma(inc, v[c][b][a][0], s0);
              s1 = fma(inc, v[c][b][a][1], s1);
              s2 = fma(inc, v[c][b][a][2], s2);
            }
          }
        const int64_t n = i + (int64_t)NXf * (j + (int64_t)NYf * k);
        const uint8_t f = fixf[n];
        T *__restrict__ xn = xf + 3 * n;
        const T x0 = xn[0], x1 = xn[1], x2 = xn[2];
        xn[0] = (f & 1) ? x0 : fma(w, s0, x0);
        xn[1] = (f & 2) ? x1 : fma(w, s1, x1);
        xn[2] = (f & 4) ? x2 : fma(w, s2, x2);
      }
}
template <typename T>
__global__ void prolong_cell_kernel(Grid gf, Grid gc, const T *__restrict__ ec, const uint8_t *__restrict__ fixf,
                                    T *__restrict__ xf, const int *skip) {
  prolong_cell_body<T>(gf, gc, ec, fixf, xf, skip);
}
template <typename T>
__global__ void prolong_cell_group_kernel(Grid gf, Grid gc, GroupTab<TransferArgs<T>> t) {
  const TransferArgs<T> &a = t.v[blockIdx.z];
  prolong_cell_body<T>(gf, gc, a.in, a.fixed, a.out, a.skip);
}
inline int64_t prolong_cells(const Grid &gf) {
  return (int64_t)((gf.NX() + 1) / 2) * ((gf.NY() + 1) / 2) * ((gf.NZ() + 1) / 2);
}

template <typename T>
__global__ void prolong_add_kernel(Grid gf, Grid gc, const T *__restrict__ ec, const uint8_t *__restrict__ fixf,
                                   T *__restrict__ xf, const int *skip) {
  prolong_add_body<T>(gf, gc, ec, fixf, xf, skip);
}
template <typename T>
__global__ void prolong_add_group_kernel(Grid gf, Grid gc, GroupTab<TransferArgs<T>> t) {
  const TransferArgs<T> &a = t.v[blockIdx.z];
  prolong_add_body<T>(gf, gc, a.in, a.fixed, a.out, a.skip);
}

hipError_t launch_prolong_add(hipStream_t s, Grid gf, Grid gc, const double *ec,
                              const uint8_t *fixf, double *xf, const int *skip) {
  if (gf.nnodes() >= INT32_MAX) return hipErrorInvalidValue;
  if (gf.nnodes() >= kProlongCellNodes)
    prolong_cell_kernel<double><<<nblocks(prolong_cells(gf)), kBs, 0, s>>>(gf, gc, ec, fixf, xf, skip);
  else
    prolong_add_kernel<double><<<nblocks(gf.nnodes()), kBs, 0, s>>>(gf, gc, ec, fixf, xf, skip);
  return hipGetLastError();
}
hipError_t launch_prolong_add(hipStream_t s, Grid gf, Grid gc, const float *ec,
                              const uint8_t *fixf, float *xf, const int *skip) {
  if (gf.nnodes() >= INT32_MAX) return hipErrorInvalidValue;
  if (gf.nnodes() >= kProlongCellNodes)
    prolong_cell_kernel<float><<<nblocks(prolong_cells(gf)), kBs, 0, s>>>(gf, gc, ec, fixf, xf, skip);
  else
    prolong_add_kernel<float><<<nblocks(gf.nnodes()), kBs, 0, s>>>(gf, gc, ec, fixf, xf, skip);
  return hipGetLastError();
}

// coarse dof fixed iff the fine dof at the coincident node (clamped into the
// fine grid) is fixed
__global__ void coarse_fixed_kernel(Grid gf, Grid gc, const uint8_t *fixf, uint8_t *fixc) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= gc.nnodes()) return;
  const int I = (int)(m % gc.NX());
  const int J = (int)((m / gc.NX()) % gc.NY());
  const int K = (int)(m / ((int64_t)gc.NX() * gc.NY()));
  const int i = min(2 * I, gf.nx), j = min(2 * J, gf.ny), k = min(2 * K, gf.nz);
  fixc[m] = fixf[i + (int64_t)gf.NX() * (j + (int64_t)gf.NY() * k)];
}

hipError_t launch_coarse_fixed(hipStream_t s, Grid gf, Grid gc, const uint8_t *fixf, uint8_t *fixc) {
  coarse_fixed_kernel<<<nblocks(gc.nnodes()), kBs, 0, s>>>(gf, gc, fixf, fixc);
  return hipGetLastError();
}

// Dense n x n operator of a (small) level, row-major, on a zeroed matrix; thread
// per row: the row of dof (node i, component c) collects E_e KE[3 li + c][3 lb + d]
// over the elements around i.  Fixed rows/columns become identity rows/columns.
__global__ void zero_kernel(int64_t n, double *A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) A[t] = 0.0;
}
__global__ void zero_group_kernel(int64_t n, GroupTab<AssembleArgs> t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t.v[blockIdx.z].A[i] = 0.0;
}

// One thread per row.  The row's dof couples with the 3 components of the 27
// nodes around its node; those 81 entries are summed in registers over the up
// to 8 elements around the node (element order e = 0..7, so every entry gets
// the same additions in the same order as an in-place accumulation) and each is
// written once; the rest of the row stays zero, as do fixed columns.  Threads
// go component-major (all rows of component 0, then 1, then 2), so a wave has
// one component and the element matrix entries are compile-time indices.
template <int C>
__device__ __forceinline__ void dense_assemble_row(const Grid &g, const double *E, const Kappa &kap,
                                                   const uint8_t *fixed, double *Ar, int i, int j, int k) {
  double acc[27][3];
#pragma unroll
  for (int o = 0; o < 27; ++o)
#pragma unroll
    for (int d = 0; d < 3; ++d) acc[o][d] = 0.0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
    const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
    if (ei < 0 || ei >= g.nx || ej < 0 || ej >= g.ny || ek < 0 || ek >= g.nz) continue;
    const double Ee = E[ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek)];
    const int li = corner_of(1 - ex, 1 - ey, 1 - ez);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int o = (ex + cx(b)) + 3 * (ey + cy(b)) + 9 * (ez + cz(b));  // neighbour (di, dj, dk) + 1
#pragma unroll
      for (int d = 0; d < 3; ++d) acc[o][d] += Ee * TOPO_KE(kap, 3 * li + C, 3 * b + d);
    }
  }
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const int ni = i + o % 3 - 1, nj = j + (o / 3) % 3 - 1, nk = k + o / 9 - 1;
    if (ni < 0 || ni >= g.NX() || nj < 0 || nj >= g.NY() || nk < 0 || nk >= g.NZ()) continue;
    const int64_t nb = ni + (int64_t)g.NX() * (nj + (int64_t)g.NY() * nk);
    const uint8_t fb = fixed[nb];
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (!((fb >> d) & 1)) Ar[3 * nb + d] = acc[o][d];
  }
}
__device__ __forceinline__ void dense_assemble_body(Grid g, const double *E, const Kappa &kap,
                                                    const uint8_t *fixed, double *A) {
  const int64_t nn = g.nnodes(), n = g.ndof();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int comp = (int)(t / nn);
  const int64_t node = t - comp * nn, row = 3 * node + comp;
  double *Ar = A + row * n;
  if ((fixed[node] >> comp) & 1) {
    Ar[row] = 1.0;
    return;
  }
  const int i = (int)(node % g.NX());
  const int j = (int)((node / g.NX()) % g.NY());
  const int k = (int)(node / ((int64_t)g.NX() * g.NY()));
  if (comp == 0) dense_assemble_row<0>(g, E, kap, fixed, Ar, i, j, k);
  else if (comp == 1) dense_assemble_row<1>(g, E, kap, fixed, Ar, i, j, k);
  else dense_assemble_row<2>(g, E, kap, fixed, Ar, i, j, k);
}
__global__ __launch_bounds__(kBs) void dense_assemble_kernel(Grid g, const double *E, Kappa kap, const uint8_t *fixed,
                                      double *A) {
  dense_assemble_body(g, E, kap, fixed, A);
}
__global__ __launch_bounds__(kBs) void dense_assemble_group_kernel(Grid g, GroupTab<AssembleArgs> t) {
  const AssembleArgs &a = t.v[blockIdx.z];
  dense_assemble_body(g, a.E, a.kap, a.fixed, a.A);
}

hipError_t launch_dense_assemble(hipStream_t s, Grid g, const double *E, const Kappa &kap,
                                 const uint8_t *fixed, double *A) {
  zero_kernel<<<nblocks(g.ndof() * g.ndof()), kBs, 0, s>>>(g.ndof() * g.ndof(), A);
  dense_assemble_kernel<<<nblocks(g.ndof()), kBs, 0, s>>>(g, E, kap, fixed, A);
  return hipGetLastError();
}

hipError_t launch_dense_assemble_group(hipStream_t s, int G, Grid g, const AssembleArgs *a) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  const GroupTab<AssembleArgs> t = group_tab(G, a);
  zero_group_kernel<<<dim3(nblocks(g.ndof() * g.ndof()), 1, G), kBs, 0, s>>>(g.ndof() * g.ndof(), t);
  dense_assemble_group_kernel<<<dim3(nblocks(g.ndof()), 1, G), kBs, 0, s>>>(g, t);
  return hipGetLastError();
}

// In-place Gauss-Jordan inversion of an SPD matrix (no pivoting is needed for
// SPD matrices).  Up to kLdsDense rows one workgroup eliminates the whole matrix
// in LDS.  Larger matrices use the blocked form over panels of kGjNb columns K:
//   P = A_KK^-1                                  (one workgroup, in LDS)
//   C = A_iK for i outside K (saved), A_Kj <- P A_Kj for j outside K
//   A_ij <- A_ij - C_i A_Kj,  A_iK <- -C_i P,  A_KK <- P
// (the scalar elimination step applied to blocks), three launches per panel.
constexpr int kInvThreads = 1024;
constexpr int kMaxDense = 2048;
constexpr int kLdsDense = 140;  // n*n doubles + pivot row/column fit in 160 KB of LDS
constexpr int kGjNb = 64;       // panel width of the blocked elimination
constexpr int kGjQ = 32;        // inner-dimension chunk staged in LDS by the tile kernels

// One chunk of kGjQ inner indices of a 64 x 64 tile product on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64): wave w owns the 32 x 32 quadrant (w / 2, w % 2)
// as 2 x 2 tiles of 16 x 16.  Operand lanes: X[i][k] from lane i + 16 k, Y[k][j]
// from lane j + 16 k; result row (lane / 16) + 4 r, column lane % 16 in acc[r].
typedef double f64x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void gj_mfma_chunk(const double (*Xs)[kGjQ + 1], const double (*Ys)[kGjNb],
                                              f64x4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = (w >> 1) * 32, c0 = (w & 1) * 32, li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int q = 0; q < kGjQ; q += 4) {
    double a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = Xs[r0 + 16 * t + li][q + lk];
      b[t] = Ys[q + lk][c0 + 16 * t + li];
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
  }
}
// tile row and column of acc[ti][tj][r] of this lane
__device__ __forceinline__ int gj_acc_row(int ti, int r) {
  return ((threadIdx.x >> 6) >> 1) * 32 + 16 * ti + ((threadIdx.x & 63) >> 4) + 4 * r;
}
__device__ __forceinline__ int gj_acc_col(int tj) { return ((threadIdx.x >> 6) & 1) * 32 + 16 * tj + (threadIdx.x & 15); }

__device__ __forceinline__ double gj_update(double a, int i, int j, int k, double inv,
                                            const double *col, const double *rowk) {
  if (i == k) return (j == k) ? inv : rowk[j] * inv;
  if (j == k) return -col[i] * inv;
  return a - col[i] * rowk[j] * inv;
}

// Gauss-Jordan on the m x m row-major matrix M in LDS by the whole workgroup
// (col and rowk: m doubles of LDS each)
__device__ void gj_invert_lds(int m, double *M, double *col, double *rowk) {
  const int mm = m * m;
  for (int k = 0; k < m; ++k) {
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
      col[t] = M[t * m + k];
      rowk[t] = M[k * m + t];
    }
    __syncthreads();
    const double inv = 1.0 / col[k];
    for (int idx = threadIdx.x; idx < mm; idx += blockDim.x) {
      const int i = idx / m, j = idx - (idx / m) * m;
      M[idx] = gj_update(M[idx], i, j, k, inv, col, rowk);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void dense_invert_lds_body(int n, double *A) {
  extern __shared__ double lds[];
  double *M = lds;            // n*n
  double *col = lds + n * n;  // n
  double *rowk = col + n;     // n
  const int nn = n * n;
  for (int t = threadIdx.x; t < nn; t += blockDim.x) M[t] = A[t];
  __syncthreads();
  gj_invert_lds(n, M, col, rowk);
  for (int t = threadIdx.x; t < nn; t += blockDim.x) A[t] = M[t];
}
__global__ __launch_bounds__(kInvThreads) void dense_invert_lds_kernel(int n, double *A) {
  dense_invert_lds_body(n, A);
}
// one workgroup per matrix of the group
__global__ __launch_bounds__(kInvThreads) void dense_invert_lds_group_kernel(int n, GroupTab<double *> A) {
  dense_invert_lds_body(n, A.v[blockIdx.z]);
}

// a double from lane `lane` of the wave (two 32-bit register reads)
__device__ __forceinline__ double read_lane_f64(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, lane);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// P = A_KK^-1 for the panel K = [k0, k0 + kb), the block padded to kGjNb x kGjNb
// with the identity.  Four waves; lane c of wave w holds column c of rows
// 16 w .. 16 w + 15 in registers.  Gauss-Jordan steps on a symmetric matrix
// keep it symmetric within the eliminated indices and within the remaining
// ones and antisymmetric between the two sets, so the pivot column of step k
// is the pivot row with the signs of its eliminated entries flipped.  The wave
// holding row k publishes through LDS the row scaled by the reciprocal pivot,
// its signed copy (the column) and the reciprocal; after the step's barrier
// every wave reads them in one batch, and each element update is one product
// and one fused multiply-add.  The wave holding row k + 1 updates and publishes
// it before its other rows, so the next division overlaps them; one barrier
// per step (double-buffered LDS).  Steps past kb (the identity padding) change
// nothing in the kb x kb block and are skipped by 16s.
__device__ __forceinline__ void gj_publish(double mk, int k, int c, double *prow, double *pcol, double *pinv) {
  const double inv = 1.0 / read_lane_f64(mk, k);  // 1 / M[k][k]
  prow[c] = mk * inv;
  pcol[c] = c < k ? -mk : mk;  // M[c][k]
  if (c == 0) *pinv = inv;
}

// one elimination step on the wave's rows but row `skip`: column k becomes
// -M[r][k] / M[k][k] (keep 0, coef 1 / M[k][k]), every other column subtracts
// M[r][k] times the scaled pivot row (keep 1)
__device__ __forceinline__ void gj_rows(double (&M)[16], const double (&pc)[16], double keep, double coef,
                                        int skip) {
#pragma unroll
  for (int i = 0; i < 16; ++i)
    if (i != skip) M[i] = fma(-pc[i], coef, keep * M[i]);
}

__device__ __forceinline__ void gj_panel_inv_body(int n, const double *A, int k0, int kb, double *P) {
  __shared__ double prow[2][kGjNb], pcol[2][kGjNb], pinv[2];
  const int c = threadIdx.x % kGjNb;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kGjNb);  // wave-uniform
  double M[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = 16 * w + i;
    M[i] = (r < kb && c < kb) ? A[(int64_t)(k0 + r) * n + k0 + c] : (r == c ? 1.0 : 0.0);
  }
  if (w == 0) gj_publish(M[0], 0, c, prow[0], pcol[0], &pinv[0]);
  for (int kw = 0; kw < 4 && 16 * kw < kb; ++kw) {
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 16 * kw + kk, b = k & 1;
      __syncthreads();
      double pc[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) pc[i] = pcol[b][16 * w + i];
      const double pr = prow[b][c], inv = pinv[b];
      const double keep = c == k ? 0.0 : 1.0, coef = c == k ? inv : pr;
      const int in = (kk + 1) % 16;  // register of row k + 1 in its wave
      if (k + 1 < kGjNb && w == (k + 1) / 16) {
        M[in] = fma(-pc[in], coef, keep * M[in]);
        gj_publish(M[in], k + 1, c, prow[b ^ 1], pcol[b ^ 1], &pinv[b ^ 1]);
        gj_rows(M, pc, keep, coef, in);
      } else {
        gj_rows(M, pc, keep, coef, -1);
      }
      if (w == kw) M[kk] = c == k ? inv : pr;  // the pivot row itself
    }
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = 16 * w + i;
    if (r < kb && c < kb) P[r * kb + c] = M[i];
  }
}
__global__ __launch_bounds__(256) void gj_panel_inv_kernel(int n, const double *A, int k0, int kb,
                                                           double *P) {
  gj_panel_inv_body(n, A, k0, kb, P);
}
__global__ __launch_bounds__(256) void gj_panel_inv_group_kernel(int n, GroupTab<double *> A, int k0, int kb,
                                                                 GroupTab<double *> W) {
  gj_panel_inv_body(n, A.v[blockIdx.z], k0, kb, W.v[blockIdx.z]);
}

// Blocks 0..nt-1: A_Kj <- P A_Kj on column tile j (the panel's own tile skipped);
// one block reads its whole kb x kGjNb input before writing it back.
// Blocks nt..2nt-1: C_i = A_iK on row tile i (rows outside K), C row-major n x kb.
// The two roles touch disjoint parts of A.
__device__ __forceinline__ void gj_panel_rows_body(int n, double *A, int k0, int kb, const double *P, double *C) {
  const int nt = (n + kGjNb - 1) / kGjNb, kt = k0 / kGjNb;
  if ((int)blockIdx.x >= nt) {
    const int it = blockIdx.x - nt;
    if (it == kt) return;
    const int i0 = it * kGjNb, rows = min(kGjNb, n - i0);
    for (int t = threadIdx.x; t < rows * kb; t += blockDim.x) {
      const int r = t / kb, q = t % kb;
      C[(int64_t)(i0 + r) * kb + q] = A[(int64_t)(i0 + r) * n + k0 + q];
    }
    return;
  }
  const int jt = blockIdx.x;
  if (jt == kt) return;
  const int j0 = jt * kGjNb, cols = min(kGjNb, n - j0);
  __shared__ double Ps[kGjNb][kGjQ + 1];
  __shared__ double Bs[kGjQ][kGjNb];
  f64x4 acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = f64x4{0.0, 0.0, 0.0, 0.0};
  constexpr int NL = kGjNb * kGjQ / 256;
  for (int q0 = 0; q0 < kb; q0 += kGjQ) {
    double pv[NL], bv[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {  // every load of the chunk before the first LDS store
      const int t = threadIdx.x + 256 * u;
      const int r = t / kGjQ, q = t % kGjQ;
      pv[u] = (r < kb && q0 + q < kb) ? P[r * kb + q0 + q] : 0.0;
      const int qb = t / kGjNb, c = t % kGjNb;
      bv[u] = (q0 + qb < kb && c < cols) ? A[(int64_t)(k0 + q0 + qb) * n + j0 + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int t = threadIdx.x + 256 * u;
      Ps[t / kGjQ][t % kGjQ] = pv[u];
      Bs[t / kGjNb][t % kGjNb] = bv[u];
    }
    __syncthreads();
    gj_mfma_chunk(Ps, Bs, acc);
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = gj_acc_row(ti, q), c = gj_acc_col(tj);
        if (r < kb && c < cols) A[(int64_t)(k0 + r) * n + j0 + c] = acc[ti][tj][q];
      }
}
__global__ __launch_bounds__(256) void gj_panel_rows_kernel(int n, double *A, int k0, int kb,
                                                            const double *P, double *C) {
  gj_panel_rows_body(n, A, k0, kb, P, C);
}
__global__ __launch_bounds__(256) void gj_panel_rows_group_kernel(int n, GroupTab<double *> A, int k0, int kb,
                                                                  GroupTab<double *> W) {
  double *P = W.v[blockIdx.z];
  gj_panel_rows_body(n, A.v[blockIdx.z], k0, kb, P, P + kGjNb * kGjNb);
}

// Tile (i, j) of kGjNb x kGjNb: A_ij <- A_ij - C_i A_Kj (j outside K), A_iK <- -C_i P,
// A_KK <- P; the panel's rows are otherwise final already.
__device__ __forceinline__ void gj_update_body(int n, double *A, int k0, int kb, const double *P,
                                               const double *C) {
  const int kt = k0 / kGjNb, it = blockIdx.y, jt = blockIdx.x;
  const int i0 = it * kGjNb, j0 = jt * kGjNb;
  const int rows = min(kGjNb, n - i0), cols = min(kGjNb, n - j0);
  if (it == kt) {
    if (jt == kt)
      for (int t = threadIdx.x; t < kb * kb; t += blockDim.x)
        A[(int64_t)(k0 + t / kb) * n + k0 + t % kb] = P[t];
    return;
  }
  const bool panel = jt == kt;
  __shared__ double Cs[kGjNb][kGjQ + 1];
  __shared__ double Bs[kGjQ][kGjNb];
  f64x4 acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = f64x4{0.0, 0.0, 0.0, 0.0};
  // the tile entries this lane updates, loaded first (their latency hides
  // behind the staging and the products)
  double old[2][2][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = gj_acc_row(ti, q), c = gj_acc_col(tj);
        old[ti][tj][q] = (!panel && r < rows && c < cols) ? A[(int64_t)(i0 + r) * n + j0 + c] : 0.0;
      }
  constexpr int NL = kGjNb * kGjQ / 256;
  for (int q0 = 0; q0 < kb; q0 += kGjQ) {
    double cv[NL], bv[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {  // every load of the chunk before the first LDS store
      const int t = threadIdx.x + 256 * u;
      const int r = t / kGjQ, q = t % kGjQ;
      cv[u] = (r < rows && q0 + q < kb) ? C[(int64_t)(i0 + r) * kb + q0 + q] : 0.0;
      const int qb = t / kGjNb, c = t % kGjNb;
      bv[u] = 0.0;
      if (q0 + qb < kb && c < cols)
        bv[u] = panel ? P[(q0 + qb) * kb + c] : A[(int64_t)(k0 + q0 + qb) * n + j0 + c];
    }
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int t = threadIdx.x + 256 * u;
      Cs[t / kGjQ][t % kGjQ] = cv[u];
      Bs[t / kGjNb][t % kGjNb] = bv[u];
    }
    __syncthreads();
    gj_mfma_chunk(Cs, Bs, acc);
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = gj_acc_row(ti, q), c = gj_acc_col(tj);
        if (r < rows && c < cols)
          A[(int64_t)(i0 + r) * n + j0 + c] = panel ? -acc[ti][tj][q] : old[ti][tj][q] - acc[ti][tj][q];
      }
}
__global__ __launch_bounds__(256) void gj_update_kernel(int n, double *A, int k0, int kb,
                                                        const double *P, const double *C) {
  gj_update_body(n, A, k0, kb, P, C);
}
__global__ __launch_bounds__(256) void gj_update_group_kernel(int n, GroupTab<double *> A, int k0, int kb,
                                                              GroupTab<double *> W) {
  const double *P = W.v[blockIdx.z];
  gj_update_body(n, A.v[blockIdx.z], k0, kb, P, P + kGjNb * kGjNb);
}

size_t dense_invert_work(int n) {
  return n <= kLdsDense ? 0 : (size_t)kGjNb * kGjNb + (size_t)n * kGjNb;
}

hipError_t launch_dense_invert(hipStream_t s, int n, double *A, double *work) {
  if (n < 1 || n > kMaxDense) return hipErrorInvalidValue;
  if (n <= kLdsDense) {
    const size_t shm = ((size_t)n * n + 2 * (size_t)n) * sizeof(double);
    (void)hipFuncSetAttribute((const void *)dense_invert_lds_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    dense_invert_lds_kernel<<<1, kInvThreads, shm, s>>>(n, A);
    return hipGetLastError();
  }
  if (!work) return hipErrorInvalidValue;
  double *P = work, *C = work + kGjNb * kGjNb;
  const int nt = (n + kGjNb - 1) / kGjNb;
  for (int k0 = 0; k0 < n; k0 += kGjNb) {
    const int kb = std::min(kGjNb, n - k0);
    gj_panel_inv_kernel<<<1, 256, 0, s>>>(n, A, k0, kb, P);
    gj_panel_rows_kernel<<<2 * nt, 256, 0, s>>>(n, A, k0, kb, P, C);
    gj_update_kernel<<<dim3(nt, nt), 256, 0, s>>>(n, A, k0, kb, P, C);
  }
  return hipGetLastError();
}

hipError_t launch_dense_invert_group(hipStream_t s, int G, int n, double *const *A, double *const *work) {
  if (!group_ok(G) || n < 1 || n > kMaxDense) return hipErrorInvalidValue;
  const GroupTab<double *> a = group_tab(G, A);
  if (n <= kLdsDense) {
    const size_t shm = ((size_t)n * n + 2 * (size_t)n) * sizeof(double);
    (void)hipFuncSetAttribute((const void *)dense_invert_lds_group_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    dense_invert_lds_group_kernel<<<dim3(1, 1, G), kInvThreads, shm, s>>>(n, a);
    return hipGetLastError();
  }
  for (int i = 0; i < G; ++i)
    if (!work[i]) return hipErrorInvalidValue;
  const GroupTab<double *> w = group_tab(G, work);
  const int nt = (n + kGjNb - 1) / kGjNb;
  for (int k0 = 0; k0 < n; k0 += kGjNb) {
    const int kb = std::min(kGjNb, n - k0);
    gj_panel_inv_group_kernel<<<dim3(1, 1, G), 256, 0, s>>>(n, a, k0, kb, w);
    gj_panel_rows_group_kernel<<<dim3(2 * nt, 1, G), 256, 0, s>>>(n, a, k0, kb, w);
    gj_update_group_kernel<<<dim3(nt, nt, G), 256, 0, s>>>(n, a, k0, kb, w);
  }
  return hipGetLastError();
}

// y = A x, one wave per row; A is the FP64 inverse in every precision (the
// products and the row sum run in FP64, single-precision vectors are widened and
// the result rounded once): the coarse operator is ill-conditioned, and an FP32
// copy of its inverse loses percents of accuracy at a thousand dofs
template <typename T>
__device__ __forceinline__ void dense_matvec_rows(int n, const double *A, const T *x, T *y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (row >= n) return;
  // four independent partial sums per lane so the row's loads overlap
  const double *Ar = A + (int64_t)row * n;
  double t0 = 0, t1 = 0, t2 = 0, t3 = 0;
  int c = lane;
  for (; c + 192 < n; c += 256) {
    t0 = fma(Ar[c], (double)x[c], t0);
    t1 = fma(Ar[c + 64], (double)x[c + 64], t1);
    t2 = fma(Ar[c + 128], (double)x[c + 128], t2);
    t3 = fma(Ar[c + 192], (double)x[c + 192], t3);
  }
  for (; c < n; c += 64) t0 = fma(Ar[c], (double)x[c], t0);
  double t = (t0 + t1) + (t2 + t3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
  if (lane == 0) y[row] = (T)t;
}
template <typename T>
__device__ __forceinline__ void dense_matvec_body(int n, const double *A, const T *x, T *y, const int *skip) {
  if (skip && *skip) return;
  dense_matvec_rows<T>(n, A, x, y);
}

// The coarsest solve fused with the restriction into it: every block forms the
// whole coarsest right-hand side R r_f in LDS (restrict_node: the values of the
// transfer kernel) and then its rows of x = Ainv b (the sums of the mat-vec),
// one launch instead of two; the coarsest b itself is not stored (nothing
// else reads it).  n = 3 nnodes(gc) <= kMaxDense.
template <typename T>
__device__ __forceinline__ void restrict_solve_body(const Grid &gf, const Grid &gc, const T *rf,
                                                    const uint8_t *fixc, int n, const double *A, T *y,
                                                    const int *skip) {
  if (skip && *skip) return;
  __shared__ T bs[kMaxDense];
  const int nn = (int)gc.nnodes();
  for (int m = threadIdx.x; m < nn; m += blockDim.x) {
    T o[3];
    restrict_node<T>(gf, gc, rf, fixc, m, o);
    bs[3 * m + 0] = o[0];
    bs[3 * m + 1] = o[1];
    bs[3 * m + 2] = o[2];
  }
  __syncthreads();
  dense_matvec_rows<T>(n, A, bs, y);
}
constexpr int kRsThreads = 512;  // the restriction phase covers 512 coarse nodes in one round
template <typename T>
__global__ __launch_bounds__(kRsThreads) void restrict_solve_kernel(Grid gf, Grid gc, const T *rf,
                                                                    const uint8_t *fixc, int n, const double *A,
                                                                    T *y, const int *skip) {
  restrict_solve_body<T>(gf, gc, rf, fixc, n, A, y, skip);
}
template <typename T>
__global__ __launch_bounds__(kRsThreads) void restrict_solve_group_kernel(Grid gf, Grid gc, int n,
                                                                          GroupTab<RestrictSolveArgs<T>> t) {
  const RestrictSolveArgs<T> &a = t.v[blockIdx.z];
  restrict_solve_body<T>(gf, gc, a.rf, a.fixed, n, a.A, a.y, a.skip);
}

template <typename T>
__global__ void dense_matvec_kernel(int n, const double *A, const T *x, T *y, const int *skip) {
  dense_matvec_body<T>(n, A, x, y, skip);
}
template <typename T>
__global__ void dense_matvec_group_kernel(int n, GroupTab<MatvecArgs<T>> t) {
  const MatvecArgs<T> &a = t.v[blockIdx.z];
  dense_matvec_body<T>(n, a.A, a.x, a.y, a.skip);
}

hipError_t launch_dense_matvec(hipStream_t s, int n, const double *A, const double *x, double *y,
                               const int *skip) {
  const int rows_per_block = kBs / 64;
  dense_matvec_kernel<double><<<(unsigned)((n + rows_per_block - 1) / rows_per_block), kBs, 0, s>>>(n, A, x, y, skip);
  return hipGetLastError();
}
hipError_t launch_dense_matvec(hipStream_t s, int n, const double *A, const float *x, float *y,
                               const int *skip) {
  const int rows_per_block = kBs / 64;
  dense_matvec_kernel<float><<<(unsigned)((n + rows_per_block - 1) / rows_per_block), kBs, 0, s>>>(n, A, x, y, skip);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_solve(hipStream_t s, Grid gf, Grid gc, const T *rf, const uint8_t *fixc, int n,
                                 const double *A, T *y, const int *skip) {
  if (n != gc.ndof() || n > kMaxDense || gf.nnodes() >= INT32_MAX) return hipErrorInvalidValue;
  const int rows_per_block = kRsThreads / 64;
  restrict_solve_kernel<T><<<(unsigned)((n + rows_per_block - 1) / rows_per_block), kRsThreads, 0, s>>>(
      gf, gc, rf, fixc, n, A, y, skip);
  return hipGetLastError();
}
template hipError_t launch_restrict_solve<double>(hipStream_t, Grid, Grid, const double *, const uint8_t *, int,
                                                  const double *, double *, const int *);
template hipError_t launch_restrict_solve<float>(hipStream_t, Grid, Grid, const float *, const uint8_t *, int,
                                                 const double *, float *, const int *);
template <typename T>
hipError_t launch_restrict_solve_group(hipStream_t s, int G, Grid gf, Grid gc, int n,
                                       const RestrictSolveArgs<T> *a) {
  if (G < 1 || G > kMaxGroup || n != gc.ndof() || n > kMaxDense || gf.nnodes() >= INT32_MAX)
    return hipErrorInvalidValue;
  GroupTab<RestrictSolveArgs<T>> t{};
  for (int i = 0; i < G; ++i) t.v[i] = a[i];
  const int rows_per_block = kRsThreads / 64;
  restrict_solve_group_kernel<T><<<dim3((unsigned)((n + rows_per_block - 1) / rows_per_block), 1, G), kRsThreads, 0,
                                   s>>>(gf, gc, n, t);
  return hipGetLastError();
}
template hipError_t launch_restrict_solve_group<double>(hipStream_t, int, Grid, Grid, int,
                                                        const RestrictSolveArgs<double> *);
template hipError_t launch_restrict_solve_group<float>(hipStream_t, int, Grid, Grid, int,
                                                       const RestrictSolveArgs<float> *);

// grouped launchers: one launch for G problems of the same grids
template <typename T>
hipError_t launch_restrict_group(hipStream_t s, int G, Grid gf, Grid gc, const TransferArgs<T> *a) {
  if (G < 1 || G > kMaxGroup || gf.nnodes() >= INT32_MAX) return hipErrorInvalidValue;
  GroupTab<TransferArgs<T>> t{};
  for (int i = 0; i < G; ++i) t.v[i] = a[i];
  restrict_group_kernel<T><<<dim3(nblocks(gc.nnodes()), 1, G), kBs, 0, s>>>(gf, gc, t);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_prolong_add_group(hipStream_t s, int G, Grid gf, Grid gc, const TransferArgs<T> *a) {
  if (G < 1 || G > kMaxGroup || gf.nnodes() >= INT32_MAX) return hipErrorInvalidValue;
  GroupTab<TransferArgs<T>> t{};
  for (int i = 0; i < G; ++i) t.v[i] = a[i];
  if (gf.nnodes() >= kProlongCellNodes)
    prolong_cell_group_kernel<T><<<dim3(nblocks(prolong_cells(gf)), 1, G), kBs, 0, s>>>(gf, gc, t);
  else
    prolong_add_group_kernel<T><<<dim3(nblocks(gf.nnodes()), 1, G), kBs, 0, s>>>(gf, gc, t);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_dense_matvec_group(hipStream_t s, int G, int n, const MatvecArgs<T> *a) {
  if (G < 1 || G > kMaxGroup) return hipErrorInvalidValue;
  GroupTab<MatvecArgs<T>> t{};
  for (int i = 0; i < G; ++i) t.v[i] = a[i];
  const int rows_per_block = kBs / 64;
  dense_matvec_group_kernel<T><<<dim3((unsigned)((n + rows_per_block - 1) / rows_per_block), 1, G), kBs, 0, s>>>(n, t);
  return hipGetLastError();
}
template hipError_t launch_restrict_group<double>(hipStream_t, int, Grid, Grid, const TransferArgs<double> *);
template hipError_t launch_restrict_group<float>(hipStream_t, int, Grid, Grid, const TransferArgs<float> *);
template hipError_t launch_prolong_add_group<double>(hipStream_t, int, Grid, Grid, const TransferArgs<double> *);
template hipError_t launch_prolong_add_group<float>(hipStream_t, int, Grid, Grid, const TransferArgs<float> *);
template hipError_t launch_dense_matvec_group<double>(hipStream_t, int, int, const MatvecArgs<double> *);
template hipError_t launch_dense_matvec_group<float>(hipStream_t, int, int, const MatvecArgs<float> *);

}  // namespace topo
