// Geometric multigrid pieces: trilinear transfers between a grid and the grid of
// half the resolution (odd fine counts round up: the coarse grid extends half a
// coarse element past the fine domain), coarse Dirichlet flags, and the dense
// coarsest-level operator with its explicit inverse.
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
__global__ void restrict_kernel(Grid gf, Grid gc, const T *__restrict__ rf,
                                const uint8_t *__restrict__ fixc, T *__restrict__ rc,
                                const int *skip) {
  if (skip && *skip) return;
  const int m = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (m >= (int)gc.nnodes()) return;
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
  rc[3 * (int64_t)m + 0] = (f & 1) ? T(0) : s0;
  rc[3 * (int64_t)m + 1] = (f & 2) ? T(0) : s1;
  rc[3 * (int64_t)m + 2] = (f & 4) ? T(0) : s2;
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
__global__ void prolong_add_kernel(Grid gf, Grid gc, const T *__restrict__ ec,
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
  const uint8_t f = fixf[n];
  T *__restrict__ xn = xf + 3 * (int64_t)n;
  if (!(f & 1)) xn[0] = fma(w, s0, xn[0]);
  if (!(f & 2)) xn[1] = fma(w, s1, xn[1]);
  if (!(f & 4)) xn[2] = fma(w, s2, xn[2]);
}

hipError_t launch_prolong_add(hipStream_t s, Grid gf, Grid gc, const double *ec,
                              const uint8_t *fixf, double *xf, const int *skip) {
  if (gf.nnodes() >= INT32_MAX) return hipErrorInvalidValue;
  prolong_add_kernel<double><<<nblocks(gf.nnodes()), kBs, 0, s>>>(gf, gc, ec, fixf, xf, skip);
  return hipGetLastError();
}
hipError_t launch_prolong_add(hipStream_t s, Grid gf, Grid gc, const float *ec,
                              const uint8_t *fixf, float *xf, const int *skip) {
  if (gf.nnodes() >= INT32_MAX) return hipErrorInvalidValue;
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

// Dense n x n operator of a (small) level, row-major; thread per row: the row of
// dof (node i, component c) collects E_e KE[3 li + c][3 lb + d] over the elements
// around i.  Fixed rows/columns become identity rows/columns.
__global__ void dense_assemble_kernel(Grid g, const double *E, Kappa kap, const uint8_t *fixed,
                                      double *A) {
  const int64_t n = g.ndof();
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  double *Ar = A + row * n;
  for (int64_t c = 0; c < n; ++c) Ar[c] = 0.0;
  const int64_t node = row / 3;
  const int comp = (int)(row % 3);
  if ((fixed[node] >> comp) & 1) {
    Ar[row] = 1.0;
    return;
  }
  const int i = (int)(node % g.NX());
  const int j = (int)((node / g.NX()) % g.NY());
  const int k = (int)(node / ((int64_t)g.NX() * g.NY()));
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
    const int ei = i - 1 + ex, ej = j - 1 + ey, ek = k - 1 + ez;
    if (ei < 0 || ei >= g.nx || ej < 0 || ej >= g.ny || ek < 0 || ek >= g.nz) continue;
    const double Ee = E[ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek)];
    const int li = corner_of(1 - ex, 1 - ey, 1 - ez);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int64_t nb = (ei + cx(b)) + (int64_t)g.NX() * ((ej + cy(b)) + (int64_t)g.NY() * (ek + cz(b)));
      const uint8_t fb = fixed[nb];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if ((fb >> d) & 1) continue;
        const double kv = comp == 0 ? TOPO_KE(kap, 3 * li + 0, 3 * b + d)
                          : comp == 1 ? TOPO_KE(kap, 3 * li + 1, 3 * b + d)
                                      : TOPO_KE(kap, 3 * li + 2, 3 * b + d);
        Ar[3 * nb + d] += Ee * kv;
      }
    }
  }
}

hipError_t launch_dense_assemble(hipStream_t s, Grid g, const double *E, const Kappa &kap,
                                 const uint8_t *fixed, double *A) {
  dense_assemble_kernel<<<nblocks(g.ndof()), kBs, 0, s>>>(g, E, kap, fixed, A);
  return hipGetLastError();
}

// In-place Gauss-Jordan inversion of an SPD matrix (no pivoting is needed for
// SPD matrices) by one workgroup.  Small matrices live in LDS for the whole
// elimination; larger ones stay in global memory and each thread updates its
// entries in register batches so the loads of a batch are in flight together.
constexpr int kInvThreads = 1024;
constexpr int kMaxDense = 2048;
constexpr int kLdsDense = 140;  // n*n doubles + pivot row/column fit in 160 KB of LDS
constexpr int kInvBatch = 8;

__device__ __forceinline__ double gj_update(double a, int i, int j, int k, double inv,
                                            const double *col, const double *rowk) {
  if (i == k) return (j == k) ? inv : rowk[j] * inv;
  if (j == k) return -col[i] * inv;
  return a - col[i] * rowk[j] * inv;
}

__global__ __launch_bounds__(kInvThreads) void dense_invert_lds_kernel(int n, double *A) {
  extern __shared__ double lds[];
  double *M = lds;                     // n*n
  double *col = lds + n * n;           // n
  double *rowk = col + n;              // n
  const int nn = n * n;
  for (int t = threadIdx.x; t < nn; t += blockDim.x) M[t] = A[t];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      col[t] = M[t * n + k];
      rowk[t] = M[k * n + t];
    }
    __syncthreads();
    const double inv = 1.0 / col[k];
    for (int idx = threadIdx.x; idx < nn; idx += blockDim.x) {
      const int i = idx / n, j = idx - (idx / n) * n;
      M[idx] = gj_update(M[idx], i, j, k, inv, col, rowk);
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < nn; t += blockDim.x) A[t] = M[t];
}

__global__ __launch_bounds__(kInvThreads) void dense_invert_kernel(int n, double *A) {
  __shared__ double col[kMaxDense];
  __shared__ double rowk[kMaxDense];
  const int64_t nn = (int64_t)n * n;
  for (int k = 0; k < n; ++k) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      col[t] = A[(int64_t)t * n + k];
      rowk[t] = A[(int64_t)k * n + t];
    }
    __syncthreads();
    const double inv = 1.0 / col[k];
    for (int64_t base = threadIdx.x; base < nn; base += (int64_t)blockDim.x * kInvBatch) {
      double v[kInvBatch];
#pragma unroll
      for (int b = 0; b < kInvBatch; ++b) {
        const int64_t idx = base + (int64_t)b * blockDim.x;
        v[b] = idx < nn ? A[idx] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < kInvBatch; ++b) {
        const int64_t idx = base + (int64_t)b * blockDim.x;
        if (idx < nn) {
          const int i = (int)(idx / n), j = (int)(idx % n);
          A[idx] = gj_update(v[b], i, j, k, inv, col, rowk);
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_dense_invert(hipStream_t s, int n, double *A) {
  if (n > kMaxDense) return hipErrorInvalidValue;
  if (n <= kLdsDense) {
    const size_t shm = ((size_t)n * n + 2 * (size_t)n) * sizeof(double);
    (void)hipFuncSetAttribute((const void *)dense_invert_lds_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    dense_invert_lds_kernel<<<1, kInvThreads, shm, s>>>(n, A);
  } else {
    dense_invert_kernel<<<1, kInvThreads, 0, s>>>(n, A);
  }
  return hipGetLastError();
}

// y = A x, one wave per row
template <typename T>
__global__ void dense_matvec_kernel(int n, const T *A, const T *x, T *y,
                                    const int *skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (row >= n) return;
  T t = 0;
  for (int c = lane; c < n; c += 64) t = fma(A[(int64_t)row * n + c], x[c], t);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
  if (lane == 0) y[row] = t;
}

hipError_t launch_dense_matvec(hipStream_t s, int n, const double *A, const double *x, double *y,
                               const int *skip) {
  const int rows_per_block = kBs / 64;
  dense_matvec_kernel<double><<<(unsigned)((n + rows_per_block - 1) / rows_per_block), kBs, 0, s>>>(n, A, x, y, skip);
  return hipGetLastError();
}
hipError_t launch_dense_matvec(hipStream_t s, int n, const float *A, const float *x, float *y,
                               const int *skip) {
  const int rows_per_block = kBs / 64;
  dense_matvec_kernel<float><<<(unsigned)((n + rows_per_block - 1) / rows_per_block), kBs, 0, s>>>(n, A, x, y, skip);
  return hipGetLastError();
}

}  // namespace topo
