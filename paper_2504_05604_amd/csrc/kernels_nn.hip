// Kernels of the convolutional preconditioner network: every convolution, its
// transpose and its weight gradient is one implicit GEMM whose B operand is
// gathered from the activation tensor while it is staged into LDS (no im2col
// buffer), plus the input/output scaling, the training loss, bias/ReLU
// gradients and the Adam update.
//
// Activations are channel-major over a batch, X[c][b][v] with v the node index
// (x fastest), so channel concatenation is adjacency in memory.  Arithmetic is
// FP32 with FP32 accumulation; every reduction has a fixed order (no atomics).
#include <algorithm>

#include "nn.h"
#include "reduce_dev.h"

namespace topo {

namespace {
constexpr int kBs = 256;
inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBs - 1) / kBs); }
__device__ __forceinline__ bool skipped(const int *skip) { return skip != nullptr && *skip != 0; }
}  // namespace

// ---------------------------------------------------------------------------
// implicit GEMM
constexpr int kTK = 16;

// coordinates (batch, x, y, z) of a column on a node grid
struct Col {
  int b, x, y, z;
  bool ok;
};

__device__ __forceinline__ Col decode(int n, int N, const Dim3 &g) {
  Col c;
  c.ok = n < N;
  const int64_t V = g.count();
  const int nn = c.ok ? n : 0;
  c.b = (int)(nn / V);
  int64_t o = nn - (int64_t)c.b * V;
  c.x = (int)(o % g.x);
  o /= g.x;
  c.y = (int)(o % g.y);
  c.z = (int)(o / g.y);
  return c;
}

// X[ch][b][p] at p = o*s + t - 1 (CONV / WGRAD gather); 0 outside gi
__device__ __forceinline__ float gather_conv(const float *__restrict__ src, const ConvGeo &g, int ch,
                                             const Col &c, int t) {
  const int px = c.x * g.stride + t % 3 - 1;
  const int py = c.y * g.stride + (t / 3) % 3 - 1;
  const int pz = c.z * g.stride + t / 9 - 1;
  if (px < 0 || px >= g.gi.x || py < 0 || py >= g.gi.y || pz < 0 || pz >= g.gi.z) return 0.0f;
  const int64_t Vi = g.gi.count();
  return src[((int64_t)ch * g.B + c.b) * Vi + px + (int64_t)g.gi.x * (py + (int64_t)g.gi.y * pz)];
}

// Y[ch][b][q] with q*s = p - t + 1 (CONVT gather; c holds the fine point p)
__device__ __forceinline__ float gather_convt(const float *__restrict__ src, const ConvGeo &g, int ch,
                                              const Col &c, int t) {
  int qx = c.x - (t % 3 - 1), qy = c.y - ((t / 3) % 3 - 1), qz = c.z - (t / 9 - 1);
  if (qx < 0 || qy < 0 || qz < 0) return 0.0f;
  if (g.stride == 2) {
    if ((qx | qy | qz) & 1) return 0.0f;
    qx >>= 1;
    qy >>= 1;
    qz >>= 1;
  }
  if (qx >= g.go.x || qy >= g.go.y || qz >= g.go.z) return 0.0f;
  const int64_t Vo = g.go.count();
  return src[((int64_t)ch * g.B + c.b) * Vo + qx + (int64_t)g.go.x * (qy + (int64_t)g.go.y * qz)];
}

// 256 threads as 16 x 16; thread (tx, ty) owns rows ty + 16 i (i < RM) and
// columns tx + 16 j (j < RN) of a (16 RM) x (16 RN) tile.  K is staged in slabs
// of 16 through LDS.  blockIdx.z selects a slice of K of length kchunk whose
// partial result goes to C + z * M * ldc.
template <int MODE, int RM, int RN>
__global__ __launch_bounds__(256) void igemm_kernel(GemmArgs a, int kchunk) {
  if (skipped(a.skip)) return;
  constexpr int TM = 16 * RM, TN = 16 * RN;
  __shared__ float As[kTK][TM + 1];
  __shared__ float Bs[kTK][TN + 1];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kb = blockIdx.z * kchunk, ke = min(a.K, kb + kchunk);
  float *C = a.C + (int64_t)blockIdx.z * a.M * a.ldc;
  const ConvGeo &g = a.geo;

  // n-major B loads: each thread always loads column n0 + tid % TN
  constexpr bool kNMajor = MODE != GB_PLAINT && MODE != GB_WGRAD;
  Col col{};
  if (kNMajor) {
    const int n = n0 + tid % TN;
    if (MODE == GB_CONV) col = decode(n, a.N, g.go);
    else if (MODE == GB_CONVT) col = decode(n, a.N, g.gi);
    else col.ok = n < a.N;
  }
  const bool a_kfast = a.sak == 1;

  float acc[RM][RN];
#pragma unroll
  for (int i = 0; i < RM; ++i)
#pragma unroll
    for (int j = 0; j < RN; ++j) acc[i][j] = 0.0f;

  for (int k0 = kb; k0 < ke; k0 += kTK) {
    // A tile (TK x TM)
    if (a_kfast) {
      for (int t = tid; t < kTK * TM; t += 256) {
        const int kk = t % kTK, mm = t / kTK;
        const int m = m0 + mm, k = k0 + kk;
        As[kk][mm] = (m < a.M && k < ke) ? a.A[(int64_t)m * a.sam + k] : 0.0f;
      }
    } else {
      for (int t = tid; t < kTK * TM; t += 256) {
        const int kk = t / TM, mm = t % TM;
        const int m = m0 + mm, k = k0 + kk;
        As[kk][mm] = (m < a.M && k < ke) ? a.A[(int64_t)m * a.sam + (int64_t)k * a.sak] : 0.0f;
      }
    }
    // B tile (TK x TN)
    if (kNMajor) {
      const int nn = tid % TN;
#pragma unroll
      for (int i = 0; i < kTK * TN / 256; ++i) {
        const int kk = tid / TN + i * (256 / TN);
        const int k = k0 + kk;
        float v = 0.0f;
        if (col.ok && k < ke) {
          if (MODE == GB_PLAIN) v = a.src[(int64_t)k * a.N + n0 + nn];
          else if (MODE == GB_CONV) v = gather_conv(a.src, g, k / 27, col, k % 27);
          else v = gather_convt(a.src, g, k / 27, col, k % 27);
        }
        Bs[kk][nn] = v;
      }
    } else {
      const int kk = tid % kTK;
      const int k = k0 + kk;
      Col kc{};
      if (MODE == GB_WGRAD) kc = decode(k, ke, g.go);
#pragma unroll
      for (int i = 0; i < kTK * TN / 256; ++i) {
        const int nn = tid / kTK + i * (256 / kTK);
        const int n = n0 + nn;
        float v = 0.0f;
        if (k < ke && n < a.N) {
          if (MODE == GB_PLAINT) v = a.src[(int64_t)n * a.K + k];
          else v = gather_conv(a.src, g, n / 27, kc, n % 27);
        }
        Bs[kk][nn] = v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kTK; ++kk) {
      float av[RM], bv[RN];
#pragma unroll
      for (int i = 0; i < RM; ++i) av[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < RN; ++j) bv[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) acc[i][j] = fmaf(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < RM; ++i) {
    const int m = m0 + ty + 16 * i;
    if (m >= a.M) continue;
    const float bias = a.bias ? a.bias[m] : 0.0f;
#pragma unroll
    for (int j = 0; j < RN; ++j) {
      const int n = n0 + tx + 16 * j;
      if (n >= a.N) continue;
      float *c = C + (int64_t)m * a.ldc + n;
      float v = acc[i][j] + bias;
      if (a.accumulate) v += *c;
      if (a.relu) v = fmaxf(v, 0.0f);
      *c = v;
    }
  }
}

// out[m][n] (+)= sum over slices z of part[z][m][n], z in order
__global__ void sum_slices_kernel(int M, int N, int nz, const float *part, float *out, int64_t ldc,
                                  int accumulate, const int *skip) {
  if (skipped(skip)) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t MN = (int64_t)M * N;
  if (i >= MN) return;
  float t = 0.0f;
  for (int z = 0; z < nz; ++z) t += part[(int64_t)z * MN + i];
  float *o = out + (i / N) * ldc + i % N;
  *o = accumulate ? *o + t : t;
}

template <int MODE, int RM, int RN>
static hipError_t igemm_launch(hipStream_t s, const GemmArgs &a, int kz, int kchunk) {
  constexpr int TM = 16 * RM, TN = 16 * RN;
  const dim3 grid((unsigned)((a.N + TN - 1) / TN), (unsigned)((a.M + TM - 1) / TM), (unsigned)kz);
  igemm_kernel<MODE, RM, RN><<<grid, 256, 0, s>>>(a, kchunk);
  return hipGetLastError();
}

template <int MODE>
static hipError_t igemm_shape(hipStream_t s, const GemmArgs &a, int kz, int kchunk) {
  if (a.M <= 16) return igemm_launch<MODE, 1, 8>(s, a, kz, kchunk);
  if (a.M <= 32) return igemm_launch<MODE, 2, 8>(s, a, kz, kchunk);
  return igemm_launch<MODE, 4, 4>(s, a, kz, kchunk);
}

static hipError_t igemm_mode(hipStream_t s, int mode, const GemmArgs &a, int kz, int kchunk) {
  switch (mode) {
    case GB_PLAIN: return igemm_shape<GB_PLAIN>(s, a, kz, kchunk);
    case GB_PLAINT: return igemm_shape<GB_PLAINT>(s, a, kz, kchunk);
    case GB_CONV: return igemm_shape<GB_CONV>(s, a, kz, kchunk);
    case GB_CONVT: return igemm_shape<GB_CONVT>(s, a, kz, kchunk);
    case GB_WGRAD: return igemm_shape<GB_WGRAD>(s, a, kz, kchunk);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_igemm(hipStream_t s, int mode, const GemmArgs &a, float *split_buf, int64_t split_cap) {
  if (a.M <= 0 || a.N <= 0 || a.K <= 0) return hipErrorInvalidValue;
  const int TM = a.M <= 16 ? 16 : (a.M <= 32 ? 32 : 64);
  const int TN = a.M <= 32 ? 128 : 64;
  const int64_t tiles = (int64_t)((a.N + TN - 1) / TN) * ((a.M + TM - 1) / TM);
  // few output tiles and a long reduction (weight gradients): split K
  int kz = 1;
  if (split_buf && tiles < 512 && a.K >= 2048) {
    kz = (int)std::min<int64_t>({64, (a.K + 1023) / 1024, (1024 + tiles - 1) / tiles});
    while (kz > 1 && (int64_t)kz * a.M * a.N > split_cap) --kz;
  }
  if (kz <= 1) return igemm_mode(s, mode, a, 1, a.K);
  const int kchunk = ((a.K + kz - 1) / kz + kTK - 1) / kTK * kTK;
  kz = (a.K + kchunk - 1) / kchunk;
  GemmArgs p = a;
  p.C = split_buf;
  p.ldc = a.N;
  p.bias = nullptr;
  p.relu = 0;
  p.accumulate = 0;
  hipError_t e = igemm_mode(s, mode, p, kz, kchunk);
  if (e != hipSuccess) return e;
  const int64_t MN = (int64_t)a.M * a.N;
  sum_slices_kernel<<<nblocks(MN), kBs, 0, s>>>(a.M, a.N, kz, split_buf, a.C, a.ldc, a.accumulate, a.skip);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void transpose_w_kernel(int co, int ci, int taps, const float *W, float *WT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over W
  if (i >= (int64_t)co * ci * taps) return;
  const int t = (int)(i % taps);
  const int c = (int)((i / taps) % ci);
  const int o = (int)(i / ((int64_t)taps * ci));
  WT[((int64_t)c * co + o) * taps + t] = W[i];
}

hipError_t launch_transpose_w(hipStream_t s, int co, int ci, int taps, const float *W, float *WT) {
  transpose_w_kernel<<<nblocks((int64_t)co * ci * taps), kBs, 0, s>>>(co, ci, taps, W, WT);
  return hipGetLastError();
}

__global__ void relu_back_kernel(int64_t n, const float *Y, float *dY) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(Y[i] > 0.0f)) dY[i] = 0.0f;
}

hipError_t launch_relu_back(hipStream_t s, int64_t n, const float *Y, float *dY) {
  relu_back_kernel<<<nblocks(n), kBs, 0, s>>>(n, Y, dY);
  return hipGetLastError();
}

// Bias gradient in two fixed-order stages: blocks (channel c, slice p) sum a
// contiguous slice of channel c's row into partials[c * P + p], then one thread
// per channel adds its P partials in order.
__global__ void bias_grad_part_kernel(int64_t N, int P, const float *dY, double *partials) {
  const int c = blockIdx.y, p = blockIdx.x;
  const int64_t len = (N + P - 1) / P, i0 = (int64_t)p * len, i1 = min(N, i0 + len);
  double t = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) t += dY[(int64_t)c * N + i];
  __shared__ double part[kMaxRed];
  double v[1] = {t};
  block_reduce_store<1, false>(v, part, 0);
  __syncthreads();
  if (threadIdx.x == 0) partials[(int64_t)c * P + p] = part[0];
}

__global__ void bias_grad_sum_kernel(int C, int P, const double *partials, float *db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double t = 0.0;
  for (int p = 0; p < P; ++p) t += partials[(int64_t)c * P + p];
  db[c] = (float)t;
}

hipError_t launch_bias_grad(hipStream_t s, int C, int64_t N, const float *dY, float *db, const Reducer &red) {
  if (!db) return hipSuccess;
  const int64_t cap = (int64_t)red.max_blocks * kMaxRed;
  int P = (int)std::min<int64_t>({64, (N + 4095) / 4096, cap / std::max(1, C)});
  if (P < 1) P = 1;
  if ((int64_t)P * C > cap) return hipErrorInvalidValue;
  bias_grad_part_kernel<<<dim3((unsigned)P, (unsigned)C), kBs, 0, s>>>(N, P, dY, red.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  bias_grad_sum_kernel<<<(C + 255) / 256, 256, 0, s>>>(C, P, red.partials, db);
  return hipGetLastError();
}

__global__ void adam_kernel(int64_t n, float *w, const float *g, float *m, float *v, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(hipStream_t s, int64_t n, float *w, const float *g, float *m, float *v, float lr,
                       float b1, float b2, float eps, int step) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  adam_kernel<<<nblocks(n), kBs, 0, s>>>(n, w, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// solver-side input
__global__ void node_density_kernel(Grid g, const double *xphys, float *rho) {
  const int64_t V = g.nnodes();
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  const int i = (int)(n % g.NX()), j = (int)((n / g.NX()) % g.NY()), k = (int)(n / ((int64_t)g.NX() * g.NY()));
  double sum = 0.0;
  int cnt = 0;
  for (int e = 0; e < 8; ++e) {
    const int ei = i - 1 + (e & 1), ej = j - 1 + ((e >> 1) & 1), ek = k - 1 + (e >> 2);
    if (ei < 0 || ei >= g.nx || ej < 0 || ej >= g.ny || ek < 0 || ek >= g.nz) continue;
    sum += xphys[ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek)];
    ++cnt;
  }
  rho[n] = (float)(sum / cnt);
}

hipError_t launch_node_density(hipStream_t s, const Grid &g, const double *xphys, float *rho) {
  node_density_kernel<<<nblocks(g.nnodes()), kBs, 0, s>>>(g, xphys, rho);
  return hipGetLastError();
}

__global__ void nn_input_resid_kernel(int64_t V, const double *r, const double *rr, double *scale, float *X1,
                                      const int *skip) {
  if (skipped(skip)) return;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double q = sqrt(rr[0] / (double)(3 * V));
  const double sc = q > 0.0 ? q : 1.0;
  if (n == 0) scale[0] = sc;
  if (n >= V) return;
  const double inv = 1.0 / sc;
#pragma unroll
  for (int c = 0; c < 3; ++c) X1[(int64_t)c * V + n] = (float)(r[3 * n + c] * inv);
}

hipError_t launch_nn_input_resid(hipStream_t s, int64_t V, const double *r, const double *rr, double *scale,
                                 float *X1, const int *skip) {
  nn_input_resid_kernel<<<nblocks(V), kBs, 0, s>>>(V, r, rr, scale, X1, skip);
  return hipGetLastError();
}

__global__ void pair_out_kernel(int64_t n, const double *r, const double *ustar, const double *u, float *dr,
                                float *de) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dr[i] = (float)r[i];
  de[i] = (float)(ustar[i] - u[i]);
}

hipError_t launch_pair_out(hipStream_t s, int64_t n, const double *r, const double *ustar, const double *u,
                           float *dr, float *de) {
  pair_out_kernel<<<nblocks(n), kBs, 0, s>>>(n, r, ustar, u, dr, de);
  return hipGetLastError();
}

// training input: one block per sample for the rms, then the gather
__global__ void rms_train_kernel(int64_t n, const int *idx, const float *r, float *scale) {
  const float *rb = r + (int64_t)idx[blockIdx.x] * n;
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) t = fma((double)rb[i], (double)rb[i], t);
  __shared__ double part[kMaxRed];
  double v[1] = {t};
  block_reduce_store<1, false>(v, part, 0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double q = sqrt(part[0] / (double)n);
    scale[blockIdx.x] = (float)(q > 0.0 ? q : 1.0);
  }
}

__global__ void nn_input_train_kernel(int64_t V, int B, const int *idx, const float *rho, const float *r,
                                      const float *scale, float *X) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (n >= V) return;
  const int64_t p = idx[b];
  const float inv = 1.0f / scale[b];
  X[(int64_t)b * V + n] = rho[p * V + n];
  for (int c = 0; c < 3; ++c) X[((int64_t)(1 + c) * B + b) * V + n] = r[(p * V + n) * 3 + c] * inv;
}

hipError_t launch_nn_input_train(hipStream_t s, int64_t V, int B, const int *idx, const float *rho,
                                 const float *r, float *scale, float *X) {
  rms_train_kernel<<<B, 1024, 0, s>>>(3 * V, idx, r, scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  nn_input_train_kernel<<<dim3(nblocks(V), B), kBs, 0, s>>>(V, B, idx, rho, r, scale, X);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void nn_output_flex_kernel(int64_t V, const float *out, const double *scale, const uint8_t *fixed,
                                      const double *r, double *z, double *partials, const int *skip) {
  if (skipped(skip)) return;
  const double s = scale[0];
  double rzn = 0.0, rzo = 0.0, zz = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < V; n += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t f = fixed[n];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t d = 3 * n + c;
      const double zn = ((f >> c) & 1) ? 0.0 : s * (double)out[(int64_t)c * V + n];
      const double rv = r[d];
      rzo = fma(rv, z[d], rzo);
      rzn = fma(rv, zn, rzn);
      zz = fma(zn, zn, zz);
      z[d] = zn;
    }
  }
  double v[3] = {rzn, rzo, zz};
  block_reduce_store<3, false>(v, partials, blockIdx.x);
}

hipError_t launch_nn_output_flex(hipStream_t s, int64_t V, const float *out, const double *scale,
                                 const uint8_t *fixed, const double *r, double *z, const Reducer &red,
                                 const Fin &fin, const int *skip) {
  const unsigned nb = std::min<unsigned>(nblocks(V), 1024u);
  if ((int)nb > red.max_blocks) return hipErrorInvalidValue;
  nn_output_flex_kernel<<<nb, kBs, 0, s>>>(V, out, scale, fixed, r, z, red.partials, skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(s, red, (int)nb, 3, fin, skip);
}

__global__ void nn_output_kernel(int64_t V, const float *out, const double *scale, const uint8_t *fixed,
                                 double *z) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= V) return;
  const double s = scale[0];
  const uint8_t f = fixed[n];
  for (int c = 0; c < 3; ++c) z[3 * n + c] = ((f >> c) & 1) ? 0.0 : s * (double)out[(int64_t)c * V + n];
}

hipError_t launch_nn_output(hipStream_t s, int64_t V, const float *out, const double *scale,
                            const uint8_t *fixed, double *z) {
  nn_output_kernel<<<nblocks(V), kBs, 0, s>>>(V, out, scale, fixed, z);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// loss, two passes.  Pass 1 reduces per sample and per block
//   mode 0 (relative):  (d.d, t.t) with d = y - t, and writes dout = d;
//   mode 1 (cosine):    (y.t, y.y, t.t), writes dout = t and zeroes y on fixed dofs;
// all over the free dofs (fixed entries of dout are 0).  Pass 2 sums each
// sample's partials in block order, stores the sample loss and turns dout into
// the gradient of the batch mean:
//   mode 0: 2 d / (t.t B);  mode 1: (a/b y - t) / (sqrt(b c) B), a = y.t, b = y.y, c = t.t.
constexpr int kLossBlocks = 64;

__global__ void loss_terms_kernel(int64_t V, int B, int mode, const int *idx, float *out, const float *e,
                                  const uint8_t *fixed, const float *scale, float *dout, double *partials) {
  const int b = blockIdx.y;
  const int64_t p = idx[b];
  const float inv = 1.0f / scale[b];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < V; n += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t f = fixed[p * V + n];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t o = ((int64_t)c * B + b) * V + n;
      const bool fr = !((f >> c) & 1);
      const float t = fr ? e[(p * V + n) * 3 + c] * inv : 0.0f;
      if (mode == 0) {
        const float d = fr ? out[o] - t : 0.0f;
        s0 += (double)d * d;
        s1 += (double)t * t;
        dout[o] = d;
      } else {
        const float y = fr ? out[o] : 0.0f;
        s0 += (double)y * t;
        s1 += (double)y * y;
        s2 += (double)t * t;
        out[o] = y;
        dout[o] = t;
      }
    }
  }
  double v[3] = {s0, s1, s2};
  block_reduce_store<3, false>(v, partials, b * kLossBlocks + blockIdx.x);
}

__global__ void loss_scale_kernel(int64_t V, int B, int mode, const double *partials, const float *out,
                                  float *dout, double *loss) {
  const int b = blockIdx.y;
  __shared__ float coef[2];
  if (threadIdx.x == 0) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < kLossBlocks; ++q)
      for (int k = 0; k < 3; ++k) s[k] += partials[(size_t)(b * kLossBlocks + q) * kMaxRed + k];
    double l, c0, c1;
    if (mode == 0) {
      const double den = s[1] > 0.0 ? s[1] : 1.0;
      l = s[0] / den;
      c0 = 2.0 / (den * B);  // dout = c0 d
      c1 = 0.0;
    } else {
      const double a = s[0], yy = s[1] > 0.0 ? s[1] : 1.0, tt = s[2] > 0.0 ? s[2] : 1.0;
      const double q = sqrt(yy * tt);
      l = 1.0 - a / q;
      c0 = 1.0 / (q * B);  // dout = c0 (c1 y - t)
      c1 = a / yy;
    }
    if (blockIdx.x == 0) loss[b] = l;
    coef[0] = (float)c0;
    coef[1] = (float)c1;
  }
  __syncthreads();
  const float c0 = coef[0], c1 = coef[1];
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < V; n += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t o = ((int64_t)c * B + b) * V + n;
      dout[o] = mode == 0 ? c0 * dout[o] : c0 * (c1 * out[o] - dout[o]);
    }
}

hipError_t launch_nn_loss(hipStream_t s, int mode, int64_t V, int B, const int *idx, float *out,
                          const float *e, const uint8_t *fixed, const float *scale, float *dout,
                          const Reducer &red, double *loss) {
  if (B * kLossBlocks > red.max_blocks || (mode != 0 && mode != 1)) return hipErrorInvalidValue;
  loss_terms_kernel<<<dim3(kLossBlocks, B), kBs, 0, s>>>(V, B, mode, idx, out, e, fixed, scale, dout, red.partials);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  loss_scale_kernel<<<dim3(kLossBlocks, B), kBs, 0, s>>>(V, B, mode, red.partials, out, dout, loss);
  return hipGetLastError();
}

}  // namespace topo
