// BF16 matrix-core variant of the network's implicit GEMM (same operand modes
// and epilogue as the FP32 kernel in kernels_nn.hip): operands are rounded to
// BF16 while they are staged into LDS and multiplied on the gfx950 matrix
// cores with v_mfma_f32_16x16x32_bf16, accumulating in FP32.
//
// Block = 4 waves side by side along N; each wave owns all 16*MT rows of the
// block tile and 16*NT columns, i.e. MT x NT accumulator tiles of 16 x 16.
// K advances in slabs of 32.  Fragment layout of the instruction (one wave):
//   A (16 x 32): lane l holds row l % 16, k = 8 (l / 16) .. +7
//   B (32 x 16): lane l holds column l % 16, k = 8 (l / 16) .. +7
//   D (16 x 16): lane l holds column l % 16, rows 4 (l / 16) .. +3
// so both operands are stored in LDS k-contiguous (row = m or n) and every lane
// reads its fragment with one 16-byte load.
#include <algorithm>

#include "nn.h"

namespace topo {

namespace {
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
constexpr int kKs = 32;       // k per slab
constexpr int kPitch = 40;    // LDS row pitch in bf16 (32 + 8 keeps 16-byte alignment)
__device__ __forceinline__ bool skipped(const int *skip) { return skip != nullptr && *skip != 0; }

struct Pos {
  int b, x, y, z;
};

__device__ __forceinline__ Pos decode_pos(int64_t n, const Dim3 &g) {
  const int64_t V = g.count();
  Pos p;
  p.b = (int)(n / V);
  int64_t o = n - (int64_t)p.b * V;
  p.x = (int)(o % g.x);
  o /= g.x;
  p.y = (int)(o % g.y);
  p.z = (int)(o / g.y);
  return p;
}

__device__ __forceinline__ void advance(Pos &p, const Dim3 &g) {
  if (++p.x < g.x) return;
  p.x = 0;
  if (++p.y < g.y) return;
  p.y = 0;
  if (++p.z < g.z) return;
  p.z = 0;
  ++p.b;
}

// X[ch][b][o*s + t - 1] on gi (0 outside)
__device__ __forceinline__ float gat_conv(const float *__restrict__ src, const ConvGeo &g, int ch, const Pos &c,
                                          int t) {
  const int px = c.x * g.stride + t % 3 - 1;
  const int py = c.y * g.stride + (t / 3) % 3 - 1;
  const int pz = c.z * g.stride + t / 9 - 1;
  if (px < 0 || px >= g.gi.x || py < 0 || py >= g.gi.y || pz < 0 || pz >= g.gi.z) return 0.0f;
  return src[((int64_t)ch * g.B + c.b) * g.gi.count() + px + (int64_t)g.gi.x * (py + (int64_t)g.gi.y * pz)];
}

// Y[ch][b][q] with q s = p - t + 1 (p on gi, q on go)
__device__ __forceinline__ float gat_convt(const float *__restrict__ src, const ConvGeo &g, int ch, const Pos &c,
                                           int t) {
  int qx = c.x - (t % 3 - 1), qy = c.y - ((t / 3) % 3 - 1), qz = c.z - (t / 9 - 1);
  if (qx < 0 || qy < 0 || qz < 0) return 0.0f;
  if (g.stride == 2) {
    if ((qx | qy | qz) & 1) return 0.0f;
    qx >>= 1;
    qy >>= 1;
    qz >>= 1;
  }
  if (qx >= g.go.x || qy >= g.go.y || qz >= g.go.z) return 0.0f;
  return src[((int64_t)ch * g.B + c.b) * g.go.count() + qx + (int64_t)g.go.x * (qy + (int64_t)g.go.y * qz)];
}
}  // namespace

template <int MODE, int MT, int NT>
__global__ __launch_bounds__(256) void igemm_mfma_kernel(GemmArgs a, int kchunk) {
  if (skipped(a.skip)) return;
  constexpr int TM = 16 * MT, TN = 64 * NT;
  constexpr bool kNMajor = MODE != GB_PLAINT && MODE != GB_WGRAD;
  __shared__ __attribute__((aligned(16))) __bf16 As[TM * kPitch];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[TN * kPitch];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kb = blockIdx.z * kchunk, ke = min(a.K, kb + kchunk);
  float *C = a.C + (int64_t)blockIdx.z * a.M * a.ldc;
  const ConvGeo &g = a.geo;

  // B staging: each thread owns one column of the slab and KPT consecutive k
  constexpr int TPC = 256 / TN;       // threads per column (1 or 2)
  constexpr int KPT = kKs / TPC;      // k per thread (32 or 16)
  const int bcol = tid / TPC;         // column within the block tile
  const int bk0 = (tid % TPC) * KPT;  // first k of this thread within a slab
  const int n_b = n0 + bcol;
  const bool col_ok = n_b < a.N;
  Pos pcol{};
  if (kNMajor && col_ok) {
    if (MODE == GB_CONV) pcol = decode_pos(n_b, g.go);
    else if (MODE == GB_CONVT) pcol = decode_pos(n_b, g.gi);
  }
  // A staging: thread -> (row, 8 consecutive k)
  const int arow = tid >> 2, ak0 = (tid & 3) * 8;

  f32x4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = kb; k0 < ke; k0 += kKs) {
    // ---- A slab [TM][32]
    if (arow < TM) {
      const int m = m0 + arow;
      bf16x8 v;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = k0 + ak0 + q;
        v[q] = (__bf16)((m < a.M && k < ke) ? a.A[(int64_t)m * a.sam + (int64_t)k * a.sak] : 0.0f);
      }
      *reinterpret_cast<bf16x8 *>(&As[arow * kPitch + ak0]) = v;
    }
    // ---- B slab [TN][32] (column-major: k contiguous)
    if (kNMajor) {
      __bf16 vals[KPT];
#pragma unroll
      for (int q = 0; q < KPT; ++q) {
        const int k = k0 + bk0 + q;
        float v = 0.0f;
        if (col_ok && k < ke) {
          if (MODE == GB_PLAIN) v = a.src[(int64_t)k * a.N + n_b];
          else if (MODE == GB_CONV) v = gat_conv(a.src, g, k / 27, pcol, k % 27);
          else v = gat_convt(a.src, g, k / 27, pcol, k % 27);
        }
        vals[q] = (__bf16)v;
      }
#pragma unroll
      for (int q = 0; q < KPT; q += 8) {
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = vals[q + e];
        *reinterpret_cast<bf16x8 *>(&Bs[bcol * kPitch + bk0 + q]) = v;
      }
    } else {
      // k runs over spatial positions (b, o) on go, column n = (ci, t) or ci.
      // The lanes take consecutive k (one position each, so a column's gather
      // is one contiguous run), every thread all columns c0 + 8 j of the tile.
      constexpr int CPT = TN / (256 / kKs);
      const int kk = tid % kKs, c0 = tid / kKs;
      const int k = k0 + kk;
      const bool k_ok = k < ke;
      Pos pk{};
      if (MODE == GB_WGRAD && k_ok) pk = decode_pos(k, g.go);
      float v[CPT];
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        const int n = n0 + c0 + 8 * j;
        v[j] = 0.0f;
        if (k_ok && n < a.N) {
          if (MODE == GB_PLAINT) v[j] = a.src[(int64_t)n * a.K + k];
          else v[j] = gat_conv(a.src, g, n / 27, pk, n % 27);
        }
      }
#pragma unroll
      for (int j = 0; j < CPT; ++j) Bs[(c0 + 8 * j) * kPitch + kk] = (__bf16)v[j];
    }
    __syncthreads();
    // ---- matrix-core products
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 af[MT], bfr[NT];
#pragma unroll
    for (int i = 0; i < MT; ++i) af[i] = *reinterpret_cast<const bf16x8 *>(&As[(16 * i + fr) * kPitch + fk]);
#pragma unroll
    for (int j = 0; j < NT; ++j)
      bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs[(wave * 16 * NT + 16 * j + fr) * kPitch + fk]);
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }

  // ---- epilogue: D lane layout = column lane % 16, rows 4 (lane / 16) + r
  const int col_l = lane & 15, row_l = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + 16 * i + row_l + r;
      if (m >= a.M) continue;
      const float bias = a.bias ? a.bias[m] : 0.0f;
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int n = n0 + wave * 16 * NT + 16 * j + col_l;
        if (n >= a.N) continue;
        float *c = C + (int64_t)m * a.ldc + n;
        float v = acc[i][j][r] + bias;
        if (a.accumulate) v += *c;
        if (a.relu) v = fmaxf(v, 0.0f);
        *c = v;
      }
    }
}

template <int MODE, int MT, int NT>
static hipError_t mfma_launch(hipStream_t s, const GemmArgs &a, int kz, int kchunk) {
  constexpr int TM = 16 * MT, TN = 64 * NT;
  const dim3 grid((unsigned)((a.N + TN - 1) / TN), (unsigned)((a.M + TM - 1) / TM), (unsigned)kz);
  igemm_mfma_kernel<MODE, MT, NT><<<grid, 256, 0, s>>>(a, kchunk);
  return hipGetLastError();
}

template <int MODE>
static hipError_t mfma_shape(hipStream_t s, const GemmArgs &a, int kz, int kchunk) {
  if (a.M <= 16) return mfma_launch<MODE, 1, 4>(s, a, kz, kchunk);
  if (a.M <= 32) return mfma_launch<MODE, 2, 4>(s, a, kz, kchunk);
  return mfma_launch<MODE, 4, 2>(s, a, kz, kchunk);
}

static hipError_t mfma_mode(hipStream_t s, int mode, const GemmArgs &a, int kz, int kchunk) {
  switch (mode) {
    case GB_PLAIN: return mfma_shape<GB_PLAIN>(s, a, kz, kchunk);
    case GB_PLAINT: return mfma_shape<GB_PLAINT>(s, a, kz, kchunk);
    case GB_CONV: return mfma_shape<GB_CONV>(s, a, kz, kchunk);
    case GB_CONVT: return mfma_shape<GB_CONVT>(s, a, kz, kchunk);
    case GB_WGRAD: return mfma_shape<GB_WGRAD>(s, a, kz, kchunk);
  }
  return hipErrorInvalidValue;
}

// out[m][n] (+)= sum over slices z of part[z][m][n], z in order
__global__ void mfma_sum_slices_kernel(int M, int N, int nz, const float *part, float *out, int64_t ldc,
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

hipError_t launch_igemm_bf16(hipStream_t s, int mode, const GemmArgs &a, float *split_buf, int64_t split_cap) {
  if (a.M <= 0 || a.N <= 0 || a.K <= 0) return hipErrorInvalidValue;
  const int TM = a.M <= 16 ? 16 : (a.M <= 32 ? 32 : 64);
  const int TN = a.M <= 32 ? 256 : 128;
  const int64_t tiles = (int64_t)((a.N + TN - 1) / TN) * ((a.M + TM - 1) / TM);
  int kz = 1;
  if (split_buf && tiles < 512 && a.K >= 2048) {
    kz = (int)std::min<int64_t>({64, (a.K + 1023) / 1024, (1024 + tiles - 1) / tiles});
    while (kz > 1 && (int64_t)kz * a.M * a.N > split_cap) --kz;
  }
  if (kz <= 1) return mfma_mode(s, mode, a, 1, a.K);
  const int kchunk = ((a.K + kz - 1) / kz + kKs - 1) / kKs * kKs;
  kz = (a.K + kchunk - 1) / kchunk;
  GemmArgs p = a;
  p.C = split_buf;
  p.ldc = a.N;
  p.bias = nullptr;
  p.relu = 0;
  p.accumulate = 0;
  hipError_t e = mfma_mode(s, mode, p, kz, kchunk);
  if (e != hipSuccess) return e;
  const int64_t MN = (int64_t)a.M * a.N;
  mfma_sum_slices_kernel<<<(unsigned)((MN + 255) / 256), 256, 0, s>>>(a.M, a.N, kz, split_buf, a.C, a.ldc,
                                                                      a.accumulate, a.skip);
  return hipGetLastError();
}

}  // namespace topo
