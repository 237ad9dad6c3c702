// Direct 3x3x3 convolutions of the preconditioner network on the matrix cores
// (BF16 operands, FP32 accumulation): the GB_CONV and GB_CONVT operand modes of
// the implicit GEMM (nn.h), with the activations staged per block in LDS.
//
// A block produces the outputs of a brick of 16 x BY x BZ positions q for all
// (up to 16 MT) output channels.  Per chunk of CC source channels it stages the
// source brick (the positions the brick's taps reach, zero outside the grid)
// in LDS as [position][channel] BF16, so a matrix-core B fragment -- 8
// consecutive channels of one tap at one output position -- is one 16-byte LDS
// read; the weights come pre-packed as [row][tap][channel] BF16 (packed once
// per weight update), so an A fragment is one 16-byte global read.  A K-slab of
// the v_mfma_f32_16x16x32_bf16 instruction covers 32 / CC taps of the chunk.
//
// Output position of brick point q: p = OS q + r.  OS = 1 except for the
// transpose of a stride-2 convolution, which is split into its 8 parity classes
// r: a class takes only the taps d with r - d even (1 to 8 of the 27) and reads
// the coarse source at q + (r - d) / 2, so no product with a structural zero is
// formed.  Source positions per tap: convolution (stride S) S q + d, transpose
// of a stride-1 convolution q - d.
#include <algorithm>

#include "nn.h"

namespace topo {

namespace {
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
constexpr int kBX = 16;
__device__ __forceinline__ bool skipped(const int *skip) { return skip != nullptr && *skip != 0; }

struct TapE {
  int t, ex, ey, ez;  // weight tap, source offset
};
}  // namespace

// Wp[m][t][c] = A(m, c*27 + t) as BF16, zero for m >= M or c >= Kch
__global__ void pack_bf16_kernel(const float *__restrict__ A, int64_t sam, int64_t sak, int M, int Kch, int Mp,
                                 int Cp, __bf16 *__restrict__ Wp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)Mp * 27 * Cp;
  if (i >= total) return;
  const int m = (int)(i / (27 * Cp));
  const int r = (int)(i % (27 * Cp));
  const int t = r / Cp, c = r % Cp;
  const float v = (m < M && c < Kch) ? A[(int64_t)m * sam + (int64_t)(c * 27 + t) * sak] : 0.0f;
  Wp[i] = (__bf16)v;
}

hipError_t launch_pack_bf16(hipStream_t s, const float *A, int64_t sam, int64_t sak, int M, int Kch, int Mp, int Cp,
                            void *Wp) {
  const int64_t total = (int64_t)Mp * 27 * Cp;
  pack_bf16_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(A, sam, sak, M, Kch, Mp, Cp, (__bf16 *)Wp);
  return hipGetLastError();
}

// MODE: GB_CONV or GB_CONVT; OS: 2 for the parity-class transpose of a
// stride-2 convolution, else 1; S: source stride of q (2 for a stride-2
// convolution, else 1)
template <int MODE, int OS, int S, int CC, int MT, int BY, int BZ>
__global__ __launch_bounds__(256) void conv_mfma_kernel(GemmArgs a) {
  if (skipped(a.skip)) return;
  constexpr int CCP = CC + 8;                         // LDS pitch per position (16-byte aligned, spreads banks)
  constexpr int EMIN = (OS == 2) ? 0 : -1;            // smallest source offset of a tap
  constexpr int ESPAN = (OS == 2) ? 2 : 3;            // offsets EMIN .. EMIN + ESPAN - 1
  constexpr int SX = S * (kBX - 1) + ESPAN, SY = S * (BY - 1) + ESPAN, SZ = S * (BZ - 1) + ESPAN;
  constexpr int SP = SX * SY * SZ;                    // source positions of the brick
  constexpr int NT = BY * BZ / 4;                     // 16-wide output fragments per wave
  constexpr int TPS = 32 / CC;                        // taps per K-slab
  static_assert(BY * BZ % 4 == 0 && (CC == 16 || CC == 32), "shape");
  __shared__ __attribute__((aligned(16))) __bf16 sb[SP * CCP];
  __shared__ TapE taps[27];
  __shared__ int ntap_sh;

  const ConvGeo &g = a.geo;
  // source and output grids of the mode
  const Dim3 gs = MODE == GB_CONV ? g.gi : g.go;
  const Dim3 gout = MODE == GB_CONV ? g.go : g.gi;
  const Dim3 gq = OS == 2 ? Dim3{(gout.x + 1) / 2, (gout.y + 1) / 2, (gout.z + 1) / 2} : gout;
  const int tx = (gq.x + kBX - 1) / kBX, ty = (gq.y + BY - 1) / BY, tz = (gq.z + BZ - 1) / BZ;
  int id = blockIdx.x;
  const int bxi = id % tx;
  id /= tx;
  const int byi = id % ty;
  id /= ty;
  const int bzi = id % tz;
  id /= tz;
  const int cls = OS == 2 ? id % 8 : 0;
  const int b = OS == 2 ? id / 8 : id;
  const int rx = cls & 1, ry = (cls >> 1) & 1, rz = cls >> 2;
  const int qx0 = bxi * kBX, qy0 = byi * BY, qz0 = bzi * BZ;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  if (tid == 0) {
    int n = 0;
    for (int t = 0; t < 27; ++t) {
      const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
      if (MODE == GB_CONV) {
        taps[n++] = TapE{t, dx, dy, dz};
      } else if (OS == 1) {
        taps[n++] = TapE{t, -dx, -dy, -dz};
      } else if (((rx - dx) & 1) == 0 && ((ry - dy) & 1) == 0 && ((rz - dz) & 1) == 0) {
        taps[n++] = TapE{t, (rx - dx) / 2, (ry - dy) / 2, (rz - dz) / 2};
      }
    }
    ntap_sh = n;
  }
  // source brick origin (in source-grid positions)
  const int sx0 = S * qx0 + EMIN, sy0 = S * qy0 + EMIN, sz0 = S * qz0 + EMIN;
  const int Kch = a.K / 27;
  const int64_t Vs = gs.count();
  const __bf16 *__restrict__ Wp = reinterpret_cast<const __bf16 *>(a.wpack);
  const int Cp = a.wp_cp;

  f32x4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int col = lane & 15, kg = lane >> 4;
  const int kc = (kg % (CC / 8)) * 8;  // channel offset of this lane's 8 k within the chunk
  const int tsub = kg / (CC / 8);      // which tap of the K-slab
  // LDS position of output fragment j's column `col` for source offset 0 (relative to EMIN)
  int fpos[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int f = wave * NT + j, fy = f % BY, fz = f / BY;
    fpos[j] = (S * col - EMIN) + SX * ((S * fy - EMIN) + SY * (S * fz - EMIN));
  }

  for (int c0 = 0; c0 < Kch; c0 += CC) {
    __syncthreads();  // previous chunk's reads done (and the tap list written)
    // stage the source brick for channels c0 .. c0 + CC - 1: a thread takes a
    // position and loads its CC channels (consecutive threads on consecutive x,
    // so each channel's loads coalesce; all CC loads in flight at once), then
    // stores them as CC/8 16-byte LDS writes
    for (int pos = tid; pos < SP; pos += 256) {
      const int lx = pos % SX, ly = (pos / SX) % SY, lz = pos / (SX * SY);
      const int gx = sx0 + lx, gy = sy0 + ly, gz = sz0 + lz;
      const bool in = gx >= 0 && gx < gs.x && gy >= 0 && gy < gs.y && gz >= 0 && gz < gs.z;
      const int64_t sp = in ? gx + (int64_t)gs.x * (gy + (int64_t)gs.y * gz) : 0;
      float v[CC];
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        const int ch = min(c0 + c, Kch - 1);
        const float t = a.src[((int64_t)ch * g.B + b) * Vs + sp];
        v[c] = (in && c0 + c < Kch) ? t : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < CC / 8; ++q) {
        bf16x8 w;
#pragma unroll
        for (int e = 0; e < 8; ++e) w[e] = (__bf16)v[8 * q + e];
        *reinterpret_cast<bf16x8 *>(&sb[pos * CCP + 8 * q]) = w;
      }
    }
    __syncthreads();
    const int ntap = ntap_sh;
    // the weight fragments of the next K-slab are loaded while this one multiplies
    auto load_a = [&](int t0, bf16x8 (&af)[MT]) {
      const int ti = t0 + tsub;
      const bool live = ti < ntap;
      const int t = taps[live ? ti : ntap - 1].t;
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        const int m = 16 * i + col;
        af[i] = *reinterpret_cast<const bf16x8 *>(Wp + ((int64_t)m * 27 + t) * Cp + c0 + kc);
        if (!live) af[i] = bf16x8{};
      }
    };
    bf16x8 anext[MT];
    load_a(0, anext);
    for (int t0 = 0; t0 < ntap; t0 += TPS) {
      const int ti = t0 + tsub;
      const TapE tp = taps[ti < ntap ? ti : ntap - 1];
      bf16x8 af[MT], bfr[NT];
#pragma unroll
      for (int i = 0; i < MT; ++i) af[i] = anext[i];
      if (t0 + TPS < ntap) load_a(t0 + TPS, anext);
      const int shift = tp.ex + SX * (tp.ey + SY * tp.ez);
#pragma unroll
      for (int j = 0; j < NT; ++j) bfr[j] = *reinterpret_cast<const bf16x8 *>(&sb[(fpos[j] + shift) * CCP + kc]);
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
  }

  // epilogue: D lane layout = column lane % 16, rows 4 (lane / 16) + r
  const int64_t Vo = gout.count();
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int f = wave * NT + j, fy = f % BY, fz = f / BY;
    const int px = OS * (qx0 + col) + rx, py = OS * (qy0 + fy) + ry, pz = OS * (qz0 + fz) + rz;
    if (qx0 + col >= gq.x || px >= gout.x || py >= gout.y || pz >= gout.z) continue;
    const int64_t n = (int64_t)b * Vo + px + (int64_t)gout.x * (py + (int64_t)gout.y * pz);
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = 16 * i + 4 * kg + r;
        if (m >= a.M) continue;
        float *c = a.C + (int64_t)m * a.ldc + n;
        float v = acc[i][j][r] + (a.bias ? a.bias[m] : 0.0f);
        if (a.accumulate) v += *c;
        if (a.relu) v = fmaxf(v, 0.0f);
        *c = v;
      }
  }
}

namespace {
template <int MODE, int OS, int S, int CC, int MT, int BY, int BZ>
hipError_t conv_launch(hipStream_t s, const GemmArgs &a) {
  const ConvGeo &g = a.geo;
  const Dim3 gout = MODE == GB_CONV ? g.go : g.gi;
  const Dim3 gq = OS == 2 ? Dim3{(gout.x + 1) / 2, (gout.y + 1) / 2, (gout.z + 1) / 2} : gout;
  const int64_t blocks = (int64_t)((gq.x + kBX - 1) / kBX) * ((gq.y + BY - 1) / BY) * ((gq.z + BZ - 1) / BZ) *
                         (OS == 2 ? 8 : 1) * g.B;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  conv_mfma_kernel<MODE, OS, S, CC, MT, BY, BZ><<<(unsigned)blocks, 256, 0, s>>>(a);
  return hipGetLastError();
}

template <int MODE, int OS, int S, int CC, int BY, int BZ>
hipError_t conv_mt(hipStream_t s, const GemmArgs &a) {
  if (a.M <= 16) return conv_launch<MODE, OS, S, CC, 1, BY, BZ>(s, a);
  if (a.M <= 32) return conv_launch<MODE, OS, S, CC, 2, BY, BZ>(s, a);
  return conv_launch<MODE, OS, S, CC, 4, BY, BZ>(s, a);
}

template <int MODE, int OS, int S, int BY, int BZ>
hipError_t conv_cc(hipStream_t s, const GemmArgs &a) {
  if (a.wp_cc == 16) return conv_mt<MODE, OS, S, 16, BY, BZ>(s, a);
  return conv_mt<MODE, OS, S, 32, BY, BZ>(s, a);
}
}  // namespace

bool conv_bf16_supported(int mode, const GemmArgs &a) {
  if (!a.wpack || (mode != GB_CONV && mode != GB_CONVT)) return false;
  if (a.M < 1 || a.M > 64 || a.K % 27 != 0 || (a.wp_cc != 16 && a.wp_cc != 32)) return false;
  if (a.wp_cp < a.K / 27 || a.wp_cp % a.wp_cc != 0) return false;
  // the pack holds 16, 32 or 64 rows: as many as the kernel's row fragments read
  if (a.wp_mp != (a.M <= 16 ? 16 : (a.M <= 32 ? 32 : 64))) return false;
  return a.geo.stride == 1 || a.geo.stride == 2;
}

hipError_t launch_conv_bf16(hipStream_t s, int mode, const GemmArgs &a) {
  if (!conv_bf16_supported(mode, a)) return hipErrorInvalidValue;
  if (mode == GB_CONV) {
    if (a.geo.stride == 2) return conv_cc<GB_CONV, 1, 2, 2, 2>(s, a);
    return conv_cc<GB_CONV, 1, 1, 4, 4>(s, a);
  }
  if (a.geo.stride == 2) return conv_cc<GB_CONVT, 2, 1, 4, 4>(s, a);
  return conv_cc<GB_CONVT, 1, 1, 4, 4>(s, a);
}

}  // namespace topo
