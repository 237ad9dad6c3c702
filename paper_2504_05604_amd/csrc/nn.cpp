// Host side of the convolutional preconditioner network: parameter layout,
// activation workspaces, forward and backward passes as sequences of implicit
// GEMMs, and the training loop (Adam on batches of stored pairs).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "nn.h"

using namespace topo;

namespace topo {

void NnWork::release() {
  for (void *a : allocs) (void)hipFree(a);
  allocs.clear();
  x = e0a = cat0 = d1 = cat1 = d2 = b2 = t1 = t0 = out = nullptr;
  dout = dt0 = dcat0 = dt1 = dcat1 = dd2 = db2 = split = nullptr;
  scale = nullptr;
  idx = nullptr;
  loss = nullptr;
  split_cap = 0;
  g0 = g1 = g2 = Dim3{};
  B = 0;
  grads = false;
}

template <typename T>
static hipError_t walloc(std::vector<void *> &allocs, T **p, int64_t count) {
  hipError_t e = hipMalloc((void **)p, (size_t)std::max<int64_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) allocs.push_back((void *)*p);
  else *p = nullptr;
  return e;
}

#define NN_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      return e_ == hipErrorOutOfMemory ? TOPO_ENOMEM : TOPO_EDEVICE;                      \
    }                                                                                     \
  } while (0)

static topo_status prepare_impl(const int c[3], NnWork &w, Dim3 g0, int B, bool grads) {
  if (w.B == B && w.g0.x == g0.x && w.g0.y == g0.y && w.g0.z == g0.z && (w.grads || !grads)) return TOPO_OK;
  w.release();
  w.g0 = g0;
  w.g1 = half_up(g0);
  w.g2 = half_up(w.g1);
  w.B = B;
  w.grads = grads;
  const int64_t N0 = B * g0.count(), N1 = B * w.g1.count(), N2 = B * w.g2.count();
  const int c0 = c[0], c1 = c[1], c2 = c[2];
  auto &A = w.allocs;
  NN_HIP(walloc(A, &w.x, 4 * N0));
  NN_HIP(walloc(A, &w.e0a, c0 * N0));
  NN_HIP(walloc(A, &w.cat0, 2 * c0 * N0));
  NN_HIP(walloc(A, &w.d1, c1 * N1));
  NN_HIP(walloc(A, &w.cat1, 2 * c1 * N1));
  NN_HIP(walloc(A, &w.d2, c2 * N2));
  NN_HIP(walloc(A, &w.b2, c2 * N2));
  NN_HIP(walloc(A, &w.t1, c1 * N1));
  NN_HIP(walloc(A, &w.t0, c0 * N0));
  NN_HIP(walloc(A, &w.out, 3 * N0));
  NN_HIP(walloc(A, &w.scale, B));
  NN_HIP(walloc(A, &w.idx, B));
  NN_HIP(walloc(A, &w.loss, B));
  if (grads) {
    NN_HIP(walloc(A, &w.dout, 3 * N0));
    NN_HIP(walloc(A, &w.dt0, c0 * N0));
    NN_HIP(walloc(A, &w.dcat0, 2 * c0 * N0));
    NN_HIP(walloc(A, &w.dt1, c1 * N1));
    NN_HIP(walloc(A, &w.dcat1, 2 * c1 * N1));
    NN_HIP(walloc(A, &w.db2, c2 * N2));
    NN_HIP(walloc(A, &w.dd2, c2 * N2));
    // split-K partials of the largest weight gradient, up to 64 slices
    const int64_t wmax = std::max<int64_t>({(int64_t)c2 * c2 * 27, (int64_t)c1 * 2 * c1 * 27,
                                            (int64_t)c0 * 2 * c0 * 27, (int64_t)c2 * c1 * 27});
    w.split_cap = 64 * wmax;
    NN_HIP(walloc(A, &w.split, w.split_cap));
  }
  return TOPO_OK;
}

static hipError_t run_gemm(const topo_nn *nn, hipStream_t s, int mode, const GemmArgs &a, float *split,
                           int64_t cap) {
  if (nn->precision != TOPO_PREC_BF16) return launch_igemm(s, mode, a, split, cap);
  if (conv_bf16_supported(mode, a)) return launch_conv_bf16(s, mode, a);
  return launch_igemm_bf16(s, mode, a, split, cap);
}

// attaches the BF16 weight pack of layer L in orientation o (0: A = W, 1: A = WT)
static GemmArgs with_pack(const topo_nn *nn, int L, int o, GemmArgs a) {
  if (nn->pack && nn->pk_mp[L][o] > 0) {
    a.wpack = nn->pack + nn->pk_off[L][o];
    a.wp_mp = nn->pk_mp[L][o];
    a.wp_cp = nn->pk_cp[L][o];
    a.wp_cc = nn->pk_cc[L][o];
  }
  return a;
}

static GemmArgs gemm(int M, int N, int K, const float *A, int64_t sam, int64_t sak, const float *src,
                     ConvGeo geo, float *C, const float *bias, bool relu, bool acc, const int *skip) {
  GemmArgs a{};
  a.M = M;
  a.N = N;
  a.K = K;
  a.A = A;
  a.sam = sam;
  a.sak = sak;
  a.src = src;
  a.geo = geo;
  a.C = C;
  a.ldc = N;
  a.bias = bias;
  a.relu = relu ? 1 : 0;
  a.accumulate = acc ? 1 : 0;
  a.skip = skip;
  return a;
}

// y = act(conv_s(x; layer) + b): x on gi (ci channels), y on ceil(gi / s)
static hipError_t conv_fwd(const topo_nn *nn, int L, hipStream_t s, int B, Dim3 gi, int stride, const float *x,
                           float *y, bool relu, const int *skip) {
  const NnLayer &l = nn->layer[L];
  const Dim3 go = stride == 2 ? half_up(gi) : gi;
  const int K = l.ci * 27;
  const GemmArgs a = gemm(l.co, (int)(B * go.count()), K, nn->W + l.w_off, K, 1, x, ConvGeo{B, gi, go, stride},
                          y, nn->W + l.b_off, relu, false, skip);
  return run_gemm(nn, s, GB_CONV, with_pack(nn, L, 0, a), nullptr, 0);
}

// y = conv_2^T(x; layer) + b: x on the coarse grid (co channels), y on gf (ci channels)
static hipError_t up_fwd(const topo_nn *nn, int L, hipStream_t s, int B, Dim3 gf, const float *x, float *y,
                         const int *skip) {
  const NnLayer &l = nn->layer[L];
  const int K = l.co * 27;
  const GemmArgs a = gemm(l.ci, (int)(B * gf.count()), K, nn->WT + l.w_off, K, 1, x,
                          ConvGeo{B, gf, half_up(gf), 2}, y, nn->W + l.b_off, false, false, skip);
  return run_gemm(nn, s, GB_CONVT, with_pack(nn, L, 1, a), nullptr, 0);
}

}  // namespace topo

topo_nn::~topo_nn() {
  work.release();
  for (void *a : allocs) (void)hipFree(a);
}

namespace topo {

topo_status nn_prepare(const topo_nn *nn, NnWork &w, Dim3 g0, int B, bool grads) {
  return prepare_impl(nn->c, w, g0, B, grads);
}

topo_status nn_refresh(topo_nn *nn, hipStream_t s) {
  for (int L = 0; L < L_COUNT; ++L) {
    const NnLayer &l = nn->layer[L];
    NN_HIP(launch_transpose_w(s, l.co, l.ci, l.taps, nn->W + l.w_off, nn->WT + l.w_off));
    for (int o = 0; o < 2; ++o) {
      if (!nn->pack || nn->pk_mp[L][o] == 0) continue;
      const int M = o ? l.ci : l.co, Kch = o ? l.co : l.ci;
      const float *A = o ? nn->WT + l.w_off : nn->W + l.w_off;
      NN_HIP(launch_pack_bf16(s, A, (int64_t)Kch * 27, 1, M, Kch, nn->pk_mp[L][o], nn->pk_cp[L][o],
                              nn->pack + nn->pk_off[L][o]));
    }
  }
  return TOPO_OK;
}

topo_status nn_forward(topo_nn *nn, NnWork &w, hipStream_t s, const int *skip) {
  const int B = w.B;
  const int64_t N0 = B * w.g0.count(), N1 = B * w.g1.count();
  const int c0 = nn->c[0], c1 = nn->c[1];
  float *s0 = w.cat0 + c0 * N0, *s1 = w.cat1 + c1 * N1;
  NN_HIP(conv_fwd(nn, L_ENC0A, s, B, w.g0, 1, w.x, w.e0a, true, skip));
  NN_HIP(conv_fwd(nn, L_ENC0B, s, B, w.g0, 1, w.e0a, s0, true, skip));
  NN_HIP(conv_fwd(nn, L_DOWN1, s, B, w.g0, 2, s0, w.d1, true, skip));
  NN_HIP(conv_fwd(nn, L_ENC1B, s, B, w.g1, 1, w.d1, s1, true, skip));
  NN_HIP(conv_fwd(nn, L_DOWN2, s, B, w.g1, 2, s1, w.d2, true, skip));
  NN_HIP(conv_fwd(nn, L_ENC2B, s, B, w.g2, 1, w.d2, w.b2, true, skip));
  NN_HIP(up_fwd(nn, L_UP1, s, B, w.g1, w.b2, w.cat1, skip));
  NN_HIP(conv_fwd(nn, L_DEC1, s, B, w.g1, 1, w.cat1, w.t1, true, skip));
  NN_HIP(up_fwd(nn, L_UP0, s, B, w.g0, w.t1, w.cat0, skip));
  NN_HIP(conv_fwd(nn, L_DEC0, s, B, w.g0, 1, w.cat0, w.t0, true, skip));
  const NnLayer &h = nn->layer[L_HEAD];
  const GemmArgs a = gemm(3, (int)N0, c0, nn->W + h.w_off, c0, 1, w.t0, ConvGeo{B, w.g0, w.g0, 1}, w.out,
                          nn->W + h.b_off, false, false, skip);
  NN_HIP(run_gemm(nn, s, GB_PLAIN, a, nullptr, 0));
  return TOPO_OK;
}

// Gradients of a convolution y = act(conv_s(x)) given dL/dy (already masked by
// the activation): weight and bias gradients into G, dL/dx into dx (added when acc).
static topo_status conv_back(topo_nn *nn, NnWork &w, int L, hipStream_t s, Dim3 gi, int stride, const float *x,
                             float *dy, float *dx, bool acc) {
  const NnLayer &l = nn->layer[L];
  const int B = w.B;
  const Dim3 go = stride == 2 ? half_up(gi) : gi;
  const int Ko = (int)(B * go.count()), Ni = (int)(B * gi.count());
  const ConvGeo geo{B, gi, go, stride};
  NN_HIP(run_gemm(nn, s, GB_WGRAD, gemm(l.co, l.ci * 27, Ko, dy, Ko, 1, x, geo, nn->G + l.w_off, nullptr, false,
                                        false, nullptr),
                      w.split, w.split_cap));
  NN_HIP(launch_bias_grad(s, l.co, Ko, dy, nn->G + l.b_off, nn->red));
  if (dx)
    NN_HIP(run_gemm(nn, s, GB_CONVT,
                    with_pack(nn, L, 1, gemm(l.ci, Ni, l.co * 27, nn->WT + l.w_off, l.co * 27, 1, dy, geo, dx,
                                             nullptr, false, acc, nullptr)),
                    nullptr, 0));
  return TOPO_OK;
}

// Gradients of an up layer y = conv_2^T(xc) + b on gf given dL/dy
static topo_status up_back(topo_nn *nn, NnWork &w, int L, hipStream_t s, Dim3 gf, const float *xc,
                           const float *dy, float *dxc) {
  const NnLayer &l = nn->layer[L];
  const int B = w.B;
  const Dim3 gc = half_up(gf);
  const int Kc = (int)(B * gc.count()), Nf = (int)(B * gf.count());
  const ConvGeo geo{B, gf, gc, 2};
  NN_HIP(run_gemm(nn, s, GB_WGRAD, gemm(l.co, l.ci * 27, Kc, xc, Kc, 1, dy, geo, nn->G + l.w_off, nullptr, false,
                                        false, nullptr),
                      w.split, w.split_cap));
  NN_HIP(launch_bias_grad(s, l.ci, Nf, dy, nn->G + l.b_off, nn->red));
  NN_HIP(run_gemm(nn, s, GB_CONV,
                  with_pack(nn, L, 0, gemm(l.co, Kc, l.ci * 27, nn->W + l.w_off, l.ci * 27, 1, dy, geo, dxc,
                                           nullptr, false, false, nullptr)),
                  nullptr, 0));
  return TOPO_OK;
}

topo_status nn_backward(topo_nn *nn, NnWork &w, hipStream_t s) {
  const int B = w.B;
  const int64_t N0 = B * w.g0.count(), N1 = B * w.g1.count(), N2 = B * w.g2.count();
  const int c0 = nn->c[0], c1 = nn->c[1], c2 = nn->c[2];
  float *s0 = w.cat0 + c0 * N0, *s1 = w.cat1 + c1 * N1;
  float *ds0 = w.dcat0 + c0 * N0, *ds1 = w.dcat1 + c1 * N1;
  topo_status st;
  // head: out = W t0 + b
  {
    const NnLayer &h = nn->layer[L_HEAD];
    const ConvGeo geo{B, w.g0, w.g0, 1};
    NN_HIP(run_gemm(nn, s, GB_PLAINT, gemm(3, c0, (int)N0, w.dout, N0, 1, w.t0, geo, nn->G + h.w_off, nullptr,
                                           false, false, nullptr),
                        w.split, w.split_cap));
    NN_HIP(launch_bias_grad(s, 3, N0, w.dout, nn->G + h.b_off, nn->red));
    NN_HIP(run_gemm(nn, s, GB_PLAIN, gemm(c0, (int)N0, 3, nn->W + h.w_off, 1, c0, w.dout, geo, w.dt0, nullptr,
                                          false, false, nullptr),
                        nullptr, 0));
  }
  NN_HIP(launch_relu_back(s, c0 * N0, w.t0, w.dt0));
  if ((st = conv_back(nn, w, L_DEC0, s, w.g0, 1, w.cat0, w.dt0, w.dcat0, false)) != TOPO_OK) return st;
  if ((st = up_back(nn, w, L_UP0, s, w.g0, w.t1, w.dcat0, w.dt1)) != TOPO_OK) return st;
  NN_HIP(launch_relu_back(s, c1 * N1, w.t1, w.dt1));
  if ((st = conv_back(nn, w, L_DEC1, s, w.g1, 1, w.cat1, w.dt1, w.dcat1, false)) != TOPO_OK) return st;
  if ((st = up_back(nn, w, L_UP1, s, w.g1, w.b2, w.dcat1, w.db2)) != TOPO_OK) return st;
  NN_HIP(launch_relu_back(s, c2 * N2, w.b2, w.db2));
  if ((st = conv_back(nn, w, L_ENC2B, s, w.g2, 1, w.d2, w.db2, w.dd2, false)) != TOPO_OK) return st;
  NN_HIP(launch_relu_back(s, c2 * N2, w.d2, w.dd2));
  if ((st = conv_back(nn, w, L_DOWN2, s, w.g1, 2, s1, w.dd2, ds1, true)) != TOPO_OK) return st;
  NN_HIP(launch_relu_back(s, c1 * N1, s1, ds1));
  if ((st = conv_back(nn, w, L_ENC1B, s, w.g1, 1, w.d1, ds1, w.dt1, false)) != TOPO_OK) return st;  // dt1 := dd1
  NN_HIP(launch_relu_back(s, c1 * N1, w.d1, w.dt1));
  if ((st = conv_back(nn, w, L_DOWN1, s, w.g0, 2, s0, w.dt1, ds0, true)) != TOPO_OK) return st;
  NN_HIP(launch_relu_back(s, c0 * N0, s0, ds0));
  if ((st = conv_back(nn, w, L_ENC0B, s, w.g0, 1, w.e0a, ds0, w.dt0, false)) != TOPO_OK) return st;  // dt0 := de0a
  NN_HIP(launch_relu_back(s, c0 * N0, w.e0a, w.dt0));
  return conv_back(nn, w, L_ENC0A, s, w.g0, 1, w.x, w.dt0, nullptr, false);
}

}  // namespace topo

// ---------------------------------------------------------------------------
// C ABI
// column indices of the implicit GEMMs are 32-bit: batch * V must stay below 2^30
static bool valid_nodes(const int32_t nodes[3], int64_t batch = 1) {
  return nodes && nodes[0] >= 2 && nodes[1] >= 2 && nodes[2] >= 2 &&
         (int64_t)nodes[0] * nodes[1] * nodes[2] * batch <= ((int64_t)1 << 30);
}

extern "C" topo_status topo_nn_create(const int32_t channels[3], void *hip_stream, topo_nn **out) {
  if (!out) return set_error("NULL out"), TOPO_EINVAL;
  *out = nullptr;
  int c[3] = {16, 32, 64};
  if (channels)
    for (int i = 0; i < 3; ++i) {
      if (channels[i] < 1 || channels[i] > 1024) return set_error("channel count %d out of range", channels[i]), TOPO_EINVAL;
      c[i] = channels[i];
    }
  topo_nn *nn = new (std::nothrow) topo_nn();
  if (!nn) return set_error("host allocation failed"), TOPO_ENOMEM;
  std::memcpy(nn->c, c, sizeof(c));
  nn->stream = (hipStream_t)hip_stream;
  const int c0 = c[0], c1 = c[1], c2 = c[2];
  // (co, ci, taps, up) in storage order; up layers store the forward convolution
  // coarse <- fine, and their bias has the fine channel count
  const int shapes[L_COUNT][4] = {{c0, 4, 27, 0},  {c0, c0, 27, 0},     {c1, c0, 27, 0}, {c1, c1, 27, 0},
                                  {c2, c1, 27, 0}, {c2, c2, 27, 0},     {c2, c1, 27, 1}, {c1, 2 * c1, 27, 0},
                                  {c1, c0, 27, 1}, {c0, 2 * c0, 27, 0}, {3, c0, 1, 0}};
  int64_t off = 0;
  for (int L = 0; L < L_COUNT; ++L) {
    NnLayer &l = nn->layer[L];
    l.co = shapes[L][0];
    l.ci = shapes[L][1];
    l.taps = shapes[L][2];
    l.up = shapes[L][3] != 0;
    l.w_off = off;
    off += (int64_t)l.co * l.ci * l.taps;
    l.b_off = off;
    l.nb = l.up ? l.ci : l.co;
    off += l.nb;
  }
  nn->nparams = off;
  hipError_t e = hipSuccess;
  float **bufs[] = {&nn->W, &nn->WT, &nn->G, &nn->m, &nn->v};
  for (float **b : bufs) {
    if ((e = walloc(nn->allocs, b, off)) != hipSuccess) break;
    if ((e = hipMemsetAsync(*b, 0, off * sizeof(float), nn->stream)) != hipSuccess) break;
  }
  // BF16 weight packs (layers with at most 64 rows in an orientation)
  if (e == hipSuccess) {
    int64_t poff = 0;
    for (int L = 0; L < L_COUNT; ++L) {
      const NnLayer &l = nn->layer[L];
      if (l.taps != 27) continue;
      for (int o = 0; o < 2; ++o) {
        const int M = o ? l.ci : l.co, Kch = o ? l.co : l.ci;
        if (M > 64) continue;
        const int cc = Kch <= 16 ? 16 : 32;
        nn->pk_mp[L][o] = M <= 16 ? 16 : (M <= 32 ? 32 : 64);
        nn->pk_cc[L][o] = cc;
        nn->pk_cp[L][o] = (Kch + cc - 1) / cc * cc;
        nn->pk_off[L][o] = poff;
        poff += (int64_t)nn->pk_mp[L][o] * 27 * nn->pk_cp[L][o];
      }
    }
    e = walloc(nn->allocs, &nn->pack, poff);
    if (e == hipSuccess) e = hipMemsetAsync(nn->pack, 0, (size_t)std::max<int64_t>(poff, 1) * 2, nn->stream);
  }
  if (e == hipSuccess) {
    nn->red.max_blocks = 64 * 64;
    e = walloc(nn->allocs, &nn->red.partials, (int64_t)nn->red.max_blocks * kMaxRed);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(nn->stream);
  if (e != hipSuccess) {
    set_error("network allocation failed: %s", hipGetErrorString(e));
    delete nn;
    return e == hipErrorOutOfMemory ? TOPO_ENOMEM : TOPO_EDEVICE;
  }
  *out = nn;
  return TOPO_OK;
}

extern "C" void topo_nn_destroy(topo_nn *nn) { delete nn; }

extern "C" topo_status topo_nn_set_precision(topo_nn *nn, int32_t precision) {
  if (!nn) return set_error("NULL argument"), TOPO_EINVAL;
  if (precision != TOPO_PREC_FP32 && precision != TOPO_PREC_BF16)
    return set_error("network precision must be TOPO_PREC_FP32 or TOPO_PREC_BF16"), TOPO_EINVAL;
  nn->precision = precision;
  return TOPO_OK;
}

extern "C" topo_status topo_nn_n_params(const topo_nn *nn, int64_t *n) {
  if (!nn || !n) return set_error("NULL argument"), TOPO_EINVAL;
  *n = nn->nparams;
  return TOPO_OK;
}

extern "C" topo_status topo_nn_set_weights(topo_nn *nn, const float *h_blob, int64_t n) {
  if (!nn || !h_blob) return set_error("NULL argument"), TOPO_EINVAL;
  if (n != nn->nparams) return set_error("weight count %lld != %lld", (long long)n, (long long)nn->nparams), TOPO_EINVAL;
  hipStream_t s = nn->stream;
  TOPO_HIP(hipMemcpyAsync(nn->W, h_blob, n * sizeof(float), hipMemcpyHostToDevice, s));
  TOPO_HIP(hipMemsetAsync(nn->m, 0, n * sizeof(float), s));
  TOPO_HIP(hipMemsetAsync(nn->v, 0, n * sizeof(float), s));
  nn->adam_step = 0;
  topo_status st = nn_refresh(nn, s);
  if (st != TOPO_OK) return st;
  TOPO_HIP(hipStreamSynchronize(s));
  return TOPO_OK;
}

extern "C" topo_status topo_nn_get_weights(const topo_nn *nn, float *h_blob, int64_t n) {
  if (!nn || !h_blob) return set_error("NULL argument"), TOPO_EINVAL;
  if (n != nn->nparams) return set_error("weight count %lld != %lld", (long long)n, (long long)nn->nparams), TOPO_EINVAL;
  TOPO_HIP(hipMemcpyAsync(h_blob, nn->W, n * sizeof(float), hipMemcpyDeviceToHost, nn->stream));
  TOPO_HIP(hipStreamSynchronize(nn->stream));
  return TOPO_OK;
}

extern "C" topo_status topo_nn_forward(topo_nn *nn, const int32_t nodes[3], int32_t batch, const float *d_in,
                                       float *d_out) {
  if (!nn || !d_in || !d_out) return set_error("NULL argument"), TOPO_EINVAL;
  if (batch < 1 || batch > 64 || !valid_nodes(nodes, batch)) return set_error("invalid grid or batch"), TOPO_EINVAL;
  const Dim3 g0{nodes[0], nodes[1], nodes[2]};
  topo_status st = nn_prepare(nn, nn->work, g0, batch, false);
  if (st != TOPO_OK) return st;
  hipStream_t s = nn->stream;
  const int64_t N0 = batch * g0.count();
  TOPO_HIP(hipMemcpyAsync(nn->work.x, d_in, 4 * N0 * sizeof(float), hipMemcpyDeviceToDevice, s));
  st = nn_forward(nn, nn->work, s, nullptr);
  if (st != TOPO_OK) return st;
  TOPO_HIP(hipMemcpyAsync(d_out, nn->work.out, 3 * N0 * sizeof(float), hipMemcpyDeviceToDevice, s));
  return TOPO_OK;
}

static bool valid_data(const float *rho, const float *r, const float *e, const uint8_t *fixed) {
  return rho && r && e && fixed;
}

// input, forward, loss and gradient of one batch (indices already on the device)
static topo_status batch_step(topo_nn *nn, int mode, int64_t V, const float *d_rho, const float *d_r,
                              const float *d_e, const uint8_t *d_fixed, double *d_loss) {
  NnWork &w = nn->work;
  hipStream_t s = nn->stream;
  TOPO_HIP(launch_nn_input_train(s, V, w.B, w.idx, d_rho, d_r, w.scale, w.x));
  topo_status st = nn_forward(nn, w, s, nullptr);
  if (st != TOPO_OK) return st;
  TOPO_HIP(launch_nn_loss(s, mode, V, w.B, w.idx, w.out, d_e, d_fixed, w.scale, w.dout, nn->red, d_loss));
  return nn_backward(nn, w, s);
}

extern "C" topo_status topo_nn_loss_grad(topo_nn *nn, const int32_t nodes[3], int64_t n_samples,
                                         const float *d_rho, const float *d_r, const float *d_e,
                                         const uint8_t *d_fixed, int32_t batch, const int32_t *h_index,
                                         int32_t loss_mode, double *h_loss, float *d_grad) {
  if (!nn || !valid_data(d_rho, d_r, d_e, d_fixed) || !h_index) return set_error("NULL argument"), TOPO_EINVAL;
  if (batch < 1 || batch > 64 || !valid_nodes(nodes, batch)) return set_error("invalid grid or batch"), TOPO_EINVAL;
  if (loss_mode != TOPO_LOSS_REL && loss_mode != TOPO_LOSS_COS) return set_error("unknown loss %d", loss_mode), TOPO_EINVAL;
  for (int b = 0; b < batch; ++b)
    if (h_index[b] < 0 || h_index[b] >= n_samples) return set_error("sample index out of range"), TOPO_EINVAL;
  const Dim3 g0{nodes[0], nodes[1], nodes[2]};
  topo_status st = nn_prepare(nn, nn->work, g0, batch, true);
  if (st != TOPO_OK) return st;
  hipStream_t s = nn->stream;
  TOPO_HIP(hipMemcpyAsync(nn->work.idx, h_index, batch * sizeof(int32_t), hipMemcpyHostToDevice, s));
  st = batch_step(nn, loss_mode, g0.count(), d_rho, d_r, d_e, d_fixed, nn->work.loss);
  if (st != TOPO_OK) return st;
  if (d_grad) TOPO_HIP(hipMemcpyAsync(d_grad, nn->G, nn->nparams * sizeof(float), hipMemcpyDeviceToDevice, s));
  std::vector<double> l(batch);
  TOPO_HIP(hipMemcpyAsync(l.data(), nn->work.loss, batch * sizeof(double), hipMemcpyDeviceToHost, s));
  TOPO_HIP(hipStreamSynchronize(s));
  if (h_loss) {
    double t = 0.0;
    for (double v : l) t += v;
    *h_loss = t / batch;
  }
  return TOPO_OK;
}

// splitmix64 (Steele, Lea, Flood 2014) drives the per-epoch shuffles
static uint64_t splitmix64(uint64_t &x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

extern "C" void topo_default_train_opts(topo_train_opts *o) {
  if (!o) return;
  o->epochs = 10;
  o->batch = 4;
  o->lr = 1e-3;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->eps = 1e-8;
  o->seed = 0;
  o->loss = TOPO_LOSS_REL;
}

extern "C" topo_status topo_nn_train(topo_nn *nn, const int32_t nodes[3], int64_t n_samples, const float *d_rho,
                                     const float *d_r, const float *d_e, const uint8_t *d_fixed,
                                     const topo_train_opts *opts, double *h_epoch_loss, topo_train_stats *h_stats) {
  if (!nn || !valid_data(d_rho, d_r, d_e, d_fixed) || !opts) return set_error("NULL argument"), TOPO_EINVAL;
  if (!valid_nodes(nodes) || n_samples < 1 || n_samples > (1ll << 30)) return set_error("invalid grid or sample count"), TOPO_EINVAL;
  if (opts->epochs < 0 || opts->batch < 1 || opts->batch > 64 || !(opts->lr > 0.0) || !(opts->beta1 >= 0.0) ||
      !(opts->beta1 < 1.0) || !(opts->beta2 >= 0.0) || !(opts->beta2 < 1.0) || !(opts->eps > 0.0) ||
      (opts->loss != TOPO_LOSS_REL && opts->loss != TOPO_LOSS_COS))
    return set_error("invalid training options"), TOPO_EINVAL;
  const int B = (int)std::min<int64_t>(opts->batch, n_samples);
  if (!valid_nodes(nodes, B)) return set_error("grid too large for the batch"), TOPO_EINVAL;
  const int64_t steps_per_epoch = n_samples / B;
  const Dim3 g0{nodes[0], nodes[1], nodes[2]};
  topo_status st = nn_prepare(nn, nn->work, g0, B, true);
  if (st != TOPO_OK) return st;
  hipStream_t s = nn->stream;
  std::vector<void *> tmp;
  struct Free {
    std::vector<void *> &v;
    ~Free() {
      for (void *p : v) (void)hipFree(p);
    }
  } guard{tmp};
  int *d_perm = nullptr;
  double *d_loss = nullptr;
  const int64_t total = (int64_t)opts->epochs * steps_per_epoch;
  TOPO_HIP(walloc(tmp, &d_perm, (int64_t)opts->epochs * n_samples));
  TOPO_HIP(walloc(tmp, &d_loss, std::max<int64_t>(1, total * B)));
  // every epoch's permutation, uploaded once
  std::vector<int32_t> perm((size_t)opts->epochs * n_samples);
  uint64_t state = opts->seed;
  for (int ep = 0; ep < opts->epochs; ++ep) {
    int32_t *p = perm.data() + (size_t)ep * n_samples;
    for (int64_t i = 0; i < n_samples; ++i) p[i] = (int32_t)i;
    for (int64_t i = n_samples - 1; i > 0; --i) {
      const int64_t j = (int64_t)(splitmix64(state) % (uint64_t)(i + 1));
      std::swap(p[i], p[j]);
    }
  }
  if (!perm.empty())
    TOPO_HIP(hipMemcpyAsync(d_perm, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  hipEvent_t e0, e1;
  TOPO_HIP(hipEventCreate(&e0));
  TOPO_HIP(hipEventCreate(&e1));
  TOPO_HIP(hipEventRecord(e0, s));
  NnWork &w = nn->work;
  int *own_idx = w.idx;
  for (int ep = 0; ep < opts->epochs && st == TOPO_OK; ++ep) {
    for (int64_t k = 0; k < steps_per_epoch && st == TOPO_OK; ++k) {
      const int64_t step = (int64_t)ep * steps_per_epoch + k;
      w.idx = d_perm + (size_t)ep * n_samples + k * B;
      st = batch_step(nn, opts->loss, g0.count(), d_rho, d_r, d_e, d_fixed, d_loss + step * B);
      if (st != TOPO_OK) break;
      ++nn->adam_step;
      hipError_t he = launch_adam(s, nn->nparams, nn->W, nn->G, nn->m, nn->v, (float)opts->lr, (float)opts->beta1,
                                  (float)opts->beta2, (float)opts->eps, nn->adam_step);
      if (he != hipSuccess) {
        set_error("adam: %s", hipGetErrorString(he));
        st = TOPO_EDEVICE;
      }
      if (st == TOPO_OK) st = nn_refresh(nn, s);
    }
  }
  w.idx = own_idx;
  (void)hipEventRecord(e1, s);
  std::vector<double> losses((size_t)std::max<int64_t>(1, total * B));
  if (st == TOPO_OK && total > 0)
    TOPO_HIP(hipMemcpyAsync(losses.data(), d_loss, total * B * sizeof(double), hipMemcpyDeviceToHost, s));
  TOPO_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != TOPO_OK) return st;
  std::vector<double> ep_loss(opts->epochs, 0.0);
  for (int ep = 0; ep < opts->epochs; ++ep) {
    double t = 0.0;
    for (int64_t i = 0; i < steps_per_epoch * B; ++i) t += losses[(size_t)(ep * steps_per_epoch * B + i)];
    ep_loss[ep] = steps_per_epoch > 0 ? t / (steps_per_epoch * B) : 0.0;
    if (h_epoch_loss) h_epoch_loss[ep] = ep_loss[ep];
  }
  if (h_stats) {
    h_stats->steps = (int32_t)total;
    h_stats->loss_first = opts->epochs ? ep_loss.front() : 0.0;
    h_stats->loss_last = opts->epochs ? ep_loss.back() : 0.0;
    h_stats->ms = ms;
  }
  return TOPO_OK;
}
