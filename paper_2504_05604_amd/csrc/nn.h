// Internal declarations of the convolutional preconditioner network (not part
// of the ABI): node-grid geometry, the implicit-GEMM convolution kernels, the
// network's parameter layout and activation workspaces.
#pragma once

#include <vector>

#include "internal.h"

namespace topo {

// node grid of one network level (x fastest)
struct Dim3 {
  int x, y, z;
  __host__ __device__ int64_t count() const { return (int64_t)x * y * z; }
};
inline Dim3 half_up(Dim3 d) { return Dim3{(d.x + 1) / 2, (d.y + 1) / 2, (d.z + 1) / 2}; }

// ---------------------------------------------------------------------------
// Implicit GEMM:  C[m][n] = act(sum_k A(m,k) B(k,n) + bias[m]) (+ C if accumulate)
// A(m,k) = A[m*sam + k*sak] (weights, their transposes or a gradient);
// B(k,n) is gathered on the fly from an activation tensor laid out [C][batch][V]:
enum GemmB {
  GB_PLAIN = 0,  // B(k,n) = src[k*N + n]                     (1x1x1 convolution)
  GB_PLAINT = 1, // B(k,n) = src[n*K + k]                     (1x1x1 weight gradient)
  GB_CONV = 2,   // k = (ci,t), n = (b,o) on go: src[ci][b][o*s + t - 1] on gi (0 outside)
  GB_CONVT = 3,  // k = (co,t), n = (b,p) on gi: src[co][b][(p - t + 1)/s] on go when exact
  GB_WGRAD = 4   // k = (b,o) on go, n = (ci,t): src[ci][b][o*s + t - 1] on gi
};
// Convolution geometry: 3x3x3 taps t = 9 (dz+1) + 3 (dy+1) + (dx+1), padding 1,
// stride s; gi is the fine (input) grid, go = ceil(gi / s) the output grid.
struct ConvGeo {
  int B;
  Dim3 gi, go;
  int stride;
};
struct GemmArgs {
  int M, N, K;
  const float *A;
  int64_t sam, sak;
  const float *src;
  ConvGeo geo;
  float *C;
  int64_t ldc;
  const float *bias;  // may be NULL
  int relu;
  int accumulate;
  const int *skip;    // device flag: return at once when non-zero (may be NULL)
  // BF16 direct-convolution path (GB_CONV / GB_CONVT): A packed as
  // [wp_mp rows][27 taps][wp_cp channels] BF16, channels in chunks of wp_cc
  const void *wpack;
  int wp_mp, wp_cp, wp_cc;
};
// split_buf (split_cap floats) enables a split reduction over long K (weight
// gradients); NULL runs unsplit.
hipError_t launch_igemm(hipStream_t s, int mode, const GemmArgs &a, float *split_buf, int64_t split_cap);
// the same product with operands rounded to BF16 on the matrix cores (FP32 accumulation)
hipError_t launch_igemm_bf16(hipStream_t s, int mode, const GemmArgs &a, float *split_buf, int64_t split_cap);

// Wp[m][t][c] = A(m, c*27 + t) as BF16 (zero for m >= M, c >= Kch), Mp x 27 x Cp
hipError_t launch_pack_bf16(hipStream_t s, const float *A, int64_t sam, int64_t sak, int M, int Kch, int Mp, int Cp,
                            void *Wp);
// direct 3x3x3 convolution on the matrix cores (kernels_nn_conv.hip) for the
// GB_CONV / GB_CONVT modes when a.wpack is set and the shape is supported
bool conv_bf16_supported(int mode, const GemmArgs &a);
hipError_t launch_conv_bf16(hipStream_t s, int mode, const GemmArgs &a);

// WT[ci][co*taps + t] = W[co][ci*taps + t]
hipError_t launch_transpose_w(hipStream_t s, int co, int ci, int taps, const float *W, float *WT);
// dY *= (Y > 0)
hipError_t launch_relu_back(hipStream_t s, int64_t n, const float *Y, float *dY);
// db[c] = sum_n dY[c][n]  (db may be NULL: nothing)
hipError_t launch_bias_grad(hipStream_t s, int C, int64_t N, const float *dY, float *db, const Reducer &red);
hipError_t launch_adam(hipStream_t s, int64_t n, float *w, const float *g, float *m, float *v, float lr,
                       float b1, float b2, float eps, int step);

// network inputs: X[0][b] = node density, X[1+c][b] = r_c / scale_b.
// Solver side: rho = mean of the element densities around each node (once per
// operator), then per application scale = sqrt(rr / ndof) (rr = r.r, already
// formed by the CG loop) and the scaled residual into channels 1..3.
hipError_t launch_node_density(hipStream_t s, const Grid &g, const double *xphys, float *rho);
hipError_t launch_nn_input_resid(hipStream_t s, int64_t V, const double *r, const double *rr, double *scale,
                                 float *X1, const int *skip);
// training pairs: dr = (float) r, de = (float)(ustar - u)
hipError_t launch_pair_out(hipStream_t s, int64_t n, const double *r, const double *ustar, const double *u,
                           float *dr, float *de);
// From training samples (float): rho [P][V], r [P][V*3]; idx[b] selects the sample.
hipError_t launch_nn_input_train(hipStream_t s, int64_t V, int B, const int *idx, const float *rho,
                                 const float *r, float *scale, float *X);
// z_new = scale * out (zero on fixed dofs), written over z; reduces
// (r.z_new, r.z_old, z_new.z_new) for the flexible CG update and the safeguard.
hipError_t launch_nn_output_flex(hipStream_t s, int64_t V, const float *out, const double *scale,
                                 const uint8_t *fixed, const double *r, double *z, const Reducer &red,
                                 const Fin &fin, const int *skip);
// plain output (no reductions): z = scale * out, zero on fixed dofs
hipError_t launch_nn_output(hipStream_t s, int64_t V, const float *out, const double *scale,
                            const uint8_t *fixed, double *z);
// per-sample loss over the free dofs m of y = out against t = e/scale:
// mode 0 ||(y - t) m||^2 / ||t m||^2, mode 1 1 - (y m).(t m) / (|y m| |t m|);
// dout = d(mean loss)/d out; loss[b] receives each sample's value.  Mode 1
// zeroes out on fixed dofs.
hipError_t launch_nn_loss(hipStream_t s, int mode, int64_t V, int B, const int *idx, float *out,
                          const float *e, const uint8_t *fixed, const float *scale, float *dout,
                          const Reducer &red, double *loss);

// ---------------------------------------------------------------------------
// Parameter layout: per layer the weight [co][ci][k^3] then the bias, in the
// order below; "up" layers are transposes of stride-2 convolutions, so their
// weight is stored as the forward convolution's [c_coarse][c_fine][27] and their
// bias has c_fine entries.
enum NnLayerId { L_ENC0A, L_ENC0B, L_DOWN1, L_ENC1B, L_DOWN2, L_ENC2B, L_UP1, L_DEC1, L_UP0, L_DEC0, L_HEAD, L_COUNT };
struct NnLayer {
  int co, ci, taps;   // forward-convolution shape of the stored weight
  bool up;
  int64_t w_off, b_off, nb;
};

struct NnWork {  // activations of one grid and batch
  Dim3 g0{}, g1{}, g2{};
  int B = 0;
  float *x = nullptr, *e0a = nullptr, *cat0 = nullptr, *d1 = nullptr, *cat1 = nullptr, *d2 = nullptr,
        *b2 = nullptr, *t1 = nullptr, *t0 = nullptr, *out = nullptr;
  // gradients (allocated on request)
  float *dout = nullptr, *dt0 = nullptr, *dcat0 = nullptr, *dt1 = nullptr, *dcat1 = nullptr, *dd2 = nullptr,
        *db2 = nullptr, *split = nullptr;
  int64_t split_cap = 0;
  float *scale = nullptr;  // [B]
  int *idx = nullptr;      // [B]
  double *loss = nullptr;  // [B]
  std::vector<void *> allocs;
  bool grads = false;
  void release();
  ~NnWork() { release(); }
};

}  // namespace topo

struct topo_nn {
  int c[3] = {16, 32, 64};
  hipStream_t stream = nullptr;
  topo::NnLayer layer[topo::L_COUNT];
  int64_t nparams = 0;
  float *W = nullptr, *WT = nullptr, *G = nullptr, *m = nullptr, *v = nullptr;
  // BF16 packs of the 3x3x3 weights for the direct-convolution kernels, per
  // layer in two orientations: [0] rows = output channels of the stored
  // convolution (A = W), [1] rows = its input channels (A = WT); refreshed with WT
  uint16_t *pack = nullptr;
  int64_t pk_off[topo::L_COUNT][2] = {};
  int pk_mp[topo::L_COUNT][2] = {}, pk_cp[topo::L_COUNT][2] = {}, pk_cc[topo::L_COUNT][2] = {};
  int adam_step = 0;
  int precision = TOPO_PREC_FP32;  // arithmetic of the convolutions: FP32 or BF16 operands
  topo::Reducer red{};
  topo::NnWork work;  // workspace of the API calls
  std::vector<void *> allocs;
  ~topo_nn();
};

namespace topo {
// (re)allocates w for grid g0 (nodes) and batch B when they differ
topo_status nn_prepare(const topo_nn *nn, NnWork &w, Dim3 g0, int B, bool grads);
// refreshes the transposed weights after W changed
topo_status nn_refresh(topo_nn *nn, hipStream_t s);
// forward of w.x -> w.out
topo_status nn_forward(topo_nn *nn, NnWork &w, hipStream_t s, const int *skip);
// backward from w.dout: parameter gradients into nn->G
topo_status nn_backward(topo_nn *nn, NnWork &w, hipStream_t s);
}  // namespace topo
