// Host side of libtopo: argument validation, setup (element stiffness, filter
// stencil, multigrid hierarchy, workspaces), the conjugate-gradient solve with a
// multigrid or Jacobi preconditioner, and the SIMP iteration driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "ke_code.h"
#include "nn.h"

namespace topo {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

// ---------------------------------------------------------------------------
// H8 element stiffness (Finite Element Analysis section): KE = int B^T D B over
// the unit cube with a 2x2x2 Gauss rule, isotropic D for E = 1 and Poisson
// ratio nu, Voigt order xx, yy, zz, xy, yz, zx with engineering shears.
static void element_stiffness(double nu, double KE[576]) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  double D[6][6] = {};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) D[a][b] = lam + (a == b ? 2.0 * mu : 0.0);
  D[3][3] = D[4][4] = D[5][5] = mu;
  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  std::fill(KE, KE + 576, 0.0);
  for (int qa = 0; qa < 2; ++qa)
    for (int qb = 0; qb < 2; ++qb)
      for (int qc = 0; qc < 2; ++qc) {
        const double p[3] = {gp[qa], gp[qb], gp[qc]};
        double B[6][24] = {};
        for (int n = 0; n < 8; ++n) {
          const int c[3] = {cx(n), cy(n), cz(n)};
          double gr[3];
          for (int d = 0; d < 3; ++d) {
            double v = c[d] ? 1.0 : -1.0;
            for (int o = 0; o < 3; ++o)
              if (o != d) v *= c[o] ? p[o] : 1.0 - p[o];
            gr[d] = v;
          }
          B[0][3 * n + 0] = gr[0];
          B[1][3 * n + 1] = gr[1];
          B[2][3 * n + 2] = gr[2];
          B[3][3 * n + 0] = gr[1];
          B[3][3 * n + 1] = gr[0];
          B[4][3 * n + 1] = gr[2];
          B[4][3 * n + 2] = gr[1];
          B[5][3 * n + 0] = gr[2];
          B[5][3 * n + 2] = gr[0];
        }
        double DB[6][24];
        for (int r = 0; r < 6; ++r)
          for (int j = 0; j < 24; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += D[r][k] * B[k][j];
            DB[r][j] = s;
          }
        for (int i = 0; i < 24; ++i)
          for (int j = 0; j < 24; ++j) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += B[k][i] * DB[k][j];
            KE[i * 24 + j] += 0.125 * s;
          }
      }
}

// Largest eigenvalue of a symmetric n x n matrix by cyclic Jacobi rotations.
static double sym_max_eig(std::vector<double> A, int n) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  double m = A[0];
  for (int i = 1; i < n; ++i) m = std::max(m, A[i * n + i]);
  return m;
}

// ---------------------------------------------------------------------------
template <typename T>
static hipError_t dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void **)p, count * sizeof(T));
}

constexpr double kChebRatio = 30.0;  // Chebyshev interval [lam_max / ratio, lam_max]
// node-column kernel: fuse the first smoothing step into the operator pass below
// this many nodes (above, that kernel is arithmetic bound and forming the operand
// on the fly doubles its loads); the element-column kernel always fuses it
constexpr int64_t kFuseFirstStepBelow = 400000;

// Multigrid level data in one precision.
template <typename T>
struct LevelBufs {
  T *E = nullptr;     // moduli incl. the 2^level stiffness scale
  T *dinv = nullptr;  // inverse Jacobi diagonal (0 on fixed dofs)
  T *b = nullptr, *x = nullptr, *res = nullptr, *d0 = nullptr, *d1 = nullptr;
};

struct Level {
  Grid g{};
  double *E = nullptr;       // moduli incl. the 2^level stiffness scale
  double *dinv = nullptr;    // inverse Jacobi diagonal (0 on fixed dofs)
  uint8_t *fixed = nullptr;  // per node, bit c = dof c fixed
  double *b = nullptr, *x = nullptr, *res = nullptr, *d0 = nullptr, *d1 = nullptr;
  LevelBufs<float> f32;      // single-precision copy for the mixed-precision preconditioner
  int shape = -1;            // K.u launch shape of the smoothing passes (-1: by grid size)
  const float *ke32 = nullptr;  // element matrix for the single-precision matrix-core K.u
  const void *ke16 = nullptr;
};

template <typename T>
LevelBufs<T> bufs(Level &L);
template <>
LevelBufs<double> bufs<double>(Level &L) {
  LevelBufs<double> b;
  b.E = L.E;
  b.dinv = L.dinv;
  b.b = L.b;
  b.x = L.x;
  b.res = L.res;
  b.d0 = L.d0;
  b.d1 = L.d1;
  return b;
}
template <>
LevelBufs<float> bufs<float>(Level &L) {
  return L.f32;
}

}  // namespace topo

using namespace topo;

struct topo_ctx {
  topo_problem prob{};
  topo_opts opts{};
  hipStream_t stream = nullptr;
  Grid g{};
  int64_t nel = 0, ndof = 0, nnodes = 0, n_design = 0;
  double target = 0.0;
  // constants
  Kappa kap{};
  double lam_max = 0.0;  // top of the Chebyshev smoothing interval (cheb_upper x the element bound)
  // problem data
  double *f = nullptr;
  int8_t *mask = nullptr;
  // filter
  FilterArgs filt{};
  int *d_off = nullptr;
  double *d_w = nullptr, *Hs = nullptr, *sD = nullptr, *volw = nullptr;
  // multigrid
  std::vector<Level> lv;
  double *Ainv = nullptr;
  double *Awork = nullptr;  // blocked inversion workspace (larger coarsest levels)
  int coarse_due = 0;       // SIMP iterations until the coarse inverse is recomputed
  int ncoarse = 0;
  bool mixed = false;        // single-precision preconditioner
  KappaT<float> kap32{};
  // CG vectors (level-0 b / x double as the V-cycle's rhs / result)
  double *u = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  float *z32 = nullptr;      // z of the single-precision multigrid preconditioner
  // SIMP work
  double *xphys = nullptr, *ce = nullptr, *dc = nullptr, *dcf = nullptr, *oc_a = nullptr,
         *tmp = nullptr, *xnew = nullptr;
  // reductions and scalars
  Scalars *sc = nullptr;
  Scalars *h_sc = nullptr;  // pinned mirror
  Reducer red{};
  int have_u = 0;
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  // the coarse inverse of a SIMP iteration, built on a stream of its own while
  // the warm start and the start of the solve run; joined before the V-cycle
  hipStream_t side = nullptr;
  hipEvent_t side_ev[2] = {};
  bool inv_pending = false;
  hipGraph_t cg_graph[3] = {};
  hipGraphExec_t cg_exec[3] = {};    // chunk of CG iterations, per preconditioner kind
  int cg_prev_iters[3] = {};          // iterations of the last solve, per preconditioner kind
  // CG's stopping test left to the next finest-level RES0 pass: r.r partials
  const double *chk_parts = nullptr;
  int chk_n = 0;
  // learned preconditioner
  int shape_cg = -1;                 // K.u launch shape of the CG product (-1: by grid size)
  size_t tail_start = 0;             // first level of the one-workgroup V-cycle tail (0: none)
  topo_nn *nn = nullptr;
  int nn_graph_precision = -1;       // network precision the captured learned chunk uses
  NnWork nnw;                        // activations (batch 1) on the node grid
  double *nn_scale = nullptr;        // rms of the residual of the current application
  double *ustar = nullptr;           // training-pair generation: converged solution
  double *u_prev = nullptr;          // extrapolated warm start: the solution before the last
  int n_warm = 0;                    // consecutive solutions available for the warm start
  double *basis[4] = {};             // projected warm start: the last solutions (ring)
  int nbasis = 0, basis_next = 0;
  double *gram = nullptr;            // its Gram matrix and right-hand side on the device
  std::vector<void *> allocs;

  template <typename T>
  hipError_t alloc(T **p_, size_t count) {
    hipError_t e = dalloc(p_, count);
    if (e == hipSuccess) allocs.push_back((void *)*p_);
    return e;
  }
  void drop_graphs() {
    for (int k = 0; k < 3; ++k) {
      if (cg_exec[k]) (void)hipGraphExecDestroy(cg_exec[k]);
      if (cg_graph[k]) (void)hipGraphDestroy(cg_graph[k]);
      cg_exec[k] = nullptr;
      cg_graph[k] = nullptr;
    }
  }
  ~topo_ctx() {
    drop_graphs();
    nnw.release();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (side) {
      (void)hipStreamSynchronize(side);
      (void)hipStreamDestroy(side);
    }
    for (hipEvent_t e : side_ev)
      if (e) (void)hipEventDestroy(e);
    for (void *a : allocs) (void)hipFree(a);
    if (h_sc) (void)hipHostFree(h_sc);
  }
};

#define TOPO_ALLOC(ptr, count)                                               \
  do {                                                                       \
    hipError_t ae_ = ctx->alloc(&(ptr), (count));                            \
    if (ae_ != hipSuccess) {                                                 \
      set_error("device allocation of %s (%zu elements) failed: %s", #ptr,   \
                (size_t)(count), hipGetErrorString(ae_));                    \
      return ae_ == hipErrorOutOfMemory ? TOPO_ENOMEM : TOPO_EDEVICE;        \
    }                                                                        \
  } while (0)

extern "C" void topo_default_opts(topo_opts *o) {
  if (!o) return;
  o->precision = TOPO_PREC_FP64;
  o->precond = TOPO_PRECOND_MG;
  o->mg_levels = 0;
  o->mg_max_coarse_dof = 1500;
  // measured at 160x80x80: one step on the finest level and four below give the
  // fewest V-cycle launches for the iteration count
  o->cheb_degree = 1;
  o->cheb_degree_coarse = 4;
  o->rtol = 1e-8;
  o->max_iters = 1000;
  o->warm_start = 3;
  o->oc_tol = 1e-12;
  o->check_every = 3;
  o->use_graphs = 1;
  o->nn_max_iters = 200;
  o->autotune = 0;
  o->coarse_tail_nodes = 0;  // per-level launches measured faster with the element-column kernel
  o->mfma_smoothing = 0;
  o->ku_kernel = TOPO_KU_AUTO;
  o->ku_shape = -1;
  o->coarse_refresh = 1;
  for (int l = 0; l < 8; ++l) o->cheb_degree_level[l] = 0;
  o->group_launch = 1;
  o->cheb_upper = 1.0;
}

extern "C" const char *topo_last_error(void) { return g_err; }

static topo_status validate(const topo_problem *P, const topo_opts *O) {
  if (!P || !O) return set_error("NULL problem or options"), TOPO_EINVAL;
  if (P->nelx < 1 || P->nely < 1 || P->nelz < 1)
    return set_error("grid sizes must be >= 1"), TOPO_EINVAL;
  const int64_t nel = (int64_t)P->nelx * P->nely * P->nelz;
  const int64_t ndof = 3 * (int64_t)(P->nelx + 1) * (P->nely + 1) * (P->nelz + 1);
  if (ndof > ((int64_t)1 << 40)) return set_error("grid too large"), TOPO_EINVAL;
  if (!(P->E0 > 0) || !(P->Emin > 0) || !(P->Emin < P->E0))
    return set_error("need 0 < Emin < E0"), TOPO_EINVAL;
  if (!(P->nu > -1.0 && P->nu < 0.5)) return set_error("nu must lie in (-1, 0.5)"), TOPO_EINVAL;
  if (!(P->penal >= 1.0)) return set_error("penal must be >= 1"), TOPO_EINVAL;
  if (!(P->rmin > 0.0) || P->rmin > 16.0) return set_error("rmin must lie in (0, 16]"), TOPO_EINVAL;
  if (!(P->volfrac > 0.0 && P->volfrac <= 1.0)) return set_error("volfrac must lie in (0, 1]"), TOPO_EINVAL;
  if (!(P->move > 0.0) || !(P->eta > 0.0)) return set_error("move and eta must be > 0"), TOPO_EINVAL;
  if (P->filter != TOPO_FILTER_DENSITY && P->filter != TOPO_FILTER_SENSITIVITY)
    return set_error("unknown filter mode %d", P->filter), TOPO_EINVAL;
  if (P->vol_mode != TOPO_VOL_DESIGN && P->vol_mode != TOPO_VOL_ALL)
    return set_error("unknown vol_mode %d", P->vol_mode), TOPO_EINVAL;
  if (!P->f) return set_error("load vector f is NULL"), TOPO_EINVAL;
  if (P->n_fixed < 6 || !P->fixed_dofs)
    return set_error("at least 6 fixed dofs are needed to remove rigid-body motion"), TOPO_EINVAL;
  for (int64_t i = 0; i < P->n_fixed; ++i)
    if (P->fixed_dofs[i] < 0 || P->fixed_dofs[i] >= ndof)
      return set_error("fixed dof %lld out of range [0, %lld)", (long long)P->fixed_dofs[i], (long long)ndof), TOPO_EINVAL;
  int64_t nd = nel;
  if (P->mask) {
    nd = 0;
    for (int64_t e = 0; e < nel; ++e) {
      if (P->mask[e] < 0 || P->mask[e] > 2)
        return set_error("mask value %d at element %lld not in {0,1,2}", (int)P->mask[e], (long long)e), TOPO_EINVAL;
      nd += P->mask[e] == 0;
    }
  }
  if (nd == 0) return set_error("no design element"), TOPO_EINVAL;
  if (P->vol_mode == TOPO_VOL_ALL) {
    int64_t ns = 0;
    if (P->mask)
      for (int64_t e = 0; e < nel; ++e) ns += P->mask[e] == 2;
    if (!(P->volfrac * (double)nel - (double)ns > 0.0))
      return set_error("volfrac * nel must exceed the number of fixed-solid elements"), TOPO_EINVAL;
  }
  if (O->precision != TOPO_PREC_FP64 && O->precision != TOPO_PREC_FP32 && O->precision != TOPO_PREC_BF16)
    return set_error("unknown precision %d", O->precision), TOPO_EINVAL;
  if (O->precond != TOPO_PRECOND_JACOBI && O->precond != TOPO_PRECOND_MG && O->precond != TOPO_PRECOND_LEARNED)
    return set_error("unknown preconditioner %d", O->precond), TOPO_EINVAL;
  if (O->precond == TOPO_PRECOND_LEARNED && O->nn_max_iters < 1)
    return set_error("nn_max_iters must be >= 1"), TOPO_EINVAL;
  if (O->cheb_degree < 1 || O->cheb_degree > 16) return set_error("cheb_degree must lie in [1, 16]"), TOPO_EINVAL;
  if (O->cheb_degree_coarse < 0 || O->cheb_degree_coarse > 16)
    return set_error("cheb_degree_coarse must lie in [0, 16]"), TOPO_EINVAL;
  if (!(O->rtol > 0.0) || O->max_iters < 1) return set_error("rtol > 0 and max_iters >= 1 required"), TOPO_EINVAL;
  if (!(O->oc_tol > 0.0)) return set_error("oc_tol must be > 0"), TOPO_EINVAL;
  if (O->mg_levels < 0 || O->mg_levels > 16) return set_error("mg_levels must lie in [0, 16]"), TOPO_EINVAL;
  if (O->coarse_tail_nodes < 0) return set_error("coarse_tail_nodes must be >= 0"), TOPO_EINVAL;
  if (O->warm_start < 0 || O->warm_start > 3) return set_error("warm_start must be 0, 1, 2 or 3"), TOPO_EINVAL;
  if (O->coarse_refresh < 1) return set_error("coarse_refresh must be >= 1"), TOPO_EINVAL;
  if (O->group_launch != 0 && O->group_launch != 1) return set_error("group_launch must be 0 or 1"), TOPO_EINVAL;
  if (O->autotune < 0 || O->autotune > 2) return set_error("autotune must be 0, 1 or 2"), TOPO_EINVAL;
  if (!(O->cheb_upper > 0.0 && O->cheb_upper <= 1.0)) return set_error("cheb_upper must lie in (0, 1]"), TOPO_EINVAL;
  for (int l = 0; l < 8; ++l)
    if (O->cheb_degree_level[l] < 0 || O->cheb_degree_level[l] > 16)
      return set_error("cheb_degree_level[%d] must lie in [0, 16]", l), TOPO_EINVAL;
  if (O->ku_kernel != TOPO_KU_AUTO && O->ku_kernel != TOPO_KU_NODE && O->ku_kernel != TOPO_KU_ELEMENT)
    return set_error("unknown ku_kernel %d", O->ku_kernel), TOPO_EINVAL;
  if (!(O->ku_shape == -1 || (O->ku_shape >= 0 && O->ku_shape < kKuShapes) ||
        (O->ku_shape >= kKuShapeHada && O->ku_shape < kKuShapeHada + kKuShapesHada)))
    return set_error("ku_shape must be -1, 0..%d or %d..%d", kKuShapes - 1, kKuShapeHada,
                     kKuShapeHada + kKuShapesHada - 1), TOPO_EINVAL;
  return TOPO_OK;
}

static std::vector<Grid> mg_hierarchy(Grid g, const topo_opts &o) {
  std::vector<Grid> dims{g};
  const int cap = o.mg_levels > 0 ? o.mg_levels : 16;
  while ((int)dims.size() < cap) {
    const Grid c = dims.back();
    if (o.mg_levels == 0 && c.ndof() <= o.mg_max_coarse_dof) break;
    if (std::min(c.nx, std::min(c.ny, c.nz)) < 2) break;
    dims.push_back(Grid{(c.nx + 1) / 2, (c.ny + 1) / 2, (c.nz + 1) / 2});
  }
  return dims;
}

static topo_status autotune(topo_ctx *ctx);

extern "C" topo_status topo_setup(const topo_problem *P, const topo_opts *O, void *hip_stream,
                                  topo_ctx **out) {
  if (!out) return set_error("out is NULL"), TOPO_EINVAL;
  *out = nullptr;
  topo_opts defaults;
  topo_default_opts(&defaults);
  if (!O) O = &defaults;
  topo_status st = validate(P, O);
  if (st != TOPO_OK) return st;
  int device = 0;
  TOPO_HIP(hipGetDevice(&device));
  TOPO_HIP(hipSetDevice(device));
  std::unique_ptr<topo_ctx> c(new topo_ctx());
  topo_ctx *ctx = c.get();
  ctx->prob = *P;
  ctx->prob.mask = nullptr;
  ctx->prob.fixed_dofs = nullptr;
  ctx->prob.f = nullptr;
  ctx->opts = *O;
  ctx->stream = (hipStream_t)hip_stream;
  hipStream_t s = ctx->stream;
  Grid g{P->nelx, P->nely, P->nelz};
  ctx->g = g;
  ctx->nel = g.nel();
  ctx->nnodes = g.nnodes();
  ctx->ndof = g.ndof();

  // element stiffness and the Jacobi-scaled bound lambda_max(diag(KE)^-1 KE),
  // whose cheb_upper-th part is the top of the smoothers' Chebyshev interval
  double KE[576];
  element_stiffness(P->nu, KE);
  double KEd[24];
  for (int i = 0; i < 24; ++i) KEd[i] = KE[i * 24 + i];
  {
    std::vector<double> S(576);
    for (int i = 0; i < 24; ++i)
      for (int j = 0; j < 24; ++j) S[i * 24 + j] = KE[i * 24 + j] / std::sqrt(KEd[i] * KEd[j]);
    ctx->lam_max = O->cheb_upper * sym_max_eig(S, 24);
  }
  // the kernels use the exact compile-time form of KE; check it against the
  // quadrature once (they agree to rounding for every nu)
  ctx->kap = make_kappa(P->nu);
  ctx->kap32 = to_float(ctx->kap);
  ctx->mixed = O->precision != TOPO_PREC_FP64;
  for (int I = 0; I < 576; ++I) {
    const double v = kKeTable.sign[I] * ctx->kap.k[kKeTable.idx[I]];
    if (std::fabs(v - KE[I]) > 1e-12 * (1.0 + std::fabs(KE[I])))
      return set_error("internal: element stiffness tables disagree"), TOPO_EINVAL;
  }

  // host-side staging of the problem arrays
  std::vector<int8_t> hmask(ctx->nel, 0);
  if (P->mask) std::memcpy(hmask.data(), P->mask, ctx->nel);
  ctx->n_design = std::count(hmask.begin(), hmask.end(), (int8_t)0);
  // volume target of the design-element sum
  if (P->vol_mode == TOPO_VOL_ALL)
    ctx->target = P->volfrac * (double)ctx->nel - (double)std::count(hmask.begin(), hmask.end(), (int8_t)2);
  else
    ctx->target = P->volfrac * (double)ctx->n_design;
  std::vector<uint8_t> hfix(ctx->nnodes, 0);
  for (int64_t i = 0; i < P->n_fixed; ++i) hfix[P->fixed_dofs[i] / 3] |= (uint8_t)(1u << (P->fixed_dofs[i] % 3));
  std::vector<double> hf(P->f, P->f + ctx->ndof);
  for (int64_t n = 0; n < ctx->nnodes; ++n)
    for (int cc = 0; cc < 3; ++cc)
      if ((hfix[n] >> cc) & 1) hf[3 * n + cc] = 0.0;  // loads on fixed dofs are eliminated
  double ff = 0.0;
  for (double v : hf) ff += v * v;
  if (ff == 0.0) return set_error("load vector is zero on the free dofs"), TOPO_EINVAL;

  TOPO_ALLOC(ctx->f, ctx->ndof);
  TOPO_ALLOC(ctx->mask, ctx->nel);
  TOPO_HIP(hipMemcpyAsync(ctx->f, hf.data(), ctx->ndof * sizeof(double), hipMemcpyHostToDevice, s));
  TOPO_HIP(hipMemcpyAsync(ctx->mask, hmask.data(), ctx->nel, hipMemcpyHostToDevice, s));

  // multigrid hierarchy (level 0 only when Jacobi is used)
  // (the learned preconditioner keeps the hierarchy for its fallback)
  std::vector<Grid> dims = O->precond != TOPO_PRECOND_JACOBI ? mg_hierarchy(g, *O) : std::vector<Grid>{g};
  ctx->lv.resize(dims.size());
  for (size_t l = 0; l < dims.size(); ++l) {
    Level &L = ctx->lv[l];
    L.g = dims[l];
    TOPO_ALLOC(L.E, L.g.nel());
    TOPO_ALLOC(L.dinv, L.g.ndof());
    TOPO_ALLOC(L.fixed, L.g.nnodes());
    TOPO_ALLOC(L.res, L.g.ndof());
    TOPO_ALLOC(L.d0, L.g.ndof());
    TOPO_ALLOC(L.d1, L.g.ndof());
    if (l > 0) {
      TOPO_ALLOC(L.b, L.g.ndof());
      TOPO_ALLOC(L.x, L.g.ndof());
    }
    if (O->precision != TOPO_PREC_FP64) {
      TOPO_ALLOC(L.f32.E, L.g.nel());
      TOPO_ALLOC(L.f32.dinv, L.g.ndof());
      TOPO_ALLOC(L.f32.b, L.g.ndof());
      TOPO_ALLOC(L.f32.x, L.g.ndof());
      TOPO_ALLOC(L.f32.res, L.g.ndof());
      TOPO_ALLOC(L.f32.d0, L.g.ndof());
      TOPO_ALLOC(L.f32.d1, L.g.ndof());
    }
  }
  if (O->precision != TOPO_PREC_FP64) {
    // element matrix for the single-precision matrix-core K.u: FP32 [32][24] and
    // BF16 [32][32] (round to nearest even), zero padded
    std::vector<float> k32(32 * 24, 0.0f);
    std::vector<uint16_t> k16(32 * 32, 0);
    for (int r = 0; r < 24; ++r)
      for (int c = 0; c < 24; ++c) {
        const float v = (float)KE[r * 24 + c];
        k32[r * 24 + c] = v;
        uint32_t bits;
        std::memcpy(&bits, &v, 4);
        bits += 0x7FFFu + ((bits >> 16) & 1u);
        k16[r * 32 + c] = (uint16_t)(bits >> 16);
      }
    float *d32 = nullptr;
    uint16_t *d16 = nullptr;
    TOPO_ALLOC(d32, k32.size());
    TOPO_ALLOC(d16, k16.size());
    TOPO_HIP(hipMemcpyAsync(d32, k32.data(), k32.size() * sizeof(float), hipMemcpyHostToDevice, s));
    TOPO_HIP(hipMemcpyAsync(d16, k16.data(), k16.size() * sizeof(uint16_t), hipMemcpyHostToDevice, s));
    TOPO_HIP(hipStreamSynchronize(s));  // host staging goes out of scope
    for (Level &L : ctx->lv) {
      L.ke32 = d32;
      L.ke16 = d16;
      // BF16 mode: every smoothing pass on the matrix cores with BF16 operands;
      // FP32 mode: on the FP32 matrix cores when asked to (else by grid size)
      if (O->precision == TOPO_PREC_BF16) L.shape = kKuShapeMfmaBf16;
      else if (O->mfma_smoothing) L.shape = kKuShapeMfma;
    }
  }
  TOPO_HIP(hipMemcpyAsync(ctx->lv[0].fixed, hfix.data(), ctx->nnodes, hipMemcpyHostToDevice, s));
  for (size_t l = 1; l < dims.size(); ++l)
    TOPO_HIP(launch_coarse_fixed(s, dims[l - 1], dims[l], ctx->lv[l - 1].fixed, ctx->lv[l].fixed));
  if (dims.size() > 1) {
    ctx->ncoarse = (int)dims.back().ndof();
    if (ctx->ncoarse > 2048) return set_error("coarsest level has %d dofs (> 2048); allow more levels", ctx->ncoarse), TOPO_EINVAL;
    TOPO_ALLOC(ctx->Ainv, (size_t)ctx->ncoarse * ctx->ncoarse);
    if (dense_invert_work(ctx->ncoarse)) TOPO_ALLOC(ctx->Awork, dense_invert_work(ctx->ncoarse));
  }

  // CG and SIMP vectors
  TOPO_ALLOC(ctx->u, ctx->ndof);
  TOPO_ALLOC(ctx->r, ctx->ndof);
  TOPO_ALLOC(ctx->z, ctx->ndof);
  TOPO_ALLOC(ctx->p, ctx->ndof);
  TOPO_ALLOC(ctx->q, ctx->ndof);
  TOPO_ALLOC(ctx->tmp, ctx->ndof);
  TOPO_ALLOC(ctx->xphys, ctx->nel);
  TOPO_ALLOC(ctx->ce, ctx->nel);
  TOPO_ALLOC(ctx->dc, ctx->nel);
  TOPO_ALLOC(ctx->dcf, ctx->nel);
  TOPO_ALLOC(ctx->oc_a, ctx->nel);
  TOPO_ALLOC(ctx->xnew, ctx->nel);
  TOPO_ALLOC(ctx->nn_scale, 1);
  TOPO_HIP(hipMemsetAsync(ctx->u, 0, ctx->ndof * sizeof(double), s));
  TOPO_HIP(hipMemsetAsync(ctx->z, 0, ctx->ndof * sizeof(double), s));
  if (ctx->mixed) {
    TOPO_ALLOC(ctx->z32, ctx->ndof);
    TOPO_HIP(hipMemsetAsync(ctx->z32, 0, ctx->ndof * sizeof(float), s));
  }
  TOPO_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  ctx->lv[0].b = ctx->r;
  ctx->lv[0].x = ctx->z;

  // one-workgroup tail of the V-cycle: the levels below coarse_tail_nodes nodes
  // (never the finest level, whose last pass also forms r.z)
  if (dims.size() > 1 && O->coarse_tail_nodes > 0) {
    const bool fp32 = O->precision != TOPO_PREC_FP64;
    auto level_bytes = [&](const Grid &g) { return fp32 ? tail_level_bytes<float>(g) : tail_level_bytes<double>(g); };
    const int nco = (int)dims.back().ndof();
    size_t bytes = level_bytes(dims.back()) + (fp32 ? tail_solve_bytes<float>(nco) : tail_solve_bytes<double>(nco));
    size_t t = dims.size() - 1;
    // the element scratch is sized by the finest tail level, the one being added
    auto scratch_bytes = [&](const Grid &g) { return fp32 ? tail_scratch_bytes<float>(g) : tail_scratch_bytes<double>(g); };
    while (t > 1 && dims[t - 1].nnodes() <= O->coarse_tail_nodes &&
           bytes + level_bytes(dims[t - 1]) + scratch_bytes(dims[t - 1]) <= kTailMaxLds &&
           dims.size() - t < (size_t)kTailMaxLevels) {
      bytes += level_bytes(dims[t - 1]);
      --t;
    }
    if (dims.size() - t >= 2 && bytes <= kTailMaxLds) ctx->tail_start = t;
    if (ctx->tail_start)
      TOPO_HIP(fp32 ? prepare_vcycle_tail_t<float>(kTailMaxLds) : prepare_vcycle_tail_t<double>(kTailMaxLds));
  }

  // reductions
  // enough partials for every K.u launch shape on the finest grid and for the vector kernels
  const int64_t nb_nodes = (ctx->nnodes + 255) / 256;
  const int64_t nb_ku = ku_max_blocks(g);
  if (nb_ku >= INT32_MAX) return set_error("grid too large for the K.u launch shapes"), TOPO_EINVAL;
  ctx->red.max_blocks = (int)std::max<int64_t>({16384, nb_nodes + 1, nb_ku + 1});
  TOPO_ALLOC(ctx->red.partials, (size_t)ctx->red.max_blocks * kMaxRed);
  TOPO_ALLOC(ctx->sc, 1);
  TOPO_HIP(hipMemsetAsync(ctx->sc, 0, sizeof(Scalars), s));
  if (hipHostMalloc((void **)&ctx->h_sc, sizeof(Scalars), hipHostMallocDefault) != hipSuccess) {
    ctx->h_sc = nullptr;
    return set_error("pinned host allocation failed"), TOPO_ENOMEM;
  }

  // filter stencil: offsets with |d| < rmin, weights rmin - |d|
  std::vector<int> off;
  std::vector<double> w;
  const int R = (int)std::ceil(P->rmin) - 1;
  for (int dk = -R; dk <= R; ++dk)
    for (int dj = -R; dj <= R; ++dj)
      for (int di = -R; di <= R; ++di) {
        const double d = std::sqrt((double)(di * di + dj * dj + dk * dk));
        if (d < P->rmin) {
          off.push_back(di);
          off.push_back(dj);
          off.push_back(dk);
          w.push_back(P->rmin - d);
        }
      }
  TOPO_ALLOC(ctx->d_off, off.size());
  TOPO_ALLOC(ctx->d_w, w.size());
  TOPO_ALLOC(ctx->Hs, ctx->nel);
  TOPO_ALLOC(ctx->sD, ctx->nel);
  TOPO_ALLOC(ctx->volw, ctx->nel);
  TOPO_HIP(hipMemcpyAsync(ctx->d_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, s));
  TOPO_HIP(hipMemcpyAsync(ctx->d_w, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, s));
  ctx->filt = FilterArgs{g, (int)w.size(), ctx->d_off, ctx->d_w, ctx->Hs, ctx->sD, ctx->mask, R, {}};
  for (int q = 0; q < 16; ++q) {
    const double d = std::sqrt((double)q);  // the same weight expression as the offset list's
    ctx->filt.wsq[q] = d < P->rmin ? P->rmin - d : 0.0;
  }
  TOPO_HIP(launch_filter_hs(s, ctx->filt, ctx->Hs));
  TOPO_HIP(launch_design_scale(s, ctx->nel, ctx->mask, ctx->Hs, ctx->sD));
  if (P->filter == TOPO_FILTER_DENSITY) {
    TOPO_HIP(launch_filter(s, TOPO_FILTER_VOLW, ctx->filt, nullptr, nullptr, ctx->volw));
  } else {
    std::vector<double> hv(ctx->nel);
    for (int64_t e = 0; e < ctx->nel; ++e) hv[e] = hmask[e] == 0 ? 1.0 : 0.0;
    TOPO_HIP(hipMemcpyAsync(ctx->volw, hv.data(), ctx->nel * sizeof(double), hipMemcpyHostToDevice, s));
    TOPO_HIP(hipStreamSynchronize(s));  // hv goes out of scope
  }
  // launch shapes by grid size within the chosen K.u kernel (the matrix-core
  // modes above keep theirs); the autotuner may replace them
  for (Level &L : ctx->lv)
    if (L.shape < 0) L.shape = O->ku_shape >= 0 ? O->ku_shape : ku_shape_for(L.g, KU_CHEB, O->ku_kernel, ctx->mixed);
  ctx->shape_cg = O->ku_shape >= 0 ? O->ku_shape : ku_shape_for(g, KU_STORE_DOT, O->ku_kernel);
  if (O->autotune) {
    st = autotune(ctx);
    if (st != TOPO_OK) return st;
  }
  TOPO_HIP(hipStreamSynchronize(s));
  *out = c.release();
  return TOPO_OK;
}

extern "C" void topo_destroy(topo_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
}

extern "C" topo_status topo_sizes(const topo_ctx *ctx, int64_t *nel, int64_t *ndof, int32_t *levels) {
  if (!ctx) return set_error("ctx is NULL"), TOPO_EINVAL;
  if (nel) *nel = ctx->nel;
  if (ndof) *ndof = ctx->ndof;
  if (levels) *levels = (int32_t)ctx->lv.size();
  return TOPO_OK;
}

// ---------------------------------------------------------------------------
static KuArgs ku_args(topo_ctx *ctx, const Level &L, const double *u) {
  KuArgs a{};
  a.g = L.g;
  a.E = L.E;
  a.u = u;
  a.fixed = L.fixed;
  a.dinv = L.dinv;
  return a;
}

template <typename T>
static KuArgsT<T> ku_args_t(Level &L, const T *u) {
  const LevelBufs<T> B = bufs<T>(L);
  KuArgsT<T> a{};
  a.g = L.g;
  a.E = B.E;
  a.u = u;
  a.fixed = L.fixed;
  a.dinv = B.dinv;
  a.ke32 = L.ke32;
  a.ke16 = L.ke16;
  return a;
}

template <typename T>
static const KappaT<T> &kappa_of(const topo_ctx *ctx);
template <>
const KappaT<double> &kappa_of<double>(const topo_ctx *ctx) {
  return ctx->kap;
}
template <>
const KappaT<float> &kappa_of<float>(const topo_ctx *ctx) {
  return ctx->kap32;
}

// ---------------------------------------------------------------------------
// Initial guess of a solve from the last few solutions: the combination U alpha
// of the stored solutions U that is closest to the new solution in the energy
// norm of the new operator, i.e. (U^T K U) alpha = U^T f.  The small Gram
// system is solved on the host through its eigen-decomposition (directions with
// eigenvalues below 1e-12 of the largest, i.e. nearly repeated solutions, are
// dropped).
constexpr int kMaxBasis = 4;

// symmetric eigen-decomposition by cyclic Jacobi rotations: A = V diag(w) V^T
static void sym_eig(std::vector<double> A, int n, std::vector<double> &w, std::vector<double> &V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, scale = 0.0;
    for (int p = 0; p < n; ++p) {
      scale += A[p * n + p] * A[p * n + p];
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    }
    if (off <= 1e-30 * scale) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - sn * akq;
          A[k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - sn * aqk;
          A[q * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - sn * vkq;
          V[k * n + q] = sn * vkp + c * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

// the dot products of column j of the Gram matrix: basis[0..j] against b
// (j = nbasis with b = f: the right-hand side g)
static MultiDotArgs gram_column(const topo_ctx *ctx, int j, const double *b) {
  MultiDotArgs m{};
  m.nv = std::min(j + 1, ctx->nbasis);
  for (int i = 0; i < m.nv; ++i) m.a[i] = ctx->basis[i];
  m.b = b;
  return m;
}

// Coefficients of the Galerkin projection u = sum_i alpha_i u_i of the new
// solution onto the stored ones: G alpha = g, G solved through its eigenpairs
// with the (numerically) null directions dropped.  h: the Gram matrix read
// back from the device (layout above).  False when a coefficient is not finite.
static bool projection_coefficients(const double *h, int nb, double *alpha) {
  std::vector<double> G(nb * nb), w, V;
  for (int j = 0; j < nb; ++j)
    for (int i = 0; i <= j; ++i) G[i * nb + j] = G[j * nb + i] = h[j * kMaxBasis + i];
  sym_eig(G, nb, w, V);
  double wmax = 0.0;
  for (double v : w) wmax = std::max(wmax, v);
  for (int i = 0; i < kMaxBasis; ++i) alpha[i] = 0.0;
  for (int k = 0; k < nb; ++k) {
    if (!(w[k] > 1e-12 * wmax)) continue;
    double qg = 0.0;
    for (int i = 0; i < nb; ++i) qg += V[i * nb + k] * h[kMaxBasis * kMaxBasis + i];
    for (int i = 0; i < nb; ++i) alpha[i] += V[i * nb + k] * qg / w[k];
  }
  for (int i = 0; i < nb; ++i)
    if (!std::isfinite(alpha[i])) return false;
  return true;
}

static topo_status projected_start(topo_ctx *ctx) {
  hipStream_t s = ctx->stream;
  const int nb = ctx->nbasis;
  Level &L0 = ctx->lv[0];
  // Gram matrix G_ij = u_i . K u_j (column j: i <= j, at gram[j kMaxBasis + i])
  // and g_i = u_i . f (at gram[kMaxBasis^2 + i])
  for (int j = 0; j < nb; ++j) {
    KuArgs a = ku_args(ctx, L0, ctx->basis[j]);
    a.y = ctx->tmp;
    TOPO_HIP(launch_ku(s, KU_STORE, a, ctx->kap, ctx->red, fin_sum(nullptr)));
    TOPO_HIP(launch_multi_dot(s, ctx->ndof, gram_column(ctx, j, ctx->tmp), ctx->red,
                              fin_sum(&ctx->gram[j * kMaxBasis])));
  }
  TOPO_HIP(launch_multi_dot(s, ctx->ndof, gram_column(ctx, nb, ctx->f), ctx->red,
                            fin_sum(&ctx->gram[kMaxBasis * kMaxBasis])));
  double h[kMaxBasis * kMaxBasis + kMaxBasis];
  TOPO_HIP(hipMemcpyAsync(h, ctx->gram, sizeof(h), hipMemcpyDeviceToHost, s));
  TOPO_HIP(hipStreamSynchronize(s));
  double alpha[kMaxBasis];
  if (!projection_coefficients(h, nb, alpha)) return TOPO_OK;  // keep the plain warm start
  const double *vs[kMaxBasis];
  for (int i = 0; i < nb; ++i) vs[i] = ctx->basis[i];
  TOPO_HIP(launch_combine(s, ctx->ndof, nb, vs, alpha, ctx->u));
  return TOPO_OK;
}

// ---------------------------------------------------------------------------
// Launch-shape autotuner: times every K.u launch shape (nodes per thread column
// x threads per block) on this context's grids and keeps the fastest, for the CG
// product on the finest level and for the smoothing passes on every level.
static topo_status time_ku_shapes(topo_ctx *ctx, const std::vector<int> &shapes,
                                  const std::function<hipError_t(int)> &launch, int *best) {
  hipStream_t s = ctx->stream;
  hipEvent_t e0, e1;
  TOPO_HIP(hipEventCreate(&e0));
  TOPO_HIP(hipEventCreate(&e1));
  float best_ms = 0.f;
  *best = -1;
  for (int shape : shapes) {
    TOPO_HIP(launch(shape));  // warm-up
    TOPO_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r) TOPO_HIP(launch(shape));
    TOPO_HIP(hipEventRecord(e1, s));
    TOPO_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    TOPO_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (*best < 0 || ms < best_ms) best_ms = ms, *best = shape;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return TOPO_OK;
}

template <typename T>
static topo_status tune_smoothing(topo_ctx *ctx, Level &L) {
  const LevelBufs<T> B = bufs<T>(L);
  const int64_t nd = L.g.ndof();
  hipStream_t s = ctx->stream;
  TOPO_HIP(hipMemsetAsync(B.E, 0, L.g.nel() * sizeof(T), s));
  for (T *v : {B.dinv, B.b, B.x, B.res, B.d0, B.d1}) TOPO_HIP(hipMemsetAsync(v, 0, nd * sizeof(T), s));
  KuArgsT<T> c = ku_args_t<T>(L, B.d0);
  c.res = B.res;
  c.x = B.x;
  c.dout = B.d1;
  c.c1 = (T)0.5;
  c.c2 = (T)0.5;
  const KappaT<T> &kap = kappa_of<T>(ctx);
  // single precision may also take the matrix-core kernel (same arithmetic up to rounding)
  return time_ku_shapes(ctx, ku_tunable_shapes(std::is_same<T, float>::value, ctx->opts.ku_kernel), [&](int shape) {
    return launch_ku(s, KU_CHEB, c, kap, ctx->red, fin_sum(nullptr), shape);
  }, &L.shape);
}

// Shapes found by the autotuner, per device and per tuning problem (grids of
// every level, operator precision, kernel family): later contexts with the same
// key take them without timing (autotune 1); autotune 2 times again and
// replaces the entry.  Any entry is a valid choice, as every shape computes the
// same products.
namespace {
struct TunedShapes {
  int shape_cg = -1;
  std::vector<int> level;
};
std::mutex g_tune_mu;
std::map<std::string, TunedShapes> g_tune_cache;
}  // namespace

static std::string tune_key(const topo_ctx *ctx) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::string k = std::to_string(dev) + "|" + std::to_string(ctx->opts.precision) + "|" +
                  std::to_string(ctx->mixed) + "|" + std::to_string(ctx->opts.ku_kernel) + "|" +
                  std::to_string(ctx->lv.size());
  for (const Level &L : ctx->lv)
    k += "|" + std::to_string(L.g.nx) + "x" + std::to_string(L.g.ny) + "x" + std::to_string(L.g.nz);
  return k;
}

static topo_status autotune_timed(topo_ctx *ctx);

static topo_status autotune(topo_ctx *ctx) {
  const std::string key = tune_key(ctx);
  if (ctx->opts.autotune == 1) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end() && it->second.level.size() == ctx->lv.size()) {
      ctx->shape_cg = it->second.shape_cg;
      for (size_t l = 0; l < ctx->lv.size(); ++l) ctx->lv[l].shape = it->second.level[l];
      return TOPO_OK;
    }
  }
  topo_status st = autotune_timed(ctx);
  if (st != TOPO_OK) return st;
  TunedShapes t;
  t.shape_cg = ctx->shape_cg;
  for (const Level &L : ctx->lv) t.level.push_back(L.shape);
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_cache[key] = t;
  return TOPO_OK;
}

extern "C" void topo_clear_tuning_cache(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_cache.clear();
}

static topo_status autotune_timed(topo_ctx *ctx) {
  hipStream_t s = ctx->stream;
  Level &L0 = ctx->lv[0];
  const int64_t nd = ctx->ndof;
  TOPO_HIP(hipMemsetAsync(L0.E, 0, ctx->nel * sizeof(double), s));
  TOPO_HIP(hipMemsetAsync(ctx->p, 0, nd * sizeof(double), s));
  KuArgs a = ku_args(ctx, L0, ctx->p);
  a.y = ctx->q;
  topo_status st = time_ku_shapes(ctx, ku_tunable_shapes(false, ctx->opts.ku_kernel), [&](int shape) {
    return launch_ku(s, KU_STORE_DOT, a, ctx->kap, ctx->red, fin_sum(&ctx->sc->red[0]), shape);
  }, &ctx->shape_cg);
  if (st != TOPO_OK) return st;
  if (ctx->lv.size() < 2) return TOPO_OK;  // Jacobi: no smoothing passes
  if (ctx->opts.precision == TOPO_PREC_BF16) return TOPO_OK;  // BF16 operands: one fixed kernel
  for (Level &L : ctx->lv) {
    st = ctx->mixed ? tune_smoothing<float>(ctx, L) : tune_smoothing<double>(ctx, L);
    if (st != TOPO_OK) return st;
  }
  return TOPO_OK;
}

// level-0 modulus from xphys, then the coarse moduli, diagonals and (unless the
// previous one is kept) the coarse inverse
// The context's stream waits for a coarse inverse still being built on the side stream.
static topo_status join_inverse(topo_ctx *ctx) {
  if (!ctx->inv_pending) return TOPO_OK;
  ctx->inv_pending = false;
  TOPO_HIP(hipStreamWaitEvent(ctx->stream, ctx->side_ev[1], 0));
  return TOPO_OK;
}

// The side stream of ctx (created on first use) set to start after everything
// enqueued on s so far; side_end marks the work enqueued on it since as the
// pending coarse inverse.
static topo_status side_begin(topo_ctx *ctx, hipStream_t s, hipStream_t *side) {
  if (!ctx->side) {
    TOPO_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    for (hipEvent_t &e : ctx->side_ev) TOPO_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  TOPO_HIP(hipEventRecord(ctx->side_ev[0], s));
  TOPO_HIP(hipStreamWaitEvent(ctx->side, ctx->side_ev[0], 0));
  *side = ctx->side;
  return TOPO_OK;
}
static topo_status side_end(topo_ctx *ctx) {
  TOPO_HIP(hipEventRecord(ctx->side_ev[1], ctx->side));
  ctx->inv_pending = true;
  return TOPO_OK;
}

// overlap_inverse: the coarse inverse goes to the side stream and is joined by
// join_inverse (pcg_run does so before its first V-cycle)
static topo_status prepare_operator(topo_ctx *ctx, const double *d_xphys, bool refresh_coarse = true,
                                    bool overlap_inverse = false) {
  hipStream_t s = ctx->stream;
  topo_status js = join_inverse(ctx);
  if (js != TOPO_OK) return js;
  const topo_problem &P = ctx->prob;
  // in mixed precision every kernel also writes the single-precision copy
  const bool m = ctx->mixed;
  TOPO_HIP(launch_simp_modulus(s, ctx->nel, d_xphys, P.E0, P.Emin, P.penal, 1.0, ctx->lv[0].E,
                               m ? ctx->lv[0].f32.E : nullptr));
  for (size_t l = 0; l < ctx->lv.size(); ++l) {
    Level &L = ctx->lv[l];
    if (l > 0) TOPO_HIP(launch_coarsen_moduli(s, ctx->lv[l - 1].g, L.g, ctx->lv[l - 1].E, L.E, m ? L.f32.E : nullptr));
    TOPO_HIP(launch_diag(s, L.g, L.E, ctx->kap, L.fixed, L.dinv, m ? L.f32.dinv : nullptr));
  }
  if (ctx->lv.size() > 1 && refresh_coarse) {
    const Level &C = ctx->lv.back();
    hipStream_t si = s;
    if (overlap_inverse) {
      // after the coarsest moduli (and everything before them on the stream)
      const topo_status ss = side_begin(ctx, s, &si);
      if (ss != TOPO_OK) return ss;
    }
    TOPO_HIP(launch_dense_assemble(si, C.g, C.E, ctx->kap, C.fixed, ctx->Ainv));
    TOPO_HIP(launch_dense_invert(si, ctx->ncoarse, ctx->Ainv, ctx->Awork));
    if (overlap_inverse) {
      const topo_status se = side_end(ctx);
      if (se != TOPO_OK) return se;
    }
  }
  // a direct call leaves a fresh inverse; the SIMP loop counts from here
  ctx->coarse_due = refresh_coarse ? ctx->opts.coarse_refresh : ctx->coarse_due;
  // network input channel 0 (node density) is fixed for the whole solve
  if (ctx->nn) TOPO_HIP(launch_node_density(s, ctx->g, d_xphys, ctx->nnw.x));
  return TOPO_OK;
}

// Chebyshev polynomial smoothing in D^-1 A on [lam_max / kChebRatio, lam_max].
struct Cheb {
  double theta, delta, sigma;
  explicit Cheb(double lam_max) {
    const double hi = lam_max, lo = hi / kChebRatio;
    theta = 0.5 * (hi + lo);
    delta = 0.5 * (hi - lo);
    sigma = theta / delta;
  }
};

// Chebyshev degree of level l: cheb_degree_level[l] when set, else cheb_degree
// on the finest and cheb_degree_coarse (when set) below it
static int level_degree(const topo_ctx *ctx, size_t l) {
  if (l < 8 && ctx->opts.cheb_degree_level[l] > 0) return ctx->opts.cheb_degree_level[l];
  return (l == 0 || ctx->opts.cheb_degree_coarse == 0) ? ctx->opts.cheb_degree : ctx->opts.cheb_degree_coarse;
}
static int level_degree(const topo_ctx *ctx, const Level &L) { return level_degree(ctx, (size_t)(&L - &ctx->lv[0])); }

// Pre-smoothing from x = 0 (cheb_degree steps); on exit x and res = b - A x.
// On small grids the first step's operand d0 = b dinv / theta is formed inside
// the operator pass.
template <typename T>
static topo_status pre_smooth(topo_ctx *ctx, Level &L, const int *skip) {
  hipStream_t s = ctx->stream;
  const int deg = level_degree(ctx, L);
  const Cheb ch(ctx->lam_max);
  const KappaT<T> &kap = kappa_of<T>(ctx);
  const LevelBufs<T> B = bufs<T>(L);
  double rho = 1.0 / ch.sigma;
  T *dcur = B.d0, *dnext = B.d1;
  KuArgsT<T> a = ku_args_t<T>(L, nullptr);
  a.b = B.b;
  a.res = B.res;
  a.x = B.x;
  a.s0 = (T)(1.0 / ch.theta);
  a.skip = skip;
  if (deg == 1) {
    if (&L == &ctx->lv[0] && ctx->chk_n) {
      a.chk_parts = ctx->chk_parts;
      a.chk_n = ctx->chk_n;
      a.chk_sc = ctx->sc;
      ctx->chk_n = 0;
    }
    TOPO_HIP(launch_ku(s, KU_RES0, a, kap, ctx->red, fin_sum(nullptr), L.shape));
    return TOPO_OK;
  }
  double rho_new = 1.0 / (2.0 * ch.sigma - rho);
  const bool element_kernel = L.shape >= kKuShapeHada && L.shape < kKuShapeHada + kKuShapesHada;
  if (L.g.nnodes() >= kFuseFirstStepBelow && !element_kernel) {
    // large grids, node-column kernel: the first direction gets its own pass
    TOPO_HIP(launch_cheb_first(s, L.g.ndof(), B.b, B.dinv, (T)(1.0 / ch.theta), dnext, B.x, B.res, skip));
    KuArgsT<T> c = ku_args_t<T>(L, dnext);
    c.res = B.res;
    c.x = B.x;
    c.dout = dcur;
    c.c1 = (T)(rho_new * rho);
    c.c2 = (T)(2.0 * rho_new / ch.delta);
    c.skip = skip;
    TOPO_HIP(launch_ku(s, KU_CHEB, c, kap, ctx->red, fin_sum(nullptr), L.shape));
  } else {
    a.dout = dcur;
    a.c1 = (T)(rho_new * rho);
    a.c2 = (T)(2.0 * rho_new / ch.delta);
    TOPO_HIP(launch_ku(s, KU_CHEB0, a, kap, ctx->red, fin_sum(nullptr), L.shape));
  }
  rho = rho_new;
  for (int k = 2; k < deg; ++k) {
    rho_new = 1.0 / (2.0 * ch.sigma - rho);
    KuArgsT<T> c = ku_args_t<T>(L, dcur);
    c.res = B.res;
    c.x = B.x;
    c.dout = dnext;
    c.c1 = (T)(rho_new * rho);
    c.c2 = (T)(2.0 * rho_new / ch.delta);
    c.skip = skip;
    TOPO_HIP(launch_ku(s, KU_CHEB, c, kap, ctx->red, fin_sum(nullptr), L.shape));
    std::swap(dcur, dnext);
    rho = rho_new;
  }
  KuArgsT<T> r = ku_args_t<T>(L, dcur);
  r.res = B.res;
  r.skip = skip;
  TOPO_HIP(launch_ku(s, KU_RESUPD, r, kap, ctx->red, fin_sum(nullptr), L.shape));
  return TOPO_OK;
}

// Where the finest level of a single-precision V-cycle hands its result to
// flexible CG: z (single precision, holding the previous z), r and the finalize.
struct FlexOut {
  float *z;
  const double *r;
  Fin fin;
  int *defer;  // when set, a pass that forms the dots leaves them as partials (their count here)
};

// Post-smoothing from the current x (cheb_degree steps).  With dot_with set,
// the last pass also reduces dot_with . x into fin; with flex set (single
// precision, finest level) the result goes to flex->z with the flexible-CG dot
// products, fused into the last update when the degree is 1.
template <typename T>
static topo_status post_smooth(topo_ctx *ctx, Level &L, const int *skip, const T *dot_with,
                               const Fin &fin, const FlexOut *flex = nullptr, int *defer_dot = nullptr) {
  hipStream_t s = ctx->stream;
  const int deg = level_degree(ctx, L);
  const Cheb ch(ctx->lam_max);
  const KappaT<T> &kap = kappa_of<T>(ctx);
  const LevelBufs<T> B = bufs<T>(L);
  double rho = 1.0 / ch.sigma;
  T *dcur = B.d0, *dnext = B.d1;
  KuArgsT<T> a = ku_args_t<T>(L, B.x);
  a.b = B.b;
  a.res = B.res;
  a.dout = dcur;
  a.s0 = (T)(1.0 / ch.theta);
  a.skip = skip;
  // degree 1 into flex_dot: it forms the direction from res itself
  bool fused_last = false;
  if constexpr (std::is_same<T, float>::value) {
    fused_last = deg == 1 && flex;
    if (fused_last && !ku_matrix_core_shape(L.shape)) {
      // ... or, with the vector kernels, the operator pass forms z and the
      // flexible-CG dot products itself (res is not needed afterwards)
      a.rflex = flex->r;
      a.zflex = flex->z;
      TOPO_HIP(launch_ku(s, KU_RESID_FLEX, a, kap, ctx->red, flex->fin, L.shape, flex->defer));
      return TOPO_OK;
    }
  }
  if (fused_last) a.dout = nullptr;
  TOPO_HIP(launch_ku(s, KU_RESID_START, a, kap, ctx->red, fin_sum(nullptr), L.shape));
  if (deg == 1) {
    if constexpr (std::is_same<T, float>::value) {
      if (flex) {
        TOPO_HIP(launch_flex_dot(s, L.g.ndof(), B.res, B.dinv, (T)(1.0 / ch.theta), B.x, flex->r, flex->z,
                                 ctx->red, flex->fin, skip));
        return TOPO_OK;
      }
    }
    if constexpr (std::is_same<T, double>::value) {
      if (dot_with && defer_dot) {
        // the last update and the dot product in one pass, its partials left
        // for the consumer (no finalize; the unused step is not stored)
        TOPO_HIP(launch_cheb_last_dot(s, L.g.ndof(), B.res, B.dinv, 1.0 / ch.theta, B.x, dot_with, ctx->red,
                                      defer_dot, skip));
        return TOPO_OK;
      }
    }
    TOPO_HIP(launch_cheb_start(s, L.g.ndof(), B.res, B.dinv, (T)(1.0 / ch.theta), dnext, B.x, skip));
    if (dot_with) {
      if constexpr (std::is_same<T, double>::value)
        TOPO_HIP(launch_dot(s, L.g.ndof(), dot_with, B.x, ctx->red, fin, skip));
    }
    return TOPO_OK;
  }
  for (int k = 1; k < deg; ++k) {
    const double rho_new = 1.0 / (2.0 * ch.sigma - rho);
    KuArgsT<T> c = ku_args_t<T>(L, dcur);
    c.res = B.res;
    c.x = B.x;
    c.dout = dnext;
    c.c1 = (T)(rho_new * rho);
    c.c2 = (T)(2.0 * rho_new / ch.delta);
    c.dot_with = (k == deg - 1) ? dot_with : nullptr;
    if (k == deg - 1) c.dout = nullptr;  // last step: only x is needed afterwards
    c.skip = skip;
    TOPO_HIP(launch_ku(s, k == 1 ? KU_CHEB_ADD : KU_CHEB, c, kap, ctx->red, fin, L.shape));
    std::swap(dcur, dnext);
    rho = rho_new;
  }
  if constexpr (std::is_same<T, float>::value) {
    if (flex)
      TOPO_HIP(launch_flex_dot(s, L.g.ndof(), nullptr, nullptr, 0.f, B.x, flex->r, flex->z, ctx->red, flex->fin,
                               skip));
  }
  return TOPO_OK;
}

// z = M r: V-cycle from level l with rhs b into x of that level; with dot_fin
// set (level 0 in double precision) the last smoothing pass reduces r.z into it
// levels tail_start .. coarsest in one launch (same arithmetic as the per-level passes)
template <typename T>
static topo_status vcycle_tail(topo_ctx *ctx, const int *skip) {
  TailArgs<T> a{};
  a.nlev = (int)(ctx->lv.size() - ctx->tail_start);
  for (int q = 0; q < a.nlev; ++q) {
    Level &L = ctx->lv[ctx->tail_start + q];
    const LevelBufs<T> B = bufs<T>(L);
    a.L[q] = TailLevel<T>{L.g, B.E, B.dinv, L.fixed, B.b, B.x, B.res, B.d0, B.d1,
                          level_degree(ctx, ctx->tail_start + q)};
  }
  a.Ainv = ctx->Ainv;
  a.ncoarse = ctx->ncoarse;
  a.hw = hada_work(kappa_of<T>(ctx));
  a.deg = 1;  // the most steps of any tail level (never the finest level): coefficients up to it
  for (int q = 0; q < a.nlev; ++q) a.deg = std::max(a.deg, a.L[q].deg);
  const Cheb ch(ctx->lam_max);
  a.s0 = (T)(1.0 / ch.theta);
  double rho = 1.0 / ch.sigma;
  for (int k = 1; k < a.deg && k < kTailMaxDeg; ++k) {
    const double rho_new = 1.0 / (2.0 * ch.sigma - rho);
    a.c1[k] = (T)(rho_new * rho);
    a.c2[k] = (T)(2.0 * rho_new / ch.delta);
    rho = rho_new;
  }
  a.skip = skip;
  TOPO_HIP(launch_vcycle_tail_t<T>(ctx->stream, a));
  return TOPO_OK;
}

template <typename T>
static topo_status vcycle(topo_ctx *ctx, size_t l, const int *skip, const Fin *dot_fin,
                          const FlexOut *flex = nullptr, int *defer_dot = nullptr) {
  hipStream_t s = ctx->stream;
  Level &L = ctx->lv[l];
  const LevelBufs<T> B = bufs<T>(L);
  if (l + 1 == ctx->lv.size()) {
    TOPO_HIP(launch_dense_matvec(s, ctx->ncoarse, ctx->Ainv, B.b, B.x, skip));
    return TOPO_OK;
  }
  if (ctx->tail_start && l == ctx->tail_start) return vcycle_tail<T>(ctx, skip);
  topo_status st = pre_smooth<T>(ctx, L, skip);
  if (st != TOPO_OK) return st;
  Level &C = ctx->lv[l + 1];
  const LevelBufs<T> BC = bufs<T>(C);
  if (l + 2 == ctx->lv.size()) {
    // the next level is the coarsest: restriction and dense solve in one launch
    TOPO_HIP(launch_restrict_solve<T>(s, L.g, C.g, B.res, C.fixed, ctx->ncoarse, ctx->Ainv, BC.x, skip));
  } else {
    TOPO_HIP(launch_restrict(s, L.g, C.g, B.res, C.fixed, BC.b, skip));
    st = vcycle<T>(ctx, l + 1, skip, nullptr);
    if (st != TOPO_OK) return st;
  }
  TOPO_HIP(launch_prolong_add(s, L.g, C.g, BC.x, L.fixed, B.x, skip));
  return post_smooth<T>(ctx, L, skip, dot_fin ? B.b : nullptr, dot_fin ? *dot_fin : fin_sum(nullptr), flex,
                        defer_dot);
}

// z = M r; the r.z finalize sets rz_new, beta = rz_new / rz and rz = rz_new.
// In mixed precision the whole V-cycle runs in single precision after a
// narrowing of r, and its result stays in single precision in ctx->z32 (CG
// widens it exactly where it reads it); its last pass forms r.z_new and r.z_old
// in double for the flexible update.
//
// The learned preconditioner (kind TOPO_PRECOND_LEARNED) maps the residual
// through the network (its rms comes from rr, formed by the caller) and feeds
// the flexible update with the safeguard test of FIN_RZ_SAFE.
static topo_status precondition(topo_ctx *ctx, int kind, const int *skip, bool have_r32 = false,
                                int *defer = nullptr) {
  hipStream_t s = ctx->stream;
  Level &L0 = ctx->lv[0];
  const Fin fin{FIN_RZ, &ctx->sc->rz_new, ctx->sc};
  if (kind == TOPO_PRECOND_LEARNED) {
    NnWork &w = ctx->nnw;
    const int64_t V = ctx->nnodes;
    TOPO_HIP(launch_nn_input_resid(s, V, ctx->r, &ctx->sc->rr, ctx->nn_scale, w.x + V, skip));
    topo_status st = nn_forward(ctx->nn, w, s, skip);
    if (st != TOPO_OK) return st;
    const Fin safe{FIN_RZ_SAFE, &ctx->sc->red[0], ctx->sc};
    TOPO_HIP(launch_nn_output_flex(s, V, w.out, ctx->nn_scale, L0.fixed, ctx->r, ctx->z, ctx->red, safe, skip));
    return TOPO_OK;
  }
  if (kind == TOPO_PRECOND_JACOBI || ctx->lv.size() == 1) {
    TOPO_HIP(launch_jacobi(s, ctx->ndof, ctx->r, L0.dinv, ctx->z, ctx->red, fin, skip));
    return TOPO_OK;
  }
  if (!ctx->mixed) return vcycle<double>(ctx, 0, skip, &fin, nullptr, defer);
  if (!have_r32) TOPO_HIP(launch_convert(s, ctx->ndof, ctx->r, L0.f32.b, skip));
  const FlexOut flex{ctx->z32, ctx->r, Fin{FIN_RZ_FLEX, &ctx->sc->red[0], ctx->sc}, defer};
  return vcycle<float>(ctx, 0, skip, nullptr, &flex);
}

// whether the preconditioner of this kind leaves z in ctx->z32 (else ctx->z)
static bool z_single(const topo_ctx *ctx, int kind) {
  return ctx->mixed && kind == TOPO_PRECOND_MG && ctx->lv.size() > 1;
}

static hipError_t update_p(topo_ctx *ctx, int kind, int first, const int *skip) {
  return z_single(ctx, kind) ? launch_cg_update_p(ctx->stream, ctx->ndof, ctx->sc, ctx->z32, ctx->p, first, skip)
                             : launch_cg_update_p(ctx->stream, ctx->ndof, ctx->sc, ctx->z, ctx->p, first, skip);
}

static topo_status read_scalars(topo_ctx *ctx) {
  TOPO_HIP(hipMemcpyAsync(ctx->h_sc, ctx->sc, sizeof(Scalars), hipMemcpyDeviceToHost, ctx->stream));
  TOPO_HIP(hipStreamSynchronize(ctx->stream));
  return TOPO_OK;
}

// One CG iteration on ctx->u; after convergence (sc->cg_done) every kernel
// returns immediately, so chunks of iterations can be enqueued (or replayed
// from a graph) without a host round trip per iteration.
static topo_status cg_body(topo_ctx *ctx, int kind) {
  hipStream_t s = ctx->stream;
  const int *skip = &ctx->sc->cg_done;
  Level &L0 = ctx->lv[0];
  KuArgs a = ku_args(ctx, L0, ctx->p);
  a.y = ctx->q;
  a.skip = skip;
  // p.q stays as block partials, summed by every block of the update (no
  // finalize launch between the two)
  int npq = 0;
  TOPO_HIP(launch_ku(s, KU_STORE_DOT, a, ctx->kap, ctx->red, fin_sum(&ctx->sc->pq), ctx->shape_cg, &npq));
  const Fin check{FIN_CG_CHECK, &ctx->sc->rr, ctx->sc};
  // a single-precision multigrid preconditioner takes the residual in FP32, written
  // by the same pass
  float *r32 = z_single(ctx, kind) ? L0.f32.b : nullptr;
  // where the V-cycle starts with a RES0 pass on a 256-thread element-column
  // shape, that pass takes the stopping test on the r.r partials itself (no
  // finalize launch); cg_iters is counted by the update then
  const bool stop_in_pass = kind == TOPO_PRECOND_MG && ctx->lv.size() > 1 && level_degree(ctx, 0) == 1 &&
                            L0.shape >= kKuShapeHada &&
                            L0.shape < kKuShapeHada + kKuShapesHada &&
                            ku_hada_block_threads(L0.shape - kKuShapeHada) == 256;
  int nrr = 0;
  TOPO_HIP(launch_cg_update_xr_pq(s, ctx->ndof, ctx->sc, ctx->u, ctx->r, ctx->p, ctx->q, ctx->red, npq, check, skip,
                                  r32, stop_in_pass ? &nrr : nullptr));
  if (stop_in_pass) {
    ctx->chk_parts = ctx->red.partials + 1;
    ctx->chk_n = nrr;
  }
  // r.z (or the flexible pair of a single-precision V-cycle) stays as partials
  // where the V-cycle's last pass forms it, summed by every block of the p update
  int nrz = 0;
  topo_status st = precondition(ctx, kind, skip, r32 != nullptr, kind == TOPO_PRECOND_MG ? &nrz : nullptr);
  if (ctx->chk_n) {
    ctx->chk_n = 0;
    return set_error("internal: the CG stopping test was not taken by the first V-cycle pass"), TOPO_EINVAL;
  }
  if (st != TOPO_OK) return st;
  if (nrz > 0 && z_single(ctx, kind))
    TOPO_HIP(launch_cg_update_p_flex(s, ctx->ndof, ctx->sc, ctx->z32, ctx->p, ctx->red, nrz, skip));
  else if (nrz > 0)
    TOPO_HIP(launch_cg_update_p_rz(s, ctx->ndof, ctx->sc, ctx->z, ctx->p, ctx->red, nrz, skip));
  else
    TOPO_HIP(update_p(ctx, kind, 0, skip));
  return TOPO_OK;
}

// Enqueues one chunk of check_every CG iterations: the captured graph when graphs
// are on (captured on first use; every pointer it holds is owned by the context),
// direct launches otherwise.
static topo_status cg_chunk(topo_ctx *ctx, int kind) {
  const int chunk = std::max(1, ctx->opts.check_every);
  if (!ctx->opts.use_graphs) {
    for (int c = 0; c < chunk; ++c) {
      topo_status st = cg_body(ctx, kind);
      if (st != TOPO_OK) return st;
    }
    return TOPO_OK;
  }
  if (kind == TOPO_PRECOND_LEARNED && ctx->cg_exec[kind] && ctx->nn_graph_precision != ctx->nn->precision) {
    (void)hipGraphExecDestroy(ctx->cg_exec[kind]);
    (void)hipGraphDestroy(ctx->cg_graph[kind]);
    ctx->cg_exec[kind] = nullptr;
    ctx->cg_graph[kind] = nullptr;
  }
  if (!ctx->cg_exec[kind]) {
    if (kind == TOPO_PRECOND_LEARNED) ctx->nn_graph_precision = ctx->nn->precision;
    hipStream_t user = ctx->stream;
    ctx->stream = ctx->cap_stream;
    TOPO_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
    topo_status st = TOPO_OK;
    for (int c = 0; c < chunk && st == TOPO_OK; ++c) st = cg_body(ctx, kind);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &graph);
    ctx->stream = user;
    if (st != TOPO_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    TOPO_HIP(ce);
    ctx->cg_graph[kind] = graph;
    TOPO_HIP(hipGraphInstantiate(&ctx->cg_exec[kind], graph, nullptr, nullptr, 0));
  }
  TOPO_HIP(hipGraphLaunch(ctx->cg_exec[kind], ctx->stream));
  return TOPO_OK;
}

// How many chunks to enqueue before the next host check of the convergence
// flag.  Each check is a round trip (copy, synchronize, next launch) that leaves
// the device idle; chunks enqueued past convergence only cost their launches,
// since every kernel in them returns at once.  From the mean rate at which r.r
// has fallen since the solve started, the chunks expected to stay short of the
// tolerance (three quarters of the estimate) go in together; before any
// iteration, three fifths of the previous solve's iterations with this
// preconditioner; without either, one chunk.  Never more chunks than the
// iteration cap leaves room for.
static int chunks_ahead(const topo_ctx *ctx, int kind, int max_iters) {
  const int chunk = std::max(1, ctx->opts.check_every);
  const Scalars &h = *ctx->h_sc;
  const int it = h.cg_iters;
  const double rr = h.rr, rr0 = h.rr_start, goal = h.rtol2 * h.ff;
  const int room = std::max(1, (max_iters - it + chunk - 1) / chunk);
  int n = 1;
  if (it == 0) {
    n = 3 * ctx->cg_prev_iters[kind] / (5 * chunk);
  } else if (rr0 > 0.0 && rr > 0.0 && rr < rr0 && goal < rr && std::isfinite(rr0)) {
    const double per_iter = std::log(rr / rr0) / it;     // < 0
    const double rest = std::log(goal / rr) / per_iter;  // iterations still needed at that rate
    n = (int)(0.75 * rest / chunk);
  }
  return std::max(1, std::min(std::min(n, room), 64));
}

// One run of (flexible) PCG with preconditioner `kind` and iteration cap
// max_iters, from ctx->u; the scalars end in ctx->h_sc.
static topo_status pcg_run(topo_ctx *ctx, int kind, int max_iters) {
  hipStream_t s = ctx->stream;
  Level &L0 = ctx->lv[0];
  const int64_t n = ctx->ndof;
  TOPO_HIP(launch_zero_fixed(s, ctx->nnodes, L0.fixed, ctx->u));
  // r = f - K u, rr
  {
    KuArgs a = ku_args(ctx, L0, ctx->u);
    a.y = ctx->r;
    a.b = ctx->f;
    TOPO_HIP(launch_ku(s, KU_RESID, a, ctx->kap, ctx->red, fin_sum(&ctx->sc->rr)));
  }
  TOPO_HIP(launch_dot(s, n, ctx->f, ctx->f, ctx->red, fin_sum(&ctx->sc->ff)));
  const double rtol = ctx->opts.rtol;
  // iteration count 0; done at once if the initial guess already meets the tolerance
  TOPO_HIP(launch_cg_start(s, ctx->sc, rtol * rtol, max_iters));
  // the flexible update reads the previous z: start it from zero
  if (z_single(ctx, kind)) TOPO_HIP(hipMemsetAsync(ctx->z32, 0, n * sizeof(float), s));
  else if (kind == TOPO_PRECOND_LEARNED || ctx->mixed) TOPO_HIP(hipMemsetAsync(ctx->z, 0, n * sizeof(double), s));
  // first direction (skipped on the device when already converged)
  // the coarse inverse of this SIMP iteration may still be in the making
  topo_status st = join_inverse(ctx);
  if (st != TOPO_OK) return st;
  st = precondition(ctx, kind, &ctx->sc->cg_done);
  if (st != TOPO_OK) return st;
  TOPO_HIP(update_p(ctx, kind, 1, &ctx->sc->cg_done));
  // with the previous solve's count as a guide the first chunks go in at once
  // (on an already converged start they return at once); otherwise the state
  // is read first
  const int chunk = std::max(1, ctx->opts.check_every);
  int ahead = std::min(3 * ctx->cg_prev_iters[kind] / (5 * chunk), std::min(64, (max_iters + chunk - 1) / chunk));
  if (ahead < 1) {
    st = read_scalars(ctx);
    if (st != TOPO_OK) return st;
  }
  for (;;) {
    if (ahead < 1) {
      if (ctx->h_sc->cg_done) break;
      ahead = chunks_ahead(ctx, kind, max_iters);
    }
    for (int c = 0; c < ahead; ++c) {
      st = cg_chunk(ctx, kind);
      if (st != TOPO_OK) return st;
    }
    ahead = 0;
    st = read_scalars(ctx);
    if (st != TOPO_OK) return st;
  }
  ctx->cg_prev_iters[kind] = ctx->h_sc->cg_iters;
  return TOPO_OK;
}

// PCG on the operator prepared by prepare_operator; solution in/out ctx->u.
// With the learned preconditioner, a failed safeguard test or nn_max_iters
// iterations without convergence restart the solve from the current iterate
// with the multigrid (or Jacobi) preconditioner.
static topo_status pcg(topo_ctx *ctx, topo_solve_stats *stats) {
  const int base = ctx->lv.size() > 1 ? TOPO_PRECOND_MG : TOPO_PRECOND_JACOBI;
  int kind = ctx->opts.precond == TOPO_PRECOND_JACOBI ? TOPO_PRECOND_JACOBI : base;
  int fallbacks = 0, learned = 0, total = 0;
  const int cap = ctx->opts.max_iters;
  topo_status st;
  if (ctx->opts.precond == TOPO_PRECOND_LEARNED) {
    if (!ctx->nn) return set_error("TOPO_PRECOND_LEARNED needs a network (topo_set_nn)"), TOPO_EINVAL;
    st = pcg_run(ctx, TOPO_PRECOND_LEARNED, std::min(cap, ctx->opts.nn_max_iters));
    if (st != TOPO_OK) return st;
    learned = total = ctx->h_sc->cg_iters;
    const bool ok = !ctx->h_sc->nn_fallback && std::isfinite(ctx->h_sc->rr) &&
                    ctx->h_sc->rr <= ctx->opts.rtol * ctx->opts.rtol * ctx->h_sc->ff;
    if (ok) kind = -1;
    else ++fallbacks;
  }
  if (kind >= 0) {
    st = pcg_run(ctx, kind, std::max(1, cap - total));
    if (st != TOPO_OK) return st;
    total += ctx->h_sc->cg_iters;
  }
  const double ff = ctx->h_sc->ff;
  const double rtol = ctx->opts.rtol;
  const double relres = std::sqrt(ctx->h_sc->rr / ff);
  if (stats) {
    stats->iters = total;
    stats->relres = relres;
    stats->converged = relres <= rtol;
    stats->fallbacks = fallbacks;
    stats->learned_iters = learned;
  }
  if (!std::isfinite(relres)) return set_error("CG diverged (non-finite residual)"), TOPO_ENOTCONVERGED;
  if (relres > rtol)
    return set_error("CG reached max_iters=%d with relres %.3e", ctx->opts.max_iters, relres), TOPO_ENOTCONVERGED;
  return TOPO_OK;
}

// ---------------------------------------------------------------------------
// Grouped CG: the contexts of a group (at most kMaxGroup, built with the same
// options on grids of the same size, so their hierarchies, launch shapes and
// smoother polynomials coincide) share one stream, and every pass of their CG
// iterations -- the operator product, the vector updates, every smoothing
// pass, transfer and coarse solve of the V-cycle, every finalize -- is one
// launch for all of them.  Each problem's blocks compute exactly what its own
// launch computes (same partials, same order), so the results are
// bit-identical to solving each problem alone; a converged problem's blocks
// return at once (its cg_done flag).
namespace topo {

// whether a context can take part in grouped CG, and the key that must match
std::string group_key(const topo_ctx *ctx) {
  const topo_opts &o = ctx->opts;
  if (o.precond != TOPO_PRECOND_MG || ctx->lv.size() < 2 || ctx->tail_start != 0) return "";
  if (o.precision == TOPO_PREC_BF16 || o.mfma_smoothing) return "";
  const bool is_hada = [&] {
    auto el = [](int sh) { return sh >= kKuShapeHada && sh < kKuShapeHada + kKuShapesHada; };
    if (!el(ctx->shape_cg)) return false;
    for (const Level &L : ctx->lv)
      if (!el(L.shape)) return false;
    return true;
  }();
  if (!is_hada) return "";
  std::string k = std::to_string(ctx->prob.nu) + "|" + std::to_string(ctx->mixed) + "|" + std::to_string(ctx->shape_cg) +
                  "|" + std::to_string(ctx->lam_max);
  for (size_t l = 0; l < ctx->lv.size(); ++l) {
    const Level &L = ctx->lv[l];
    k += "|" + std::to_string(L.g.nx) + "x" + std::to_string(L.g.ny) + "x" + std::to_string(L.g.nz) + "s" +
         std::to_string(L.shape) + "d" + std::to_string(level_degree(ctx, l));
  }
  return k;
}

// the launch shapes of src (same grids) for dst: every shape computes the same
// products, so this changes at most the rounding of reductions
void group_adopt_shapes(topo_ctx *dst, const topo_ctx *src) {
  if (dst->lv.size() != src->lv.size()) return;
  dst->shape_cg = src->shape_cg;
  for (size_t l = 0; l < dst->lv.size(); ++l) dst->lv[l].shape = src->lv[l].shape;
}
void ctx_set_stream(topo_ctx *ctx, hipStream_t s) { ctx->stream = s; }
Grid ctx_grid(const topo_ctx *ctx) { return ctx->g; }

static std::vector<Reducer> group_reds(const Group &G) {
  std::vector<Reducer> r;
  for (topo_ctx *c : G.c) r.push_back(c->red);
  return r;
}

template <typename T>
static topo_status group_pre_smooth(const Group &G, size_t l) {
  const int n = G.n();
  topo_ctx *c0 = G.c[0];
  const int deg = level_degree(c0, l);
  const Cheb ch(c0->lam_max);
  const KappaT<T> &kap = kappa_of<T>(c0);
  const std::vector<Reducer> red = group_reds(G);
  const std::vector<Fin> fin(n, fin_sum(nullptr));
  const int shape = c0->lv[l].shape;
  std::vector<KuArgsT<T>> a(n);
  std::vector<T *> dcur(n), dnext(n);
  for (int i = 0; i < n; ++i) {
    Level &L = G.c[i]->lv[l];
    const LevelBufs<T> B = bufs<T>(L);
    dcur[i] = B.d0;
    dnext[i] = B.d1;
    a[i] = ku_args_t<T>(L, nullptr);
    a[i].b = B.b;
    a[i].res = B.res;
    a[i].x = B.x;
    a[i].s0 = (T)(1.0 / ch.theta);
    a[i].skip = &G.c[i]->sc->cg_done;
  }
  if (deg == 1) {
    TOPO_HIP(launch_ku_group<T>(G.s, KU_RES0, n, a.data(), kap, red.data(), fin.data(), shape));
    return TOPO_OK;
  }
  double rho = 1.0 / ch.sigma;
  double rho_new = 1.0 / (2.0 * ch.sigma - rho);
  for (int i = 0; i < n; ++i) {
    a[i].dout = dcur[i];
    a[i].c1 = (T)(rho_new * rho);
    a[i].c2 = (T)(2.0 * rho_new / ch.delta);
  }
  TOPO_HIP(launch_ku_group<T>(G.s, KU_CHEB0, n, a.data(), kap, red.data(), fin.data(), shape));
  rho = rho_new;
  for (int k = 2; k < deg; ++k) {
    rho_new = 1.0 / (2.0 * ch.sigma - rho);
    for (int i = 0; i < n; ++i) {
      Level &L = G.c[i]->lv[l];
      const LevelBufs<T> B = bufs<T>(L);
      KuArgsT<T> c = ku_args_t<T>(L, dcur[i]);
      c.res = B.res;
      c.x = B.x;
      c.dout = dnext[i];
      c.c1 = (T)(rho_new * rho);
      c.c2 = (T)(2.0 * rho_new / ch.delta);
      c.skip = &G.c[i]->sc->cg_done;
      a[i] = c;
      std::swap(dcur[i], dnext[i]);
    }
    TOPO_HIP(launch_ku_group<T>(G.s, KU_CHEB, n, a.data(), kap, red.data(), fin.data(), shape));
    rho = rho_new;
  }
  for (int i = 0; i < n; ++i) {
    Level &L = G.c[i]->lv[l];
    KuArgsT<T> r = ku_args_t<T>(L, dcur[i]);
    r.res = bufs<T>(L).res;
    r.skip = &G.c[i]->sc->cg_done;
    a[i] = r;
  }
  TOPO_HIP(launch_ku_group<T>(G.s, KU_RESUPD, n, a.data(), kap, red.data(), fin.data(), shape));
  return TOPO_OK;
}

// post-smoothing; on the finest level the result goes to CG: in single
// precision through flex_dot into z32 (flexible update), in double with the
// r.z reduction of the last pass (FIN_RZ)
template <typename T>
static topo_status group_post_smooth(const Group &G, size_t l, bool finest, int *defer = nullptr) {
  const int n = G.n();
  topo_ctx *c0 = G.c[0];
  const int deg = level_degree(c0, l);
  const Cheb ch(c0->lam_max);
  const KappaT<T> &kap = kappa_of<T>(c0);
  const std::vector<Reducer> red = group_reds(G);
  constexpr bool single = std::is_same<T, float>::value;
  std::vector<Fin> fin(n, fin_sum(nullptr));
  if (finest && !single)
    for (int i = 0; i < n; ++i) fin[i] = Fin{FIN_RZ, &G.c[i]->sc->rz_new, G.c[i]->sc};
  std::vector<Fin> flexfin(n);
  for (int i = 0; i < n; ++i) flexfin[i] = Fin{FIN_RZ_FLEX, &G.c[i]->sc->red[0], G.c[i]->sc};
  const int shape = c0->lv[l].shape;
  std::vector<KuArgsT<T>> a(n);
  std::vector<T *> dcur(n), dnext(n);
  const bool fused_last = single && deg == 1 && finest;
  for (int i = 0; i < n; ++i) {
    Level &L = G.c[i]->lv[l];
    const LevelBufs<T> B = bufs<T>(L);
    dcur[i] = B.d0;
    dnext[i] = B.d1;
    a[i] = ku_args_t<T>(L, B.x);
    a[i].b = B.b;
    a[i].res = B.res;
    a[i].dout = fused_last ? nullptr : dcur[i];
    a[i].s0 = (T)(1.0 / ch.theta);
    a[i].skip = &G.c[i]->sc->cg_done;
  }
  if constexpr (single) {
    if (fused_last) {  // the operator pass forms z and the flexible-CG dots (post_smooth)
      for (int i = 0; i < n; ++i) {
        a[i].rflex = G.c[i]->r;
        a[i].zflex = G.c[i]->z32;
      }
      TOPO_HIP(launch_ku_group<T>(G.s, KU_RESID_FLEX, n, a.data(), kap, red.data(), flexfin.data(), shape, defer));
      return TOPO_OK;
    }
  }
  TOPO_HIP(launch_ku_group<T>(G.s, KU_RESID_START, n, a.data(), kap, red.data(), fin.data(), shape));
  const int64_t nd = c0->lv[l].g.ndof();
  if (deg == 1) {
    if constexpr (single) {
      if (finest) {
        std::vector<FlexArgs> f(n);
        for (int i = 0; i < n; ++i) {
          const LevelBufs<float> B = bufs<float>(G.c[i]->lv[l]);
          f[i] = FlexArgs{B.res, B.dinv, B.x, G.c[i]->r, G.c[i]->z32, &G.c[i]->sc->cg_done};
        }
        TOPO_HIP(launch_flex_dot_group(G.s, n, nd, (float)(1.0 / ch.theta), f.data(), red.data(), flexfin.data()));
        return TOPO_OK;
      }
    }
    std::vector<ChebStartArgs<T>> cs(n);
    for (int i = 0; i < n; ++i) {
      const LevelBufs<T> B = bufs<T>(G.c[i]->lv[l]);
      cs[i] = ChebStartArgs<T>{B.res, B.dinv, dnext[i], B.x, &G.c[i]->sc->cg_done};
    }
    TOPO_HIP(launch_cheb_start_group<T>(G.s, n, nd, (T)(1.0 / ch.theta), cs.data()));
    if constexpr (!single) {
      if (finest) {
        std::vector<DotArgs> d(n);
        for (int i = 0; i < n; ++i)
          d[i] = DotArgs{G.c[i]->lv[l].b, G.c[i]->lv[l].x, &G.c[i]->sc->cg_done};
        TOPO_HIP(launch_dot_group(G.s, n, nd, d.data(), red.data(), fin.data()));
      }
    }
    return TOPO_OK;
  }
  double rho = 1.0 / ch.sigma;
  for (int k = 1; k < deg; ++k) {
    const double rho_new = 1.0 / (2.0 * ch.sigma - rho);
    for (int i = 0; i < n; ++i) {
      Level &L = G.c[i]->lv[l];
      const LevelBufs<T> B = bufs<T>(L);
      KuArgsT<T> c = ku_args_t<T>(L, dcur[i]);
      c.res = B.res;
      c.x = B.x;
      c.dout = dnext[i];
      c.c1 = (T)(rho_new * rho);
      c.c2 = (T)(2.0 * rho_new / ch.delta);
      c.dot_with = (k == deg - 1 && finest && !single) ? (const T *)B.b : nullptr;
      if (k == deg - 1) c.dout = nullptr;
      c.skip = &G.c[i]->sc->cg_done;
      a[i] = c;
      std::swap(dcur[i], dnext[i]);
    }
    TOPO_HIP(launch_ku_group<T>(G.s, k == 1 ? KU_CHEB_ADD : KU_CHEB, n, a.data(), kap, red.data(), fin.data(),
                                shape));
    rho = rho_new;
  }
  if constexpr (single) {
    if (finest) {
      std::vector<FlexArgs> f(n);
      for (int i = 0; i < n; ++i) {
        const LevelBufs<float> B = bufs<float>(G.c[i]->lv[l]);
        f[i] = FlexArgs{nullptr, nullptr, B.x, G.c[i]->r, G.c[i]->z32, &G.c[i]->sc->cg_done};
      }
      TOPO_HIP(launch_flex_dot_group(G.s, n, nd, 0.f, f.data(), red.data(), flexfin.data()));
    }
  }
  return TOPO_OK;
}

// defer: where the finest level's last pass forms the flexible-CG dots, they
// stay as partials (their count there) for the grouped p update
template <typename T>
static topo_status group_vcycle(const Group &G, size_t l, int *defer = nullptr) {
  const int n = G.n();
  topo_ctx *c0 = G.c[0];
  if (l + 1 == c0->lv.size()) {
    std::vector<MatvecArgs<T>> m(n);
    for (int i = 0; i < n; ++i) {
      const LevelBufs<T> B = bufs<T>(G.c[i]->lv[l]);
      m[i] = MatvecArgs<T>{G.c[i]->Ainv, B.b, B.x, &G.c[i]->sc->cg_done};
    }
    TOPO_HIP(launch_dense_matvec_group<T>(G.s, n, c0->ncoarse, m.data()));
    return TOPO_OK;
  }
  topo_status st = group_pre_smooth<T>(G, l);
  if (st != TOPO_OK) return st;
  std::vector<TransferArgs<T>> t(n);
  if (l + 2 == c0->lv.size()) {
    // the next level is the coarsest: restriction and dense solve in one launch
    std::vector<RestrictSolveArgs<T>> r(n);
    for (int i = 0; i < n; ++i) {
      Level &L = G.c[i]->lv[l], &C = G.c[i]->lv[l + 1];
      r[i] = RestrictSolveArgs<T>{bufs<T>(L).res, C.fixed, G.c[i]->Ainv, bufs<T>(C).x, &G.c[i]->sc->cg_done};
    }
    TOPO_HIP(launch_restrict_solve_group<T>(G.s, n, c0->lv[l].g, c0->lv[l + 1].g, c0->ncoarse, r.data()));
  } else {
    for (int i = 0; i < n; ++i) {
      Level &L = G.c[i]->lv[l], &C = G.c[i]->lv[l + 1];
      t[i] = TransferArgs<T>{bufs<T>(L).res, C.fixed, bufs<T>(C).b, &G.c[i]->sc->cg_done};
    }
    TOPO_HIP(launch_restrict_group<T>(G.s, n, c0->lv[l].g, c0->lv[l + 1].g, t.data()));
    st = group_vcycle<T>(G, l + 1);
    if (st != TOPO_OK) return st;
  }
  for (int i = 0; i < n; ++i) {
    Level &L = G.c[i]->lv[l], &C = G.c[i]->lv[l + 1];
    t[i] = TransferArgs<T>{bufs<T>(C).x, L.fixed, bufs<T>(L).x, &G.c[i]->sc->cg_done};
  }
  TOPO_HIP(launch_prolong_add_group<T>(G.s, n, c0->lv[l].g, c0->lv[l + 1].g, t.data()));
  return group_post_smooth<T>(G, l, l == 0, l == 0 ? defer : nullptr);
}

static topo_status group_update_p(const Group &G, int first) {
  const int n = G.n();
  const bool zs = G.c[0]->mixed;
  std::vector<PArgs> a(n);
  for (int i = 0; i < n; ++i)
    a[i] = PArgs{G.c[i]->sc, zs ? (const void *)G.c[i]->z32 : (const void *)G.c[i]->z, G.c[i]->p,
                 &G.c[i]->sc->cg_done};
  TOPO_HIP(launch_cg_update_p_group(G.s, n, G.c[0]->ndof, zs, a.data(), first));
  return TOPO_OK;
}

static topo_status group_precondition(const Group &G) {
  return G.c[0]->mixed ? group_vcycle<float>(G, 0) : group_vcycle<double>(G, 0);
}

// one CG iteration of every problem of the group (the multigrid preconditioner)
static topo_status group_cg_body(const Group &G) {
  const int n = G.n();
  topo_ctx *c0 = G.c[0];
  const std::vector<Reducer> red = group_reds(G);
  std::vector<KuArgs> a(n);
  std::vector<Fin> fpq(n), fchk(n);
  std::vector<XrArgs> xr(n);
  for (int i = 0; i < n; ++i) {
    topo_ctx *c = G.c[i];
    a[i] = ku_args(c, c->lv[0], c->p);
    a[i].y = c->q;
    a[i].skip = &c->sc->cg_done;
    fpq[i] = fin_sum(&c->sc->pq);
    fchk[i] = Fin{FIN_CG_CHECK, &c->sc->rr, c->sc};
    xr[i] = XrArgs{c->sc, c->u, c->r, c->p, c->q, c->mixed ? c->lv[0].f32.b : nullptr, &c->sc->cg_done};
  }
  // p.q summed by every block of the update, and in mixed precision the
  // flexible dots by every block of the p update (as cg_body does)
  int npq = 0;
  TOPO_HIP(launch_ku_group<double>(G.s, KU_STORE_DOT, n, a.data(), c0->kap, red.data(), fpq.data(), c0->shape_cg,
                                   &npq));
  TOPO_HIP(launch_cg_update_xr_group_pq(G.s, n, c0->ndof, xr.data(), red.data(), npq, fchk.data()));
  if (!c0->mixed) {
    topo_status st = group_vcycle<double>(G, 0);
    if (st != TOPO_OK) return st;
    return group_update_p(G, 0);
  }
  int nrz = 0;
  topo_status st = group_vcycle<float>(G, 0, &nrz);
  if (st != TOPO_OK) return st;
  if (nrz < 1) return group_update_p(G, 0);
  std::vector<PArgs> pa(n);
  for (int i = 0; i < n; ++i) pa[i] = PArgs{G.c[i]->sc, G.c[i]->z32, G.c[i]->p, &G.c[i]->sc->cg_done};
  TOPO_HIP(launch_cg_update_p_flex_group(G.s, n, c0->ndof, pa.data(), red.data(), nrz));
  return TOPO_OK;
}

// the scalars of every problem of the group into their pinned mirrors, one wait
static topo_status group_read_scalars(const Group &G) {
  for (topo_ctx *c : G.c)
    TOPO_HIP(hipMemcpyAsync(c->h_sc, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, G.s));
  TOPO_HIP(hipStreamSynchronize(G.s));
  return TOPO_OK;
}

// Multigrid-preconditioned (flexible in mixed precision) CG of every problem
// of the group from its own u, to its own tolerance: the per-problem set-up,
// then grouped chunks of check_every iterations (captured once as a graph when
// the contexts use graphs) until every problem has converged.
topo_status group_pcg(Group &G, hipGraph_t *graph_out, hipGraphExec_t *exec, hipStream_t cap_stream,
                      topo_solve_stats *stats) {
  const int n = G.n();
  for (topo_ctx *c : G.c)
    if (c->stream != G.s) return set_error("grouped CG: the contexts must use the group's stream"), TOPO_EINVAL;
  // coarse inverses that iterate_pre left on the members' side streams
  for (topo_ctx *c : G.c) {
    const topo_status js = join_inverse(c);
    if (js != TOPO_OK) return js;
  }
  // r = f - K u, rr, ff and the stopping test of every member (the launches of
  // pcg_run's start, shared by the group)
  {
    topo_ctx *c0 = G.c[0];
    const int64_t nd = c0->ndof;
    const std::vector<Reducer> red = group_reds(G);
    std::vector<const uint8_t *> fx(n);
    std::vector<double *> uu(n);
    std::vector<KuArgs> a(n);
    std::vector<Fin> frr(n), fff(n);
    std::vector<DotArgs> ff(n);
    std::vector<CgStartArgs> cs(n);
    for (int i = 0; i < n; ++i) {
      topo_ctx *c = G.c[i];
      fx[i] = c->lv[0].fixed;
      uu[i] = c->u;
      a[i] = ku_args(c, c->lv[0], c->u);
      a[i].y = c->r;
      a[i].b = c->f;
      frr[i] = fin_sum(&c->sc->rr);
      fff[i] = fin_sum(&c->sc->ff);
      ff[i] = DotArgs{c->f, c->f, nullptr};
      cs[i] = CgStartArgs{c->sc, c->opts.rtol * c->opts.rtol, c->opts.max_iters};
    }
    TOPO_HIP(launch_zero_fixed_group(G.s, n, c0->nnodes, fx.data(), uu.data()));
    TOPO_HIP(launch_ku_group<double>(G.s, KU_RESID, n, a.data(), c0->kap, red.data(), frr.data(),
                                     ku_shape_for(c0->g, KU_RESID, TOPO_KU_AUTO, false)));
    TOPO_HIP(launch_dot_group(G.s, n, nd, ff.data(), red.data(), fff.data()));
    TOPO_HIP(launch_cg_start_group(G.s, n, cs.data()));
    if (c0->mixed) {
      std::vector<void *> z(n);
      std::vector<ConvertArgs> cv(n);
      for (int i = 0; i < n; ++i) {
        z[i] = G.c[i]->z32;
        cv[i] = ConvertArgs{G.c[i]->r, G.c[i]->lv[0].f32.b, &G.c[i]->sc->cg_done};
      }
      TOPO_HIP(launch_copy_group(G.s, n, nd * (int64_t)sizeof(float), nullptr, z.data()));
      TOPO_HIP(launch_convert_group(G.s, n, nd, cv.data()));
    }
  }
  topo_status st = group_precondition(G);
  if (st != TOPO_OK) return st;
  st = group_update_p(G, 1);
  if (st != TOPO_OK) return st;
  const int chunk = std::max(1, G.c[0]->opts.check_every);
  const bool graphs = G.c[0]->opts.use_graphs && graph_out != nullptr && exec != nullptr && cap_stream != nullptr;
  if (graphs && !*exec) {
    Group cap = G;
    cap.s = cap_stream;
    TOPO_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed));
    for (int k = 0; k < chunk && st == TOPO_OK; ++k) st = group_cg_body(cap);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(cap_stream, &graph);
    if (st != TOPO_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    TOPO_HIP(ce);
    const hipError_t ie = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(graph);
      *exec = nullptr;
      TOPO_HIP(ie);
    }
    *graph_out = graph;
  }
  st = group_read_scalars(G);
  if (st != TOPO_OK) return st;
  for (;;) {
    // chunks before the next check: the fewest that any unconverged member asks for
    int ahead = 0;
    for (int i = 0; i < n; ++i) {
      const topo_ctx *c = G.c[i];
      if (c->h_sc->cg_done) continue;
      const int want = chunks_ahead(c, TOPO_PRECOND_MG, c->opts.max_iters);
      ahead = ahead ? std::min(ahead, want) : want;
    }
    if (!ahead) break;
    for (int a = 0; a < ahead; ++a) {
      if (graphs) {
        TOPO_HIP(hipGraphLaunch(*exec, G.s));
      } else {
        for (int k = 0; k < chunk; ++k) {
          st = group_cg_body(G);
          if (st != TOPO_OK) return st;
        }
      }
    }
    st = group_read_scalars(G);
    if (st != TOPO_OK) return st;
  }
  for (topo_ctx *c : G.c) c->cg_prev_iters[TOPO_PRECOND_MG] = c->h_sc->cg_iters;
  topo_status result = TOPO_OK;
  for (int i = 0; i < n; ++i) {
    topo_ctx *c = G.c[i];
    const double relres = std::sqrt(c->h_sc->rr / c->h_sc->ff);
    if (stats) {
      stats[i] = topo_solve_stats{};
      stats[i].iters = c->h_sc->cg_iters;
      stats[i].relres = relres;
      stats[i].converged = relres <= c->opts.rtol;
    }
    if (!(relres <= c->opts.rtol)) {
      set_error("CG of a grouped problem reached max_iters=%d with relres %.3e", c->opts.max_iters, relres);
      result = TOPO_ENOTCONVERGED;
    }
  }
  return result;
}

}  // namespace topo

extern "C" topo_status topo_apply_K(topo_ctx *ctx, const double *d_xphys, const double *d_u, double *d_y) {
  if (!ctx || !d_xphys || !d_u || !d_y) return set_error("NULL argument"), TOPO_EINVAL;
  if (d_u == d_y) return set_error("d_u and d_y must not alias"), TOPO_EINVAL;
  hipStream_t s = ctx->stream;
  const topo_problem &P = ctx->prob;
  Level &L0 = ctx->lv[0];
  TOPO_HIP(launch_simp_modulus(s, ctx->nel, d_xphys, P.E0, P.Emin, P.penal, 1.0, L0.E));
  TOPO_HIP(launch_copy_masked(s, ctx->nnodes, L0.fixed, d_u, ctx->tmp));
  KuArgs a = ku_args(ctx, L0, ctx->tmp);
  a.y = d_y;
  TOPO_HIP(launch_ku(s, KU_STORE, a, ctx->kap, ctx->red, fin_sum(nullptr), ctx->shape_cg));
  // identity rows return the caller's u (not the zeroed copy) on fixed dofs
  TOPO_HIP(launch_copy_fixed(s, ctx->nnodes, L0.fixed, d_u, d_y));
  return TOPO_OK;
}

extern "C" topo_status topo_apply_precond(topo_ctx *ctx, const double *d_xphys, const double *d_r,
                                          double *d_z) {
  if (!ctx || !d_xphys || !d_r || !d_z) return set_error("NULL argument"), TOPO_EINVAL;
  if (d_r == d_z) return set_error("d_r and d_z must not alias"), TOPO_EINVAL;
  hipStream_t s = ctx->stream;
  topo_status st = prepare_operator(ctx, d_xphys);
  if (st != TOPO_OK) return st;
  TOPO_HIP(hipMemcpyAsync(ctx->r, d_r, ctx->ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
  int kind = ctx->opts.precond;
  if (kind == TOPO_PRECOND_LEARNED) {
    if (!ctx->nn) return set_error("TOPO_PRECOND_LEARNED needs a network (topo_set_nn)"), TOPO_EINVAL;
    TOPO_HIP(launch_dot(s, ctx->ndof, ctx->r, ctx->r, ctx->red, fin_sum(&ctx->sc->rr)));
    TOPO_HIP(hipMemsetAsync(ctx->z, 0, ctx->ndof * sizeof(double), s));
  } else if (kind == TOPO_PRECOND_MG && ctx->lv.size() == 1) {
    kind = TOPO_PRECOND_JACOBI;
  }
  st = precondition(ctx, kind, nullptr);
  if (st != TOPO_OK) return st;
  if (z_single(ctx, kind)) TOPO_HIP(launch_convert(s, ctx->ndof, ctx->z32, d_z));
  else TOPO_HIP(hipMemcpyAsync(d_z, ctx->z, ctx->ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
  return TOPO_OK;
}

extern "C" topo_status topo_solve(topo_ctx *ctx, const double *d_xphys, double *d_u, topo_solve_stats *st_out) {
  if (!ctx || !d_xphys || !d_u) return set_error("NULL argument"), TOPO_EINVAL;
  hipEvent_t e0, e1;
  TOPO_HIP(hipEventCreate(&e0));
  TOPO_HIP(hipEventCreate(&e1));
  TOPO_HIP(hipEventRecord(e0, ctx->stream));
  topo_status st = prepare_operator(ctx, d_xphys);
  topo_solve_stats stats{};
  if (st == TOPO_OK) {
    TOPO_HIP(hipMemcpyAsync(ctx->u, d_u, ctx->ndof * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    st = pcg(ctx, &stats);
    TOPO_HIP(hipMemcpyAsync(d_u, ctx->u, ctx->ndof * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    ctx->have_u = 1;
    ctx->n_warm = 0;  // a caller's solve starts a new sequence for the extrapolated
    ctx->nbasis = 0;  // and the projected warm starts
  }
  (void)hipEventRecord(e1, ctx->stream);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  stats.ms = ms;
  if (st_out) *st_out = stats;
  return st;
}

extern "C" topo_status topo_sensitivity(topo_ctx *ctx, const double *d_xphys, const double *d_u,
                                        double *d_ce, double *d_dc, double *h_compliance) {
  if (!ctx || !d_xphys || !d_u || !d_ce || !d_dc) return set_error("NULL argument"), TOPO_EINVAL;
  hipStream_t s = ctx->stream;
  const topo_problem &P = ctx->prob;
  TOPO_HIP(launch_sensitivity(s, ctx->g, ctx->kap, d_u, d_xphys, P.E0, P.Emin, P.penal, d_ce, d_dc));
  if (h_compliance) {
    TOPO_HIP(launch_dot(s, ctx->ndof, ctx->f, d_u, ctx->red, fin_sum(&ctx->sc->comp)));
    topo_status st = read_scalars(ctx);
    if (st != TOPO_OK) return st;
    *h_compliance = ctx->h_sc->comp;
  }
  return TOPO_OK;
}

extern "C" topo_status topo_filter(topo_ctx *ctx, int32_t op, const double *d_in, const double *d_aux,
                                   double *d_out) {
  if (!ctx || !d_out) return set_error("NULL argument"), TOPO_EINVAL;
  if (op < TOPO_FILTER_FWD || op > TOPO_FILTER_VOLW) return set_error("unknown filter op %d", op), TOPO_EINVAL;
  if (op != TOPO_FILTER_VOLW && !d_in) return set_error("d_in is NULL"), TOPO_EINVAL;
  if (op == TOPO_FILTER_SENS && !d_aux) return set_error("d_aux (x) is NULL"), TOPO_EINVAL;
  if (d_out == d_in || (d_aux && d_out == d_aux)) return set_error("d_out must not alias an input"), TOPO_EINVAL;
  TOPO_HIP(launch_filter(ctx->stream, op, ctx->filt, d_in, d_aux, d_out));
  return TOPO_OK;
}

static topo_status oc_update(topo_ctx *ctx, const double *d_x, const double *d_dc, const double *d_dv,
                             double *d_xnew) {
  hipStream_t s = ctx->stream;
  const topo_problem &P = ctx->prob;
  TOPO_HIP(launch_oc_prepare(s, ctx->nel, d_x, d_dc, d_dv, ctx->mask, P.eta, ctx->target, ctx->oc_a,
                             ctx->sc, ctx->red));
  const int passes = oc_pass_launches(ctx->opts.oc_tol);
  for (int pass = 0; pass < passes; ++pass)
    TOPO_HIP(launch_oc_pass(s, ctx->nel, d_x, ctx->oc_a, d_dc, d_dv, ctx->mask, P.move, P.eta,
                            ctx->opts.oc_tol, ctx->sc, ctx->red));
  TOPO_HIP(launch_oc_final(s, ctx->nel, d_x, ctx->oc_a, d_dc, d_dv, ctx->mask, P.move, P.eta, d_xnew,
                           ctx->sc, ctx->red));
  return TOPO_OK;
}

extern "C" topo_status topo_oc_update(topo_ctx *ctx, const double *d_x, const double *d_dc,
                                      const double *d_dv, double *d_xnew, double *h_change,
                                      double *h_lambda) {
  if (!ctx || !d_x || !d_dc || !d_dv || !d_xnew) return set_error("NULL argument"), TOPO_EINVAL;
  if (d_xnew == d_x || d_xnew == d_dc || d_xnew == d_dv) return set_error("d_xnew must not alias an input"), TOPO_EINVAL;
  topo_status st = oc_update(ctx, d_x, d_dc, d_dv, d_xnew);
  if (st != TOPO_OK) return st;
  if (h_change || h_lambda) {
    st = read_scalars(ctx);
    if (st != TOPO_OK) return st;
    if (h_change) *h_change = ctx->h_sc->change;
    if (h_lambda) *h_lambda = ctx->h_sc->lambda;
  }
  return TOPO_OK;
}

// One SIMP iteration in three parts (the solve in between), so that a batch
// can solve the problems of a group together: iterate_pre runs the filter and
// the operator set-up and forms the initial guess, iterate_post the
// sensitivities, the filter adjoint and the OC update, and fills the stats.
// ev: 6 events (phase boundaries).
namespace topo {
topo_status iterate_pre(topo_ctx *ctx, double *d_x, hipEvent_t *ev) {
  hipStream_t s = ctx->stream;
  const topo_problem &P = ctx->prob;
  (void)hipEventRecord(ev[0], s);
  // physical density
  if (P.filter == TOPO_FILTER_DENSITY) {
    TOPO_HIP(launch_filter(s, TOPO_FILTER_FWD, ctx->filt, d_x, nullptr, ctx->xphys));
  } else {
    TOPO_HIP(hipMemcpyAsync(ctx->xphys, d_x, ctx->nel * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  (void)hipEventRecord(ev[1], s);
  // modulus, operator hierarchy and the initial guess (warm start from the last u)
  if (!ctx->opts.warm_start || !ctx->have_u) {
    TOPO_HIP(hipMemsetAsync(ctx->u, 0, ctx->ndof * sizeof(double), s));
    ctx->n_warm = 0;
    ctx->nbasis = 0;
  } else if (ctx->opts.warm_start == 2) {
    // extrapolated start 2 u_k - u_{k-1} once two solutions are known
    if (!ctx->u_prev) TOPO_ALLOC(ctx->u_prev, ctx->ndof);
    if (ctx->n_warm >= 2) TOPO_HIP(launch_extrapolate(s, ctx->ndof, ctx->u, ctx->u_prev));
    else TOPO_HIP(hipMemcpyAsync(ctx->u_prev, ctx->u, ctx->ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  // the coarse inverse is recomputed every coarse_refresh SIMP iterations; in
  // between the previous one (still SPD) preconditions the coarsest level
  const bool refresh = ctx->coarse_due <= 0;
  topo_status st = prepare_operator(ctx, ctx->xphys, refresh, true);
  --ctx->coarse_due;
  if (st == TOPO_OK && ctx->opts.warm_start == 3 && ctx->nbasis > 0) st = projected_start(ctx);
  return st;
}

topo_status iterate_post(topo_ctx *ctx, double *d_x, const topo_solve_stats &ss, hipEvent_t *ev,
                         topo_iter_stats *o) {
  hipStream_t s = ctx->stream;
  const topo_problem &P = ctx->prob;
  ctx->have_u = 1;
  ++ctx->n_warm;
  if (ctx->opts.warm_start == 3) {
    if (!ctx->gram) TOPO_ALLOC(ctx->gram, kMaxBasis * kMaxBasis + kMaxBasis);
    double *&slot = ctx->basis[ctx->basis_next];
    if (!slot) TOPO_ALLOC(slot, ctx->ndof);
    TOPO_HIP(hipMemcpyAsync(slot, ctx->u, ctx->ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
    ctx->basis_next = (ctx->basis_next + 1) % kMaxBasis;
    ctx->nbasis = std::min(ctx->nbasis + 1, kMaxBasis);
  }
  (void)hipEventRecord(ev[2], s);
  // sensitivities and compliance
  TOPO_HIP(launch_sensitivity(s, ctx->g, ctx->kap, ctx->u, ctx->xphys, P.E0, P.Emin, P.penal, ctx->ce, ctx->dc));
  TOPO_HIP(launch_dot(s, ctx->ndof, ctx->f, ctx->u, ctx->red, fin_sum(&ctx->sc->comp)));
  (void)hipEventRecord(ev[3], s);
  // filtered sensitivities and OC update
  if (P.filter == TOPO_FILTER_DENSITY)
    TOPO_HIP(launch_filter(s, TOPO_FILTER_ADJ, ctx->filt, ctx->dc, nullptr, ctx->dcf));
  else
    TOPO_HIP(launch_filter(s, TOPO_FILTER_SENS, ctx->filt, ctx->dc, d_x, ctx->dcf));
  (void)hipEventRecord(ev[4], s);
  topo_status st = oc_update(ctx, d_x, ctx->dcf, ctx->volw, ctx->xnew);
  if (st != TOPO_OK) return st;
  TOPO_HIP(hipMemcpyAsync(d_x, ctx->xnew, ctx->nel * sizeof(double), hipMemcpyDeviceToDevice, s));
  (void)hipEventRecord(ev[5], s);
  if (o) {
    st = read_scalars(ctx);
    if (st != TOPO_OK) return st;
    fill_stats(ctx, ss, ev, o);
  }
  return TOPO_OK;
}

// the stats of one SIMP iteration from the scalars already read back and the
// six phase events
void fill_stats(const topo_ctx *ctx, const topo_solve_stats &ss, hipEvent_t *ev, topo_iter_stats *o) {
  o->c = ctx->h_sc->comp;
  o->volume = ctx->h_sc->volume;
  o->change = ctx->h_sc->change;
  o->lambda = ctx->h_sc->lambda;
  o->pcg_iters = ss.iters;
  o->converged = ss.converged;
  o->relres = ss.relres;
  o->fallbacks = ss.fallbacks;
  o->learned_iters = ss.learned_iters;
  float t[5];
  for (int k = 0; k < 5; ++k) (void)hipEventElapsedTime(&t[k], ev[k], ev[k + 1]);
  float tot = 0.f;
  (void)hipEventElapsedTime(&tot, ev[0], ev[5]);
  o->ms_total = tot;
  o->ms_filter = t[0] + t[3];
  o->ms_solve = t[1];
  o->ms_sens = t[2];
  o->ms_oc = t[4];
}

// ---------------------------------------------------------------------------
// The rest of a SIMP iteration of a group (iterate_pre / iterate_post of every
// member, with one launch per step for the whole group).  The members must be
// in lockstep (the same warm-start history and coarse refresh count), which
// they are when set up and iterated together; members whose filters differ in
// reach or mode share the launches of their own kind.
bool group_lockstep(const Group &G) {
  const topo_ctx *a = G.c[0];
  for (const topo_ctx *c : G.c) {
    if (c->nn || !c->oc_a) return false;
    if (c->nel != a->nel || c->ndof != a->ndof || c->lv.size() != a->lv.size() || c->ncoarse != a->ncoarse ||
        c->mixed != a->mixed)
      return false;
    if (c->opts.warm_start != a->opts.warm_start || c->have_u != a->have_u || c->n_warm != a->n_warm ||
        c->nbasis != a->nbasis || c->basis_next != a->basis_next || c->coarse_due != a->coarse_due)
      return false;
  }
  return true;
}

// op for each member's problem: TOPO_FILTER_* per member (-1: none); members
// with the same operation and stencil reach share a launch
static topo_status group_filter(const Group &G, const std::vector<int> &op, const std::vector<FilterCall> &call) {
  const int n = G.n();
  std::vector<bool> done(n, false);
  for (int i = 0; i < n; ++i) {
    if (done[i] || op[i] < 0) continue;
    const int R = call[i].f.R;
    const bool tiled = R >= 1 && R <= kFilterTiledMaxR;
    std::vector<FilterCall> part;
    for (int j = i; j < n; ++j) {
      const int Rj = call[j].f.R;
      const bool tj = Rj >= 1 && Rj <= kFilterTiledMaxR;
      if (done[j] || op[j] != op[i] || tj != tiled || (tiled && Rj != R)) continue;
      part.push_back(call[j]);
      done[j] = true;
    }
    TOPO_HIP(launch_filter_group(G.s, op[i], (int)part.size(), part.data()));
  }
  return TOPO_OK;
}

// prepare_operator for every member
// The grouped coarse inverse goes to the first member's side stream (joined by
// group_pcg before the first V-cycle).
static topo_status group_prepare_operator(const Group &G, bool refresh) {
  const int n = G.n();
  topo_ctx *c0 = G.c[0];
  hipStream_t s = G.s;
  for (topo_ctx *c : G.c) {
    const topo_status js = join_inverse(c);
    if (js != TOPO_OK) return js;
  }
  std::vector<ModulusArgs> ma(n);
  for (int i = 0; i < n; ++i) {
    const topo_problem &P = G.c[i]->prob;
    ma[i] = ModulusArgs{G.c[i]->xphys, P.E0, P.Emin, P.penal, G.c[i]->lv[0].E,
                        c0->mixed ? G.c[i]->lv[0].f32.E : nullptr};
  }
  TOPO_HIP(launch_simp_modulus_group(s, n, c0->nel, ma.data()));
  for (size_t l = 0; l < c0->lv.size(); ++l) {
    std::vector<const double *> ef(n);
    std::vector<double *> ec(n);
    std::vector<float *> ec32(n);
    std::vector<DiagArgs> da(n);
    for (int i = 0; i < n; ++i) {
      Level &L = G.c[i]->lv[l];
      if (l > 0) ef[i] = G.c[i]->lv[l - 1].E, ec[i] = L.E, ec32[i] = c0->mixed ? L.f32.E : nullptr;
      da[i] = DiagArgs{L.E, G.c[i]->kap, L.fixed, L.dinv, c0->mixed ? L.f32.dinv : nullptr};
    }
    if (l > 0)
      TOPO_HIP(launch_coarsen_moduli_group(s, n, c0->lv[l - 1].g, c0->lv[l].g, ef.data(), ec.data(), ec32.data()));
    TOPO_HIP(launch_diag_group(s, n, c0->lv[l].g, da.data()));
  }
  if (c0->lv.size() > 1 && refresh) {
    std::vector<AssembleArgs> aa(n);
    std::vector<double *> A(n), W(n);
    for (int i = 0; i < n; ++i) {
      const Level &C = G.c[i]->lv.back();
      aa[i] = AssembleArgs{C.E, G.c[i]->kap, C.fixed, G.c[i]->Ainv};
      A[i] = G.c[i]->Ainv;
      W[i] = G.c[i]->Awork;
    }
    hipStream_t si = s;
    const topo_status ss = side_begin(c0, s, &si);
    if (ss != TOPO_OK) return ss;
    TOPO_HIP(launch_dense_assemble_group(si, n, c0->lv.back().g, aa.data()));
    TOPO_HIP(launch_dense_invert_group(si, n, c0->ncoarse, A.data(), W.data()));
    const topo_status se = side_end(c0);
    if (se != TOPO_OK) return se;
  }
  for (topo_ctx *c : G.c) c->coarse_due = refresh ? c->opts.coarse_refresh : c->coarse_due;
  return TOPO_OK;
}

// projected_start for every member: the Gram matrices together, one wait,
// the combinations of the members whose projection is usable
static topo_status group_projected_start(const Group &G) {
  const int n = G.n();
  topo_ctx *c0 = G.c[0];
  hipStream_t s = G.s;
  const int nb = c0->nbasis;
  const std::vector<Reducer> red = group_reds(G);
  const int shape = ku_shape_for(c0->g, KU_STORE, TOPO_KU_AUTO, false);
  std::vector<KuArgs> a(n);
  std::vector<MultiDotArgs> md(n);
  std::vector<Fin> fin(n), nofin(n, fin_sum(nullptr));
  for (int j = 0; j < nb; ++j) {
    for (int i = 0; i < n; ++i) {
      topo_ctx *c = G.c[i];
      a[i] = ku_args(c, c->lv[0], c->basis[j]);
      a[i].y = c->tmp;
      md[i] = gram_column(c, j, c->tmp);
      fin[i] = fin_sum(&c->gram[j * kMaxBasis]);
    }
    TOPO_HIP(launch_ku_group<double>(s, KU_STORE, n, a.data(), c0->kap, red.data(), nofin.data(), shape));
    TOPO_HIP(launch_multi_dot_group(s, n, c0->ndof, md.data(), red.data(), fin.data()));
  }
  for (int i = 0; i < n; ++i) {
    md[i] = gram_column(G.c[i], nb, G.c[i]->f);
    fin[i] = fin_sum(&G.c[i]->gram[kMaxBasis * kMaxBasis]);
  }
  TOPO_HIP(launch_multi_dot_group(s, n, c0->ndof, md.data(), red.data(), fin.data()));
  constexpr int kGram = kMaxBasis * kMaxBasis + kMaxBasis;
  std::vector<double> h((size_t)n * kGram);
  for (int i = 0; i < n; ++i)
    TOPO_HIP(hipMemcpyAsync(&h[(size_t)i * kGram], G.c[i]->gram, kGram * sizeof(double), hipMemcpyDeviceToHost, s));
  TOPO_HIP(hipStreamSynchronize(s));
  std::vector<Combo> cb;
  std::vector<double *> uu;
  for (int i = 0; i < n; ++i) {
    double alpha[kMaxBasis];
    if (!projection_coefficients(&h[(size_t)i * kGram], nb, alpha)) continue;  // plain warm start
    Combo c{};
    c.n = nb;
    for (int k = 0; k < nb; ++k) {
      c.v[k] = G.c[i]->basis[k];
      c.alpha[k] = alpha[k];
    }
    cb.push_back(c);
    uu.push_back(G.c[i]->u);
  }
  if (!cb.empty()) TOPO_HIP(launch_combine_group(s, (int)cb.size(), c0->ndof, cb.data(), uu.data()));
  return TOPO_OK;
}

topo_status group_pre(const Group &G, double *const *d_x, hipEvent_t *ev) {
  const int n = G.n();
  topo_ctx *c0 = G.c[0];
  hipStream_t s = G.s;
  (void)hipEventRecord(ev[0], s);
  // physical densities
  {
    std::vector<int> op(n);
    std::vector<FilterCall> call(n);
    std::vector<const void *> src;
    std::vector<void *> dst;
    for (int i = 0; i < n; ++i) {
      topo_ctx *c = G.c[i];
      const bool density = c->prob.filter == TOPO_FILTER_DENSITY;
      op[i] = density ? TOPO_FILTER_FWD : -1;
      call[i] = FilterCall{c->filt, d_x[i], nullptr, c->xphys};
      if (!density) src.push_back(d_x[i]), dst.push_back(c->xphys);
    }
    topo_status st = group_filter(G, op, call);
    if (st != TOPO_OK) return st;
    if (!src.empty())
      TOPO_HIP(launch_copy_group(s, (int)src.size(), c0->nel * (int64_t)sizeof(double), src.data(), dst.data()));
  }
  (void)hipEventRecord(ev[1], s);
  // initial guesses
  std::vector<double *> uu(n), up(n);
  for (int i = 0; i < n; ++i) uu[i] = G.c[i]->u;
  if (!c0->opts.warm_start || !c0->have_u) {
    std::vector<void *> d(uu.begin(), uu.end());
    TOPO_HIP(launch_copy_group(s, n, c0->ndof * (int64_t)sizeof(double), nullptr, d.data()));
    for (topo_ctx *c : G.c) c->n_warm = 0, c->nbasis = 0;
  } else if (c0->opts.warm_start == 2) {
    for (int i = 0; i < n; ++i) {
      topo_ctx *ctx = G.c[i];
      if (!ctx->u_prev) TOPO_ALLOC(ctx->u_prev, ctx->ndof);
      up[i] = ctx->u_prev;
    }
    if (c0->n_warm >= 2) {
      TOPO_HIP(launch_extrapolate_group(s, n, c0->ndof, uu.data(), up.data()));
    } else {
      std::vector<const void *> a(uu.begin(), uu.end());
      std::vector<void *> b(up.begin(), up.end());
      TOPO_HIP(launch_copy_group(s, n, c0->ndof * (int64_t)sizeof(double), a.data(), b.data()));
    }
  }
  const bool refresh = c0->coarse_due <= 0;
  topo_status st = group_prepare_operator(G, refresh);
  for (topo_ctx *c : G.c) --c->coarse_due;
  if (st == TOPO_OK && c0->opts.warm_start == 3 && c0->nbasis > 0) st = group_projected_start(G);
  return st;
}

topo_status group_post(const Group &G, double *const *d_x, const topo_solve_stats *ss, hipEvent_t *ev,
                       topo_iter_stats *const *o) {
  const int n = G.n();
  topo_ctx *c0 = G.c[0];
  hipStream_t s = G.s;
  for (topo_ctx *c : G.c) c->have_u = 1, ++c->n_warm;
  if (c0->opts.warm_start == 3) {
    std::vector<const void *> a(n);
    std::vector<void *> b(n);
    for (int i = 0; i < n; ++i) {
      topo_ctx *ctx = G.c[i];
      if (!ctx->gram) TOPO_ALLOC(ctx->gram, kMaxBasis * kMaxBasis + kMaxBasis);
      double *&slot = ctx->basis[ctx->basis_next];
      if (!slot) TOPO_ALLOC(slot, ctx->ndof);
      a[i] = ctx->u;
      b[i] = slot;
      ctx->basis_next = (ctx->basis_next + 1) % kMaxBasis;
      ctx->nbasis = std::min(ctx->nbasis + 1, kMaxBasis);
    }
    TOPO_HIP(launch_copy_group(s, n, c0->ndof * (int64_t)sizeof(double), a.data(), b.data()));
  }
  (void)hipEventRecord(ev[2], s);
  // sensitivities and compliances
  {
    std::vector<SensArgs> sa(n);
    std::vector<DotArgs> fu(n);
    std::vector<Fin> fin(n);
    for (int i = 0; i < n; ++i) {
      topo_ctx *c = G.c[i];
      const topo_problem &P = c->prob;
      sa[i] = SensArgs{c->kap, c->u, c->xphys, P.E0, P.Emin, P.penal, c->ce, c->dc};
      fu[i] = DotArgs{c->f, c->u, nullptr};
      fin[i] = fin_sum(&c->sc->comp);
    }
    TOPO_HIP(launch_sensitivity_group(s, n, c0->g, sa.data()));
    const std::vector<Reducer> red = group_reds(G);
    TOPO_HIP(launch_dot_group(s, n, c0->ndof, fu.data(), red.data(), fin.data()));
  }
  (void)hipEventRecord(ev[3], s);
  // filtered sensitivities
  {
    std::vector<int> op(n);
    std::vector<FilterCall> call(n);
    for (int i = 0; i < n; ++i) {
      topo_ctx *c = G.c[i];
      const bool density = c->prob.filter == TOPO_FILTER_DENSITY;
      op[i] = density ? TOPO_FILTER_ADJ : TOPO_FILTER_SENS;
      call[i] = FilterCall{c->filt, c->dc, density ? nullptr : d_x[i], c->dcf};
    }
    topo_status st = group_filter(G, op, call);
    if (st != TOPO_OK) return st;
  }
  (void)hipEventRecord(ev[4], s);
  // OC updates into xnew, then the designs
  {
    std::vector<OcArgs> oa(n);
    std::vector<const void *> a(n);
    std::vector<void *> b(n);
    for (int i = 0; i < n; ++i) {
      topo_ctx *c = G.c[i];
      const topo_problem &P = c->prob;
      oa[i] = OcArgs{d_x[i], c->dcf, c->volw, c->mask, P.move, P.eta, c->opts.oc_tol, c->target,
                     c->oc_a, c->xnew, c->sc};
      a[i] = c->xnew;
      b[i] = d_x[i];
    }
    const std::vector<Reducer> red = group_reds(G);
    TOPO_HIP(launch_oc_update_group(s, n, c0->nel, oa.data(), red.data()));
    TOPO_HIP(launch_copy_group(s, n, c0->nel * (int64_t)sizeof(double), a.data(), b.data()));
  }
  (void)hipEventRecord(ev[5], s);
  bool any = false;
  for (int i = 0; i < n; ++i) any = any || o[i];
  if (any) {
    for (topo_ctx *c : G.c) TOPO_HIP(hipMemcpyAsync(c->h_sc, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    TOPO_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i)
      if (o[i]) fill_stats(G.c[i], ss[i], ev, o[i]);
  }
  return TOPO_OK;
}
}  // namespace topo

extern "C" topo_status topo_iterate(topo_ctx *ctx, double *d_x, int32_t n_iter, topo_iter_stats *h_stats) {
  if (!ctx || !d_x || n_iter < 0) return set_error("invalid argument"), TOPO_EINVAL;
  hipEvent_t ev[6];
  for (auto &e : ev) TOPO_HIP(hipEventCreate(&e));
  topo_status result = TOPO_OK;
  for (int it = 0; it < n_iter; ++it) {
    topo_status st = iterate_pre(ctx, d_x, ev);
    topo_solve_stats ss{};
    if (st == TOPO_OK) st = pcg(ctx, &ss);
    if (st != TOPO_OK && st != TOPO_ENOTCONVERGED) return st;
    if (st == TOPO_ENOTCONVERGED) result = st;
    st = iterate_post(ctx, d_x, ss, ev, h_stats ? &h_stats[it] : nullptr);
    if (st != TOPO_OK) return st;
  }
  TOPO_HIP(hipStreamSynchronize(ctx->stream));
  for (auto &e : ev) (void)hipEventDestroy(e);
  return result;
}

extern "C" topo_status topo_time_operator(topo_ctx *ctx, int32_t reps, double *h_ms) {
  if (!ctx || reps < 1 || !h_ms) return set_error("invalid argument"), TOPO_EINVAL;
  hipStream_t s = ctx->stream;
  Level &L0 = ctx->lv[0];
  KuArgs a = ku_args(ctx, L0, ctx->u);
  a.y = ctx->tmp;
  hipEvent_t e0, e1;
  TOPO_HIP(hipEventCreate(&e0));
  TOPO_HIP(hipEventCreate(&e1));
  // the plain product (no dot product, hence no finalize launch between the
  // events), in the CG product's launch shape
  TOPO_HIP(launch_ku(s, KU_STORE, a, ctx->kap, ctx->red, fin_sum(nullptr), ctx->shape_cg));  // warm caches
  TOPO_HIP(hipEventRecord(e0, s));
  for (int i = 0; i < reps; ++i)
    TOPO_HIP(launch_ku(s, KU_STORE, a, ctx->kap, ctx->red, fin_sum(nullptr), ctx->shape_cg));
  TOPO_HIP(hipEventRecord(e1, s));
  TOPO_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  TOPO_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *h_ms = (double)ms / reps;
  return TOPO_OK;
}

extern "C" topo_status topo_get_state(topo_ctx *ctx, double *d_u, double *d_xphys) {
  if (!ctx) return set_error("ctx is NULL"), TOPO_EINVAL;
  if (d_u) TOPO_HIP(hipMemcpyAsync(d_u, ctx->u, ctx->ndof * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  if (d_xphys) TOPO_HIP(hipMemcpyAsync(d_xphys, ctx->xphys, ctx->nel * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  return TOPO_OK;
}

extern "C" topo_status topo_set_nn(topo_ctx *ctx, topo_nn *nn) {
  if (!ctx) return set_error("ctx is NULL"), TOPO_EINVAL;
  // the captured learned-preconditioner chunk refers to the network's buffers
  if (ctx->cg_exec[TOPO_PRECOND_LEARNED]) (void)hipGraphExecDestroy(ctx->cg_exec[TOPO_PRECOND_LEARNED]);
  if (ctx->cg_graph[TOPO_PRECOND_LEARNED]) (void)hipGraphDestroy(ctx->cg_graph[TOPO_PRECOND_LEARNED]);
  ctx->cg_exec[TOPO_PRECOND_LEARNED] = nullptr;
  ctx->cg_graph[TOPO_PRECOND_LEARNED] = nullptr;
  ctx->nn = nullptr;
  if (!nn) {
    TOPO_HIP(hipStreamSynchronize(ctx->stream));
    ctx->nnw.release();
    return TOPO_OK;
  }
  const Dim3 g0{ctx->g.NX(), ctx->g.NY(), ctx->g.NZ()};
  if (g0.count() > ((int64_t)1 << 30)) return set_error("grid too large for the network"), TOPO_EUNSUPPORTED;
  topo_status st = nn_prepare(nn, ctx->nnw, g0, 1, false);
  if (st != TOPO_OK) return st;
  ctx->nn = nn;
  return TOPO_OK;
}

extern "C" topo_status topo_nn_make_pairs(topo_ctx *ctx, const double *d_xphys, int32_t n, const int32_t *h_iters,
                                          float *d_rho, float *d_r, float *d_e, uint8_t *d_fixed) {
  if (!ctx || !d_xphys || !h_iters || !d_rho || !d_r || !d_e || !d_fixed) return set_error("NULL argument"), TOPO_EINVAL;
  if (n < 1) return set_error("n must be >= 1"), TOPO_EINVAL;
  for (int i = 0; i < n; ++i)
    if (h_iters[i] < 0) return set_error("iteration counts must be >= 0"), TOPO_EINVAL;
  hipStream_t s = ctx->stream;
  if (!ctx->ustar) TOPO_ALLOC(ctx->ustar, ctx->ndof);
  const int base = ctx->lv.size() > 1 ? TOPO_PRECOND_MG : TOPO_PRECOND_JACOBI;
  topo_status st = prepare_operator(ctx, d_xphys);
  if (st != TOPO_OK) return st;
  // converged solution
  const double rtol_user = ctx->opts.rtol;
  ctx->opts.rtol = std::min(rtol_user, 1e-10);
  TOPO_HIP(hipMemsetAsync(ctx->u, 0, ctx->ndof * sizeof(double), s));
  st = pcg_run(ctx, base, ctx->opts.max_iters);
  const double rtol2 = ctx->opts.rtol * ctx->opts.rtol;
  ctx->opts.rtol = rtol_user;
  if (st != TOPO_OK) return st;
  if (!(ctx->h_sc->rr <= rtol2 * ctx->h_sc->ff))
    return set_error("reference solve did not converge (relres %.3e)", std::sqrt(ctx->h_sc->rr / ctx->h_sc->ff)),
           TOPO_ENOTCONVERGED;
  TOPO_HIP(hipMemcpyAsync(ctx->ustar, ctx->u, ctx->ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
  const int64_t V = ctx->nnodes;
  TOPO_HIP(launch_node_density(s, ctx->g, d_xphys, d_rho));
  Level &L0 = ctx->lv[0];
  for (int i = 0; i < n; ++i) {
    if (i > 0) TOPO_HIP(hipMemcpyAsync(d_rho + (size_t)i * V, d_rho, V * sizeof(float), hipMemcpyDeviceToDevice, s));
    TOPO_HIP(hipMemcpyAsync(d_fixed + (size_t)i * V, L0.fixed, V, hipMemcpyDeviceToDevice, s));
    TOPO_HIP(hipMemsetAsync(ctx->u, 0, ctx->ndof * sizeof(double), s));
    if (h_iters[i] > 0) {
      st = pcg_run(ctx, base, h_iters[i]);
      if (st != TOPO_OK) return st;
    }
    // true residual of the iterate, and its error against the converged solution
    KuArgs a = ku_args(ctx, L0, ctx->u);
    a.y = ctx->r;
    a.b = ctx->f;
    TOPO_HIP(launch_ku(s, KU_RESID, a, ctx->kap, ctx->red, fin_sum(&ctx->sc->red[0])));
    TOPO_HIP(launch_pair_out(s, ctx->ndof, ctx->r, ctx->ustar, ctx->u, d_r + (size_t)i * 3 * V,
                             d_e + (size_t)i * 3 * V));
  }
  TOPO_HIP(hipStreamSynchronize(s));
  ctx->have_u = 0;  // the next warm start must not use a truncated iterate
  return TOPO_OK;
}
