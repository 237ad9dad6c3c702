// Internal declarations of libtopo (not part of the ABI).
#pragma once

#include <string>
#include <vector>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/topo.h"

namespace topo {

// ---------------------------------------------------------------------------
// grid geometry
struct Grid {
  int nx, ny, nz;  // elements per axis
  __host__ __device__ int NX() const { return nx + 1; }
  __host__ __device__ int NY() const { return ny + 1; }
  __host__ __device__ int NZ() const { return nz + 1; }
  __host__ __device__ int64_t nel() const { return (int64_t)nx * ny * nz; }
  __host__ __device__ int64_t nnodes() const { return (int64_t)(nx + 1) * (ny + 1) * (nz + 1); }
  __host__ __device__ int64_t ndof() const { return 3 * nnodes(); }
};

// Local node a of an element sits at corner (cx(a), cy(a), cz(a)) of the unit cube.
__host__ __device__ constexpr int cx(int a) { return (a == 1 || a == 2 || a == 5 || a == 6) ? 1 : 0; }
__host__ __device__ constexpr int cy(int a) { return (a == 2 || a == 3 || a == 6 || a == 7) ? 1 : 0; }
__host__ __device__ constexpr int cz(int a) { return a >= 4 ? 1 : 0; }
__host__ __device__ constexpr int corner_of(int x, int y, int z) {
  return z * 4 + (y ? (x ? 2 : 3) : (x ? 1 : 0));
}

// ---------------------------------------------------------------------------
// deterministic reductions: each reducing kernel stores one partial per block,
// a one-block finalize kernel sums them in block order.
constexpr int kMaxRed = 4;  // values reduced together in one kernel

struct Reducer {
  double *partials;  // [max_blocks * kMaxRed]
  int max_blocks;
};

// ---------------------------------------------------------------------------
// error state
void set_error(const char *fmt, ...);
#define TOPO_HIP(call)                                                           \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ::topo::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),   \
                        __FILE__, __LINE__);                                     \
      return TOPO_EDEVICE;                                                       \
    }                                                                            \
  } while (0)

// ---------------------------------------------------------------------------
// device scalar block of the CG loop and the OC search
constexpr int kOcCand = 63;  // candidate multipliers evaluated per pass
struct Scalars {
  double rr, rz, rz_new, pq, ff, alpha, beta, comp;  // CG / compliance
  double red[8];                                     // scratch results of reductions
  // OC multiplier search
  double l1, l2, target, vconst, change, volume, lambda;
  int oc_done, oc_pass;
  int cg_done, cg_iters;  // device-side CG convergence state
  int cg_max;             // iteration cap of the running solve
  int nn_fallback;        // learned preconditioner failed its safeguard test
  double rtol2;           // squared relative tolerance of the running solve
  double rr_start;        // r.r when the running solve started
  double rz_old;          // r.z as the x/r update found it (read by the fused flexible p update)
  double oc_lam[64];
};

// the 10 distinct values of the element matrix (their placement: ke_code.h)
template <typename T>
struct KappaT {
  T k[10];
};
using Kappa = KappaT<double>;
// the element matrix's 8 distinct entries in the sum/difference basis of the
// element's corners, in the form the kernels apply them (see ke_code.h)
template <typename T>
struct HadaW {
  T w[8];
};

// ---------------------------------------------------------------------------
// kernel launchers (kernels_*.hip)

// What a finalize does with the reduced value (see finalize_kernel):
//   FIN_CG_CHECK  (out = rr): count the iteration, raise cg_done at convergence
//                 (rr <= rtol2 ff) or at the iteration cap cg_max
//   FIN_RZ        (out = rz_new): beta = rz_new / rz, then rz = rz_new
//   FIN_RZ_FLEX   (out = r.z_new, r.z_old): flexible (Polak-Ribiere) beta
//   FIN_RZ_SAFE   (out = r.z_new, r.z_old, z.z): as FIN_RZ_FLEX, and when
//                 r.z_new <= kSafeEps ||r|| ||z|| (or any of them is not finite)
//                 raise nn_fallback and cg_done
enum FinMode { FIN_SUM = 0, FIN_MAX = 1, FIN_CG_CHECK = 2, FIN_RZ = 3, FIN_RZ_FLEX = 4, FIN_RZ_SAFE = 5 };
constexpr double kSafeEps = 1e-6;
struct Fin {
  int mode;
  double *out;      // device result slot(s)
  Scalars *sc;      // all modes but FIN_SUM / FIN_MAX
};
inline Fin fin_sum(double *out) { return Fin{FIN_SUM, out, nullptr}; }
inline Fin fin_max(double *out) { return Fin{FIN_MAX, out, nullptr}; }

// sums nparts partials (slot-major, k-th value at [slot*kMaxRed + k]) into fin.out[0..n)
hipError_t launch_finalize(hipStream_t s, const Reducer &red, int nparts, int n, const Fin &fin,
                           const int *skip = nullptr);

// E_e = Emin + xphys^p (E0 - Emin), times scale.  The set-up kernels below
// also write a single-precision copy of their result where one is passed (E32,
// Ec32, dinv32 may be NULL): the FP64 value rounded once.
hipError_t launch_simp_modulus(hipStream_t s, int64_t nel, const double *xphys, double E0,
                               double Emin, double penal, double scale, double *E, float *E32 = nullptr);
// E_c = 2 * mean of the 8 children (missing children count as 0)
hipError_t launch_coarsen_moduli(hipStream_t s, Grid gf, Grid gc, const double *Ef, double *Ec,
                                 float *Ec32 = nullptr);
// dinv_i = 1 / sum_{e ni i} E_e KE_{li,li}; 0 on fixed dofs
hipError_t launch_diag(hipStream_t s, Grid g, const double *E, const Kappa &kap,
                       const uint8_t *fixed, double *dinv, float *dinv32 = nullptr);

// K.u variants (matrix-free, identity rows on fixed dofs); the input vector must
// be zero on fixed dofs.
enum KuEpi {
  KU_STORE = 0,        // y = Au
  KU_STORE_DOT = 1,    // y = Au, reduce u.y
  KU_RESID = 2,        // y = b - Au, reduce y.y
  KU_RES0 = 3,         // operand d0 = b dinv s0: x = d0; res = b - A d0
  KU_CHEB0 = 4,        // operand d0 = b dinv s0: res = b - A d0; dout = c1 d0 + c2 res dinv; x = d0 + dout
  KU_CHEB = 5,         // res -= Au; dout = c1 u + c2 res dinv; x += dout      [reduce dot_with.x]
                       // (dout = NULL: the last step, only x is stored)
  KU_CHEB_ADD = 6,     // as KU_CHEB with x += u + dout (u = the pending step)  [reduce dot_with.x]
  KU_RESUPD = 7,       // res -= Au
  KU_RESID_START = 8,  // res = b - Au; dout = res dinv s0 (x not updated: the next
                       // KU_CHEB_ADD adds dout; dout null: not stored)
  KU_RESID_FLEX = 9,   // the end of a degree-1 post-smoothing handed to flexible CG:
                       // res = b - Au (not stored), z_new = u + res dinv s0 into zflex
                       // (u = x), reduce rflex.z_new and rflex.z_old (z_old: zflex before)
};
// values an epilogue reduces (0: none)
inline int ku_ndot(KuEpi epi) { return epi == KU_RESID_FLEX ? 2 : 1; }
template <typename T>
struct KuArgsT {
  Grid g;
  const T *E;
  const T *u;             // stencil operand
  T *y;                   // STORE, STORE_DOT, RESID output
  const T *b;             // right-hand side
  const uint8_t *fixed;   // per node, bit c set if dof c is fixed
  T *res, *x, *dout;      // smoother vectors
  const T *dinv;          // inverse Jacobi diagonal (0 on fixed dofs)
  T c1, c2, s0;
  const T *dot_with;      // CHEB / CHEB_ADD: if set, reduce dot_with . x_new
  const int *skip;        // device flag: return at once when non-zero (may be NULL)
  const float *ke32;      // matrix-core shapes: KE as FP32 [32][24] (rows 24.. zero)
  const void *ke16;       // ... and as BF16 [32][32] (zero padded)
  const double *rflex;    // RESID_FLEX: the conjugate-gradient residual (FP64)
  T *zflex;               // RESID_FLEX: the preconditioned residual, read and replaced
  // RES0 on an element-column shape of 256 threads: CG's r.r as chk_n block
  // partials (value 0 of each slot); every block first takes the stopping test
  // of FIN_CG_CHECK on their sum (the x/r update has counted the iteration)
  // and returns when CG has stopped; block 0 stores r.r and raises cg_done
  const double *chk_parts;
  int chk_n;
  Scalars *chk_sc;
};
using KuArgs = KuArgsT<double>;
// threads per block of element-column shape `which` (relative to kKuShapeHada)
int ku_hada_block_threads(int which);
// fin receives the reduction of STORE_DOT / RESID / CHEB with dot_with
// shape: launch shape index (-1 = chosen from the grid size)
// defer_parts: no finalize launch; the block partials stay in red (value 0 of
// each slot) for the next kernel to sum, and their count is stored here
hipError_t launch_ku(hipStream_t s, KuEpi epi, const KuArgs &a, const Kappa &kap, const Reducer &red,
                     const Fin &fin, int shape = -1, int *defer_parts = nullptr);
// single-precision operator (smoothing passes only: no reducing epilogues but
// RESID_FLEX's, which defer_parts can leave as partials as above)
hipError_t launch_ku(hipStream_t s, KuEpi epi, const KuArgsT<float> &a, const KappaT<float> &kap,
                     const Reducer &red, const Fin &fin, int shape = -1, int *defer_parts = nullptr);
// launch shape by grid size within a K.u kernel family (TOPO_KU_*), for the
// double- or the single-precision operator
int ku_shape_for(const Grid &g, KuEpi epi, int family, bool single = false);
// launch shapes: 0..3 the node-column vector kernel (FP64 and FP32), 4 the FP32
// matrix-core kernel (single precision only), 5 the matrix-core kernel with BF16
// operands (single precision only; changes the arithmetic, chosen only in BF16
// mode), 6..10 the element-column kernel in the sum/difference basis
constexpr int kKuShapes = 4;
constexpr int kKuShapeMfma = 4, kKuShapeMfmaBf16 = 5;
inline bool ku_matrix_core_shape(int shape) { return shape == kKuShapeMfma || shape == kKuShapeMfmaBf16; }
constexpr int kKuShapeHada = 6, kKuShapesHada = 9;
hipError_t launch_ku_mfma(hipStream_t s, KuEpi epi, const KuArgsT<float> &a, bool bf16);
template <typename T>
hipError_t launch_ku_hada(hipStream_t s, KuEpi epi, const KuArgsT<T> &a, const KappaT<T> &kap,
                          const Reducer &red, int which, int *nparts);
template <typename T>
hipError_t launch_ku_hada_group(hipStream_t s, KuEpi epi, int G, const KuArgsT<T> *a, const KappaT<T> &kap,
                                const Reducer *red, int which, int *nparts);
// most block partials any K.u launch shape writes on this grid
int64_t ku_max_blocks(const Grid &g);
int64_t ku_hada_max_blocks(const Grid &g);
// shapes the autotuner times within a K.u kernel family (TOPO_KU_*; with AUTO,
// single precision adds the FP32 matrix-core kernel)
std::vector<int> ku_tunable_shapes(bool single, int family);

// vector kernels
hipError_t launch_zero_fixed(hipStream_t s, int64_t nnodes, const uint8_t *fixed, double *v);
hipError_t launch_copy_masked(hipStream_t s, int64_t nnodes, const uint8_t *fixed, const double *in,
                              double *out);
// out[d] = in[d] on fixed dofs only
hipError_t launch_copy_fixed(hipStream_t s, int64_t nnodes, const uint8_t *fixed, const double *in,
                             double *out);
hipError_t launch_dot(hipStream_t s, int64_t n, const double *a, const double *b, const Reducer &red,
                      const Fin &fin, const int *skip = nullptr);
// x += alpha p; r -= alpha q; fin.out = r.r (alpha = sc->rz / sc->pq); with
// FIN_CG_CHECK the finalize also runs the device-side convergence test
hipError_t launch_cg_update_xr(hipStream_t s, int64_t n, Scalars *sc, double *x, double *r,
                               const double *p, const double *q, const Reducer &red,
                               const Fin &fin, const int *skip = nullptr, float *r32 = nullptr);
// The same with p.q still as npq block partials in red (left by launch_ku with
// defer_parts): every block sums them in the finalize kernel's order (so alpha
// is bit for bit the one of the unfused pair), block 0 stores p.q, and the r.r
// partials go to value 1 of each slot, apart from the ones being read.
// defer_rr: no finalize launch either; block 0 counts the iteration, the r.r
// partials stay at red.partials + 1 and their count is stored here, for a
// RES0 pass with chk_parts to take the stopping test
hipError_t launch_cg_update_xr_pq(hipStream_t s, int64_t n, Scalars *sc, double *x, double *r,
                                  const double *p, const double *q, const Reducer &red, int npq,
                                  const Fin &fin, const int *skip = nullptr, float *r32 = nullptr,
                                  int *defer_rr = nullptr);
// cg_iters = 0; rtol2, cg_max stored; nn_fallback = 0; cg_done = (rr <= rtol2 ff)
hipError_t launch_cg_start(hipStream_t s, Scalars *sc, double rtol2, int max_iters);
// z = r * dinv; fin.out = r.z
hipError_t launch_jacobi(hipStream_t s, int64_t n, const double *r, const double *dinv, double *z,
                         const Reducer &red, const Fin &fin, const int *skip = nullptr);
// p = z + beta p (p = z if first); beta is set by the FIN_RZ finalize of r.z;
// z in double or (single-precision preconditioner) in single precision
hipError_t launch_cg_update_p(hipStream_t s, int64_t n, Scalars *sc, const double *z, double *p,
                              int first, const int *skip = nullptr);
hipError_t launch_cg_update_p(hipStream_t s, int64_t n, Scalars *sc, const float *z, double *p,
                              int first, const int *skip = nullptr);
// The flexible update with r.z_new and r.z_old still as nrz block partials in
// red (left by RESID_FLEX with defer_parts): every block sums them in the
// finalize kernel's order and forms beta = (r.z_new - r.z_old) / sc->rz_old as
// FIN_RZ_FLEX does from sc->rz (sc->rz_old is the copy the x/r update made of
// it); block 0 stores the sums in sc->red[0..1], beta and sc->rz = r.z_new.
hipError_t launch_cg_update_p_flex(hipStream_t s, int64_t n, Scalars *sc, const float *z, double *p,
                                   const Reducer &red, int nrz, const int *skip = nullptr);
// The same for an FP64 preconditioner: r.z as nrz block partials (left by
// launch_cheb_last_dot), beta = r.z / sc->rz_old as FIN_RZ forms it; block 0
// stores sc->rz_new, beta and sc->rz = r.z.
hipError_t launch_cg_update_p_rz(hipStream_t s, int64_t n, Scalars *sc, const double *z, double *p,
                                 const Reducer &red, int nrz, const int *skip = nullptr);
// Degree-1 post-smoothing's update with the V-cycle's r.z: x += res dinv
// inv_theta, and r.x as block partials in red (value 0 of each slot) in
// launch_dot's order and grid, so that their sum is bit for bit the one of
// launch_cheb_start + launch_dot; the count goes to *nparts (no finalize).
hipError_t launch_cheb_last_dot(hipStream_t s, int64_t n, const double *res, const double *dinv, double inv_theta,
                                double *x, const double *r, const Reducer &red, int *nparts,
                                const int *skip = nullptr);
// Chebyshev first step from x = 0: d = r dinv / theta; x = d; res = r
hipError_t launch_cheb_first(hipStream_t s, int64_t n, const double *r, const double *dinv,
                             double inv_theta, double *d, double *x, double *res,
                             const int *skip = nullptr);
// d = res dinv / theta; x += d
hipError_t launch_cheb_start(hipStream_t s, int64_t n, const double *res, const double *dinv,
                             double inv_theta, double *d, double *x, const int *skip = nullptr);
hipError_t launch_cheb_first(hipStream_t s, int64_t n, const float *r, const float *dinv,
                             float inv_theta, float *d, float *x, float *res, const int *skip = nullptr);
hipError_t launch_cheb_start(hipStream_t s, int64_t n, const float *res, const float *dinv,
                             float inv_theta, float *d, float *x, const int *skip = nullptr);
// out = (float) in, and out = (double) in
hipError_t launch_convert(hipStream_t s, int64_t n, const double *in, float *out,
                          const int *skip = nullptr);
hipError_t launch_convert(hipStream_t s, int64_t n, const float *in, double *out,
                          const int *skip = nullptr);
// u = sum_k alpha_k v_k, 1 <= nv <= 4
hipError_t launch_combine(hipStream_t s, int64_t n, int nv, const double *const *v, const double *alpha, double *u);
// u = sum_k alpha_k v_k over the first n of up to 4 vectors
struct Combo {
  const double *v[4];
  double alpha[4];
  int n;
};
// nv <= kMaxRed dot products a_k . b in one pass; fin.out[k] = a_k . b, each
// bit-identical to launch_dot of the same pair
struct MultiDotArgs {
  const double *a[kMaxRed];
  const double *b;
  int nv;
};
hipError_t launch_multi_dot(hipStream_t s, int64_t n, const MultiDotArgs &m, const Reducer &red, const Fin &fin);
// u_prev <- u and u <- 2 u - u_prev (previous u_prev)
hipError_t launch_extrapolate(hipStream_t s, int64_t n, double *u, double *u_prev);
// z_new = x (+ res dinv inv_theta when res is given); fin.out[0] = r.z_new,
// fin.out[1] = r.z_old with z_old the previous content of z; z = z_new (FIN_RZ_FLEX)
hipError_t launch_flex_dot(hipStream_t s, int64_t n, const float *res, const float *dinv, float inv_theta,
                           const float *x, const double *r, float *z, const Reducer &red, const Fin &fin,
                           const int *skip = nullptr);

// multigrid transfers
hipError_t launch_restrict(hipStream_t s, Grid gf, Grid gc, const double *rf, const uint8_t *fixc,
                           double *rc, const int *skip = nullptr);
hipError_t launch_prolong_add(hipStream_t s, Grid gf, Grid gc, const double *ec,
                              const uint8_t *fixf, double *xf, const int *skip = nullptr);
hipError_t launch_restrict(hipStream_t s, Grid gf, Grid gc, const float *rf, const uint8_t *fixc,
                           float *rc, const int *skip = nullptr);
hipError_t launch_prolong_add(hipStream_t s, Grid gf, Grid gc, const float *ec,
                              const uint8_t *fixf, float *xf, const int *skip = nullptr);
hipError_t launch_coarse_fixed(hipStream_t s, Grid gf, Grid gc, const uint8_t *fixf, uint8_t *fixc);
// dense coarsest-level operator, inverse and application
hipError_t launch_dense_assemble(hipStream_t s, Grid g, const double *E, const Kappa &kap,
                                 const uint8_t *fixed, double *A);
// in-place inverse of an SPD n x n matrix; work: dense_invert_work(n) doubles
// (none for small n)
size_t dense_invert_work(int n);
hipError_t launch_dense_invert(hipStream_t s, int n, double *A, double *work);
hipError_t launch_dense_matvec(hipStream_t s, int n, const double *A, const double *x, double *y,
                               const int *skip = nullptr);
hipError_t launch_dense_matvec(hipStream_t s, int n, const double *A, const float *x, float *y,
                               const int *skip = nullptr);

// The coarse end of the V-cycle in one workgroup (kernels_tail.hip): levels
// L[0] (finest of the tail) .. L[nlev-1] (coarsest, solved with Ainv).
template <typename T>
struct TailLevel {
  Grid g;
  const T *E;              // moduli incl. the level's stiffness scale
  const T *dinv;           // inverse Jacobi diagonal (0 on fixed dofs)
  const uint8_t *fixed;    // per node, bit c = dof c fixed
  T *b, *x, *res, *d0, *d1;
  int deg;                 // Chebyshev steps per smoothing on this level
};
constexpr int kTailMaxLevels = 8;
constexpr int kTailMaxDeg = 17;
constexpr int kTailThreads = 512;
template <typename T>
struct TailArgs {
  int nlev;
  TailLevel<T> L[kTailMaxLevels];
  const double *Ainv;                  // dense inverse of the coarsest operator (ncoarse^2, FP64)
  int ncoarse;
  HadaW<T> hw;                         // element matrix, sum/difference basis (see ke_code.h)
  int deg;                             // Chebyshev degree per smoothing
  T s0;                                // 1 / theta
  T c1[kTailMaxDeg], c2[kTailMaxDeg];  // step k: d_k = c1[k] d_{k-1} + c2[k] D^-1 r
  const int *skip;
};
// LDS bytes of the tail, per level E | dinv | b | x | res | d0 | d1 | fixed
// (16-byte aligned)
constexpr size_t kTailMaxLds = 158 * 1024;  // dynamic part; the kernel adds < 1 KB of static LDS
template <typename T>
__host__ __device__ inline size_t tail_level_bytes(const Grid &g) {
  return ((size_t)(g.nel() + 6 * g.ndof()) * sizeof(T) + 15) / 16 * 16 + (size_t)((g.nnodes() + 15) / 16) * 16;
}
// per-element products of one operator pass (24 values per element), sized by
// the finest (largest) level of the tail, after the levels and the solve partials
template <typename T>
__host__ __device__ inline size_t tail_scratch_bytes(const Grid &finest) {
  return (size_t)24 * finest.nel() * sizeof(T);
}
// partial sums of the coarsest solve (kColParts per row)
constexpr int kColParts = 4;
template <typename T>
__host__ __device__ inline size_t tail_solve_bytes(int ncoarse) {
  return (size_t)kColParts * ncoarse * sizeof(double);  // FP64 in every precision
}
// ---------------------------------------------------------------------------
// Grouped launches (kernels_*.hip): the problems of a group have identical
// grids and launch shapes, so one launch serves all of them -- the kernel takes
// a table of per-problem arguments by value and blockIdx.z picks the entry.
// Each problem's blocks do exactly what its own launch would (same partial
// sums, same order), so results are bit-identical to one launch per problem.
constexpr int kMaxGroup = 8;
template <class A>
struct GroupTab {
  A v[kMaxGroup];
};
// defer_parts (STORE_DOT, RESID_FLEX): no finalize, as for launch_ku
template <typename T>
hipError_t launch_ku_group(hipStream_t s, KuEpi epi, int G, const KuArgsT<T> *a, const KappaT<T> &kap,
                           const Reducer *red, const Fin *fin, int shape, int *defer_parts = nullptr);
// finalize of G reductions of nparts partials each (partials of red[i], skip[i])
hipError_t launch_finalize_group(hipStream_t s, int G, const Reducer *red, int nparts, int n, const Fin *fin,
                                 const int *const *skip);
struct XrArgs {
  Scalars *sc;
  double *x, *r;
  const double *p, *q;
  float *r32;
  const int *skip;
};
hipError_t launch_cg_update_xr_group(hipStream_t s, int G, int64_t n, const XrArgs *a, const Reducer *red,
                                     const Fin *fin);
// launch_cg_update_xr_pq for each problem of a group (p.q as npq partials in
// red[i], r.r to value 1 of each slot and its finalize)
hipError_t launch_cg_update_xr_group_pq(hipStream_t s, int G, int64_t n, const XrArgs *a, const Reducer *red,
                                        int npq, const Fin *fin);
struct PArgs {
  Scalars *sc;
  const void *z;  // double, or float when zsingle
  double *p;
  const int *skip;
};
hipError_t launch_cg_update_p_group(hipStream_t s, int G, int64_t n, bool zsingle, const PArgs *a, int first);
// launch_cg_update_p_flex for each problem of a group (z in single precision)
hipError_t launch_cg_update_p_flex_group(hipStream_t s, int G, int64_t n, const PArgs *a, const Reducer *red,
                                         int nrz);
struct FlexArgs {
  const float *res, *dinv, *x;
  const double *r;
  float *z;
  const int *skip;
};
hipError_t launch_flex_dot_group(hipStream_t s, int G, int64_t n, float inv_theta, const FlexArgs *a,
                                 const Reducer *red, const Fin *fin);
template <typename T>
struct ChebStartArgs {
  const T *res, *dinv;
  T *d, *x;
  const int *skip;
};
template <typename T>
hipError_t launch_cheb_start_group(hipStream_t s, int G, int64_t n, T inv_theta, const ChebStartArgs<T> *a);
struct DotArgs {
  const double *a, *b;
  const int *skip;
};
hipError_t launch_dot_group(hipStream_t s, int G, int64_t n, const DotArgs *a, const Reducer *red, const Fin *fin);
template <typename T>
struct TransferArgs {
  const T *in;
  const uint8_t *fixed;  // fixed flags of the output level
  T *out;
  const int *skip;
};
template <typename T>
hipError_t launch_restrict_group(hipStream_t s, int G, Grid gf, Grid gc, const TransferArgs<T> *a);
template <typename T>
hipError_t launch_prolong_add_group(hipStream_t s, int G, Grid gf, Grid gc, const TransferArgs<T> *a);
template <typename T>
struct MatvecArgs {
  const double *A;
  const T *x;
  T *y;
  const int *skip;
};
template <typename T>
hipError_t launch_dense_matvec_group(hipStream_t s, int G, int n, const MatvecArgs<T> *a);
// the restriction of r_f onto the coarsest level and x = Ainv of it in one
// launch (the coarsest right-hand side is not stored); n = gc.ndof()
template <typename T>
hipError_t launch_restrict_solve(hipStream_t s, Grid gf, Grid gc, const T *rf, const uint8_t *fixc, int n,
                                 const double *A, T *y, const int *skip);
template <typename T>
struct RestrictSolveArgs {
  const T *rf;
  const uint8_t *fixed;  // of the coarsest level
  const double *A;
  T *y;
  const int *skip;
};
template <typename T>
hipError_t launch_restrict_solve_group(hipStream_t s, int G, Grid gf, Grid gc, int n,
                                       const RestrictSolveArgs<T> *a);

hipError_t launch_zero_fixed_group(hipStream_t s, int G, int64_t nnodes, const uint8_t *const *fixed,
                                   double *const *v);
struct CgStartArgs {
  Scalars *sc;
  double rtol2;
  int max_iters;
};
hipError_t launch_cg_start_group(hipStream_t s, int G, const CgStartArgs *a);
struct ConvertArgs {
  const double *in;
  float *out;
  const int *skip;
};
hipError_t launch_convert_group(hipStream_t s, int G, int64_t n, const ConvertArgs *a);
hipError_t launch_extrapolate_group(hipStream_t s, int G, int64_t n, double *const *u, double *const *u_prev);
hipError_t launch_combine_group(hipStream_t s, int G, int64_t n, const Combo *c, double *const *u);
hipError_t launch_multi_dot_group(hipStream_t s, int G, int64_t n, const MultiDotArgs *m, const Reducer *red,
                                  const Fin *fin);
// dst[i] <- src[i] (bytes, a multiple of 4); src == NULL: dst[i] <- 0
hipError_t launch_copy_group(hipStream_t s, int G, int64_t bytes, const void *const *src, void *const *dst);

struct ModulusArgs {
  const double *xphys;
  double E0, Emin, penal;
  double *E;
  float *E32;  // may be NULL
};
hipError_t launch_simp_modulus_group(hipStream_t s, int G, int64_t nel, const ModulusArgs *a);
hipError_t launch_coarsen_moduli_group(hipStream_t s, int G, Grid gf, Grid gc, const double *const *Ef,
                                       double *const *Ec, float *const *Ec32);
struct DiagArgs {
  const double *E;
  Kappa kap;
  const uint8_t *fixed;
  double *dinv;
  float *dinv32;  // may be NULL
};
hipError_t launch_diag_group(hipStream_t s, int G, Grid g, const DiagArgs *a);
struct AssembleArgs {
  const double *E;
  Kappa kap;
  const uint8_t *fixed;
  double *A;
};
hipError_t launch_dense_assemble_group(hipStream_t s, int G, Grid g, const AssembleArgs *a);
// G in-place inversions of n x n SPD matrices A[i] (work[i]: dense_invert_work(n) doubles)
hipError_t launch_dense_invert_group(hipStream_t s, int G, int n, double *const *A, double *const *work);

template <typename T>
hipError_t launch_vcycle_tail_t(hipStream_t s, const TailArgs<T> &a);

// Grouped CG over contexts (topo.cpp), used by the batch: the members share the
// group's stream; key "" = the context cannot be grouped.
struct Group {
  std::vector<topo_ctx *> c;
  hipStream_t s = nullptr;
  int n() const { return (int)c.size(); }
};
std::string group_key(const topo_ctx *ctx);
void group_adopt_shapes(topo_ctx *dst, const topo_ctx *src);
void ctx_set_stream(topo_ctx *ctx, hipStream_t s);
Grid ctx_grid(const topo_ctx *ctx);
// graph/exec: the captured chunk of grouped CG iterations (made on first use,
// owned by the caller, kept together as the single-context path keeps its own)
topo_status group_pcg(Group &G, hipGraph_t *graph, hipGraphExec_t *exec, hipStream_t cap_stream,
                      topo_solve_stats *stats);
topo_status iterate_pre(topo_ctx *ctx, double *d_x, hipEvent_t *ev);
topo_status iterate_post(topo_ctx *ctx, double *d_x, const topo_solve_stats &ss, hipEvent_t *ev,
                         topo_iter_stats *o);
void fill_stats(const topo_ctx *ctx, const topo_solve_stats &ss, hipEvent_t *ev, topo_iter_stats *o);
// iterate_pre / iterate_post of every member of a group, one launch per step
// for the whole group (ev: 6 events of the group; o[i] may be NULL); only for
// groups in lockstep (group_lockstep)
bool group_lockstep(const Group &G);
topo_status group_pre(const Group &G, double *const *d_x, hipEvent_t *ev);
topo_status group_post(const Group &G, double *const *d_x, const topo_solve_stats *ss, hipEvent_t *ev,
                       topo_iter_stats *const *o);
// raises the kernel's dynamic LDS limit (call once before launching)
template <typename T>
hipError_t prepare_vcycle_tail_t(size_t smem_bytes);

// sensitivities: ce = u_e^T KE u_e, dc = -p xphys^(p-1) (E0-Emin) ce
hipError_t launch_sensitivity(hipStream_t s, Grid g, const Kappa &kap, const double *u,
                              const double *xphys, double E0, double Emin, double penal, double *ce,
                              double *dc);

// filter
struct FilterArgs {
  Grid g;
  int noff;
  const int *off;       // noff x 3 (di, dj, dk)
  const double *w;      // noff weights
  const double *Hs;     // nel
  const double *sD;     // nel: design/Hs
  const int8_t *mask;   // nel
  // tiled stencil (reach R = ceil(rmin) - 1 in 1..kFilterTiledMaxR): the weight
  // of an offset d depends on |d|^2 only; wsq[q] = max(0, rmin - sqrt(q)) for
  // q < (R+1)^2 (offsets with |d|^2 >= (R+1)^2 > rmin^2 never contribute)
  int R;
  double wsq[16];
};
constexpr int kFilterTiledMaxR = 3;
hipError_t launch_filter_hs(hipStream_t s, const FilterArgs &f, double *Hs);
hipError_t launch_filter(hipStream_t s, int op, const FilterArgs &f, const double *in,
                         const double *aux, double *out);
hipError_t launch_design_scale(hipStream_t s, int64_t nel, const int8_t *mask, const double *Hs,
                               double *sD);
// grouped filter (FWD, ADJ or SENS) of G problems on one grid with the same
// stencil reach; every problem gets exactly its own launch's result
struct FilterCall {
  FilterArgs f;
  const double *in, *aux;
  double *out;
};
hipError_t launch_filter_group(hipStream_t s, int op, int G, const FilterCall *c);
struct SensArgs {
  Kappa kap;
  const double *u, *xphys;
  double E0, Emin, penal;
  double *ce, *dc;
};
hipError_t launch_sensitivity_group(hipStream_t s, int G, Grid g, const SensArgs *a);

// OC update with device-side multisection.  a (nel) holds the per-element
// coefficients x (max(0,-dc)/dv)^eta between the passes; with a == nullptr
// every pass recomputes them from x, dc and dv (the same bits).  Partials: the
// pass kernels use kOcPassBlocks x kOcStride slots, the prepare and final
// reductions kOcReduceBlocks x kMaxRed.
constexpr int kOcPassBlocks = 512, kOcReduceBlocks = 1024, kOcStride = 64;
constexpr int kOcPartials = kOcPassBlocks * kOcStride > kOcReduceBlocks * kMaxRed
                                ? kOcPassBlocks * kOcStride : kOcReduceBlocks * kMaxRed;
// Multisection passes launched for a final relative bracket width tol: from the
// initial 1e80 bracket two geometric passes (each shrinks the log-range 64-fold)
// leave a bracket within a factor 2, a relative width of at most 1/3, which each
// linear pass shrinks 64-fold; one pass spare, at most kOcMaxPasses (passes
// after convergence return at once).  10 for tol = 1e-12.
constexpr int kOcMaxPasses = 16;
inline int oc_pass_launches(double tol) {
  int n = 3;
  for (double w = 1.0 / 3.0; w >= tol && n < kOcMaxPasses; w /= 64.0) ++n;
  return n;
}
hipError_t launch_oc_prepare(hipStream_t s, int64_t nel, const double *x, const double *dc,
                             const double *dv, const int8_t *mask, double eta, double target,
                             double *a, Scalars *sc, const Reducer &red);
hipError_t launch_oc_pass(hipStream_t s, int64_t nel, const double *x, const double *a,
                          const double *dc, const double *dv, const int8_t *mask, double move,
                          double eta, double tol, Scalars *sc, const Reducer &red);
hipError_t launch_oc_final(hipStream_t s, int64_t nel, const double *x, const double *a,
                           const double *dc, const double *dv, const int8_t *mask, double move,
                           double eta, double *xnew, Scalars *sc, const Reducer &red);
// prepare, the multisection passes and the final update of G problems with nel
// elements each, every launch shared by the group (a: stored coefficients)
struct OcArgs {
  const double *x, *dc, *dv;
  const int8_t *mask;
  double move, eta, tol, target;
  double *a, *xnew;
  Scalars *sc;
};
hipError_t launch_oc_update_group(hipStream_t s, int G, int64_t nel, const OcArgs *o, const Reducer *red);

}  // namespace topo
