/*
 * topo.h -- C ABI of libtopo: the per-iteration hot path of 3D SIMP compliance
 * minimisation on a structured grid of 8-node trilinear hexahedra (PyTopo3D,
 * arXiv 2504.05604), implemented with hand-written HIP kernels for gfx950.
 *
 * Problem statement (paper, Finite Element Analysis / Optimality Criteria /
 * Sensitivity Filtering sections): a nelx x nely x nelz grid of unit hexahedra,
 * element moduli E_e = Emin + rho_e^p (E0 - Emin) (modified SIMP), equilibrium
 * K(E) u = f with fixed displacements applied by elimination, compliance
 * c = f^T u, element sensitivities, a cone-weight filter of radius rmin, and an
 * Optimality Criteria update with move limits under a volume fraction that
 * excludes passive (obstacle) elements.
 *
 * Numbering (the paper leaves it open):
 *   element e = i + nelx*(j + nely*k),
 *   node    n = i + (nelx+1)*(j + (nely+1)*k),
 *   dof       = 3*n + c  (c = 0,1,2 for x,y,z; node-interleaved "AoS").
 * Local element node order: (0,0,0),(1,0,0),(1,1,0),(0,1,0),(0,0,1),(1,0,1),
 * (1,1,1),(0,1,1).
 *
 * Pointers: arguments named d_* are DEVICE pointers owned by the caller
 * (contiguous FP64 arrays of the stated length, allocated on the device the
 * context was created on); h_* are HOST pointers.  topo_setup copies every host
 * array it is given; the context owns all its device workspaces.
 *
 * Streams and threads: every call enqueues its work on the stream given to
 * topo_setup (NULL = the default stream) and returns after enqueueing, except
 * calls that write h_* outputs, which synchronise that stream.  A context must
 * not be used from two threads at once.
 *
 * Errors: no call aborts or throws; a non-OK status leaves a message retrievable
 * with topo_last_error() (thread-local).  Argument validation happens before
 * any device work.
 */
#ifndef TOPO_H
#define TOPO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct topo_ctx topo_ctx; /* opaque, library-owned */

typedef enum {
  TOPO_OK = 0,
  TOPO_EINVAL = 1,          /* invalid argument or problem definition        */
  TOPO_ENOMEM = 2,          /* device allocation failed                      */
  TOPO_EDEVICE = 3,         /* HIP runtime error                             */
  TOPO_ENOTCONVERGED = 4,   /* solver hit max_iters; outputs hold last iterate */
  TOPO_EUNSUPPORTED = 5     /* option combination not implemented            */
} topo_status;

/* filter modes (Sensitivity Filtering section) */
enum { TOPO_FILTER_DENSITY = 0, TOPO_FILTER_SENSITIVITY = 1 };
/* volume target of the OC update (Optimality Criteria section; the paper does
 * not say how obstacle elements count).  DESIGN: the design-element sum of the
 * physical density equals volfrac * (number of design elements), passive
 * elements outside both sides.  ALL: the sum over every element (fixed-solid
 * elements count 1, fixed-void 0) equals volfrac * nel, i.e. the design-element
 * sum equals volfrac * nel - (number of fixed-solid elements). */
enum { TOPO_VOL_DESIGN = 0, TOPO_VOL_ALL = 1 };
/* filter operations for topo_filter */
enum {
  TOPO_FILTER_FWD = 0,  /* out = (H in)/Hs, passive elements reset to 0 (void) / 1 (solid) */
  TOPO_FILTER_ADJ = 1,  /* out = H (in_D / Hs): in restricted to design elements          */
  TOPO_FILTER_SENS = 2, /* out = H (aux * in) / (Hs * max(1e-3, aux)); aux = x             */
  TOPO_FILTER_VOLW = 3  /* out = H (1_D / Hs): filtered volume weights (in, aux unused)    */
};
/* precision of the multigrid preconditioner.  FP32: smoothing, transfers and
 * the coarse solve run in single precision (FP32 accumulation) and the CG
 * recurrence switches to the flexible (Polak-Ribiere) update; the CG operator,
 * vectors, inner products and stopping test stay FP64, so the solution meets
 * the same FP64 residual tolerance.  BF16: as FP32, and every smoothing
 * operator pass multiplies BF16-rounded element matrix and displacements on the
 * matrix cores (FP32 accumulation). */
enum { TOPO_PREC_FP64 = 0, TOPO_PREC_FP32 = 1, TOPO_PREC_BF16 = 2 };
/* K.u kernels (Finite Element Analysis section: y = sum_e E_e KE u_e, never assembled).
 * NODE: one thread per node column applies the 24 x 24 element matrix rows of
 * the 8 elements around each node.  ELEMENT: one thread per element column works
 * in the per-axis sum/difference basis of the element's corners, where KE splits
 * into eight 3 x 3 parity blocks (21 multiply-adds per element), and neighbouring
 * threads add their corner contributions through LDS.  AUTO: ELEMENT. */
enum { TOPO_KU_AUTO = 0, TOPO_KU_NODE = 1, TOPO_KU_ELEMENT = 2 };
/* preconditioner of the conjugate-gradient solve.  LEARNED: the convolutional
 * network attached with topo_set_nn (see below), used inside flexible CG with a
 * restart on the multigrid preconditioner when the safeguard fails. */
enum { TOPO_PRECOND_JACOBI = 0, TOPO_PRECOND_MG = 1, TOPO_PRECOND_LEARNED = 2 };

/* Problem definition; all arrays are host arrays copied by topo_setup. */
typedef struct {
  int32_t nelx, nely, nelz;   /* elements per axis, each >= 1                        */
  double E0, Emin;            /* solid and void moduli, E0 > Emin > 0                */
  double nu;                  /* Poisson ratio, -1 < nu < 0.5                        */
  double penal;               /* SIMP penalty p >= 1                                 */
  double rmin;                /* filter radius in element units, > 0                 */
  double volfrac;             /* volume fraction of the design elements, (0, 1]      */
  double move;                /* OC move limit, > 0                                  */
  double eta;                 /* OC damping exponent, > 0                            */
  int32_t filter;             /* TOPO_FILTER_DENSITY | TOPO_FILTER_SENSITIVITY       */
  int32_t vol_mode;           /* TOPO_VOL_DESIGN (0) | TOPO_VOL_ALL (1)               */
  const int8_t *mask;         /* nel entries: 0 design, 1 void, 2 solid; NULL = all design */
  const int64_t *fixed_dofs;  /* n_fixed constrained dofs (homogeneous), any order   */
  int64_t n_fixed;
  const double *f;            /* ndof nodal loads; entries on fixed dofs are ignored */
} topo_problem;

/* Solver options; topo_default_opts fills every field. */
typedef struct {
  int32_t precision;          /* TOPO_PREC_*                                          */
  int32_t precond;            /* TOPO_PRECOND_*                                       */
  int32_t mg_levels;          /* 0 = automatic (coarsest <= mg_max_coarse_dof)         */
  int32_t mg_max_coarse_dof;  /* automatic depth: stop coarsening at or below this     */
  int32_t cheb_degree;        /* Chebyshev smoother degree per pre/post smoothing      */
  int32_t cheb_degree_coarse; /* the same below the finest level (0: cheb_degree)        */
  double rtol;                /* stop when ||r||_2 <= rtol ||f||_2 (free dofs)         */
  int32_t max_iters;          /* CG iteration cap per solve                           */
  int32_t warm_start;         /* topo_iterate: 0 start each solve from zero, 1 from the
                                 last u, 2 from the extrapolation 2 u_k - u_{k-1}, 3 from
                                 the combination of the last 4 solutions closest to the
                                 new solution in the new operator's energy norm          */
  double oc_tol;              /* relative width of the final multiplier bracket        */
  int32_t check_every;        /* CG iterations per chunk; the host checks convergence
                                 after one or more chunks (the device stops iterating
                                 at convergence within a chunk)                        */
  int32_t use_graphs;         /* replay chunks of CG iterations from a captured HIP graph */
  int32_t nn_max_iters;       /* LEARNED: flexible-CG iterations before the solve restarts
                                 on the multigrid preconditioner                       */
  int32_t autotune;           /* 1: at setup, take the K.u launch shapes found earlier in
                                 this process for the same grids, precision and kernel
                                 family, else time every shape on this problem's grids
                                 and keep (and remember) the fastest; 2: always time
                                 afresh and replace what is remembered; 0: shapes by
                                 grid size                                              */
  int32_t coarse_tail_nodes;  /* multigrid levels (below the finest) with at most this many
                                 nodes run as one single-workgroup launch; 0 = off        */
  int32_t mfma_smoothing;     /* FP32 preconditioner: smoothing operator passes on the FP32
                                 matrix cores (else the vector-unit kernels)              */
  int32_t ku_kernel;          /* TOPO_KU_*: which matrix-free K.u kernel the solver runs;
                                 every choice computes the same product up to rounding    */
  int32_t ku_shape;           /* -1: launch shapes by grid size (or autotuned); else one
                                 launch shape for every level and the CG product:
                                 0..3 node-column kernel, nodes per thread column x
                                 threads = 8x256, 8x128, 2x128, 1x64; 6..14 element-column
                                 kernel, node planes per slab x tile = 8x32x8, 8x16x16,
                                 4x16x8 (next plane loaded ahead), 2x8x8 (ahead), 1x8x8,
                                 8x32x8 (ahead), 8x16x16 (ahead), 8x32x8 (planes staged
                                 through LDS), 8x16x16 (staged); 4 and 5, the matrix-core
                                 kernels, are chosen through precision / mfma_smoothing  */
  int32_t coarse_refresh;     /* topo_iterate: recompute the coarsest level's dense inverse
                                 every this many SIMP iterations (1 = every iteration); in
                                 between the last one (an SPD matrix, so the V-cycle stays
                                 a valid preconditioner) serves; other entry points always
                                 recompute it                                            */
  int32_t cheb_degree_level[8]; /* per multigrid level, finest first: a Chebyshev degree
                                 in [1, 16] that replaces cheb_degree / cheb_degree_coarse
                                 on that level; 0 = not set (the level above the exact
                                 coarsest solve never smooths more than 16 steps)      */
  int32_t group_launch;       /* topo_iterate_batch: problems with equal grids (multigrid
                                 preconditioner in FP64 or FP32 on the element-column
                                 kernel) are solved together, up to 8 per group, every CG
                                 pass one launch for the whole group (results identical to
                                 solving each alone with the group's launch shapes);
                                 0 = every problem on its own stream                  */
  double cheb_upper;          /* the smoothers' Chebyshev interval is [c lb / 30, c lb], c =
                                 cheb_upper in (0, 1], lb = lambda_max(diag(KE)^-1 KE), which
                                 bounds lambda_max(D^-1 A) for any densities (c = 1, the
                                 default, is valid always).  A smaller c smooths the top
                                 of the spectrum harder and fits while lambda_max(D^-1 A)
                                 stays below c lb: filtered SIMP designs measure 0.58-0.72,
                                 unfiltered random densities up to 0.85, an isolated solid
                                 element in void 1.  Convergence to rtol is checked on the
                                 true residual whatever c is                           */
} topo_opts;

typedef struct {
  int32_t iters;       /* CG iterations taken (all phases)           */
  int32_t converged;   /* 1 if relres <= rtol                        */
  double relres;       /* ||f - K u|| / ||f|| (recursive residual)   */
  double ms;           /* wall time of the solve on the stream       */
  int32_t fallbacks;   /* LEARNED: restarts on the multigrid preconditioner */
  int32_t learned_iters; /* LEARNED: iterations taken with the network  */
} topo_solve_stats;

typedef struct {
  double c;            /* compliance f^T u                                      */
  double volume;       /* design-element sum of the physical density after update */
  double change;       /* max |x_new - x|                                       */
  double lambda;       /* volume multiplier                                     */
  int32_t pcg_iters;   /* CG iterations of this iteration's solve               */
  int32_t converged;
  double relres;
  double ms_total, ms_filter, ms_solve, ms_sens, ms_oc; /* phase times (hipEvents) */
  int32_t fallbacks;   /* LEARNED: restarts of this iteration's solve on the multigrid
                          preconditioner (a safeguard event, not an error)         */
  int32_t learned_iters; /* LEARNED: CG iterations of this solve taken with the network */
} topo_iter_stats;

/* Fills *opts with defaults: FP64, MG, automatic depth (coarsest <= 1500 dofs),
 * Chebyshev degree 1 on the finest level and 4 below (cheb_degree_coarse),
 * rtol 1e-8, max_iters 1000, projected warm start (3), oc_tol 1e-12,
 * check_every 3, use_graphs 1, nn_max_iters 200, autotune 0, coarse_tail_nodes 0,
 * mfma_smoothing 0, ku_kernel TOPO_KU_AUTO, ku_shape -1, coarse_refresh 1,
 * cheb_degree_level all 0, group_launch 1, cheb_upper 1. */
void topo_default_opts(topo_opts *opts);

/* Validates the problem, copies its arrays to the device, builds the element
 * stiffness matrix (Finite Element Analysis section: precomputed H8 matrix), the
 * filter stencil and row sums (Sensitivity Filtering section), the multigrid
 * hierarchy and all workspaces.  hip_stream is a hipStream_t or NULL.
 * Errors: TOPO_EINVAL (sizes < 1, non-positive rmin/move/eta, volfrac outside
 * (0,1], Emin <= 0 or >= E0, mask codes outside {0,1,2}, unknown vol_mode, a
 * TOPO_VOL_ALL target not above zero (the fixed-solid elements alone exceed
 * volfrac * nel), fixed dofs out of range, fewer than 6 fixed dofs, no design
 * element, NULL f), TOPO_ENOMEM,
 * TOPO_EDEVICE.  On error *out is NULL. */
topo_status topo_setup(const topo_problem *problem, const topo_opts *opts, void *hip_stream,
                       topo_ctx **out);

/* Releases the context and its device memory (NULL is accepted). */
void topo_destroy(topo_ctx *ctx);

/* Thread-local message of the last non-OK status ("" if none). */
const char *topo_last_error(void);

/* Sizes of the problem held by ctx (any pointer may be NULL). */
topo_status topo_sizes(const topo_ctx *ctx, int64_t *nel, int64_t *ndof, int32_t *mg_levels);

/* Matrix-free operator (Finite Element Analysis section, K U = F with the
 * constraints eliminated): d_y = K(E(d_xphys)) d_u on free dofs with the fixed
 * entries of d_u taken as zero, and d_y = d_u on fixed dofs (identity rows).
 * E = Emin + xphys^p (E0 - Emin).  d_xphys: nel, d_u, d_y: ndof (must not alias). */
topo_status topo_apply_K(topo_ctx *ctx, const double *d_xphys, const double *d_u, double *d_y);

/* Solves K(E(d_xphys)) u = f on the free dofs by preconditioned conjugate
 * gradients (Finite Element Analysis section: the linear solve of K U = F).
 * d_u (ndof) holds the initial guess on entry (its fixed entries are zeroed)
 * and the solution on exit.  Returns TOPO_ENOTCONVERGED if max_iters was hit
 * (d_u then holds the last iterate).  h_stats may be NULL. */
topo_status topo_solve(topo_ctx *ctx, const double *d_xphys, double *d_u, topo_solve_stats *h_stats);

/* One application of the solver's preconditioner z = M r for the operator of
 * d_xphys: the symmetric multigrid V-cycle (TOPO_PRECOND_MG: Chebyshev-Jacobi
 * smoothing, trilinear transfers, rediscretised coarse levels, exact coarsest
 * solve) or z = r / diag(K) (TOPO_PRECOND_JACOBI).  This is the inner operator
 * of topo_solve, exposed so it can be checked on its own.  d_r must be zero on
 * fixed dofs; d_z receives zeros there.  d_xphys: nel; d_r, d_z: ndof. */
topo_status topo_apply_precond(topo_ctx *ctx, const double *d_xphys, const double *d_r, double *d_z);

/* Element energies and compliance sensitivities (Optimality Criteria section):
 * d_ce[e] = u_e^T KE u_e, d_dc[e] = -p xphys_e^(p-1) (E0 - Emin) ce_e (nel each);
 * *h_compliance = f^T u if h_compliance is not NULL (synchronises). */
topo_status topo_sensitivity(topo_ctx *ctx, const double *d_xphys, const double *d_u, double *d_ce,
                             double *d_dc, double *h_compliance);

/* Cone-weight filter (Sensitivity Filtering section), op = TOPO_FILTER_*.
 * d_in, d_aux, d_out: nel each; d_aux is x for TOPO_FILTER_SENS, else ignored.
 * d_out must not alias d_in or d_aux. */
topo_status topo_filter(topo_ctx *ctx, int32_t op, const double *d_in, const double *d_aux,
                        double *d_out);

/* OC update with move limits (Optimality Criteria section).  For design
 * elements x_new = clamp(x (max(0,-dc)/(lambda dv))^eta, max(0,x-move),
 * min(1,x+move)); passive elements keep x.  lambda is chosen so that the volume
 * measure sum_j dv_j x_new_j (over all elements) equals the problem's target
 * (TOPO_VOL_DESIGN: volfrac * (number of design elements); TOPO_VOL_ALL:
 * volfrac * nel - (number of fixed-solid elements)); dv is therefore the volume weight vector: H(1_D/Hs) for the
 * density filter (TOPO_FILTER_VOLW), 1 on design and 0 on passive elements for
 * the sensitivity filter.  The multiplier bracket is narrowed until its relative
 * width is below oc_tol (down to about 1e-16: the number of passes enqueued
 * grows with -log(oc_tol) and is capped at 16, enough for 1e-16 from the
 * initial [1e-40, 1e40] bracket).  d_x, d_dc, d_dv, d_xnew: nel (d_xnew must
 * not alias).
 * h_change = max |x_new - x|, h_lambda (either may be NULL; synchronises if not). */
topo_status topo_oc_update(topo_ctx *ctx, const double *d_x, const double *d_dc, const double *d_dv,
                           double *d_xnew, double *h_change, double *h_lambda);

/* The OC update of topo_oc_update without a context, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): this call allocates nothing.  Its search
 * state and partial sums live in one fixed array of the library per GPU (about
 * 260 KB, held until the process ends; its size does not depend on nel), so
 * calls that overlap on one GPU (concurrent streams or threads) race and must
 * be serialised by the caller; each call fully rewrites the state it reads.
 * Arguments: nel >= 1 elements; d_x, d_dc, d_dv, d_xnew (nel FP64 each) and
 * d_mask (nel int8: 0 design, 1 void, 2 solid) on the current device, d_xnew
 * not aliasing an input; move, eta, oc_tol > 0; target > 0 is the volume the
 * sum of d_dv * x_new over all elements must meet (volfrac * number of design
 * elements for the density filter, plus the passive elements' d_dv * x).  The
 * update is the one topo_oc_update computes with the same inputs (same kernels
 * and order of summation).  d_result (device, 3 FP64: max |x_new - x|, the
 * volume sum_j dv_j x_new_j and lambda) may be NULL.  Enqueued on hip_stream
 * (NULL = default stream); returns without synchronising.  Errors: TOPO_EINVAL
 * (validation, before any device work), TOPO_EDEVICE. */
topo_status topo_oc_update_noalloc(int64_t nel, const double *d_x, const double *d_dc, const double *d_dv,
                                   const int8_t *d_mask, double move, double eta, double target,
                                   double oc_tol, void *hip_stream, double *d_xnew, double *d_result);

/* n_iter SIMP iterations in the order of the Workflow section (filter ->
 * modulus -> solve -> sensitivities -> filter adjoint -> OC update) on the
 * design d_x (nel, in/out).  h_stats (n_iter entries) may be NULL.  The last
 * displacement is kept in the context for the next call's warm start and can be
 * read with topo_get_displacement. */
topo_status topo_iterate(topo_ctx *ctx, double *d_x, int32_t n_iter, topo_iter_stats *h_stats);

/* Measurement helper: times `reps` back-to-back launches of the finest-level
 * matrix-free operator kernel (y = K u in the launch shape of the
 * conjugate-gradient product, with the context's current moduli and
 * displacement as operand; no reduction, so no other kernel runs between the
 * events) between two hipEvents on the context's stream; *h_ms_per_launch =
 * elapsed / reps.  Call after topo_iterate or topo_solve.  Writes only the
 * context's scratch vector. */
topo_status topo_time_operator(topo_ctx *ctx, int32_t reps, double *h_ms_per_launch);

/* Forgets every launch shape the autotuner (topo_opts.autotune 1) remembers in
 * this process; contexts already set up keep theirs.  Thread-safe. */
void topo_clear_tuning_cache(void);

/* Copies the context's current displacement (ndof) to d_u / physical density
 * (nel) to d_xphys; either may be NULL. */
topo_status topo_get_state(topo_ctx *ctx, double *d_u, double *d_xphys);

/* ------------------------------------------------------------------------
 * Before and after the loop (Workflow and Key Features section: STL design
 * domains in, the optimised design out as an STL mesh).  Element (i, j, k)
 * occupies [o + h i, o + h (i+1)] x ... with origin o (h_origin: 3 doubles on
 * the host, NULL = 0) and element size h > 0.
 */

/* Binary STL of the thresholded design: every face between an element with
 * d_xphys > threshold and an element at or below it (or outside the grid) as
 * two triangles with the outward unit normal, counter-clockwise seen from
 * outside; elements in numbering order, faces in the order -x, +x, -y, +y, -z,
 * +z.  The mesh is closed and encloses exactly the solid elements.  Writes
 * *h_ntri (the triangle count); if d_stl is not NULL also the whole file image
 * into d_stl (device, stl_bytes >= 84 + 50 ntri: 80-byte header, uint32 count,
 * 50-byte triangle records).  Calling with d_stl NULL first gives the size.
 * d_xphys: nel FP64 (device).  Allocates temporary device memory; synchronises
 * hip_stream.  Errors: TOPO_EINVAL (sizes, NULL arguments, buffer too small,
 * more than 2^32 - 1 triangles), TOPO_ENOMEM, TOPO_EDEVICE. */
topo_status topo_surface_stl(int32_t nelx, int32_t nely, int32_t nelz, const double *d_xphys, double threshold,
                             const double *h_origin, double h, void *hip_stream, uint8_t *d_stl,
                             int64_t stl_bytes, int64_t *h_ntri);

/* Element mask from a closed triangle mesh (an STL design domain or obstacle):
 * d_mask[e] = code_inside where the element's centroid lies inside the mesh
 * (odd number of crossings of the ray from the centroid along +z), else
 * code_outside; e.g. a domain gives 0 (design) inside and 1 (void) outside for
 * topo_problem.mask.  d_tri: ntri x 3 vertices x (x, y, z) float32 (device), in
 * any orientation.  *h_bad_columns (may be NULL) counts the element columns
 * whose vertical line crossed the mesh an odd number of times (or more than 128
 * times): zero for a closed mesh.  Allocates temporary device memory;
 * synchronises hip_stream.  Errors: TOPO_EINVAL, TOPO_ENOMEM, TOPO_EDEVICE. */
topo_status topo_voxelize(const float *d_tri, int64_t ntri, int32_t nelx, int32_t nely, int32_t nelz,
                          const double *h_origin, double h, int8_t code_inside, int8_t code_outside,
                          void *hip_stream, int8_t *d_mask, int64_t *h_bad_columns);

/* ------------------------------------------------------------------------
 * Batches of independent problems.  Each problem gets its own context on its
 * own stream (created by the batch), so kernels of different problems overlap
 * on the device; topo_iterate_batch drives them from a pool of n_threads host
 * threads (0 = min(8, n)), largest problems first.  Results of every problem
 * are those of topo_iterate on a context of its own with the same options.
 */
typedef struct topo_batch topo_batch;
/* Sets up n problems (the array is read during the call only).  Errors as for
 * topo_setup, with the failing problem's index in the message. */
topo_status topo_setup_batch(const topo_problem *problems, int32_t n, const topo_opts *opts, int32_t n_threads,
                             topo_batch **out);
void topo_destroy_batch(topo_batch *batch);
/* The context of problem i (owned by the batch), e.g. for topo_get_state. */
topo_status topo_batch_context(topo_batch *batch, int32_t i, topo_ctx **out);
/* n_iter SIMP iterations of every problem i on d_x[i] (device, nel_i, in/out);
 * h_stats (n * n_iter entries, problem-major) may be NULL.  Returns after all
 * problems are done; TOPO_ENOTCONVERGED if any solve hit max_iters. */
topo_status topo_iterate_batch(topo_batch *batch, double *const *d_x, int32_t n_iter, topo_iter_stats *h_stats);

/* ------------------------------------------------------------------------
 * Learned preconditioner.  A three-level convolutional encoder-decoder on the
 * node grid maps the node density (mean of the adjacent elements' physical
 * densities) and the residual scaled by its root-mean-square to a correction
 * z ~ K^{-1} r, rescaled and zeroed on fixed dofs.  Layers (3x3x3 zero-padded
 * cross-correlations, ReLU after each but the up layers and the head):
 *   enc0a 4->c0, enc0b c0->c0 (= s0), down1 c0->c1 stride 2, enc1b c1->c1 (= s1),
 *   down2 c1->c2 stride 2, enc2b c2->c2, up1 = transpose of a stride-2
 *   convolution c2->c1 (+bias), dec1 on [up1, s1] 2c1->c1, up0 c1->c0 (+bias),
 *   dec0 on [up0, s0] 2c0->c0, head 1x1x1 c0->3.
 * Coarse grids have ceil(n/2) nodes per axis.  Parameters are one FP32 blob:
 * per layer its weight [c_out][c_in][taps] (taps z-major, then y, then x) and
 * its bias, in the order above; an up layer stores the weight of the stride-2
 * convolution it transposes, [c_coarse][c_fine][27], and a c_fine bias.  With
 * (16, 32, 64) channels there are 354611 parameters.
 *
 * Network activations are channel-major over a batch: [C][batch][V] with
 * V = NX*NY*NZ nodes, x fastest (node numbering above).  nodes[3] = (NX, NY, NZ).
 * Training samples are stored per sample: rho [n][V] (node density), r and
 * e [n][3V] (dof order), fixed [n][V] (bit c set when dof c of the node is
 * fixed).  With y = net(rho, r/s), s = rms(r), t = e/s and m the free dofs,
 * the loss of a sample is
 *   TOPO_LOSS_REL:    ||(y - t) m||^2 / ||t m||^2,
 *   TOPO_LOSS_COS:    1 - (y m).(t m) / (|y m| |t m|)
 *                     (blind to a positive scaling of y, as flexible CG is);
 * a batch's loss is the mean over its samples.
 */
typedef struct topo_nn topo_nn;
enum { TOPO_LOSS_REL = 0, TOPO_LOSS_COS = 1 };

typedef struct {
  int32_t epochs;          /* passes over the samples (a fresh shuffle each)      */
  int32_t batch;           /* samples per Adam step, 1..64                         */
  double lr, beta1, beta2, eps; /* Adam (Kingma and Ba 2015) with bias correction */
  uint64_t seed;           /* shuffle seed                                         */
  int32_t loss;            /* TOPO_LOSS_*                                          */
} topo_train_opts;

typedef struct {
  int32_t steps;           /* Adam steps taken                                     */
  double loss_first;       /* mean sample loss over the first epoch                */
  double loss_last;        /* ... over the last epoch                              */
  double ms;               /* wall time on the stream                              */
} topo_train_stats;

/* Creates a network with channels (c0, c1, c2) (NULL = 16, 32, 64) and zero
 * weights; hip_stream as in topo_setup.  Errors: TOPO_EINVAL, TOPO_ENOMEM. */
topo_status topo_nn_create(const int32_t channels[3], void *hip_stream, topo_nn **out);
void topo_nn_destroy(topo_nn *nn);
/* Arithmetic of the network's convolutions (forward, backward and inside the
 * solver): TOPO_PREC_FP32 (default; FP32 operands and accumulation) or
 * TOPO_PREC_BF16 (operands rounded to BF16 on the matrix cores, FP32
 * accumulation; activations, gradients and master weights stay FP32). */
topo_status topo_nn_set_precision(topo_nn *nn, int32_t precision);
topo_status topo_nn_n_params(const topo_nn *nn, int64_t *n);
/* Copies n = n_params FP32 parameters from the host (layout above) and resets
 * the Adam moments.  Synchronises. */
topo_status topo_nn_set_weights(topo_nn *nn, const float *h_blob, int64_t n);
topo_status topo_nn_get_weights(const topo_nn *nn, float *h_blob, int64_t n);
/* d_out[3][batch][V] = net(d_in[4][batch][V]) (raw network, no scaling). */
topo_status topo_nn_forward(topo_nn *nn, const int32_t nodes[3], int32_t batch, const float *d_in,
                            float *d_out);
/* Mean loss (TOPO_LOSS_*) of the samples h_index[0..batch) (host indices into
 * n_samples) and its gradient with respect to the parameters (d_grad, n_params;
 * may be NULL).  *h_loss may be NULL.  Synchronises. */
topo_status topo_nn_loss_grad(topo_nn *nn, const int32_t nodes[3], int64_t n_samples, const float *d_rho,
                              const float *d_r, const float *d_e, const uint8_t *d_fixed, int32_t batch,
                              const int32_t *h_index, int32_t loss_mode, double *h_loss, float *d_grad);
/* Fills *opts: 10 epochs, batch 4, lr 1e-3, betas 0.9 / 0.999, eps 1e-8, seed 0,
 * TOPO_LOSS_REL. */
void topo_default_train_opts(topo_train_opts *opts);
/* Adam training over the stored samples; the last partial batch of an epoch is
 * dropped.  h_epoch_loss (epochs entries) and h_stats may be NULL.  Synchronises. */
topo_status topo_nn_train(topo_nn *nn, const int32_t nodes[3], int64_t n_samples, const float *d_rho,
                          const float *d_r, const float *d_e, const uint8_t *d_fixed,
                          const topo_train_opts *opts, double *h_epoch_loss, topo_train_stats *h_stats);

/* Attaches nn (NULL detaches) as the network of TOPO_PRECOND_LEARNED for ctx.
 * The context keeps its own activation buffers; nn must outlive the attachment,
 * and later topo_nn_set_weights / topo_nn_train calls take effect at once. */
topo_status topo_set_nn(topo_ctx *ctx, topo_nn *nn);

/* Training pairs from the conjugate-gradient iterates of one density field:
 * solves K(E(d_xphys)) u* = f to min(rtol, 1e-10) with the multigrid
 * preconditioner, then for each i restarts from u = 0, takes h_iters[i] >= 0
 * iterations and stores r_i = f - K u_i and e_i = u* - u_i (= K^{-1} r_i).
 * Writes d_rho[i][V] (node density), d_r[i][3V], d_e[i][3V] (FP32) and
 * d_fixed[i][V] for i < n.  Synchronises. */
topo_status topo_nn_make_pairs(topo_ctx *ctx, const double *d_xphys, int32_t n, const int32_t *h_iters,
                               float *d_rho, float *d_r, float *d_e, uint8_t *d_fixed);

#ifdef __cplusplus
}
#endif

#endif /* TOPO_H */
