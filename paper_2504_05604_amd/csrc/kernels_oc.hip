// OC design update with move limits (Optimality Criteria section) and a
// device-side multisection search for the volume multiplier.
//
// For design element j, a_j = x_j (max(0,-dc_j)/dv_j)^eta, so the candidate at
// multiplier lambda is clamp(a_j lambda^-eta, max(0, x_j - move), min(1, x_j + move)).
// The volume V(lambda) = sum_j dv_j x_new_j is non-increasing in lambda.  Each
// pass evaluates V at kOcCand multipliers inside the current bracket (geometric
// spacing while the bracket spans more than a factor 2, linear after) and keeps
// the sub-interval in which V crosses the target; the bracket shrinks by a
// factor 64 per pass instead of 2 per bisection step, and the host never waits.
#include <algorithm>

#include "group_host.h"
#include "internal.h"
#include "reduce_dev.h"

namespace topo {

namespace {
constexpr int kBs = 256;
static_assert(kOcStride >= kOcCand, "one partial slot per candidate");
inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBs - 1) / kBs); }
}  // namespace

__device__ __forceinline__ double oc_value(double x, double a, double lam_pow, double move) {
  const double lo = fmax(0.0, x - move), hi = fmin(1.0, x + move);
  return fmin(hi, fmax(lo, a * lam_pow));
}

// a_e of a design element: read from the array the prepare pass stored, or
// (kStored false, for callers without a per-element workspace) recomputed from
// x, dc and dv by the same expression, so both give the same bits
__device__ __forceinline__ double oc_coef(double x, double dc, double dv, double eta) {
  const double B = fmax(0.0, -dc) / dv;
  return x * pow(B, eta);
}
template <bool kStored>
__device__ __forceinline__ double oc_a_of(const double *__restrict__ a, const double *__restrict__ dc,
                                          const double *__restrict__ dv, double x, double eta, int64_t e) {
  if constexpr (kStored) return a[e];
  else return oc_coef(x, dc[e], dv[e], eta);
}

// candidate c of the bracket [l1, l2] (one lane per candidate)
__device__ __forceinline__ double oc_candidate(double l1, double l2, int c) {
  const bool geo = l1 > 0.0 && l2 > 2.0 * l1;
  const double t = (double)(c + 1) / (double)(kOcCand + 1);
  return geo ? l1 * pow(l2 / l1, t) : l1 + (l2 - l1) * t;
}

__device__ __forceinline__ void oc_prepare_body(int64_t nel, const double *__restrict__ x,
                                                const double *__restrict__ dc, const double *__restrict__ dv,
                                                const int8_t *__restrict__ mask, double eta,
                                                double *__restrict__ a, double *partials) {
  double cst = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nel;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (mask[e] == 0) {
      if (a) a[e] = oc_coef(x[e], dc[e], dv[e], eta);
    } else {
      if (a) a[e] = 0.0;
      cst = fma(dv[e], x[e], cst);
    }
  }
  double v[1] = {cst};
  block_reduce_store<1, false>(v, partials, blockIdx.x);
}
__global__ void oc_prepare_kernel(int64_t nel, const double *__restrict__ x,
                                  const double *__restrict__ dc, const double *__restrict__ dv,
                                  const int8_t *__restrict__ mask, double eta,
                                  double *__restrict__ a, double *partials) {
  oc_prepare_body(nel, x, dc, dv, mask, eta, a, partials);
}
__global__ void oc_prepare_group_kernel(int64_t nel, GroupTab<OcArgs> t, GroupTab<double *> part) {
  const OcArgs &o = t.v[blockIdx.z];
  oc_prepare_body(nel, o.x, o.dc, o.dv, o.mask, o.eta, o.a, part.v[blockIdx.z]);
}

// one wave: lane 0 the scalars, lane c candidate c
__device__ __forceinline__ void oc_init_body(Scalars *sc, double target) {
  constexpr double l1 = 1e-40, l2 = 1e40;  // the multiplier is positive; l1 stands for the lower end 0
  const int c = threadIdx.x;
  if (c == 0) {
    sc->target = target;
    sc->l1 = l1;
    sc->l2 = l2;
    sc->oc_done = 0;
    sc->oc_pass = 0;
  }
  if (c < kOcCand) sc->oc_lam[c] = oc_candidate(l1, l2, c);
}
__global__ void oc_init_kernel(Scalars *sc, double target) { oc_init_body(sc, target); }
// one wave per problem
__global__ void oc_init_group_kernel(GroupTab<OcArgs> t) {
  const OcArgs &o = t.v[blockIdx.x];
  oc_init_body(o.sc, o.target);
}

// Partial volumes of one block for every candidate multiplier.  A thread takes
// its elements e0, e0 + S, e0 + 2S, ... (S threads in the grid) in groups of
// kOcGroup: the loads of the next group are issued before the arithmetic of the
// current one, and each candidate's lambda^-eta, read once from LDS, serves the
// whole group.  Elements outside the design (mask) or past nel contribute exact
// zeros (x_new of x = a = 0 is 0, weighted by 0), so every accumulator adds the
// same terms in the same order as a plain element-by-element loop.
constexpr int kOcGroup = 4;
template <bool kStored>
__device__ __forceinline__ void oc_pass_body(int64_t nel, const double *__restrict__ x,
                                             const double *__restrict__ a, const double *__restrict__ dc,
                                             const double *__restrict__ dv, const int8_t *__restrict__ mask,
                                             double move, double eta, const Scalars *sc, double *partials) {
  if (sc->oc_done) return;
  __shared__ double lampow[kOcCand];
  __shared__ double sh[kOcCand][kBs / 64];
  for (int c = threadIdx.x; c < kOcCand; c += blockDim.x) lampow[c] = pow(sc->oc_lam[c], -eta);
  __syncthreads();
  double part[kOcCand];
#pragma unroll
  for (int c = 0; c < kOcCand; ++c) part[c] = 0.0;
  constexpr int U = kOcGroup;
  const int64_t S = (int64_t)gridDim.x * blockDim.x;
  // raw loads of a group (clamped index: in bounds, selected at use)
  struct Grp {
    double x[U], q[U], w[U];  // q: a (stored) or dc (recomputed)
    int8_t m[U];
  };
  auto fetch = [&](int64_t eb, Grp &g) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t ec = min(eb + u * S, nel - 1);
      g.x[u] = x[ec];
      g.q[u] = kStored ? a[ec] : dc[ec];
      g.w[u] = dv[ec];
      g.m[u] = mask[ec];
    }
  };
  Grp cur, nxt;
  int64_t eb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (eb < nel) fetch(eb, cur);
  for (; eb < nel; eb += U * S) {
    if (eb + U * S < nel) fetch(eb + U * S, nxt);
    double xe[U], ae[U], we[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = eb + u * S < nel && cur.m[u] == 0;
      const double ar = kStored ? cur.q[u] : oc_coef(cur.x[u], cur.q[u], cur.w[u], eta);
      xe[u] = ok ? cur.x[u] : 0.0;
      ae[u] = ok ? ar : 0.0;
      we[u] = ok ? cur.w[u] : 0.0;
    }
    // an index the compiler cannot see through: keeps the 63 reads of lampow
    // inside the loop (hoisted, they would hold 126 more registers)
    int l0 = 0;
    asm volatile("" : "+v"(l0));
#pragma unroll
    for (int c = 0; c < kOcCand; ++c) {
      const double lp = lampow[c + l0];
#pragma unroll
      for (int u = 0; u < U; ++u) part[c] = fma(we[u], oc_value(xe[u], ae[u], lp, move), part[c]);
    }
    cur = nxt;
  }
  // the wave's sums of the 64 accumulators (the last one zero) by recursive
  // halving: at distance k a lane keeps half of its current range, adds its
  // partner's copy of that half and hands the other half over, so lane c ends
  // with candidate c (63 exchanges instead of 63 separate wave reductions)
  const int lane = threadIdx.x & 63, wid = threadIdx.x / 64;
  double v[64];
#pragma unroll
  for (int c = 0; c < 64; ++c) v[c] = c < kOcCand ? part[c] : 0.0;
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) {
    const bool upper = (lane & k) != 0;
#pragma unroll
    for (int i = 0; i < k; ++i) {
      const double send = upper ? v[i] : v[k + i];
      const double keep = upper ? v[k + i] : v[i];
      v[i] = keep + __shfl_xor(send, k, 64);
    }
  }
  if (lane < kOcCand) sh[lane][wid] = v[0];
  __syncthreads();
  for (int c = threadIdx.x; c < kOcCand; c += blockDim.x) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) t += sh[c][w];
    partials[(size_t)blockIdx.x * kOcStride + c] = t;
  }
}
template <bool kStored>
__global__ __launch_bounds__(kBs) void oc_pass_kernel(int64_t nel, const double *__restrict__ x,
                                                      const double *__restrict__ a,
                                                      const double *__restrict__ dc,
                                                      const double *__restrict__ dv,
                                                      const int8_t *__restrict__ mask, double move,
                                                      double eta, const Scalars *sc,
                                                      double *partials) {
  oc_pass_body<kStored>(nel, x, a, dc, dv, mask, move, eta, sc, partials);
}
__global__ __launch_bounds__(kBs) void oc_pass_group_kernel(int64_t nel, GroupTab<OcArgs> t,
                                                            GroupTab<double *> part) {
  const OcArgs &o = t.v[blockIdx.z];
  oc_pass_body<true>(nel, o.x, o.a, o.dc, o.dv, o.mask, o.move, o.eta, o.sc, part.v[blockIdx.z]);
}

// Sums the pass partials and keeps the crossing sub-interval.  Wave w of the
// 16 reads partial rows w, w + 16, ... with lane = candidate (each load one
// contiguous row, every load of the lane in flight at once: the loop is
// unrolled to the largest count), into four running sums (row index / 16 mod
// 4); the first wave adds the 16 wave sums in a fixed pairwise order.
// nparts <= kOcPassBlocks.
constexpr int kSelThreads = 1024;
__device__ __forceinline__ void oc_select_body(int nparts, double tol, Scalars *sc, const double *partials) {
  if (sc->oc_done) return;
  constexpr int kW = kSelThreads / 64, kPer = (kOcPassBlocks + kW - 1) / kW;
  __shared__ double Vw[kW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int b = w + kW * j;
    acc[j & 3] += (b < nparts && lane < kOcCand) ? partials[(size_t)b * kOcStride + lane] : 0.0;
  }
  Vw[w][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (threadIdx.x >= 64) return;
  double t[kW];
#pragma unroll
  for (int q = 0; q < kW; ++q) t[q] = Vw[q][lane];
#pragma unroll
  for (int h = kW / 2; h >= 1; h /= 2)
#pragma unroll
    for (int q = 0; q < h; ++q) t[q] += t[q + h];
  const double Vc = t[0] + sc->vconst;
  // the crossing: V is non-increasing in lambda, and the bracket keeps the last
  // candidate above the target and the first one at or below it (a scan over
  // the candidates stopping at the first one not above); one wave, lane = candidate
  const double target = sc->target;
  const bool above = lane < kOcCand && Vc > target;
  const unsigned long long m = __ballot(above);
  const int first_below = __builtin_ctzll(~m);  // lane kOcCand (never above) bounds it
  double l1 = sc->l1, l2 = sc->l2;
  if (first_below > 0) l1 = sc->oc_lam[first_below - 1];
  if (first_below < kOcCand) l2 = sc->oc_lam[first_below];
  const int pass = sc->oc_pass + 1;
  const bool done = (l2 - l1) / (l1 + l2) < tol || pass >= 64;
  // every lane has read what it needs (the new values depend on those reads)
  if (lane == 0) {
    sc->l1 = l1;
    sc->l2 = l2;
    sc->oc_pass = pass;
    sc->oc_done = done ? 1 : 0;
  }
  if (!done && lane < kOcCand) sc->oc_lam[lane] = oc_candidate(l1, l2, lane);
}
__global__ __launch_bounds__(kSelThreads) void oc_select_kernel(int nparts, double tol, Scalars *sc,
                                                                const double *partials) {
  oc_select_body(nparts, tol, sc, partials);
}
// one block per problem
__global__ __launch_bounds__(kSelThreads) void oc_select_group_kernel(int nparts, GroupTab<OcArgs> t,
                                                                      GroupTab<double *> part) {
  const OcArgs &o = t.v[blockIdx.x];
  oc_select_body(nparts, o.tol, o.sc, part.v[blockIdx.x]);
}

template <bool kStored>
__device__ __forceinline__ void oc_final_body(int64_t nel, const double *__restrict__ x,
                                              const double *__restrict__ a, const double *__restrict__ dc,
                                              const double *__restrict__ dv, const int8_t *__restrict__ mask,
                                              double move, double eta, double *__restrict__ xnew, Scalars *sc,
                                              double *partials) {
  const double lam = 0.5 * (sc->l1 + sc->l2);
  const double lp = pow(lam, -eta);
  double chg = 0.0, vol = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nel;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double xe = x[e];
    const double xn = mask[e] == 0 ? oc_value(xe, oc_a_of<kStored>(a, dc, dv, xe, eta, e), lp, move) : xe;
    xnew[e] = xn;
    chg = fmax(chg, fabs(xn - xe));
    vol = fma(dv[e], xn, vol);
  }
  double vm[1] = {chg};
  block_reduce_store<1, true>(vm, partials, blockIdx.x);
  double vs[1] = {vol};
  block_reduce_store<1, false>(vs, partials + 1, blockIdx.x);
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->lambda = lam;
}
template <bool kStored>
__global__ void oc_final_kernel(int64_t nel, const double *__restrict__ x,
                                const double *__restrict__ a, const double *__restrict__ dc,
                                const double *__restrict__ dv, const int8_t *__restrict__ mask,
                                double move, double eta, double *__restrict__ xnew, Scalars *sc,
                                double *partials) {
  oc_final_body<kStored>(nel, x, a, dc, dv, mask, move, eta, xnew, sc, partials);
}
__global__ void oc_final_group_kernel(int64_t nel, GroupTab<OcArgs> t, GroupTab<double *> part) {
  const OcArgs &o = t.v[blockIdx.z];
  oc_final_body<true>(nel, o.x, o.a, o.dc, o.dv, o.mask, o.move, o.eta, o.xnew, o.sc, part.v[blockIdx.z]);
}

static unsigned oc_blocks(int64_t nel, int cap) {
  unsigned nb = nblocks((nel + 3) / 4);
  if (nb > (unsigned)cap) nb = (unsigned)cap;
  return nb < 1u ? 1u : nb;
}

hipError_t launch_oc_prepare(hipStream_t s, int64_t nel, const double *x, const double *dc,
                             const double *dv, const int8_t *mask, double eta, double target,
                             double *a, Scalars *sc, const Reducer &red) {
  const unsigned nb = oc_blocks(nel, kOcReduceBlocks);
  oc_prepare_kernel<<<nb, kBs, 0, s>>>(nel, x, dc, dv, mask, eta, a, red.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_finalize(s, red, (int)nb, 1, fin_sum(&sc->vconst));
  if (e != hipSuccess) return e;
  oc_init_kernel<<<1, 64, 0, s>>>(sc, target);
  return hipGetLastError();
}

hipError_t launch_oc_pass(hipStream_t s, int64_t nel, const double *x, const double *a,
                          const double *dc, const double *dv, const int8_t *mask, double move,
                          double eta, double tol, Scalars *sc, const Reducer &red) {
  const unsigned nb = oc_blocks(nel, kOcPassBlocks);
  if (a)
    oc_pass_kernel<true><<<nb, kBs, 0, s>>>(nel, x, a, dc, dv, mask, move, eta, sc, red.partials);
  else
    oc_pass_kernel<false><<<nb, kBs, 0, s>>>(nel, x, a, dc, dv, mask, move, eta, sc, red.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  oc_select_kernel<<<1, kSelThreads, 0, s>>>((int)nb, tol, sc, red.partials);
  return hipGetLastError();
}

hipError_t launch_oc_final(hipStream_t s, int64_t nel, const double *x, const double *a,
                           const double *dc, const double *dv, const int8_t *mask, double move,
                           double eta, double *xnew, Scalars *sc, const Reducer &red) {
  const unsigned nb = oc_blocks(nel, kOcReduceBlocks);
  if (a)
    oc_final_kernel<true><<<nb, kBs, 0, s>>>(nel, x, a, dc, dv, mask, move, eta, xnew, sc, red.partials);
  else
    oc_final_kernel<false><<<nb, kBs, 0, s>>>(nel, x, a, dc, dv, mask, move, eta, xnew, sc, red.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_finalize(s, red, (int)nb, 1, fin_max(&sc->change));
  if (e != hipSuccess) return e;
  Reducer r2{red.partials + 1, red.max_blocks};
  return launch_finalize(s, r2, (int)nb, 1, fin_sum(&sc->volume));
}


// ---------------------------------------------------------------------------
// The same update for G problems with equally many elements: every launch
// above serves the whole group (stored coefficients only)
hipError_t launch_oc_update_group(hipStream_t s, int G, int64_t nel, const OcArgs *o, const Reducer *red) {
  if (!group_ok(G)) return hipErrorInvalidValue;
  for (int i = 0; i < G; ++i)
    if (!o[i].a) return hipErrorInvalidValue;
  const GroupTab<OcArgs> t = group_tab(G, o);
  const GroupTab<double *> part = group_partials(G, red);
  const int *noskip[kMaxGroup] = {};
  Fin fin[kMaxGroup];
  // prepare: coefficients and the volume of the passive elements
  const unsigned nr = oc_blocks(nel, kOcReduceBlocks);
  oc_prepare_group_kernel<<<dim3(nr, 1, G), kBs, 0, s>>>(nel, t, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int i = 0; i < G; ++i) fin[i] = fin_sum(&o[i].sc->vconst);
  e = launch_finalize_group(s, G, red, (int)nr, 1, fin, noskip);
  if (e != hipSuccess) return e;
  oc_init_group_kernel<<<G, 64, 0, s>>>(t);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // multisection passes
  const unsigned np = oc_blocks(nel, kOcPassBlocks);
  double tol = o[0].tol;  // enough passes for the tightest member
  for (int i = 1; i < G; ++i) tol = std::min(tol, o[i].tol);
  const int passes = oc_pass_launches(tol);
  for (int pass = 0; pass < passes; ++pass) {
    oc_pass_group_kernel<<<dim3(np, 1, G), kBs, 0, s>>>(nel, t, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    oc_select_group_kernel<<<G, kSelThreads, 0, s>>>((int)np, t, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // final: new design, its change and volume
  oc_final_group_kernel<<<dim3(nr, 1, G), kBs, 0, s>>>(nel, t, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int i = 0; i < G; ++i) fin[i] = fin_max(&o[i].sc->change);
  e = launch_finalize_group(s, G, red, (int)nr, 1, fin, noskip);
  if (e != hipSuccess) return e;
  Reducer r2[kMaxGroup];
  for (int i = 0; i < G; ++i) {
    r2[i] = Reducer{red[i].partials + 1, red[i].max_blocks};
    fin[i] = fin_sum(&o[i].sc->volume);
  }
  return launch_finalize_group(s, G, r2, (int)nr, 1, fin, noskip);
}

}  // namespace topo
