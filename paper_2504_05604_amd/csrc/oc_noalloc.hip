// OC update without a context and without any allocation: the multisection
// search state and its per-block partial sums live in a fixed device array of
// this library (one copy per GPU, held until the process ends).  For callers
// that cannot allocate device memory.
#include <cmath>
#include <cstddef>
#include <mutex>

#include "internal.h"

namespace topo {

namespace {
// scratch layout (doubles): the Scalars block of the search, then the partials
constexpr size_t kScalarDoubles = (sizeof(Scalars) + 255) / 256 * 256 / sizeof(double);
constexpr size_t kScratchDoubles = kScalarDoubles + (size_t)kOcPartials;
static_assert(sizeof(Scalars) <= kScalarDoubles * sizeof(double), "scalar block fits");
}  // namespace

// The fixed workspace (about 260 KB).  Host code never uses this name as an
// address: it stands for a device symbol, whose address on each GPU comes from
// hipGetSymbolAddress below.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The scratch address on the current device, looked up once per device with
// that device current.
topo_status scratch_on_current_device(double **out) {
  int dev = 0;
  TOPO_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error("device %d out of range", dev), TOPO_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error("hipGetSymbolAddress of the OC scratch failed: %s", hipGetErrorString(e)), TOPO_EDEVICE;
    g_scratch_ptr[dev] = (double *)p;
  }
  *out = g_scratch_ptr[dev];
  return TOPO_OK;
}
}  // namespace

}  // namespace topo

using namespace topo;

extern "C" topo_status topo_oc_update_noalloc(int64_t nel, const double *d_x, const double *d_dc,
                                              const double *d_dv, const int8_t *d_mask, double move,
                                              double eta, double target, double oc_tol, void *hip_stream,
                                              double *d_xnew, double *d_result) {
  if (nel < 1) return set_error("nel must be >= 1"), TOPO_EINVAL;
  if (!d_x || !d_dc || !d_dv || !d_mask || !d_xnew) return set_error("NULL argument"), TOPO_EINVAL;
  if (d_xnew == d_x || d_xnew == d_dc || d_xnew == d_dv) return set_error("d_xnew must not alias an input"), TOPO_EINVAL;
  if (!(move > 0.0) || !(eta > 0.0)) return set_error("move and eta must be > 0"), TOPO_EINVAL;
  if (!(oc_tol > 0.0)) return set_error("oc_tol must be > 0"), TOPO_EINVAL;
  if (!(target > 0.0) || !std::isfinite(target)) return set_error("target must be positive and finite"), TOPO_EINVAL;
  double *ws = nullptr;
  topo_status st = scratch_on_current_device(&ws);
  if (st != TOPO_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  Scalars *sc = (Scalars *)ws;
  const Reducer red{ws + kScalarDoubles, kOcPartials / kMaxRed};
  // the search state is fully written by the prepare launches (bracket, target,
  // pass count, candidates, the passive elements' volume): nothing to clear
  TOPO_HIP(launch_oc_prepare(s, nel, d_x, d_dc, d_dv, d_mask, eta, target, nullptr, sc, red));
  const int passes = oc_pass_launches(oc_tol);
  for (int pass = 0; pass < passes; ++pass)
    TOPO_HIP(launch_oc_pass(s, nel, d_x, nullptr, d_dc, d_dv, d_mask, move, eta, oc_tol, sc, red));
  TOPO_HIP(launch_oc_final(s, nel, d_x, nullptr, d_dc, d_dv, d_mask, move, eta, d_xnew, sc, red));
  if (d_result) {
    static_assert(offsetof(Scalars, volume) == offsetof(Scalars, change) + sizeof(double) &&
                      offsetof(Scalars, lambda) == offsetof(Scalars, change) + 2 * sizeof(double),
                  "change, volume and lambda are adjacent");
    TOPO_HIP(hipMemcpyAsync(d_result, &sc->change, 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  return TOPO_OK;
}
