// gp_query_noalloc: the PIP / P2P query with a library-held workspace, for callers that
// cannot allocate device memory (code under graph capture, tight serving loops).
//
// The workspace is a file-scope device array.  Host code never uses the array's name as
// a device address (on the host it names a stand-in, not device memory): the device
// address of each GPU's copy is looked up once per device with hipGetSymbolAddress and
// kept, and only that address is handed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gp_internal.h"

namespace gp {
gp_status set_error(gp_status code, const char *fmt, ...);
gp_status run_query_tuned(const gp_grid *g, gp_kind kind, int64_t n, const double *px,
                          const double *py, int32_t *out_id, double *out_dist,
                          gp_precision prec, void *ws, size_t ws_bytes, hipStream_t s,
                          gp_stats *stats, const gp_tuning *t);
}  // namespace gp

using namespace gp;

namespace {

constexpr int kMaxDevices = 64;

// One copy per GPU the library runs on, held until the process ends.
__device__ __align__(256) unsigned char scratch[GP_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device, once known

// Device address of the current device's scratch array (looked up on first use).
gp_status scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(GP_E_INVALID_ARG, "device %d is beyond the %d the library tracks", dev,
                     kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(GP_E_HIP, "hipGetSymbolAddress of the scratch array failed: %s",
                       hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GP_OK;
}

}  // namespace

extern "C" gp_status gp_query_noalloc(const gp_grid *grid, gp_kind kind, int64_t n,
                                      const double *px, const double *py, int32_t *out_id,
                                      double *out_dist, gp_precision prec, void *hip_stream) {
  if (!grid) return set_error(GP_E_INVALID_ARG, "null grid");
  if (kind != GP_PIP && kind != GP_P2P) return set_error(GP_E_INVALID_ARG, "bad kind");
  size_t need = 0;
  gp_status rc = gp_workspace_bytes(grid, n, prec, &need);
  if (rc) return rc;
  if (need > (size_t)GP_NOALLOC_SCRATCH_BYTES)
    return set_error(GP_E_CAPACITY,
                     "%lld points need %zu bytes of workspace, more than the %zu of the "
                     "library's scratch", (long long)n, need, (size_t)GP_NOALLOC_SCRATCH_BYTES);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(GP_E_HIP, "hipGetDevice failed");
  void *ws = nullptr;
  rc = scratch_address(dev, &ws);
  if (rc) return rc;
  return run_query_tuned(grid, kind, n, px, py, out_id, out_dist, prec, ws,
                         (size_t)GP_NOALLOC_SCRATCH_BYTES, (hipStream_t)hip_stream, nullptr,
                         nullptr);
}
