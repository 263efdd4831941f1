// mgx_decompose_noalloc: the decomposition for callers that cannot allocate
// device memory.  Its tables and workspace live in one file-scope device
// array; each device holds its own copy of it from the library's load until
// the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mgx.h"
#include "placed.hpp"

namespace {

static_assert(MGX_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

// The level tables followed by the decomposition's workspace.  In host code
// this name is a stand-in for the symbol, not a device address: the kernels
// get the per-device address that hipGetSymbolAddress returns.
__device__ __align__(256) char scratch[MGX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current).
mgx_status scratch_ptr(char **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MGX_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return MGX_ERR_HIP;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MGX_ERR_HIP;
    g_ptr[dev] = p;
  }
  *out = (char *)g_ptr[dev];
  return MGX_OK;
}

}  // namespace

extern "C" mgx_status mgx_decompose_noalloc(const void *u, void *u_mc, mgx_dtype dtype, int ndim,
                                             const int64_t *dims, const double *const *coords, int stop_level,
                                             hipStream_t stream) {
  char *region = nullptr;
  mgx_status s = scratch_ptr(&region);
  if (s) return s;
  return mgx::decompose_placed(u, u_mc, dtype, ndim, dims, coords, stop_level, region, MGX_NOALLOC_SCRATCH_BYTES,
                               stream);
}
