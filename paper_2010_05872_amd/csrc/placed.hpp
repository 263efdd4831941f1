// Decomposition on device memory the caller places (internal to libmgx):
// the entry point that allocates nothing hands its static array here.
#pragma once

#include <cstddef>
#include <cstdint>

#include "mgx.h"

namespace mgx {

// mgx_decompose of a 1-D to 3-D field with every piece of device memory
// besides u and u_mc inside `region` (region_bytes, 256-byte aligned): the
// plan's level tables are copied there from host memory on `stream`
// (hipMemcpyAsync from pageable memory), followed by the workspace.  No
// device allocation, no event, no tracing.  MGX_ERR_WORKSPACE when tables
// and workspace do not fit; MGX_ERR_SHAPE for ndim = 4; otherwise the
// errors of mgx_decompose.
mgx_status decompose_placed(const void *u, void *u_mc, mgx_dtype dtype, int ndim, const int64_t *dims,
                            const double *const *coords, int stop_level, char *region, size_t region_bytes,
                            hipStream_t stream);

}  // namespace mgx
