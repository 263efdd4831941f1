// Per-level Shannon entropy of quantization labels (sort-based histogram).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace mgx {
// Workspace bytes for n labels in nlev levels.
size_t entropy_workspace(int64_t n, int nlev);
// bits_out[i]: entropy in bits per label of level qa.first + i, whose label
// count is level_count[i].  Synchronizes st.
hipError_t label_entropy(const int32_t *labels, const QuantArgs &qa, const int64_t *level_count, char *ws,
                         hipStream_t st, double *bits_out);
}  // namespace mgx
