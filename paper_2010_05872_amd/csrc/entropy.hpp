// Per-level Shannon entropy of quantization labels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "kernels4.hpp"

namespace mgx {
// Workspace bytes for n labels in nlev levels.
size_t entropy_workspace(int64_t n, int nlev);
// bits_out[i]: entropy in bits per label of level qa.first + i, whose label
// count is level_count[i].  Synchronizes st.  A: QuantArgs (1-D to 3-D) or
// Quant4Args (4-D).  known_max (host, nullable): each level's max |label| as
// the quantizer reported it, which saves the pass that finds it; labels
// beyond it make the call count again without it.
template <typename A>
hipError_t label_entropy(const int32_t *labels, const A &qa, const int64_t *level_count, char *ws, hipStream_t st,
                         double *bits_out, const int32_t *known_max = nullptr);
// max_abs[i] (device, zeroed by the caller) = largest |label| of level
// qa.first + i, leaving out INT32_MIN labels (out-of-range coefficients).
// Asynchronous on st.
template <typename A>
hipError_t label_max_abs(const int32_t *labels, const A &qa, int *max_abs, hipStream_t st);
}  // namespace mgx
