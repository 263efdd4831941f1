// Index arithmetic of four-axis boxes (device code): exact 32-bit division by
// precomputed magics, flat index -> axis indices, and the level of an element
// of a 4-D level-centric array (Sec. 5.1), shared by the 4-D kernels and the
// label entropy.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels4.hpp"
#include "levelpos.hpp"

namespace mgx {

__device__ __forceinline__ uint32_t udiv(uint32_t n, const Div32 &v) {
  return v.d == 1 ? n : (uint32_t)__umul64hi((uint64_t)n, v.mag);
}

// Axis indices of flat index i of a box whose dims 3, 2, 1 divide as d3, d2, d1.
__device__ __forceinline__ void split4(uint32_t i, const Div32 &d3, const Div32 &d2, const Div32 &d1, int j[4]) {
  const uint32_t r = udiv(i, d3);
  j[3] = (int)(i - r * d3.d);
  const uint32_t r2 = udiv(r, d2);
  j[2] = (int)(r - r2 * d2.d);
  const uint32_t r3 = udiv(r2, d1);
  j[1] = (int)(r2 - r3 * d1.d);
  j[0] = (int)r3;
}

// The level of flat element i: the largest of its four positions' levels.
__device__ __forceinline__ int elem_level(uint32_t i, const Quant4Args &a) {
  int j[4];
  split4(i, a.d3, a.d2, a.d1, j);
  int l = a.first;
#pragma unroll
  for (int k = 0; k < 4; k++) l = max(l, pos_level((uint32_t)j[k], a.off[k], a.first));
  return l;
}

}  // namespace mgx
