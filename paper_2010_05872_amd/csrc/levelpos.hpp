// Level of an element of a level-centric array (Sec. 5.1) from its position,
// shared by the quantization passes and the label entropy.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace mgx {

// The level of a position is the smallest l whose box holds it.  Along an
// axis with n - 1 = 2^m, the level-l box has 2^(m-L+l) + 1 nodes, so position
// p >= 2 lies in level max(first, bitlength(p-1) - (m - L)); positions 0 and
// 1 are in every box.
__device__ __forceinline__ int pos_level(uint32_t p, int off, int first) {
  if (p < 2) return first;
  const int bl = 32 - __clz((int)(p - 1));
  return max(first, bl - off);
}

// The level of flat element idx = (z * n1 + y) * n2 + x (all < 2^32);
// divisions by precomputed magics.
__device__ __forceinline__ int elem_level(uint32_t idx, const QuantArgs &a) {
  const uint32_t row = (uint32_t)__umul64hi((uint64_t)idx, a.mag2);
  const uint32_t x = idx - row * (uint32_t)a.n2;
  const uint32_t z = a.n1 == 1 ? row : (uint32_t)__umul64hi((uint64_t)row, a.mag1);
  const uint32_t y = row - z * (uint32_t)a.n1;
  int l = pos_level(x, a.off[2], a.first);
  l = max(l, pos_level(y, a.off[1], a.first));
  l = max(l, pos_level(z, a.off[0], a.first));
  return l;
}

}  // namespace mgx
