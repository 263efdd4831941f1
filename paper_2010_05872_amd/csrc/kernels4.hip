// HIP kernels for four-axis fields on gfx950 (the 4-D QMCPACK field of
// Sec. 6, Table 2), arXiv 2010.05872.
//
// The method is the one of Sec. 2 on a grid with four axes.  A level runs as
//   k_coef4<DEC>      coefficients c = V - Pi V on N*_l (Pi over up to 16
//                     nodal corners), stored at level-centric positions
//                     (Sec. 5.1);
//   k_sweep4 x 4      the load vector (R M)^{x4} V, one axis after the other
//                     (Sec. 5.2 applies the fused mass-restriction stencil per
//                     axis), each sweep halving one axis, the contiguous axis
//                     first so later sweeps read already reduced boxes;
//   Thomas solves     the 3-D path's solve kernels with the other axes folded
//                     into (outer, inner) line sets.
// Recomposition: k_sweep4<GATHER> reads the coefficients straight from u_mc,
// the same solves subtract the correction, and k_coef4<REC> adds the
// interpolant.  These kernels are memory-bound elementwise passes: one thread
// per output node, consecutive threads on consecutive contiguous indices.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels4.hpp"

namespace mgx {
namespace {

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

template <typename T, bool DEC>
__global__ void __launch_bounds__(256) k_coef4(Coef4Args<T> a) {
  const int m1 = a.ax[1].m, m2 = a.ax[2].m, m3 = a.ax[3].m;
  const int c1 = a.ax[1].c, c2 = a.ax[2].c, c3 = a.ax[3].c;
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < a.n; i += stride) {
    int j[4];
    split4((uint32_t)i, a.d3, a.d2, a.d1, j);
    int odd = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) odd |= (j[k] & 1) << k;
    if (odd == 0) {
      if (!DEC)
        a.out[j[0] * a.op[0] + j[1] * a.op[1] + j[2] * a.op[2] + j[3]] =
            a.nodal[(((int64_t)(j[0] >> 1) * c1 + (j[1] >> 1)) * c2 + (j[2] >> 1)) * c3 + (j[3] >> 1)];
      continue;
    }
    // interpolant over the nodal corners: for each odd axis the left (bit 0)
    // and right (bit 1) neighbour
    T pred = T(0);
    for (int cn = 0; cn < 16; cn++) {
      if (cn & ~odd) continue;
      T w = T(1);
      int q[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        if ((odd >> k) & 1) {
          if ((cn >> k) & 1) {
            q[k] = j[k] + 1;
            w *= a.ax[k].wr[j[k]];
          } else {
            q[k] = j[k] - 1;
            w *= a.ax[k].wl[j[k]];
          }
        } else {
          q[k] = j[k];
        }
      }
      const T v = DEC ? a.V[(((int64_t)q[0] * m1 + q[1]) * m2 + q[2]) * m3 + q[3]]
                      : a.nodal[(((int64_t)(q[0] >> 1) * c1 + (q[1] >> 1)) * c2 + (q[2] >> 1)) * c3 + (q[3] >> 1)];
      pred += w * v;
    }
    int64_t pos = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int p = (j[k] & 1) ? a.ax[k].c + (j[k] >> 1) : (j[k] >> 1);
      pos += (k < 3) ? (int64_t)p * a.up[k] : (int64_t)p;
    }
    if (DEC)
      a.umc_w[pos] = a.V[i] - pred;
    else
      a.out[j[0] * a.op[0] + j[1] * a.op[1] + j[2] * a.op[2] + j[3]] = a.umc_r[pos] + pred;
  }
}

template <typename T, bool GATHER>
__global__ void __launch_bounds__(256) k_sweep4(Sweep4Args<T> a) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < a.n; i += stride) {
    const uint32_t t = udiv((uint32_t)i, a.dinner);
    const uint32_t ii = (uint32_t)i - t * a.inner;
    const uint32_t o = udiv(t, a.dc);
    const int J = (int)(t - o * (uint32_t)a.c);
    T acc = T(0);
    if (!GATHER) {
      const T *row = a.in + (int64_t)o * a.m * a.inner + ii;
#pragma unroll
      for (int d = 0; d < 5; d++) {
        const int jj = 2 * J + d - 2;
        if (jj < 0 || jj >= a.m) continue;
        acc += a.w5[5 * J + d] * row[(int64_t)jj * a.inner];
      }
    } else {
      // o = (j0 m1 + j1) m2 + j2 of the level box; the sweep runs along axis 3
      const uint32_t r = udiv(o, a.dm2);
      const int j2 = (int)(o - r * (uint32_t)a.m2);
      const int j0 = (int)udiv(r, a.dm1);
      const int j1 = (int)(r - (uint32_t)j0 * (uint32_t)a.m1);
      const bool nodal_row = ((j0 | j1 | j2) & 1) == 0;
      auto lc = [&](int j, int k) { return (j & 1) ? a.cc[k] + (j >> 1) : (j >> 1); };
      const int64_t base = (int64_t)lc(j0, 0) * a.up[0] + (int64_t)lc(j1, 1) * a.up[1] + (int64_t)lc(j2, 2) * a.up[2];
#pragma unroll
      for (int d = 0; d < 5; d++) {
        const int jj = 2 * J + d - 2;
        if (jj < 0 || jj >= a.m) continue;
        if (nodal_row && (jj & 1) == 0) continue;  // nodal node: component zero
        acc += a.w5[5 * J + d] * a.umc[base + lc(jj, 3)];
      }
    }
    a.out[i] = acc;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_copy4(Copy4Args<T> a) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < a.n; i += stride) {
    int j[4];
    split4((uint32_t)i, a.d3, a.d2, a.d1, j);
    a.dst[j[0] * a.dp[0] + j[1] * a.dp[1] + j[2] * a.dp[2] + j[3]] =
        a.src[j[0] * a.sp[0] + j[1] * a.sp[1] + j[2] * a.sp[2] + j[3]];
  }
}

// Level of position p along an axis with n - 1 = 2^(L + off): the smallest
// level whose box (2^(l + off) + 1 nodes) holds it, at least `first`.
__device__ __forceinline__ int axis_pos_level(uint32_t p, int off, int first) {
  if (p < 2) return first;
  const int bl = 32 - __clz((int)(p - 1));
  return max(first, bl - off);
}

__device__ __forceinline__ int level4(uint32_t i, const Quant4Args &a) {
  int j[4];
  split4(i, a.d3, a.d2, a.d1, j);
  int l = a.first;
#pragma unroll
  for (int k = 0; k < 4; k++) l = max(l, axis_pos_level((uint32_t)j[k], a.off[k], a.first));
  return l;
}

template <typename T>
__global__ void __launch_bounds__(256) k_quantize4(const T *__restrict__ umc, int32_t *__restrict__ labels,
                                                   Quant4Args a) {
  __shared__ double s_q[kMaxLevelsK];
  __shared__ int s_max[kMaxLevelsK];
  __shared__ unsigned long long s_ovf, s_nan;
  if (threadIdx.x < kMaxLevelsK) {
    s_q[threadIdx.x] = a.q[threadIdx.x];
    s_max[threadIdx.x] = 0;
  }
  if (threadIdx.x == 0) s_ovf = s_nan = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  unsigned long long ovf = 0, nan = 0;
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  // every thread of the workgroup runs the same iterations (wave-wide
  // reductions below); elements past the end are inactive
  for (uint64_t b0 = (uint64_t)blockIdx.x * 256u; b0 < a.n; b0 += stride) {
    const uint64_t i = b0 + threadIdx.x;
    const bool in = i < a.n;
    const int l = in ? level4((uint32_t)i, a) : a.first;
    int absl = 0;
    if (in) {
      const double t = (double)umc[i] / s_q[l - a.first];
      int32_t lab;
      if (!(fabs(t) < 2147483647.0)) {
        lab = INT32_MIN;
        if (isnan(t) || isinf(t))
          nan++;
        else
          ovf++;
      } else {
        lab = (int32_t)rint(t);
        absl = lab < 0 ? -lab : lab;
      }
      labels[i] = lab;
    }
    if (a.stats_max) {
      // per-level maxima: one reduction per distinct level in the wave
      unsigned long long todo = __ballot(in);
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int L0 = __shfl(l, leader);
        const bool mine = in && l == L0;
        int m = mine ? absl : 0;
        for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
        if (lane == leader) atomicMax(&s_max[L0 - a.first], m);
        todo &= ~__ballot(mine);
      }
    }
  }
  if (a.stats_max) {
    if (ovf) atomicAdd(&s_ovf, ovf);
    if (nan) atomicAdd(&s_nan, nan);
    __syncthreads();
    if (threadIdx.x < a.nlev && s_max[threadIdx.x] > 0) atomicMax(&a.stats_max[threadIdx.x], s_max[threadIdx.x]);
    if (threadIdx.x == 0) {
      if (s_ovf) atomicAdd(a.stats_ovf, s_ovf);
      if (s_nan) atomicAdd(a.stats_nan, s_nan);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_dequantize4(const int32_t *__restrict__ labels, T *__restrict__ umc,
                                                     Quant4Args a) {
  __shared__ double s_q[kMaxLevelsK];
  if (threadIdx.x < kMaxLevelsK) s_q[threadIdx.x] = a.q[threadIdx.x];
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < a.n; i += stride) {
    const int l = level4((uint32_t)i, a);
    umc[i] = (T)((double)labels[i] * s_q[l - a.first]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_pad4(Pad4Args<T> a) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < a.n; i += stride) {
    int j[4];
    split4((uint32_t)i, a.d3, a.d2, a.d1, j);
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) s = s * a.nsrc[k] + min(j[k], a.nsrc[k] - 1);
    a.dst[i] = a.src[s];
  }
}

unsigned grid_for(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

template <typename T>
hipError_t launch_coef4(Coef4Args<T> a, bool dec, hipStream_t st) {
  if (a.n == 0) return hipSuccess;
  if (dec)
    hipLaunchKernelGGL((k_coef4<T, true>), dim3(grid_for(a.n)), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_coef4<T, false>), dim3(grid_for(a.n)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep4(Sweep4Args<T> a, bool gather, hipStream_t st) {
  if (a.n == 0) return hipSuccess;
  if (gather)
    hipLaunchKernelGGL((k_sweep4<T, true>), dim3(grid_for(a.n)), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_sweep4<T, false>), dim3(grid_for(a.n)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy4(Copy4Args<T> a, hipStream_t st) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_copy4<T>), dim3(grid_for(a.n)), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_quantize4(const T *umc, int32_t *labels, Quant4Args a, hipStream_t st) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_quantize4<T>), dim3(grid_for(a.n)), dim3(256), 0, st, umc, labels, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dequantize4(const int32_t *labels, T *umc, Quant4Args a, hipStream_t st) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_dequantize4<T>), dim3(grid_for(a.n)), dim3(256), 0, st, labels, umc, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pad4(Pad4Args<T> a, hipStream_t st) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_pad4<T>), dim3(grid_for(a.n)), dim3(256), 0, st, a);
  return hipGetLastError();
}

#define MGX_INST4(T)                                                                     \
  template hipError_t launch_coef4<T>(Coef4Args<T>, bool, hipStream_t);                  \
  template hipError_t launch_sweep4<T>(Sweep4Args<T>, bool, hipStream_t);                \
  template hipError_t launch_copy4<T>(Copy4Args<T>, hipStream_t);                        \
  template hipError_t launch_quantize4<T>(const T *, int32_t *, Quant4Args, hipStream_t); \
  template hipError_t launch_dequantize4<T>(const int32_t *, T *, Quant4Args, hipStream_t); \
  template hipError_t launch_pad4<T>(Pad4Args<T>, hipStream_t);
MGX_INST4(float)
MGX_INST4(double)

}  // namespace mgx
