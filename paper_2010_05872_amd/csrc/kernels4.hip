// HIP kernels for four-axis fields on gfx950 (the 4-D QMCPACK field of
// Sec. 6, Table 2), arXiv 2010.05872.
//
// The method is the one of Sec. 2 on a grid with four axes.  A level runs as
//   k_coef4<DEC>      coefficients c = V - Pi V on N*_l (Pi over up to 16
//                     nodal corners), stored at level-centric positions
//                     (Sec. 5.1), one thread per column marching along axis 0;
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
#include "levelpos4.hpp"

namespace mgx {
namespace {

// Quantization label of a coefficient and a coefficient of a label: the
// operations of the separate (de)quantization passes (Sec. 4.1), so labels
// written or read by the level kernels equal theirs bit for bit.
template <typename T>
__device__ __forceinline__ int32_t label4(T v, double q) {
  const double t = (double)v / q;
  return !(fabs(t) < 2147483647.0) ? INT32_MIN : (int32_t)rint(t);
}
// A label of INT32_MIN counted: rng[0] for a finite |c/q| >= 2^31 - 1,
// rng[1] for a c/q that is not finite.
template <typename T>
__device__ __forceinline__ void count_range4(unsigned long long *rng, T v, double q) {
  const double t = (double)v / q;
  atomicAdd(&rng[(isnan(t) || isinf(t)) ? 1 : 0], 1ull);
}
// (the product is rounded on its own, never contracted into a following add)
template <typename T>
__device__ __forceinline__ T unlabel4(int32_t l, double q) {
#pragma clang fp contract(off)
  return (T)((double)l * q);
}

// One thread per column (j1, j2, j3) of the level box and chunk of plane
// pairs (blockIdx.y), marching along axis 0.
// The interpolant factors: Pi V(j) = wl0 Q(j0 - 1) + wr0 Q(j0 + 1) for odd j0
// and Q(j0) for even j0, where Q(p) is the interpolant over axes 1..3 of
// plane p at the column (the value itself when the column is nodal in axes
// 1..3).  Q of each even plane is computed once and kept for the odd plane
// after it, so every value of the level box is read about once.
template <typename T, bool DEC, bool LAB>
__global__ void __launch_bounds__(256) k_coef4(Coef4Args<T> a) {
  const int m1 = a.ax[1].m, m2 = a.ax[2].m, m3 = a.ax[3].m;
  const int c1 = a.ax[1].c, c2 = a.ax[2].c, c3 = a.ax[3].c;
  const uint32_t col = blockIdx.x * 256u + threadIdx.x;
  if (col >= a.ncol) return;
  int j[4];
  {
    const uint32_t r = udiv(col, a.d3);
    j[3] = (int)(col - r * a.d3.d);
    const uint32_t r2 = udiv(r, a.d2);
    j[2] = (int)(r - r2 * a.d2.d);
    j[1] = (int)r2;
  }
  // the column's nodal neighbours in axes 1..3 (level-l box for DEC, coarse
  // box for REC): per axis the left (or, on an even index, the own) offset and
  // the right one, with their weights
  int64_t lo[4], hi[4];
  T wlo[4], whi[4];
  bool od[4];
  {
    const int64_t str[4] = {0, DEC ? (int64_t)m2 * m3 : (int64_t)c2 * c3, DEC ? m3 : c3, 1};
#pragma unroll
    for (int k = 1; k < 4; k++) {
      od[k] = j[k] & 1;
      const int jl = od[k] ? j[k] - 1 : j[k], jr = od[k] ? j[k] + 1 : j[k];
      lo[k] = (DEC ? jl : (jl >> 1)) * str[k];
      hi[k] = (DEC ? jr : (jr >> 1)) * str[k];
      wlo[k] = od[k] ? a.ax[k].wl[j[k]] : T(1);
      whi[k] = od[k] ? a.ax[k].wr[j[k]] : T(0);
    }
  }
  const bool odd = od[1] || od[2] || od[3];
  const int64_t plane = DEC ? (int64_t)m1 * m2 * m3 : (int64_t)c1 * c2 * c3;
  // no aliasing between the level box, the coarse box and the outputs: the
  // loads of the next plane pair may pass the stores of the previous one
  const T *__restrict__ src = DEC ? a.V : a.nodal;
  const T *__restrict__ V = a.V;
  T *__restrict__ umc_w = a.umc_w;
  int32_t *__restrict__ lab_w = a.lab_w;
  const T *__restrict__ umc_r = a.umc_r;
  const int32_t *__restrict__ lab_r = a.lab_r;
  T *__restrict__ out = a.out;
  // Q(p): the interpolant over axes 1..3 at the column in plane p of src
  // (fine plane index for DEC, coarse for REC), nested one axis at a time
  auto Q = [&](int p) {
    const T *b = src + (int64_t)p * plane;
    auto row = [&](int64_t o) { return od[3] ? wlo[3] * b[o + lo[3]] + whi[3] * b[o + hi[3]] : b[o + lo[3]]; };
    auto pln = [&](int64_t o) { return od[2] ? wlo[2] * row(o + lo[2]) + whi[2] * row(o + hi[2]) : row(o + lo[2]); };
    return od[1] ? wlo[1] * pln(lo[1]) + whi[1] * pln(hi[1]) : pln(lo[1]);
  };
  // level-centric offsets of the column in u_mc, and its output offset
  auto lcp = [&](int jj, int k) { return (jj & 1) ? a.ax[k].c + (jj >> 1) : (jj >> 1); };
  const int64_t ucol = (int64_t)lcp(j[1], 1) * a.up[1] + (int64_t)lcp(j[2], 2) * a.up[2] + lcp(j[3], 3);
  const int64_t vcol = ((int64_t)j[1] * m2 + j[2]) * m3 + j[3];
  const int64_t ocol = j[1] * a.op[1] + j[2] * a.op[2] + j[3];
  const int cc0 = a.ax[0].c;
  // decompose: store coefficient c at u_mc offset u (and / or its label)
  auto put = [&](int64_t u, T c) {
    if (!LAB || umc_w) umc_w[u] = c;
    if (LAB) {
      const int32_t l = label4<T>(c, a.qc);
      lab_w[u] = l;
      if (l == INT32_MIN && a.rng) count_range4(a.rng, c, a.qc);
    }
  };
  // recompose: the coefficient at u_mc offset u
  auto get = [&](int64_t u) { return LAB ? unlabel4<T>(lab_r[u], a.qc) : umc_r[u]; };
  // this chunk's pairs (even plane 2J, odd plane 2J+1), J0 <= J < J1; the
  // last chunk also takes the last even plane
  const int npair = cc0 - 1;
  const int J0 = (int)blockIdx.y * a.jchunk;
  const int J1 = min(npair, J0 + a.jchunk);
  const bool last = J1 == npair;
  T qprev = Q(DEC ? 2 * J0 : J0);
  // one plane pair per iteration (unrolling measured slower for the
  // recomposition kernel, equal for the decomposition)
  auto pair = [&](int J) {
    const int je = 2 * J;
    const T qnext = Q(DEC ? je + 2 : J + 1);
    const T ve = DEC ? V[je * plane + vcol] : (odd ? get((int64_t)J * a.up[0] + ucol) : T(0));
    const int64_t u = (int64_t)(cc0 + J) * a.up[0] + ucol;
    const T vo = DEC ? V[(je + 1) * plane + vcol] : get(u);
    const T pred = a.ax[0].wl[je + 1] * qprev + a.ax[0].wr[je + 1] * qnext;
    if (DEC) {
      if (odd) put((int64_t)J * a.up[0] + ucol, ve - qprev);
      put(u, vo - pred);
    } else {
      out[je * a.op[0] + ocol] = odd ? ve + qprev : qprev;
      out[(je + 1) * a.op[0] + ocol] = vo + pred;
    }
    qprev = qnext;
  };
  for (int J = J0; J < J1; J++) pair(J);
  if (!last) return;
  // the last (even) plane
  const int J = J1;
  const int je = 2 * J;
  if (DEC) {
    if (odd) put((int64_t)J * a.up[0] + ucol, V[je * plane + vcol] - qprev);
  } else {
    out[je * a.op[0] + ocol] = odd ? get((int64_t)J * a.up[0] + ucol) + qprev : qprev;
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
        const int64_t u = base + lc(jj, 3);
        acc += a.w5[5 * J + d] * (a.lab ? unlabel4<T>(a.lab[u], a.qc) : a.umc[u]);
      }
    }
    a.out[i] = acc;
  }
}

// The same sweep as one march per (o, i) column along the axis (inner >=
// kSweepMarchInner: consecutive threads on consecutive i, coalesced): output J
// needs inputs 2J-2 .. 2J+2, of which 2J-2 .. 2J carry over from output J-1,
// so each input row is read once per chunk (plus two rows at its start).
template <typename T>
__global__ void __launch_bounds__(256) k_sweep4_march(Sweep4Args<T> a) {
  const uint64_t col = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  const uint64_t ncol = (uint64_t)a.n / (uint64_t)a.c;  // outer * inner
  if (col >= ncol) return;
  const uint32_t o = udiv((uint32_t)col, a.dinner);
  const uint32_t ii = (uint32_t)col - o * a.inner;
  const T *__restrict__ row = a.in + (int64_t)o * a.m * a.inner + ii;
  T *__restrict__ out = a.out + (int64_t)o * a.c * a.inner + ii;
  const T *__restrict__ w5 = a.w5;
  const int64_t inner = a.inner;
  const int m = a.m;
  auto x = [&](int j) { return (j >= 0 && j < m) ? row[(int64_t)j * inner] : T(0); };
  const int J0 = (int)blockIdx.y * a.jchunk, J1 = min(a.c, J0 + a.jchunk);
  T xm2 = x(2 * J0 - 2), xm1 = x(2 * J0 - 1), x0 = x(2 * J0);
  for (int J = J0; J < J1; J++) {
    const T x1 = x(2 * J + 1), x2 = x(2 * J + 2);
    const T *w = w5 + 5 * J;
    T acc = T(0);
    if (2 * J - 2 >= 0) acc += w[0] * xm2;
    if (2 * J - 1 >= 0) acc += w[1] * xm1;
    acc += w[2] * x0;
    if (2 * J + 1 < m) acc += w[3] * x1;
    if (2 * J + 2 < m) acc += w[4] * x2;
    out[(int64_t)J * inner] = acc;
    xm2 = x0;
    xm1 = x1;
    x0 = x2;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_copy4(Copy4Args<T> a) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < a.n; i += stride) {
    int j[4];
    split4((uint32_t)i, a.d3, a.d2, a.d1, j);
    const int64_t si = j[0] * a.sp[0] + j[1] * a.sp[1] + j[2] * a.sp[2] + j[3];
    const int64_t di = j[0] * a.dp[0] + j[1] * a.dp[1] + j[2] * a.dp[2] + j[3];
    const T v = a.lab_r ? unlabel4<T>(a.lab_r[si], a.q) : a.src[si];
    if (a.dst) a.dst[di] = v;
    if (a.lab_w) {
      const int32_t l = label4<T>(v, a.q);
      a.lab_w[di] = l;
      if (l == INT32_MIN && a.rng) count_range4(a.rng, v, a.q);
    }
  }
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
    const int l = in ? elem_level((uint32_t)i, a) : a.first;
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
    const int l = elem_level((uint32_t)i, a);
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

#ifndef MGX_GRID4_MAX
#define MGX_GRID4_MAX 65536
#endif
unsigned grid_for(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  if (g > MGX_GRID4_MAX) g = MGX_GRID4_MAX;
  return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

template <typename T>
hipError_t launch_coef4(Coef4Args<T> a, bool dec, hipStream_t st) {
  if (a.ncol == 0) return hipSuccess;
  if (a.jchunk < 1 || a.nchunk < 1) return hipErrorInvalidValue;
  const dim3 grid((a.ncol + 255) / 256, a.nchunk);
  if (dec && a.lab_w)
    hipLaunchKernelGGL((k_coef4<T, true, true>), grid, dim3(256), 0, st, a);
  else if (dec)
    hipLaunchKernelGGL((k_coef4<T, true, false>), grid, dim3(256), 0, st, a);
  else if (a.lab_r)
    hipLaunchKernelGGL((k_coef4<T, false, true>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_coef4<T, false, false>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep4(Sweep4Args<T> a, bool gather, hipStream_t st) {
  if (a.n == 0) return hipSuccess;
  if (!gather && a.inner >= (uint32_t)kSweepMarchInner) {
    if (a.jchunk < 1 || a.nchunk < 1 || (int64_t)a.jchunk * a.nchunk < a.c) return hipErrorInvalidValue;
    const uint64_t ncol = (uint64_t)a.n / (uint64_t)a.c;
    hipLaunchKernelGGL((k_sweep4_march<T>), dim3((unsigned)((ncol + 255) / 256), a.nchunk), dim3(256), 0, st, a);
    return hipGetLastError();
  }
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
