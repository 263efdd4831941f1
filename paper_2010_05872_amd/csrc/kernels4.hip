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
#include <type_traits>

#include "kernels4.hpp"
#include "levelpos4.hpp"

namespace mgx {
namespace {

// A uniform table entry through the constant address space: a scalar load,
// so waiting for it never waits for the vector loads in flight.
template <typename T>
__device__ __forceinline__ T ldu4(const T *p, int i) {
  return ((const __attribute__((address_space(4))) T *)p)[i];
}

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
// pairs (the logical block's row), marching along axis 0.  A wave takes 60
// consecutive columns (lanes 2..61) plus two on either side (lanes 0, 1, 62,
// 63, which only load): the axis-3 neighbours j3 - 1, j3 + 1 of a column with odd j3
// (never the first or last of its row) are then the neighbouring lanes, whose
// values come by lane shuffles, so a lane loads Q's corners only at its own
// j3.  With a.g the decomposition also takes the first load-vector sweep
// (R M along axis 3) of the planes it reads: the lane of an even j3 = 2 J3
// sums w5[5 J3 + d] x(j3 + d - 2) over the lanes j3 - 2 .. j3 + 2 of its row
// (terms outside the row skipped, the order of k_sweep4), so the level box is
// read once for both.
// The interpolant factors: Pi V(j) = wl0 Q(j0 - 1) + wr0 Q(j0 + 1) for odd j0
// and Q(j0) for even j0, where Q(p) is the interpolant over axes 1..3 of
// plane p at the column (the value itself when the column is nodal in axes
// 1..3).  Q of each even plane is computed once and kept for the odd plane
// after it, so every value of the level box is read about once.
// Memory: a pair's words (the 8 corners of Q's stencil in the next even plane
// -- on an axis where the column is even both corners are the same node --,
// and the pair's own two values) are loaded together, without branches, and
// two pairs ahead: pair J+2's loads are issued before pair J's stores (three
// register buffers, the loop unrolled three times).  One counter covers both
// loads and stores and drains in order, so waiting for pair J's words also
// waits for whatever was issued before them; one pair ahead, that was the
// previous pair's stores and most of pair J+1's loads.  The arithmetic is
// that of the nested form (per axis: wl x(lo) + wr x(hi) on odd, x(lo) on
// even), unchanged.
constexpr int kCoefHalo = 2;                     // load-only lanes on either side of a wave
constexpr int kCoefCols = 64 - 2 * kCoefHalo;  // output columns per wave of k_coef4
// Workgroups are dispatched to the 8 XCDs (each with its own L2) in turn.
// Logical block of the b-th workgroup of nb: each XCD takes a contiguous
// range of logical blocks, columns first and then chunks, so the rows
// j1 - 1 and j1 + 1 whose nodes a column's interpolant reads, and the lines
// that two neighbouring workgroups share, are fetched into one L2.  The
// order is that of the three-axis level kernels (xcd_remap in kernels.hip),
// with 64-bit block counts, since a four-axis grid's blocks times chunks
// may pass 2^31.
__device__ __forceinline__ uint64_t xcd_block4(uint64_t b, uint64_t nb) {
  const uint64_t q = nb >> 3, r = nb & 7, xcd = b & 7;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + (b >> 3);
}

template <typename T, bool DEC, bool LAB>
__global__ void __launch_bounds__(256) k_coef4(Coef4Args<T> a) {
  const int m1 = a.ax[1].m, m2 = a.ax[2].m, m3 = a.ax[3].m;
  const int c1 = a.ax[1].c, c2 = a.ax[2].c, c3 = a.ax[3].c;
  const int lane = threadIdx.x & 63;
  const uint64_t lb = xcd_block4(blockIdx.x + (uint64_t)blockIdx.y * gridDim.x, (uint64_t)gridDim.x * gridDim.y);
  const uint64_t bx = lb % gridDim.x, by = lb / gridDim.x;
  const int64_t wcol = ((int64_t)bx * 4 + (threadIdx.x >> 6)) * kCoefCols - kCoefHalo + lane;
  // every lane runs the march (the shuffles need the whole wave); only the
  // inner lanes of real columns store
  const bool active = lane >= kCoefHalo && lane < kCoefHalo + kCoefCols && wcol < (int64_t)a.ncol;
  const uint32_t col = (uint32_t)min(max(wcol, (int64_t)0), (int64_t)a.ncol - 1);
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
  // offsets of the 4 corner rows at the lane's own axis-3 position (bit 1:
  // axis 1, bit 0: axis 2); the own position is j3 (DEC) or the coarse j3 >> 1
  // (REC), whose axis-3 neighbours are: DEC lanes - 1 and + 1; REC the own
  // value and lane + 1 (for odd j3, (j3 - 1) / 2 and (j3 + 1) / 2)
  const int64_t own3 = DEC ? j[3] : (j[3] >> 1);
  int64_t coff[4];
#pragma unroll
  for (int c = 0; c < 4; c++) coff[c] = ((c & 2) ? hi[1] : lo[1]) + ((c & 1) ? hi[2] : lo[2]) + own3;
  // Q from the 4 loaded corner rows, nested one axis at a time (axis 3 first,
  // as wl x(lo) + wr x(hi) on an odd index and x(lo) on an even one)
  auto Qof = [&](const T (&x)[4]) {
    T r[4];
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const T dn = __shfl_down(x[c], 1);
      const T lo3v = DEC ? __shfl_up(x[c], 1) : x[c];
      r[c] = od[3] ? wlo[3] * lo3v + whi[3] * dn : x[c];
    }
    auto pln = [&](int b) { return od[2] ? wlo[2] * r[b] + whi[2] * r[b + 1] : r[b]; };
    return od[1] ? wlo[1] * pln(0) + whi[1] * pln(2) : pln(0);
  };
  // level-centric offsets of the column in u_mc, and its output offset
  auto lcp = [&](int jj, int k) { return (jj & 1) ? a.ax[k].c + (jj >> 1) : (jj >> 1); };
  const int64_t ucol = (int64_t)lcp(j[1], 1) * a.up[1] + (int64_t)lcp(j[2], 2) * a.up[2] + lcp(j[3], 3);
  const int64_t vcol = ((int64_t)j[1] * m2 + j[2]) * m3 + j[3];
  const int64_t ocol = j[1] * a.op[1] + j[2] * a.op[2] + j[3];
  const int cc0 = a.ax[0].c;
  // the fused axis-3 sweep: the lane's 5 weights (even j3 = 2 J3) and output row
  const bool gout = DEC && a.g && active && !(j[3] & 1);
  const int J3 = j[3] >> 1;
  T g5[5];
#pragma unroll
  for (int d = 0; d < 5; d++) g5[d] = (DEC && a.g && !(j[3] & 1)) ? a.ax[3].w5[5 * J3 + d] : T(0);
  const int64_t gplane = (int64_t)m1 * m2 * c3;
  const int64_t grow = ((int64_t)j[1] * m2 + j[2]) * c3 + J3;
  // the sweep output of plane p from the lane's value v of that plane (all
  // lanes shuffle; the even lanes store)
  auto sweep3 = [&](int p, T v) {
    if (!DEC || !a.g) return;
    T x[5];
    x[0] = __shfl_up(v, 2);
    x[1] = __shfl_up(v, 1);
    x[2] = v;
    x[3] = __shfl_down(v, 1);
    x[4] = __shfl_down(v, 2);
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < 5; d++) {
      const int jj = j[3] + d - 2;
      if (jj < 0 || jj >= m3) continue;
      acc += g5[d] * x[d];
    }
    if (gout) a.g[(int64_t)p * gplane + grow] = acc;
  };
  // decompose: store coefficient c at u_mc offset u (and / or its label)
  auto put = [&](int64_t u, T c) {
    if (!LAB || umc_w) umc_w[u] = c;
    if (LAB) {
      const int32_t l = label4<T>(c, a.qc);
      lab_w[u] = l;
      if (l == INT32_MIN && a.rng) count_range4(a.rng, c, a.qc);
    }
  };
  // recompose: a pair's coefficient words stay raw (labels) until used
  using W = typename std::conditional<(!DEC && LAB), int32_t, T>::type;
  auto val = [&](W w) -> T {
    if constexpr (!DEC && LAB)
      return unlabel4<T>(w, a.qc);
    else
      return w;
  };
  const W *__restrict__ cw = DEC ? nullptr : (LAB ? (const W *)lab_r : (const W *)umc_r);
  // this chunk's pairs (even plane 2J, odd plane 2J+1), J0 <= J < J1; the
  // last chunk also takes the last even plane
  const int npair = cc0 - 1;
  const int J0 = (int)by * a.jchunk;
  const int J1 = min(npair, J0 + a.jchunk);
  const bool last = J1 == npair;
  // the words of pair J: the corners of Q in plane 2J+2 (DEC) or J+1 (REC,
  // coarse), the even plane's value and the odd plane's; plane indices are
  // clamped into the box for J = npair (only its even value is used)
  struct Words {
    T q[4];
    W e, o;
  };
  const int plast = DEC ? 2 * npair : npair;  // the last even plane (fine or coarse index)
  auto fetch = [&](int J, Words &w) {
    const T *b = src + (int64_t)min(DEC ? 2 * J + 2 : J + 1, plast) * plane;
#pragma unroll
    for (int c = 0; c < 4; c++) w.q[c] = b[coff[c]];
    if constexpr (DEC) {
      w.e = V[(int64_t)(2 * J) * plane + vcol];
      w.o = V[(int64_t)min(2 * J + 1, plast) * plane + vcol];
    } else {
      w.e = cw[(int64_t)J * a.up[0] + ucol];
      w.o = cw[(int64_t)(cc0 + min(J, npair - 1)) * a.up[0] + ucol];
    }
  };
  T qprev;
  {
    const T *b = src + (int64_t)(DEC ? 2 * J0 : J0) * plane;
    T x[4];
#pragma unroll
    for (int c = 0; c < 4; c++) x[c] = b[coff[c]];
    qprev = Qof(x);
  }
  auto pair = [&](int J, const Words &w) {
    const int je = 2 * J;
    const T qnext = Qof(w.q);
    const int64_t u = (int64_t)(cc0 + J) * a.up[0] + ucol;
    const T pred = ldu4(a.ax[0].wl, je + 1) * qprev + ldu4(a.ax[0].wr, je + 1) * qnext;
    if (DEC) {
      sweep3(je, val(w.e));
      sweep3(je + 1, val(w.o));
    }
    if (active) {
      if (DEC) {
        if (odd) put((int64_t)J * a.up[0] + ucol, val(w.e) - qprev);
        put(u, val(w.o) - pred);
      } else {
        out[je * a.op[0] + ocol] = odd ? val(w.e) + qprev : qprev;
        out[(je + 1) * a.op[0] + ocol] = val(w.o) + pred;
      }
    }
    qprev = qnext;
  };
  // the last (even) plane, from the words of pair J1
  auto finish = [&](const Words &w) {
    if (!last) return;
    const int J = J1;
    if (DEC) sweep3(2 * J, val(w.e));
    if (!active) return;
    if (DEC) {
      if (odd) put((int64_t)J * a.up[0] + ucol, val(w.e) - qprev);
    } else {
      out[(2 * J) * a.op[0] + ocol] = odd ? val(w.e) + qprev : qprev;
    }
  };
  Words w0, w1, w2;
  fetch(J0, w0);
  fetch(min(J0 + 1, J1), w1);
  for (int J = J0;;) {
    if (J == J1) {
      finish(w0);
      break;
    }
    fetch(min(J + 2, J1), w2);
    pair(J, w0);
    if (++J == J1) {
      finish(w1);
      break;
    }
    fetch(min(J + 2, J1), w0);
    pair(J, w1);
    if (++J == J1) {
      finish(w2);
      break;
    }
    fetch(min(J + 2, J1), w1);
    pair(J, w2);
    ++J;
  }
}

// One output per thread and step of a grid-stride loop, kSweepU steps taken
// together: their inputs are all loaded (at positions clamped into the row or
// the array, without branches) before any output is computed or stored, so a
// thread has kSweepU outputs' loads in flight instead of one's.  The terms are
// summed as before (a term outside the row, or at a nodal node of a gathered
// row, is skipped), in the same order.
constexpr int kSweepU = 4;
constexpr int kSweepLdsW = 2560;
// The sweep's loop; weights from wt_src (LDS or global, per WLDS).
template <typename T, bool GATHER, bool LABG, bool WLDS>
__device__ __forceinline__ void sweep4_body(const Sweep4Args<T> &a, const T *__restrict__ wt_src) {
  // LABG: the gathered inputs are labels, raw until summed
  using W = typename std::conditional<LABG, int32_t, T>::type;
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  const uint64_t lb = xcd_block4(blockIdx.x, gridDim.x);  // neighbouring blocks under one L2
  for (uint64_t i0 = lb * 256u + threadIdx.x; i0 < a.n; i0 += kSweepU * stride) {
    W x[kSweepU][5];
    T wt[kSweepU][5];  // the stencil weights, read with the inputs
    int Js[kSweepU];
    bool skipn[kSweepU];  // gather: a nodal row, whose even inputs are zero
#pragma unroll
    for (int u = 0; u < kSweepU; u++) {
      const uint64_t iu = i0 + (uint64_t)u * stride;
      const uint32_t i = (uint32_t)min(iu, (uint64_t)a.n - 1);
      // the gathering sweep runs along the contiguous axis (inner = 1)
      const uint32_t t = GATHER ? i : udiv(i, a.dinner);
      const uint32_t ii = GATHER ? 0u : i - t * a.inner;
      const uint32_t o = udiv(t, a.dc);
      const int J = (int)(t - o * (uint32_t)a.c);
      Js[u] = J;
      skipn[u] = false;
#pragma unroll
      for (int d = 0; d < 5; d++) {
        if constexpr (WLDS)
          wt[u][d] = ((const __attribute__((address_space(3))) T *)wt_src)[5 * J + d];
        else
          wt[u][d] = wt_src[5 * J + d];
      }
      if constexpr (!GATHER) {
        const T *row = a.in + (int64_t)o * a.m * a.inner + ii;
#pragma unroll
        for (int d = 0; d < 5; d++) {
          const int jj = min(max(2 * J + d - 2, 0), a.m - 1);
          x[u][d] = row[(int64_t)jj * a.inner];
        }
      } else {
        // o = (j0 m1 + j1) m2 + j2 of the level box; the sweep runs along axis 3
        const uint32_t r = udiv(o, a.dm2);
        const int j2 = (int)(o - r * (uint32_t)a.m2);
        const int j0 = (int)udiv(r, a.dm1);
        const int j1 = (int)(r - (uint32_t)j0 * (uint32_t)a.m1);
        skipn[u] = ((j0 | j1 | j2) & 1) == 0;
        auto lc = [&](int j, int k) { return (j & 1) ? a.cc[k] + (j >> 1) : (j >> 1); };
        // element indices in 32 bits (4-D boxes hold fewer than 2^32 nodes)
        const uint32_t base = (uint32_t)lc(j0, 0) * (uint32_t)a.up[0] + (uint32_t)lc(j1, 1) * (uint32_t)a.up[1] +
                              (uint32_t)lc(j2, 2) * (uint32_t)a.up[2];
        // taps 2J-2 .. 2J+2 along axis 3: even ones at J-1, J, J+1 of the row's
        // even part, odd ones at J-1, J of its odd part (from cc[3]); a tap
        // outside the axis reads a node inside it and is dropped by its weight
        const uint32_t Jm = max(J - 1, 0), Jp = min(J + 1, a.c - 1), Jo = min(J, a.c - 2);
        const uint32_t qo = base + (uint32_t)a.cc[3];
        const uint32_t q[5] = {base + Jm, qo + Jm, base + (uint32_t)J, qo + Jo, base + Jp};
#pragma unroll
        for (int d = 0; d < 5; d++) {
          if constexpr (LABG)
            x[u][d] = a.lab[q[d]];
          else
            x[u][d] = (W)a.umc[q[d]];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kSweepU; u++) {
      const uint64_t iu = i0 + (uint64_t)u * stride;
      if (iu >= a.n) break;
      const int J = Js[u];
      T acc = T(0);
#pragma unroll
      for (int d = 0; d < 5; d++) {
        // taps outside the axis, and (gather) nodal nodes, whose component is
        // zero, add nothing; selected rather than branched around
        const bool in = d < 2 ? J > 0 : (d > 2 ? J < a.c - 1 : true);
        const bool use = in && !(GATHER && skipn[u] && (d & 1) == 0);
        T v;
        if constexpr (LABG)
          v = unlabel4<T>(x[u][d], a.qc);
        else
          v = x[u][d];
        const T acc1 = acc + wt[u][d] * v;
        acc = use ? acc1 : acc;
      }
      a.out[iu] = acc;
    }
  }
}

// The stencil weights of the axis (5 per output index) are copied to LDS
// when they fit kSweepLdsW entries, so that only the inputs go through the
// texture/address units (the sweeps are bound by their load instructions).
// The stencil weights of the axis (5 per output index) are copied to LDS
// when they fit kSweepLdsW entries, so that only the inputs go through the
// texture/address units (the sweeps are bound by their load instructions).
template <typename T, bool GATHER, bool LABG>
__global__ void __launch_bounds__(256) k_sweep4(Sweep4Args<T> a) {
  __shared__ T s_w[kSweepLdsW];
  if (5 * a.c <= kSweepLdsW) {
    for (int k = threadIdx.x; k < 5 * a.c; k += 256) s_w[k] = a.w5[k];
    __syncthreads();
    sweep4_body<T, GATHER, LABG, true>(a, s_w);
  } else {
    sweep4_body<T, GATHER, LABG, false>(a, a.w5);
  }
}

// The same sweep as one march per (o, i) column along the axis (inner >=
// kSweepMarchInner: consecutive threads on consecutive i, coalesced): output J
// needs inputs 2J-2 .. 2J+2, of which 2J-2 .. 2J carry over from output J-1,
// so each input row is read once per chunk (plus two rows at its start).  The
// two new inputs of output J+1 are loaded before output J is computed and
// stored (two register pairs, the loop unrolled twice), so the march keeps
// one output's loads in flight; inputs outside the axis load a clamped
// position and count as zero.
template <typename T>
__global__ void __launch_bounds__(256) k_sweep4_march(Sweep4Args<T> a) {
  // logical block: each XCD takes a contiguous range of columns (as k_coef4)
  const uint64_t lb = xcd_block4(blockIdx.x + (uint64_t)blockIdx.y * gridDim.x, (uint64_t)gridDim.x * gridDim.y);
  const uint64_t bx = lb % gridDim.x, by = lb / gridDim.x;
  const uint64_t col = bx * 256u + threadIdx.x;
  const uint64_t ncol = (uint64_t)a.n / (uint64_t)a.c;  // outer * inner
  if (col >= ncol) return;
  const uint32_t o = udiv((uint32_t)col, a.dinner);
  const uint32_t ii = (uint32_t)col - o * a.inner;
  const T *__restrict__ row = a.in + (int64_t)o * a.m * a.inner + ii;
  T *__restrict__ out = a.out + (int64_t)o * a.c * a.inner + ii;
  const T *__restrict__ w5 = a.w5;
  const int64_t inner = a.inner;
  const int m = a.m;
  auto ld = [&](int j) { return row[(int64_t)min(max(j, 0), m - 1) * inner]; };
  auto x = [&](int j, T v) { return (j >= 0 && j < m) ? v : T(0); };
  const int J0 = (int)by * a.jchunk, J1 = min(a.c, J0 + a.jchunk);
  if (J0 >= J1) return;
  T xm2 = x(2 * J0 - 2, ld(2 * J0 - 2)), xm1 = x(2 * J0 - 1, ld(2 * J0 - 1)), x0 = x(2 * J0, ld(2 * J0));
  auto step = [&](int J, T r1, T r2) {
    const T x1 = x(2 * J + 1, r1), x2 = x(2 * J + 2, r2);
    // J is the same on every lane: the weights come through scalar loads
    T acc = T(0);
    if (2 * J - 2 >= 0) acc += ldu4(w5, 5 * J) * xm2;
    if (2 * J - 1 >= 0) acc += ldu4(w5, 5 * J + 1) * xm1;
    acc += ldu4(w5, 5 * J + 2) * x0;
    if (2 * J + 1 < m) acc += ldu4(w5, 5 * J + 3) * x1;
    if (2 * J + 2 < m) acc += ldu4(w5, 5 * J + 4) * x2;
    out[(int64_t)J * inner] = acc;
    xm2 = x0;
    xm1 = x1;
    x0 = x2;
  };
  T a1 = ld(2 * J0 + 1), a2 = ld(2 * J0 + 2), b1, b2;
  for (int J = J0;;) {
    b1 = ld(2 * J + 3);
    b2 = ld(2 * J + 4);
    step(J, a1, a2);
    if (++J == J1) break;
    a1 = ld(2 * J + 3);
    a2 = ld(2 * J + 4);
    step(J, b1, b2);
    if (++J == J1) break;
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

// Four consecutive destination nodes per thread: one index split per four
// nodes (the split was most of the per-node work), the four source reads
// issued together, one 16-byte store (two for FP64) where the four are whole.
// A quad that runs past a destination row's end continues in the next row.
template <typename T>
__global__ void __launch_bounds__(256) k_pad4(Pad4Args<T> a) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  const uint32_t nq = (a.n + 3u) / 4u;
  const int n1 = a.ndst[1], n2 = a.ndst[2], n3 = a.ndst[3], s3 = a.nsrc[3];
  const bool vec = ((uintptr_t)a.dst & 15u) == 0;
  for (uint64_t t = (uint64_t)blockIdx.x * 256u + threadIdx.x; t < nq; t += stride) {
    const uint32_t i0 = (uint32_t)t * 4u;
    int j[4];
    split4(i0, a.d3, a.d2, a.d1, j);
    // source row of destination row (j0, j1, j2), the last real one past the edges
    auto srow = [&]() -> int64_t {
      int64_t r = 0;
#pragma unroll
      for (int k = 0; k < 3; k++) r = r * a.nsrc[k] + min(j[k], a.nsrc[k] - 1);
      return r * s3;
    };
    int64_t rb = srow();
    int col = j[3];
    T v[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
      if (col == n3) {  // into the next destination row
        col = 0;
        if (++j[2] == n2) {
          j[2] = 0;
          if (++j[1] == n1) {
            j[1] = 0;
            ++j[0];
          }
        }
        rb = srow();
      }
      const bool in = i0 + (uint32_t)e < a.n;
      v[e] = a.src[in ? rb + min(col, s3 - 1) : 0];
      ++col;
    }
    if (vec && i0 + 4u <= a.n) {
      if constexpr (sizeof(T) == 4) {
        *(float4 *)(a.dst + i0) = make_float4(v[0], v[1], v[2], v[3]);
      } else {
        *(double2 *)(a.dst + i0) = make_double2(v[0], v[1]);
        *(double2 *)(a.dst + i0 + 2) = make_double2(v[2], v[3]);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; e++)
        if (i0 + (uint32_t)e < a.n) a.dst[i0 + e] = v[e];
    }
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
  const dim3 grid((a.ncol + 4 * kCoefCols - 1) / (4 * kCoefCols), a.nchunk);
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
  const unsigned g = grid_for((a.n + kSweepU - 1) / kSweepU);
  if (gather && a.lab)
    hipLaunchKernelGGL((k_sweep4<T, true, true>), dim3(g), dim3(256), 0, st, a);
  else if (gather)
    hipLaunchKernelGGL((k_sweep4<T, true, false>), dim3(g), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_sweep4<T, false, false>), dim3(g), dim3(256), 0, st, a);
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
  // one quad per thread: a grid-stride loop would make each iteration's reads
  // wait for the previous iteration's stores (one vector memory counter)
  const uint64_t g = ((uint64_t)a.n + 1023) / 1024;
  hipLaunchKernelGGL((k_pad4<T>), dim3((unsigned)(g > 0 ? g : 1)), dim3(256), 0, st, a);
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
