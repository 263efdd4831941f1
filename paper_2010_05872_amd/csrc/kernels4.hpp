// Four-axis fields (the 4-D QMCPACK field of Sec. 6, Table 2): kernel
// argument blocks and launchers (internal to libmgx).
//
// Boxes are C order (n0, n1, n2, n3) with axis 3 contiguous.  Every level
// box is compact except u_mc, which keeps the finest grid's pitches.  Flat
// element indices are 32-bit (a box holds fewer than 2^32 nodes) and split
// into axis indices by multiplication with precomputed magics.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace mgx {

// Exact n / d for n, d < 2^32: mag = ceil(2^64 / d) (d = 1: mag = 0, n / 1 = n).
struct Div32 {
  uint32_t d = 1;
  uint64_t mag = 0;
};
inline Div32 make_div32(uint32_t d) {
  Div32 v;
  v.d = d;
  v.mag = d < 2 ? 0 : (~(uint64_t)0) / d + 1;
  return v;
}

template <typename T>
struct Axis4 {
  const T *wl, *wr;  // interpolation weights of the left / right nodal neighbour at odd nodes [m]
  const T *w5;       // the R M stencil, 5 per coarse node [5c]
  int m, c;          // level-l and level-(l-1) node counts
};

// Coefficients of one level (decomposition) or its recomposition, one
// thread per column (j1, j2, j3) of the level-l box, marching along axis 0.
//   decompose: u_mc[lc(j)] = V(j) - Pi V(j) at every coefficient node j
//   recompose: out(j) = u_mc[lc(j)] + Pi nodal(j) at coefficient nodes,
//              out(j) = nodal(j / 2) at nodal nodes
// Pi: the multilinear interpolant from the 2^(#odd axes) nodal corners.
template <typename T>
struct Coef4Args {
  Axis4<T> ax[4];
  const T *V;           // decompose: level-l box, compact
  const T *nodal;       // recompose: corrected nodal values, compact (c0, c1, c2, c3)
  T *umc_w;             // decompose: u_mc out
  const T *umc_r;       // recompose: u_mc in
  int64_t up[3];        // u_mc pitches of axes 0..2
  T *out;               // recompose: level-l box out
  int64_t op[3];        // its pitches
  uint32_t ncol;        // m1 m2 m3
  Div32 d3, d2;         // by m3, m2
  int jchunk, nchunk;   // plane pairs per chunk of the march, chunks (nchunk * jchunk >= c0 - 1)
  // quantization labels (u_mc's layout) of the level's coefficients, bin
  // width qc: decompose writes them (umc_w may then be null), recompose reads
  // them instead of u_mc
  int32_t *lab_w;
  const int32_t *lab_r;
  double qc;
  // decompose with labels: counts of labels set to INT32_MIN, [0] finite
  // |c/q| >= 2^31 - 1, [1] c/q not finite (null: not counted)
  unsigned long long *rng;
  // decompose (nullable): also the first load-vector sweep, R M along axis 3
  // of the level box, out (m0, m1, m2, c3) compact, as k_sweep4 computes it
  T *g;
};

// One load-vector sweep R M along one axis: in (outer, m, inner) ->
// out (outer, c, inner), both compact: out(o, J, i) = sum_d w5[5J + d] in(o, 2J + d - 2, i).
// GATHER (the first recomposition sweep, along axis 3): the input is the
// level's multilevel component, u_mc at level-centric positions and zero at
// nodal nodes; then outer = m0 m1 m2 and inner = 1.
template <typename T>
struct Sweep4Args {
  const T *w5;
  int m, c;
  const T *in;
  T *out;
  uint32_t n;          // outer * c * inner
  uint32_t inner;
  Div32 dinner, dc;    // by inner, by c
  // gather only
  const T *umc;
  int64_t up[3];
  int m1, m2;          // level box sizes of axes 1, 2
  int cc[4];           // level-(l-1) node counts (level-centric offsets of odd indices)
  Div32 dm2, dm1;      // by m2, m1
  const int32_t *lab;  // non-null: read labels (times qc) instead of u_mc
  double qc;
  // march form (inner >= kSweepMarchInner, no gather): one thread per (o, i)
  // column and chunk of jchunk outputs along the axis
  int jchunk, nchunk;
};
constexpr int kSweepMarchInner = 32;

// 4-D box copy with pitches (axis 3 contiguous on both sides).  With lab_r
// the values are labels (at the source's positions) times q; with lab_w the
// values' labels are written at the destination's positions (dst may then
// be null).
template <typename T>
struct Copy4Args {
  const T *src;
  int64_t sp[3];
  T *dst;
  int64_t dp[3];
  uint32_t n;          // b0 b1 b2 b3
  int b[4];
  Div32 d3, d2, d1;
  const int32_t *lab_r;
  int32_t *lab_w;
  double q;
  unsigned long long *rng;  // with lab_w: out-of-range counts as Coef4Args::rng (nullable)
};

// Quantization of a 4-D u_mc (level-centric layout), Sec. 4.1: the level of
// a position is the largest of its axes' levels; label = rint(c / q_l) in FP64.
struct Quant4Args {
  uint32_t n;          // n0 n1 n2 n3
  int nd[4];
  Div32 d3, d2, d1;
  int off[4];          // log2(n_k - 1) - L per axis
  int first, nlev;
  double q[kMaxLevelsK];
  int *stats_max;      // [nlev], nullable (no statistics)
  unsigned long long *stats_ovf, *stats_nan;
};

// Edge padding of a non-dyadic 4-D box to a dyadic one (each dummy node takes
// the value of the nearest real node): destination node j takes source node
// min(j, nsrc - 1) on every axis.  With nsrc >= ndst the same gather crops.
template <typename T>
struct Pad4Args {
  const T *src;
  T *dst;
  int nsrc[4], ndst[4];
  uint32_t n;          // destination node count
  Div32 d3, d2, d1;    // by the destination's dims 3, 2, 1
};

template <typename T> hipError_t launch_coef4(Coef4Args<T> a, bool dec, hipStream_t st);  // labels: a.lab_w / a.lab_r
template <typename T> hipError_t launch_sweep4(Sweep4Args<T> a, bool gather, hipStream_t st);
template <typename T> hipError_t launch_copy4(Copy4Args<T> a, hipStream_t st);
template <typename T> hipError_t launch_quantize4(const T *umc, int32_t *labels, Quant4Args a, hipStream_t st);
template <typename T> hipError_t launch_dequantize4(const int32_t *labels, T *umc, Quant4Args a, hipStream_t st);
template <typename T> hipError_t launch_pad4(Pad4Args<T> a, hipStream_t st);

}  // namespace mgx
