// HIP kernels for gfx950 (MI355X): multilevel decomposition / recomposition
// (arXiv 2010.05872, Sec. 2 and Sec. 5) and level-wise quantization (Sec. 4.1).
//
// One decomposition level l (box m0 x m1 x m2 -> coarse c0 x c1 x c2) runs as
//   k_load_vector<DEC>  the coefficients c = V - Pi_{l-1} V on N*_l, stored at
//                       their level-centric positions (Sec. 5.1) and / or as
//                       quantization labels, and the load vector
//                       F = (R M)^{x3} V, in one pass over the level box
//                       (z-march over tiles staged in LDS);
//   k_solve_contig      coarse mass-matrix solve along the contiguous axis
//                       (one wavefront scan of the Thomas recurrences);
//   k_solve_twisted     solves along the strided axes (two-ended Thomas, one
//                       line per lane, up to 65 nodes; k_solve_seg from 129
//                       nodes, MGX_SEG_MINC: segments of a line on the waves of
//                       a workgroup; k_solve_strided for the longest), the
//                       last one storing Q_{l-1} u = M_c^{-1} F.
// Mass apply, restriction and the solve act on different tensor axes, so the
// three load-vector stencils run first, on the fine grid, and the three
// solves afterwards on the 8x smaller coarse grid.  Recomposition uses
// k_load_vector<REC> on the stored coefficients (or labels), the same solves
// with the correction subtracted, and k_interp_plane / k_interp_add.  Levels
// whose boxes fit in LDS run in one workgroup (k_tail_dec / k_tail_rec).
// Also here: the quantization passes, the adjoint's prolongation
// (k_prolong_mass), the adaptive decomposition's estimate, the dummy-node
// padding.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.hpp"
#include "levelpos.hpp"

// Tuning parameters (compile-time; overridable with -D for measurements).
#ifndef MGX_STENCIL_DEPTH
#define MGX_STENCIL_DEPTH 2
#endif
#ifndef MGX_INTERP_PLANE
#define MGX_INTERP_PLANE 1
#endif
#ifndef MGX_INTERP_NP
#define MGX_INTERP_NP 2
#endif
#ifndef MGX_INTERP_AHEAD
#define MGX_INTERP_AHEAD 2
#endif
#ifndef MGX_REC_DEPTH
#define MGX_REC_DEPTH 4
#endif
#ifndef MGX_STENCIL_WAVES
#define MGX_STENCIL_WAVES 4
#endif
#ifndef MGX_REC_WAVES
#define MGX_REC_WAVES MGX_STENCIL_WAVES
#endif
#ifndef MGX_SEG_MINC  // shortest strided lines solved in segments over several waves
#define MGX_SEG_MINC 129
#endif
#ifndef MGX_DEEP_CH
#define MGX_DEEP_CH 32
#endif
#ifndef MGX_F32_TX
#define MGX_F32_TX 32
#endif
#ifndef MGX_F32_TY
#define MGX_F32_TY 16
#endif
#ifndef MGX_F32_DEC_TX
#define MGX_F32_DEC_TX 64
#endif
#ifndef MGX_F32_DEC_TY
#define MGX_F32_DEC_TY 8
#endif
#ifndef MGX_F32_DEC_NT
#define MGX_F32_DEC_NT MGX_F32_NT
#endif
#ifndef MGX_F32_RECLAB_TX
#define MGX_F32_RECLAB_TX 32
#endif
#ifndef MGX_F32_RECLAB_TY
#define MGX_F32_RECLAB_TY 16
#endif
#ifndef MGX_F32_INTERP_TX
#define MGX_F32_INTERP_TX 64
#endif
#ifndef MGX_F32_INTERP_TY
#define MGX_F32_INTERP_TY 8
#endif
#ifndef MGX_F32_NT
#define MGX_F32_NT 512
#endif
#ifndef MGX_F64_TY
#define MGX_F64_TY 16
#endif
#ifndef MGX_F64_NT
#define MGX_F64_NT 256
#endif

namespace mgx {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Give every XCD a contiguous range of logical tiles so that tiles that
// share halo rows run under the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, idx = b >> 3;
  const int base = xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q;
  return base + idx;
}

// Load of a uniform table entry through the constant address space: the
// compiler emits a scalar load (counted separately from vector memory
// operations), so waiting for it never waits for in-flight vector loads or
// stores.
template <typename T>
__device__ __forceinline__ T ldu(const T *p, int i) {
  return ((const __attribute__((address_space(4))) T *)p)[i];
}

// Element access at a 32-bit byte offset from a (wave-uniform) base pointer:
// lets the compiler use the scalar-base + 32-bit vector-offset addressing
// form instead of 64-bit per-lane address arithmetic.
template <typename T>
__device__ __forceinline__ T ld_at(const T *base, uint32_t byte_off) {
  return *(const T *)((const char *)base + byte_off);
}
template <typename T>
__device__ __forceinline__ void st_at(T *base, uint32_t byte_off, T v) {
  *(T *)((char *)base + byte_off) = v;
}

// The quantizer's decision for one coefficient: rint(c / q) in FP64 (a
// correctly rounded division, ties to even), INT32_MIN when out of range or
// not finite -- the same operations as the quantization pass, so labels
// written by the level kernels equal that pass's labels bit for bit.
template <typename T>
__device__ __forceinline__ int32_t label_of(T v, double q) {
  const double t = (double)v / q;
  return !(fabs(t) < 2147483647.0) ? INT32_MIN : (int32_t)rint(t);
}
// 1/q rounded to FP32 for the fast path below; NaN (fast path never taken)
// when it falls outside FP32's normal range.
__device__ __forceinline__ float label_rcp(double q) {
  const double r = 1.0 / q;
  return (r >= 1.1754943508222875e-38 && r <= 3.4028234663852886e38) ? (float)r : __builtin_nanf("");
}
// The same decision for an FP32 coefficient, mostly without the FP64
// division.  t = v * rq in FP32 is within about 2^-23 |v/q| of the exact
// quotient (two roundings of 2^-24, one in rq and one in the product), and
// the FP64 quotient within 2^-53 of it.  With r = rint(t), d = |t - r| is
// exact and 0.5 - d is t's distance to the nearest half-integer; when that
// exceeds |t| 2^-21, both quotients sit strictly inside the same interval
// between half-integers and round to r.  The test d + |t| 2^-21 < 0.5 is a
// single FMA (its rounding cannot turn a sum >= 0.5 into one below), it
// fails for |t| >= 2^20 (labels stay far inside int32) and for non-finite
// t; there *ok is false and the FP64 division decides.  Relies on IEEE
// subnormals (the kernels are compiled without flush to zero).
__device__ __forceinline__ int32_t label_fast(float v, float rq, bool &ok) {
  const float t = v * rq;
  const float r = rintf(t);
  ok = __builtin_fmaf(fabsf(t), 0x1p-21f, fabsf(t - r)) < 0.5f;
  return (int32_t)(ok ? r : 0.0f);
}
__device__ __forceinline__ int32_t label_fast(double, float, bool &ok) {
  ok = false;  // FP64 coefficients: always the division
  return 0;
}
template <typename T>
__device__ __forceinline__ int32_t label_of(T v, double q, float rq) {
  bool ok;
  const int32_t l = label_fast(v, rq, ok);
  if (__builtin_expect(ok, 1)) return l;
  return label_of<T>(v, q);
}
// Counts a coefficient whose label is INT32_MIN: rng[0] when c/q is finite
// (|c/q| >= 2^31 - 1), rng[1] when it is not.  Callers reach it only where the
// label came from the FP64 division, which fields without such coefficients
// take rarely or never.
template <typename T>
__device__ __forceinline__ void count_out_of_range(unsigned long long *rng, T v, double q) {
  const double t = (double)v / q;
  atomicAdd(&rng[(isnan(t) || isinf(t)) ? 1 : 0], 1ull);
}
// A coefficient from its label (the dequantization pass's operations).
template <typename T>
__device__ __forceinline__ T from_label(int32_t l, double q) {
  return (T)((double)l * q);
}
// Byte offset of the label of the element at byte offset off of a T array.
template <typename T>
__device__ __forceinline__ uint32_t lab_off(uint32_t off) {
  return sizeof(T) == 4 ? off : off >> 1;
}

// Two adjacent elements (a at byte offset off, b after it) in one store
// instruction, or only a.  The pair is aligned to the element size only (the
// offset of an odd row or an odd plane of an odd-pitch box is not a multiple
// of twice the element size); gfx9 global stores take such addresses.
template <typename T>
__device__ __forceinline__ void st_pair(T *base, uint32_t byte_off, T a, T b, bool two) {
  typedef T pair_t __attribute__((ext_vector_type(2), aligned(sizeof(T))));
  if (two) {
    pair_t v;
    v.x = a;
    v.y = b;
    *(pair_t *)((char *)base + byte_off) = v;
  } else {
    *(T *)((char *)base + byte_off) = a;
  }
}

// Column of region column q in a de-interleaved LDS row: even columns first,
// then odd ones (stride-1 reads in the restriction along x).
template <int TX>
__device__ __forceinline__ int zcol(int q) {
  return (q & 1) ? (TX + 3) + (q >> 1) : (q >> 1);
}

// Slot o of a (TY+1) x (TX+1) grid of per-tile work items (coarse outputs or
// 2x2 fine blocks): the TY x TX interior first, then the last column, then
// the last row.  Interior tiles own only the interior items, so with one
// item per thread every thread of such a tile gets exactly one and the
// per-thread loops over items are balanced across waves; slots past the
// grid give r = TY and c > TX (callers test o against the grid size).
template <int TX, int TY>
__device__ __forceinline__ void tile_slot(int o, int &r, int &c) {
  if (o < TX * TY) {
    r = o / TX;
    c = o - r * TX;
  } else if (o < TX * TY + TY + 1) {
    r = o - TX * TY;
    c = TX;
  } else {
    r = TY;
    c = o - (TX * TY + TY + 1);
  }
}

__device__ __forceinline__ int64_t lc_pos(int j, int c) {
  // level-centric position of level index j on an axis with c coarse nodes
  return (j & 1) ? (int64_t)c + (j >> 1) : (int64_t)(j >> 1);
}

// Returns v unchanged but opaque to the optimizer, so that per-element index
// arithmetic is recomputed inside plane loops instead of being hoisted into
// dozens of live registers (an empty asm statement: no instruction emitted).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// ---------------------------------------------------------------------------
// k_load_vector: load vector of one level (+ coefficients when decomposing)
// ---------------------------------------------------------------------------
//
// DEC: reads the level box V = Q_l u and
//   - writes the coefficients c = V - Pi_{l-1} V of the nodes in N*_l to
//     their level-centric positions (Sec. 2 steps 2-3, Sec. 5.1), and
//   - writes the load vector F = (R M)^{x3} V of V itself.  The solves then
//     give M_c^{-1} F = Q_{l-1} u directly: the correction of Sec. 2 step 4
//     equals Q_{l-1}u - Pi_{l-1}Q_l u, and R M P = M_c, so nodal values plus
//     correction is the L2 projection of V (identical up to rounding).
// REC: reads the stored coefficients z (zero on N_{l-1}) and writes
//   F = (R M)^{x3} z, whose solve is the correction of recomposition.
//
// Tile: coarse columns [X0,X1) x rows [Y0,Y1) x planes [Z0,Z1); the last tile
// along an axis also takes the final coarse node (c = 2^k+1).  The fine
// region read is [2Y0-2, 2Y1] x [2X0-2, 2X1] (restriction reach 2); the
// coefficients written are those of the owned nodes [2Y0, min(2Y1,m1)) x
// [2X0, min(2X1,m2)) of the owned planes.  The kernel marches over fine
// planes j = 2Z0-2 .. 2Z1; plane j adds its yx-restricted values into the
// load vector of the up to three coarse planes it touches.  Rows are stored
// de-interleaved in LDS (even columns first), so both the restriction and
// the interpolation corners read consecutive LDS words.  Planes are fetched
// DEPTH iterations ahead into register buffers.
// LAB: 0 no labels; 1 labels (decompose: written, recompose: read); 2
// (decompose) labels and the largest |label| written, reduced into a.smax.
// WC false: the coefficients are not written (a.umc_w is null), known at
// compile time, so the labels-only decomposition carries no per-node test.
template <typename T, int TX, int TY, int NT, bool DEC, int LAB, bool WC = true>
__device__ __forceinline__ void load_vector_body(const StencilArgs<T> a, const int lb) {
  constexpr int HR = 2 * TY + 5;  // region rows incl. halo and the extension
  constexpr int W = 2 * TX + 5;   // region row pitch
  constexpr int E = TX + 3;       // even columns of a region row
  constexpr int GW = TX + 1;      // coarse columns per tile (max)
  constexpr int GH = TY + 1;      // coarse rows per tile (max)
  constexpr int NE = (HR * W + NT - 1) / NT;  // region elements per thread
  constexpr int NV = DEC ? 4 : 2;             // ring of planes kept in LDS
  constexpr int AHEAD = DEC ? 2 : 1;          // plane committed at iteration j is j + AHEAD
  // register buffers in flight (FP64 recomposition: two, within 128 VGPRs)
  constexpr int DEPTH = DEC ? MGX_STENCIL_DEPTH : (sizeof(T) == 8 ? 2 : MGX_REC_DEPTH);
  constexpr int XRS = NT / GW;                // x-restriction: rows per sweep
  constexpr int XR = (HR + XRS - 1) / XRS;    // x-restriction: rows per thread
  constexpr int NOUT = (GH * GW + NT - 1) / NT;  // y-restriction outputs per thread
  constexpr int NB = NOUT;                       // 2x2 coefficient blocks per thread

  // a fetched word: a label when recomposing from labels, else a value
  using R = typename std::conditional<(!DEC && LAB != 0), int32_t, T>::type;
  __shared__ T sV[NV][HR * W];
  // x-restricted rows of the plane, double-buffered by plane parity: the one
  // barrier per plane then separates every LDS write from the reads of the
  // same words (x-restriction of plane j+2 vs y-restriction of plane j;
  // commit of plane j+AHEAD vs the reads of that slot one iteration before)
  __shared__ T sGbuf[2][HR * GW];

  const int tid = threadIdx.x;
  const int m0 = a.ax[0].m, m1 = a.ax[1].m, m2 = a.ax[2].m;
  const int c0 = a.ax[0].c, c1 = a.ax[1].c, c2 = a.ax[2].c;
  const int tx = lb % a.ntx;
  const int t2 = lb / a.ntx;
  const int ty = t2 % a.nty;
  const int tz = t2 / a.nty;
  const int X0 = tx * TX, X1 = (tx == a.ntx - 1) ? c2 : X0 + TX;
  const int Y0 = ty * TY, Y1 = (ty == a.nty - 1) ? c1 : Y0 + TY;
  const int Z0 = tz * a.tz, Z1 = (tz == a.nzc - 1) ? c0 : Z0 + a.tz;
  const int nX = X1 - X0, nY = Y1 - Y0;
  const int r0 = 2 * Y0 - 2, q0 = 2 * X0 - 2;  // fine row / column at region 0 (even)
  const int nr = 2 * nY + 3, nq = 2 * nX + 3;
  const int fr = min(2 * Y1, m1) - 2 * Y0;  // owned fine rows
  const int fq = min(2 * X1, m2) - 2 * X0;  // owned fine columns
  const int own_p0 = 2 * Z0, own_p1 = min(2 * Z1, m0);
  const float rq = a.rqc;

  // ---- plane loads: global and LDS offsets of this thread's NE region
  //      elements (the same in every plane) ----
  int goff[NE], loff[NE];
  unsigned valid = 0, inlds = 0, yxeven = 0;
#pragma unroll
  for (int k = 0; k < NE; k++) {
    const int idx = tid + NT * k;
    const int r = idx / W, q = idx - r * W;
    const int j1 = r0 + r, j2 = q0 + q;
    const bool in = idx < nr * W && q < nq && j1 >= 0 && j1 < m1 && j2 >= 0 && j2 < m2;
    valid |= (unsigned)in << k;
    inlds |= (unsigned)(idx < HR * W) << k;
    yxeven |= (unsigned)(!(j1 & 1) && !(j2 & 1)) << k;
    loff[k] = r * W + zcol<TX>(q);
    // byte offsets within a plane
    if (DEC)
      goff[k] = in ? (j1 * (int)a.vp1 + j2) * (int)sizeof(T) : 0;
    else
      goff[k] = in ? (int)(lc_pos(j1, c1) * a.up1 + lc_pos(j2, c2)) * (int)sizeof(T) : 0;
  }
  // issue the loads of fine plane j into registers.  Every lane issues every
  // load (masked lanes read a valid element), so the number of outstanding
  // memory operations is static and later waits can be partial.  The words
  // are kept raw (labels unconverted, masked lanes unmasked) until the
  // commit: an operation on a loaded value at the fetch would make the
  // compiler wait for the load there and drain the prefetch.
  auto fetch = [&](int j, R (&st)[NE]) {
    const bool pin = j >= 0 && j < m0;
    const T *base = DEC ? a.V + (int64_t)(pin ? j : 0) * a.vp0 : a.umc_r + (pin ? lc_pos(j, c0) : 0) * a.up0;
    const int32_t *lbase = (!DEC && LAB) ? a.lab_r + (pin ? lc_pos(j, c0) : 0) * a.up0 : nullptr;
    // recomposition: nodal nodes (all indices even) carry no multilevel
    // component; their lanes read the plane's first element instead (one
    // shared line) rather than the coarse corner
    const bool skip_nodal = !DEC && !(j & 1);
#pragma unroll
    for (int k = 0; k < NE; k++) {
      const uint32_t off = (skip_nodal && ((yxeven >> k) & 1u)) ? 0u : (uint32_t)goff[k];
      if constexpr (!DEC && LAB)
        st[k] = ld_at(lbase, lab_off<T>(off));
      else
        st[k] = ld_at(base, off);
    }
  };
  // the words of plane j into LDS slot `slot`: zeros outside the grid and,
  // when recomposing, at nodal nodes; labels times the bin width
  auto commit = [&](int slot, int j, const R (&st)[NE]) {
    const bool pin = j >= 0 && j < m0;
    const bool skip_nodal = !DEC && !(j & 1);
    const unsigned keep = pin ? (skip_nodal ? (valid & ~yxeven) : valid) : 0u;
#pragma unroll
    for (int k = 0; k < NE; k++) {
      // every element but the last of each thread lies in the region
      // ((NE - 1) NT < HR WL): only the last needs the (divergent) test
      if (k < NE - 1 || ((inlds >> k) & 1u)) {
        T v;
        if constexpr (!DEC && LAB)
          v = from_label<T>(st[k], a.qc);
        else
          v = st[k];
        sV[slot][loff[k]] = ((keep >> k) & 1u) ? v : T(0);
      }
    }
  };
  auto slot_of = [&](int j) { return (j + 4) % NV; };

  // ---- x-restriction role: coarse column xX, region rows xr0 + XRS i ----
  const int xX = tid % GW, xr0 = tid / GW;
  const bool xact = tid < XRS * GW && xX < nX;
  T xw[5];
#pragma unroll
  for (int d = 0; d < 5; d++) xw[d] = xact ? a.ax[2].w5[(X0 + xX) * 5 + d] : T(0);

  // ---- y-restriction role: coarse outputs (Y, X), weights and offsets ----
  T yw[NOUT][5];
  int foff[NOUT], ysrc[NOUT];
  unsigned yact = 0;
#pragma unroll
  for (int k = 0; k < NOUT; k++) {
    const int o = tid + NT * k;
    int Y, X;
    tile_slot<TX, TY>(o, Y, X);
    const bool act = o < GH * GW && Y < nY && X < nX;
    yact |= (unsigned)act << k;
#pragma unroll
    for (int d = 0; d < 5; d++) yw[k][d] = act ? a.ax[1].w5[(Y0 + Y) * 5 + d] : T(0);
    foff[k] = act ? ((Y0 + Y) * (int)a.fp1 + X0 + X) * (int)sizeof(T) : 0;
    ysrc[k] = (2 * Y) * GW + X;
  }

  // ---- coefficient role (decomposition): 2x2 blocks of owned fine nodes
  //      (rows 2ca, 2ca+1; columns 2cb, 2cb+1) sharing their nodal corners ----
  int cR0[NB], cE0[NB], cRowE[NB], cColE[NB];
  T cwxl[NB], cwxr[NB], cwyl[NB], cwyr[NB];
  unsigned cn = 0;  // 4 bits per block: nodes 00, 01, 10, 11 inside the owned box
  if (DEC) {
#pragma unroll
    for (int k = 0; k < NB; k++) {
      const int o = tid + NT * k;
      int ca, cb;
      tile_slot<TX, TY>(o, ca, cb);
      const bool blk = o < GH * GW;
      const bool r0ok = blk && 2 * ca < fr, r1ok = blk && 2 * ca + 1 < fr;
      const bool q0ok = 2 * cb < fq, q1ok = 2 * cb + 1 < fq;
      cn |= (unsigned)((r0ok && q0ok) | ((r0ok && q1ok) << 1) | ((r1ok && q0ok) << 2) | ((r1ok && q1ok) << 3))
            << (4 * k);
      cR0[k] = (2 * ca + 2) * W;  // region row of owned row 2ca
      cE0[k] = cb + 1;            // de-interleaved position of region column 2cb+2 (even)
      cRowE[k] = (int)((Y0 + ca) * a.up1) * (int)sizeof(T);
      cColE[k] = (X0 + cb) * (int)sizeof(T);
      cwxl[k] = q1ok ? a.ax[2].wl[2 * X0 + 2 * cb + 1] : T(0);
      cwxr[k] = q1ok ? a.ax[2].wr[2 * X0 + 2 * cb + 1] : T(0);
      cwyl[k] = r1ok ? a.ax[1].wl[2 * Y0 + 2 * ca + 1] : T(0);
      cwyr[k] = r1ok ? a.ax[1].wr[2 * Y0 + 2 * ca + 1] : T(0);
    }
  }
  const int rowOdd = (int)(c1 * a.up1) * (int)sizeof(T);  // level-centric shift of odd rows (bytes)
  const int colOdd = c2 * (int)sizeof(T);                   // ... and of odd columns

  int lmax = 0;  // LAB == 2: largest |label| this thread wrote
  T acc[3][NOUT];
#pragma unroll
  for (int s = 0; s < 3; s++)
#pragma unroll
    for (int k = 0; k < NOUT; k++) acc[s][k] = T(0);

  // one plane of the march; st holds plane j + AHEAD on entry and receives
  // plane j + AHEAD + DEPTH on exit.  The commit of plane j + AHEAD goes to a
  // slot this iteration does not read (last read two iterations ago).
  auto plane = [&](int j, R (&st)[NE]) {
    commit(slot_of(j + AHEAD), j + AHEAD, st);
    const bool plane_in = (j >= 0 && j < m0);
    const int pz = j & 1;
    const int s0 = slot_of(j);
    T *const sG = sGbuf[j & 1];
    // ---- restriction along x of plane j: sG[r][X] ----
    if (plane_in && xact) {
#pragma unroll
      for (int i = 0; i < XR; i++) {
        const int r = xr0 + XRS * i;
        if (r < nr) {
          const int b = r * W + xX;
          sG[r * GW + xX] = xw[0] * sV[s0][b] + xw[1] * sV[s0][b + E] + xw[2] * sV[s0][b + 1] +
                            xw[3] * sV[s0][b + E + 1] + xw[4] * sV[s0][b + 2];
        }
      }
    }
    // ---- coefficients of the owned nodes of plane j (decomposition) ----
    if (DEC && (a.umc_w != nullptr || LAB) && plane_in && j >= own_p0 && j < own_p1) {
      T *const cbase = a.umc_w + lc_pos(j, c0) * a.up0;
      int32_t *const lbase = LAB ? a.lab_w + lc_pos(j, c0) * a.up0 : nullptr;
      const bool wc = WC && a.umc_w != nullptr;
      // the coefficients cv[p0..3] of one 2x2 block (nodes 00, 01, 10, 11 at
      // byte offsets oE + {0, colOdd, rowOdd, rowOdd + colOdd}) to u_mc and /
      // or their labels, for the nodes in f.  Labels are stored from the FP32
      // fast path; the rare ones it cannot decide are then overwritten (same
      // lane, same address: the stores stay in order) with the FP64 decision.
      auto emit = [&](const int p0, const unsigned f, const uint32_t oE, const T (&cv)[4]) {
        unsigned slow = 0;
#pragma unroll
        for (int p = p0; p < 4; p++) {
          const uint32_t off = oE + ((p & 1) ? colOdd : 0u) + ((p & 2) ? rowOdd : 0u);
          if ((f >> p) & 1u) {
            if (wc) st_at(cbase, off, cv[p]);
            if (LAB) {
              bool ok;
              const int32_t lf = label_fast(cv[p], rq, ok);
              st_at(lbase, lab_off<T>(off), lf);
              slow |= (unsigned)!ok << p;
              if (LAB == 2) lmax = max(lmax, lf < 0 ? -lf : lf);  // 0 where !ok
            }
          }
        }
        if (LAB && __builtin_expect(slow != 0u, 0)) {
#pragma unroll
          for (int p = p0; p < 4; p++)
            if ((slow >> p) & 1u) {
              const uint32_t off = oE + ((p & 1) ? colOdd : 0u) + ((p & 2) ? rowOdd : 0u);
              const int32_t lab = label_of<T>(cv[p], a.qc);
              st_at(lbase, lab_off<T>(off), lab);
              if (lab == INT32_MIN && a.rng) count_out_of_range(a.rng, cv[p], a.qc);
              if (LAB == 2 && lab != INT32_MIN) lmax = max(lmax, lab < 0 ? -lab : lab);
            }
        }
      };
      if (!pz) {
        // even plane: corners in the plane itself; node 00 is nodal
#pragma unroll
        for (int k = 0; k < NB; k++) {
          const unsigned f = (cn >> (4 * k)) & 0xEu;
          if (f) {
            const int R0 = cR0[k], R2 = cR0[k] + 2 * W, e0 = cE0[k];
            const T C00 = sV[s0][R0 + e0], C02 = sV[s0][R0 + e0 + 1];
            const T C20 = sV[s0][R2 + e0], C22 = sV[s0][R2 + e0 + 1];
            const T t0 = cwxl[k] * C00 + cwxr[k] * C02, t2 = cwxl[k] * C20 + cwxr[k] * C22;
            const T cv[4] = {T(0), sV[s0][R0 + E + e0] - t0, sV[s0][R0 + W + e0] - (cwyl[k] * C00 + cwyr[k] * C20),
                             sV[s0][R0 + W + E + e0] - (cwyl[k] * t0 + cwyr[k] * t2)};
            emit(1, f, (uint32_t)(cRowE[k] + cColE[k]), cv);
          }
        }
      } else {
        // odd plane: corners on the even planes j-1 and j+1
        const int sa = slot_of(j - 1), sb = slot_of(j + 1);
        const T wzl = ldu(a.ax[0].wl, j), wzr = ldu(a.ax[0].wr, j);
#pragma unroll
        for (int k = 0; k < NB; k++) {
          const unsigned f = (cn >> (4 * k)) & 0xFu;
          if (f) {
            const int R0 = cR0[k], R2 = cR0[k] + 2 * W, e0 = cE0[k];
            const T A00 = sV[sa][R0 + e0], A02 = sV[sa][R0 + e0 + 1], A20 = sV[sa][R2 + e0], A22 = sV[sa][R2 + e0 + 1];
            const T B00 = sV[sb][R0 + e0], B02 = sV[sb][R0 + e0 + 1], B20 = sV[sb][R2 + e0], B22 = sV[sb][R2 + e0 + 1];
            const T wxl = cwxl[k], wxr = cwxr[k], wyl = cwyl[k], wyr = cwyr[k];
            const T ta0 = wxl * A00 + wxr * A02, ta2 = wxl * A20 + wxr * A22;
            const T tb0 = wxl * B00 + wxr * B02, tb2 = wxl * B20 + wxr * B22;
            const T cv[4] = {
                sV[s0][R0 + e0] - (wzl * A00 + wzr * B00), sV[s0][R0 + E + e0] - (wzl * ta0 + wzr * tb0),
                sV[s0][R0 + W + e0] - (wzl * (wyl * A00 + wyr * A20) + wzr * (wyl * B00 + wyr * B20)),
                sV[s0][R0 + W + E + e0] - (wzl * (wyl * ta0 + wyr * ta2) + wzr * (wyl * tb0 + wyr * tb2))};
            emit(0, f, (uint32_t)(cRowE[k] + cColE[k]), cv);
          }
        }
      }
    }
    __syncthreads();
    // ---- restriction along y, accumulation along z ----
    if (plane_in) {
      const int Jc = j >> 1;  // j even: Z = Jc-1, Jc, Jc+1; j odd: Z = Jc, Jc+1
      T wz0, wz1, wz2;
      if (!pz) {
        wz0 = Jc - 1 >= 0 ? ldu(a.ax[0].w5, (Jc - 1) * 5 + 4) : T(0);
        wz1 = ldu(a.ax[0].w5, Jc * 5 + 2);
        wz2 = Jc + 1 < c0 ? ldu(a.ax[0].w5, (Jc + 1) * 5 + 0) : T(0);
      } else {
        wz0 = ldu(a.ax[0].w5, Jc * 5 + 3);
        wz1 = Jc + 1 < c0 ? ldu(a.ax[0].w5, (Jc + 1) * 5 + 1) : T(0);
        wz2 = T(0);
      }
#pragma unroll
      for (int k = 0; k < NOUT; k++) {
        if ((yact >> k) & 1u) {
          const int b = ysrc[k];
          const T gyx = yw[k][0] * sG[b] + yw[k][1] * sG[b + GW] + yw[k][2] * sG[b + 2 * GW] +
                        yw[k][3] * sG[b + 3 * GW] + yw[k][4] * sG[b + 4 * GW];
          acc[0][k] += wz0 * gyx;
          acc[1][k] += wz1 * gyx;
          acc[2][k] += wz2 * gyx;
        }
      }
    }
    // after an even plane j, coarse plane j/2 - 1 is complete
    if (!pz) {
      const int Zdone = (j >> 1) - 1;
      if (Zdone >= Z0 && Zdone < Z1) {
        T *const fbase = a.F + (int64_t)Zdone * a.fp0;
#pragma unroll
        for (int k = 0; k < NOUT; k++)
          if ((yact >> k) & 1u) st_at(fbase, (uint32_t)foff[k], acc[0][k]);
      }
#pragma unroll
      for (int k = 0; k < NOUT; k++) {
        acc[0][k] = acc[1][k];
        acc[1][k] = acc[2][k];
        acc[2][k] = T(0);
      }
    }
    // the loads for plane j + AHEAD + DEPTH are issued after every store of
    // this iteration, so the commit DEPTH iterations later needs a partial
    // wait only
    fetch(j + AHEAD + DEPTH, st);
  };

  const int jstart = 2 * Z0 - 2, jend = 2 * Z1;  // both even
  R st[DEPTH][NE];
  {
    // the planes before the march and the first DEPTH planes of it are all
    // requested before the first commit waits
    R p0[NE], p1[NE];
    fetch(jstart, p0);
    if (DEC) fetch(jstart + 1, p1);
#pragma unroll
    for (int d = 0; d < DEPTH; d++) fetch(jstart + AHEAD + d, st[d]);
    commit(slot_of(jstart), jstart, p0);
    if (DEC) commit(slot_of(jstart + 1), jstart + 1, p1);
  }
  __syncthreads();
  int j = jstart;
  for (; j + DEPTH - 1 <= jend; j += DEPTH) {
#pragma unroll
    for (int d = 0; d < DEPTH; d++) plane(j + d, st[d]);
  }
#pragma unroll
  for (int d = 0; d < DEPTH - 1; d++)
    if (j + d <= jend) plane(j + d, st[d]);
  if (LAB == 2) {  // the level's largest |label|: one atomic per wave
    for (int off = 32; off > 0; off >>= 1) lmax = max(lmax, __shfl_xor(lmax, off));
    if ((tid & 63) == 0 && lmax > 0) atomicMax(a.smax, lmax);
  }
}

template <typename T, int TX, int TY, int NT, bool DEC, int LAB, bool WC = true>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(DEC ? MGX_STENCIL_WAVES : MGX_REC_WAVES, 8)))
k_load_vector(StencilArgs<T> a) {
  if (a.gate && *a.gate == 0) return;
  load_vector_body<T, TX, TY, NT, DEC, LAB, WC>(a, xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// k_solve_contig: Thomas solve along the contiguous axis, one line per group
// of G lanes, E nodes per lane, line length c = G*E + 1.
// The forward elimination f'_J = f_J - mult_J f'_{J-1} and the back
// substitution y_J = invd_J f'_J - qsup_J y_{J+1} are first-order affine
// recurrences; each lane composes its E maps, the group scans the composed
// maps with shuffles, and each lane then replays its E steps.
// ---------------------------------------------------------------------------
template <typename T, int E, int G>
__device__ __forceinline__ void solve_contig_body(const SolveArgs<T> a, const int bx) {
  const int lane = threadIdx.x & 63;
  const int li = lane % G;
  const int64_t line = ((int64_t)bx * 4 + (threadIdx.x >> 6)) * (64 / G) + lane / G;
  const bool active = line < a.nlines;
  const int c = G * E + 1;
  T *row = a.F + (active ? line : 0) * a.pitch;
  const int J0 = li * E;

  T f[E], mu[E];
#pragma unroll
  for (int e = 0; e < E; e++) {
    f[e] = row[J0 + e];
    mu[e] = a.mult[J0 + e];  // mult[0] = 0: the first map is constant
  }
  // forward: compose x -> -mu x + f over the lane's nodes
  T A = T(1), B = T(0);
#pragma unroll
  for (int e = 0; e < E; e++) {
    A = -mu[e] * A;
    B = -mu[e] * B + f[e];
  }
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    T Ap = __shfl_up(A, off, G);
    T Bp = __shfl_up(B, off, G);
    if (li >= off) {
      B = A * Bp + B;
      A = A * Ap;
    }
  }
  T xin = __shfl_up(B, 1, G);  // state before the lane's first node
  if (li == 0) xin = T(0);
  T x = xin;
#pragma unroll
  for (int e = 0; e < E; e++) {
    x = -mu[e] * x + f[e];
    f[e] = x;  // f'
  }
  // last node c-1 on the group's last lane
  const T fl = row[c - 1];
  T ylast = a.invd[c - 1] * (fl - a.mult[c - 1] * x);
  ylast = __shfl(ylast, G - 1, G);
  // backward: x -> -qsup x + invd f' over nodes in descending order
  T iv[E], qs[E];
#pragma unroll
  for (int e = 0; e < E; e++) {
    iv[e] = a.invd[J0 + e];
    qs[e] = a.qsup[J0 + e];
  }
  A = T(1);
  B = T(0);
#pragma unroll
  for (int e = E - 1; e >= 0; e--) {
    A = -qs[e] * A;
    B = -qs[e] * B + iv[e] * f[e];
  }
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    T An = __shfl_down(A, off, G);
    T Bn = __shfl_down(B, off, G);
    if (li + off < G) {
      B = A * Bn + B;
      A = A * An;
    }
  }
  T An = __shfl_down(A, 1, G);
  T Bn = __shfl_down(B, 1, G);
  if (li == G - 1) {
    An = T(1);
    Bn = T(0);
  }
  x = An * ylast + Bn;
#pragma unroll
  for (int e = E - 1; e >= 0; e--) {
    x = -qs[e] * x + iv[e] * f[e];
    f[e] = x;
  }
  if (active) {
#pragma unroll
    for (int e = 0; e < E; e++) row[J0 + e] = f[e];
    if (li == G - 1) row[c - 1] = ylast;
  }
}

template <typename T, int E, int G>
__global__ void __launch_bounds__(256) k_solve_contig(SolveArgs<T> a) {
  if (a.gate && *a.gate == 0) return;
  solve_contig_body<T, E, G>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// k_solve_strided: Thomas solve along a strided axis of the coarse box.
// One thread per line, consecutive lanes on consecutive contiguous indices
// (coalesced rows).  The line is processed in chunks of CH nodes whose loads
// are issued together, the next chunk's loads before the current chunk's
// stores, so one memory latency is paid per chunk rather than per node.  The
// forward sweep writes f' in place; the backward sweep reads it back.  With
// APPLY the solution is not stored but added (sign +1, decomposition) or
// subtracted (sign -1, recomposition) to the nodal values: out = in + sign*y.
// ---------------------------------------------------------------------------
template <typename T, int MODE, int CH>
__device__ __forceinline__ void solve_strided_body(const StridedArgs<T> a, const int bx, const int o) {
  constexpr bool APPLY = MODE == kSolveApply;
  const int x = bx * 256 + threadIdx.x;
  if (x >= a.nx) return;
  T *p = a.F + (int64_t)o * a.so + x;
  const int c = a.c;
  const int64_t s = a.sj;
  const int nch = (c + CH - 1) / CH;
  T v[CH], w[CH];
  // ---- forward elimination ----
#pragma unroll
  for (int k = 0; k < CH; k++) v[k] = k < c ? p[k * s] : T(0);
  T fp = T(0);
  for (int ch = 0; ch < nch; ch++) {
    const int J0 = ch * CH;
    if (ch + 1 < nch) {
#pragma unroll
      for (int k = 0; k < CH; k++) w[k] = (J0 + CH + k < c) ? p[(int64_t)(J0 + CH + k) * s] : T(0);
    }
#pragma unroll
    for (int k = 0; k < CH; k++) {
      const int J = J0 + k;
      if (J < c) {
        fp = v[k] - a.mult[J] * fp;  // mult[0] = 0
        v[k] = fp;
      }
    }
#pragma unroll
    for (int k = 0; k < CH; k++)
      if (J0 + k < c) p[(int64_t)(J0 + k) * s] = v[k];
#pragma unroll
    for (int k = 0; k < CH; k++) v[k] = w[k];
  }
  // ---- back substitution, from the last chunk down ----
  T iv[CH], iw[CH];
  {
    const int J0 = (nch - 1) * CH;
#pragma unroll
    for (int k = 0; k < CH; k++) {
      const bool in = J0 + k < c;
      v[k] = in ? p[(int64_t)(J0 + k) * s] : T(0);
      if (APPLY) iv[k] = in ? a.in[(int64_t)(J0 + k) * a.ij + (int64_t)o * a.io + x] : T(0);
    }
  }
  T y = T(0);
  for (int ch = nch - 1; ch >= 0; ch--) {
    const int J0 = ch * CH;
    if (ch > 0) {
#pragma unroll
      for (int k = 0; k < CH; k++) {
        w[k] = p[(int64_t)(J0 - CH + k) * s];
        if (APPLY) iw[k] = a.in[(int64_t)(J0 - CH + k) * a.ij + (int64_t)o * a.io + x];
      }
    }
#pragma unroll
    for (int k = CH - 1; k >= 0; k--) {
      const int J = J0 + k;
      if (J < c) {
        y = a.invd[J] * v[k] - a.qsup[J] * y;  // qsup[c-1] = 0
        v[k] = y;
      }
    }
#pragma unroll
    for (int k = 0; k < CH; k++) {
      const int J = J0 + k;
      if (J < c) {
        if (APPLY)
          a.out[(int64_t)J * a.oj + (int64_t)o * a.oo + x] = iv[k] + a.sign * v[k];
        else if (MODE == kSolveStore)
          a.out[(int64_t)J * a.oj + (int64_t)o * a.oo + x] = v[k];
        else
          p[(int64_t)J * s] = v[k];
      }
    }
#pragma unroll
    for (int k = 0; k < CH; k++) {
      v[k] = w[k];
      if (APPLY) iv[k] = iw[k];
    }
  }
}

// ---------------------------------------------------------------------------
// k_solve_seg: Thomas solve along a strided axis for lines too long for the
// two-ended register solve.  Each line is cut into P = blockDim.x / 64
// segments of SEG nodes (the last segment also takes the final node): one
// wave per segment, one lane per line, lanes on consecutive lines, i.e. on
// consecutive contiguous indices (coalesced).  Both sweeps are first-order
// affine recurrences (forward f'_J = f_J - mult_J f'_{J-1}, backward
// y_J = invd_J f'_J - qsup_J y_{J+1}); every lane composes the maps of its
// segment in registers (f'_J = A_J + B_J f'_in, y_J = C_J + D_J y_out), the
// segments' maps are chained through LDS, and each lane replays its segment
// with the value entering it.  Every node is read once and written once.
// ---------------------------------------------------------------------------
constexpr int kSegMaxWaves = 16;

template <typename T, int SEG, int MODE>
__device__ __forceinline__ void solve_seg_body(const StridedArgs<T> a, const int b) {
  __shared__ T sA[kSegMaxWaves][64], sB[kSegMaxWaves][64];
  const int P = (int)(blockDim.x >> 6);
  const int lane = (int)(threadIdx.x & 63);
  const int s = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform: scalar table loads
  const int64_t line = (int64_t)b * 64 + lane;
  const bool act = line < (int64_t)a.nx * a.nouter;
  const int o = act ? (int)(line / a.nx) : 0;
  const int x = act ? (int)(line - (int64_t)o * a.nx) : 0;
  T *const p = a.F + (int64_t)o * a.so + x;
  const int64_t sj = a.sj;
  const int J0 = s * SEG;
  const bool last = s == P - 1;  // this segment also holds node c - 1
  T v[SEG + 1];
#pragma unroll
  for (int k = 0; k < SEG; k++) v[k] = act ? p[(int64_t)(J0 + k) * sj] : T(0);
  v[SEG] = (act && last) ? p[(int64_t)(J0 + SEG) * sj] : T(0);
  // apply: the nodal values are requested now and arrive during the solve (read
  // next to each store, every read would wait for the stores before it)
  T nod[MODE == kSolveApply ? SEG + 1 : 1];
  if (MODE == kSolveApply) {
    const T *const q = a.in + (int64_t)o * a.io + x;  // lanes past the lines read line 0
#pragma unroll
    for (int k = 0; k < SEG; k++) nod[k] = q[(int64_t)(J0 + k) * a.ij];
    if (last) nod[SEG] = q[(int64_t)(J0 + SEG) * a.ij];
  }
  // ---- forward: the segment's map from zero, and its multiplier ----
  T A = T(0), B = T(1);
#pragma unroll
  for (int k = 0; k < SEG; k++) {
    const T m = ldu(a.mult, J0 + k);  // mult[0] = 0
    A = v[k] - m * A;
    B = -m * B;
    v[k] = A;
  }
  if (last) {
    const T m = ldu(a.mult, J0 + SEG);
    A = v[SEG] - m * A;
    B = -m * B;
    v[SEG] = A;
  }
  sA[s][lane] = A;
  sB[s][lane] = B;
  __syncthreads();
  T fin = T(0);
  for (int t = 0; t < s; t++) fin = sA[t][lane] + sB[t][lane] * fin;
  __syncthreads();  // sA / sB are reused by the backward exchange
  {
    T Bk = T(1);
#pragma unroll
    for (int k = 0; k < SEG; k++) {
      Bk = -ldu(a.mult, J0 + k) * Bk;
      v[k] = v[k] + Bk * fin;
    }
    if (last) {
      Bk = -ldu(a.mult, J0 + SEG) * Bk;
      v[SEG] = v[SEG] + Bk * fin;
    }
  }
  // ---- backward: y from the segment's end (qsup[c-1] = 0 ends the line) ----
  T C = T(0), D = T(1);
  if (last) {
    C = ldu(a.invd, J0 + SEG) * v[SEG];
    D = T(0);
    v[SEG] = C;
  }
#pragma unroll
  for (int k = SEG - 1; k >= 0; k--) {
    const T q = ldu(a.qsup, J0 + k);
    C = ldu(a.invd, J0 + k) * v[k] - q * C;
    D = -q * D;
    v[k] = C;
  }
  sA[s][lane] = C;
  sB[s][lane] = D;
  __syncthreads();
  T yout = T(0);
  for (int t = P - 1; t > s; t--) yout = sA[t][lane] + sB[t][lane] * yout;
  {
    T Dk = last ? T(0) : T(1);
#pragma unroll
    for (int k = SEG - 1; k >= 0; k--) {
      Dk = -ldu(a.qsup, J0 + k) * Dk;
      v[k] = v[k] + Dk * yout;
    }
  }
  if (!act) return;
  auto put = [&](const int k, const T y) {
    const int J = J0 + k;
    if (MODE == kSolveApply)
      a.out[(int64_t)J * a.oj + (int64_t)o * a.oo + x] = nod[MODE == kSolveApply ? k : 0] + a.sign * y;
    else if (MODE == kSolveStore)
      a.out[(int64_t)J * a.oj + (int64_t)o * a.oo + x] = y;
    else
      p[(int64_t)J * sj] = y;
  };
#pragma unroll
  for (int k = 0; k < SEG; k++) put(k, v[k]);
  if (last) put(SEG, v[SEG]);
}

template <typename T, int SEG, int MODE>
__global__ void __launch_bounds__(64 * kSegMaxWaves) k_solve_seg(StridedArgs<T> a) {
  if (a.gate && *a.gate == 0) return;
  solve_seg_body<T, SEG, MODE>(a, blockIdx.x);
}

template <typename T, int MODE, int CH>
__global__ void __launch_bounds__(256) k_solve_strided(StridedArgs<T> a) {
  if (a.gate && *a.gate == 0) return;
  solve_strided_body<T, MODE, CH>(a, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// k_solve_twisted: Thomas solve along a strided axis of the coarse box as a
// two-ended ("twisted") factorization of the same tridiagonal matrix.  A
// workgroup takes 128 consecutive lines in (outer, x) order: waves 0-1
// eliminate rows 0..K-1 from the top, waves 2-3 rows C-1..K+1 from the
// bottom (C = 2K+1), each lane keeping its half line in registers; the two
// values next to the middle row K are swapped through LDS, the middle row is
// solved, and both halves back-substitute outwards.  A direct method (the
// same matrix factored from both ends), every element read once and written
// once; the row index is uniform per wave, so row offsets and the factor
// tables are scalar operands.
// ---------------------------------------------------------------------------
template <typename T, int C, int MODE>
__device__ __forceinline__ void solve_twisted_body(const StridedArgs<T> a, const int b) {
  constexpr int K = C / 2;
  __shared__ T sE[2][128];
  const int wave = threadIdx.x >> 6;
  const int half = wave >> 1;  // 0: top rows, 1: bottom rows (uniform per wave)
  const int line = (wave & 1) * 64 + (threadIdx.x & 63);
  // lines numbered over (outer, x) with x fastest, 128 per workgroup: no
  // workgroup is left nearly empty by an extent of 2^k + 1
  const int64_t g = (int64_t)b * 128 + line;
  const bool active = g < (int64_t)a.nx * a.nouter;
  const int o = active ? (int)(g / a.nx) : 0;
  const int x = active ? (int)(g - (int64_t)o * a.nx) : 0;
  T *p = a.F + (int64_t)o * a.so + x;
  const int64_t s = a.sj;
  T r[K];
  if (!half) {
#pragma unroll
    for (int i = 0; i < K; i++) r[i] = p[(int64_t)i * s];
  } else {
#pragma unroll
    for (int i = 0; i < K; i++) r[i] = p[(int64_t)(C - 1 - i) * s];
  }
  const T fK = p[(int64_t)K * s];
  T e = r[0];
  if (!half) {
#pragma unroll
    for (int i = 1; i < K; i++) {
      e = r[i] - a.mult[i] * e;
      r[i] = e;
    }
  } else {
#pragma unroll
    for (int i = 1; i < K; i++) {
      e = r[i] - a.multb[C - 1 - i] * e;
      r[i] = e;
    }
  }
  sE[half][line] = e;  // f'_{K-1} (top) or g'_{K+1} (bottom)
  __syncthreads();
  const T yK = a.mid[0] * (fK - a.mid[1] * sE[0][line] - a.mid[2] * sE[1][line]);
  T y = yK;
  if (!half) {
#pragma unroll
    for (int i = K - 1; i >= 0; i--) {
      y = a.invd[i] * r[i] - a.qsup[i] * y;
      r[i] = y;
    }
  } else {
#pragma unroll
    for (int i = K - 1; i >= 0; i--) {
      const int J = C - 1 - i;
      y = a.invdb[J] * r[i] - a.qsub[J] * y;
      r[i] = y;
    }
  }
  if (!active) return;
  if (MODE == kSolveApply || MODE == kSolveStore) {
    const T *in = a.in + (int64_t)o * a.io + x;
    T *out = a.out + (int64_t)o * a.oo + x;
    constexpr int CHA = 16;
#pragma unroll
    for (int i0 = 0; i0 < K; i0 += CHA) {
      T iv[CHA];
      if (MODE == kSolveApply) {
#pragma unroll
        for (int k = 0; k < CHA; k++) {
          const int i = i0 + k;
          if (i < K) iv[k] = in[(int64_t)(half ? C - 1 - i : i) * a.ij];
        }
      }
#pragma unroll
      for (int k = 0; k < CHA; k++) {
        const int i = i0 + k;
        if (i < K)
          out[(int64_t)(half ? C - 1 - i : i) * a.oj] = MODE == kSolveApply ? iv[k] + a.sign * r[i] : r[i];
      }
    }
    if (!half) out[(int64_t)K * a.oj] = MODE == kSolveApply ? in[(int64_t)K * a.ij] + a.sign * yK : yK;
  } else {
    if (!half) {
#pragma unroll
      for (int i = 0; i < K; i++) p[(int64_t)i * s] = r[i];
      p[(int64_t)K * s] = yK;
    } else {
#pragma unroll
      for (int i = 0; i < K; i++) p[(int64_t)(C - 1 - i) * s] = r[i];
    }
  }
}

template <typename T, int C, int MODE>
__global__ void __launch_bounds__(256) k_solve_twisted(StridedArgs<T> a) {
  if (a.gate && *a.gate == 0) return;
  solve_twisted_body<T, C, MODE>(a, blockIdx.x);
}

// Last step for one-dimensional fields (no strided solve): out = in + sign * F
// (recomposition) or out = F (decomposition) over a row of the coarse box.
template <typename T>
__device__ __forceinline__ void apply_body(const StridedArgs<T> a, const int bx) {
  const int x = bx * 256 + threadIdx.x;
  if (x >= a.nx) return;
  a.out[x] = a.in ? a.in[x] + a.sign * a.F[x] : a.F[x];
}

template <typename T>
__global__ void __launch_bounds__(256) k_apply(StridedArgs<T> a) {
  if (a.gate && *a.gate == 0) return;
  apply_body<T>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// k_interp_add: recomposition step 4 — Q_l u = coefficient + Pi_{l-1} of the
// corrected nodal values (and the nodal values themselves on N_{l-1}).
// Tile as in k_load_vector.  The kernel marches over coarse planes J with a
// four-slot LDS ring of nodal planes and emits fine planes 2J and 2J+1.
// Each thread owns 2x2 blocks of fine nodes (rows 2a, 2a+1; columns 2b,
// 2b+1) that share four nodal corners per coarse plane; its weights and
// offsets are fixed for the whole march, and the coefficients of the next
// coarse plane are fetched into registers while the current one is done.
// ---------------------------------------------------------------------------
template <typename T, int TX, int TY, int NT, bool LAB>
__device__ __forceinline__ void interp_add_body(const InterpArgs<T> a, const int lb) {
  constexpr int NW = TX + 2;  // nodal tile pitch
  constexpr int NH = TY + 2;
  constexpr int BW = TX + 1;  // 2x2 blocks per tile row (max)
  constexpr int BH = TY + 1;
  constexpr int NB = (BH * BW + NT - 1) / NT;
  constexpr int NN = (NH * NW + NT - 1) / NT;
  constexpr int NR = 4;  // nodal ring slots
  constexpr int AH = MGX_INTERP_AHEAD;  // steps of coefficients and nodal planes in flight
  __shared__ T sN[NR][NH * NW];

  const int tid = threadIdx.x;
  const int m0 = a.ax[0].m, m1 = a.ax[1].m, m2 = a.ax[2].m;
  const int c0 = a.ax[0].c, c1 = a.ax[1].c, c2 = a.ax[2].c;
  const int tx = lb % a.ntx;
  const int t2 = lb / a.ntx;
  const int ty = t2 % a.nty;
  const int tz = t2 / a.nty;
  const int X0 = tx * TX, X1 = (tx == a.ntx - 1) ? c2 : X0 + TX;
  const int Y0 = ty * TY, Y1 = (ty == a.nty - 1) ? c1 : Y0 + TY;
  const int Z0 = tz * a.tz, Z1 = (tz == a.nzc - 1) ? c0 : Z0 + a.tz;
  const int nX = X1 - X0, nY = Y1 - Y0;
  const int ncx = min(nX + 1, c2 - X0), ncy = min(nY + 1, c1 - Y0);  // nodal tile extent
  const int fq = min(2 * X1, m2) - 2 * X0;  // owned fine columns
  const int fr = min(2 * Y1, m1) - 2 * Y0;  // owned fine rows
  constexpr int ES = (int)sizeof(T);

  // ---- nodal plane loads: NN elements per thread ----
  int noff[NN];
  unsigned nvalid = 0, ninlds = 0;
#pragma unroll
  for (int k = 0; k < NN; k++) {
    const int idx = tid + NT * k;
    const int r = idx / NW, q = idx - r * NW;
    const bool ok = idx < NH * NW && r < ncy && q < ncx;
    nvalid |= (unsigned)ok << k;
    ninlds |= (unsigned)(idx < NH * NW) << k;
    noff[k] = ok ? ((Y0 + r) * (int)a.np1 + X0 + q) * ES : 0;
  }
  auto fetch_nodal = [&](int J, T (&v)[NN]) {
    const bool pin = J < c0;
    const T *src = a.nodal + (int64_t)(pin ? J : 0) * a.np0;
#pragma unroll
    for (int k = 0; k < NN; k++) {
      const T x = ld_at(src, (uint32_t)noff[k]);
      v[k] = (pin && ((nvalid >> k) & 1u)) ? x : T(0);
    }
  };
  auto commit_nodal = [&](int slot, const T (&v)[NN]) {
#pragma unroll
    for (int k = 0; k < NN; k++)
      if ((ninlds >> k) & 1u) sN[slot][tid + NT * k] = v[k];
  };

  // ---- 2x2 blocks ----
  // byte offsets of the block's coefficients in a level-centric plane:
  // (even row, even col), (even, odd), (odd, even), (odd, odd).  Positions of
  // nodes outside the owned box fall back to the even ones (and a block
  // outside the box to the tile origin), so every load stays in the level box.
  int bN[NB], bEE[NB], bEO[NB], bOE[NB], bOO[NB], bOut[NB];
  T bwxl[NB], bwxr[NB], bwyl[NB], bwyr[NB];
  unsigned bn = 0;  // 4 bits per block: nodes 00, 01, 10, 11 inside the owned box
#pragma unroll
  for (int k = 0; k < NB; k++) {
    const int o = tid + NT * k;
    int ba, bb;
    tile_slot<TX, TY>(o, ba, bb);
    const bool blk = o < BH * BW;
    const bool r0ok = blk && 2 * ba < fr, r1ok = blk && 2 * ba + 1 < fr;
    const bool q0ok = 2 * bb < fq, q1ok = 2 * bb + 1 < fq;
    bn |= (unsigned)((r0ok && q0ok) | ((r0ok && q1ok) << 1) | ((r1ok && q0ok) << 2) | ((r1ok && q1ok) << 3)) << (4 * k);
    const bool inbox = r0ok && q0ok;
    bN[k] = inbox ? ba * NW + bb : 0;
    const int rE = (int)((Y0 + (inbox ? ba : 0)) * a.up1) * ES;
    const int rO = r1ok && inbox ? rE + (int)(c1 * a.up1) * ES : rE;
    const int cE = (X0 + (inbox ? bb : 0)) * ES;
    const int cO = q1ok && inbox ? cE + c2 * ES : cE;
    bEE[k] = rE + cE;
    bEO[k] = rE + cO;
    bOE[k] = rO + cE;
    bOO[k] = rO + cO;
    bOut[k] = inbox ? ((2 * (Y0 + ba)) * (int)a.op1 + 2 * (X0 + bb)) * ES : 0;
    bwxl[k] = q1ok ? a.ax[2].wl[2 * X0 + 2 * bb + 1] : T(0);
    bwxr[k] = q1ok ? a.ax[2].wr[2 * X0 + 2 * bb + 1] : T(0);
    bwyl[k] = r1ok ? a.ax[1].wl[2 * Y0 + 2 * ba + 1] : T(0);
    bwyr[k] = r1ok ? a.ax[1].wr[2 * Y0 + 2 * ba + 1] : T(0);
  }
  const int outRow = (int)a.op1 * ES;

  // coefficients of coarse plane J: fine plane 2J (nodes 01, 10, 11) and
  // 2J+1 (nodes 00, 01, 10, 11), 7 per block
  auto fetch_coef = [&](int J, T (&cv)[NB][7]) {
    const bool pin = J < Z1;
    const bool odd_in = pin && 2 * J + 1 < m0;
    const int64_t pe = (int64_t)(pin ? J : 0) * a.up0, po = (int64_t)(odd_in ? c0 + J : 0) * a.up0;
    if (LAB) {
      const int32_t *be = a.lab + pe, *bo = a.lab + po;
#pragma unroll
      for (int k = 0; k < NB; k++) {
        cv[k][0] = from_label<T>(ld_at(be, lab_off<T>((uint32_t)bEO[k])), a.qc);
        cv[k][1] = from_label<T>(ld_at(be, lab_off<T>((uint32_t)bOE[k])), a.qc);
        cv[k][2] = from_label<T>(ld_at(be, lab_off<T>((uint32_t)bOO[k])), a.qc);
        cv[k][3] = from_label<T>(ld_at(bo, lab_off<T>((uint32_t)bEE[k])), a.qc);
        cv[k][4] = from_label<T>(ld_at(bo, lab_off<T>((uint32_t)bEO[k])), a.qc);
        cv[k][5] = from_label<T>(ld_at(bo, lab_off<T>((uint32_t)bOE[k])), a.qc);
        cv[k][6] = from_label<T>(ld_at(bo, lab_off<T>((uint32_t)bOO[k])), a.qc);
      }
    } else {
      const T *be = a.umc + pe, *bo = a.umc + po;
#pragma unroll
      for (int k = 0; k < NB; k++) {
        cv[k][0] = ld_at(be, (uint32_t)bEO[k]);
        cv[k][1] = ld_at(be, (uint32_t)bOE[k]);
        cv[k][2] = ld_at(be, (uint32_t)bOO[k]);
        cv[k][3] = ld_at(bo, (uint32_t)bEE[k]);
        cv[k][4] = ld_at(bo, (uint32_t)bEO[k]);
        cv[k][5] = ld_at(bo, (uint32_t)bOE[k]);
        cv[k][6] = ld_at(bo, (uint32_t)bOO[k]);
      }
    }
  };

  auto step = [&](int J, T (&cv)[NB][7], T (&nv)[NN]) {
    commit_nodal((J + 2) % NR, nv);  // plane J+2; its slot was last read two steps ago
    __syncthreads();
    const int sa = J % NR, sb = (J + 1) % NR;
    const bool odd_in = 2 * J + 1 < m0;
    const T wzl = odd_in ? ldu(a.ax[0].wl, 2 * J + 1) : T(0);
    const T wzr = odd_in ? ldu(a.ax[0].wr, 2 * J + 1) : T(0);
    T *const oe = a.out + (int64_t)(2 * J) * a.op0;
    T *const oo = a.out + (int64_t)(odd_in ? 2 * J + 1 : 2 * J) * a.op0;
#pragma unroll
    for (int k = 0; k < NB; k++) {
      const unsigned f = bn >> (4 * k);
      if (!(f & 0xFu)) continue;
      const T wxl = bwxl[k], wxr = bwxr[k], wyl = bwyl[k], wyr = bwyr[k];
      const int n = bN[k];
      const T A00 = sN[sa][n], A01 = sN[sa][n + 1], A10 = sN[sa][n + NW], A11 = sN[sa][n + NW + 1];
      // interpolants of plane J at the block's nodes
      const T ea = wxl * A00 + wxr * A01;
      const T eb = wxl * A10 + wxr * A11;
      const T e10 = wyl * A00 + wyr * A10;
      const T e11 = wyl * ea + wyr * eb;
      const uint32_t o0 = (uint32_t)bOut[k];
      if (f & 1u) st_at(oe, o0, A00);
      if (f & 2u) st_at(oe, o0 + ES, cv[k][0] + ea);
      if (f & 4u) st_at(oe, o0 + outRow, cv[k][1] + e10);
      if (f & 8u) st_at(oe, o0 + outRow + ES, cv[k][2] + e11);
      if (odd_in) {
        const T B00 = sN[sb][n], B01 = sN[sb][n + 1], B10 = sN[sb][n + NW], B11 = sN[sb][n + NW + 1];
        const T fa = wxl * B00 + wxr * B01;
        const T fb = wxl * B10 + wxr * B11;
        const T f10 = wyl * B00 + wyr * B10;
        const T f11 = wyl * fa + wyr * fb;
        if (f & 1u) st_at(oo, o0, cv[k][3] + (wzl * A00 + wzr * B00));
        if (f & 2u) st_at(oo, o0 + ES, cv[k][4] + (wzl * ea + wzr * fa));
        if (f & 4u) st_at(oo, o0 + outRow, cv[k][5] + (wzl * e10 + wzr * f10));
        if (f & 8u) st_at(oo, o0 + outRow + ES, cv[k][6] + (wzl * e11 + wzr * f11));
      }
    }
    // loads for step J+AH after every store of this step (partial waits later)
    fetch_coef(J + AH, cv);
    fetch_nodal(J + 2 + AH, nv);
  };

  T nv[AH][NN];
  T cv[AH][NB][7];
  fetch_nodal(Z0, nv[0]);
  commit_nodal(Z0 % NR, nv[0]);
  fetch_nodal(Z0 + 1, nv[0]);
  commit_nodal((Z0 + 1) % NR, nv[0]);
#pragma unroll
  for (int k = 0; k < AH; k++) {
    fetch_nodal(Z0 + 2 + k, nv[k]);
    fetch_coef(Z0 + k, cv[k]);
  }
  int J = Z0;
  for (; J + AH - 1 < Z1; J += AH) {
#pragma unroll
    for (int k = 0; k < AH; k++) step(J + k, cv[k], nv[k]);
  }
#pragma unroll
  for (int k = 0; k < AH - 1; k++)
    if (J + k < Z1) step(J + k, cv[k], nv[k]);
}

template <typename T, int TX, int TY, int NT, bool LAB>
__global__ void __launch_bounds__(NT) k_interp_add(InterpArgs<T> a) {
  interp_add_body<T, TX, TY, NT, LAB>(a, xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// k_interp_plane: the interpolate-add step with one coarse plane J per
// workgroup (fine planes 2J and 2J+1 of one tile).  Consecutive workgroups
// (on the same XCD after the remap) take neighbouring tiles of the same
// plane, so the stores of the chip advance through memory as one compact
// front instead of one front per z-marching workgroup.  Each thread owns one
// 2x2 block of fine nodes; all loads are issued before the first wait.
// ---------------------------------------------------------------------------
template <typename T, int TX, int TY, int NTP, bool LAB>
__device__ __forceinline__ void interp_plane_body(const InterpArgs<T> a, const int lb) {
  constexpr int NP = MGX_INTERP_NP;   // coarse planes per workgroup
  constexpr int NW = TX + 2, NH = TY + 2, BW = TX + 1;
  constexpr int NNP = ((NP + 1) * NH * NW + NTP - 1) / NTP;  // nodal loads per thread (planes J0 .. J0+NP)
  constexpr int ES = (int)sizeof(T);
  __shared__ T sN[NP + 1][NH * NW];
  const int tid = threadIdx.x;
  const int m0 = a.ax[0].m, m1 = a.ax[1].m, m2 = a.ax[2].m;
  const int c0 = a.ax[0].c, c1 = a.ax[1].c, c2 = a.ax[2].c;
  const int tx = lb % a.ntx;
  const int t2 = lb / a.ntx;
  const int ty = t2 % a.nty;
  const int J0 = (t2 / a.nty) * NP;
  const int X0 = tx * TX, X1 = (tx == a.ntx - 1) ? c2 : X0 + TX;
  const int Y0 = ty * TY, Y1 = (ty == a.nty - 1) ? c1 : Y0 + TY;
  const int ncx = min(X1 - X0 + 1, c2 - X0), ncy = min(Y1 - Y0 + 1, c1 - Y0);
  const int fq = min(2 * X1, m2) - 2 * X0;
  const int fr = min(2 * Y1, m1) - 2 * Y0;
  // nodal planes J0 .. J0+NP (zeros outside the box)
  T nv[NNP];
#pragma unroll
  for (int k = 0; k < NNP; k++) {
    const int idx = tid + NTP * k;
    const int p = idx / (NH * NW), rem = idx - p * (NH * NW);
    const int r = rem / NW, q = rem - r * NW;
    const int Jp = J0 + p;
    const bool ok = idx < (NP + 1) * NH * NW && r < ncy && q < ncx && Jp < c0;
    const T *src = a.nodal + (int64_t)(ok ? Jp : 0) * a.np0;
    const T x = ld_at(src, (uint32_t)(ok ? ((Y0 + r) * (int)a.np1 + X0 + q) * ES : 0));
    nv[k] = ok ? x : T(0);
  }
  // this thread's 2x2 block and its coefficients in every plane pair
  const int ba = tid / BW, bb = tid - ba * BW;
  const bool blk = ba < TY + 1;
  const bool r0ok = blk && 2 * ba < fr, r1ok = blk && 2 * ba + 1 < fr;
  const bool q0ok = 2 * bb < fq, q1ok = 2 * bb + 1 < fq;
  const bool inbox = r0ok && q0ok;
  const int rE = (int)((Y0 + (inbox ? ba : 0)) * a.up1) * ES;
  const int rO = r1ok && inbox ? rE + (int)(c1 * a.up1) * ES : rE;
  const int cE = (X0 + (inbox ? bb : 0)) * ES;
  const int cO = q1ok && inbox ? cE + c2 * ES : cE;
  auto coef = [&](int64_t plane, int off) -> T {
    if (LAB) return from_label<T>(ld_at(a.lab + plane, lab_off<T>((uint32_t)off)), a.qc);
    return ld_at(a.umc + plane, (uint32_t)off);
  };
  T cv[NP][7];
#pragma unroll
  for (int p = 0; p < NP; p++) {
    const int J = min(J0 + p, c0 - 1);
    const bool odd_in = 2 * J + 1 < m0;
    const int64_t pe = (int64_t)J * a.up0, po = (int64_t)(odd_in ? c0 + J : J) * a.up0;
    cv[p][0] = coef(pe, rE + cO);
    cv[p][1] = coef(pe, rO + cE);
    cv[p][2] = coef(pe, rO + cO);
    cv[p][3] = coef(po, rE + cE);
    cv[p][4] = coef(po, rE + cO);
    cv[p][5] = coef(po, rO + cE);
    cv[p][6] = coef(po, rO + cO);
  }
  const T wxl = q1ok ? a.ax[2].wl[2 * X0 + 2 * bb + 1] : T(0), wxr = q1ok ? a.ax[2].wr[2 * X0 + 2 * bb + 1] : T(0);
  const T wyl = r1ok ? a.ax[1].wl[2 * Y0 + 2 * ba + 1] : T(0), wyr = r1ok ? a.ax[1].wr[2 * Y0 + 2 * ba + 1] : T(0);
#pragma unroll
  for (int k = 0; k < NNP; k++) {
    const int idx = tid + NTP * k;
    if (idx < (NP + 1) * NH * NW) (&sN[0][0])[idx] = nv[k];
  }
  __syncthreads();
  if (!inbox) return;
  const int n = ba * NW + bb;
  const uint32_t o0 = (uint32_t)(((2 * (Y0 + ba)) * (int)a.op1 + 2 * (X0 + bb)) * ES);
  const uint32_t orow = (uint32_t)((int)a.op1 * ES);
  T A00 = sN[0][n], A01 = sN[0][n + 1], A10 = sN[0][n + NW], A11 = sN[0][n + NW + 1];
  T ea = wxl * A00 + wxr * A01, eb = wxl * A10 + wxr * A11;
  T e10 = wyl * A00 + wyr * A10, e11 = wyl * ea + wyr * eb;
#pragma unroll
  for (int p = 0; p < NP; p++) {
    const int J = J0 + p;
    if (J >= c0) break;
    const bool odd_in = 2 * J + 1 < m0;
    T *const oe = a.out + (int64_t)(2 * J) * a.op0;
    // each fine row's even and odd column in one store
    st_pair(oe, o0, A00, cv[p][0] + ea, q1ok);
    if (r1ok) st_pair(oe, o0 + orow, cv[p][1] + e10, cv[p][2] + e11, q1ok);
    if (!odd_in) break;
    const T B00 = sN[p + 1][n], B01 = sN[p + 1][n + 1], B10 = sN[p + 1][n + NW], B11 = sN[p + 1][n + NW + 1];
    const T fa = wxl * B00 + wxr * B01, fb = wxl * B10 + wxr * B11;
    const T f10 = wyl * B00 + wyr * B10, f11 = wyl * fa + wyr * fb;
    const T wzl = ldu(a.ax[0].wl, 2 * J + 1), wzr = ldu(a.ax[0].wr, 2 * J + 1);
    T *const oo = a.out + (int64_t)(2 * J + 1) * a.op0;
    st_pair(oo, o0, cv[p][3] + (wzl * A00 + wzr * B00), cv[p][4] + (wzl * ea + wzr * fa), q1ok);
    if (r1ok) st_pair(oo, o0 + orow, cv[p][5] + (wzl * e10 + wzr * f10), cv[p][6] + (wzl * e11 + wzr * f11), q1ok);
    // plane J + 1's interpolant serves the next pair's even plane
    A00 = B00;
    ea = fa;
    e10 = f10;
    e11 = f11;
  }
}
template <typename T, int TX, int TY, int NTP, bool LAB>
__global__ void __launch_bounds__(NTP) k_interp_plane(InterpArgs<T> a) {
  interp_plane_body<T, TX, TY, NTP, LAB>(a, xcd_remap(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// k_prolong_mass: one level of the adjoint (not in the paper).  Applies the
// transpose of the fused load-vector operator, (M P) along every axis, to a
// coarse box y and combines the level-l result with the level's other terms:
//   kProlongRecAdj: lc_out[x] = fine[x] - ((M P) y)(x) at coefficient nodes,
//   kProlongDecAdj: out[x] = ((M P) y)(x) + (x a coefficient node ? lc_in[x]
//                                            : -r[x/2]).
// Along one axis, (M P)[j][I] = (R M)[I][j] = w5[I][j - 2I + 2]: fine node 2I
// takes coarse I-1, I, I+1 (entries 4, 2, 0) and fine node 2I+1 takes I, I+1
// (entries 3, 1).  Tile as in k_interp_add.  The kernel marches over coarse
// planes; each thread keeps, for its fixed fine positions, the 2-D product
// (M P)_y (M P)_x of coarse planes J-1, J, J+1 in registers and combines
// them along z into fine planes 2J and 2J+1.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void mp_weights(const T *w5, int c, int j, T &w0, T &w1, T &w2) {
  const int I = j >> 1;
  if (!(j & 1)) {
    w0 = I - 1 >= 0 ? w5[(I - 1) * 5 + 4] : T(0);
    w1 = w5[I * 5 + 2];
    w2 = I + 1 < c ? w5[(I + 1) * 5 + 0] : T(0);
  } else {
    w0 = T(0);
    w1 = w5[I * 5 + 3];
    w2 = I + 1 < c ? w5[(I + 1) * 5 + 1] : T(0);
  }
}

template <typename T, int TX, int TY, int NT, int MODE>
__global__ void __launch_bounds__(NT) k_prolong_mass(ProlongArgs<T> a) {
  constexpr int CW = TX + 3, CH = TY + 3;          // coarse tile with halo, from (Y0-1, X0-1)
  constexpr int FW = 2 * TX + 1, FH = 2 * TY + 1;  // owned fine extent (max)
  constexpr int NP = (FW * FH + NT - 1) / NT;
  constexpr int NC = (CW * CH + NT - 1) / NT;
  constexpr int ES = (int)sizeof(T);
  __shared__ T sC[2][CH * CW];
  __shared__ T sWx[3][FW], sWy[3][FH];

  const int tid = threadIdx.x;
  const int m0 = a.ax[0].m, m1 = a.ax[1].m, m2 = a.ax[2].m;
  const int c0 = a.ax[0].c, c1 = a.ax[1].c, c2 = a.ax[2].c;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = lb % a.ntx;
  const int t2 = lb / a.ntx;
  const int ty = t2 % a.nty;
  const int tz = t2 / a.nty;
  const int X0 = tx * TX, X1 = (tx == a.ntx - 1) ? c2 : X0 + TX;
  const int Y0 = ty * TY, Y1 = (ty == a.nty - 1) ? c1 : Y0 + TY;
  const int Z0 = tz * a.tz, Z1 = (tz == a.nzc - 1) ? c0 : Z0 + a.tz;
  const int fq = min(2 * X1, m2) - 2 * X0;  // owned fine columns
  const int fr = min(2 * Y1, m1) - 2 * Y0;  // owned fine rows

  for (int q = tid; q < FW; q += NT) {
    T w0 = T(0), w1 = T(0), w2 = T(0);
    if (q < fq) mp_weights(a.ax[2].w5, c2, 2 * X0 + q, w0, w1, w2);
    sWx[0][q] = w0;
    sWx[1][q] = w1;
    sWx[2][q] = w2;
  }
  for (int r = tid; r < FH; r += NT) {
    T w0 = T(0), w1 = T(0), w2 = T(0);
    if (r < fr) mp_weights(a.ax[1].w5, c1, 2 * Y0 + r, w0, w1, w2);
    sWy[0][r] = w0;
    sWy[1][r] = w1;
    sWy[2][r] = w2;
  }

  // ---- coarse plane loads (zeros outside the box) ----
  int coff[NC];
  unsigned cvalid = 0;
#pragma unroll
  for (int k = 0; k < NC; k++) {
    const int idx = tid + NT * k;
    const int r = idx / CW, q = idx - r * CW;
    const int J1 = Y0 - 1 + r, J2 = X0 - 1 + q;
    const bool ok = idx < CH * CW && J1 >= 0 && J1 < c1 && J2 >= 0 && J2 < c2;
    cvalid |= (unsigned)ok << k;
    coff[k] = ok ? (J1 * (int)a.yp1 + J2) * ES : 0;
  }
  auto fetch = [&](int K, T (&v)[NC]) {
    const bool pin = K >= 0 && K < c0;
    const T *base = a.y + (int64_t)(pin ? K : 0) * a.yp0;
#pragma unroll
    for (int k = 0; k < NC; k++) {
      const T x = ld_at(base, (uint32_t)coff[k]);
      v[k] = (pin && ((cvalid >> k) & 1u)) ? x : T(0);
    }
  };
  auto commit = [&](int slot, const T (&v)[NC]) {
#pragma unroll
    for (int k = 0; k < NC; k++)
      if (tid + NT * k < CH * CW) sC[slot][tid + NT * k] = v[k];
  };

  // ---- owned fine positions ----
  int pbase[NP], prq[NP], lcoff[NP], boff[NP], roff[NP];
  unsigned pval = 0, pnod = 0;
#pragma unroll
  for (int k = 0; k < NP; k++) {
    const int p = tid + NT * k;
    const int r = p / FW, q = p - r * FW;
    const bool ok = p < FW * FH && r < fr && q < fq;
    pval |= (unsigned)ok << k;
    const int j1 = 2 * Y0 + r, j2 = 2 * X0 + q;
    pnod |= (unsigned)(!(j1 & 1) && !(j2 & 1)) << k;
    pbase[k] = ok ? (r >> 1) * CW + (q >> 1) : 0;
    prq[k] = ok ? (r << 16) | q : 0;
    lcoff[k] = ok ? (int)(lc_pos(j1, c1) * a.up1 + lc_pos(j2, c2)) * ES : 0;
    if (MODE == kProlongRecAdj)
      boff[k] = ok ? (j1 * (int)a.fp1 + j2) * ES : 0;
    else
      boff[k] = ok ? (j1 * (int)a.op1 + j2) * ES : 0;
    roff[k] = ok ? ((j1 >> 1) * (int)a.rp1 + (j2 >> 1)) * ES : 0;
  }

  auto computeH = [&](int slot, T (&H)[NP]) {
#pragma unroll
    for (int k = 0; k < NP; k++) {
      H[k] = T(0);
      if ((pval >> k) & 1u) {
        const int r = prq[k] >> 16, q = prq[k] & 0xFFFF, b = pbase[k];
        const T wx0 = sWx[0][q], wx1 = sWx[1][q], wx2 = sWx[2][q];
        const T *C = &sC[slot][b];
        const T h0 = wx0 * C[0] + wx1 * C[1] + wx2 * C[2];
        const T h1 = wx0 * C[CW] + wx1 * C[CW + 1] + wx2 * C[CW + 2];
        const T h2 = wx0 * C[2 * CW] + wx1 * C[2 * CW + 1] + wx2 * C[2 * CW + 2];
        H[k] = sWy[0][r] * h0 + sWy[1][r] * h1 + sWy[2][r] * h2;
      }
    }
  };

  auto output = [&](int J, const T (&Hm)[NP], const T (&H0)[NP], const T (&Hp)[NP]) {
    const T we0 = J - 1 >= 0 ? ldu(a.ax[0].w5, (J - 1) * 5 + 4) : T(0);
    const T we1 = ldu(a.ax[0].w5, J * 5 + 2);
    const T we2 = J + 1 < c0 ? ldu(a.ax[0].w5, (J + 1) * 5 + 0) : T(0);
    const bool odd_in = 2 * J + 1 < m0;
    const T wo1 = odd_in ? ldu(a.ax[0].w5, J * 5 + 3) : T(0);
    const T wo2 = odd_in && J + 1 < c0 ? ldu(a.ax[0].w5, (J + 1) * 5 + 1) : T(0);
    if (MODE == kProlongRecAdj) {
      const T *fe = a.fine + (int64_t)(2 * J) * a.fp0;
      const T *fo = a.fine + (int64_t)(odd_in ? 2 * J + 1 : 2 * J) * a.fp0;
      T *le = a.lc_out + (int64_t)J * a.up0;
      T *lo = a.lc_out + (int64_t)(odd_in ? c0 + J : J) * a.up0;
#pragma unroll
      for (int k = 0; k < NP; k++) {
        if (!((pval >> k) & 1u)) continue;
        if (!((pnod >> k) & 1u))
          st_at(le, (uint32_t)lcoff[k], ld_at(fe, (uint32_t)boff[k]) - (we0 * Hm[k] + we1 * H0[k] + we2 * Hp[k]));
        if (odd_in) st_at(lo, (uint32_t)lcoff[k], ld_at(fo, (uint32_t)boff[k]) - (wo1 * H0[k] + wo2 * Hp[k]));
      }
    } else {
      T *oe = a.out + (int64_t)(2 * J) * a.op0;
      T *oo = a.out + (int64_t)(odd_in ? 2 * J + 1 : 2 * J) * a.op0;
      const T *le = a.lc_in + (int64_t)J * a.up0;
      const T *lo = a.lc_in + (int64_t)(odd_in ? c0 + J : J) * a.up0;
      const T *rb = a.r + (int64_t)J * a.rp0;
#pragma unroll
      for (int k = 0; k < NP; k++) {
        if (!((pval >> k) & 1u)) continue;
        const T other = ((pnod >> k) & 1u) ? -ld_at(rb, (uint32_t)roff[k]) : ld_at(le, (uint32_t)lcoff[k]);
        st_at(oe, (uint32_t)boff[k], (we0 * Hm[k] + we1 * H0[k] + we2 * Hp[k]) + other);
        if (odd_in) st_at(oo, (uint32_t)boff[k], (wo1 * H0[k] + wo2 * Hp[k]) + ld_at(lo, (uint32_t)lcoff[k]));
      }
    }
  };

  // slot of coarse plane K: (K - Z0 + 1) & 1
  T creg[NC];
  T Hm[NP], H0[NP], Hp[NP];
  fetch(Z0 - 1, creg);
  commit(0, creg);
  fetch(Z0, creg);
  __syncthreads();
  computeH(0, Hm);
  commit(1, creg);
  fetch(Z0 + 1, creg);
  __syncthreads();
  computeH(1, H0);
  for (int J = Z0; J < Z1; J++) {
    const int s = (J - Z0) & 1;  // slot of plane J+1
    commit(s, creg);
    fetch(J + 2, creg);
    __syncthreads();
    computeH(s, Hp);
    output(J, Hm, H0, Hp);
#pragma unroll
    for (int k = 0; k < NP; k++) {
      Hm[k] = H0[k];
      H0[k] = Hp[k];
    }
  }
}

template <typename T>
__device__ __forceinline__ void copy_box_body(const CopyArgs<T> a, const int b, const int nb) {
  const int64_t n = (int64_t)a.n0 * a.n1 * a.n2;
  for (int64_t i = b * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)nb * 256) {
    const int64_t r = i / a.n2;
    const int i2 = (int)(i - r * a.n2);
    const int i0 = (int)(r / a.n1), i1 = (int)(r - (int64_t)i0 * a.n1);
    a.dst[i0 * a.dp0 + i1 * a.dp1 + i2] = a.src[i0 * a.sp0 + i1 * a.sp1 + i2];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_copy_box(CopyArgs<T> a) {
  copy_box_body<T>(a, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_pad_edge(PadArgs<T> a) {
  const int64_t n = (int64_t)a.p0 * a.p1 * a.p2;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t r = i / a.p2;
    const int i2 = (int)(i - r * a.p2);
    const int i0 = (int)(r / a.p1), i1 = (int)(r - (int64_t)i0 * a.p1);
    const int j0 = min(i0, a.n0 - 1), j1 = min(i1, a.n1 - 1), j2 = min(i2, a.n2 - 1);
    a.dst[i] = a.src[((int64_t)j0 * a.n1 + j1) * a.n2 + j2];
  }
}

template <typename T>
hipError_t launch_pad_edge(PadArgs<T> a, hipStream_t st) {
  if (a.n0 < 1 || a.n1 < 1 || a.n2 < 1 || a.p0 < a.n0 || a.p1 < a.n1 || a.p2 < a.n2) return hipErrorInvalidValue;
  int64_t blocks = ((int64_t)a.p0 * a.p1 * a.p2 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((k_pad_edge<T>), dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Quantization (Sec. 4.1): label = rint(c / q_l) in FP64, the level of an
// element from its position (levelpos.hpp).  The array is processed flat,
// four consecutive elements per thread.
// ---------------------------------------------------------------------------
// Four consecutive elements of T / int32 as one 16-byte (float, int32) or
// two 16-byte (double) accesses when the buffers are 16-byte aligned.
template <typename T, bool VEC>
__device__ __forceinline__ void load4(const T *p, uint32_t base, uint32_t N, T (&v)[4]) {
  if (VEC && base + 3 < N) {
    if constexpr (sizeof(T) == 4) {
      const float4 t = *(const float4 *)(p + base);
      v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else {
      const double2 t0 = *(const double2 *)(p + base), t1 = *(const double2 *)(p + base + 2);
      v[0] = t0.x; v[1] = t0.y; v[2] = t1.x; v[3] = t1.y;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++) v[e] = base + e < N ? p[base + e] : T(0);
  }
}

template <typename T, bool VEC>
__device__ __forceinline__ void store4(T *p, uint32_t base, uint32_t N, const T (&v)[4]) {
  if (VEC && base + 3 < N) {
    if constexpr (sizeof(T) == 4) {
      *(float4 *)(p + base) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
      *(double2 *)(p + base) = make_double2(v[0], v[1]);
      *(double2 *)(p + base + 2) = make_double2(v[2], v[3]);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++)
      if (base + e < N) p[base + e] = v[e];
  }
}

__device__ __forceinline__ void load4i(const int32_t *p, uint32_t base, uint32_t N, int32_t (&v)[4], bool vec) {
  if (vec && base + 3 < N) {
    const int4 t = *(const int4 *)(p + base);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++) v[e] = base + e < N ? p[base + e] : 0;
  }
}

__device__ __forceinline__ void store4i(int32_t *p, uint32_t base, uint32_t N, const int32_t (&v)[4], bool vec) {
  if (vec && base + 3 < N) {
    *(int4 *)(p + base) = make_int4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++)
      if (base + e < N) p[base + e] = v[e];
  }
}

template <typename T, bool STATS, bool VEC>
__device__ __forceinline__ void quantize_body(const T *__restrict__ umc, int32_t *__restrict__ labels,
                                              const QuantArgs &a, const int b, const int nb) {
  __shared__ int s_max[kMaxLevelsK];
  __shared__ double s_q[kMaxLevelsK];
  __shared__ unsigned long long s_ovf, s_nan;
  if (threadIdx.x < kMaxLevelsK) {
    s_q[threadIdx.x] = a.q[threadIdx.x];
    if (STATS) s_max[threadIdx.x] = 0;
  }
  if (STATS && threadIdx.x == 0) {
    s_ovf = 0;
    s_nan = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  unsigned long long my_ovf = 0, my_nan = 0;
  const uint32_t N = (uint32_t)a.n;
  const uint32_t stride = (uint32_t)nb * 256u * 4u;
  for (uint32_t base = ((uint32_t)b * 256u + threadIdx.x) * 4u; base < N; base += stride) {
    int lev[4], absl[4];
    bool sel[4];
    int nsel = 0;
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const bool in = base + e < N;
      lev[e] = in ? elem_level(base + e, a) : a.first;
      sel[e] = in && lev[e] >= a.sel_lo && lev[e] <= a.sel_hi;
      nsel += sel[e] ? 1 : 0;
      absl[e] = 0;
    }
    if (nsel > 0) {
      T v[4];
      if (nsel == 4) {
        load4<T, VEC>(umc, base, N, v);
      } else {
#pragma unroll
        for (int e = 0; e < 4; e++) v[e] = sel[e] ? umc[base + e] : T(0);
      }
      int32_t lab[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const double t = (double)v[e] / s_q[lev[e] - a.first];
        if (!(fabs(t) < 2147483647.0)) {
          lab[e] = INT32_MIN;
          if (sel[e]) {
            if (isnan(t) || isinf(t))
              my_nan++;
            else
              my_ovf++;
          }
        } else {
          lab[e] = (int32_t)rint(t);
          absl[e] = sel[e] ? (lab[e] < 0 ? -lab[e] : lab[e]) : 0;
        }
      }
      if (nsel == 4) {
        store4i(labels, base, N, lab, VEC);
      } else {
#pragma unroll
        for (int e = 0; e < 4; e++)
          if (sel[e]) labels[base + e] = lab[e];
      }
    }
    if (STATS) {
      // per-level maxima: reduce each distinct level present in the wave
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const bool in = sel[e];
        unsigned long long todo = __ballot(in);
        while (todo) {
          const int leader = __ffsll((long long)todo) - 1;
          const int L0 = __shfl(lev[e], leader);
          const bool mine = in && lev[e] == L0;
          int m = mine ? absl[e] : 0;
          for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
          if (lane == leader) atomicMax(&s_max[L0 - a.first], m);
          todo &= ~__ballot(mine);
        }
      }
    }
  }
  if (!STATS && a.stats_ovf) {
    // out-of-range counts without the other statistics (rare: per thread)
    if (my_ovf) atomicAdd(a.stats_ovf, my_ovf);
    if (my_nan) atomicAdd(a.stats_nan, my_nan);
  }
  if (STATS) {
    for (int off = 32; off > 0; off >>= 1) {
      my_ovf += __shfl_xor(my_ovf, off);
      my_nan += __shfl_xor(my_nan, off);
    }
    if (lane == 0) {
      atomicAdd(&s_ovf, my_ovf);
      atomicAdd(&s_nan, my_nan);
    }
    __syncthreads();
    if (threadIdx.x < a.nlev) atomicMax(&a.stats_max[threadIdx.x], s_max[threadIdx.x]);
    if (threadIdx.x == 0) {
      atomicAdd(a.stats_ovf, s_ovf);
      atomicAdd(a.stats_nan, s_nan);
    }
  }
}

template <typename T, bool STATS, bool VEC>
__global__ void __launch_bounds__(256) k_quantize(const T *__restrict__ umc, int32_t *__restrict__ labels,
                                                  QuantArgs a) {
  quantize_body<T, STATS, VEC>(umc, labels, a, blockIdx.x, gridDim.x);
}

template <typename T, bool VEC>
__device__ __forceinline__ void dequantize_body(const int32_t *__restrict__ labels, T *__restrict__ umc,
                                                const QuantArgs &a, const int b, const int nb) {
  __shared__ double s_q[kMaxLevelsK];
  if (threadIdx.x < kMaxLevelsK) s_q[threadIdx.x] = a.q[threadIdx.x];
  __syncthreads();
  const uint32_t N = (uint32_t)a.n;
  const uint32_t stride = (uint32_t)nb * 256u * 4u;
  for (uint32_t base = ((uint32_t)b * 256u + threadIdx.x) * 4u; base < N; base += stride) {
    int lev[4];
    bool sel[4];
    int nsel = 0;
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const bool in = base + e < N;
      lev[e] = in ? elem_level(base + e, a) : a.first;
      sel[e] = in && lev[e] >= a.sel_lo && lev[e] <= a.sel_hi;
      nsel += sel[e] ? 1 : 0;
    }
    if (nsel == 0) continue;
    int32_t lab[4];
    if (nsel == 4) {
      load4i(labels, base, N, lab, VEC);
    } else {
#pragma unroll
      for (int e = 0; e < 4; e++) lab[e] = sel[e] ? labels[base + e] : 0;
    }
    T v[4];
#pragma unroll
    for (int e = 0; e < 4; e++) v[e] = (T)((double)lab[e] * s_q[lev[e] - a.first]);
    if (nsel == 4) {
      store4<T, VEC>(umc, base, N, v);
    } else {
#pragma unroll
      for (int e = 0; e < 4; e++)
        if (sel[e]) umc[base + e] = v[e];
    }
  }
}

template <typename T, bool VEC>
__global__ void __launch_bounds__(256) k_dequantize(const int32_t *__restrict__ labels, T *__restrict__ umc,
                                                    QuantArgs a) {
  dequantize_body<T, VEC>(labels, umc, a, blockIdx.x, gridDim.x);
}

// Quantization restricted to the corner box b0 x b1 x b2 of the array (the
// coarser levels' coefficients): every element of the box is visited once,
// one element per thread and iteration.
template <typename T>
__device__ __forceinline__ void quantize_box_body(const T *__restrict__ umc, int32_t *__restrict__ labels,
                                                  const QuantArgs &a, const int b, const int nb) {
  __shared__ double s_q[kMaxLevelsK];
  if (threadIdx.x < kMaxLevelsK) s_q[threadIdx.x] = a.q[threadIdx.x];
  __syncthreads();
  const uint32_t B = (uint32_t)a.bn;
  int lmax = 0;  // largest |label| written (kept when one level is selected and stats_max is set)
  for (uint32_t i = (uint32_t)b * 256u + threadIdx.x; i < B; i += (uint32_t)nb * 256u) {
    const uint32_t row = (uint32_t)__umul64hi((uint64_t)i, a.bmag2);
    const uint32_t x = i - row * (uint32_t)a.b2;
    const uint32_t z = a.b1 == 1 ? row : (uint32_t)__umul64hi((uint64_t)row, a.bmag1);
    const uint32_t y = row - z * (uint32_t)a.b1;
    int l = pos_level(x, a.off[2], a.first);
    l = max(l, pos_level(y, a.off[1], a.first));
    l = max(l, pos_level(z, a.off[0], a.first));
    if (l < a.sel_lo || l > a.sel_hi) continue;
    const uint32_t idx = (z * (uint32_t)a.n1 + y) * (uint32_t)a.n2 + x;
    const double t = (double)umc[a.box_compact ? i : idx] / s_q[l - a.first];
    const bool out = !(fabs(t) < 2147483647.0);
    const int32_t lab = out ? INT32_MIN : (int32_t)rint(t);
    labels[idx] = lab;
    if (out && a.stats_ovf) atomicAdd((isnan(t) || isinf(t)) ? a.stats_nan : a.stats_ovf, 1ull);
    if (!out) lmax = max(lmax, lab < 0 ? -lab : lab);
  }
  if (a.stats_max && a.sel_lo == a.sel_hi) {  // every lane reaches this point
    for (int off = 32; off > 0; off >>= 1) lmax = max(lmax, __shfl_xor(lmax, off));
    if ((threadIdx.x & 63) == 0 && lmax > 0) atomicMax(&a.stats_max[a.sel_lo - a.first], lmax);
  }
}

template <typename T>
__device__ __forceinline__ void dequantize_box_body(const int32_t *__restrict__ labels, T *__restrict__ umc,
                                                    const QuantArgs &a, const int b, const int nb) {
  __shared__ double s_q[kMaxLevelsK];
  if (threadIdx.x < kMaxLevelsK) s_q[threadIdx.x] = a.q[threadIdx.x];
  __syncthreads();
  const uint32_t B = (uint32_t)a.bn;
  for (uint32_t i = (uint32_t)b * 256u + threadIdx.x; i < B; i += (uint32_t)nb * 256u) {
    const uint32_t row = (uint32_t)__umul64hi((uint64_t)i, a.bmag2);
    const uint32_t x = i - row * (uint32_t)a.b2;
    const uint32_t z = a.b1 == 1 ? row : (uint32_t)__umul64hi((uint64_t)row, a.bmag1);
    const uint32_t y = row - z * (uint32_t)a.b1;
    int l = pos_level(x, a.off[2], a.first);
    l = max(l, pos_level(y, a.off[1], a.first));
    l = max(l, pos_level(z, a.off[0], a.first));
    if (l < a.sel_lo || l > a.sel_hi) continue;
    const uint32_t idx = (z * (uint32_t)a.n1 + y) * (uint32_t)a.n2 + x;
    umc[a.box_compact ? i : idx] = (T)((double)labels[idx] * s_q[l - a.first]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_quantize_box(const T *__restrict__ umc, int32_t *__restrict__ labels,
                                                      QuantArgs a) {
  quantize_box_body<T>(umc, labels, a, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_dequantize_box(const int32_t *__restrict__ labels, T *__restrict__ umc,
                                                        QuantArgs a) {
  dequantize_box_body<T>(labels, umc, a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// k_adaptive_estimate: the error estimate of the adaptive decomposition
// (Sec. 4.2, Alg. 1 lines 4-9) on the level-l box V = Q_l u.  One thread per
// sampled 3^3 block: it loads the 4x4x4 region of level indices 2a-1 .. 2a+2
// per axis (the block and its Lorenzo neighbours), and for each of the 19
// coefficient nodes adds |u - Lorenzo prediction| and |u - multilinear
// interpolant| (FP64, weights of the level's coordinates).  Each workgroup
// writes its two sums; k_adaptive_decide adds them up.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kEstimateThreads) k_adaptive_estimate(EstimateArgs<T> a) {
  if (a.gate && *a.gate == 0) return;
  __shared__ double sl[kEstimateThreads], si[kEstimateThreads];
  const int nb = a.nb0 * a.nb1 * a.nb2;
  const int b = blockIdx.x * kEstimateThreads + threadIdx.x;
  double el = 0.0, ei = 0.0;
  if (b < nb) {
    const int b2 = b % a.nb2, r = b / a.nb2, b1 = r % a.nb1, b0 = r / a.nb1;
    const int a0 = 1 + 4 * b0, a1 = 1 + 4 * b1, a2 = 1 + 4 * b2;
    // region R[i0][i1][i2] = V at level indices (2a0-1+i0, 2a1-1+i1, 2a2-1+i2)
    double R[4][4][4];
    const T *base = a.V + (int64_t)(2 * a0 - 1) * a.vp0 + (int64_t)(2 * a1 - 1) * a.vp1 + (2 * a2 - 1);
#pragma unroll
    for (int i0 = 0; i0 < 4; i0++)
#pragma unroll
      for (int i1 = 0; i1 < 4; i1++)
#pragma unroll
        for (int i2 = 0; i2 < 4; i2++) R[i0][i1][i2] = (double)base[i0 * a.vp0 + i1 * a.vp1 + i2];
    // weights of the odd (middle) level index of the block on each axis
    const double l0 = a.wl[0][2 * a0 + 1], r0 = a.wr[0][2 * a0 + 1];
    const double l1 = a.wl[1][2 * a1 + 1], r1 = a.wr[1][2 * a1 + 1];
    const double l2 = a.wl[2][2 * a2 + 1], r2 = a.wr[2][2 * a2 + 1];
#pragma unroll
    for (int q0 = 0; q0 < 3; q0++)
#pragma unroll
      for (int q1 = 0; q1 < 3; q1++)
#pragma unroll
        for (int q2 = 0; q2 < 3; q2++) {
          if (q0 != 1 && q1 != 1 && q2 != 1) continue;
          const int i0 = q0 + 1, i1 = q1 + 1, i2 = q2 + 1;
          const double x = R[i0][i1][i2];
          const double lor = R[i0][i1 - 1][i2] + R[i0 - 1][i1][i2] + R[i0][i1][i2 - 1] - R[i0 - 1][i1 - 1][i2] -
                             R[i0][i1 - 1][i2 - 1] - R[i0 - 1][i1][i2 - 1] + R[i0 - 1][i1 - 1][i2 - 1];
          // multilinear interpolant from the nodal corners (block positions 0 and 2)
          double pred = 0.0;
#pragma unroll
          for (int c = 0; c < 8; c++) {
            const int c0 = c & 1, c1 = (c >> 1) & 1, c2 = (c >> 2) & 1;
            if ((q0 != 1 && c0) || (q1 != 1 && c1) || (q2 != 1 && c2)) continue;
            const double w0 = q0 != 1 ? 1.0 : (c0 ? r0 : l0);
            const double w1 = q1 != 1 ? 1.0 : (c1 ? r1 : l1);
            const double w2 = q2 != 1 ? 1.0 : (c2 ? r2 : l2);
            const int j0 = q0 != 1 ? i0 : 1 + 2 * c0, j1 = q1 != 1 ? i1 : 1 + 2 * c1, j2 = q2 != 1 ? i2 : 1 + 2 * c2;
            pred += w0 * w1 * w2 * R[j0][j1][j2];
          }
          el += fabs(x - lor);
          ei += fabs(x - pred);
        }
  }
  sl[threadIdx.x] = el;
  si[threadIdx.x] = ei;
  __syncthreads();
  for (int h = kEstimateThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sl[threadIdx.x] += sl[threadIdx.x + h];
      si[threadIdx.x] += si[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.partial[2 * blockIdx.x] = sl[0];
    a.partial[2 * blockIdx.x + 1] = si[0];
  }
}

template <typename T>
hipError_t launch_adaptive_estimate(EstimateArgs<T> a, int nblocks, hipStream_t st) {
  if (nblocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_adaptive_estimate<T>), dim3((unsigned)nblocks), dim3(kEstimateThreads), 0, st, a);
  return hipGetLastError();
}

// k_adaptive_decide: one workgroup adds the estimate's per-workgroup sums
// (thread t takes workgroups t, t + 256, ... in order, then a fixed tree), so
// the totals do not depend on timing.  With a state it takes the decision of
// Sec. 4.2 on the device: the decomposition stops at this level when the
// Lorenzo estimate (sum + penalty) is below the interpolation's, and the
// level kernels that follow, gated on state[0], then do nothing.  Once the
// state says stop, later decisions leave it as it is.
__global__ void __launch_bounds__(kEstimateThreads) k_adaptive_decide(DecideArgs a) {
  if (a.state && !a.first && a.state[0] == 0) return;
  __shared__ double sl[kEstimateThreads], si[kEstimateThreads];
  double x = 0.0, y = 0.0;
  for (int i = threadIdx.x; i < a.nwg; i += kEstimateThreads) {
    x += a.partial[2 * i];
    y += a.partial[2 * i + 1];
  }
  sl[threadIdx.x] = x;
  si[threadIdx.x] = y;
  __syncthreads();
  for (int h = kEstimateThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sl[threadIdx.x] += sl[threadIdx.x + h];
      si[threadIdx.x] += si[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (a.sums) {
    a.sums[0] = sl[0];
    a.sums[1] = si[0];
  }
  if (a.state) {
    if (sl[0] + a.pen_lor < si[0] + a.pen_int) {
      a.state[0] = 0;
      a.state[1] = a.level;
    } else {
      a.state[0] = 1;
      if (a.first) a.state[1] = 0;
    }
  }
}

hipError_t launch_adaptive_decide(DecideArgs a, hipStream_t st) {
  if (a.nwg < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_adaptive_decide, dim3(1), dim3(kEstimateThreads), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <typename T>
struct Tiles;
template <>
struct Tiles<float> {
  static constexpr int TX = MGX_F32_TX, TY = MGX_F32_TY, NT = MGX_F32_NT;
};
template <>
struct Tiles<double> {
  static constexpr int TX = 16, TY = MGX_F64_TY, NT = MGX_F64_NT;
};
// Tiles of the decomposition's load-vector kernel (single-field launches)
template <typename T>
struct DecTiles : Tiles<T> {};
template <>
struct DecTiles<float> {
  static constexpr int TX = MGX_F32_DEC_TX, TY = MGX_F32_DEC_TY, NT = MGX_F32_DEC_NT;
};
// Tiles of the recomposition's load-vector kernel reading labels (measured
// faster with wider rows; the kernel on coefficients keeps the tiles above)
template <typename T>
struct RecLabTiles : Tiles<T> {};
template <>
struct RecLabTiles<float> {
  static constexpr int TX = MGX_F32_RECLAB_TX, TY = MGX_F32_RECLAB_TY, NT = MGX_F32_NT;
};
// Tiles of the interpolation kernels (wider rows than the load vector's:
// longer store runs per row, measured faster on MI355X)
template <typename T>
struct InterpTiles : Tiles<T> {};
template <>
struct InterpTiles<float> {
  static constexpr int TX = MGX_F32_INTERP_TX, TY = MGX_F32_INTERP_TY, NT = MGX_F32_NT;
};

// Tiles of TX x TY coarse columns/rows (the last tile takes the extra node of
// c = 2^k + 1) and z-chunks of tz coarse planes.  Returns false when an axis
// length does not satisfy the tiling assumption (c - 1 a multiple of the
// tile, or smaller than it), so that no kernel is launched on a bad shape.
static bool tile_grid(int c0, int c1, int c2, int TX, int TY, int *ntx, int *nty, int *nzc, int *tz,
                      const Tuning &tn = Tuning{}) {
  if (c0 < 1 || c1 < 1 || c2 < 1) return false;
  if ((c2 - 1) >= TX && (c2 - 1) % TX != 0) return false;
  if ((c1 - 1) >= TY && (c1 - 1) % TY != 0) return false;
  *ntx = (c2 - 1) / TX > 0 ? (c2 - 1) / TX : 1;
  *nty = (c1 - 1) / TY > 0 ? (c1 - 1) / TY : 1;
  const int per = *ntx * *nty;
  int want = (tn.target_blocks + per - 1) / per;
  // large levels keep z-chunks of >= min_zchunk coarse planes (halo re-reads
  // stay small); small levels take one coarse plane per workgroup (latency
  // bound)
  const int64_t cn = (int64_t)c0 * c1 * c2;
  const bool large = cn >= (1 << 20);
  const int mz0 = cn >= (1 << 24) ? tn.min_zchunk : tn.mid_zchunk;
  const int mz = mz0 > 0 ? mz0 : 1;
  int maxz = large ? (c0 / mz > 0 ? c0 / mz : 1) : c0;
  if (want > maxz) want = maxz;
  if (want < 1) want = 1;
  *nzc = want;
  *tz = c0 / want;
  return true;
}

template <typename T, typename TL, bool DEC, int LAB>
hipError_t launch_load_vector_t(StencilArgs<T> a, hipStream_t st, Tuning tn) {
  constexpr int TX = TL::TX, TY = TL::TY, NT = TL::NT;
  if (!tile_grid(a.ax[0].c, a.ax[1].c, a.ax[2].c, TX, TY, &a.ntx, &a.nty, &a.nzc, &a.tz, tn))
    return hipErrorInvalidValue;
  dim3 grid(a.ntx * a.nty * a.nzc);
  if constexpr (DEC && LAB != 0) {
    if (!a.umc_w) {  // labels only
      hipLaunchKernelGGL((k_load_vector<T, TX, TY, NT, DEC, LAB, false>), grid, dim3(NT), 0, st, a);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_load_vector<T, TX, TY, NT, DEC, LAB>), grid, dim3(NT), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_load_vector(StencilArgs<T> a, bool dec, hipStream_t st, Tuning tn) {
  if (dec) {
    if (a.lab_w && a.smax) return launch_load_vector_t<T, DecTiles<T>, true, 2>(a, st, tn);
    if (a.lab_w) return launch_load_vector_t<T, DecTiles<T>, true, 1>(a, st, tn);
    return launch_load_vector_t<T, DecTiles<T>, true, 0>(a, st, tn);
  }
  if (a.lab_r) return launch_load_vector_t<T, RecLabTiles<T>, false, 1>(a, st, tn);
  return launch_load_vector_t<T, Tiles<T>, false, 0>(a, st, tn);
}

// Large levels take the one-plane-per-workgroup interpolation (compact store
// front); smaller ones the z-marching kernel.
template <typename T>
static bool interp_plane(const InterpArgs<T> &a) {
  return MGX_INTERP_PLANE && (int64_t)a.ax[0].c * a.ax[1].c * a.ax[2].c >= (1 << 20);
}
template <typename T>
constexpr int interp_plane_threads() {
  return ((InterpTiles<T>::TY + 1) * (InterpTiles<T>::TX + 1) + 63) / 64 * 64;
}

template <typename T>
hipError_t launch_interp_add(InterpArgs<T> a, hipStream_t st, Tuning tn) {
  constexpr int TX = InterpTiles<T>::TX, TY = InterpTiles<T>::TY, NT = InterpTiles<T>::NT;
  if (!tile_grid(a.ax[0].c, a.ax[1].c, a.ax[2].c, TX, TY, &a.ntx, &a.nty, &a.nzc, &a.tz, tn))
    return hipErrorInvalidValue;
  if (interp_plane(a)) {
    // MGX_INTERP_NP coarse planes per workgroup
    constexpr int NTP = interp_plane_threads<T>();
    a.nzc = (a.ax[0].c + MGX_INTERP_NP - 1) / MGX_INTERP_NP;
    a.tz = MGX_INTERP_NP;
    dim3 grid(a.ntx * a.nty * a.nzc);
    if (a.lab)
      hipLaunchKernelGGL((k_interp_plane<T, TX, TY, NTP, true>), grid, dim3(NTP), 0, st, a);
    else
      hipLaunchKernelGGL((k_interp_plane<T, TX, TY, NTP, false>), grid, dim3(NTP), 0, st, a);
    return hipGetLastError();
  }
  dim3 grid(a.ntx * a.nty * a.nzc);
  if (a.lab)
    hipLaunchKernelGGL((k_interp_add<T, TX, TY, NT, true>), grid, dim3(NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_interp_add<T, TX, TY, NT, false>), grid, dim3(NT), 0, st, a);
  return hipGetLastError();
}

template <typename T, int E, int G>
static void launch_contig_eg(SolveArgs<T> a, hipStream_t st) {
  const int64_t lines_per_block = 4 * (64 / G);
  dim3 grid((unsigned)((a.nlines + lines_per_block - 1) / lines_per_block));
  hipLaunchKernelGGL((k_solve_contig<T, E, G>), grid, dim3(256), 0, st, a);
}

template <typename T>
hipError_t launch_solve_contig(SolveArgs<T> a, hipStream_t st) {
  switch (a.c) {
    case 3: launch_contig_eg<T, 1, 2>(a, st); break;
    case 5: launch_contig_eg<T, 1, 4>(a, st); break;
    case 9: launch_contig_eg<T, 1, 8>(a, st); break;
    case 17: launch_contig_eg<T, 1, 16>(a, st); break;
    case 33: launch_contig_eg<T, 1, 32>(a, st); break;
    case 65: launch_contig_eg<T, 1, 64>(a, st); break;
    case 129: launch_contig_eg<T, 2, 64>(a, st); break;
    case 257: launch_contig_eg<T, 4, 64>(a, st); break;
    case 513: launch_contig_eg<T, 8, 64>(a, st); break;
    case 1025: launch_contig_eg<T, 16, 64>(a, st); break;
    case 2049: launch_contig_eg<T, 32, 64>(a, st); break;
    case 4097: launch_contig_eg<T, 64, 64>(a, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int C>
static void launch_twisted_c(StridedArgs<T> a, int mode, hipStream_t st) {
  dim3 grid((unsigned)(((int64_t)a.nx * a.nouter + 127) / 128));
  if (mode == kSolveApply)
    hipLaunchKernelGGL((k_solve_twisted<T, C, kSolveApply>), grid, dim3(256), 0, st, a);
  else if (mode == kSolveStore)
    hipLaunchKernelGGL((k_solve_twisted<T, C, kSolveStore>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_solve_twisted<T, C, kSolveInPlace>), grid, dim3(256), 0, st, a);
}

template <typename T, int CH>
static void launch_chunked(StridedArgs<T> a, int mode, hipStream_t st) {
  dim3 grid((unsigned)((a.nx + 255) / 256), (unsigned)a.nouter);
  if (mode == kSolveApply)
    hipLaunchKernelGGL((k_solve_strided<T, kSolveApply, CH>), grid, dim3(256), 0, st, a);
  else if (mode == kSolveStore)
    hipLaunchKernelGGL((k_solve_strided<T, kSolveStore, CH>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_solve_strided<T, kSolveInPlace, CH>), grid, dim3(256), 0, st, a);
}

// Segment length of the segmented solve (register budget: SEG + 1 values per
// lane) and whether a line of c nodes takes it: longer than the two-ended
// solve handles, and at most kSegMaxWaves segments.
template <typename T>
constexpr int seg_len() {
  return sizeof(T) == 8 ? 16 : 32;
}
template <typename T>
static bool strided_seg(int c) {
  return c >= MGX_SEG_MINC && (c - 1) % seg_len<T>() == 0 && (c - 1) / seg_len<T>() >= 2 &&
         (c - 1) / seg_len<T>() <= kSegMaxWaves;
}

template <typename T>
static hipError_t launch_seg(StridedArgs<T> a, int mode, hipStream_t st) {
  constexpr int SEG = seg_len<T>();
  const int P = (a.c - 1) / SEG;
  dim3 grid((unsigned)(((int64_t)a.nx * a.nouter + 63) / 64));
  if (mode == kSolveApply)
    hipLaunchKernelGGL((k_solve_seg<T, SEG, kSolveApply>), grid, dim3(64 * P), 0, st, a);
  else if (mode == kSolveStore)
    hipLaunchKernelGGL((k_solve_seg<T, SEG, kSolveStore>), grid, dim3(64 * P), 0, st, a);
  else
    hipLaunchKernelGGL((k_solve_seg<T, SEG, kSolveInPlace>), grid, dim3(64 * P), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_solve_strided(StridedArgs<T> a, int mode, hipStream_t st) {
  // lines of MGX_SEG_MINC nodes and more: segments of the line on the waves
  // of a workgroup (measured faster at 257 fp32 nodes: 34 against 40 us per
  // in-place pass of the 513^3 field's finest level; at 129, 5 us off the
  // 513^3 step); shorter ones: the two-ended register solve (half a line in
  // registers)
  if (strided_seg<T>(a.c)) return launch_seg<T>(a, mode, st);
  switch (a.c) {
    case 3: launch_twisted_c<T, 3>(a, mode, st); return hipGetLastError();
    case 5: launch_twisted_c<T, 5>(a, mode, st); return hipGetLastError();
    case 9: launch_twisted_c<T, 9>(a, mode, st); return hipGetLastError();
    case 17: launch_twisted_c<T, 17>(a, mode, st); return hipGetLastError();
    case 33: launch_twisted_c<T, 33>(a, mode, st); return hipGetLastError();
    case 65: launch_twisted_c<T, 65>(a, mode, st); return hipGetLastError();
    case 129: launch_twisted_c<T, 129>(a, mode, st); return hipGetLastError();
    default: break;
  }
  // the longest lines: chunked sweeps; few lines (one wave per SIMD or less)
  // use deep chunks to keep enough loads in flight
  const bool deep = (int64_t)a.nx * a.nouter < (1 << 18);
  constexpr int CS = sizeof(T) == 8 ? 8 : 16;
  constexpr int CD = sizeof(T) == 8 ? MGX_DEEP_CH / 2 : MGX_DEEP_CH;
  if (deep)
    launch_chunked<T, CD>(a, mode, st);
  else
    launch_chunked<T, CS>(a, mode, st);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply(StridedArgs<T> a, hipStream_t st) {
  dim3 grid((unsigned)((a.nx + 255) / 256));
  hipLaunchKernelGGL((k_apply<T>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_mass(ProlongArgs<T> a, int mode, hipStream_t st) {
  constexpr int TX = Tiles<T>::TX, TY = Tiles<T>::TY, NT = Tiles<T>::NT;
  if (!tile_grid(a.ax[0].c, a.ax[1].c, a.ax[2].c, TX, TY, &a.ntx, &a.nty, &a.nzc, &a.tz))
    return hipErrorInvalidValue;
  dim3 grid(a.ntx * a.nty * a.nzc);
  if (mode == kProlongRecAdj)
    hipLaunchKernelGGL((k_prolong_mass<T, TX, TY, NT, kProlongRecAdj>), grid, dim3(NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_prolong_mass<T, TX, TY, NT, kProlongDecAdj>), grid, dim3(NT), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy_box(CopyArgs<T> a, hipStream_t st) {
  const int64_t n = (int64_t)a.n0 * a.n1 * a.n2;
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL((k_copy_box<T>), dim3((unsigned)g), dim3(256), 0, st, a);
  return hipGetLastError();
}

static unsigned quant_grid(int64_t n) {
  int64_t g = (n + 1023) / 1024;
  if (g > 8192) g = 8192;
  return (unsigned)(g > 0 ? g : 1);
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

template <typename T>
hipError_t launch_quantize(const T *umc, int32_t *labels, QuantArgs a, bool stats, hipStream_t st) {
  if (a.box && !stats) {
    int64_t g = (a.bn + 255) / 256;
    hipLaunchKernelGGL((k_quantize_box<T>), dim3((unsigned)(g < 1 ? 1 : (g > 8192 ? 8192 : g))), dim3(256), 0, st,
                       umc, labels, a);
    return hipGetLastError();
  }
  dim3 grid(quant_grid(a.n));
  const bool vec = aligned16(umc) && aligned16(labels);
  if (stats) {
    if (vec)
      hipLaunchKernelGGL((k_quantize<T, true, true>), grid, dim3(256), 0, st, umc, labels, a);
    else
      hipLaunchKernelGGL((k_quantize<T, true, false>), grid, dim3(256), 0, st, umc, labels, a);
  } else {
    if (vec)
      hipLaunchKernelGGL((k_quantize<T, false, true>), grid, dim3(256), 0, st, umc, labels, a);
    else
      hipLaunchKernelGGL((k_quantize<T, false, false>), grid, dim3(256), 0, st, umc, labels, a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dequantize(const int32_t *labels, T *umc, QuantArgs a, hipStream_t st) {
  if (a.box) {
    int64_t g = (a.bn + 255) / 256;
    hipLaunchKernelGGL((k_dequantize_box<T>), dim3((unsigned)(g < 1 ? 1 : (g > 8192 ? 8192 : g))), dim3(256), 0,
                       st, labels, umc, a);
    return hipGetLastError();
  }
  dim3 grid(quant_grid(a.n));
  if (aligned16(umc) && aligned16(labels))
    hipLaunchKernelGGL((k_dequantize<T, true>), grid, dim3(256), 0, st, labels, umc, a);
  else
    hipLaunchKernelGGL((k_dequantize<T, false>), grid, dim3(256), 0, st, labels, umc, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tail of the hierarchy in one workgroup.  Every level of the tail has at
// most kTailBox nodes per axis, so a step is too small to fill the chip and a
// launch per step is latency bound.  One workgroup of 1024 threads runs all
// the tail's levels with the same arithmetic as the tiled kernels, entirely
// in LDS, phase by phase with a workgroup barrier between phases:
// coefficients, the load vector as three separable 5-point passes (x, y, z)
// and the three Thomas solves.  Global memory is touched once per level for
// the coefficients and once for the tail's input or output box.
// ---------------------------------------------------------------------------
constexpr int kTailThreads = 1024;
constexpr int kTailM = kTailBox, kTailC = (kTailBox + 1) / 2;
constexpr int kTailV = kTailM * kTailM * kTailM;   // a level box
constexpr int kTailG1 = kTailM * kTailM * kTailC;  // after the x pass
constexpr int kTailG2 = kTailM * kTailC * kTailC;  // after the y pass
constexpr int kTailF = kTailC * kTailC * kTailC;   // a coarse box
constexpr int kTailLds = kTailV + kTailG1 + kTailG2 + 2 * kTailF;
// per level and axis: wl, wr (m each), w5 (5c), mult, invd, qsup (c each)
constexpr int kTailTab = 2 * kTailM + 8 * kTailC;

// LDS-typed pointers for the tail: with generic pointers the compiler emits
// flat accesses, which wait on the vector memory counter too, so every LDS
// read would first wait for the level's label and coefficient stores.
template <typename T>
using lds = __attribute__((address_space(3))) T;

// One axis of one tail level, its tables in LDS: wl, wr (m each), w5 (5c),
// mult, invd, qsup (c each), laid out in that order from b.
template <typename T>
struct TailTab {
  lds<const T> *b;
  int m, c;
  uint32_t mm, cm;  // division magics as in TailAxis
  __device__ __forceinline__ T wl(int j) const { return b[j]; }
  __device__ __forceinline__ T wr(int j) const { return b[m + j]; }
  __device__ __forceinline__ T w5(int i) const { return b[2 * m + i]; }
  __device__ __forceinline__ T mult(int j) const { return b[2 * m + 5 * c + j]; }
  __device__ __forceinline__ T invd(int j) const { return b[2 * m + 6 * c + j]; }
  __device__ __forceinline__ T qsup(int j) const { return b[2 * m + 7 * c + j]; }
};

// Copies the tables of the tail's levels into LDS (they are read inside
// dependent chains, e.g. every step of a line solve) and fills their views.
// Each pair of waves takes one (level, axis) slot per round, 128 words, and
// every round's load is issued before the first word is stored.  Ends with a
// workgroup barrier.
template <typename T>
__device__ __forceinline__ void tail_tables(const TailArgs<T> &a, lds<T> *sT, TailTab<T> (&ax)[kTailMax][3]) {
  static_assert(kTailTab <= 128, "one slot per pair of waves");
  constexpr int kSlots = kTailThreads / 128, kRounds = (kTailMax * 3 + kSlots - 1) / kSlots;
  const int tid = threadIdx.x, q = tid & 127;
  const int s0 = __builtin_amdgcn_readfirstlane(tid >> 7);
  T v[kRounds];
  bool st[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; r++) {
    const int sl = s0 + kSlots * r;
    st[r] = false;
    v[r] = T(0);
    if (sl < 3 * a.nlev) {
      const TailAxis<T> &g = a.ax[sl / 3][sl % 3];
      const int m = g.m, c = g.c;
      const T *src = q < m           ? g.wl + q
                     : q < 2 * m     ? g.wr + (q - m)
                     : q < 2 * m + 5 * c ? g.w5 + (q - 2 * m)
                     : q < 2 * m + 6 * c ? g.mult + (q - 2 * m - 5 * c)
                     : q < 2 * m + 7 * c ? g.invd + (q - 2 * m - 6 * c)
                                         : g.qsup + min(q - 2 * m - 7 * c, c - 1);
      st[r] = q < 2 * m + 8 * c;
      v[r] = *src;
    }
  }
#pragma unroll
  for (int r = 0; r < kRounds; r++)
    if (st[r]) sT[(s0 + kSlots * r) * kTailTab + q] = v[r];
  if (tid < 3 * a.nlev) {
    const TailAxis<T> &g = a.ax[tid / 3][tid % 3];
    ax[tid / 3][tid % 3] = TailTab<T>{sT + tid * kTailTab, g.m, g.c, g.mm, g.cm};
  }
  __syncthreads();
}

__device__ __forceinline__ int lcp(int j, int c) { return (j & 1) ? c + (j >> 1) : (j >> 1); }

// q / d and q % d for the tail's small boxes, from d's magic (TailAxis::mm,
// cm): one multiply instead of an integer division sequence.  The phases of
// a tail step split a linear index into box coordinates for every node, and
// with one workgroup on one CU those divisions were most of their time.
__device__ __forceinline__ int tdiv(int q, int d, uint32_t mg) {
  return d > 1 ? (int)__umulhi((uint32_t)q, mg) : q;
}

// Weights and corner offsets (along one axis) of the multilinear interpolant
// at level index j: corners lo/hi in units of the coarse index.
template <typename T>
__device__ __forceinline__ void tail_corner(const TailTab<T> &ax, int j, int &lo, int &hi, T &wlo, T &whi) {
  const int odd = j & 1;
  const T l = ax.wl(j), r = ax.wr(j);
  lo = (j - odd) >> 1;
  hi = (j + odd) >> 1;
  wlo = odd ? l : T(1);
  whi = odd ? r : T(0);
}

// Interpolant at level node (j0,j1,j2) from a coarse box C (pitches cp0, cp1).
// All eight corners are read and summed in a fixed order; a corner of weight
// zero (an even index) adds a signed zero, which leaves the sum's value as
// it is.  Without branches the reads of a node go out together.
template <typename T>
__device__ __forceinline__ T tail_interp(const lds<T> *C, int cp0, int cp1, int cp2, const TailTab<T> (&ax)[3],
                                         int j0, int j1, int j2) {
  int lo[3], hi[3];
  T wlo[3], whi[3];
  tail_corner(ax[0], j0, lo[0], hi[0], wlo[0], whi[0]);
  tail_corner(ax[1], j1, lo[1], hi[1], wlo[1], whi[1]);
  tail_corner(ax[2], j2, lo[2], hi[2], wlo[2], whi[2]);
  T acc = T(0);
#pragma unroll
  for (int c = 0; c < 8; c++) {
    const T w = ((c & 1) ? whi[0] : wlo[0]) * ((c & 2) ? whi[1] : wlo[1]) * ((c & 4) ? whi[2] : wlo[2]);
    acc += w * C[((c & 1) ? hi[0] : lo[0]) * cp0 + ((c & 2) ? hi[1] : lo[1]) * cp1 +
                 ((c & 4) ? hi[2] : lo[2]) * cp2];
  }
  return acc;
}

// F = (R M)^{x3} of the level box V (compact, in LDS), via g1 and g2.
template <typename T>
__device__ __forceinline__ void tail_load_vector(const TailTab<T> (&ax)[3], const lds<T> *V, lds<T> *g1, lds<T> *g2,
                                                 lds<T> *F) {
  const int m0 = ax[0].m, m1 = ax[1].m, m2 = ax[2].m, c0 = ax[0].c, c1 = ax[1].c, c2 = ax[2].c;
  const int tid = threadIdx.x;
  const uint32_t c1g = ax[1].cm, c2g = ax[2].cm;
  for (int i = tid; i < m0 * m1 * c2; i += kTailThreads) {
    const int r = tdiv(i, c2, c2g), X = i - r * c2;
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < 5; d++) {  // taps outside the box: weight 0 on a node inside
      const int x = 2 * X + d - 2;
      const bool in = x >= 0 && x < m2;
      const T w = ax[2].w5(X * 5 + d);
      acc += (in ? w : T(0)) * V[r * m2 + (in ? x : 0)];
    }
    g1[i] = acc;
  }
  __syncthreads();
  for (int i = tid; i < m0 * c1 * c2; i += kTailThreads) {
    const int r = tdiv(i, c2, c2g), X = i - r * c2, z = tdiv(r, c1, c1g), Y = r - z * c1;
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < 5; d++) {
      const int y = 2 * Y + d - 2;
      const bool in = y >= 0 && y < m1;
      const T w = ax[1].w5(Y * 5 + d);
      acc += (in ? w : T(0)) * g1[(z * m1 + (in ? y : 0)) * c2 + X];
    }
    g2[i] = acc;
  }
  __syncthreads();
  for (int i = tid; i < c0 * c1 * c2; i += kTailThreads) {
    const int r = tdiv(i, c2, c2g), X = i - r * c2, Z = tdiv(r, c1, c1g), Y = r - Z * c1;
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < 5; d++) {
      const int z = 2 * Z + d - 2;
      const bool in = z >= 0 && z < m0;
      const T w = ax[0].w5(Z * 5 + d);
      acc += (in ? w : T(0)) * g2[((in ? z : 0) * c1 + Y) * c2 + X];
    }
    F[i] = acc;
  }
  __syncthreads();
}

// Thomas solves of the coarse mass matrix along x, y and z, in place on F.
// A thread takes one line: its values and factors are read into registers
// first (lines have at most kTailC nodes), so the two sweeps' dependent
// chains run in registers rather than through LDS round trips.
template <typename T>
__device__ __forceinline__ void tail_solves(const TailTab<T> (&ax)[3], lds<T> *F) {
  const int c0 = ax[0].c, c1 = ax[1].c, c2 = ax[2].c;
  const int tid = threadIdx.x;
  const int n[3] = {c0, c1, c2};
  const int stride[3] = {c1 * c2, c2, 1};
  for (int k = 2; k >= 0; k--) {
    const int c = n[k];
    const int o1 = k == 0 ? 1 : 0, o2 = k == 2 ? 1 : 2;
    const int nl = n[o1] * n[o2];
    const TailTab<T> &t = ax[k];
    if (tid < nl) {
      const int t1 = tdiv(tid, n[o2], o2 == 2 ? ax[2].cm : ax[1].cm);
      lds<T> *p = F + t1 * stride[o1] + (tid - t1 * n[o2]) * stride[o2];
      const int s = stride[k];
      T x[kTailC], mu[kTailC], iv[kTailC], qs[kTailC];
#pragma unroll
      for (int J = 0; J < kTailC; J++) {
        const int Jc = min(J, c - 1);
        x[J] = p[Jc * s];
        mu[J] = t.mult(Jc);
        iv[J] = t.invd(Jc);
        qs[J] = t.qsup(Jc);
      }
#pragma unroll
      for (int J = 1; J < kTailC; J++) {
        const T f = x[J] - mu[J] * x[J - 1];
        x[J] = J < c ? f : x[J];
      }
      T y = T(0);
#pragma unroll
      for (int J = kTailC - 1; J >= 0; J--) {
        const T b = J == c - 1 ? iv[J] * x[J] : iv[J] * x[J] - qs[J] * y;
        y = J < c ? b : y;
        x[J] = y;
      }
#pragma unroll
      for (int J = 0; J < kTailC; J++)
        if (J < c) p[J * s] = x[J];
    }
    __syncthreads();
  }
}

template <typename T>
__device__ __forceinline__ void tail_dec_body(const TailArgs<T> &a) {
  __shared__ T sm_[kTailLds];
  __shared__ T sT_[kTailMax * 3 * kTailTab];
  lds<T> *const sm = (lds<T> *)sm_, *const sT = (lds<T> *)sT_;
  lds<T> *const sV = sm, *const g1 = sV + kTailV, *const g2 = g1 + kTailG1, *const fA = g2 + kTailG2,
                *const fB = fA + kTailF;
  const int tid = threadIdx.x;
  __shared__ TailTab<T> tabs[kTailMax][3];  // views of sT
  tail_tables<T>(a, sT, tabs);
  {  // the level-lt box into LDS (all loads issued before the first wait)
    const int m0 = a.ax[0][0].m, m1 = a.ax[0][1].m, m2 = a.ax[0][2].m, n = m0 * m1 * m2;
    const uint32_t m1g = a.ax[0][1].mm, m2g = a.ax[0][2].mm;
    constexpr int R = (kTailV + kTailThreads - 1) / kTailThreads;
    T r[R];
#pragma unroll
    for (int k = 0; k < R; k++) {
      const int q = min(tid + k * kTailThreads, n - 1);  // lanes past the box reload its last node
      const int t = tdiv(q, m2, m2g), j2 = q - t * m2, j0 = tdiv(t, m1, m1g), j1 = t - j0 * m1;
      r[k] = a.src[j0 * a.sp0 + j1 * a.sp1 + j2];
    }
#pragma unroll
    for (int k = 0; k < R; k++)
      if (tid + k * kTailThreads < n) sV[tid + k * kTailThreads] = r[k];
    __syncthreads();
  }
  const lds<T> *V = sV;
  int lmax = 0;  // with a.smax: largest |label| of the current level written by this thread
  for (int i = 0; i < a.nlev; i++) {
    const TailTab<T>(&ax)[3] = tabs[i];
    const int m1 = ax[1].m, m2 = ax[2].m, c0 = ax[0].c, c1 = ax[1].c, c2 = ax[2].c;
    const int m0 = ax[0].m;
    const double qi = a.q[i];
    const float rqi = label_rcp(qi);
    // coefficients of the level's non-nodal nodes, at level-centric positions
    const uint32_t m1g = ax[1].mm, m2g = ax[2].mm;
    for (int q = tid; q < m0 * m1 * m2; q += kTailThreads) {
      const int r = tdiv(q, m2, m2g), j2 = q - r * m2, j0 = tdiv(r, m1, m1g), j1 = r - j0 * m1;
      // nodal corners of V at level indices: the interpolant reads V at
      // 2*lo, 2*hi, i.e. a coarse view with doubled pitches.  Computed at
      // nodal nodes too (no divergence), stored only at the others.
      const T v = V[q] - tail_interp<T>(V, 2 * m1 * m2, 2 * m2, 2, ax, j0, j1, j2);
      if (!((j0 | j1 | j2) & 1)) continue;
      const int64_t pos = lcp(j0, c0) * a.up0 + lcp(j1, c1) * a.up1 + lcp(j2, c2);
      if (a.umc) a.umc[pos] = v;
      if (a.lab_w) {
        const int32_t lab = label_of(v, qi, rqi);
        a.lab_w[pos] = lab;
        if (lab == INT32_MIN && a.rng) count_out_of_range(a.rng, v, qi);
        if (lab != INT32_MIN) lmax = max(lmax, lab < 0 ? -lab : lab);
      }
    }
    if (a.smax && lmax > 0) atomicMax(&a.smax[a.nlev - i], lmax);  // level lt - i; the tail is small
    lmax = 0;
    // Q_{l-1} u = Mc^{-1} (R M)^{x3} V (as in the tiled decomposition)
    lds<T> *F = (i & 1) ? fB : fA;
    tail_load_vector<T>(ax, V, g1, g2, F);
    tail_solves<T>(ax, F);
    if (i == a.nlev - 1) {
      const double qs = a.q[a.nlev];
      const float rqs = label_rcp(qs);
      for (int q = tid; q < c0 * c1 * c2; q += kTailThreads) {
        const int r = tdiv(q, c2, ax[2].cm), X = q - r * c2, Z = tdiv(r, c1, ax[1].cm), Y = r - Z * c1;
        const int64_t pos = Z * a.up0 + Y * a.up1 + X;
        const T f = F[q];
        if (a.umc) a.umc[pos] = f;
        if (a.lab_w) {
          const int32_t lab = label_of(f, qs, rqs);
          a.lab_w[pos] = lab;
          if (lab == INT32_MIN && a.rng) count_out_of_range(a.rng, f, qs);
          if (lab != INT32_MIN) lmax = max(lmax, lab < 0 ? -lab : lab);
        }
      }
      if (a.smax && lmax > 0) atomicMax(&a.smax[0], lmax);
    }
    V = F;
  }
}

template <typename T>
__device__ __forceinline__ void tail_rec_body(const TailArgs<T> &a) {
  __shared__ T sm_[kTailLds];
  __shared__ T sT_[kTailMax * 3 * kTailTab];
  lds<T> *const sm = (lds<T> *)sm_, *const sT = (lds<T> *)sT_;
  lds<T> *const sZ = sm, *const g1 = sZ + kTailV, *const g2 = g1 + kTailG1, *const fA = g2 + kTailG2,
                *const vB = fA + kTailF;
  const int tid = threadIdx.x;
  __shared__ TailTab<T> tabs[kTailMax][3];  // views of sT
  tail_tables<T>(a, sT, tabs);
  const T *U = a.umc_r;
  // nodal values of the level below: the stop box of u_mc first
  {
    const TailTab<T>(&ax)[3] = tabs[a.nlev - 1];
    const int c0 = ax[0].c, c1 = ax[1].c, c2 = ax[2].c;
    const double qs = a.q[a.nlev];
    for (int q = tid; q < c0 * c1 * c2; q += kTailThreads) {
      const int r = tdiv(q, c2, ax[2].cm), X = q - r * c2, Z = tdiv(r, c1, ax[1].cm), Y = r - Z * c1;
      const int64_t pos = Z * a.up0 + Y * a.up1 + X;
      vB[q] = a.lab_r ? from_label<T>(a.lab_r[pos], qs) : U[pos];
    }
  }
  for (int i = 0; i < a.nlev; i++) {
    const TailTab<T>(&ax)[3] = tabs[a.nlev - 1 - i];
    const int m0 = ax[0].m, m1 = ax[1].m, m2 = ax[2].m, c0 = ax[0].c, c1 = ax[1].c, c2 = ax[2].c;
    // the level's coefficients (zero at nodal nodes) into LDS, all loads
    // issued before the first wait
    {
      const int n = m0 * m1 * m2;
      const double qi = a.q[a.nlev - 1 - i];
      constexpr int R = (kTailV + kTailThreads - 1) / kTailThreads;
      int64_t pos[R];
      unsigned coef = 0;
#pragma unroll
      for (int k = 0; k < R; k++) {
        const int q = tid + k * kTailThreads;
        const int qc = min(q, n - 1);
        const int t = tdiv(qc, m2, ax[2].mm), j2 = qc - t * m2, j0 = tdiv(t, m1, ax[1].mm), j1 = t - j0 * m1;
        const bool cf = q < n && ((j0 | j1 | j2) & 1);
        coef |= (unsigned)cf << k;
        pos[k] = cf ? lcp(j0, c0) * a.up0 + lcp(j1, c1) * a.up1 + lcp(j2, c2) : 0;
      }
      // every load issued unconditionally (nodal lanes read element 0) and
      // converted only after the last one, so the thread waits once
      T r[R];
      if (a.lab_r) {
        int32_t w[R];
#pragma unroll
        for (int k = 0; k < R; k++) w[k] = a.lab_r[pos[k]];
#pragma unroll
        for (int k = 0; k < R; k++) r[k] = ((coef >> k) & 1u) ? from_label<T>(w[k], qi) : T(0);
      } else {
#pragma unroll
        for (int k = 0; k < R; k++) r[k] = U[pos[k]];
#pragma unroll
        for (int k = 0; k < R; k++) r[k] = ((coef >> k) & 1u) ? r[k] : T(0);
      }
#pragma unroll
      for (int k = 0; k < R; k++)
        if (tid + k * kTailThreads < n) sZ[tid + k * kTailThreads] = r[k];
    }
    __syncthreads();
    // correction from the coefficients, subtracted from the nodal values
    tail_load_vector<T>(ax, sZ, g1, g2, fA);
    tail_solves<T>(ax, fA);
    for (int q = tid; q < c0 * c1 * c2; q += kTailThreads) fA[q] = vB[q] - fA[q];
    __syncthreads();
    // level box: nodal values, coefficients plus the interpolant
    const bool last = i == a.nlev - 1;
    for (int q = tid; q < m0 * m1 * m2; q += kTailThreads) {
      const int r = tdiv(q, m2, ax[2].mm), j2 = q - r * m2, j0 = tdiv(r, m1, ax[1].mm), j1 = r - j0 * m1;
      const T vc = sZ[q] + tail_interp<T>(fA, c1 * c2, c2, 1, ax, j0, j1, j2);
      const T vn = fA[((j0 >> 1) * c1 + (j1 >> 1)) * c2 + (j2 >> 1)];
      const T v = ((j0 | j1 | j2) & 1) ? vc : vn;
      if (last)
        a.dst[j0 * a.dp0 + j1 * a.dp1 + j2] = v;
      else
        vB[q] = v;  // the next level's nodal values (its coarse box)
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(kTailThreads) k_tail_dec(TailArgs<T> a) {
  tail_dec_body<T>(a);
}

template <typename T>
__global__ void __launch_bounds__(kTailThreads) k_tail_rec(TailArgs<T> a) {
  tail_rec_body<T>(a);
}

// ---------------------------------------------------------------------------
// Multi-field launches.  One grid covers several ops of one kernel instance
// (for example the load-vector step of every field of a batch at the same
// level depth): workgroup g belongs to op f with start[f] <= g < start[f+1]
// and runs the op's body with local index g - start[f].  The op arguments
// are read from device memory; they are uniform per workgroup.
// ---------------------------------------------------------------------------
template <typename T>
struct MultiArgs {
  const OpArgs<T> *__restrict__ args;
  const int *__restrict__ start;
  int n;
};

// The op's arguments, read through the constant address space (the buffer is
// written before the launch and only read during it).  Pointers loaded from
// constant memory are known to be global; loaded through a generic pointer,
// every access through them would be a flat instruction, whose waits also
// wait for the LDS operations in flight.  Used by the stencil and solve
// kernels (the elementwise and tail kernels index their arguments
// dynamically, which a copy would place in scratch).
// (The host compilation pass also type-checks this device function but never
// runs it; the copy out of the constant address space is a device-pass
// construct, so the host pass reads the generic pointer.)
template <typename T>
__device__ __forceinline__ OpArgs<T> op_args(const MultiArgs<T> &m, int f) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(4))) OpArgs<T> *)m.args)[f];
#else
  return m.args[f];
#endif
}

__device__ __forceinline__ int find_op(const int *__restrict__ start, int n, int g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, int TX, int TY, int NT, bool DEC, int LAB>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(DEC ? MGX_STENCIL_WAVES : MGX_REC_WAVES, 8)))
k_load_vector_multi(MultiArgs<T> m) {
  const int g = xcd_remap(blockIdx.x, gridDim.x);
  const int f = find_op(m.start, m.n, g);
  load_vector_body<T, TX, TY, NT, DEC, LAB>(op_args(m, f).st, g - m.start[f]);
}

template <typename T, int TX, int TY, int NT, bool LAB>
__global__ void __launch_bounds__(NT) k_interp_add_multi(MultiArgs<T> m) {
  const int g = xcd_remap(blockIdx.x, gridDim.x);
  const int f = find_op(m.start, m.n, g);
  interp_add_body<T, TX, TY, NT, LAB>(op_args(m, f).ia, g - m.start[f]);
}

template <typename T, int TX, int TY, int NTP, bool LAB>
__global__ void __launch_bounds__(NTP) k_interp_plane_multi(MultiArgs<T> m) {
  const int g = xcd_remap(blockIdx.x, gridDim.x);
  const int f = find_op(m.start, m.n, g);
  interp_plane_body<T, TX, TY, NTP, LAB>(op_args(m, f).ia, g - m.start[f]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_quantize_box_multi(MultiArgs<T> m) {
  const int g = blockIdx.x;
  const int f = find_op(m.start, m.n, g);
  const QuantJob<T> &j = m.args[f].qj;
  quantize_box_body<T>(j.umc, j.labels, j.a, g - m.start[f], m.start[f + 1] - m.start[f]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_dequantize_box_multi(MultiArgs<T> m) {
  const int g = blockIdx.x;
  const int f = find_op(m.start, m.n, g);
  const DequantJob<T> &j = m.args[f].dj;
  dequantize_box_body<T>(j.labels, j.umc, j.a, g - m.start[f], m.start[f + 1] - m.start[f]);
}

template <typename T, int E, int G>
__global__ void __launch_bounds__(256) k_solve_contig_multi(MultiArgs<T> m) {
  const int g = blockIdx.x;
  const int f = find_op(m.start, m.n, g);
  solve_contig_body<T, E, G>(op_args(m, f).so, g - m.start[f]);
}

template <typename T, int C, int MODE>
__global__ void __launch_bounds__(256) k_solve_twisted_multi(MultiArgs<T> m) {
  const int g = blockIdx.x;
  const int f = find_op(m.start, m.n, g);
  const StridedArgs<T> a = op_args(m, f).sd;
  solve_twisted_body<T, C, MODE>(a, g - m.start[f]);
}

template <typename T, int MODE, int CH>
__global__ void __launch_bounds__(256) k_solve_strided_multi(MultiArgs<T> m) {
  const int g = blockIdx.x;
  const int f = find_op(m.start, m.n, g);
  const StridedArgs<T> a = op_args(m, f).sd;
  const int b = g - m.start[f], nbx = (a.nx + 255) / 256;
  solve_strided_body<T, MODE, CH>(a, b % nbx, b / nbx);
}

template <typename T, int SEG, int MODE>
__global__ void __launch_bounds__(64 * kSegMaxWaves) k_solve_seg_multi(MultiArgs<T> m) {
  const int g = blockIdx.x;
  const int f = find_op(m.start, m.n, g);
  solve_seg_body<T, SEG, MODE>(op_args(m, f).sd, g - m.start[f]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_apply_multi(MultiArgs<T> m) {
  const int g = blockIdx.x;
  const int f = find_op(m.start, m.n, g);
  apply_body<T>(op_args(m, f).sd, g - m.start[f]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_copy_box_multi(MultiArgs<T> m) {
  const int g = blockIdx.x;
  const int f = find_op(m.start, m.n, g);
  copy_box_body<T>(op_args(m, f).cp, g - m.start[f], m.start[f + 1] - m.start[f]);
}

template <typename T, bool VEC, bool STATS>
__global__ void __launch_bounds__(256) k_quantize_multi(MultiArgs<T> m) {
  const int g = blockIdx.x;
  const int f = find_op(m.start, m.n, g);
  const QuantJob<T> &j = m.args[f].qj;
  quantize_body<T, STATS, VEC>(j.umc, j.labels, j.a, g - m.start[f], m.start[f + 1] - m.start[f]);
}

template <typename T, bool VEC>
__global__ void __launch_bounds__(256) k_dequantize_multi(MultiArgs<T> m) {
  const int g = blockIdx.x;
  const int f = find_op(m.start, m.n, g);
  const DequantJob<T> &j = m.args[f].dj;
  dequantize_body<T, VEC>(j.labels, j.umc, j.a, g - m.start[f], m.start[f + 1] - m.start[f]);
}

template <typename T>
__global__ void __launch_bounds__(kTailThreads) k_tail_dec_multi(MultiArgs<T> m) {
  tail_dec_body<T>(m.args[find_op(m.start, m.n, blockIdx.x)].tl);
}

template <typename T>
__global__ void __launch_bounds__(kTailThreads) k_tail_rec_multi(MultiArgs<T> m) {
  tail_rec_body<T>(m.args[find_op(m.start, m.n, blockIdx.x)].tl);
}

// ---- op dispatch (host) ----
// line length c of the contiguous solve -> (E, G) instance index
static int contig_index(int c) {
  switch (c) {
    case 3: return 0;
    case 5: return 1;
    case 9: return 2;
    case 17: return 3;
    case 33: return 4;
    case 65: return 5;
    case 129: return 6;
    case 257: return 7;
    case 513: return 8;
    case 1025: return 9;
    case 2049: return 10;
    case 4097: return 11;
    default: return -1;
  }
}
static int contig_group(int c) {  // G: lanes per line
  return c <= 65 ? (c - 1) : 64;
}

template <typename T>
static bool strided_twisted(int c) {
  return c <= 129 && !strided_seg<T>(c);
}
template <typename T>
static bool strided_deep(const StridedArgs<T> &a) {
  return (int64_t)a.nx * a.nouter < (1 << 18);
}

static int grid_cap(int64_t blocks) {
  if (blocks > 8192) blocks = 8192;
  return (int)(blocks > 0 ? blocks : 1);
}

template <typename T>
int op_blocks(int kind, int mode, OpArgs<T> &a, const Tuning &tn) {
  constexpr int TX = Tiles<T>::TX, TY = Tiles<T>::TY;
  (void)mode;
  switch (kind) {
    case kOpLoadVecDec:
    case kOpLoadVecRec: {
      StencilArgs<T> &s = a.st;
      if (!tile_grid(s.ax[0].c, s.ax[1].c, s.ax[2].c, TX, TY, &s.ntx, &s.nty, &s.nzc, &s.tz, tn)) return -1;
      return s.ntx * s.nty * s.nzc;
    }
    case kOpInterpAdd: {
      InterpArgs<T> &s = a.ia;
      constexpr int IX = InterpTiles<T>::TX, IY = InterpTiles<T>::TY;
      if (!tile_grid(s.ax[0].c, s.ax[1].c, s.ax[2].c, IX, IY, &s.ntx, &s.nty, &s.nzc, &s.tz, tn)) return -1;
      if (interp_plane(s)) {
        s.nzc = (s.ax[0].c + MGX_INTERP_NP - 1) / MGX_INTERP_NP;
        s.tz = MGX_INTERP_NP;
      }
      return s.ntx * s.nty * s.nzc;
    }
    case kOpSolveContig: {
      if (contig_index(a.so.c) < 0) return -1;
      const int64_t lpb = 4 * (64 / contig_group(a.so.c));
      return (int)((a.so.nlines + lpb - 1) / lpb);
    }
    case kOpSolveStrided: {
      if (strided_twisted<T>(a.sd.c)) return (int)(((int64_t)a.sd.nx * a.sd.nouter + 127) / 128);
      if (strided_seg<T>(a.sd.c)) return (int)(((int64_t)a.sd.nx * a.sd.nouter + 63) / 64);
      return (int)(((int64_t)a.sd.nx + 255) / 256 * a.sd.nouter);
    }
    case kOpApply: return (a.sd.nx + 255) / 256;
    case kOpQuantize: return grid_cap(a.qj.a.box ? (a.qj.a.bn + 255) / 256 : (a.qj.a.n + 1023) / 1024);
    case kOpDequantize: return grid_cap(a.dj.a.box ? (a.dj.a.bn + 255) / 256 : (a.dj.a.n + 1023) / 1024);
    case kOpCopyBox: return grid_cap(((int64_t)a.cp.n0 * a.cp.n1 * a.cp.n2 + 255) / 256);
    case kOpTailDec:
    case kOpTailRec: return 1;
  }
  return -1;
}

template <typename T>
int op_key(int kind, int mode, const OpArgs<T> &a) {
  switch (kind) {
    case kOpSolveContig: return a.so.c;
    case kOpLoadVecDec: return a.st.lab_w ? (a.st.smax ? 2 : 1) : 0;
    case kOpLoadVecRec: return a.st.lab_r ? 1 : 0;
    case kOpInterpAdd: return (interp_plane(a.ia) ? 1 : 0) | (a.ia.lab ? 2 : 0);
    case kOpSolveStrided: return (a.sd.c << 4) | (mode << 1) | (strided_deep(a.sd) ? 1 : 0);
    // flat passes with statistics (per-level maxima and counts): 4 | vector form
    case kOpQuantize:
      return a.qj.a.box ? 2 : ((a.qj.a.stats_max ? 4 : 0) | (aligned16(a.qj.umc) && aligned16(a.qj.labels)));
    case kOpDequantize: return a.dj.a.box ? 2 : (aligned16(a.dj.umc) && aligned16(a.dj.labels));
    default: return 0;
  }
}

template <typename T>
hipError_t launch_op(int kind, int mode, OpArgs<T> a, const Tuning &tn, hipStream_t st) {
  switch (kind) {
    case kOpLoadVecDec: return launch_load_vector<T>(a.st, true, st, tn);
    case kOpLoadVecRec: return launch_load_vector<T>(a.st, false, st, tn);
    case kOpInterpAdd: return launch_interp_add<T>(a.ia, st, tn);
    case kOpSolveContig: return launch_solve_contig<T>(a.so, st);
    case kOpSolveStrided: return launch_solve_strided<T>(a.sd, mode, st);
    case kOpApply: return launch_apply<T>(a.sd, st);
    case kOpQuantize:  // the flat pass with statistics when they are asked for
      return launch_quantize<T>(a.qj.umc, a.qj.labels, a.qj.a, !a.qj.a.box && a.qj.a.stats_max != nullptr, st);
    case kOpDequantize: return launch_dequantize<T>(a.dj.labels, a.dj.umc, a.dj.a, st);
    case kOpCopyBox: return launch_copy_box<T>(a.cp, st);
    case kOpTailDec:
      hipLaunchKernelGGL((k_tail_dec<T>), dim3(1), dim3(kTailThreads), 0, st, a.tl);
      return hipGetLastError();
    case kOpTailRec:
      hipLaunchKernelGGL((k_tail_rec<T>), dim3(1), dim3(kTailThreads), 0, st, a.tl);
      return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

#define MGX_MULTI(KERNEL, NT_)                                                    \
  do {                                                                            \
    hipLaunchKernelGGL((KERNEL), dim3((unsigned)total), dim3(NT_), 0, st, m);     \
  } while (0)

template <typename T, int C>
static void twisted_multi(int mode, MultiArgs<T> m, int total, hipStream_t st) {
  if (mode == kSolveApply) MGX_MULTI((k_solve_twisted_multi<T, C, kSolveApply>), 256);
  else if (mode == kSolveStore) MGX_MULTI((k_solve_twisted_multi<T, C, kSolveStore>), 256);
  else MGX_MULTI((k_solve_twisted_multi<T, C, kSolveInPlace>), 256);
}

template <typename T, int CH>
static void chunked_multi(int mode, MultiArgs<T> m, int total, hipStream_t st) {
  if (mode == kSolveApply) MGX_MULTI((k_solve_strided_multi<T, kSolveApply, CH>), 256);
  else if (mode == kSolveStore) MGX_MULTI((k_solve_strided_multi<T, kSolveStore, CH>), 256);
  else MGX_MULTI((k_solve_strided_multi<T, kSolveInPlace, CH>), 256);
}

template <typename T>
hipError_t launch_op_multi(int kind, int key, const OpArgs<T> *dargs, const int *dstart, int n, int total,
                           hipStream_t st) {
  constexpr int TX = Tiles<T>::TX, TY = Tiles<T>::TY, NT = Tiles<T>::NT;
  if (n <= 0 || total <= 0) return hipSuccess;
  MultiArgs<T> m{dargs, dstart, n};
  switch (kind) {
    case kOpLoadVecDec:
      if (key == 2) MGX_MULTI((k_load_vector_multi<T, TX, TY, NT, true, 2>), NT);
      else if (key) MGX_MULTI((k_load_vector_multi<T, TX, TY, NT, true, 1>), NT);
      else MGX_MULTI((k_load_vector_multi<T, TX, TY, NT, true, 0>), NT);
      break;
    case kOpLoadVecRec:
      if (key) MGX_MULTI((k_load_vector_multi<T, TX, TY, NT, false, 1>), NT);
      else MGX_MULTI((k_load_vector_multi<T, TX, TY, NT, false, 0>), NT);
      break;
    case kOpInterpAdd: {
      constexpr int IX = InterpTiles<T>::TX, IY = InterpTiles<T>::TY, INT = InterpTiles<T>::NT;
      constexpr int NTP = interp_plane_threads<T>();
      switch (key) {
        case 0: MGX_MULTI((k_interp_add_multi<T, IX, IY, INT, false>), INT); break;
        case 1: MGX_MULTI((k_interp_plane_multi<T, IX, IY, NTP, false>), NTP); break;
        case 2: MGX_MULTI((k_interp_add_multi<T, IX, IY, INT, true>), INT); break;
        default: MGX_MULTI((k_interp_plane_multi<T, IX, IY, NTP, true>), NTP); break;
      }
      break;
    }
    case kOpApply: MGX_MULTI((k_apply_multi<T>), 256); break;
    case kOpCopyBox: MGX_MULTI((k_copy_box_multi<T>), 256); break;
    case kOpTailDec: MGX_MULTI((k_tail_dec_multi<T>), kTailThreads); break;
    case kOpTailRec: MGX_MULTI((k_tail_rec_multi<T>), kTailThreads); break;
    case kOpQuantize:
      switch (key) {
        case 2: MGX_MULTI((k_quantize_box_multi<T>), 256); break;
        case 1: MGX_MULTI((k_quantize_multi<T, true, false>), 256); break;
        case 5: MGX_MULTI((k_quantize_multi<T, true, true>), 256); break;
        case 4: MGX_MULTI((k_quantize_multi<T, false, true>), 256); break;
        default: MGX_MULTI((k_quantize_multi<T, false, false>), 256); break;
      }
      break;
    case kOpDequantize:
      if (key == 2) MGX_MULTI((k_dequantize_box_multi<T>), 256);
      else if (key) MGX_MULTI((k_dequantize_multi<T, true>), 256);
      else MGX_MULTI((k_dequantize_multi<T, false>), 256);
      break;
    case kOpSolveContig:
      switch (key) {
        case 3: MGX_MULTI((k_solve_contig_multi<T, 1, 2>), 256); break;
        case 5: MGX_MULTI((k_solve_contig_multi<T, 1, 4>), 256); break;
        case 9: MGX_MULTI((k_solve_contig_multi<T, 1, 8>), 256); break;
        case 17: MGX_MULTI((k_solve_contig_multi<T, 1, 16>), 256); break;
        case 33: MGX_MULTI((k_solve_contig_multi<T, 1, 32>), 256); break;
        case 65: MGX_MULTI((k_solve_contig_multi<T, 1, 64>), 256); break;
        case 129: MGX_MULTI((k_solve_contig_multi<T, 2, 64>), 256); break;
        case 257: MGX_MULTI((k_solve_contig_multi<T, 4, 64>), 256); break;
        case 513: MGX_MULTI((k_solve_contig_multi<T, 8, 64>), 256); break;
        case 1025: MGX_MULTI((k_solve_contig_multi<T, 16, 64>), 256); break;
        case 2049: MGX_MULTI((k_solve_contig_multi<T, 32, 64>), 256); break;
        case 4097: MGX_MULTI((k_solve_contig_multi<T, 64, 64>), 256); break;
        default: return hipErrorInvalidValue;
      }
      break;
    case kOpSolveStrided: {
      const int c = key >> 4, mode = (key >> 1) & 7;
      const bool deep = key & 1;
      if (strided_seg<T>(c)) {  // one op kind per launch: every line of it has c nodes
        constexpr int SEG = seg_len<T>();
        const int NTS = 64 * ((c - 1) / SEG);
        if (mode == kSolveApply) MGX_MULTI((k_solve_seg_multi<T, SEG, kSolveApply>), NTS);
        else if (mode == kSolveStore) MGX_MULTI((k_solve_seg_multi<T, SEG, kSolveStore>), NTS);
        else MGX_MULTI((k_solve_seg_multi<T, SEG, kSolveInPlace>), NTS);
        break;
      }
      switch (c) {
        case 3: twisted_multi<T, 3>(mode, m, total, st); break;
        case 5: twisted_multi<T, 5>(mode, m, total, st); break;
        case 9: twisted_multi<T, 9>(mode, m, total, st); break;
        case 17: twisted_multi<T, 17>(mode, m, total, st); break;
        case 33: twisted_multi<T, 33>(mode, m, total, st); break;
        case 65: twisted_multi<T, 65>(mode, m, total, st); break;
        case 129: twisted_multi<T, 129>(mode, m, total, st); break;
        default: {
            constexpr int CS = sizeof(T) == 8 ? 8 : 16;
            constexpr int CD = sizeof(T) == 8 ? MGX_DEEP_CH / 2 : MGX_DEEP_CH;
            if (deep) chunked_multi<T, CD>(mode, m, total, st);
            else chunked_multi<T, CS>(mode, m, total, st);
          }
      }
      break;
    }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
#undef MGX_MULTI

#define MGX_INSTANTIATE(T)                                                                    \
  template hipError_t launch_load_vector<T>(StencilArgs<T>, bool, hipStream_t, Tuning);       \
  template hipError_t launch_interp_add<T>(InterpArgs<T>, hipStream_t, Tuning);               \
  template int op_blocks<T>(int, int, OpArgs<T> &, const Tuning &);                           \
  template int op_key<T>(int, int, const OpArgs<T> &);                                        \
  template hipError_t launch_op<T>(int, int, OpArgs<T>, const Tuning &, hipStream_t);         \
  template hipError_t launch_op_multi<T>(int, int, const OpArgs<T> *, const int *, int, int, hipStream_t); \
  template hipError_t launch_solve_contig<T>(SolveArgs<T>, hipStream_t);                      \
  template hipError_t launch_solve_strided<T>(StridedArgs<T>, int, hipStream_t);              \
  template hipError_t launch_apply<T>(StridedArgs<T>, hipStream_t);                           \
  template hipError_t launch_prolong_mass<T>(ProlongArgs<T>, int, hipStream_t);               \
  template hipError_t launch_copy_box<T>(CopyArgs<T>, hipStream_t);                           \
  template hipError_t launch_adaptive_estimate<T>(EstimateArgs<T>, int, hipStream_t);         \
  template hipError_t launch_pad_edge<T>(PadArgs<T>, hipStream_t);                             \
  template hipError_t launch_quantize<T>(const T *, int32_t *, QuantArgs, bool, hipStream_t); \
  template hipError_t launch_dequantize<T>(const int32_t *, T *, QuantArgs, hipStream_t);

MGX_INSTANTIATE(float)
MGX_INSTANTIATE(double)

}  // namespace mgx
