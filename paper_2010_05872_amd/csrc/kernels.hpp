// Kernel argument blocks and host launchers (internal to libmgx).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mgx {

constexpr int kMaxLevelsK = 16;

// What the last solve of a level does with the solution y.
constexpr int kSolveInPlace = 0;  // y replaces the load vector
constexpr int kSolveApply = 1;    // out = in + sign * y (recomposition)
constexpr int kSolveStore = 2;    // out = y (decomposition: y = Q_{l-1} u)

// Tables of one axis at the level being processed (see plan.hpp).
template <typename T>
struct AxisTab {
  const T *wl, *wr;               // interpolation weights at odd fine nodes [m]
  const T *w5;                    // load-vector stencil, 5 per coarse node [5c]
  const T *mult, *invd, *qsup;    // Thomas factors of the coarse mass matrix [c]
  const T *multb, *invdb, *qsub;  // the same, eliminating from the last row [c]
  const T *mid;                   // middle-row factors of the two-ended solve [3]
  int m, c;                       // fine and coarse node counts
};

template <typename T>
struct StencilArgs {
  AxisTab<T> ax[3];
  const T *V;                 // level-l box (decompose), compact
  int64_t vp0, vp1;           // its plane and row pitches
  T *umc_w;                   // u_mc (decompose writes coefficients; null: load vector only)
  const T *umc_r;             // u_mc (recompose reads coefficients)
  int64_t up0, up1;           // u_mc pitches (finest grid)
  T *F;                       // load vector out, coarse box
  int64_t fp0, fp1;
  int32_t *lab_w;             // decompose: also write the quantization labels (u_mc's layout)
  const int32_t *lab_r;       // recompose: read labels instead of coefficients
  double qc;                  // bin width q_l of the level's coefficients (labels)
  float rqc;                  // 1/q_l rounded to FP32 (NaN outside FP32's normal range)
  // decompose with labels: counts of coefficients whose label is INT32_MIN,
  // [0] finite |c/q| >= 2^31 - 1, [1] c/q not finite (null: not counted)
  unsigned long long *rng;
  int *smax;                  // decompose with labels: the level's max |label| (atomicMax; null: not taken)
  const int *gate;            // nullable: the launch does nothing while *gate == 0 (adaptive decomposition)
  int ntx, nty, nzc, tz;      // set by the launcher
};

template <typename T>
struct InterpArgs {
  AxisTab<T> ax[3];
  const T *nodal;             // corrected nodal values, coarse box
  int64_t np0, np1;
  const T *umc;               // coefficients (level-centric)
  int64_t up0, up1;
  T *out;                     // level-l box out
  int64_t op0, op1;
  const int32_t *lab;         // non-null: read labels (times qc) instead of coefficients
  double qc;
  int ntx, nty, nzc, tz;
};

template <typename T>
struct SolveArgs {            // contiguous-axis solve, in place on F rows
  T *F;
  int64_t nlines, pitch;
  int c;
  const T *mult, *invd, *qsup;
  const int *gate;            // as StencilArgs::gate
};

// Adaptive decomposition estimate (3-D): one thread per sampled 3^3 block
// (level-l cells a with a % 4 == 1 per axis) of the level-l box V.
template <typename T>
struct EstimateArgs {
  const T *V;
  int64_t vp0, vp1;
  int nb0, nb1, nb2;            // sampled cells per axis
  const double *wl[3], *wr[3];  // FP64 interpolation weights of level l, by level index
  double *partial;              // per workgroup: sum |u - Lorenzo|, sum |u - interpolant|
  const int *gate;              // as StencilArgs::gate
};

// The estimate's decision: the partial sums of one estimate launch added up
// (fixed order), and the adaptive decomposition's state updated on the device.
struct DecideArgs {
  const double *partial;        // [2 * nwg] from the estimate
  int nwg;
  double *sums;                 // nullable: the two totals out
  int *state;                   // nullable: [0] 1 while the decomposition goes on, [1] its stop level
  int level;                    // the level the estimate was taken on
  int first;                    // nonzero: the first decision (initialises the state, ignores [0])
  double pen_lor, pen_int;      // penalty terms added to the two sums before they are compared
};

template <typename T>
struct StridedArgs {          // strided-axis solve (optionally applying)
  T *F;
  int c;                      // line length
  int64_t sj;                 // element stride along the line
  int nx;                     // contiguous extent (threads)
  int64_t so;                 // stride between outer lines
  int nouter;
  const T *mult, *invd, *qsup;
  const T *multb, *invdb, *qsub, *mid;
  const T *in;                // apply: nodal in (index J*ij + o*io + x); unused by store
  int64_t ij, io;
  T *out;                     // apply: nodal out (index J*oj + o*oo + x)
  int64_t oj, oo;
  T sign;
  const int *gate;            // as StencilArgs::gate
};

// Adjoint: the transposed load-vector operator (M P) along every axis, from a
// coarse box y to the level-l box, combined with the level's other terms.
constexpr int kProlongRecAdj = 0;  // lc_out[x] = fine[x] - (MP)y at coefficient nodes
constexpr int kProlongDecAdj = 1;  // out[x] = (MP)y + (coef node ? lc_in[x] : -r[x/2])

template <typename T>
struct ProlongArgs {
  AxisTab<T> ax[3];           // w5 (the R M stencil), m, c
  const T *y;                 // coarse box
  int64_t yp0, yp1;
  const T *fine;              // recompose adjoint: level-l box in
  int64_t fp0, fp1;
  T *lc_out;                  // recompose adjoint: coefficient gradient out (level-centric)
  const T *lc_in;             // decompose adjoint: coefficient gradient in (level-centric)
  int64_t up0, up1;           // level-centric array pitches
  const T *r;                 // decompose adjoint: R of the coefficient gradient, coarse box
  int64_t rp0, rp1;
  T *out;                     // decompose adjoint: level-l box out
  int64_t op0, op1;
  int ntx, nty, nzc, tz;
};

template <typename T>
struct CopyArgs {             // strided copy of an n0 x n1 x n2 box
  const T *src;
  int64_t sp0, sp1;
  T *dst;
  int64_t dp0, dp1;
  int n0, n1, n2;
};

// Dummy-node padding of a non-dyadic box (n0 x n1 x n2) to a dyadic one
// (p0 x p1 x p2, every p_k >= n_k): each padded node takes the value of the
// nearest real node (index clamped to n_k - 1).
template <typename T>
struct PadArgs {
  const T *src;
  T *dst;
  int n0, n1, n2, p0, p1, p2;
};
template <typename T> hipError_t launch_pad_edge(PadArgs<T> a, hipStream_t st);

// The coarse tail of the hierarchy (every level box at most kTailBox nodes
// per axis) in one workgroup: all its levels in one launch instead of one
// latency-bound launch per step and level.
constexpr int kTailBox = 17;
constexpr int kTailMax = 6;  // levels of a tail (17 -> 3 takes 3 steps)

template <typename T>
struct TailAxis {
  const T *wl, *wr, *w5, *mult, *invd, *qsup;
  int m, c;
  // ceil(2^32 / m) and ceil(2^32 / c), 0 for 1: the tail's index splits
  // (q / m as the high half of q * mm, exact for q * m < 2^32)
  uint32_t mm, cm;
};
// ceil(2^32 / d) for the tail's divisions (d >= 1; 0 for d = 1)
inline uint32_t tail_magic(int64_t d) { return d > 1 ? (uint32_t)((((uint64_t)1 << 32) + d - 1) / d) : 0u; }

template <typename T>
struct TailArgs {
  TailAxis<T> ax[kTailMax][3];  // [i][k]: level lt - i, lt the tail's finest level
  int nlev;                      // levels lt .. lt - nlev + 1 are processed
  const T *src;                  // decompose: the level-lt box (Q_lt u)
  int64_t sp0, sp1;
  T *umc;                        // decompose: coefficients and stop box out
  const T *umc_r;                // recompose: coefficients and stop box in
  int64_t up0, up1;
  T *dst;                        // recompose: the level-lt box out
  int64_t dp0, dp1;
  int32_t *lab_w;                // decompose: also (umc null: only) write labels
  const int32_t *lab_r;          // recompose: read labels instead of coefficients
  double q[kTailMax + 1];        // bin widths: q[i] of level lt - i, q[nlev] of the stop box
  unsigned long long *rng;       // decompose: out-of-range counts as StencilArgs::rng (nullable)
  int *smax;                     // decompose: max |label| per level from the stop level up:
                                 // smax[nlev - i] of level lt - i, smax[0] of the stop box (nullable)
};

struct QuantArgs {
  int64_t n;                  // element count (< 2^32)
  int n1, n2;                 // padded dims 1 and 2
  uint64_t mag1, mag2;        // ceil(2^64 / n1), ceil(2^64 / n2): exact 32-bit division
  int off[3];                 // log2(n_k - 1) - L per axis (0 for padded axes)
  int first, nlev;            // levels first .. first+nlev-1
  int sel_lo, sel_hi;         // only elements of levels sel_lo .. sel_hi are read and written
  int box;                    // nonzero: visit only the corner box b0 x b1 x b2 of the array
  int b1, b2;
  int64_t bn;                 // b0 * b1 * b2
  uint64_t bmag1, bmag2;      // ceil(2^64 / b1), ceil(2^64 / b2)
  int box_compact;            // box mode: the coefficient side is a compact b0 x b1 x b2 buffer
  double q[kMaxLevelsK];      // bin width per level
  int *stats_max;             // [nlev] device
  // out-of-range counts, added to whenever they are set (nullable)
  unsigned long long *stats_ovf, *stats_nan;
};

// Launch shape of the tiled stencil kernels: the workgroups a launch aims
// for, and the fewest coarse planes one workgroup marches through on large
// levels (smaller levels take one coarse plane per workgroup).
#ifndef MGX_TUNE_TARGET
#define MGX_TUNE_TARGET 2048
#endif
#ifndef MGX_TUNE_MINZ
#define MGX_TUNE_MINZ 8
#endif
#ifndef MGX_TUNE_MIDZ
#define MGX_TUNE_MIDZ 8
#endif
struct Tuning {
  int target_blocks = MGX_TUNE_TARGET;
  int min_zchunk = MGX_TUNE_MINZ;  // levels of at least 2^24 coarse nodes
  int mid_zchunk = MGX_TUNE_MIDZ;  // levels of 2^20 .. 2^24 coarse nodes
};

template <typename T> hipError_t launch_load_vector(StencilArgs<T> a, bool dec, hipStream_t st, Tuning tn = {});
template <typename T> hipError_t launch_interp_add(InterpArgs<T> a, hipStream_t st, Tuning tn = {});
template <typename T> hipError_t launch_solve_contig(SolveArgs<T> a, hipStream_t st);
template <typename T> hipError_t launch_solve_strided(StridedArgs<T> a, int mode, hipStream_t st);
template <typename T> hipError_t launch_apply(StridedArgs<T> a, hipStream_t st);
template <typename T> hipError_t launch_prolong_mass(ProlongArgs<T> a, int mode, hipStream_t st);
template <typename T> hipError_t launch_copy_box(CopyArgs<T> a, hipStream_t st);
template <typename T>
hipError_t launch_quantize(const T *umc, int32_t *labels, QuantArgs a, bool stats, hipStream_t st);
template <typename T>
hipError_t launch_dequantize(const int32_t *labels, T *umc, QuantArgs a, hipStream_t st);

// ---- ops: one kernel launch of one field, and multi-field launches ----
enum OpKind {
  kOpLoadVecDec, kOpLoadVecRec, kOpSolveContig, kOpSolveStrided, kOpApply, kOpInterpAdd,
  kOpQuantize, kOpDequantize, kOpCopyBox, kOpTailDec, kOpTailRec
};

template <typename T>
struct QuantJob {
  const T *umc;
  int32_t *labels;
  QuantArgs a;
};
template <typename T>
struct DequantJob {
  const int32_t *labels;
  T *umc;
  QuantArgs a;
};

template <typename T>
union OpArgs {
  StencilArgs<T> st;
  SolveArgs<T> so;
  StridedArgs<T> sd;
  InterpArgs<T> ia;
  QuantJob<T> qj;
  DequantJob<T> dj;
  CopyArgs<T> cp;
  TailArgs<T> tl;
};

template <typename T> hipError_t launch_adaptive_estimate(EstimateArgs<T> a, int nblocks, hipStream_t st);
hipError_t launch_adaptive_decide(DecideArgs a, hipStream_t st);
constexpr int kEstimateThreads = 256;

// Workgroups of one op (fills the tile-grid fields of stencil ops); -1 when
// the shape is not launchable.
template <typename T> int op_blocks(int kind, int mode, OpArgs<T> &a, const Tuning &tn);
// Ops of one kind with equal key run the same kernel instance, so a single
// multi-field launch can take them all.
template <typename T> int op_key(int kind, int mode, const OpArgs<T> &a);
// One op on its own grid.
template <typename T> hipError_t launch_op(int kind, int mode, OpArgs<T> a, const Tuning &tn, hipStream_t st);
// n ops of equal (kind, key) in one launch: dargs[n] and dstart[n+1] (prefix
// sums of the ops' workgroup counts, dstart[n] = total) live in device memory.
template <typename T>
hipError_t launch_op_multi(int kind, int key, const OpArgs<T> *dargs, const int *dstart, int n, int total,
                           hipStream_t st);

}  // namespace mgx
