/*
 * mgx — MGARD+ multilevel decomposition, recomposition and level-wise
 * quantization on AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The method is that of "MGARD+: Optimizing Multilevel Methods for
 * Error-bounded Scientific Data Reduction" (arXiv 2010.05872).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - Arrays are C order with shape dims[0] x ... x dims[ndim-1]; the last axis
 *   is contiguous.  1 <= ndim <= 3, and ndim = 4 (four-axis fields such as
 *   the QMCPACK data of Sec. 6, Table 2) where an entry point says so.  Every
 *   dims[k] must be 2^m + 1 with 1 <= m <= 13 (3 <= n <= 8193); a 4-D field
 *   has fewer than 2^32 nodes.  Every call that quantizes or dequantizes
 *   (mgx_quantize, mgx_dequantize, their _levels forms, the fused calls, the
 *   batched calls with labels, mgx_label_entropy) indexes the field with 32
 *   bits and returns MGX_ERR_SHAPE for 2^32 nodes or more, whatever ndim.
 * - Four-axis fields: mgx_num_levels, mgx_workspace_size, mgx_decompose,
 *   mgx_recompose, mgx_recompose_to, mgx_quantize, mgx_dequantize,
 *   mgx_quantize_levels, mgx_dequantize_levels, mgx_decompose_quantize,
 *   mgx_dequantize_recompose, mgx_label_entropy,
 *   mgx_label_entropy_workspace_size, mgx_linf_constant, mgx_level_tolerances
 *   (kappa = 4), mgx_dyadic_dims, mgx_pad and mgx_crop accept ndim = 4; every
 *   other entry point returns MGX_ERR_SHAPE for it.  The layouts, the level-centric order and the
 *   tolerance schedule are those of 1-D to 3-D fields with four axes.
 * - The level count L = min_k m_k - 1: all axes coarsen together and the
 *   coarsest grid N_0 has 3 nodes on the shortest axis.  Level l keeps every
 *   2^(L-l)-th node of the input grid N_L (Sec. 2).
 * - coords is NULL or an array of ndim host pointers; coords[k] is NULL
 *   (meaning coordinates 0, 1, ..., dims[k]-1) or dims[k] finite, strictly
 *   increasing doubles.  Coordinates are copied into a cached plan; the
 *   caller may free them after the call returns.
 * - stop_level l~ in [0, L]: levels L ... l~+1 are decomposed and Q_{l~} u is
 *   kept (the stop level of Algorithm 1).
 * - Device pointers (u, u_mc, labels, workspace) are caller-owned device
 *   memory on the current HIP device; the library never frees them.  They
 *   must be aligned to their element size.
 * - Every call validates its arguments on the host before any launch.  A
 *   non-MGX_OK status means nothing was enqueued.  Launches are asynchronous
 *   on `stream`; errors reported by the HIP runtime at launch time become
 *   MGX_ERR_HIP.  No call throws across the ABI.
 * - The multilevel coefficients u_mc use the level-centric layout of Sec. 5.1:
 *   along every axis, at every level from the finest down, the nodal (even)
 *   indices of the level are moved to the front of the level's box and the
 *   coefficient (odd) indices follow, both in increasing order.  So the box
 *   [0, n_k^(l)) on every axis holds level l, its corner box
 *   [0, n_k^(l-1)) holds level l-1, and the box of the stop level holds
 *   Q_{l~} u in natural order.  u_mc has the same shape as u.
 * - Calls that use the same workspace must not overlap; calls on different
 *   streams with distinct workspaces may run concurrently.
 */
#ifndef MGX_H
#define MGX_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The *_ENUM_MAX members only widen each enum to every non-negative int, so
 * that a C caller's out-of-range value is a value of the type the library
 * (written in C++) can test and reject; they are never valid arguments. */
typedef enum { MGX_F32 = 0, MGX_F64 = 1, MGX_DTYPE_ENUM_MAX = 0x7fffffff } mgx_dtype;

typedef enum {
  MGX_OK = 0,
  MGX_ERR_ARG = 1,       /* null pointer, in/out aliasing, bad enum value      */
  MGX_ERR_SHAPE = 2,     /* ndim not in [1,3] (or 4 where supported), or some dims[k] != 2^m+1, 1<=m<=13 */
  MGX_ERR_COORDS = 3,    /* non-finite or not strictly increasing coordinates  */
  MGX_ERR_LEVEL = 4,     /* stop_level outside [0, L]                          */
  MGX_ERR_TOL = 5,       /* tolerance not positive and finite, or 0 < C < 1    */
  MGX_ERR_RANGE = 6,     /* a quantization label overflowed int32 or a
                            coefficient was not finite (quantize with stats)    */
  MGX_ERR_WORKSPACE = 7, /* workspace NULL or smaller than mgx_workspace_size  */
  MGX_ERR_HIP = 8,       /* the HIP runtime reported an error                  */
  MGX_STATUS_ENUM_MAX = 0x7fffffff
} mgx_status;

#define MGX_MAX_LEVELS 16

/* Per-call quantization statistics (filled by mgx_quantize when requested).
 * Entry i of max_abs_label belongs to level first_level + i; labels of
 * out-of-range coefficients are excluded from it. */
typedef struct {
  int32_t first_level;                   /* the stop level l~                   */
  int32_t num_levels;                    /* L + 1 - l~                          */
  int32_t max_abs_label[MGX_MAX_LEVELS]; /* max |label| per level              */
  int64_t n_overflow;                    /* finite |c/q_l| >= 2^31 - 1         */
  int64_t n_nonfinite;                   /* c/q_l not finite (NaN or Inf input) */
} mgx_quant_stats;

/* Human-readable name of a status code (static storage). */
const char *mgx_status_string(mgx_status s);

/* Finest level index L for this shape, or -MGX_ERR_SHAPE. */
int mgx_num_levels(int ndim, const int64_t *dims);

/* Workspace bytes needed by mgx_decompose / mgx_recompose for this shape,
 * dtype and stop level (0 on invalid arguments).  About 0.3 N element sizes:
 * two compact coarse boxes for the nodal values and one coarse load-vector
 * box. */
size_t mgx_workspace_size(mgx_dtype dtype, int ndim, const int64_t *dims, int stop_level);

/* Multilevel decomposition (Sec. 2, decomposition steps 1-6, with the
 * level-centric output layout of Sec. 5.1):
 * for l = L ... l~+1, coefficients u_mc[N*_l] = ((I - Pi_{l-1}) Q_l u)(x),
 * then Q_{l-1} u = Pi_{l-1} Q_l u + Q_{l-1}(I - Pi_{l-1}) Q_l u, where the
 * correction is the L2 projection of the multilevel component (mass matrix
 * apply, restriction, tridiagonal solve per axis).
 *   u        in:  device, dims, dtype, natural order.  Not modified.
 *   u_mc     out: device, dims, dtype, level-centric layout.  Must not
 *                 overlap u.
 *   workspace, workspace_bytes: device scratch of at least
 *                 mgx_workspace_size(...) bytes, contents undefined after.
 * Errors: MGX_ERR_ARG, _SHAPE, _COORDS, _LEVEL, _WORKSPACE, _HIP. */
mgx_status mgx_decompose(const void *u, void *u_mc, mgx_dtype dtype, int ndim,
                         const int64_t *dims, const double *const *coords, int stop_level,
                         void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Multilevel recomposition (Sec. 2, recomposition steps 1-5): the exact
 * inverse of mgx_decompose.  For l = l~+1 ... L: the correction computed
 * from the level-l coefficients is subtracted from Q_{l-1} u, giving
 * Pi_{l-1} Q_l u on N_{l-1}, and the interpolant is added back to the
 * coefficients on N*_l.
 *   u_mc     in:  device, level-centric layout.  Not modified.
 *   u        out: device, natural order.  Must not overlap u_mc.
 * Errors as mgx_decompose. */
mgx_status mgx_recompose(const void *u_mc, void *u, mgx_dtype dtype, int ndim,
                         const int64_t *dims, const double *const *coords, int stop_level,
                         void *workspace, size_t workspace_bytes, hipStream_t stream);

/* L2 variant of level-wise quantization (Sec. 4.1, the cost-optimal bin
 * widths under the L2 error budget): tau_l = tol_l2 / sqrt(c_l2 h_l^d #N_L)
 * for l = stop_level .. L (tau_out[l - stop_level], host), so that
 * sum_l #N*_l h_l^d tau_l^2 = tol_l2^2 / c_l2.  h_l^d is the level's cell
 * volume (extent / intervals on every real axis).  c_l2 <= 0 takes
 * mgx_l2_constant.  Errors: MGX_ERR_TOL (tol_l2 not positive and finite,
 * c_l2 not finite), _LEVEL, _SHAPE, _COORDS. */
mgx_status mgx_level_tolerances_l2(int ndim, const int64_t *dims, const double *const *coords, double tol_l2,
                                   int stop_level, double c_l2, double *tau_out);

/* Level-wise quantization with caller-given tolerances tau[0 .. L-stop]
 * (host; level stop_level + i uses tau[i], bin width 2 tau[i]), e.g. from
 * mgx_level_tolerances_l2; otherwise as mgx_quantize / mgx_dequantize.
 * MGX_ERR_TOL if some tau[i] is not positive and finite. */
mgx_status mgx_quantize_levels(const void *u_mc, int32_t *labels, mgx_dtype dtype, int ndim, const int64_t *dims,
                               const double *const *coords, int stop_level, const double *tau,
                               mgx_quant_stats *stats, hipStream_t stream);
mgx_status mgx_dequantize_levels(const int32_t *labels, void *u_mc, mgx_dtype dtype, int ndim, const int64_t *dims,
                                 const double *const *coords, int stop_level, const double *tau,
                                 hipStream_t stream);

/* Shannon entropy of the labels of each level, in bits per label (Sec. 4.1:
 * the estimated cost of storing the labels): bits_out[l - stop_level] =
 * -sum_k p_k log2 p_k over the distinct labels k of level l (the stop
 * level's whole box counts as one level), host, L + 1 - stop_level entries.
 * labels: device, level-centric layout of that stop level.  The counts come
 * from one histogram pass when the levels' label ranges (2 max|label| + 1
 * each) add up to at most 2^26; wider ranges are counted by a radix sort of
 * (level, label) keys.  Workspace: mgx_label_entropy_workspace_size bytes
 * (enough for either: about 20 bytes per label, at least 292 MiB), must not
 * overlap labels.  Synchronizes `stream`.
 * Errors: MGX_ERR_ARG, _SHAPE, _LEVEL, _WORKSPACE, _HIP. */
mgx_status mgx_label_entropy(const int32_t *labels, int ndim, const int64_t *dims, int stop_level, double *bits_out,
                             void *workspace, size_t workspace_bytes, hipStream_t stream);
size_t mgx_label_entropy_workspace_size(int ndim, const int64_t *dims, int stop_level);

/* mgx_label_entropy with the statistics of the quantizing call that wrote
 * the labels (stats: host, as returned by mgx_quantize, mgx_quantize_levels
 * or mgx_decompose_quantize with the same shape and stop level): its per-level
 * max |label| sets the histogram's key ranges, so the labels are read once
 * instead of twice.  Statistics of another stop level, or that count
 * out-of-range labels, are not used (the call then finds the maxima itself);
 * a label beyond its level's stated maximum is detected and the call counts
 * again with the maxima found on the labels, so wrong statistics cost time,
 * never correctness.  Same results, workspace and errors as
 * mgx_label_entropy (MGX_ERR_ARG for a null stats). */
mgx_status mgx_label_entropy_bounded(const int32_t *labels, int ndim, const int64_t *dims, int stop_level,
                                     const mgx_quant_stats *stats, double *bits_out, void *workspace,
                                     size_t workspace_bytes, hipStream_t stream);

/* Non-dyadic sizes (the dummy nodes of Sec. 6.2.2): an axis of n nodes is
 * padded to the next 2^m + 1 >= n (m >= 1) with dummy nodes after the last
 * real node, each carrying the value of the nearest real node; the padded
 * field goes through the dyadic path (coordinates, if any, continued with
 * the last spacing by the caller) and the result is cropped back.  The L-inf
 * bound then holds on every real node.
 *   mgx_dyadic_dims  padded_out: host, ndim entries.  MGX_ERR_SHAPE if some
 *                    n < 2.
 *   mgx_pad          u (device, dims) -> u_pad (device, padded dims).
 *   mgx_crop         u_pad (device, padded dims) -> u (device, dims).
 * u and u_pad must not overlap.  Errors: MGX_ERR_ARG, MGX_ERR_SHAPE,
 * MGX_ERR_HIP. */
mgx_status mgx_dyadic_dims(int ndim, const int64_t *dims, int64_t *padded_out);
mgx_status mgx_pad(const void *u, void *u_pad, mgx_dtype dtype, int ndim, const int64_t *dims,
                   hipStream_t stream);
mgx_status mgx_crop(const void *u_pad, void *u, mgx_dtype dtype, int ndim, const int64_t *dims,
                    hipStream_t stream);

/* Adaptive decomposition (Sec. 4.2 "Adaptive decomposition", Alg. 1 lines
 * 1-16), 3-D fields only.  Before decomposing level l (from L down), the
 * Lorenzo predictor and the multilinear interpolation are compared on
 * sampled 3^3 blocks of Q_l u (the level-l cells a with a % 4 == 1 on every
 * axis, one block in four per axis): E = sum over their coefficient nodes of
 * |u - prediction| plus the penalty factors of Sec. 4.2 (Lorenzo 1.22,
 * interpolation edge 0.369, plane 0.259, cube 0.182) times tau0, the
 * tolerance of the coarsest level when the decomposition stops at l
 * (mgx_level_tolerances with stop level l).  The decomposition stops at the
 * first level whose Lorenzo estimate is the lower one, else at level 0.
 *   u, u_mc       as mgx_decompose; u_mc holds the decomposition to the
 *                 chosen stop level (the level-centric layout of that stop).
 *   tol_linf, c_linf  as mgx_quantize.
 *   stop_level_out    out: host, the chosen stop level.
 *   workspace     mgx_workspace_size(dtype, ..., 0) bytes.
 * The decisions are taken on the device: every level's estimate, decision
 * and kernels are enqueued at once, the levels below the stop doing nothing,
 * and `stream` is synchronized once, at the end, to read the stop level.
 * Errors: MGX_ERR_SHAPE for fewer than three real axes; otherwise as
 * mgx_decompose and mgx_quantize (MGX_ERR_TOL). */
mgx_status mgx_decompose_adaptive(const void *u, void *u_mc, mgx_dtype dtype, int ndim, const int64_t *dims,
                                  const double *const *coords, double tol_linf, double c_linf,
                                  int *stop_level_out, void *workspace, size_t workspace_bytes,
                                  hipStream_t stream);

/* The estimate alone, on a level box v (device, natural order, the level-
 * `level` grid of a field of shape dims, holding Q_level u): sums_out[0] =
 * sum |u - Lorenzo prediction|, sums_out[1] = sum |u - multilinear
 * interpolant| over the sampled coefficient nodes (FP64), counts_out[0..2] =
 * sampled edge, plane and cube nodes (host arrays).  Workspace:
 * mgx_adaptive_workspace_size bytes.  Synchronizes `stream`. */
mgx_status mgx_adaptive_estimate(const void *v, mgx_dtype dtype, int ndim, const int64_t *dims,
                                 const double *const *coords, int level, double *sums_out, int64_t *counts_out,
                                 void *workspace, size_t workspace_bytes, hipStream_t stream);
size_t mgx_adaptive_workspace_size(int ndim, const int64_t *dims);

/* Progressive recomposition: the recomposition stopped after level
 * target_level, giving Q_target u, the coarse representation of the field
 * on the level-target grid (the partial reconstruction that data refactoring
 * offers, Sec. 1; the analysis on decomposed representations, Sec. 6.2.2).
 *   u_mc          in:  device, level-centric layout of a decomposition to
 *                 stop_level.  Not modified.
 *   u_t           out: device, the level-target box in natural order, node
 *                 counts (n_k - 1) / 2^(L - target_level) + 1 per real axis
 *                 (dims unchanged on padded axes).  Must not overlap u_mc or
 *                 the workspace.
 *   target_level  stop_level <= target_level <= L; L gives mgx_recompose's
 *                 result, stop_level a copy of the stop level's box.
 * Workspace as mgx_recompose (mgx_workspace_size with stop_level).
 * Errors: MGX_ERR_LEVEL for a target outside [stop_level, L]; otherwise as
 * mgx_recompose. */
mgx_status mgx_recompose_to(const void *u_mc, void *u_t, mgx_dtype dtype, int ndim, const int64_t *dims,
                            const double *const *coords, int stop_level, int target_level, void *workspace,
                            size_t workspace_bytes, hipStream_t stream);

/* mgx_decompose followed by mgx_quantize in one call, with the same results
 * (Sec. 4.1 quantization of the Sec. 2 decomposition, Alg. 1's quantize
 * step): every kernel that produces coefficients of a level also writes
 * their labels, so no separate pass over u_mc is made.
 *   u_mc     out: device, level-centric layout, or NULL: then only labels
 *            are written (the stop level's box goes through the workspace).
 *   labels   out: device, int32, same shape; must not overlap u, u_mc or
 *            the workspace.  A coefficient whose |c/q_l| >= 2^31-1 or that
 *            is not finite gets INT32_MIN.
 *   stats    NULL: fully asynchronous; out-of-range coefficients are not
 *            reported.  Non-NULL (host): the level kernels also reduce the
 *            per-level max |label| (one atomic per wave) and count
 *            out-of-range coefficients (on their rare exact-division path),
 *            the call waits for the stream, fills *stats as mgx_quantize does
 *            and returns MGX_ERR_RANGE when some coefficient was out of
 *            range.  Four-axis fields take the per-level maxima in one more
 *            pass over the labels.
 * Errors as mgx_decompose and mgx_quantize (MGX_ERR_TOL, MGX_ERR_RANGE). */
mgx_status mgx_decompose_quantize(const void *u, void *u_mc, int32_t *labels, mgx_dtype dtype, int ndim,
                                  const int64_t *dims, const double *const *coords, double tol_linf,
                                  int stop_level, double c_linf, void *workspace, size_t workspace_bytes,
                                  mgx_quant_stats *stats, hipStream_t stream);

/* mgx_dequantize(labels) followed by mgx_recompose into u, with the same
 * results.
 *   u_mc     NULL: the recomposition's kernels read each coefficient as its
 *            label times the level's bin width (no u_mc pass); or device,
 *            dtype: the dequantized coefficients are written there first and
 *            recomposed from.
 *   labels   in: device, int32; must not overlap u, u_mc or the workspace.
 * Errors as mgx_recompose and mgx_dequantize. */
mgx_status mgx_dequantize_recompose(const int32_t *labels, void *u_mc, void *u, mgx_dtype dtype, int ndim,
                                    const int64_t *dims, const double *const *coords, double tol_linf,
                                    int stop_level, double c_linf, void *workspace, size_t workspace_bytes,
                                    hipStream_t stream);

/* ---- Decomposition without allocation ----
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * mgx_decompose with the same results (the same kernels), but its level
 * tables and its workspace live in a static device array of the library,
 * MGX_NOALLOC_SCRATCH_BYTES per device, held from the library's load until
 * the process ends.  The call allocates no device memory: the tables (a few
 * hundred KB at most) are copied from host memory into the array on `stream`
 * (hipMemcpyAsync from pageable memory, which may wait for the copy), then
 * the level kernels run with the array as their workspace.  No part of the
 * array needs to start at zero: every call writes what it reads.  Every
 * call on one device shares that device's array: calls that overlap on one
 * device (other streams, other host threads) race; calls in order on one
 * stream do not.  Tracing (mgx_trace_enable) does not record these calls.
 *   u, u_mc, dtype, ndim, dims, coords, stop_level: as mgx_decompose.
 * Errors: MGX_ERR_WORKSPACE when the tables (256-byte aligned) plus
 * mgx_workspace_size(...) exceed MGX_NOALLOC_SCRATCH_BYTES (e.g. 257^3 fp32
 * fits, 513^3 fp32 does not); MGX_ERR_SHAPE for ndim = 4; otherwise those of
 * mgx_decompose. */
#define MGX_NOALLOC_SCRATCH_BYTES (32u << 20)
mgx_status mgx_decompose_noalloc(const void *u, void *u_mc, mgx_dtype dtype, int ndim, const int64_t *dims,
                                 const double *const *coords, int stop_level, hipStream_t stream);

/* ---- Adjoints (project extension, not in the paper) ----
 * The transposes of the linear maps mgx_decompose (D) and mgx_recompose
 * (R = D^{-1}): for all x, y, <D x, y> = <x, D^T y>.  They let gradients of
 * a loss on a reconstructed field flow back to the coefficients and the
 * input.  Per level they run the transposed steps of Sec. 2 in reverse
 * order: the coarse solve, the transposed load-vector stencil (M P per
 * axis, the transpose of the fused R M of Sec. 5.2) and the restriction R.
 * Workspace: at least mgx_adjoint_workspace_size(...) bytes (the forward
 * workspace plus one more coarse load-vector box). */
size_t mgx_adjoint_workspace_size(mgx_dtype dtype, int ndim, const int64_t *dims, int stop_level);

/* g_u = D^T g_mc.
 *   g_mc     in:  device, dims, dtype, level-centric layout (the layout of
 *                 mgx_decompose's output).  Not modified.
 *   g_u      out: device, natural order.  Must not overlap g_mc.
 * Errors as mgx_decompose (MGX_ERR_WORKSPACE against the adjoint size). */
mgx_status mgx_decompose_adjoint(const void *g_mc, void *g_u, mgx_dtype dtype, int ndim,
                                 const int64_t *dims, const double *const *coords, int stop_level,
                                 void *workspace, size_t workspace_bytes, hipStream_t stream);

/* g_mc = R^T g_u.
 *   g_u      in:  device, natural order.  Not modified.
 *   g_mc     out: device, level-centric layout.  Must not overlap g_u.
 * Errors as mgx_decompose_adjoint. */
mgx_status mgx_recompose_adjoint(const void *g_u, void *g_mc, mgx_dtype dtype, int ndim,
                                 const int64_t *dims, const double *const *coords, int stop_level,
                                 void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ---- Batched fields (project extension, not in the paper) ----
 * Many independent fields of uneven shapes in one graph launch.  The
 * library records every field's launch sequence (the steps of
 * mgx_decompose / mgx_recompose, and the quantizer when labels are given),
 * runs the same step of all fields as one multi-field kernel launch (one per
 * kernel instance), captures the whole sequence into a HIP graph once per
 * batch (keyed by the field list and the workspace pointer) and replays it.
 * The first call of a batch also picks the launch shape of the tiled
 * stencil kernels by timing candidate graphs (autotuning; it synchronizes
 * the stream), unless mgx_batch_set_autotune(0).  The paper processes each
 * field separately (one field per core, Sec. 6). */
typedef struct {
  const void *in;            /* decompose: u; recompose: u_mc (unused when labels is set)   */
  void *out;                 /* decompose: u_mc; recompose: u                               */
  mgx_dtype dtype;
  int ndim;
  int64_t dims[3];           /* C order, first ndim entries used                            */
  const double *coords[3];   /* per axis, NULL: 0 .. n-1                                    */
  int stop_level;
  double tol_linf;           /* with labels: the absolute L-infinity tolerance              */
  double c_linf;             /* <= 0: library default                                       */
  int32_t *labels;           /* decompose: labels out (NULL: no quantization);
                                recompose: labels in (NULL: recompose from in)              */
  void *coef;                /* recompose from labels: NULL, the level kernels read the
                                labels; or a device buffer (dims, dtype) that receives the
                                dequantized coefficients first                             */
  mgx_quant_stats *stats;    /* decompose with labels: NULL, or host statistics of this
                                field as mgx_decompose_quantize fills them (the batched call
                                then waits for the stream); unused otherwise               */
} mgx_field;

typedef struct {
  int launches;              /* kernel launches in the batch's graph                        */
  int target_blocks;         /* chosen launch shape of the stencil kernels                  */
  int min_zchunk;
  double tuned_ms;           /* time of the chosen graph during tuning (0: not tuned)       */
  int tune_source;           /* 0: default shape, 1: timed by this process, 2: read from the
                                tuning cache file (MGX_TUNE_CACHE)                         */
} mgx_batch_info;

/* Workspace bytes for mgx_decompose_batched / mgx_recompose_batched (the
 * sum of the fields' mgx_workspace_size, each 256-byte aligned; 0 on
 * invalid fields). */
size_t mgx_batch_workspace_size(int nfields, const mgx_field *fields);

/* Every field as mgx_decompose, with labels != NULL as
 * mgx_decompose_quantize (labels written by the level kernels; the same
 * labels as mgx_quantize).  A field with stats != NULL gets the statistics
 * of mgx_decompose_quantize: the call then waits for the stream and returns
 * MGX_ERR_RANGE when some such field had an out-of-range coefficient (every
 * field's stats are filled).  Outputs and labels of different fields must
 * not overlap.  Errors: those of the single-field calls (the first failing
 * field decides), MGX_ERR_WORKSPACE, MGX_ERR_HIP, MGX_ERR_RANGE. */
mgx_status mgx_decompose_batched(int nfields, const mgx_field *fields, void *workspace,
                                 size_t workspace_bytes, hipStream_t stream);

/* Every field as mgx_recompose; with labels != NULL as
 * mgx_dequantize_recompose: coef NULL reads the labels in the level kernels,
 * otherwise the labels are dequantized into coef first and recomposed from
 * it (the same results either way). */
mgx_status mgx_recompose_batched(int nfields, const mgx_field *fields, void *workspace,
                                 size_t workspace_bytes, hipStream_t stream);

/* Frees what the library caches across calls: the level plans of every
 * (shape, coordinates) seen so far, with their device tables, and the
 * captured graphs of batches.  Those caches otherwise grow with the number
 * of distinct shapes, coordinate sets and batches a process uses, until it
 * ends.  Synchronizes every device that holds cached memory.  No other call
 * of the library may run, on any thread, while this one does; later calls
 * rebuild what they need.  The statistics buffer and the static array of
 * mgx_decompose_noalloc are not affected.  Errors: MGX_ERR_HIP. */
mgx_status mgx_release_cached(void);

/* Autotuning of batches on first use: 1 (default) or 0 (default shape).
 * With the environment variable MGX_TUNE_CACHE set to a file path, tuned
 * shapes persist across processes: a batch met for the first time is
 * looked up there by a signature of its fields' dtypes, dims, stop levels,
 * label / coefficient / statistics use and coordinate values (not their
 * addresses) and built with the stored shape without timing; each shape
 * timed is appended as one text line.  Read at every first meeting of a
 * batch; an unreadable or unwritable file is ignored. */
mgx_status mgx_batch_set_autotune(int on);

/* Shape of the most recent batched call of this thread. */
mgx_status mgx_batch_last_info(mgx_batch_info *info);

/* Level-wise quantization (Sec. 4.1, eq. (LinfTau); Algorithm 1, quantize
 * step).  tau_l~ = (1-kappa)/(1-kappa^(L+1-l~)) * tol_linf / C and
 * tau_l = kappa tau_{l-1} with kappa = sqrt(2^d), all in FP64 in that
 * operation order; q_l = 2 tau_l.  Every coefficient c of level l (the
 * level-l~ box counts as level l~) becomes label = rint(c / q_l), computed
 * in FP64 with a correctly rounded division and ties to even, so that
 * |c - label q_l| <= tau_l.
 *   u_mc     in:  device, level-centric layout.
 *   labels   out: device int32, dims.  A coefficient whose |c/q_l| >= 2^31-1
 *                 or is not finite gets INT32_MIN.
 *   tol_linf absolute L-infinity tolerance tau > 0.
 *   c_linf   the constant C_{L^inf} (>= 1), or <= 0 for the library default
 *            mgx_linf_constant(...).
 *   stats    NULL: fully asynchronous, no reductions.  Non-NULL: the call
 *            also reduces per-level max |label| and the overflow/non-finite
 *            counts, waits for the stream, fills *stats and returns
 *            MGX_ERR_RANGE when any label overflowed.
 * Errors: MGX_ERR_ARG, _SHAPE, _COORDS, _LEVEL, _TOL, _RANGE, _HIP. */
mgx_status mgx_quantize(const void *u_mc, int32_t *labels, mgx_dtype dtype, int ndim,
                        const int64_t *dims, const double *const *coords, double tol_linf,
                        int stop_level, double c_linf, mgx_quant_stats *stats,
                        hipStream_t stream);

/* Dequantization: c~ = (double)label * q_l, rounded to dtype (nearest).
 *   labels   in:  device int32, level-centric positions.
 *   u_mc     out: device, dtype.
 * Errors: MGX_ERR_ARG, _SHAPE, _COORDS, _LEVEL, _TOL, _HIP. */
mgx_status mgx_dequantize(const int32_t *labels, void *u_mc, mgx_dtype dtype, int ndim,
                          const int64_t *dims, const double *const *coords, double tol_linf,
                          int stop_level, double c_linf, hipStream_t stream);

/* The default C_{L^inf} (Sec. 4.1, eq. (LInfNormEstimator)).  The paper cites
 * its value without printing it; the library uses the rigorous bound
 * max(1, max over levels l~ < l <= L of 1 + prod_k ||Mc_k^-1 R_k M_k||_inf),
 * the per-level amplification of a coefficient error through recomposition.
 * Host, synchronous.  Returns a negative value on invalid arguments. */
double mgx_linf_constant(int ndim, const int64_t *dims, const double *const *coords,
                         int stop_level);

/* The default C_{L^2} of the L2 estimator (Sec. 4.1, eq. (L2NormEstimator)),
 * which the paper cites without printing.  The quantization error of level l
 * recomposes to (I - Q_{l-1}) e_l (e_l the level-l interpolant of the
 * level's coefficient errors; e_l itself on the stop box); these pieces are
 * L2-orthogonal across levels and I - Q_{l-1} does not increase the norm, so
 * ||u - u~||^2 <= sum_l lambda_max(M_l) sum |delta_l|^2.  Bounding
 * lambda_max(M_l) by the product of the axes' largest mass-matrix row sums,
 * max_j (h_{j-1} + h_j) / 2, gives C = max over levels l~ <= l <= L of that
 * product over h_l^d (the cell volume of mgx_level_tolerances_l2): exactly 1
 * on uniform grids.  Host, synchronous; negative on invalid arguments. */
double mgx_l2_constant(int ndim, const int64_t *dims, const double *const *coords, int stop_level);

/* tau_out[0 .. L-l~] = tolerances of levels l~ ... L as used by
 * mgx_quantize.  Host, synchronous. */
mgx_status mgx_level_tolerances(int ndim, const int64_t *dims, const double *const *coords,
                                double tol_linf, int stop_level, double c_linf,
                                double *tau_out);

/* Kernel tracing.  While enabled, every kernel this library launches is
 * bracketed by two HIP events recorded on the stream it is launched on, and
 * mgx_trace_read reports the summed durations per (kernel, level).  Meant
 * for measurement: the events cost a few microseconds per launch.  Tracing
 * state is process-wide; enable/read are not meant to race with launches
 * from other host threads. */
typedef struct {
  char name[40];     /* e.g. "load_vector_dec", "solve_contig"             */
  int32_t level;     /* level l being decomposed/recomposed, -1 if none  */
  int32_t count;     /* launches recorded                               */
  double total_ms;   /* summed event-to-event time                      */
} mgx_kernel_time;

/* on != 0 starts recording (and clears earlier records); 0 stops. */
mgx_status mgx_trace_enable(int on);
/* Waits for the recorded events, writes up to max aggregated entries to
 * out (host), clears the records and returns the number of entries, or -1
 * on a HIP error. */
int mgx_trace_read(mgx_kernel_time *out, int max);

#ifdef __cplusplus
}
#endif
#endif /* MGX_H */
