// C ABI of libmgx (include/mgx.h): argument validation, workspace layout and
// the per-level launch sequences of decomposition and recomposition.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "entropy.hpp"
#include "kernels.hpp"
#include "kernels4.hpp"
#include "mgx.h"
#include "placed.hpp"
#include "plan.hpp"

namespace mgx {
namespace {

size_t elem_size(mgx_dtype d) { return d == MGX_F64 ? 8 : 4; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int64_t round4(int64_t v) { return (v + 3) / 4 * 4; }

struct Layout {
  size_t offA = 0, offB = 0, offF = 0, offG = 0, offS = 0, offE = 0, total = 0;
  int lt = -1;  // finest level of the single-workgroup tail, -1: none
};

// Finest level whose box has at most kTailBox nodes on every axis (the
// tail runs levels lt .. stop+1 in one workgroup), or -1.
int tail_level(const int64_t n[3], const bool real[3], int L, int stop) {
  for (int l = L; l > stop; l--) {
    bool ok = true;
    for (int k = 0; k < 3; k++)
      if (real[k] && (n[k] - 1) / ((int64_t)1 << (L - l)) + 1 > kTailBox) ok = false;
    if (ok) return l;
  }
  return -1;
}

// Two compact coarse boxes (levels L-1 and L-2) for nodal values and one
// coarse box with padded rows for the load vector.
// The adjoints need one more load-vector sized box (G).
Layout layout(const int64_t n[3], const bool real[3], int L, int stop, size_t es, bool adjoint = false) {
  Layout w;
  if (stop >= L) return w;
  int64_t cA = 1, cB = 1, cF = 1;
  for (int k = 0; k < 3; k++) {
    int64_t a = real[k] ? (n[k] - 1) / 2 + 1 : 1;
    int64_t b = real[k] ? (n[k] - 1) / 4 + 1 : 1;
    cA *= a;
    cB *= b;
    cF *= (k == 2) ? round4(a) : a;
  }
  size_t off = 0;
  w.offA = off;
  off = align_up(off + (size_t)cA * es, 256);
  w.offB = off;
  if (L - stop >= 2) off = align_up(off + (size_t)cB * es, 256);
  w.offF = off;
  off = align_up(off + (size_t)cF * es, 256);
  w.offG = off;
  if (adjoint) off = align_up(off + (size_t)cF * es, 256);
  w.lt = tail_level(n, real, L, stop);
  // the stop box, compact (paths that work on labels without u_mc)
  int64_t cS = 1;
  for (int k = 0; k < 3; k++) cS *= real[k] ? (n[k] - 1) / ((int64_t)1 << (L - stop)) + 1 : 1;
  w.offS = off;
  off = align_up(off + (size_t)cS * es, 256);
  // the adaptive decomposition's decision state (two ints)
  w.offE = off;
  off += 256;
  w.total = off;
  return w;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + nb && y < x + na;
}

mgx_status hip_status(hipError_t e) { return e == hipSuccess ? MGX_OK : MGX_ERR_HIP; }

// ---- kernel tracing (mgx_trace_enable / mgx_trace_read) ----
struct TraceRec {
  const char *name;
  int level;
  hipEvent_t a, b;
};
struct Tracer {
  std::mutex mu;
  bool on = false;
  std::vector<TraceRec> recs;
  std::vector<hipEvent_t> pool;
};
Tracer &tracer() {
  static Tracer *t = new Tracer();
  return *t;
}
hipEvent_t take_event(Tracer &t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
// Runs launch() bracketed by events on st when tracing is on.
template <class F>
hipError_t traced(const char *name, int level, hipStream_t st, F &&launch) {
  Tracer &t = tracer();
  if (!t.on) return launch();
  std::lock_guard<std::mutex> g(t.mu);
  hipEvent_t a = take_event(t), b = take_event(t);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, st);
  t.recs.push_back({name, level, a, b});
  return e;
}

template <typename T>
AxisTab<T> axis_tab(const Plan *P, int l, int k, const T *tab) {
  const AxisLevel &a = P->ax[l][k];
  AxisTab<T> t;
  t.wl = tab + a.off_wl;
  t.wr = tab + a.off_wr;
  t.w5 = tab + a.off_w5;
  t.mult = tab + a.off_mult;
  t.invd = tab + a.off_invd;
  t.qsup = tab + a.off_qsup;
  t.multb = tab + a.off_multb;
  t.invdb = tab + a.off_invdb;
  t.qsub = tab + a.off_qsub;
  t.mid = tab + a.off_mid;
  t.m = (int)a.m;
  t.c = (int)a.c;
  return t;
}

// Sink of the launch sequences below.  Immediately launched (single field,
// traced when tracing is on), or recorded for a multi-field batch: the
// batch runs ops of equal (step, phase) of all its fields together, where
// step counts levels from the finest and phase counts ops within a level.
template <typename T>
struct RecordedOp {
  int kind, mode, step, phase;
  const char *name;
  int level;
  OpArgs<T> a;
};

template <typename T>
struct Emitter {
  hipStream_t st = nullptr;
  Tuning tn{};
  std::vector<RecordedOp<T>> *rec = nullptr;
  bool untraced = false;  // never bracket launches with events (callers that must not allocate)
  // immediate mode only: called before and after each launch with (kind, level)
  std::function<hipError_t(int, int)> before, after;
  // immediate mode only: the device flag that gates the stencil and solve
  // launches (they do nothing while it is 0), null: ungated
  const int *gate = nullptr;
  int base = 0, step = 0, phase = 0;
  void begin_step(int s) {
    step = base + s;
    phase = 0;
  }
  hipError_t op(int kind, int mode, const char *name, int level, const OpArgs<T> &in) {
    OpArgs<T> a = in;
    if (gate) {
      switch (kind) {
        case kOpLoadVecDec:
        case kOpLoadVecRec: a.st.gate = gate; break;
        case kOpSolveContig: a.so.gate = gate; break;
        case kOpSolveStrided:
        case kOpApply: a.sd.gate = gate; break;
        default: return hipErrorInvalidValue;
      }
    }
    if (rec) {
      rec->push_back({kind, mode, step, phase++, name, level, a});
      return hipSuccess;
    }
    hipError_t e;
    if (untraced) return launch_op<T>(kind, mode, a, tn, st);
    if (before && (e = before(kind, level)) != hipSuccess) return e;
    e = traced(name, level, st, [&] { return launch_op<T>(kind, mode, a, tn, st); });
    if (e == hipSuccess && after) e = after(kind, level);
    return e;
  }
};

// The coarse solves of one level on F (c0 x c1 x c2, pitches fp0,fp1), one
// per real axis, the contiguous axis first.  The last one either stores the
// solution (decomposition: out = Q_{l-1} u), applies it to the nodal values
// (recomposition: out = in - correction) or leaves it in F (in place).
template <typename T>
hipError_t solve_level(int level, const AxisTab<T> ax[3], const bool real[3], T *F, int64_t fp0, int64_t fp1,
                       int last_mode, const T *in, int64_t ip0, int64_t ip1, T *out, int64_t op0, int64_t op1,
                       Emitter<T> &em) {
  const int c0 = ax[0].c, c1 = ax[1].c, c2 = ax[2].c;
  hipError_t e;
  {
    OpArgs<T> o{};
    o.so = SolveArgs<T>{F, (int64_t)c0 * c1, fp1, c2, ax[2].mult, ax[2].invd, ax[2].qsup};
    if ((e = em.op(kOpSolveContig, 0, "solve_contig", level, o)) != hipSuccess) return e;
  }
  const T sign = T(-1);
  if (!real[1]) {  // 1-D: the solved row is the result
    OpArgs<T> o{};
    StridedArgs<T> &s = o.sd;
    s.F = F;
    s.nx = c2;
    s.in = last_mode == kSolveApply ? in : nullptr;
    s.out = out;
    s.sign = sign;
    return em.op(kOpApply, 0, "finish_1d", level, o);
  }
  auto strided = [&](int k, int mode, const char *name) {
    OpArgs<T> o{};
    StridedArgs<T> &s = o.sd;
    s.F = F;
    s.c = ax[k].c;
    s.sj = k == 1 ? fp1 : fp0;  // line stride
    s.nx = c2;
    s.so = k == 1 ? fp0 : fp1;  // outer stride (plane for the y solve, row for the z solve)
    s.nouter = k == 1 ? c0 : c1;
    s.mult = ax[k].mult;
    s.invd = ax[k].invd;
    s.qsup = ax[k].qsup;
    s.multb = ax[k].multb;
    s.invdb = ax[k].invdb;
    s.qsub = ax[k].qsub;
    s.mid = ax[k].mid;
    if (mode != kSolveInPlace) {
      s.in = in;
      s.ij = k == 1 ? ip1 : ip0;
      s.io = k == 1 ? ip0 : ip1;
      s.out = out;
      s.oj = k == 1 ? op1 : op0;
      s.oo = k == 1 ? op0 : op1;
      s.sign = sign;
    }
    return em.op(kOpSolveStrided, mode, name, level, o);
  };
  const char *last_name = last_mode == kSolveApply   ? "solve_strided_apply"
                          : last_mode == kSolveStore ? "solve_strided_store"
                                                     : "solve_strided";
  if (!real[0]) return strided(1, last_mode, last_name);  // 2-D
  if ((e = strided(1, kSolveInPlace, "solve_strided")) != hipSuccess) return e;
  return strided(0, last_mode, last_name);
}

template <typename T>
hipError_t copy_box(const T *src, int64_t sp0, int64_t sp1, T *dst, int64_t dp0, int64_t dp1, int n0, int n1,
                    int n2, int level, Emitter<T> &em) {
  OpArgs<T> o{};
  o.cp = CopyArgs<T>{src, sp0, sp1, dst, dp0, dp1, n0, n1, n2};
  return em.op(kOpCopyBox, 0, "copy_box", level, o);
}

template <typename T>
OpArgs<T> tail_args(const Plan *P, int stop, const T *tab, char *ws, const Layout &lay) {
  OpArgs<T> o{};
  TailArgs<T> &t = o.tl;
  t.nlev = lay.lt - stop;
  for (int i = 0; i < t.nlev; i++)
    for (int k = 0; k < 3; k++) {
      const AxisLevel &a = P->ax[lay.lt - i][k];
      t.ax[i][k] = TailAxis<T>{tab + a.off_wl,   tab + a.off_wr, tab + a.off_w5,  tab + a.off_mult,
                               tab + a.off_invd, tab + a.off_qsup, (int)a.m,      (int)a.c,
                               tail_magic(a.m),  tail_magic(a.c)};
    }
  (void)ws;
  return o;
}

void quant_box(const Plan *P, QuantArgs &qa, int level);

// Node counts of the level-l box along each axis (1 on padded axes).
void level_box(const Plan *P, int l, int64_t m[3]) {
  for (int k = 0; k < 3; k++) m[k] = P->real[k] ? (P->n[k] - 1) / ((int64_t)1 << (P->L - l)) + 1 : 1;
}

// 1/q in FP64 rounded to FP32, NaN outside FP32's normal range: the factor
// of the decomposition kernels' FP32 label shortcut (the same rounding the
// device-side label_rcp performs).
float label_rcp_host(double q) {
  const double r = 1.0 / q;
  return (r >= 1.1754943508222875e-38 && r <= 3.4028234663852886e38) ? (float)r : std::nanf("");
}

// With labels (and the quantizer's arguments qa), every kernel that writes
// coefficients also writes their labels, and u_mc may be null (labels only).
template <typename T>
mgx_status run_decompose(Plan *P, int stop, const T *u, T *umc, char *ws, const Layout &lay, const T *tab,
                         Emitter<T> &em, int32_t *labels = nullptr, const QuantArgs *qa = nullptr) {
  const int L = P->L;
  const int64_t n1 = P->n[1], n2 = P->n[2];
  const int64_t up0 = n1 * n2, up1 = n2;
  if (stop == L) {
    em.begin_step(0);
    if (umc && copy_box<T>(u, up0, up1, umc, up0, up1, (int)P->n[0], (int)n1, (int)n2, L, em) != hipSuccess)
      return MGX_ERR_HIP;
    if (labels) {
      OpArgs<T> o{};
      o.qj = QuantJob<T>{u, labels, *qa};  // at stop == L, u_mc is u itself
      em.begin_step(1);
      if (em.op(kOpQuantize, 0, "quantize", -1, o) != hipSuccess) return MGX_ERR_HIP;
    }
    return MGX_OK;
  }
  T *A = (T *)(ws + lay.offA), *B = (T *)(ws + lay.offB), *F = (T *)(ws + lay.offF);
  T *S = (T *)(ws + lay.offS);  // the stop box when u_mc is not written
  const T *src = u;
  int64_t sp0 = up0, sp1 = up1;
  const int lowest = lay.lt > stop ? lay.lt : stop;  // tiled levels L .. lowest+1
  for (int l = L; l > lowest; l--) {
    em.begin_step(L - l);
    AxisTab<T> ax[3] = {axis_tab(P, l, 0, tab), axis_tab(P, l, 1, tab), axis_tab(P, l, 2, tab)};
    const int c1 = ax[1].c, c2 = ax[2].c;
    const int64_t cp1 = c2, cp0 = (int64_t)c1 * c2;
    const int64_t fp1 = round4(c2), fp0 = (int64_t)c1 * fp1;
    OpArgs<T> o{};
    StencilArgs<T> &s = o.st;
    for (int k = 0; k < 3; k++) s.ax[k] = ax[k];
    s.V = src;
    s.vp0 = sp0;
    s.vp1 = sp1;
    s.umc_w = umc;
    s.up0 = up0;
    s.up1 = up1;
    s.F = F;
    s.fp0 = fp0;
    s.fp1 = fp1;
    if (labels) {
      s.lab_w = labels;
      s.qc = qa->q[l - stop];
      s.rqc = label_rcp_host(s.qc);
      s.rng = qa->stats_ovf;  // [0] overflow, [1] non-finite (stats_nan follows it)
      s.smax = qa->stats_max ? qa->stats_max + (l - stop) : nullptr;
    }
    hipError_t e = em.op(kOpLoadVecDec, 0, labels ? "load_vector_dec+q" : "load_vector_dec", l, o);
    if (e != hipSuccess) return MGX_ERR_HIP;
    // Q_{l-1} u goes to the compact box of level l-1, or into the corner of
    // u_mc after the last decomposed level (the compact stop box without u_mc)
    const bool last = (l == stop + 1);
    T *dst = last ? (umc ? umc : S) : (((L - 1 - (l - 1)) % 2 == 0) ? A : B);
    const int64_t op0 = (last && umc) ? up0 : cp0, op1 = (last && umc) ? up1 : cp1;
    e = solve_level<T>(l, ax, P->real, F, fp0, fp1, kSolveStore, nullptr, 0, 0, dst, op0, op1, em);
    if (e != hipSuccess) return MGX_ERR_HIP;
    src = dst;
    sp0 = cp0;
    sp1 = cp1;
  }
  if (lay.lt > stop) {  // levels lt .. stop+1 in one workgroup
    em.begin_step(L - lay.lt);
    OpArgs<T> o = tail_args<T>(P, stop, tab, ws, lay);
    o.tl.src = src;
    o.tl.sp0 = sp0;
    o.tl.sp1 = sp1;
    o.tl.umc = umc;
    o.tl.up0 = up0;
    o.tl.up1 = up1;
    if (labels) {
      o.tl.lab_w = labels;
      for (int i = 0; i < o.tl.nlev; i++) o.tl.q[i] = qa->q[lay.lt - i - stop];
      o.tl.q[o.tl.nlev] = qa->q[0];
      o.tl.rng = qa->stats_ovf;
      o.tl.smax = qa->stats_max;
    }
    if (em.op(kOpTailDec, 0, labels ? "tail_dec+q" : "tail_dec", lay.lt, o) != hipSuccess) return MGX_ERR_HIP;
  } else if (labels) {  // the stop box's labels, after the last level
    QuantArgs b = *qa;
    quant_box(P, b, stop);
    b.sel_lo = b.sel_hi = stop;
    b.box_compact = umc ? 0 : 1;
    OpArgs<T> o{};
    o.qj = QuantJob<T>{umc ? umc : S, labels, b};
    em.begin_step(L - stop);
    if (em.op(kOpQuantize, 0, "quantize_box", -1, o) != hipSuccess) return MGX_ERR_HIP;
  }
  return MGX_OK;
}

// With labels (and qa), the coefficients are read as labels times the
// level's bin width (u_mc unused, may be null).  With top < L the
// recomposition stops after level top and u receives Q_top u as the compact
// level-top box (progressive recomposition; coefficients from u_mc only).
template <typename T>
mgx_status run_recompose(Plan *P, int stop, const T *umc, T *u, char *ws, const Layout &lay0, const T *tab,
                         Emitter<T> &em, const int32_t *labels = nullptr, const QuantArgs *qa = nullptr,
                         int top = -1) {
  const int L = P->L;
  if (top < 0) top = L;
  if (top < stop || top > L || (labels && top != L)) return MGX_ERR_LEVEL;
  Layout lay = lay0;
  if (lay.lt > top) lay.lt = top;  // the single-workgroup tail ends at the target level
  const int64_t n1 = P->n[1], n2 = P->n[2];
  const int64_t up0 = n1 * n2, up1 = n2;
  int64_t tm[3];
  level_box(P, top, tm);
  const int64_t tp1 = tm[2], tp0 = tm[1] * tm[2];  // output pitches (level-top box)
  if (stop == top) {
    em.begin_step(0);
    if (labels) {
      OpArgs<T> o{};
      o.dj = DequantJob<T>{labels, u, *qa};
      return hip_status(em.op(kOpDequantize, 0, "dequantize", -1, o));
    }
    return hip_status(copy_box<T>(umc, up0, up1, u, tp0, tp1, (int)tm[0], (int)tm[1], (int)tm[2], top, em));
  }
  T *A = (T *)(ws + lay.offA), *B = (T *)(ws + lay.offB), *F = (T *)(ws + lay.offF);
  T *S = (T *)(ws + lay.offS);
  const bool sbox = labels && !(lay.lt > stop);  // stop box dequantized into S first
  if (sbox) {
    QuantArgs b = *qa;
    quant_box(P, b, stop);
    b.sel_lo = b.sel_hi = stop;
    b.box_compact = 1;
    OpArgs<T> o{};
    o.dj = DequantJob<T>{labels, S, b};
    em.begin_step(0);
    if (em.op(kOpDequantize, 0, "dequantize_box", -1, o) != hipSuccess) return MGX_ERR_HIP;
  }
  int first_tiled = stop + 1;
  if (lay.lt > stop) {  // levels stop+1 .. lt in one workgroup, into the level-lt box
    em.begin_step(0);
    OpArgs<T> o = tail_args<T>(P, stop, tab, ws, lay);
    o.tl.umc_r = umc;
    o.tl.up0 = up0;
    o.tl.up1 = up1;
    if (labels) {
      o.tl.lab_r = labels;
      for (int i = 0; i < o.tl.nlev; i++) o.tl.q[i] = qa->q[lay.lt - i - stop];
      o.tl.q[o.tl.nlev] = qa->q[0];
    }
    if (lay.lt == top) {
      o.tl.dst = u;
      o.tl.dp0 = tp0;
      o.tl.dp1 = tp1;
    } else {
      const AxisLevel &a1 = P->ax[lay.lt][1], &a2 = P->ax[lay.lt][2];
      o.tl.dst = ((L - 1 - lay.lt) % 2 == 0) ? A : B;
      o.tl.dp1 = a2.m;
      o.tl.dp0 = a1.m * a2.m;
    }
    if (em.op(kOpTailRec, 0, labels ? "tail_rec+q" : "tail_rec", lay.lt, o) != hipSuccess) return MGX_ERR_HIP;
    first_tiled = lay.lt + 1;
  }
  for (int l = first_tiled; l <= top; l++) {
    em.begin_step(l - stop - 1 + ((lay.lt > stop || sbox) ? 1 : 0));
    AxisTab<T> ax[3] = {axis_tab(P, l, 0, tab), axis_tab(P, l, 1, tab), axis_tab(P, l, 2, tab)};
    const int c1 = ax[1].c, c2 = ax[2].c;
    const int m1 = ax[1].m, m2 = ax[2].m;
    T *nb = ((L - 1 - (l - 1)) % 2 == 0) ? A : B;  // level l-1 nodal values
    const int64_t cp1 = c2, cp0 = (int64_t)c1 * c2;
    const int64_t fp1 = round4(c2), fp0 = (int64_t)c1 * fp1;
    const bool first = (l == stop + 1);  // with a tail, level lt+1 reads the tail's box nb
    const T *nin = first ? (sbox ? S : umc) : nb;
    const int64_t ip0 = (first && !sbox) ? up0 : cp0, ip1 = (first && !sbox) ? up1 : cp1;
    OpArgs<T> o{};
    StencilArgs<T> &s = o.st;
    for (int k = 0; k < 3; k++) s.ax[k] = ax[k];
    s.umc_r = umc;
    s.up0 = up0;
    s.up1 = up1;
    s.F = F;
    s.fp0 = fp0;
    s.fp1 = fp1;
    if (labels) {
      s.lab_r = labels;
      s.qc = qa->q[l - stop];
    }
    hipError_t e = em.op(kOpLoadVecRec, 0, labels ? "load_vector_rec+q" : "load_vector_rec", l, o);
    if (e != hipSuccess) return MGX_ERR_HIP;
    e = solve_level<T>(l, ax, P->real, F, fp0, fp1, kSolveApply, nin, ip0, ip1, nb, cp0, cp1, em);
    if (e != hipSuccess) return MGX_ERR_HIP;
    OpArgs<T> oi{};
    InterpArgs<T> &ia = oi.ia;
    for (int k = 0; k < 3; k++) ia.ax[k] = ax[k];
    ia.nodal = nb;
    ia.np0 = cp0;
    ia.np1 = cp1;
    ia.umc = umc;
    ia.up0 = up0;
    ia.up1 = up1;
    if (labels) {
      ia.lab = labels;
      ia.qc = qa->q[l - stop];
    }
    if (l == top) {
      ia.out = u;
      ia.op0 = tp0;
      ia.op1 = tp1;
    } else {
      ia.out = ((L - 1 - l) % 2 == 0) ? A : B;
      ia.op1 = m2;
      ia.op0 = (int64_t)m1 * m2;
    }
    e = em.op(kOpInterpAdd, 0, labels ? "interp_add+q" : "interp_add", l, oi);
    if (e != hipSuccess) return MGX_ERR_HIP;
  }
  return MGX_OK;
}

mgx_status tolerances(Plan *P, int ndim, double tol, int stop, double c_linf, double *tau);

// ---- adaptive decomposition (Sec. 4.2, Alg. 1 lines 1-16) ----
// Penalty factors of the estimate (Sec. 4.2, 3-D, in units of tau0).
constexpr double kPenLorenzo = 1.22, kPenEdge = 0.369, kPenPlane = 0.259, kPenCube = 0.182;

// Sampled 3^3 blocks of the estimate on level l (cells a = 1, 5, 9, ... per
// axis) and its sampled edge, plane and cube nodes (12, 6, 1 per block).
int64_t estimate_blocks(const Plan *P, int l, int nbk[3], int64_t counts[3]) {
  int64_t m[3];
  level_box(P, l, m);
  for (int k = 0; k < 3; k++) {
    const int64_t cells = (m[k] - 1) / 2;
    nbk[k] = cells > 1 ? (int)((cells - 2) / 4 + 1) : 0;
  }
  const int64_t nb = (int64_t)nbk[0] * nbk[1] * nbk[2];
  counts[0] = 12 * nb;
  counts[1] = 6 * nb;
  counts[2] = nb;
  return nb;
}

int estimate_workgroups(int64_t nb) { return (int)((nb + kEstimateThreads - 1) / kEstimateThreads); }

// Enqueues the estimate on the level-l box V (pitches vp0, vp1) and the
// decision kernel on st; nothing waits.  part: the per-workgroup sums;
// sums (nullable): the two totals; state (nullable): the decision state,
// which also gates the estimate unless this is the first decision.
template <typename T>
mgx_status enqueue_estimate(Plan *P, int l, const T *V, int64_t vp0, int64_t vp1, const double *tab64, double *part,
                            double *sums, int *state, bool first, double tau0, hipStream_t st) {
  int nbk[3];
  int64_t cnt[3];
  const int64_t nb = estimate_blocks(P, l, nbk, cnt);
  const int nwg = estimate_workgroups(nb);
  if (nb > 0) {
    EstimateArgs<T> a{};
    a.V = V;
    a.vp0 = vp0;
    a.vp1 = vp1;
    a.nb0 = nbk[0];
    a.nb1 = nbk[1];
    a.nb2 = nbk[2];
    for (int k = 0; k < 3; k++) {
      a.wl[k] = tab64 + P->ax[l][k].off_wl;
      a.wr[k] = tab64 + P->ax[l][k].off_wr;
    }
    a.partial = part;
    a.gate = first ? nullptr : state;
    if (traced("adaptive_estimate", l, st, [&] { return launch_adaptive_estimate<T>(a, nwg, st); }) != hipSuccess)
      return MGX_ERR_HIP;
  }
  DecideArgs d{};
  d.partial = part;
  d.nwg = nwg;
  d.sums = sums;
  d.state = state;
  d.level = l;
  d.first = first ? 1 : 0;
  d.pen_lor = kPenLorenzo * tau0 * (double)(cnt[0] + cnt[1] + cnt[2]);
  d.pen_int = (kPenEdge * (double)cnt[0] + kPenPlane * (double)cnt[1] + kPenCube * (double)cnt[2]) * tau0;
  if (traced("adaptive_decide", l, st, [&] { return launch_adaptive_decide(d, st); }) != hipSuccess)
    return MGX_ERR_HIP;
  return MGX_OK;
}

// All levels are enqueued at once, decided on the device: per level from L
// the estimate of Q_l u and its decision, then the level's kernels, which
// run only while the decision state says go on.  One wait at the end reads
// the stop level; Q_stop u (u itself, or the compact A/B box the last run
// level wrote, untouched by the gated levels below) is then copied into
// u_mc's corner.  The estimate's partial sums use the load vector's buffer
// F, which the level's kernels overwrite only after the decision.
template <typename T>
mgx_status run_decompose_adaptive(Plan *P, int ndim, const T *u, T *umc, double tol, double c_linf, char *ws,
                                  const Layout &lay, const T *tab, const double *tab64, hipStream_t st,
                                  int *stop_out) {
  const int L = P->L;
  const int64_t n1 = P->n[1], n2 = P->n[2];
  const int64_t up0 = n1 * n2, up1 = n2;
  T *A = (T *)(ws + lay.offA), *B = (T *)(ws + lay.offB), *F = (T *)(ws + lay.offF);
  double *part = (double *)(ws + lay.offF);
  int *state = (int *)(ws + lay.offE);
  Emitter<T> em;
  em.st = st;
  em.gate = state;
  const T *src = u;
  int64_t sp0 = up0, sp1 = up1;
  for (int l = L; l >= 1; l--) {
    double tau[kMaxLevels];
    mgx_status s = tolerances(P, ndim, tol, l, c_linf, tau);
    if (s) return s;
    if ((s = enqueue_estimate<T>(P, l, src, sp0, sp1, tab64, part, nullptr, state, l == L, tau[0], st))) return s;
    AxisTab<T> ax[3] = {axis_tab(P, l, 0, tab), axis_tab(P, l, 1, tab), axis_tab(P, l, 2, tab)};
    const int c1 = ax[1].c, c2 = ax[2].c;
    const int64_t cp1 = c2, cp0 = (int64_t)c1 * c2;
    const int64_t fp1 = round4(c2), fp0 = (int64_t)c1 * fp1;
    OpArgs<T> o{};
    StencilArgs<T> &sa = o.st;
    for (int k = 0; k < 3; k++) sa.ax[k] = ax[k];
    sa.V = src;
    sa.vp0 = sp0;
    sa.vp1 = sp1;
    sa.umc_w = umc;
    sa.up0 = up0;
    sa.up1 = up1;
    sa.F = F;
    sa.fp0 = fp0;
    sa.fp1 = fp1;
    if (em.op(kOpLoadVecDec, 0, "load_vector_dec", l, o) != hipSuccess) return MGX_ERR_HIP;
    T *dst = ((L - 1 - (l - 1)) % 2 == 0) ? A : B;
    if (solve_level<T>(l, ax, P->real, F, fp0, fp1, kSolveStore, nullptr, 0, 0, dst, cp0, cp1, em) != hipSuccess)
      return MGX_ERR_HIP;
    src = dst;
    sp0 = cp0;
    sp1 = cp1;
  }
  int stop = -1;
  if (hipMemcpyAsync(&stop, state + 1, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return MGX_ERR_HIP;
  if (stop < 0 || stop > L) return MGX_ERR_HIP;
  int64_t m[3];
  level_box(P, stop, m);
  if (stop < L) {  // Q_s u for s < L sits in the box level s + 1 wrote
    src = ((L - 1 - stop) % 2 == 0) ? A : B;
    sp0 = m[1] * m[2];
    sp1 = m[2];
  } else {
    src = u;
    sp0 = up0;
    sp1 = up1;
  }
  em.gate = nullptr;
  if (copy_box<T>(src, sp0, sp1, umc, up0, up1, (int)m[0], (int)m[1], (int)m[2], stop, em) != hipSuccess)
    return MGX_ERR_HIP;
  *stop_out = stop;
  return MGX_OK;
}

// Tables of level l with the load-vector stencil replaced by the restriction
// R = P^T alone (adjoint passes).
template <typename T>
AxisTab<T> restrict_tab(const Plan *P, int l, int k, const T *tab) {
  AxisTab<T> t = axis_tab(P, l, k, tab);
  t.w5 = tab + P->ax[l][k].off_p5;
  return t;
}

// Adjoint of decomposition (not in the paper): g_u = D^T g_mc.  D is the
// product of the level maps D_L first ... D_{stop+1} last, so the transpose
// runs the levels upwards.  Per level, with gW the gradient of the coarse
// values and gz that of the level's coefficients:
//   y = Mc^{-1} gW,  r = R gz,
//   g_V = (M P)^{x3} y + gz at coefficient nodes, - r at nodal nodes.
template <typename T>
mgx_status run_decompose_adjoint(Plan *P, int stop, const T *gmc, T *gu, char *ws, const Layout &lay,
                                 const T *tab, hipStream_t st) {
  Emitter<T> em;
  em.st = st;
  const int L = P->L;
  const int64_t n1 = P->n[1], n2 = P->n[2];
  const int64_t up0 = n1 * n2, up1 = n2;
  if (stop == L) return hip_status(hipMemcpyAsync(gu, gmc, sizeof(T) * P->n[0] * up0, hipMemcpyDeviceToDevice, st));
  T *A = (T *)(ws + lay.offA), *B = (T *)(ws + lay.offB), *F = (T *)(ws + lay.offF), *G = (T *)(ws + lay.offG);
  for (int l = stop + 1; l <= L; l++) {
    AxisTab<T> ax[3] = {axis_tab(P, l, 0, tab), axis_tab(P, l, 1, tab), axis_tab(P, l, 2, tab)};
    const int c0 = ax[0].c, c1 = ax[1].c, c2 = ax[2].c;
    const int m1 = ax[1].m, m2 = ax[2].m;
    const int64_t cp1 = c2, cp0 = (int64_t)c1 * c2;
    const int64_t fp1 = round4(c2), fp0 = (int64_t)c1 * fp1;
    const bool first = (l == stop + 1);
    const T *gW = first ? gmc : (((L - 1 - (l - 1)) % 2 == 0) ? A : B);
    const int64_t wp0 = first ? up0 : cp0, wp1 = first ? up1 : cp1;
    hipError_t e = copy_box<T>(gW, wp0, wp1, F, fp0, fp1, c0, c1, c2, l, em);
    if (e != hipSuccess) return MGX_ERR_HIP;
    e = solve_level<T>(l, ax, P->real, F, fp0, fp1, kSolveInPlace, nullptr, 0, 0, F, fp0, fp1, em);
    if (e != hipSuccess) return MGX_ERR_HIP;
    StencilArgs<T> s{};
    for (int k = 0; k < 3; k++) s.ax[k] = restrict_tab(P, l, k, tab);
    s.umc_r = gmc;
    s.up0 = up0;
    s.up1 = up1;
    s.F = G;
    s.fp0 = fp0;
    s.fp1 = fp1;
    e = traced("restrict_coef", l, st, [&] { return launch_load_vector<T>(s, false, st); });
    if (e != hipSuccess) return MGX_ERR_HIP;
    ProlongArgs<T> pa{};
    for (int k = 0; k < 3; k++) pa.ax[k] = ax[k];
    pa.y = F;
    pa.yp0 = fp0;
    pa.yp1 = fp1;
    pa.lc_in = gmc;
    pa.up0 = up0;
    pa.up1 = up1;
    pa.r = G;
    pa.rp0 = fp0;
    pa.rp1 = fp1;
    if (l == L) {
      pa.out = gu;
      pa.op0 = up0;
      pa.op1 = up1;
    } else {
      pa.out = ((L - 1 - l) % 2 == 0) ? A : B;
      pa.op1 = m2;
      pa.op0 = (int64_t)m1 * m2;
    }
    e = traced("prolong_mass_dec_adj", l, st, [&] { return launch_prolong_mass<T>(pa, kProlongDecAdj, st); });
    if (e != hipSuccess) return MGX_ERR_HIP;
  }
  return MGX_OK;
}

// Adjoint of recomposition: g_mc = R^T g_u, levels downwards.  Per level,
// with g_V the gradient of the level-l values:
//   a = R g_V (the gradient of the coarse values), y = Mc^{-1} a,
//   gz = g_V - (M P)^{x3} y at the coefficient nodes.
template <typename T>
mgx_status run_recompose_adjoint(Plan *P, int stop, const T *gu, T *gmc, char *ws, const Layout &lay,
                                 const T *tab, hipStream_t st) {
  Emitter<T> em;
  em.st = st;
  const int L = P->L;
  const int64_t n1 = P->n[1], n2 = P->n[2];
  const int64_t up0 = n1 * n2, up1 = n2;
  if (stop == L) return hip_status(hipMemcpyAsync(gmc, gu, sizeof(T) * P->n[0] * up0, hipMemcpyDeviceToDevice, st));
  T *A = (T *)(ws + lay.offA), *B = (T *)(ws + lay.offB), *F = (T *)(ws + lay.offF);
  for (int l = L; l > stop; l--) {
    AxisTab<T> ax[3] = {axis_tab(P, l, 0, tab), axis_tab(P, l, 1, tab), axis_tab(P, l, 2, tab)};
    const int c0 = ax[0].c, c1 = ax[1].c, c2 = ax[2].c;
    const int m1 = ax[1].m, m2 = ax[2].m;
    const int64_t cp1 = c2, cp0 = (int64_t)c1 * c2;
    const int64_t fp1 = round4(c2), fp0 = (int64_t)c1 * fp1;
    const T *gV = (l == L) ? gu : (((L - 1 - l) % 2 == 0) ? A : B);
    const int64_t vp0 = (l == L) ? up0 : (int64_t)m1 * m2, vp1 = (l == L) ? up1 : m2;
    StencilArgs<T> s{};
    for (int k = 0; k < 3; k++) s.ax[k] = restrict_tab(P, l, k, tab);
    s.V = gV;
    s.vp0 = vp0;
    s.vp1 = vp1;
    s.umc_w = nullptr;
    s.up0 = up0;
    s.up1 = up1;
    s.F = F;
    s.fp0 = fp0;
    s.fp1 = fp1;
    hipError_t e = traced("restrict_field", l, st, [&] { return launch_load_vector<T>(s, true, st); });
    if (e != hipSuccess) return MGX_ERR_HIP;
    // the coarse gradient: the stop box of g_mc, or the next level's input
    const bool last = (l == stop + 1);
    T *gW = last ? gmc : (((L - 1 - (l - 1)) % 2 == 0) ? A : B);
    const int64_t wp0 = last ? up0 : cp0, wp1 = last ? up1 : cp1;
    e = copy_box<T>(F, fp0, fp1, gW, wp0, wp1, c0, c1, c2, l, em);
    if (e != hipSuccess) return MGX_ERR_HIP;
    e = solve_level<T>(l, ax, P->real, F, fp0, fp1, kSolveInPlace, nullptr, 0, 0, F, fp0, fp1, em);
    if (e != hipSuccess) return MGX_ERR_HIP;
    ProlongArgs<T> pa{};
    for (int k = 0; k < 3; k++) pa.ax[k] = ax[k];
    pa.y = F;
    pa.yp0 = fp0;
    pa.yp1 = fp1;
    pa.fine = gV;
    pa.fp0 = vp0;
    pa.fp1 = vp1;
    pa.lc_out = gmc;
    pa.up0 = up0;
    pa.up1 = up1;
    e = traced("prolong_mass_rec_adj", l, st, [&] { return launch_prolong_mass<T>(pa, kProlongRecAdj, st); });
    if (e != hipSuccess) return MGX_ERR_HIP;
  }
  return MGX_OK;
}

// Common validation of decompose / recompose.
// With placed != null the tables are not looked up on the device (the caller
// copies them to memory of its own) and *tab stays untouched.
mgx_status prepare(const void *in, void *out, mgx_dtype dtype, int ndim, const int64_t *dims,
                   const double *const *coords, int stop, void *ws, size_t ws_bytes, Plan **plan,
                   Layout *lay, const void **tab, bool adjoint = false, int may_null = 0, bool placed = false) {
  if (dtype != MGX_F32 && dtype != MGX_F64) return MGX_ERR_ARG;
  int64_t n[3];
  bool real[3];
  int L;
  int st = parse_shape(ndim, dims, n, real, &L);
  if (st) return (mgx_status)st;
  // may_null: 1 = in, 2 = out may be null (the fused calls' u_mc)
  if ((!in && !(may_null & 1)) || (!out && !(may_null & 2))) return MGX_ERR_ARG;
  const size_t es = elem_size(dtype);
  const size_t bytes = (size_t)(n[0] * n[1] * n[2]) * es;
  if (in && out && overlaps(in, bytes, out, bytes)) return MGX_ERR_ARG;
  Plan *P = get_plan(ndim, dims, coords, &st);
  if (!P) return (mgx_status)st;
  if (stop < 0 || stop > L) return MGX_ERR_LEVEL;
  *lay = layout(n, real, L, stop, es, adjoint);
  if (lay->total > 0) {
    if (!ws || ws_bytes < lay->total) return MGX_ERR_WORKSPACE;
    if ((in && overlaps(ws, lay->total, in, bytes)) || (out && overlaps(ws, lay->total, out, bytes)))
      return MGX_ERR_ARG;
  }
  *plan = P;
  if (placed) return MGX_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MGX_ERR_HIP;
  int herr = 0;
  *tab = P->device_tables(dev, dtype == MGX_F64, &herr);
  if (!*tab) return MGX_ERR_HIP;
  return MGX_OK;
}

// Level tolerances of Sec. 4.1, eq. (LinfTau) with the stop level of
// Algorithm 1, in a fixed FP64 operation order.
// C: the L-infinity constant (c_linf when given, else the plan's default).
mgx_status tau_schedule(double C, int L, int ndim, double tol, int stop, double *tau) {
  if (!(tol > 0.0) || !std::isfinite(tol)) return MGX_ERR_TOL;
  if (!(C >= 1.0) || !std::isfinite(C)) return MGX_ERR_TOL;
  volatile double kappa = std::sqrt((double)(1 << ndim));
  double p = 1.0;
  for (int i = 0; i < L + 1 - stop; i++) p = p * kappa;
  double t = ((1.0 - kappa) / (1.0 - p)) * (tol / C);
  tau[0] = t;
  for (int l = 1; l <= L - stop; l++) tau[l] = tau[l - 1] * kappa;
  return MGX_OK;
}

mgx_status tolerances(Plan *P, int ndim, double tol, int stop, double c_linf, double *tau) {
  if (std::isnan(c_linf) || std::isinf(c_linf)) return MGX_ERR_TOL;
  if (!(tol > 0.0) || !std::isfinite(tol)) return MGX_ERR_TOL;
  return tau_schedule(c_linf > 0.0 ? c_linf : P->linf_constant(stop), P->L, ndim, tol, stop, tau);
}

// tau_in (optional): the tolerances of levels stop .. L given by the caller
// instead of the L-infinity schedule of tol.
mgx_status quant_args(int ndim, const int64_t *dims, const double *const *coords, double tol, int stop,
                      double c_linf, QuantArgs *qa, Plan **plan, const double *tau_in = nullptr) {
  int st = 0;
  Plan *P = get_plan(ndim, dims, coords, &st);
  if (!P) return (mgx_status)st;
  if (stop < 0 || stop > P->L) return MGX_ERR_LEVEL;
  double tau[kMaxLevels];
  if (tau_in) {
    for (int i = 0; i <= P->L - stop; i++) {
      if (!(tau_in[i] > 0.0) || !std::isfinite(tau_in[i])) return MGX_ERR_TOL;
      tau[i] = tau_in[i];
    }
  } else {
    mgx_status s = tolerances(P, ndim, tol, stop, c_linf, tau);
    if (s) return s;
  }
  const int L = P->L;
  std::memset(qa, 0, sizeof(*qa));
  qa->n = P->n[0] * P->n[1] * P->n[2];
  if (qa->n >= ((int64_t)1 << 32)) return MGX_ERR_SHAPE;  // flat 32-bit indexing
  qa->n1 = (int)P->n[1];
  qa->n2 = (int)P->n[2];
  auto magic = [](uint64_t d) -> uint64_t { return d < 2 ? 0 : (~(uint64_t)0) / d + 1; };
  qa->mag1 = magic((uint64_t)qa->n1);
  qa->mag2 = magic((uint64_t)qa->n2);
  for (int k = 0; k < 3; k++) {
    int m = 0;
    if (P->real[k])
      while (((int64_t)1 << m) < P->n[k] - 1) m++;
    qa->off[k] = P->real[k] ? m - L : 0;
  }
  qa->first = stop;
  qa->nlev = L + 1 - stop;
  qa->sel_lo = stop;
  qa->sel_hi = L;
  for (int i = 0; i < qa->nlev; i++) qa->q[i] = 2.0 * tau[i];
  *plan = P;
  return MGX_OK;
}

struct StatsBuf {
  std::mutex mu;
  std::vector<void *> per_dev;
};
StatsBuf &stats_buf() {
  static StatsBuf *s = new StatsBuf();
  return *s;
}

// The statistics buffer of the current device (per-level max |label| and the
// out-of-range counts), cleared on `stream`; nullptr on a HIP error.  The
// caller holds stats_buf().mu until it has read the buffer back.
char *stats_device(hipStream_t stream) {
  StatsBuf &sb = stats_buf();
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  if ((int)sb.per_dev.size() <= dev) sb.per_dev.resize(dev + 1, nullptr);
  const size_t sbytes = sizeof(int) * kMaxLevels + 2 * sizeof(unsigned long long);
  if (!sb.per_dev[dev] && hipMalloc(&sb.per_dev[dev], sbytes) != hipSuccess) return nullptr;
  if (hipMemsetAsync(sb.per_dev[dev], 0, sbytes, stream) != hipSuccess) return nullptr;
  return (char *)sb.per_dev[dev];
}

// Waits for `stream` and fills *stats from the buffer; MGX_ERR_RANGE when some
// label overflowed or some coefficient was not finite.
mgx_status stats_read(const char *base, int first, int nlev, mgx_quant_stats *stats, hipStream_t stream) {
  const size_t sbytes = sizeof(int) * kMaxLevels + 2 * sizeof(unsigned long long);
  char host[sizeof(int) * kMaxLevels + 2 * sizeof(unsigned long long)];
  if (hipMemcpyAsync(host, base, sbytes, hipMemcpyDeviceToHost, stream) != hipSuccess) return MGX_ERR_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return MGX_ERR_HIP;
  std::memset(stats, 0, sizeof(*stats));
  stats->first_level = first;
  stats->num_levels = nlev;
  std::memcpy(stats->max_abs_label, host, sizeof(int) * nlev);
  unsigned long long ovf, nan;
  std::memcpy(&ovf, host + sizeof(int) * kMaxLevels, sizeof(ovf));
  std::memcpy(&nan, host + sizeof(int) * kMaxLevels + sizeof(ovf), sizeof(nan));
  stats->n_overflow = (int64_t)ovf;
  stats->n_nonfinite = (int64_t)nan;
  return (ovf || nan) ? MGX_ERR_RANGE : MGX_OK;
}

// The corner box of a level (level L-1: the coarser levels' coefficients)
// as the visited region of a quantization pass.
void quant_box(const Plan *P, QuantArgs &qa, int level = -1) {
  const int L = P->L;
  if (level < 0) level = L - 1;
  int64_t b[3];
  for (int k = 0; k < 3; k++) b[k] = P->real[k] ? (P->n[k] - 1) / ((int64_t)1 << (L - level)) + 1 : 1;
  auto magic = [](uint64_t d) -> uint64_t { return d < 2 ? 0 : (~(uint64_t)0) / d + 1; };
  qa.box = 1;
  qa.b1 = (int)b[1];
  qa.b2 = (int)b[2];
  qa.bn = b[0] * b[1] * b[2];
  qa.bmag1 = magic((uint64_t)b[1]);
  qa.bmag2 = magic((uint64_t)b[2]);
  (void)L;
}

// The fused calls: the level kernels write (decomposition) or read
// (recomposition) the labels themselves.
template <typename T>
mgx_status run_decompose_quantize(Plan *P, int stop, const T *u, T *umc, int32_t *labels, QuantArgs qa, char *ws,
                                  const Layout &lay, const T *tab, hipStream_t st) {
  Emitter<T> em;
  em.st = st;
  return run_decompose<T>(P, stop, u, umc, ws, lay, tab, em, labels, &qa);
}

template <typename T>
mgx_status run_dequantize_recompose(Plan *P, int stop, const int32_t *labels, T *umc, T *u, QuantArgs qa,
                                    char *ws, const Layout &lay, const T *tab, hipStream_t st) {
  Emitter<T> em;
  em.st = st;
  if (!umc)  // coefficients read from the labels by the level kernels
    return run_recompose<T>(P, stop, nullptr, u, ws, lay, tab, em, labels, &qa);
  if (traced("dequantize", -1, st, [&] { return launch_dequantize<T>(labels, umc, qa, st); }) != hipSuccess)
    return MGX_ERR_HIP;
  return run_recompose<T>(P, stop, umc, u, ws, lay, tab, em);
}

// ---- batches of fields (multi-field launches in one captured graph) ----
struct BatchField {
  Plan *P = nullptr;
  const void *tab = nullptr;
  Layout lay;
  size_t ws_off = 0;
};

mgx_status batch_validate(int nfields, const mgx_field *f, bool dec, std::vector<BatchField> &out,
                          size_t *ws_total, bool check_ptrs = true) {
  if (nfields < 1 || !f) return MGX_ERR_ARG;
  out.assign(nfields, BatchField{});
  size_t off = 0;
  int dev = 0;
  if (check_ptrs && hipGetDevice(&dev) != hipSuccess) return MGX_ERR_HIP;
  for (int i = 0; i < nfields; i++) {
    const mgx_field &x = f[i];
    if (x.dtype != MGX_F32 && x.dtype != MGX_F64) return MGX_ERR_ARG;
    int64_t n[3];
    bool real[3];
    int L;
    int st = parse_shape(x.ndim, x.dims, n, real, &L);
    if (st) return (mgx_status)st;
    const size_t es = elem_size(x.dtype);
    const size_t bytes = (size_t)(n[0] * n[1] * n[2]) * es;
    if (check_ptrs) {
      if (!x.out) return MGX_ERR_ARG;
      if (dec || !x.labels) {
        if (!x.in || overlaps(x.in, bytes, x.out, bytes)) return MGX_ERR_ARG;
      } else if (x.coef && overlaps(x.coef, bytes, x.out, bytes)) {
        return MGX_ERR_ARG;
      }
      if (x.labels && overlaps(x.labels, (size_t)(n[0] * n[1] * n[2]) * 4, x.out, bytes)) return MGX_ERR_ARG;
    }
    Plan *P = get_plan(x.ndim, x.dims, x.coords, &st);
    if (!P) return (mgx_status)st;
    if (x.stop_level < 0 || x.stop_level > L) return MGX_ERR_LEVEL;
    BatchField &b = out[i];
    b.P = P;
    b.lay = layout(n, real, L, x.stop_level, es);
    b.ws_off = off;
    off = align_up(off + b.lay.total, 256);
    if (check_ptrs) {
      int herr = 0;
      b.tab = P->device_tables(dev, x.dtype == MGX_F64, &herr);
      if (!b.tab) return MGX_ERR_HIP;
    }
  }
  *ws_total = off;
  return MGX_OK;
}

// Bytes of one field's statistics slot in a batch: per-level max |label|
// (kMaxLevels ints) then the overflow and non-finite counts.
constexpr size_t kStatSlot = 128;
static_assert(sizeof(int) * kMaxLevels + 2 * sizeof(unsigned long long) <= kStatSlot, "statistics slot");

// stat: the field's statistics slot (device), or null.
template <typename T>
mgx_status batch_record(const mgx_field &x, const BatchField &b, char *ws, bool dec,
                        std::vector<RecordedOp<T>> &ops, char *stat = nullptr) {
  Emitter<T> em;
  em.rec = &ops;
  char *w = ws + b.ws_off;
  if (dec) {
    if (x.labels) {  // labels written by the level kernels
      QuantArgs qa;
      Plan *P;
      mgx_status s = quant_args(x.ndim, x.dims, x.coords, x.tol_linf, x.stop_level, x.c_linf, &qa, &P);
      if (s) return s;
      if (stat) {  // the level kernels reduce their statistics there
        qa.stats_max = (int *)stat;
        qa.stats_ovf = (unsigned long long *)(stat + sizeof(int) * kMaxLevels);
        qa.stats_nan = qa.stats_ovf + 1;
      }
      return run_decompose<T>(b.P, x.stop_level, (const T *)x.in, (T *)x.out, w, b.lay, (const T *)b.tab, em,
                              x.labels, &qa);
    }
    return run_decompose<T>(b.P, x.stop_level, (const T *)x.in, (T *)x.out, w, b.lay, (const T *)b.tab, em);
  }
  const T *src = (const T *)x.in;
  if (x.labels && !x.coef) {  // coefficients read from the labels by the level kernels
    QuantArgs qa;
    Plan *P;
    mgx_status s = quant_args(x.ndim, x.dims, x.coords, x.tol_linf, x.stop_level, x.c_linf, &qa, &P);
    if (s) return s;
    return run_recompose<T>(b.P, x.stop_level, nullptr, (T *)x.out, w, b.lay, (const T *)b.tab, em, x.labels, &qa);
  }
  if (x.labels) {
    QuantArgs qa;
    Plan *P;
    mgx_status s = quant_args(x.ndim, x.dims, x.coords, x.tol_linf, x.stop_level, x.c_linf, &qa, &P);
    if (s) return s;
    OpArgs<T> o{};
    o.dj = DequantJob<T>{x.labels, (T *)x.coef, qa};
    em.begin_step(0);
    if (em.op(kOpDequantize, 0, "dequantize", -1, o) != hipSuccess) return MGX_ERR_HIP;
    em.base = 1;
    src = (const T *)x.coef;
  }
  return run_recompose<T>(b.P, x.stop_level, src, (T *)x.out, w, b.lay, (const T *)b.tab, em);
}

// Multi-field launches of one dtype: ops sorted by (step, phase, kind, key);
// each run of equal values is one launch.  Argument tables are appended to
// blob (host) at 256-byte aligned offsets.
struct BatchLaunch {
  int kind, key, n, total;
  size_t args_off, start_off;
  bool f64;
};

template <typename T>
mgx_status batch_plan(std::vector<RecordedOp<T>> ops, const Tuning &tn, std::vector<BatchLaunch> &launches,
                      std::vector<char> &blob) {
  std::vector<int> blocks(ops.size()), keys(ops.size());
  for (size_t i = 0; i < ops.size(); i++) {
    blocks[i] = op_blocks<T>(ops[i].kind, ops[i].mode, ops[i].a, tn);
    if (blocks[i] < 0) return MGX_ERR_SHAPE;
    keys[i] = op_key<T>(ops[i].kind, ops[i].mode, ops[i].a);
  }
  std::vector<size_t> idx(ops.size());
  for (size_t i = 0; i < idx.size(); i++) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
    const RecordedOp<T> &x = ops[a], &y = ops[b];
    if (x.step != y.step) return x.step < y.step;
    if (x.phase != y.phase) return x.phase < y.phase;
    if (x.kind != y.kind) return x.kind < y.kind;
    return keys[a] < keys[b];
  });
  size_t i = 0;
  while (i < idx.size()) {
    size_t j = i + 1;
    const RecordedOp<T> &h = ops[idx[i]];
    while (j < idx.size()) {
      const RecordedOp<T> &o = ops[idx[j]];
      if (o.step != h.step || o.phase != h.phase || o.kind != h.kind || keys[idx[j]] != keys[idx[i]]) break;
      j++;
    }
    BatchLaunch L{};
    L.kind = h.kind;
    L.key = keys[idx[i]];
    L.n = (int)(j - i);
    L.f64 = sizeof(T) == 8;
    L.args_off = align_up(blob.size(), 256);
    blob.resize(L.args_off + sizeof(OpArgs<T>) * L.n);
    std::vector<int> start(L.n + 1, 0);
    for (size_t k = i; k < j; k++) {
      std::memcpy(blob.data() + L.args_off + sizeof(OpArgs<T>) * (k - i), &ops[idx[k]].a, sizeof(OpArgs<T>));
      start[k - i + 1] = start[k - i] + blocks[idx[k]];
    }
    L.total = start[L.n];
    L.start_off = align_up(blob.size(), 256);
    blob.resize(L.start_off + sizeof(int) * (L.n + 1));
    std::memcpy(blob.data() + L.start_off, start.data(), sizeof(int) * (L.n + 1));
    if (L.total > 0) launches.push_back(L);
    i = j;
  }
  return MGX_OK;
}

// ---- persisted autotuning ----
// A batch's best launch shape depends on its fields' shapes, not on where
// they live, so the tuned shapes can outlive the process: with the
// environment variable MGX_TUNE_CACHE naming a file, a batch met for the
// first time looks its signature up there (a line "<signature> <target
// blocks> <min z chunk> <mid z chunk> <ms>") and is built with the shape it
// finds, without timing; a batch that is timed appends its line.  The
// signature covers the direction and, per field, the dtype, dims, stop
// level, which of labels / coefficients / statistics are used, and a hash
// of the coordinate values.  An unreadable file is ignored.
uint64_t fnv1a(const void *p, size_t n, uint64_t h) {
  const unsigned char *c = (const unsigned char *)p;
  for (size_t i = 0; i < n; i++) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

std::string batch_signature(int nfields, const mgx_field *f, bool dec) {
  uint64_t h[2] = {1469598103934665603ull, 7809847782465536322ull};  // two seeds: 128 bits
  auto put = [&](const void *p, size_t n) {
    h[0] = fnv1a(p, n, h[0]);
    h[1] = fnv1a(p, n, h[1]);
  };
  const char d = dec ? 'D' : 'R';
  put(&d, 1);
  put(&nfields, sizeof(nfields));
  for (int i = 0; i < nfields; i++) {
    const mgx_field &x = f[i];
    const int32_t v[5] = {(int32_t)x.dtype, x.ndim, x.stop_level, x.labels ? 1 : 0,
                          (x.labels && !dec && x.coef) || (dec && x.labels && x.stats) ? 1 : 0};
    put(v, sizeof(v));
    for (int a = 0; a < x.ndim && a < 3; a++) {
      put(&x.dims[a], sizeof(int64_t));
      const char has = x.coords[a] ? 1 : 0;
      put(&has, 1);
      if (x.coords[a]) put(x.coords[a], sizeof(double) * (size_t)x.dims[a]);
    }
  }
  char buf[40];
  std::snprintf(buf, sizeof(buf), "%016llx%016llx", (unsigned long long)h[0], (unsigned long long)h[1]);
  return buf;
}

// The tuned shape of a signature in the cache file, if any.
bool tune_cache_find(const std::string &sig, Tuning *tn, double *ms) {
  const char *path = std::getenv("MGX_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE *fp = std::fopen(path, "r");
  if (!fp) return false;
  char line[256];
  bool found = false;
  while (std::fgets(line, sizeof(line), fp)) {
    char key[64];
    Tuning t;
    double m = 0.0;
    if (std::sscanf(line, "%63s %d %d %d %lf", key, &t.target_blocks, &t.min_zchunk, &t.mid_zchunk, &m) == 5 &&
        sig == key && t.target_blocks > 0 && t.min_zchunk > 0 && t.mid_zchunk > 0) {
      *tn = t;  // the last matching line wins
      *ms = m;
      found = true;
    }
  }
  std::fclose(fp);
  return found;
}

void tune_cache_add(const std::string &sig, const Tuning &tn, double ms) {
  const char *path = std::getenv("MGX_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *fp = std::fopen(path, "a");
  if (!fp) return;
  std::fprintf(fp, "%s %d %d %d %.6f\n", sig.c_str(), tn.target_blocks, tn.min_zchunk, tn.mid_zchunk, ms);
  std::fclose(fp);
}

struct BatchEntry {
  hipGraphExec_t exec = nullptr;
  void *dev = nullptr;
  void *stat = nullptr;       // statistics slots of the fields that ask for them
  std::vector<int> slot;      // per field: its slot, or -1
  int nslot = 0;
  int launches = 0;
  Tuning tn{};
  double tuned_ms = 0.0;
  int tune_source = 0;        // 0 default shape, 1 timed here, 2 read from the tuning cache file
};

// A field of a decomposition batch that asks for statistics.
bool batch_wants_stats(const mgx_field &x, bool dec) { return dec && x.labels && x.stats; }

struct BatchCache {
  std::mutex mu;
  std::unordered_map<std::string, BatchEntry> map;
  std::vector<std::string> order;
  std::vector<hipStream_t> streams;  // per device: the capture / tuning stream
};
BatchCache &batch_cache() {
  static BatchCache *c = new BatchCache();
  return *c;
}
std::atomic<int> g_batch_autotune{1};
thread_local mgx_batch_info g_batch_info{};

void batch_entry_free(BatchEntry &e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.dev) (void)hipFree(e.dev);
  if (e.stat) (void)hipFree(e.stat);
  e.exec = nullptr;
  e.dev = nullptr;
  e.stat = nullptr;
}

// Records every field, plans the launches for tn, uploads the argument
// tables and captures the launches on cs into an executable graph.
mgx_status batch_build(int nfields, const mgx_field *f, const std::vector<BatchField> &bf, char *ws, bool dec,
                       const Tuning &tn, hipStream_t cs, BatchEntry &out) {
  std::vector<RecordedOp<float>> o32;
  std::vector<RecordedOp<double>> o64;
  out.slot.assign(nfields, -1);
  out.nslot = 0;
  for (int i = 0; i < nfields; i++)
    if (batch_wants_stats(f[i], dec)) out.slot[i] = out.nslot++;
  if (out.nslot > 0 && hipMalloc(&out.stat, kStatSlot * out.nslot) != hipSuccess) return MGX_ERR_HIP;
  for (int i = 0; i < nfields; i++) {
    char *stat = out.slot[i] >= 0 ? (char *)out.stat + kStatSlot * out.slot[i] : nullptr;
    mgx_status s = f[i].dtype == MGX_F32 ? batch_record<float>(f[i], bf[i], ws, dec, o32, stat)
                                         : batch_record<double>(f[i], bf[i], ws, dec, o64, stat);
    if (s) {
      batch_entry_free(out);
      return s;
    }
  }
  std::vector<BatchLaunch> launches;
  std::vector<char> blob;
  mgx_status s = batch_plan<float>(o32, tn, launches, blob);
  if (!s) s = batch_plan<double>(o64, tn, launches, blob);
  void *dev = nullptr;
  if (!s && hipMalloc(&dev, blob.size() > 0 ? blob.size() : 256) != hipSuccess) s = MGX_ERR_HIP;
  if (s) {
    batch_entry_free(out);
    return s;
  }
  if (!blob.empty() && hipMemcpy(dev, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(dev);
    batch_entry_free(out);
    return MGX_ERR_HIP;
  }
  char *d = (char *)dev;
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipFree(dev);
    batch_entry_free(out);
    return MGX_ERR_HIP;
  }
  hipError_t le = hipSuccess;
  for (const BatchLaunch &L : launches) {
    if (L.f64)
      le = launch_op_multi<double>(L.kind, L.key, (const OpArgs<double> *)(d + L.args_off),
                                   (const int *)(d + L.start_off), L.n, L.total, cs);
    else
      le = launch_op_multi<float>(L.kind, L.key, (const OpArgs<float> *)(d + L.args_off),
                                  (const int *)(d + L.start_off), L.n, L.total, cs);
    if (le != hipSuccess) break;
  }
  hipError_t ce = hipStreamEndCapture(cs, &graph);
  if (le != hipSuccess || ce != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipFree(dev);
    batch_entry_free(out);
    return MGX_ERR_HIP;
  }
  hipGraphExec_t exec = nullptr;
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    (void)hipFree(dev);
    batch_entry_free(out);
    return MGX_ERR_HIP;
  }
  out.exec = exec;
  out.dev = dev;
  out.launches = (int)launches.size();
  out.tn = tn;
  return MGX_OK;
}

// Mean time of one replay of e on cs (ms), or a negative value on error.
double batch_time(const BatchEntry &e, hipStream_t cs, int reps) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0;
  double ms = -1.0;
  if (hipGraphLaunch(e.exec, cs) == hipSuccess && hipStreamSynchronize(cs) == hipSuccess &&
      hipEventRecord(a, cs) == hipSuccess) {
    bool ok = true;
    for (int r = 0; r < reps && ok; r++) ok = hipGraphLaunch(e.exec, cs) == hipSuccess;
    float t = 0.f;
    if (ok && hipEventRecord(b, cs) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
        hipEventElapsedTime(&t, a, b) == hipSuccess)
      ms = t / reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms;
}

// The key of a batch's graph: every member the recorded launches depend on
// (never the struct's raw bytes: its padding and unused entries are
// arbitrary in a caller's struct, and the stats pointer itself may change
// from call to call; only whether it is set matters).
std::string batch_key(int nfields, const mgx_field *f, const void *ws, bool dec, const std::vector<BatchField> &bf) {
  std::string k;
  auto put = [&](const void *p, size_t n) { k.append((const char *)p, n); };
  k.push_back(dec ? 'D' : 'R');
  put(&ws, sizeof(ws));
  for (int i = 0; i < nfields; i++) {
    const mgx_field &x = f[i];
    put(&x.in, sizeof(x.in));
    put(&x.out, sizeof(x.out));
    put(&x.dtype, sizeof(x.dtype));
    put(&x.ndim, sizeof(x.ndim));
    for (int a = 0; a < x.ndim && a < 3; a++) put(&x.dims[a], sizeof(int64_t));
    put(&x.stop_level, sizeof(x.stop_level));
    put(&x.labels, sizeof(x.labels));
    if (x.labels) {
      put(&x.tol_linf, sizeof(x.tol_linf));
      put(&x.c_linf, sizeof(x.c_linf));
      if (!dec) put(&x.coef, sizeof(x.coef));
    }
    k.push_back(batch_wants_stats(x, dec) ? 'S' : '-');
    put(&bf[i].P, sizeof(Plan *));  // coordinates by content
  }
  return k;
}

mgx_status run_batched(int nfields, const mgx_field *f, void *ws, size_t ws_bytes, hipStream_t stream, bool dec) {
  std::vector<BatchField> bf;
  size_t need = 0;
  mgx_status s = batch_validate(nfields, f, dec, bf, &need);
  if (s) return s;
  if (need > 0 && (!ws || ws_bytes < need)) return MGX_ERR_WORKSPACE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MGX_ERR_HIP;
  BatchCache &C = batch_cache();
  std::lock_guard<std::mutex> g(C.mu);
  if ((int)C.streams.size() <= dev) C.streams.resize(dev + 1, nullptr);
  if (!C.streams[dev] && hipStreamCreateWithFlags(&C.streams[dev], hipStreamNonBlocking) != hipSuccess)
    return MGX_ERR_HIP;
  hipStream_t cs = C.streams[dev];
  const std::string key = batch_key(nfields, f, ws, dec, bf);
  auto it = C.map.find(key);
  Tuning cached;
  double cached_ms = 0.0;
  std::string sig;
  if (it == C.map.end() && g_batch_autotune.load()) sig = batch_signature(nfields, f, dec);
  if (it == C.map.end()) {
    BatchEntry best;
    if (!sig.empty() && tune_cache_find(sig, &cached, &cached_ms)) {
      s = batch_build(nfields, f, bf, (char *)ws, dec, cached, cs, best);
      if (s) return s;
      best.tuned_ms = cached_ms;
      best.tune_source = 2;
    } else if (g_batch_autotune.load()) {
      // candidate launch shapes of the stencil kernels; inputs must be ready
      if (hipStreamSynchronize(stream) != hipSuccess) return MGX_ERR_HIP;
      const Tuning cand[] = {{2048, 8, 8}, {512, 4, 4}, {128, 2, 2}, {8192, 8, 4}};
      double best_ms = -1.0;
      for (const Tuning &tn : cand) {
        BatchEntry e;
        s = batch_build(nfields, f, bf, (char *)ws, dec, tn, cs, e);
        if (s) {
          batch_entry_free(best);
          return s;
        }
        const double ms = batch_time(e, cs, 3);
        if (ms < 0.0) {
          batch_entry_free(e);
          batch_entry_free(best);
          return MGX_ERR_HIP;
        }
        if (best_ms < 0.0 || ms < best_ms) {
          batch_entry_free(best);
          best = e;
          best_ms = ms;
          best.tuned_ms = ms;
          best.tune_source = 1;
        } else {
          batch_entry_free(e);
        }
      }
      tune_cache_add(sig, best.tn, best_ms);
    } else {
      s = batch_build(nfields, f, bf, (char *)ws, dec, Tuning{}, cs, best);
      if (s) return s;
    }
    if (C.order.size() >= 32) {  // bounded cache: drop the oldest batch
      auto old = C.map.find(C.order.front());
      if (old != C.map.end()) {
        (void)hipStreamSynchronize(cs);
        batch_entry_free(old->second);
        C.map.erase(old);
      }
      C.order.erase(C.order.begin());
    }
    it = C.map.emplace(key, best).first;
    C.order.push_back(key);
  }
  const BatchEntry &e = it->second;
  g_batch_info.launches = e.launches;
  g_batch_info.target_blocks = e.tn.target_blocks;
  g_batch_info.min_zchunk = e.tn.min_zchunk;
  g_batch_info.tuned_ms = e.tuned_ms;
  g_batch_info.tune_source = e.tune_source;
  if (e.nslot > 0 && hipMemsetAsync(e.stat, 0, kStatSlot * e.nslot, stream) != hipSuccess) return MGX_ERR_HIP;
  hipError_t le = traced(dec ? "decompose_batched" : "recompose_batched", -2, stream,
                         [&] { return hipGraphLaunch(e.exec, stream); });
  if (le != hipSuccess || e.nslot == 0) return hip_status(le);
  // statistics (reduced by the level kernels): one read-back
  std::vector<QuantArgs> qas(nfields);
  for (int i = 0; i < nfields; i++) {
    if (e.slot[i] < 0) continue;
    Plan *P;
    if ((s = quant_args(f[i].ndim, f[i].dims, f[i].coords, f[i].tol_linf, f[i].stop_level, f[i].c_linf, &qas[i],
                        &P)))
      return s;
  }
  std::vector<char> host(kStatSlot * e.nslot);
  if (hipMemcpyAsync(host.data(), e.stat, host.size(), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return MGX_ERR_HIP;
  bool range = false;
  for (int i = 0; i < nfields; i++) {
    if (e.slot[i] < 0) continue;
    const char *h = host.data() + kStatSlot * e.slot[i];
    mgx_quant_stats *st = f[i].stats;
    std::memset(st, 0, sizeof(*st));
    st->first_level = qas[i].first;
    st->num_levels = qas[i].nlev;
    std::memcpy(st->max_abs_label, h, sizeof(int) * qas[i].nlev);
    unsigned long long ovf, nan;
    std::memcpy(&ovf, h + sizeof(int) * kMaxLevels, sizeof(ovf));
    std::memcpy(&nan, h + sizeof(int) * kMaxLevels + sizeof(ovf), sizeof(nan));
    st->n_overflow = (int64_t)ovf;
    st->n_nonfinite = (int64_t)nan;
    range = range || ovf || nan;
  }
  return range ? MGX_ERR_RANGE : MGX_OK;
}

// ---- four-axis fields (the 4-D QMCPACK field of Sec. 6, Table 2) ----
// A 4-D plan is four 1-D plans, one per axis.  Level l of the 4-D hierarchy
// (L = min_k L_k, every axis halving together) is level l + off_k of axis k's
// own hierarchy, off_k = L_k - L.
struct Plan4 {
  Plan *ax[4] = {};
  int off[4] = {};
  int64_t n[4] = {};
  int L = 0;
  int64_t m(int l, int k) const { return (n[k] - 1) / ((int64_t)1 << (L - l)) + 1; }
  int64_t count(int l) const { return m(l, 0) * m(l, 1) * m(l, 2) * m(l, 3); }
  // 1 + prod_k ||Mc^-1 R M||_inf, maximised over the levels above stop
  double linf_constant(int stop) const {
    double C = 1.0;
    for (int l = L; l > stop; l--) {
      double prod = 1.0;
      for (int k = 0; k < 4; k++) prod *= ax[k]->axis_norm[l + off[k]][2];
      if (1.0 + prod > C) C = 1.0 + prod;
    }
    return C;
  }
};

// Shape of a 4-D field: every dim 2^m + 1 (1 <= m <= 13), fewer than 2^32 nodes.
int parse_shape4(const int64_t *dims, int *L) {
  if (!dims) return MGX_ERR_SHAPE;
  int Lmin = 1 << 30;
  int64_t total = 1;
  for (int k = 0; k < 4; k++) {
    int64_t n[3];
    bool real[3];
    int Lk;
    if (parse_shape(1, &dims[k], n, real, &Lk)) return MGX_ERR_SHAPE;
    Lmin = std::min(Lmin, Lk);
    total *= dims[k];
  }
  if (total >= ((int64_t)1 << 32)) return MGX_ERR_SHAPE;  // flat 32-bit indexing
  *L = Lmin;
  return MGX_OK;
}

mgx_status get_plan4(const int64_t *dims, const double *const *coords, Plan4 *p) {
  int L;
  int st = parse_shape4(dims, &L);
  if (st) return (mgx_status)st;
  p->L = L;
  for (int k = 0; k < 4; k++) {
    const double *ck = coords ? coords[k] : nullptr;
    p->ax[k] = get_plan(1, &dims[k], ck ? &ck : nullptr, &st);
    if (!p->ax[k]) return (mgx_status)st;
    p->off[k] = p->ax[k]->L - L;
    p->n[k] = dims[k];
  }
  return MGX_OK;
}

// Workspace: the first two sweeps' outputs (A, B; later sweeps and the load
// vector reuse them) and two compact level-(L-1) boxes (C, D).
struct Layout4 {
  size_t offA = 0, offB = 0, offC = 0, offD = 0, total = 0;
};
Layout4 layout4(const int64_t n[4], int L, int stop, size_t es) {
  Layout4 w;
  if (stop >= L) return w;
  int64_t c[4];
  for (int k = 0; k < 4; k++) c[k] = (n[k] - 1) / 2 + 1;
  const int64_t a = n[0] * n[1] * n[2] * c[3], b = n[0] * n[1] * c[2] * c[3], cc = c[0] * c[1] * c[2] * c[3];
  size_t off = 0;
  w.offA = off;
  off = align_up(off + (size_t)a * es, 256);
  w.offB = off;
  off = align_up(off + (size_t)b * es, 256);
  w.offC = off;
  off = align_up(off + (size_t)cc * es, 256);
  w.offD = off;
  off = align_up(off + (size_t)cc * es, 256);
  w.total = off;
  return w;
}

template <typename T>
struct Level4 {
  AxisTab<T> ax[4];
  int64_t m[4], c[4];
};

template <typename T>
mgx_status level4_tabs(const Plan4 &P, int l, bool fp64, Level4<T> *lv) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MGX_ERR_HIP;
  for (int k = 0; k < 4; k++) {
    int herr = 0;
    const T *tab = (const T *)P.ax[k]->device_tables(dev, fp64, &herr);
    if (!tab) return MGX_ERR_HIP;
    lv->ax[k] = axis_tab(P.ax[k], l + P.off[k], 2, tab);
    lv->m[k] = lv->ax[k].m;
    lv->c[k] = lv->ax[k].c;
  }
  return MGX_OK;
}

template <typename T>
Axis4<T> axis4(const AxisTab<T> &t) {
  return Axis4<T>{t.wl, t.wr, t.w5, t.m, t.c};
}

// Chunks of the coefficient kernels' march along axis 0: about 16 M threads
// in flight on large levels, at least 16 plane pairs per chunk.
#ifndef MGX_MARCH_THREADS
#define MGX_MARCH_THREADS (1 << 24)
#endif
#ifndef MGX_MARCH_MINPAIRS
#define MGX_MARCH_MINPAIRS 16
#endif
template <typename T>
void march_chunks(Coef4Args<T> &a, int64_t c0) {
  const int64_t npair = c0 - 1;
  int64_t want = (int64_t)MGX_MARCH_THREADS / std::max<int64_t>(a.ncol, 1);
  want = std::min<int64_t>(want, std::max<int64_t>(npair / MGX_MARCH_MINPAIRS, 1));
  want = std::max<int64_t>(want, 1);
  a.jchunk = (int)std::max<int64_t>((npair + want - 1) / want, 1);
  a.nchunk = npair > 0 ? (int)((npair + a.jchunk - 1) / a.jchunk) : 1;
}

// One sweep of R M along axis k of (outer, m_k, inner) -> (outer, c_k, inner).
template <typename T>
hipError_t sweep4(const char *name, const AxisTab<T> &t, const T *in, T *out, int64_t outer, int64_t inner,
                  int level, hipStream_t st) {
  Sweep4Args<T> a{};
  a.w5 = t.w5;
  a.m = t.m;
  a.c = t.c;
  a.in = in;
  a.out = out;
  a.n = (uint32_t)(outer * t.c * inner);
  a.inner = (uint32_t)inner;
  a.dinner = make_div32((uint32_t)inner);
  a.dc = make_div32((uint32_t)t.c);
  // march form: about MGX_MARCH_THREADS threads, at least 8 outputs per chunk
  const int64_t ncol = outer * inner;
  int64_t want = std::max<int64_t>((int64_t)MGX_MARCH_THREADS / std::max<int64_t>(ncol, 1), 1);
  want = std::min<int64_t>(want, std::max<int64_t>(t.c / 8, 1));
  a.jchunk = (int)((t.c + want - 1) / want);
  a.nchunk = (int)((t.c + a.jchunk - 1) / a.jchunk);
  return traced(name, level, st, [&] { return launch_sweep4<T>(a, false, st); });
}

// Thomas solves of the coarse box (c0, c1, c2, c3) in place, axis 3 first;
// the axis-0 solve applies out = in - y when `in` is given (recomposition).
template <typename T>
hipError_t solves4(const Level4<T> &lv, T *F, const T *in, T *out, int level, hipStream_t st) {
  const int64_t c0 = lv.c[0], c1 = lv.c[1], c2 = lv.c[2], c3 = lv.c[3];
  hipError_t e;
  {
    SolveArgs<T> a{F, c0 * c1 * c2, c3, (int)c3, lv.ax[3].mult, lv.ax[3].invd, lv.ax[3].qsup};
    if ((e = traced("solve_contig", level, st, [&] { return launch_solve_contig<T>(a, st); })) != hipSuccess)
      return e;
  }
  // axis k: lines of stride sj, x over the contiguous run of the later axes,
  // `nouter` runs of stride so
  auto strided = [&](int k, int64_t sj, int64_t nouter, int mode) {
    StridedArgs<T> a{};
    a.F = F;
    a.c = (int)lv.c[k];
    a.sj = sj;
    a.nx = (int)sj;
    a.so = sj * lv.c[k];
    a.nouter = (int)nouter;
    const AxisTab<T> &t = lv.ax[k];
    a.mult = t.mult;
    a.invd = t.invd;
    a.qsup = t.qsup;
    a.multb = t.multb;
    a.invdb = t.invdb;
    a.qsub = t.qsub;
    a.mid = t.mid;
    if (mode == kSolveApply) {
      a.in = in;
      a.ij = sj;
      a.io = sj * lv.c[k];
      a.out = out;
      a.oj = sj;
      a.oo = sj * lv.c[k];
      a.sign = T(-1);
    }
    // long lines take a (runs x 256-column) grid whose second dimension is limited
    const bool twisted = a.c <= (sizeof(T) == 4 ? 257 : 129);
    if (!twisted && nouter > 65535) return hipErrorInvalidValue;
    return traced(mode == kSolveApply ? "solve_strided_apply" : "solve_strided", level, st,
                  [&] { return launch_solve_strided<T>(a, mode, st); });
  };
  if ((e = strided(2, c3, c0 * c1, kSolveInPlace)) != hipSuccess) return e;
  if ((e = strided(1, c2 * c3, c0, kSolveInPlace)) != hipSuccess) return e;
  return strided(0, c1 * c2 * c3, 1, in ? kSolveApply : kSolveInPlace);
}

// lab_r: read labels times q instead of src; lab_w: also (dst null: only)
// write the labels of the values at the destination positions.
template <typename T>
hipError_t copy4(const T *src, const int64_t sp[3], T *dst, const int64_t dp[3], const int64_t b[4], int level,
                 hipStream_t st, const int32_t *lab_r = nullptr, int32_t *lab_w = nullptr, double q = 0.0,
                 unsigned long long *rng = nullptr) {
  Copy4Args<T> a{};
  a.src = src;
  a.dst = dst;
  a.lab_r = lab_r;
  a.lab_w = lab_w;
  a.q = q;
  a.rng = rng;
  for (int k = 0; k < 3; k++) {
    a.sp[k] = sp[k];
    a.dp[k] = dp[k];
  }
  for (int k = 0; k < 4; k++) a.b[k] = (int)b[k];
  a.n = (uint32_t)(b[0] * b[1] * b[2] * b[3]);
  a.d3 = make_div32((uint32_t)b[3]);
  a.d2 = make_div32((uint32_t)b[2]);
  a.d1 = make_div32((uint32_t)b[1]);
  const char *name = lab_w ? "copy4+q" : lab_r ? "copy4_dq" : "copy4";
  return traced(name, level, st, [&] { return launch_copy4<T>(a, st); });
}

void compact_pitches(const int64_t b[4], int64_t p[3]) {
  p[2] = b[3];
  p[1] = b[2] * b[3];
  p[0] = b[1] * b[2] * b[3];
}

// Decomposition of a 4-D field, levels L .. stop+1 (Sec. 2): per level the
// coefficients, the four load-vector sweeps and the four solves, whose result
// Q_{l-1} u = Mc^{-1} (R M)^{x4} V is the next level's box.
// With labels (bin widths qa->q by level from stop), the level kernels also
// (umc null: only) write the quantization labels.
template <typename T>
mgx_status run_decompose4(const Plan4 &P, int stop, const T *u, T *umc, char *ws, const Layout4 &lay,
                          hipStream_t st, int32_t *labels = nullptr, const Quant4Args *qa = nullptr) {
  const int L = P.L;
  const int64_t N = P.count(L);
  int64_t up[3];
  compact_pitches(P.n, up);
  if (stop == L) {
    if (!labels) return hip_status(hipMemcpyAsync(umc, u, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
    return copy4<T>(u, up, umc, up, P.n, L, st, nullptr, labels, qa->q[0], qa->stats_ovf) != hipSuccess
               ? MGX_ERR_HIP
               : MGX_OK;
  }
  T *A = (T *)(ws + lay.offA), *B = (T *)(ws + lay.offB);
  const T *V = u;
  for (int l = L; l > stop; l--) {
    Level4<T> lv;
    mgx_status s = level4_tabs<T>(P, l, sizeof(T) == 8, &lv);
    if (s) return s;
    const int64_t *m = lv.m, *c = lv.c;
    Coef4Args<T> ca{};
    for (int k = 0; k < 4; k++) ca.ax[k] = axis4(lv.ax[k]);
    ca.V = V;
    ca.umc_w = umc;
    if (labels) {
      ca.lab_w = labels;
      ca.qc = qa->q[l - stop];
      ca.rng = qa->stats_ovf;  // [0] overflow, [1] non-finite (stats_nan follows it)
    }
    for (int k = 0; k < 3; k++) ca.up[k] = up[k];
    ca.ncol = (uint32_t)(m[1] * m[2] * m[3]);
    ca.d3 = make_div32((uint32_t)m[3]);
    ca.d2 = make_div32((uint32_t)m[2]);
    march_chunks(ca, c[0]);
    ca.g = A;  // the coefficient march also takes the axis-3 sweep
    if (traced(labels ? "coef4_dec+q" : "coef4_dec", l, st, [&] { return launch_coef4<T>(ca, true, st); }) !=
        hipSuccess)
      return MGX_ERR_HIP;
    if (sweep4<T>("sweep4_a2", lv.ax[2], A, B, m[0] * m[1], c[3], l, st) != hipSuccess ||
        sweep4<T>("sweep4_a1", lv.ax[1], B, A, m[0], c[2] * c[3], l, st) != hipSuccess ||
        sweep4<T>("sweep4_a0", lv.ax[0], A, B, 1, c[1] * c[2] * c[3], l, st) != hipSuccess)
      return MGX_ERR_HIP;
    if (solves4<T>(lv, B, nullptr, nullptr, l, st) != hipSuccess) return MGX_ERR_HIP;
    V = B;
  }
  int64_t b[4], bp[3];
  for (int k = 0; k < 4; k++) b[k] = P.m(stop, k);
  compact_pitches(b, bp);
  return copy4<T>(B, bp, umc, up, b, stop, st, nullptr, labels, labels ? qa->q[0] : 0.0,
                  labels ? qa->stats_ovf : nullptr) != hipSuccess
             ? MGX_ERR_HIP
             : MGX_OK;
}

// Recomposition, levels stop+1 .. L: the load vector of the level's
// coefficients (read from u_mc), the solves subtracting the correction from
// the nodal values, then coefficients plus interpolant.
// With labels, the coefficients are read as labels times their level's bin
// width instead of from umc (which may then be null).  top (progressive
// recomposition): the last level recomposed, u then receives the compact
// level-top box Q_top u; -1 means L.
template <typename T>
mgx_status run_recompose4(const Plan4 &P, int stop, const T *umc, T *u, char *ws, const Layout4 &lay,
                          hipStream_t st, const int32_t *labels = nullptr, const Quant4Args *qa = nullptr,
                          int top = -1) {
  const int L = P.L;
  const int64_t N = P.count(L);
  int64_t up[3];
  compact_pitches(P.n, up);
  if (top < 0) top = L;
  if (top < L) {
    // Q_top u: the recomposition stopped after level top, out compact
    int64_t b[4], bp[3];
    for (int k = 0; k < 4; k++) b[k] = P.m(stop, k);
    compact_pitches(b, bp);
    if (top == stop)  // the stop box itself
      return copy4<T>(umc, up, u, bp, b, stop, st, labels, nullptr, labels ? qa->q[0] : 0.0) != hipSuccess
                 ? MGX_ERR_HIP
                 : MGX_OK;
  }
  if (stop == L) {
    if (!labels) return hip_status(hipMemcpyAsync(u, umc, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
    return copy4<T>(umc, up, u, up, P.n, L, st, labels, nullptr, qa->q[0]) != hipSuccess ? MGX_ERR_HIP : MGX_OK;
  }
  T *A = (T *)(ws + lay.offA), *B = (T *)(ws + lay.offB), *C = (T *)(ws + lay.offC), *D = (T *)(ws + lay.offD);
  {
    int64_t b[4], bp[3];
    for (int k = 0; k < 4; k++) b[k] = P.m(stop, k);
    compact_pitches(b, bp);
    if (copy4<T>(umc, up, D, bp, b, stop, st, labels, nullptr, labels ? qa->q[0] : 0.0) != hipSuccess)
      return MGX_ERR_HIP;
  }
  for (int l = stop + 1; l <= top; l++) {
    Level4<T> lv;
    mgx_status s = level4_tabs<T>(P, l, sizeof(T) == 8, &lv);
    if (s) return s;
    const int64_t *m = lv.m, *c = lv.c;
    Sweep4Args<T> g{};
    g.w5 = lv.ax[3].w5;
    g.m = (int)m[3];
    g.c = (int)c[3];
    g.out = A;
    g.n = (uint32_t)(m[0] * m[1] * m[2] * c[3]);
    g.inner = 1;
    g.dinner = make_div32(1);
    g.dc = make_div32((uint32_t)c[3]);
    g.umc = umc;
    for (int k = 0; k < 3; k++) g.up[k] = up[k];
    g.m1 = (int)m[1];
    g.m2 = (int)m[2];
    for (int k = 0; k < 4; k++) g.cc[k] = (int)c[k];
    g.dm2 = make_div32((uint32_t)m[2]);
    g.dm1 = make_div32((uint32_t)m[1]);
    if (labels) {
      g.lab = labels;
      g.qc = qa->q[l - stop];
    }
    if (traced(labels ? "sweep4_gather+q" : "sweep4_gather", l, st, [&] { return launch_sweep4<T>(g, true, st); }) != hipSuccess ||
        sweep4<T>("sweep4_a2", lv.ax[2], A, B, m[0] * m[1], c[3], l, st) != hipSuccess ||
        sweep4<T>("sweep4_a1", lv.ax[1], B, A, m[0], c[2] * c[3], l, st) != hipSuccess ||
        sweep4<T>("sweep4_a0", lv.ax[0], A, B, 1, c[1] * c[2] * c[3], l, st) != hipSuccess)
      return MGX_ERR_HIP;
    if (solves4<T>(lv, B, D, C, l, st) != hipSuccess) return MGX_ERR_HIP;
    Coef4Args<T> ca{};
    for (int k = 0; k < 4; k++) ca.ax[k] = axis4(lv.ax[k]);
    ca.nodal = C;
    ca.umc_r = umc;
    if (labels) {
      ca.lab_r = labels;
      ca.qc = qa->q[l - stop];
    }
    for (int k = 0; k < 3; k++) ca.up[k] = up[k];
    ca.out = l == top ? u : D;  // the level-top box (at top = L the whole field) or the next level's nodal box
    compact_pitches(m, ca.op);
    ca.ncol = (uint32_t)(m[1] * m[2] * m[3]);
    ca.d3 = make_div32((uint32_t)m[3]);
    ca.d2 = make_div32((uint32_t)m[2]);
    march_chunks(ca, c[0]);
    if (traced(labels ? "coef4_rec+q" : "coef4_rec", l, st, [&] { return launch_coef4<T>(ca, false, st); }) !=
        hipSuccess)
      return MGX_ERR_HIP;
  }
  return MGX_OK;
}

// Validation of a 4-D decompose / recompose.
// may_null: 1 = in, 2 = out may be null (the fused calls' u_mc).
mgx_status prepare4(const void *in, void *out, mgx_dtype dtype, const int64_t *dims, const double *const *coords,
                    int stop, void *ws, size_t ws_bytes, Plan4 *P, Layout4 *lay, int may_null = 0) {
  if (dtype != MGX_F32 && dtype != MGX_F64) return MGX_ERR_ARG;
  int L;
  int st = parse_shape4(dims, &L);
  if (st) return (mgx_status)st;
  if ((!in && !(may_null & 1)) || (!out && !(may_null & 2))) return MGX_ERR_ARG;
  const size_t es = elem_size(dtype);
  const size_t bytes = (size_t)(dims[0] * dims[1] * dims[2] * dims[3]) * es;
  if (in && out && overlaps(in, bytes, out, bytes)) return MGX_ERR_ARG;
  mgx_status s = get_plan4(dims, coords, P);
  if (s) return s;
  if (stop < 0 || stop > L) return MGX_ERR_LEVEL;
  *lay = layout4(P->n, L, stop, es);
  if (lay->total > 0) {
    if (!ws || ws_bytes < lay->total) return MGX_ERR_WORKSPACE;
    if ((in && overlaps(ws, lay->total, in, bytes)) || (out && overlaps(ws, lay->total, out, bytes)))
      return MGX_ERR_ARG;
  }
  return MGX_OK;
}

mgx_status decompose4(const void *u, void *u_mc, mgx_dtype dtype, const int64_t *dims, const double *const *coords,
                      int stop, void *ws, size_t ws_bytes, hipStream_t st) {
  Plan4 P;
  Layout4 lay;
  mgx_status s = prepare4(u, u_mc, dtype, dims, coords, stop, ws, ws_bytes, &P, &lay);
  if (s) return s;
  if (dtype == MGX_F32) return run_decompose4<float>(P, stop, (const float *)u, (float *)u_mc, (char *)ws, lay, st);
  return run_decompose4<double>(P, stop, (const double *)u, (double *)u_mc, (char *)ws, lay, st);
}

mgx_status recompose4(const void *u_mc, void *u, mgx_dtype dtype, const int64_t *dims, const double *const *coords,
                      int stop, void *ws, size_t ws_bytes, hipStream_t st) {
  Plan4 P;
  Layout4 lay;
  mgx_status s = prepare4(u_mc, u, dtype, dims, coords, stop, ws, ws_bytes, &P, &lay);
  if (s) return s;
  if (dtype == MGX_F32) return run_recompose4<float>(P, stop, (const float *)u_mc, (float *)u, (char *)ws, lay, st);
  return run_recompose4<double>(P, stop, (const double *)u_mc, (double *)u, (char *)ws, lay, st);
}

// Quantization arguments of a 4-D field (Sec. 4.1): tau_in, when given,
// replaces the L-infinity schedule of tol.
mgx_status quant_args4(const int64_t *dims, const double *const *coords, double tol, int stop, double c_linf,
                       const double *tau_in, Quant4Args *qa) {
  Plan4 P;
  mgx_status s = get_plan4(dims, coords, &P);
  if (s) return s;
  const int L = P.L;
  if (stop < 0 || stop > L) return MGX_ERR_LEVEL;
  double tau[kMaxLevels];
  if (tau_in) {
    for (int i = 0; i <= L - stop; i++) {
      if (!(tau_in[i] > 0.0) || !std::isfinite(tau_in[i])) return MGX_ERR_TOL;
      tau[i] = tau_in[i];
    }
  } else {
    if (std::isnan(c_linf) || std::isinf(c_linf)) return MGX_ERR_TOL;
    if (!(tol > 0.0) || !std::isfinite(tol)) return MGX_ERR_TOL;
    s = tau_schedule(c_linf > 0.0 ? c_linf : P.linf_constant(stop), L, 4, tol, stop, tau);
    if (s) return s;
  }
  *qa = Quant4Args{};
  qa->n = (uint32_t)P.count(L);
  for (int k = 0; k < 4; k++) {
    qa->nd[k] = (int)P.n[k];
    qa->off[k] = P.ax[k]->L + 1 - L;  // log2(n_k - 1) - L
  }
  qa->d3 = make_div32((uint32_t)P.n[3]);
  qa->d2 = make_div32((uint32_t)P.n[2]);
  qa->d1 = make_div32((uint32_t)P.n[1]);
  qa->first = stop;
  qa->nlev = L + 1 - stop;
  for (int i = 0; i < qa->nlev; i++) qa->q[i] = 2.0 * tau[i];
  return MGX_OK;
}

}  // namespace
}  // namespace mgx

namespace mgx {

mgx_status decompose_placed(const void *u, void *u_mc, mgx_dtype dtype, int ndim, const int64_t *dims,
                            const double *const *coords, int stop_level, char *region, size_t region_bytes,
                            hipStream_t stream) {
  if (ndim == 4) return MGX_ERR_SHAPE;
  if (!region) return MGX_ERR_ARG;
  if (dtype != MGX_F32 && dtype != MGX_F64) return MGX_ERR_ARG;
  // the plan (host) first: its table size decides where the workspace starts
  int st = 0;
  int64_t n[3];
  bool real[3];
  int L;
  if ((st = parse_shape(ndim, dims, n, real, &L)) != 0) return (mgx_status)st;
  Plan *P = get_plan(ndim, dims, coords, &st);
  if (!P) return (mgx_status)st;
  const bool f64 = dtype == MGX_F64;
  const void *host_tab = f64 ? (const void *)P->tab64.data() : (const void *)P->tab32.data();
  const size_t tab_bytes = f64 ? P->tab64.size() * sizeof(double) : P->tab32.size() * sizeof(float);
  const size_t ws_off = align_up(tab_bytes, 256);
  if (ws_off > region_bytes) return MGX_ERR_WORKSPACE;
  Layout lay;
  const void *unused = nullptr;
  mgx_status s = prepare(u, u_mc, dtype, ndim, dims, coords, stop_level, region + ws_off, region_bytes - ws_off, &P,
                         &lay, &unused, false, 0, true);
  if (s) return s;
  if (overlaps(region, ws_off, u, (size_t)(n[0] * n[1] * n[2]) * elem_size(dtype)) ||
      overlaps(region, ws_off, u_mc, (size_t)(n[0] * n[1] * n[2]) * elem_size(dtype)))
    return MGX_ERR_ARG;
  if (hipMemcpyAsync(region, host_tab, tab_bytes, hipMemcpyHostToDevice, stream) != hipSuccess) return MGX_ERR_HIP;
  if (!f64) {
    Emitter<float> em;
    em.st = stream;
    em.untraced = true;
    return run_decompose<float>(P, stop_level, (const float *)u, (float *)u_mc, region + ws_off, lay,
                                (const float *)region, em);
  }
  Emitter<double> em;
  em.st = stream;
  em.untraced = true;
  return run_decompose<double>(P, stop_level, (const double *)u, (double *)u_mc, region + ws_off, lay,
                               (const double *)region, em);
}

// The 4-D gather of mgx_pad and mgx_crop: dst (ddims) node j takes src
// (sdims) node min(j, sdims - 1) per axis.
template <typename T>
Pad4Args<T> pad4_args(const T *src, T *dst, const int64_t *sdims, const int64_t *ddims) {
  Pad4Args<T> a{};
  a.src = src;
  a.dst = dst;
  for (int k = 0; k < 4; k++) {
    a.nsrc[k] = (int)sdims[k];
    a.ndst[k] = (int)ddims[k];
  }
  a.n = (uint32_t)(ddims[0] * ddims[1] * ddims[2] * ddims[3]);
  a.d3 = make_div32((uint32_t)ddims[3]);
  a.d2 = make_div32((uint32_t)ddims[2]);
  a.d1 = make_div32((uint32_t)ddims[1]);
  return a;
}

}  // namespace mgx

using namespace mgx;

extern "C" {

const char *mgx_status_string(mgx_status s) {
  switch (s) {
    case MGX_OK: return "ok";
    case MGX_ERR_ARG: return "invalid argument";
    case MGX_ERR_SHAPE: return "invalid shape (ndim 1..4, each dim 2^m+1 with 1<=m<=13)";
    case MGX_ERR_COORDS: return "coordinates not finite or not strictly increasing";
    case MGX_ERR_LEVEL: return "stop level out of range";
    case MGX_ERR_TOL: return "invalid tolerance or L-infinity constant";
    case MGX_ERR_RANGE: return "quantization label out of int32 range or non-finite coefficient";
    case MGX_ERR_WORKSPACE: return "workspace missing or too small";
    case MGX_ERR_HIP: return "HIP runtime error";
    default: break;
  }
  return "unknown status";
}

int mgx_num_levels(int ndim, const int64_t *dims) {
  if (ndim == 4) {
    int L4;
    int st4 = parse_shape4(dims, &L4);
    return st4 ? -st4 : L4;
  }
  int64_t n[3];
  bool real[3];
  int L;
  int st = parse_shape(ndim, dims, n, real, &L);
  return st ? -st : L;
}

size_t mgx_workspace_size(mgx_dtype dtype, int ndim, const int64_t *dims, int stop_level) {
  if (dtype != MGX_F32 && dtype != MGX_F64) return 0;
  if (ndim == 4) {
    int L4;
    if (parse_shape4(dims, &L4) || stop_level < 0 || stop_level > L4) return 0;
    return layout4(dims, L4, stop_level, elem_size(dtype)).total;
  }
  int64_t n[3];
  bool real[3];
  int L;
  if (parse_shape(ndim, dims, n, real, &L)) return 0;
  if (stop_level < 0 || stop_level > L) return 0;
  return layout(n, real, L, stop_level, elem_size(dtype)).total;
}

mgx_status mgx_decompose(const void *u, void *u_mc, mgx_dtype dtype, int ndim, const int64_t *dims,
                         const double *const *coords, int stop_level, void *workspace, size_t workspace_bytes,
                         hipStream_t stream) {
  if (ndim == 4) return decompose4(u, u_mc, dtype, dims, coords, stop_level, workspace, workspace_bytes, stream);
  Plan *P;
  Layout lay;
  const void *tab;
  mgx_status s = prepare(u, u_mc, dtype, ndim, dims, coords, stop_level, workspace, workspace_bytes, &P, &lay, &tab);
  if (s) return s;
  if (dtype == MGX_F32) {
    Emitter<float> em;
    em.st = stream;
    return run_decompose<float>(P, stop_level, (const float *)u, (float *)u_mc, (char *)workspace, lay,
                                (const float *)tab, em);
  }
  Emitter<double> em;
  em.st = stream;
  return run_decompose<double>(P, stop_level, (const double *)u, (double *)u_mc, (char *)workspace, lay,
                               (const double *)tab, em);
}

mgx_status mgx_recompose(const void *u_mc, void *u, mgx_dtype dtype, int ndim, const int64_t *dims,
                         const double *const *coords, int stop_level, void *workspace, size_t workspace_bytes,
                         hipStream_t stream) {
  if (ndim == 4) return recompose4(u_mc, u, dtype, dims, coords, stop_level, workspace, workspace_bytes, stream);
  Plan *P;
  Layout lay;
  const void *tab;
  mgx_status s = prepare(u_mc, u, dtype, ndim, dims, coords, stop_level, workspace, workspace_bytes, &P, &lay, &tab);
  if (s) return s;
  if (dtype == MGX_F32) {
    Emitter<float> em;
    em.st = stream;
    return run_recompose<float>(P, stop_level, (const float *)u_mc, (float *)u, (char *)workspace, lay,
                                (const float *)tab, em);
  }
  Emitter<double> em;
  em.st = stream;
  return run_recompose<double>(P, stop_level, (const double *)u_mc, (double *)u, (char *)workspace, lay,
                               (const double *)tab, em);
}

mgx_status mgx_recompose_to(const void *u_mc, void *u_t, mgx_dtype dtype, int ndim, const int64_t *dims,
                            const double *const *coords, int stop_level, int target_level, void *workspace,
                            size_t workspace_bytes, hipStream_t stream) {
  if (ndim == 4) {
    Plan4 P4;
    Layout4 lay4;
    mgx_status s4 = prepare4(u_mc, nullptr, dtype, dims, coords, stop_level, workspace, workspace_bytes, &P4, &lay4, 2);
    if (s4) return s4;
    if (target_level < stop_level || target_level > P4.L) return MGX_ERR_LEVEL;
    if (!u_t) return MGX_ERR_ARG;
    const size_t es = elem_size(dtype);
    const size_t in_bytes = (size_t)P4.count(P4.L) * es, out_bytes = (size_t)P4.count(target_level) * es;
    if (overlaps(u_t, out_bytes, u_mc, in_bytes) || (lay4.total > 0 && overlaps(u_t, out_bytes, workspace, lay4.total)))
      return MGX_ERR_ARG;
    if (dtype == MGX_F32)
      return run_recompose4<float>(P4, stop_level, (const float *)u_mc, (float *)u_t, (char *)workspace, lay4, stream,
                                   nullptr, nullptr, target_level);
    return run_recompose4<double>(P4, stop_level, (const double *)u_mc, (double *)u_t, (char *)workspace, lay4,
                                  stream, nullptr, nullptr, target_level);
  }
  Plan *P;
  Layout lay;
  const void *tab;
  mgx_status s = prepare(u_mc, nullptr, dtype, ndim, dims, coords, stop_level, workspace, workspace_bytes, &P, &lay,
                         &tab, false, 2);
  if (s) return s;
  if (target_level < stop_level || target_level > P->L) return MGX_ERR_LEVEL;
  if (!u_t) return MGX_ERR_ARG;
  const size_t es = elem_size(dtype);
  const size_t in_bytes = (size_t)(P->n[0] * P->n[1] * P->n[2]) * es;
  int64_t tm[3];
  level_box(P, target_level, tm);
  const size_t out_bytes = (size_t)(tm[0] * tm[1] * tm[2]) * es;
  if (overlaps(u_t, out_bytes, u_mc, in_bytes) || (lay.total > 0 && overlaps(u_t, out_bytes, workspace, lay.total)))
    return MGX_ERR_ARG;
  if (dtype == MGX_F32) {
    Emitter<float> em;
    em.st = stream;
    return run_recompose<float>(P, stop_level, (const float *)u_mc, (float *)u_t, (char *)workspace, lay,
                                (const float *)tab, em, nullptr, nullptr, target_level);
  }
  Emitter<double> em;
  em.st = stream;
  return run_recompose<double>(P, stop_level, (const double *)u_mc, (double *)u_t, (char *)workspace, lay,
                               (const double *)tab, em, nullptr, nullptr, target_level);
}

mgx_status mgx_decompose_adaptive(const void *u, void *u_mc, mgx_dtype dtype, int ndim, const int64_t *dims,
                                  const double *const *coords, double tol_linf, double c_linf, int *stop_level_out,
                                  void *workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!stop_level_out) return MGX_ERR_ARG;
  Plan *P;
  Layout lay;
  const void *tab;
  mgx_status s = prepare(u, u_mc, dtype, ndim, dims, coords, 0, workspace, workspace_bytes, &P, &lay, &tab);
  if (s) return s;
  if (ndim != 3 || !P->real[0]) return MGX_ERR_SHAPE;
  double tau[kMaxLevels];
  if ((s = tolerances(P, ndim, tol_linf, P->L, c_linf, tau))) return s;
  int dev = 0, herr = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MGX_ERR_HIP;
  const double *tab64 = (const double *)P->device_tables(dev, true, &herr);
  if (!tab64) return MGX_ERR_HIP;
  if (P->L < 1) {  // nothing to decompose
    *stop_level_out = 0;
    return hipMemcpyAsync(u_mc, u, (size_t)(P->n[0] * P->n[1] * P->n[2]) * elem_size(dtype),
                          hipMemcpyDeviceToDevice, stream) == hipSuccess
               ? MGX_OK
               : MGX_ERR_HIP;
  }
  if (dtype == MGX_F32)
    return run_decompose_adaptive<float>(P, ndim, (const float *)u, (float *)u_mc, tol_linf, c_linf,
                                         (char *)workspace, lay, (const float *)tab, tab64, stream, stop_level_out);
  return run_decompose_adaptive<double>(P, ndim, (const double *)u, (double *)u_mc, tol_linf, c_linf,
                                        (char *)workspace, lay, (const double *)tab, tab64, stream, stop_level_out);
}

mgx_status mgx_adaptive_estimate(const void *v, mgx_dtype dtype, int ndim, const int64_t *dims,
                                 const double *const *coords, int level, double *sums_out, int64_t *counts_out,
                                 void *workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!v || !sums_out || !counts_out || (dtype != MGX_F32 && dtype != MGX_F64)) return MGX_ERR_ARG;
  int st = 0;
  Plan *P = get_plan(ndim, dims, coords, &st);
  if (!P) return (mgx_status)st;
  if (ndim != 3 || !P->real[0]) return MGX_ERR_SHAPE;
  if (level < 1 || level > P->L) return MGX_ERR_LEVEL;
  const size_t need = mgx_adaptive_workspace_size(ndim, dims);
  if (!workspace || workspace_bytes < need) return MGX_ERR_WORKSPACE;
  int64_t m[3];
  level_box(P, level, m);
  if (overlaps(workspace, need, v, (size_t)(m[0] * m[1] * m[2]) * elem_size(dtype))) return MGX_ERR_ARG;
  int dev = 0, herr = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MGX_ERR_HIP;
  const double *tab64 = (const double *)P->device_tables(dev, true, &herr);
  if (!tab64) return MGX_ERR_HIP;
  int nbk[3];
  const int nwg = estimate_workgroups(estimate_blocks(P, level, nbk, counts_out));
  double *part = (double *)workspace, *sums = part + 2 * (int64_t)nwg;
  const mgx_status s = dtype == MGX_F32 ? enqueue_estimate<float>(P, level, (const float *)v, m[1] * m[2], m[2], tab64, part, sums,
                                                 nullptr, true, 0.0, stream)
                                        : enqueue_estimate<double>(P, level, (const double *)v, m[1] * m[2], m[2],
                                                                   tab64, part, sums, nullptr, true, 0.0, stream);
  if (s) return s;
  double h[2];
  if (hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return MGX_ERR_HIP;
  sums_out[0] = h[0];
  sums_out[1] = h[1];
  return MGX_OK;
}

mgx_status mgx_dyadic_dims(int ndim, const int64_t *dims, int64_t *padded_out) {
  if (ndim < 1 || ndim > 4 || !dims || !padded_out) return MGX_ERR_ARG;
  for (int k = 0; k < ndim; k++) {
    if (dims[k] < 2 || dims[k] > ((int64_t)1 << 30) + 1) return MGX_ERR_SHAPE;
    int64_t p = 3;
    while (p < dims[k]) p = 2 * p - 1;  // 2^m + 1 -> 2^(m+1) + 1
    padded_out[k] = p;
  }
  return MGX_OK;
}

// Box extents of dims padded to three axes (leading axes of 1).
static void box3(int ndim, const int64_t *d, int64_t out[3]) {
  for (int k = 0; k < 3; k++) {
    const int src = k - (3 - ndim);
    out[k] = src >= 0 ? d[src] : 1;
  }
}

mgx_status mgx_pad(const void *u, void *u_pad, mgx_dtype dtype, int ndim, const int64_t *dims,
                   hipStream_t stream) {
  if (!u || !u_pad || (dtype != MGX_F32 && dtype != MGX_F64)) return MGX_ERR_ARG;
  int64_t pd[4];
  mgx_status s = mgx_dyadic_dims(ndim, dims, pd);
  if (s) return s;
  if (ndim == 4) {
    const int64_t nn = dims[0] * dims[1] * dims[2] * dims[3], pn = pd[0] * pd[1] * pd[2] * pd[3];
    const size_t es = elem_size(dtype);
    if (pn >= ((int64_t)1 << 32) || overlaps(u, (size_t)nn * es, u_pad, (size_t)pn * es)) return MGX_ERR_ARG;
    return hip_status(dtype == MGX_F32 ? launch_pad4<float>(pad4_args((const float *)u, (float *)u_pad, dims, pd), stream)
                                       : launch_pad4<double>(pad4_args((const double *)u, (double *)u_pad, dims, pd),
                                                             stream));
  }
  int64_t n[3], p[3];
  box3(ndim, dims, n);
  box3(ndim, pd, p);
  const size_t es = elem_size(dtype);
  if ((p[0] * p[1] * p[2]) > INT32_MAX || overlaps(u, (size_t)(n[0] * n[1] * n[2]) * es, u_pad,
                                                   (size_t)(p[0] * p[1] * p[2]) * es))
    return MGX_ERR_ARG;
  hipError_t e;
  if (dtype == MGX_F32)
    e = launch_pad_edge<float>(PadArgs<float>{(const float *)u, (float *)u_pad, (int)n[0], (int)n[1], (int)n[2],
                                              (int)p[0], (int)p[1], (int)p[2]},
                               stream);
  else
    e = launch_pad_edge<double>(PadArgs<double>{(const double *)u, (double *)u_pad, (int)n[0], (int)n[1], (int)n[2],
                                                (int)p[0], (int)p[1], (int)p[2]},
                                stream);
  return hip_status(e);
}

mgx_status mgx_crop(const void *u_pad, void *u, mgx_dtype dtype, int ndim, const int64_t *dims,
                    hipStream_t stream) {
  if (!u || !u_pad || (dtype != MGX_F32 && dtype != MGX_F64)) return MGX_ERR_ARG;
  int64_t pd[4];
  mgx_status s = mgx_dyadic_dims(ndim, dims, pd);
  if (s) return s;
  if (ndim == 4) {
    const int64_t nn = dims[0] * dims[1] * dims[2] * dims[3], pn = pd[0] * pd[1] * pd[2] * pd[3];
    const size_t es = elem_size(dtype);
    if (pn >= ((int64_t)1 << 32) || overlaps(u, (size_t)nn * es, u_pad, (size_t)pn * es)) return MGX_ERR_ARG;
    return hip_status(dtype == MGX_F32
                          ? launch_pad4<float>(pad4_args((const float *)u_pad, (float *)u, pd, dims), stream)
                          : launch_pad4<double>(pad4_args((const double *)u_pad, (double *)u, pd, dims), stream));
  }
  int64_t n[3], p[3];
  box3(ndim, dims, n);
  box3(ndim, pd, p);
  const size_t es = elem_size(dtype);
  if ((p[0] * p[1] * p[2]) > INT32_MAX || overlaps(u, (size_t)(n[0] * n[1] * n[2]) * es, u_pad,
                                                   (size_t)(p[0] * p[1] * p[2]) * es))
    return MGX_ERR_ARG;
  hipError_t e;
  if (dtype == MGX_F32)
    e = launch_copy_box<float>(CopyArgs<float>{(const float *)u_pad, p[1] * p[2], p[2], (float *)u, n[1] * n[2], n[2],
                                               (int)n[0], (int)n[1], (int)n[2]},
                               stream);
  else
    e = launch_copy_box<double>(CopyArgs<double>{(const double *)u_pad, p[1] * p[2], p[2], (double *)u, n[1] * n[2],
                                                 n[2], (int)n[0], (int)n[1], (int)n[2]},
                                stream);
  return hip_status(e);
}

size_t mgx_adaptive_workspace_size(int ndim, const int64_t *dims) {
  int64_t n[3];
  bool real[3];
  int L;
  if (parse_shape(ndim, dims, n, real, &L)) return 0;
  int64_t nb = 1;
  for (int k = 0; k < 3; k++) {
    const int64_t cells = real[k] ? (n[k] - 1) / 2 : 0;
    nb *= cells > 1 ? (cells - 2) / 4 + 1 : 1;
  }
  // per-workgroup sums of the finest level, then the two totals
  return (size_t)(((nb + kEstimateThreads - 1) / kEstimateThreads) * 2 + 2) * sizeof(double);
}

size_t mgx_adjoint_workspace_size(mgx_dtype dtype, int ndim, const int64_t *dims, int stop_level) {
  if (dtype != MGX_F32 && dtype != MGX_F64) return 0;
  int64_t n[3];
  bool real[3];
  int L;
  if (parse_shape(ndim, dims, n, real, &L)) return 0;
  if (stop_level < 0 || stop_level > L) return 0;
  return layout(n, real, L, stop_level, elem_size(dtype), true).total;
}

mgx_status mgx_decompose_adjoint(const void *g_mc, void *g_u, mgx_dtype dtype, int ndim, const int64_t *dims,
                                 const double *const *coords, int stop_level, void *workspace,
                                 size_t workspace_bytes, hipStream_t stream) {
  Plan *P;
  Layout lay;
  const void *tab;
  mgx_status s = prepare(g_mc, g_u, dtype, ndim, dims, coords, stop_level, workspace, workspace_bytes, &P, &lay,
                         &tab, true);
  if (s) return s;
  if (dtype == MGX_F32)
    return run_decompose_adjoint<float>(P, stop_level, (const float *)g_mc, (float *)g_u, (char *)workspace, lay,
                                        (const float *)tab, stream);
  return run_decompose_adjoint<double>(P, stop_level, (const double *)g_mc, (double *)g_u, (char *)workspace, lay,
                                       (const double *)tab, stream);
}

mgx_status mgx_recompose_adjoint(const void *g_u, void *g_mc, mgx_dtype dtype, int ndim, const int64_t *dims,
                                 const double *const *coords, int stop_level, void *workspace,
                                 size_t workspace_bytes, hipStream_t stream) {
  Plan *P;
  Layout lay;
  const void *tab;
  mgx_status s = prepare(g_u, g_mc, dtype, ndim, dims, coords, stop_level, workspace, workspace_bytes, &P, &lay,
                         &tab, true);
  if (s) return s;
  if (dtype == MGX_F32)
    return run_recompose_adjoint<float>(P, stop_level, (const float *)g_u, (float *)g_mc, (char *)workspace, lay,
                                        (const float *)tab, stream);
  return run_recompose_adjoint<double>(P, stop_level, (const double *)g_u, (double *)g_mc, (char *)workspace, lay,
                                       (const double *)tab, stream);
}

// 4-D quantization; with stats, the per-level maxima and the out-of-range
// counts come back like those of the 3-D pass.
static mgx_status quantize4_common(const void *u_mc, int32_t *labels, mgx_dtype dtype, const int64_t *dims,
                                   const double *const *coords, double tol_linf, int stop_level, double c_linf,
                                   const double *tau_in, mgx_quant_stats *stats, hipStream_t stream) {
  int L4;
  int st4 = parse_shape4(dims, &L4);
  if (st4) return (mgx_status)st4;
  if (!u_mc || !labels) return MGX_ERR_ARG;
  const size_t cnt = (size_t)(dims[0] * dims[1] * dims[2] * dims[3]);
  if (overlaps(u_mc, cnt * elem_size(dtype), labels, cnt * 4)) return MGX_ERR_ARG;
  Quant4Args qa;
  mgx_status s = quant_args4(dims, coords, tol_linf, stop_level, c_linf, tau_in, &qa);
  if (s) return s;
  if (!stats) {
    hipError_t e = traced("quantize4", -1, stream, [&] {
      return dtype == MGX_F32 ? launch_quantize4<float>((const float *)u_mc, labels, qa, stream)
                              : launch_quantize4<double>((const double *)u_mc, labels, qa, stream);
    });
    return hip_status(e);
  }
  std::lock_guard<std::mutex> g(stats_buf().mu);
  char *base = stats_device(stream);
  if (!base) return MGX_ERR_HIP;
  qa.stats_max = (int *)base;
  qa.stats_ovf = (unsigned long long *)(base + sizeof(int) * kMaxLevels);
  qa.stats_nan = qa.stats_ovf + 1;
  hipError_t e = traced("quantize4_stats", -1, stream, [&] {
    return dtype == MGX_F32 ? launch_quantize4<float>((const float *)u_mc, labels, qa, stream)
                            : launch_quantize4<double>((const double *)u_mc, labels, qa, stream);
  });
  if (e != hipSuccess) return MGX_ERR_HIP;
  return stats_read(base, qa.first, qa.nlev, stats, stream);
}

static mgx_status quantize_common(const void *u_mc, int32_t *labels, mgx_dtype dtype, int ndim,
                                  const int64_t *dims, const double *const *coords, double tol_linf,
                                  int stop_level, double c_linf, const double *tau_in, mgx_quant_stats *stats,
                                  hipStream_t stream) {
  if (dtype != MGX_F32 && dtype != MGX_F64) return MGX_ERR_ARG;
  if (ndim == 4) return quantize4_common(u_mc, labels, dtype, dims, coords, tol_linf, stop_level, c_linf, tau_in,
                                         stats, stream);
  int64_t n[3];
  bool real[3];
  int L;
  int st = parse_shape(ndim, dims, n, real, &L);
  if (st) return (mgx_status)st;
  if (!u_mc || !labels) return MGX_ERR_ARG;
  const size_t cnt = (size_t)(n[0] * n[1] * n[2]);
  if (overlaps(u_mc, cnt * elem_size(dtype), labels, cnt * 4)) return MGX_ERR_ARG;
  QuantArgs qa;
  Plan *P;
  mgx_status s = quant_args(ndim, dims, coords, tol_linf, stop_level, c_linf, &qa, &P, tau_in);
  if (s) return s;
  if (!stats) {
    hipError_t e = traced("quantize", -1, stream, [&] {
      return dtype == MGX_F32 ? launch_quantize<float>((const float *)u_mc, labels, qa, false, stream)
                              : launch_quantize<double>((const double *)u_mc, labels, qa, false, stream);
    });
    return hip_status(e);
  }
  std::lock_guard<std::mutex> g(stats_buf().mu);
  char *base = stats_device(stream);
  if (!base) return MGX_ERR_HIP;
  qa.stats_max = (int *)base;
  qa.stats_ovf = (unsigned long long *)(base + sizeof(int) * kMaxLevels);
  qa.stats_nan = qa.stats_ovf + 1;
  hipError_t e = traced("quantize_stats", -1, stream, [&] {
    return dtype == MGX_F32 ? launch_quantize<float>((const float *)u_mc, labels, qa, true, stream)
                            : launch_quantize<double>((const double *)u_mc, labels, qa, true, stream);
  });
  if (e != hipSuccess) return MGX_ERR_HIP;
  return stats_read(base, qa.first, qa.nlev, stats, stream);
}

static mgx_status dequantize_common(const int32_t *labels, void *u_mc, mgx_dtype dtype, int ndim,
                                    const int64_t *dims, const double *const *coords, double tol_linf,
                                    int stop_level, double c_linf, const double *tau_in, hipStream_t stream) {
  if (dtype != MGX_F32 && dtype != MGX_F64) return MGX_ERR_ARG;
  if (ndim == 4) {
    int L4;
    int st4 = parse_shape4(dims, &L4);
    if (st4) return (mgx_status)st4;
    if (!u_mc || !labels) return MGX_ERR_ARG;
    const size_t cnt = (size_t)(dims[0] * dims[1] * dims[2] * dims[3]);
    if (overlaps(u_mc, cnt * elem_size(dtype), labels, cnt * 4)) return MGX_ERR_ARG;
    Quant4Args qa;
    mgx_status s4 = quant_args4(dims, coords, tol_linf, stop_level, c_linf, tau_in, &qa);
    if (s4) return s4;
    hipError_t e = traced("dequantize4", -1, stream, [&] {
      return dtype == MGX_F32 ? launch_dequantize4<float>(labels, (float *)u_mc, qa, stream)
                              : launch_dequantize4<double>(labels, (double *)u_mc, qa, stream);
    });
    return hip_status(e);
  }
  int64_t n[3];
  bool real[3];
  int L;
  int st = parse_shape(ndim, dims, n, real, &L);
  if (st) return (mgx_status)st;
  if (!u_mc || !labels) return MGX_ERR_ARG;
  const size_t cnt = (size_t)(n[0] * n[1] * n[2]);
  if (overlaps(u_mc, cnt * elem_size(dtype), labels, cnt * 4)) return MGX_ERR_ARG;
  QuantArgs qa;
  Plan *P;
  mgx_status s = quant_args(ndim, dims, coords, tol_linf, stop_level, c_linf, &qa, &P, tau_in);
  if (s) return s;
  hipError_t e = traced("dequantize", -1, stream, [&] {
    return dtype == MGX_F32 ? launch_dequantize<float>(labels, (float *)u_mc, qa, stream)
                            : launch_dequantize<double>(labels, (double *)u_mc, qa, stream);
  });
  return hip_status(e);
}

mgx_status mgx_quantize(const void *u_mc, int32_t *labels, mgx_dtype dtype, int ndim, const int64_t *dims,
                        const double *const *coords, double tol_linf, int stop_level, double c_linf,
                        mgx_quant_stats *stats, hipStream_t stream) {
  return quantize_common(u_mc, labels, dtype, ndim, dims, coords, tol_linf, stop_level, c_linf, nullptr, stats,
                         stream);
}

mgx_status mgx_dequantize(const int32_t *labels, void *u_mc, mgx_dtype dtype, int ndim, const int64_t *dims,
                          const double *const *coords, double tol_linf, int stop_level, double c_linf,
                          hipStream_t stream) {
  return dequantize_common(labels, u_mc, dtype, ndim, dims, coords, tol_linf, stop_level, c_linf, nullptr, stream);
}

mgx_status mgx_quantize_levels(const void *u_mc, int32_t *labels, mgx_dtype dtype, int ndim, const int64_t *dims,
                               const double *const *coords, int stop_level, const double *tau,
                               mgx_quant_stats *stats, hipStream_t stream) {
  if (!tau) return MGX_ERR_ARG;
  return quantize_common(u_mc, labels, dtype, ndim, dims, coords, 1.0, stop_level, 0.0, tau, stats, stream);
}

mgx_status mgx_dequantize_levels(const int32_t *labels, void *u_mc, mgx_dtype dtype, int ndim, const int64_t *dims,
                                 const double *const *coords, int stop_level, const double *tau,
                                 hipStream_t stream) {
  if (!tau) return MGX_ERR_ARG;
  return dequantize_common(labels, u_mc, dtype, ndim, dims, coords, 1.0, stop_level, 0.0, tau, stream);
}

size_t mgx_label_entropy_workspace_size(int ndim, const int64_t *dims, int stop_level) {
  if (ndim == 4) {
    int L4;
    if (parse_shape4(dims, &L4) || stop_level < 0 || stop_level > L4) return 0;
    return entropy_workspace(dims[0] * dims[1] * dims[2] * dims[3], L4 + 1 - stop_level);
  }
  int64_t n[3];
  bool real[3];
  int L;
  if (parse_shape(ndim, dims, n, real, &L) || stop_level < 0 || stop_level > L) return 0;
  return entropy_workspace(n[0] * n[1] * n[2], L + 1 - stop_level);
}

// known_max: host, the quantizer's per-level maxima, or null.
static mgx_status entropy_common(const int32_t *labels, int ndim, const int64_t *dims, int stop_level,
                                 double *bits_out, void *workspace, size_t workspace_bytes, const int32_t *known_max,
                                 hipStream_t stream) {
  if (!labels || !bits_out) return MGX_ERR_ARG;
  if (ndim == 4) {
    int L4;
    int st4 = parse_shape4(dims, &L4);
    if (st4) return (mgx_status)st4;
    if (stop_level < 0 || stop_level > L4) return MGX_ERR_LEVEL;
    const int64_t cnt4 = dims[0] * dims[1] * dims[2] * dims[3];
    const size_t need4 = entropy_workspace(cnt4, L4 + 1 - stop_level);
    if (need4 == 0) return MGX_ERR_SHAPE;
    if (!workspace || workspace_bytes < need4) return MGX_ERR_WORKSPACE;
    if (overlaps(workspace, need4, labels, (size_t)cnt4 * 4)) return MGX_ERR_ARG;
    double ones4[kMaxLevels];
    for (int i = 0; i < kMaxLevels; i++) ones4[i] = 1.0;
    Quant4Args qa4;
    mgx_status s4 = quant_args4(dims, nullptr, 1.0, stop_level, 0.0, ones4, &qa4);
    if (s4) return s4;
    Plan4 P4;
    if ((s4 = get_plan4(dims, nullptr, &P4))) return s4;
    int64_t count4[kMaxLevels], prev4 = 0;
    for (int l = stop_level; l <= L4; l++) {
      count4[l - stop_level] = P4.count(l) - prev4;
      prev4 = P4.count(l);
    }
    return hip_status(label_entropy(labels, qa4, count4, (char *)workspace, stream, bits_out, known_max));
  }
  int64_t n[3];
  bool real[3];
  int L;
  int st = parse_shape(ndim, dims, n, real, &L);
  if (st) return (mgx_status)st;
  if (stop_level < 0 || stop_level > L) return MGX_ERR_LEVEL;
  const int64_t cnt = n[0] * n[1] * n[2];
  const size_t need = entropy_workspace(cnt, L + 1 - stop_level);
  if (need == 0) return MGX_ERR_SHAPE;
  if (!workspace || workspace_bytes < need) return MGX_ERR_WORKSPACE;
  if (overlaps(workspace, need, labels, (size_t)cnt * 4)) return MGX_ERR_ARG;
  double ones[kMaxLevels];
  for (int i = 0; i < kMaxLevels; i++) ones[i] = 1.0;
  QuantArgs qa;
  Plan *P;
  mgx_status s = quant_args(ndim, dims, nullptr, 1.0, stop_level, 0.0, &qa, &P, ones);
  if (s) return s;
  // labels per level: the stop level's whole box, then each finer level's new nodes
  int64_t count[kMaxLevels], prev = 0;
  for (int l = stop_level; l <= L; l++) {
    int64_t m[3];
    level_box(P, l, m);
    const int64_t box = m[0] * m[1] * m[2];
    count[l - stop_level] = box - prev;
    prev = box;
  }
  return hip_status(label_entropy(labels, qa, count, (char *)workspace, stream, bits_out, known_max));
}

mgx_status mgx_label_entropy(const int32_t *labels, int ndim, const int64_t *dims, int stop_level, double *bits_out,
                             void *workspace, size_t workspace_bytes, hipStream_t stream) {
  return entropy_common(labels, ndim, dims, stop_level, bits_out, workspace, workspace_bytes, nullptr, stream);
}

mgx_status mgx_label_entropy_bounded(const int32_t *labels, int ndim, const int64_t *dims, int stop_level,
                                     const mgx_quant_stats *stats, double *bits_out, void *workspace,
                                     size_t workspace_bytes, hipStream_t stream) {
  if (!stats) return MGX_ERR_ARG;
  const int L = mgx_num_levels(ndim, dims);
  if (L < 0) return (mgx_status)-L;
  if (stop_level < 0 || stop_level > L) return MGX_ERR_LEVEL;
  // statistics of another stop level, or with out-of-range labels (left out
  // of the maxima): the maxima are found on the labels instead
  bool use = stats->first_level == stop_level && stats->num_levels == L + 1 - stop_level &&
             stats->n_overflow == 0 && stats->n_nonfinite == 0;
  for (int i = 0; use && i < stats->num_levels; i++)
    if (stats->max_abs_label[i] < 0) use = false;
  return entropy_common(labels, ndim, dims, stop_level, bits_out, workspace, workspace_bytes,
                        use ? stats->max_abs_label : nullptr, stream);
}

double mgx_linf_constant(int ndim, const int64_t *dims, const double *const *coords, int stop_level) {
  if (ndim == 4) {
    Plan4 P4;
    if (get_plan4(dims, coords, &P4) || stop_level < 0 || stop_level > P4.L) return -1.0;
    return P4.linf_constant(stop_level);
  }
  int st = 0;
  Plan *P = get_plan(ndim, dims, coords, &st);
  if (!P || stop_level < 0 || stop_level > P->L) return -1.0;
  return P->linf_constant(stop_level);
}

mgx_status mgx_level_tolerances(int ndim, const int64_t *dims, const double *const *coords, double tol_linf,
                                int stop_level, double c_linf, double *tau_out) {
  if (!tau_out) return MGX_ERR_ARG;
  if (ndim == 4) {
    Plan4 P4;
    mgx_status s4 = get_plan4(dims, coords, &P4);
    if (s4) return s4;
    if (stop_level < 0 || stop_level > P4.L) return MGX_ERR_LEVEL;
    if (std::isnan(c_linf) || std::isinf(c_linf)) return MGX_ERR_TOL;
    if (!(tol_linf > 0.0) || !std::isfinite(tol_linf)) return MGX_ERR_TOL;
    return tau_schedule(c_linf > 0.0 ? c_linf : P4.linf_constant(stop_level), P4.L, 4, tol_linf, stop_level,
                        tau_out);
  }
  int st = 0;
  Plan *P = get_plan(ndim, dims, coords, &st);
  if (!P) return (mgx_status)st;
  if (stop_level < 0 || stop_level > P->L) return MGX_ERR_LEVEL;
  return tolerances(P, ndim, tol_linf, stop_level, c_linf, tau_out);
}

double mgx_l2_constant(int ndim, const int64_t *dims, const double *const *coords, int stop_level) {
  int st = 0;
  Plan *P = get_plan(ndim, dims, coords, &st);
  if (!P || stop_level < 0 || stop_level > P->L) return -1.0;
  return P->l2_constant(stop_level);
}

mgx_status mgx_level_tolerances_l2(int ndim, const int64_t *dims, const double *const *coords, double tol_l2,
                                   int stop_level, double c_l2, double *tau_out) {
  if (!tau_out) return MGX_ERR_ARG;
  int st = 0;
  Plan *P = get_plan(ndim, dims, coords, &st);
  if (!P) return (mgx_status)st;
  if (stop_level < 0 || stop_level > P->L) return MGX_ERR_LEVEL;
  if (!(tol_l2 > 0.0) || !std::isfinite(tol_l2) || !std::isfinite(c_l2)) return MGX_ERR_TOL;
  if (!(c_l2 > 0.0)) c_l2 = P->l2_constant(stop_level);
  const double nL = (double)(P->n[0] * P->n[1] * P->n[2]);
  for (int l = stop_level; l <= P->L; l++) {
    // h_l^d: the level's cell volume, extent / intervals on every real axis
    double hd = 1.0;
    for (int k = 0; k < 3; k++) {
      if (!P->real[k]) continue;
      const int64_t m = (P->n[k] - 1) / ((int64_t)1 << (P->L - l)) + 1;
      hd = hd * ((P->X[k][P->n[k] - 1] - P->X[k][0]) / (double)(m - 1));
    }
    tau_out[l - stop_level] = tol_l2 / std::sqrt(c_l2 * hd * nL);
  }
  return MGX_OK;
}

mgx_status mgx_trace_enable(int on) {
  Tracer &t = tracer();
  std::lock_guard<std::mutex> g(t.mu);
  for (auto &r : t.recs) {
    (void)hipEventSynchronize(r.b);
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
  }
  t.recs.clear();
  t.on = on != 0;
  return MGX_OK;
}

int mgx_trace_read(mgx_kernel_time *out, int max) {
  Tracer &t = tracer();
  std::lock_guard<std::mutex> g(t.mu);
  std::vector<mgx_kernel_time> agg;
  bool ok = true;
  for (auto &r : t.recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ok = false;
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
    size_t i = 0;
    for (; i < agg.size(); i++)
      if (agg[i].level == r.level && std::strncmp(agg[i].name, r.name, sizeof(agg[i].name)) == 0) break;
    if (i == agg.size()) {
      mgx_kernel_time k;
      std::memset(&k, 0, sizeof(k));
      std::strncpy(k.name, r.name, sizeof(k.name) - 1);
      k.level = r.level;
      agg.push_back(k);
    }
    agg[i].count += 1;
    agg[i].total_ms += ms;
  }
  t.recs.clear();
  if (!ok) return -1;
  int n = (int)agg.size() < max ? (int)agg.size() : max;
  for (int i = 0; i < n; i++) out[i] = agg[i];
  return n;
}

mgx_status mgx_decompose_quantize(const void *u, void *u_mc, int32_t *labels, mgx_dtype dtype, int ndim,
                                  const int64_t *dims, const double *const *coords, double tol_linf, int stop_level,
                                  double c_linf, void *workspace, size_t workspace_bytes, mgx_quant_stats *stats,
                                  hipStream_t stream) {
  if (!labels) return MGX_ERR_ARG;  // checked before any HIP call
  // with stats: the statistics buffer (held until it is read back) takes the
  // level kernels' per-level maxima and out-of-range counts (four axes: the
  // counts, then one pass over the labels for the maxima)
  std::unique_lock<std::mutex> stats_lock;
  char *sbase = nullptr;
  auto attach = [&](int **mx, unsigned long long **ovf, unsigned long long **nan) -> mgx_status {
    if (!stats) return MGX_OK;
    stats_lock = std::unique_lock<std::mutex>(stats_buf().mu);
    if (!(sbase = stats_device(stream))) return MGX_ERR_HIP;
    *mx = (int *)sbase;
    *ovf = (unsigned long long *)(sbase + sizeof(int) * kMaxLevels);
    *nan = *ovf + 1;
    return MGX_OK;
  };
  if (ndim == 4) {  // labels written by the level kernels, u_mc optional
    Quant4Args qa;
    mgx_status s4 = quant_args4(dims, coords, tol_linf, stop_level, c_linf, nullptr, &qa);
    if (s4) return s4;
    Plan4 P4;
    Layout4 lay4;
    if ((s4 = prepare4(u, u_mc, dtype, dims, coords, stop_level, workspace, workspace_bytes, &P4, &lay4, 2)))
      return s4;
    const size_t cnt = (size_t)P4.count(P4.L), es = elem_size(dtype);
    if ((u_mc && overlaps(labels, cnt * 4, u_mc, cnt * es)) || overlaps(labels, cnt * 4, u, cnt * es) ||
        (lay4.total > 0 && overlaps(labels, cnt * 4, workspace, lay4.total)))
      return MGX_ERR_ARG;
    int *mx = nullptr;
    if ((s4 = attach(&mx, &qa.stats_ovf, &qa.stats_nan))) return s4;
    if (dtype == MGX_F32)
      s4 = run_decompose4<float>(P4, stop_level, (const float *)u, (float *)u_mc, (char *)workspace, lay4, stream,
                                 labels, &qa);
    else
      s4 = run_decompose4<double>(P4, stop_level, (const double *)u, (double *)u_mc, (char *)workspace, lay4,
                                  stream, labels, &qa);
    if (s4 || !stats) return s4;
    if (label_max_abs<Quant4Args>(labels, qa, mx, stream) != hipSuccess) return MGX_ERR_HIP;
    return stats_read(sbase, qa.first, qa.nlev, stats, stream);
  }
  if (dtype != MGX_F32 && dtype != MGX_F64) return MGX_ERR_ARG;
  QuantArgs qa;
  Plan *Pq;
  mgx_status s = quant_args(ndim, dims, coords, tol_linf, stop_level, c_linf, &qa, &Pq);
  if (s) return s;
  Plan *P;
  Layout lay;
  const void *tab;
  if ((s = prepare(u, u_mc, dtype, ndim, dims, coords, stop_level, workspace, workspace_bytes, &P, &lay, &tab, false,
                   2)))
    return s;
  const size_t cnt = (size_t)(P->n[0] * P->n[1] * P->n[2]);
  if ((u_mc && overlaps(labels, cnt * 4, u_mc, cnt * elem_size(dtype))) ||
      overlaps(labels, cnt * 4, u, cnt * elem_size(dtype)) ||
      (lay.total > 0 && overlaps(labels, cnt * 4, workspace, lay.total)))
    return MGX_ERR_ARG;
  if ((s = attach(&qa.stats_max, &qa.stats_ovf, &qa.stats_nan))) return s;  // the level kernels take them all
  if (dtype == MGX_F32)
    s = run_decompose_quantize<float>(P, stop_level, (const float *)u, (float *)u_mc, labels, qa, (char *)workspace,
                                      lay, (const float *)tab, stream);
  else
    s = run_decompose_quantize<double>(P, stop_level, (const double *)u, (double *)u_mc, labels, qa,
                                       (char *)workspace, lay, (const double *)tab, stream);
  if (s || !stats) return s;
  return stats_read(sbase, qa.first, qa.nlev, stats, stream);
}

mgx_status mgx_dequantize_recompose(const int32_t *labels, void *u_mc, void *u, mgx_dtype dtype, int ndim,
                                    const int64_t *dims, const double *const *coords, double tol_linf,
                                    int stop_level, double c_linf, void *workspace, size_t workspace_bytes,
                                    hipStream_t stream) {
  if (!labels) return MGX_ERR_ARG;  // labels and tolerance checked before any HIP call
  if (ndim == 4) {  // with u_mc: dequantize into it, then recompose; without: straight from the labels
    Quant4Args qa;
    mgx_status s4 = quant_args4(dims, coords, tol_linf, stop_level, c_linf, nullptr, &qa);
    if (s4) return s4;
    Plan4 P4;
    Layout4 lay4;
    if ((s4 = prepare4(u_mc, u, dtype, dims, coords, stop_level, workspace, workspace_bytes, &P4, &lay4, 1)))
      return s4;
    const size_t cnt = (size_t)P4.count(P4.L), es = elem_size(dtype);
    if ((u_mc && overlaps(labels, cnt * 4, u_mc, cnt * es)) || overlaps(labels, cnt * 4, u, cnt * es) ||
        (lay4.total > 0 && overlaps(labels, cnt * 4, workspace, lay4.total)))
      return MGX_ERR_ARG;
    if (u_mc) {
      if ((s4 = dequantize_common(labels, u_mc, dtype, 4, dims, coords, tol_linf, stop_level, c_linf, nullptr,
                                  stream)))
        return s4;
      return recompose4(u_mc, u, dtype, dims, coords, stop_level, workspace, workspace_bytes, stream);
    }
    if (dtype == MGX_F32)
      return run_recompose4<float>(P4, stop_level, nullptr, (float *)u, (char *)workspace, lay4, stream, labels, &qa);
    return run_recompose4<double>(P4, stop_level, nullptr, (double *)u, (char *)workspace, lay4, stream, labels, &qa);
  }
  if (dtype != MGX_F32 && dtype != MGX_F64) return MGX_ERR_ARG;
  QuantArgs qa;
  Plan *Pq;
  mgx_status s = quant_args(ndim, dims, coords, tol_linf, stop_level, c_linf, &qa, &Pq);
  if (s) return s;
  Plan *P;
  Layout lay;
  const void *tab;
  if ((s = prepare(u_mc, u, dtype, ndim, dims, coords, stop_level, workspace, workspace_bytes, &P, &lay, &tab, false,
                   1)))
    return s;
  const size_t cnt = (size_t)(P->n[0] * P->n[1] * P->n[2]);
  if ((u_mc && overlaps(labels, cnt * 4, u_mc, cnt * elem_size(dtype))) ||
      overlaps(labels, cnt * 4, u, cnt * elem_size(dtype)) ||
      (lay.total > 0 && overlaps(labels, cnt * 4, workspace, lay.total)))
    return MGX_ERR_ARG;
  if (dtype == MGX_F32)
    return run_dequantize_recompose<float>(P, stop_level, labels, (float *)u_mc, (float *)u, qa, (char *)workspace,
                                           lay, (const float *)tab, stream);
  return run_dequantize_recompose<double>(P, stop_level, labels, (double *)u_mc, (double *)u, qa,
                                          (char *)workspace, lay, (const double *)tab, stream);
}

size_t mgx_batch_workspace_size(int nfields, const mgx_field *fields) {
  std::vector<BatchField> bf;
  size_t need = 0;
  if (batch_validate(nfields, fields, true, bf, &need, false) != MGX_OK) return 0;
  return need;
}

mgx_status mgx_decompose_batched(int nfields, const mgx_field *fields, void *workspace, size_t workspace_bytes,
                                 hipStream_t stream) {
  return run_batched(nfields, fields, workspace, workspace_bytes, stream, true);
}

mgx_status mgx_recompose_batched(int nfields, const mgx_field *fields, void *workspace, size_t workspace_bytes,
                                 hipStream_t stream) {
  return run_batched(nfields, fields, workspace, workspace_bytes, stream, false);
}

mgx_status mgx_release_cached(void) {
  bool err = false;
  {
    BatchCache &C = batch_cache();
    std::lock_guard<std::mutex> g(C.mu);
    if (!C.map.empty()) {
      int cur = 0, ndev = 0;
      if (hipGetDevice(&cur) != hipSuccess || hipGetDeviceCount(&ndev) != hipSuccess) return MGX_ERR_HIP;
      for (int d = 0; d < ndev; d++)  // graphs may still run on any device
        if (hipSetDevice(d) != hipSuccess || hipDeviceSynchronize() != hipSuccess) err = true;
      if (hipSetDevice(cur) != hipSuccess) err = true;
      for (auto &kv : C.map) batch_entry_free(kv.second);
      C.map.clear();
      C.order.clear();
    }
  }
  if (release_plans()) err = true;
  return err ? MGX_ERR_HIP : MGX_OK;
}

mgx_status mgx_batch_set_autotune(int on) {
  g_batch_autotune.store(on ? 1 : 0);
  return MGX_OK;
}

mgx_status mgx_batch_last_info(mgx_batch_info *info) {
  if (!info) return MGX_ERR_ARG;
  *info = g_batch_info;
  return MGX_OK;
}

}  // extern "C"
