// Shannon entropy of the quantization labels of every level (Sec. 4.1: the
// cost of storing the labels is estimated by the entropy of their
// distribution): per level H = log2(N) - (1/N) sum_k c_k log2 c_k over the
// counts c_k of its distinct labels.  One pass finds each level's largest
// |label|.  When the levels' label ranges, laid end to end, fit in kHistBins
// keys, the counts come from one histogram pass (the finest levels counted in
// LDS first) and the terms are summed per level in a fixed order; otherwise
// (very wide ranges) the keys (level, label) are radix sorted and equal keys
// counted.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "entropy.hpp"
#include "kernels.hpp"
#include "levelpos.hpp"
#include "levelpos4.hpp"

namespace mgx {

namespace {

constexpr int64_t kHistBins = (int64_t)1 << 26;  // histogram keys (256 MB of counts)
constexpr int kLdsBins = 12288;         // LDS counters per workgroup (48 KB)
constexpr int kHistThreads = 512;       // threads of a counting workgroup (8 waves: two fit a CU's LDS)
constexpr int kHistBlocks = 512;        // workgroups of the counting pass
constexpr int kTermBlocks = 512;
constexpr int kFoldChunks = 16;         // slice chunks of the fold (y extent of its grid)
constexpr int kThreads = 256;

// The labels counted in LDS first: level l's labels in [-half[l], half[l]]
// (half < 0: none) at LDS offset off[l].  The finest levels hold most labels.
struct LdsMap {
  int half[kMaxLevelsK];
  int off[kMaxLevelsK];
};

// The histogram's keys: level l's labels -maxabs[l] .. maxabs[l] take keys
// koff[l] .. koff[l+1]-1 (passed by value: no copy to the device).
struct KeyMap {
  int64_t koff[kMaxLevelsK + 1];
  unsigned maxabs[kMaxLevelsK];
};

unsigned grid_of(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  if (g > 8192) g = 8192;
  return (unsigned)(g > 0 ? g : 1);
}

// Workgroups of a range pass: about four 16-byte words per thread and load.
unsigned range_grid(int64_t n) {
  int64_t g = (n + (int64_t)kThreads * 16 - 1) / ((int64_t)kThreads * 16);
  if (g > 4096) g = 4096;
  return (unsigned)(g > 0 ? g : 1);
}

// 16-byte loads in flight per thread in the passes over the labels, which
// are bound by memory latency with one load at a time.
constexpr int kLoads = 4;

// f(i, v) for every label v = labels[i], i < n, spread over the grid.  With
// vec (labels 16-byte aligned) four labels come with one load and each
// thread has kLoads loads in flight: workgroup b's iteration takes kLoads
// consecutive runs of blockDim.x 16-byte words.  The labels past the last
// whole word (and every label without vec) go one per thread.
template <class F>
__device__ __forceinline__ void for_each_label(const int32_t *__restrict__ labels, uint64_t n, bool vec, F &&f) {
  const uint64_t nt = blockDim.x, nthreads = (uint64_t)gridDim.x * nt;
  uint64_t done = 0;
  if (vec) {
    const uint64_t n4 = n / 4;
    const int4 *__restrict__ w4 = (const int4 *)labels;
    for (uint64_t q0 = (uint64_t)blockIdx.x * nt * kLoads + threadIdx.x; q0 < n4; q0 += nthreads * kLoads) {
      int4 w[kLoads];
#pragma unroll
      for (int u = 0; u < kLoads; u++) {
        const uint64_t q = q0 + (uint64_t)u * nt;
        w[u] = q < n4 ? w4[q] : make_int4(0, 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < kLoads; u++) {
        const uint64_t q = q0 + (uint64_t)u * nt;
        if (q < n4) {
          f(4 * q, w[u].x);
          f(4 * q + 1, w[u].y);
          f(4 * q + 2, w[u].z);
          f(4 * q + 3, w[u].w);
        }
      }
    }
    done = n4 * 4;
  }
  for (uint64_t i = done + (uint64_t)blockIdx.x * nt + threadIdx.x; i < n; i += nthreads) f(i, labels[i]);
}

// Rows of a level-centric array: the last axis (len labels) and the
// level of a row's position on the other axes.
__device__ __forceinline__ uint32_t row_len(const QuantArgs &a) { return (uint32_t)a.n2; }
__device__ __forceinline__ int row_off(const QuantArgs &a) { return a.off[2]; }
__device__ __forceinline__ int row_level(uint32_t r, const QuantArgs &a) {
  const uint32_t z = a.n1 == 1 ? r : (uint32_t)__umul64hi((uint64_t)r, a.mag1);
  const uint32_t y = r - z * (uint32_t)a.n1;
  return max(pos_level(y, a.off[1], a.first), pos_level(z, a.off[0], a.first));
}
__device__ __forceinline__ uint32_t row_len(const Quant4Args &a) { return (uint32_t)a.nd[3]; }
__device__ __forceinline__ int row_off(const Quant4Args &a) { return a.off[3]; }
__device__ __forceinline__ int row_level(uint32_t r, const Quant4Args &a) {
  const uint32_t r2 = udiv(r, a.d2);
  const uint32_t j2 = r - r2 * a.d2.d;
  const uint32_t j0 = udiv(r2, a.d1);
  const uint32_t j1 = r2 - j0 * a.d1.d;
  return max(max(pos_level(j0, a.off[0], a.first), pos_level(j1, a.off[1], a.first)),
             pos_level(j2, a.off[2], a.first));
}

// f(level, label) for every label, or ftop(label) for labels known to be of
// the finest level.  Rows of at least 64 labels go one per wave at a time,
// in pieces of up to 1024 labels (16 loads of 64): the row's level is found
// once; a row of the finest level (three in four rows of a 3-D field) holds
// only finest-level labels, and in other rows a label's level is the larger
// of the row's and that of its position along the row, so no label needs
// the divisions of elem_level.  A wave loads its next piece before it
// processes the current one (two register buffers, the loop unrolled twice
// so that no loaded value is copied before use), which keeps two pieces of
// loads in flight.  Lanes past the piece's end load its last label again (in
// bounds, not processed).  Shorter rows take elem_level per label (vec:
// labels 16-byte aligned).
template <typename A, class FT, class F>
__device__ __forceinline__ void for_each_level_label(const int32_t *__restrict__ labels, const A &a, bool vec,
                                                     FT &&ftop, F &&f) {
  const uint32_t len = row_len(a);
  if (len < 64) {
    for_each_label(labels, (uint64_t)a.n, vec, [&](uint64_t i, int32_t v) { f(elem_level((uint32_t)i, a), v); });
    return;
  }
  constexpr int J = 16;
  constexpr uint32_t P = 64 * J;
  const int top = a.first + a.nlev - 1;
  const uint32_t cpr = (len + P - 1) / P;  // pieces per row
  const uint32_t npieces = (uint32_t)((uint64_t)a.n / len) * cpr;
  const int offx = row_off(a);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
  uint32_t p = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (p >= npieces) return;
  auto fetch = [&](uint32_t q, int32_t (&v)[J]) {
    q = min(q, npieces - 1);
    const uint32_t r = cpr == 1 ? q : q / cpr, x0 = (q - r * cpr) * P;
    const uint32_t last = min(len - x0, P) - 1;
    const int32_t *__restrict__ row = labels + (uint64_t)r * len + x0;
#pragma unroll
    for (int j = 0; j < J; j++) v[j] = row[min(j * 64 + lane, last)];
  };
  auto process = [&](uint32_t q, const int32_t (&v)[J]) {
    const uint32_t r = cpr == 1 ? q : q / cpr, x0 = (q - r * cpr) * P;
    const uint32_t m = min(len - x0, P);
    const int lr = row_level(r, a);
    if (lr == top) {
#pragma unroll
      for (int j = 0; j < J; j++) {
        if ((j + 1) * 64 <= (int)m)
          ftop(v[j]);
        else if (j * 64 < (int)m && j * 64 + lane < m)
          ftop(v[j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < J; j++) {
        const uint32_t x = j * 64 + lane;
        if (x < m) f(max(lr, pos_level(x0 + x, offx, a.first)), v[j]);
      }
    }
  };
  int32_t va[J], vb[J];
  fetch(p, va);
  for (;;) {
    fetch(p + nwaves, vb);
    process(p, va);
    p += nwaves;
    if (p >= npieces) break;
    fetch(p + nwaves, va);
    process(p, vb);
    p += nwaves;
    if (p >= npieces) break;
  }
}

// Largest |label| of every level (an overflowed label, INT32_MIN, counts as
// 2^31, or with SKIP_OUT as 0: the quantizer's statistics leave it out).
// A: the (de)quantization arguments of a 1-D to 3-D (QuantArgs) or 4-D
// (Quant4Args) field; elem_level(i, a) gives the level of flat element i.
// The two finest levels (nearly all labels) keep their maxima in registers;
// the coarser ones go to LDS atomics.
template <typename A, bool SKIP_OUT>
__global__ void __launch_bounds__(kThreads) k_ent_range(const int32_t *__restrict__ labels, A a, int vec,
                                                        unsigned *__restrict__ maxabs) {
  __shared__ unsigned s_max[kMaxLevelsK];
  if (threadIdx.x < kMaxLevelsK) s_max[threadIdx.x] = 0;
  __syncthreads();
  const int top = a.first + a.nlev - 1;
  unsigned m0 = 0, m1 = 0;  // levels top and top - 1
  auto mag = [](int32_t v) {
    return (SKIP_OUT && v == INT32_MIN) ? 0u : v < 0 ? 0u - (unsigned)v : (unsigned)v;
  };
  for_each_level_label(
      labels, a, vec != 0, [&](int32_t v) { m0 = max(m0, mag(v)); },
      [&](int l, int32_t v) {
        const unsigned m = mag(v);
        // selects, not branches, for the two finest levels
        m0 = max(m0, l == top ? m : 0u);
        m1 = max(m1, l == top - 1 ? m : 0u);
        if (l < top - 1 && m) atomicMax(&s_max[l - a.first], m);
      });
  for (int off = 32; off > 0; off >>= 1) {
    m0 = max(m0, (unsigned)__shfl_xor((int)m0, off));
    m1 = max(m1, (unsigned)__shfl_xor((int)m1, off));
  }
  if ((threadIdx.x & 63) == 0) {
    if (m0) atomicMax(&s_max[top - a.first], m0);
    if (m1) atomicMax(&s_max[top - 1 - a.first], m1);  // (m1 stays 0 with one level)
  }
  __syncthreads();
  if (threadIdx.x < a.nlev && s_max[threadIdx.x]) atomicMax(&maxabs[threadIdx.x], s_max[threadIdx.x]);
}

// Counts of the keys koff[l] + maxabs[l] + label: a label inside its level's
// LDS window is counted in LDS, the others with global atomics.  Each
// workgroup then stores its LDS counters, bins 0 .. used-1, to its own slice
// slices[blockIdx.x * kLdsBins + j] (k_ent_fold adds the slices up).  A label
// beyond its level's maxabs (only when maxabs came from the caller) is not
// counted but added to *esc.
template <typename A>
__global__ void __launch_bounds__(kHistThreads) k_ent_hist(const int32_t *__restrict__ labels, A a, int vec,
                                                       KeyMap km, LdsMap lm, int used,
                                                       unsigned *__restrict__ hist, unsigned *__restrict__ slices,
                                                       unsigned *__restrict__ esc) {
  __shared__ unsigned s_h[kLdsBins + 1];   // the last counter takes the adds of labels counted elsewhere
  __shared__ int64_t s_base[kMaxLevelsK];  // key of label 0 of each level
  __shared__ int4 s_info[kMaxLevelsK];     // per level: LDS half width, LDS offset + half, maxabs
  for (int i = threadIdx.x; i <= kLdsBins; i += kHistThreads) s_h[i] = 0;
  if (threadIdx.x < kMaxLevelsK) {
    const bool in = threadIdx.x < a.nlev;
    s_base[threadIdx.x] = in ? km.koff[threadIdx.x] + (int64_t)km.maxabs[threadIdx.x] : 0;
    s_info[threadIdx.x] = make_int4(lm.half[threadIdx.x], lm.off[threadIdx.x] + lm.half[threadIdx.x],
                                    in ? (int)km.maxabs[threadIdx.x] : 0, 0);
  }
  __syncthreads();
  unsigned out = 0;
  const int top = a.nlev - 1;
  const int4 ftop = s_info[top];
  // one label of level l (info f): counted in LDS, globally, or as beyond maxabs
  auto count = [&](int l, const int4 &f, int32_t v) {
    const unsigned av = v < 0 ? 0u - (unsigned)v : (unsigned)v;
    const bool over = av > (unsigned)f.z;
    const bool lds = !over && f.x >= 0 && (unsigned)v + (unsigned)f.x <= 2u * (unsigned)f.x;
    out += over ? 1u : 0u;
    // every lane adds in LDS (0 at the spare counter unless counted there)
    atomicAdd(&s_h[lds ? f.y + v : kLdsBins], lds ? 1u : 0u);
    if (!lds && !over) atomicAdd(&hist[s_base[l] + v], 1u);
  };
  for_each_level_label(
      labels, a, vec != 0, [&](int32_t v) { count(top, ftop, v); },
      [&](int la, int32_t v) {
        const int l = la - a.first;
        count(l, s_info[l], v);
      });
  if (out) atomicAdd(esc, out);
  __syncthreads();
  unsigned *mine = slices + (int64_t)blockIdx.x * kLdsBins;
  for (int j = threadIdx.x; j < used; j += kHistThreads) mine[j] = s_h[j];
}

// hist[key of LDS bin j] = the sum over the hb slices of bin j.  Grid
// (bins / kThreads, chunks): the y-th chunk of slices is added with kLoads*2
// loads in flight and its sum added atomically (integer sums: any order).
__global__ void __launch_bounds__(kThreads) k_ent_fold(const unsigned *__restrict__ slices, int hb, int used,
                                                       KeyMap km, LdsMap lm, int nlev, unsigned *__restrict__ hist) {
  constexpr int U = 2 * kLoads;
  const int j = blockIdx.x * kThreads + threadIdx.x;
  if (j >= used) return;
  const int per = (hb + gridDim.y - 1) / gridDim.y;
  const int b0 = blockIdx.y * per, b1 = min(hb, b0 + per);
  unsigned sum = 0;
  for (int b = b0; b < b1; b += U) {
    unsigned c[U];
#pragma unroll
    for (int u = 0; u < U; u++) c[u] = b + u < b1 ? slices[(int64_t)(b + u) * kLdsBins + j] : 0u;
#pragma unroll
    for (int u = 0; u < U; u++) sum += c[u];
  }
  if (!sum) return;
  for (int l = 0; l < nlev; l++) {
    const int h = lm.half[l];
    if (h >= 0 && j >= lm.off[l] && j <= lm.off[l] + 2 * h) {
      atomicAdd(&hist[km.koff[l] + (int64_t)km.maxabs[l] + (j - lm.off[l] - h)], sum);
      return;
    }
  }
}

// Per level, the sum of c log2 c over its keys koff[l] .. koff[l+1]-1: block
// b takes the b-th of gridDim.x equal slices of every level, its threads
// read the slice coalesced (kLoads*2 loads in flight), and the sums are
// reduced in a fixed order (deterministic).  partial[b * nlev + l].
__global__ void __launch_bounds__(kThreads) k_ent_terms(const unsigned *__restrict__ hist, KeyMap km, int nlev,
                                                        double *__restrict__ partial) {
  constexpr int U = 2 * kLoads;
  __shared__ double s_sum[kThreads];
  for (int q = 0; q < nlev; q++) {
    const int64_t k0 = km.koff[q], k1 = km.koff[q + 1];
    const int64_t per = (k1 - k0 + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = k0 + (int64_t)blockIdx.x * per, b1 = min(k1, b0 + per);
    double acc = 0.0;
    for (int64_t k = b0 + threadIdx.x; k < b1; k += (int64_t)U * kThreads) {
      unsigned c[U];
#pragma unroll
      for (int u = 0; u < U; u++) c[u] = k + u * kThreads < b1 ? hist[k + u * kThreads] : 0u;
#pragma unroll
      for (int u = 0; u < U; u++)
        if (c[u] > 1) acc += (double)c[u] * log2((double)c[u]);
    }
    s_sum[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) s_sum[threadIdx.x] += s_sum[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * nlev + q] = s_sum[0];
    __syncthreads();
  }
}

// sums[l] = the sum over the nb blocks of partial[b * nlev + l] in a fixed
// order (thread t adds blocks t, t + 256, ..., then a fixed tree).
__global__ void __launch_bounds__(kThreads) k_ent_final(const double *__restrict__ partial, int nb, int nlev,
                                                        double *__restrict__ sums) {
  __shared__ double s_sum[kThreads];
  for (int q = 0; q < nlev; q++) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) acc += partial[(int64_t)b * nlev + q];
    s_sum[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) s_sum[threadIdx.x] += s_sum[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) sums[q] = s_sum[0];
    __syncthreads();
  }
}

// ---- sort path ----
// Keys (level - first) << 32 | label with its sign bit flipped: ascending key
// order is level, then label.
template <typename A>
__global__ void __launch_bounds__(kThreads) k_ent_keys(const int32_t *__restrict__ labels, A a,
                                                       uint64_t *__restrict__ keys) {
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < (uint64_t)a.n; i += stride) {
    const int l = elem_level((uint32_t)i, a);
    keys[i] = ((uint64_t)(uint32_t)(l - a.first) << 32) | (uint64_t)((uint32_t)labels[i] ^ 0x80000000u);
  }
}

// c log2 c of every run of equal keys, and the first run of every level.
__global__ void __launch_bounds__(kThreads) k_ent_run_terms(const uint64_t *__restrict__ uniq,
                                                            const int *__restrict__ cnt, const int *__restrict__ nruns,
                                                            double *__restrict__ terms, int *__restrict__ first_run) {
  const int n = *nruns;
  for (int r = blockIdx.x * kThreads + threadIdx.x; r < n; r += gridDim.x * kThreads) {
    const double c = (double)cnt[r];
    terms[r] = c * log2(c);
    const int lv = (int)(uniq[r] >> 32);
    if (r == 0 || (int)(uniq[r - 1] >> 32) != lv) first_run[lv] = r;
  }
}

__global__ void k_fill_int(int *p, int n, int v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

// Temp bytes of the library calls for n keys (no launch).
size_t sort_temp(int64_t n) {
  size_t a = 0, b = 0, c = 0;
  (void)hipcub::DeviceRadixSort::SortKeys(nullptr, a, (const uint64_t *)nullptr, (uint64_t *)nullptr, (int)n);
  (void)hipcub::DeviceRunLengthEncode::Encode(nullptr, b, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                              (int *)nullptr, (int *)nullptr, (int)n);
  (void)hipcub::DeviceReduce::Sum(nullptr, c, (const double *)nullptr, (double *)nullptr, (int)n);
  return std::max(std::max(a, b), c);
}

__global__ void k_fill_u32(unsigned *p, int64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (uint64_t)n; i += stride) p[i] = 0u;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace: the small arrays first, then either the histogram or the sort
// path's buffers (both start at `big`).
struct Parts {
  unsigned *maxabs;
  double *partial;
  int *nruns, *first_run;
  double *sums;
  unsigned *esc;  // labels beyond the caller's maxima
  char *big;
};

size_t small_bytes() {
  return align256(sizeof(unsigned) * kMaxLevelsK) +
         align256(sizeof(double) * kTermBlocks * kMaxLevelsK) + 256 + align256(sizeof(int) * kMaxLevelsK) +
         align256(sizeof(double) * kMaxLevelsK) + 256;
}

// The histogram path: the counts, then the workgroups' LDS counter slices.
size_t slices_offset() { return align256((size_t)kHistBins * 4); }
size_t hist_bytes() { return slices_offset() + align256((size_t)kHistBlocks * kLdsBins * 4); }

size_t sort_bytes(int64_t n) { return 2 * align256((size_t)n * 8) + align256((size_t)n * 4) + align256(sort_temp(n)); }

Parts carve(char *ws) {
  Parts p;
  size_t off = 0;
  p.maxabs = (unsigned *)(ws + off);
  off += align256(sizeof(unsigned) * kMaxLevelsK);
  p.partial = (double *)(ws + off);
  off += align256(sizeof(double) * kTermBlocks * kMaxLevelsK);
  p.nruns = (int *)(ws + off);
  off += 256;
  p.first_run = (int *)(ws + off);
  off += align256(sizeof(int) * kMaxLevelsK);
  p.sums = (double *)(ws + off);
  off += align256(sizeof(double) * kMaxLevelsK);
  p.esc = (unsigned *)(ws + off);
  off += 256;
  p.big = ws + off;
  return p;
}

// The sort path: sums of c log2 c per level into s.
template <typename A>
hipError_t sort_sums(const int32_t *labels, const A &qa, const Parts &p, hipStream_t st, double *s) {
  const int64_t n = qa.n;
  const int nlev = qa.nlev;
  uint64_t *keys_a = (uint64_t *)p.big;
  uint64_t *keys_b = (uint64_t *)(p.big + align256((size_t)n * 8));
  int *cnt = (int *)(p.big + 2 * align256((size_t)n * 8));
  void *temp = p.big + 2 * align256((size_t)n * 8) + align256((size_t)n * 4);
  const size_t temp_bytes = sort_temp(n);
  hipError_t e;
  hipLaunchKernelGGL((k_ent_keys<A>), dim3(grid_of(n)), dim3(kThreads), 0, st, labels, qa, keys_a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  size_t tb = temp_bytes;
  if ((e = hipcub::DeviceRadixSort::SortKeys(temp, tb, keys_a, keys_b, (int)n, 0, 64, st)) != hipSuccess) return e;
  tb = temp_bytes;
  // distinct keys into keys_a (free after the sort), their counts into cnt
  if ((e = hipcub::DeviceRunLengthEncode::Encode(temp, tb, keys_b, keys_a, cnt, p.nruns, (int)n, st)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, p.first_run, nlev, -1);
  double *terms = (double *)keys_b;  // the sorted keys are no longer needed
  hipLaunchKernelGGL(k_ent_run_terms, dim3(grid_of(n)), dim3(kThreads), 0, st, keys_a, cnt, p.nruns, terms,
                     p.first_run);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int nruns = 0;
  std::vector<int> first((size_t)nlev);
  if ((e = hipMemcpyAsync(&nruns, p.nruns, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipMemcpyAsync(first.data(), p.first_run, sizeof(int) * (size_t)nlev, hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  // per level: the sum over its runs (levels are contiguous in key order)
  for (int l = 0; l < nlev; l++) {
    if (first[l] < 0) continue;
    int end = nruns;
    for (int k = l + 1; k < nlev; k++)
      if (first[k] >= 0) {
        end = first[k];
        break;
      }
    tb = temp_bytes;
    if ((e = hipcub::DeviceReduce::Sum(temp, tb, terms + first[l], p.sums + l, end - first[l], st)) != hipSuccess)
      return e;
  }
  if ((e = hipMemcpyAsync(s, p.sums, sizeof(double) * (size_t)nlev, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  for (int l = 0; l < nlev; l++)
    if (first[l] < 0) s[l] = 0.0;  // (no labels of that level; its slot was not written)
  return hipSuccess;
}

}  // namespace

size_t entropy_workspace(int64_t n, int nlev) {
  if (n < 1 || n > INT32_MAX || nlev < 1 || nlev > kMaxLevelsK) return 0;
  return small_bytes() + std::max(hist_bytes(), sort_bytes(n));
}

template <typename A>
hipError_t label_entropy(const int32_t *labels, const A &qa, const int64_t *level_count, char *ws, hipStream_t st,
                         double *bits_out, const int32_t *known_max) {
  const int nlev = qa.nlev;
  Parts p = carve(ws);
  hipError_t e;
  const int vec = ((uintptr_t)labels & 15) == 0;
  std::vector<unsigned> mx(kMaxLevelsK, 0u);
  if (known_max) {  // the caller's maxima (the quantizer's statistics): no range pass
    for (int l = 0; l < nlev; l++) mx[l] = (unsigned)known_max[l];
    if ((e = hipMemcpyAsync(p.maxabs, mx.data(), sizeof(unsigned) * kMaxLevelsK, hipMemcpyHostToDevice, st)) !=
        hipSuccess)
      return e;
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, p.maxabs, (int64_t)kMaxLevelsK);
    hipLaunchKernelGGL((k_ent_range<A, false>), dim3(range_grid(qa.n)), dim3(kThreads), 0, st, labels, qa, vec,
                       p.maxabs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(mx.data(), p.maxabs, sizeof(unsigned) * kMaxLevelsK, hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return e;
  }
  // the levels' key ranges end to end: level l takes 2 maxabs[l] + 1 keys
  std::vector<int64_t> koff(kMaxLevelsK + 1, 0);
  for (int l = 0; l < nlev; l++) koff[l + 1] = koff[l] + 2 * (int64_t)mx[l] + 1;
  for (int l = nlev + 1; l <= kMaxLevelsK; l++) koff[l] = koff[nlev];
  const int64_t R = koff[nlev];
  KeyMap km;
  for (int l = 0; l <= kMaxLevelsK; l++) km.koff[l] = koff[l];
  for (int l = 0; l < kMaxLevelsK; l++) km.maxabs[l] = mx[l];
  // LDS counters: the finest level first, then the next, each up to half the
  // counters (or its whole label range)
  LdsMap lm;
  int used = 0;
  for (int l = nlev - 1; l >= 0; l--) {
    const int room = (kLdsBins - used - 1) / 2;
    const int want = (int)std::min<int64_t>((int64_t)mx[l], l == nlev - 1 ? (kLdsBins / 2 - 1) / 2 : room);
    lm.half[l] = room > 0 ? std::min(want, room) : -1;
    lm.off[l] = used;
    if (lm.half[l] >= 0) used += 2 * lm.half[l] + 1;
  }
  for (int l = nlev; l < kMaxLevelsK; l++) {
    lm.half[l] = -1;
    lm.off[l] = 0;
  }
  std::vector<double> s((size_t)nlev, 0.0);
  if (R > kHistBins) {
    if ((e = sort_sums(labels, qa, p, st, s.data())) != hipSuccess) return e;
  } else {
    unsigned *hist = (unsigned *)p.big, *slices = (unsigned *)(p.big + slices_offset());
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, p.esc, (int64_t)1);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_of(R)), dim3(kThreads), 0, st, hist, R);
    const unsigned hb = std::min<unsigned>(grid_of(qa.n), kHistBlocks);
    hipLaunchKernelGGL((k_ent_hist<A>), dim3(hb), dim3(kHistThreads), 0, st, labels, qa, vec, km, lm, used, hist,
                       slices, p.esc);
    hipLaunchKernelGGL(k_ent_fold, dim3((unsigned)((used + kThreads - 1) / kThreads), kFoldChunks), dim3(kThreads),
                       0, st, slices, (int)hb, used, km, lm, nlev, hist);
    hipLaunchKernelGGL(k_ent_terms, dim3(kTermBlocks), dim3(kThreads), 0, st, hist, km, nlev, p.partial);
    hipLaunchKernelGGL(k_ent_final, dim3(1), dim3(kThreads), 0, st, p.partial, kTermBlocks, nlev, p.sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the sums and the escape count (p.esc follows p.sums) in one copy
    static_assert(sizeof(double) * kMaxLevelsK <= 256, "sums slot");
    double back[256 / sizeof(double) + 1];
    if ((e = hipMemcpyAsync(back, p.sums, 256 + sizeof(unsigned), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return e;
    unsigned esc;
    std::memcpy(&esc, back + 256 / sizeof(double), sizeof(unsigned));
    // some label beyond the caller's maxima: count again with the exact ones
    if (esc) return label_entropy(labels, qa, level_count, ws, st, bits_out, nullptr);
    for (int l = 0; l < nlev; l++) s[l] = back[l];
  }
  for (int l = 0; l < nlev; l++) {
    const double N = (double)level_count[l];
    bits_out[l] = N <= 0.0 ? 0.0 : std::log2(N) - s[l] / N;
  }
  return hipSuccess;
}

template <typename A>
hipError_t label_max_abs(const int32_t *labels, const A &qa, int *max_abs, hipStream_t st) {
  hipLaunchKernelGGL((k_ent_range<A, true>), dim3(range_grid(qa.n)), dim3(kThreads), 0, st, labels, qa,
                     (int)(((uintptr_t)labels & 15) == 0), (unsigned *)max_abs);
  return hipGetLastError();
}

template hipError_t label_max_abs<QuantArgs>(const int32_t *, const QuantArgs &, int *, hipStream_t);
template hipError_t label_max_abs<Quant4Args>(const int32_t *, const Quant4Args &, int *, hipStream_t);
template hipError_t label_entropy<QuantArgs>(const int32_t *, const QuantArgs &, const int64_t *, char *,
                                             hipStream_t, double *, const int32_t *);
template hipError_t label_entropy<Quant4Args>(const int32_t *, const Quant4Args &, const int64_t *, char *,
                                              hipStream_t, double *, const int32_t *);

}  // namespace mgx
