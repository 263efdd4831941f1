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
constexpr int kHistBlocks = 1024;       // workgroups of the counting pass (few: small flushes)
constexpr int kTermBlocks = 512;
constexpr int kThreads = 256;

// The labels counted in LDS first: level l's labels in [-half[l], half[l]]
// (half < 0: none) at LDS offset off[l].  The finest levels hold most labels.
struct LdsMap {
  int half[kMaxLevelsK];
  int off[kMaxLevelsK];
};

unsigned grid_of(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  if (g > 8192) g = 8192;
  return (unsigned)(g > 0 ? g : 1);
}

// Largest |label| of every level (an overflowed label, INT32_MIN, counts as
// 2^31, or with SKIP_OUT as 0: the quantizer's statistics leave it out).
// A: the (de)quantization arguments of a 1-D to 3-D (QuantArgs) or 4-D
// (Quant4Args) field; elem_level(i, a) gives the level of flat element i.
template <typename A, bool SKIP_OUT>
__global__ void __launch_bounds__(kThreads) k_ent_range(const int32_t *__restrict__ labels, A a,
                                                        unsigned *__restrict__ maxabs) {
  __shared__ unsigned s_max[kMaxLevelsK];
  if (threadIdx.x < kMaxLevelsK) s_max[threadIdx.x] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  // every thread of the workgroup runs the same iterations (wave-wide reductions)
  for (uint64_t b0 = (uint64_t)blockIdx.x * kThreads; b0 < (uint64_t)a.n; b0 += stride) {
    const uint64_t i = b0 + threadIdx.x;
    const bool in = i < (uint64_t)a.n;
    const int l = in ? elem_level((uint32_t)i, a) : a.first;
    const int32_t v = in ? labels[i] : 0;
    const unsigned m = (SKIP_OUT && v == INT32_MIN) ? 0u : v < 0 ? 0u - (unsigned)v : (unsigned)v;
    unsigned long long todo = __ballot(in);
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int L0 = __shfl(l, leader);
      const bool mine = in && l == L0;
      unsigned r = mine ? m : 0u;
      for (int off = 32; off > 0; off >>= 1) r = max(r, (unsigned)__shfl_xor((int)r, off));
      if (lane == leader) atomicMax(&s_max[L0 - a.first], r);
      todo &= ~__ballot(mine);
    }
  }
  __syncthreads();
  if (threadIdx.x < a.nlev) atomicMax(&maxabs[threadIdx.x], s_max[threadIdx.x]);
}

// Counts of the keys off[l] + label + maxabs[l] in [wb, wb + nb).
template <typename A>
__global__ void __launch_bounds__(kThreads) k_ent_hist(const int32_t *__restrict__ labels, A a,
                                                       const unsigned *__restrict__ maxabs, const int64_t *__restrict__ koff,
                                                       LdsMap lm, int64_t wb, int64_t nb, unsigned *__restrict__ hist) {
  __shared__ unsigned s_h[kLdsBins];
  __shared__ int64_t s_base[kMaxLevelsK];  // key of label 0 of each level
  for (int i = threadIdx.x; i < kLdsBins; i += kThreads) s_h[i] = 0;
  if (threadIdx.x < kMaxLevelsK)
    s_base[threadIdx.x] = threadIdx.x < a.nlev ? koff[threadIdx.x] + (int64_t)maxabs[threadIdx.x] : 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * kThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < (uint64_t)a.n; i += stride) {
    const int l = elem_level((uint32_t)i, a) - a.first;
    const int32_t v = labels[i];
    const int64_t k = s_base[l] + v - wb;
    if (k < 0 || k >= nb) continue;
    const int h = lm.half[l];
    if (v >= -h && v <= h)
      atomicAdd(&s_h[lm.off[l] + v + h], 1u);
    else
      atomicAdd(&hist[k], 1u);
  }
  __syncthreads();
  // counted only inside [wb, wb + nb), so every flushed key lies in it
  for (int l = 0; l < a.nlev; l++) {
    const int h = lm.half[l];
    for (int j = threadIdx.x; j <= 2 * h; j += kThreads) {
      const unsigned c = s_h[lm.off[l] + j];
      if (c) atomicAdd(&hist[s_base[l] + (j - h) - wb], c);
    }
  }
}

// Per level, the sum of c log2 c over the bins [wb, wb + nb): block b takes a
// contiguous bin range, each thread a contiguous part of it, and the per-level
// sums are reduced in a fixed order (deterministic).  partial[b * nlev + l].
__global__ void __launch_bounds__(kThreads) k_ent_terms(const unsigned *__restrict__ hist, int64_t wb, int64_t nb,
                                                        const int64_t *__restrict__ koff, int nlev,
                                                        double *__restrict__ partial) {
  __shared__ double s_sum[kMaxLevelsK][kThreads];
  __shared__ int64_t s_off[kMaxLevelsK + 1];
  for (int l = 0; l < kMaxLevelsK; l++) s_sum[l][threadIdx.x] = 0.0;
  if (threadIdx.x <= kMaxLevelsK) s_off[threadIdx.x] = koff[min((int)threadIdx.x, nlev)];
  __syncthreads();
  const int64_t per_block = (nb + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per_block, b1 = min(nb, b0 + per_block);
  const int64_t per_thread = (per_block + kThreads - 1) / kThreads;
  const int64_t t0 = b0 + (int64_t)threadIdx.x * per_thread, t1 = min(b1, t0 + per_thread);
  int l = 0;
  double acc = 0.0;
  for (int64_t k = t0; k < t1; k++) {
    const int64_t key = wb + k;
    while (l + 1 < nlev && key >= s_off[l + 1]) {
      s_sum[l][threadIdx.x] += acc;
      acc = 0.0;
      l++;
    }
    const unsigned c = hist[k];
    if (c > 1) acc += (double)c * log2((double)c);
  }
  if (t0 < t1) s_sum[l][threadIdx.x] += acc;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int q = 0; q < nlev; q++) s_sum[q][threadIdx.x] += s_sum[q][threadIdx.x + h];
    __syncthreads();
  }
  if ((int)threadIdx.x < nlev) partial[(int64_t)blockIdx.x * nlev + threadIdx.x] = s_sum[threadIdx.x][0];
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
  int64_t *koff;
  double *partial;
  int *nruns, *first_run;
  double *sums;
  char *big;
};

size_t small_bytes() {
  return align256(sizeof(unsigned) * kMaxLevelsK) + align256(sizeof(int64_t) * (kMaxLevelsK + 1)) +
         align256(sizeof(double) * kTermBlocks * kMaxLevelsK) + 256 + align256(sizeof(int) * kMaxLevelsK) +
         align256(sizeof(double) * kMaxLevelsK);
}

size_t sort_bytes(int64_t n) { return 2 * align256((size_t)n * 8) + align256((size_t)n * 4) + align256(sort_temp(n)); }

Parts carve(char *ws) {
  Parts p;
  size_t off = 0;
  p.maxabs = (unsigned *)(ws + off);
  off += align256(sizeof(unsigned) * kMaxLevelsK);
  p.koff = (int64_t *)(ws + off);
  off += align256(sizeof(int64_t) * (kMaxLevelsK + 1));
  p.partial = (double *)(ws + off);
  off += align256(sizeof(double) * kTermBlocks * kMaxLevelsK);
  p.nruns = (int *)(ws + off);
  off += 256;
  p.first_run = (int *)(ws + off);
  off += align256(sizeof(int) * kMaxLevelsK);
  p.sums = (double *)(ws + off);
  off += align256(sizeof(double) * kMaxLevelsK);
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
  return small_bytes() + std::max(align256((size_t)kHistBins * 4), sort_bytes(n));
}

template <typename A>
hipError_t label_entropy(const int32_t *labels, const A &qa, const int64_t *level_count, char *ws, hipStream_t st,
                         double *bits_out) {
  const int nlev = qa.nlev;
  Parts p = carve(ws);
  hipError_t e;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, p.maxabs, (int64_t)kMaxLevelsK);
  hipLaunchKernelGGL((k_ent_range<A, false>), dim3(grid_of(qa.n)), dim3(kThreads), 0, st, labels, qa, p.maxabs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  std::vector<unsigned> mx(kMaxLevelsK);
  if ((e = hipMemcpyAsync(mx.data(), p.maxabs, sizeof(unsigned) * kMaxLevelsK, hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  // the levels' key ranges end to end: level l takes 2 maxabs[l] + 1 keys
  std::vector<int64_t> koff(kMaxLevelsK + 1, 0);
  for (int l = 0; l < nlev; l++) koff[l + 1] = koff[l] + 2 * (int64_t)mx[l] + 1;
  for (int l = nlev + 1; l <= kMaxLevelsK; l++) koff[l] = koff[nlev];
  const int64_t R = koff[nlev];
  if ((e = hipMemcpyAsync(p.koff, koff.data(), sizeof(int64_t) * (kMaxLevelsK + 1), hipMemcpyHostToDevice, st)) !=
      hipSuccess)
    return e;
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
  std::vector<double> s((size_t)nlev, 0.0), part((size_t)kTermBlocks * nlev);
  if (R > kHistBins) {
    if ((e = sort_sums(labels, qa, p, st, s.data())) != hipSuccess) return e;
  } else {
    unsigned *hist = (unsigned *)p.big;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_of(R)), dim3(kThreads), 0, st, hist, R);
    const unsigned hb = std::min<unsigned>(grid_of(qa.n), kHistBlocks);
    hipLaunchKernelGGL((k_ent_hist<A>), dim3(hb), dim3(kThreads), 0, st, labels, qa, p.maxabs, p.koff, lm, (int64_t)0,
                       R, hist);
    hipLaunchKernelGGL(k_ent_terms, dim3(kTermBlocks), dim3(kThreads), 0, st, hist, (int64_t)0, R, p.koff, nlev,
                       p.partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(part.data(), p.partial, sizeof(double) * part.size(), hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return e;
    for (int b = 0; b < kTermBlocks; b++)
      for (int l = 0; l < nlev; l++) s[l] += part[(size_t)b * nlev + l];
  }
  for (int l = 0; l < nlev; l++) {
    const double N = (double)level_count[l];
    bits_out[l] = N <= 0.0 ? 0.0 : std::log2(N) - s[l] / N;
  }
  return hipSuccess;
}

template <typename A>
hipError_t label_max_abs(const int32_t *labels, const A &qa, int *max_abs, hipStream_t st) {
  hipLaunchKernelGGL((k_ent_range<A, true>), dim3(grid_of(qa.n)), dim3(kThreads), 0, st, labels, qa,
                     (unsigned *)max_abs);
  return hipGetLastError();
}

template hipError_t label_max_abs<QuantArgs>(const int32_t *, const QuantArgs &, int *, hipStream_t);
template hipError_t label_max_abs<Quant4Args>(const int32_t *, const Quant4Args &, int *, hipStream_t);
template hipError_t label_entropy<QuantArgs>(const int32_t *, const QuantArgs &, const int64_t *, char *,
                                             hipStream_t, double *);
template hipError_t label_entropy<Quant4Args>(const int32_t *, const Quant4Args &, const int64_t *, char *,
                                              hipStream_t, double *);

}  // namespace mgx
