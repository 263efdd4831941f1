// Shannon entropy of the quantization labels of every level (Sec. 4.1: the
// cost of storing the labels is estimated by the entropy of their
// distribution).  Keys (level, label) are sorted, equal keys counted, and
// per level H = log2(N) - (1/N) sum_k c_k log2 c_k over its distinct labels.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstdint>
#include <vector>

#include "entropy.hpp"
#include "kernels.hpp"

namespace mgx {

namespace {

__global__ void __launch_bounds__(256) k_entropy_terms(const uint64_t *__restrict__ uniq, const int *__restrict__ cnt,
                                                     const int *__restrict__ nruns, double *__restrict__ terms,
                                                     int *__restrict__ first_run) {
  const int n = *nruns;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    const double c = (double)cnt[r];
    terms[r] = c * log2(c);
    const int lv = (int)(uniq[r] >> 32);
    if (r == 0 || (int)(uniq[r - 1] >> 32) != lv) first_run[lv] = r;
  }
}

__global__ void k_fill_int(int *p, int n, int v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

struct Parts {
  uint64_t *keys_a, *keys_b;
  int *cnt, *nruns, *first_run;
  double *sums;
  void *temp;
  size_t temp_bytes;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Temp bytes of the library calls for n keys (no launch).
size_t temp_need(int64_t n) {
  size_t a = 0, b = 0, c = 0;
  hipcub::DeviceRadixSort::SortKeys(nullptr, a, (const uint64_t *)nullptr, (uint64_t *)nullptr, (int)n);
  hipcub::DeviceRunLengthEncode::Encode(nullptr, b, (const uint64_t *)nullptr, (uint64_t *)nullptr, (int *)nullptr,
                                        (int *)nullptr, (int)n);
  hipcub::DeviceReduce::Sum(nullptr, c, (const double *)nullptr, (double *)nullptr, (int)n);
  size_t m = a > b ? a : b;
  return m > c ? m : c;
}

Parts carve(char *ws, int64_t n, int nlev) {
  Parts p;
  size_t off = 0;
  p.keys_a = (uint64_t *)(ws + off);
  off += align256((size_t)n * 8);
  p.keys_b = (uint64_t *)(ws + off);
  off += align256((size_t)n * 8);
  p.cnt = (int *)(ws + off);
  off += align256((size_t)n * 4);
  p.nruns = (int *)(ws + off);
  off += 256;
  p.first_run = (int *)(ws + off);
  off += align256(sizeof(int) * (size_t)nlev);
  p.sums = (double *)(ws + off);
  off += align256(sizeof(double) * (size_t)nlev);
  p.temp = ws + off;
  p.temp_bytes = temp_need(n);
  return p;
}

}  // namespace

size_t entropy_workspace(int64_t n, int nlev) {
  if (n < 1 || n > INT32_MAX) return 0;
  size_t off = 2 * align256((size_t)n * 8) + align256((size_t)n * 4) + 256 + align256(sizeof(int) * (size_t)nlev) +
               align256(sizeof(double) * (size_t)nlev);
  return off + align256(temp_need(n));
}

hipError_t label_entropy(const int32_t *labels, const QuantArgs &qa, const int64_t *level_count, char *ws,
                         hipStream_t st, double *bits_out) {
  const int64_t n = qa.n;
  const int nlev = qa.nlev;
  Parts p = carve(ws, n, nlev);
  hipError_t e;
  if ((e = launch_entropy_keys(labels, p.keys_a, qa, st)) != hipSuccess) return e;
  size_t tb = p.temp_bytes;
  if ((e = hipcub::DeviceRadixSort::SortKeys(p.temp, tb, p.keys_a, p.keys_b, (int)n, 0, 64, st)) != hipSuccess)
    return e;
  tb = p.temp_bytes;
  // distinct keys into keys_a (free after the sort), their counts into cnt
  if ((e = hipcub::DeviceRunLengthEncode::Encode(p.temp, tb, p.keys_b, p.keys_a, p.cnt, p.nruns, (int)n, st)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, p.first_run, nlev, -1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  double *terms = (double *)p.keys_b;  // the sorted keys are no longer needed
  int blocks = (int)((n + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_entropy_terms, dim3((unsigned)blocks), dim3(256), 0, st, p.keys_a, p.cnt, p.nruns, terms,
                     p.first_run);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int nruns = 0;
  std::vector<int> first((size_t)nlev);
  if ((e = hipMemcpyAsync(&nruns, p.nruns, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipMemcpyAsync(first.data(), p.first_run, sizeof(int) * (size_t)nlev, hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  // per level: the sum of c log2 c over its runs (levels are contiguous in key order)
  std::vector<double> s((size_t)nlev, 0.0);
  for (int l = 0; l < nlev; l++) {
    if (first[l] < 0) continue;
    int end = nruns;
    for (int k = l + 1; k < nlev; k++)
      if (first[k] >= 0) {
        end = first[k];
        break;
      }
    tb = p.temp_bytes;
    if ((e = hipcub::DeviceReduce::Sum(p.temp, tb, terms + first[l], p.sums + l, end - first[l], st)) != hipSuccess)
      return e;
  }
  if ((e = hipMemcpyAsync(s.data(), p.sums, sizeof(double) * (size_t)nlev, hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  for (int l = 0; l < nlev; l++) {
    const double N = (double)level_count[l];
    bits_out[l] = (first[l] < 0 || N <= 0.0) ? 0.0 : std::log2(N) - s[l] / N;
  }
  return hipSuccess;
}

}  // namespace mgx
