// Host-side paths of libmgx under AddressSanitizer and UBSan (built by
// tests/test_host_sanitizers.py with the host objects instrumented): level
// plans on uniform, random and tanh-like coordinates, the constants and
// tolerance schedules, the batch workspace sizing, and the argument
// validation of the device entry points (every case here fails validation
// before any HIP call, so no device memory is touched).  Exits nonzero on a
// wrong answer; the sanitizers abort on a memory or undefined-behaviour
// error.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mgx.h"

static int g_fail = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      g_fail = 1;                                                  \
    }                                                              \
  } while (0)

static std::vector<double> coords_of(int64_t n, int kind) {
  std::vector<double> x(n);
  unsigned s = 12345u + (unsigned)n;
  double acc = 0.0;
  for (int64_t i = 0; i < n; i++) {
    if (kind == 0) {
      x[i] = (double)i;
    } else if (kind == 1) {
      s = s * 1664525u + 1013904223u;
      acc += 0.25 + (double)(s >> 8) / (double)(1u << 24);
      x[i] = acc;
    } else {
      x[i] = std::tanh(2.0 * ((double)i / (double)(n - 1) - 1.0));
    }
  }
  return x;
}

int main() {
  const int64_t shapes[][3] = {{65, 0, 0}, {17, 33, 0}, {9, 17, 5}, {33, 9, 129}, {3, 3, 3}, {257, 5, 9}};
  const int ndims[] = {1, 2, 3, 3, 3, 3};
  for (int si = 0; si < 6; si++) {
    const int nd = ndims[si];
    const int64_t *d = shapes[si];
    const int L = mgx_num_levels(nd, d);
    CHECK(L >= 0);
    for (int kind = 0; kind < 3; kind++) {
      std::vector<std::vector<double>> X(nd);
      std::vector<const double *> cp(nd);
      for (int k = 0; k < nd; k++) {
        X[k] = coords_of(d[k], kind);
        cp[k] = X[k].data();
      }
      for (int stop = 0; stop <= L; stop++) {
        const double C = mgx_linf_constant(nd, d, cp.data(), stop);
        CHECK(C >= 1.0 && std::isfinite(C));
        const double C2 = mgx_l2_constant(nd, d, cp.data(), stop);
        CHECK(C2 > 0.0 && std::isfinite(C2));
        if (kind == 0) CHECK(C2 == 1.0);
        std::vector<double> tau(L + 1 - stop), tau2(L + 1 - stop);
        CHECK(mgx_level_tolerances(nd, d, cp.data(), 1e-3, stop, 0.0, tau.data()) == MGX_OK);
        double sum = 0.0;
        for (double t : tau) sum += t;
        CHECK(std::fabs(sum * C - 1e-3) <= 1e-15);
        CHECK(mgx_level_tolerances_l2(nd, d, cp.data(), 1.0, stop, 0.0, tau2.data()) == MGX_OK);
        CHECK(mgx_workspace_size(MGX_F32, nd, d, stop) <= mgx_workspace_size(MGX_F64, nd, d, stop));
      }
      CHECK(mgx_linf_constant(nd, d, cp.data(), L + 1) < 0.0);
    }
    // invalid coordinates: one repeated value
    std::vector<double> bad = coords_of(d[0], 1);
    bad[d[0] / 2] = bad[d[0] / 2 - 1];
    std::vector<const double *> cb(nd, nullptr);
    cb[0] = bad.data();
    CHECK(mgx_linf_constant(nd, d, cb.data(), 0) < 0.0);
    double tau[16];
    CHECK(mgx_level_tolerances(nd, d, cb.data(), 1.0, 0, 0.0, tau) == MGX_ERR_COORDS);
  }
  // shapes and levels
  const int64_t badshape[3] = {10, 9, 9};
  CHECK(mgx_num_levels(3, badshape) == -MGX_ERR_SHAPE);
  const int64_t big[1] = {(int64_t)1 << 40};
  CHECK(mgx_num_levels(1, big) == -MGX_ERR_SHAPE);
  CHECK(mgx_num_levels(0, badshape) == -MGX_ERR_SHAPE);
  CHECK(mgx_num_levels(5, badshape) == -MGX_ERR_SHAPE);
  int64_t padded[4];
  const int64_t odd[4] = {288, 115, 69, 69};
  CHECK(mgx_dyadic_dims(4, odd, padded) == MGX_OK);
  CHECK(padded[0] == 513 && padded[1] == 129 && padded[2] == 129 && padded[3] == 129);
  const int64_t one[1] = {1};
  CHECK(mgx_dyadic_dims(1, one, padded) == MGX_ERR_SHAPE);
  // device entry points: validation before any HIP call.  The pointers are
  // distinct made-up addresses, never dereferenced: each call below fails
  // its host-side checks first.
  const int64_t d3[3] = {9, 9, 9};
  void *a = (void *)0x10000000, *b = (void *)0x20000000, *w = (void *)0x30000000;
  const size_t wb = (size_t)1 << 20;
  CHECK(mgx_decompose(nullptr, b, MGX_F32, 3, d3, nullptr, 0, w, wb, nullptr) == MGX_ERR_ARG);
  CHECK(mgx_decompose(a, b, (mgx_dtype)7, 3, d3, nullptr, 0, w, wb, nullptr) == MGX_ERR_ARG);
  CHECK(mgx_decompose(a, a, MGX_F32, 3, d3, nullptr, 0, w, wb, nullptr) == MGX_ERR_ARG);
  CHECK(mgx_decompose(a, b, MGX_F32, 3, badshape, nullptr, 0, w, wb, nullptr) == MGX_ERR_SHAPE);
  CHECK(mgx_decompose(a, b, MGX_F32, 3, d3, nullptr, 0, w, 16, nullptr) == MGX_ERR_WORKSPACE);
  CHECK(mgx_recompose(a, b, MGX_F64, 3, d3, nullptr, 9, w, wb, nullptr) == MGX_ERR_LEVEL);
  CHECK(mgx_quantize(a, (int32_t *)b, MGX_F32, 3, d3, nullptr, -1.0, 0, 0.0, nullptr, nullptr) == MGX_ERR_TOL);
  CHECK(mgx_quantize(a, (int32_t *)b, MGX_F32, 3, d3, nullptr, NAN, 0, 0.0, nullptr, nullptr) == MGX_ERR_TOL);
  CHECK(mgx_dequantize((const int32_t *)a, b, MGX_F32, 3, d3, nullptr, 1.0, 0, 0.5, nullptr) == MGX_ERR_TOL);
  CHECK(mgx_decompose_quantize(a, nullptr, nullptr, MGX_F32, 3, d3, nullptr, 1.0, 0, 0.0, w, wb, nullptr,
                               nullptr) == MGX_ERR_ARG);
  CHECK(mgx_decompose_quantize(a, nullptr, (int32_t *)b, MGX_F32, 3, d3, nullptr, -2.0, 0, 0.0, w, wb, nullptr,
                               nullptr) == MGX_ERR_TOL);
  CHECK(mgx_dequantize_recompose(nullptr, nullptr, b, MGX_F32, 3, d3, nullptr, 1.0, 0, 0.0, w, wb, nullptr) ==
        MGX_ERR_ARG);
  CHECK(mgx_dequantize_recompose((const int32_t *)a, nullptr, b, MGX_F64, 3, d3, nullptr, 1.0, 0, 0.5, w, wb,
                                 nullptr) == MGX_ERR_TOL);
  const int64_t d4[4] = {5, 5, 5, 5};
  CHECK(mgx_decompose_quantize(a, nullptr, (int32_t *)b, MGX_F32, 4, d4, nullptr, 0.0, 0, 0.0, w, wb, nullptr,
                               nullptr) == MGX_ERR_TOL);
  double taul2[8];
  CHECK(mgx_level_tolerances_l2(3, d3, nullptr, 1.0, 0, NAN, taul2) == MGX_ERR_TOL);
  CHECK(mgx_level_tolerances_l2(3, d3, nullptr, 0.0, 0, 1.0, taul2) == MGX_ERR_TOL);
  // batches: workspace sizing only (host), including a field with stats
  mgx_quant_stats st;
  mgx_field f[3];
  std::memset(f, 0, sizeof(f));
  const int64_t fd[3][3] = {{33, 65, 33}, {17, 257, 0}, {129, 0, 0}};
  for (int i = 0; i < 3; i++) {
    f[i].dtype = i == 1 ? MGX_F64 : MGX_F32;
    f[i].ndim = 3 - i;
    for (int k = 0; k < f[i].ndim; k++) f[i].dims[k] = fd[i][k];
    f[i].stats = &st;
  }
  const size_t ws = mgx_batch_workspace_size(3, f);
  CHECK(ws >= mgx_workspace_size(MGX_F32, 3, fd[0], 0));
  f[1].dims[1] = 100;
  CHECK(mgx_batch_workspace_size(3, f) == 0);
  // dropping the caches, then building plans again
  const double c_before = mgx_linf_constant(3, fd[0], nullptr, 0);
  CHECK(mgx_release_cached() == MGX_OK);
  CHECK(mgx_linf_constant(3, fd[0], nullptr, 0) == c_before);
  CHECK(mgx_release_cached() == MGX_OK);
  for (int s = 0; s <= 8; s++) CHECK(mgx_status_string((mgx_status)s) != nullptr);
  CHECK(mgx_status_string((mgx_status)99) != nullptr);
  if (!g_fail) std::printf("host sanitizer driver: ok\n");
  return g_fail;
}
