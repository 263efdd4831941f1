/* The C oracle under AddressSanitizer and UBSan (built by
 * tests/test_host_sanitizers.py): decomposition, recomposition (full and to
 * each level), adjoints, quantization, the level maps, the constants and the
 * adaptive decomposition on small 1-D to 4-D grids with default and random
 * coordinates, plus the error paths.  Exits nonzero on a wrong answer. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mgard_oracle.h"

static int fail = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      fail = 1;                                                    \
    }                                                              \
  } while (0)

static unsigned rng_state = 2010u;
static double rnd(void) {
  rng_state = rng_state * 1664525u + 1013904223u;
  return (double)(rng_state >> 8) / (double)(1u << 24) - 0.5;
}

int main(void) {
  const int64_t shapes[][4] = {{17, 0, 0, 0}, {9, 17, 0, 0}, {5, 9, 17, 0}, {9, 9, 9, 0}, {5, 9, 5, 9}};
  const int ndims[] = {1, 2, 3, 3, 4};
  for (int si = 0; si < 5; si++) {
    const int nd = ndims[si];
    const int64_t *d = shapes[si];
    int64_t n = 1;
    for (int k = 0; k < nd; k++) n *= d[k];
    const int L = mgo_num_levels(nd, d);
    CHECK(L >= 1);
    double *X[4] = {0};
    for (int k = 0; k < nd; k++) {
      X[k] = malloc(sizeof(double) * d[k]);
      double acc = 0.0;
      for (int64_t i = 0; i < d[k]; i++) X[k][i] = (acc += 0.6 + rnd());
    }
    const double *const *cs[2] = {NULL, (const double *const *)X};
    double *u = malloc(sizeof(double) * n), *v = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    int32_t *lab = malloc(sizeof(int32_t) * n);
    int8_t *lev = malloc(n);
    int64_t *pos = malloc(sizeof(int64_t) * n);
    for (int64_t i = 0; i < n; i++) u[i] = rnd();
    for (int c = 0; c < 2; c++) {
      for (int stop = 0; stop <= L; stop++) {
        memcpy(v, u, sizeof(double) * n);
        CHECK(mgo_decompose(v, nd, d, cs[c], stop) == MGO_OK);
        memcpy(w, v, sizeof(double) * n);
        CHECK(mgo_recompose(w, nd, d, cs[c], stop) == MGO_OK);
        double err = 0.0;
        for (int64_t i = 0; i < n; i++) err = fmax(err, fabs(w[i] - u[i]));
        CHECK(err < 1e-12);
        for (int t = stop; t <= L; t++) {
          memcpy(w, v, sizeof(double) * n);
          CHECK(mgo_recompose_to(w, nd, d, cs[c], stop, t) == MGO_OK);
        }
        memcpy(w, v, sizeof(double) * n);
        CHECK(mgo_decompose_adjoint(w, nd, d, cs[c], stop) == MGO_OK);
        CHECK(mgo_recompose_adjoint(w, nd, d, cs[c], stop) == MGO_OK);
        CHECK(mgo_quantize(v, lab, nd, d, cs[c], 1e-3, stop, 0.0) == MGO_OK);
        CHECK(mgo_dequantize(lab, w, nd, d, cs[c], 1e-3, stop, 0.0) == MGO_OK);
        CHECK(mgo_level_map(lev, nd, d, stop) == MGO_OK);
        CHECK(mgo_level_centric_index(pos, nd, d, stop) == MGO_OK);
        CHECK(mgo_linf_constant(nd, d, cs[c], stop) >= 1.0);
      }
      CHECK(mgo_decompose(v, nd, d, cs[c], L + 1) == MGO_ERR_LEVEL);
      if (nd == 3) {
        int stop = -1;
        memcpy(v, u, sizeof(double) * n);
        CHECK(mgo_decompose_adaptive(v, nd, d, cs[c], 1e-2, 0.0, &stop) == MGO_OK);
        CHECK(stop >= 0 && stop <= L);
      }
    }
    /* a NaN: the quantizer reports the range error */
    memcpy(v, u, sizeof(double) * n);
    v[n / 2] = NAN;
    CHECK(mgo_quantize(v, lab, nd, d, NULL, 1e-3, 0, 0.0) == MGO_ERR_RANGE);
    /* non-increasing coordinates */
    X[0][1] = X[0][0];
    CHECK(mgo_decompose(v, nd, d, (const double *const *)X, 0) == MGO_ERR_COORDS);
    for (int k = 0; k < nd; k++) free(X[k]);
    free(u);
    free(v);
    free(w);
    free(lab);
    free(lev);
    free(pos);
  }
  const int64_t bad[2] = {10, 9};
  CHECK(mgo_num_levels(2, bad) == -MGO_ERR_SHAPE);
  double X[9], Y[5];
  for (int i = 0; i < 9; i++) X[i] = i * i + i;
  double g[9], o[9], f[5], sub[5], diag[5], sup[5];
  for (int i = 0; i < 9; i++) g[i] = rnd();
  mgo_mass_apply_1d(X, 9, g, o);
  mgo_restrict_1d(X, 9, g, f);
  mgo_coarse_mass_1d(X, 9, sub, diag, sup);
  mgo_project_line_1d(X, 9, g, Y);
  CHECK(mgo_axis_operator_norm(X, 9) > 0.0);
  if (!fail) printf("oracle sanitizer driver: ok\n");
  return fail;
}
