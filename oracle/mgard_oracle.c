/*
 * Plain FP64 CPU oracle for MGARD+ multilevel decomposition, recomposition
 * and level-wise quantization (arXiv 2010.05872).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may use it.  It shares no source, header, table or helper
 * with the HIP path.
 *
 * Everything here is single threaded, unblocked and unfused: it follows the
 * paper's definitions step by step so that a reader can check it by eye.
 *
 * Layout: arrays are C order with shape (n_0, ..., n_{d-1}); the last axis is
 * contiguous.  The multilevel coefficients u_mc are kept "interleaved", i.e.
 * indexed by the node of the finest grid N_L exactly as in Sec. 2 (u_mc[x]
 * holds the coefficient of the coarsest level that contains x).  The
 * level-centric layout of Sec. 5.1 is produced by mgo_level_centric_index.
 */
#include "mgard_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Grid hierarchy (Sec. 2, Table 1).                                          */
/* Axes are padded to MGO_D = 4 at the front: a padded axis has one node and  */
/* never coarsens.  1-D to 3-D fields and the 4-D fields of Sec. 6 share the  */
/* same code.                                                                 */
/* ------------------------------------------------------------------------ */

#define MGO_D 4

typedef struct {
  int d;              /* spatial dimension (number of real axes) */
  int64_t n[MGO_D];   /* node counts, padded axes have n = 1 */
  int real[MGO_D];    /* 1 for a real (coarsening) axis */
  double *X[MGO_D];   /* owned copies of the fine coordinates */
  int L;              /* finest level index */
} grid_t;

static int is_dyadic_plus_one(int64_t n, int *m) {
  if (n < 3) return 0;
  int64_t t = n - 1;
  int k = 0;
  while ((t & 1) == 0) { t >>= 1; k++; }
  if (t != 1) return 0;
  *m = k;
  return 1;
}

static void grid_free(grid_t *g) {
  for (int k = 0; k < MGO_D; k++) { free(g->X[k]); g->X[k] = NULL; }
}

/* The level count: every axis halves together, and the coarsest grid N_0 has
 * three nodes on the shortest axis (the example grids of Sec. 6 are
 * decomposed down to 3^d nodes). */
static int grid_init(grid_t *g, int ndim, const int64_t *dims,
                     const double *const *coords) {
  memset(g, 0, sizeof(*g));
  if (ndim < 1 || ndim > MGO_D || dims == NULL) return MGO_ERR_SHAPE;
  g->d = ndim;
  int mmin = 1 << 30;
  for (int k = 0; k < MGO_D; k++) {
    int src = k - (MGO_D - ndim);
    if (src < 0) { g->n[k] = 1; g->real[k] = 0; continue; }
    int m;
    if (!is_dyadic_plus_one(dims[src], &m)) return MGO_ERR_SHAPE;
    g->n[k] = dims[src];
    g->real[k] = 1;
    if (m < mmin) mmin = m;
  }
  g->L = mmin - 1;
  for (int k = 0; k < MGO_D; k++) {
    int src = k - (MGO_D - ndim);
    g->X[k] = (double *)malloc(sizeof(double) * (size_t)g->n[k]);
    if (!g->X[k]) { grid_free(g); return MGO_ERR_ALLOC; }
    for (int64_t i = 0; i < g->n[k]; i++) {
      double x = (src >= 0 && coords && coords[src]) ? coords[src][i] : (double)i;
      if (!isfinite(x)) { grid_free(g); return MGO_ERR_COORDS; }
      if (i > 0 && !(x > g->X[k][i - 1])) { grid_free(g); return MGO_ERR_COORDS; }
      g->X[k][i] = x;
    }
  }
  return MGO_OK;
}

/* Advances the multi-index j through the box m[0..MGO_D-1] in C order (last
 * axis fastest); returns 0 after the last index.  A loop over a whole box is
 * "j = 0; do { ... } while (next_index(j, m));" (boxes are never empty). */
static int next_index(int64_t *j, const int64_t *m) {
  for (int k = MGO_D - 1; k >= 0; k--) {
    if (++j[k] < m[k]) return 1;
    j[k] = 0;
  }
  return 0;
}

static int64_t box_total(const int64_t *m) {
  int64_t t = 1;
  for (int k = 0; k < MGO_D; k++) t *= m[k];
  return t;
}

/* Number of level-l nodes along axis k: N_l keeps every 2^(L-l)-th node. */
static int64_t level_size(const grid_t *g, int k, int l) {
  if (!g->real[k]) return 1;
  return (g->n[k] - 1) / ((int64_t)1 << (g->L - l)) + 1;
}

/* Level-l coordinates along axis k. */
static void level_coords(const grid_t *g, int k, int l, double *Xl) {
  int64_t s = (int64_t)1 << (g->L - l);
  int64_t m = level_size(g, k, l);
  for (int64_t j = 0; j < m; j++) Xl[j] = g->real[k] ? g->X[k][j * s] : 0.0;
}

/* ------------------------------------------------------------------------ */
/* One-dimensional building blocks on a line with nodes X_0 < ... < X_{m-1}. */
/* ------------------------------------------------------------------------ */

/* Weight of the left and right nodal neighbour when piecewise linear
 * interpolation predicts the odd node j from nodes j-1 and j+1 (Sec. 2,
 * operator Pi; on uniform grids both weights are 1/2, eq. of Sec. 4.2). */
static double w_left(const double *X, int64_t j)  { return (X[j + 1] - X[j]) / (X[j + 1] - X[j - 1]); }
static double w_right(const double *X, int64_t j) { return (X[j] - X[j - 1]) / (X[j + 1] - X[j - 1]); }

/* Mass matrix of the piecewise linear hat functions on X applied to g:
 * (Mg)_j = h_{j-1}/6 g_{j-1} + (h_{j-1}+h_j)/3 g_j + h_j/6 g_{j+1}
 * with h_j = X_{j+1}-X_j and terms beyond the ends dropped. */
void mgo_mass_apply_1d(const double *X, int64_t m, const double *g, double *out) {
  for (int64_t j = 0; j < m; j++) {
    double hl = (j > 0) ? X[j] - X[j - 1] : 0.0;
    double hr = (j < m - 1) ? X[j + 1] - X[j] : 0.0;
    double acc = (hl + hr) / 3.0 * g[j];
    if (j > 0) acc += hl / 6.0 * g[j - 1];
    if (j < m - 1) acc += hr / 6.0 * g[j + 1];
    out[j] = acc;
  }
}

/* Restriction R = P^T, P the prolongation by linear interpolation from the
 * even nodes: f_J = g_{2J} + w_right(2J-1) g_{2J-1} + w_left(2J+1) g_{2J+1}. */
void mgo_restrict_1d(const double *X, int64_t m, const double *g, double *f) {
  int64_t mc = (m + 1) / 2;
  for (int64_t J = 0; J < mc; J++) {
    int64_t j = 2 * J;
    double acc = g[j];
    if (j - 1 >= 0) acc += w_right(X, j - 1) * g[j - 1];
    if (j + 1 <= m - 1) acc += w_left(X, j + 1) * g[j + 1];
    f[J] = acc;
  }
}

/* Tridiagonal coarse mass matrix on the even nodes of X (spacing
 * H_J = X_{2J+2}-X_{2J}): sub H_{J-1}/6, diag (H_{J-1}+H_J)/3, sup H_J/6.
 * On a uniform grid of fine spacing h this is the matrix printed in Sec. 5.4. */
void mgo_coarse_mass_1d(const double *X, int64_t m, double *sub, double *diag, double *sup) {
  int64_t mc = (m + 1) / 2;
  for (int64_t J = 0; J < mc; J++) {
    double Hl = (J > 0) ? X[2 * J] - X[2 * J - 2] : 0.0;
    double Hr = (J < mc - 1) ? X[2 * J + 2] - X[2 * J] : 0.0;
    sub[J] = Hl / 6.0;
    diag[J] = (Hl + Hr) / 3.0;
    sup[J] = Hr / 6.0;
  }
}

/* Thomas algorithm (forward elimination, back substitution, no pivoting;
 * the coarse mass matrix is symmetric and diagonally dominant). In place. */
static void thomas_solve(int64_t mc, const double *sub, const double *diag,
                         const double *sup, double *f, double *work) {
  /* work holds the modified diagonal */
  work[0] = diag[0];
  for (int64_t J = 1; J < mc; J++) {
    double mult = sub[J] / work[J - 1];
    work[J] = diag[J] - mult * sup[J - 1];
    f[J] = f[J] - mult * f[J - 1];
  }
  f[mc - 1] = f[mc - 1] / work[mc - 1];
  for (int64_t J = mc - 2; J >= 0; J--) f[J] = (f[J] - sup[J] * f[J + 1]) / work[J];
}

/* L2 projection onto the coarse line of a fine-line function z:
 * y = Mc^{-1} R M z (mass apply, restriction, tridiagonal solve). */
void mgo_project_line_1d(const double *X, int64_t m, const double *z, double *y) {
  int64_t mc = (m + 1) / 2;
  double *g = (double *)malloc(sizeof(double) * (size_t)m);
  double *sub = (double *)malloc(sizeof(double) * (size_t)mc * 4);
  double *diag = sub + mc, *sup = sub + 2 * mc, *work = sub + 3 * mc;
  mgo_mass_apply_1d(X, m, z, g);
  mgo_restrict_1d(X, m, g, y);
  mgo_coarse_mass_1d(X, m, sub, diag, sup);
  thomas_solve(mc, sub, diag, sup, y, work);
  free(g);
  free(sub);
}

/* ------------------------------------------------------------------------ */
/* Correction computation (Sec. 2, step 4): the L2 projection onto V_{l-1} of */
/* the multilevel component z, one axis after the other, the contiguous axis  */
/* first ("row sweep, then column sweep", Sec. 5.1).                          */
/* z has level-l shape m[]; y receives the level-(l-1) shape.                 */
/* Along axis k the array is (outer, a[k], inner): outer the product of the   */
/* axes before k, inner of the axes after it; a line is one (outer, inner).  */
/* ------------------------------------------------------------------------ */
static int correction_box(const int64_t *m_in, const int *real,
                          double *const *Xl, const double *z, double *y) {
  int64_t a[MGO_D];
  for (int k = 0; k < MGO_D; k++) a[k] = m_in[k];
  double *cur = (double *)malloc(sizeof(double) * (size_t)box_total(a));
  if (!cur) return MGO_ERR_ALLOC;
  memcpy(cur, z, sizeof(double) * (size_t)box_total(a));
  for (int k = MGO_D - 1; k >= 0; k--) {
    if (!real[k]) continue;
    int64_t mk = a[k], mc = (mk + 1) / 2;
    int64_t outer = 1, inner = 1;
    for (int i = 0; i < k; i++) outer *= a[i];
    for (int i = k + 1; i < MGO_D; i++) inner *= a[i];
    double *next = (double *)malloc(sizeof(double) * (size_t)(outer * mc * inner));
    double *line = (double *)malloc(sizeof(double) * (size_t)mk);
    double *res = (double *)malloc(sizeof(double) * (size_t)mc);
    if (!next || !line || !res) { free(cur); free(next); free(line); free(res); return MGO_ERR_ALLOC; }
    for (int64_t o = 0; o < outer; o++) {
      for (int64_t i = 0; i < inner; i++) {
        for (int64_t j = 0; j < mk; j++) line[j] = cur[(o * mk + j) * inner + i];
        mgo_project_line_1d(Xl[k], mk, line, res);
        for (int64_t J = 0; J < mc; J++) next[(o * mc + J) * inner + i] = res[J];
      }
    }
    free(line);
    free(res);
    free(cur);
    cur = next;
    a[k] = mc;
  }
  memcpy(y, cur, sizeof(double) * (size_t)box_total(a));
  free(cur);
  return MGO_OK;
}

int mgo_correction(const double *z, double *y, int ndim, const int64_t *dims,
                   const double *const *coords) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, coords);
  if (st) return st;
  st = correction_box(g.n, g.real, g.X, z, y);
  grid_free(&g);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Level-l view of the interleaved array: level index (j_0, ..., j_3) is the */
/* fine node (j_0 s, ..., j_3 s), s = 2^(L-l).                                */
/* ------------------------------------------------------------------------ */
typedef struct {
  double *v;
  int64_t stride[MGO_D]; /* fine-array stride times s, per axis */
  int64_t m[MGO_D];
  double *Xl[MGO_D];
  int real[MGO_D];
} level_view_t;

static int view_init(level_view_t *w, const grid_t *g, double *v, int l) {
  int64_t s = (int64_t)1 << (g->L - l);
  int64_t fs[MGO_D];
  fs[MGO_D - 1] = 1;
  for (int k = MGO_D - 2; k >= 0; k--) fs[k] = fs[k + 1] * g->n[k + 1];
  w->v = v;
  for (int k = 0; k < MGO_D; k++) w->Xl[k] = NULL;
  for (int k = 0; k < MGO_D; k++) {
    w->real[k] = g->real[k];
    w->m[k] = level_size(g, k, l);
    w->stride[k] = g->real[k] ? fs[k] * s : 0;
    w->Xl[k] = (double *)malloc(sizeof(double) * (size_t)w->m[k]);
    if (!w->Xl[k]) return MGO_ERR_ALLOC;
    level_coords(g, k, l, w->Xl[k]);
  }
  return MGO_OK;
}

static void view_free(level_view_t *w) {
  for (int k = 0; k < MGO_D; k++) { free(w->Xl[k]); w->Xl[k] = NULL; }
}

static double *at(const level_view_t *w, const int64_t *j) {
  int64_t off = 0;
  for (int k = 0; k < MGO_D; k++) off += j[k] * w->stride[k];
  return w->v + off;
}

/* Piecewise multilinear interpolant Pi_{l-1} at the level-l node j, built
 * from the 2^(#odd axes) nodal corners (eq. of Sec. 4.2: edge, plane and cube
 * nodes use 2, 4 and 8 corners with weights 1/2, 1/4, 1/8 on uniform grids;
 * a node odd on all four axes of a 4-D grid uses 16). */
static double interpolant(const level_view_t *w, const int64_t *j) {
  int odd[MGO_D];
  for (int k = 0; k < MGO_D; k++) odd[k] = w->real[k] && (j[k] & 1);
  double pred = 0.0;
  for (int c = 0; c < (1 << MGO_D); c++) {
    int64_t q[MGO_D];
    double wt = 1.0;
    int skip = 0;
    for (int k = 0; k < MGO_D; k++) {
      int bit = (c >> k) & 1;
      if (!odd[k]) {
        if (bit) { skip = 1; break; }
        q[k] = j[k];
      } else if (bit == 0) {
        q[k] = j[k] - 1;
        wt *= w_left(w->Xl[k], j[k]);
      } else {
        q[k] = j[k] + 1;
        wt *= w_right(w->Xl[k], j[k]);
      }
    }
    if (skip) continue;
    pred += wt * *at(w, q);
  }
  return pred;
}

static int is_nodal(const level_view_t *w, const int64_t *j) {
  for (int k = 0; k < MGO_D; k++)
    if (w->real[k] && (j[k] & 1)) return 0;
  return 1;
}

/* The multilevel component (I - Pi_{l-1}) Q_l u as a level-l box: the value
 * stored at coefficient nodes, zero at nodal nodes. */
static double *component_box(const level_view_t *w) {
  double *z = (double *)malloc(sizeof(double) * (size_t)box_total(w->m));
  if (!z) return NULL;
  size_t t = 0;
  int64_t j[MGO_D] = {0};
  do {
    z[t++] = is_nodal(w, j) ? 0.0 : *at(w, j);
  } while (next_index(j, w->m));
  return z;
}

/* Level-(l-1) box size of the view. */
static void coarse_shape(const level_view_t *w, int64_t *mc) {
  for (int k = 0; k < MGO_D; k++) mc[k] = w->real[k] ? (w->m[k] + 1) / 2 : 1;
}

/* The level-l index of the nodal node with coarse index J. */
static void nodal_of(const level_view_t *w, const int64_t *J, int64_t *j) {
  for (int k = 0; k < MGO_D; k++) j[k] = w->real[k] ? 2 * J[k] : 0;
}

/* Add sign * y (level-(l-1) box) to the nodal values. */
static void apply_correction(const level_view_t *w, const double *y, double sign) {
  int64_t mc[MGO_D], J[MGO_D] = {0}, j[MGO_D];
  coarse_shape(w, mc);
  size_t t = 0;
  do {
    nodal_of(w, J, j);
    *at(w, j) += sign * y[t++];
  } while (next_index(J, mc));
}

static size_t coarse_total(const level_view_t *w) {
  int64_t mc[MGO_D];
  coarse_shape(w, mc);
  return (size_t)box_total(mc);
}

/* One decomposition step Q_l u -> (Q_{l-1} u, coefficients on N*_l), Sec. 2
 * steps 2-5. */
static int decompose_level(const grid_t *g, double *v, int l) {
  level_view_t w;
  int st = view_init(&w, g, v, l);
  if (st) { view_free(&w); return st; }
  /* steps 2+3 (coefficient computation): subtract the interpolant at every
   * coefficient node; nodal corners are never modified, so order is free. */
  {
    int64_t j[MGO_D] = {0};
    do {
      if (!is_nodal(&w, j)) {
        double pred = interpolant(&w, j);
        *at(&w, j) -= pred;
      }
    } while (next_index(j, w.m));
  }
  /* step 4 (correction computation) */
  double *z = component_box(&w);
  double *y = (double *)malloc(sizeof(double) * coarse_total(&w));
  if (!z || !y) { free(z); free(y); view_free(&w); return MGO_ERR_ALLOC; }
  st = correction_box(w.m, w.real, w.Xl, z, y);
  /* step 5 (correction application): nodal values become Q_{l-1} u */
  if (!st) apply_correction(&w, y, +1.0);
  free(z);
  free(y);
  view_free(&w);
  return st;
}

/* One recomposition step (Sec. 2, recomposition steps 2-4). */
static int recompose_level(const grid_t *g, double *v, int l) {
  level_view_t w;
  int st = view_init(&w, g, v, l);
  if (st) { view_free(&w); return st; }
  double *z = component_box(&w);
  double *y = (double *)malloc(sizeof(double) * coarse_total(&w));
  if (!z || !y) { free(z); free(y); view_free(&w); return MGO_ERR_ALLOC; }
  /* step 2: correction from the coefficients; step 3: subtract it */
  st = correction_box(w.m, w.real, w.Xl, z, y);
  if (!st) apply_correction(&w, y, -1.0);
  /* step 4: add the interpolant of the corrected nodal values */
  if (!st) {
    int64_t j[MGO_D] = {0};
    do {
      if (!is_nodal(&w, j)) {
        double pred = interpolant(&w, j);
        *at(&w, j) += pred;
      }
    } while (next_index(j, w.m));
  }
  free(z);
  free(y);
  view_free(&w);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Adjoint (transpose) of decomposition and recomposition.                   */
/* Not part of the paper: the transposes of the level maps above, written    */
/* out step by step in reverse order.  A decomposition level is              */
/*   D_l = (I + S^T C Z)(I - E),                                             */
/* E the interpolant at the coefficient nodes (zero rows at nodal nodes), Z  */
/* the restriction to coefficient nodes, C the per-axis projection of        */
/* correction_box and S^T the scatter of a coarse box onto the nodal nodes.  */
/* A recomposition level is R_l = (I + E)(I - S^T C Z).  So                  */
/*   D_l^T = (I - E^T)(I + Z C^T S),   R_l^T = (I - Z C^T S)(I + E^T),       */
/* with C^T = prod_k M P Mc^{-1} along each axis (M and Mc are symmetric and */
/* R = P^T).                                                                 */
/* ------------------------------------------------------------------------ */

/* Transpose of mgo_project_line_1d: out = M P Mc^{-1} y (coarse -> fine). */
void mgo_project_line_adjoint_1d(const double *X, int64_t m, const double *y, double *out) {
  int64_t mc = (m + 1) / 2;
  double *a = (double *)malloc(sizeof(double) * (size_t)mc);
  double *b = (double *)malloc(sizeof(double) * (size_t)m);
  double *sub = (double *)malloc(sizeof(double) * (size_t)mc * 4);
  double *diag = sub + mc, *sup = sub + 2 * mc, *work = sub + 3 * mc;
  memcpy(a, y, sizeof(double) * (size_t)mc);
  mgo_coarse_mass_1d(X, m, sub, diag, sup);
  thomas_solve(mc, sub, diag, sup, a, work);
  /* prolongation P: even nodes copy, odd nodes interpolate (transpose of R) */
  for (int64_t j = 0; j < m; j++) {
    if ((j & 1) == 0) b[j] = a[j / 2];
    else b[j] = w_left(X, j) * a[(j - 1) / 2] + w_right(X, j) * a[(j + 1) / 2];
  }
  mgo_mass_apply_1d(X, m, b, out);
  free(a);
  free(b);
  free(sub);
}

/* C^T: coarse box y (shape of the level-(l-1) grid) -> level-l box out.
 * The forward projection runs the axes from the last to the first; its
 * transpose runs them from the first to the last. */
static int correction_box_adjoint(const int64_t *m_out, const int *real,
                                  double *const *Xl, const double *y, double *out) {
  int64_t a[MGO_D];
  for (int k = 0; k < MGO_D; k++) a[k] = real[k] ? (m_out[k] + 1) / 2 : m_out[k];
  double *cur = (double *)malloc(sizeof(double) * (size_t)box_total(a));
  if (!cur) return MGO_ERR_ALLOC;
  memcpy(cur, y, sizeof(double) * (size_t)box_total(a));
  for (int k = 0; k < MGO_D; k++) {
    if (!real[k]) continue;
    int64_t mc = a[k], mk = m_out[k];
    int64_t outer = 1, inner = 1;
    for (int i = 0; i < k; i++) outer *= a[i];
    for (int i = k + 1; i < MGO_D; i++) inner *= a[i];
    double *next = (double *)malloc(sizeof(double) * (size_t)(outer * mk * inner));
    double *line = (double *)malloc(sizeof(double) * (size_t)mc);
    double *res = (double *)malloc(sizeof(double) * (size_t)mk);
    if (!next || !line || !res) { free(cur); free(next); free(line); free(res); return MGO_ERR_ALLOC; }
    for (int64_t o = 0; o < outer; o++) {
      for (int64_t i = 0; i < inner; i++) {
        for (int64_t J = 0; J < mc; J++) line[J] = cur[(o * mc + J) * inner + i];
        mgo_project_line_adjoint_1d(Xl[k], mk, line, res);
        for (int64_t j = 0; j < mk; j++) next[(o * mk + j) * inner + i] = res[j];
      }
    }
    free(line);
    free(res);
    free(cur);
    cur = next;
    a[k] = mk;
  }
  memcpy(out, cur, sizeof(double) * (size_t)box_total(a));
  free(cur);
  return MGO_OK;
}

/* sign * E^T: every coefficient node x sends weight * g(x) to each nodal
 * corner of its interpolant (the corner weights of interpolant()). */
static void scatter_interpolant_transpose(const level_view_t *w, double sign) {
  int64_t j[MGO_D] = {0};
  do {
    if (is_nodal(w, j)) continue;
    double gx = *at(w, j);
    int odd[MGO_D];
    for (int k = 0; k < MGO_D; k++) odd[k] = w->real[k] && (j[k] & 1);
    for (int c = 0; c < (1 << MGO_D); c++) {
      int64_t q[MGO_D];
      double wt = 1.0;
      int skip = 0;
      for (int k = 0; k < MGO_D; k++) {
        int bit = (c >> k) & 1;
        if (!odd[k]) {
          if (bit) { skip = 1; break; }
          q[k] = j[k];
        } else if (bit == 0) {
          q[k] = j[k] - 1;
          wt *= w_left(w->Xl[k], j[k]);
        } else {
          q[k] = j[k] + 1;
          wt *= w_right(w->Xl[k], j[k]);
        }
      }
      if (skip) continue;
      *at(w, q) += sign * wt * gx;
    }
  } while (next_index(j, w->m));
}

/* Nodal values of the level-l view as a coarse box (the operator S). */
static void gather_nodal(const level_view_t *w, double *y) {
  int64_t mc[MGO_D], J[MGO_D] = {0}, j[MGO_D];
  coarse_shape(w, mc);
  size_t t = 0;
  do {
    nodal_of(w, J, j);
    y[t++] = *at(w, j);
  } while (next_index(J, mc));
}

/* g(x) += sign * t(x) at the coefficient nodes (the operator Z^T). */
static void add_at_coefficients(const level_view_t *w, const double *t, double sign) {
  size_t i = 0;
  int64_t j[MGO_D] = {0};
  do {
    if (!is_nodal(w, j)) *at(w, j) += sign * t[i];
    i++;
  } while (next_index(j, w->m));
}

/* D_l^T = (I - E^T)(I + Z C^T S), applied in place to the level-l view. */
static int decompose_level_adjoint(const grid_t *g, double *v, int l) {
  level_view_t w;
  int st = view_init(&w, g, v, l);
  if (st) { view_free(&w); return st; }
  double *y = (double *)malloc(sizeof(double) * coarse_total(&w));
  double *t = (double *)malloc(sizeof(double) * (size_t)box_total(w.m));
  if (!y || !t) { free(y); free(t); view_free(&w); return MGO_ERR_ALLOC; }
  gather_nodal(&w, y);
  st = correction_box_adjoint(w.m, w.real, w.Xl, y, t);
  if (!st) {
    add_at_coefficients(&w, t, +1.0);
    scatter_interpolant_transpose(&w, -1.0);
  }
  free(y);
  free(t);
  view_free(&w);
  return st;
}

/* R_l^T = (I - Z C^T S)(I + E^T), applied in place to the level-l view. */
static int recompose_level_adjoint(const grid_t *g, double *v, int l) {
  level_view_t w;
  int st = view_init(&w, g, v, l);
  if (st) { view_free(&w); return st; }
  double *y = (double *)malloc(sizeof(double) * coarse_total(&w));
  double *t = (double *)malloc(sizeof(double) * (size_t)box_total(w.m));
  if (!y || !t) { free(y); free(t); view_free(&w); return MGO_ERR_ALLOC; }
  scatter_interpolant_transpose(&w, +1.0);
  gather_nodal(&w, y);
  st = correction_box_adjoint(w.m, w.real, w.Xl, y, t);
  if (!st) add_at_coefficients(&w, t, -1.0);
  free(y);
  free(t);
  view_free(&w);
  return st;
}

int mgo_decompose_adjoint(double *v, int ndim, const int64_t *dims,
                          const double *const *coords, int stop_level) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, coords);
  if (st) return st;
  if (stop_level < 0 || stop_level > g.L) { grid_free(&g); return MGO_ERR_LEVEL; }
  /* D = D_{stop+1} ... D_L, so D^T applies D_{stop+1}^T first */
  for (int l = stop_level + 1; l <= g.L && !st; l++) st = decompose_level_adjoint(&g, v, l);
  grid_free(&g);
  return st;
}

int mgo_recompose_adjoint(double *v, int ndim, const int64_t *dims,
                          const double *const *coords, int stop_level) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, coords);
  if (st) return st;
  if (stop_level < 0 || stop_level > g.L) { grid_free(&g); return MGO_ERR_LEVEL; }
  /* R = R_L ... R_{stop+1}, so R^T applies R_L^T first */
  for (int l = g.L; l > stop_level && !st; l--) st = recompose_level_adjoint(&g, v, l);
  grid_free(&g);
  return st;
}

int mgo_num_levels(int ndim, const int64_t *dims) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, NULL);
  if (st) return -st;
  int L = g.L;
  grid_free(&g);
  return L;
}

int mgo_decompose(double *v, int ndim, const int64_t *dims,
                  const double *const *coords, int stop_level) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, coords);
  if (st) return st;
  if (stop_level < 0 || stop_level > g.L) { grid_free(&g); return MGO_ERR_LEVEL; }
  for (int l = g.L; l > stop_level && !st; l--) st = decompose_level(&g, v, l);
  grid_free(&g);
  return st;
}

int mgo_recompose(double *v, int ndim, const int64_t *dims,
                  const double *const *coords, int stop_level) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, coords);
  if (st) return st;
  if (stop_level < 0 || stop_level > g.L) { grid_free(&g); return MGO_ERR_LEVEL; }
  for (int l = stop_level + 1; l <= g.L && !st; l++) st = recompose_level(&g, v, l);
  grid_free(&g);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Adaptive decomposition (Sec. 4.2, "Adaptive decomposition"; Alg. 1 lines  */
/* 1-16): before decomposing level l, compare the Lorenzo predictor with the */
/* multilinear interpolation on sampled 3^d blocks of Q_l u; stop where the  */
/* Lorenzo estimate is the lower one.                                         */
/* ------------------------------------------------------------------------ */

/* Penalty factors of Sec. 4.2 (3-D, in units of tau): Lorenzo, and the
 * interpolation's edge, plane and cube nodes. */
#define MGO_PEN_LORENZO 1.22
#define MGO_PEN_EDGE 0.369
#define MGO_PEN_PLANE 0.259
#define MGO_PEN_CUBE 0.182

/* Sums over the sampled blocks of level l (3-D fields only): one 3^3 block
 * (level-l cell) in four along every axis, the cells a with a % 4 == 1, so
 * that every Lorenzo neighbour (index - 1 on any subset of the axes) lies in
 * the grid.  For each coefficient node x of a sampled block (at least one odd
 * level index): s_lorenzo += |u(x) - Lorenzo prediction(x)|, s_interp +=
 * |u(x) - multilinear interpolant(x)|; counts[0..2] = sampled edge, plane and
 * cube nodes (1, 2, 3 odd indices).  v is the interleaved array holding
 * Q_l u on the level-l grid. */
int mgo_adaptive_estimate(const double *v, int ndim, const int64_t *dims, const double *const *coords,
                          int level, double *s_lorenzo, double *s_interp, int64_t *counts) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, coords);
  if (st) return st;
  if (g.d != 3) { grid_free(&g); return MGO_ERR_SHAPE; }
  if (level < 1 || level > g.L) { grid_free(&g); return MGO_ERR_LEVEL; }
  level_view_t w;
  st = view_init(&w, &g, (double *)v, level);
  if (st) { view_free(&w); grid_free(&g); return st; }
  double sl = 0.0, si = 0.0;
  int64_t cnt[3] = {0, 0, 0};
  int64_t cells[3];
  /* the three real axes of a 3-D field are axes 1..3 of the padded grid */
#define U3(a, b, c) (*at(&w, (const int64_t[MGO_D]){0, (a), (b), (c)}))
  for (int k = 0; k < 3; k++) cells[k] = (w.m[k + 1] - 1) / 2;
  for (int64_t a0 = 1; a0 < cells[0]; a0 += 4)
    for (int64_t a1 = 1; a1 < cells[1]; a1 += 4)
      for (int64_t a2 = 1; a2 < cells[2]; a2 += 4)
        for (int r0 = 0; r0 < 3; r0++)
          for (int r1 = 0; r1 < 3; r1++)
            for (int r2 = 0; r2 < 3; r2++) {
              int64_t j[MGO_D] = {0, 2 * a0 + r0, 2 * a1 + r1, 2 * a2 + r2};
              int nodd = (r0 == 1) + (r1 == 1) + (r2 == 1);
              if (nodd == 0) continue;
              int64_t x0 = j[1], x1 = j[2], x2 = j[3];
              double x = U3(x0, x1, x2);
              double lor = U3(x0, x1 - 1, x2) + U3(x0 - 1, x1, x2) + U3(x0, x1, x2 - 1) -
                           U3(x0 - 1, x1 - 1, x2) - U3(x0, x1 - 1, x2 - 1) - U3(x0 - 1, x1, x2 - 1) +
                           U3(x0 - 1, x1 - 1, x2 - 1);
              sl += fabs(x - lor);
              si += fabs(x - interpolant(&w, j));
              cnt[nodd - 1]++;
            }
#undef U3
  view_free(&w);
  grid_free(&g);
  *s_lorenzo = sl;
  *s_interp = si;
  for (int k = 0; k < 3; k++) counts[k] = cnt[k];
  return MGO_OK;
}

/* The estimated errors E_Lorenzo and E_interp of level l from the sums and
 * counts above and tau0, the coarsest level's tolerance when the
 * decomposition stops at l (Alg. 1 line 3: the level tolerances with stop
 * level l). */
void mgo_adaptive_errors(double s_lorenzo, double s_interp, const int64_t *counts, double tau0,
                         double *e_lorenzo, double *e_interp) {
  double n = (double)(counts[0] + counts[1] + counts[2]);
  *e_lorenzo = s_lorenzo + MGO_PEN_LORENZO * tau0 * n;
  *e_interp = s_interp + (MGO_PEN_EDGE * (double)counts[0] + MGO_PEN_PLANE * (double)counts[1] +
                          MGO_PEN_CUBE * (double)counts[2]) * tau0;
}

/* In place: decomposition of u (natural order) level by level from L, each
 * level preceded by the estimate; stops at the first level l whose Lorenzo
 * estimate is below the interpolation's (*stop_out = l), else at level 0.
 * The result equals mgo_decompose with stop level *stop_out. */
int mgo_decompose_adaptive(double *v, int ndim, const int64_t *dims, const double *const *coords,
                           double tol, double c_linf, int *stop_out) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, coords);
  if (st) return st;
  if (g.d != 3) { grid_free(&g); return MGO_ERR_SHAPE; }
  int L = g.L, stop = 0;
  double *tau = (double *)malloc(sizeof(double) * (size_t)(L + 1));
  if (!tau) { grid_free(&g); return MGO_ERR_ALLOC; }
  for (int l = L; l >= 1 && !st; l--) {
    st = mgo_level_tolerances(ndim, dims, coords, tol, l, c_linf, tau);
    if (st) break;
    double sl, si, el, ei;
    int64_t cnt[3];
    st = mgo_adaptive_estimate(v, ndim, dims, coords, l, &sl, &si, cnt);
    if (st) break;
    mgo_adaptive_errors(sl, si, cnt, tau[0], &el, &ei);
    if (el < ei) { stop = l; break; }
    st = decompose_level(&g, v, l);
  }
  free(tau);
  grid_free(&g);
  if (!st) *stop_out = stop;
  return st;
}

/* Progressive (partial) recomposition: the recomposition of Sec. 2 stopped
 * after level target_level.  The interleaved array then holds Q_target u on
 * the level-target grid N_target (the nodes whose indices are multiples of
 * 2^(L - target) on every real axis): the coarse representation that data
 * refactoring retrieves without the finer components (Sec. 1; the analysis
 * on decomposed representations of Sec. 6.2.2).  target = L is the full
 * recomposition; target = stop leaves the array unchanged. */
int mgo_recompose_to(double *v, int ndim, const int64_t *dims,
                     const double *const *coords, int stop_level, int target_level) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, coords);
  if (st) return st;
  if (stop_level < 0 || stop_level > g.L || target_level < stop_level || target_level > g.L) {
    grid_free(&g);
    return MGO_ERR_LEVEL;
  }
  for (int l = stop_level + 1; l <= target_level && !st; l++) st = recompose_level(&g, v, l);
  grid_free(&g);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Level membership and the level-centric reordering (Sec. 5.1).              */
/* ------------------------------------------------------------------------ */

/* Level of fine index i along one real axis: the coarsest level whose grid
 * contains it, with everything in N_{stop} reported as level stop. */
static int axis_level(int64_t i, int L, int stop) {
  int64_t sstop = (int64_t)1 << (L - stop);
  if (i % sstop == 0) return stop;
  int tz = 0;
  while (((i >> tz) & 1) == 0) tz++;
  return L - tz;
}

int mgo_level_map(int8_t *lev, int ndim, const int64_t *dims, int stop_level) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, NULL);
  if (st) return st;
  if (stop_level < 0 || stop_level > g.L) { grid_free(&g); return MGO_ERR_LEVEL; }
  size_t t = 0;
  int64_t i[MGO_D] = {0};
  do {
    int lv = stop_level;
    for (int k = 0; k < MGO_D; k++) {
      if (!g.real[k]) continue;
      int a = axis_level(i[k], g.L, stop_level);
      if (a > lv) lv = a;
    }
    lev[t++] = (int8_t)lv;
  } while (next_index(i, g.n));
  grid_free(&g);
  return MGO_OK;
}

/* Level-centric reordering of Sec. 5.1.  At every level l, from the finest
 * down, the level-l grid (which sits in the corner box [0, m_l) on every
 * axis) is reordered: along each axis its nodal (even) indices move to the
 * front, keeping their order, and its coefficient (odd) indices follow.  The
 * next level only reorders the nodal block (its own grid), so a level-l
 * coefficient stays where the level-l reordering put it.  A node of N*_l
 * with level indices j_k therefore lands at j_k/2 (even j_k) or
 * c_k + (j_k-1)/2 (odd j_k) on each axis, c_k the level-(l-1) node count;
 * a node of N_stop keeps its natural position in the stop-level box. */
int mgo_level_centric_index(int64_t *pos, int ndim, const int64_t *dims, int stop_level) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, NULL);
  if (st) return st;
  if (stop_level < 0 || stop_level > g.L) { grid_free(&g); return MGO_ERR_LEVEL; }
  size_t t = 0;
  int64_t i[MGO_D] = {0};
  do {
    int lv = stop_level;
    for (int k = 0; k < MGO_D; k++)
      if (g.real[k]) {
        int a = axis_level(i[k], g.L, stop_level);
        if (a > lv) lv = a;
      }
    int64_t s = (int64_t)1 << (g.L - lv);
    int64_t off = 0;
    for (int k = 0; k < MGO_D; k++) {
      int64_t j = i[k] / s; /* level-lv index (the node is in N_lv) */
      int64_t p;
      if (lv == stop_level) {
        p = j;
      } else {
        int64_t c = level_size(&g, k, lv - 1);
        p = (j & 1) ? c + (j - 1) / 2 : j / 2;
      }
      off = off * g.n[k] + p;
    }
    pos[t++] = off;
  } while (next_index(i, g.n));
  grid_free(&g);
  return MGO_OK;
}

/* ------------------------------------------------------------------------ */
/* L-infinity constant and level tolerances (Sec. 4.1).                       */
/* ------------------------------------------------------------------------ */

/* The paper takes C_{L^inf} from a cited analysis and prints no value.  This
 * oracle uses the rigorous per-level bound: a change delta of the level-l
 * coefficients moves the reconstruction by at most
 * (1 + prod_k ||Mc_k^{-1} R_k M_k||_inf) ||delta||_inf, and finer
 * recomposition steps only interpolate it.  The 1-D operator is built column
 * by column from unit vectors. */
double mgo_axis_operator_norm(const double *X, int64_t m) {
  int64_t mc = (m + 1) / 2;
  double *A = (double *)calloc((size_t)(mc * m), sizeof(double)); /* A[J*m + j] */
  double *e = (double *)calloc((size_t)m, sizeof(double));
  double *col = (double *)malloc(sizeof(double) * (size_t)mc);
  for (int64_t j = 0; j < m; j++) {
    memset(e, 0, sizeof(double) * (size_t)m);
    e[j] = 1.0;
    mgo_project_line_1d(X, m, e, col);
    for (int64_t J = 0; J < mc; J++) A[J * m + j] = col[J];
  }
  double best = 0.0;
  for (int64_t J = 0; J < mc; J++) {
    double s = 0.0;
    for (int64_t j = 0; j < m; j++) s += fabs(A[J * m + j]);
    if (s > best) best = s;
  }
  free(A);
  free(e);
  free(col);
  return best;
}

double mgo_linf_constant(int ndim, const int64_t *dims, const double *const *coords,
                         int stop_level) {
  grid_t g;
  if (grid_init(&g, ndim, dims, coords)) return -1.0;
  if (stop_level < 0 || stop_level > g.L) { grid_free(&g); return -1.0; }
  double C = 1.0;
  for (int l = g.L; l > stop_level; l--) {
    double prod = 1.0;
    for (int k = 0; k < MGO_D; k++) {
      if (!g.real[k]) continue;
      int64_t m = level_size(&g, k, l);
      double *Xl = (double *)malloc(sizeof(double) * (size_t)m);
      level_coords(&g, k, l, Xl);
      prod *= mgo_axis_operator_norm(Xl, m);
      free(Xl);
    }
    if (1.0 + prod > C) C = 1.0 + prod;
  }
  grid_free(&g);
  return C;
}

/* Level tolerances of eq. (LinfTau) with the stop level of Algorithm 1:
 * kappa = sqrt(2^d), tau_stop = (1-kappa)/(1-kappa^(L+1-stop)) * tau/C and
 * tau_l = kappa tau_{l-1}.  Fixed operation order, no contraction. */
int mgo_level_tolerances(int ndim, const int64_t *dims, const double *const *coords,
                         double tol, int stop_level, double c_linf, double *tau) {
  grid_t g;
  int st = grid_init(&g, ndim, dims, coords);
  if (st) return st;
  int L = g.L;
  grid_free(&g);
  if (stop_level < 0 || stop_level > L) return MGO_ERR_LEVEL;
  if (!(tol > 0.0) || !isfinite(tol)) return MGO_ERR_TOL;
  double C = c_linf;
  if (!(C > 0.0)) C = mgo_linf_constant(ndim, dims, coords, stop_level);
  if (!(C >= 1.0) || !isfinite(C)) return MGO_ERR_TOL;
  double kappa = sqrt((double)(1 << ndim));
  double p = 1.0;
  for (int i = 0; i < L + 1 - stop_level; i++) p = p * kappa;
  tau[0] = ((1.0 - kappa) / (1.0 - p)) * (tol / C);
  for (int l = 1; l <= L - stop_level; l++) tau[l] = tau[l - 1] * kappa;
  return MGO_OK;
}

/* ------------------------------------------------------------------------ */
/* Level-wise quantization (Sec. 4.1, Algorithm 1 quantize step).             */
/* Bins of width q_l = 2 tau_l anchored at zero; the reconstruction is the    */
/* bin centre label * q_l, so |c - c~| <= q_l / 2 = tau_l.                    */
/* ------------------------------------------------------------------------ */
int mgo_quantize(const double *u_mc, int32_t *labels, int ndim, const int64_t *dims,
                 const double *const *coords, double tol, int stop_level, double c_linf) {
  int L = mgo_num_levels(ndim, dims);
  if (L < 0) return -L;
  if (stop_level < 0 || stop_level > L) return MGO_ERR_LEVEL;
  double tau[64];
  int st = mgo_level_tolerances(ndim, dims, coords, tol, stop_level, c_linf, tau);
  if (st) return st;
  size_t total = 1;
  for (int k = 0; k < ndim; k++) total *= (size_t)dims[k];
  int8_t *lev = (int8_t *)malloc(total);
  if (!lev) return MGO_ERR_ALLOC;
  mgo_level_map(lev, ndim, dims, stop_level);
  int bad = 0;
  for (size_t t = 0; t < total; t++) {
    double q = 2.0 * tau[lev[t] - stop_level];
    double x = u_mc[t] / q;
    if (!isfinite(x) || fabs(x) >= 2147483647.0) { labels[t] = INT32_MIN; bad = 1; continue; }
    labels[t] = (int32_t)rint(x);
  }
  free(lev);
  return bad ? MGO_ERR_RANGE : MGO_OK;
}

int mgo_dequantize(const int32_t *labels, double *u_mc, int ndim, const int64_t *dims,
                   const double *const *coords, double tol, int stop_level, double c_linf) {
  int L = mgo_num_levels(ndim, dims);
  if (L < 0) return -L;
  if (stop_level < 0 || stop_level > L) return MGO_ERR_LEVEL;
  double tau[64];
  int st = mgo_level_tolerances(ndim, dims, coords, tol, stop_level, c_linf, tau);
  if (st) return st;
  size_t total = 1;
  for (int k = 0; k < ndim; k++) total *= (size_t)dims[k];
  int8_t *lev = (int8_t *)malloc(total);
  if (!lev) return MGO_ERR_ALLOC;
  mgo_level_map(lev, ndim, dims, stop_level);
  for (size_t t = 0; t < total; t++) {
    double q = 2.0 * tau[lev[t] - stop_level];
    u_mc[t] = (double)labels[t] * q;
  }
  free(lev);
  return MGO_OK;
}
