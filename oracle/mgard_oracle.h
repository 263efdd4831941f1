/*
 * Plain FP64 CPU oracle for MGARD+ (arXiv 2010.05872) decomposition,
 * recomposition and level-wise quantization.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product library.
 *
 * Arrays are C order, last axis contiguous, and are indexed by the nodes of
 * the finest grid N_L ("interleaved" u_mc, Sec. 2).  coords is NULL or an
 * array of ndim pointers, each NULL (meaning 0, 1, ..., n-1) or n strictly
 * increasing finite values.  All functions are synchronous and allocate
 * their own scratch memory.
 */
#ifndef MGARD_ORACLE_H
#define MGARD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MGO_OK = 0,
  MGO_ERR_SHAPE = 2,   /* ndim not in [1,4] or some n_k not 2^m+1, m >= 1 */
  MGO_ERR_COORDS = 3,  /* non-finite or non-increasing coordinates */
  MGO_ERR_LEVEL = 4,   /* stop level outside [0, L] */
  MGO_ERR_TOL = 5,     /* tolerance not positive and finite, or C < 1 */
  MGO_ERR_RANGE = 6,   /* a quantization label does not fit int32 */
  MGO_ERR_ALLOC = 9
};

/* Finest level index L (coarsest grid has 3 nodes on the shortest axis),
 * or minus an error code. */
int mgo_num_levels(int ndim, const int64_t *dims);

/* In place: u (natural order) -> interleaved u_mc, levels L .. stop+1. */
int mgo_decompose(double *v, int ndim, const int64_t *dims,
                  const double *const *coords, int stop_level);
/* In place: interleaved u_mc -> u (exact inverse of mgo_decompose). */
int mgo_recompose(double *v, int ndim, const int64_t *dims,
                  const double *const *coords, int stop_level);

/* Adaptive decomposition (Sec. 4.2; Alg. 1 lines 1-16), 3-D fields only.
 * Sums of |u - Lorenzo prediction| and |u - multilinear interpolant| over the
 * coefficient nodes of the sampled 3^3 blocks of level `level` (cells a with
 * a % 4 == 1 per axis) of the interleaved array, and the sampled edge, plane
 * and cube node counts. */
int mgo_adaptive_estimate(const double *v, int ndim, const int64_t *dims, const double *const *coords,
                          int level, double *s_lorenzo, double *s_interp, int64_t *counts);
/* E_Lorenzo and E_interp: the sums plus the penalty factors times tau0. */
void mgo_adaptive_errors(double s_lorenzo, double s_interp, const int64_t *counts, double tau0,
                         double *e_lorenzo, double *e_interp);
/* In place: the adaptive decomposition; *stop_out receives the stop level. */
int mgo_decompose_adaptive(double *v, int ndim, const int64_t *dims, const double *const *coords,
                           double tol, double c_linf, int *stop_out);

/* In place: the recomposition stopped after level target_level (stop <=
 * target <= L); the level-target grid of v then holds Q_target u. */
int mgo_recompose_to(double *v, int ndim, const int64_t *dims,
                     const double *const *coords, int stop_level, int target_level);

/* Transposes (adjoints) of mgo_decompose and mgo_recompose, in place on the
 * interleaved layout: for all x, y, <D x, y> = <x, D^T y>. */
int mgo_decompose_adjoint(double *v, int ndim, const int64_t *dims,
                          const double *const *coords, int stop_level);
int mgo_recompose_adjoint(double *v, int ndim, const int64_t *dims,
                          const double *const *coords, int stop_level);
void mgo_project_line_adjoint_1d(const double *X, int64_t m, const double *y, double *out);

/* The correction Q_{l-1}(I - Pi_{l-1}) of a single level: z is a full
 * level box of shape dims (zeros expected at even-index nodes), y receives
 * the coarse box of shape (dims+1)/2. */
int mgo_correction(const double *z, double *y, int ndim, const int64_t *dims,
                   const double *const *coords);

/* One-dimensional pieces on a line of m nodes with coordinates X. */
void mgo_mass_apply_1d(const double *X, int64_t m, const double *g, double *out);
void mgo_restrict_1d(const double *X, int64_t m, const double *g, double *f);
void mgo_coarse_mass_1d(const double *X, int64_t m, double *sub, double *diag, double *sup);
void mgo_project_line_1d(const double *X, int64_t m, const double *z, double *y);
double mgo_axis_operator_norm(const double *X, int64_t m);

/* lev[t] = level of fine node t (levels at or below stop reported as stop). */
int mgo_level_map(int8_t *lev, int ndim, const int64_t *dims, int stop_level);
/* pos[t] = flat index of fine node t in the level-centric layout. */
int mgo_level_centric_index(int64_t *pos, int ndim, const int64_t *dims, int stop_level);

/* Rigorous L-infinity constant (C >= 1), or a negative value on bad input. */
double mgo_linf_constant(int ndim, const int64_t *dims, const double *const *coords,
                         int stop_level);
/* tau[0 .. L-stop] = tolerances of levels stop .. L.  c_linf <= 0 selects
 * mgo_linf_constant. */
int mgo_level_tolerances(int ndim, const int64_t *dims, const double *const *coords,
                         double tol, int stop_level, double c_linf, double *tau);

/* label = rint(c / (2 tau_level)); INT32_MIN and MGO_ERR_RANGE on overflow
 * or a non-finite quotient.  Interleaved layout. */
int mgo_quantize(const double *u_mc, int32_t *labels, int ndim, const int64_t *dims,
                 const double *const *coords, double tol, int stop_level, double c_linf);
int mgo_dequantize(const int32_t *labels, double *u_mc, int ndim, const int64_t *dims,
                   const double *const *coords, double tol, int stop_level, double c_linf);

#ifdef __cplusplus
}
#endif
#endif
