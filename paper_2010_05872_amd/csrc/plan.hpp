// Host-side level plan: per-axis, per-level tables for the HIP kernels.
//
// For every level l (1..L) and axis k the plan holds, in FP64 and FP32:
//   wl, wr  interpolation weights of the left/right nodal neighbour at each
//           odd node (operator Pi of Sec. 2; 1/2 and 1/2 on uniform axes),
//   w5      the load vector of the correction as one 5-point stencil per
//           coarse node: mass matrix apply followed by restriction fused
//           into one operator (Sec. 5.2, Lemma 1, generalised to per-node
//           spacings), so F_J = sum_d w5[J][d] z_{2J+d-2},
//   mult, invd, qsup  precomputed Thomas factors of the coarse mass matrix
//           (Sec. 5.4, reuse of intermediate variables): forward
//           f'_J = f_J - mult_J f'_{J-1}, backward
//           y_J = invd_J f'_J - qsup_J y_{J+1},
//   p5      the restriction R = P^T alone, in the layout of w5 (adjoint),
//   multb, invdb, qsub, mid  the same elimination run from the last row up
//           (g'_J = f_J - multb_J g'_{J+1}, y_J = invdb_J g'_J - qsub_J y_{J-1})
//           and the row K = c/2 where the two meet:
//           y_K = mid[0] (f_K - mid[1] f'_{K-1} - mid[2] g'_{K+1}).
// The common factor h_l of Sec. 5.4 needs no separate elimination: the
// factors are tabulated once per axis and level, so no per-element product
// with h_l remains.
#pragma once

#include <cstddef>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace mgx {

constexpr int kMaxLevels = 16;
constexpr int kMaxLog2 = 13;  // dims up to 2^13 + 1

struct AxisLevel {
  int64_t m = 1;       // fine (level-l) node count along the axis
  int64_t c = 1;       // coarse (level l-1) node count
  bool real = false;   // false for padded axes (ndim < 3)
  size_t off_wl = 0, off_wr = 0, off_w5 = 0, off_mult = 0, off_invd = 0, off_qsup = 0;
  // factors of the elimination from the last row upwards and of the middle
  // row, for the two-ended (twisted) factorization of the same matrix
  size_t off_multb = 0, off_invdb = 0, off_qsub = 0, off_mid = 0;
  // the restriction R = P^T alone as a 5-point stencil in the layout of w5
  // (0, weight of fine 2J-1, 1, weight of fine 2J+1, 0): used by the adjoint
  size_t off_p5 = 0;
};

struct Plan {
  int ndim = 0;
  int64_t n[3] = {1, 1, 1};  // padded to three axes, axis 2 contiguous
  bool real[3] = {false, false, false};
  int L = 0;
  std::vector<double> X[3];                  // fine coordinates
  AxisLevel ax[kMaxLevels][3];               // [l][k], l = 1..L
  double level_amp[kMaxLevels] = {};         // 1 + prod_k ||Mc^-1 R M||_inf at level l
  double axis_norm[kMaxLevels][3] = {};      // ||Mc^-1 R M||_inf of axis k at level l (real axes)
  std::vector<double> tab64;                 // all tables, FP64
  std::vector<float> tab32;                  // same, rounded to FP32
  // device copies, one per device ordinal
  std::mutex dev_mu;
  std::vector<void *> dtab64, dtab32;

  const void *device_tables(int device, bool fp64, int *hip_err);
  double linf_constant(int stop) const;
  // C_L2 of the L2 estimator (Sec. 4.1): max over levels stop..L of
  // prod_k (largest row sum of the axis mass matrix) / h_l^d, the level's
  // mass-matrix eigenvalue bound over its cell volume; 1 on uniform grids.
  double l2_constant(int stop) const;
};

// Shape checks shared by every entry point.  Returns 0 or an mgx_status.
int parse_shape(int ndim, const int64_t *dims, int64_t n[3], bool real[3], int *L);

// Looks up or builds the plan for (ndim, dims, coords).  Returns nullptr and
// sets *status on invalid coordinates.  Plans live until release_plans().
Plan *get_plan(int ndim, const int64_t *dims, const double *const *coords, int *status);

// Drops every cached plan and frees its device tables (after synchronizing
// each device that holds some; the current device is restored).  No other
// call of the library may run meanwhile.  Returns nonzero if the HIP runtime
// reported an error.
int release_plans();

}  // namespace mgx
