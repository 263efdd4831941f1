// Level plan construction and caching (host).  See plan.hpp.
#include "plan.hpp"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <unordered_map>

#include "mgx.h"

namespace mgx {

int parse_shape(int ndim, const int64_t *dims, int64_t n[3], bool real[3], int *L) {
  if (ndim < 1 || ndim > 3 || dims == nullptr) return MGX_ERR_SHAPE;
  int mmin = 1 << 30;
  for (int k = 0; k < 3; k++) {
    int src = k - (3 - ndim);
    if (src < 0) {
      n[k] = 1;
      real[k] = false;
      continue;
    }
    int64_t v = dims[src];
    if (v < 3) return MGX_ERR_SHAPE;
    int64_t t = v - 1;
    int m = 0;
    while ((t & 1) == 0) {
      t >>= 1;
      m++;
    }
    if (t != 1 || m < 1 || m > kMaxLog2) return MGX_ERR_SHAPE;
    n[k] = v;
    real[k] = true;
    if (m < mmin) mmin = m;
  }
  *L = mmin - 1;
  return MGX_OK;
}

namespace {

// Tables of one axis at one level, built from the level-l coordinates Y
// (m nodes).  Appends to tab and records the offsets.
void build_axis(const std::vector<double> &Y, AxisLevel &a, std::vector<double> &tab) {
  const int64_t m = (int64_t)Y.size();
  const int64_t c = (m + 1) / 2;
  a.m = m;
  a.c = c;
  auto h = [&](int64_t j) { return (j >= 0 && j + 1 < m) ? Y[j + 1] - Y[j] : 0.0; };
  // interpolation weights at odd nodes
  a.off_wl = tab.size();
  for (int64_t j = 0; j < m; j++)
    tab.push_back((j & 1) ? (Y[j + 1] - Y[j]) / (Y[j + 1] - Y[j - 1]) : 0.0);
  a.off_wr = tab.size();
  for (int64_t j = 0; j < m; j++)
    tab.push_back((j & 1) ? (Y[j] - Y[j - 1]) / (Y[j + 1] - Y[j - 1]) : 0.0);
  // fine mass matrix rows: (M z)_j = lo_j z_{j-1} + di_j z_j + up_j z_{j+1}
  auto lo = [&](int64_t j) { return h(j - 1) / 6.0; };
  auto di = [&](int64_t j) { return (h(j - 1) + h(j)) / 3.0; };
  auto up = [&](int64_t j) { return h(j) / 6.0; };
  // restriction weights: coarse J collects fine 2J (1), 2J-1 (its right
  // interpolation weight) and 2J+1 (its left interpolation weight)
  auto rl = [&](int64_t J) {  // weight of fine 2J-1
    int64_t j = 2 * J - 1;
    return j >= 1 ? (Y[j] - Y[j - 1]) / (Y[j + 1] - Y[j - 1]) : 0.0;
  };
  auto rr = [&](int64_t J) {  // weight of fine 2J+1
    int64_t j = 2 * J + 1;
    return j <= m - 2 ? (Y[j + 1] - Y[j]) / (Y[j + 1] - Y[j - 1]) : 0.0;
  };
  // fused load-vector stencil (R M) on offsets -2..2 around fine 2J
  a.off_w5 = tab.size();
  for (int64_t J = 0; J < c; J++) {
    const int64_t j = 2 * J;
    double w[5] = {0, 0, 0, 0, 0};
    // row 2J of M, weight 1
    if (j - 1 >= 0) w[1] += lo(j);
    w[2] += di(j);
    if (j + 1 < m) w[3] += up(j);
    // row 2J-1 of M, weight rl
    if (j - 1 >= 0) {
      double r = rl(J);
      if (j - 2 >= 0) w[0] += r * lo(j - 1);
      w[1] += r * di(j - 1);
      w[2] += r * up(j - 1);
    }
    // row 2J+1 of M, weight rr
    if (j + 1 < m) {
      double r = rr(J);
      w[2] += r * lo(j + 1);
      w[3] += r * di(j + 1);
      if (j + 2 < m) w[4] += r * up(j + 1);
    }
    for (int d = 0; d < 5; d++) tab.push_back(w[d]);
  }
  // restriction alone, same layout (the transpose of the prolongation P)
  a.off_p5 = tab.size();
  for (int64_t J = 0; J < c; J++) {
    const int64_t j = 2 * J;
    tab.push_back(0.0);
    tab.push_back(j - 1 >= 0 ? rl(J) : 0.0);
    tab.push_back(1.0);
    tab.push_back(j + 1 < m ? rr(J) : 0.0);
    tab.push_back(0.0);
  }
  // coarse mass matrix on the even nodes and its Thomas factors
  std::vector<double> sub(c), dia(c), sup(c), dp(c);
  for (int64_t J = 0; J < c; J++) {
    double Hl = J > 0 ? Y[2 * J] - Y[2 * J - 2] : 0.0;
    double Hr = J + 1 < c ? Y[2 * J + 2] - Y[2 * J] : 0.0;
    sub[J] = Hl / 6.0;
    dia[J] = (Hl + Hr) / 3.0;
    sup[J] = Hr / 6.0;
  }
  a.off_mult = tab.size();
  std::vector<double> mult(c, 0.0);
  dp[0] = dia[0];
  for (int64_t J = 1; J < c; J++) {
    mult[J] = sub[J] / dp[J - 1];
    dp[J] = dia[J] - mult[J] * sup[J - 1];
  }
  for (int64_t J = 0; J < c; J++) tab.push_back(mult[J]);
  a.off_invd = tab.size();
  for (int64_t J = 0; J < c; J++) tab.push_back(1.0 / dp[J]);
  a.off_qsup = tab.size();
  for (int64_t J = 0; J < c; J++) tab.push_back(sup[J] / dp[J]);
  // elimination from the last row upwards
  std::vector<double> ep(c), multb(c, 0.0);
  ep[c - 1] = dia[c - 1];
  for (int64_t J = c - 2; J >= 0; J--) {
    multb[J] = sup[J] / ep[J + 1];
    ep[J] = dia[J] - multb[J] * sub[J + 1];
  }
  a.off_multb = tab.size();
  for (int64_t J = 0; J < c; J++) tab.push_back(multb[J]);
  a.off_invdb = tab.size();
  for (int64_t J = 0; J < c; J++) tab.push_back(1.0 / ep[J]);
  a.off_qsub = tab.size();
  for (int64_t J = 0; J < c; J++) tab.push_back(sub[J] / ep[J]);
  // the middle row K, where the two eliminations meet
  const int64_t K = c / 2;
  a.off_mid = tab.size();
  if (c >= 3) {
    const double al = sub[K] / dp[K - 1];
    const double be = sup[K] / ep[K + 1];
    tab.push_back(1.0 / (dia[K] - al * sup[K - 1] - be * sub[K + 1]));
    tab.push_back(al);
    tab.push_back(be);
  } else {
    tab.push_back(1.0 / dia[0]);
    tab.push_back(0.0);
    tab.push_back(0.0);
  }
}

// Trivial tables of a padded axis (one node, identity operators).
void build_padded(AxisLevel &a, std::vector<double> &tab) {
  a.m = 1;
  a.c = 1;
  a.real = false;
  a.off_wl = tab.size();
  tab.push_back(0.0);
  a.off_wr = tab.size();
  tab.push_back(0.0);
  a.off_w5 = tab.size();
  for (int d = 0; d < 5; d++) tab.push_back(d == 2 ? 1.0 : 0.0);
  a.off_p5 = tab.size();
  for (int d = 0; d < 5; d++) tab.push_back(d == 2 ? 1.0 : 0.0);
  a.off_mult = tab.size();
  tab.push_back(0.0);
  a.off_invd = tab.size();
  tab.push_back(1.0);
  a.off_qsup = tab.size();
  tab.push_back(0.0);
  a.off_multb = tab.size();
  tab.push_back(0.0);
  a.off_invdb = tab.size();
  tab.push_back(1.0);
  a.off_qsub = tab.size();
  tab.push_back(0.0);
  a.off_mid = tab.size();
  tab.push_back(1.0);
  tab.push_back(0.0);
  tab.push_back(0.0);
}

// ||Mc^-1 (R M)||_inf of one axis, from the tabulated stencil and factors:
// column j of R M has at most three nonzeros (coarse rows around j), and each
// column of the product is one tridiagonal solve.
double axis_norm(const AxisLevel &a, const std::vector<double> &tab) {
  const int64_t m = a.m, c = a.c;
  const double *w5 = &tab[a.off_w5];
  const double *mult = &tab[a.off_mult];
  const double *invd = &tab[a.off_invd];
  const double *qsup = &tab[a.off_qsup];
  std::vector<double> rowsum(c, 0.0), col(c);
  for (int64_t j = 0; j < m; j++) {
    std::fill(col.begin(), col.end(), 0.0);
    for (int64_t J = (j / 2 > 0 ? j / 2 - 1 : 0); J <= j / 2 + 1 && J < c; J++) {
      int64_t d = j - 2 * J + 2;
      if (d >= 0 && d < 5) col[J] = w5[5 * J + d];
    }
    for (int64_t J = 1; J < c; J++) col[J] -= mult[J] * col[J - 1];
    col[c - 1] *= invd[c - 1];
    for (int64_t J = c - 2; J >= 0; J--) col[J] = invd[J] * col[J] - qsup[J] * col[J + 1];
    for (int64_t J = 0; J < c; J++) rowsum[J] += std::fabs(col[J]);
  }
  double best = 0.0;
  for (double s : rowsum) best = s > best ? s : best;
  return best;
}

struct Cache {
  std::mutex mu;
  std::unordered_map<std::string, std::unique_ptr<Plan>> plans;
};

Cache &cache() {
  static Cache *c = new Cache();  // intentionally leaked: device tables live until exit
  return *c;
}

}  // namespace

double Plan::linf_constant(int stop) const {
  double C = 1.0;
  for (int l = L; l > stop; l--) C = level_amp[l] > C ? level_amp[l] : C;
  return C;
}

double Plan::l2_constant(int stop) const {
  double best = 0.0;
  for (int l = stop; l <= L; l++) {
    double ratio = 1.0;
    for (int k = 0; k < 3; k++) {
      if (!real[k]) continue;
      const int64_t s = (int64_t)1 << (L - l);
      const int64_t m = (n[k] - 1) / s + 1;
      // row j of the level's 1-D mass matrix sums to (h_{j-1} + h_j) / 2
      double rmax = 0.0;
      for (int64_t j = 0; j < m; j++) {
        const double hl = j > 0 ? X[k][j * s] - X[k][(j - 1) * s] : 0.0;
        const double hr = j + 1 < m ? X[k][(j + 1) * s] - X[k][j * s] : 0.0;
        const double r = (hl + hr) / 2.0;
        rmax = r > rmax ? r : rmax;
      }
      ratio *= rmax / ((X[k][n[k] - 1] - X[k][0]) / (double)(m - 1));
    }
    best = ratio > best ? ratio : best;
  }
  return best;
}

const void *Plan::device_tables(int device, bool fp64, int *hip_err) {
  std::lock_guard<std::mutex> g(dev_mu);
  auto &vec = fp64 ? dtab64 : dtab32;
  if ((int)vec.size() <= device) vec.resize(device + 1, nullptr);
  if (vec[device] == nullptr) {
    size_t bytes = fp64 ? tab64.size() * sizeof(double) : tab32.size() * sizeof(float);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      *hip_err = (int)e;
      return nullptr;
    }
    e = hipMemcpy(p, fp64 ? (const void *)tab64.data() : (const void *)tab32.data(), bytes,
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(p);
      *hip_err = (int)e;
      return nullptr;
    }
    vec[device] = p;
  }
  return vec[device];
}

int release_plans() {
  Cache &C = cache();
  std::lock_guard<std::mutex> g(C.mu);
  int err = 0, cur = -1;
  bool any = false;
  for (auto &kv : C.plans) {
    Plan &p = *kv.second;
    std::lock_guard<std::mutex> gd(p.dev_mu);
    for (std::vector<void *> *v : {&p.dtab64, &p.dtab32})
      for (size_t d = 0; d < v->size(); d++)
        if ((*v)[d]) {
          if (!any && hipGetDevice(&cur) != hipSuccess) cur = -1;
          any = true;
          // the tables may still be read by work enqueued on that device
          if (hipSetDevice((int)d) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
              hipFree((*v)[d]) != hipSuccess)
            err = 1;
          (*v)[d] = nullptr;
        }
  }
  C.plans.clear();
  if (any && cur >= 0 && hipSetDevice(cur) != hipSuccess) err = 1;
  return err;
}

Plan *get_plan(int ndim, const int64_t *dims, const double *const *coords, int *status) {
  int64_t n[3];
  bool real[3];
  int L;
  int st = parse_shape(ndim, dims, n, real, &L);
  if (st) {
    *status = st;
    return nullptr;
  }
  // key: ndim, dims and the raw coordinate bytes (or a marker for defaults)
  std::string key;
  key.append((const char *)&ndim, sizeof(ndim));
  for (int k = 0; k < 3; k++) key.append((const char *)&n[k], sizeof(int64_t));
  for (int k = 0; k < ndim; k++) {
    const double *ck = coords ? coords[k] : nullptr;
    char tag = ck ? 1 : 0;
    key.push_back(tag);
    if (ck) key.append((const char *)ck, sizeof(double) * (size_t)dims[k]);
  }
  Cache &C = cache();
  {
    std::lock_guard<std::mutex> g(C.mu);
    auto it = C.plans.find(key);
    if (it != C.plans.end()) return it->second.get();
  }
  auto p = std::make_unique<Plan>();
  p->ndim = ndim;
  p->L = L;
  for (int k = 0; k < 3; k++) {
    p->n[k] = n[k];
    p->real[k] = real[k];
    int src = k - (3 - ndim);
    p->X[k].resize(n[k]);
    for (int64_t i = 0; i < n[k]; i++) {
      double x = (src >= 0 && coords && coords[src]) ? coords[src][i] : (double)i;
      if (!std::isfinite(x) || (i > 0 && !(x > p->X[k][i - 1]))) {
        *status = MGX_ERR_COORDS;
        return nullptr;
      }
      p->X[k][i] = x;
    }
  }
  for (int l = 1; l <= L; l++) {
    double prod = 1.0;
    for (int k = 0; k < 3; k++) {
      AxisLevel &a = p->ax[l][k];
      if (!real[k]) {
        build_padded(a, p->tab64);
        continue;
      }
      a.real = true;
      int64_t s = (int64_t)1 << (L - l);
      std::vector<double> Y;
      for (int64_t i = 0; i < n[k]; i += s) Y.push_back(p->X[k][i]);
      build_axis(Y, a, p->tab64);
      p->axis_norm[l][k] = axis_norm(a, p->tab64);
      prod *= p->axis_norm[l][k];
    }
    p->level_amp[l] = 1.0 + prod;
  }
  if (p->tab64.empty()) p->tab64.push_back(0.0);  // L = 0: no levels, keep a valid device allocation
  p->tab32.resize(p->tab64.size());
  for (size_t i = 0; i < p->tab64.size(); i++) p->tab32[i] = (float)p->tab64[i];
  std::lock_guard<std::mutex> g(C.mu);
  auto it = C.plans.find(key);
  if (it != C.plans.end()) return it->second.get();
  Plan *raw = p.get();
  C.plans.emplace(std::move(key), std::move(p));
  return raw;
}

}  // namespace mgx
