// Selection of the kernel parameters (Section 5.1), p = 2.
//
// A net of 2N points (m + 1 digits) whose first N points form an m-digit net
// (true when every C_j is upper triangular: the last output digit does not
// depend on the first m index digits).  The spline is fitted to f at the
// first half and its cost is sum (f - Sf)^2 over the second half; the second
// half is the first half shifted by x_N (digital nets are groups), so Sf
// there is a group convolution of the spline coefficients with
// K(. (+) x_N, 0), computed with Walsh transforms (run_split_cost).  The
// weights are gamma_j = beta j^q; (alpha, beta, q) minimise the cost by the
// Nelder-Mead simplex method in the unconstrained coordinates
// (log(alpha - 1), log beta, q).
#include <algorithm>
#include <array>
#include <cmath>

#include "fdwt_internal.h"

namespace fdwt {

namespace {

struct Split {
  fdwt_net* tr = nullptr;        // the first half as an m-digit net
  std::vector<uint32_t> delta;   // x_N per coordinate, (m + 1)-digit integers
  float* ft = nullptr;           // forward transform of the first half's values
  const float* fval = nullptr;   // values at the second half
  hipStream_t st = nullptr;
  ~Split() {
    if (ft) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(ft);
    }
    if (tr) fdwt_net_free(tr);
  }
};

int split_setup(const Net& n2, const float* f2, Split& sp, hipStream_t st) {
  if (n2.p != 2) return fail(FDWT_EUNSUPPORTED, "kernel-parameter selection is defined for p = 2 (Section 5.1)");
  if (n2.m < 2) return fail(FDWT_EINVAL, "the net needs m >= 2 digits (two halves of at least 2 points)");
  const int m2 = n2.m, m = m2 - 1, s = n2.s;
  const int64_t N = int64_t(1) << m;
  auto C = [&](int j, int r, int c) { return (int)n2.C[((size_t)j * m2 + r) * m2 + c]; };
  for (int j = 0; j < s; ++j)
    for (int c = 0; c < m; ++c)
      if (C(j, m, c)) return fail(FDWT_EINVAL, "the first half of the net is not an m-digit net");
  std::vector<uint8_t> lead((size_t)s * m * m);
  for (int j = 0; j < s; ++j)
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < m; ++c) lead[((size_t)j * m + r) * m + c] = (uint8_t)C(j, r, c);
  if (int rc = fdwt_net_generate(2, m, s, lead.data(), &sp.tr)) return rc;
  sp.delta.assign(s, 0u);
  for (int j = 0; j < s; ++j)
    for (int r = 0; r < m2; ++r)
      if (C(j, r, m)) sp.delta[j] |= 1u << (m2 - 1 - r);
  sp.st = st;
  FDWT_HIP(hipMalloc(&sp.ft, (size_t)N * sizeof(float)));
  if (int rc = fwt_run(2, m, false, K_F32, f2, K_F32, K_F32, sp.ft, 1, 1.0 / (double)N, st)) return rc;
  sp.fval = f2 + N;
  return FDWT_OK;
}

int split_eval(Split& sp, const double prm[3], float* sf, double* cost) {
  Net& tr = sp.tr->n;
  std::vector<double> gam(tr.s);
  for (int j = 0; j < tr.s; ++j) gam[j] = prm[1] * std::pow((double)(j + 1), prm[2]);  // gamma_j = beta j^q
  const fdwt_kernel kern{prm[0], gam.data(), tr.s};
  return run_split_cost(tr, tr.sc, sp.delta.data(), sp.ft, sp.fval, &kern, sf, cost, sp.st);
}

std::array<double, 3> to_params(const std::array<double, 3>& th) {
  return {1.0 + std::exp(th[0]), std::exp(th[1]), th[2]};
}

}  // namespace

int split_cost_call(const Net& n2, const float* f2, const double prm[3], float* sf, double* cost, hipStream_t st) {
  Split sp;
  if (int rc = split_setup(n2, f2, sp, st)) return rc;
  return split_eval(sp, prm, sf, cost);
}

int kernel_tune_call(const Net& n2, const float* f2, const double start[3], int max_evals, fdwt_kernel_fit* out,
                     hipStream_t st) {
  Split sp;
  if (int rc = split_setup(n2, f2, sp, st)) return rc;
  using V = std::array<double, 3>;
  int evals = 0, rc = FDWT_OK;
  auto cost = [&](const V& th) {
    const V prm = to_params(th);
    double c = 0.0;
    if (!rc) rc = split_eval(sp, prm.data(), nullptr, &c);
    ++evals;
    return std::isfinite(c) ? c : HUGE_VAL;
  };
  // Initial simplex: the start and a step of 0.5 along each coordinate.
  std::array<V, 4> x;
  std::array<double, 4> fx;
  x[0] = {std::log(start[0] - 1.0), std::log(start[1]), start[2]};
  for (int i = 1; i < 4; ++i) {
    x[i] = x[0];
    x[i][i - 1] += 0.5;
  }
  for (int i = 0; i < 4; ++i) fx[i] = cost(x[i]);
  std::array<int, 4> ord = {0, 1, 2, 3};
  while (!rc && evals < max_evals) {
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return fx[a] < fx[b]; });
    const int b = ord[0], w = ord[3], sw = ord[2];
    double ext = 0.0;
    for (int i = 1; i < 4; ++i)
      for (int k = 0; k < 3; ++k) ext = std::max(ext, std::fabs(x[ord[i]][k] - x[b][k]));
    if (ext <= 1e-4 && fx[w] - fx[b] <= 1e-10 * std::fabs(fx[b]) + 1e-300) break;
    V c = {0.0, 0.0, 0.0};
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) c[k] += x[ord[i]][k] / 3.0;
    auto along = [&](double t) {  // c + t (c - x_w)
      V v;
      for (int k = 0; k < 3; ++k) v[k] = c[k] + t * (c[k] - x[w][k]);
      return v;
    };
    const V xr = along(1.0);
    const double fr = cost(xr);
    if (fr < fx[b]) {
      const V xe = along(2.0);
      const double fe = cost(xe);
      if (fe < fr) x[w] = xe, fx[w] = fe;
      else x[w] = xr, fx[w] = fr;
    } else if (fr < fx[sw]) {
      x[w] = xr, fx[w] = fr;
    } else {
      const bool outside = fr < fx[w];
      const V xc = along(outside ? 0.5 : -0.5);
      const double fc = cost(xc);
      if (fc < (outside ? fr : fx[w])) {
        x[w] = xc, fx[w] = fc;
      } else {  // shrink towards the best vertex
        for (int i = 1; i < 4; ++i) {
          const int v = ord[i];
          for (int k = 0; k < 3; ++k) x[v][k] = x[b][k] + 0.5 * (x[v][k] - x[b][k]);
          fx[v] = cost(x[v]);
        }
      }
    }
  }
  if (rc) return rc;
  int best = 0;
  for (int i = 1; i < 4; ++i)
    if (fx[i] < fx[best]) best = i;
  const V prm = to_params(x[best]);
  out->alpha = prm[0];
  out->beta = prm[1];
  out->q = prm[2];
  out->cost = fx[best];
  out->evaluations = evals;
  return FDWT_OK;
}

}  // namespace fdwt
