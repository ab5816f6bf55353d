// Test-function families sampled on the device (fdwt_sample), shared by the
// sampling kernels (net.hip) and the p = 2 first pass that samples its own
// input (fwt.hip): both evaluate f(x_n) with exactly these operations, in
// this order, so the fused transform equals sampling then transforming bit
// for bit.
#pragma once

#include "fdwt_internal.h"

namespace fdwt {

// Test-function families.  The first three work in float on x = X p^-m;
// the Asian payoff (Section 5.3) works in double on the exact quotient.
struct FamilyArgs {
  int s;
  float a[kMaxS];
  float inv1a[kMaxS];  // 1 / (1 + a_j), Section 5.2 function
  // Asian call: log S0, K, drift (r - sigma^2/2) T/s, sigma sqrt(T/s),
  // discount exp(-rT), 1/(s + 1) (the mean runs over S_0..S_s).
  double g[6];
};

// Standard normal quantile: the rational approximation 26.2.23 of
// Abramowitz and Stegun (absolute error below 4.5e-4) on the smaller tail,
// refined by three Newton steps on Phi(x) = erfc(-x/sqrt 2)/2 (quadratic
// convergence); u = 0 and u = 1 map to -inf and +inf.
__device__ __forceinline__ double inv_normal(double u) {
  if (u <= 0.0) return -INFINITY;
  if (u >= 1.0) return INFINITY;
  const double pl = u < 0.5 ? u : 1.0 - u;  // exact for u = X p^-m
  const double t = sqrt(-2.0 * log(pl));
  double x = -(t - (2.515517 + t * (0.802853 + t * 0.010328)) / (1.0 + t * (1.432788 + t * (0.189269 + t * 0.001308))));
  const double sqrt2pi = 2.5066282746310002;
  for (int k = 0; k < 3; ++k) {
    const double e = 0.5 * erfc(-x * 0.70710678118654752) - pl;  // Phi(x) - pl, accurate in the tail
    x -= e * sqrt2pi * exp(0.5 * x * x);
  }
  return u < 0.5 ? x : -x;
}

template <int FAM>
struct FamState {
  using T = float;
};
template <>
struct FamState<FDWT_FAMILY_ASIAN> {
  using T = double2;  // (log S_j, sum of S_1..S_j)
};

template <int FAM>
__device__ __forceinline__ typename FamState<FAM>::T fam_init(const FamilyArgs& fa) {
  if constexpr (FAM == FDWT_FAMILY_ASIAN) return make_double2(fa.g[0], exp(fa.g[0]));  // S_0 in the mean
  else return FAM == FDWT_FAMILY_EXP ? 0.0f : 1.0f;
}
// One coordinate: X its integer value, inv_f / inv_d the factor p^-m (inv_f
// is used only for p = 2, where it is a power of two).
template <int FAM, bool ODD>
__device__ __forceinline__ void fam_step(typename FamState<FAM>::T& acc, const FamilyArgs& fa, float a, float inv1a,
                                         uint32_t X, float inv_f, double inv_d) {
  if constexpr (FAM == FDWT_FAMILY_ASIAN) {
    acc.x += fa.g[2] + fa.g[3] * inv_normal((double)X * inv_d);
    acc.y += exp(acc.x);
  } else {
    const float x = ODD ? (float)((double)X * inv_d) : (float)X * inv_f;
    if constexpr (FAM == FDWT_FAMILY_PRODUCT) acc = acc * (1.0f + a * (x - 0.5f));
    else if constexpr (FAM == FDWT_FAMILY_EXP) acc = acc + a * x * x;
    else acc = acc * ((fabsf(4.0f * x - 2.0f) + a) * inv1a);
  }
}
template <int FAM>
__device__ __forceinline__ float fam_final(typename FamState<FAM>::T acc, const FamilyArgs& fa) {
  if constexpr (FAM == FDWT_FAMILY_ASIAN) return (float)(fa.g[4] * fmax(acc.y * fa.g[5] - fa.g[1], 0.0));
  else if constexpr (FAM == FDWT_FAMILY_EXP) return expf(-acc);
  else return acc;
}

// Family parameters for the device (a: the caller's fdwt_sample values).
FamilyArgs make_family_args(const Net& net, int family, const double* a);
// p = 2 forward transform of the family sampled on the device, with the
// sampling done inside the first pass (fwt.hip); FDWT_EUNSUPPORTED, with
// nothing enqueued, when the net is too small for that pass.
int fwt_p2_forward_family(const Net& net, int family, const FamilyArgs& fa, float* out, hipStream_t st);

}  // namespace fdwt
