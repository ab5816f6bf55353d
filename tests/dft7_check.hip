// The 7-point DFT codelet (Rader's algorithm) run on the host against the
// definition y_h = sum_n x_n w^(n h), in float and double, both directions.
#include <hip/hip_runtime.h>
#include <cmath>
#include <complex>
#include <cstdio>
#include "dev_math.h"
using namespace fdwt;
template <bool INV, class C> double check() {
  double worst = 0;
  for (int trial = 0; trial < 100; ++trial) {
    C x[7]; std::complex<double> xr[7];
    for (int n = 0; n < 7; ++n) { double a = std::sin(1.3 * n + trial), b = std::cos(0.7 * n * n + 2 * trial); x[n].x = a; x[n].y = b; xr[n] = {a, b}; }
    Dft<7, INV>::run(x, 1);
    for (int h = 0; h < 7; ++h) {
      std::complex<double> r = 0;
      for (int n = 0; n < 7; ++n) r += xr[n] * std::polar(1.0, (INV ? 2 : -2) * M_PI * n * h / 7.0);
      worst = std::max(worst, std::abs(std::complex<double>(x[h].x, x[h].y) - r));
    }
  }
  return worst;
}
int main() {
  const double ef = std::max(check<false, float2>(), check<true, float2>());
  const double ed = std::max(check<false, double2>(), check<true, double2>());
  printf("float %.3g double %.3g\n", ef, ed);
  return (ef < 2e-6 && ed < 1e-13) ? 0 : 1;
}
