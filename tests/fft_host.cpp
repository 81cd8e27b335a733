// Host build of the product's FFT butterflies (test code only): runs the
// Stockham stage sequence of fft.hpp on one line so the host test suite can
// compare it with numpy's FFT.
#include "fft.hpp"

#include <cmath>
#include <vector>

extern "C" int fft_line_host(double* data, int n, int sign) {
  using nbs::cd;
  int rad[8];
  const int ns = nbs::fft_factor(n, rad);
  if (ns < 0) return -1;
  std::vector<cd> a(n), b(n), tw(n);
  for (int i = 0; i < n; ++i) a[i] = cd{data[2 * i], data[2 * i + 1]};
  for (int m = 0; m < n; ++m) {
    const double ph = 2.0 * M_PI * m / n;
    tw[m] = cd{std::cos(ph), sign * std::sin(ph)};
  }
  cd* src = a.data();
  cd* dst = b.data();
  int Ns = 1;
  for (int s = 0; s < ns; ++s) {
    const int p = rad[s];
    for (int j = 0; j < n / p; ++j) nbs::stockham_butterfly(src, 1, dst, 1, n, p, Ns, j, tw.data(), sign);
    std::swap(src, dst);
    Ns *= p;
  }
  for (int i = 0; i < n; ++i) { data[2 * i] = src[i].re; data[2 * i + 1] = src[i].im; }
  return ns;
}
