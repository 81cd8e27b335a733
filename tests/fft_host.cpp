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

// The register-resident transform of fft_reg.hpp for the lengths the device
// code instantiates.
#include "fft_reg.hpp"

template <int N> static void reg_line(double* data, int sign) {
  nbs::cd v[N];
  for (int i = 0; i < N; ++i) v[i] = nbs::cd{data[2 * i], data[2 * i + 1]};
  if (sign < 0) nbs::fft_reg<N, -1>(v);
  else nbs::fft_reg<N, 1>(v);
  for (int i = 0; i < N; ++i) { data[2 * i] = v[i].re; data[2 * i + 1] = v[i].im; }
}

extern "C" int fft_reg_line_host(double* data, int n, int sign) {
  switch (n) {
#define NBS_REG_CASE(N) case N: reg_line<N>(data, sign); return 1;
    NBS_REG_CASE(2) NBS_REG_CASE(3) NBS_REG_CASE(4) NBS_REG_CASE(5) NBS_REG_CASE(6) NBS_REG_CASE(8)
    NBS_REG_CASE(10) NBS_REG_CASE(12) NBS_REG_CASE(16) NBS_REG_CASE(20) NBS_REG_CASE(24) NBS_REG_CASE(32)
    NBS_REG_CASE(40) NBS_REG_CASE(48)
#undef NBS_REG_CASE
  }
  return -1;
}

// The constexpr twiddle table against the C library's long double cos and
// sin (the extra precision keeps the reference's own argument rounding out
// of the comparison).
extern "C" double twiddle_max_err(int n) {
  long double err = 0;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int m = 0; m < n; ++m) {
    double c = 0, s = 0;
    nbs::ct::sincos_frac(m, n, c, s);
    const long double ph = 2.0L * pi * m / n;
    err = std::fmax(err, std::fabs((long double)c - std::cos(ph)));
    err = std::fmax(err, std::fabs((long double)s - std::sin(ph)));
  }
  return (double)err;
}
