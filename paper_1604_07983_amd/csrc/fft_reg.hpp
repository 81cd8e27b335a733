// fft_reg.hpp -- a whole length-N line transform held in registers.
//
// The same self-sorting Stockham stage sequence as fft.hpp (radix 4 first,
// then 2, 3, 5), but with N a template parameter: every loop is unrolled,
// every index and every twiddle factor is a compile-time constant, so one
// thread transforms one line without local memory or barriers.
//
// The twiddles exp(2 pi i m / N) come from a constexpr table.  cos and sin
// are evaluated at compile time by their Taylor series on [0, pi/4] after an
// exact reduction of the integer m (quadrant, then the half quadrant), which
// keeps them within an ulp or two of the correctly rounded values.
#pragma once

#include "cx.hpp"
#include "fft.hpp"

namespace nbs {

namespace ct {

constexpr double kPi = 3.14159265358979323846264338327950288;

// sin and cos of x in [0, pi/4] by their Taylor series (terms to x^27 and
// x^26), summed by Horner's rule from the smallest term.
constexpr void sincos_small(double x, double& s, double& c) {
  const double x2 = x * x;
  double ps = 1.0, pc = 1.0;
  for (int k = 13; k >= 1; --k) {
    ps = 1.0 - x2 / ((2.0 * k) * (2.0 * k + 1.0)) * ps;
    pc = 1.0 - x2 / ((2.0 * k - 1.0) * (2.0 * k)) * pc;
  }
  s = x * ps;
  c = pc;
}

// cos and sin of 2 pi m / n for integers 0 <= m < n.
constexpr void sincos_frac(int m, int n, double& c, double& s) {
  const int q = (4 * m) / n;   // quadrant
  int r = 4 * m - q * n;       // angle inside it = (pi/2) r / n
  bool swap = false;
  if (2 * r > n) {             // use the complement pi/2 - angle
    r = n - r;
    swap = true;
  }
  double sp = 0.0, cp = 0.0;
  sincos_small(0.5 * kPi * r / n, sp, cp);
  if (swap) {
    const double t = sp;
    sp = cp;
    cp = t;
  }
  switch (q) {
    case 0: c = cp; s = sp; break;
    case 1: c = -sp; s = cp; break;
    case 2: c = -cp; s = -sp; break;
    default: c = sp; s = -cp; break;
  }
}

template <int N> struct Twiddles {
  double c[N], s[N];
};

template <int N> constexpr Twiddles<N> make_twiddles() {
  Twiddles<N> t{};
  for (int m = 0; m < N; ++m) sincos_frac(m, N, t.c[m], t.s[m]);
  return t;
}

// Radix of stage S of a length-N transform (0 once the stages are done).
constexpr int radix_at(int n, int S) {
  int st = 0;
  for (int p : {4, 2, 3, 5}) {
    while (n % p == 0) {
      if (st == S) return p;
      n /= p;
      ++st;
    }
  }
  return 0;
}

constexpr bool supported(int n) {
  for (int p : {4, 2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

}  // namespace ct

// Stage S (stride NS = product of the radices already applied) and all later
// ones, in place on v.  SIGN is the sign of the exponent.
template <int N, int SIGN, int S, int NS, typename T>
__host__ __device__ inline void fft_reg_stage(cx<T> (&v)[N]) {
  constexpr int P = ct::radix_at(N, S);
  if constexpr (P != 0) {
    constexpr ct::Twiddles<N> tw = ct::make_twiddles<N>();
    constexpr int step = N / (NS * P);
    cx<T> w[N];
#pragma unroll
    for (int j = 0; j < N / P; ++j) {
      const int k = j % NS;
      cx<T> x[P];
#pragma unroll
      for (int r = 0; r < P; ++r) x[r] = v[j + r * (N / P)];
#pragma unroll
      for (int r = 1; r < P; ++r) {
        const int m = (k * r * step) % N;
        if (m != 0) x[r] = x[r] * cx<T>{(T)tw.c[m], (T)(SIGN * tw.s[m])};
      }
      small_dft<P>(x, SIGN);
      const int base = (j / NS) * NS * P + k;
#pragma unroll
      for (int r = 0; r < P; ++r) w[base + r * NS] = x[r];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = w[i];
    fft_reg_stage<N, SIGN, S + 1, NS * P>(v);
  }
}

// y_k = sum_m v_m exp(SIGN 2 pi i m k / N), in place, unnormalised.
template <int N, int SIGN, typename T> __host__ __device__ inline void fft_reg(cx<T> (&v)[N]) {
  static_assert(ct::supported(N), "FFT length must be 2,3,5-smooth");
  fft_reg_stage<N, SIGN, 0, 1>(v);
}

}  // namespace nbs
