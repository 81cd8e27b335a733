// fft.hpp -- building blocks of the in-house mixed-radix FFT (radix 2, 3, 4, 5).
//
// Each 1-D transform is a self-sorting Stockham sequence of radix-p stages:
// stage s with N_s = product of the radices already applied takes, for every
// butterfly j in [0, n/p), the p inputs in[j + r n/p], twiddles them by
// exp(sign 2 pi i (j mod N_s) r / (N_s p)), applies the length-p DFT and
// stores output r at (j div N_s) N_s p + (j mod N_s) + r N_s
// (Govindaraju et al., SC'08).  No bit reversal pass is needed.
//
// The functions are __host__ __device__ so the host test suite can run the
// same butterflies on the CPU against a library DFT.
#pragma once

#include "cx.hpp"

namespace nbs {

// Radices for n (4s first, then 2, 3, 5); returns the stage count or -1 if n
// has a prime factor above 5 or needs more than 8 stages.
__host__ __device__ inline int fft_factor(int n, int rad[8]) {
  int ns = 0;
  while (n % 4 == 0 && ns < 8) { rad[ns++] = 4; n /= 4; }
  while (n % 2 == 0 && ns < 8) { rad[ns++] = 2; n /= 2; }
  while (n % 3 == 0 && ns < 8) { rad[ns++] = 3; n /= 3; }
  while (n % 5 == 0 && ns < 8) { rad[ns++] = 5; n /= 5; }
  return n == 1 ? ns : -1;
}

// In-place length-P DFT, y_k = sum_r v_r exp(sign 2 pi i r k / P).
template <int P, typename T> __host__ __device__ inline void small_dft(cx<T>* v, int sign) {
  if constexpr (P == 2) {
    const cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (P == 4) {
    const cx<T> s02 = v[0] + v[2], d02 = v[0] - v[2], s13 = v[1] + v[3], d13 = v[1] - v[3];
    const cx<T> rot = mul_si(d13, sign);
    v[0] = s02 + s13;
    v[2] = s02 - s13;
    v[1] = d02 + rot;
    v[3] = d02 - rot;
  } else if constexpr (P == 3) {
    const T h = (T)0.86602540378443864676;  // sin(pi/3)
    const cx<T> t1 = v[1] + v[2], t2 = v[1] - v[2];
    const cx<T> m = v[0] - (T)0.5 * t1;
    const cx<T> rot = mul_si(h * t2, sign);
    v[0] = v[0] + t1;
    v[1] = m + rot;
    v[2] = m - rot;
  } else {
    static_assert(P == 5, "radix");
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;  // cos 2pi/5, cos 4pi/5
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;   // sin 2pi/5, sin 4pi/5
    const cx<T> a1 = v[1] + v[4], b1 = v[1] - v[4], a2 = v[2] + v[3], b2 = v[2] - v[3];
    const cx<T> m1 = v[0] + c1 * a1 + c2 * a2, m2 = v[0] + c2 * a1 + c1 * a2;
    const cx<T> r1 = mul_si(s1 * b1 + s2 * b2, sign), r2 = mul_si(s2 * b1 - s1 * b2, sign);
    v[0] = v[0] + a1 + a2;
    v[1] = m1 + r1;
    v[4] = m1 - r1;
    v[2] = m2 + r2;
    v[3] = m2 - r2;
  }
}

// One butterfly of a radix-P Stockham stage.  tw[m] = exp(sign 2 pi i m / n).
// Strides: element i of the line is at in[i * is] / out[i * os].
template <int P, typename T>
__host__ __device__ inline void stockham_butterfly_p(const cx<T>* in, int is, cx<T>* out, int os, int n, int Ns,
                                                     int j, const cx<T>* tw, int sign) {
  cx<T> v[P];
  const int stride = n / P;
  const int k = j % Ns;
#pragma unroll
  for (int r = 0; r < P; ++r) v[r] = in[(j + r * stride) * is];
  if (Ns > 1) {
    const int step = n / (Ns * P);
#pragma unroll
    for (int r = 1; r < P; ++r) v[r] = v[r] * tw[(k * r * step) % n];
  }
  small_dft<P>(v, sign);
  const int base = (j / Ns) * Ns * P + k;
#pragma unroll
  for (int r = 0; r < P; ++r) out[(base + r * Ns) * os] = v[r];
}

template <typename T>
__host__ __device__ inline void stockham_butterfly(const cx<T>* in, int is, cx<T>* out, int os, int n, int p,
                                                   int Ns, int j, const cx<T>* tw, int sign) {
  switch (p) {
    case 4: stockham_butterfly_p<4>(in, is, out, os, n, Ns, j, tw, sign); break;
    case 2: stockham_butterfly_p<2>(in, is, out, os, n, Ns, j, tw, sign); break;
    case 3: stockham_butterfly_p<3>(in, is, out, os, n, Ns, j, tw, sign); break;
    default: stockham_butterfly_p<5>(in, is, out, os, n, Ns, j, tw, sign); break;
  }
}

}  // namespace nbs
