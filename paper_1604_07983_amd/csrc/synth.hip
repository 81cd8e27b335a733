// synth.hip -- the seeded synthetic propagators of synth.py generated on the
// device (input generation only; none of the method's arithmetic): the
// value at (seed, flavour, t, site, row, col) is a counter-based SplitMix64
// draw (Steele, Lea and Flood) turned into a complex normal deviate by the
// Box-Muller transform and damped by exp(-m ((t - t0) mod T)).  Integer
// steps are exact; the FP64 log, cos and sin may differ from the host's in
// the last bit.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ __launch_bounds__(256) void k_synth(T* out, uint64_t key, long long n_el, long long e0, double damp) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_el) return;
  const uint64_t n = 2 * (uint64_t)(e0 + i);
  const uint64_t z1 = mix64(key + (n + 1) * kGolden);
  const uint64_t z2 = mix64(key + (n + 2) * kGolden);
  const double u1 = ((double)(z1 >> 11) + 1.0) * 0x1p-53;
  const double u2 = (double)(z2 >> 11) * 0x1p-53;
  const double rad = sqrt(-log(u1));
  const double ang = 2.0 * 3.14159265358979323846 * u2;
  out[2 * i] = (T)(rad * cos(ang) * damp);
  out[2 * i + 1] = (T)(rad * sin(ang) * damp);
}

}  // namespace

extern "C" {

// One flavour's propagator on one slice t of an L^3 lattice into out
// ([V][12][12] complex, interleaved; complex128 if fp64 else complex64) on
// stream: key = SplitMix64 output 0 of the seed, damp = exp(-m ((t - t0) mod T))
// computed by the caller.  Returns 0 or a HIP error code.
int nbs_synth_slice(void* out, int fp64, uint64_t seed, long long V, int t, double damp, void* stream) {
  const uint64_t key = mix64(seed + kGolden);
  const long long n_el = V * 144;
  const long long e0 = (long long)t * V * 144;
  const unsigned blocks = (unsigned)((n_el + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL(k_synth<double>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (double*)out, key, n_el, e0,
                       damp);
  else
    hipLaunchKernelGGL(k_synth<float>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (float*)out, key, n_el, e0,
                       damp);
  return (int)hipGetLastError();
}

}  // extern "C"
