// kernels.hip -- HIP kernels for gfx950 (MI355X) of the NBS four-point function.
//
//   k_nbb       normal baryon blocks, Eq. (5) / Sec. 3(i) Eq. (8)
//   k_fft_pass  one axis of the in-house batched 3-D FFT (Eq. (6))
//   k_contract  effective blocks and their products, Sec. 3(ii)-(iii),
//               Eqs. (9)-(10), driven by the compiled SoA program
//   k_absmax / k_scale_exps / k_channel_scale   per-slice power-of-two
//               scale of the precision form and its exact undo
#include <hip/hip_runtime.h>

#include "cx.hpp"
#include "fft.hpp"
#include "kernels.hpp"

namespace nbs {

// ---------------------------------------------------------------------------
// per-slice scale (precision form): max |Re|,|Im| of each flavour on each
// slice, kept as float bits (monotone for non-negative floats, so the
// atomic max is exact and order independent).
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(unsigned* p, unsigned v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kThreads) void k_absmax(const cf* S, unsigned* maxbits, long long per_slice) {
  const int t = blockIdx.y;
  const cf* base = S + (long long)t * per_slice;
  float m = 0.f;
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < per_slice;
       i += (long long)gridDim.x * kThreads) {
    const cf v = base[i];
    m = fmaxf(m, fmaxf(fabsf(v.re), fabsf(v.im)));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  __shared__ float red[kThreads / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) m = fmaxf(m, red[w]);
    atomicMax(&maxbits[t], __float_as_uint(m));
  }
}

__global__ void k_scale_exps(const unsigned* maxbits, int* exps, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float m = __uint_as_float(maxbits[i]);
  int e = 0;
  if (m > 0.f) frexpf(m, &e);  // m = f 2^e, f in [0.5, 1): S 2^-e has max in [0.5, 1)
  exps[i] = e;
}

__global__ void k_channel_scale(const int* exps, const int* chan_nf, double* oscale, int n_ch, int t_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ch * t_count) return;
  const int c = i / t_count, t = i % t_count;
  int e = 0;
  for (int f = 0; f < 3; ++f) e += chan_nf[3 * c + f] * exps[f * t_count + t];
  oscale[i] = ldexp(1.0, e);
}

// ---------------------------------------------------------------------------
// Normal baryon blocks.  One workgroup per (site, slice): the three
// propagators are staged in LDS, the diquarks
//   D_{f1 f2}[c][j1][j2] = sum eps_abc (C g5)_{be ga} S_f1[(be,a)][j1] S_f2[(ga,b)][j2]
// are formed once per flavour pair, then every block
//   N_{f1 f2 f3}[al][j1][j2][j3] = sum_c D_{f1 f2}[c][j1][j2] S_f3[(al,c)][j3]
// is written as 3456 contiguous complex values.
// ---------------------------------------------------------------------------
template <typename Tin, typename T>
__global__ __launch_bounds__(kThreads) void k_nbb(NbbArgs a) {
  __shared__ cx<T> S[3][144];
  __shared__ cx<T> D[4][432];  // octet operators need at most 4 diquark flavour pairs
  const int site = blockIdx.x, t = blockIdx.y;
  const long long sbase = ((long long)t * a.V + site) * 144;
  for (int i = threadIdx.x; i < 3 * 144; i += kThreads) {
    const int f = i / 144, e = i % 144;
    if (!a.flavour_used[f]) continue;
    const cx<Tin> v = reinterpret_cast<const cx<Tin>*>(a.S[f])[sbase + e];
    T sc = (T)1;
    if (a.scale_exp) sc = (T)ldexp(1.0, -a.scale_exp[f * a.t_count + t]);
    S[f][e] = cx<T>{(T)v.re * sc, (T)v.im * sc};
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a.n_dq * 432; i += kThreads) {
    const int d = i / 432, r = i % 432;
    const int c = r / 144, j1 = (r / 12) % 12, j2 = r % 12;
    const cx<T>* S1 = S[a.dq_f1[d]];
    const cx<T>* S2 = S[a.dq_f2[d]];
    cx<T> acc{0, 0};
    // eps_abc: (a,b) = (c+1, c+2) is cyclic (+1), (c+2, c+1) anti-cyclic (-1)
#pragma unroll
    for (int cyc = 0; cyc < 2; ++cyc) {
      const int ca = cyc == 0 ? (c + 1) % 3 : (c + 2) % 3;
      const int cb = cyc == 0 ? (c + 2) % 3 : (c + 1) % 3;
      const T e = cyc == 0 ? (T)1 : (T)-1;
#pragma unroll
      for (int be = 0; be < 4; ++be) {
        const int ga = be ^ 1;                 // (C g5)_{be, be^1} = +1 for even be, -1 for odd
        const T g = (be & 1) ? -e : e;
        const cx<T> p = S1[(3 * be + ca) * 12 + j1] * S2[(3 * ga + cb) * 12 + j2];
        acc.re = fma(g, p.re, acc.re);
        acc.im = fma(g, p.im, acc.im);
      }
    }
    D[d][r] = acc;
  }
  __syncthreads();
  for (int slot = 0; slot < a.n_types; ++slot) {
    const cx<T>* Dd = D[a.type_dq[slot]];
    const cx<T>* S3 = S[a.type_f3[slot]];
    cx<T>* out = reinterpret_cast<cx<T>*>(a.Nq) + ((long long)(t * a.n_types + slot) * a.V + site) * kBlockEntries;
    for (int o = threadIdx.x; o < kBlockEntries; o += kThreads) {
      const int al = o / 1728, j12 = (o / 12) % 144, j3 = o % 12;
      cx<T> v{0, 0};
#pragma unroll
      for (int c = 0; c < 3; ++c) cmac(v, Dd[c * 144 + j12], S3[(3 * al + c) * 12 + j3]);
      out[o] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// One axis of the batched 3-D DFT in FP64 arithmetic.  A workgroup takes a
// tile of OB outer indices x IB contiguous inner indices x the full length n,
// stages it in LDS (coalesced: runs of IB consecutive elements), runs the
// Stockham stages on every line and writes the tile back.
// ---------------------------------------------------------------------------
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kThreads) void k_fft_pass(FftArgs a) {
  extern __shared__ cd smem_fft[];
  const int n = a.n, IB = a.IB, OB = a.OB, ld = n + 1;
  const long long n_itiles = a.inner / IB;
  const long long tile = blockIdx.x;
  const long long o0 = (tile / n_itiles) * OB, i0 = (tile % n_itiles) * IB;
  const int ob = (int)((a.outer - o0) < OB ? (a.outer - o0) : OB);
  const int lines = ob * IB;
  cd* tw = smem_fft;
  cd* A = tw + n;
  cd* B = A + OB * IB * ld;
  for (int m = threadIdx.x; m < n; m += kThreads) {
    double s, c;
    sincospi(2.0 * m / n, &s, &c);
    tw[m] = cd{c, a.sign * s};
  }
  const cx<Tin>* in = reinterpret_cast<const cx<Tin>*>(a.in);
  const int total = lines * n;
  for (int e = threadIdx.x; e < total; e += kThreads) {
    const int ib = e % IB, rest = e / IB, in_ = rest % n, o = rest / n;
    const long long g = ((o0 + o) * n + in_) * a.inner + i0 + ib;
    A[(o * IB + ib) * ld + in_] = conv<double>(in[g]);
  }
  __syncthreads();
  int rad[8];
  const int ns = fft_factor(n, rad);
  cd* src = A;
  cd* dst = B;
  int Ns = 1;
  for (int s = 0; s < ns; ++s) {
    const int p = rad[s], nb = n / p, work = lines * nb;
    for (int w = threadIdx.x; w < work; w += kThreads) {
      const int line = w / nb, j = w % nb;
      stockham_butterfly(src + line * ld, 1, dst + line * ld, 1, n, p, Ns, j, tw, a.sign);
    }
    __syncthreads();
    cd* tmp = src;
    src = dst;
    dst = tmp;
    Ns *= p;
  }
  cx<Tout>* out = reinterpret_cast<cx<Tout>*>(a.out);
  for (int e = threadIdx.x; e < total; e += kThreads) {
    const int ib = e % IB, rest = e / IB, in_ = rest % n, o = rest / n;
    const long long g = ((o0 + o) * n + in_) * a.inner + i0 + ib;
    double f = a.gscale;
    if (a.oscale) f *= a.oscale[(o0 + o) / a.oscale_div];
    const cd v = src[(o * IB + ib) * ld + in_];
    out[g] = conv<Tout>(cd{v.re * f, v.im * f});
  }
}

// ---------------------------------------------------------------------------
// Effective blocks and their products.  One workgroup per (channel group,
// momentum q, slice) runs the group's chunks:
//   load N~_type(+q or -q) into LDS (when the program says so),
//   EBB: E[e] += sum_terms coef * N~[idx]           (Eq. (9), SoA tables)
//   MEB: partial[item][r1, r2] = sum_k E1[r1][k] E2[r2][k]   (Eq. (10))
//   ACC: F~[channel][spin] += sum coef * partial      (sum over diagrams)
// The blockIdx -> work mapping keeps every group of one momentum on the same
// XCD so they share N~(q), N~(-q) in that XCD's L2.
// ---------------------------------------------------------------------------
template <typename T, int R1>
__device__ inline void meb_item(const cx<T>* E, int e1, int e2, int K, int k0, int kn, cx<T>* out) {
  constexpr int R2 = 16 / R1;
  cx<T> acc[16];
#pragma unroll
  for (int o = 0; o < 16; ++o) acc[o] = cx<T>{0, 0};
  for (int k = k0; k < k0 + kn; ++k) {
    cx<T> x[R1], y[R2];
#pragma unroll
    for (int r = 0; r < R1; ++r) x[r] = E[e1 + r * K + k];
#pragma unroll
    for (int r = 0; r < R2; ++r) y[r] = E[e2 + r * K + k];
#pragma unroll
    for (int r1 = 0; r1 < R1; ++r1)
#pragma unroll
      for (int r2 = 0; r2 < R2; ++r2) cmac(acc[r1 * R2 + r2], x[r1], y[r2]);
  }
#pragma unroll
  for (int o = 0; o < 16; ++o) out[o] = acc[o];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_contract(ContractArgs a) {
  extern __shared__ char smem_raw[];
  cx<T>* slot = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* E = slot + kBlockEntries;
  cx<T>* part = E + a.e_budget;
  cx<T>* acc = part + a.item_budget * 16;

  const long long nb8 = (a.n_blocks + 7) / 8 * 8;
  const long long b = blockIdx.x;
  const long long logical = (b % 8) * (nb8 / 8) + b / 8;
  if (logical >= a.n_blocks) return;
  const int g = (int)(logical % a.n_groups);
  const long long qt = logical / a.n_groups;
  const int t = (int)(qt / a.V), q = (int)(qt % a.V);
  const int qx = q % a.Lx, qy = (q / a.Lx) % a.Ly, qz = q / (a.Lx * a.Ly);
  const int mq = (a.Lx - qx) % a.Lx + a.Lx * ((a.Ly - qy) % a.Ly + a.Ly * ((a.Lz - qz) % a.Lz));
  const int tid = threadIdx.x;

  const int gch0 = a.group_ch[g], nch = a.group_ch[g + 1] - gch0;
  for (int i = tid; i < nch * 16; i += kThreads) acc[i] = cx<T>{0, 0};

  const cx<T>* Nq = reinterpret_cast<const cx<T>*>(a.Nq);
  for (int c = a.group_chunk[g]; c < a.group_chunk[g + 1]; ++c) {
    const int esize = a.chunk_esize[c];
    for (int i = tid; i < esize; i += kThreads) E[i] = cx<T>{0, 0};
    __syncthreads();
    for (int s = a.chunk_step[c]; s < a.chunk_step[c + 1]; ++s) {
      if (a.step_load[s]) {
        const int site = a.step_side[s] ? mq : q;
        const cx<T>* src = Nq + ((long long)(t * a.n_types + a.step_type[s]) * a.V + site) * kBlockEntries;
        for (int i = tid; i < kBlockEntries; i += kThreads) slot[i] = src[i];
        __syncthreads();
      }
      for (int it = a.step_ebb[s] + tid; it < a.step_ebb[s + 1]; it += kThreads) {
        cx<T> v{0, 0};
        for (int k = a.ebb_term[it]; k < a.ebb_term[it + 1]; ++k) {
          const int tm = a.terms[k];
          const T cf = (T)(tm >> 16);
          const cx<T> x = slot[tm & 0xffff];
          v.re = fma(cf, x.re, v.re);
          v.im = fma(cf, x.im, v.im);
        }
        E[a.ebb_e[it]] += v;
      }
      __syncthreads();
    }
    const int m0 = a.chunk_meb[c], m1 = a.chunk_meb[c + 1];
    for (int it = m0 + tid; it < m1; it += kThreads) {
      cx<T>* out = part + (it - m0) * 16;
      const int r1 = a.meb_rows1[it];
      if (r1 == 4)
        meb_item<T, 4>(E, a.meb_e1[it], a.meb_e2[it], a.meb_K[it], a.meb_k0[it], a.meb_kn[it], out);
      else if (r1 == 2)
        meb_item<T, 2>(E, a.meb_e1[it], a.meb_e2[it], a.meb_K[it], a.meb_k0[it], a.meb_kn[it], out);
      else
        meb_item<T, 8>(E, a.meb_e1[it], a.meb_e2[it], a.meb_K[it], a.meb_k0[it], a.meb_kn[it], out);
    }
    __syncthreads();
    for (int it = a.chunk_acc[c] + tid; it < a.chunk_acc[c + 1]; it += kThreads) {
      cx<T> v{0, 0};
      for (int k = a.acc_src_range[it]; k < a.acc_src_range[it + 1]; ++k) {
        const T cf = (T)a.acc_coef[k];
        const cx<T> x = part[a.acc_src[k]];
        v.re = fma(cf, x.re, v.re);
        v.im = fma(cf, x.im, v.im);
      }
      acc[a.acc_target[it]] += v;
    }
    __syncthreads();
  }
  cx<T>* Ft = reinterpret_cast<cx<T>*>(a.Ft);
  for (int i = tid; i < nch * 16; i += kThreads) {
    const int ch = a.group_channels[gch0 + i / 16], s = i % 16;
    Ft[(((long long)ch * a.t_count + t) * 16 + s) * a.V + q] = acc[i];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_u32(unsigned* p, unsigned v, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_absmax(const void* S, unsigned* maxbits, long long per_slice, int t_count, hipStream_t st) {
  long long blocks = (per_slice + kThreads * 8 - 1) / (kThreads * 8);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_absmax, dim3((unsigned)blocks, t_count), dim3(kThreads), 0, st,
                     reinterpret_cast<const cf*>(S), maxbits, per_slice);
  return hipGetLastError();
}

hipError_t launch_scale_exps(const unsigned* maxbits, int* exps, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_exps, dim3((n + 63) / 64), dim3(64), 0, st, maxbits, exps, n);
  return hipGetLastError();
}

hipError_t launch_channel_scale(const int* exps, const int* chan_nf, double* oscale, int n_ch, int t_count,
                                hipStream_t st) {
  const int n = n_ch * t_count;
  hipLaunchKernelGGL(k_channel_scale, dim3((n + 63) / 64), dim3(64), 0, st, exps, chan_nf, oscale, n_ch, t_count);
  return hipGetLastError();
}

hipError_t launch_nbb(int prec, const NbbArgs& a, hipStream_t st) {
  dim3 grid(a.V, a.t_count);
  if (prec == 0)
    hipLaunchKernelGGL((k_nbb<double, double>), grid, dim3(kThreads), 0, st, a);
  else
    hipLaunchKernelGGL((k_nbb<float, float>), grid, dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fft_pass(int kind, const FftArgs& a, hipStream_t st) {
  const long long tiles = ((a.outer + a.OB - 1) / a.OB) * (a.inner / a.IB);
  const size_t lds = sizeof(cd) * (a.n + 2 * (size_t)a.OB * a.IB * (a.n + 1));
  dim3 grid((unsigned)tiles);
  static bool attr_set = false;
  if (!attr_set) {
    const int mx = 160 * 1024;
    (void)hipFuncSetAttribute((const void*)k_fft_pass<double, double>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)k_fft_pass<float, float>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    (void)hipFuncSetAttribute((const void*)k_fft_pass<float, double>, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    attr_set = true;
  }
  if (kind == 0)
    hipLaunchKernelGGL((k_fft_pass<double, double>), grid, dim3(kThreads), lds, st, a);
  else if (kind == 1)
    hipLaunchKernelGGL((k_fft_pass<float, float>), grid, dim3(kThreads), lds, st, a);
  else
    hipLaunchKernelGGL((k_fft_pass<float, double>), grid, dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

size_t contract_lds_bytes(int prec, int e_budget, int item_budget, int max_gch) {
  const size_t el = prec == 0 ? sizeof(cd) : sizeof(cf);
  return el * ((size_t)kBlockEntries + e_budget + (size_t)item_budget * 16 + (size_t)max_gch * 16);
}

hipError_t launch_contract(int prec, const ContractArgs& a, hipStream_t st) {
  const size_t lds = contract_lds_bytes(prec, a.e_budget, a.item_budget, a.max_gch);
  const long long nb8 = (a.n_blocks + 7) / 8 * 8;
  dim3 grid((unsigned)nb8);
  hipError_t e;
  if (prec == 0) {
    e = hipFuncSetAttribute((const void*)k_contract<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_contract<double>, grid, dim3(kThreads), lds, st, a);
  } else {
    e = hipFuncSetAttribute((const void*)k_contract<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_contract<float>, grid, dim3(kThreads), lds, st, a);
  }
  return hipGetLastError();
}

}  // namespace nbs
