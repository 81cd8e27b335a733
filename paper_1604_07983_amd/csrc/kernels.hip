// kernels.hip -- HIP kernels for gfx950 (MI355X) of the NBS four-point function.
//
//   k_nbb       normal baryon blocks, Eq. (5) / Sec. 4(i) Eq. (8)
//   k_fft_line  one axis of the in-house batched 3-D FFT (Eq. (6)), one line
//               per thread in registers
//   k_fft_line2 the same for 64, 80 and 96 points, two threads per line
//   k_fft_pass  the same through LDS tiles, for the lengths k_fft_line lacks
//   k_fft_plane the x and y axes of square planes of block fields together
//   k_fft_cube  all three axes of 8^3 and 16^3 block fields in one pass;
//               k_fft_cube_inv the inverse of contiguous 8^3 and 16^3 fields
//   k_contract  effective blocks and their products, Sec. 4(ii)-(iii),
//               Eqs. (9)-(10), driven by the compiled SoA program (lane
//               teams); k_contract_seg the same as segments on the matrix
//               cores
//   k_two_point zero-momentum single-baryon correlators from the blocks
//   k_absmax / k_scale_exps / k_channel_scale   per-slice power-of-two
//               scale of the precision form and its exact undo
#include <hip/hip_runtime.h>

#include <cfloat>
#include <limits>
#include <type_traits>

#include "cx.hpp"
#include "fft.hpp"
#include "fft_reg.hpp"
#include "kernels.hpp"

namespace nbs {

// Lane moves within rows of 16 lanes (DPP), for floats and doubles.
template <int CTRL> __device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

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
  // m = f 2^e, f in [0.5, 1): S 2^-e has max in [0.5, 1); an infinite
  // maximum (non-finite input, reported by the block kernel) keeps scale 1
  if (m > 0.f && m <= FLT_MAX) frexpf(m, &e);
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
// Normal baryon blocks, per sink operator.  One workgroup per (site, slice):
// the three propagators are staged in LDS, the diquarks
//   D_{f1 f2}[c][j1][j2] = sum eps_abc (C g5)_{be ga} S_f1[(be,a)][j1] S_f2[(ga,b)][j2]
// are formed once per flavour pair, then every operator block
//   N_op[al][j0][j1][j2] = sum_k w_k sum_c D_k[c][i0][i1] S_{f3,k}[(al,c)][i2],
//   (i0, i1, i2) = (j_pi(0), j_pi(1), j_pi(2)),
// (the Lambda and Sigma0 blocks as combinations of the X_u, X_d, X_s blocks,
// Sec. 4(i)) is written in the block layout of BlockLayout: operators with
// a same-flavour slot pair antisymmetrised in it and packed (1584 complex
// per site), the others whole (3456).
// ---------------------------------------------------------------------------
// Index p of the pair (a, b), a < b, of 12 x 12, and its inverse: the 66
// pairs by bands of equal difference d = b - a (d = 1 .. 11, a = 0 ..
// 11 - d), band d starting at band_start(d) = (d - 1)(24 - d) / 2.  Along a
// band both (a, b) and (b, a) move by one step of each index, so a staged
// block is unpacked with additions only.
__host__ __device__ inline int band_start(int d) { return (d - 1) * (24 - d) / 2; }
__host__ __device__ inline int pair_index(int a, int b) { return band_start(b - a) + a; }
__host__ __device__ inline void pair_decode(int p, int& a, int& b) {
  // the largest d with band_start(d) <= p, from the quadratic, then checked
  int d = (int)((25.0f - sqrtf((float)(529 - 8 * p))) * 0.5f);
  if (d < 1) d = 1;
  if (d > 11) d = 11;
  if (band_start(d) > p) --d;
  if (d < 11 && band_start(d + 1) <= p) ++d;
  a = p - band_start(d);
  b = a + d;
}

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
    // NaN fails every comparison; infinities exceed the largest finite value
    constexpr Tin kMax = std::numeric_limits<Tin>::max();
    if (!(fabs(v.re) <= kMax && fabs(v.im) <= kMax)) atomicOr(a.nonfinite, 1u);
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
        const int ga = be ^ 1;  // (C g5)_{be, be^1} = +1 for even be, -1 for odd
        const T g = (be & 1) ? -e : e;
        const cx<T> p = S1[(3 * be + ca) * 12 + j1] * S2[(3 * ga + cb) * 12 + j2];
        acc.re = fma(g, p.re, acc.re);
        acc.im = fma(g, p.im, acc.im);
      }
    }
    D[d][r] = acc;
  }
  __syncthreads();
  for (int op = 0; op < a.n_ops; ++op) {
    cx<T>* out = reinterpret_cast<cx<T>*>(a.Nq) + block_offset(a.lay, op, a.t_count, t, a.V, site);
    const int nt = a.op_nterm[op];
    const int pair = a.lay.pair[op];
    // N_op[al][j0][j1][j2]
    auto pick = [](int m, int j0, int j1, int j2) { return m == 0 ? j0 : (m == 1 ? j1 : j2); };
    auto entry = [&](int al, int j0, int j1, int j2) {
      cx<T> v{0, 0};
      for (int k = 0; k < nt; ++k) {
        const int pm = a.op_perm[op][k];
        const int i0 = pick(pm & 3, j0, j1, j2), i1 = pick((pm >> 2) & 3, j0, j1, j2),
                  i2 = pick((pm >> 4) & 3, j0, j1, j2);
        const cx<T>* Dd = D[a.op_dq[op][k]];
        const cx<T>* S3 = S[a.op_f3[op][k]];
        cx<T> u{0, 0};
#pragma unroll
        for (int c = 0; c < 3; ++c) cmac(u, Dd[c * 144 + i0 * 12 + i1], S3[(3 * al + c) * 12 + i2]);
        const T w = (T)a.op_w[op][k];
        v.re = fma(w, u.re, v.re);
        v.im = fma(w, u.im, v.im);
      }
      return v;
    };
    const int ne = a.lay.ne[op];
    for (int o = threadIdx.x; o < ne; o += kThreads) {
      int al, j0, j1, j2;
      if (pair < 0) {
        al = o / 1728;
        j0 = (o / 144) % 12;
        j1 = (o / 12) % 12;
        j2 = o % 12;
      } else {
        // packed: (al, j_s3, pair index of j_s1 < j_s2)
        const int s1 = pair & 3, s2 = (pair >> 2) & 3;
        al = o / 792;
        const int r = o - 792 * al, js3 = r / 66;
        int pa, pb;
        pair_decode(r - 66 * js3, pa, pb);
        int j[3];
        j[3 - s1 - s2] = js3;
        j[s1] = pa;
        j[s2] = pb;
        j0 = j[0];
        j1 = j[1];
        j2 = j[2];
      }
      cx<T> v = entry(al, j0, j1, j2);
      if (pair >= 0) {
        // antisymmetrised in the same-flavour slot pair: N - N(s1 <-> s2)
        const int s1 = pair & 3, s2 = (pair >> 2) & 3;
        const int a1 = pick(s1, j0, j1, j2), a2 = pick(s2, j0, j1, j2);
        if (a1 == a2) {
          v = cx<T>{0, 0};
        } else {
          // the third slot keeps its index; the pair's indices are exchanged
          const int k0 = s1 == 0 ? a2 : (s2 == 0 ? a1 : j0);
          const int k1 = s1 == 1 ? a2 : (s2 == 1 ? a1 : j1);
          const int k2 = s1 == 2 ? a2 : (s2 == 2 ? a1 : j2);
          v = v - entry(al, k0, k1, k2);
        }
      }
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
  const long long tile = a.unit0 + blockIdx.x;
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

// One axis of the batched transform with the whole line in registers: thread
// (o, i) transforms the N elements o N inner + i + k inner, k < N.  Adjacent
// threads take adjacent i, so every load and store of a wavefront is one
// contiguous run.  Arithmetic in FP64 whatever the storage type.  Lines up
// to 48 points; 64, 80 and 96 take two threads per line (k_fft_line2).
template <int N, int SIGN, typename Tin, typename Tout>
__global__ __launch_bounds__(kThreads) void k_fft_line(FftArgs a) {
  using AT = double;
  const long long gid = a.unit0 + (long long)blockIdx.x * kThreads + threadIdx.x;
  if (gid >= a.outer * a.inner) return;
  const long long o = gid / a.inner, i = gid - o * a.inner;
  const long long base = o * N * a.inner + i;
  const cx<Tin>* in = reinterpret_cast<const cx<Tin>*>(a.in);
  cx<AT> v[N];
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = conv<AT>(in[base + k * a.inner]);
  fft_reg<N, SIGN>(v);
  double f = a.gscale;
  if (a.oscale) f *= a.oscale[o / a.oscale_div];
  const AT fa = (AT)f;
  cx<Tout>* out = reinterpret_cast<cx<Tout>*>(a.out);
#pragma unroll
  for (int k = 0; k < N; ++k) out[base + k * a.inner] = conv<Tout>(cx<AT>{v[k].re * fa, v[k].im * fa});
}

// Lines of N = 2 M points (64, 80, 96) with FP64 arithmetic, two threads
// per line: thread r (r = 0, 1; adjacent lanes) loads the points 2 m + r,
// transforms them (length M, registers), and the pair combines the halves
// by decimation in time, X[k] = E[k] + w^k O[k], X[k + M] = E[k] - w^k O[k]
// with w = exp(SIGN 2 pi i / N), exchanging one half through a DPP lane
// swap; thread r writes X[r M .. r M + M).
template <int N, int SIGN, typename Tin, typename Tout>
__global__ __launch_bounds__(kThreads) void k_fft_line2(FftArgs a) {
  constexpr int M = N / 2;
  const long long gid = 2 * a.unit0 + (long long)blockIdx.x * kThreads + threadIdx.x;
  const long long line = gid >> 1;
  const int r = (int)(gid & 1);
  // both threads of a pair are in range together (the grid covers 2 x lines)
  if (line >= a.outer * a.inner) return;
  const long long o = line / a.inner, i = line - o * a.inner;
  const long long base = o * N * a.inner + i;
  const cx<Tin>* in = reinterpret_cast<const cx<Tin>*>(a.in);
  cd v[M];
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = conv<double>(in[base + (2 * m + r) * a.inner]);
  fft_reg<M, SIGN>(v);
  constexpr ct::Twiddles<N> tw = ct::make_twiddles<N>();
  double f = a.gscale;
  if (a.oscale) f *= a.oscale[o / a.oscale_div];
  cx<Tout>* out = reinterpret_cast<cx<Tout>*>(a.out);
#pragma unroll
  for (int k = 0; k < M; ++k) {
    // the partner's value of this k (lane ^ 1)
    const cd w{dpp_move<0xB1>(v[k].re), dpp_move<0xB1>(v[k].im)};
    const cd E = r ? w : v[k], O = r ? v[k] : w;
    const cd t = O * cd{tw.c[k], SIGN * tw.s[k]};
    const cd x = r ? E - t : E + t;
    out[base + (k + r * M) * a.inner] = conv<Tout>(cd{x.re * f, x.im * f});
  }
}

// The x and y axes of a forward transform in one pass.  Workgroup (plane,
// field tile) loads the N x N x IB tile (runs of IB fields, so adjacent
// threads read adjacent fields), transforms every x line, then every y line,
// each thread one line in registers (fft_reg), and stores the tile back:
// one HBM read and one write for two axes.  The tile is kept in LDS in the
// storage type (the precision form keeps complex64 between the axes, as it
// does between passes); arithmetic is FP64.
template <int N, int IB, typename T, int NT>
__global__ __launch_bounds__(NT) void k_fft_plane(FftPlaneArgs a) {
  extern __shared__ __align__(16) char smem_plane[];
  cx<T>* tile = reinterpret_cast<cx<T>*>(smem_plane);  // [y][x][f]
  const long long n_ftiles = a.inner / IB;
  // consecutive field tiles (halves of one 128-byte run when IB x element
  // is 64 bytes) on the same XCD at about the same time, so that they
  // share its L2
  const long long per = (a.n_units + 7) / 8;
  const long long local = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (local >= a.n_units) return;
  const long long wg = a.unit0 + local;
  const long long plane = wg / n_ftiles, f0 = (wg % n_ftiles) * IB;
  const cx<T>* in = reinterpret_cast<const cx<T>*>(a.in) + plane * N * N * a.inner + f0;
  cx<T>* out = reinterpret_cast<cx<T>*>(a.out) + plane * N * N * a.inner + f0;
  constexpr int kTile = N * N * IB;
  for (int e = threadIdx.x; e < kTile; e += NT) {
    const int f = e % IB, xy = e / IB;
    tile[e] = in[(long long)xy * a.inner + f];
  }
  __syncthreads();
  // lines along x: (y, f) -> elements (y N + x) IB + f
  for (int l = threadIdx.x; l < N * IB; l += NT) {
    const int f = l % IB, y = l / IB;
    cd v[N];
#pragma unroll
    for (int x = 0; x < N; ++x) v[x] = conv<double>(tile[(y * N + x) * IB + f]);
    fft_reg<N, -1>(v);
#pragma unroll
    for (int x = 0; x < N; ++x) tile[(y * N + x) * IB + f] = conv<T>(v[x]);
  }
  __syncthreads();
  // lines along y: (x, f)
  for (int l = threadIdx.x; l < N * IB; l += NT) {
    const int f = l % IB, x = l / IB;
    cd v[N];
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = conv<double>(tile[(y * N + x) * IB + f]);
    fft_reg<N, -1>(v);
#pragma unroll
    for (int y = 0; y < N; ++y) tile[(y * N + x) * IB + f] = conv<T>(v[y]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kTile; e += NT) {
    const int f = e % IB, xy = e / IB;
    out[(long long)xy * a.inner + f] = tile[e];
  }
}

// All three axes of a forward block transform on a cubic lattice in one
// pass.  Workgroup (cube, field tile) keeps the N^3 x IB tile in registers:
// LP lanes share the z column (x, y) of the tile's IB fields, lane l of
// them holding fields l, l + LP, ..., so that adjacent lanes load adjacent
// fields of a site.  The x and y axes go through LDS, ZB planes of z at a
// time: the threads write the planes, transform every x line, then every y
// line, of each (plane, field), each line by one thread in registers, and
// read their values back; the z axis is then transformed in registers and
// stored: one HBM read and one write for the three axes.  Rows in LDS are
// padded to N + 1 entries, so that the x lines, whose threads differ in y,
// fall in different banks, and the planes of the fields lie 8 entries off
// a multiple of the bank cycle, so that the lanes of one site do too.
// Values are rounded to the storage type after each axis, in the order x,
// y, z, and the arithmetic is FP64, as in the separate passes, so the
// results are the same bit for bit.  In place is allowed: a workgroup reads
// its whole tile before writing it.
template <int N, int IB, int LP, int ZB, typename T>
__global__ __launch_bounds__(N * N * LP) void k_fft_cube(FftPlaneArgs a) {
  constexpr int NT = N * N * LP, FT = IB / LP, SY = N + 1, SP = N * SY + 8, LINES = ZB * IB * N;
  static_assert(N % ZB == 0 && IB % LP == 0, "cube tile shape");
  extern __shared__ __align__(16) char smem_cube[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_cube);  // [plane][field][y][x], rows padded
  const long long n_ftiles = a.inner / IB;
  // consecutive field tiles of a cube, which share 128-byte runs, on the
  // same XCD at about the same time
  const long long per = (a.n_units + 7) / 8;
  const long long local = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (local >= a.n_units) return;
  const long long wg = a.unit0 + local;
  const long long cube = wg / n_ftiles, f0 = (wg % n_ftiles) * IB;
  constexpr long long V = (long long)N * N * N;
  const int lane = threadIdx.x % LP, col = threadIdx.x / LP, px = col % N, py = col / N;
  const cx<T>* in = reinterpret_cast<const cx<T>*>(a.in) + cube * V * a.inner + f0 + lane;
  cx<T>* out = reinterpret_cast<cx<T>*>(a.out) + cube * V * a.inner + f0 + lane;
  cx<T> R[FT][N];
  // every load issued before the first use
#pragma unroll
  for (int z = 0; z < N; ++z)
#pragma unroll
    for (int j = 0; j < FT; ++j) R[j][z] = in[((long long)(z * N + py) * N + px) * a.inner + j * LP];
#pragma unroll
  for (int b = 0; b < N / ZB; ++b) {
#pragma unroll
    for (int k = 0; k < ZB; ++k)
#pragma unroll
      for (int j = 0; j < FT; ++j) buf[(k * IB + lane + j * LP) * SP + py * SY + px] = R[j][b * ZB + k];
    __syncthreads();
    // x lines: (plane and field, y)
    for (int l = threadIdx.x; l < LINES; l += NT) {
      cx<T>* row = buf + (l / N) * SP + (l % N) * SY;
      cd v[N];
#pragma unroll
      for (int x = 0; x < N; ++x) v[x] = conv<double>(row[x]);
      fft_reg<N, -1>(v);
#pragma unroll
      for (int x = 0; x < N; ++x) row[x] = conv<T>(v[x]);
    }
    __syncthreads();
    // y lines: (plane and field, x)
    for (int l = threadIdx.x; l < LINES; l += NT) {
      cx<T>* cl = buf + (l / N) * SP + (l % N);
      cd v[N];
#pragma unroll
      for (int y = 0; y < N; ++y) v[y] = conv<double>(cl[y * SY]);
      fft_reg<N, -1>(v);
#pragma unroll
      for (int y = 0; y < N; ++y) cl[y * SY] = conv<T>(v[y]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ZB; ++k)
#pragma unroll
      for (int j = 0; j < FT; ++j) R[j][b * ZB + k] = buf[(k * IB + lane + j * LP) * SP + py * SY + px];
    if (b + 1 < N / ZB) __syncthreads();
  }
  // z lines in registers
#pragma unroll
  for (int j = 0; j < FT; ++j) {
    cd v[N];
#pragma unroll
    for (int z = 0; z < N; ++z) v[z] = conv<double>(R[j][z]);
    fft_reg<N, -1>(v);
#pragma unroll
    for (int z = 0; z < N; ++z) R[j][z] = conv<T>(v[z]);
  }
#pragma unroll
  for (int z = 0; z < N; ++z)
#pragma unroll
    for (int j = 0; j < FT; ++j) out[((long long)(z * N + py) * N + px) * a.inner + j * LP] = R[j][z];
}

// The inverse transform of the relative sum (Eq. (6)) on a cubic lattice
// in one pass: the fields are contiguous N^3 cubes (one per channel, slice
// and spin pair), so a workgroup loads one cube into LDS in runs of N
// entries, transforms every x line, then every y line, then every z line
// (each by one thread in registers, FP64), and stores it scaled by
// gscale oscale[cube / oscale_div] straight from the z lines.  Rows are
// padded to N + 1 entries (the x lines' threads differ in y).  In place is
// allowed: the cube is read whole before it is written.
template <int N, typename Tin>
__global__ __launch_bounds__(N * N) void k_fft_cube_inv(FftArgs a) {
  constexpr int NT = N * N, SY = N + 1, SZ = N * SY;
  constexpr long long V = (long long)N * N * N;
  extern __shared__ __align__(16) char smem_cinv[];
  cd* tile = reinterpret_cast<cd*>(smem_cinv);  // [z][y][x], x padded
  const long long cube = a.unit0 + blockIdx.x;
  if (cube >= a.outer) return;
  const cx<Tin>* in = reinterpret_cast<const cx<Tin>*>(a.in) + cube * V;
  cd* out = reinterpret_cast<cd*>(a.out) + cube * V;
  for (int e = threadIdx.x; e < N * N * N; e += NT) {
    const int x = e % N, yz = e / N;
    tile[(yz / N) * SZ + (yz % N) * SY + x] = conv<double>(in[e]);
  }
  __syncthreads();
  const int pp = threadIdx.x % N, qq = threadIdx.x / N;
  {
    // x lines (y, z) = (pp, qq)
    cd* row = tile + qq * SZ + pp * SY;
    cd v[N];
#pragma unroll
    for (int x = 0; x < N; ++x) v[x] = row[x];
    fft_reg<N, 1>(v);
#pragma unroll
    for (int x = 0; x < N; ++x) row[x] = v[x];
  }
  __syncthreads();
  {
    // y lines (x, z) = (pp, qq)
    cd* cl = tile + qq * SZ + pp;
    cd v[N];
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = cl[y * SY];
    fft_reg<N, 1>(v);
#pragma unroll
    for (int y = 0; y < N; ++y) cl[y * SY] = v[y];
  }
  __syncthreads();
  {
    // z lines (x, y) = (pp, qq), scaled and stored
    cd* cl = tile + qq * SY + pp;
    cd v[N];
#pragma unroll
    for (int z = 0; z < N; ++z) v[z] = cl[z * SZ];
    fft_reg<N, 1>(v);
    double f = a.gscale;
    if (a.oscale) f *= a.oscale[cube / a.oscale_div];
#pragma unroll
    for (int z = 0; z < N; ++z) out[(z * N + qq) * N + pp] = cd{v[z].re * f, v[z].im * f};
  }
}

// ---------------------------------------------------------------------------
// Effective blocks and their products (Sec. 4(ii)-(iii), Eqs. (9)-(10)).
//
// One workgroup per (sink-operator group, momentum q, slice) stages the two
// operator blocks N~_op1(q) and N~_op2(-q) in LDS, then every wavefront works
// through 64-lane tasks without further barriers: a team of 1, 4 or 16 lanes
// owns one block product, each lane takes a slice of the shared source
// indices xi~ = (x_A, x_B), generates the effective-block entries
//   E[al, labels][x_A][x_B] = sum_maps sign sum_{source tensor} coef N~[...]
// from index arithmetic, accumulates the 4 x 4 (or 8 x 2) product, and the
// team is reduced with cross-lane shuffles.  Finally each channel output
// sums its products with their diagram coefficients.
// The blockIdx -> work mapping keeps every group of one momentum on the same
// XCD so they share N~(q), N~(-q) in that XCD's L2.
// ---------------------------------------------------------------------------
struct BlkShape {
  int kA, loneA, kB, loneB, nA, nB, KB;
  bool l3, l4;
};

__device__ __forceinline__ BlkShape decode_shape(int mask) {
  BlkShape s;
  int lone[2], in[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int bits = (mask >> (3 * h)) & 7;
    in[h] = __popc(bits);
    lone[h] = -1;
    if (in[h] == 2) lone[h] = (~bits & 1) ? 0 : ((~bits & 2) ? 1 : 2);
    if (in[h] == 1) lone[h] = (bits & 1) ? 0 : ((bits & 2) ? 1 : 2);
  }
  s.kA = in[0]; s.loneA = lone[0]; s.kB = in[1]; s.loneB = lone[1];
  s.nA = in[0] == 3 ? 24 : (in[0] == 2 ? (lone[0] == 2 ? 8 : 2) : 1);
  s.nB = in[1] == 3 ? 24 : (in[1] == 2 ? (lone[1] == 2 ? 8 : 2) : 1);
  s.KB = lone[1] < 0 ? 1 : (lone[1] == 2 ? 3 : 12);
  s.l3 = (mask >> 2) & 1;
  s.l4 = (mask >> 5) & 1;
  return s;
}

__device__ __forceinline__ int eps3(int a, int b, int c) { return (a - b) * (b - c) * (c - a) / 2; }

// Term t of the source tensor eps_{c1 c2 c3} (C g5)_{s1 s2} delta_{s3 al} of
// one source baryon, restricted to the block: sets j0..j2 (3 spin + colour)
// of the baryon's quarks that lie in the block and returns the coefficient.
// in = quarks of the baryon in the block; lone = its lone quark (local index);
// x = the shared index of the lone quark (3 spin + colour, or colour alone
// for the third quark whose spin is the label al).
__device__ __forceinline__ int part_term(int in, int lone, int x, int al, int t, int& j0, int& j1, int& j2) {
  if (in == 3) {
    const int cp = t >> 2, sp = t & 3;
    const int c0 = cp < 3 ? cp : cp - 3;
    const int c1 = cp < 3 ? (c0 + 1) % 3 : (c0 + 2) % 3;
    const int c2 = cp < 3 ? (c0 + 2) % 3 : (c0 + 1) % 3;
    j0 = 3 * sp + c0;
    j1 = 3 * (sp ^ 1) + c1;
    j2 = 3 * al + c2;
    return (cp < 3 ? 1 : -1) * ((sp & 1) ? -1 : 1);
  }
  if (in == 2) {
    if (lone == 2) {
      const int c2 = x, cc = t >> 2, sp = t & 3;
      const int c0 = cc == 0 ? (c2 + 1) % 3 : (c2 + 2) % 3;
      const int c1 = cc == 0 ? (c2 + 2) % 3 : (c2 + 1) % 3;
      j0 = 3 * sp + c0;
      j1 = 3 * (sp ^ 1) + c1;
      return (cc == 0 ? 1 : -1) * ((sp & 1) ? -1 : 1);
    }
    const int sa = x / 3, ca = x % 3, sb = sa ^ 1;
    const int o1 = (ca + 1) % 3, o2 = (ca + 2) % 3;
    const int cb = t == 0 ? o1 : o2, c2 = t == 0 ? o2 : o1;
    const int g = lone == 0 ? ((sa & 1) ? -1 : 1) : ((sb & 1) ? -1 : 1);
    const int e = lone == 0 ? eps3(ca, cb, c2) : eps3(cb, ca, c2);
    if (lone == 0) j1 = 3 * sb + cb; else j0 = 3 * sb + cb;
    j2 = 3 * al + c2;
    return e * g;
  }
  if (in == 1) {
    if (lone == 2) j2 = 3 * al + x;
    else if (lone == 1) j1 = x;
    else j0 = x;
  }
  return 1;
}


__device__ __forceinline__ int lds_index(int i) {
  const int al = i / 1728, j0 = (i / 144) % 12, j1 = (i / 12) % 12, j2 = i % 12;
  return al * kLdsAl + j0 * kLdsJ0 + j1 * kLdsJ1 + j2;
}

// Entry i of an operator's stored block (BlockLayout) written into a staged
// block in LDS: unpacked entries at their place; a packed entry (pair
// (s1, s2), j_s1 < j_s2) at (j_s1, j_s2) and negated at (j_s2, j_s1).
template <typename T> __device__ __forceinline__ void put_entry(cx<T>* slot, int pair, int i, cx<T> v) {
  if (pair < 0) {
    slot[lds_index(i)] = v;
    return;
  }
  const int s1 = pair & 3, s2 = (pair >> 2) & 3;
  const int al = i / 792, r = i - 792 * al, js3 = r / 66;
  int a, b;
  pair_decode(r - 66 * js3, a, b);
  int j[3];
  j[3 - s1 - s2] = js3;
  j[s1] = a;
  j[s2] = b;
  slot[al * kLdsAl + j[0] * kLdsJ0 + j[1] * kLdsJ1 + j[2]] = v;
  j[s1] = b;
  j[s2] = a;
  slot[al * kLdsAl + j[0] * kLdsJ0 + j[1] * kLdsJ1 + j[2]] = cx<T>{-v.re, -v.im};
}

// The 288 entries with j_s1 = j_s2 of a staged packed block are zero.
template <typename T> __device__ __forceinline__ void zero_pair_diagonal(cx<T>* slot, int pair, int tid, int nt) {
  if (pair < 0) return;
  const int s1 = pair & 3, s2 = (pair >> 2) & 3;
  for (int k = tid; k < 288; k += nt) {
    const int al = k / 144, js3 = (k / 12) % 12, a = k % 12;
    int j[3];
    j[3 - s1 - s2] = js3;
    j[s1] = a;
    j[s2] = a;
    slot[al * kLdsAl + j[0] * kLdsJ0 + j[1] * kLdsJ1 + j[2]] = cx<T>{0, 0};
  }
}

__device__ __forceinline__ int pick6(int m, int j0, int j1, int j2, int j3, int j4, int j5) {
  return m == 0 ? j0 : m == 1 ? j1 : m == 2 ? j2 : m == 3 ? j3 : m == 4 ? j4 : j5;
}

// Stride of source quark q in N~[al][slot0][slot1][slot2] under map mp
// (slot i is contracted with quark m_i): 144, 12, 1, or 0 if q is not in the block.
__device__ __forceinline__ int quark_stride(int mp, int q) {
  return ((mp & 7) == q ? kLdsJ0 : 0) + (((mp >> 3) & 7) == q ? kLdsJ1 : 0) + (((mp >> 6) & 7) == q ? 1 : 0);
}

// rows r of a block -> (al, a3, a4): r = (al * n3 + a3) * n4 + a4
__device__ __forceinline__ void decode_row(const BlkShape& sh, int r, int& al, int& a3, int& a4) {
  const int n4 = sh.l4 ? 2 : 1, n3 = sh.l3 ? 2 : 1;
  a4 = sh.l4 ? r % 2 : 0;
  a3 = sh.l3 ? (r / n4) % 2 : 0;
  al = r / (n3 * n4);
}

// Row r = (al, a3, a4) enters the address of every term linearly:
//   al * 1728 + 3 a3 * stride(quark 2) + 3 a4 * stride(quark 5).
template <int R>
__device__ __forceinline__ void row_offsets(const BlkShape& sh, int mp, int ro[R]) {
  const int s2 = 3 * quark_stride(mp, 2), s5 = 3 * quark_stride(mp, 5);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int al, a3, a4;
    decode_row(sh, r, al, a3, a4);
    ro[r] = al * kLdsAl + a3 * s2 + a4 * s5;
  }
}

template <typename T, int R>
__device__ __forceinline__ void add_rows(const cx<T>* slot, int base, T c, const int ro[R], cx<T> e[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const cx<T> x = slot[base + ro[r]];
    e[r].re = fma(c, x.re, e[r].re);
    e[r].im = fma(c, x.im, e[r].im);
  }
}

// Entries E[r][x_A][x_B] of the R rows of one block at one shared index:
// each source-tensor term is generated once and read for all rows.
template <typename T, int R>
__device__ __forceinline__ void block_rows(const cx<T>* slot, const BlkShape& sh, int nmaps, int mp0, int mp1,
                                  const int ro0[R], const int ro1[R], int xA, int xB, cx<T> e[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) e[r] = cx<T>{0, 0};
  const int sg0 = ((mp0 >> 9) & 1) ? -1 : 1, sg1 = ((mp1 >> 9) & 1) ? -1 : 1;
  for (int ta = 0; ta < sh.nA; ++ta) {
    int j0 = 0, j1 = 0, j2 = 0;
    const int cA = part_term(sh.kA, sh.loneA, xA, 0, ta, j0, j1, j2);
    for (int tb = 0; tb < sh.nB; ++tb) {
      int j3 = 0, j4 = 0, j5 = 0;
      const int c = cA * part_term(sh.kB, sh.loneB, xB, 0, tb, j3, j4, j5);
      const int b0 = pick6(mp0 & 7, j0, j1, j2, j3, j4, j5) * kLdsJ0 +
                     pick6((mp0 >> 3) & 7, j0, j1, j2, j3, j4, j5) * kLdsJ1 +
                     pick6((mp0 >> 6) & 7, j0, j1, j2, j3, j4, j5);
      add_rows<T, R>(slot, b0, (T)(sg0 * c), ro0, e);
      if (nmaps > 1) {
        const int b1 = pick6(mp1 & 7, j0, j1, j2, j3, j4, j5) * kLdsJ0 +
                       pick6((mp1 >> 3) & 7, j0, j1, j2, j3, j4, j5) * kLdsJ1 +
                       pick6((mp1 >> 6) & 7, j0, j1, j2, j3, j4, j5);
        add_rows<T, R>(slot, b1, (T)(sg1 * c), ro1, e);
      }
    }
  }
}

// Generic lane work (used for products of two full projections, K = 1):
// k runs over [k0, k0 + nk) and every entry is generated from part_term.
template <typename T, int R1>
__device__ __forceinline__ void lane_work_generic(const cx<T>* slotA, const cx<T>* slotB, const int* d, int k0, int nk,
                                         cx<T> acc[16]) {
  constexpr int R2 = 16 / R1;
  const BlkShape s1 = decode_shape(d[0]), s2 = decode_shape(d[8]);
  const int nm1 = d[1], nm2 = d[9];
  const int p10 = d[2], p11 = d[3], p20 = d[10], p21 = d[11];
  int ro10[R1], ro11[R1], ro20[R2], ro21[R2];
  row_offsets<R1>(s1, p10, ro10);
  row_offsets<R1>(s1, p11, ro11);
  row_offsets<R2>(s2, p20, ro20);
  row_offsets<R2>(s2, p21, ro21);
  const int KB = d[17];
  for (int k = k0; k < k0 + nk; ++k) {
    const int xA = k / KB, xB = k - xA * KB;
    cx<T> e1[R1], e2[R2];
    block_rows<T, R1>(slotA, s1, nm1, p10, p11, ro10, ro11, xA, xB, e1);
    block_rows<T, R2>(slotB, s2, nm2, p20, p21, ro20, ro21, xA, xB, e2);
#pragma unroll
    for (int r1 = 0; r1 < R1; ++r1)
#pragma unroll
      for (int r2 = 0; r2 < R2; ++r2) cmac(acc[r1 * R2 + r2], e1[r1], e2[r2]);
  }
}

// Universal table of the source-tensor terms of a quark pair inside a block
// (the third quark of that source baryon, the lone one, sits in the other
// block with shared index x): entry = j_p | j_q << 4 | (coef < 0) << 8 with
// (p, q) the pair's quarks in order, label spin 0.  Lone quark 0 or 1:
// 12 values of x, 2 terms; lone quark 2: 3 values (its colour), 8 terms.
constexpr int kPairTable = 72;
__device__ __forceinline__ int pair_index(int lone, int x, int t) { return lone < 2 ? lone * 24 + x * 2 + t : 48 + x * 8 + t; }

__device__ __forceinline__ void build_pair_table(int* tp, int tid, int nthreads) {
  for (int i = tid; i < kPairTable; i += nthreads) {
    const int lone = i < 24 ? 0 : (i < 48 ? 1 : 2);
    const int x = lone < 2 ? (i - 24 * lone) / 2 : (i - 48) / 8;
    const int t = lone < 2 ? (i - 24 * lone) % 2 : (i - 48) % 8;
    int j0 = 0, j1 = 0, j2 = 0;
    const int c = part_term(2, lone, x, 0, t, j0, j1, j2);
    const int jp = lone == 0 ? j1 : j0, jq = lone == 2 ? j1 : j2;
    tp[i] = jp | (jq << 4) | ((c < 0) << 8);
  }
}

// Products of a pair+single block with its complementary single+pair block
// (K = 9, 36, 144).  Side Y is where block 1 holds a quark pair: the lane
// fixes y on that side, so block 1's pair terms are formed once per lane,
// and walks z over the other side, where block 1 only shifts by z * stride
// and block 2's pair terms come from the universal table.
template <typename T, int R1>
__device__ __forceinline__ void lane_work_split(const cx<T>* slotA, const cx<T>* slotB, const int* d, const int* tp,
                                       int y, int z0, int zstep, cx<T> acc[16]) {
  constexpr int R2 = 16 / R1;
  const BlkShape s1 = decode_shape(d[0]), s2 = decode_shape(d[8]);
  const bool pairA = s1.kA == 2;                    // block 1's pair is in source baryon A
  const int base1 = pairA ? 0 : 3, base2 = pairA ? 3 : 0;
  const int lone1 = pairA ? s1.loneA : s1.loneB;    // lone quark (local) of block 1's pair baryon
  const int lone2 = pairA ? s2.loneB : s2.loneA;    // lone quark (local) of block 2's pair baryon
  const int Kz = lone2 == 2 ? 3 : 12;
  const int nP1 = lone1 == 2 ? 8 : 2, nP2 = lone2 == 2 ? 8 : 2;
  const int p1 = base1 + (lone1 == 0 ? 1 : 0), q1 = base1 + (lone1 == 2 ? 1 : 2);
  const int p2 = base2 + (lone2 == 0 ? 1 : 0), q2 = base2 + (lone2 == 2 ? 1 : 2);
  const int ys = base1 + lone1, zs = base2 + lone2;  // the single quarks: in block 2 (y) and block 1 (z)
  const int nm1 = d[1], nm2 = d[9];
  const int mp1[2] = {d[2], d[3]}, mp2[2] = {d[10], d[11]};
  int ro1[2][R1], ro2[2][R2];
  row_offsets<R1>(s1, mp1[0], ro1[0]);
  row_offsets<R1>(s1, mp1[1], ro1[1]);
  row_offsets<R2>(s2, mp2[0], ro2[0]);
  row_offsets<R2>(s2, mp2[1], ro2[1]);
  // block 1: fixed pair terms for this lane, z-stride of its single quark
  int off1[2][8], zst1[2];
  T c1[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int e = t < nP1 ? tp[pair_index(lone1, y, t)] : 0;
    c1[t] = (e >> 8) & 1 ? (T)-1 : (T)1;
#pragma unroll
    for (int m = 0; m < 2; ++m)
      off1[m][t] = (e & 15) * quark_stride(mp1[m], p1) + ((e >> 4) & 15) * quark_stride(mp1[m], q1);
  }
  T sg1[2], sg2[2];
  int yo2[2], st2p[2], st2q[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    zst1[m] = quark_stride(mp1[m], zs);
    sg1[m] = ((mp1[m] >> 9) & 1) ? (T)-1 : (T)1;
    sg2[m] = ((mp2[m] >> 9) & 1) ? (T)-1 : (T)1;
    yo2[m] = y * quark_stride(mp2[m], ys);
    st2p[m] = quark_stride(mp2[m], p2);
    st2q[m] = quark_stride(mp2[m], q2);
  }
  for (int z = z0; z < Kz; z += zstep) {
    cx<T> e1[R1], e2[R2];
#pragma unroll
    for (int r = 0; r < R1; ++r) e1[r] = cx<T>{0, 0};
#pragma unroll
    for (int r = 0; r < R2; ++r) e2[r] = cx<T>{0, 0};
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (m >= nm1) break;
      const int zo = z * zst1[m];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (t >= nP1) break;
        add_rows<T, R1>(slotA, off1[m][t] + zo, sg1[m] * c1[t], ro1[m], e1);
      }
    }
    for (int t = 0; t < nP2; ++t) {
      const int e = tp[pair_index(lone2, z, t)];
      const T c = (e >> 8) & 1 ? (T)-1 : (T)1;
      const int jp = e & 15, jq = (e >> 4) & 15;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        if (m >= nm2) break;
        add_rows<T, R2>(slotB, yo2[m] + jp * st2p[m] + jq * st2q[m], sg2[m] * c, ro2[m], e2);
      }
    }
#pragma unroll
    for (int r1 = 0; r1 < R1; ++r1)
#pragma unroll
      for (int r2 = 0; r2 < R2; ++r2) cmac(acc[r1 * R2 + r2], e1[r1], e2[r2]);
  }
}

// Class-specialised form of lane_work_split: rows, pair-term counts and map
// counts are compile-time, so the loop over z is straight-line code, and the
// per-map offsets come precomputed from the product descriptor.
template <int R>
__device__ __forceinline__ int row_offset(int r, int wlo, int whi) {
  // rows r = (al n3 + a3) n4 + a4: label bits below the spin al
  if constexpr (R == 2) return r * kLdsAl;
  else if constexpr (R == 4) return (r & 1) * wlo + (r >> 1) * kLdsAl;
  else return (r & 1) * wlo + ((r >> 1) & 1) * whi + (r >> 2) * kLdsAl;
}

template <typename T, int R1, int NP1, int NP2>
__device__ __forceinline__ void lane_split_fixed(const cx<T>* slotA, const cx<T>* slotB, const int* d, const int* tp,
                                                 int y, int z0, int zstep, int nm1, int nm2, cx<T> acc[16]) {
  // nm1, nm2 (1 or 2 maps per block) are wavefront-uniform: the compiler
  // packs tasks by class, and the class includes the map counts
  constexpr int R2 = 16 / R1;
  constexpr int KZ = NP2 == 8 ? 3 : 12;
  const int lone1 = d[20], lone2 = d[21];
  int e1d[2][6], e2d[2][6];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      e1d[m][k] = m < nm1 ? d[24 + 6 * m + k] : 0;
      e2d[m][k] = m < nm2 ? d[36 + 6 * m + k] : 0;
    }
  int ro1[2][R1], ro2[2][R2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
#pragma unroll
    for (int r = 0; r < R1; ++r) ro1[m][r] = row_offset<R1>(r, e1d[m][3], e1d[m][4]);
#pragma unroll
    for (int r = 0; r < R2; ++r) ro2[m][r] = row_offset<R2>(r, e2d[m][3], e2d[m][4]);
  }
  // block 1: this lane's pair terms (fixed y), z moves its single quark
  int off1[2][NP1];
  T cc1[2][NP1];
#pragma unroll
  for (int t = 0; t < NP1; ++t) {
    const int e = tp[pair_index(lone1, y, t)];
    const int jp = e & 15, jq = (e >> 4) & 15;
    const int c = ((e >> 8) & 1) ? -1 : 1;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      off1[m][t] = jp * e1d[m][0] + jq * e1d[m][1];
      cc1[m][t] = (T)(e1d[m][5] * c);
    }
  }
  int yo2[2];
  T sg2[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    yo2[m] = y * e2d[m][0];
    sg2[m] = (T)e2d[m][5];
  }
  const int tz0 = pair_index(lone2, 0, 0), tzs = NP2;  // table row of z is tz0 + z * NP2
#pragma unroll 1
  for (int z = z0; z < KZ; z += zstep) {
    cx<T> e1[R1], e2[R2];
#pragma unroll
    for (int r = 0; r < R1; ++r) e1[r] = cx<T>{0, 0};
#pragma unroll
    for (int r = 0; r < R2; ++r) e2[r] = cx<T>{0, 0};
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (m < nm1) {
        const int zo = z * e1d[m][2];
#pragma unroll
        for (int t = 0; t < NP1; ++t) add_rows<T, R1>(slotA, off1[m][t] + zo, cc1[m][t], ro1[m], e1);
      }
    }
#pragma unroll
    for (int t = 0; t < NP2; ++t) {
      const int e = tp[tz0 + z * tzs + t];
      const T c = ((e >> 8) & 1) ? (T)-1 : (T)1;
      const int jp = e & 15, jq = (e >> 4) & 15;
#pragma unroll
      for (int m = 0; m < 2; ++m)
        if (m < nm2) add_rows<T, R2>(slotB, yo2[m] + jp * e2d[m][1] + jq * e2d[m][2], sg2[m] * c, ro2[m], e2);
    }
#pragma unroll
    for (int r1 = 0; r1 < R1; ++r1)
#pragma unroll
      for (int r2 = 0; r2 < R2; ++r2) cmac(acc[r1 * R2 + r2], e1[r1], e2[r2]);
  }
}

// The 4 x 4-row split shapes of the precision form on matrix cores.  A quad
// of lanes walks one stream of shared indices (fixed y, z = z0, z0 + zstep,
// ...); quad lane r builds row r of both effective blocks, E1[r](y, z) and
// E2[r](y, z), and v_mfma_f32_4x4x1f32 (16 independent 4 x 4 outer products,
// one per quad: lane 4b + i gives row i of A and column i of B of block b)
// accumulates E1 E2^T as re.re, re.im, im.re, im.im.  Every lane of the
// wavefront runs the loop (the matrix instruction is wavefront-wide); lanes
// of idle quads feed zeros.
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int NP1, int NP2>
__device__ __forceinline__ void lane_split_mfma(const cf* slotA, const cf* slotB, const int* d, const int* tp, int y,
                                                int z0, int zstep, int nm1, int nm2, int r, bool live, f32x4& crr,
                                                f32x4& cri, f32x4& cir, f32x4& cii) {
  constexpr int KZ = NP2 == 8 ? 3 : 12;
  const int lone1 = d[20], lone2 = d[21];
  int e1d[2][6], e2d[2][6];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      e1d[m][k] = m < nm1 ? d[24 + 6 * m + k] : 0;
      e2d[m][k] = m < nm2 ? d[36 + 6 * m + k] : 0;
    }
  int ro1[2], ro2[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    ro1[m] = row_offset<4>(r, e1d[m][3], e1d[m][4]);
    ro2[m] = row_offset<4>(r, e2d[m][3], e2d[m][4]);
  }
  int off1[2][NP1];
  float cc1[2][NP1];
#pragma unroll
  for (int t = 0; t < NP1; ++t) {
    const int e = tp[pair_index(lone1, y, t)];
    const int jp = e & 15, jq = (e >> 4) & 15;
    const int c = ((e >> 8) & 1) ? -1 : 1;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      off1[m][t] = jp * e1d[m][0] + jq * e1d[m][1] + ro1[m];
      cc1[m][t] = (float)(e1d[m][5] * c);
    }
  }
  int yo2[2];
  float sg2[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    yo2[m] = y * e2d[m][0] + ro2[m];
    sg2[m] = (float)e2d[m][5];
  }
  const int tz0 = pair_index(lone2, 0, 0);
  const int nsteps = (KZ + zstep - 1) / zstep;  // the same for every lane of the task
#pragma unroll 1
  for (int s = 0; s < nsteps; ++s) {
    const int zt = z0 + s * zstep;
    const bool ok = live && zt < KZ;
    const int z = ok ? zt : 0;
    cf e1{0.f, 0.f}, e2{0.f, 0.f};
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (m < nm1) {
        const int zo = z * e1d[m][2];
#pragma unroll
        for (int t = 0; t < NP1; ++t) {
          const cf x = slotA[off1[m][t] + zo];
          e1.re = fmaf(cc1[m][t], x.re, e1.re);
          e1.im = fmaf(cc1[m][t], x.im, e1.im);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NP2; ++t) {
      const int e = tp[tz0 + z * NP2 + t];
      const float c = ((e >> 8) & 1) ? -1.f : 1.f;
      const int jp = e & 15, jq = (e >> 4) & 15;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        if (m < nm2) {
          const cf x = slotB[yo2[m] + jp * e2d[m][1] + jq * e2d[m][2]];
          const float cs = sg2[m] * c;
          e2.re = fmaf(cs, x.re, e2.re);
          e2.im = fmaf(cs, x.im, e2.im);
        }
      }
    }
    if (!ok) e1 = e2 = cf{0.f, 0.f};
    crr = __builtin_amdgcn_mfma_f32_4x4x1f32(e1.re, e2.re, crr, 0, 0, 0);
    cri = __builtin_amdgcn_mfma_f32_4x4x1f32(e1.re, e2.im, cri, 0, 0, 0);
    cir = __builtin_amdgcn_mfma_f32_4x4x1f32(e1.im, e2.re, cir, 0, 0, 0);
    cii = __builtin_amdgcn_mfma_f32_4x4x1f32(e1.im, e2.im, cii, 0, 0, 0);
  }
}

// Product of two full projections (K = 1): E1[a1 a3'] and E2[a2 a4'] are
// sums of the 24 source-tensor terms of one baryon each.  A 16-lane team
// shares the terms (lane u takes terms u and u + 16), reduces E1 and E2
// across the team, and lane 0 forms the 4 x 4 outer product (the other lanes
// contribute zero to the team sum that follows).
template <typename T>
__device__ __forceinline__ void lane_full(const cx<T>* slotA, const cx<T>* slotB, const int* d, int u, int nm1, int nm2,
                                          cx<T> acc[16]) {
  // nm1, nm2 are wavefront-uniform (part of the product class)
  const BlkShape s1 = decode_shape(d[0]), s2 = decode_shape(d[8]);
  int mp1[2] = {d[2], d[3]}, mp2[2] = {d[10], d[11]};
  cx<T> e1[4], e2[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) e1[r] = e2[r] = cx<T>{0, 0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = u + 16 * h;
    if (t < 24) {
      // block 1
      {
        int j0 = 0, j1 = 0, j2 = 0, j3 = 0, j4 = 0, j5 = 0;
        const int c = s1.kA == 3 ? part_term(3, -1, 0, 0, t, j0, j1, j2) : part_term(3, -1, 0, 0, t, j3, j4, j5);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          if (m < nm1) {
            int ro[4];
            row_offsets<4>(s1, mp1[m], ro);
            const int b = pick6(mp1[m] & 7, j0, j1, j2, j3, j4, j5) * kLdsJ0 +
                          pick6((mp1[m] >> 3) & 7, j0, j1, j2, j3, j4, j5) * kLdsJ1 +
                          pick6((mp1[m] >> 6) & 7, j0, j1, j2, j3, j4, j5);
            add_rows<T, 4>(slotA, b, (T)((((mp1[m] >> 9) & 1) ? -1 : 1) * c), ro, e1);
          }
        }
      }
      // block 2
      {
        int j0 = 0, j1 = 0, j2 = 0, j3 = 0, j4 = 0, j5 = 0;
        const int c = s2.kA == 3 ? part_term(3, -1, 0, 0, t, j0, j1, j2) : part_term(3, -1, 0, 0, t, j3, j4, j5);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          if (m < nm2) {
            int ro[4];
            row_offsets<4>(s2, mp2[m], ro);
            const int b = pick6(mp2[m] & 7, j0, j1, j2, j3, j4, j5) * kLdsJ0 +
                          pick6((mp2[m] >> 3) & 7, j0, j1, j2, j3, j4, j5) * kLdsJ1 +
                          pick6((mp2[m] >> 6) & 7, j0, j1, j2, j3, j4, j5);
            add_rows<T, 4>(slotB, b, (T)((((mp2[m] >> 9) & 1) ? -1 : 1) * c), ro, e2);
          }
        }
      }
    }
  }
#pragma unroll
  for (int dd = 1; dd < 16; dd <<= 1) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      e1[r].re += __shfl_xor(e1[r].re, dd);
      e1[r].im += __shfl_xor(e1[r].im, dd);
      e2[r].re += __shfl_xor(e2[r].re, dd);
      e2[r].im += __shfl_xor(e2[r].im, dd);
    }
  }
  if (u == 0) {
#pragma unroll
    for (int r1 = 0; r1 < 4; ++r1)
#pragma unroll
      for (int r2 = 0; r2 < 4; ++r2) cmac(acc[r1 * 4 + r2], e1[r1], e2[r2]);
  }
}

// Dispatch on the (wavefront-uniform) product class.
template <typename T, int R1, int NP1, int NP2>
__device__ __forceinline__ void split_maps(int nmc, const cx<T>* sA, const cx<T>* sB, const int* d, const int* tp,
                                           int y, int z0, int zs, cx<T> acc[16]) {
  lane_split_fixed<T, R1, NP1, NP2>(sA, sB, d, tp, y, z0, zs, 1 + (nmc >> 1), 1 + (nmc & 1), acc);
}

template <typename T>
__device__ __forceinline__ void run_product(int cls, const cx<T>* sA, const cx<T>* sB, const int* d, const int* tp, int y,
                                   int z0, int zs, cx<T> acc[16]) {
  if (cls < 4) {
    lane_full<T>(sA, sB, d, y, 1 + (cls >> 1), 1 + (cls & 1), acc);
  } else if (cls < 8) {
    split_maps<T, 4, 2, 2>(cls - 4, sA, sB, d, tp, y, z0, zs, acc);
  } else if (cls < 12) {
    split_maps<T, 8, 2, 8>(cls - 8, sA, sB, d, tp, y, z0, zs, acc);
  } else if (cls < 16) {
    split_maps<T, 2, 8, 2>(cls - 12, sA, sB, d, tp, y, z0, zs, acc);
  } else if (cls < 20) {
    split_maps<T, 4, 8, 8>(cls - 16, sA, sB, d, tp, y, z0, zs, acc);
  } else {
    const int rows1 = d[18];
    if (rows1 == 4)
      lane_work_split<T, 4>(sA, sB, d, tp, y, z0, zs, acc);
    else if (rows1 == 2)
      lane_work_split<T, 2>(sA, sB, d, tp, y, z0, zs, acc);
    else
      lane_work_split<T, 8>(sA, sB, d, tp, y, z0, zs, acc);
  }
}

size_t contract_lds_bytes(int prec, int max_gprod, int max_gcontrib, int max_gch, int max_gtask) {
  const size_t el = prec == 0 ? sizeof(cd) : sizeof(cf);
  const size_t real = prec == 0 ? sizeof(double) : sizeof(float);
  return el * (2 * (size_t)kLdsBlock + (size_t)max_gprod * 16) + real * max_gcontrib +
         sizeof(int) * (kPairTable + max_gcontrib + max_gch + 1 + (size_t)max_gtask * 64 + 1);
}

// The geometry owning (slice, momentum) pair `logical` (geometries in
// order of their first pair).  The table is read with vector loads; every field
// is moved to scalar registers explicitly (it is wavefront-uniform), which
// keeps vector registers free for the product loops.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni64(long long v) {
  const unsigned lo = (unsigned)uni((int)(unsigned)(v & 0xffffffffLL));
  const unsigned hi = (unsigned)uni((int)(unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ ContractGeom find_geometry(const ContractGeom* geo, int n_geom, long long logical) {
  int gi = 0;
  for (int k = 1; k < n_geom; ++k)
    if (logical >= uni64(geo[k].block0)) gi = k;
  gi = uni(gi);
  ContractGeom G;
  G.Nq = (const void*)uni64((long long)geo[gi].Nq);
  G.Ft = (void*)uni64((long long)geo[gi].Ft);
  G.V = uni(geo[gi].V);
  G.Lx = uni(geo[gi].Lx);
  G.Ly = uni(geo[gi].Ly);
  G.Lz = uni(geo[gi].Lz);
  G.t_count = uni(geo[gi].t_count);
  G.pad = 0;
  G.block0 = uni64(geo[gi].block0);
  G.qorder = (const int*)uni64((long long)geo[gi].qorder);
  return G;
}

// ---- team sums: reduce-scatter across the lanes of a team ----------------
// Each step pairs every lane with a partner that differs in one lane bit
// (row_mirror flips bits 0-3, row_half_mirror bits 0-2, the quad mirror bits
// 0-1, the quad swap bit 0; all within a 16-lane row, as DPP moves), keeps
// the half of its values selected by that bit and adds the partner's copy of
// that half.  After the steps for bits 3..0 lane l of a row holds output
// l & 15 summed over the row (4- and 8-lane teams take the steps for bits
// 1..0 and 2..0 and keep 4 and 2 outputs per lane); rows of 32- and 64-lane
// teams are added with cross-row shuffles.  About 15 complex
// moves per lane instead of 16 per butterfly step, and a fixed order.
template <int CTRL, int NV, typename T>
__device__ __forceinline__ void rs_step(const cx<T>* in, cx<T>* out, bool upper) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const cx<T> lo = in[i], hi = in[NV + i];
    const cx<T> keep = upper ? hi : lo, send = upper ? lo : hi;
    out[i] = cx<T>{keep.re + dpp_move<CTRL>(send.re), keep.im + dpp_move<CTRL>(send.im)};
  }
}

constexpr int kDppRowMirror = 0x140, kDppRowHalfMirror = 0x141, kDppQuadMirror = 0x1B, kDppQuadSwap = 0xB1;
constexpr int kDppQuadSwap2 = 0x4E;  // quad_perm [2, 3, 0, 1]: partner lane ^ 2

template <typename T>
__device__ __forceinline__ void team_reduce_store(const cx<T> acc[16], int lg, int lane, int p, cx<T>* R) {
  const bool b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1, b1 = (lane >> 1) & 1, b0 = lane & 1;
  if (lg == 2) {
    cx<T> v8[8], v4[4];
    rs_step<kDppQuadMirror, 8, T>(acc, v8, b1);
    rs_step<kDppQuadSwap, 4, T>(v8, v4, b0);
    if (p != 0xfff) {
      const int o0 = 8 * b1 + 4 * b0;
#pragma unroll
      for (int k = 0; k < 4; ++k) R[p * 16 + o0 + k] = v4[k];
    }
    return;
  }
  if (lg == 3) {
    cx<T> v8[8], v4[4], v2[2];
    rs_step<kDppRowHalfMirror, 8, T>(acc, v8, b2);
    rs_step<kDppQuadMirror, 4, T>(v8, v4, b1);
    rs_step<kDppQuadSwap, 2, T>(v4, v2, b0);
    if (p != 0xfff) {
      const int o0 = 8 * b2 + 4 * b1 + 2 * b0;
      R[p * 16 + o0] = v2[0];
      R[p * 16 + o0 + 1] = v2[1];
    }
    return;
  }
  cx<T> v8[8], v4[4], v2[2], v1[1];
  rs_step<kDppRowMirror, 8, T>(acc, v8, b3);
  rs_step<kDppRowHalfMirror, 4, T>(v8, v4, b2);
  rs_step<kDppQuadMirror, 2, T>(v4, v2, b1);
  rs_step<kDppQuadSwap, 1, T>(v2, v1, b0);
  cx<T> v = v1[0];
  if (lg >= 5) {
    v.re += __shfl_xor(v.re, 16);
    v.im += __shfl_xor(v.im, 16);
  }
  if (lg >= 6) {
    v.re += __shfl_xor(v.re, 32);
    v.im += __shfl_xor(v.im, 32);
  }
  if (p != 0xfff && (lane & ((1 << lg) - 1)) < 16) R[p * 16 + (lane & 15)] = v;
}

// Team sums of the matrix-core classes: lane 4 q + j of a quad holds
// R[i][j] for i = 0..3 of its quad's shared indices.  The four quads of a
// 16-lane row are added by two DPP row shifts (Hillis-Steele: afterwards the
// row's last quad holds the row's sum), rows by cross-row shuffles; the last
// quad of the team's first row writes.
constexpr int kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;

__device__ __forceinline__ void quad_team_store(const cf v_in[4], int lg, int lane, int p, cf* R) {
  cf v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = v_in[i];
    v[i].re += dpp_move<kDppRowShr4>(v[i].re);
    v[i].im += dpp_move<kDppRowShr4>(v[i].im);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i].re += dpp_move<kDppRowShr8>(v[i].re);
    v[i].im += dpp_move<kDppRowShr8>(v[i].im);
  }
  if (lg >= 5) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i].re += __shfl_xor(v[i].re, 16);
      v[i].im += __shfl_xor(v[i].im, 16);
    }
  }
  if (lg >= 6) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i].re += __shfl_xor(v[i].re, 32);
      v[i].im += __shfl_xor(v[i].im, 32);
    }
  }
  const int tl = lane & ((1 << lg) - 1);
  if (p != 0xfff && tl >= 12 && tl < 16) {
    const int j = lane & 3;
#pragma unroll
    for (int i = 0; i < 4; ++i) R[p * 16 + i * 4 + j] = v[i];
  }
}

// The contraction's dynamic LDS: the two operator blocks, the group's
// products, its channel contributions (coefficients, words, offsets per
// channel), the pair table, the task lane words and the task counter.
template <typename T> struct ContractLds {
  cx<T>*slotA, *slotB, *R;
  T* ccoef;
  int *tp, *cword, *coff, *tword, *counter;
};

template <typename T, typename Args>
__device__ __forceinline__ ContractLds<T> contract_lds(char* base, const Args& a) {
  ContractLds<T> l;
  l.slotA = reinterpret_cast<cx<T>*>(base);
  l.slotB = l.slotA + kLdsBlock;
  l.R = l.slotB + kLdsBlock;
  l.ccoef = reinterpret_cast<T*>(l.R + a.max_gprod * 16);
  l.tp = reinterpret_cast<int*>(l.ccoef + a.max_gcontrib);
  l.cword = l.tp + kPairTable;
  l.coff = l.cword + a.max_gcontrib;
  l.tword = l.coff + a.max_gch + 1;
  l.counter = l.tword + a.max_gtask * 64;
  return l;
}

// NT threads per workgroup: 512 for FP64 (the two staged blocks take most of
// the LDS, one workgroup per CU), 256 for the precision form (two workgroups
// per CU, so one stages while the other computes).  The channel compiler
// balances each group's tasks over NT / 64 wavefronts.
constexpr int kIdleClass = 30;

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_contract(ContractArgs a) {
  constexpr int kContractThreads = NT;
  extern __shared__ __align__(16) char smem_raw[];

  // consecutive logical workgroups on one XCD (hardware deals workgroups
  // round-robin over the 8 XCDs)
  const long long nb8 = (a.n_chunk + 7) / 8 * 8;
  const long long b = blockIdx.x;
  const long long local = (b % 8) * (nb8 / 8) + b / 8;
  if (local >= a.n_chunk) return;
  const long long logical = a.block0 + local;
  // consecutive logical workgroups share (slice, momentum): chunk-minor
  const long long qtl = logical / a.n_gchunk;
  const int chunk = (int)(logical - qtl * a.n_gchunk);
  build_pair_table(contract_lds<T>(smem_raw, a).tp, threadIdx.x, kContractThreads);

  // the workgroup walks its chunk of sink-operator groups for its (q,
  // slice); the compiler orders the groups so that consecutive ones share an
  // operator where possible, and a block stays in LDS while its operator
  // does not change
  const ContractGeom G = find_geometry(a.geo, a.n_geom, qtl);
  const long long qt = qtl - G.block0;
  const int t = (int)(qt / G.V), q = (int)(qt % G.V);
  const int qx = q % G.Lx, qy = (q / G.Lx) % G.Ly, qz = q / (G.Lx * G.Ly);
  const int mq = (G.Lx - qx) % G.Lx + G.Lx * ((G.Ly - qy) % G.Ly + G.Ly * ((G.Lz - qz) % G.Lz));
  const int gbeg = a.gchunk[chunk], gend = a.gchunk[chunk + 1];
  for (int g = gbeg; g < gend; ++g) {
  // in double precision the arguments are read again from the argument
  // segment in every group (through a pointer the compiler cannot follow),
  // so that scalar registers need not hold them across the product loop
  using kargs = const __attribute__((address_space(4))) ContractArgs*;
  kargs ka = (kargs)__builtin_amdgcn_kernarg_segment_ptr();
  if constexpr (sizeof(T) == 8) asm volatile("" : "+s"(ka));
  const __attribute__((address_space(4))) ContractArgs& A = *ka;
  const ContractLds<T> lds = contract_lds<T>(smem_raw, A);
  cx<T>* const slotA = lds.slotA;
  cx<T>* const slotB = lds.slotB;
  cx<T>* const R = lds.R;
  T* const ccoef = lds.ccoef;
  const int* const tp = lds.tp;
  int* const cword = lds.cword;
  int* const coff = lds.coff;
  int* const tword = lds.tword;
  int& task_counter = *lds.counter;
  const bool newA = g == gbeg || A.group_op1[g] != A.group_op1[g - 1];
  // in double precision the thread index is made opaque per group so that
  // per-thread addresses are recomputed here instead of being held in
  // registers across the product loop (where they would spill)
  int tid = threadIdx.x;
  if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(tid));
  // stage the two operator blocks, the group's channel contributions and
  // the pair table
  const cx<T>* Nq = reinterpret_cast<const cx<T>*>(G.Nq);
  // first entry of operator op's block at site (A lives in the constant
  // address space, so the layout is read field by field)
  auto boff = [&](int op, int site) {
    return (long long)A.lay.cum[op] * G.t_count * G.V + ((long long)t * G.V + site) * A.lay.ne[op];
  };
  const cx<T>* srcA = Nq + boff(A.group_op1[g], q);
  const cx<T>* srcB = Nq + boff(A.group_op2[g], mq);
  const int neA = A.lay.ne[A.group_op1[g]], neB = A.lay.ne[A.group_op2[g]];
  const int prA = A.lay.pair[A.group_op1[g]], prB = A.lay.pair[A.group_op2[g]];
  constexpr int kPer = (kBlockEntries + kContractThreads - 1) / kContractThreads;
  const int gc0 = A.group_ch[g], nch = A.group_ch[g + 1] - gc0;
  const int cbase = A.ch_contrib[gc0], ncon = A.ch_contrib[gc0 + nch] - cbase;
  // staging paths with and without each block, so that none keeps
  // registers for a block it does not load
  auto stage = [&](auto with_a, auto with_b) {
    constexpr bool kA = decltype(with_a)::value, kB = decltype(with_b)::value;
    // every global load of the staging (both blocks, the group's channel
    // contributions) is issued before the first LDS store.  The block
    // pointers come from the geometry table: state that they address global
    // memory, so the loads are global loads that may all be in flight.
    using gptr = const __attribute__((address_space(1))) cx<T>*;
    const gptr gA = (gptr)srcA;
    const gptr gB = (gptr)srcB;
    cx<T> va[kA ? kPer : 1], vb[kB ? kPer : 1];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = tid + k * kContractThreads;
      if constexpr (kA) {
        const int ii = i < neA ? i : neA - 1;
        va[k] = cx<T>{gA[ii].re, gA[ii].im};
      }
      if constexpr (kB) {
        const int ii = i < neB ? i : neB - 1;
        vb[k] = cx<T>{gB[ii].re, gB[ii].im};
      }
    }
    const bool has_con = tid < ncon;
    const int cw = has_con ? A.contrib_prod[cbase + tid] : 0;
    const double cc = has_con ? A.contrib_coef[cbase + tid] : 0.0;
    const int co = tid <= nch ? A.ch_contrib[gc0 + tid] - cbase : 0;
    const int tw0 = A.group_task[g], ntw = (A.group_task[g + 1] - tw0) * 64;
    constexpr int kTwPer = 3;  // lane words per thread staged with the blocks
    int tw[kTwPer];
#pragma unroll
    for (int k = 0; k < kTwPer; ++k) {
      const int i = tid + k * kContractThreads;
      tw[k] = i < ntw ? A.task_lanes[(long long)tw0 * 64 + i] : 0;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = tid + k * kContractThreads;
      if constexpr (kA)
        if (i < neA) put_entry(slotA, prA, i, va[k]);
      if constexpr (kB)
        if (i < neB) put_entry(slotB, prB, i, vb[k]);
    }
    if constexpr (kA) zero_pair_diagonal(slotA, prA, tid, kContractThreads);
    if constexpr (kB) zero_pair_diagonal(slotB, prB, tid, kContractThreads);
    if (has_con) {
      cword[tid] = cw;
      ccoef[tid] = (T)cc;
    }
    if (tid <= nch) coff[tid] = co;
#pragma unroll
    for (int k = 0; k < kTwPer; ++k) {
      const int i = tid + k * kContractThreads;
      if (i < ntw) tword[i] = tw[k];
    }
    for (int i = tid + kTwPer * kContractThreads; i < ntw; i += kContractThreads)
      tword[i] = A.task_lanes[(long long)tw0 * 64 + i];
    for (int i = tid + kContractThreads; i < ncon; i += kContractThreads) {
      cword[i] = A.contrib_prod[cbase + i];
      ccoef[i] = (T)A.contrib_coef[cbase + i];
    }
  };
  // FP64 (one workgroup per CU): after the first group, half of the
  // wavefronts stage the next group's blocks while the other half forms the
  // channel sums (below), so the HBM latency of the staging overlaps that
  // work.  The precision form has a second workgroup on the CU to cover it.
  // stage_blocks: the blocks of group gg whose operator changed, by the NTH
  // threads from `first`, every global load before the first LDS store.
  constexpr bool kOverlap = sizeof(T) == 8;
  auto stage_blocks = [&](int gg, auto with_a, auto with_b, int first, auto nthreads) {
    constexpr bool kA = decltype(with_a)::value, kB = decltype(with_b)::value;
    constexpr int NTH = decltype(nthreads)::value;
    constexpr int kP = (kBlockEntries + NTH - 1) / NTH;
    using gptr = const __attribute__((address_space(1))) cx<T>*;
    const gptr gA = (gptr)(Nq + boff(A.group_op1[gg], q));
    const gptr gB = (gptr)(Nq + boff(A.group_op2[gg], mq));
    const int nA = A.lay.ne[A.group_op1[gg]], nB = A.lay.ne[A.group_op2[gg]];
    const int pA = A.lay.pair[A.group_op1[gg]], pB = A.lay.pair[A.group_op2[gg]];
    const int lt = tid - first;
    cx<T> va[kA ? kP : 1], vb[kB ? kP : 1];
#pragma unroll
    for (int k = 0; k < kP; ++k) {
      const int i = lt + k * NTH;
      if constexpr (kA) {
        const int ii = i < nA ? i : nA - 1;
        va[k] = cx<T>{gA[ii].re, gA[ii].im};
      }
      if constexpr (kB) {
        const int ii = i < nB ? i : nB - 1;
        vb[k] = cx<T>{gB[ii].re, gB[ii].im};
      }
    }
#pragma unroll
    for (int k = 0; k < kP; ++k) {
      const int i = lt + k * NTH;
      if constexpr (kA)
        if (i < nA) put_entry(slotA, pA, i, va[k]);
      if constexpr (kB)
        if (i < nB) put_entry(slotB, pB, i, vb[k]);
    }
    if constexpr (kA) zero_pair_diagonal(slotA, pA, lt, NTH);
    if constexpr (kB) zero_pair_diagonal(slotB, pB, lt, NTH);
  };
  auto stage_blocks_of = [&](int gg, int first, auto nthreads) {
    const bool nA = gg == gbeg || A.group_op1[gg] != A.group_op1[gg - 1];
    const bool nB = gg == gbeg || A.group_op2[gg] != A.group_op2[gg - 1];
    if (nA && nB)
      stage_blocks(gg, std::true_type{}, std::true_type{}, first, nthreads);
    else if (nA)
      stage_blocks(gg, std::true_type{}, std::false_type{}, first, nthreads);
    else if (nB)
      stage_blocks(gg, std::false_type{}, std::true_type{}, first, nthreads);
  };
  if constexpr (kOverlap) {
    if (g == gbeg) stage_blocks_of(g, 0, std::integral_constant<int, kContractThreads>{});
    stage(std::false_type{}, std::false_type{});  // contributions and task words
  } else {
    const bool newB = g == gbeg || A.group_op2[g] != A.group_op2[g - 1];
    if (newA && newB)
      stage(std::true_type{}, std::true_type{});
    else if (newA)
      stage(std::true_type{}, std::false_type{});
    else if (newB)
      stage(std::false_type{}, std::true_type{});
    else
      stage(std::false_type{}, std::false_type{});
  }
  if (tid == 0) task_counter = 0;
  __syncthreads();

  const int pbase = A.group_prod[g];
  const int lane = tid & 63;
  const int ntask = A.group_task[g + 1] - A.group_task[g];
  // every wavefront claims the next task (tasks come longest first); which
  // wavefront runs a task does not change its arithmetic
  for (;;) {
    int claim = 0;
    if (lane == 0) claim = atomicAdd(&task_counter, 1);
    const int tix = __builtin_amdgcn_readfirstlane(__shfl(claim, 0));
    if (tix >= ntask) break;
    const int w = tword[tix * 64 + lane];
    const int p = w & 0xfff, lg = (w >> 16) & 7;
    const int cls = __builtin_amdgcn_readfirstlane((w >> 26) & 31);
    if (cls == kIdleClass) continue;
    cx<T> acc[16];
#pragma unroll
    for (int o = 0; o < 16; ++o) acc[o] = cx<T>{0, 0};
    if constexpr (sizeof(T) == 4) {
      if (cls >= 20 && cls < 28) {
        // matrix-core classes (20 + 4 b' + map counts): the whole wavefront
        // runs the loop; idle lanes use product 0's descriptor and feed zeros
        const bool live = p != 0xfff;
        const int* d = A.prod_desc + (long long)(pbase + (live ? p : 0)) * kProdInts;
        const int y = live ? (w >> 12) & 15 : 0, z0 = (w >> 19) & 15, zs = 1 << ((w >> 23) & 7);
        const int nmc = (cls - 20) & 3, nm1 = 1 + (nmc >> 1), nm2 = 1 + (nmc & 1);
        f32x4 crr = {0.f, 0.f, 0.f, 0.f}, cri = crr, cir = crr, cii = crr;
        const cf* sA = reinterpret_cast<const cf*>(slotA);
        const cf* sB = reinterpret_cast<const cf*>(slotB);
        if (cls < 24)
          lane_split_mfma<2, 2>(sA, sB, d, tp, y, z0, zs, nm1, nm2, lane & 3, live, crr, cri, cir, cii);
        else
          lane_split_mfma<8, 8>(sA, sB, d, tp, y, z0, zs, nm1, nm2, lane & 3, live, crr, cri, cir, cii);
        cf v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = cf{crr[i] - cii[i], cri[i] + cir[i]};
        const int pt = __shfl(p, lane & ~((1 << lg) - 1));
        quad_team_store(v, lg, lane, pt, reinterpret_cast<cf*>(R));
        continue;
      }
    }
    if (cls < 4) {
      // full projections: the whole wavefront runs the team code (it
      // shuffles); idle lanes compute on product 0 and drop the result
      const int y = (w >> 12) & 15;
      const int* d = A.prod_desc + (long long)(pbase + (p != 0xfff ? p : 0)) * kProdInts;
      run_product<T>(cls, slotA, slotB, d, tp, y, 0, 1, acc);
      if (p == 0xfff) {
#pragma unroll
        for (int o = 0; o < 16; ++o) acc[o] = cx<T>{0, 0};
      }
    } else if (p != 0xfff) {
      const int y = (w >> 12) & 15, z0 = (w >> 19) & 15, zs = 1 << ((w >> 23) & 7);
      run_product<T>(cls, slotA, slotB, A.prod_desc + (long long)(pbase + p) * kProdInts, tp, y, z0, zs, acc);
    }
    if (cls < 4) {
      // lane_full left the whole product in the team's first lane
      if (p != 0xfff && ((w >> 12) & 15) == 0) {
#pragma unroll
        for (int o = 0; o < 16; ++o) R[p * 16 + o] = acc[o];
      }
    } else {
      // the team's product (its first lane is never idle)
      const int pt = __shfl(p, lane & ~((1 << lg) - 1));
      team_reduce_store<T>(acc, lg, lane, pt, R);
    }
  }
  __syncthreads();

  const bool split = kOverlap && g + 1 < gend;
  if (split && tid >= kContractThreads / 2) {
    stage_blocks_of(g + 1, kContractThreads / 2, std::integral_constant<int, kContractThreads / 2>{});
  } else {
  // channel sums: 8 lanes per output (spin s of local channel cl), each
  // summing every 8th contribution, then a fixed-order shuffle reduction.
  // The geometry is read again here rather than kept live through the
  // product loop above, where registers are scarce.
  const ContractGeom G2 = find_geometry(A.geo, A.n_geom, qtl);
  const long long qt2 = qtl - G2.block0;
  const int t2 = (int)(qt2 / G2.V), q2 = (int)(qt2 % G2.V);
  cx<T>* Ft = reinterpret_cast<cx<T>*>(G2.Ft);
  const int nacc = split ? kContractThreads / 2 : kContractThreads;
  for (int i0 = 0; i0 < nch * 16 * 8; i0 += nacc) {
    const int i = i0 + tid;
    const int o = i >> 3, sub = i & 7;
    const int cl = o >> 4, s = o & 15;
    cx<T> v{0, 0};
    if (cl < nch) {
      const int a1 = (s >> 3) & 1, a2 = (s >> 2) & 1, a3 = (s >> 1) & 1, a4 = s & 1;
      for (int c = coff[cl] + sub; c < coff[cl + 1]; c += 8) {
        const int w = cword[c];
        const int p = w & 0xffff, rows2 = 16 / ((w >> 16) & 15);
        const bool l3 = (w >> 20) & 1, l4 = (w >> 21) & 1;
        const int r1 = (a1 * (l3 ? 2 : 1) + (l3 ? a3 : 0)) * (l4 ? 2 : 1) + (l4 ? a4 : 0);
        const int r2 = (a2 * (l3 ? 1 : 2) + (l3 ? 0 : a3)) * (l4 ? 1 : 2) + (l4 ? 0 : a4);
        const T cf = ccoef[c];
        const cx<T> x = R[p * 16 + r1 * rows2 + r2];
        v.re = fma(cf, x.re, v.re);
        v.im = fma(cf, x.im, v.im);
      }
    }
#pragma unroll
    for (int dd = 1; dd < 8; dd <<= 1) {
      v.re += __shfl_xor(v.re, dd);
      v.im += __shfl_xor(v.im, dd);
    }
    if (cl < nch && sub == 0) {
      const int ch = A.group_channels[gc0 + cl];
      Ft[(((long long)ch * G2.t_count + t2) * 16 + s) * G2.V + q2] = v;
    }
  }
  }
  __syncthreads();  // LDS is restaged for the next group
  }
}

// ---------------------------------------------------------------------------
// Effective blocks and their products on the matrix cores (Sec. 4(ii)-(iii),
// Eqs. (9)-(10)).
//
// One workgroup per (slice, momentum q) walks the sink-operator groups as
// the lane-team kernel above does, staging the two operator blocks in LDS.
// The products of a group come as segments (compiler.hpp): a 16-lane team
// takes one segment, and at every step lane (h, x) forms row x of both
// effective blocks at shared-index slot k' = 4 s + h from the staged blocks
// (the source-tensor sums of Eq. (9): two terms per entry where the block
// holds a quark pair with a spin-colour lone partner, eight where the lone
// partner is a third quark, 24 for a whole baryon), and the team's matrix
// product accumulates E_A E_B^T: v_mfma_f64_4x4x4f64 (4 blocks of
// 4 x 4 x 4, lanes 16 k + 4 b + i) in FP64, v_mfma_f32_4x4x1f32 (16 blocks
// of 4 x 4 x 1, lanes 4 b + i) in the precision form, where the four quads
// of a team hold four slots k' and are summed at the end.  Complex products
// take three accumulators: re re, im im and the two cross terms.
// Segments of one product write separate result slots, summed before the
// channel sums, so the result does not depend on the order in which
// wavefronts finish.
// ---------------------------------------------------------------------------
template <typename T> struct SegAcc;
template <> struct SegAcc<double> {
  double rr, ii, ri;
};
template <> struct SegAcc<float> {
  f32x4 rr, ii, ri;
};

__device__ __forceinline__ void seg_zero(SegAcc<double>& c) { c.rr = c.ii = c.ri = 0.0; }
__device__ __forceinline__ void seg_zero(SegAcc<float>& c) {
  c.rr = f32x4{0.f, 0.f, 0.f, 0.f};
  c.ii = c.rr;
  c.ri = c.rr;
}
__device__ __forceinline__ void seg_mma(SegAcc<double>& c, cd a, cd b) {
  c.rr = __builtin_amdgcn_mfma_f64_4x4x4f64(a.re, b.re, c.rr, 0, 0, 0);
  c.ii = __builtin_amdgcn_mfma_f64_4x4x4f64(a.im, b.im, c.ii, 0, 0, 0);
  c.ri = __builtin_amdgcn_mfma_f64_4x4x4f64(a.re, b.im, c.ri, 0, 0, 0);
  c.ri = __builtin_amdgcn_mfma_f64_4x4x4f64(a.im, b.re, c.ri, 0, 0, 0);
}
__device__ __forceinline__ void seg_mma(SegAcc<float>& c, cf a, cf b) {
  c.rr = __builtin_amdgcn_mfma_f32_4x4x1f32(a.re, b.re, c.rr, 0, 0, 0);
  c.ii = __builtin_amdgcn_mfma_f32_4x4x1f32(a.im, b.im, c.ii, 0, 0, 0);
  c.ri = __builtin_amdgcn_mfma_f32_4x4x1f32(a.re, b.im, c.ri, 0, 0, 0);
  c.ri = __builtin_amdgcn_mfma_f32_4x4x1f32(a.im, b.re, c.ri, 0, 0, 0);
}

// Lane roles: team tm (0..3) of the wavefront, shared-index slot h (0..3),
// row x (0..3).  FP64: lane 16 h + 4 tm + x (the 4 x 4 x 4 block layout);
// FP32: lane 16 tm + 4 h + x (quad 4 tm + h of the 4 x 4 x 1 layout).
template <typename T> __device__ __forceinline__ void seg_roles(int lane, int& tm, int& h, int& x) {
  x = lane & 3;
  if constexpr (sizeof(T) == 8) {
    h = lane >> 4;
    tm = (lane >> 2) & 3;
  } else {
    tm = lane >> 4;
    h = (lane >> 2) & 3;
  }
}

// Sum over the four slots h of a team (the lanes that differ in h only).
template <typename T> __device__ __forceinline__ T seg_hsum(T v) {
  constexpr int s0 = sizeof(T) == 8 ? 16 : 4, s1 = sizeof(T) == 8 ? 32 : 8;
  v += __shfl_xor(v, s0);
  v += __shfl_xor(v, s1);
  return v;
}

// FP32 lanes 16 tm + 4 h + x: sum over h into the lanes with h = 3 (DPP row
// shifts by 4 and 8 lanes within the 16-lane row, Hillis-Steele).
__device__ __forceinline__ float seg_hsum_last(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x114, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x118, 0xF, 0xF, true));
  return v;
}

__device__ __forceinline__ int seg_row(int r, const int* w) {
  return (r & 1) * w[0] + ((r >> 1) & 1) * w[1] + ((r >> 2) & 1) * w[2];
}

// Pair of a source baryon whose lone quark (quark 0 or 1, shared index
// v = 3 s + c) sits in the other block: two terms, the pair's quark p at
// 3 (s ^ 1) + (c + 1 + t) % 3 and its third quark q (spin: a label) at colour
// (c + 2 - t) % 3, coefficient (t ? -1 : 1) (s odd ? -1 : 1).  The entry is
// S[o0] - S[o1]: the offsets come in the order that absorbs the sign.
__device__ __forceinline__ void seg_pair2(int v, int up, int uq, int& o0, int& o1) {
  const int sp = v / 3, c = v - 3 * sp;
  const int c1 = c == 2 ? 0 : c + 1, c2 = c == 0 ? 2 : c - 1;
  const int jp = 3 * (sp ^ 1);
  const int a = (jp + c1) * up + c2 * uq, b = (jp + c2) * up + c1 * uq;
  o0 = (sp & 1) ? b : a;
  o1 = (sp & 1) ? a : b;
}

// Pair of a source baryon whose lone quark is its third quark (shared index
// v = its colour c): terms (cc, sp) with quark p at 3 sp + (c + 1 + cc) % 3,
// quark q at 3 (sp ^ 1) + (c + 2 - cc) % 3, coefficient (cc ? -1 : 1)
// (sp odd ? -1 : 1).  Colour parts of the two colour orders.
__device__ __forceinline__ void seg_pair8(int c, int up, int uq, int& o0, int& o1) {
  const int c1 = c == 2 ? 0 : c + 1, c2 = c == 0 ? 2 : c - 1;
  o0 = c1 * up + c2 * uq;
  o1 = c2 * up + c1 * uq;
}

// Entry of a side with an eight-term pair: sum over the spin sp of the
// pair's first quark (spin offsets so[sp]) and the two colour orders.
template <typename T>
__device__ __forceinline__ cx<T> seg_entry8(const cx<T>* S, int base, const int so[4], int o0, int o1) {
  cx<T> e{0, 0};
#pragma unroll
  for (int sp = 0; sp < 4; ++sp) {
    const cx<T> u = S[base + so[sp] + o0], w = S[base + so[sp] + o1];
    if (sp & 1) {
      e.re += w.re - u.re;
      e.im += w.im - u.im;
    } else {
      e.re += u.re - w.re;
      e.im += u.im - w.im;
    }
  }
  return e;
}

template <typename T> __device__ __forceinline__ cx<T> cdiff(cx<T> u, cx<T> w) { return cx<T>{u.re - w.re, u.im - w.im}; }

// One segment of a team.  d: the team's descriptor; SA, SB: the staged
// blocks of sides A and B; R: result slots (16 complex each).
template <typename T>
__device__ __forceinline__ void seg_run(const int* d, const cx<T>* S1, const cx<T>* S2, cx<T>* R, int rstride, int shape,
                                        int nsteps, int lane) {
  int tm, h, x;
  seg_roles<T>(lane, tm, h, x);
  (void)tm;
  const bool live = d[0] != kSegIdle;
  const int s0 = d[1], hdr = d[3];
  const bool transposed = (hdr >> 17) & 1;
  const cx<T>* SA = transposed ? S2 : S1;
  const cx<T>* SB = transposed ? S1 : S2;
  int wa[3] = {d[7], d[8], d[9]}, wb[3] = {d[13], d[14], d[15]};
  const int uAs = d[4], uAp = d[5], uAq = d[6];
  const int uBs = d[10], uBp = d[11], uBq = d[12];
  SegAcc<T> acc, acc2;
  seg_zero(acc);
  seg_zero(acc2);
  const cx<T> zero{0, 0};
  if (shape == kSegC144) {
    // v1 = s / 3 (side A's pair, side B's single quark), v2 = 4 (s % 3) + h.
    // Teams without a segment compute from in-range offsets (their
    // descriptor is zero) and store nothing; the matrix blocks of the
    // other teams do not see their values.  Per value of v1 all twelve
    // block reads are issued before any is used.
    const int roA = seg_row(x, wa) + h * uAs, roB = seg_row(x, wb);
    const int stepA = 4 * uAs;
    int oB[3][2];
#pragma unroll
    for (int m = 0; m < 3; ++m) seg_pair2(4 * m + h, uBp, uBq, oB[m][0], oB[m][1]);
    for (int it = 0; it < nsteps / 3; ++it) {
      const int v1 = s0 / 3 + it;
      int oA0, oA1;
      seg_pair2(v1, uAp, uAq, oA0, oA1);
      const int bA0 = roA + oA0, bA1 = roA + oA1, bB = roB + v1 * uBs;
      cx<T> ua[3], wa_[3], ub[3], wb_[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        ua[m] = SA[bA0 + m * stepA];
        wa_[m] = SA[bA1 + m * stepA];
        ub[m] = SB[bB + oB[m][0]];
        wb_[m] = SB[bB + oB[m][1]];
      }
#pragma unroll
      for (int m = 0; m < 3; ++m) seg_mma(acc, cdiff(ua[m], wa_[m]), cdiff(ub[m], wb_[m]));
    }
  } else if (shape == kSegC36) {
    // side A has 8 rows: two accumulators, rows x (acc) and x + 4 (acc2);
    // side B has 2 rows, fed on lanes x < 2 (zero on the others).  Step s
    // covers k = 4 s + h = 12 v2 + v1: v2 = s / 3 (side A's single quark,
    // side B's pair), v1 = 4 (s % 3) + h (side A's pair, side B's single).
    const int roA0 = seg_row(x, wa), roA1 = seg_row(x + 4, wa);
    const int roB = seg_row(x & 1, wb) + h * uBs;
    const bool bl = x < 2;
    int so[4];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) so[sp] = 3 * sp * uBp + 3 * (sp ^ 1) * uBq;
    for (int it = 0; it < nsteps / 3; ++it) {
      const int v2 = s0 / 3 + it;
      int o0, o1;
      seg_pair8(v2, uBp, uBq, o0, o1);
      const int bA0 = roA0 + v2 * uAs, bA1 = roA1 + v2 * uAs;
#pragma unroll 1
      for (int m = 0; m < 3; ++m) {
        int p0, p1;
        seg_pair2(4 * m + h, uAp, uAq, p0, p1);
        const cx<T> a0 = cdiff(SA[bA0 + p0], SA[bA0 + p1]);
        const cx<T> a1 = cdiff(SA[bA1 + p0], SA[bA1 + p1]);
        cx<T> b = zero;
        if (bl) b = seg_entry8<T>(SB, roB + 4 * m * uBs, so, o0, o1);
        seg_mma(acc, a0, b);
        seg_mma(acc2, a1, b);
      }
    }
  } else if (shape == kSegC9) {
    // k' = 4 s + h = 3 v1 + v2 < 9
    const int roA = seg_row(x, wa), roB = seg_row(x, wb);
    int soA[4], soB[4];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
      soA[sp] = 3 * sp * uAp + 3 * (sp ^ 1) * uAq;
      soB[sp] = 3 * sp * uBp + 3 * (sp ^ 1) * uBq;
    }
    for (int it = 0; it < nsteps; ++it) {
      const int kk = 4 * (s0 + it) + h;
      const int v1 = kk / 3, v2 = kk - 3 * v1;
      cx<T> a = zero, b = zero;
      if (kk < 9) {
        int o0, o1;
        seg_pair8(v1, uAp, uAq, o0, o1);
        a = seg_entry8<T>(SA, roA + v2 * uAs, soA, o0, o1);
        seg_pair8(v2, uBp, uBq, o0, o1);
        b = seg_entry8<T>(SB, roB + v1 * uBs, soB, o0, o1);
      }
      seg_mma(acc, a, b);
    }
  } else {
    // two whole baryons: lane h takes the terms with the first quark's spin
    // h, (C g5)_{h, h ^ 1} = (h odd ? -1 : 1), and the six colour orders
    const int roA = seg_row(x, wa), roB = seg_row(x, wb);
    auto whole = [&](const cx<T>* S, int ro, int u2, int u0, int u1) {
      const int b = ro + 3 * h * u0 + 3 * (h ^ 1) * u1;
      cx<T> e{0, 0};
#pragma unroll
      for (int cp = 0; cp < 6; ++cp) {
        const int c0 = cp < 3 ? cp : cp - 3;
        const int c1 = cp < 3 ? (c0 + 1) % 3 : (c0 + 2) % 3;
        const int c2 = cp < 3 ? (c0 + 2) % 3 : (c0 + 1) % 3;
        const cx<T> v = S[b + c0 * u0 + c1 * u1 + c2 * u2];
        if (cp < 3) {
          e.re += v.re;
          e.im += v.im;
        } else {
          e.re -= v.re;
          e.im -= v.im;
        }
      }
      if (h & 1) e = cx<T>{-e.re, -e.im};
      return e;
    };
    cx<T> a = whole(SA, roA, uAs, uAp, uAq), b = whole(SB, roB, uBs, uBp, uBq);
    a.re = seg_hsum(a.re);
    a.im = seg_hsum(a.im);
    b.re = seg_hsum(b.re);
    b.im = seg_hsum(b.im);
    if (h != 0) a = b = zero;
    seg_mma(acc, a, b);
  }
  // results: D[i][j] = sum_k E_A[i][k] E_B[j][k] (for the 8 x 2 shape D
  // of acc2 holds side A's rows i + 4); canonical slot entry r1 * rows2 + r2
  // with (r1, r2) the rows of blocks 1 and 2
  const T sgn = ((hdr >> 16) & 1) ? (T)-1 : (T)1;
  const int slot = hdr & 0xffff;
  auto put = [&](int i, int j, int b, T re, T im) {
    int idx;
    if (shape == kSegC36) {
      const int ra = i + 4 * b;
      idx = transposed ? j * 8 + ra : ra * 2 + j;
    } else {
      idx = i * 4 + j;
    }
    R[slot * rstride + idx] = cx<T>{sgn * re, sgn * im};
  };
  if constexpr (sizeof(T) == 8) {
    if (live) {
      if (shape == kSegC36) {
        if (x < 2) {
          put(h, x, 0, acc.rr - acc.ii, acc.ri);
          put(h, x, 1, acc2.rr - acc2.ii, acc2.ri);
        }
      } else {
        put(h, x, 0, acc.rr - acc.ii, acc.ri);
      }
    }
  } else {
    // the four quads of the team hold partial sums over their slots h:
    // summed into the quad h = 3
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc.rr[i] = seg_hsum_last(acc.rr[i]);
      acc.ii[i] = seg_hsum_last(acc.ii[i]);
      acc.ri[i] = seg_hsum_last(acc.ri[i]);
    }
    if (shape == kSegC36) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc2.rr[i] = seg_hsum_last(acc2.rr[i]);
        acc2.ii[i] = seg_hsum_last(acc2.ii[i]);
        acc2.ri[i] = seg_hsum_last(acc2.ri[i]);
      }
    }
    if (live && h == 3) {
      if (shape == kSegC36) {
        if (x < 2) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            put(i, x, 0, acc.rr[i] - acc.ii[i], acc.ri[i]);
            put(i, x, 1, acc2.rr[i] - acc2.ii[i], acc2.ri[i]);
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) put(i, x, 0, acc.rr[i] - acc.ii[i], acc.ri[i]);
      }
    }
  }
}

// LDS of the segment contraction: the two blocks, the result slots, one set
// of task descriptors, two sets of channel tables (coefficients, product
// words, segment words, channel offsets: the group being summed and the
// next one), the task counter and the claimed work item.
size_t contract_seg_lds_bytes(int prec, int max_gslots, int max_gcontrib, int max_gch, int max_gstask, int rstride) {
  const size_t el = prec == 0 ? sizeof(cd) : sizeof(cf);
  const size_t real = prec == 0 ? sizeof(double) : sizeof(float);
  return el * (2 * (size_t)kLdsBlock + (size_t)max_gslots * rstride) + 2 * real * max_gcontrib +
         sizeof(int) * ((size_t)max_gstask * kSegTeams * kSegInts + 2 * (2 * (size_t)max_gcontrib + max_gch + 1) + 2);
}

// One operator block moved from HBM to LDS in chunks of four consecutive
// entries (one run of the last slot index), kChunks per thread: the loads
// can be issued early and the registers written to LDS later.
constexpr int kBlockChunks = kBlockEntries / 4;

__device__ __forceinline__ int chunk_lds_base(int c) {
  const int r = c / 3, j2 = 4 * (c - 3 * r);
  const int al = r / 144, rr = r - 144 * al;
  const int j0 = rr / 12, j1 = rr - 12 * j0;
  return al * kLdsAl + j0 * kLdsJ0 + j1 * kLdsJ1 + j2;
}

template <typename T, int NT> struct BlockRegs {
  static constexpr int kCh = (kBlockChunks + NT - 1) / NT;
  cx<T> v[kCh][4];
  int nch = 0, pair = -1;  // chunks of the stored block, its packed pair
  // ne entries (kBlockEntries, or kPackedEntries for a packed block with
  // pair pr) from HBM, four consecutive per chunk
  __device__ __forceinline__ void load(const cx<T>* src, int ne, int pr, int tid) {
    using gptr = const __attribute__((address_space(1))) cx<T>*;
    const gptr g = (gptr)src;
    // uniform over the workgroup: scalar registers
    nch = __builtin_amdgcn_readfirstlane(ne / 4);
    pair = __builtin_amdgcn_readfirstlane(pr);
#pragma unroll
    for (int k = 0; k < kCh; ++k) {
      const int c = tid + k * NT;
      const int cc = c < nch ? c : nch - 1;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[k][e] = cx<T>{g[4 * cc + e].re, g[4 * cc + e].im};
    }
  }
  // into a staged block in LDS (a packed block unpacked, its diagonal
  // zeroed unless the slot's previous block was packed in the same pair:
  // slot_pair tracks that, -2 at the start)
  __device__ __forceinline__ void store(cx<T>* slot, int tid, int& slot_pair) const {
    if (pair < 0) {
#pragma unroll
      for (int k = 0; k < kCh; ++k) {
        const int c = tid + k * NT;
        if (c < nch) {
          const int b = chunk_lds_base(c);
#pragma unroll
          for (int e = 0; e < 4; ++e) slot[b + e] = v[k][e];
        }
      }
      slot_pair = -1;
      return;
    }
    const int s1 = pair & 3, s2 = (pair >> 2) & 3, s3 = 3 - s1 - s2;
    const int u1 = s1 == 0 ? kLdsJ0 : s1 == 1 ? kLdsJ1 : 1, u2 = s2 == 0 ? kLdsJ0 : s2 == 1 ? kLdsJ1 : 1;
    const int u3 = s3 == 0 ? kLdsJ0 : s3 == 1 ? kLdsJ1 : 1;
#pragma unroll
    for (int k = 0; k < kCh; ++k) {
      const int c = tid + k * NT;
      if (c < nch) {
        // the chunk's first entry decoded once, then stepped along its band
        // of pairs (direct position (a, a + d), mirrored (a + d, a))
        const int i = 4 * c;
        const int al = i / 792, r0 = i - 792 * al;
        int j3 = r0 / 66, pa, pb;
        pair_decode(r0 - 66 * j3, pa, pb);
        int d = pb - pa, left = 11 - pb;  // pairs after this one in its band
        int base = al * kLdsAl + j3 * u3;
        const int uu = u1 + u2;
        int od = base + pa * u1 + pb * u2, om = base + pb * u1 + pa * u2;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const cx<T> x = v[k][e];
          slot[od] = x;
          slot[om] = cx<T>{-x.re, -x.im};
          if (left > 0) {
            od += uu;
            om += uu;
            --left;
          } else {
            if (d < 11) {
              ++d;
            } else {
              // the next j_s3, or after j_s3 = 11 the next al
              d = 1;
              if (++j3 == 12) {
                j3 = 0;
                base += kLdsAl - 11 * u3;
              } else {
                base += u3;
              }
            }
            od = base + d * u2;
            om = base + d * u1;
            left = 11 - d;
          }
        }
      }
    }
    if (slot_pair != pair) zero_pair_diagonal(slot, pair, tid, NT);
    slot_pair = pair;
  }
};

// One group's tables (task descriptors, channel contributions) read into
// registers while the previous group computes, written to LDS when it is
// done with them.  Descriptor ints beyond kTd per thread and contributions
// beyond one per thread are copied straight from global memory.  In the
// precision form (two workgroups per CU, no registers to spare) everything
// is copied at the store: the other workgroup hides that latency.
template <typename T, int NT> struct GroupTables {
  static constexpr bool kRegs = sizeof(T) == 8;
  static constexpr int kTd = kRegs ? (NT >= 1024 ? 2 : 3) : 1;
  int td[kTd];
  int cw = 0, ce = 0, co = 0;
  T cc = 0;
  long long tb = 0, cbase = 0;
  int ntd = 0, ncon = 0, nch = 0, gc0 = 0;
  __device__ __forceinline__ void load(const ContractArgs& a, int g, int tid) {
    gc0 = a.group_ch[g];
    nch = a.group_ch[g + 1] - gc0;
    cbase = a.ch_contrib[gc0];
    ncon = (int)(a.ch_contrib[gc0 + nch] - cbase);
    tb = (long long)a.group_stask[g] * (kSegTeams * kSegInts);
    ntd = (a.group_stask[g + 1] - a.group_stask[g]) * (kSegTeams * kSegInts);
    if constexpr (kRegs) {
#pragma unroll
      for (int k = 0; k < kTd; ++k) {
        const int i = tid + k * NT;
        td[k] = i < ntd ? a.seg_task[tb + i] : 0;
      }
      if (tid < ncon) {
        cw = a.contrib_prod[cbase + tid];
        ce = a.contrib_ext[cbase + tid];
        cc = (T)a.contrib_coef[cbase + tid];
      }
      if (tid <= nch) co = (int)(a.ch_contrib[gc0 + tid] - cbase);
    }
  }
  __device__ __forceinline__ void store(const ContractArgs& a, int* tdesc, int* cword, int* cext, T* ccoef, int* coff,
                                        int tid) const {
    const int nr = kRegs ? NT : 0;
    if constexpr (kRegs) {
#pragma unroll
      for (int k = 0; k < kTd; ++k) {
        const int i = tid + k * NT;
        if (i < ntd) tdesc[i] = td[k];
      }
      if (tid < ncon) {
        cword[tid] = cw;
        cext[tid] = ce;
        ccoef[tid] = cc;
      }
      if (tid <= nch) coff[tid] = co;
    }
    for (int i = (kRegs ? kTd * NT : 0) + tid; i < ntd; i += NT) tdesc[i] = a.seg_task[tb + i];
    for (int i = nr + tid; i < ncon; i += NT) {
      cword[i] = a.contrib_prod[cbase + i];
      cext[i] = a.contrib_ext[cbase + i];
      ccoef[i] = (T)a.contrib_coef[cbase + i];
    }
    for (int i = nr + tid; i <= nch; i += NT) coff[i] = (int)(a.ch_contrib[gc0 + i] - cbase);
  }
};

// One work item: (geometry, slice, momentum, range of groups) number
// `local` of the launch.  Ends with a barrier, so the LDS can be reused.
template <typename T, int NT> __device__ __forceinline__ void contract_seg_item(const ContractArgs& a, long long local) {
  extern __shared__ __align__(16) char smem_raw[];
  const long long logical = a.block0 + local;
  const long long qtl = logical / a.n_gchunk;
  const int chunk = (int)(logical - qtl * a.n_gchunk);
  const ContractGeom G = find_geometry(a.geo, a.n_geom, qtl);
  const long long qt = qtl - G.block0;
  const int t = (int)(qt / G.V), q = uni(G.qorder[qt % G.V]);
  const int qx = q % G.Lx, qy = (q / G.Lx) % G.Ly, qz = q / (G.Lx * G.Ly);
  const int mq = (G.Lx - qx) % G.Lx + G.Lx * ((G.Ly - qy) % G.Ly + G.Ly * ((G.Lz - qz) % G.Lz));
  cx<T>* const slotA = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* const slotB = slotA + kLdsBlock;
  cx<T>* const R = slotB + kLdsBlock;
  // channel tables in two sets [2][...]: the group being summed, the next
  const int rstride = a.rstride;
  T* const ccoef = reinterpret_cast<T*>(R + a.max_gslots * rstride);
  int* const tdesc = reinterpret_cast<int*>(ccoef + 2 * a.max_gcontrib);
  int* const cword = tdesc + a.max_gstask * (kSegTeams * kSegInts);
  int* const cext = cword + 2 * a.max_gcontrib;
  int* const coff = cext + 2 * a.max_gcontrib;
  int* const counter = coff + 2 * (a.max_gch + 1);
  const int tid = threadIdx.x, lane = tid & 63;
  const cx<T>* Nq = reinterpret_cast<const cx<T>*>(G.Nq);
  const int gbeg = a.gchunk[chunk], gend = a.gchunk[chunk + 1];
  auto block_src = [&](int op, int qq) { return Nq + block_offset(a.lay, op, G.t_count, t, G.V, qq); };
  // the packed pair of the block each slot holds (-1 whole, -2 none yet)
  int pairA = -2, pairB = -2;
  // the first group's blocks and tables
  {
    BlockRegs<T, NT> ra, rb;
    GroupTables<T, NT> tg;
    const int op1 = a.group_op1[gbeg], op2 = a.group_op2[gbeg];
    ra.load(block_src(op1, q), a.lay.ne[op1], a.lay.pair[op1], tid);
    rb.load(block_src(op2, mq), a.lay.ne[op2], a.lay.pair[op2], tid);
    tg.load(a, gbeg, tid);
    ra.store(slotA, tid, pairA);
    rb.store(slotB, tid, pairB);
    tg.store(a, tdesc, cword, cext, ccoef, coff, tid);
    if (tid == 0) *counter = 0;
  }
  __syncthreads();
  for (int g = gbeg; g < gend; ++g) {
    const int cur = (g - gbeg) & 1, nxt = cur ^ 1;
    // the next group's changed block (the walk changes one operator at a
    // time where it can) and its tables go into registers now and into LDS
    // once this group's products are done, so that their latency overlaps
    // the products
    const bool more = g + 1 < gend;
    const bool nA = more && a.group_op1[g + 1] != a.group_op1[g];
    const bool nB = more && a.group_op2[g + 1] != a.group_op2[g];
    BlockRegs<T, NT> pf;
    auto load_next = [&](BlockRegs<T, NT>& r, bool side_a) {
      const int op = side_a ? a.group_op1[g + 1] : a.group_op2[g + 1];
      r.load(block_src(op, side_a ? q : mq), a.lay.ne[op], a.lay.pair[op], tid);
    };
    if (nA)
      load_next(pf, true);
    else if (nB)
      load_next(pf, false);
    using Tables = GroupTables<T, NT>;
    Tables tn;
    if (Tables::kRegs && more) tn.load(a, g + 1, tid);

    // products: wavefronts claim tasks (longest first) from the counter
    const int ntask = a.group_stask[g + 1] - a.group_stask[g];
    for (;;) {
      int claim = 0;
      if (lane == 0) claim = atomicAdd(counter, 1);
      const int tix = __builtin_amdgcn_readfirstlane(claim);
      if (tix >= ntask) break;
      int tm, h, x;
      seg_roles<T>(lane, tm, h, x);
      (void)h;
      (void)x;
      const int* dt = tdesc + tix * (kSegTeams * kSegInts);
      const int shape = __builtin_amdgcn_readfirstlane(dt[0]);
      const int nsteps = __builtin_amdgcn_readfirstlane(dt[2]);
      int d[kSegInts];
#pragma unroll
      for (int k = 0; k < kSegInts; ++k) d[k] = dt[tm * kSegInts + k];
      seg_run<T>(d, slotA, slotB, R, rstride, shape, nsteps, lane);
    }
    __syncthreads();  // results complete; blocks, descriptors, counter free

    // channel sums: 8 lanes per output (spin s of local channel cl); each
    // contribution adds its product's result slot and extra segment slots
    {
      const int* cw_ = cword + cur * a.max_gcontrib;
      const int* ce_ = cext + cur * a.max_gcontrib;
      const T* cc_ = ccoef + cur * a.max_gcontrib;
      const int* co_ = coff + cur * (a.max_gch + 1);
      const int gc0 = a.group_ch[g], nch = a.group_ch[g + 1] - gc0;
      cx<T>* Ft = reinterpret_cast<cx<T>*>(G.Ft);
      for (int i0 = 0; i0 < nch * 16 * 8; i0 += NT) {
        const int i = i0 + tid;
        const int o = i >> 3, sub = i & 7;
        const int cl = o >> 4, s = o & 15;
        cx<T> v{0, 0};
        if (cl < nch) {
          const int a1 = (s >> 3) & 1, a2 = (s >> 2) & 1, a3 = (s >> 1) & 1, a4 = s & 1;
          for (int c = co_[cl] + sub; c < co_[cl + 1]; c += 8) {
            const int w = cw_[c];
            const int p = w & 0xffff, rows2 = 16 / ((w >> 16) & 15);
            const bool l3 = (w >> 20) & 1, l4 = (w >> 21) & 1;
            const int r1 = (a1 * (l3 ? 2 : 1) + (l3 ? a3 : 0)) * (l4 ? 2 : 1) + (l4 ? a4 : 0);
            const int r2 = (a2 * (l3 ? 1 : 2) + (l3 ? 0 : a3)) * (l4 ? 1 : 2) + (l4 ? 0 : a4);
            const int e = ce_[c], ne = e >> 16, e0 = e & 0xffff, ro = r1 * rows2 + r2;
            cx<T> xv = R[p * rstride + ro];
            for (int k = 0; k < ne; ++k) xv += R[(e0 + k) * rstride + ro];
            const T cf = cc_[c];
            v.re = fma(cf, xv.re, v.re);
            v.im = fma(cf, xv.im, v.im);
          }
        }
        // sum of the 8 lanes of the output: DPP moves within each 8-lane
        // half row (partners lane ^ 1, lane ^ 2, then the mirrored quad)
        v.re += dpp_move<kDppQuadSwap>(v.re);
        v.im += dpp_move<kDppQuadSwap>(v.im);
        v.re += dpp_move<kDppQuadSwap2>(v.re);
        v.im += dpp_move<kDppQuadSwap2>(v.im);
        v.re += dpp_move<kDppRowHalfMirror>(v.re);
        v.im += dpp_move<kDppRowHalfMirror>(v.im);
        if (cl < nch && sub == 0) {
          const int ch = a.group_channels[gc0 + cl];
          Ft[(((long long)ch * G.t_count + t) * 16 + s) * G.V + q] = v;
        }
      }
    }
    // the next group's block and tables (the channel sums read neither the
    // blocks, nor the descriptors, nor the other table set)
    if (nA) {
      pf.store(slotA, tid, pairA);
      if (nB) {
        BlockRegs<T, NT> rb;
        load_next(rb, false);
        rb.store(slotB, tid, pairB);
      }
    } else if (nB) {
      pf.store(slotB, tid, pairB);
    }
    if (more) {
      if (!Tables::kRegs) tn.load(a, g + 1, tid);
      tn.store(a, tdesc, cword + nxt * a.max_gcontrib, cext + nxt * a.max_gcontrib, ccoef + nxt * a.max_gcontrib,
               coff + nxt * (a.max_gch + 1), tid);
    }
    if (tid == 0) *counter = 0;
    __syncthreads();
  }
}

// Work items [0, n_chunk) in eight equal shares, item x * per + k of share
// x, where the share of XCD x holds every range of groups of one momentum
// (its pair q, -q in one L2).  One workgroup per item (workgroup b takes
// item k = b / 8 of share b % 8), or, in the persistent variant, as many
// workgroups as stay resident, each claiming items of its XCD's share from
// a counter in a.queue (zeroed before the launch) and then those of the
// other shares; every workgroup leaves once every counter has passed its
// share's end.  (Separate kernels: the claim loop costs registers.)
template <typename T, int NT, bool kPersist> __device__ __forceinline__ void contract_seg_body(const ContractArgs& a) {
  const long long per = (a.n_chunk + 7) / 8;
  const int xcd = blockIdx.x % 8;
  if constexpr (!kPersist) {
    const long long local = xcd * per + blockIdx.x / 8;
    if (local < a.n_chunk) contract_seg_item<T, NT>(a, local);
    return;
  }
  // the int after the task counter (the item's LDS layout)
  extern __shared__ __align__(16) char smem_raw[];
  cx<T>* const R = reinterpret_cast<cx<T>*>(smem_raw) + 2 * kLdsBlock;
  T* const ccoef = reinterpret_cast<T*>(R + a.max_gslots * a.rstride);
  int* const claim = reinterpret_cast<int*>(ccoef + 2 * a.max_gcontrib) + a.max_gstask * (kSegTeams * kSegInts) +
                     2 * (2 * a.max_gcontrib + a.max_gch + 1) + 1;
  for (int off = 0; off < 8; ++off) {
    const int share = (xcd + off) & 7;
    for (;;) {
      if (threadIdx.x == 0) *claim = (int)atomicAdd(&a.queue[share], 1u);
      __syncthreads();
      const long long k = *claim;
      __syncthreads();  // read by every thread before the next claim
      if (k >= per) break;
      const long long local = share * per + k;
      if (local < a.n_chunk) contract_seg_item<T, NT>(a, local);
    }
  }
}

template <typename T, int NT, bool kPersist = false>
__global__ __launch_bounds__(NT) void k_contract_seg(ContractArgs a) {
  contract_seg_body<T, NT, kPersist>(a);
}
// Precision form, 512 threads: four wavefronts per SIMD (registers for two
// workgroups per CU), so that one stages blocks while the other computes.
template <> __global__ __launch_bounds__(512, 4) void k_contract_seg<float, 512, false>(ContractArgs a) {
  contract_seg_body<float, 512, false>(a);
}
template <> __global__ __launch_bounds__(512, 4) void k_contract_seg<float, 512, true>(ContractArgs a) {
  contract_seg_body<float, 512, true>(a);
}

// ---------------------------------------------------------------------------
// Zero-momentum single-baryon two-point functions (Eq. (1) with one baryon
// on each side): workgroup (pair, slice), one wavefront.  Lane i takes the
// (term, source spin, source-tensor term) items i, i + 64, ...: the source
// tensor eps (C g5) delta of Eq. (4) for one baryon has 24 non-zero
// (colour, spin) assignments per source spin; each item reads both sink
// spins of the block entry the term's map selects.  FP64 accumulation,
// fixed-order shuffle reduction.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_two_point(TwoPointArgs a) {
  const int k = blockIdx.x, t = blockIdx.y, lane = threadIdx.x;
  const int slot = a.slot[k], pair = a.lay.pair[slot];
  const cx<T>* N = reinterpret_cast<const cx<T>*>(a.Nq) + block_offset(a.lay, slot, a.t_count, t, a.V, 0);  // q = 0
  double acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = 0.0;
  const int items = a.n_terms[k] * 48;
  for (int i = lane; i < items; i += 64) {
    const int term = i / 48, r = i - term * 48, ap = r / 24, s = r - ap * 24;
    int j[3] = {0, 0, 0};
    const int c = part_term(3, -1, 0, ap, s, j[0], j[1], j[2]);
    const int mp = a.term_map[k][term];
    const int jj[3] = {j[mp & 3], j[(mp >> 2) & 3], j[(mp >> 4) & 3]};
    // the stored entry: whole blocks at (j0, j1, j2); packed blocks at the
    // ordered pair, negated for j_s1 > j_s2, zero for j_s1 = j_s2
    int idx = (jj[0] * 12 + jj[1]) * 12 + jj[2], stride = 1728;
    double w = a.term_coef[k][term] * c;
    if (pair >= 0) {
      const int s1 = pair & 3, s2 = (pair >> 2) & 3, pa = jj[s1], pb = jj[s2];
      if (pa == pb) w = 0.0;
      if (pa > pb) w = -w;
      idx = pa == pb ? 0 : jj[3 - s1 - s2] * 66 + (pa < pb ? pair_index(pa, pb) : pair_index(pb, pa));
      stride = 792;
    }
#pragma unroll
    for (int al = 0; al < 2; ++al) {
      const cx<T> v = N[al * stride + idx];
      acc[4 * al + 2 * ap] = fma(w, (double)v.re, acc[4 * al + 2 * ap]);
      acc[4 * al + 2 * ap + 1] = fma(w, (double)v.im, acc[4 * al + 2 * ap + 1]);
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] += __shfl_xor(acc[i], d);
  if (lane == 0) {
    int e = 0;
    if (a.exps)
      for (int f = 0; f < 3; ++f) e += a.nf[k][f] * a.exps[f * a.t_count + t];
    const double sc = ldexp(a.slot_coef[k], e);
    cd* C = reinterpret_cast<cd*>(a.C) + ((long long)k * a.t_count + t) * 4;
#pragma unroll
    for (int o = 0; o < 4; ++o) C[o] = cd{acc[2 * o] * sc, acc[2 * o + 1] * sc};
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_two_point(int prec, const TwoPointArgs& a, hipStream_t st) {
  if (a.n_pairs < 1 || a.n_pairs > kMaxTwoPointPairs || a.t_count < 1) return hipErrorInvalidValue;
  const dim3 grid(a.n_pairs, a.t_count);
  if (prec == 0)
    hipLaunchKernelGGL(k_two_point<double>, grid, dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL(k_two_point<float>, grid, dim3(64), 0, st, a);
  return hipGetLastError();
}

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

namespace {

template <int N, int SIGN, typename Tin, typename Tout> hipError_t launch_line(const FftArgs& a, hipStream_t st) {
  const long long lines = a.outer * a.inner;
  for (long long l0 = 0; l0 < lines; l0 += kMaxLaunchItems) {
    FftArgs c = a;
    c.unit0 = l0;
    const long long n = lines - l0 < kMaxLaunchItems ? lines - l0 : kMaxLaunchItems;
    hipLaunchKernelGGL((k_fft_line<N, SIGN, Tin, Tout>), dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, st, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int N> hipError_t launch_line_kind(int kind, const FftArgs& a, hipStream_t st) {
  if (kind == 0) return a.sign < 0 ? launch_line<N, -1, double, double>(a, st) : launch_line<N, 1, double, double>(a, st);
  if (kind == 1) return launch_line<N, -1, float, float>(a, st);  // forward transform of the precision form
  return launch_line<N, 1, float, double>(a, st);                  // first inverse pass of the precision form
}

// Long lines, two threads per line.
template <int N, int SIGN, typename Tin, typename Tout> hipError_t launch_line2(const FftArgs& a, hipStream_t st) {
  const long long lines = a.outer * a.inner;
  const long long per = kMaxLaunchItems / 2;
  for (long long l0 = 0; l0 < lines; l0 += per) {
    FftArgs c = a;
    c.unit0 = l0;
    const long long n = lines - l0 < per ? lines - l0 : per;
    hipLaunchKernelGGL((k_fft_line2<N, SIGN, Tin, Tout>), dim3((unsigned)((2 * n + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, st, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int N> hipError_t launch_line2_kind(int kind, const FftArgs& a, hipStream_t st) {
  if (kind == 0) return a.sign < 0 ? launch_line2<N, -1, double, double>(a, st) : launch_line2<N, 1, double, double>(a, st);
  if (kind == 1) return launch_line2<N, -1, float, float>(a, st);
  return launch_line2<N, 1, float, double>(a, st);
}

}  // namespace

bool fft_line_supported(int n, int kind) {
  switch (n) {
    case 2: case 3: case 4: case 5: case 6: case 8: case 10: case 12: case 16: case 20: case 24: case 32:
    case 40: case 48:
      return true;
    case 64: case 80: case 96:
      return true;
  }
  return false;
}

namespace {
// fields per workgroup: runs of at least 128 bytes (16 fields at most) in a
// tile of at most 128 KB of LDS
template <typename T> constexpr int plane_ib(int n) {
  int ib = 1;
  while (ib < 16 && ib * (int)sizeof(cx<T>) < 128) ib *= 2;
  while (ib > 1 && (long long)n * n * ib * (long long)sizeof(cx<T>) > 128 * 1024) ib /= 2;
  return ib;
}

// threads of a plane workgroup: 512 where the tile leaves one workgroup per
// CU (complex64 planes of 32 and 40 points), else 256
template <typename T> constexpr int plane_threads(int n) { return sizeof(T) == 8 || n < 32 ? kThreads : 512; }

template <int N, typename T> hipError_t launch_plane_t(const FftPlaneArgs& a, hipStream_t st) {
  constexpr int IB = plane_ib<T>(N);
  constexpr int NT = plane_threads<T>(N);
  if (a.IB != IB) return hipErrorInvalidValue;
  const size_t lds = sizeof(cx<T>) * N * N * IB;
  const long long wgs = a.planes * (a.inner / IB);
  const long long chunk = kMaxLaunchItems / NT / 8 * 8;
  for (long long w0 = 0; w0 < wgs; w0 += chunk) {
    FftPlaneArgs c = a;
    c.unit0 = w0;
    c.n_units = wgs - w0 < chunk ? wgs - w0 : chunk;
    hipLaunchKernelGGL((k_fft_plane<N, IB, T, NT>), dim3((unsigned)((c.n_units + 7) / 8 * 8)), dim3(NT), lds, st, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace

namespace {
// Shape of the cube workgroups, measured at 16^3: runs of 32 bytes per site
// (16-byte runs, and 64-byte runs that leave one workgroup per CU, measured
// slower), LDS batches of 8 planes (all 16 measured slower); FP64 fields
// shared by lane pairs (one field per thread measured faster than two);
// complex64 fields four to a thread (lane teams of four, which need
// 1024-thread workgroups, measured slower).
template <typename T> constexpr int cube_ib() { return 32 / (int)sizeof(cx<T>); }
template <typename T> constexpr int cube_lp() { return sizeof(T) == 8 ? 2 : 1; }
template <typename T> constexpr int cube_zb(int n) { return n < 8 ? n : 8; }
template <int N, typename T> constexpr size_t cube_lds() {
  return sizeof(cx<T>) * (size_t)cube_zb<T>(N) * cube_ib<T>() * (N * (N + 1) + 8);
}

template <int N, typename T> hipError_t launch_cube_t(const FftPlaneArgs& a, hipStream_t st) {
  constexpr int IB = cube_ib<T>(), LP = cube_lp<T>(), ZB = cube_zb<T>(N);
  constexpr int NT = N * N * LP;
  constexpr size_t lds = cube_lds<N, T>();
  if (a.IB != IB || a.inner % IB != 0) return hipErrorInvalidValue;
  const long long wgs = a.planes * (a.inner / IB);
  const long long chunk = kMaxLaunchItems / NT / 8 * 8;
  for (long long w0 = 0; w0 < wgs; w0 += chunk) {
    FftPlaneArgs c = a;
    c.unit0 = w0;
    c.n_units = wgs - w0 < chunk ? wgs - w0 : chunk;
    hipLaunchKernelGGL((k_fft_cube<N, IB, LP, ZB, T>), dim3((unsigned)((c.n_units + 7) / 8 * 8)), dim3(NT), lds, st,
                       c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace

int fft_cube_fields(int n, long long inner, int kind) {
  if (kind != 0 && kind != 1) return 0;
  if (n != 8 && n != 16) return 0;
  const int ib = kind == 0 ? cube_ib<double>() : cube_ib<float>();
  return inner % ib == 0 ? ib : 0;
}

hipError_t launch_fft_cube(int kind, int n, const FftPlaneArgs& a, hipStream_t st) {
  if (kind == 0) {
    if (n == 8) return launch_cube_t<8, double>(a, st);
    if (n == 16) return launch_cube_t<16, double>(a, st);
  } else if (kind == 1) {
    if (n == 8) return launch_cube_t<8, float>(a, st);
    if (n == 16) return launch_cube_t<16, float>(a, st);
  }
  return hipErrorInvalidValue;
}

int fft_plane_fields(int n, long long inner, int kind) {
  if (kind != 0 && kind != 1) return 0;
  if (n != 8 && n != 16 && n != 24 && n != 32 && n != 40) return 0;
  const int ib = kind == 0 ? (n == 8 ? plane_ib<double>(8) : n == 16 ? plane_ib<double>(16) : n == 24 ? plane_ib<double>(24)
                                      : n == 32 ? plane_ib<double>(32) : plane_ib<double>(40))
                           : (n == 8 ? plane_ib<float>(8) : n == 16 ? plane_ib<float>(16) : n == 24 ? plane_ib<float>(24)
                                      : n == 32 ? plane_ib<float>(32) : plane_ib<float>(40));
  const int el = kind == 0 ? 16 : 8;
  return inner % ib == 0 && ib * el >= 64 ? ib : 0;
}

namespace {
template <int N> constexpr size_t cube_inv_lds() { return sizeof(cd) * (size_t)N * N * (N + 1); }

template <int N, typename Tin> hipError_t launch_cube_inv_t(const FftArgs& a, hipStream_t st) {
  constexpr int NT = N * N;
  constexpr size_t lds = cube_inv_lds<N>();
  const long long chunk = kMaxLaunchItems / NT;
  for (long long c0 = 0; c0 < a.outer; c0 += chunk) {
    FftArgs c = a;
    c.unit0 = c0;
    const long long n = a.outer - c0 < chunk ? a.outer - c0 : chunk;
    hipLaunchKernelGGL((k_fft_cube_inv<N, Tin>), dim3((unsigned)n), dim3(NT), lds, st, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace

bool fft_cube_inv_supported(int n, int kind) { return (n == 8 || n == 16) && (kind == 0 || kind == 2); }

hipError_t launch_fft_cube_inv(int kind, const FftArgs& a, hipStream_t st) {
  if (a.inner != 1 || a.sign < 0 || !fft_cube_inv_supported(a.n, kind)) return hipErrorInvalidValue;
  if (kind == 0) return a.n == 8 ? launch_cube_inv_t<8, double>(a, st) : launch_cube_inv_t<16, double>(a, st);
  return a.n == 8 ? launch_cube_inv_t<8, float>(a, st) : launch_cube_inv_t<16, float>(a, st);
}

hipError_t launch_fft_plane(int kind, int n, const FftPlaneArgs& a, hipStream_t st) {
  if (kind == 0) {
    switch (n) {
      case 8: return launch_plane_t<8, double>(a, st);
      case 16: return launch_plane_t<16, double>(a, st);
      case 24: return launch_plane_t<24, double>(a, st);
      case 32: return launch_plane_t<32, double>(a, st);
      case 40: return launch_plane_t<40, double>(a, st);
    }
  } else if (kind == 1) {
    switch (n) {
      case 8: return launch_plane_t<8, float>(a, st);
      case 16: return launch_plane_t<16, float>(a, st);
      case 24: return launch_plane_t<24, float>(a, st);
      case 32: return launch_plane_t<32, float>(a, st);
      case 40: return launch_plane_t<40, float>(a, st);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fft_line(int kind, const FftArgs& a, hipStream_t st) {
  if ((kind == 1 && a.sign > 0) || (kind == 2 && a.sign < 0)) return hipErrorInvalidValue;
  switch (a.n) {
    case 2: return launch_line_kind<2>(kind, a, st);
    case 3: return launch_line_kind<3>(kind, a, st);
    case 4: return launch_line_kind<4>(kind, a, st);
    case 5: return launch_line_kind<5>(kind, a, st);
    case 6: return launch_line_kind<6>(kind, a, st);
    case 8: return launch_line_kind<8>(kind, a, st);
    case 10: return launch_line_kind<10>(kind, a, st);
    case 12: return launch_line_kind<12>(kind, a, st);
    case 16: return launch_line_kind<16>(kind, a, st);
    case 20: return launch_line_kind<20>(kind, a, st);
    case 24: return launch_line_kind<24>(kind, a, st);
    case 32: return launch_line_kind<32>(kind, a, st);
    case 40: return launch_line_kind<40>(kind, a, st);
    case 48: return launch_line_kind<48>(kind, a, st);
    // long lines: two threads per line
    case 64: return launch_line2_kind<64>(kind, a, st);
    case 80: return launch_line2_kind<80>(kind, a, st);
    case 96: return launch_line2_kind<96>(kind, a, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fft_pass(int kind, const FftArgs& a, hipStream_t st) {
  const long long tiles = ((a.outer + a.OB - 1) / a.OB) * (a.inner / a.IB);
  const size_t lds = sizeof(cd) * (a.n + 2 * (size_t)a.OB * a.IB * (a.n + 1));
  const long long chunk = kMaxLaunchItems / kThreads;
  for (long long t0 = 0; t0 < tiles; t0 += chunk) {
    FftArgs c = a;
    c.unit0 = t0;
    dim3 grid((unsigned)(tiles - t0 < chunk ? tiles - t0 : chunk));
    if (kind == 0)
      hipLaunchKernelGGL((k_fft_pass<double, double>), grid, dim3(kThreads), lds, st, c);
    else if (kind == 1)
      hipLaunchKernelGGL((k_fft_pass<float, float>), grid, dim3(kThreads), lds, st, c);
    else
      hipLaunchKernelGGL((k_fft_pass<float, double>), grid, dim3(kThreads), lds, st, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int contract_waves(int prec) { return prec == 0 ? 8 : 4; }

hipError_t prepare_kernels(int prec, int waves, size_t contract_lds, int engine) {
  const int mx = 160 * 1024;
  hipError_t e = hipSuccess;
  auto set = [&](const void* f, int bytes) {
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  };
  set((const void*)k_fft_pass<double, double>, mx);
  set((const void*)k_fft_pass<float, float>, mx);
  set((const void*)k_fft_pass<float, double>, mx);
  set((const void*)k_fft_plane<8, plane_ib<double>(8), double, plane_threads<double>(8)>, 128 * 1024);
  set((const void*)k_fft_plane<16, plane_ib<double>(16), double, plane_threads<double>(16)>, 128 * 1024);
  set((const void*)k_fft_plane<24, plane_ib<double>(24), double, plane_threads<double>(24)>, 128 * 1024);
  set((const void*)k_fft_plane<32, plane_ib<double>(32), double, plane_threads<double>(32)>, 128 * 1024);
  set((const void*)k_fft_plane<40, plane_ib<double>(40), double, plane_threads<double>(40)>, 128 * 1024);
  set((const void*)k_fft_plane<8, plane_ib<float>(8), float, plane_threads<float>(8)>, 128 * 1024);
  set((const void*)k_fft_plane<16, plane_ib<float>(16), float, plane_threads<float>(16)>, 128 * 1024);
  set((const void*)k_fft_plane<24, plane_ib<float>(24), float, plane_threads<float>(24)>, 128 * 1024);
  set((const void*)k_fft_plane<32, plane_ib<float>(32), float, plane_threads<float>(32)>, 128 * 1024);
  set((const void*)k_fft_plane<40, plane_ib<float>(40), float, plane_threads<float>(40)>, 128 * 1024);
  set((const void*)k_fft_cube_inv<16, double>, (int)cube_inv_lds<16>());
  set((const void*)k_fft_cube_inv<16, float>, (int)cube_inv_lds<16>());
  set((const void*)k_fft_cube<8, cube_ib<double>(), cube_lp<double>(), cube_zb<double>(8), double>,
      (int)cube_lds<8, double>());
  set((const void*)k_fft_cube<16, cube_ib<double>(), cube_lp<double>(), cube_zb<double>(16), double>,
      (int)cube_lds<16, double>());
  set((const void*)k_fft_cube<8, cube_ib<float>(), cube_lp<float>(), cube_zb<float>(8), float>,
      (int)cube_lds<8, float>());
  set((const void*)k_fft_cube<16, cube_ib<float>(), cube_lp<float>(), cube_zb<float>(16), float>,
      (int)cube_lds<16, float>());
  if (engine == 1) {
    if (prec == 0) {
      set(waves == 16 ? (const void*)k_contract_seg<double, 1024> : (const void*)k_contract_seg<double, 512>,
          (int)contract_lds);
      set(waves == 16 ? (const void*)k_contract_seg<double, 1024, true> : (const void*)k_contract_seg<double, 512, true>,
          (int)contract_lds);
    } else {
      set(waves == 16 ? (const void*)k_contract_seg<float, 1024> : (const void*)k_contract_seg<float, 512>,
          (int)contract_lds);
      set(waves == 16 ? (const void*)k_contract_seg<float, 1024, true> : (const void*)k_contract_seg<float, 512, true>,
          (int)contract_lds);
    }
  } else if (prec == 0) {
    set((const void*)k_contract<double, 512>, (int)contract_lds);
  } else if (waves == 8) {
    set((const void*)k_contract<float, 512>, (int)contract_lds);
  } else {
    set((const void*)k_contract<float, 256>, (int)contract_lds);
  }
  return e;
}

namespace {
template <typename T, int NT, bool SEG> hipError_t launch_contract_t(const ContractArgs& a, size_t lds, hipStream_t st) {
  hipError_t e = hipSuccess;
  if constexpr (SEG) {
    if (a.persistent) {
      // every work item in one launch of as many workgroups as stay resident
      int dev = 0, cus = 0, per_cu = 0;
      if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
      if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
      if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_contract_seg<T, NT, true>, NT,
                                                            lds)) != hipSuccess)
        return e;
      if (a.queue == nullptr || per_cu < 1 || a.n_blocks > (1LL << 31) - 8) return hipErrorInvalidValue;
      ContractArgs c = a;
      c.block0 = 0;
      c.n_chunk = a.n_blocks;
      const long long nb8 = (c.n_chunk + 7) / 8 * 8;
      const long long res = ((long long)cus * per_cu + 7) / 8 * 8;
      hipLaunchKernelGGL((k_contract_seg<T, NT, true>), dim3((unsigned)(nb8 < res ? nb8 : res)), dim3(NT), lds, st, c);
      return hipGetLastError();
    }
  }
  const long long chunk = kMaxLaunchItems / NT / 8 * 8;
  for (long long b0 = 0; b0 < a.n_blocks; b0 += chunk) {
    ContractArgs c = a;
    c.block0 = b0;
    c.n_chunk = a.n_blocks - b0 < chunk ? a.n_blocks - b0 : chunk;
    const long long nb8 = (c.n_chunk + 7) / 8 * 8;
    if constexpr (SEG)
      hipLaunchKernelGGL((k_contract_seg<T, NT>), dim3((unsigned)nb8), dim3(NT), lds, st, c);
    else
      hipLaunchKernelGGL((k_contract<T, NT>), dim3((unsigned)nb8), dim3(NT), lds, st, c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace

hipError_t launch_contract(int prec, const ContractArgs& a, hipStream_t st) {
  if (a.engine == 1) {
    if (a.rstride != 16 && a.rstride != kSegRStride) return hipErrorInvalidValue;
    const size_t lds = contract_seg_lds_bytes(prec, a.max_gslots, a.max_gcontrib, a.max_gch, a.max_gstask, a.rstride);
    if (a.waves != 8 && a.waves != 16) return hipErrorInvalidValue;
    if (prec == 0)
      return a.waves == 16 ? launch_contract_t<double, 1024, true>(a, lds, st)
                           : launch_contract_t<double, 512, true>(a, lds, st);
    return a.waves == 16 ? launch_contract_t<float, 1024, true>(a, lds, st)
                         : launch_contract_t<float, 512, true>(a, lds, st);
  }
  const size_t lds = contract_lds_bytes(prec, a.max_gprod, a.max_gcontrib, a.max_gch, a.max_gtask);
  if (prec == 0) return a.waves == 8 ? launch_contract_t<double, 512, false>(a, lds, st) : hipErrorInvalidValue;
  if (a.waves == 4) return launch_contract_t<float, 256, false>(a, lds, st);
  if (a.waves == 8) return launch_contract_t<float, 512, false>(a, lds, st);
  return hipErrorInvalidValue;
}

}  // namespace nbs
