// kernels.hpp -- host-side launch interface of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace nbs {

constexpr int kBlockEntries = 3456;  // 2 x 12 x 12 x 12 complex per normal block
constexpr int kThreads = 256;

// Operator blocks (Eq. (5)/(8) combined per Eqs. (2)-(3)) of every sink
// operator: N_op[al][j0][j1][j2] = sum_k w_k N_{trip_k}[al][j_pi(0)][j_pi(1)][j_pi(2)].
constexpr int kMaxOps = 11;

// Operator blocks in HBM.  An operator with a same-flavour slot pair
// (s1, s2) is stored antisymmetrised in that pair (N - N with the two slot
// indices exchanged) and packed: only the entries with j_s1 < j_s2, as
// [al][j_s3][p], p the index of the pair (j_s1, j_s2) among the 66 (by
// bands of equal difference j_s2 - j_s1 = 1 .. 11, ascending j_s1 within a
// band), kPackedEntries complex per site (the others are zero or negated
// copies).  Operators without a pair are stored
// as [al][j0][j1][j2], kBlockEntries complex per site.  Per geometry the
// blocks of operator op start at cum[op] * t_count * V entries and hold
// [t][site][ne[op]].
constexpr int kPackedEntries = 2 * 12 * 66;
struct BlockLayout {
  int ne[kMaxOps];    // entries per site: kBlockEntries or kPackedEntries
  int cum[kMaxOps];   // sum of ne over the earlier operators
  int pair[kMaxOps];  // s1 | s2 << 2 of the stored antisymmetrised pair, or -1
};
// first entry of the block of operator op, slice t (of t_count), site
__host__ __device__ inline long long block_offset(const BlockLayout& b, int op, int t_count, int t, long long V,
                                                  long long site) {
  return (long long)b.cum[op] * t_count * V + ((long long)t * V + site) * b.ne[op];
}

struct NbbArgs {
  const void* S[3];      // u, d, s propagators: [t_count][V][12][12]
  void* Nq;              // operator blocks, BlockLayout
  int V, t_count, n_ops;
  int n_dq, dq_f1[4], dq_f2[4];    // diquark flavour pairs
  int op_nterm[kMaxOps];
  int op_dq[kMaxOps][3], op_f3[kMaxOps][3], op_perm[kMaxOps][3];  // perm: pi(0) | pi(1) << 2 | pi(2) << 4
  double op_w[kMaxOps][3];
  BlockLayout lay;
  int flavour_used[3];
  const int* scale_exp;  // [3][t_count] power-of-two exponents (precision form) or null
  unsigned* nonfinite;   // set to 1 when a propagator entry read is NaN or infinite
};

// One axis of a batched 3-D transform on an array viewed as
// [outer][n][inner] (inner contiguous).  out may equal in.
struct FftArgs {
  const void* in;
  void* out;
  long long outer, inner;
  int n, IB, OB, sign;
  const double* oscale;   // optional per-outer-group factor oscale[o / oscale_div]
  long long oscale_div;
  double gscale;          // global factor
  long long unit0;        // first tile (LDS kernel) or line (register kernel) of this launch
};

// The x and y axes of a batched transform in one pass: the array is
// [planes][Ly][Lx][inner]; a workgroup transforms IB consecutive fields of
// one plane through LDS.  The same arguments serve the one-pass transform
// of cubic lattices, planes then counting cubes [Lz][Ly][Lx][inner].  in
// may equal out.
struct FftPlaneArgs {
  const void* in;
  void* out;
  long long planes, inner;
  int IB;
  long long unit0;    // first workgroup of this launch
  long long n_units;  // workgroups of this launch
};

// Workgroups per launch stay below this bound, so that workgroups x threads
// stays below the 2^32 work-items a dispatch can address; larger grids are
// issued as several launches with an offset.
constexpr long long kMaxLaunchItems = 1LL << 31;

// LDS layout of a staged operator block N~[al][j0][j1][j2] in the
// contraction kernel: odd strides for the two leading source indices so the
// lanes of a team (which differ in those indices) spread over the LDS banks
// (144 and 12 complex entries are multiples of the bank cycle).  The channel
// compiler precomputes per-product offsets in these units.
// The spin stride is 4 modulo 8 (complex entries) so that the rows of an
// effective block, which differ by it and by a label weight, fall in
// different LDS banks.
constexpr int kLdsJ0 = 157, kLdsJ1 = 13, kLdsAl = 1892, kLdsBlock = 2 * kLdsAl;
// Integers per block-product descriptor (layout documented in compiler.hpp).
constexpr int kProdInts = 48;
// Segment descriptors of the matrix-core contraction: integers per
// descriptor, teams (one descriptor each) per wavefront task.
constexpr int kSegInts = 16, kSegTeams = 4;
// result slots of the segment contraction: 16 complex values, spaced 17
// apart so that the lanes summing one channel output (same entry of
// different slots) fall in different LDS banks
constexpr int kSegRStride = 17;
constexpr int kSegC144 = 0, kSegC9 = 1, kSegC36 = 2, kSegC1 = 3, kSegIdle = 15;

// One geometry of a contraction launch: its blocks, its F~ output and its
// first (slice, momentum) pair: geometry i owns the pairs [block0, block0 +
// V * t_count), in geometry order.
struct ContractGeom {
  const void* Nq;  // operator blocks, BlockLayout
  void* Ft;        // [n_ch][t_count][16][V]
  int V, Lx, Ly, Lz, t_count, pad;
  long long block0;
  // momentum of the i-th workgroup of a slice: q and -q are consecutive, so
  // the two workgroups that read the same pair of blocks run together and
  // the second finds them in the cache
  const int* qorder;
};
constexpr int kMaxGeom = 32;

// Effective blocks and their products (Eqs. (9)-(10)) per (group, q, slice),
// over every geometry of the plan in one launch.
struct ContractArgs {
  const ContractGeom* geo;  // device table, n_geom entries
  int n_geom, n_ops, n_groups;
  long long n_blocks;  // n_gchunk times the sum over geometries of V * t_count
  // the sink-operator groups split into n_gchunk consecutive ranges
  // [gchunk[c], gchunk[c + 1]), one workgroup per range and (slice, momentum)
  const int* gchunk;
  int n_gchunk;
  const int *group_op1, *group_op2, *group_prod, *group_task, *group_ch, *group_channels;
  const int *ch_contrib, *contrib_prod, *prod_desc, *task_lanes;
  const double* contrib_coef;
  int max_gprod, max_gcontrib, max_gch, max_gtask;
  int waves;  // wavefronts the compiled tasks are balanced over
  // matrix-core contraction (engine 1): segment tasks per group, extra
  // result slots per product, result slots per group
  int engine;
  const int *seg_task, *group_stask, *prod_ext, *contrib_ext;
  int max_gslots, max_gstask;
  int rstride;  // complex values between result slots: kSegRStride, or 16 where that does not fit
  // persistent launch: resident workgroups claim work items from eight
  // counters (queue[8], zeroed before each launch)
  int persistent;
  unsigned* queue;
  long long block0, n_chunk;  // logical workgroups [block0, block0 + n_chunk) in this launch
  BlockLayout lay;
};

// Zero-momentum single-baryon two-point functions of one geometry: pair k
// reads the transformed block of operator slot slot[k] at q = 0 (times
// slot_coef[k], the isospin alias factor), contracts it with the
// one-baryon source tensor through term_map / term_coef (slot i with source
// quark (map >> 2 i) & 3), undoes the precision form's scale 2^(sum_f
// nf[k][f] exps[f][t]) when exps is given, and writes complex128
// C[k][t][a][a'].
constexpr int kMaxTwoPointPairs = 8, kMaxTwoPointTerms = 18;
struct TwoPointArgs {
  const void* Nq;  // operator blocks, BlockLayout
  BlockLayout lay;
  void* C;
  const int* exps;
  int V, t_count, n_pairs;
  int slot[kMaxTwoPointPairs];
  double slot_coef[kMaxTwoPointPairs];
  int nf[kMaxTwoPointPairs][3];
  int n_terms[kMaxTwoPointPairs];
  int term_map[kMaxTwoPointPairs][kMaxTwoPointTerms];
  double term_coef[kMaxTwoPointPairs][kMaxTwoPointTerms];
};
hipError_t launch_two_point(int prec, const TwoPointArgs& a, hipStream_t st);

// prec: 0 = FP64 form, 1 = precision form (complex64 storage, FP32 compute).
hipError_t launch_absmax(const void* S, unsigned* maxbits, long long per_slice, int t_count, hipStream_t st);
hipError_t launch_fill_u32(unsigned* p, unsigned v, long long n, hipStream_t st);
hipError_t launch_scale_exps(const unsigned* maxbits, int* exps, int n, hipStream_t st);
hipError_t launch_channel_scale(const int* exps, const int* chan_nf, double* oscale, int n_ch, int t_count,
                                hipStream_t st);
hipError_t launch_nbb(int prec, const NbbArgs& a, hipStream_t st);
// kind: 0 = complex128 -> complex128, 1 = complex64 -> complex64, 2 = complex64 -> complex128
hipError_t launch_fft_pass(int kind, const FftArgs& a, hipStream_t st);
// Lengths with a register-resident kernel, and its launcher (kind as above;
// the forward precision-form kind takes sign -1, the mixed kind sign +1).
bool fft_line_supported(int n, int kind);
// Square planes with a fused x-y kernel (forward transforms of the blocks,
// kinds 0 and 1); fields per workgroup for an inner extent, 0 if none fits.
int fft_plane_fields(int n, long long inner, int kind);
// fields per workgroup of the one-pass transform of an n^3 cube (0: no
// kernel for this length, storage kind or field count)
int fft_cube_fields(int n, long long inner, int kind);
hipError_t launch_fft_cube(int kind, int n, const FftPlaneArgs& a, hipStream_t st);
// the inverse transform of contiguous n^3 cubes (inner 1, sign +1) in one
// pass, kind 0 (complex128 in) or 2 (complex64 in), complex128 out
bool fft_cube_inv_supported(int n, int kind);
hipError_t launch_fft_cube_inv(int kind, const FftArgs& a, hipStream_t st);
hipError_t launch_fft_plane(int kind, int n, const FftPlaneArgs& a, hipStream_t st);
hipError_t launch_fft_line(int kind, const FftArgs& a, hipStream_t st);
size_t contract_lds_bytes(int prec, int max_gprod, int max_gcontrib, int max_gch, int max_gtask);
size_t contract_seg_lds_bytes(int prec, int max_gslots, int max_gcontrib, int max_gch, int max_gstask, int rstride);
// Wavefronts per contraction workgroup for a precision (the channel compiler
// balances each group's tasks over this many).
int contract_waves(int prec);
hipError_t launch_contract(int prec, const ContractArgs& a, hipStream_t st);
// Sets the dynamic-LDS limits of the kernels that need more than the
// default; called once per plan before any launch (and so outside any
// stream capture).
hipError_t prepare_kernels(int prec, int waves, size_t contract_lds, int engine);

}  // namespace nbs
