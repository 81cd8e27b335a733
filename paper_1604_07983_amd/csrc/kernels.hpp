// kernels.hpp -- host-side launch interface of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace nbs {

constexpr int kBlockEntries = 3456;  // 2 x 12 x 12 x 12 complex per normal block
constexpr int kThreads = 256;

// Normal baryon blocks (Eq. (5)/(8)) of every needed flavour triplet.
struct NbbArgs {
  const void* S[3];      // u, d, s propagators: [t_count][V][12][12]
  void* Nq;              // [t_count][n_types][V][3456]
  int V, t_count, n_types;
  int type_f3[27], type_dq[27];  // per type slot: third flavour, diquark slot
  int n_dq, dq_f1[9], dq_f2[9];  // diquark flavour pairs
  int flavour_used[3];
  const int* scale_exp;  // [3][t_count] power-of-two exponents (precision form) or null
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
};

// Effective blocks + products (Eqs. (9)-(10)), program interpreted per
// (channel group, momentum, slice).
struct ContractArgs {
  const void* Nq;
  void* Ft;  // [n_ch][t_count][16][V]
  int V, Lx, Ly, Lz, t_count, n_types, n_ch, n_groups;
  long long n_blocks;  // n_groups * V * t_count
  const int *group_chunk, *group_ch, *group_channels;
  const int *chunk_step, *chunk_meb, *chunk_acc, *chunk_esize;
  const int *step_type, *step_side, *step_load, *step_ebb;
  const int *ebb_e, *ebb_term, *terms;
  const int *meb_e1, *meb_e2, *meb_K, *meb_k0, *meb_kn, *meb_rows1;
  const int *acc_target, *acc_src_range, *acc_src;
  const double* acc_coef;
  int e_budget, item_budget, max_gch;
};

// prec: 0 = FP64 form, 1 = precision form (complex64 storage, FP32 compute).
hipError_t launch_absmax(const void* S, unsigned* maxbits, long long per_slice, int t_count, hipStream_t st);
hipError_t launch_fill_u32(unsigned* p, unsigned v, long long n, hipStream_t st);
hipError_t launch_scale_exps(const unsigned* maxbits, int* exps, int n, hipStream_t st);
hipError_t launch_channel_scale(const int* exps, const int* chan_nf, double* oscale, int n_ch, int t_count,
                                hipStream_t st);
hipError_t launch_nbb(int prec, const NbbArgs& a, hipStream_t st);
// kind: 0 = complex128 -> complex128, 1 = complex64 -> complex64, 2 = complex64 -> complex128
hipError_t launch_fft_pass(int kind, const FftArgs& a, hipStream_t st);
size_t contract_lds_bytes(int prec, int e_budget, int item_budget, int max_gch);
hipError_t launch_contract(int prec, const ContractArgs& a, hipStream_t st);

}  // namespace nbs
