// compiler.hpp -- channel-table compiler: from a list of two-baryon channels
// to the structure-of-arrays program the contraction kernel interprets.
//
// The paper does the "symbolical manipulations" and "diagrammatical
// classification" on the CPU and ships SoA data to the device (Sec. 3(ii),
// 3(iii)).  Here that step turns each channel into diagrams d (a split of the
// six source quarks between the two sink baryons), each diagram into a pair
// of effective blocks E1^(d)(q), E2^(d)(-q) (Eq. (9)) that absorb every
// same-flavour reordering of the quarks inside a block, and the channel into
// sum_d sigma_d sum_{xi~_d} E1 E2 (Eq. (10)).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace nbs {

enum Flavour { FU = 0, FD = 1, FS = 2 };

// One flavour triplet (f1, f2, f3) of eps_abc (f1_a C g5 f2_b) f3_c.
struct Triplet {
  int f[3];
  int code() const { return (f[0] * 3 + f[1]) * 3 + f[2]; }
};

// Weighted expansion of an interpolating field (Eqs. (2)-(3)):
// op = norm * sum_k wnum_k * triplet_k with small integers wnum.
struct OpExpansion {
  double norm;
  std::vector<Triplet> trip;
  std::vector<int> wnum;
};
OpExpansion expand_operator(int op);

struct ChannelSpec {
  int sink[2], src[2];
};

// Logical description of one diagram (for inspection and tests).
struct DiagramInfo {
  int channel, src_term, set1_mask, paper_sign, k, labels1, open_mask;
  double coef;
  int product;  // index into the product list
};

// Device program ("SoA tables") for one plan; every array is plain int32 or
// double so it can be copied to the device as is.
struct Program {
  int n_types = 0;              // type slots used
  std::vector<int> type_code;   // slot -> triplet code

  // Work groups: each owns a set of channels and a range of chunks.
  std::vector<int> group_chunk;     // n_groups + 1
  std::vector<int> group_ch;        // n_groups + 1, ranges into group_channels
  std::vector<int> group_channels;  // global channel index

  // Chunks: a set of products whose effective blocks fit the LDS budget.
  std::vector<int> chunk_step;  // n_chunks + 1
  std::vector<int> chunk_meb;   // n_chunks + 1
  std::vector<int> chunk_acc;   // n_chunks + 1
  std::vector<int> chunk_esize; // entries of the chunk's E buffer

  // Load steps: bring N~_type(side ? -q : q) into LDS (if load flag), then
  // accumulate its contributions into effective-block entries.
  std::vector<int> step_type, step_side, step_load;
  std::vector<int> step_ebb;  // n_steps + 1

  // EBB items: E[ebb_e] += sum_{terms} coef * N~[idx]
  std::vector<int> ebb_e;
  std::vector<int> ebb_term;  // n_ebb + 1
  std::vector<int> terms;     // idx | (coef << 16)

  // MEB items: partial[slot][r1 * rows2 + r2] = sum_{k in [k0, k0+kn)}
  //   E[e1 + r1 * K + k] * E[e2 + r2 * K + k]
  std::vector<int> meb_e1, meb_e2, meb_K, meb_k0, meb_kn, meb_rows1;

  // Accumulation: acc[target] += sum coef * partial[src], target =
  // local channel * 16 + spin, src = item_in_chunk * 16 + output.
  std::vector<int> acc_target;
  std::vector<int> acc_src_range;  // n_acc + 1
  std::vector<int> acc_src;
  std::vector<double> acc_coef;

  int max_group_channels = 0;
  int max_chunk_items = 0;
  int max_chunk_esize = 0;
};

struct CompileOptions {
  int e_budget = 4096;      // effective-block entries per chunk
  int item_budget = 96;     // MEB items per chunk
  int k_chunk = 16;         // shared indices per MEB item
  int max_group_channels = 32;
  int group_mode = 0;       // 0: channels sharing a sink operator pair; 1: one per channel
};

struct Compiled {
  std::vector<ChannelSpec> channels;
  std::vector<DiagramInfo> diagrams;
  Program prog;
  int n_blocks = 0, n_products = 0;
  int64_t sum_k = 0, n_entries = 0, n_terms = 0, n_wick = 0;
  std::vector<int> channel_flavour;  // [n_ch][3] quark counts (u, d, s)
};

// Returns "" on success, else an error message.
std::string compile_channels(const std::vector<ChannelSpec>& ch,
                             const CompileOptions& opt, Compiled* out);

}  // namespace nbs
