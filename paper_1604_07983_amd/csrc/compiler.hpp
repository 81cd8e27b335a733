// compiler.hpp -- channel-table compiler: from a list of two-baryon channels
// to the structure-of-arrays program the contraction kernel interprets.
//
// The paper does the "symbolical manipulations" and "diagrammatical
// classification" on the CPU and ships SoA data to the device (Sec. 4(ii),
// 3(iii)).  Here that step turns each channel into diagrams d (a split of the
// six source quarks between the two sink baryons), each diagram into a pair
// of effective blocks E1^(d)(q), E2^(d)(-q) (Eq. (9)) that absorb every
// same-flavour reordering of the quarks inside a block, and the channel into
// sum_d sigma_d sum_{xi~_d} E1 E2 (Eq. (10)).
//
// Blocks are built per sink *operator* (Sec. 4(i): the Lambda and Sigma0
// blocks are combinations of the X_u, X_d, X_s blocks), so every effective
// block reads one operator block.  The device program is coarse: per block
// product a fixed-size descriptor, per wavefront a 64-lane work list; the
// entries of an effective block are generated from index arithmetic on the
// device, not from per-term tables.
#pragma once

#include "kernels.hpp"

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

// Flavours of the three slots of an operator block: the triplet itself for
// single-term operators, (u, d, s) for the X combinations Lambda and Sigma0.
void operator_slots(int op, int fl[3]);

// The two slots of an operator block that carry the same flavour (p: the two
// u slots 0 and 2; n: the d slots 1 and 2; ...), or false when all three
// differ (X_u, X_d, X_s, Lambda, Sigma0).  For such an operator every
// flavour-respecting map of its slots onto a set of source quarks comes with
// its partner that exchanges the quarks of the two slots, with the opposite
// sign, so the stored block is the antisymmetrised one
//   A[al][j0][j1][j2] = N[al][j0][j1][j2] - N[al][j0'][j1'][j2'],
// j' = j with the indices of slots s1 and s2 exchanged, and one map of each
// partner pair (the one with m[s1] < m[s2]) reads it.
bool operator_pair(int op, int* s1, int* s2);

struct ChannelSpec {
  int sink[2], src[2];
};

// Logical description of one diagram (for inspection and tests).
struct DiagramInfo {
  int channel, src_term, set1_mask, paper_sign, k, labels1, open_mask;
  double coef;
};

// Integers per block-product descriptor (layout in kernels and tests):
//  [0] mask1 [1] nmaps1 [2..7] maps1  [8] mask2 [9] nmaps2 [10..15] maps2
//  [16] K [17] KB [18] rows1 [19] label flags of block 1 (bit0 a3, bit1 a4)
//  and, for products with a shared index (K > 1), offsets in the kernel's
//  LDS layout (kLdsJ0, kLdsJ1, 1 for the three slots of a block):
//  [20] lone1, [21] lone2: local index of the lone quark of block 1's pair
//       baryon (it sits in block 2) and of block 2's pair baryon
//  [24 + 6 m + 0..5], map m of block 1: offset unit of the pair's first and
//       second quark and of the walked (z) quark, the row weights of its
//       spin labels (least significant first), sign
//  [36 + 6 m + 0..5], map m of block 2: offset unit of the fixed (y) quark
//       and of the pair's first and second quark, row weights, sign
// A map packs m0 | m1 << 3 | m2 << 6 | (sign < 0) << 9: operator-block slot
// i is contracted with source quark m_i.  kProdInts (48) is defined with
// the kernel's LDS layout in kernels.hpp.
// Lane word of a wavefront task: product (12 bits) | y << 12 (4 bits) |
// log2(team) << 16 (3 bits) | z0 << 19 (4 bits) | zsl << 23 (3 bits) |
// class << 26 (5 bits); product 0xfff = idle lane.  For K > 1, y is the
// lane's fixed shared index on the side where block 1 holds a quark pair and
// the lane walks the other side's index z = z0, z0 + 2^zsl, ... (the team is
// 2^zsl sets of 4 or 16 lanes, lane y + set size * z0).  For K = 1 the team
// has 16 lanes whose y = 0..15 share the 24 source-tensor terms.  All teams
// of one task have the same size and class; a task of class kClassIdle is
// empty.
constexpr int kLanesPerTask = 64;

// Product classes (kernel dispatch; every task holds one class, so the
// dispatch is wavefront-uniform): 0 .. 3 = two full projections (K = 1),
// 2 (nmaps1 - 1) + (nmaps2 - 1); 4 + 4 b + 2 (nmaps1 - 1) + (nmaps2 - 1) for
// the split shapes b = 0: 4 x 4 rows, 2 + 2 pair terms (K = 144); b = 1:
// 8 x 2 rows, 2 + 8 (K = 36); b = 2: 2 x 8 rows, 8 + 2 (K = 36); b = 3: 4 x 4
// rows, 8 + 8 (K = 9); kClassSplitAny = any other split product.
constexpr int kClassFullEnd = 4;
// Precision form with matrix cores: the 4 x 4-row split shapes (b = 0, 3)
// as 20 + 4 b' + 2 (nmaps1 - 1) + (nmaps2 - 1), b' = 0 for b = 0 and 1 for
// b = 3.  Their teams are quads: the four lanes of a quad walk one stream of
// shared indices, lane r building row r of both effective blocks, and the
// quad's outer products go to v_mfma_f32_4x4x1f32 (16 blocks of 4 x 4).
constexpr int kClassMfmaBegin = 20, kClassMfmaEnd = 28;
inline bool class_is_mfma(int c) { return c >= kClassMfmaBegin && c < kClassMfmaEnd; }
constexpr int kClassIdle = 30;
constexpr int kClassSplitAny = 31;
int product_class(int K, int rows1, int lone1, int lone2, int nm1, int nm2);

// ---- segment program of the matrix-core contraction ------------------------
// Each block product F[r1][r2] = sum_k E1[r1][k] E2[r2][k] (Eq. (10)) is
// cut into segments of consecutive steps; a step feeds one 4 x 4 x 4 (FP64)
// or four 4 x 4 x 1 (FP32) matrix products of a 16-lane team, lane (h, x)
// supplying row x of both effective blocks at shared-index slot k' = 4 s + h.
// Shapes (the product class):
//   kSegC144: 4 x 4 rows, both lone quarks spin-colour (K = 144); shared
//             index k' = 12 v1 + v2, v1 = s / 3, v2 = 4 (s % 3) + h
//   kSegC9:   4 x 4 rows, both lone quarks colour only (K = 9): k' = 3 v1 + v2
//   kSegC36:  8 x 2 rows (the 2-term side A has 8 rows, the 8-term side B 2):
//             two accumulators for side A's rows x and x + 4, side B fed on
//             lanes x < 2 (zero elsewhere); k' = 12 v2 + v1, v2 = s / 3,
//             v1 = 4 (s % 3) + h
// Segments start and end on multiples of three steps.
//   kSegC1:   two full projections (K = 1): the 24 source-tensor terms of
//             each side are spread over the four h lanes and summed first
// Side A of a product is block 1 (sink operator at +q) except for the
// transposed 2 x 8 products, whose 8-row side is block 2.  On side A the
// pair of source quarks is indexed by v1 and the single quark by v2; on side
// B the pair by v2 and the single by v1.
// Descriptor (kSegInts ints):
//   [0] shape  [1] first step  [2] steps  [3] result slot | (sign < 0) << 16 |
//   transposed << 17
//   [4..9]   side A: unit of the single quark, units of the pair's two
//            quarks, row weights w0, w1, w2 (row r at (r & 1) w0 +
//            ((r >> 1) & 1) w1 + ((r >> 2) & 1) w2)
//   [10..15] side B, the same fields
// For kSegC1 the three units are those of the baryon's quarks 2, 0, 1.
// The first segment of product p writes result slot p; further segments
// take slots from the number of products on, and prod_ext[p] = first extra
// slot | count << 16 lists them; contrib_ext[c] repeats the word of
// contribution c's product, so that each channel sum adds a product's
// segments itself.
// (the shape codes kSegC144 .. kSegIdle are defined in kernels.hpp)

struct Program {
  // operator blocks built by the NBB kernel: slot -> operator code and
  // recipe N_op = sum_k w_k N_{f1 f2 f3}[al][j_{pi(0)}][j_{pi(1)}][j_{pi(2)}]
  int n_ops = 0;
  std::vector<int> op_code;
  std::vector<int> op_nterm;        // per slot
  std::vector<int> op_term_trip;    // [slot * 3 + k] triplet code
  std::vector<int> op_term_perm;    // [slot * 3 + k] pi(0) | pi(1) << 2 | pi(2) << 4
  std::vector<double> op_term_w;    // [slot * 3 + k]
  std::vector<int> op_pair;         // [slot] s1 | s2 << 2 of the antisymmetrised slot pair, or -1
  // Isospin-symmetric limit (S_d = S_u, Sec. 4(i)): slot s equals
  // op_alias_coef[s] times slot op_alias[s]; the n_canon canonical slots
  // come first and are the only ones built in that limit.
  std::vector<int> op_alias;
  std::vector<double> op_alias_coef;
  int n_canon = 0;

  // groups: channels sharing a sink operator pair
  std::vector<int> group_op1, group_op2;  // operator slots (momentum +q, -q)
  std::vector<int> group_prod;            // n_groups + 1, products (units of kProdInts)
  std::vector<int> group_task;            // n_groups + 1, tasks (units of 64 lanes)
  std::vector<int> group_ch;              // n_groups + 1, into group_channels
  std::vector<int> group_channels;        // global channel index
  std::vector<int> ch_contrib;            // per group-channel slot + 1, into contrib_*
  std::vector<int> contrib_prod;          // product (local) | rows1 << 16 | label flags << 20
  std::vector<double> contrib_coef;
  // the same groups read from canonical slots, the alias coefficients of
  // both operators folded into the channel coefficients
  std::vector<int> group_op1_iso, group_op2_iso;
  std::vector<double> contrib_coef_iso;
  std::vector<int> prod_desc;
  std::vector<int> task_lanes;
  // matrix-core program: tasks of kSegTeams segment descriptors (wavefront-
  // uniform shape and step count), per group a range of tasks, per product
  // its extra result slots
  std::vector<int> seg_task;      // [task][team][kSegInts]
  std::vector<int> group_stask;   // n_groups + 1
  std::vector<int> prod_ext;      // per product (global index)
  std::vector<int> contrib_ext;   // per contribution: prod_ext of its product
  int max_group_slots = 0;        // result slots (products + extra segments)
  int max_group_stasks = 0;
  int max_group_products = 0;
  int max_group_channels = 0;
  int max_group_contrib = 0;
  int max_group_tasks = 0;
};

struct CompileOptions {
  int max_group_products = 88;  // LDS result buffer bound per group
  int waves = 8;                // wavefronts of a contraction workgroup
  int seg_waves = 16;           // wavefronts of a matrix-core contraction workgroup
  int max_group_slots = 160;    // result slots of the matrix-core contraction
  bool split = true;            // may split a product's walked index over lanes
  bool mfma = false;            // 4 x 4-row split products on matrix cores (precision form)
  bool fp32 = false;            // precision form: the LDS bank model of 8-byte entries
};

struct Compiled {
  std::vector<ChannelSpec> channels;
  std::vector<DiagramInfo> diagrams;
  Program prog;
  int n_blocks = 0, n_products = 0;
  int64_t sum_k = 0, n_entries = 0, n_terms = 0, n_wick = 0, product_k = 0;
  std::vector<int> channel_flavour;  // [n_ch][3] quark counts (u, d, s)
};

// Returns "" on success, else an error message.
std::string compile_channels(const std::vector<ChannelSpec>& ch,
                             const CompileOptions& opt, Compiled* out);

// Zero-momentum single-baryon two-point function of a sink-operator block
// with a source operator: for each weighted flavour term of the source and
// each flavour-respecting map of the block's slots onto its three quarks
// (slot i contracted with source quark m[i]), the map and the source weight
// times the map's sign (Eq. (1) with one baryon on each side, Eqs. (2)-(5)).
struct TwoPointTerm {
  int m[3];
  double coef;
};
std::vector<TwoPointTerm> two_point_terms(int sink_op, int src_op);
// Quark flavour counts (u, d, s) of an operator's block slots.
void operator_flavour_counts(int op, int nf[3]);

}  // namespace nbs
