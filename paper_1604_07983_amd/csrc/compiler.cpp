// compiler.cpp -- channel-table compiler (see compiler.hpp).
#include "compiler.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <tuple>

namespace nbs {
namespace {

// eps_abc on {0,1,2} and C g5 = diag(i s2, i s2) (Dirac representation).
int levi(int a, int b, int c) { return (a - b) * (b - c) * (c - a) / 2; }
const int kCg5[4][4] = {{0, 1, 0, 0}, {-1, 0, 0, 0}, {0, 0, 0, 1}, {0, 0, -1, 0}};

int popcount(unsigned v) { int n = 0; for (; v; v &= v - 1) ++n; return n; }

int seq_sign(const int* s, int n) {
  int inv = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) inv += s[i] > s[j];
  return (inv & 1) ? -1 : 1;
}

// One term of an effective block: sink slot i of `type` is contracted with
// source quark m[i]; w carries the operator's integer weight and the sign of
// m as an ordering of the block's source set.
struct BlockTerm {
  int type, m[3], w;
  bool operator<(const BlockTerm& o) const {
    return std::tie(type, m[0], m[1], m[2], w) < std::tie(o.type, o.m[0], o.m[1], o.m[2], o.w);
  }
  bool operator==(const BlockTerm& o) const {
    return type == o.type && m[0] == o.m[0] && m[1] == o.m[1] && m[2] == o.m[2] && w == o.w;
  }
};

// Shape of a block determined by its source set S (bit k = source quark k).
struct Shape {
  int kA, kB;      // quarks of source baryon A (0,1,2) / B (3,4,5) inside S
  int loneA, loneB;  // the quark of a split baryon that sits alone in one block (-1: no split)
  int KA, KB;
  bool lbl3, lbl4;   // alpha_3 / alpha_4 carried by this block
  int rows() const { return 2 * (lbl3 ? 2 : 1) * (lbl4 ? 2 : 1); }
  int K() const { return KA * KB; }
};

Shape shape_of(int mask) {
  Shape s{};
  for (int half = 0; half < 2; ++half) {
    const int base = 3 * half;
    int in = 0, lone = -1;
    for (int k = 0; k < 3; ++k) in += (mask >> (base + k)) & 1;
    if (in == 2) {
      for (int k = 0; k < 3; ++k) if (!((mask >> (base + k)) & 1)) lone = base + k;
    } else if (in == 1) {
      for (int k = 0; k < 3; ++k) if ((mask >> (base + k)) & 1) lone = base + k;
    }
    const int Kp = lone < 0 ? 1 : (lone == base + 2 ? 3 : 12);
    // the label (spin of quark base+2) sits where quark base+2 is
    const bool lbl = (mask >> (base + 2)) & 1;
    if (half == 0) { s.kA = in; s.loneA = lone; s.KA = Kp; s.lbl3 = lbl; }
    else { s.kB = in; s.loneB = lone; s.KB = Kp; s.lbl4 = lbl; }
  }
  return s;
}

// Assignments of source indices j' (3 * spin + colour) to the quarks of one
// source baryon that lie in the block, for a given shared index x and label
// spin al.  The baryon tensor eps_{c1 c2 c3} (C g5)_{s1 s2} delta_{s3 al} is
// placed in the block that holds two or three of its quarks.
struct Part { int j[3]; int coef; };

std::vector<Part> source_parts(int in, int lone_local, int x, int al) {
  std::vector<Part> out;
  if (in == 0) { out.push_back({{-1, -1, -1}, 1}); return out; }
  if (in == 3) {
    for (int c0 = 0; c0 < 3; ++c0) for (int c1 = 0; c1 < 3; ++c1) for (int c2 = 0; c2 < 3; ++c2) {
      const int e = levi(c0, c1, c2);
      if (!e) continue;
      for (int s0 = 0; s0 < 4; ++s0) for (int s1 = 0; s1 < 4; ++s1) {
        if (!kCg5[s0][s1]) continue;
        out.push_back({{3 * s0 + c0, 3 * s1 + c1, 3 * al + c2}, e * kCg5[s0][s1]});
      }
    }
    return out;
  }
  if (in == 1) {  // the lone quark is here: its index is the shared one
    Part p{{-1, -1, -1}, 1};
    p.j[lone_local] = lone_local == 2 ? 3 * al + x : x;
    out.push_back(p);
    return out;
  }
  // in == 2: the lone quark is in the other block, the tensor is here
  if (lone_local == 2) {
    const int c2 = x;
    for (int c0 = 0; c0 < 3; ++c0) for (int c1 = 0; c1 < 3; ++c1) {
      const int e = levi(c0, c1, c2);
      if (!e) continue;
      for (int s0 = 0; s0 < 4; ++s0) for (int s1 = 0; s1 < 4; ++s1) {
        if (!kCg5[s0][s1]) continue;
        out.push_back({{3 * s0 + c0, 3 * s1 + c1, -1}, e * kCg5[s0][s1]});
      }
    }
    return out;
  }
  const int a = lone_local, b = 1 - a;
  const int sa = x / 3, ca = x % 3;
  for (int cb = 0; cb < 3; ++cb) for (int c2 = 0; c2 < 3; ++c2) {
    const int c0 = a == 0 ? ca : cb, c1 = a == 0 ? cb : ca;
    const int e = levi(c0, c1, c2);
    if (!e) continue;
    for (int sb = 0; sb < 4; ++sb) {
      const int g = a == 0 ? kCg5[sa][sb] : kCg5[sb][sa];
      if (!g) continue;
      Part p{{-1, -1, -1}, e * g};
      p.j[b] = 3 * sb + cb;
      p.j[2] = 3 * al + c2;
      out.push_back(p);
    }
  }
  return out;
}

struct Term { int type, idx, coef; };

// Entries of an effective block: entries[r * K + k] = list of (type, idx, coef).
std::vector<std::vector<Term>> block_entries(int mask, const std::vector<BlockTerm>& bts) {
  const Shape sh = shape_of(mask);
  const int K = sh.K(), rows = sh.rows();
  const int n3 = sh.lbl3 ? 2 : 1, n4 = sh.lbl4 ? 2 : 1;
  std::vector<std::vector<Term>> ent(rows * K);
  for (int al = 0; al < 2; ++al)
  for (int a3 = 0; a3 < n3; ++a3)
  for (int a4 = 0; a4 < n4; ++a4) {
    const int r = (al * n3 + a3) * n4 + a4;
    for (int xa = 0; xa < sh.KA; ++xa)
    for (int xb = 0; xb < sh.KB; ++xb) {
      const auto pa = source_parts(sh.kA, sh.loneA < 0 ? -1 : sh.loneA, xa, a3);
      const auto pb = source_parts(sh.kB, sh.loneB < 0 ? -1 : sh.loneB - 3, xb, a4);
      std::map<std::pair<int, int>, int> acc;
      for (const auto& A : pa)
        for (const auto& B : pb) {
          int j[6] = {A.j[0], A.j[1], A.j[2], B.j[0], B.j[1], B.j[2]};
          for (const auto& bt : bts) {
            const int idx = al * 1728 + j[bt.m[0]] * 144 + j[bt.m[1]] * 12 + j[bt.m[2]];
            acc[{bt.type, idx}] += bt.w * A.coef * B.coef;
          }
        }
      auto& e = ent[r * K + xa * sh.KB + xb];
      for (const auto& kv : acc)
        if (kv.second) e.push_back({kv.first.first, kv.first.second, kv.second});
    }
  }
  return ent;
}

// Effective block of one sink operator for source set `mask` given the
// flavours of the six source quarks.
std::vector<BlockTerm> effective_block(const OpExpansion& op, int mask, const int srcfl[6]) {
  int S[3], n = 0;
  for (int k = 0; k < 6; ++k) if ((mask >> k) & 1) S[n++] = k;
  std::vector<BlockTerm> out;
  int perm[3] = {0, 1, 2};
  for (size_t t = 0; t < op.trip.size(); ++t) {
    std::sort(perm, perm + 3);
    do {
      BlockTerm bt{};
      bt.type = op.trip[t].code();
      bool ok = true;
      for (int i = 0; i < 3; ++i) {
        bt.m[i] = S[perm[i]];
        if (op.trip[t].f[i] != srcfl[bt.m[i]]) ok = false;
      }
      if (!ok) continue;
      bt.w = op.wnum[t] * seq_sign(perm, 3);
      out.push_back(bt);
    } while (std::next_permutation(perm, perm + 3));
  }
  std::sort(out.begin(), out.end());
  return out;
}

// Permutation giving each block's source quarks in ascending order for the
// operators' first flavour terms: the representative whose sign the paper
// prints with each diagram of Eq. (7).
int paper_sign(const OpExpansion& o1, const OpExpansion& o2, int mask1, const int srcfl[6]) {
  int P[6];
  const OpExpansion* ops[2] = {&o1, &o2};
  const int masks[2] = {mask1, 0x3f & ~mask1};
  for (int side = 0; side < 2; ++side) {
    const auto& tr = ops[side]->trip;
    for (size_t t = 0; t < tr.size(); ++t) {
      int used = 0;
      bool ok = true;
      for (int i = 0; i < 3 && ok; ++i) {
        int pick = -1;
        for (int k = 0; k < 6; ++k)
          if (((masks[side] >> k) & 1) && !((used >> k) & 1) && srcfl[k] == tr[t].f[i]) { pick = k; break; }
        if (pick < 0) ok = false; else { used |= 1 << pick; P[3 * side + i] = pick; }
      }
      if (ok) break;
    }
  }
  return seq_sign(P, 6);
}

int flavour_count(const Triplet& t, int f) { return (t.f[0] == f) + (t.f[1] == f) + (t.f[2] == f); }

}  // namespace

OpExpansion expand_operator(int op) {
  OpExpansion e;
  auto T = [](int a, int b, int c) { Triplet t; t.f[0] = a; t.f[1] = b; t.f[2] = c; return t; };
  e.norm = 1.0;
  switch (op) {
    case 0: e.trip = {T(FU, FD, FU)}; e.wnum = {+1}; break;  // p
    case 1: e.trip = {T(FU, FD, FD)}; e.wnum = {-1}; break;  // n
    case 3: e.trip = {T(FU, FS, FU)}; e.wnum = {-1}; break;  // Sigma+
    case 5: e.trip = {T(FD, FS, FD)}; e.wnum = {-1}; break;  // Sigma-
    case 6: e.trip = {T(FU, FS, FS)}; e.wnum = {+1}; break;  // Xi0
    case 7: e.trip = {T(FD, FS, FS)}; e.wnum = {-1}; break;  // Xi-
    case 8: e.trip = {T(FD, FS, FU)}; e.wnum = {+1}; break;  // X_u
    case 9: e.trip = {T(FS, FU, FD)}; e.wnum = {+1}; break;  // X_d
    case 10: e.trip = {T(FU, FD, FS)}; e.wnum = {+1}; break; // X_s
    case 2:  // Lambda = (X_u + X_d - 2 X_s) / sqrt 6
      e.norm = 1.0 / std::sqrt(6.0);
      e.trip = {T(FD, FS, FU), T(FS, FU, FD), T(FU, FD, FS)};
      e.wnum = {+1, +1, -2};
      break;
    case 4:  // Sigma0 = (X_u - X_d) / sqrt 2
      e.norm = 1.0 / std::sqrt(2.0);
      e.trip = {T(FD, FS, FU), T(FS, FU, FD)};
      e.wnum = {+1, -1};
      break;
    default: e.norm = 0.0; break;
  }
  return e;
}

std::string compile_channels(const std::vector<ChannelSpec>& chans, const CompileOptions& opt,
                             Compiled* out) {
  Compiled C;
  C.channels = chans;
  const int n_ch = (int)chans.size();
  if (n_ch <= 0) return "no channels";

  // ---- 1. diagrams, effective blocks and products -------------------------
  std::map<std::pair<int, std::vector<BlockTerm>>, int> block_id[2];  // per side
  std::vector<int> block_mask[2];
  std::vector<std::vector<BlockTerm>> block_terms[2];
  std::map<std::pair<int, int>, int> product_id;
  std::vector<std::pair<int, int>> products;
  // product -> channel -> coefficient
  std::vector<std::map<int, double>> product_coef;

  for (int c = 0; c < n_ch; ++c) {
    OpExpansion op[4];
    for (int k = 0; k < 4; ++k) {
      const int code = k < 2 ? chans[c].sink[k] : chans[c].src[k - 2];
      if (code < 0 || code > 10) return "channel " + std::to_string(c) + ": bad operator code";
      op[k] = expand_operator(code);
    }
    // flavour conservation
    int nf[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (int side = 0; side < 2; ++side)
      for (int k = 0; k < 2; ++k)
        for (int f = 0; f < 3; ++f) nf[side][f] += flavour_count(op[2 * side + k].trip[0], f);
    for (int f = 0; f < 3; ++f)
      if (nf[0][f] != nf[1][f]) return "channel " + std::to_string(c) + ": flavour not conserved";
    for (int f = 0; f < 3; ++f) C.channel_flavour.push_back(nf[0][f]);

    int src_term = 0;
    for (size_t t3 = 0; t3 < op[2].trip.size(); ++t3)
      for (size_t t4 = 0; t4 < op[3].trip.size(); ++t4, ++src_term) {
        int srcfl[6];
        for (int i = 0; i < 3; ++i) {
          srcfl[i] = op[2].trip[t3].f[i];
          srcfl[3 + i] = op[3].trip[t4].f[i];
        }
        const double wsrc = op[0].norm * op[1].norm * op[2].norm * op[3].norm *
                            op[2].wnum[t3] * op[3].wnum[t4];
        for (int mask = 0; mask < 64; ++mask) {
          if (popcount(mask) != 3) continue;
          const int mask2 = 0x3f & ~mask;
          auto e1 = effective_block(op[0], mask, srcfl);
          auto e2 = effective_block(op[1], mask2, srcfl);
          if (e1.empty() || e2.empty()) continue;
          // count of Wick permutations this diagram covers (per sink term pair)
          int cross = 0;
          for (int x = 0; x < 6; ++x)
            for (int y = 0; y < 6; ++y)
              if (((mask >> x) & 1) && ((mask2 >> y) & 1) && x > y) ++cross;
          const double coef = wsrc * ((cross & 1) ? -1.0 : 1.0);
          int ids[2];
          const std::vector<BlockTerm>* es[2] = {&e1, &e2};
          const int ms[2] = {mask, mask2};
          for (int side = 0; side < 2; ++side) {
            auto key = std::make_pair(ms[side], *es[side]);
            auto it = block_id[side].find(key);
            if (it == block_id[side].end()) {
              const int id = (int)block_terms[side].size();
              block_id[side][key] = id;
              block_terms[side].push_back(*es[side]);
              block_mask[side].push_back(ms[side]);
              ids[side] = id;
            } else {
              ids[side] = it->second;
            }
          }
          auto pk = std::make_pair(ids[0], ids[1]);
          int pid;
          auto pit = product_id.find(pk);
          if (pit == product_id.end()) {
            pid = (int)products.size();
            product_id[pk] = pid;
            products.push_back(pk);
            product_coef.emplace_back();
          } else {
            pid = pit->second;
          }
          product_coef[pid][c] += coef;

          const Shape sh = shape_of(mask);
          DiagramInfo d{};
          d.channel = c;
          d.src_term = src_term;
          d.set1_mask = mask;
          d.paper_sign = paper_sign(op[0], op[1], mask, srcfl);
          d.k = sh.K();
          d.labels1 = (sh.lbl3 ? 1 : 0) | (sh.lbl4 ? 2 : 0);
          int open = 0;
          if (sh.loneA >= 0) open |= (1 << (2 * sh.loneA)) | (sh.loneA != 2 ? 1 << (2 * sh.loneA + 1) : 0);
          if (sh.loneB >= 0) open |= (1 << (2 * sh.loneB)) | (sh.loneB != 5 ? 1 << (2 * sh.loneB + 1) : 0);
          d.open_mask = open;
          d.coef = coef;
          d.product = pid;
          C.diagrams.push_back(d);
          C.sum_k += sh.K();
          // Wick permutations covered: maps of block 1 x maps of block 2,
          // per sink flavour-term pair
          std::map<std::pair<int, int>, int> cnt;
          int n1[27] = {0}, n2[27] = {0};
          for (auto& bt : e1) n1[bt.type]++;
          for (auto& bt : e2) n2[bt.type]++;
          for (int a = 0; a < 27; ++a)
            for (int b = 0; b < 27; ++b) C.n_wick += (int64_t)n1[a] * n2[b];
        }
      }
  }

  // ---- 2. entries of every block -------------------------------------------
  std::vector<std::vector<std::vector<Term>>> entries[2];
  std::set<int> used_types;
  for (int side = 0; side < 2; ++side)
    for (size_t b = 0; b < block_terms[side].size(); ++b) {
      entries[side].push_back(block_entries(block_mask[side][b], block_terms[side][b]));
      for (auto& e : entries[side].back()) {
        ++C.n_entries;
        C.n_terms += (int64_t)e.size();
        for (auto& t : e) used_types.insert(t.type);
      }
    }
  C.n_blocks = (int)(block_terms[0].size() + block_terms[1].size());
  C.n_products = (int)products.size();

  Program& P = C.prog;
  std::map<int, int> type_slot;
  for (int t : used_types) {
    type_slot[t] = (int)P.type_code.size();
    P.type_code.push_back(t);
  }
  P.n_types = (int)P.type_code.size();

  // ---- 3. groups of channels ------------------------------------------------
  std::vector<std::vector<int>> groups;
  if (opt.group_mode == 1) {
    for (int c = 0; c < n_ch; ++c) groups.push_back({c});
  } else {
    std::map<std::pair<int, int>, std::vector<int>> by_sink;
    std::vector<std::pair<int, int>> order;
    for (int c = 0; c < n_ch; ++c) {
      auto k = std::make_pair(chans[c].sink[0], chans[c].sink[1]);
      if (!by_sink.count(k)) order.push_back(k);
      by_sink[k].push_back(c);
    }
    for (auto& k : order) {
      auto& v = by_sink[k];
      for (size_t i = 0; i < v.size(); i += opt.max_group_channels)
        groups.emplace_back(v.begin() + i, v.begin() + std::min(v.size(), i + opt.max_group_channels));
    }
  }

  // products used by each channel
  std::vector<std::vector<int>> chan_products(n_ch);
  for (size_t p = 0; p < products.size(); ++p)
    for (auto& kv : product_coef[p]) chan_products[kv.first].push_back((int)p);

  P.group_chunk.push_back(0);
  P.group_ch.push_back(0);
  P.chunk_step.push_back(0);
  P.chunk_meb.push_back(0);
  P.chunk_acc.push_back(0);
  P.step_ebb.push_back(0);
  P.ebb_term.push_back(0);
  P.acc_src_range.push_back(0);

  for (auto& g : groups) {
    std::map<int, int> local;  // channel -> local index
    for (int c : g) { local[c] = (int)P.group_channels.size() - P.group_ch.back(); P.group_channels.push_back(c); }
    P.max_group_channels = std::max(P.max_group_channels, (int)g.size());
    // products of the group, ordered by their blocks so neighbours share types
    std::set<int> pset;
    for (int c : g) for (int p : chan_products[c]) pset.insert(p);
    std::vector<int> plist(pset.begin(), pset.end());
    auto type_sig = [&](int p) {
      std::set<int> t0, t1;
      for (auto& bt : block_terms[0][products[p].first]) t0.insert(bt.type);
      for (auto& bt : block_terms[1][products[p].second]) t1.insert(bt.type);
      return std::make_tuple(std::vector<int>(t0.begin(), t0.end()), std::vector<int>(t1.begin(), t1.end()),
                             products[p].first, products[p].second);
    };
    std::stable_sort(plist.begin(), plist.end(), [&](int a, int b) { return type_sig(a) < type_sig(b); });

    int slot_side = -1, slot_type = -1;
    size_t pi = 0;
    while (pi < plist.size()) {
      // greedy chunk
      std::map<std::pair<int, int>, int> eoff;  // (side, block) -> offset
      int esize = 0, items = 0;
      std::vector<int> cp;
      while (pi < plist.size()) {
        const int p = plist[pi];
        const auto& pr = products[p];
        const Shape s1 = shape_of(block_mask[0][pr.first]);
        const int K = s1.K();
        int add_e = 0;
        if (!eoff.count({0, pr.first})) add_e += s1.rows() * K;
        if (!eoff.count({1, pr.second})) add_e += (16 / s1.rows()) * K;
        const int add_i = (K + opt.k_chunk - 1) / opt.k_chunk;
        if (!cp.empty() && (esize + add_e > opt.e_budget || items + add_i > opt.item_budget)) break;
        if (!eoff.count({0, pr.first})) { eoff[{0, pr.first}] = esize; esize += s1.rows() * K; }
        if (!eoff.count({1, pr.second})) { eoff[{1, pr.second}] = esize; esize += (16 / s1.rows()) * K; }
        items += add_i;
        cp.push_back(p);
        ++pi;
      }
      if (esize > opt.e_budget || items > opt.item_budget) return "chunk exceeds LDS budget";
      P.chunk_esize.push_back(esize);
      P.max_chunk_esize = std::max(P.max_chunk_esize, esize);
      P.max_chunk_items = std::max(P.max_chunk_items, items);

      // steps: every (side, type) the chunk's entries read
      std::map<std::pair<int, int>, std::vector<std::pair<int, std::vector<Term>>>> by_step;
      for (auto& kv : eoff) {
        const int side = kv.first.first, b = kv.first.second, off = kv.second;
        const auto& ents = entries[side][b];
        for (size_t e = 0; e < ents.size(); ++e) {
          std::map<int, std::vector<Term>> per_type;
          for (auto& t : ents[e]) per_type[t.type].push_back(t);
          for (auto& pt : per_type)
            by_step[{side, pt.first}].push_back({off + (int)e, pt.second});
        }
      }
      std::vector<std::pair<int, int>> steps;
      for (auto& kv : by_step) steps.push_back(kv.first);
      // start with what the LDS slot already holds
      std::stable_partition(steps.begin(), steps.end(), [&](const std::pair<int, int>& s) {
        return s.first == slot_side && s.second == slot_type;
      });
      for (auto& st : steps) {
        const int load = !(st.first == slot_side && st.second == slot_type);
        slot_side = st.first;
        slot_type = st.second;
        P.step_side.push_back(st.first);
        P.step_type.push_back(type_slot[st.second]);
        P.step_load.push_back(load);
        for (auto& item : by_step[st]) {
          P.ebb_e.push_back(item.first);
          for (auto& t : item.second) {
            if (t.coef < -32768 || t.coef > 32767) return "term coefficient overflow";
            P.terms.push_back((t.idx & 0xffff) | (int)((unsigned)(t.coef & 0xffff) << 16));
          }
          P.ebb_term.push_back((int)P.terms.size());
        }
        P.step_ebb.push_back((int)P.ebb_e.size());
      }
      P.chunk_step.push_back((int)P.step_side.size());

      // MEB items and accumulation
      std::map<int, std::vector<std::pair<int, double>>> acc;  // target -> (src, coef)
      int item = 0;
      for (int p : cp) {
        const auto& pr = products[p];
        const Shape s1 = shape_of(block_mask[0][pr.first]);
        const int K = s1.K(), rows1 = s1.rows(), rows2 = 16 / rows1;
        const int n13 = s1.lbl3 ? 2 : 1, n14 = s1.lbl4 ? 2 : 1;
        const int n23 = s1.lbl3 ? 1 : 2, n24 = s1.lbl4 ? 1 : 2;
        const int first_item = item;
        for (int k0 = 0; k0 < K; k0 += opt.k_chunk) {
          P.meb_e1.push_back(eoff[{0, pr.first}]);
          P.meb_e2.push_back(eoff[{1, pr.second}]);
          P.meb_K.push_back(K);
          P.meb_k0.push_back(k0);
          P.meb_kn.push_back(std::min(opt.k_chunk, K - k0));
          P.meb_rows1.push_back(rows1);
          ++item;
        }
        // output o = r1 * rows2 + r2 -> spin s
        for (int o = 0; o < 16; ++o) {
          const int r1 = o / rows2, r2 = o % rows2;
          // r1 = (a1 * n13 + a3') * n14 + a4' ; r2 = (a2 * n23 + a3'') * n24 + a4''
          const int a1 = r1 / (n13 * n14), a2 = r2 / (n23 * n24);
          const int a3 = s1.lbl3 ? (r1 / n14) % n13 : (r2 / n24) % n23;
          const int a4 = s1.lbl4 ? r1 % n14 : r2 % n24;
          const int s = 8 * a1 + 4 * a2 + 2 * a3 + a4;
          for (auto& kv : product_coef[p]) {
            if (!local.count(kv.first)) continue;
            const int target = local[kv.first] * 16 + s;
            for (int it = first_item; it < item; ++it) acc[target].push_back({it * 16 + o, kv.second});
          }
        }
      }
      for (auto& kv : acc) {
        P.acc_target.push_back(kv.first);
        for (auto& sc : kv.second) {
          P.acc_src.push_back(sc.first);
          P.acc_coef.push_back(sc.second);
        }
        P.acc_src_range.push_back((int)P.acc_src.size());
      }
      P.chunk_meb.push_back((int)P.meb_e1.size());
      P.chunk_acc.push_back((int)P.acc_target.size());
    }
    P.group_chunk.push_back((int)P.chunk_esize.size());
    P.group_ch.push_back((int)P.group_channels.size());
  }
  *out = std::move(C);
  return "";
}

}  // namespace nbs
