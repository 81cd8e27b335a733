// compiler.cpp -- channel-table compiler (see compiler.hpp).
#include "compiler.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <set>
#include <tuple>

namespace nbs {
namespace {

int popcount(unsigned v) { int n = 0; for (; v; v &= v - 1) ++n; return n; }

int seq_sign(const int* s, int n) {
  int inv = 0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) inv += s[i] > s[j];
  return (inv & 1) ? -1 : 1;
}

// Shape of a block determined by its source set S (bit k = source quark k).
struct Shape {
  int kA, kB;        // quarks of source baryon A (0,1,2) / B (3,4,5) inside S
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
    const bool lbl = (mask >> (base + 2)) & 1;  // spin label sits with quark base+2
    if (half == 0) { s.kA = in; s.loneA = lone; s.KA = Kp; s.lbl3 = lbl; }
    else { s.kB = in; s.loneB = lone; s.KB = Kp; s.lbl4 = lbl; }
  }
  return s;
}

// Number of (colour, spin) terms the source tensor contributes to one entry
// of a block holding `in` quarks of a source baryon whose lone quark is lone_local.
int part_terms(int in, int lone_local) {
  if (in == 3) return 24;
  if (in == 2) return lone_local == 2 ? 8 : 2;
  return 1;
}

// A map of operator-block slots to source quarks with its sign.
struct Map {
  int m[3], sign;
  bool operator<(const Map& o) const { return std::tie(m[0], m[1], m[2], sign) < std::tie(o.m[0], o.m[1], o.m[2], o.sign); }
  bool operator==(const Map& o) const { return m[0] == o.m[0] && m[1] == o.m[1] && m[2] == o.m[2] && sign == o.sign; }
  int packed() const { return m[0] | (m[1] << 3) | (m[2] << 6) | ((sign < 0) << 9); }
};

// Effective block of a sink operator for source set `mask`: every
// flavour-respecting map of its slots onto the set, signed by the parity of
// the map as an ordering of the set (the paper's effective block, Eq. (9)).
std::vector<Map> effective_block(int op, int mask, const int srcfl[6]) {
  int fl[3];
  operator_slots(op, fl);
  int S[3], n = 0;
  for (int k = 0; k < 6; ++k) if ((mask >> k) & 1) S[n++] = k;
  std::vector<Map> out;
  int perm[3] = {0, 1, 2};
  do {
    Map mp{};
    bool ok = true;
    for (int i = 0; i < 3; ++i) {
      mp.m[i] = S[perm[i]];
      if (fl[i] != srcfl[mp.m[i]]) ok = false;
    }
    if (!ok) continue;
    mp.sign = seq_sign(perm, 3);
    out.push_back(mp);
  } while (std::next_permutation(perm, perm + 3));
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

// Kernel dispatch class of a block product (see compiler.hpp).
int product_class(int K, int rows1, int lone1, int lone2, int nm1, int nm2) {
  if (nm1 < 1 || nm1 > 2 || nm2 < 1 || nm2 > 2) return kClassSplitAny;
  if (K == 1) return (nm1 - 1) * 2 + (nm2 - 1);
  const int np1 = lone1 == 2 ? 8 : 2, np2 = lone2 == 2 ? 8 : 2;
  int base = -1;
  if (rows1 == 4 && np1 == 2 && np2 == 2) base = 4;
  if (rows1 == 8 && np1 == 2 && np2 == 8) base = 8;
  if (rows1 == 2 && np1 == 8 && np2 == 2) base = 12;
  if (rows1 == 4 && np1 == 8 && np2 == 8) base = 16;
  if (base < 0) return kClassSplitAny;
  return base + (nm1 - 1) * 2 + (nm2 - 1);
}

namespace {

struct Block {
  int mask;
  std::vector<Map> maps;
  bool operator<(const Block& o) const { return std::tie(mask, maps) < std::tie(o.mask, o.maps); }
};

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

void operator_slots(int op, int fl[3]) {
  if (op == 2 || op == 4) { fl[0] = FU; fl[1] = FD; fl[2] = FS; return; }
  const OpExpansion e = expand_operator(op);
  for (int i = 0; i < 3; ++i) fl[i] = e.trip.empty() ? -1 : e.trip[0].f[i];
}

bool operator_pair(int op, int* s1, int* s2) {
  int fl[3];
  operator_slots(op, fl);
  for (int a = 0; a < 3; ++a)
    for (int b = a + 1; b < 3; ++b)
      if (fl[a] >= 0 && fl[a] == fl[b]) {
        *s1 = a;
        *s2 = b;
        return true;
      }
  return false;
}

namespace {

// Maps of an operator block onto a source set as read from the stored
// block: for an operator with a same-flavour slot pair (s1, s2) the maps come
// in partner pairs m, m' (m' exchanges the quarks of s1 and s2, sign(m') =
// -sign(m)), and sign(m) N[m] + sign(m') N[m'] = sign(m) A[m] on the
// antisymmetrised block A, so only the partner with m[s1] < m[s2] is kept.
std::vector<Map> on_stored_block(int op, const std::vector<Map>& maps) {
  int s1 = 0, s2 = 0;
  if (!operator_pair(op, &s1, &s2)) return maps;
  std::vector<Map> out;
  for (const Map& m : maps)
    if (m.m[s1] < m.m[s2]) out.push_back(m);
  return out;
}

// Offset unit of source quark q in a block under map mp: the LDS stride of
// the slot contracted with q, 0 if q is not in the block.
int quark_unit(const Map& mp, int q) {
  return (mp.m[0] == q ? nbs::kLdsJ0 : 0) + (mp.m[1] == q ? nbs::kLdsJ1 : 0) + (mp.m[2] == q ? 1 : 0);
}

// Row weights of a block's spin labels, least significant row bit first:
// rows are r = (al n3 + a3) n4 + a4, and a label of quark 2 (5) moves the
// spin of that quark's slot, i.e. 3 units of its stride.
void label_weights(const Shape& sh, const Map& mp, int w[2]) {
  int n = 0;
  w[0] = w[1] = 0;
  if (sh.lbl4) w[n++] = 3 * quark_unit(mp, 5);
  if (sh.lbl3) w[n++] = 3 * quark_unit(mp, 2);
}

// Per-product offsets of a split product (descriptor entries 20..47).
void fill_split_offsets(const Block& b1, const Block& b2, int* d) {
  const Shape s1 = shape_of(b1.mask), s2 = shape_of(b2.mask);
  const bool pairA = s1.kA == 2;
  const int base1 = pairA ? 0 : 3, base2 = pairA ? 3 : 0;
  const int lone1 = (pairA ? s1.loneA : s1.loneB) - base1;
  const int lone2 = (pairA ? s2.loneB : s2.loneA) - base2;
  const int p1 = base1 + (lone1 == 0 ? 1 : 0), q1 = base1 + (lone1 == 2 ? 1 : 2);
  const int p2 = base2 + (lone2 == 0 ? 1 : 0), q2 = base2 + (lone2 == 2 ? 1 : 2);
  const int ys = base1 + lone1, zs = base2 + lone2;
  d[20] = lone1;
  d[21] = lone2;
  for (size_t m = 0; m < b1.maps.size() && m < 2; ++m) {
    int* e = d + 24 + 6 * m;
    int w[2];
    label_weights(s1, b1.maps[m], w);
    e[0] = quark_unit(b1.maps[m], p1);
    e[1] = quark_unit(b1.maps[m], q1);
    e[2] = quark_unit(b1.maps[m], zs);
    e[3] = w[0];
    e[4] = w[1];
    e[5] = b1.maps[m].sign;
  }
  for (size_t m = 0; m < b2.maps.size() && m < 2; ++m) {
    int* e = d + 36 + 6 * m;
    int w[2];
    label_weights(s2, b2.maps[m], w);
    e[0] = quark_unit(b2.maps[m], ys);
    e[1] = quark_unit(b2.maps[m], p2);
    e[2] = quark_unit(b2.maps[m], q2);
    e[3] = w[0];
    e[4] = w[1];
    e[5] = b2.maps[m].sign;
  }
}

// ---- segment program of the matrix-core contraction (compiler.hpp) -----------

// Row-offset generator of a block side: row r = (al n3 + a3) n4 + a4 sits at
// (r & 1) w0 + ((r >> 1) & 1) w1 + ((r >> 2) & 1) w2.
void row_generator(const Shape& sh, const Map& mp, int w[3]) {
  int lw[2];
  label_weights(sh, mp, lw);
  const int nl = (sh.lbl3 ? 1 : 0) + (sh.lbl4 ? 1 : 0);
  w[0] = nl == 0 ? nbs::kLdsAl : lw[0];
  w[1] = nl == 0 ? 0 : (nl == 1 ? nbs::kLdsAl : lw[1]);
  w[2] = nl == 2 ? nbs::kLdsAl : 0;
}

// Shape, side fields and sign of the segments of one block product (one
// map per block: operators with a same-flavour slot pair are read
// antisymmetrised).  Returns false for a shape the kernel lacks.
bool segment_fields(const Block& b1, const Block& b2, int* shape, int* steps, int hdr3, int* d) {
  const Shape s1 = shape_of(b1.mask), s2 = shape_of(b2.mask);
  if (b1.maps.size() != 1 || b2.maps.size() != 1) return false;
  const Map& m1 = b1.maps[0];
  const Map& m2 = b2.maps[0];
  int side1[6], side2[6];
  if (s1.K() == 1) {
    const int base1 = s1.kA == 3 ? 0 : 3, base2 = 3 - base1;
    side1[0] = quark_unit(m1, base1 + 2); side1[1] = quark_unit(m1, base1); side1[2] = quark_unit(m1, base1 + 1);
    side2[0] = quark_unit(m2, base2 + 2); side2[1] = quark_unit(m2, base2); side2[2] = quark_unit(m2, base2 + 1);
    *shape = kSegC1;
    *steps = 1;
  } else {
    const bool pairA = s1.kA == 2;
    const int base1 = pairA ? 0 : 3, base2 = pairA ? 3 : 0;
    const int lone1 = (pairA ? s1.loneA : s1.loneB) - base1;
    const int lone2 = (pairA ? s2.loneB : s2.loneA) - base2;
    const int p1 = base1 + (lone1 == 0 ? 1 : 0), q1 = base1 + (lone1 == 2 ? 1 : 2);
    const int p2 = base2 + (lone2 == 0 ? 1 : 0), q2 = base2 + (lone2 == 2 ? 1 : 2);
    const int ys = base1 + lone1, zs = base2 + lone2;
    // block 1: pair indexed by y, single quark zs; block 2: single ys, pair by z
    side1[0] = quark_unit(m1, zs); side1[1] = quark_unit(m1, p1); side1[2] = quark_unit(m1, q1);
    side2[0] = quark_unit(m2, ys); side2[1] = quark_unit(m2, p2); side2[2] = quark_unit(m2, q2);
    if (lone1 < 2 && lone2 < 2) { *shape = kSegC144; *steps = 36; }
    else if (lone1 == 2 && lone2 == 2) { *shape = kSegC9; *steps = 3; }
    else { *shape = kSegC36; *steps = 9; }
  }
  row_generator(s1, m1, side1 + 3);
  row_generator(s2, m2, side2 + 3);
  // the 2 x 8 products run transposed: block 2 (8 rows) is side A
  const bool transposed = *shape == kSegC36 && s1.rows() == 2;
  const int* sa = transposed ? side2 : side1;
  const int* sb = transposed ? side1 : side2;
  d[0] = *shape;
  d[3] = hdr3 | ((m1.sign * m2.sign < 0) << 16) | (transposed << 17);
  for (int i = 0; i < 6; ++i) {
    d[4 + i] = sa[i];
    d[10 + i] = sb[i];
  }
  return true;
}

// Cost of one step of a segment shape for one lane (block entries read) and
// of a segment's set-up and result store, in the same units.
double seg_step_cost(int shape) {
  return shape == kSegC144 ? 4.0 : shape == kSegC9 ? 16.0 : shape == kSegC36 ? 12.0 : 24.0;
}
constexpr double kSegOverhead = 8.0;

// LDS entries a segment's team reads, per read instruction of the kernel's
// step loop (the 4 x 4 and 8 x 2 shapes): 16 lanes in (slot h, row x)
// order, -1 where the lane is inactive.  The same index arithmetic as the
// kernel's step loop.
void seg_read_addrs(const std::vector<int>& d, std::vector<std::array<int, 16>>& out) {
  out.clear();
  const int shape = d[0], s0 = d[1], n = d[2];
  const bool tr = (d[3] >> 17) & 1;
  const int SA = tr ? nbs::kLdsBlock : 0, SB = tr ? 0 : nbs::kLdsBlock;
  const int* wa = &d[7];
  const int* wb = &d[13];
  auto row = [](int r, const int* w) { return (r & 1) * w[0] + ((r >> 1) & 1) * w[1] + ((r >> 2) & 1) * w[2]; };
  auto pair2 = [](int v, int up, int uq, int& o0, int& o1) {
    const int sp = v / 3, c = v % 3, c1 = (c + 1) % 3, c2 = (c + 2) % 3, jp = 3 * (sp ^ 1);
    const int a = (jp + c1) * up + c2 * uq, b = (jp + c2) * up + c1 * uq;
    o0 = (sp & 1) ? b : a;
    o1 = (sp & 1) ? a : b;
  };
  std::array<int, 16> A;
  if (shape == kSegC144) {
    for (int it = 0; it < n / 3; ++it) {
      const int v1 = s0 / 3 + it;
      int a0, a1;
      pair2(v1, d[5], d[6], a0, a1);
      for (int m = 0; m < 3; ++m)
        for (int which = 0; which < 4; ++which) {
          for (int h = 0; h < 4; ++h) {
            int b0, b1;
            pair2(4 * m + h, d[11], d[12], b0, b1);
            for (int x = 0; x < 4; ++x)
              A[4 * h + x] = which < 2 ? SA + row(x, wa) + h * d[4] + (which ? a1 : a0) + 4 * m * d[4]
                                       : SB + row(x, wb) + v1 * d[10] + (which == 2 ? b0 : b1);
          }
          out.push_back(A);
        }
    }
  } else if (shape == kSegC36) {
    for (int it = 0; it < n / 3; ++it) {
      const int v2 = s0 / 3 + it;
      const int c1 = (v2 + 1) % 3, c2 = (v2 + 2) % 3;
      const int o0 = c1 * d[11] + c2 * d[12], o1 = c2 * d[11] + c1 * d[12];
      for (int m = 0; m < 3; ++m)
        for (int which = 0; which < 12; ++which) {
          for (int h = 0; h < 4; ++h) {
            int p0, p1;
            pair2(4 * m + h, d[5], d[6], p0, p1);
            for (int x = 0; x < 4; ++x) {
              int a;
              if (which < 4) {
                const int bA = (which < 2 ? row(x, wa) : row(x + 4, wa)) + v2 * d[4];
                a = SA + bA + ((which & 1) ? p1 : p0);
              } else if (x >= 2) {
                a = -1;
              } else {
                const int sp = (which - 4) / 2;
                const int so = 3 * sp * d[11] + 3 * (sp ^ 1) * d[12];
                a = SB + row(x & 1, wb) + h * d[10] + 4 * m * d[10] + so + (((which - 4) & 1) ? o1 : o0);
              }
              A[4 * h + x] = a;
            }
          }
          out.push_back(A);
        }
    }
  }
}

// Extra LDS cycles of the teams' reads when they share a task: 64 banks of
// four bytes; FP64 entries (16 bytes) are served 16 lanes per cycle, one
// slot h of all four teams (lane 16 h + 4 tm + x); FP32 entries (8 bytes)
// 32 lanes per cycle, two whole teams (lane 16 tm + 4 h + x).  A cycle
// serves distinct entries in distinct bank sets; equal entries broadcast.
long long seg_conflicts(const std::vector<const std::vector<std::array<int, 16>>*>& teams, bool fp32) {
  long long extra = 0;
  if (teams.empty()) return 0;
  const size_t n = teams[0]->size();
  const int mod = fp32 ? 32 : 16;
  int cnt[32];
  int seen[64];
  auto cycle = [&](const int* addrs, int na) {
    for (int b = 0; b < mod; ++b) cnt[b] = 0;
    int ns = 0, mx = 0;
    for (int i = 0; i < na; ++i) {
      const int a = addrs[i];
      if (a < 0) continue;
      bool dup = false;
      for (int j = 0; j < ns && !dup; ++j) dup = seen[j] == a;
      if (dup) continue;
      seen[ns++] = a;
      mx = std::max(mx, ++cnt[a % mod]);
    }
    return mx > 1 ? mx - 1 : 0;
  };
  int buf[64];
  for (size_t i = 0; i < n; ++i) {
    if (!fp32) {
      for (int h = 0; h < 4; ++h) {
        int na = 0;
        for (const auto* t : teams)
          for (int x = 0; x < 4; ++x) buf[na++] = (*t)[i][4 * h + x];
        extra += cycle(buf, na);
      }
    } else {
      for (size_t g = 0; g < teams.size(); g += 2) {
        int na = 0;
        for (size_t k = g; k < std::min(teams.size(), g + 2); ++k)
          for (int e = 0; e < 16; ++e) buf[na++] = (*teams[k])[i][e];
        extra += cycle(buf, na);
      }
    }
  }
  return extra;
}

// Order the segments of one (shape, step count) so that consecutive fours
// (the tasks) read LDS with few bank conflicts: greedily, each task (FP64)
// or each pair of teams sharing a cycle (FP32) takes the segment that adds
// the fewest extra cycles.
void pack_segments(std::vector<std::vector<int>>& segs, bool fp32) {
  const int shape = segs.empty() ? -1 : segs[0][0];
  if (segs.size() <= 1 || (shape != kSegC144 && shape != kSegC36)) return;
  std::vector<std::vector<std::array<int, 16>>> addrs(segs.size());
  for (size_t i = 0; i < segs.size(); ++i) seg_read_addrs(segs[i], addrs[i]);
  const size_t unit = fp32 ? 2 : kSegTeams;
  std::vector<int> rem(segs.size());
  for (size_t i = 0; i < rem.size(); ++i) rem[i] = (int)i;
  std::vector<int> order;
  while (!rem.empty()) {
    std::vector<int> grp = {rem.front()};
    rem.erase(rem.begin());
    while (grp.size() < unit && !rem.empty()) {
      long long best = -1;
      size_t bi = 0;
      for (size_t j = 0; j < rem.size(); ++j) {
        std::vector<const std::vector<std::array<int, 16>>*> t;
        for (int k : grp) t.push_back(&addrs[k]);
        t.push_back(&addrs[rem[j]]);
        const long long c = seg_conflicts(t, fp32);
        if (best < 0 || c < best) {
          best = c;
          bi = j;
        }
      }
      grp.push_back(rem[bi]);
      rem.erase(rem.begin() + bi);
    }
    order.insert(order.end(), grp.begin(), grp.end());
  }
  std::vector<std::vector<int>> out;
  for (int i : order) out.push_back(segs[i]);
  segs = out;
}

struct SegPlan {
  std::vector<std::vector<int>> tasks;  // per task kSegTeams * kSegInts ints
  std::vector<int> ext;                 // per product
  int slots = 0;
  double makespan = 0.0;
};

// Cut the products into segments (lengths l144 and l36 steps; a multiple
// of three steps, where the 4 x 4 shape's lanes start a new v1), put
// segments of one shape and one step count four to a task, and balance the
// tasks over `waves` wavefronts longest first.
SegPlan plan_segments(const std::vector<std::vector<int>>& base, const std::vector<int>& steps, int l144, int l36,
                      int waves, bool fp32, bool pack) {
  SegPlan sp;
  const int np = (int)base.size();
  sp.ext.assign(np, 0);
  int next_slot = np;
  std::map<std::pair<int, int>, std::vector<std::vector<int>>> by_key;  // (shape, steps) -> descriptors
  for (int p = 0; p < np; ++p) {
    const int shape = base[p][0];
    const int L = shape == kSegC144 ? l144 : shape == kSegC36 ? l36 : steps[p];
    int n_extra = 0;
    for (int s0 = 0; s0 < steps[p]; s0 += L) {
      std::vector<int> d = base[p];
      const int n = std::min(L, steps[p] - s0);
      const int slot = s0 == 0 ? p : next_slot + n_extra++;
      d[1] = s0;
      d[2] = n;
      d[3] = (d[3] & ~0xffff) | slot;
      by_key[{shape, n}].push_back(d);
    }
    if (n_extra) sp.ext[p] = next_slot | (n_extra << 16);
    next_slot += n_extra;
  }
  sp.slots = next_slot;
  std::vector<double> cost;
  for (auto& kv : by_key) {
    auto& segs = kv.second;
    if (pack) pack_segments(segs, fp32);
    for (size_t i = 0; i < segs.size(); i += kSegTeams) {
      std::vector<int> t(kSegTeams * kSegInts, 0);
      for (int k = 0; k < kSegTeams; ++k) {
        int* d = t.data() + k * kSegInts;
        if (i + k < segs.size()) {
          std::copy(segs[i + k].begin(), segs[i + k].end(), d);
        } else {
          d[0] = kSegIdle;
          d[2] = kv.first.second;
        }
      }
      sp.tasks.push_back(t);
      cost.push_back(kv.first.second * seg_step_cost(kv.first.first) + kSegOverhead);
    }
  }
  std::vector<int> ord(sp.tasks.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<double> load(std::max(1, waves), 0.0);
  for (int i : ord) *std::min_element(load.begin(), load.end()) += cost[i];
  sp.makespan = *std::max_element(load.begin(), load.end());
  std::vector<std::vector<int>> sorted;
  for (int i : ord) sorted.push_back(sp.tasks[i]);
  sp.tasks = sorted;
  return sp;
}

// Lane layout of one block product inside a task (see the lane word).
struct TeamUnit {
  int p;        // product (local index)
  int cls;      // product class
  int ky;       // lanes carrying the fixed index (16 term lanes for K = 1)
  int kypad;    // ky rounded up to 4 or 16
  int kz;       // values of the walked index
  int zsl;      // the walked index is split over 2^zsl lane sets
  int quad;     // lanes per walker: 4 for matrix-core classes, else 1
  double cell;  // estimated cost of one step of one lane
};

int team_lg(const TeamUnit& u) {
  int lg = 0;
  while ((1 << lg) < (u.quad * u.kypad << u.zsl)) ++lg;
  return lg;
}

// Order in which a contraction workgroup walks the sink-operator pairs
// (operator slots at +q and -q).  A step that keeps one of the two blocks
// loads one block instead of two, so the walk moves between pairs that share
// a slot on the same side, choosing the candidate with the fewest unvisited
// neighbours (so that few pairs are left stranded), and jumps only when no
// such pair is left.  Every start is tried; the walk with the fewest block
// loads (ties: the earlier start) is returned as indices into pairs.
std::vector<int> walk_order(const std::vector<std::pair<int, int>>& pairs) {
  const int n = (int)pairs.size();
  auto shares = [&](int i, int j) { return pairs[i].first == pairs[j].first || pairs[i].second == pairs[j].second; };
  std::vector<int> best;
  int best_loads = 0;
  for (int s = 0; s < n; ++s) {
    std::vector<char> used(n, 0);
    std::vector<int> walk{s};
    used[s] = 1;
    int loads = 2;
    for (int step = 1; step < n; ++step) {
      const int cur = walk.back();
      int pick = -1, pick_deg = 0;
      bool pick_shares = false;
      for (int j = 0; j < n; ++j) {
        if (used[j]) continue;
        int deg = 0;
        for (int k = 0; k < n; ++k)
          if (!used[k] && k != j && shares(j, k)) ++deg;
        const bool sh = shares(cur, j);
        if (pick < 0 || (sh && !pick_shares) || (sh == pick_shares && deg < pick_deg)) {
          pick = j;
          pick_deg = deg;
          pick_shares = sh;
        }
      }
      loads += (pairs[pick].first != pairs[cur].first) + (pairs[pick].second != pairs[cur].second);
      used[pick] = 1;
      walk.push_back(pick);
    }
    if (best.empty() || loads < best_loads) {
      best = walk;
      best_loads = loads;
    }
  }
  return best;
}

// Packs the products into 64-lane tasks (teams of one size and one class per
// task) and, if lanes is given, emits them longest first.  Returns the
// estimated time of the busiest wavefront when W wavefronts take the tasks
// in that order, each the next one when it is free (longest processing time
// first).
double pack_tasks(const std::vector<TeamUnit>& units, int waves, std::vector<int>* lanes) {
  constexpr double kShuffleStep = 32.0;  // one team-reduction step, same units as cell
  std::vector<int> ord(units.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
  auto steps = [](const TeamUnit& u) { return (u.kz + (1 << u.zsl) - 1) >> u.zsl; };
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    const int la = team_lg(units[a]), lb = team_lg(units[b]);
    if (la != lb) return la > lb;
    if (units[a].cls != units[b].cls) return units[a].cls < units[b].cls;
    return steps(units[a]) * units[a].cell > steps(units[b]) * units[b].cell;
  });
  std::vector<std::vector<int>> tasks;
  std::vector<double> tcost;
  int cur_key = -1;
  for (int i : ord) {
    const TeamUnit& u = units[i];
    const int lg = team_lg(u);
    const int key = lg * 64 + u.cls;
    const int idle = 0xfff | (lg << 16) | (u.cls << 26);
    if (key != cur_key || tasks.back().size() == (size_t)kLanesPerTask) {
      if (!tasks.empty())
        while (tasks.back().size() < (size_t)kLanesPerTask) tasks.back().push_back(tasks.back().back() | 0xfff);
      tasks.emplace_back();
      tcost.push_back(0.0);
      cur_key = key;
    }
    for (int zs = 0; zs < (1 << u.zsl); ++zs)
      for (int y = 0; y < u.kypad; ++y) {
        const bool busy = y < u.ky && zs < u.kz;
        for (int r = 0; r < u.quad; ++r)
          tasks.back().push_back(busy ? (u.p | (y << 12) | (lg << 16) | (zs << 19) | (u.zsl << 23) | (u.cls << 26))
                                      : idle);
      }
    tcost.back() = std::max(tcost.back(), steps(u) * u.cell + lg * kShuffleStep);
  }
  if (!tasks.empty())
    while (tasks.back().size() < (size_t)kLanesPerTask) tasks.back().push_back(tasks.back().back() | 0xfff);
  std::vector<int> by_cost(tasks.size());
  for (size_t i = 0; i < tasks.size(); ++i) by_cost[i] = (int)i;
  std::stable_sort(by_cost.begin(), by_cost.end(), [&](int a, int b) { return tcost[a] > tcost[b]; });
  std::vector<std::vector<int>> bins(waves);
  std::vector<double> load(waves, 0.0);
  for (int ti : by_cost) {
    const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    bins[w].push_back(ti);
    load[w] += tcost[ti];
  }
  if (lanes) {
    // longest first: the kernel's wavefronts claim tasks in this order from
    // a workgroup counter (greedy list scheduling)
    for (int ti : by_cost) lanes->insert(lanes->end(), tasks[ti].begin(), tasks[ti].end());
  }
  return *std::max_element(load.begin(), load.end());
}

}  // namespace

std::string compile_channels(const std::vector<ChannelSpec>& chans, const CompileOptions& opt,
                             Compiled* out) {
  Compiled C;
  C.channels = chans;
  const int n_ch = (int)chans.size();
  if (n_ch <= 0) return "no channels";
  Program& P = C.prog;

  // ---- 1. operator blocks the sink side needs ------------------------------
  std::map<int, int> op_slot;
  for (int c = 0; c < n_ch; ++c)
    for (int k = 0; k < 4; ++k) {
      const int code = k < 2 ? chans[c].sink[k] : chans[c].src[k - 2];
      if (code < 0 || code > 10) return "channel " + std::to_string(c) + ": bad operator code";
    }
  for (int c = 0; c < n_ch; ++c)
    for (int k = 0; k < 2; ++k)
      if (!op_slot.count(chans[c].sink[k])) op_slot[chans[c].sink[k]] = 0;
  for (auto& kv : op_slot) {
    kv.second = (int)P.op_code.size();
    P.op_code.push_back(kv.first);
    {
      int s1 = 0, s2 = 0;
      P.op_pair.push_back(operator_pair(kv.first, &s1, &s2) ? (s1 | (s2 << 2)) : -1);
    }
    const OpExpansion e = expand_operator(kv.first);
    int sl[3];
    operator_slots(kv.first, sl);
    P.op_nterm.push_back((int)e.trip.size());
    for (int k = 0; k < 3; ++k) {
      if (k >= (int)e.trip.size()) {
        P.op_term_trip.push_back(0); P.op_term_perm.push_back(0); P.op_term_w.push_back(0.0);
        continue;
      }
      // pi(i): the operator slot holding the flavour of triplet slot i
      int pi[3], used = 0;
      for (int i = 0; i < 3; ++i) {
        pi[i] = -1;
        for (int s = 0; s < 3; ++s)
          if (!((used >> s) & 1) && sl[s] == e.trip[k].f[i]) { pi[i] = s; used |= 1 << s; break; }
        if (pi[i] < 0) return "operator slot mismatch";
      }
      P.op_term_trip.push_back(e.trip[k].code());
      P.op_term_perm.push_back(pi[0] | (pi[1] << 2) | (pi[2] << 4));
      P.op_term_w.push_back(e.norm * e.wnum[k] * seq_sign(pi, 3));
    }
  }
  P.n_ops = (int)P.op_code.size();

  // ---- 1b. the isospin-symmetric limit: with S_d = S_u a block depends on
  // its recipe with d read as u; slots whose recipes agree up to a common
  // factor and that are stored antisymmetrised in the same slot pair are one
  // block (Sigma- = Sigma+, Xi- = -Xi0; n equals -p as a plain block, but
  // the two are antisymmetrised in different slot pairs, so n keeps its own
  // block).  Canonical slots are moved to the front.
  {
    const int n = P.n_ops;
    std::vector<int> alias(n);
    std::vector<double> coef(n, 1.0);
    auto key = [&](int s, int k) {
      const int code = P.op_term_trip[3 * s + k];
      int f[3] = {code / 9, (code / 3) % 3, code % 3};
      for (int& x : f) x = x == 1 ? 0 : x;
      return std::make_pair((f[0] * 3 + f[1]) * 3 + f[2], P.op_term_perm[3 * s + k]);
    };
    for (int s = 0; s < n; ++s) {
      alias[s] = s;
      for (int s0 = 0; s0 < s; ++s0) {
        // blocks are stored antisymmetrised in their same-flavour slot pair:
        // two slots are one block only if that pair is the same (n = -p as
        // plain blocks, but their stored forms differ in the pair)
        if (alias[s0] != s0 || P.op_nterm[s0] != P.op_nterm[s] || P.op_pair[s0] != P.op_pair[s]) continue;
        bool same = true;
        double c = 0.0;
        for (int k = 0; k < P.op_nterm[s] && same; ++k) {
          if (key(s, k) != key(s0, k)) same = false;
          const double r = P.op_term_w[3 * s + k] / P.op_term_w[3 * s0 + k];
          if (k == 0) c = r;
          else if (std::fabs(r - c) > 1e-12 * std::fabs(c)) same = false;
        }
        if (same) {
          alias[s] = s0;
          coef[s] = c;
          break;
        }
      }
    }
    // canonical slots first (stable), aliased after
    std::vector<int> order;
    for (int s = 0; s < n; ++s)
      if (alias[s] == s) order.push_back(s);
    P.n_canon = (int)order.size();
    for (int s = 0; s < n; ++s)
      if (alias[s] != s) order.push_back(s);
    std::vector<int> newpos(n);
    for (int i = 0; i < n; ++i) newpos[order[i]] = i;
    Program Q = P;
    for (int i = 0; i < n; ++i) {
      const int s = order[i];
      Q.op_code[i] = P.op_code[s];
      Q.op_nterm[i] = P.op_nterm[s];
      Q.op_pair[i] = P.op_pair[s];
      for (int k = 0; k < 3; ++k) {
        Q.op_term_trip[3 * i + k] = P.op_term_trip[3 * s + k];
        Q.op_term_perm[3 * i + k] = P.op_term_perm[3 * s + k];
        Q.op_term_w[3 * i + k] = P.op_term_w[3 * s + k];
      }
    }
    Q.op_alias.assign(n, 0);
    Q.op_alias_coef.assign(n, 1.0);
    for (int s = 0; s < n; ++s) {
      Q.op_alias[newpos[s]] = newpos[alias[s]];
      Q.op_alias_coef[newpos[s]] = coef[s];
    }
    P = Q;
    for (auto& kv : op_slot) kv.second = newpos[kv.second];
  }

  // ---- 2. diagrams and products per sink-operator group --------------------
  std::map<std::pair<int, int>, std::vector<int>> by_sink;
  std::vector<std::pair<int, int>> order;
  for (int c = 0; c < n_ch; ++c) {
    auto k = std::make_pair(chans[c].sink[0], chans[c].sink[1]);
    if (!by_sink.count(k)) order.push_back(k);
    by_sink[k].push_back(c);
  }
  C.channel_flavour.assign(3 * n_ch, 0);

  P.group_prod.push_back(0);
  P.group_task.push_back(0);
  P.group_stask.push_back(0);
  std::string seg_error;
  P.group_ch.push_back(0);
  P.ch_contrib.push_back(0);
  std::set<Block> all_blocks[2];

  {
    std::vector<std::pair<int, int>> slots;
    for (const auto& k : order) slots.emplace_back(op_slot[k.first], op_slot[k.second]);
    const std::vector<int> w = walk_order(slots);
    std::vector<std::pair<int, int>> walked;
    for (int i : w) walked.push_back(order[i]);
    order = walked;
  }
  for (auto& sk : order) {
    const std::vector<int>& chs = by_sink[sk];
    // a group is flushed when its product list would exceed the LDS result buffer
    std::map<std::pair<Block, Block>, int> prod_id;
    std::vector<std::pair<Block, Block>> prods;
    std::vector<std::map<int, double>> pcoef;  // product -> channel -> coef
    auto flush = [&](const std::vector<int>& gch) {
      // products, sorted into team-size classes and packed into 64-lane tasks
      const int gbase_prod = (int)(P.prod_desc.size() / kProdInts);
      std::vector<int> order_p(prods.size());
      for (size_t i = 0; i < prods.size(); ++i) order_p[i] = (int)i;
      // Lane layout of a product (the contraction kernel's rules): K = 1 -> one
      // lane; otherwise one lane per value y of the shared index on the side
      // where block 1 holds a quark pair (Ky = 3 or 12 lanes in a team of 4 or
      // 16), each walking the Kz values of the other side.
      auto ky_of = [&](int p) {
        const Shape s1 = shape_of(prods[p].first.mask);
        return s1.K() == 1 ? 16 : (s1.kA == 2 ? s1.KA : s1.KB);  // K = 1: 16 lanes share the 24 terms
      };
      auto team = [&](int p) {
        const int ky = ky_of(p);
        return ky <= 4 ? 4 : 16;
      };
      auto kz_of = [&](int p) {
        const int K = shape_of(prods[p].first.mask).K();
        return K == 1 ? 1 : K / ky_of(p);
      };
      auto cls_of = [&](int p) {
        const Shape s1 = shape_of(prods[p].first.mask), s2 = shape_of(prods[p].second.mask);
        // lone quarks as local indices (0..2) within their source baryon
        const bool pairA = s1.kA == 2;
        const int lone1 = pairA ? s1.loneA : s1.loneB - 3, lone2 = pairA ? s2.loneB - 3 : s2.loneA;
        const int c = product_class(s1.K(), s1.rows(), lone1, lone2, (int)prods[p].first.maps.size(),
                                    (int)prods[p].second.maps.size());
        if (opt.mfma && c >= 4 && c < 8) return kClassMfmaBegin + (c - 4);
        if (opt.mfma && c >= 16 && c < 20) return kClassMfmaBegin + 4 + (c - 16);
        return c;
      };
      std::stable_sort(order_p.begin(), order_p.end(), [&](int a, int b) {
        const int ta = team(a), tb = team(b);
        if (ta != tb) return ta > tb;
        if (cls_of(a) != cls_of(b)) return cls_of(a) < cls_of(b);
        if (kz_of(a) != kz_of(b)) return kz_of(a) > kz_of(b);
        return std::make_tuple(prods[a].first.mask, prods[a].first.maps.size(), prods[a].second.maps.size()) <
               std::make_tuple(prods[b].first.mask, prods[b].first.maps.size(), prods[b].second.maps.size());
      });
      std::vector<int> local(prods.size());
      for (size_t i = 0; i < order_p.size(); ++i) local[order_p[i]] = (int)i;
      for (int p : order_p) {
        const Shape s1 = shape_of(prods[p].first.mask);
        int d[kProdInts] = {0};
        d[0] = prods[p].first.mask;
        d[1] = (int)prods[p].first.maps.size();
        for (size_t i = 0; i < prods[p].first.maps.size(); ++i) d[2 + i] = prods[p].first.maps[i].packed();
        d[8] = prods[p].second.mask;
        d[9] = (int)prods[p].second.maps.size();
        for (size_t i = 0; i < prods[p].second.maps.size(); ++i) d[10 + i] = prods[p].second.maps[i].packed();
        d[16] = s1.K();
        d[17] = s1.KB;
        d[18] = s1.rows();
        d[19] = (s1.lbl3 ? 1 : 0) | (s1.lbl4 ? 2 : 0);
        if (s1.K() > 1) fill_split_offsets(prods[p].first, prods[p].second, d);
        P.prod_desc.insert(P.prod_desc.end(), d, d + kProdInts);
        C.product_k += s1.K();
      }
      // matrix-core program: segments of each product, packed into tasks
      {
        std::vector<std::vector<int>> base;
        std::vector<int> nsteps;
        bool ok = true;
        for (int p : order_p) {
          std::vector<int> d(kSegInts, 0);
          int shape = 0, st = 0;
          if (!segment_fields(prods[p].first, prods[p].second, &shape, &st, 0, d.data())) ok = false;
          base.push_back(d);
          nsteps.push_back(st);
        }
        if (!ok) seg_error = "a block product has no matrix-core shape";
        SegPlan best;
        bool have = false;
        int bl144 = 0, bl36 = 0;
        for (int l144 : {36, 18, 12, 9, 6, 3})
          for (int l36 : {9, 6, 3}) {
            SegPlan sp = plan_segments(base, nsteps, l144, l36, opt.seg_waves, opt.fp32, false);
            if (sp.slots > opt.max_group_slots) continue;
            if (!have || sp.makespan < best.makespan - 1e-9 ||
                (std::fabs(sp.makespan - best.makespan) <= 1e-9 && sp.slots < best.slots)) {
              best = sp;
              bl144 = l144;
              bl36 = l36;
              have = true;
            }
          }
        if (!have) seg_error = "a channel group needs more result slots than the contraction holds";
        // the chosen cut, its tasks composed against LDS bank conflicts
        // (the same segments, slots and balance)
        else best = plan_segments(base, nsteps, bl144, bl36, opt.seg_waves, opt.fp32, true);
        for (const auto& t : best.tasks) P.seg_task.insert(P.seg_task.end(), t.begin(), t.end());
        P.prod_ext.insert(P.prod_ext.end(), best.ext.begin(), best.ext.end());
        P.group_stask.push_back((int)(P.seg_task.size() / (kSegTeams * kSegInts)));
        P.max_group_slots = std::max(P.max_group_slots, best.slots);
        P.max_group_stasks = std::max(P.max_group_stasks, (int)best.tasks.size());
      }
      // lanes: one team per product; the walked index may be split over
      // 2^zsl lane sets (a larger team, fewer steps per lane).  The split is
      // chosen per group by trying targets for the steps per lane and keeping
      // the one with the smallest estimated workgroup time.
      std::vector<TeamUnit> units;
      for (int p : order_p) {
        const Shape s1 = shape_of(prods[p].first.mask), s2 = shape_of(prods[p].second.mask);
        TeamUnit u{};
        u.p = local[p];
        u.cls = cls_of(p);
        u.ky = ky_of(p);
        u.kypad = team(p);
        u.kz = kz_of(p);
        u.zsl = 0;
        u.quad = class_is_mfma(u.cls) ? 4 : 1;
        const int nm1 = (int)prods[p].first.maps.size(), nm2 = (int)prods[p].second.maps.size();
        if (s1.K() == 1) {
          u.cell = 8.0 * (nm1 + nm2) + 64.0 + 32.0;
        } else {
          const int lone1 = s1.kA == 2 ? s1.loneA : s1.loneB - 3, lone2 = s1.kA == 2 ? s2.loneB - 3 : s2.loneA;
          const int np1 = lone1 == 2 ? 8 : 2, np2 = lone2 == 2 ? 8 : 2;
          u.cell = u.quad == 4 ? (double)np1 * nm1 + np2 * nm2 + 8.0
                               : (double)s1.rows() * np1 * nm1 + (double)(16 / s1.rows()) * np2 * nm2 + 32.0;
        }
        units.push_back(u);
      }
      std::vector<TeamUnit> best = units;
      double best_t = pack_tasks(units, opt.waves, nullptr);
      for (int target : {6, 4, 3, 2, 1}) {
        if (!opt.split) break;
        std::vector<TeamUnit> trial = units;
        for (auto& u : trial) {
          if (u.cls < kClassFullEnd) continue;
          while ((u.kz + (1 << u.zsl) - 1) >> u.zsl > target && (u.quad * u.kypad << (u.zsl + 1)) <= kLanesPerTask)
            ++u.zsl;
        }
        const double t = pack_tasks(trial, opt.waves, nullptr);
        if (t < best_t) {
          best_t = t;
          best = trial;
        }
      }
      std::vector<int> lanes;
      pack_tasks(best, opt.waves, &lanes);
      P.task_lanes.insert(P.task_lanes.end(), lanes.begin(), lanes.end());
      // channel contributions
      for (int c : gch) {
        P.group_channels.push_back(c);
        for (size_t p = 0; p < prods.size(); ++p) {
          auto it = pcoef[p].find(c);
          if (it == pcoef[p].end() || it->second == 0.0) continue;
          const Shape s1 = shape_of(prods[p].first.mask);
          const int lbl = (s1.lbl3 ? 1 : 0) | (s1.lbl4 ? 2 : 0);
          P.contrib_prod.push_back(local[p] | (s1.rows() << 16) | (lbl << 20));
          P.contrib_coef.push_back(it->second);
          const size_t pe = (size_t)P.group_prod.back() + (size_t)local[p];
          P.contrib_ext.push_back(pe < P.prod_ext.size() ? P.prod_ext[pe] : 0);
        }
        P.ch_contrib.push_back((int)P.contrib_prod.size());
      }
      P.group_op1.push_back(op_slot[sk.first]);
      P.group_op2.push_back(op_slot[sk.second]);
      {
        const int s1 = op_slot[sk.first], s2 = op_slot[sk.second];
        P.group_op1_iso.push_back(P.op_alias[s1]);
        P.group_op2_iso.push_back(P.op_alias[s2]);
        const double f = P.op_alias_coef[s1] * P.op_alias_coef[s2];
        for (size_t c = P.contrib_coef_iso.size(); c < P.contrib_coef.size(); ++c)
          P.contrib_coef_iso.push_back(P.contrib_coef[c] * f);
      }
      P.group_prod.push_back((int)(P.prod_desc.size() / kProdInts));
      P.group_task.push_back((int)(P.task_lanes.size() / kLanesPerTask));
      P.group_ch.push_back((int)P.group_channels.size());
      P.max_group_products = std::max(P.max_group_products, (int)prods.size());
      P.max_group_contrib = std::max(P.max_group_contrib, P.ch_contrib.back() - P.ch_contrib[P.group_ch[P.group_ch.size() - 2]]);
      P.max_group_channels = std::max(P.max_group_channels, (int)gch.size());
      P.max_group_tasks = std::max(P.max_group_tasks, P.group_task.back() - P.group_task[P.group_task.size() - 2]);
      (void)gbase_prod;
      prod_id.clear();
      prods.clear();
      pcoef.clear();
    };

    std::vector<int> gch;
    for (int c : chs) {
      OpExpansion op[4];
      for (int k = 0; k < 4; ++k) op[k] = expand_operator(k < 2 ? chans[c].sink[k] : chans[c].src[k - 2]);
      int nf[2][3] = {{0, 0, 0}, {0, 0, 0}};
      for (int side = 0; side < 2; ++side)
        for (int k = 0; k < 2; ++k)
          for (int f = 0; f < 3; ++f) nf[side][f] += flavour_count(op[2 * side + k].trip[0], f);
      for (int f = 0; f < 3; ++f)
        if (nf[0][f] != nf[1][f]) return "channel " + std::to_string(c) + ": flavour not conserved";
      for (int f = 0; f < 3; ++f) C.channel_flavour[3 * c + f] = nf[0][f];

      // products this channel needs
      std::vector<std::tuple<Block, Block, double>> mine;
      int src_term = 0;
      for (size_t t3 = 0; t3 < op[2].trip.size(); ++t3)
        for (size_t t4 = 0; t4 < op[3].trip.size(); ++t4, ++src_term) {
          int srcfl[6];
          for (int i = 0; i < 3; ++i) {
            srcfl[i] = op[2].trip[t3].f[i];
            srcfl[3 + i] = op[3].trip[t4].f[i];
          }
          const double wsrc = op[2].norm * op[3].norm * op[2].wnum[t3] * op[3].wnum[t4];
          for (int mask = 0; mask < 64; ++mask) {
            if (popcount(mask) != 3) continue;
            const int mask2 = 0x3f & ~mask;
            const std::vector<Map> full1 = effective_block(chans[c].sink[0], mask, srcfl);
            const std::vector<Map> full2 = effective_block(chans[c].sink[1], mask2, srcfl);
            if (full1.empty() || full2.empty()) continue;
            Block b1{mask, on_stored_block(chans[c].sink[0], full1)};
            Block b2{mask2, on_stored_block(chans[c].sink[1], full2)};
            int cross = 0;
            for (int x = 0; x < 6; ++x)
              for (int y = 0; y < 6; ++y)
                if (((mask >> x) & 1) && ((mask2 >> y) & 1) && x > y) ++cross;
            const double coef = wsrc * ((cross & 1) ? -1.0 : 1.0);
            mine.emplace_back(b1, b2, coef);
            all_blocks[0].insert(b1);
            all_blocks[1].insert(b2);
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
            C.diagrams.push_back(d);
            C.sum_k += sh.K();
            // Wick permutations covered, counted on the flavour triplets of the operators
            // every flavour triplet of an operator has the block's slot flavours, so
            // each (triplet, triplet) pair covers maps1 x maps2 permutations
            C.n_wick += (int64_t)op[0].trip.size() * op[1].trip.size() * full1.size() * full2.size();
          }
        }
      // new products this channel would add to the current group
      int new_p = 0;
      for (auto& m : mine)
        if (!prod_id.count({std::get<0>(m), std::get<1>(m)})) ++new_p;
      if (!prods.empty() && (int)prods.size() + new_p > opt.max_group_products) {
        flush(gch);
        gch.clear();
      }
      if ((int)mine.size() > opt.max_group_products && prods.empty() && new_p > opt.max_group_products)
        return "channel " + std::to_string(c) + " needs more products than one group holds";
      gch.push_back(c);
      for (auto& m : mine) {
        auto key = std::make_pair(std::get<0>(m), std::get<1>(m));
        auto it = prod_id.find(key);
        int pid;
        if (it == prod_id.end()) {
          pid = (int)prods.size();
          prod_id[key] = pid;
          prods.push_back(key);
          pcoef.emplace_back();
        } else {
          pid = it->second;
        }
        pcoef[pid][c] += std::get<2>(m);
      }
    }
    if (!gch.empty()) flush(gch);
  }

  if (!seg_error.empty()) return seg_error;

  // ---- 3. statistics ---------------------------------------------------------
  for (int side = 0; side < 2; ++side)
    for (const Block& b : all_blocks[side]) {
      const Shape s = shape_of(b.mask);
      const int nA = part_terms(s.kA, s.loneA < 0 ? -1 : s.loneA);
      const int nB = part_terms(s.kB, s.loneB < 0 ? -1 : s.loneB - 3);
      C.n_entries += (int64_t)s.rows() * s.K();
      C.n_terms += (int64_t)s.rows() * s.K() * (int64_t)b.maps.size() * nA * nB;
    }
  C.n_blocks = (int)(all_blocks[0].size() + all_blocks[1].size());
  C.n_products = (int)(P.prod_desc.size() / kProdInts);
  *out = std::move(C);
  return "";
}

std::vector<TwoPointTerm> two_point_terms(int sink_op, int src_op) {
  std::vector<TwoPointTerm> out;
  const OpExpansion src = expand_operator(src_op);
  for (size_t k = 0; k < src.trip.size(); ++k) {
    const int srcfl[6] = {src.trip[k].f[0], src.trip[k].f[1], src.trip[k].f[2], -1, -1, -1};
    for (const Map& mp : on_stored_block(sink_op, effective_block(sink_op, 0x7, srcfl))) {
      TwoPointTerm t;
      for (int i = 0; i < 3; ++i) t.m[i] = mp.m[i];
      t.coef = src.norm * src.wnum[k] * mp.sign;
      out.push_back(t);
    }
  }
  return out;
}

void operator_flavour_counts(int op, int nf[3]) {
  int fl[3];
  operator_slots(op, fl);
  nf[0] = nf[1] = nf[2] = 0;
  for (int i = 0; i < 3; ++i)
    if (fl[i] >= 0 && fl[i] < 3) ++nf[fl[i]];
}

}  // namespace nbs
