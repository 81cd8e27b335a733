"""CPU emulation of the compiled contraction program (test code only).

Executes the structure-of-arrays program exported by nbs_plan_table the way
the contraction kernel does: per group the two operator blocks, per 64-lane
task the lane words (product, first shared index, team size, count), the
effective-block entries generated from the source-tensor structure, the
team sums and the channel accumulation.  It lets the host test suite check
the channel compiler, the task packing and the entry generation rules
against the oracle without a GPU; it is never part of the product path.
"""
from __future__ import annotations

import numpy as np

NAMES = ("op_code", "op_nterm", "op_term_trip", "op_term_perm", "op_term_w", "op_pair", "group_op1", "group_op2",
         "group_prod", "group_task", "group_ch", "group_channels", "ch_contrib", "contrib_prod",
         "contrib_coef", "prod_desc", "task_lanes")
PROD_INTS = 48
MFMA_BEGIN, MFMA_END = 20, 28
IDLE_CLASS = 30

EPS = {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}
CG5 = {(0, 1): 1, (1, 0): -1, (2, 3): 1, (3, 2): -1}


def tables(plan):
    return {n: plan.table(n) for n in NAMES}


def operator_blocks(T, triplet_blocks):
    """Operator blocks N_op[V, 3456] from triplet blocks {code: [V, 2, 12, 12, 12]}."""
    out = []
    for s, _code in enumerate(T["op_code"]):
        acc = None
        for k in range(T["op_nterm"][s]):
            code = int(T["op_term_trip"][3 * s + k])
            pm = int(T["op_term_perm"][3 * s + k])
            pi = (pm & 3, (pm >> 2) & 3, (pm >> 4) & 3)
            sigma = [pi.index(o) for o in range(3)]  # op slot -> triplet slot
            blk = np.transpose(triplet_blocks[code], (0, 1, 2 + sigma[0], 2 + sigma[1], 2 + sigma[2]))
            term = T["op_term_w"][3 * s + k] * blk
            acc = term if acc is None else acc + term
        pair = int(T["op_pair"][s])
        if pair >= 0:
            # stored antisymmetrised in the same-flavour slot pair (s1, s2)
            s1, s2 = pair & 3, (pair >> 2) & 3
            acc = acc - np.swapaxes(acc, 2 + s1, 2 + s2)
        out.append(acc.reshape(acc.shape[0], 3456))
    return out


def _shape(mask):
    sh = {}
    for h, base in ((0, 0), (1, 3)):
        bits = (mask >> base) & 7
        n = bin(bits).count("1")
        lone = -1
        if n == 2:
            lone = [i for i in range(3) if not (bits >> i) & 1][0]
        elif n == 1:
            lone = [i for i in range(3) if (bits >> i) & 1][0]
        sh["in%d" % h], sh["lone%d" % h] = n, lone
    sh["l3"], sh["l4"] = bool((mask >> 2) & 1), bool((mask >> 5) & 1)
    return sh


def _part(n, lone, x, al):
    """(quark -> j, coef) terms of one source baryon's tensor inside a block."""
    out = []
    if n == 3:
        for (c0, c1, c2), e in EPS.items():
            for (s0, s1), g in CG5.items():
                out.append(({0: 3 * s0 + c0, 1: 3 * s1 + c1, 2: 3 * al + c2}, e * g))
    elif n == 2 and lone == 2:
        for (c0, c1, c2), e in EPS.items():
            if c2 != x:
                continue
            for (s0, s1), g in CG5.items():
                out.append(({0: 3 * s0 + c0, 1: 3 * s1 + c1}, e * g))
    elif n == 2:
        sa, ca = divmod(x, 3)
        b = 1 - lone
        for cs, e in EPS.items():
            if cs[lone] != ca:
                continue
            for sp, g in CG5.items():
                if sp[lone] != sa:
                    continue
                out.append(({b: 3 * sp[b] + cs[b], 2: 3 * al + cs[2]}, e * g))
    elif n == 1:
        out.append(({lone: 3 * al + x if lone == 2 else x}, 1))
    else:
        out.append(({}, 1))
    return out


def _entry(slot, mask, maps, r, xA, xB):
    sh = _shape(mask)
    n3, n4 = (2 if sh["l3"] else 1), (2 if sh["l4"] else 1)
    a4 = r % 2 if sh["l4"] else 0
    a3 = (r // n4) % 2 if sh["l3"] else 0
    al = r // (n3 * n4)
    v = 0j
    for ja, ca in _part(sh["in0"], sh["lone0"], xA, a3):
        for jb, cb in _part(sh["in1"], sh["lone1"], xB, a4):
            j = dict(ja)
            j.update({k + 3: vv for k, vv in jb.items()})
            for mp in maps:
                m = (mp & 7, (mp >> 3) & 7, (mp >> 6) & 7)
                sg = -1 if (mp >> 9) & 1 else 1
                v += sg * ca * cb * slot[al * 1728 + j[m[0]] * 144 + j[m[1]] * 12 + j[m[2]]]
    return v


def emulate_q(T, Nq_plus, Nq_minus, n_ch):
    """F~(q) [n_ch, 16] from operator blocks at +q (Nq_plus[slot]) and -q."""
    out = np.zeros((n_ch, 16), dtype=np.complex128)
    lanes = T["task_lanes"].reshape(-1, 64)
    desc = T["prod_desc"].reshape(-1, PROD_INTS)
    n_groups = len(T["group_prod"]) - 1
    for g in range(n_groups):
        slotA, slotB = Nq_plus[T["group_op1"][g]], Nq_minus[T["group_op2"][g]]
        pb, pe = T["group_prod"][g], T["group_prod"][g + 1]
        R = {}
        for task in range(T["group_task"][g], T["group_task"][g + 1]):
            words = lanes[task]
            lgs = {(int(w) >> 16) & 7 for w in words if int(w) & 0xFFF != 0xFFF}
            cls = {(int(w) >> 26) & 31 for w in words if int(w) & 0xFFF != 0xFFF}
            if ((int(words[0]) >> 26) & 31) == IDLE_CLASS:
                assert not lgs, "an idle task holds work"
                continue
            assert {(int(w) >> 16) & 7 for w in words} == lgs or not lgs, "idle lanes disagree on the team size"
            if not lgs:
                continue
            assert len(lgs) == 1, "a task mixes team sizes"
            assert len(cls) == 1, "a task mixes product classes"
            tl = 1 << lgs.pop()
            cls_t = cls.pop()
            for t0 in range(0, 64, tl):
                team = [int(w) for w in words[t0:t0 + tl]]
                ps = {w & 0xFFF for w in team} - {0xFFF}
                if not ps:
                    continue
                assert len(ps) == 1, "a team mixes products"
                p = ps.pop()
                assert p not in R, "product computed twice"
                d = desc[pb + p]
                K, KB, r1n = int(d[16]), int(d[17]), int(d[18])
                r2n = 16 // r1n
                m1 = [int(x) for x in d[2:2 + d[1]]]
                m2 = [int(x) for x in d[10:10 + d[9]]]
                pairA = _shape(int(d[0]))["in0"] == 2
                covered = []
                acc = np.zeros(16, dtype=np.complex128)
                if MFMA_BEGIN <= cls_t < MFMA_END:  # quads: four lanes walk one stream
                    assert tl >= 16 and all(team[i] == team[i - i % 4] for i in range(len(team)))
                    team = team[::4]
                if K == 1:  # the team shares one full-projection product
                    assert sorted(((w >> 12) & 15) for w in team if w & 0xFFF != 0xFFF) == list(range(16))
                    team = [w for w in team if (w >> 12) & 15 == 0]
                for w in team:
                    if w & 0xFFF == 0xFFF:
                        continue
                    y, z0, zs = (w >> 12) & 15, (w >> 19) & 15, 1 << ((w >> 23) & 7)
                    kz = 1 if K == 1 else (KB if pairA else K // KB)
                    for z in range(z0, kz, zs):
                        if K == 1:
                            xA = xB = 0
                        else:
                            xA, xB = (y, z) if pairA else (z, y)
                        covered.append(xA * KB + xB)
                        e1 = [_entry(slotA, int(d[0]), m1, r, xA, xB) for r in range(r1n)]
                        e2 = [_entry(slotB, int(d[8]), m2, r, xA, xB) for r in range(r2n)]
                        acc += np.outer(e1, e2).ravel()
                assert sorted(covered) == list(range(K)), "shared indices not covered exactly once"
                R[p] = acc
        assert sorted(R) == list(range(pe - pb))
        c0 = T["group_ch"][g]
        for cl in range(T["group_ch"][g + 1] - c0):
            ch = T["group_channels"][c0 + cl]
            for s in range(16):
                a1, a2, a3, a4 = (s >> 3) & 1, (s >> 2) & 1, (s >> 1) & 1, s & 1
                v = 0j
                for c in range(T["ch_contrib"][c0 + cl], T["ch_contrib"][c0 + cl + 1]):
                    w = int(T["contrib_prod"][c])
                    p = w & 0xFFFF
                    d = desc[pb + p]
                    assert (w >> 16) & 15 == d[18] and (w >> 20) & 3 == d[19]
                    l3, l4 = bool(d[19] & 1), bool(d[19] & 2)
                    rows2 = 16 // d[18]
                    r1 = (a1 * (2 if l3 else 1) + (a3 if l3 else 0)) * (2 if l4 else 1) + (a4 if l4 else 0)
                    r2 = (a2 * (1 if l3 else 2) + (0 if l3 else a3)) * (1 if l4 else 2) + (0 if l4 else a4)
                    v += T["contrib_coef"][c] * R[p][r1 * rows2 + r2]
                out[ch, s] = v
    return out


LDS_J0, LDS_J1 = 157, 13


def split_offsets(d):
    """Independent derivation of descriptor entries 20..47 of a product with
    a shared index (the per-map offsets in the kernel's LDS units)."""
    out = np.zeros(28, dtype=np.int64)
    m1 = [int(x) for x in d[2:2 + d[1]]]
    m2 = [int(x) for x in d[10:10 + d[9]]]
    sh1, sh2 = _shape(int(d[0])), _shape(int(d[8]))
    pair_a = sh1["in0"] == 2
    base1, base2 = (0, 3) if pair_a else (3, 0)
    lone1 = sh1["lone0"] if pair_a else sh1["lone1"]   # local index
    lone2 = sh2["lone1"] if pair_a else sh2["lone0"]
    others1 = [k for k in range(3) if k != lone1]
    others2 = [k for k in range(3) if k != lone2]
    p1, q1 = base1 + others1[0], base1 + others1[1]
    p2, q2 = base2 + others2[0], base2 + others2[1]
    ys, zs = base1 + lone1, base2 + lone2

    def unit(mp, q):
        slots = (mp & 7, (mp >> 3) & 7, (mp >> 6) & 7)
        return sum(w for s, w in zip(slots, (LDS_J0, LDS_J1, 1)) if s == q)

    def weights(sh, mp):
        w = []
        if sh["l4"]:
            w.append(3 * unit(mp, 5))
        if sh["l3"]:
            w.append(3 * unit(mp, 2))
        return (w + [0, 0])[:2]

    out[0], out[1] = lone1, lone2
    for m, mp in enumerate(m1):
        sg = -1 if (mp >> 9) & 1 else 1
        out[4 + 6 * m:10 + 6 * m] = [unit(mp, p1), unit(mp, q1), unit(mp, zs), *weights(sh1, mp), sg]
    for m, mp in enumerate(m2):
        sg = -1 if (mp >> 9) & 1 else 1
        out[16 + 6 * m:22 + 6 * m] = [unit(mp, ys), unit(mp, p2), unit(mp, q2), *weights(sh2, mp), sg]
    return out


# ---- the kernel's team reduction, simulated lane by lane --------------------
def _dpp_partner(ctrl, lane):
    r, i = lane & ~15, lane & 15
    if ctrl == "row_mirror":
        return r | (15 - i)
    if ctrl == "row_half_mirror":
        return r | (i & 8) | (7 - (i & 7))
    if ctrl == "quad_mirror":
        return (lane & ~3) | (3 - (lane & 3))
    if ctrl == "quad_swap":
        return lane ^ 1
    raise ValueError(ctrl)


STEPS = {2: ("quad_mirror", "quad_swap"), 3: ("row_half_mirror", "quad_mirror", "quad_swap"),
         4: ("row_mirror", "row_half_mirror", "quad_mirror", "quad_swap")}


def team_reduce(vals, lg):
    """vals: [64, 16] per-lane partial sums of a wavefront whose teams have
    2^lg lanes.  Returns {(lane, output index): value} as the kernel writes."""
    cur = {l: list(vals[l]) for l in range(64)}
    steps = STEPS[min(lg, 4)]
    for k, ctrl in zip(range(len(steps) - 1, -1, -1), steps):
        nxt = {}
        for l in range(64):
            upper = (l >> k) & 1
            n = len(cur[l]) // 2
            mine, part = cur[l], cur[_dpp_partner(ctrl, l)]
            keep = mine[n:] if upper else mine[:n]
            # the partner sends the half it does not keep, i.e. the half I keep
            recv = part[n:] if upper else part[:n]
            nxt[l] = [a + b for a, b in zip(keep, recv)]
        cur = nxt
    out = {}
    for l in range(64):
        if (l & ((1 << lg) - 1)) >= 16:
            continue
        v = cur[l]
        n = len(v)
        base = 0
        bits = min(lg, 4)
        for k in range(bits):
            base += ((l >> k) & 1) * (16 >> (bits - k))
        for j in range(n):
            out[(l, base + j)] = v[j]
    # cross-row sums of 32- and 64-lane teams
    if lg >= 5:
        res = {}
        for (l, o), v in out.items():
            tot = v
            for r in range(1, 1 << (lg - 4)):
                tot = tot + cur[l + 16 * r][0]
            res[(l, o)] = tot
        out = res
    return out



def quad_team_reduce(vals, lg):
    """Matrix-core classes: vals [64, 4] holds, per lane 4 q + j, R[i][j] for
    i = 0..3 of its quad.  Two DPP row shifts (by 4 and 8 lanes, zero fill)
    then cross-row adds; returns {(lane, i * 4 + j): value} as written."""
    cur = [list(v) for v in vals]
    for sh in (4, 8):
        nxt = []
        for l in range(64):
            src = l - sh
            same_row = src >= 0 and (src >> 4) == (l >> 4)
            nxt.append([a + (cur[src][k] if same_row else 0) for k, a in enumerate(cur[l])])
        cur = nxt
    for x in (16, 32):
        if (x == 16 and lg >= 5) or (x == 32 and lg >= 6):
            cur = [[a + b for a, b in zip(cur[l], cur[l ^ x])] for l in range(64)]
    out = {}
    for l in range(64):
        tl = l & ((1 << lg) - 1)
        if 12 <= tl < 16:
            for i in range(4):
                out[(l, i * 4 + (l & 3))] = cur[l][i]
    return out


# ---- the matrix-core contraction's segment program ---------------------------
SEG_NAMES = ("seg_task", "group_stask", "prod_ext", "contrib_ext")
SEG_INTS, SEG_TEAMS = 16, 4
SEG_C144, SEG_C9, SEG_C36, SEG_C1, SEG_IDLE = 0, 1, 2, 3, 15
LDS_AL, LDS_BLOCK = 1892, 2 * 1892


def lds_image(block):
    """A staged operator block in the kernel's LDS layout; padding is NaN so
    that a read outside the block's entries shows in the result."""
    out = np.full(LDS_BLOCK, np.nan + 0j, dtype=np.complex128)
    i = np.arange(3456)
    al, j0, j1, j2 = i // 1728, (i // 144) % 12, (i // 12) % 12, i % 12
    out[al * LDS_AL + j0 * LDS_J0 + j1 * LDS_J1 + j2] = block
    return out


def _seg_row(r, w):
    return (r & 1) * w[0] + ((r >> 1) & 1) * w[1] + ((r >> 2) & 1) * w[2]


def _pair2(v, up, uq):
    sp, c = divmod(v, 3)
    c1, c2 = (c + 1) % 3, (c + 2) % 3
    jp = 3 * (sp ^ 1)
    return (jp + c1) * up + c2 * uq, (jp + c2) * up + c1 * uq, (-1 if sp & 1 else 1)


def _entry2(S, base, o0, o1, g):
    return g * (S[base + o0] - S[base + o1])


def _entry8(S, base, up, uq, c):
    c1, c2 = (c + 1) % 3, (c + 2) % 3
    o0, o1 = c1 * up + c2 * uq, c2 * up + c1 * uq
    e = 0j
    for sp in range(4):
        so = 3 * sp * up + 3 * (sp ^ 1) * uq
        e += (-1 if sp & 1 else 1) * (S[base + so + o0] - S[base + so + o1])
    return e


def seg_run(d, S1, S2, shape, nsteps):
    """The 4 x 4 result D[i][j] of one team's segment (None for an idle team),
    computed lane by lane as the kernel does: lane (h, x) supplies row x of
    both sides at slot k' = 4 s + h, D = sum over steps and h of A B^T."""
    if d[0] == SEG_IDLE:
        return None
    s0, hdr = int(d[1]), int(d[3])
    transposed = (hdr >> 17) & 1
    SA, SB = (S2, S1) if transposed else (S1, S2)
    uAs, uAp, uAq, wa = int(d[4]), int(d[5]), int(d[6]), [int(v) for v in d[7:10]]
    uBs, uBp, uBq, wb = int(d[10]), int(d[11]), int(d[12]), [int(v) for v in d[13:16]]
    D = np.zeros((4, 4), dtype=np.complex128)
    D2 = np.zeros((4, 4), dtype=np.complex128)
    for s in range(s0, s0 + nsteps):
        A = np.zeros((4, 4), dtype=np.complex128)  # [row x][slot h]
        A2 = np.zeros((4, 4), dtype=np.complex128)  # rows x + 4 of the 8 x 2 shape
        B = np.zeros((4, 4), dtype=np.complex128)
        for h in range(4):
            for x in range(4):
                if shape == SEG_C144:
                    v1, v2 = s // 3, 4 * (s % 3) + h
                    o0, o1, g = _pair2(v1, uAp, uAq)
                    A[x, h] = _entry2(SA, _seg_row(x, wa) + v2 * uAs, o0, o1, g)
                    o0, o1, g = _pair2(v2, uBp, uBq)
                    B[x, h] = _entry2(SB, _seg_row(x, wb) + v1 * uBs, o0, o1, g)
                elif shape == SEG_C36:
                    v2, v1 = s // 3, 4 * (s % 3) + h
                    o0, o1, g = _pair2(v1, uAp, uAq)
                    A[x, h] = _entry2(SA, _seg_row(x, wa) + v2 * uAs, o0, o1, g)
                    A2[x, h] = _entry2(SA, _seg_row(x + 4, wa) + v2 * uAs, o0, o1, g)
                    if x < 2:
                        B[x, h] = _entry8(SB, _seg_row(x, wb) + v1 * uBs, uBp, uBq, v2)
                elif shape == SEG_C9:
                    kk = 4 * s + h
                    if kk < 9:
                        v1, v2 = divmod(kk, 3)
                        A[x, h] = _entry8(SA, _seg_row(x, wa) + v2 * uAs, uAp, uAq, v1)
                        B[x, h] = _entry8(SB, _seg_row(x, wb) + v1 * uBs, uBp, uBq, v2)
                else:
                    for side, (S, ro, u2, u0, u1) in enumerate(((SA, _seg_row(x, wa), uAs, uAp, uAq),
                                                                (SB, _seg_row(x, wb), uBs, uBp, uBq))):
                        b = ro + 3 * h * u0 + 3 * (h ^ 1) * u1
                        e = 0j
                        for cp in range(6):
                            c0 = cp if cp < 3 else cp - 3
                            c1 = (c0 + 1) % 3 if cp < 3 else (c0 + 2) % 3
                            c2 = (c0 + 2) % 3 if cp < 3 else (c0 + 1) % 3
                            e += (1 if cp < 3 else -1) * S[b + c0 * u0 + c1 * u1 + c2 * u2]
                        e *= -1 if h & 1 else 1
                        (A if side == 0 else B)[x, h] = e
        if shape == SEG_C1:  # summed over the four h lanes, fed on h = 0
            A = np.concatenate([A.sum(axis=1, keepdims=True), np.zeros((4, 3))], axis=1)
            B = np.concatenate([B.sum(axis=1, keepdims=True), np.zeros((4, 3))], axis=1)
        D += A @ B.T
        D2 += A2 @ B.T
    sgn = -1 if (hdr >> 16) & 1 else 1
    R = np.zeros(16, dtype=np.complex128)
    for i in range(4):
        for j in range(4):
            if shape == SEG_C36:
                if j >= 2:
                    assert D[i, j] == 0 and D2[i, j] == 0
                    continue
                for b, Db in ((0, D), (1, D2)):
                    ra = i + 4 * b
                    R[j * 8 + ra if transposed else ra * 2 + j] = sgn * Db[i, j]
            else:
                R[i * 4 + j] = sgn * D[i, j]
    return R


def emulate_q_seg(T, Nq_plus, Nq_minus, n_ch, check_slots=True):
    """F~(q) [n_ch, 16] from the segment program of the matrix-core
    contraction, following its kernel: segments into result slots, then
    channel sums in which each contribution adds its product's segment
    slots (contrib_ext)."""
    out = np.zeros((n_ch, 16), dtype=np.complex128)
    tasks = T["seg_task"].reshape(-1, SEG_TEAMS, SEG_INTS)
    n_groups = len(T["group_prod"]) - 1
    for g in range(n_groups):
        S1 = lds_image(Nq_plus[T["group_op1"][g]])
        S2 = lds_image(Nq_minus[T["group_op2"][g]])
        pb, pe = int(T["group_prod"][g]), int(T["group_prod"][g + 1])
        R = {}
        for task in tasks[T["group_stask"][g]:T["group_stask"][g + 1]]:
            shape, nsteps = int(task[0][0]), int(task[0][2])
            assert shape != SEG_IDLE, "a task led by an idle team"
            for d in task:
                assert d[0] in (shape, SEG_IDLE) and d[2] == nsteps, "a task mixes shapes or step counts"
                r = seg_run(d, S1, S2, shape, nsteps)
                if r is None:
                    continue
                slot = int(d[3]) & 0xFFFF
                assert slot not in R, "result slot written twice"
                R[slot] = r
        np_ = pe - pb
        # every slot written: a product's first segment at slot p, the
        # others at the extra slots prod_ext lists
        want = set(range(np_))
        for p in range(np_):
            ext = int(T["prod_ext"][pb + p])
            want.update((ext & 0xFFFF) + e for e in range(ext >> 16))
        if check_slots:
            assert sorted(R) == sorted(want), "result slots do not match the products' segments"
        c0 = T["group_ch"][g]
        for cl in range(T["group_ch"][g + 1] - c0):
            ch = T["group_channels"][c0 + cl]
            for s in range(16):
                a1, a2, a3, a4 = (s >> 3) & 1, (s >> 2) & 1, (s >> 1) & 1, s & 1
                v = 0j
                for c in range(T["ch_contrib"][c0 + cl], T["ch_contrib"][c0 + cl + 1]):
                    w = int(T["contrib_prod"][c])
                    p = w & 0xFFFF
                    rows1, lbl = (w >> 16) & 15, (w >> 20) & 3
                    l3, l4 = bool(lbl & 1), bool(lbl & 2)
                    rows2 = 16 // rows1
                    r1 = (a1 * (2 if l3 else 1) + (a3 if l3 else 0)) * (2 if l4 else 1) + (a4 if l4 else 0)
                    r2 = (a2 * (1 if l3 else 2) + (0 if l3 else a3)) * (1 if l4 else 2) + (0 if l4 else a4)
                    # the product's value: its first segment, then its
                    # extra segments in order (the kernel's summation order)
                    ext = int(T["contrib_ext"][c])
                    assert ext == int(T["prod_ext"][pb + p]), "contrib_ext differs from the product's prod_ext"
                    xv = R[p][r1 * rows2 + r2]
                    for e in range(ext >> 16):
                        xv = xv + R[(ext & 0xFFFF) + e][r1 * rows2 + r2]
                    v += T["contrib_coef"][c] * xv
                out[ch, s] = v
    return out
