"""CPU emulation of the compiled contraction program (test code only).

Executes the SoA tables exported by nbs_plan_table exactly as the
contraction kernel interprets them (load / EBB / MEB / ACC per chunk), on
momentum-space normal blocks supplied by the test.  It lets the host test
suite check the channel compiler and its scheduling against the oracle
without a GPU; it is never part of the product path.
"""
from __future__ import annotations

import numpy as np

NAMES = ("type_code", "group_chunk", "group_ch", "group_channels", "chunk_step", "chunk_meb",
         "chunk_acc", "chunk_esize", "step_type", "step_side", "step_load", "step_ebb", "ebb_e",
         "ebb_term", "terms", "meb_e1", "meb_e2", "meb_K", "meb_k0", "meb_kn", "meb_rows1",
         "acc_target", "acc_src_range", "acc_src", "acc_coef")


def tables(plan):
    return {n: plan.table(n) for n in NAMES}


def emulate_q(T, params, Nq_plus, Nq_minus, n_ch):
    """F~(q) [n_ch, 16] from Nq_plus[slot] = N~_type(q), Nq_minus[slot] = N~_type(-q)."""
    out = np.zeros((n_ch, 16), dtype=np.complex128)
    terms = T["terms"].astype(np.int64)
    t_idx = terms & 0xFFFF
    t_coef = (T["terms"] >> 16).astype(np.float64)  # arithmetic shift keeps the sign
    n_groups = len(T["group_chunk"]) - 1
    for g in range(n_groups):
        c0, c1 = T["group_ch"][g], T["group_ch"][g + 1]
        nch = c1 - c0
        assert nch <= params["max_group_channels"]
        acc = np.zeros(nch * 16, dtype=np.complex128)
        held = None
        slot = None
        for c in range(T["group_chunk"][g], T["group_chunk"][g + 1]):
            esize = T["chunk_esize"][c]
            assert esize <= params["e_budget"]
            E = np.zeros(esize, dtype=np.complex128)
            for s in range(T["chunk_step"][c], T["chunk_step"][c + 1]):
                want = (int(T["step_type"][s]), int(T["step_side"][s]))
                if T["step_load"][s]:
                    held = want
                    slot = (Nq_minus if want[1] else Nq_plus)[want[0]]
                assert held == want, "step reads a block the LDS slot does not hold"
                i0, i1 = T["step_ebb"][s], T["step_ebb"][s + 1]
                if i1 == i0:
                    continue
                lo, hi = T["ebb_term"][i0], T["ebb_term"][i1]
                vals = t_coef[lo:hi] * slot[t_idx[lo:hi]]
                starts = T["ebb_term"][i0:i1] - lo
                sums = np.add.reduceat(vals, starts)
                tgt = T["ebb_e"][i0:i1]
                assert len(np.unique(tgt)) == len(tgt)
                assert tgt.max() < esize
                E[tgt] += sums
            m0, m1 = T["chunk_meb"][c], T["chunk_meb"][c + 1]
            assert m1 - m0 <= params["item_budget"]
            part = np.zeros((m1 - m0) * 16, dtype=np.complex128)
            for it in range(m0, m1):
                e1, e2, K = T["meb_e1"][it], T["meb_e2"][it], T["meb_K"][it]
                k0, kn, r1 = T["meb_k0"][it], T["meb_kn"][it], T["meb_rows1"][it]
                r2 = 16 // r1
                ks = np.arange(k0, k0 + kn)
                X = E[e1 + np.arange(r1)[:, None] * K + ks[None, :]]
                Y = E[e2 + np.arange(r2)[:, None] * K + ks[None, :]]
                part[(it - m0) * 16:(it - m0 + 1) * 16] = (X @ Y.T).ravel()
            for it in range(T["chunk_acc"][c], T["chunk_acc"][c + 1]):
                a0, a1 = T["acc_src_range"][it], T["acc_src_range"][it + 1]
                acc[T["acc_target"][it]] += np.sum(T["acc_coef"][a0:a1] * part[T["acc_src"][a0:a1]])
        out[T["group_channels"][c0:c1]] = acc.reshape(nch, 16)
    return out
