"""Independent constructions used to pin the oracle (test code only).

Everything here is rebuilt from the paper's definitions and textbook
mathematics, not from the oracle's tables: gamma matrices in the Dirac
representation, the Levi-Civita symbol from permutation parity, the
operator content of Eqs. (2)-(3), and the Wick contraction of six quark
fields written as a 6x6 determinant (sum over permutations with sign),
which replaces the oracle's explicit permutation enumeration.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

U, D, S = 0, 1, 2

# Eqs. (2)-(3): operator -> [(flavours of eps (q1 Cg5 q2) q3, weight)]
_R6, _R2 = 1 / math.sqrt(6.0), 1 / math.sqrt(2.0)
OPERATORS = {
    "p": [((U, D, U), 1.0)],
    "n": [((U, D, D), -1.0)],
    "Sigma+": [((U, S, U), -1.0)],
    "Sigma-": [((D, S, D), -1.0)],
    "Xi0": [((U, S, S), 1.0)],
    "Xi-": [((D, S, S), -1.0)],
    "Xu": [((D, S, U), 1.0)],
    "Xd": [((S, U, D), 1.0)],
    "Xs": [((U, D, S), 1.0)],
    "Lambda": [((D, S, U), _R6), ((S, U, D), _R6), ((U, D, S), -2 * _R6)],
    "Sigma0": [((D, S, U), _R2), ((S, U, D), -_R2)],
}


def dirac_cg5() -> np.ndarray:
    """C gamma_5 with gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 = diag(1, 1, -1, -1),
    gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 and C = gamma_4 gamma_2."""
    s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]),
         np.array([[1, 0], [0, -1]], complex)]
    Z, I2 = np.zeros((2, 2), complex), np.eye(2, dtype=complex)
    g = [np.block([[Z, -1j * sk], [1j * sk, Z]]) for sk in s]
    g4 = np.block([[I2, Z], [Z, -I2]])
    g5 = g[0] @ g[1] @ g[2] @ g4
    C = g4 @ g[1]
    return C @ g5


def levi_civita(a: int, b: int, c: int) -> int:
    p = (a, b, c)
    if len(set(p)) < 3:
        return 0
    inv = sum(1 for i in range(3) for j in range(i + 1, 3) if p[i] > p[j])
    return -1 if inv % 2 else 1


def baryon_tensor(alpha: int, cg5: np.ndarray):
    """Non-zero entries of eps_abc (Cg5)_{be ga} with the third quark's spin
    fixed to alpha: [((j1, j2, j3), coef)], j = 3 * spin + colour."""
    out = []
    for a, b, c in itertools.permutations(range(3)):
        e = levi_civita(a, b, c)
        for be in range(4):
            for ga in range(4):
                if abs(cg5[be, ga]) > 0.5:
                    out.append(((3 * be + a, 3 * ga + b, 3 * alpha + c),
                                e * float(np.real(cg5[be, ga]))))
    return out


def site_index(L, x, y, z) -> int:
    return (x % L[0]) + L[0] * ((y % L[1]) + L[1] * (z % L[2]))


def site_coords(L, s: int):
    return s % L[0], (s // L[0]) % L[1], s // (L[0] * L[1])


def brute_force_correlator(L, props, chan, spins, r) -> complex:
    """F^{<B1 B2 B3bar B4bar>}_{a1 a2, a3 a4}(r) of Eq. (1) by expanding every
    operator into quark fields and evaluating <q1..q6 qbar'..> as the
    determinant of the 6x6 flavour-blocked propagator matrix.

    props[f] is [V, 12, 12] complex; B1 sits at X + r, B2 at X."""
    cg5 = dirac_cg5()
    a1, a2, a3, a4 = spins
    V = int(np.prod(L))
    T = [baryon_tensor(a, cg5) for a in (a1, a2, a3, a4)]
    rows = np.array([t1[0] + t2[0] for t1 in T[0] for t2 in T[1]])        # (576, 6)
    crow = np.array([t1[1] * t2[1] for t1 in T[0] for t2 in T[1]])
    cols = np.array([t3[0] + t4[0] for t3 in T[2] for t4 in T[3]])
    ccol = np.array([t3[1] * t4[1] for t3 in T[2] for t4 in T[3]])
    total = 0j
    for (f1, w1), (f2, w2), (f3, w3), (f4, w4) in itertools.product(
            *(OPERATORS[b] for b in chan)):
        sinkfl, srcfl = f1 + f2, f3 + f4
        match = np.array([[sinkfl[i] == srcfl[k] for k in range(6)] for i in range(6)], float)
        for X in range(V):
            x, y, z = site_coords(L, X)
            x1 = site_index(L, x + r[0], y + r[1], z + r[2])
            mats = np.stack([props[sinkfl[i]][x1 if i < 3 else X] for i in range(6)])
            M = mats[np.arange(6)[None, None, :, None], rows[:, None, :, None],
                     cols[None, :, None, :]] * match
            det = np.linalg.det(M)
            total += w1 * w2 * w3 * w4 * (crow @ det @ ccol)
    return total


def random_props(rng, L, n=3):
    V = int(np.prod(L))
    return [(rng.standard_normal((V, 12, 12)) + 1j * rng.standard_normal((V, 12, 12))) / math.sqrt(2)
            for _ in range(n)]


def random_su3(rng) -> np.ndarray:
    z = (rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3)))
    q, rr = np.linalg.qr(z)
    q = q * (np.diag(rr) / np.abs(np.diag(rr)))
    return q / np.linalg.det(q) ** (1.0 / 3.0)


def colour_matrix(omega: np.ndarray) -> np.ndarray:
    """12x12 action of a colour matrix on j = 3 * spin + colour."""
    return np.kron(np.eye(4), omega)
