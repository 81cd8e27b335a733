"""Separable propagators S_f(x) = phi_f(x) M_f and the closed form of their
four-point functions (test code only).

With such inputs every normal block factorises, N_t(x) = Phi_t(x) N_t[M]
with Phi_t the product of the phi of the block's three quark flavours, and
the flavour content of a sink operator is the same for every Wick
permutation.  So each channel is
    F_c,s(r) = C_c,s  sum_X Phi_B1(X + r) Phi_B2(X),
where C_c,s is the channel on constant propagators M_f divided by the
volume (F is then constant in r).  C comes from the oracle on a 2^3
lattice; the scalar correlation from numpy's FFT.
"""
from __future__ import annotations

import numpy as np

import oracle

# quark content (u, d, s) of each sink operator (Eqs. (2)-(3))
CONTENT = {"p": (2, 1, 0), "n": (1, 2, 0), "Lambda": (1, 1, 1), "Sigma+": (2, 0, 1), "Sigma0": (1, 1, 1),
           "Sigma-": (0, 2, 1), "Xi0": (1, 0, 2), "Xi-": (0, 1, 2), "Xu": (1, 1, 1), "Xd": (1, 1, 1),
           "Xs": (1, 1, 1)}


def make(L, seed=7, dtype=np.complex64):
    """Propagators of one slice, three arrays [1, Lz, Ly, Lx, 12, 12], and the
    factors: (M [3, 12, 12] complex128, phi [3, Lz, Ly, Lx] complex128)."""
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz = L
    M = (rng.standard_normal((3, 12, 12)) + 1j * rng.standard_normal((3, 12, 12))) / np.sqrt(2)
    phi = (rng.standard_normal((3, Lz, Ly, Lx)) + 1j * rng.standard_normal((3, Lz, Ly, Lx))) / np.sqrt(2)
    props = []
    for f in range(3):
        S = (phi[f][..., None, None].astype(dtype) * M[f].astype(dtype)[None, None, None])
        props.append(S[None])
    # the values the GPU sees (storage rounding included) factor exactly only
    # in FP64; for complex64 inputs the factors are taken after rounding
    return props, M, phi


def constants(chans, M):
    """C_c,s: the channels on constant propagators M_f, per site: [n_ch, 16]."""
    L = (2, 2, 2)
    S = [np.ascontiguousarray(np.broadcast_to(M[f], (8, 12, 12))) for f in range(3)]
    F = oracle.correlators(L, S, chans, mode="direct")
    return F[:, :, 0, 0, 0] / 8.0


def correlation(phi, c1, c2):
    """sum_X Phi1(X + r) Phi2(X) on the lattice of phi ([3, Lz, Ly, Lx])."""
    P1 = np.prod([phi[f] ** c1[f] for f in range(3)], axis=0)
    P2 = np.prod([phi[f] ** c2[f] for f in range(3)], axis=0)
    V = P1.size
    return np.fft.ifftn(np.fft.fftn(P1) * (V * np.fft.ifftn(P2)))


def channel(chan, C_row, phi):
    """Closed-form F of one channel: [16, Lz, Ly, Lx] complex128."""
    corr = correlation(phi, CONTENT[chan[0]], CONTENT[chan[1]])
    return C_row[:, None, None, None] * corr[None]
