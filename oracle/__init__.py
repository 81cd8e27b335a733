"""CPU oracle for the two-baryon four-point function (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it.
It is a thin ctypes wrapper around ``nbs_oracle.c``, a plain FP64
implementation of Nemura (LATTICE 2015) Sec. 2, Eqs. (1)-(6): normal
blocks by their explicit 24-term sum (Eq. (5)), every flavour-respecting
Wick permutation with its sign (Eq. (4)), and the sum over X either
directly or through the DFT correlation (Eq. (6)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbs_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libnbs_oracle.so")

# Operator codes of nbs_oracle.h, named as in Eqs. (2)-(3).
OPS = {
    "p": 0, "n": 1, "Lambda": 2, "Sigma+": 3, "Sigma0": 4, "Sigma-": 5,
    "Xi0": 6, "Xi-": 7, "Xu": 8, "Xd": 9, "Xs": 10,
}
FLAVOURS = ("u", "d", "s")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP) into oracle/_build."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
             "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        lib.ora_cg5.argtypes = [P]
        lib.ora_expand_op.argtypes = [I, P, P]
        lib.ora_normal_blocks.argtypes = [P, P, I, I, I, P]
        lib.ora_dft3.argtypes = [P, I, P, I]
        lib.ora_correlators.argtypes = [I, P, P, I, P, P]
        lib.ora_correlators_at_q.argtypes = [P, P, I, P, P, P]
        lib.ora_count_perms.argtypes = [P, P, P]
        lib.ora_two_point.argtypes = [P, P, I, P, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _props(S):
    """S: sequence of three complex128 arrays (u, d, s), each [..., 12, 12]."""
    arrs = [np.ascontiguousarray(s, dtype=np.complex128) for s in S]
    ptrs = (ctypes.c_void_p * 3)(*[a.ctypes.data for a in arrs])
    return arrs, ptrs


def _L(L):
    return np.ascontiguousarray(np.asarray(L, dtype=np.int32))


def _chans(chans):
    c = np.array([[OPS[b] if isinstance(b, str) else int(b) for b in ch] for ch in chans],
                 dtype=np.int32)
    return np.ascontiguousarray(c.reshape(-1, 4))


def cg5() -> np.ndarray:
    out = np.zeros(16)
    _load().ora_cg5(_ptr(out))
    return out.reshape(4, 4)


def expand_op(op):
    fl = np.zeros(9, dtype=np.int32)
    w = np.zeros(3)
    code = OPS[op] if isinstance(op, str) else int(op)
    n = _load().ora_expand_op(code, _ptr(fl), _ptr(w))
    return [(tuple(int(x) for x in fl[3 * k:3 * k + 3]), float(w[k])) for k in range(n)]


def normal_blocks(L, S, f1, f2, f3) -> np.ndarray:
    """N_{f1 f2 f3}(x) as complex128 [V, 2, 12, 12, 12]."""
    V = int(np.prod(L))
    arrs, ptrs = _props(S)
    out = np.zeros((V, 2, 12, 12, 12), dtype=np.complex128)
    rc = _load().ora_normal_blocks(_ptr(_L(L)), ptrs, f1, f2, f3, _ptr(out))
    assert rc == 0
    return out


def dft3(data: np.ndarray, L, sign: int) -> np.ndarray:
    """DFT over sites of a site-major array [V, nfield] (copy returned)."""
    d = np.ascontiguousarray(data, dtype=np.complex128).copy()
    V = int(np.prod(L))
    nfield = d.size // V
    rc = _load().ora_dft3(_ptr(d), nfield, _ptr(_L(L)), int(sign))
    assert rc == 0
    return d


def correlators(L, S, chans, mode: str = "fft") -> np.ndarray:
    """F for each channel on one time slice: complex128 [n_ch, 16, Lz, Ly, Lx].

    mode "direct" sums over X explicitly (Eq. (4)); "fft" uses Eq. (6)."""
    V = int(np.prod(L))
    arrs, ptrs = _props(S)
    c = _chans(chans)
    F = np.zeros((len(c), 16, V), dtype=np.complex128)
    rc = _load().ora_correlators(0 if mode == "direct" else 1, _ptr(_L(L)), ptrs,
                                 len(c), _ptr(c), _ptr(F))
    if rc:
        raise RuntimeError("oracle failed (%d)" % rc)
    return F.reshape(len(c), 16, L[2], L[1], L[0])


def correlators_at_q(L, S, chans, q) -> np.ndarray:
    """F~_c(q) (before the 1/V inverse DFT): complex128 [n_ch, 16]."""
    arrs, ptrs = _props(S)
    c = _chans(chans)
    out = np.zeros((len(c), 16), dtype=np.complex128)
    qq = np.ascontiguousarray(np.asarray(q, dtype=np.int32))
    rc = _load().ora_correlators_at_q(_ptr(_L(L)), ptrs, len(c), _ptr(c), _ptr(qq), _ptr(out))
    if rc:
        raise RuntimeError("oracle failed (%d)" % rc)
    return out


def count_perms(chan):
    c = _chans([chan])[0]
    nt = np.zeros(1, dtype=np.int32)
    npm = np.zeros(1, dtype=np.int32)
    rc = _load().ora_count_perms(_ptr(c), _ptr(nt), _ptr(npm))
    assert rc == 0
    return int(nt[0]), int(npm[0])


def two_point(L, S, pairs) -> np.ndarray:
    """Zero-momentum single-baryon two-point functions on one time slice:
    complex128 [n_pairs, 2, 2] (sink spin, source spin) for (sink, source)
    operator pairs."""
    arrs, ptrs = _props(S)
    c = np.ascontiguousarray(np.array([[OPS[b] if isinstance(b, str) else int(b) for b in pr] for pr in pairs],
                                      dtype=np.int32).reshape(-1, 2))
    out = np.zeros((len(c), 2, 2), dtype=np.complex128)
    rc = _load().ora_two_point(_ptr(_L(L)), ptrs, len(c), _ptr(c), _ptr(out))
    if rc:
        raise RuntimeError("oracle failed (%d)" % rc)
    return out
