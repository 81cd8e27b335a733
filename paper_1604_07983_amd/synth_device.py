"""The synthetic propagators of synth.py generated on the device by
libnbs_synth.so (input generation only; the same counter-based definition,
see synth.py), for workloads too large to generate on the host."""
from __future__ import annotations

import ctypes
import math
import os

from . import synth

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libnbs_synth.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError("libnbs_synth.so is not built (%s); run __graft_entry__.build()" % _LIB)
        L = ctypes.CDLL(_LIB)
        L.nbs_synth_slice.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_longlong,
                                      ctypes.c_int, ctypes.c_double, ctypes.c_void_p]
        L.nbs_synth_slice.restype = ctypes.c_int
        _lib = L
    return _lib


def fill_slice(dst, L, t, flavour, decay, T, t0=0, source=0, base=synth.SEED_BASE, stream=0):
    """Write one flavour's propagator on slice t into the device tensor dst
    ([Lz, Ly, Lx, 12, 12], complex128 or complex64)."""
    import torch
    V = int(L[0]) * int(L[1]) * int(L[2])
    assert dst.is_cuda and dst.is_contiguous() and dst.numel() == V * 144
    fp64 = 1 if dst.dtype == torch.complex128 else 0
    assert fp64 or dst.dtype == torch.complex64
    damp = math.exp(-decay * ((t - t0) % T))
    rc = lib().nbs_synth_slice(dst.data_ptr(), fp64, synth.seed_for(flavour, source, base), V, int(t), damp, stream)
    if rc != 0:
        raise RuntimeError("nbs_synth_slice failed (%d)" % rc)
