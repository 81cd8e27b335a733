"""Shared helpers of the GPU parity tests (test code only)."""
from __future__ import annotations

import numpy as np


def rel_err_per_channel(F_gpu, F_ref):
    """Per channel c: max over slices t of ||dF(., t)|| / ||F_ref(., t)|| with the
    norm over the 16 spin components and every r.  Arrays [c, t, 16, ...]."""
    d = np.asarray(F_gpu) - np.asarray(F_ref)
    num = np.sqrt((np.abs(d) ** 2).reshape(d.shape[0], d.shape[1], -1).sum(-1))
    den = np.sqrt((np.abs(F_ref) ** 2).reshape(d.shape[0], d.shape[1], -1).sum(-1))
    return (num / den).max(axis=1)


def flat_props(props, t):
    """Slice t of the three [t, Lz, Ly, Lx, 12, 12] arrays as [V, 12, 12] complex128."""
    return [np.ascontiguousarray(p[t].reshape(-1, 12, 12).astype(np.complex128)) for p in props]
