"""Run the three C-ABI stages on torch-owned device memory (marshalling only).

PyTorch provides the device buffers and the stream; every arithmetic step
happens inside libnbs's HIP kernels.
"""
from __future__ import annotations

import numpy as np

from . import binding, synth

DECAY = {"u": 0.4, "d": 0.4, "s": 0.55}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the NBS path runs only in HIP kernels")
    return torch


def device_props(props_np, prec):
    """Host arrays [t, Lz, Ly, Lx, 12, 12] -> device tensors of the form's dtype."""
    torch = _torch()
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    return [torch.from_numpy(np.ascontiguousarray(p.astype(dt, copy=False))).to("cuda") for p in props_np]


def host_props(L, T, ts, decay=DECAY, same_ud=False, t0=0, source=0, dtype=np.complex128):
    """Seeded synthetic propagators (u, d, s) on slices ts: three arrays [len(ts), Lz, Ly, Lx, 12, 12]."""
    out = []
    for f, name in enumerate("uds"):
        if same_ud and name == "d":
            out.append(out[0])
            continue
        out.append(synth.propagators(L, ts, f, decay[name], T=T, t0=t0, source=source, dtype=dtype))
    return out


class Runner:
    """A plan plus its output buffer for one window of slices."""

    def __init__(self, L, T, chans, prec=binding.NBS_FP64, t0=0, t_begin=0, t_count=None, device=0):
        torch = _torch()
        self.plan = binding.Plan(L, T, chans, prec=prec, device=device, t0=t0, t_begin=t_begin,
                                 t_count=t_count)
        self.L = tuple(L)
        self.t_count = self.plan.geom.t_count
        self.n_ch = len(chans)
        self.F = torch.empty((self.n_ch, self.t_count, 16, L[2], L[1], L[0]), dtype=torch.complex128,
                             device="cuda")

    def stream(self):
        return _torch().cuda.current_stream().cuda_stream

    def build(self, pu, pd, ps):
        self.plan.build_blocks(pu.data_ptr(), pd.data_ptr(), ps.data_ptr(), self.stream())

    def contract(self):
        self.plan.contract_channels(self.stream())

    def relative_sum(self):
        self.plan.relative_sum(self.F.data_ptr(), self.stream())

    def run(self, pu, pd, ps):
        self.build(pu, pd, ps)
        self.contract()
        self.relative_sum()
        return self.F

    def close(self):
        self.plan.close()
