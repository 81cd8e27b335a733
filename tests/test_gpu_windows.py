"""Windowed sweeps over every sink slice with inputs generated on the device.

The device generator must reproduce the host generator's propagators (same
counter-based definition; log, cos and sin may differ in the last bit), and
a sweep of graph replays on refilled buffers must give, window by window,
the oracle's correlators of the host-generated propagators."""
import numpy as np
import pytest

import oracle
from paper_1604_07983_amd import binding, channels, runner, synth, synth_device
from tests.parity_util import flat_props, rel_err_per_channel

pytestmark = pytest.mark.gpu

DECAY45 = {"u": 0.45, "d": 0.45, "s": 0.45}


def announce(msg):
    print("[case] " + msg, flush=True)


@pytest.mark.parametrize("fp64", [1, 0])
def test_device_generator_matches_host(fp64):
    import torch
    announce("device generator, fp64=%d" % fp64)
    L, T = (5, 3, 4), 6
    dt_h = np.complex128 if fp64 else np.complex64
    dt_d = torch.complex128 if fp64 else torch.complex64
    # FP64: the two libms may differ by a few ulps; FP32: one rounding of the
    # same double, so at most one float ulp apart
    tol = 1e-14 if fp64 else 2.0 ** -23
    buf = torch.empty((L[2], L[1], L[0], 12, 12), dtype=dt_d, device="cuda")
    for t, flavour, source, t0 in ((0, 0, 0, 0), (3, 1, 7, 2), (5, 2, 23, 4), (1, 0, 3, 5)):
        synth_device.fill_slice(buf, L, t, flavour, 0.45, T, t0=t0, source=source)
        torch.cuda.synchronize()
        got = buf.cpu().numpy()
        want = synth.propagator_slice(L, t, flavour, 0.45, T=T, t0=t0, source=source, dtype=dt_h)
        scale = np.abs(want.astype(np.complex128))
        dev = np.abs(got.astype(np.complex128) - want.astype(np.complex128))
        assert (dev <= tol * np.maximum(scale, 1e-300) + 1e-300).all(), (t, flavour, source, float((dev / scale).max()))


@pytest.mark.parametrize("prec,tol", [(binding.NBS_FP32_MFMA, 1e-5), (binding.NBS_FP64, 1e-12)])
def test_sweep_every_sink_slice_matches_oracle(prec, tol):
    """Two lattices of different extent (T = 6 and 4) x 2 sources: windows
    0-3 hold all four geometries, 4-5 the longer lattice's two; every
    window's F against the oracle on host-generated inputs."""
    import torch
    announce("sink-slice sweep, prec %d" % prec)
    lattices = (((4, 4, 3), 6), ((3, 5, 4), 4))
    chans = [channels.r52()[c] for c in (0, 1, 2, 12, 22, 30, 51)]
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    seen = []

    def check(win, geoms, F, ms):
        assert ms > 0
        for g, f in zip(geoms, F):
            t = (g["t0"] + win) % g["T"]
            hp = runner.host_props(g["L"], g["T"], [t], decay=DECAY45, t0=g["t0"], source=g["source"], dtype=dt)
            want = oracle.correlators(g["L"], flat_props(hp, 0), chans, mode="fft")[:, None]
            got = f.cpu().numpy()  # [channel, window slice, spin, z, y, x]
            err = rel_err_per_channel(got, want)
            assert err.max() <= tol, (win, g, float(err.max()))
            seen.append((g["L"], g["source"], t))

    ms, n_win, sites = runner.sweep_sink_slices(lattices, 2, chans, DECAY45, check, prec=prec)
    torch.cuda.synchronize()
    assert n_win == 6 and ms > 0
    assert sites == 4 * 2 * (48 + 60) + 2 * 2 * 48
    want_seen = sorted((tuple(L), i * 2 + k, t) for i, (L, T) in enumerate(lattices) for k in range(2)
                       for t in range(T))
    assert sorted((tuple(a), b, c) for a, b, c in seen) == want_seen

