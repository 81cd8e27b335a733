"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times: 16^3 x 32 (plain FP64, all 52 channels) and 32^3 x 64 (the
precision form).  The oracle cannot afford every output at these sizes, so it
is evaluated one by one at sampled momenta (F~_c(q) of all 52 channels, the
q = 0 one being the sum rule) and, for a channel subset, over a full slice.
"""
import numpy as np
import pytest

import oracle
from paper_1604_07983_amd import binding, channels, runner
from tests.parity_util import flat_props, rel_err_per_channel

pytestmark = pytest.mark.gpu

DECAY = {"u": 0.4, "d": 0.4, "s": 0.55}


def announce(msg):
    print("[case] " + msg, flush=True)


def run_window(L, T, prec, t_begin, t_count, chans):
    import torch
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, T, range(t_begin, t_begin + t_count), decay=DECAY, dtype=dt)
    dp = runner.device_props(props, prec)
    r = runner.Runner(L, T, chans, prec=prec, t_begin=t_begin, t_count=t_count)
    F = r.run(*dp)
    torch.cuda.synchronize()
    out = F.cpu().numpy()
    r.close()
    del dp
    return props, out


def check_sampled_momenta(L, props, Fg, chans, slices, qs, tol):
    """F~_c(q) = sum_r F_c(r) exp(-i q.r) of the GPU output against the oracle."""
    for ti in slices:
        Fq = np.fft.fftn(Fg[:, ti], axes=(2, 3, 4))  # [c, 16, qz, qy, qx]
        S = flat_props(props, ti)
        for q in qs:
            want = oracle.correlators_at_q(L, S, chans, q)
            got = Fq[:, :, q[2], q[1], q[0]]
            err = np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)
            assert err.max() <= tol, (ti, q, float(err.max()), int(err.argmax()))


def test_config2_fp64_16c32_all_channels():
    announce("16^3 x 32 fp64 r52")
    L, T = (16, 16, 16), 32
    chans = channels.r52()
    props, Fg = run_window(L, T, binding.NBS_FP64, 0, 32, chans)
    assert np.isfinite(Fg).all()
    check_sampled_momenta(L, props, Fg, chans, slices=(0, 31), qs=((0, 0, 0), (1, 2, 3), (15, 8, 1)),
                          tol=1e-12)
    # every slice at one momentum of its own (q = (t, 3t + 1, 5t + 2) mod 16)
    for ti in range(1, 31):
        q = (ti % 16, (3 * ti + 1) % 16, (5 * ti + 2) % 16)
        check_sampled_momenta(L, props, Fg, chans, slices=(ti,), qs=(q,), tol=1e-12)
    # a full slice for channels of each sector
    sub = [0, 1, 12, 30, 51]
    Fo = oracle.correlators(L, flat_props(props, 17), [chans[c] for c in sub], mode="fft")
    err = rel_err_per_channel(Fg[sub][:, 17:18], Fo[:, None])
    assert err.max() <= 1e-12, err


@pytest.mark.parametrize("t_begin", [0, 30, 62])
def test_config3_fp32_32c64_windows(t_begin):
    """Precision form at 32^3, two-slice windows at both ends and the middle
    of T = 64 (slices 0, 1, 30, 31, 62, 63; the latest decay by
    e^-(0.4*4+0.55*2)*63 ~ 1e-74 in some channels)."""
    announce("32^3 x 64 precision form window %d" % t_begin)
    L, T = (32, 32, 32), 64
    chans = channels.r52()
    props, Fg = run_window(L, T, binding.NBS_FP32_MFMA, t_begin, 2, chans)
    assert np.isfinite(Fg).all()
    check_sampled_momenta(L, props, Fg, chans, slices=(0, 1), qs=((0, 0, 0), (3, 30, 7)), tol=1e-5)


def test_config3_fp32_32c64_bench_window():
    """The benchmark's exact launch: 32^3 x 64, one 16-slice window (10.5 M
    contraction workgroups, more work-items than one dispatch can address, so
    the launch is split); the first and the last slice at sampled momenta,
    and the first slice over every r for a channel of the first and of the
    last strangeness sector."""
    announce("32^3 x 64 precision form, 16-slice window")
    L, T = (32, 32, 32), 64
    chans = channels.r52()
    props, Fg = run_window(L, T, binding.NBS_FP32_MFMA, 0, 16, chans)
    assert np.isfinite(Fg).all()
    check_sampled_momenta(L, props, Fg, chans, slices=(0, 15), qs=((0, 0, 0), (31, 5, 17)), tol=1e-5)
    sub = [0, 51]
    Fo = oracle.correlators(L, flat_props(props, 0), [chans[c] for c in sub], mode="fft")
    err = rel_err_per_channel(Fg[sub][:, 0:1], Fo[:, None])
    assert err.max() <= 1e-5, err


def test_config5_96cubed_slice_closed_form():
    """One slice of the 96^3 slab (the precision form, one GPU's share of a
    time-split 96^3 x 64 run), every channel against the closed form of
    separable propagators phi_f(x) M_f (the oracle's channel constants times
    a scalar correlation): the 96-point transforms, 196 GB of blocks and
    the 17.7 M-workgroup contraction at their real size."""
    import gc
    import torch
    from tests import separable
    gc.collect()
    torch.cuda.empty_cache()
    announce("96^3 slice, separable propagators")
    L, T = (96, 96, 96), 64
    chans = channels.r52()
    props, M, phi = separable.make(L, seed=11, dtype=np.complex64)
    dp = runner.device_props(props, binding.NBS_FP32_MFMA)
    r = runner.Runner(L, T, chans, prec=binding.NBS_FP32_MFMA, t_begin=0, t_count=1)
    F = r.run(*dp)
    torch.cuda.synchronize()
    r.close()
    del dp
    C = separable.constants(chans, M)
    for c, ch in enumerate(chans):
        got = F[c, 0].cpu().numpy()
        want = separable.channel(ch, C[c], phi)
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert err <= 1e-5, (c, ch, float(err))


def test_config5_96cubed_gaussian_flavour_limit():
    """Slice 0 of the 96^3 slab with the seeded Gaussian generator, u = d = s
    (one propagator, decay 0.4): pp <- pp, Sigma+ Sigma+ <- Sigma+ Sigma+ and
    Xi0 Xi0 <- Xi0 Xi0 agree everywhere (flavour relabelling, which holds at
    any size), and pp's F~(0) = sum_r F(r) matches the oracle's
    zero-momentum value computed from the same propagator."""
    import gc
    import torch
    from paper_1604_07983_amd import synth
    gc.collect()
    torch.cuda.empty_cache()
    announce("96^3 slice 0, Gaussian, u = d = s")
    L, T = (96, 96, 96), 64
    chans = [channels.r52()[c] for c in (0, 12, 50)]
    S = synth.propagator_slice(L, 0, 0, 0.4, T=T, dtype=np.complex64)
    d = torch.from_numpy(S).to("cuda").reshape(1, *S.shape)
    r = runner.Runner(L, T, chans, prec=binding.NBS_FP32_MFMA, t_begin=0, t_count=1)
    F = r.run(d, d, d)
    torch.cuda.synchronize()
    r.close()
    del d
    Fh = F[:, 0].cpu().numpy()
    del F
    torch.cuda.empty_cache()
    assert np.isfinite(Fh).all()
    for c in (1, 2):
        err = np.linalg.norm(Fh[c] - Fh[0]) / np.linalg.norm(Fh[0])
        assert err <= 1e-5, (c, float(err))
    S128 = np.ascontiguousarray(S.reshape(-1, 12, 12).astype(np.complex128))
    del S
    want = oracle.correlators_at_q(L, [S128, S128, S128], chans[:1], (0, 0, 0))[0]
    got = Fh[0].reshape(16, -1).sum(axis=1)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err <= 1e-5, float(err)


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
def test_two_point_full_slices(prec):
    """Zero-momentum octet two-point functions at 16^3 x 32 (all 32 slices
    from one build, as the benchmark calls it) against the oracle on three
    slices."""
    import torch
    announce("two-point 16^3 x 32 prec %d" % prec)
    L, T = (16, 16, 16), 32
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, T, range(T), decay=DECAY, dtype=dt)
    dp = runner.device_props(props, prec)
    r = runner.Runner(L, T, channels.r52(), prec=prec, t_count=T)
    r.build(*dp)
    pairs = [(b, b) for b in ("p", "n", "Lambda", "Sigma+", "Sigma0", "Sigma-", "Xi0", "Xi-")]
    C = r.two_point(pairs).cpu().numpy()
    torch.cuda.synchronize()
    r.close()
    del dp
    assert np.isfinite(C).all()
    tol = 1e-12 if prec == binding.NBS_FP64 else 1e-5
    for t in (0, 13, 31):
        want = oracle.two_point(L, flat_props(props, t), pairs)
        got = C[:, t]
        err = np.linalg.norm((got - want).reshape(len(pairs), -1), axis=1) / \
            np.linalg.norm(want.reshape(len(pairs), -1), axis=1)
        assert err.max() <= tol, (t, float(err.max()), int(err.argmax()))
