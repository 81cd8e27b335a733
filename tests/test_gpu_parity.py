"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (norm-wise relative error per channel, max over slices):
1e-12 for the plain FP64 form and 1e-5 for the precision form.
"""
import numpy as np
import pytest

import oracle
from paper_1604_07983_amd import binding, channels, runner
from tests.parity_util import flat_props, rel_err_per_channel

pytestmark = pytest.mark.gpu

TOL = {binding.NBS_FP64: 1e-12, binding.NBS_FP32_MFMA: 1e-5}


def announce(msg):
    print("[case] " + msg, flush=True)


def run_gpu(L, T, chans, props_np, prec, t0=0, t_begin=0, t_count=None, tuning=None, alias_ud=False):
    import torch
    dp = runner.device_props(props_np, prec)
    if alias_ud:
        dp[1] = dp[0]  # the same memory for u and d: the isospin-symmetric limit
    r = runner.Runner(L, T, chans, prec=prec, t0=t0, t_begin=t_begin, t_count=t_count)
    if tuning:
        r.plan.set_tuning(**tuning)
    F = r.run(*dp)
    torch.cuda.synchronize()
    out = F.cpu().numpy()
    r.close()
    return out


def oracle_F(L, props_np, chans, mode="fft"):
    """[c, t, 16, Lz, Ly, Lx] from the oracle, slice by slice."""
    nt = props_np[0].shape[0]
    return np.stack([oracle.correlators(L, flat_props(props_np, i), chans, mode=mode) for i in range(nt)],
                    axis=1)


def test_config1_pp_fp64_direct_sum():
    """4^3 x 8, pp only, u = d, decay 0.5, every slice against the O(V^2) direct sum."""
    announce("config1 pp 4^3x8 fp64")
    L, T = (4, 4, 4), 8
    props = runner.host_props(L, T, range(T), decay={"u": 0.5, "d": 0.5, "s": 0.5}, same_ud=True)
    chans = [("p", "p", "p", "p")]
    Fg = run_gpu(L, T, chans, props, binding.NBS_FP64)
    Fo = oracle_F(L, props, chans, mode="direct")
    err = rel_err_per_channel(Fg, Fo)
    assert err.max() <= 1e-12, err


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
def test_all_r52_channels_small_lattice(prec):
    """Every R52 channel on a non-cubic 4x2x3 lattice, three slices."""
    announce("r52 4x2x3 prec=%d" % prec)
    L, T = (4, 2, 3), 3
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, T, range(T), dtype=dt)
    chans = channels.r52()
    Fg = run_gpu(L, T, chans, props, prec)
    Fo = oracle_F(L, props, chans)
    err = rel_err_per_channel(Fg, Fo)
    assert err.max() <= TOL[prec], (err.max(), int(err.argmax()))


@pytest.mark.parametrize("sector", [(-2, 0), (-1, -1), (-3, 1)])
def test_generated_sector_tables(sector):
    """Channel tables generated from quantum numbers (every ordered octet
    pair of a strangeness and I_z sector, coupled channels included) run end
    to end against the oracle."""
    announce("generated sector %s" % (sector,))
    L, T = (4, 2, 3), 2
    props = runner.host_props(L, T, range(T), dtype=np.complex128)
    chans = channels.coupled_channels(*sector, ordered=True)
    Fg = run_gpu(L, T, chans, props, binding.NBS_FP64)
    Fo = oracle_F(L, props, chans)
    err = rel_err_per_channel(Fg, Fo)
    assert err.max() <= TOL[binding.NBS_FP64], (err.max(), int(err.argmax()))


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
def test_window_and_source_slice(prec):
    """A window t_begin = 3, t_count = 2 of T = 6 with the source at t0 = 2."""
    announce("window 6x4x2 prec=%d" % prec)
    L, T, t0, tb, tc = (6, 4, 2), 6, 2, 3, 2
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, T, range(tb, tb + tc), t0=t0, dtype=dt)
    chans = [channels.WORKED_EXAMPLE, ("Xi0", "Xi-", "Xi0", "Xi-"), ("Lambda", "Lambda", "p", "Xi-")]
    Fg = run_gpu(L, T, chans, props, prec, t0=t0, t_begin=tb, t_count=tc)
    Fo = oracle_F(L, props, chans)
    err = rel_err_per_channel(Fg, Fo)
    assert err.max() <= TOL[prec], err


def test_repeat_runs_are_bit_identical():
    announce("determinism 4^3 r52 fp64")
    L, T = (4, 4, 4), 2
    props = runner.host_props(L, T, range(T))
    chans = channels.r52()
    a = run_gpu(L, T, chans, props, binding.NBS_FP64)
    b = run_gpu(L, T, chans, props, binding.NBS_FP64)
    assert np.array_equal(a.view(np.float64), b.view(np.float64))


def test_state_errors_on_device_plan():
    announce("state errors")
    import torch
    r = runner.Runner((2, 2, 2), 2, [("p", "p", "p", "p")])
    with pytest.raises(binding.NbsError) as e:
        r.contract()
    assert e.value.status == 5
    with pytest.raises(binding.NbsError) as e:
        r.relative_sum()
    assert e.value.status == 5
    with pytest.raises(binding.NbsError) as e:
        r.plan.build_blocks(0, 0, 0, r.stream())
    assert e.value.status == 1
    assert r.plan.workspace_bytes() > 0
    r.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
def test_square_plane_lattice(prec):
    """8 x 8 x 3: square x-y planes take the fused two-axis transform."""
    announce("square plane 8x8x3 prec=%d" % prec)
    L, T = (8, 8, 3), 2
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, T, range(T), dtype=dt)
    chans = channels.r52()
    Fg = run_gpu(L, T, chans, props, prec)
    Fo = oracle_F(L, props, chans)
    err = rel_err_per_channel(Fg, Fo)
    assert err.max() <= TOL[prec], (err.max(), int(err.argmax()))


@pytest.mark.parametrize("tuning", [dict(engine=0, waves=4), dict(engine=0, mfma=1, waves=4),
                                    dict(engine=0, mfma=1, waves=8),
                                    dict(engine=0, waves=4, split=0, fft_line=0, fft_tile=2048), dict(fft_plane=1),
                                    dict(gchunk=1), dict(gchunk=2, waves=8), dict(waves=16), dict(persist=1),
                                    dict(persist=1, gchunk=1, waves=16)])
def test_precision_form_launch_shapes(tuning):
    """The precision form under other launch shapes (the lane-team engine
    with and without its matrix-core quads, 256- and 512-thread workgroups,
    no index splitting, LDS-tile transforms, the fused x-y pass, group
    ranges, 1024-thread matrix-core workgroups) on every R52 channel."""
    announce("precision form shapes %s" % tuning)
    L, T = (8, 8, 3), 2
    props = runner.host_props(L, T, range(T), dtype=np.complex64)
    chans = channels.r52()
    Fg = run_gpu(L, T, chans, props, binding.NBS_FP32_MFMA, tuning=tuning)
    Fo = oracle_F(L, props, chans)
    err = rel_err_per_channel(Fg, Fo)
    assert err.max() <= 1e-5, (err.max(), int(err.argmax()))


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
@pytest.mark.parametrize("L", [(24, 24, 2), (32, 32, 2), (40, 40, 2)])
def test_plane_pass_wide_planes(L, prec):
    """The fused x-y pass on 24^2, 32^2 and 40^2 planes (512-thread
    workgroups and XCD-paired field tiles for complex64 32^2 and 40^2)
    against the line passes and the oracle."""
    announce("plane pass %s prec=%d" % (L, prec))
    chans = [channels.r52()[c] for c in (0, 12, 22, 51)]
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, 2, range(1), dtype=dt)
    Fp = run_gpu(L, 2, chans, props, prec, t_count=1, tuning=dict(fft_plane=1))
    Fl = run_gpu(L, 2, chans, props, prec, t_count=1, tuning=dict(fft_plane=0))
    Fo = oracle_F(L, props, chans)
    for Fg in (Fp, Fl):
        err = rel_err_per_channel(Fg, Fo)
        assert err.max() <= TOL[prec], (err.max(), int(err.argmax()))


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
@pytest.mark.parametrize("L", [(64, 2, 3), (80, 2, 2), (96, 2, 2)])
def test_long_register_lines(L, prec):
    """Lines of 64, 80 and 96 points, two threads per line with FP64
    arithmetic, forward and inverse, in both forms; channels of every
    strangeness sector against the oracle."""
    announce("long lines %s prec=%d" % (L, prec))
    chans = [channels.r52()[c] for c in (0, 1, 2, 12, 22, 30, 51)]
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, 2, range(1), dtype=dt)
    Fg = run_gpu(L, 2, chans, props, prec, t_count=1)
    Fo = oracle_F(L, props, chans)
    err = rel_err_per_channel(Fg, Fo)
    assert err.max() <= TOL[prec], (err.max(), int(err.argmax()))


@pytest.mark.parametrize("tuning", [dict(gchunk=1), dict(gchunk=2), dict(persist=1), dict(persist=1, gchunk=1),
                                    dict(engine=0, waves=8),
                                    dict(engine=0, waves=8, gchunk=2), dict(waves=16)])
def test_fp64_launch_shapes(tuning):
    """Double precision with workgroups that walk one run of sink-operator
    groups in which one operator block stays, or a single group, with the
    lane-team engine, and with 1024-thread matrix-core workgroups, on every
    R52 channel."""
    announce("fp64 launch shapes %s" % tuning)
    L, T = (6, 4, 5), 2
    props = runner.host_props(L, T, range(T), dtype=np.complex128)
    chans = channels.r52()
    Fg = run_gpu(L, T, chans, props, binding.NBS_FP64, tuning=tuning)
    Fo = oracle_F(L, props, chans)
    err = rel_err_per_channel(Fg, Fo)
    assert err.max() <= 1e-12, (err.max(), int(err.argmax()))


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
def test_isospin_limit_builds_canonical_blocks_only(prec):
    """u and d given as the same memory: only p, n, Lambda, Sigma+, Sigma0,
    Xi0 blocks are built (Sec. 4(i)); every R52 channel against the oracle
    with S_d = S_u, and against the same propagators passed as two copies."""
    announce("isospin limit prec=%d" % prec)
    L, T = (4, 3, 2), 2
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, T, range(T), dtype=dt, same_ud=True)
    chans = channels.r52()
    Fi = run_gpu(L, T, chans, props, prec, alias_ud=True)
    Fc = run_gpu(L, T, chans, props, prec, alias_ud=False)
    Fo = oracle_F(L, props, chans)
    assert rel_err_per_channel(Fi, Fo).max() <= TOL[prec]
    assert rel_err_per_channel(Fi, Fc).max() <= TOL[prec]


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
@pytest.mark.parametrize("L", [(8, 8, 8), (16, 16, 16)])
def test_cube_pass(L, prec):
    """The one-pass transforms of 8^3 and 16^3 cubes (forward: the blocks,
    rounded where the separate passes round; inverse: the contiguous F
    fields) against the fused x-y pass with the z line pass, against three
    line passes (the same up to FP64 rounding order in the inverse) and
    against the oracle."""
    announce("cube pass %s prec=%d" % (L, prec))
    chans = [channels.r52()[c] for c in (0, 12, 22, 51)]
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, 2, range(1), dtype=dt)
    Fc = run_gpu(L, 2, chans, props, prec, t_count=1, tuning=dict(fft_cube=1, fft_plane=0))
    Fp = run_gpu(L, 2, chans, props, prec, t_count=1, tuning=dict(fft_cube=0, fft_plane=1))
    Fl = run_gpu(L, 2, chans, props, prec, t_count=1, tuning=dict(fft_cube=0, fft_plane=0))
    assert rel_err_per_channel(Fc, Fp).max() <= 1e-13
    assert rel_err_per_channel(Fc, Fl).max() <= 1e-13
    Fo = oracle_F(L, props, chans)
    err = rel_err_per_channel(Fc, Fo)
    assert err.max() <= TOL[prec], (err.max(), int(err.argmax()))
