"""The allocation-free entry point (nbs_four_point_static) through the C ABI
against the plan path (nbs_plan_create + the three stages) on the same
inputs, two calls in a row, the second with a smaller input; and its size
limit.  The comparison bar is the plan path's own bar against the oracle:
1e-12 (FP64) and 1e-5 (precision form), norm-wise per channel and slice."""
import numpy as np
import pytest

from paper_1604_07983_amd import binding, channels, runner
from tests.parity_util import rel_err_per_channel

pytestmark = pytest.mark.gpu

TOL = {binding.NBS_FP64: 1e-12, binding.NBS_FP32_MFMA: 1e-5}


def announce(msg):
    print("[case] " + msg, flush=True)


def _both(L, T, chans, prec, t_count, seed_shift=0):
    import torch
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, T, range(t_count), dtype=dt, t0=0, source=seed_shift)
    dp = runner.device_props(props, prec)
    r = runner.Runner(L, T, chans, prec=prec, t_begin=0, t_count=t_count)
    Fp = r.run(*dp).clone()
    torch.cuda.synchronize()
    r.close()
    Fs = torch.full((len(chans), t_count, 16, L[2], L[1], L[0]), complex("nan"), dtype=torch.complex128,
                    device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    binding.four_point_static(L, T, chans, dp[0].data_ptr(), dp[1].data_ptr(), dp[2].data_ptr(), Fs.data_ptr(),
                              prec=prec, t_begin=0, t_count=t_count, stream=stream)
    torch.cuda.synchronize()
    return Fs.cpu().numpy(), Fp.cpu().numpy()


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
def test_static_path_matches_plan_path_twice(prec):
    chans = [("p", "p", "p", "p"), channels.WORKED_EXAMPLE, ("Lambda", "Lambda", "Sigma+", "Sigma-"),
             ("Xi0", "Sigma0", "Xi-", "Sigma+")]
    for k, (L, T, tc) in enumerate((((4, 3, 2), 4, 3), ((2, 3, 2), 2, 1))):
        announce("static path prec=%d call %d L=%s t_count=%d" % (prec, k, L, tc))
        Fs, Fp = _both(L, T, chans, prec, tc, seed_shift=k)
        assert np.isfinite(Fs).all()
        err = rel_err_per_channel(Fs, Fp)
        assert err.max() <= TOL[prec], (k, err.max())


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
def test_static_path_cubic_lattice(prec):
    """An 8^3 lattice (the one-pass forward and inverse transforms) through
    the workspace, pp only so that its blocks fit."""
    L, T, tc = (8, 8, 8), 2, 1
    announce("static path cubic prec=%d L=%s" % (prec, L))
    Fs, Fp = _both(L, T, [("p", "p", "p", "p")], prec, tc)
    assert np.isfinite(Fs).all()
    assert rel_err_per_channel(Fs, Fp).max() <= TOL[prec]


def test_static_path_rejects_too_large():
    import torch
    announce("static path size limit")
    L, T = (32, 32, 32), 2
    chans = channels.r52()
    x = torch.zeros(1, dtype=torch.complex128, device="cuda")
    with pytest.raises(binding.NbsError) as ei:
        binding.four_point_static(L, T, chans, x.data_ptr(), x.data_ptr(), x.data_ptr(), x.data_ptr(), t_count=1)
    assert ei.value.status == 2 and "MiB" in str(ei.value)
