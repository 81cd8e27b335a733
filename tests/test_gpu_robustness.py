"""Failure handling forced from the host (no kernel faults): device
allocation failures injected at every allocation of nbs_plan_create, and
propagators holding NaN or infinite entries."""
import os

import numpy as np
import pytest

from paper_1604_07983_amd import binding, channels, runner

pytestmark = pytest.mark.gpu


def announce(msg):
    print("[case] " + msg, flush=True)


def test_allocation_failure_at_every_allocation(monkeypatch):
    """NBS_TEST_FAIL_ALLOC=k fails the k-th device allocation of plan
    creation: every k up to the plan's allocation count returns
    NBS_ERR_NOMEM and frees what was allocated before it; the next k builds
    the plan."""
    import torch
    announce("allocation failure walk")
    geoms = [dict(L=(4, 3, 2), T=4, t_begin=0, t_count=2), dict(L=(2, 2, 2), T=2, t_begin=0, t_count=1)]
    chans = [("p", "p", "p", "p"), channels.WORKED_EXAMPLE]
    # one plan first: the runtime loads the library's code objects (and its
    # static workspace) on first use, which is not the plan's memory
    binding.Plan(None, None, chans, geoms=geoms).close()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    k = 1
    while True:
        monkeypatch.setenv("NBS_TEST_FAIL_ALLOC", str(k))
        try:
            p = binding.Plan(None, None, chans, geoms=geoms)
        except binding.NbsError as e:
            assert e.status == 3, (k, str(e))
            k += 1
            assert k < 64
            continue
        monkeypatch.delenv("NBS_TEST_FAIL_ALLOC")
        p.close()
        break
    assert k > 10  # per geometry blocks, F~, scale tables, momentum order; then the shared tables
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert abs(free1 - free0) < (8 << 20), (free0, free1)


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
def test_nonfinite_propagators_are_reported(prec):
    import torch
    announce("non-finite inputs prec=%d" % prec)
    L, T = (4, 3, 2), 2
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, T, range(T), dtype=dt)
    chans = [("p", "p", "p", "p"), ("Lambda", "Lambda", "Sigma+", "Sigma-")]
    r = runner.Runner(L, T, chans, prec=prec)
    dp = runner.device_props(props, prec)
    F = r.run(*dp)
    torch.cuda.synchronize()
    assert not r.plan.nonfinite()
    assert torch.isfinite(F).all()
    for bad in (complex(np.nan, 0.0), complex(0.0, np.inf)):
        props_bad = [p.copy() for p in props]
        props_bad[2][1, 1, 2, 3, 5, 7] = bad  # one entry of s on slice 1
        dpb = runner.device_props(props_bad, prec)
        F = r.run(*dpb)
        torch.cuda.synchronize()
        assert r.plan.nonfinite()
        # slice 0 does not see slice 1's input
        assert torch.isfinite(F[:, 0]).all()
    r.run(*dp)
    torch.cuda.synchronize()
    assert not r.plan.nonfinite()
    r.close()
