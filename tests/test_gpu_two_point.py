"""GPU parity of the zero-momentum single-baryon two-point functions (a
by-product of the normal blocks: Eq. (1) with one baryon on each side, read
from the transformed blocks at q = 0) against the oracle, in both forms, in
the isospin-symmetric limit and in the batching form."""
import numpy as np
import pytest

import oracle
from paper_1604_07983_amd import binding, channels, runner
from tests.parity_util import flat_props

pytestmark = pytest.mark.gpu

TOL = {binding.NBS_FP64: 1e-12, binding.NBS_FP32_MFMA: 1e-5}
OCTET = ["p", "n", "Lambda", "Sigma+", "Sigma0", "Sigma-", "Xi0", "Xi-"]
MIXED = [("Lambda", "Sigma0"), ("Sigma0", "Lambda"), ("p", "n"), ("Xi0", "Xi-"), ("Lambda", "Xs"), ("Sigma+", "p")]


def announce(msg):
    print("[case] " + msg, flush=True)


def oracle_C(L, props, pairs):
    """[pair, t, 2, 2] from the oracle, slice by slice."""
    return np.stack([oracle.two_point(L, flat_props(props, t), pairs) for t in range(props[0].shape[0])], axis=1)


def check(got, want, tol):
    """Per pair and slice ||dC|| / ||C|| over the 2 x 2 spins; pairs whose
    oracle value vanishes (forbidden flavour content, or no mixing) against
    the largest diagonal magnitude of that slice."""
    scale = np.abs(want).reshape(want.shape[0], want.shape[1], -1).max(axis=(0, 2))
    for k in range(want.shape[0]):
        for t in range(want.shape[1]):
            d = np.linalg.norm(got[k, t] - want[k, t])
            n = np.linalg.norm(want[k, t])
            ref = n if n > 1e-9 * scale[t] else scale[t]
            assert d <= tol * ref, (k, t, d / ref)


def run(L, T, t_count, prec, pairs_list, alias_ud=False):
    import torch
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    props = runner.host_props(L, T, range(1, 1 + t_count), dtype=dt, same_ud=alias_ud)
    dp = runner.device_props(props, prec)
    if alias_ud:
        dp[1] = dp[0]
    r = runner.Runner(L, T, channels.r52(), prec=prec, t_begin=1, t_count=t_count)
    r.build(*dp)
    out = [r.two_point(pairs).cpu().numpy() for pairs in pairs_list]
    torch.cuda.synchronize()
    r.close()
    return props, out


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
def test_two_point_matches_oracle(prec):
    announce("two-point 4x4x4, 3 slices, prec %d" % prec)
    L = (4, 4, 4)
    diag = [(b, b) for b in OCTET]
    props, (Cd, Cm) = run(L, 8, 3, prec, [diag, MIXED])
    check(Cd, oracle_C(L, props, diag), TOL[prec])
    check(Cm, oracle_C(L, props, MIXED), TOL[prec])


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
def test_two_point_isospin_limit(prec):
    """u and d as the same memory: Sigma-, Xi- come from their aliases, n
    from its own block (equal to p's two-point function in this limit);
    Lambda and Sigma0 do not mix."""
    announce("two-point isospin limit, prec %d" % prec)
    L = (4, 4, 2)
    pairs = [("n", "n"), ("Sigma-", "Sigma-"), ("Xi-", "Xi-"), ("Lambda", "Sigma0"), ("p", "p")]
    props, (C,) = run(L, 6, 2, prec, [pairs], alias_ud=True)
    want = oracle_C(L, props, pairs)
    check(C, want, TOL[prec])
    np.testing.assert_allclose(C[0], C[4], rtol=0, atol=TOL[prec] * np.abs(C[4]).max() * 4)


def test_two_point_batch_geometries():
    import torch
    announce("two-point batching form")
    geoms = [dict(L=(4, 4, 4), T=8, t0=0, t_begin=1, t_count=2), dict(L=(6, 4, 5), T=6, t0=3, t_begin=4, t_count=2)]
    prec = binding.NBS_FP32_MFMA
    hprops = runner.host_props_many(geoms, decay={"u": 0.45, "d": 0.45, "s": 0.45}, dtype=np.complex64)
    dprops = [runner.device_props(p, prec) for p in hprops]
    br = runner.BatchRunner(geoms, channels.r52(), prec=prec)
    br.build(dprops)
    pairs = [(b, b) for b in OCTET]
    C = br.two_point(pairs)
    torch.cuda.synchronize()
    for g, pr, c in zip(geoms, hprops, C):
        check(c.cpu().numpy(), oracle_C(g["L"], pr, pairs), TOL[prec])
    br.close()


def test_two_point_argument_errors():
    announce("two-point errors")
    import torch
    r = runner.Runner((2, 2, 2), 2, [("p", "p", "p", "p")])
    with pytest.raises(binding.NbsError) as e:
        r.two_point([("p", "p")])
    assert e.value.status == 5  # before nbs_build_blocks
    props = runner.host_props((2, 2, 2), 2, range(2))
    r.build(*runner.device_props(props, binding.NBS_FP64))
    for pairs in ([("Lambda", "Lambda")], [("p", "p")] * 9, [(11, 0)]):
        with pytest.raises(binding.NbsError) as e:
            r.two_point(pairs)
        assert e.value.status == 1
    C = r.two_point([("p", "p")])
    torch.cuda.synchronize()
    check(C.cpu().numpy(), oracle_C((2, 2, 2), props, [("p", "p")]), 1e-12)
    r.close()
