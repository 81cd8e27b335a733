"""GPU parity of the batching form: one plan over several geometries
(uneven lattices, several source slices, different windows), contracted in
one launch, run eagerly, as a captured HIP graph, and after the autotuner
has picked launch shapes."""
import numpy as np
import pytest

import oracle
from paper_1604_07983_amd import binding, channels, runner
from tests.parity_util import flat_props, rel_err_per_channel

pytestmark = pytest.mark.gpu

DECAY45 = {"u": 0.45, "d": 0.45, "s": 0.45}
SUB = [0, 1, 2, 12, 22, 30, 51]  # channels of every strangeness sector


def announce(msg):
    print("[case] " + msg, flush=True)


def small_geoms():
    return [dict(L=(4, 4, 4), T=8, t0=0, t_begin=1, t_count=2),
            dict(L=(6, 4, 5), T=6, t0=3, t_begin=4, t_count=2),
            dict(L=(3, 5, 2), T=4, t0=1, t_begin=0, t_count=3),
            dict(L=(4, 4, 4), T=8, t0=4, t_begin=6, t_count=1)]


def geom_props(geoms, dtype, workers=1):
    return runner.host_props_many(geoms, decay=DECAY45, dtype=dtype, workers=workers)


def oracle_window(L, props, chans):
    tc = props[0].shape[0]
    return np.stack([oracle.correlators(L, flat_props(props, t), chans, mode="fft") for t in range(tc)], axis=1)


def check_against_oracle(geoms, hprops, F, chans, tol):
    for g, pr, Fg in zip(geoms, hprops, F):
        got = Fg.cpu().numpy()
        want = oracle_window(g["L"], pr, chans)
        err = rel_err_per_channel(got, want)
        assert err.max() <= tol, (g, float(err.max()), int(err.argmax()))


@pytest.mark.parametrize("prec,tol", [(binding.NBS_FP64, 1e-12), (binding.NBS_FP32_MFMA, 1e-5)])
def test_batch_uneven_lattices_match_oracle(prec, tol):
    import torch
    announce("batch of 4 uneven geometries, prec %d" % prec)
    geoms = small_geoms()
    chans = channels.r52()
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    hprops = geom_props(geoms, dt)
    dprops = [runner.device_props(p, prec) for p in hprops]
    br = runner.BatchRunner(geoms, chans, prec=prec)
    F = br.run(dprops)
    torch.cuda.synchronize()
    check_against_oracle(geoms, hprops, F, chans, tol)
    br.close()


@pytest.mark.parametrize("prec,tol", [(binding.NBS_FP64, 1e-12), (binding.NBS_FP32_MFMA, 1e-5)])
def test_batch_persistent_contraction(prec, tol):
    """Resident workgroups claiming (geometry, slice, momentum) items from
    the XCD counters, eagerly and in graph replays (the counters are reset
    by a fill kernel inside the graph)."""
    import torch
    announce("batch persistent contraction, prec %d" % prec)
    geoms = small_geoms()
    chans = [channels.r52()[c] for c in SUB]
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    hprops = geom_props(geoms, dt)
    dprops = [runner.device_props(p, prec) for p in hprops]
    br = runner.BatchRunner(geoms, chans, prec=prec)
    br.plan.set_tuning(persist=1)
    F = [f.clone() for f in br.run(dprops)]
    torch.cuda.synchronize()
    check_against_oracle(geoms, hprops, F, chans, tol)
    for rep in range(3):
        for f in br.F:
            f.fill_(float("nan"))
        br.run_graph(dprops)
        torch.cuda.synchronize()
        for a, b in zip(br.F, F):
            assert torch.equal(a, b), rep
    br.close()


def test_batch_graph_replays_match_eager():
    """Graph replays with eager work in between; every replay equals the
    eager result bit for bit; new output pointers trigger a new capture."""
    import torch
    announce("batch graph replays")
    geoms = small_geoms()
    chans = [channels.r52()[c] for c in SUB]
    prec = binding.NBS_FP32_MFMA
    hprops = geom_props(geoms, np.complex64)
    dprops = [runner.device_props(p, prec) for p in hprops]
    br = runner.BatchRunner(geoms, chans, prec=prec)
    eager = [f.clone() for f in br.run(dprops)]
    torch.cuda.synchronize()
    for rep in range(3):
        for f in br.F:
            f.fill_(float("nan"))
        br.run_graph(dprops)
        torch.cuda.synchronize()
        for a, b in zip(br.F, eager):
            assert torch.equal(a, b), rep
        # eager work of the program between replays
        br.run(dprops)
        torch.cuda.synchronize()
    br.F = [torch.empty_like(f) for f in br.F]
    br.run_graph(dprops)
    torch.cuda.synchronize()
    for a, b in zip(br.F, eager):
        assert torch.equal(a, b)
    br.close()


def test_autotune_keeps_parity():
    import torch
    announce("autotune on a batch")
    geoms = small_geoms()[:3]
    chans = channels.r52()
    prec = binding.NBS_FP32_MFMA
    hprops = geom_props(geoms, np.complex64)
    dprops = [runner.device_props(p, prec) for p in hprops]
    br = runner.BatchRunner(geoms, chans, prec=prec)
    tune = br.autotune(dprops)
    assert tune["waves"] in (4, 8) and tune["split"] in (0, 1) and tune["fft_line"] in (0, 1)
    assert tune["fft_tile"] in (512, 1024, 2048, 4096)
    F = br.run(dprops)
    torch.cuda.synchronize()
    check_against_oracle(geoms, hprops, F, chans, 1e-5)
    br.close()


def config4_geoms():
    """Batching workload: 24^3 x 48, 32^3 x 64, 40^3 x 40, each with 8 source
    slices t0_k = k T / 8 and the sink slice t0_k + 4 (mod T)."""
    out = []
    for L, T in (((24, 24, 24), 48), ((32, 32, 32), 64), ((40, 40, 40), 40)):
        for k in range(8):
            t0 = k * T // 8
            out.append(dict(L=L, T=T, t0=t0, t_begin=(t0 + 4) % T, t_count=1))
    return out


def test_config4_batch_full_size():
    """All 24 geometries in one plan (about 200 GB of blocks); two sources
    per lattice against the oracle at sampled momenta, all finite."""
    import torch
    torch.cuda.empty_cache()
    announce("batching form, 3 lattices x 8 sources")
    geoms = config4_geoms()
    chans = channels.r52()
    prec = binding.NBS_FP32_MFMA
    hprops = geom_props(geoms, np.complex64, workers=8)
    dprops = [runner.device_props(p, prec) for p in hprops]
    br = runner.BatchRunner(geoms, chans, prec=prec)
    F = br.run_graph(dprops)
    torch.cuda.synchronize()
    for i, g in enumerate(geoms):
        Fi = F[i]
        assert bool(torch.isfinite(Fi).all()), g
        if i % 8 not in (0, 5):
            continue
        L = g["L"]
        Fq = np.fft.fftn(Fi[:, 0].cpu().numpy(), axes=(2, 3, 4))
        S = flat_props(hprops[i], 0)
        for q in ((0, 0, 0), (1, L[1] - 2, 3)):
            want = oracle.correlators_at_q(L, S, chans, q)
            got = Fq[:, :, q[2], q[1], q[0]]
            err = np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)
            assert err.max() <= 1e-5, (g, q, float(err.max()), int(err.argmax()))
    br.close()


def test_tuning_cache_round_trip(tmp_path, monkeypatch):
    """Autotuned shapes land in the JSON cache under the architecture,
    precision, extents and channels; a second plan of the same shapes reads
    them back instead of measuring, and keeps parity."""
    import json

    import torch
    announce("tuning cache")
    monkeypatch.setenv("NBS_TUNE_CACHE", str(tmp_path / "tuning.json"))
    geoms = small_geoms()[:2]
    chans = [channels.r52()[c] for c in SUB]
    prec = binding.NBS_FP32_MFMA
    hprops = geom_props(geoms, np.complex64)
    dprops = [runner.device_props(p, prec) for p in hprops]
    br = runner.BatchRunner(geoms, chans, prec=prec)
    tune = br.autotune(dprops, cache=True)
    br.close()
    d = json.load(open(tmp_path / "tuning.json"))
    assert len(d) == 1
    key, val = next(iter(d.items()))
    assert key.startswith("gfx") and "|prec%d|" % prec in key and "4x4x4/8/2" in key
    assert val == {k: int(v) for k, v in tune.items()}
    # plant a distinct valid shape: the next plan must take it from the file
    val2 = dict(val, engine=1, waves=16 if (val["engine"], val["waves"]) == (1, 8) else 8)
    json.dump({key: val2}, open(tmp_path / "tuning.json", "w"))
    br = runner.BatchRunner(geoms, chans, prec=prec)
    assert br.autotune(dprops, cache=True) == val2
    F = br.run(dprops)
    torch.cuda.synchronize()
    check_against_oracle(geoms, hprops, F, chans, 1e-5)
    br.close()


@pytest.mark.parametrize("prec,tol", [(binding.NBS_FP64, 1e-12), (binding.NBS_FP32_MFMA, 1e-5)])
def test_batch_cubic_lattice_in_graph(prec, tol):
    """A cubic 8^3 geometry (the one-pass forward and inverse transforms)
    beside a non-cubic one (the separate passes) in one plan: eager run
    against the oracle, then graph replays with eager work in between, each
    equal to the eager result bit for bit."""
    import torch
    announce("batch with an 8^3 lattice, graph replays, prec %d" % prec)
    geoms = [dict(L=(8, 8, 8), T=4, t0=0, t_begin=1, t_count=2),
             dict(L=(6, 4, 5), T=6, t0=3, t_begin=4, t_count=1)]
    chans = [channels.r52()[c] for c in SUB]
    dt = np.complex128 if prec == binding.NBS_FP64 else np.complex64
    hprops = geom_props(geoms, dt)
    dprops = [runner.device_props(p, prec) for p in hprops]
    br = runner.BatchRunner(geoms, chans, prec=prec)
    assert br.plan.tuning()["fft_cube"] == 1
    eager = [f.clone() for f in br.run(dprops)]
    torch.cuda.synchronize()
    check_against_oracle(geoms, hprops, eager, chans, tol)
    for rep in range(3):
        for f in br.F:
            f.fill_(float("nan"))
        br.run_graph(dprops)
        torch.cuda.synchronize()
        for a, b in zip(br.F, eager):
            assert torch.equal(a, b), rep
        br.run(dprops)
        torch.cuda.synchronize()
    br.close()
