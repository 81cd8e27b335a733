"""Benchmark of the NBS hot path on one MI355X.

A step is one pass of the whole path over one window of time slices:
nbs_build_blocks (normal blocks + forward 3-D FFT), nbs_contract_channels
(effective blocks and their products) and nbs_relative_sum (inverse FFT),
on synthetic seeded propagators already resident in HBM.

Default workload: plain FP64 form, 16^3 x 32 lattice, all 52 channels of the
R52 table, u, d, s propagators with decay rates 0.4 / 0.4 / 0.55.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    # name: (L, T, t_begin, t_count, prec, decay, label)
    "fp64_16c32": ((16, 16, 16), 32, 0, 32, 0, {"u": 0.4, "d": 0.4, "s": 0.55},
                   "plain FP64, 16^3x32, 52 channels (R52), u/d/s decay 0.4/0.4/0.55"),
    "fp32_32c64": ((32, 32, 32), 64, 0, 16, 1, {"u": 0.4, "d": 0.4, "s": 0.55},
                   "precision form (FP32 blocks/contractions, FP64 FFT), 32^3x64, 52 channels, "
                   "window of 16 slices"),
}

# The batching form: 24^3 x 48, 32^3 x 64 and 40^3 x 40 lattices, 8 source
# slices each (t0_k = k T / 8, seeds per source), the sink slice t0_k + 4,
# all 24 geometries in one plan and one captured graph, decay 0.45.
BATCH_LATTICES = (((24, 24, 24), 48), ((32, 32, 32), 64), ((40, 40, 40), 40))


def batch_geoms():
    out = []
    for L, T in BATCH_LATTICES:
        for k in range(8):
            t0 = k * T // 8
            out.append(dict(L=L, T=T, t0=t0, t_begin=(t0 + 4) % T, t_count=1))
    return out


PEAK = {"hbm": 8.0e12, "fp64": 78.6e12, "fp32_vector": 157.3e12}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="fp64_16c32", choices=sorted(CONFIGS) + ["batch_c4", "fp32_96c8"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (the reference kernel for HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of 1 GiB, five times: the FETCH_SIZE and
    WRITE_SIZE counters read on it give the scale between counter units and
    bytes actually moved."""
    import torch
    n = 1 << 30
    x = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}), flush=True)


def measured_traffic(config):
    """HBM bytes of one nbs_contract_channels call from the byte counters
    recorded in profiles/k_contract_traffic.json, or None when the kernel
    source has changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_contract_traffic.json")
    src = os.path.join(ROOT, "paper_1604_07983_amd", "csrc", "kernels.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != sha or config not in rec.get("configs", {}):
        return None
    return rec["configs"][config]["bytes_per_call"]


def program_work(plan):
    """Algorithmic work per momentum site of the contraction: (EBB flops,
    MEB flops).  EBB: every distinct effective-block entry is a sum of
    (real coefficient x complex block entry) terms, 4 flops each; MEB: each
    block product costs 16 complex multiply-adds per shared index, 8 flops
    each (products shared by several channels counted once)."""
    import numpy as np
    info = plan.info()
    desc = plan.table("prod_desc").reshape(-1, plan.params()["prod_ints"])
    return 4.0 * info["n_terms"], 8.0 * 16 * float(desc[:, 16].astype(np.int64).sum())


def cpu_baseline(L):
    """The oracle (DFT-correlation mode, all 52 channels) on one time slice of
    the workload's lattice (for lattices above 16^3, a 16^3 slice) with the
    same generator: a bounded sample of the per-site work."""
    import numpy as np
    import oracle
    from paper_1604_07983_amd import channels, runner
    L = tuple(min(x, 16) for x in L)
    props = runner.host_props(L, 32, [5])
    S = [np.ascontiguousarray(p[0].reshape(-1, 12, 12)) for p in props]
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        cores = min(cores, int(omp))
    t = time.perf_counter()
    oracle.correlators(L, S, channels.r52(), mode="fft")
    dt = time.perf_counter() - t
    V = L[0] * L[1] * L[2]
    return {"value": V * 52 / dt, "unit": "site-channels/s", "cores": cores, "kind": "oracle",
            "sample": "oracle DFT-correlation mode, all 52 channels, one slice of a %dx%dx%d lattice "
                      "(%d sites), %.1f s" % (L[0], L[1], L[2], V, dt)}


def time_two_point(r, stream, reps=10):
    """Zero-momentum two-point functions of the eight octet baryons from the
    built blocks (a by-product of the build stage, timed apart from the
    step): average time of one call over reps calls."""
    import torch
    pairs = [(b, b) for b in ("p", "n", "Lambda", "Sigma+", "Sigma0", "Sigma-", "Xi0", "Xi-")]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    r.two_point(pairs)
    ev[0].record(stream)
    for _ in range(reps):
        r.two_point(pairs)
    ev[1].record(stream)
    torch.cuda.synchronize()
    return {"pairs": len(pairs), "ms": ev[0].elapsed_time(ev[1]) / reps}


def bench_batch(args):
    """The batching form: one step = one launch of the captured graph over
    all 24 geometries (build, contraction in one launch, inverse transforms)."""
    import numpy as np
    import torch
    from paper_1604_07983_amd import binding, channels, runner
    geoms = batch_geoms()
    chans = channels.r52()
    decay = {"u": 0.45, "d": 0.45, "s": 0.45}
    print("[bench] generating propagators for %d geometries" % len(geoms), file=sys.stderr, flush=True)
    hprops = runner.host_props_many(geoms, decay=decay, dtype=np.complex64, workers=8)
    dprops = [runner.device_props(p, binding.NBS_FP32_MFMA) for p in hprops]
    del hprops
    br = runner.BatchRunner(geoms, chans, prec=binding.NBS_FP32_MFMA)
    print("[bench] autotune", file=sys.stderr, flush=True)
    tune = br.autotune(dprops)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        br.run_graph(dprops)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        br.run_graph(dprops)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    # the contraction alone, timed on the same stream, for the roofline
    ec = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ec[0].record(stream)
    for _ in range(args.steps):
        br.contract()
    ec[1].record(stream)
    torch.cuda.synchronize()
    contract_ms = ec[0].elapsed_time(ec[1]) / args.steps
    sites = sum(g["L"][0] * g["L"][1] * g["L"][2] * g["t_count"] for g in geoms)
    ebb_f, meb_f = program_work(br.plan)
    flops = (ebb_f + meb_f) * sites
    roof = {"bound": "alu", "achieved": flops / (contract_ms * 1e-3) / 1e12, "peak": PEAK["fp32_vector"] / 1e12,
            "unit": "TFLOP/s", "traffic": None, "kernel": "k_contract (effective blocks + products, all geometries)"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    out = {
        "metric": "NBS site-channels/sec + GFLOP/s, FP32-MFMA batched vs FP64 plain at stated rel err",
        "value": sites * len(chans) / (ms_step * 1e-3), "unit": "site-channels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batching form: 24^3x48, 32^3x64, 40^3x40 lattices x 8 source slices, one sink "
                               "slice each, 52 channels, complex64, decay 0.45, one captured graph",
                   "geometries": len(geoms), "channels": len(chans), "sites_per_step": sites, "tuning": tune},
        "stage_ms": {"graph_step": ms_step, "contract_channels": contract_ms},
        "roofline": roof,
    }
    br.close()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline((16, 16, 16))
    print(json.dumps(out), flush=True)


def bench_slab96(args):
    """One GPU's share of a time-split 96^3 x 64 run: slices 0..7, all 52
    channels, precision form.  One slice's blocks take 196 GB, so a step
    runs the three stages slice by slice on one single-slice plan (the
    output buffer is reused per slice)."""
    import numpy as np
    import torch
    from paper_1604_07983_amd import binding, channels, runner
    L, T, n_slices = (96, 96, 96), 64, 8
    chans = channels.r52()
    geoms = [dict(L=L, T=T, t0=0, t_begin=t, t_count=1, source=0) for t in range(n_slices)]
    print("[bench] generating 96^3 propagators for %d slices" % n_slices, file=sys.stderr, flush=True)
    hprops = runner.host_props_many(geoms, decay={"u": 0.4, "d": 0.4, "s": 0.55}, dtype=np.complex64, workers=8)
    dprops = [runner.device_props(hp, binding.NBS_FP32_MFMA) for hp in hprops]
    del hprops
    r = runner.Runner(L, T, chans, prec=binding.NBS_FP32_MFMA, t_begin=0, t_count=1)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        for t in range(n_slices):
            if ev is not None:
                ev[t][0].record(stream)
            r.build(*dprops[t])
            if ev is not None:
                ev[t][1].record(stream)
            r.contract()
            if ev is not None:
                ev[t][2].record(stream)
            r.relative_sum()
            if ev is not None:
                ev[t][3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)
    evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(n_slices)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
        print("[bench] step %d done" % k, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage = np.array([[[e[i].elapsed_time(e[i + 1]) for i in range(3)] for e in ek] for ek in evs])  # ms
    ms_step = wall * 1e3 / args.steps
    V = L[0] * L[1] * L[2]
    sites = V * n_slices
    two_point = time_two_point(r, stream)
    ebb_f, meb_f = program_work(r.plan)
    contract_ms = float(stage[:, :, 1].mean())
    roof = {"bound": "alu", "achieved": (ebb_f + meb_f) * V / (contract_ms * 1e-3) / 1e12,
            "peak": PEAK["fp32_vector"] / 1e12, "unit": "TFLOP/s", "traffic": None,
            "kernel": "k_contract (effective blocks + products)"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    out = {
        "metric": "NBS site-channels/sec + GFLOP/s, FP32-MFMA batched vs FP64 plain at stated rel err",
        "value": sites * len(chans) / (ms_step * 1e-3), "unit": "site-channels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "96^3 slab: slices 0-7 of T = 64, 52 channels, precision form, one slice at a time",
                   "lattice": list(L), "T": T, "slices": n_slices, "channels": len(chans), "sites_per_step": sites},
        "two_point": two_point,
        "stage_ms_per_slice": {"build_blocks": float(stage[:, :, 0].mean()), "contract_channels": contract_ms,
                               "relative_sum": float(stage[:, :, 2].mean())},
        "roofline": roof,
    }
    r.close()
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(a time-slice split would need no communication; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.config == "batch_c4":
        bench_batch(args)
        return
    if args.config == "fp32_96c8":
        bench_slab96(args)
        return
    import numpy as np
    import torch
    from paper_1604_07983_amd import binding, channels, runner

    L, T, tb, tc, prec, decay, label = CONFIGS[args.config]
    chans = channels.r52()
    V = L[0] * L[1] * L[2]
    dt = np.complex128 if prec == 0 else np.complex64
    print("[bench] generating propagators %s" % (L,), file=sys.stderr, flush=True)
    props = runner.host_props(L, T, range(tb, tb + tc), decay=decay, dtype=dt)
    dp = runner.device_props(props, prec)
    del props
    r = runner.Runner(L, T, chans, prec=prec, t_begin=tb, t_count=tc)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        r.build(*dp)
        if ev:
            ev[1].record(stream)
        r.contract()
        if ev:
            ev[2].record(stream)
        r.relative_sum()
        if ev:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(3)] for e in evs])  # ms
    ms_step = wall * 1e3 / args.steps
    sites = V * tc
    value = sites * len(chans) / (ms_step * 1e-3)

    two_point = time_two_point(r, stream)
    ebb_f, meb_f = program_work(r.plan)
    contract_ms = float(stage[:, 1].mean())
    contract_flops = (ebb_f + meb_f) * sites
    # FFT traffic: three passes, each reads and writes every block entry
    el = 16 if prec == 0 else 8
    n_types = r.plan.info()["n_types"]
    build_bytes = sites * (3 * 144 * el + n_types * 3456 * el * (1 + 2 * 3))
    total_flops = contract_flops + sites * (n_types * 3456 * 3 * 8 + n_types * 3456 * 5 * np.log2(V) * 1.0)
    roof = {"bound": "alu", "achieved": contract_flops / (contract_ms * 1e-3) / 1e12,
            "peak": PEAK["fp64"] / 1e12 if prec == 0 else PEAK["fp32_vector"] / 1e12,
            "unit": "TFLOP/s", "traffic": measured_traffic(args.config),
            "kernel": "k_contract (effective blocks + products)",
            "algorithmic_bytes": float(sites * n_types * 3456 * el + len(chans) * 16 * sites * el)}
    roof["frac"] = roof["achieved"] / roof["peak"]
    # whole-step roofline: per stage the larger of its algorithmic flops at
    # the vector peak and its algorithmic bytes at the HBM peak (propagators
    # read, blocks written once and transformed with one read and one write,
    # blocks read once by the contraction, F~ written, read and F written)
    peak = PEAK["fp64"] if prec == 0 else PEAK["fp32_vector"]
    blocks = sites * n_types * 3456 * el
    fields = sites * len(chans) * 16
    parts = {"build_blocks": max(sites * n_types * 3456 * (3 * 8 + 5 * np.log2(V)) / peak,
                                 (sites * 3 * 144 * el + 3 * blocks) / PEAK["hbm"]),
             "contract_channels": max(contract_flops / peak, (blocks + fields * el) / PEAK["hbm"]),
             "relative_sum": max(fields * 5 * np.log2(V) / PEAK["fp64"], fields * (el + 16) / PEAK["hbm"])}
    step_roof_ms = sum(parts.values()) * 1e3
    out = {
        "metric": "NBS site-channels/sec + GFLOP/s, FP32-MFMA batched vs FP64 plain at stated rel err",
        "value": value, "unit": "site-channels/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32", "data": "synthetic",
        "config": {"workload": label, "lattice": list(L), "T": T, "slices": tc, "channels": len(chans),
                   "sites_per_step": sites},
        "gflops": total_flops / (ms_step * 1e-3) / 1e9,
        "stage_ms": {"build_blocks": float(stage[:, 0].mean()), "contract_channels": contract_ms,
                     "relative_sum": float(stage[:, 2].mean())},
        "build_hbm_gbs": build_bytes / (stage[:, 0].mean() * 1e-3) / 1e9,
        "two_point": two_point,
        "roofline": roof,
        "step_roofline": {"ms": step_roof_ms, "frac": step_roof_ms / ms_step,
                          "parts_ms": {k: v * 1e3 for k, v in parts.items()}},
    }
    r.close()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(L)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
