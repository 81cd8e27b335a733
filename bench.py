"""Benchmark of the NBS hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic input
already resident in HBM: nbs_build_blocks (normal blocks + forward 3-D FFT),
nbs_contract_channels (effective blocks and their products) and
nbs_relative_sum (inverse FFT).

The default run measures both forms the metric compares and prints one JSON
line:
  - plain FP64 (the line's `value`): 16^3 x 32 lattice, all 52 channels of the
    R52 table, u, d, s propagators decaying as exp(-0.4 t), exp(-0.4 t),
    exp(-0.55 t); a step covers the 32 slices;
  - batched FP32 (precision form, batching form): 24^3 x 48, 32^3 x 64 and
    40^3 x 40 lattices with 8 source slices each, decay 0.45; a step is one
    window, one sink slice of each of the 24 (lattice, source) geometries,
    run as one captured graph after the on-device autotuner.
The oracle (cpu_baseline leg) is timed on the host on one 16^3 slice of the
FP64 workload; the same oracle outputs give the FP64 leg's error per channel
over that whole slice, and the oracle at sampled momenta of two batched
geometries gives the FP32 leg's error per channel.

Other workloads: --config fp32_32c64 (precision form, 32^3 x 64, a window of
16 slices), batch_c4 (the batched leg alone), batch_c4_full (every sink slice
of the batching workload, window by window, inputs generated on the device),
fp32_96c8 (96^3 slab, slices 0-7, slice by slice), --copy-calibration (a
plain device copy, the reference kernel for the HBM byte counters).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NBS site-channels/sec + GFLOP/s, FP32-MFMA batched vs FP64 plain at stated rel err"

PLAIN = {
    # name: (L, T, t_begin, t_count, prec, decay, label)
    "fp64_16c32": ((16, 16, 16), 32, 0, 32, 0, {"u": 0.4, "d": 0.4, "s": 0.55},
                   "plain FP64, 16^3x32, 52 channels (R52), u/d/s decay 0.4/0.4/0.55, all 32 slices per step"),
    "fp32_32c64": ((32, 32, 32), 64, 0, 16, 1, {"u": 0.4, "d": 0.4, "s": 0.55},
                   "precision form (FP32 blocks/contractions, FP64 FFT), 32^3x64, 52 channels, "
                   "window of 16 slices per step"),
}

# The batching form: 24^3 x 48, 32^3 x 64 and 40^3 x 40 lattices, 8 source
# slices each (t0_k = k T / 8, seeds per source); one window = one sink slice
# of every geometry, t0_k + 4 (mod T) by default.
BATCH_LATTICES = (((24, 24, 24), 48), ((32, 32, 32), 64), ((40, 40, 40), 40))
BATCH_DECAY = {"u": 0.45, "d": 0.45, "s": 0.45}

PEAK = {"hbm": 8.0e12, "fp64": 78.6e12, "fp32_mfma": 157.3e12}


def batch_geoms(sep=4):
    out = []
    for L, T in BATCH_LATTICES:
        for k in range(8):
            t0 = k * T // 8
            out.append(dict(L=L, T=T, t0=t0, t_begin=(t0 + sep) % T, t_count=1, source=k))
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="default",
                    choices=["default"] + sorted(PLAIN) + ["batch_c4", "batch_c4_full", "fp32_96c8"])
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (no cpu_baseline and no rel err)")
    ap.add_argument("--no-batched", action="store_true", help="default workload without the batched FP32 leg")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched leg with the default launch shapes (no on-device autotuner, no tuning cache)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (the reference kernel for HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


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


def contraction_work(plan):
    """Work per momentum site of one slice, from the compiled channel table:
    (algorithmic flops, flops with products shared across channels, bytes).
      products (Eq. (10)): 8 flops per complex multiply-add, 16 per shared
        index of every diagram (sum over diagrams of |xi~_d|), or of every
        distinct product when products shared by channels count once;
      effective blocks (Eq. (9)): 2 flops per (sign x block entry) term of
        every effective-block entry the products read;
      bytes: the operator blocks read once and F~ written once."""
    import numpy as np
    info = plan.info()
    desc = plan.table("prod_desc").reshape(-1, plan.params()["prod_ints"])
    K = desc[:, 16].astype(np.int64)
    rows1 = desc[:, 18].astype(np.int64)

    def nterms(mask):
        out = np.ones(len(mask), dtype=np.int64)
        for h in range(2):
            bits = (mask >> (3 * h)) & 7
            n = ((bits & 1) + ((bits >> 1) & 1) + ((bits >> 2) & 1))
            lone2 = (n == 2) & ((bits & 4) == 0)  # the baryon's third quark is the lone one
            out *= np.where(n == 3, 24, np.where(n == 2, np.where(lone2, 8, 2), 1))
        return out

    terms = (K * (rows1 * nterms(desc[:, 0].astype(np.int64)) +
                  (16 // rows1) * nterms(desc[:, 8].astype(np.int64)))).sum()
    ebb = 2.0 * float(terms)
    meb = 8.0 * 16 * float(info["sum_k"])
    meb_shared = 8.0 * 16 * float(K.sum())
    return ebb + meb, ebb + meb_shared, ebb, meb


def roofline(prec, flops_site, flops_shared_site, sites, t_ms, traffic):
    peak = PEAK["fp64"] if prec == 0 else PEAK["fp32_mfma"]
    ach = flops_site * sites / (t_ms * 1e-3)
    out = {"bound": "mfma", "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
           "frac": ach / peak, "traffic": traffic,
           "kernel": "k_contract_seg (effective blocks and their products, matrix cores)",
           "flops_per_site": flops_site,
           "frac_products_shared": flops_shared_site * sites / (t_ms * 1e-3) / peak}
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    return min(cores, int(omp)) if omp else cores


def rel_err_channels(got, want):
    """Per channel: ||got - want|| / ||want|| over the remaining axes."""
    import numpy as np
    d = (got - want).reshape(got.shape[0], -1)
    w = want.reshape(want.shape[0], -1)
    return np.linalg.norm(d, axis=1) / np.linalg.norm(w, axis=1)


def plain_leg(args, name):
    """One geometry, all slices of the window per step."""
    import numpy as np
    import torch
    from paper_1604_07983_amd import binding, channels, runner

    L, T, tb, tc, prec, decay, label = PLAIN[name]
    chans = channels.r52()
    V = L[0] * L[1] * L[2]
    dt = np.complex128 if prec == 0 else np.complex64
    log("generating propagators %s x %d slices" % (L, tc))
    props = runner.host_props(L, T, range(tb, tb + tc), decay=decay, dtype=dt)
    dp = runner.device_props(props, prec)
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
    log("%s warmup done" % name)
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
    # complex entries per site of the stored operator blocks: operators with
    # a same-flavour slot pair are stored antisymmetrised and packed (1584),
    # the others whole (3456)
    stored = int(sum(1584 if pr >= 0 else 3456 for pr in r.plan.table("op_pair")))
    tune = r.plan.tuning()
    fl, fl_sh, ebb, meb = contraction_work(r.plan)
    contract_ms = float(stage[:, 1].mean())
    el = 16 if prec == 0 else 8
    passes = 1 + 2 * transform_passes(tune, L)
    build_bytes = sites * (3 * 144 * el + stored * el * passes)
    blocks = sites * stored * el
    fields = sites * len(chans) * 16
    peak = PEAK["fp64"] if prec == 0 else PEAK["fp32_mfma"]
    # whole-step roofline: per stage the larger of its flops at the peak and
    # its algorithmic bytes at the HBM peak (propagators read, blocks written
    # once and transformed with one read and one write, blocks read once by
    # the contraction, F~ written, read and F written)
    parts = {"build_blocks": max(sites * stored * (3 * 8 + 5 * np.log2(V)) / peak,
                                 (sites * 3 * 144 * el + 3 * blocks) / PEAK["hbm"]),
             "contract_channels": max(fl * sites / peak, (blocks + fields * el) / PEAK["hbm"]),
             "relative_sum": max(fields * 5 * np.log2(V) / PEAK["fp64"], fields * (el + 16) / PEAK["hbm"])}
    step_roof_ms = sum(parts.values()) * 1e3
    total_flops = fl * sites + sites * stored * (3 * 8 + 5 * np.log2(V)) + fields * 5 * np.log2(V)
    leg = {
        "workload": label, "lattice": list(L), "T": T, "slices": tc, "channels": len(chans),
        "sites_per_step": sites, "ms_per_step": ms_step, "value": sites * len(chans) / (ms_step * 1e-3),
        "unit": "site-channels/s", "dtype": "f64" if prec == 0 else "f32",
        "gflops": total_flops / (ms_step * 1e-3) / 1e9,
        "stage_ms": {"build_blocks": float(stage[:, 0].mean()), "contract_channels": contract_ms,
                     "relative_sum": float(stage[:, 2].mean())},
        "build_hbm_gbs": build_bytes / (stage[:, 0].mean() * 1e-3) / 1e9,
        "build_block_passes": passes,
        "roofline": roofline(prec, fl, fl_sh, sites, contract_ms, measured_traffic(name)),
        "step_roofline": {"ms": step_roof_ms, "frac": step_roof_ms / ms_step,
                          "parts_ms": {k: v * 1e3 for k, v in parts.items()}},
        "tuning": tune,
        "two_point": time_two_point(r, stream),
    }
    # the sample the oracle checks: one slice of the output
    ts = min(5, tc - 1)
    sample = {"L": L, "S": [np.ascontiguousarray(p[ts].reshape(-1, 12, 12).astype(np.complex128)) for p in props],
              "F": r.F[:, ts].cpu().numpy(), "chans": chans, "slice": tb + ts}
    r.close()
    del dp
    return leg, sample


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


def batch_leg(args):
    """The batching form: a step is one launch of the captured graph over the
    24 geometries of one window (build, one contraction launch over all
    geometries, inverse transforms)."""
    import numpy as np
    import torch
    from paper_1604_07983_amd import binding, channels, runner
    geoms = batch_geoms()
    chans = channels.r52()
    log("generating propagators for %d geometries" % len(geoms))
    hprops = runner.host_props_many(geoms, decay=BATCH_DECAY, dtype=np.complex64, workers=8)
    dprops = [runner.device_props(p, binding.NBS_FP32_MFMA) for p in hprops]
    # the oracle's sample: the 24^3 geometry of source 0 and the 32^3 one of
    # source 3, host copies of their inputs
    pick = [0, 11]
    S_sample = {i: [np.ascontiguousarray(p[0].reshape(-1, 12, 12).astype(np.complex128)) for p in hprops[i]]
                for i in pick}
    del hprops
    br = runner.BatchRunner(geoms, chans, prec=binding.NBS_FP32_MFMA)
    if args.no_autotune:
        tune = br.plan.tuning()
    else:
        log("autotune (or the tuning cache)")
        tune = br.autotune(dprops, cache=True)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        br.run_graph(dprops)
    torch.cuda.synchronize()
    log("batched warmup done")
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
    F_sample = {i: br.F[i][:, 0].cpu().numpy() for i in pick}
    # the contraction alone, timed on the same stream, for the roofline
    ec = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ec[0].record(stream)
    for _ in range(args.steps):
        br.contract()
    ec[1].record(stream)
    torch.cuda.synchronize()
    contract_ms = ec[0].elapsed_time(ec[1]) / args.steps
    sites = sum(g["L"][0] * g["L"][1] * g["L"][2] * g["t_count"] for g in geoms)
    fl, fl_sh, _, _ = contraction_work(br.plan)
    leg = {
        "workload": "batching form: 24^3x48, 32^3x64, 40^3x40 lattices x 8 source slices (t0 = k T / 8), "
                    "one sink slice each (t0 + 4) per step, 52 channels, complex64, decay 0.45, one captured graph",
        "geometries": len(geoms), "channels": len(chans), "sites_per_step": sites, "ms_per_step": ms_step,
        "value": sites * len(chans) / (ms_step * 1e-3), "unit": "site-channels/s", "dtype": "f32",
        "stage_ms": {"graph_step": ms_step, "contract_channels": contract_ms},
        "roofline": roofline(1, fl, fl_sh, sites, contract_ms, measured_traffic("batch_c4")),
        "tuning": tune,
    }
    br.close()
    del dprops
    sample = {"geoms": [geoms[i] for i in pick], "S": [S_sample[i] for i in pick], "F": [F_sample[i] for i in pick],
              "chans": chans}
    return leg, sample


def cpu_baseline(fp64_sample, batch_sample):
    """The oracle on the host cores: all 52 channels of one 16^3 slice of the
    FP64 workload (timed; DFT-correlation mode), which also gives the FP64
    leg's error per channel over that whole slice; and the oracle's F~(q) at
    two momenta of two batched geometries for the FP32 leg's error per
    channel (max over the samples)."""
    import numpy as np
    import oracle
    L, S, chans = fp64_sample["L"], fp64_sample["S"], fp64_sample["chans"]
    t = time.perf_counter()
    Fo = oracle.correlators(L, S, chans, mode="fft")
    dt = time.perf_counter() - t
    V = L[0] * L[1] * L[2]
    cores = host_cores()
    base = {"value": V * len(chans) / dt, "unit": "site-channels/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "oracle DFT-correlation mode, all 52 channels, slice %d of the 16^3 x 32 FP64 workload "
                      "(%d sites), %.1f s on %d threads" % (fp64_sample["slice"], V, dt, cores)}
    err64 = rel_err_channels(fp64_sample["F"], Fo)
    errs = {"fp64_plain": {"max": float(err64.max()), "per_channel": [float(e) for e in err64],
                           "over": "every r and spin of slice %d (norm-wise per channel)" % fp64_sample["slice"]}}
    if batch_sample is not None:
        qs = ((0, 0, 0), (3, 1, 2))
        per = np.zeros(len(batch_sample["chans"]))
        for g, S, F in zip(batch_sample["geoms"], batch_sample["S"], batch_sample["F"]):
            Fq = np.fft.fftn(F, axes=(2, 3, 4))  # [c, 16, qz, qy, qx]
            for q in qs:
                want = oracle.correlators_at_q(g["L"], S, batch_sample["chans"], q)
                got = Fq[:, :, q[2], q[1], q[0]]
                per = np.maximum(per, rel_err_channels(got, want))
        errs["fp32_batched"] = {"max": float(per.max()), "per_channel": [float(e) for e in per],
                                "over": "F~(q) at q = (0,0,0), (3,1,2) of the 24^3 source-0 and 32^3 source-3 "
                                        "geometries, 16 spins (norm-wise per channel)"}
    return base, errs


def bench_default(args):
    fp64, s64 = plain_leg(args, "fp64_16c32")
    fp32b, sb = (None, None) if args.no_batched else batch_leg(args)
    out = {
        "metric": METRIC, "value": fp64["value"], "unit": "site-channels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": fp64["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": fp64["workload"], "lattice": fp64["lattice"], "T": fp64["T"],
                   "slices": fp64["slices"], "channels": fp64["channels"],
                   "sites_per_step": fp64["sites_per_step"]},
        "gflops": fp64["gflops"],
        "roofline": fp64["roofline"],
        "legs": {"fp64_plain": fp64},
    }
    if fp32b is not None:
        out["legs"]["fp32_batched"] = fp32b
        out["batched_fp32_vs_fp64_plain"] = fp32b["value"] / fp64["value"]
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"], out["rel_err"] = cpu_baseline(s64, sb)
    print(json.dumps(out), flush=True)


def bench_plain(args):
    leg, sample = plain_leg(args, args.config)
    out = {"metric": METRIC, "value": leg["value"], "unit": "site-channels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": leg["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": leg["dtype"], "data": "synthetic",
           "config": {"workload": leg["workload"], "lattice": leg["lattice"], "T": leg["T"], "slices": leg["slices"],
                      "channels": leg["channels"], "sites_per_step": leg["sites_per_step"]},
           "gflops": leg["gflops"], "roofline": leg["roofline"], "legs": {args.config: leg}}
    print(json.dumps(out), flush=True)


def bench_batch(args):
    leg, _ = batch_leg(args)
    out = {"metric": METRIC, "value": leg["value"], "unit": "site-channels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": leg["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": leg["workload"], "geometries": leg["geometries"], "channels": leg["channels"],
                      "sites_per_step": leg["sites_per_step"]},
           "roofline": leg["roofline"], "legs": {"fp32_batched": leg}}
    print(json.dumps(out), flush=True)


def bench_batch_full(args):
    """The batching workload in full: every sink slice of the 8 sources of
    each lattice (24^3 x 48, 32^3 x 64, 40^3 x 40: 1216 slice-geometries) as
    windows of one sink slice per geometry (a step is one window: one replay
    of the plan's captured graph on input buffers that the device generator
    refills between replays), F drained per window into sums of |F|^2 per
    (lattice, source, sink slice, channel).  The rate counts graph time only;
    generation and draining are reported beside it."""
    import numpy as np
    import torch
    from paper_1604_07983_amd import binding, channels, runner
    chans = channels.r52()
    checks = {}

    def drain(win, geoms, F, ms):
        sums = [(f.abs() ** 2).sum(dim=(1, 2, 3, 4, 5)).cpu().numpy() for f in F]
        for g, sm in zip(geoms, sums):
            checks[(g["L"][0], g["source"], (g["t0"] + win) % g["T"])] = sm
        if win % 8 == 0:
            log("window %d: %.1f ms" % (win, ms))

    t_wall = time.perf_counter()
    graph_ms, n_win, sites = runner.sweep_sink_slices(BATCH_LATTICES, 8, chans, BATCH_DECAY, drain,
                                                      prec=binding.NBS_FP32_MFMA, autotune=not args.no_autotune,
                                                      log=log)
    wall = time.perf_counter() - t_wall
    keys = sorted(checks)
    table = np.stack([checks[k] for k in keys])
    assert np.isfinite(table).all()
    digest = hashlib.sha256(np.ascontiguousarray(table).tobytes()).hexdigest()
    per_lat = {"%d^3" % L[0]: float(sum(checks[k].sum() for k in keys if k[0] == L[0])) for L, _ in BATCH_LATTICES}
    out = {
        "metric": METRIC, "value": sites * len(chans) / (graph_ms * 1e-3), "unit": "site-channels/s",
        "n_gpus": 1, "steps": n_win, "warmup": 0, "ms_per_step": graph_ms / n_win, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic (generated on the device)",
        "config": {"workload": "batching form in full: every sink slice of 8 sources on 24^3x48, 32^3x64, 40^3x40 "
                               "(1216 slice-geometries), windows of one sink slice per geometry, 52 channels, "
                               "complex64, decay 0.45", "slice_geometries": len(keys), "windows": n_win,
                   "sites": sites},
        "graph_ms_total": graph_ms, "wall_s_with_capture_generation_draining": wall,
        "checksums": {"sum_abs2_per_lattice": per_lat, "table_sha256": digest,
                      "table": "sum over r and spins of |F|^2 per (lattice, source, sink slice, channel)"},
    }
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
    log("generating 96^3 propagators for %d slices" % n_slices)
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
    log("warmup done")
    evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(n_slices)]
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
        log("step %d done" % k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage = np.array([[[e[i].elapsed_time(e[i + 1]) for i in range(3)] for e in ek] for ek in evs])  # ms
    ms_step = wall * 1e3 / args.steps
    V = L[0] * L[1] * L[2]
    sites = V * n_slices
    fl, fl_sh, _, _ = contraction_work(r.plan)
    contract_ms = float(stage[:, :, 1].mean())
    out = {
        "metric": METRIC, "value": sites * len(chans) / (ms_step * 1e-3), "unit": "site-channels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "96^3 slab: slices 0-7 of T = 64, 52 channels, precision form, one slice at a time",
                   "lattice": list(L), "T": T, "slices": n_slices, "channels": len(chans), "sites_per_step": sites},
        "two_point": time_two_point(r, stream),
        "stage_ms_per_slice": {"build_blocks": float(stage[:, :, 0].mean()), "contract_channels": contract_ms,
                               "relative_sum": float(stage[:, :, 2].mean())},
        "roofline": roofline(1, fl, fl_sh, V, contract_ms, None),
    }
    r.close()
    print(json.dumps(out), flush=True)


def transform_passes(tune, L):
    """HBM passes (one read and one write of the blocks each) of the forward
    block transform: one for 8^3 and 16^3 cubes with the one-pass kernel on,
    two with the fused x-y pass on a square plane, else three line passes."""
    if tune["fft_cube"] and L[0] == L[1] == L[2] and L[0] in (8, 16):
        return 1
    if tune["fft_plane"] and L[0] == L[1] and L[0] in (8, 16, 24, 32, 40):
        return 2
    return 3


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: nothing here uses a second GPU (a split by time slice would need "
              "no communication between GPUs)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
    elif args.config == "default":
        bench_default(args)
    elif args.config == "batch_c4":
        bench_batch(args)
    elif args.config == "batch_c4_full":
        bench_batch_full(args)
    elif args.config == "fp32_96c8":
        bench_slab96(args)
    else:
        bench_plain(args)


if __name__ == "__main__":
    main()
