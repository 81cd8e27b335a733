"""Run the three C-ABI stages on torch-owned device memory (marshalling only).

PyTorch provides the device buffers and the stream; every arithmetic step
happens inside libnbs's HIP kernels.
"""
from __future__ import annotations

import hashlib
import json
import os

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


def _props_job(args):
    L, T, ts, decay, t0, source, dtype = args
    return host_props(L, T, ts, decay=decay, t0=t0, source=source, dtype=dtype)


def host_props_many(geoms, decay=DECAY, dtype=np.complex128, workers=8):
    """host_props for every geometry (source index: the geometry's "source"
    key, else its position in the list), generated in a process pool."""
    jobs = [(tuple(g["L"]), g["T"], list(range(g.get("t_begin", 0), g.get("t_begin", 0) + g["t_count"])), decay,
             g.get("t0", 0), g.get("source", k), dtype) for k, g in enumerate(geoms)]
    if workers <= 1 or len(jobs) == 1:
        return [_props_job(j) for j in jobs]
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=min(workers, len(jobs)), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_props_job, jobs))


def tune_cache_path():
    """File of autotuned launch shapes: $NBS_TUNE_CACHE, else
    ~/.cache/nbs/tuning.json."""
    return os.environ.get("NBS_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "nbs", "tuning.json")


def _tune_key(plan, geoms):
    torch = _torch()
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    # launch shapes depend on the extents and window lengths, not on which
    # slices a window holds
    g = ";".join("%s/%d/%d" % ("x".join(map(str, x["L"])), x["T"], x.get("t_count") or x["T"]) for x in geoms)
    codes = [[binding.OPS[b] if isinstance(b, str) else int(b) for b in c] for c in plan.chans]
    ch = hashlib.sha256(np.asarray(codes, dtype=np.int32).tobytes()).hexdigest()[:16]
    return "%s|prec%d|%s|%s" % (arch, plan.prec, g, ch)


def _tune_cache_load():
    try:
        with open(tune_cache_path()) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _tune_cache_store(key, tune):
    path = tune_cache_path()
    d = _tune_cache_load()
    d[key] = {k: int(v) for k, v in tune.items()}
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


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

    def two_point(self, pairs):
        """C[pair, t, a, a'] (complex128, on the device) from the built blocks."""
        torch = _torch()
        C = torch.empty((len(pairs), self.t_count, 2, 2), dtype=torch.complex128, device="cuda")
        self.plan.two_point(pairs, C.data_ptr(), self.stream())
        return C

    def close(self):
        self.plan.close()


class BatchRunner:
    """The batching form: one plan over several geometries (uneven lattices,
    source slices, windows), one output buffer per geometry."""

    def __init__(self, geoms, chans, prec=binding.NBS_FP32_MFMA, device=0):
        torch = _torch()
        self.geoms = [dict(g) for g in geoms]
        self.plan = binding.Plan(None, None, chans, prec=prec, device=device, geoms=self.geoms)
        self.n_ch = len(chans)
        self.F = []
        for i, g in enumerate(self.geoms):
            L = g["L"]
            tc = self.plan.geoms[i].t_count
            self.F.append(torch.empty((self.n_ch, tc, 16, L[2], L[1], L[0]), dtype=torch.complex128, device="cuda"))

    def stream(self):
        return _torch().cuda.current_stream().cuda_stream

    @staticmethod
    def _split(props):
        return ([p[0].data_ptr() for p in props], [p[1].data_ptr() for p in props], [p[2].data_ptr() for p in props])

    def build(self, props):
        """props: per geometry the (u, d, s) device tensors."""
        self.plan.build_blocks(*self._split(props), self.stream())

    def contract(self):
        self.plan.contract_channels(self.stream())

    def relative_sum(self):
        self.plan.relative_sum([f.data_ptr() for f in self.F], self.stream())

    def run(self, props):
        self.build(props)
        self.contract()
        self.relative_sum()
        return self.F

    def two_point(self, pairs):
        """Per geometry C[pair, t, a, a'] (complex128, on the device)."""
        torch = _torch()
        C = [torch.empty((len(pairs), self.plan.geoms[i].t_count, 2, 2), dtype=torch.complex128, device="cuda")
             for i in range(len(self.geoms))]
        self.plan.two_point(pairs, [c.data_ptr() for c in C], self.stream())
        return C

    def run_graph(self, props):
        self.plan.run_graph(*self._split(props), [f.data_ptr() for f in self.F], self.stream())
        return self.F

    def autotune(self, props, cache=False):
        """nbs_plan_autotune with the caller's propagators; with cache=True
        the chosen shapes are kept in a JSON file keyed by (GPU architecture,
        precision, geometries, channels) and reused instead of measuring
        again."""
        key = _tune_key(self.plan, self.geoms) if cache else None
        if key is not None:
            hit = _tune_cache_load().get(key)
            if hit is not None:
                self.plan.set_tuning(**hit)
                # leave the plan built, as nbs_plan_autotune does
                self.build(props)
                return self.plan.tuning()
        self.plan.autotune(*self._split(props), self.stream())
        tune = self.plan.tuning()
        if key is not None:
            _tune_cache_store(key, tune)
        return tune

    def close(self):
        self.plan.close()


def sink_slice_phases(lattices):
    """Split the sink-slice windows of several lattices into phases: window w
    holds sink slice t0 + w of every source of the lattices with T > w, so a
    phase is a run of windows with the same set of lattices."""
    phases, w = [], 0
    maxT = max(T for _, T in lattices)
    while w < maxT:
        lats = [(tuple(L), T) for L, T in lattices if T > w]
        w_end = min(T for _, T in lats)
        phases.append((w, w_end, lats))
        w = w_end
    return phases


def sweep_sink_slices(lattices, n_sources, chans, decay, on_window, prec=binding.NBS_FP32_MFMA, autotune=False,
                      log=None):
    """Every sink slice of n_sources source slices (t0 = k T / n_sources) per
    lattice, as windows of one sink slice per geometry: one plan per phase
    (sink_slice_phases), its graph captured once on fixed input buffers that
    the device generator refills before each replay.  Source numbering: the
    k-th source of the i-th lattice is i * n_sources + k.  After each replay
    on_window(window, geoms, F, graph_ms) is called with the plan's outputs
    (F on the device; the caller drains what it needs before returning).
    Returns (graph milliseconds in total, windows, sites in total)."""
    torch = _torch()
    from . import synth_device
    stream = torch.cuda.current_stream()
    dt = torch.complex128 if prec == binding.NBS_FP64 else torch.complex64
    total_ms, n_win, n_sites = 0.0, 0, 0
    index = {(tuple(L), T): i for i, (L, T) in enumerate(lattices)}
    for w0, w1, lats in sink_slice_phases(lattices):
        geoms = []
        for L, T in lats:
            for k in range(n_sources):
                t0 = k * T // n_sources
                geoms.append(dict(L=L, T=T, t0=t0, t_begin=(t0 + w0) % T, t_count=1,
                                  source=index[(L, T)] * n_sources + k))
        if log:
            log("windows %d-%d: %d geometries" % (w0, w1 - 1, len(geoms)))
        bufs = [[torch.empty((1, g["L"][2], g["L"][1], g["L"][0], 12, 12), dtype=dt, device="cuda")
                 for _ in range(3)] for g in geoms]

        def fill(win):
            for g, b in zip(geoms, bufs):
                t = (g["t0"] + win) % g["T"]
                for f, name in enumerate("uds"):
                    synth_device.fill_slice(b[f], g["L"], t, f, decay[name], g["T"], t0=g["t0"], source=g["source"],
                                            stream=stream.cuda_stream)

        br = BatchRunner(geoms, chans, prec=prec)
        try:
            fill(w0)
            if autotune:
                br.autotune(bufs, cache=True)
            br.run_graph(bufs)  # the capture; later replays read the refilled buffers
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            for win in range(w0, w1):
                fill(win)
                e0.record(stream)
                br.run_graph(bufs)
                e1.record(stream)
                e1.synchronize()
                ms = e0.elapsed_time(e1)
                total_ms += ms
                n_win += 1
                n_sites += sum(g["L"][0] * g["L"][1] * g["L"][2] for g in geoms)
                on_window(win, geoms, br.F, ms)
        finally:
            br.close()
            del bufs
    return total_ms, n_win, n_sites
