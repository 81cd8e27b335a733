"""Host tests of the channel-table compiler and the C ABI (no GPU work).

The compiled diagrams are checked against the paper's worked example, and
the compiled SoA program is executed on the CPU by tests/program_emulator.py
against the oracle's momentum-space correlators.
"""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import oracle
from paper_1604_07983_amd import binding, channels
from tests import physics_ref as ref
from tests import program_emulator as emu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def host_plan(chans, L=(4, 4, 4), T=8, prec=binding.NBS_FP64):
    return binding.Plan(L, T, chans, prec=prec, device=-1)


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "nbs.h")).read()
    declared = set(re.findall(r"^\s*(?:nbs_status|const char\*)\s+(nbs_\w+)\s*\(", hdr, re.M))
    assert declared == set(binding.SYMBOLS)
    lib = ctypes.CDLL(binding._LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def _open_names(mask):
    names = []
    for k in range(6):
        if (mask >> (2 * k)) & 1:
            names.append("c%d" % (k + 1))
        if (mask >> (2 * k + 1)) & 1:
            names.append("alpha%d" % (k + 1))
    return names


def test_worked_example_diagrams_match_paper():
    g = json.load(open(os.path.join(GOLDEN, "worked_example_pLambda_pXu.json")))
    p = host_plan([tuple(g["channel"])])
    ds = p.diagrams()
    got = sorted((tuple(sorted(_open_names(d["open_mask"]))),
                  tuple(l for b, l in ((1, "alpha3"), (2, "alpha4")) if d["labels1"] & b),
                  d["sign"]) for d in ds)
    want = sorted((tuple(sorted(x["open"])), tuple(x["first_block_labels"]), x["sign"])
                  for x in g["diagrams"])
    assert got == want
    info = p.info()
    assert info["sum_k"] == g["effective_iterations"]
    assert info["n_diagrams"] == 6
    # naive count (Nc! Na)^B Nu! Nd! Ns! 2^(NLambda+NSigma0-B) of Sec. 2
    assert 576 * info["n_wick_perms"] // 3 // 2 == g["naive_iterations"]


def test_r52_table_counts():
    """Regression values of the R52 reading (derived by enumeration)."""
    ch = channels.r52()
    assert len(ch) == 52 and len(set(ch)) == 52
    info = host_plan(ch).info()
    assert info["n_diagrams"] == 640
    assert info["sum_k"] == 41920
    assert info["n_wick_perms"] == 3376
    assert info["n_types"] == 8  # operator blocks: p n Lambda Sigma0 Sigma+ Sigma- Xi0 Xi-
    # every channel's Wick permutation count agrees with the oracle's enumeration
    total = sum(oracle.count_perms(c)[1] for c in ch)
    assert total == info["n_wick_perms"]


@pytest.mark.parametrize("chan", [("p", "p", "p", "p"), ("Lambda", "Lambda", "Sigma+", "Sigma-"),
                                  ("Xi0", "Sigma0", "Xi-", "Sigma+")])
def test_per_channel_wick_counts(chan):
    p = host_plan([chan])
    assert p.info()["n_wick_perms"] == oracle.count_perms(chan)[1]


def _momentum_operator_blocks(L, S, T):
    V = int(np.prod(L))
    trip = {}
    for s in range(len(T["op_code"])):
        for k in range(T["op_nterm"][s]):
            code = int(T["op_term_trip"][3 * s + k])
            if code not in trip:
                trip[code] = oracle.normal_blocks(L, S, code // 9, (code // 3) % 3, code % 3)
    ops = emu.operator_blocks(T, trip)
    return [oracle.dft3(o.reshape(V, 3456), L, -1) for o in ops]


def _neg(L, q):
    x, y, z = q % L[0], (q // L[0]) % L[1], q // (L[0] * L[1])
    return ((-x) % L[0]) + L[0] * (((-y) % L[1]) + L[1] * ((-z) % L[2]))


@pytest.mark.parametrize("prec", [binding.NBS_FP64, binding.NBS_FP32_MFMA])
@pytest.mark.parametrize("chans,L,qs", [
    ([channels.WORKED_EXAMPLE, ("p", "p", "p", "p")], (2, 2, 2), None),
    ([("Lambda", "Lambda", "Sigma+", "Sigma-"), ("Xi0", "Sigma0", "Xi-", "Sigma+"),
      ("n", "Xi0", "Lambda", "Lambda")], (2, 2, 2), [0, 3, 5]),
    (channels.r52(), (2, 3, 2), [0, 7]),
])
def test_compiled_program_reproduces_oracle(chans, L, qs, prec, mfma=False):
    """The compiled program, run by the CPU emulator with the kernel's rules,
    gives the oracle's F~(q) (built from explicit Wick permutations)."""
    rng = np.random.default_rng(101)
    S = ref.random_props(rng, L)
    p = host_plan(chans, L=L, T=4, prec=prec)
    if mfma:
        p.set_tuning(mfma=1)
    T = emu.tables(p)
    Nt = _momentum_operator_blocks(L, S, T)
    V = int(np.prod(L))
    for q in (qs if qs is not None else range(V)):
        mq = _neg(L, q)
        got = emu.emulate_q(T, [n[q] for n in Nt], [n[mq] for n in Nt], len(chans))
        qv = (q % L[0], (q // L[0]) % L[1], q // (L[0] * L[1]))
        want = oracle.correlators_at_q(L, S, chans, qv)
        err = np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)
        assert err.max() < 1e-12, (q, err.max(), int(err.argmax()))


@pytest.mark.parametrize("chans,L,qs", [
    ([channels.WORKED_EXAMPLE, ("p", "p", "p", "p")], (2, 2, 2), None),
    ([("Lambda", "Lambda", "Sigma+", "Sigma-"), ("Xi0", "Sigma0", "Xi-", "Sigma+"),
      ("n", "Xi0", "Lambda", "Lambda")], (2, 2, 2), [0, 3, 5]),
    (channels.r52(), (2, 3, 2), [0, 7]),
])
def test_segment_program_reproduces_oracle(chans, L, qs):
    """The matrix-core contraction's segment program, run lane by lane by the
    CPU emulator (block padding read as NaN, every result slot written once),
    gives the oracle's F~(q)."""
    rng = np.random.default_rng(103)
    S = ref.random_props(rng, L)
    p = host_plan(chans, L=L, T=4)
    T = emu.tables(p)
    T.update({n: p.table(n) for n in emu.SEG_NAMES})
    Nt = _momentum_operator_blocks(L, S, T)
    V = int(np.prod(L))
    for q in (qs if qs is not None else range(V)):
        mq = _neg(L, q)
        got = emu.emulate_q_seg(T, [n[q] for n in Nt], [n[mq] for n in Nt], len(chans))
        qv = (q % L[0], (q // L[0]) % L[1], q // (L[0] * L[1]))
        want = oracle.correlators_at_q(L, S, chans, qv)
        err = np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)
        assert err.max() < 1e-12, (q, err.max(), int(err.argmax()))


def test_segment_program_shapes_and_balance():
    """Every R52 product has a matrix-core shape; tasks hold four segments of
    one shape and step count; segments of a product cover its steps once."""
    p = host_plan(channels.r52())
    tasks = p.table("seg_task").reshape(-1, emu.SEG_TEAMS, emu.SEG_INTS)
    gs, gp, ext = p.table("group_stask"), p.table("group_prod"), p.table("prod_ext")
    full = {emu.SEG_C144: 36, emu.SEG_C9: 3, emu.SEG_C36: 9, emu.SEG_C1: 1}
    for g in range(len(gp) - 1):
        np_ = gp[g + 1] - gp[g]
        steps = {}
        for t in tasks[gs[g]:gs[g + 1]]:
            for d in t:
                if d[0] == emu.SEG_IDLE:
                    continue
                slot = int(d[3]) & 0xFFFF
                steps.setdefault(int(d[0]), []).append((slot, int(d[1]), int(d[2])))
        # map extra slots back to their products and check coverage
        owner = {p_: p_ for p_ in range(np_)}
        for p_ in range(np_):
            e = int(ext[gp[g] + p_])
            for k in range(e >> 16):
                owner[(e & 0xFFFF) + k] = p_
        cover = {}
        align = {emu.SEG_C144: 3, emu.SEG_C36: 3, emu.SEG_C9: 3, emu.SEG_C1: 1}
        for shape, segs in steps.items():
            for slot, s0, n in segs:
                # segments start and end where the kernel's per-lane pair
                # indices start a new value
                assert s0 % align[shape] == 0 and n % align[shape] == 0, (shape, s0, n)
                cover.setdefault(owner[slot], []).append((s0, n, shape))
        assert sorted(cover) == list(range(np_))
        for p_, segs in cover.items():
            shapes = {sh for _, _, sh in segs}
            assert len(shapes) == 1
            sh = shapes.pop()
            got = sorted(s for s0, n, _ in segs for s in range(s0, s0 + n))
            assert got == list(range(full[sh])), (g, p_)


# ---- ABI argument checking (host only) -------------------------------------

def _create(L=(4, 4, 4), T=8, chans=(("p", "p", "p", "p"),), prec=0, device=-1, n_geom=1, **kw):
    h = ctypes.c_void_p()
    g = binding.make_geometry(L, T, **kw)
    ch = binding.make_channels(list(chans))
    st = binding.lib().nbs_plan_create(ctypes.byref(h), ctypes.byref(g), n_geom, ch, len(chans), prec, device)
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(L=(7, 4, 4)), 1), (dict(L=(1, 4, 4)), 1), (dict(L=(256, 4, 4)), 1),
    (dict(T=8, t_begin=6, t_count=4), 1), (dict(T=8, t0=8), 1), (dict(prec=5), 1),
    (dict(chans=(("p", "p", "p", "n"),)), 1), (dict(chans=((0, 0, 0, 11),)), 1),
    (dict(n_geom=33), 2), (dict(n_geom=0), 1), (dict(device=-7), 1),
])
def test_plan_create_rejects_bad_arguments(kw, status):
    st, h = _create(**kw)
    assert st == status
    assert not h.value


def _create_many(geoms, device=-1):
    h = ctypes.c_void_p()
    arr = (binding.Geometry * len(geoms))()
    for i, g in enumerate(geoms):
        arr[i] = binding.make_geometry(**g)
    ch = binding.make_channels([("p", "p", "p", "p")])
    st = binding.lib().nbs_plan_create(ctypes.byref(h), arr, len(geoms), ch, 1, 1, device)
    return st, h


def test_batched_plan_takes_uneven_geometries():
    geoms = [dict(L=(24, 24, 24), T=48, t0=6 * k, t_begin=(6 * k + 3) % 48, t_count=1) for k in range(8)]
    geoms += [dict(L=(40, 40, 40), T=40, t0=5 * k, t_begin=(5 * k + 3) % 40, t_count=1) for k in range(8)]
    geoms += [dict(L=(6, 10, 9), T=8, t0=1, t_begin=0, t_count=8)]
    st, h = _create_many(geoms)
    assert st == 0 and h.value
    binding.lib().nbs_plan_destroy(h)


@pytest.mark.parametrize("bad", [dict(L=(7, 4, 4), T=8), dict(L=(4, 4, 4), T=8, t_begin=7, t_count=2)])
def test_batched_plan_rejects_any_bad_geometry(bad):
    geoms = [dict(L=(4, 4, 4), T=8), dict(L=(6, 6, 6), T=12), bad]
    st, h = _create_many(geoms)
    assert st == 1 and not h.value


def test_compute_calls_on_host_only_plan_are_state_errors():
    p = host_plan([("p", "p", "p", "p")])
    L = binding.lib()
    z = (ctypes.c_void_p * 1)(1)
    assert L.nbs_build_blocks(p.handle, z, z, z, None) == 5
    assert L.nbs_contract_channels(p.handle, None) == 5
    assert L.nbs_relative_sum(p.handle, z, None) == 5
    assert L.nbs_run_graph(p.handle, z, z, z, z, None) == 5
    assert L.nbs_plan_autotune(p.handle, z, z, z, None) == 5
    assert L.nbs_two_point(p.handle, None, 0, z, None) == 5
    assert b"host-only" in L.nbs_last_error(p.handle)
    tune = p.tuning()
    assert tune["fft_line"] == 1 and tune["fft_tile"] == 1024 and tune["split"] == 1 and tune["fft_plane"] == 1
    assert L.nbs_plan_destroy(None) == 0
    assert L.nbs_status_string(3) == b"out of device memory"


def test_precomputed_split_offsets():
    """Descriptor entries 20..47 (per-map LDS offsets the kernel uses for
    split products) against an independent derivation from masks and maps."""
    p = host_plan(channels.r52())
    desc = p.table("prod_desc").reshape(-1, p.params()["prod_ints"])
    n = 0
    for d in desc:
        if d[16] == 1:
            assert not d[20:].any()
            continue
        want = emu.split_offsets(d)
        assert np.array_equal(d[20:48], want), (d[:20], d[20:], want)
        n += 1
    assert n > 300


@pytest.mark.parametrize("lg", [2, 3, 4, 5, 6])
def test_team_reduce_scatter_owns_every_output_once(lg):
    """The kernel's team sums (DPP reduce-scatter, then cross-row adds),
    simulated lane by lane: every output of every team is written once, by a
    lane of that team, with the sum over the team's lanes."""
    rng = np.random.default_rng(lg)
    vals = rng.standard_normal((64, 16))
    out = emu.team_reduce(vals, lg)
    T = 1 << lg
    seen = {}
    for (lane, o), v in out.items():
        team = lane // T
        assert (team, o) not in seen
        seen[(team, o)] = v
    for team in range(64 // T):
        for o in range(16):
            assert np.isclose(seen[(team, o)], vals[team * T:(team + 1) * T, o].sum())


@pytest.mark.parametrize("lg", [4, 5, 6])
def test_quad_team_sums(lg):
    """Team sums of the matrix-core classes, simulated lane by lane: each of a
    team's 16 outputs is written once, with the sum over its quads."""
    rng = np.random.default_rng(10 + lg)
    vals = rng.standard_normal((64, 4))
    out = emu.quad_team_reduce(vals, lg)
    T = 1 << lg
    seen = {}
    for (lane, o), v in out.items():
        key = (lane // T, o)
        assert key not in seen
        seen[key] = v
    for team in range(64 // T):
        for o in range(16):
            i, j = divmod(o, 4)
            want = sum(vals[l, i] for l in range(team * T, (team + 1) * T) if l % 4 == j)
            assert np.isclose(seen[(team, o)], want)


def test_matrix_core_classes_only_where_enabled():
    """The matrix-core classes appear only in the precision form and only when
    the tuning enables them (the autotuner's candidate; off by default)."""
    p = host_plan(channels.r52(), prec=binding.NBS_FP32_MFMA)
    assert p.tuning()["mfma"] == 0
    c32 = (p.table("task_lanes") >> 26) & 31
    assert not ((c32 >= 20) & (c32 < 28)).any()
    q = host_plan(channels.r52())
    c64 = (q.table("task_lanes") >> 26) & 31
    assert not ((c64 >= 20) & (c64 < 28)).any()


def test_matrix_core_program_reproduces_oracle():
    """The precision form's program with matrix-core classes (quad teams)."""
    test_compiled_program_reproduces_oracle(channels.r52(), (2, 3, 2), [0, 7], binding.NBS_FP32_MFMA, mfma=True)
    p = host_plan(channels.r52(), prec=binding.NBS_FP32_MFMA)
    p.set_tuning(mfma=1)
    c = (p.table("task_lanes") >> 26) & 31
    assert ((c >= 20) & (c < 28)).mean() > 0.3


def test_set_tuning_rejects_bad_shapes():
    p = host_plan([("p", "p", "p", "p")])
    for kw in (dict(fft_tile=300), dict(waves=4), dict(mfma=1), dict(gchunk=3), dict(engine=0, waves=16),
               dict(engine=0, waves=8, persist=1)):
        with pytest.raises(binding.NbsError):
            p.set_tuning(**kw)
    # the matrix-core engine with 8-wavefront workgroups, one per work item,
    # by default
    assert p.tuning()["waves"] == 8 and p.tuning()["engine"] == 1 and p.tuning()["persist"] == 0
    p.set_tuning(persist=1)
    assert p.tuning()["persist"] == 1
    p.set_tuning(persist=0)
    p.set_tuning(engine=0, waves=8)
    assert p.tuning()["waves"] == 8 and p.tuning()["engine"] == 0


def test_transform_tuning_bits():
    """The block transform's shapes: the one-pass cube transform on by
    default in both forms, round-tripped with the other bits; unknown bits
    of the first word are rejected and leave the plan unchanged."""
    import ctypes
    for prec in (binding.NBS_FP64, binding.NBS_FP32_MFMA):
        p = host_plan([("p", "p", "p", "p")], prec=prec)
        t = p.tuning()
        assert t["fft_cube"] == 1 and t["fft_line"] == 1 and t["fft_plane"] == (1 if prec == binding.NBS_FP64 else 0)
        p.set_tuning(fft_cube=0, fft_plane=1)
        assert p.tuning()["fft_cube"] == 0 and p.tuning()["fft_plane"] == 1
        p.set_tuning(fft_cube=1)
        assert p.tuning()["fft_cube"] == 1 and p.tuning()["fft_plane"] == 1
        before = p.tuning()
        L = binding.lib()
        for word0 in (1 << 3, -1):
            arr = (ctypes.c_int32 * 4)(word0, before["fft_tile"], before["waves"], 1 | (1 << 4))
            assert L.nbs_plan_set_tuning(p.handle, arr) == 1  # NBS_ERR_INVALID
        assert p.tuning() == before


def test_group_range_modes():
    """Contraction workgroups per (slice, momentum): by default one that
    walks every group; every mode is accepted and reported back."""
    assert host_plan([("p", "p", "p", "p")]).tuning()["gchunk"] == 0
    p = host_plan(channels.r52(), prec=binding.NBS_FP32_MFMA)
    assert p.tuning()["gchunk"] == 0
    for m in (1, 2, 0):
        p.set_tuning(gchunk=m)
        assert p.tuning()["gchunk"] == m
    # the groups come in an order in which consecutive groups share an
    # operator block where possible: R52's 20 sink-operator pairs (7 operators
    # at +q, 8 at -q) are walked with 21 block loads, one per group plus the
    # first block, against 25 for the pairs in sorted order
    o1, o2 = p.table("group_op1"), p.table("group_op2")
    pairs = list(zip(o1.tolist(), o2.tolist()))
    assert len(set(pairs)) == len(pairs) == 20

    def loads(seq):
        return 2 + sum((a[0] != b[0]) + (a[1] != b[1]) for a, b in zip(seq, seq[1:]))
    assert loads(pairs) == 21 < loads(sorted(pairs))


def test_isospin_aliases_of_the_octet():
    """With S_d = S_u: Sigma- = Sigma+ and Xi- = -Xi0 as stored blocks
    (Sec. 4(i)); n = -p holds for the plain blocks, but the stored n block is
    antisymmetrised in its two d slots and the p block in its two u slots,
    so n is built.  The canonical slots come first."""
    p = host_plan(channels.r52())
    codes = list(p.table("op_code"))
    alias = p.table("op_alias")
    coef = p.table("op_alias_coef")
    name = {v: k for k, v in channels.OPS.items()}
    got = {name[c]: (name[codes[alias[s]]], coef[s]) for s, c in enumerate(codes) if alias[s] != s}
    assert got == {"Sigma-": ("Sigma+", 1.0), "Xi-": ("Xi0", -1.0)}
    canon = [s for s in range(len(codes)) if alias[s] == s]
    assert canon == list(range(len(canon))) and len(canon) == 6


def test_isospin_program_reproduces_oracle():
    """The aliased group tables on blocks of the canonical slots only, with
    S_d = S_u, against the oracle."""
    rng = np.random.default_rng(202)
    L = (2, 3, 2)
    S = ref.random_props(rng, L)
    S = [S[0], S[0], S[2]]
    chans = channels.r52()
    p = host_plan(chans, L=L, T=4)
    T = emu.tables(p)
    Nt = _momentum_operator_blocks(L, S, T)
    Ti = dict(T)
    Ti["group_op1"], Ti["group_op2"] = p.table("group_op1_iso"), p.table("group_op2_iso")
    Ti["contrib_coef"] = p.table("contrib_coef_iso")
    alias = p.table("op_alias")
    assert all(alias[s] < len([a for a in range(len(alias)) if alias[a] == a]) for s in range(len(alias)))
    for q in (0, 5):
        mq = _neg(L, q)
        got = emu.emulate_q(Ti, [n[q] for n in Nt], [n[mq] for n in Nt], len(chans))
        qv = (q % L[0], (q // L[0]) % L[1], q // (L[0] * L[1]))
        want = oracle.correlators_at_q(L, S, chans, qv)
        err = np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)
        assert err.max() < 1e-12, (q, err.max())


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built HIP library every entry point raises (no fallback)."""
    monkeypatch.setattr(binding, "_LIB_PATH", "/nonexistent/libnbs.so")
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(ImportError):
        binding.lib()
    with pytest.raises(ImportError):
        binding.Plan((4, 4, 4), 8, [("p", "p", "p", "p")], device=-1)
