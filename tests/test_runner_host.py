"""Host-side scheduling of the runner: the phases of a sweep over every sink
slice (no GPU needed)."""
from paper_1604_07983_amd import runner


def test_sink_slice_phases_batching_workload():
    lats = (((24, 24, 24), 48), ((32, 32, 32), 64), ((40, 40, 40), 40))
    ph = runner.sink_slice_phases(lats)
    assert [(a, b, [T for _, T in c]) for a, b, c in ph] == [(0, 40, [48, 64, 40]), (40, 48, [48, 64]),
                                                             (48, 64, [64])]
    # 8 sources per lattice: every (source, sink slice) pair exactly once
    assert sum((b - a) * len(c) * 8 for a, b, c in ph) == 8 * (48 + 64 + 40) == 1216


def test_sink_slice_phases_equal_extents():
    ph = runner.sink_slice_phases((((4, 4, 4), 6), ((6, 6, 6), 6)))
    assert [(a, b, len(c)) for a, b, c in ph] == [(0, 6, 2)]
