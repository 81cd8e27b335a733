"""Channel tables from quantum numbers and from text (host only)."""
import os

import pytest

from paper_1604_07983_amd import binding, channels

QUARKS = {"p": "uud", "n": "udd", "Lambda": "uds", "Sigma+": "uus", "Sigma0": "uds", "Sigma-": "dds",
          "Xi0": "uss", "Xi-": "dss"}


def test_octet_quantum_numbers_follow_the_quark_content():
    for b, (S, tz) in channels.OCTET.items():
        q = QUARKS[b]
        assert S == -q.count("s")
        assert tz == q.count("u") - q.count("d")


def test_every_sector_compiles():
    """All channels of every (S, I_z) sector: flavour is conserved, so the
    channel compiler accepts the whole list."""
    total = 0
    for S, tz in channels.sectors():
        ch = channels.coupled_channels(S, tz)
        p = binding.Plan((4, 4, 4), 8, ch, device=-1)
        assert p.info()["n_channels"] == len(ch)
        total += len(ch)
    assert total > 52


def test_r52_rows_lie_in_generated_sectors():
    """Each R52 row is a channel of the sector of its sink pair (with the
    pairs taken in either order)."""
    for b1, b2, b3, b4 in channels.r52():
        S = channels.OCTET[b1][0] + channels.OCTET[b2][0]
        tz = channels.OCTET[b1][1] + channels.OCTET[b2][1]
        gen = set(channels.coupled_channels(S, tz, ordered=True))
        assert (b1, b2, b3, b4) in gen


def test_sector_sizes():
    assert channels.octet_pairs(0, 2) == [("p", "p")]
    assert channels.octet_pairs(0, 0) == [("p", "n")]
    assert sorted(channels.octet_pairs(-1, 1)) == sorted([("p", "Lambda"), ("p", "Sigma0"), ("n", "Sigma+")])
    assert len(channels.coupled_channels(-2, 0)) == len(channels.octet_pairs(-2, 0)) ** 2
    assert len(channels.octet_pairs(-2, 0)) == 6  # Lambda Lambda, Lambda Sigma0, Sigma0 Sigma0, Sigma+ Sigma-, p Xi-, n Xi0


def test_parse_and_load_table(tmp_path):
    text = "# a small table\np p p p\nLambda, Lambda, Sigma+, Sigma-   # coupled\n\n"
    assert channels.parse_table(text) == [("p", "p", "p", "p"), ("Lambda", "Lambda", "Sigma+", "Sigma-")]
    f = tmp_path / "t.txt"
    f.write_text("\n".join(" ".join(c) for c in channels.r52()))
    assert channels.load_table(str(f)) == channels.r52()
    with pytest.raises(ValueError):
        channels.parse_table("p p p Omega")
    with pytest.raises(ValueError):
        channels.parse_table("p p p")


def test_non_conserving_table_is_rejected_by_the_compiler():
    with pytest.raises(binding.NbsError):
        binding.Plan((4, 4, 4), 8, channels.parse_table("p p p n"), device=-1)
