"""Channel tables (data): operator names and the 52-channel reading R52.

The paper computes 52 octet two-baryon channels but only cites the
companion paper's Tables 1-4 for the list (Sec. 4(iii)).  R52 is a reading:
particle-basis operators, isospin-symmetric coupled sectors at I_z = I, and
u<->d-independent representatives of the S = -2, I_z = 0 block.  A corrected
list drops in here without code changes.
"""
from __future__ import annotations

# Operator codes of include/nbs.h (Eqs. (2)-(3)).
OPS = {
    "p": 0, "n": 1, "Lambda": 2, "Sigma+": 3, "Sigma0": 4, "Sigma-": 5,
    "Xi0": 6, "Xi-": 7, "Xu": 8, "Xd": 9, "Xs": 10,
}


def _block(sinks, sources):
    return [(a, b, c, d) for (a, b) in sinks for (c, d) in sources]


def r52():
    """The 52 channels (B1, B2, B3, B4) = <B1 B2 | B3bar B4bar>."""
    ch = []
    # S = 0
    ch += [("p", "p", "p", "p"), ("p", "n", "p", "n")]
    # S = -1
    s1 = [("p", "Lambda"), ("p", "Sigma0"), ("n", "Sigma+")]
    ch += _block(s1, s1)
    ch += [("p", "Sigma+", "p", "Sigma+")]
    # S = -2
    ch += [("Sigma+", "Sigma+", "Sigma+", "Sigma+")]
    s2 = [("p", "Xi0"), ("Lambda", "Sigma+"), ("Sigma0", "Sigma+")]
    ch += _block(s2, s2)
    ch += _block([("Lambda", "Lambda"), ("Sigma0", "Sigma0")],
                 [("Lambda", "Lambda"), ("Sigma0", "Sigma0"), ("Sigma+", "Sigma-"), ("p", "Xi-")])
    ch += _block([("p", "Xi-"), ("Sigma+", "Sigma-")],
                 [("Lambda", "Lambda"), ("Sigma0", "Sigma0"), ("Sigma+", "Sigma-"), ("p", "Xi-"),
                  ("n", "Xi0")])
    # S = -3
    s3 = [("Xi0", "Lambda"), ("Xi0", "Sigma0"), ("Xi-", "Sigma+")]
    ch += _block(s3, s3)
    ch += [("Xi0", "Sigma+", "Xi0", "Sigma+")]
    # S = -4
    ch += [("Xi0", "Xi0", "Xi0", "Xi0"), ("Xi0", "Xi-", "Xi0", "Xi-")]
    assert len(ch) == 52
    return ch


# The paper's worked example, Eq. (7): <p Lambda | pbar Xu-bar>.
WORKED_EXAMPLE = ("p", "Lambda", "p", "Xu")


# ---- channel tables from quantum numbers, and from text --------------------
# Strangeness and twice the third isospin component of the octet operators
# (Eqs. (2)-(3)).
OCTET = {
    "p": (0, 1), "n": (0, -1), "Lambda": (-1, 0), "Sigma+": (-1, 2), "Sigma0": (-1, 0), "Sigma-": (-1, -2),
    "Xi0": (-2, 1), "Xi-": (-2, -1),
}


def octet_pairs(S, two_Iz, ordered=False):
    """Two-baryon states (B1, B2) of the octet with total strangeness S and
    total 2 I_z.  Unordered pairs (B1 listed first in OCTET order) unless
    ordered=True."""
    names = list(OCTET)
    out = []
    for i, a in enumerate(names):
        for j, b in enumerate(names):
            if not ordered and j < i:
                continue
            if OCTET[a][0] + OCTET[b][0] == S and OCTET[a][1] + OCTET[b][1] == two_Iz:
                out.append((a, b))
    return out


def coupled_channels(S, two_Iz, ordered=False):
    """Every channel <B1 B2 | B3bar B4bar> of one (S, I_z) sector: all sink
    pairs times all source pairs of the sector."""
    pairs = octet_pairs(S, two_Iz, ordered)
    return _block(pairs, pairs)


def sectors():
    """The (S, 2 I_z) sectors with at least one octet pair."""
    out = []
    for S in range(0, -5, -1):
        for tz in range(-4, 5):
            if octet_pairs(S, tz):
                out.append((S, tz))
    return out


def parse_table(text):
    """Channels from text: one per line, four operator names
    (B1 B2 B3 B4 for <B1 B2 | B3bar B4bar>) separated by blanks or commas;
    '#' starts a comment.  Unknown names raise ValueError; flavour
    conservation is checked by the channel compiler (nbs_plan_create)."""
    out = []
    for k, line in enumerate(text.splitlines(), 1):
        line = line.split("#", 1)[0].replace(",", " ").strip()
        if not line:
            continue
        f = line.split()
        if len(f) != 4 or any(x not in OPS for x in f):
            raise ValueError("line %d: expected four operator names of %s, got %r" % (k, sorted(OPS), line))
        out.append(tuple(f))
    return out


def load_table(path):
    with open(path) as fh:
        return parse_table(fh.read())
