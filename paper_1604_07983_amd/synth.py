"""Seeded synthetic quark propagators (inputs only; none of the method's arithmetic).

Stand-in for solved lattice propagators: the paper's gauge configurations
and solver are not available, so every input is a counter-based draw.
The value at (seed, flavour, t, site, row, col) is

    key  = splitmix64_output_0(seed)                  seed = base + flavour + 16*k
    n    = 2 * (((t * V + site) * 12 + row) * 12 + col)
    u1   = ((splitmix64(key, n)     >> 11) + 1) * 2^-53      in (0, 1]
    u2   =  (splitmix64(key, n + 1) >> 11)      * 2^-53      in [0, 1)
    S    = sqrt(-ln u1) * (cos 2 pi u2 + i sin 2 pi u2) * exp(-m_f * ((t - t0) mod T))

i.e. i.i.d. CN(0, 1) entries (Box-Muller) damped like a propagator from a
wall source at t0.  splitmix64(key, n) is output n of Steele, Lea and
Flood's SplitMix64 generator started at state ``key``:
mix(key + (n + 1) * 0x9E3779B97F4A7C15) with the published mix function.

Both the oracle-side tests and the GPU path consume the same bytes from
this module (or from a device kernel implementing the same definition).
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
SEED_BASE = 20260101
FLAVOUR_INDEX = {"u": 0, "d": 1, "s": 2}


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int) -> np.uint64:
    with np.errstate(over="ignore"):
        return _mix64(np.array([seed], dtype=np.uint64) + GOLDEN)[0]


def seed_for(flavour: int, source: int = 0, base: int = SEED_BASE) -> int:
    return base + flavour + 16 * source


def propagator_slice(L, t: int, flavour: int, decay: float, *, T: int,
                     t0: int = 0, source: int = 0, base: int = SEED_BASE,
                     dtype=np.complex128) -> np.ndarray:
    """Propagator of one flavour on time slice t: array [Lz, Ly, Lx, 12, 12]."""
    Lx, Ly, Lz = (int(v) for v in L)
    V = Lx * Ly * Lz
    key = stream_key(seed_for(flavour, source, base))
    out = np.empty(V * 144, dtype=dtype)
    damp = np.exp(-decay * ((t - t0) % T))
    chunk = 1 << 21
    with np.errstate(over="ignore"):
        for start in range(0, V * 144, chunk):
            stop = min(V * 144, start + chunk)
            e = np.arange(start, stop, dtype=np.uint64) + np.uint64(t * V * 144)
            n = e * np.uint64(2)
            z1 = _mix64(key + (n + np.uint64(1)) * GOLDEN)
            z2 = _mix64(key + (n + np.uint64(2)) * GOLDEN)
            u1 = ((z1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
            u2 = (z2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
            rad = np.sqrt(-np.log(u1))
            ang = 2.0 * np.pi * u2
            val = (rad * np.cos(ang) + 1j * (rad * np.sin(ang))) * damp
            out[start:stop] = val.astype(dtype)
    return out.reshape(Lz, Ly, Lx, 12, 12)


def propagators(L, ts, flavour: int, decay: float, **kw) -> np.ndarray:
    """Stack of slices: [len(ts), Lz, Ly, Lx, 12, 12]."""
    return np.stack([propagator_slice(L, int(t), flavour, decay, **kw) for t in ts])
