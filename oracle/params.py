"""Method constants from Section 2 (oracle side).  Test infrastructure only."""
from __future__ import annotations

from math import gcd, pi


def ntones(fs: int, f_comb: int) -> int:
    """Number of comb tones (= fold bins) over the band and its mirrored half: N = fs / f_comb (Section 2)."""
    if fs % f_comb:
        raise ValueError("fs must be a multiple of f_comb")
    return fs // f_comb


def rotator_period(fs: int, f_offset: int) -> int:
    """Shortest repeat length of the sampled rotator, Eq. 4: fs / gcd(fs, f_offset)."""
    return fs // gcd(fs, f_offset)


def phase_step(fs: int, f_offset: int) -> float:
    """Rotator phase increment per sample, Eq. 5: 2 pi f_offset / fs (radians)."""
    return 2.0 * pi * f_offset / fs
