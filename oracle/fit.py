"""Amplitude, phase and delay from per-tone correlations (oracle side, numpy FP64).

Test infrastructure only.  Readings of the paper used here (it fixes none of
them): the amplitude is |C_k| / L; the phase is arg C_k in (-pi, pi]; a
lower-sideband stream reports the complex conjugate; the delay is the
least-squares slope of the tone phases, unwrapped along increasing tone
frequency f_k = f_offset + k*f_comb over the tones with 0 < f_k < fs/2,
divided by 2*pi (the phases of Eq. 1 grow as 2*pi*f_k*t_d).
"""
from __future__ import annotations

import numpy as np


def tone_freqs(fs: int, f_comb: int, f_offset: int) -> np.ndarray:
    n = fs // f_comb
    return f_offset + f_comb * np.arange(n, dtype=np.float64)


def in_band(fs: int, f_comb: int, f_offset: int) -> np.ndarray:
    """Indices k of the tones with 0 < f_k < fs/2 (the non-mirror half of the band)."""
    f = f_offset + f_comb * np.arange(fs // f_comb, dtype=np.int64)
    return np.nonzero((f > 0) & (2 * f < fs))[0]


def delay_fit(phase: np.ndarray, freqs: np.ndarray) -> float:
    """t_d = slope / (2 pi) of the least-squares line through the unwrapped phases."""
    if len(phase) < 2:
        return 0.0
    u = np.unwrap(np.asarray(phase, dtype=np.float64))
    f = np.asarray(freqs, dtype=np.float64)
    fm = f.mean()
    um = u.mean()
    slope = np.sum((f - fm) * (u - um)) / np.sum((f - fm) ** 2)
    return float(slope / (2.0 * np.pi))


def results(C: np.ndarray, nsamples: int, fs: int, f_comb: int, f_offset: int, sideband: int = 1):
    """(amp[N], phase[N], delay) from the C_k of all N tones."""
    C = np.asarray(C, dtype=np.complex128)
    if sideband < 0:
        C = np.conj(C)
    amp = np.abs(C) / float(nsamples) if nsamples else np.zeros(C.size)
    phase = np.angle(C)
    k = in_band(fs, f_comb, f_offset)
    delay = delay_fit(phase[k], tone_freqs(fs, f_comb, f_offset)[k])
    return amp, phase, delay
