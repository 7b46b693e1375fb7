"""Delay at the power peak of the folded pulse, and the delay-corrected band-pass (oracle side, numpy FP64).

Test infrastructure only.  Section 2 notes that bin b of the fold P[b]
stands for a time delay of b / fs and that the delay can be read off near the
largest bin by a hyperbolic fit over its neighbours; Section 3 takes the
group delay at the position of maximum power.  The paper gives no formula.
Readings used here:

* the peak bin b0 is the first bin of largest power |P[b]|^2;
* the pulse of N tones of equal amplitude is a periodic sinc whose envelope
  is c / |sin(pi (b - x0) / N)| -- near the peak the hyperbola c / |b - x0|,
  made periodic.  Fitting it through the amplitudes of b0 and of its larger
  cyclic neighbour b0 + s (s = +1 or -1) gives the offset d in [0, 1/2]:
  tan(u d) = a_s sin(u) / (a_0 + a_s cos(u)), u = pi / N.  Equal neighbours
  give d = 0.  The fit is exact for an equal-amplitude comb at any delay;
* the pulse position pos = b0 + s d is taken in (-N/2, N/2] bins;
* the delay is reported in the sign convention of the phase-slope delay (a
  tone phase that grows as 2 pi f_k t_d): an upper-sideband comb delayed by
  t_d folds into a pulse at bin -t_d fs (mod N), so delay = -pos / fs; a
  lower-sideband stream (reported as the conjugate spectrum, whose pulse is
  conj(P[-b])) gives +pos / fs.
"""
from __future__ import annotations

import math

import numpy as np


def pulse_peak(P, fs: int, sideband: int = 1):
    """(b0, signed offset s*d, delay_s, peak_power) of the pulse P[b] (power not normalised)."""
    P = np.asarray(P, dtype=np.complex128)
    n = P.size
    power = P.real * P.real + P.imag * P.imag
    b0 = int(np.argmax(power))
    a_0 = math.sqrt(power[b0])
    a_m = math.sqrt(power[(b0 - 1) % n])
    a_p = math.sqrt(power[(b0 + 1) % n])
    if a_p > a_m:
        s, a_s = 1, a_p
    elif a_m > a_p:
        s, a_s = -1, a_m
    else:
        s, a_s = 0, 0.0
    u = math.pi / n
    d = math.atan2(a_s * math.sin(u), a_0 + a_s * math.cos(u)) / u if s else 0.0
    pos = b0 + s * d
    if pos > n / 2.0:
        pos -= n
    delay = (-pos if sideband > 0 else pos) / float(fs)
    return b0, float(s * d), float(delay), float(power[b0])


def bandpass(C, fs: int, f_comb: int, f_offset: int, delay: float, sideband: int = 1):
    """Band-pass corrected for a group delay (Section 3): arg(C_k exp(-j 2 pi f_k delay)) for every tone.

    C are the raw correlations of :func:`oracle.correlate`; a lower-sideband
    stream is reported as their conjugate (as :func:`oracle.results` does)
    before the correction; f_k = f_offset + k f_comb.  A comb whose tone
    phases grow as 2 pi f_k t_d, corrected by t_d, has flat phases.
    """
    C = np.asarray(C, dtype=np.complex128)
    if sideband < 0:
        C = np.conj(C)
    f = f_offset + f_comb * np.arange(C.size, dtype=np.float64)
    return np.angle(C * np.exp(-2j * np.pi * f * delay))


def refine(C, fs: int, f_comb: int, f_offset: int, t0: float, iters: int, sideband: int = 1):
    """Multi-pass delay refinement (Section 2: a coarse delay from the pulse, then repeated passes that
    counter-rotate by the current estimate and measure the residual phase).

    Reading used here: the counter-rotation by a delay t is applied to the tone responses, which is what
    counter-rotating the input by that delay does to them -- every tone k turns by exp(-j 2 pi f_k t),
    f_k = f_offset + k f_comb.  Starting from t0, each pass takes the residual phases
    psi_k = arg(C_k exp(-j 2 pi f_k t)) of the in-band tones (0 < f_k < fs/2), unwraps them along
    increasing f_k, fits the least-squares line psi = a + 2 pi f t_res and moves the estimate to
    t + t_res.  A lower-sideband stream is reported as the conjugate spectrum first (as
    :func:`oracle.results` does).

    Returns (delays, a, rms): delays[0] = t0 and delays[i] the estimate after pass i (seconds), then the
    last pass's intercept a (rad, the line's phase at f = 0) and the rms of its phase residuals about
    the line (rad).
    """
    from .fit import in_band, tone_freqs

    if iters < 1:
        raise ValueError("at least one pass")
    C = np.asarray(C, dtype=np.complex128)
    if sideband < 0:
        C = np.conj(C)
    k = in_band(fs, f_comb, f_offset)
    f = tone_freqs(fs, f_comb, f_offset)[k]
    Ck = C[k]
    delays = [float(t0)]
    t = float(t0)
    a = rms = 0.0
    for _ in range(iters):
        psi = np.unwrap(np.angle(Ck * np.exp(-2j * np.pi * f * t)))
        fm, um = f.mean(), psi.mean()
        slope = np.sum((f - fm) * (psi - um)) / np.sum((f - fm) ** 2)
        a = float(um - slope * fm)
        rms = float(np.sqrt(np.mean((psi - a - slope * f) ** 2)))
        t = t + float(slope / (2.0 * np.pi))
        delays.append(t)
    return np.asarray(delays), a, rms
