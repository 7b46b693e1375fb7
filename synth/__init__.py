"""Seeded synthetic baseband streams carrying a multi-tone phase-calibration comb.

This module only *makes inputs*.  It holds none of the extraction method's
arithmetic (no rotation, no folding, no transform): it evaluates the signal
model of Section 2, Eq. 1 -- galaxy noise plus N equally spaced sinusoids at
``i*f_comb + f_offset`` with phases ``phi_i = 2*pi*(i*f_comb + f_offset)*t_d``
(+ an optional per-tone jitter) -- then quantises and packs the samples the
way a VLBI recorder stores them (2-bit or 8-bit, Section 1).  Both the FP64
oracle and the HIP library consume the very same packed bytes.

Conventions (the paper is silent on them; the readings are stated here):

* 2-bit: thresholds ``{-0.98, 0, +0.98}`` give offset-binary codes 0..3 that
  stand for the levels ``{-3, -1, +1, +3}``; byte ``j`` holds samples
  ``4j..4j+3`` with sample ``4j+q`` in bits ``[2q, 2q+1]`` (LSB first).
* 8-bit: two's-complement int8, round-half-even then clamp to [-128, 127].

Random numbers come from counter-based Philox generators: numpy's Philox on
the host, torch's Philox on the device.  A stream is a pure function of its
parameters and seed, so any chunk can be regenerated independently.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import gcd
from typing import Optional, Sequence

import numpy as np

TWO_BIT_THRESHOLDS = (-0.98, 0.0, 0.98)


@dataclass(frozen=True)
class CombSpec:
    """Parameters of one synthetic stream (frequencies in integer Hz)."""

    fs: int
    f_comb: int
    f_offset: int
    nbits: int
    amp: float          # per-tone amplitude, in units of the noise sigma's scale
    t_d: float          # instrumental delay in seconds (Eq. 1 phases)
    sigma: float = 1.0  # noise standard deviation
    jitter: float = 0.0  # per-tone phase jitter drawn from U(-jitter, +jitter) rad
    seed: Sequence[int] = field(default=(0,))

    @property
    def ntones(self) -> int:
        return self.fs // self.f_comb

    @property
    def samples_per_byte(self) -> int:
        return 8 // self.nbits


def _check(spec: CombSpec) -> None:
    if spec.fs <= 0 or spec.f_comb <= 0 or spec.fs % spec.f_comb:
        raise ValueError("fs must be a positive multiple of f_comb")
    if not (0 <= spec.f_offset < spec.fs):
        raise ValueError("f_offset must lie in [0, fs)")
    if spec.nbits not in (2, 8):
        raise ValueError("nbits must be 2 or 8")


def tone_jitter(spec: CombSpec) -> np.ndarray:
    """Per-tone phase jitter eps_i ~ U(-jitter, +jitter), seeded by ``spec.seed``."""
    n = spec.ntones
    if spec.jitter == 0.0:
        return np.zeros(n)
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence(list(spec.seed) + [0x4A17])))
    return rng.uniform(-spec.jitter, spec.jitter, size=n)


def tone_phases(spec: CombSpec) -> np.ndarray:
    """Injected phases phi_i = 2*pi*(i*f_comb + f_offset)*t_d + eps_i (Eq. 1)."""
    i = np.arange(spec.ntones, dtype=np.float64)
    f = i * spec.f_comb + spec.f_offset
    return 2.0 * np.pi * f * spec.t_d + tone_jitter(spec)


def comb_period_length(spec: CombSpec) -> int:
    """Length after which the sampled comb repeats exactly: fs / gcd(fs, f_comb, f_offset)."""
    return spec.fs // gcd(gcd(spec.fs, spec.f_comb), spec.f_offset)


def comb_period(spec: CombSpec) -> np.ndarray:
    """One exact period of the noiseless comb p[n] of Eq. 1, in FP64.

    The argument of each sine is reduced exactly with integer arithmetic,
    ``((i*f_comb + f_offset) * n) mod fs``, before it is scaled to radians, so
    the period is accurate to FP64 rounding for any period length.
    """
    _check(spec)
    per = comb_period_length(spec)
    g = spec.fs // per
    n = np.arange(per, dtype=np.int64)
    phi = tone_phases(spec)
    out = np.zeros(per, dtype=np.float64)
    for i in range(spec.ntones):
        a = ((i * spec.f_comb + spec.f_offset) // g) % per
        m = (a * n) % per
        out += np.sin(2.0 * np.pi * m / per + phi[i])
    return spec.amp * out


def comb_values(spec: CombSpec, start: int, count: int) -> np.ndarray:
    """The noiseless comb of Eq. 1 at samples start .. start+count-1: the same values, to the bit, as
    ``comb_period(spec)`` at those indices modulo the period (same integer reduction, same per-tone
    summation order), without building a whole period -- for periods far longer than the range."""
    _check(spec)
    per = comb_period_length(spec)
    g = spec.fs // per
    n = np.arange(start, start + count, dtype=np.int64) % per
    phi = tone_phases(spec)
    out = np.zeros(count, dtype=np.float64)
    for i in range(spec.ntones):
        a = ((i * spec.f_comb + spec.f_offset) // g) % per
        m = (a * n) % per
        out += np.sin(2.0 * np.pi * m / per + phi[i])
    return spec.amp * out


def _quantise_host(x: np.ndarray, nbits: int) -> np.ndarray:
    if nbits == 2:
        t0, t1, t2 = TWO_BIT_THRESHOLDS
        return ((x > t0).astype(np.uint8) + (x > t1) + (x > t2)).astype(np.uint8)
    return np.clip(np.rint(x), -128, 127).astype(np.int8).view(np.uint8)


def pack_2bit(codes: np.ndarray) -> np.ndarray:
    """Pack codes 0..3 four per byte, sample 4j+q into bits [2q, 2q+1] of byte j."""
    c = np.asarray(codes, dtype=np.uint8).reshape(-1, 4)
    return (c[:, 0] | (c[:, 1] << 2) | (c[:, 2] << 4) | (c[:, 3] << 6)).astype(np.uint8)


def levels_2bit(codes: np.ndarray) -> np.ndarray:
    """Offset-binary code c -> level 2c - 3 (used only by tests that build expected samples)."""
    return 2 * np.asarray(codes, dtype=np.int64) - 3


def make_stream(spec: CombSpec, nsamples: int, n0: int = 0, chunk: int = 1 << 22,
                noise_seed_extra: Sequence[int] = ()) -> np.ndarray:
    """Packed bytes (numpy uint8) for samples n0 .. n0+nsamples-1 of the stream.

    Noise is drawn per fixed-size block of the *global* sample index, so a
    sub-range of the stream is bit-identical to the same samples cut out of a
    longer generation (``n0`` and ``chunk`` must then be multiples of 4 for
    2-bit packing).
    """
    _check(spec)
    spb = spec.samples_per_byte
    if nsamples % spb or n0 % spb:
        raise ValueError("nsamples and n0 must be multiples of the samples per byte")
    per = comb_period_length(spec)
    # a period longer than the range: evaluate the comb at the samples generated instead
    direct = spec.amp != 0.0 and per > nsamples
    comb = comb_period(spec) if spec.amp != 0.0 and not direct else None
    out = np.empty(nsamples // spb, dtype=np.uint8)
    blk = 1 << 16
    pos = 0
    while pos < nsamples:
        g = n0 + pos
        b0 = g // blk
        take = min(nsamples - pos, (b0 + 1) * blk - g, chunk)
        rng = np.random.Generator(np.random.Philox(
            np.random.SeedSequence(list(spec.seed) + list(noise_seed_extra) + [int(b0)])))
        noise = rng.standard_normal(blk)
        off = g - b0 * blk
        x = spec.sigma * noise[off:off + take]
        if direct:
            x = x + comb_values(spec, g, take)
        elif comb is not None:
            idx = (np.arange(g, g + take, dtype=np.int64)) % per
            x = x + comb[idx]
        q = _quantise_host(x, spec.nbits)
        if spec.nbits == 2:
            out[pos // 4:(pos + take) // 4] = pack_2bit(q)
        else:
            out[pos:pos + take] = q
        pos += take
    return out


def make_stream_device(spec: CombSpec, nsamples: int, device: str = "cuda", chunk: int = 1 << 26):
    """Packed bytes as a torch uint8 tensor generated on ``device`` (fast path for large inputs).

    Uses torch's counter-based Philox generator seeded from ``spec.seed``; the
    bytes differ from :func:`make_stream` (different generator) but are just
    as reproducible.  Tests hand the *same* tensor, copied to the host, to the
    oracle.
    """
    import torch

    _check(spec)
    spb = spec.samples_per_byte
    if nsamples % spb:
        raise ValueError("nsamples must be a multiple of the samples per byte")
    per = comb_period_length(spec)
    if spec.amp != 0.0 and per > nsamples:
        # a period longer than the range: the comb at samples 0 .. nsamples-1 (indices stay below per)
        host = comb_values(spec, 0, nsamples)
    else:
        host = comb_period(spec) if spec.amp != 0.0 else np.zeros(per)
    comb = torch.as_tensor(host, dtype=torch.float32, device=device)
    seed = 0
    for s in spec.seed:
        seed = (seed * 1000003 + int(s) + 1) % (1 << 62)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    out = torch.empty(nsamples // spb, dtype=torch.uint8, device=device)
    chunk = max(spb * per, (chunk // (spb * per)) * spb * per) if per < chunk else chunk - chunk % spb
    pos = 0
    while pos < nsamples:
        take = min(chunk, nsamples - pos)
        idx = torch.arange(pos, pos + take, device=device, dtype=torch.int64) % per
        x = torch.randn(take, generator=gen, device=device, dtype=torch.float32) * spec.sigma + comb[idx]
        if spec.nbits == 2:
            t0, t1, t2 = TWO_BIT_THRESHOLDS
            c = (x > t0).to(torch.uint8) + (x > t1).to(torch.uint8) + (x > t2).to(torch.uint8)
            c = c.view(-1, 4)
            out[pos // 4:(pos + take) // 4] = c[:, 0] | (c[:, 1] << 2) | (c[:, 2] << 4) | (c[:, 3] << 6)
        else:
            out[pos:pos + take] = torch.clamp(torch.round(x), -128, 127).to(torch.int8).view(torch.uint8)
        pos += take
    return out


# ---------------------------------------------------------------------------
# Named workloads (the sizes, value distributions and structure of the
# evaluation configurations).  ``nsamples`` is the full size; tests use prefixes.
# ---------------------------------------------------------------------------

WORKLOADS = {
    # fs=32 MHz, N=32, f_offset=0: integer fold, bit-exact
    "small_2bit_fo0": dict(spec=CombSpec(32_000_000, 1_000_000, 0, 2, amp=0.05, t_d=10e-9, seed=(1, 0, 0)),
                           nsamples=1 << 24),
    # fs=64 MHz, N=64, f_offset=10 kHz (rotator period 6400), 2-bit, 2^30 samples
    "fold2_64M_10k": dict(spec=CombSpec(64_000_000, 1_000_000, 10_000, 2, amp=0.02, t_d=3.7e-9,
                                        jitter=0.1, seed=(2, 0, 0)),
                          nsamples=1 << 30),
    # fs=1024 MHz, N=1024, f_offset=510 kHz (rotator period 102400), 8-bit, 2^33 in 2^28 chunks
    "wide8_1024M_510k": dict(spec=CombSpec(1_024_000_000, 1_000_000, 510_000, 8, amp=1.0, t_d=125e-9,
                                           sigma=20.0, seed=(3, 0, 0)),
                             nsamples=1 << 33, chunk=1 << 28),
    # fs=64 MHz, N=64, f_offset=10008 Hz (rotator period 8e6 samples: the longest fold periods AUTO still
    # folds; the per-sample forms run on it too), 2-bit, 2^30 samples
    "osc2_64M_10008": dict(spec=CombSpec(64_000_000, 1_000_000, 10_008, 2, amp=0.02, t_d=3.7e-9,
                                         jitter=0.1, seed=(6, 0, 0)),
                           nsamples=1 << 30),
}


def batch_specs(nstreams: int = 64, seed: int = 4, nbits: Optional[int] = 2) -> list:
    """Stream mix of the precision study: fs ~ U{16..512} MHz, f_offset ~ U{0,10,250,510} kHz."""
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, 0xBA7C])))
    fss = [16, 32, 64, 128, 256, 512]
    fos = [0, 10_000, 250_000, 510_000]
    out = []
    for s in range(nstreams):
        fs = int(fss[rng.integers(len(fss))]) * 1_000_000
        fo = int(fos[rng.integers(len(fos))])
        td = float(rng.uniform(0.0, 20e-9))
        nb = nbits if nbits is not None else int((2, 8)[rng.integers(2)])
        if nb == 2:
            out.append(CombSpec(fs, 1_000_000, fo, 2, amp=0.02, t_d=td, seed=(seed, s, 0)))
        else:
            out.append(CombSpec(fs, 1_000_000, fo, 8, amp=1.0, t_d=td, sigma=20.0, seed=(seed, s, 0)))
    return out


def served_specs(nstreams: int = 256, seed: int = 5) -> list:
    """Stream mix of the serving study: 16 stations x 16 channels, each with
    fs ~ U{32..512} MHz, f_offset ~ U{0,10,250,510} kHz, 2- or 8-bit with p = 1/2."""
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, 0x5E7E])))
    fss = [32, 64, 128, 256, 512]
    fos = [0, 10_000, 250_000, 510_000]
    out = []
    for s in range(nstreams):
        fs = int(fss[rng.integers(len(fss))]) * 1_000_000
        fo = int(fos[rng.integers(len(fos))])
        td = float(rng.uniform(0.0, 20e-9))
        if rng.integers(2) == 0:
            out.append(CombSpec(fs, 1_000_000, fo, 2, amp=0.02, t_d=td, seed=(seed, s, 0)))
        else:
            out.append(CombSpec(fs, 1_000_000, fo, 8, amp=1.0, t_d=td, sigma=20.0, seed=(seed, s, 0)))
    return out


def served_trace(nstreams: int, seconds: float, offered_sps: float = 200e9, seed: int = 5):
    """Chunk arrivals of the serving study: Poisson in time at rate offered_sps / E[chunk],
    chunk sizes 2^U{20..24} samples, each to a stream drawn uniformly.

    Returns (arrival times in s, stream index, samples) as numpy arrays."""
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, 0x7A3C])))
    sizes = 2 ** np.arange(20, 25)
    rate = offered_sps / sizes.mean()
    n = int(rate * seconds * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    keep = t < seconds
    t = t[keep]
    sid = rng.integers(0, nstreams, size=n)[keep]
    ns = sizes[rng.integers(0, sizes.size, size=n)][keep].astype(np.int64)
    return t, sid.astype(np.int64), ns
