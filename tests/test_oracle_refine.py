"""Pins of the oracle's multi-pass delay refinement (Section 2; CPU only).

The refinement counter-rotates the tone responses by the current delay,
unwraps the residual phases over the in-band tones and moves the delay by
the least-squares slope.  Pinned to closed forms of the noiseless Eq. 1 comb
(phases phi_k - pi/2 with phi_k = 2 pi f_k t_d + eps_k): the delay is t_d
plus the least-squares slope of the injected jitter, the intercept -pi/2
plus the jitter's intercept, the rms the jitter's residual about its line;
a start several samples off still converges; later passes are a fixed point;
the lower sideband is the conjugate.  Planted mistakes (sign of the
counter-rotation, the offset frequency dropped, no unwrap, the update sign)
each break a pin.
"""
import types

import numpy as np
import pytest

import synth
from tests.test_oracle import _closed_form


def _ls(f, y):
    fm, ym = f.mean(), y.mean()
    slope = np.sum((f - fm) * (y - ym)) / np.sum((f - fm) ** 2)
    a = ym - slope * fm
    return slope, a, float(np.sqrt(np.mean((y - a - slope * f) ** 2)))


CASES = [
    (64_000_000, 10_000, 3.7e-9, 0.0),
    (64_000_000, 10_000, 3.7e-9, 0.1),
    (16_000_000, 250_000, -120e-9, 0.0),
    (32_000_000, 510_000, 410e-9, 0.05),   # 0.41 of the 1 us ambiguity
]


def _comb(fs, fo, td, jit):
    spec = synth.CombSpec(fs, 1_000_000, fo, 2, amp=0.3, t_d=td, jitter=jit, seed=(9,))
    L = synth.comb_period_length(spec) * 4
    return spec, _closed_form(spec, L)


def _expected(spec):
    import oracle

    k = oracle.in_band(spec.fs, spec.f_comb, spec.f_offset)
    f = oracle.tone_freqs(spec.fs, spec.f_comb, spec.f_offset)[k]
    eps = synth.tone_jitter(spec)[k] if spec.jitter else np.zeros(k.size)
    s, a, rms = _ls(f, eps)
    return spec.t_d + s / (2 * np.pi), -np.pi / 2 + a, rms


@pytest.mark.parametrize("fs,fo,td,jit", CASES)
def test_refine_closed_form(fs, fo, td, jit):
    import oracle

    spec, C = _comb(fs, fo, td, jit)
    t_want, a_want, rms_want = _expected(spec)
    for t0 in (td, td + 3.0 / fs, td - 2.5 / fs):
        d, a, rms = oracle.refine(C, fs, 1_000_000, fo, t0, 3)
        assert d[0] == t0
        assert abs(d[1] - t_want) < 1e-17 and abs(d[3] - t_want) < 1e-17
        assert abs(a - a_want) < 1e-9
        assert abs(rms - rms_want) < 1e-9


def test_refine_fixed_point_and_sideband():
    import oracle

    spec, C = _comb(64_000_000, 10_000, 3.7e-9, 0.1)
    d, a, rms = oracle.refine(C, spec.fs, 1_000_000, spec.f_offset, 0.0, 5)
    assert np.abs(np.diff(d[1:])).max() < 1e-20
    dl, al, rl = oracle.refine(np.conj(C), spec.fs, 1_000_000, spec.f_offset, 0.0, 5, sideband=-1)
    assert np.array_equal(d, dl) and a == al and rms == rl


def test_refine_start_from_pulse_peak():
    """Section 2's sequence: the coarse delay from the pulse peak, then the passes."""
    import oracle

    spec, C = _comb(32_000_000, 510_000, 410e-9, 0.05)
    _, _, t0, _ = oracle.pulse_peak(np.fft.ifft(C), spec.fs)
    d, _, _ = oracle.refine(C, spec.fs, 1_000_000, spec.f_offset, t0, 2)
    assert abs(d[-1] - _expected(spec)[0]) < 1e-17


REFINE_MUTANTS = {
    "counter_rotation_sign": ("np.exp(-2j * np.pi * f * t)", "np.exp(2j * np.pi * f * t)"),
    "no_offset_frequency": ("f = tone_freqs(fs, f_comb, f_offset)[k]", "f = tone_freqs(fs, f_comb, 0)[k]"),
    "no_unwrap": ("psi = np.unwrap(np.angle(Ck * np.exp(-2j * np.pi * f * t)))",
                  "psi = np.angle(Ck * np.exp(-2j * np.pi * f * t))"),
    "update_sign": ("t = t + float(slope / (2.0 * np.pi))", "t = t - float(slope / (2.0 * np.pi))"),
}


def _variant(old, new):
    import oracle.pulse as op

    src = open(op.__file__).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("oracle.pulse_variant")
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), "pulse_variant", "exec"), mod.__dict__)
    return mod


def _refine_pins_hold(m) -> bool:
    for fs, fo, td, jit in CASES:
        spec, C = _comb(fs, fo, td, jit)
        t_want, a_want, _ = _expected(spec)
        for t0 in (td + 3.0 / fs, td - 2.5 / fs):
            d, a, _ = m.refine(C, fs, 1_000_000, fo, t0, 2)
            if abs(d[-1] - t_want) > 1e-17 or abs(a - a_want) > 1e-9:
                return False
    return True


def test_refine_pins_hold_on_oracle():
    import oracle.pulse as op

    assert _refine_pins_hold(op)


@pytest.mark.parametrize("name", sorted(REFINE_MUTANTS))
def test_refine_pins_catch_mutant(name):
    assert not _refine_pins_hold(_variant(*REFINE_MUTANTS[name])), name
