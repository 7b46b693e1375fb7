"""Planted-mistake check of the oracle's pins (CPU only).

Each mutant is the oracle's C source with one plausible mistake planted in a
temporary copy (a flipped rotation sign, a dropped offset term, a wrong phase
index, a swapped bit order, a dropped tail, cos/sin swapped, ...).  The set of
pins below -- the same kinds of evidence as in test_oracle.py -- must pass on
the real oracle and fail on every mutant.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import synth
from oracle import core
from tests.test_oracle import _closed_form, _np_levels, _read_golden

MUTANTS = {
    "rotation_sign": ("*s = -sin(ang);", "*s = sin(ang);"),
    "cos_sin_swapped": ("*c = cos(ang);\n    *s = -sin(ang);", "*c = sin(ang);\n    *s = -cos(ang);"),
    "offset_dropped": ("((k * fc + fo) / g) % P", "((k * fc) / g) % P"),
    "phase_index_off_by_one": ("(uint64_t)((n0 + i0) % P)", "(uint64_t)((n0 + i0 + 1) % P)"),
    "global_index_ignored": ("(uint64_t)((n0 + i0) % P)", "(uint64_t)((i0) % P)"),
    "angle_reduction_sign": ("ang = -ORC_TWO_PI * (double)(P - m) / (double)P;",
                             "ang = ORC_TWO_PI * (double)(P - m) / (double)P;"),
    "bit_order_reversed": ("(2 * (int)(i & 3))", "(2 * (3 - (int)(i & 3)))"),
    "level_map_inverted": ("return 2 * code - 3;", "return 3 - 2 * code;"),
    "int8_read_unsigned": ("return (int)(int8_t)packed[i];", "return (int)packed[i];"),
    "tail_dropped": ("(nsamples + ORC_BLOCK - 1) / ORC_BLOCK", "nsamples / ORC_BLOCK"),
    "fold_ignores_n0": ("int64_t b = n0 % nbins;", "int64_t b = 0;"),
}


def _mp_corr(levels, n0, fs, fc, fo, k):
    mp.mp.dps = 30
    f = k * fc + fo
    acc = mp.mpc(0)
    for i, x in enumerate(levels):
        if x:
            acc += int(x) * mp.expj(-2 * mp.pi * mp.mpf(f * (n0 + i)) / fs)
    return complex(acc)


def _pins_hold(o) -> bool:
    """True when every pin holds for oracle binding ``o``."""
    # decoder fixtures
    for row in _read_golden("decode.txt"):
        lhs, rhs = row.split(":")
        parts = lhs.split()
        data = np.array([int(h, 16) for h in parts[1:]], dtype=np.uint8)
        want = np.array([int(v) for v in rhs.split()])
        if not np.array_equal(o.decode(data, int(parts[0]), want.size).astype(np.int64), want):
            return False
    # brute force, tiny packed inputs, both sample formats
    for fs, fc, fo, nbits, L, n0 in ((16_000_000, 1_000_000, 10_000, 2, 256, 1234),
                                     (16_000_000, 1_000_000, 250_000, 8, 128, 77)):
        rng = np.random.default_rng(L + nbits)
        packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
        lv = _np_levels(packed, nbits, L)
        tones = [0, 3, 9, 15]
        got = o.correlate(packed, nbits, L, fs, fc, fo, n0=n0, tones=tones)
        for t, c in zip(tones, got):
            if abs(c - _mp_corr(lv, n0, fs, fc, fo, t)) > 1e-12 * np.abs(lv).sum():
                return False
    # library FFT special case with a global offset
    fs, fc, fo = 16_000_000, 1_000_000, 10_000
    P = fs // math.gcd(math.gcd(fs, fc), fo)
    x = np.random.default_rng(1).standard_normal(P)
    got = o.correlate_f64(x, fs, fc, fo, n0=4321)
    X = np.fft.fft(x)
    g = fs // P
    for k in range(fs // fc):
        a = (k * fc + fo) // g
        if abs(got[k] - np.exp(-2j * np.pi * ((a * 4321) % P) / P) * X[a % P]) > 1e-9:
            return False
    # closed form of the noiseless comb
    spec = synth.CombSpec(16_000_000, 1_000_000, 10_000, 2, amp=0.3, t_d=3.7e-9)
    per = synth.comb_period(spec)
    got = o.correlate_f64(np.tile(per, 2), spec.fs, spec.f_comb, spec.f_offset)
    if np.max(np.abs(got - _closed_form(spec, 2 * per.size))) > 1e-9:
        return False
    # integer fold against a reshape-sum
    rng = np.random.default_rng(2)
    packed = rng.integers(0, 256, size=1000, dtype=np.uint8)
    lv = _np_levels(packed, 2, 4000)
    want = np.zeros(64, dtype=np.int64)
    np.add.at(want, (np.arange(4000) + 4 * 33) % 64, lv)
    if not np.array_equal(o.fold_int(packed, 2, 4000, 64, n0=4 * 33), want):
        return False
    return True


def test_pins_hold_on_oracle(oracle_lib):
    assert _pins_hold(core)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = core.source_text()
    assert src.count(old) >= 1, name
    variant = core.build_variant(src.replace(old, new), str(tmp_path / ("mut_%s.so" % name)))
    assert not _pins_hold(variant), name
