"""Pins of the oracle's rotated fold and pulse-peak delay (CPU only).

The rotated bins P[b] of Eqs. 2-3 are tied to 40-digit brute force, to the
exact integer fold when f_offset = 0, to the per-tone correlation through the
identity DFT(P) = C_k of Section 2, to the closed form of a single impulse,
and to chunking with a global sample index.  The pulse-peak delay (Sections
2-3) is tied to closed forms: a single-bin pulse, the pulse of an
equal-amplitude comb at any delay, and the noiseless Eq. 1 comb, whose pulse
delay must agree with the phase-slope delay.  Planted mistakes in the C
source of the fold must each break a pin.
"""

import mpmath as mp
import numpy as np
import pytest

import synth
from oracle import core
from tests.test_oracle import _closed_form, _np_levels


def _mp_fold(levels, n0, fs, fo, N):
    mp.mp.dps = 40
    out = [mp.mpc(0)] * N
    for i, x in enumerate(levels):
        if x:
            out[(n0 + i) % N] += int(x) * mp.expj(-2 * mp.pi * mp.mpf(fo * (n0 + i)) / fs)
    return np.array([complex(v) for v in out])


BRUTE = [
    (16_000_000, 10_000, 16, 2, 1024, 0),
    (16_000_000, 250_000, 16, 2, 512, 12345),
    (64_000_000, 10_007, 32, 8, 400, 10 ** 9 + 3),   # prime offset: no phasor table
    (24_000_000, 510_000, 24, 8, 300, 2 ** 33 + 1),  # large global index
]


@pytest.mark.parametrize("fs,fo,N,nbits,L,n0", BRUTE)
def test_fold_rot_mpmath_bruteforce(oracle_lib, fs, fo, N, nbits, L, n0):
    rng = np.random.default_rng(L + fo)
    packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
    lv = _np_levels(packed, nbits, L)
    got = oracle_lib.fold_rot(packed, nbits, L, fs, fo, N, n0=n0)
    want = _mp_fold(lv, n0, fs, fo, N)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(lv).sum()


@pytest.mark.parametrize("nbits,N,L,n0", [(2, 32, 4096, 0), (2, 64, 4000, 132), (8, 1024, 5000, 77)])
def test_fold_rot_f0_is_integer_fold(oracle_lib, nbits, N, L, n0):
    rng = np.random.default_rng(N + L)
    packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
    got = oracle_lib.fold_rot(packed, nbits, L, 32_000_000, 0, N, n0=n0)
    want = oracle_lib.fold_int(packed, nbits, L, N, n0=n0)
    assert np.array_equal(got.real, want.astype(np.float64))
    assert not np.any(got.imag)


@pytest.mark.parametrize("fs,fc,fo,nbits,L,n0", [
    (64_000_000, 1_000_000, 10_000, 2, 6400 * 8, 0),
    (16_000_000, 1_000_000, 250_000, 8, 20_000, 999),
    (32_000_000, 2_000_000, 10_007, 2, 8192, 2 ** 31 + 12),
    (1_024_000_000, 1_000_000, 510_000, 8, 1 << 16, 3 << 28),
])
def test_fold_rot_dft_is_correlation(oracle_lib, fs, fc, fo, nbits, L, n0):
    """Section 2: the DFT of the rotated bins gives every tone's C_k."""
    rng = np.random.default_rng(fs % 997 + L)
    packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
    N = fs // fc
    P = oracle_lib.fold_rot(packed, nbits, L, fs, fo, N, n0=n0)
    C = oracle_lib.correlate(packed, nbits, L, fs, fc, fo, n0=n0)
    scale = np.abs(_np_levels(packed, nbits, L)).sum()
    assert np.abs(np.fft.fft(P) - C).max() <= 1e-12 * scale


def test_fold_rot_impulse(oracle_lib):
    """One nonzero 8-bit sample x at global index n lands in bin n mod N as x exp(-j 2 pi f_o n / fs)."""
    fs, fo, N, L = 64_000_000, 10_000, 64, 1000
    for i, x, n0 in ((0, 5, 0), (517, -128, 6400 * 3 + 11), (999, 127, 10 ** 12 + 7)):
        packed = np.zeros(L, dtype=np.uint8)
        packed[i] = np.uint8(x & 0xFF)
        got = oracle_lib.fold_rot(packed, 8, L, fs, fo, N, n0=n0)
        n = n0 + i
        want = np.zeros(N, dtype=np.complex128)
        want[n % N] = x * np.exp(-2j * np.pi * ((fo * n) % fs) / fs)
        assert np.abs(got - want).max() <= 1e-14 * abs(x)


def test_fold_rot_chunking(oracle_lib):
    fs, fo, N = 64_000_000, 10_000, 64
    rng = np.random.default_rng(5)
    L = 4 * 6000
    packed = rng.integers(0, 256, size=L // 4, dtype=np.uint8)
    whole = oracle_lib.fold_rot(packed, 2, L, fs, fo, N, n0=40)
    cut = 4 * 1234
    parts = oracle_lib.fold_rot(packed[:cut // 4], 2, cut, fs, fo, N, n0=40) + \
        oracle_lib.fold_rot(packed[cut // 4:], 2, L - cut, fs, fo, N, n0=40 + cut)
    assert np.abs(whole - parts).max() <= 1e-11


# ------------------------------------------------------------- pulse-peak delay

@pytest.mark.parametrize("N,b0", [(64, 0), (64, 5), (64, 32), (64, 33), (64, 63), (1, 0), (2, 1), (1024, 700)])
def test_pulse_peak_single_bin(oracle_lib, N, b0):
    fs = 64_000_000
    P = np.zeros(N, dtype=np.complex128)
    P[b0] = 3.0 - 4.0j
    b, off, delay, power = oracle_lib.pulse_peak(P, fs)
    pos = b0 - N if b0 > N / 2 else b0
    assert (b, off, power) == (b0, 0.0, 25.0)
    assert delay == -pos / fs
    assert oracle_lib.pulse_peak(P, fs, sideband=-1)[2] == pos / fs


def test_pulse_peak_empty_and_flat(oracle_lib):
    assert oracle_lib.pulse_peak(np.zeros(64), 64_000_000) == (0, 0.0, 0.0, 0.0)
    b, off, delay, _ = oracle_lib.pulse_peak(np.ones(16), 16_000_000)
    assert (b, off, delay) == (0, 0.0, 0.0)


@pytest.mark.parametrize("N", [16, 64, 1024])
@pytest.mark.parametrize("tau", [0.0, 0.25, 0.5, 0.77, 3.7, -5.3, -0.49])
def test_pulse_peak_equal_comb_any_delay(oracle_lib, N, tau):
    """N equal tones delayed by tau samples (C_k = exp(j 2 pi k tau / N)): exact tau from the pulse."""
    fs = N * 1_000_000
    k = np.arange(N)
    C = np.exp(2j * np.pi * k * tau / N) * np.exp(0.3j) * 1e6
    P = np.fft.ifft(C)
    _, _, delay, _ = oracle_lib.pulse_peak(P, fs)
    assert abs(delay * fs - tau) < 1e-9
    # the conjugate spectrum (a lower-sideband stream) has its pulse at conj(P[-b]) and the opposite delay
    Pm = np.conj(np.roll(P[::-1], 1))
    _, _, d_lsb, _ = oracle_lib.pulse_peak(Pm, fs, sideband=-1)
    assert abs(d_lsb - delay) < 1e-9 / fs


@pytest.mark.parametrize("fs,fo,td", [
    (64_000_000, 10_000, 3.7e-9),
    (16_000_000, 250_000, -120e-9),
    (32_000_000, 510_000, 10e-9),
])
def test_pulse_delay_agrees_with_slope_delay(oracle_lib, fs, fo, td):
    """Noiseless Eq. 1 comb (closed-form C_k): the pulse-peak delay and the phase-slope delay are both t_d."""
    spec = synth.CombSpec(fs, 1_000_000, fo, 2, amp=0.3, t_d=td, seed=(9,))
    L = synth.comb_period_length(spec) * 4
    C = _closed_form(spec, L)
    _, _, slope_delay = oracle_lib.results(C, L, fs, 1_000_000, fo)
    _, _, pulse_delay, _ = oracle_lib.pulse_peak(np.fft.ifft(C), fs)
    assert abs(slope_delay - td) < 1e-15
    assert abs(pulse_delay - td) < 1e-15


def test_pulse_delay_from_quantised_stream(oracle_lib):
    """8-bit quantised noisy comb: the pulse of the oracle's own fold recovers t_d to a small fraction of a sample."""
    spec = synth.CombSpec(64_000_000, 1_000_000, 10_000, 8, amp=1.0, t_d=37e-9, sigma=20.0, seed=(3, 1, 0))
    L = 6400 * 160
    packed = synth.make_stream(spec, L)
    P = oracle_lib.fold_rot(packed, 8, L, spec.fs, spec.f_offset, spec.ntones)
    _, _, delay, _ = oracle_lib.pulse_peak(P, spec.fs)
    assert abs(delay - spec.t_d) * spec.fs < 0.05


# ------------------------------------------------------------- planted mistakes

FOLD_MUTANTS = {
    "bin_step_wrong": ("(uint64_t)(nbins % P)) % (uint64_t)P);", "(uint64_t)((nbins + 1) % P)) % (uint64_t)P);"),
    "first_sample_ignores_n0": ("const int64_t i0 = ((b - n0 % nbins) % nbins + nbins) % nbins;",
                                "const int64_t i0 = b;"),
    "phase_start_local": ("% nbins;\n        int64_t m = (int64_t)(((unsigned __int128)(uint64_t)a * (uint64_t)((n0 + i0)",
                          "% nbins;\n        int64_t m = (int64_t)(((unsigned __int128)(uint64_t)a * (uint64_t)((i0)"),
    "offset_reduced_wrong": ("const int64_t a = (fo / g) % P; /* phase index step per sample */",
                             "const int64_t a = (fo / g + 1) % P; /* phase index step per sample */"),
}


def _fold_pins_hold(o) -> bool:
    for fs, fo, N, nbits, L, n0 in BRUTE[:3]:
        rng = np.random.default_rng(L + fo)
        packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
        lv = _np_levels(packed, nbits, L)
        if np.abs(o.fold_rot(packed, nbits, L, fs, fo, N, n0=n0) - _mp_fold(lv, n0, fs, fo, N)).max() > \
                1e-13 * np.abs(lv).sum():
            return False
    return True


def test_fold_pins_hold_on_oracle(oracle_lib):
    assert _fold_pins_hold(core)


@pytest.mark.parametrize("name", sorted(FOLD_MUTANTS))
def test_fold_pins_catch_mutant(tmp_path, name):
    old, new = FOLD_MUTANTS[name]
    src = core.source_text()
    assert src.count(old) == 1, name
    variant = core.build_variant(src.replace(old, new), str(tmp_path / ("mut_%s.so" % name)))
    assert not _fold_pins_hold(variant), name


# ------------------------------------------------------------- delay-corrected band-pass

@pytest.mark.parametrize("fs,fo,td,jit", [
    (64_000_000, 10_000, 3.7e-9, 0.0),
    (64_000_000, 10_000, 3.7e-9, 0.1),
    (16_000_000, 250_000, -120e-9, 0.0),
    (32_000_000, 510_000, 10e-9, 0.05),
])
def test_bandpass_of_noiseless_comb_is_flat(oracle_lib, fs, fo, td, jit):
    """Closed-form C_k of the Eq. 1 comb corrected by its own t_d: phase -pi/2 + eps_k for every tone."""
    spec = synth.CombSpec(fs, 1_000_000, fo, 2, amp=0.3, t_d=td, jitter=jit, seed=(9,))
    L = synth.comb_period_length(spec) * 4
    C = _closed_form(spec, L)
    got = oracle_lib.bandpass(C, fs, 1_000_000, fo, td)
    want = np.angle(np.exp(1j * (synth.tone_jitter(spec) - np.pi / 2)))
    assert np.abs(np.angle(np.exp(1j * (got - want)))).max() < 1e-9
    # raw correlations that are the conjugate of these, read as a lower sideband, give the same band-pass
    got_l = oracle_lib.bandpass(np.conj(C), fs, 1_000_000, fo, td, sideband=-1)
    assert np.abs(np.angle(np.exp(1j * (got_l - want)))).max() < 1e-9


def test_bandpass_zero_delay_is_the_phase(oracle_lib):
    rng = np.random.default_rng(3)
    C = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    assert np.array_equal(oracle_lib.bandpass(C, 64_000_000, 1_000_000, 10_000, 0.0), np.angle(C))


PULSE_MUTANTS = {
    "delay_sign": ("delay = (-pos if sideband > 0 else pos) / float(fs)", "delay = (pos if sideband > 0 else -pos) / float(fs)"),
    "neighbour_swapped": ("if a_p > a_m:\n        s, a_s = 1, a_p", "if a_p > a_m:\n        s, a_s = -1, a_p"),
    "envelope_period": ("u = math.pi / n", "u = 2.0 * math.pi / n"),
    "plain_hyperbola": ("d = math.atan2(a_s * math.sin(u), a_0 + a_s * math.cos(u)) / u if s else 0.0",
                        "d = a_s / (a_0 + a_s) if s else 0.0"),
    "no_wrap": ("    if pos > n / 2.0:\n        pos -= n\n", ""),
    "bandpass_sign": ("np.exp(-2j * np.pi * f * delay)", "np.exp(2j * np.pi * f * delay)"),
    "bandpass_no_offset": ("f = f_offset + f_comb * np.arange", "f = f_comb * np.arange"),
}


def _pulse_variant(old, new):
    import types

    import oracle.pulse as op

    src = open(op.__file__).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("pulse_variant")
    exec(compile(src.replace(old, new), "pulse_variant", "exec"), mod.__dict__)
    return mod


def _pulse_pins_hold(m) -> bool:
    fs, N = 64_000_000, 64
    P = np.zeros(N, dtype=np.complex128)
    P[50] = 1.0
    if m.pulse_peak(P, fs)[2] != 14 / fs:
        return False
    for tau in (0.25, 3.7, -5.3):
        k = np.arange(N)
        Pc = np.fft.ifft(np.exp(2j * np.pi * k * tau / N))
        if abs(m.pulse_peak(Pc, N * 1_000_000)[2] * N * 1_000_000 - tau) > 1e-9:
            return False
    spec = synth.CombSpec(64_000_000, 1_000_000, 10_000, 2, amp=0.3, t_d=3.7e-9, seed=(9,))
    C = _closed_form(spec, synth.comb_period_length(spec) * 4)
    got = m.bandpass(C, spec.fs, 1_000_000, 10_000, spec.t_d)
    return bool(np.abs(np.angle(np.exp(1j * (got + np.pi / 2)))).max() < 1e-9)


def test_pulse_pins_hold_on_oracle():
    import oracle.pulse as op

    assert _pulse_pins_hold(op)


@pytest.mark.parametrize("name", sorted(PULSE_MUTANTS))
def test_pulse_pins_catch_mutant(name):
    assert not _pulse_pins_hold(_pulse_variant(*PULSE_MUTANTS[name])), name
