"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test ties the oracle to something the paper or the mathematics fixes:
printed constants (Eq. 4, Eq. 5), hand-built decoder cases, 40-digit brute
force on tiny inputs, library FFTs in the special cases where the per-tone
correlation *is* a DFT bin, closed forms of the noiseless Eq. 1 comb,
symmetry/linearity invariants, and the least-squares delay of known phases.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import synth
from tests.conftest import golden_path


def _read_golden(name):
    rows = []
    with open(golden_path(name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line)
    return rows


def _np_levels(packed, nbits, nsamples):
    """Test-local decoder (same convention as the golden decode fixture)."""
    b = np.asarray(packed, dtype=np.uint8)
    if nbits == 2:
        codes = (b[:, None] >> np.array([0, 2, 4, 6], dtype=np.uint8)) & 3
        return (2 * codes.astype(np.int64) - 3).reshape(-1)[:nsamples]
    return b.view(np.int8).astype(np.int64)[:nsamples]


# ---------------------------------------------------------------- printed values

def test_paper_constants(oracle_lib):
    rows = _read_golden("paper_constants.txt")
    assert len(rows) == 3
    for row in rows:
        name, fs, fc, fo, val = row.split()
        fs, fc, fo = int(fs), int(fc), int(fo)
        if name == "rotator_period":
            assert oracle_lib.rotator_period(fs, fo) == int(val)
        elif name == "ntones":
            assert oracle_lib.ntones(fs, fc) == int(val)
        elif name == "phase_step":
            assert abs(oracle_lib.phase_step(fs, fo) - float(val)) < 1e-17
        else:
            raise AssertionError(name)


def test_decoder_golden(oracle_lib):
    for row in _read_golden("decode.txt"):
        lhs, rhs = row.split(":")
        parts = lhs.split()
        nbits = int(parts[0])
        data = np.array([int(h, 16) for h in parts[1:]], dtype=np.uint8)
        want = np.array([int(v) for v in rhs.split()], dtype=np.int64)
        got = oracle_lib.decode(data, nbits, want.size).astype(np.int64)
        np.testing.assert_array_equal(got, want)
        np.testing.assert_array_equal(_np_levels(data, nbits, want.size), want)


def test_generator_packing_matches_decoder(oracle_lib):
    rng = np.random.default_rng(7)
    codes = rng.integers(0, 4, size=4096).astype(np.uint8)
    packed = synth.pack_2bit(codes)
    np.testing.assert_array_equal(oracle_lib.decode(packed, 2, codes.size), synth.levels_2bit(codes))


# ---------------------------------------------------------------- brute force

def _mp_correlate(levels, n0, fs, fc, fo, k):
    mp.mp.dps = 40
    f = k * fc + fo
    acc = mp.mpc(0)
    for i, x in enumerate(levels):
        if x:
            acc += int(x) * mp.expj(-2 * mp.pi * mp.mpf(f * (n0 + i)) / fs)
    return complex(acc)


@pytest.mark.parametrize("fs,fc,fo,nbits,L,n0", [
    (16_000_000, 1_000_000, 10_000, 2, 1024, 0),
    (16_000_000, 1_000_000, 250_000, 2, 512, 12345),
    (32_000_000, 1_000_000, 0, 8, 768, 7),
    (64_000_000, 2_000_000, 10_007, 8, 400, 10 ** 9 + 3),   # prime offset: no phasor table
    (24_000_000, 1_000_000, 510_000, 2, 256, 2 ** 33 + 1),  # large global index
])
def test_mpmath_bruteforce(oracle_lib, fs, fc, fo, nbits, L, n0):
    rng = np.random.default_rng(fs % 1000 + L + fo)
    packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
    lv = _np_levels(packed, nbits, L)
    N = fs // fc
    tones = sorted(set([0, 1, N // 2, N - 1, int(rng.integers(N))]))
    got = oracle_lib.correlate(packed, nbits, L, fs, fc, fo, n0=n0, tones=tones)
    scale = np.abs(lv).sum()
    for t, c in zip(tones, got):
        want = _mp_correlate(lv, n0, fs, fc, fo, t)
        assert abs(c - want) <= 1e-13 * scale, (t, c, want)


# ---------------------------------------------------------------- library FFT special case

@pytest.mark.parametrize("fs,fc,fo,reps,n0", [
    (16_000_000, 1_000_000, 10_000, 2, 0),
    (64_000_000, 1_000_000, 250_000, 3, 0),
    (32_000_000, 1_000_000, 0, 5, 0),
    (16_000_000, 1_000_000, 510_000, 1, 987654321),
])
def test_fft_special_case(oracle_lib, fs, fc, fo, reps, n0):
    """With L a multiple of P = fs/gcd(fs,f_comb,f_offset), C_k is bin m_k of an L-point FFT."""
    g = math.gcd(math.gcd(fs, fc), fo)
    P = fs // g
    L = P * reps
    rng = np.random.default_rng(L)
    x = rng.standard_normal(L)
    N = fs // fc
    got = oracle_lib.correlate_f64(x, fs, fc, fo, n0=n0)
    X = np.fft.fft(x)
    for k in range(N):
        a = (k * fc + fo) // g
        m = (a * reps) % L
        shift = np.exp(-2j * np.pi * ((a * n0) % P) / P)
        assert abs(got[k] - shift * X[m]) <= 1e-11 * np.sqrt(L), k


def test_fft_special_case_packed(oracle_lib):
    fs, fc, fo = 32_000_000, 1_000_000, 10_000
    P = fs // math.gcd(math.gcd(fs, fc), fo)  # 3200
    L = 2 * P
    rng = np.random.default_rng(3)
    for nbits in (2, 8):
        packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
        x = _np_levels(packed, nbits, L).astype(np.float64)
        got = oracle_lib.correlate(packed, nbits, L, fs, fc, fo)
        X = np.fft.fft(x)
        g = fs // P
        for k in range(fs // fc):
            m = (((k * fc + fo) // g) * 2) % L
            assert abs(got[k] - X[m]) <= 1e-11 * np.abs(x).sum()


# ---------------------------------------------------------------- integer fold (Eq. 2)

@pytest.mark.parametrize("nbits,N,L,n0", [(2, 32, 4096 + 12, 0), (2, 64, 10000, 4 * 777), (8, 1024, 5000, 3)])
def test_fold_int_matches_reshape(oracle_lib, nbits, N, L, n0):
    rng = np.random.default_rng(N + L)
    packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
    x = _np_levels(packed, nbits, L)
    want = np.zeros(N, dtype=np.int64)
    np.add.at(want, (np.arange(L) + n0) % N, x)
    got = oracle_lib.fold_int(packed, nbits, L, N, n0=n0)
    np.testing.assert_array_equal(got, want)


def test_core_identity_f0(oracle_lib):
    """f_offset = 0: the DFT of the Eq. 2 bins equals the per-tone correlation (two oracle functions)."""
    fs, fc = 32_000_000, 1_000_000
    N = fs // fc
    rng = np.random.default_rng(11)
    L = 4 * 3001
    packed = rng.integers(0, 256, size=L // 4, dtype=np.uint8)
    for n0 in (0, 4 * 5):
        P = oracle_lib.fold_int(packed, 2, L, N, n0=n0).astype(np.float64)
        C = oracle_lib.correlate(packed, 2, L, fs, fc, 0, n0=n0)
        np.testing.assert_allclose(np.fft.fft(P), C, rtol=0, atol=1e-9 * np.abs(P).sum())
        assert C[0].real == pytest.approx(P.sum(), abs=1e-9)


# ---------------------------------------------------------------- closed forms of Eq. 1

def _closed_form(spec, L):
    """C_k of the noiseless comb over L samples (L a multiple of the comb period)."""
    fs, fc, fo = spec.fs, spec.f_comb, spec.f_offset
    N = fs // fc
    phi = synth.tone_phases(spec)
    out = np.zeros(N, dtype=np.complex128)
    for k in range(N):
        fk = k * fc + fo
        v = np.exp(1j * phi[k])
        for m in range(N):
            if (m * fc + fo + fk) % fs == 0:
                v -= np.exp(-1j * phi[m])
        out[k] = spec.amp * L / 2j * v
    return out


@pytest.mark.parametrize("fs,fo,td,jit", [
    (16_000_000, 10_000, 3.7e-9, 0.0),
    (64_000_000, 10_000, 3.7e-9, 0.1),
    (16_000_000, 250_000, 12e-9, 0.0),
    (32_000_000, 0, 10e-9, 0.0),
    (32_000_000, 500_000, 7e-9, 0.0),   # f_offset = f_comb / 2: tone k meets its mirror N-1-k
])
def test_closed_form_noiseless(oracle_lib, fs, fo, td, jit):
    spec = synth.CombSpec(fs, 1_000_000, fo, 2, amp=0.3, t_d=td, jitter=jit, seed=(9,))
    per = synth.comb_period(spec)
    L = 3 * per.size
    x = np.tile(per, 3)
    got = oracle_lib.correlate_f64(x, spec.fs, spec.f_comb, spec.f_offset)
    want = _closed_form(spec, L)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * spec.amp * L)


def test_closed_form_f0_amplitude():
    """f_offset = 0 (Section 2, Eq. 2 case): |C_k|/L = A |sin(pi fs t_d)| and arg C_k = phi_k - pi fs t_d."""
    spec = synth.CombSpec(32_000_000, 1_000_000, 0, 2, amp=0.05, t_d=10e-9)
    import oracle

    per = synth.comb_period(spec)
    L = 2 * per.size
    C = oracle.correlate_f64(np.tile(per, 2), spec.fs, spec.f_comb, 0)
    s = math.sin(math.pi * spec.fs * spec.t_d)
    phi = synth.tone_phases(spec)
    for k in range(1, spec.ntones):
        assert abs(abs(C[k]) / L - spec.amp * abs(s)) < 1e-14
        d = np.angle(C[k] * np.exp(-1j * (phi[k] - math.pi * spec.fs * spec.t_d)))
        assert abs(d) < 1e-12
    assert abs(C[0]) < 1e-12 * L


# ---------------------------------------------------------------- invariants

def test_linearity_and_chunking(oracle_lib):
    fs, fc, fo = 16_000_000, 1_000_000, 10_000
    rng = np.random.default_rng(5)
    L = 50_000
    x = rng.standard_normal(L)
    y = rng.standard_normal(L)
    cx = oracle_lib.correlate_f64(x, fs, fc, fo)
    cy = oracle_lib.correlate_f64(y, fs, fc, fo)
    cxy = oracle_lib.correlate_f64(x + 2.5 * y, fs, fc, fo)
    np.testing.assert_allclose(cxy, cx + 2.5 * cy, rtol=0, atol=1e-10)
    for cut in (1, 12_345, 49_999):
        a = oracle_lib.correlate_f64(x[:cut], fs, fc, fo, n0=0)
        b = oracle_lib.correlate_f64(x[cut:], fs, fc, fo, n0=cut)
        np.testing.assert_allclose(a + b, cx, rtol=0, atol=1e-10)


def test_packed_chunking(oracle_lib):
    spec = synth.CombSpec(64_000_000, 1_000_000, 10_000, 2, amp=0.02, t_d=3.7e-9, seed=(2, 1))
    L = 1 << 18
    b = synth.make_stream(spec, L)
    whole = oracle_lib.correlate(b, 2, L, spec.fs, spec.f_comb, spec.f_offset)
    cut = 4 * 12_345
    p1 = oracle_lib.correlate(b[:cut // 4], 2, cut, spec.fs, spec.f_comb, spec.f_offset)
    p2 = oracle_lib.correlate(b[cut // 4:], 2, L - cut, spec.fs, spec.f_comb, spec.f_offset, n0=cut)
    np.testing.assert_allclose(p1 + p2, whole, rtol=0, atol=1e-8)
    # regenerating a sub-range of the stream gives the same bytes
    np.testing.assert_array_equal(synth.make_stream(spec, L - cut, n0=cut), b[cut // 4:])


def test_long_period_comb_evaluated_directly():
    """For a comb period longer than the range generated, the generator evaluates the comb at the samples
    themselves: the same values, to the bit, as the period table at those indices (and so the same bytes
    for a sub-range cut out of a longer generation, across a period boundary too)."""
    spec = synth.CombSpec(4_000_000, 1_000_000, 1_001, 2, amp=0.3, t_d=2e-9, seed=(9, 1))
    per = synth.comb_period(spec)
    assert per.size == 4_000_000
    for start, count in [(0, 4096), (3_998_000, 5000), (123_457, 1)]:
        idx = np.arange(start, start + count) % per.size
        np.testing.assert_array_equal(synth.comb_values(spec, start, count), per[idx])
    whole = synth.make_stream(spec, 8_000_000)            # two periods: the table path
    part = synth.make_stream(spec, 1 << 16, n0=3_990_000)  # shorter than the period: the direct path
    np.testing.assert_array_equal(part, whole[3_990_000 // 4:(3_990_000 + (1 << 16)) // 4])


def test_conjugate_symmetry(oracle_lib):
    rng = np.random.default_rng(8)
    x = rng.standard_normal(7777)
    fs, fc = 16_000_000, 1_000_000
    N = fs // fc
    C = oracle_lib.correlate_f64(x, fs, fc, 0)
    for k in range(1, N):
        assert abs(C[N - k] - np.conj(C[k])) < 1e-10
    C = oracle_lib.correlate_f64(x, fs, fc, fc // 2)
    for k in range(N):
        assert abs(C[N - 1 - k] - np.conj(C[k])) < 1e-10


# ---------------------------------------------------------------- amplitude / phase / delay

@pytest.mark.parametrize("fs,fo,td,jit", [
    (64_000_000, 10_000, 3.7e-9, 0.0),
    (64_000_000, 10_000, 3.7e-9, 0.1),
    (32_000_000, 0, 10e-9, 0.0),
    (16_000_000, 250_000, -40e-9, 0.0),
])
def test_delay_fit_noiseless(oracle_lib, fs, fo, td, jit):
    spec = synth.CombSpec(fs, 1_000_000, fo, 2, amp=0.1, t_d=td, jitter=jit, seed=(21,))
    per = synth.comb_period(spec)
    L = 2 * per.size
    C = oracle_lib.correlate_f64(np.tile(per, 2), spec.fs, spec.f_comb, spec.f_offset)
    amp, phase, delay = oracle_lib.results(C, L, spec.fs, spec.f_comb, spec.f_offset)
    k = oracle_lib.in_band(spec.fs, spec.f_comb, spec.f_offset)
    f = spec.f_offset + spec.f_comb * k.astype(np.float64)
    if jit == 0.0:
        assert abs(delay - td) < 1e-15
    else:
        phi = synth.tone_phases(spec)[k] - np.pi / 2
        want = np.polyfit(f, phi, 1)[0] / (2 * np.pi)
        assert abs(delay - want) < 1e-15
    if fo != 0:
        phi = synth.tone_phases(spec) - np.pi / 2
        assert np.max(np.abs(np.angle(np.exp(1j * (phase - phi))))) < 1e-12
        np.testing.assert_allclose(amp, spec.amp / 2, rtol=1e-12)
    # lower sideband: conjugate phases, negated delay
    amp2, phase2, delay2 = oracle_lib.results(C, L, spec.fs, spec.f_comb, spec.f_offset, sideband=-1)
    np.testing.assert_allclose(amp2, amp)
    assert abs(delay2 + delay) < 1e-15


def test_in_band_tones(oracle_lib):
    np.testing.assert_array_equal(oracle_lib.in_band(32_000_000, 1_000_000, 0), np.arange(1, 16))
    np.testing.assert_array_equal(oracle_lib.in_band(64_000_000, 1_000_000, 10_000), np.arange(0, 32))
    assert oracle_lib.in_band(1_024_000_000, 1_000_000, 510_000).size == 512


@pytest.mark.parametrize("nbits", [2, 8])
def test_statistical_recovery(oracle_lib, nbits):
    """Quantised comb + noise: C_k lies within 6 noise sigma of its expectation.

    The expectation is exact: the mean quantiser output given the comb value
    p is E[level] = 2 * sum_t Phi((p - t) / sigma) - 3 for the 2-bit thresholds t
    (Gaussian noise), or p itself for 8-bit with sigma = 20 LSB (rounding and
    clipping are negligible there).  Its C_k follows from an FFT of one comb
    period, since L is a multiple of the period.  The injected phases are then
    recovered to within the same noise bound.
    """
    from scipy.special import ndtr

    if nbits == 2:
        spec = synth.CombSpec(64_000_000, 1_000_000, 10_000, 2, amp=0.02, t_d=3.7e-9, seed=(31,))
    else:
        spec = synth.CombSpec(64_000_000, 1_000_000, 10_000, 8, amp=1.0, t_d=25e-9, sigma=20.0, seed=(32,))
    L = 655 * 6400
    L -= L % 4
    per = synth.comb_period(spec)
    P = per.size
    reps = L // P
    L = reps * P
    b = synth.make_stream(spec, L)
    C = oracle_lib.correlate(b, nbits, L, spec.fs, spec.f_comb, spec.f_offset)
    if nbits == 2:
        ev = 2.0 * sum(ndtr((per - t) / spec.sigma) for t in synth.TWO_BIT_THRESHOLDS) - 3.0
        var = 9.0 * 2 * ndtr(-0.98) + 1.0 * (1 - 2 * ndtr(-0.98))
    else:
        ev = per.copy()
        var = spec.sigma ** 2
    X = np.fft.fft(ev) * reps
    g = spec.fs // P
    N = spec.ntones
    Cexp = np.array([X[((k * spec.f_comb + spec.f_offset) // g) % P] for k in range(N)])
    sig = np.sqrt(var * L / 2)          # per-component noise standard deviation of C_k
    assert np.max(np.abs(C - Cexp)) < 6 * sig, (np.max(np.abs(C - Cexp)) / sig)
    amp, phase, delay = oracle_lib.results(C, L, spec.fs, spec.f_comb, spec.f_offset)
    k = oracle_lib.in_band(spec.fs, spec.f_comb, spec.f_offset)
    phi = synth.tone_phases(spec) - np.pi / 2
    err = np.angle(np.exp(1j * (phase[k] - phi[k])))
    assert np.max(np.abs(err)) < 6 * sig / np.min(np.abs(Cexp[k])) + 1e-3


# ---------------------------------------------------------------- correlation with a supplied rotator

def _exact_tables(fs, fc, fo, rows):
    N = fs // fc
    u = np.exp(-2j * np.pi * ((fo * N * np.arange(rows)) % fs) / fs)
    v = np.exp(-2j * np.pi * ((fo * np.arange(N)) % fs) / fs)
    return u, v


@pytest.mark.parametrize("fs,fc,fo,nbits,rows,L,n0", [
    (64_000_000, 1_000_000, 10_000, 2, 100, 4 * 20_011, 4 * 3),
    (16_000_000, 1_000_000, 250_000, 8, 4, 9_999, 17),
    (24_000_000, 1_000_000, 500_000, 2, 2, 4 * 777, 0),
])
def test_rotator_form_with_exact_tables_is_plain_correlation(oracle_lib, fs, fc, fo, nbits, rows, L, n0):
    """With the exact factor tables the rotator form reduces to the plain definition."""
    rng = np.random.default_rng(rows + L)
    packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
    u, v = _exact_tables(fs, fc, fo, rows)
    got = oracle_lib.correlate_rotator(packed, nbits, L, fs // fc, u, v, n0=n0)
    want = oracle_lib.correlate(packed, nbits, L, fs, fc, fo, n0=n0)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-10 * np.abs(_np_levels(packed, nbits, L)).sum())


def test_rotator_form_bruteforce_rounded_tables(oracle_lib):
    """Perturbed tables: 40-digit brute force of the rotator-form definition."""
    fs, fc, fo, rows = 16_000_000, 1_000_000, 10_000, 100
    N = fs // fc
    u, v = _exact_tables(fs, fc, fo, rows)
    u = u.real.astype(np.float16).astype(float) + 1j * u.imag.astype(np.float16).astype(float)
    rng = np.random.default_rng(4)
    L, n0 = 300, 4 * 401
    packed = rng.integers(0, 256, size=L // 4, dtype=np.uint8)
    lv = _np_levels(packed, 2, L)
    got = oracle_lib.correlate_rotator(packed, 2, L, N, u, v, n0=n0, tones=[0, 5, 15])
    mp.mp.dps = 40
    for t, c in zip([0, 5, 15], got):
        acc = mp.mpc(0)
        for i, x in enumerate(lv):
            q = (n0 + i) % (rows * N)
            col, row = q % N, q // N
            r = mp.mpc(u[row].real, u[row].imag) * mp.mpc(v[col].real, v[col].imag)
            acc += int(x) * r * mp.expj(-2 * mp.pi * mp.mpf(t * col) / N)
        assert abs(c - complex(acc)) < 1e-12 * np.abs(lv).sum()
