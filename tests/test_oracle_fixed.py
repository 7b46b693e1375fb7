"""Pins of the oracle's fixed-point rotator fold (Section 4.8's integer rotator; CPU only).

orc_fold_table_int sums x[n] * T[n mod R] into bin n mod N exactly in
integers; fixed_rotator gives the rotator of Eq. 3 over one period (Eq. 4)
scaled by 2^17 and rounded.  Pinned to a plain Python loop on tiny inputs,
to the integer fold of Eq. 2 for the unit table, to the exact rotator at
the quarter-rate offset, to the rounding bound of every entry and of the
bins against the FP64 rotated fold, and to chunking with a global index.
Planted mistakes in the C source each break a pin.
"""
import numpy as np
import pytest

from oracle import core
from tests.test_oracle import _np_levels


def _py_fold(levels, n0, N, table):
    R = len(table)
    re = [0] * N
    im = [0] * N
    for i, x in enumerate(levels):
        n = n0 + i
        t = table[n % R]
        re[n % N] += int(x) * int(t.real)
        im[n % N] += int(x) * int(t.imag)
    return np.array(re, dtype=np.int64), np.array(im, dtype=np.int64)


TINY = [(2, 16, 7, 400, 0), (8, 24, 100, 333, 12345), (8, 64, 1, 256, 2 ** 40 + 3), (2, 32, 6400, 1024, 99)]


@pytest.mark.parametrize("nbits,N,R,L,n0", TINY)
def test_fold_table_int_python_loop(oracle_lib, nbits, N, R, L, n0):
    rng = np.random.default_rng(N * R + L)
    packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
    table = rng.integers(-40000, 40000, size=R) + 1j * rng.integers(-40000, 40000, size=R)
    got = oracle_lib.fold_table_int(packed, nbits, L, N, table, n0=n0)
    want = _py_fold(_np_levels(packed, nbits, L), n0, N, table)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_unit_table_is_integer_fold(oracle_lib):
    rng = np.random.default_rng(5)
    for nbits, N, L, n0 in ((2, 32, 4096, 0), (8, 1024, 5000, 77)):
        packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
        re, im = oracle_lib.fold_table_int(packed, nbits, L, N, np.ones(7, dtype=complex), n0=n0)
        assert np.array_equal(re, oracle_lib.fold_int(packed, nbits, L, N, n0=n0)) and not im.any()


def test_fixed_rotator_entries():
    """Integers within 2^-18 sqrt(2) (times 2^17) of the exact rotator; exact at the quarter rate."""
    T = core.fixed_rotator(16_000_000, 4_000_000)
    assert np.array_equal(T, np.array([131072, -131072j, -131072, 131072j]))
    for fs, fo in ((64_000_000, 10_000), (1_024_000_000, 510_000), (64_000_000, 10_008)):
        T = core.fixed_rotator(fs, fo)
        R = fs // np.gcd(fs, fo)
        assert T.size == R and T[0] == 131072
        assert np.array_equal(T.real, np.round(T.real)) and np.array_equal(T.imag, np.round(T.imag))
        r = np.arange(R)
        exact = np.exp(-2j * np.pi * ((fo * r) % fs) / fs)
        assert np.abs(T / 131072.0 - exact).max() <= 2 ** -18 * np.sqrt(2) + 1e-15


@pytest.mark.parametrize("fs,fo,nbits,N,L,n0", [(64_000_000, 10_000, 2, 64, 6400 * 5 + 44, 3),
                                                (1_024_000_000, 510_000, 8, 1024, 300_000, 2 ** 28 + 5)])
def test_fixed_bins_within_rounding_of_fp64_fold(oracle_lib, fs, fo, nbits, N, L, n0):
    rng = np.random.default_rng(L)
    packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
    T = core.fixed_rotator(fs, fo)
    re, im = oracle_lib.fold_table_int(packed, nbits, L, N, T, n0=n0)
    P = oracle_lib.fold_rot(packed, nbits, L, fs, fo, N, n0=n0)
    lv = np.abs(_np_levels(packed, nbits, L))
    bound = np.bincount((n0 + np.arange(L)) % N, weights=lv, minlength=N) * 2 ** -18 * np.sqrt(2)
    assert np.all(np.abs((re + 1j * im) / 131072.0 - P) <= bound + 1e-9)


def test_fixed_chunking(oracle_lib):
    rng = np.random.default_rng(8)
    L, N = 8000, 64
    packed = rng.integers(0, 256, size=L // 4, dtype=np.uint8)
    T = core.fixed_rotator(64_000_000, 10_000)
    whole = oracle_lib.fold_table_int(packed, 2, L, N, T, n0=1000)
    a = oracle_lib.fold_table_int(packed[:500], 2, 2000, N, T, n0=1000)
    b = oracle_lib.fold_table_int(packed[500:], 2, 6000, N, T, n0=3000)
    assert np.array_equal(whole[0], a[0] + b[0]) and np.array_equal(whole[1], a[1] + b[1])


FIXED_MUTANTS = {
    "table_index_local": ("int64_t b = n0 % nbins, r = n0 % R;", "int64_t b = n0 % nbins, r = 0;"),
    "bin_index_local": ("int64_t b = n0 % nbins, r = n0 % R;", "int64_t b = 0, r = n0 % R;"),
    "imag_sign": ("im[b] += x * t_im[r];", "im[b] -= x * t_im[r];"),
    "table_wraps_late": ("if (++r == R) r = 0;", "if (++r > R) r = 0;"),
}


def _fixed_pins_hold(o) -> bool:
    for nbits, N, R, L, n0 in TINY:
        rng = np.random.default_rng(N * R + L)
        packed = rng.integers(0, 256, size=L * nbits // 8, dtype=np.uint8)
        table = rng.integers(-40000, 40000, size=R) + 1j * rng.integers(-40000, 40000, size=R)
        got = o.fold_table_int(packed, nbits, L, N, table, n0=n0)
        want = _py_fold(_np_levels(packed, nbits, L), n0, N, table)
        if not (np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])):
            return False
    return True


def test_fixed_pins_hold_on_oracle(oracle_lib):
    assert _fixed_pins_hold(core)


@pytest.mark.parametrize("name", sorted(FIXED_MUTANTS))
def test_fixed_pins_catch_mutant(tmp_path, name):
    old, new = FIXED_MUTANTS[name]
    src = core.source_text()
    assert src.count(old) == 1, name
    variant = core.build_variant(src.replace(old, new), str(tmp_path / ("mut_%s.so" % name)))
    assert not _fixed_pins_hold(variant), name
