"""ctypes wrapper over the plain-C FP64 oracle (``pcal_oracle.c``).  Test infrastructure only."""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcal_oracle.c")
_LIB = os.path.join(_HERE, "libpcal_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE FP64: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _bind(path: str):
    lib = ctypes.CDLL(path)
    i64, i32, p = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    lib.orc_correlate_packed.argtypes = [p, i32, i64, i64, i64, i64, i64, i32, p, i32, p, p]
    lib.orc_correlate_f64.argtypes = [p, i64, i64, i64, i64, i64, i32, p, i32, p, p]
    lib.orc_fold_int.argtypes = [p, i32, i64, i64, i64, p]
    lib.orc_decode.argtypes = [p, i32, i64, p]
    lib.orc_correlate_rotator.argtypes = [p, i32, i64, i64, i64, i64, p, p, p, p, i32, p, i32, p, p]
    lib.orc_fold_rot.argtypes = [p, i32, i64, i64, i64, i64, i64, i32, p, p]
    lib.orc_fold_table_int.argtypes = [p, i32, i64, i64, i64, i64, p, p, p, p]
    for f in (lib.orc_correlate_packed, lib.orc_correlate_f64, lib.orc_fold_int, lib.orc_decode,
              lib.orc_max_threads, lib.orc_correlate_rotator, lib.orc_fold_rot, lib.orc_fold_table_int):
        f.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _bind(_LIB)
    return _lib


class Variant:
    """The same entry points bound to another build of the oracle source (used by mutation tests)."""

    def __init__(self, path: str):
        self._l = _bind(path)

    def __getattr__(self, name):
        fn = globals()[name]

        def call(*a, **kw):
            global _lib
            saved = _lib
            _lib = self._l
            try:
                return fn(*a, **kw)
            finally:
                _lib = saved
        return call


def build_variant(source: str, path: str) -> "Variant":
    """Compile oracle C source text (e.g. with a planted mistake) to ``path`` and bind it."""
    src = path + ".c"
    with open(src, "w") as fh:
        fh.write(source)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=gnu11", "-shared", "-fPIC",
                    "-o", path, src, "-lm"], check=True)
    return Variant(path)


def source_text() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _bytes(packed) -> np.ndarray:
    if hasattr(packed, "detach"):  # a torch tensor: take a host copy
        packed = packed.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(packed, dtype=np.uint8))


def _tones(fs: int, fc: int, tones: Optional[Sequence[int]]) -> np.ndarray:
    if tones is None:
        tones = range(fs // fc)
    return np.ascontiguousarray(np.asarray(list(tones), dtype=np.int32))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def correlate(packed, nbits: int, nsamples: int, fs: int, fc: int, fo: int, n0: int = 0,
              tones: Optional[Sequence[int]] = None, nthreads: int = 0) -> np.ndarray:
    """C_k for the requested tones (default: all N) of packed 2-/8-bit samples; complex128."""
    b = _bytes(packed)
    need = (nsamples * nbits + 7) // 8
    if b.size < need:
        raise ValueError("packed buffer holds fewer than nsamples samples")
    t = _tones(fs, fc, tones)
    re = np.zeros(t.size)
    im = np.zeros(t.size)
    rc = _load().orc_correlate_packed(_ptr(b), nbits, nsamples, n0, fs, fc, fo, t.size, _ptr(t),
                                      nthreads, _ptr(re), _ptr(im))
    if rc:
        raise ValueError("oracle rejected the arguments (code %d)" % rc)
    return re + 1j * im


def correlate_f64(x, fs: int, fc: int, fo: int, n0: int = 0, tones: Optional[Sequence[int]] = None,
                  nthreads: int = 0) -> np.ndarray:
    """C_k of real FP64 samples (used by the closed-form checks on unquantised combs)."""
    xs = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    t = _tones(fs, fc, tones)
    re = np.zeros(t.size)
    im = np.zeros(t.size)
    rc = _load().orc_correlate_f64(_ptr(xs), xs.size, n0, fs, fc, fo, t.size, _ptr(t), nthreads,
                                   _ptr(re), _ptr(im))
    if rc:
        raise ValueError("oracle rejected the arguments (code %d)" % rc)
    return re + 1j * im


def correlate_rotator(packed, nbits: int, nsamples: int, nbins: int, u, v, n0: int = 0,
                      tones: Optional[Sequence[int]] = None, nthreads: int = 0) -> np.ndarray:
    """C_k with the rotator read from tables: U (rows, complex) times V (nbins, complex).

    Equals :func:`correlate` for the exact tables U[m] = exp(-j w_o N m),
    V[b] = exp(-j w_o b); with rounded tables it is what an extraction that
    rotates by the rounded values computes in exact arithmetic.
    """
    b = _bytes(packed)
    u = np.asarray(u, dtype=np.complex128)
    v = np.asarray(v, dtype=np.complex128)
    if v.size != nbins:
        raise ValueError("v needs nbins entries")
    ur, ui = np.ascontiguousarray(u.real), np.ascontiguousarray(u.imag)
    vr, vi = np.ascontiguousarray(v.real), np.ascontiguousarray(v.imag)
    t = np.ascontiguousarray(np.asarray(list(range(nbins)) if tones is None else list(tones), dtype=np.int32))
    re = np.zeros(t.size)
    im = np.zeros(t.size)
    rc = _load().orc_correlate_rotator(_ptr(b), nbits, nsamples, n0, nbins, u.size, _ptr(ur), _ptr(ui), _ptr(vr),
                                       _ptr(vi), t.size, _ptr(t), nthreads, _ptr(re), _ptr(im))
    if rc:
        raise ValueError("oracle rejected the arguments (code %d)" % rc)
    return re + 1j * im


def fold_int(packed, nbits: int, nsamples: int, nbins: int, n0: int = 0) -> np.ndarray:
    """Eq. 2 integer bins: P[b] = sum of x[n], n = b (mod nbins), int64."""
    b = _bytes(packed)
    out = np.zeros(nbins, dtype=np.int64)
    rc = _load().orc_fold_int(_ptr(b), nbits, nsamples, n0, nbins, _ptr(out))
    if rc:
        raise ValueError("oracle rejected the arguments (code %d)" % rc)
    return out


def fold_rot(packed, nbits: int, nsamples: int, fs: int, f_offset: int, nbins: int, n0: int = 0,
             nthreads: int = 0) -> np.ndarray:
    """Eqs. 2-3 rotated bins: P[b] = sum of x[n] exp(-j 2 pi f_offset n / fs), n = b (mod nbins), complex."""
    b = _bytes(packed)
    re = np.zeros(nbins)
    im = np.zeros(nbins)
    rc = _load().orc_fold_rot(_ptr(b), nbits, nsamples, n0, fs, f_offset, nbins, nthreads, _ptr(re), _ptr(im))
    if rc:
        raise ValueError("oracle rejected the arguments (code %d)" % rc)
    return re + 1j * im


def fold_table_int(packed, nbits: int, nsamples: int, nbins: int, table, n0: int = 0):
    """Eqs. 2-3 with an integer rotator table T (complex, integer parts, length R = the rotator period):
    P[b] = sum of x[n] T[n mod R] over n = b (mod nbins), exact; returns (re, im) as int64 arrays."""
    b = _bytes(packed)
    t = np.asarray(table)
    tr = np.ascontiguousarray(np.asarray(t.real, dtype=np.int32))
    ti = np.ascontiguousarray(np.asarray(t.imag, dtype=np.int32))
    if not (np.array_equal(tr, t.real) and np.array_equal(ti, t.imag)):
        raise ValueError("table entries must be integers within int32")
    re = np.zeros(nbins, dtype=np.int64)
    im = np.zeros(nbins, dtype=np.int64)
    rc = _load().orc_fold_table_int(_ptr(b), nbits, nsamples, n0, nbins, tr.size, _ptr(tr), _ptr(ti), _ptr(re),
                                    _ptr(im))
    if rc:
        raise ValueError("oracle rejected the arguments (code %d)" % rc)
    return re, im


def fixed_rotator(fs: int, f_offset: int, frac_bits: int = 17) -> np.ndarray:
    """The rotator exp(-j 2 pi f_offset r / fs) over one period R = fs / gcd(fs, f_offset) (Eq. 4), scaled by
    2^frac_bits and rounded to the nearest integer (ties to even): the fixed-point rotator of Section 4.8.
    Complex array whose parts are integers."""
    from math import gcd

    R = fs // gcd(fs, f_offset)
    r = np.arange(R, dtype=np.int64)
    idx = (f_offset * r) % fs                                  # exact phase index
    ang = 2.0 * np.pi * idx.astype(np.float64) / float(fs)
    scale = float(1 << frac_bits)
    return np.rint(scale * np.cos(ang)) - 1j * np.rint(scale * np.sin(ang))


def decode(packed, nbits: int, nsamples: int) -> np.ndarray:
    """Sample levels (int8) decoded by the oracle's own unpacker."""
    b = _bytes(packed)
    out = np.zeros(nsamples, dtype=np.int8)
    rc = _load().orc_decode(_ptr(b), nbits, nsamples, _ptr(out))
    if rc:
        raise ValueError("oracle rejected the arguments (code %d)" % rc)
    return out
