"""Helpers shared by the GPU tests: tolerances and comparisons against the oracle."""
import sys

import numpy as np

# Contract tolerances for rotated streams (amplitude relative, phase in radians),
# stated against the FP64 oracle.
AMP_RTOL = 1e-5
PHASE_ATOL = 1e-4
# The FP64 form rotates exact integer sums with an FP64 table: its error is a
# few FP64 roundings per term, far below the contract.
F64_RTOL = 1e-10


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def compare_spectra(got, want, amp_rtol=AMP_RTOL, phase_atol=PHASE_ATOL, rel_floor=1e-5):
    """Max relative amplitude error and max wrapped phase error over tones.

    Tones whose magnitude is below rel_floor * max|C| carry no signal (for
    example the DC tone of an f_offset = 0 comb); they are compared by their
    absolute error against rel_floor * max|C| instead.
    """
    got = np.asarray(got)
    want = np.asarray(want)
    scale = np.abs(want).max()
    strong = np.abs(want) >= rel_floor * scale
    amp_err = np.abs(np.abs(got[strong]) - np.abs(want[strong])) / np.abs(want[strong])
    ph_err = np.abs(np.angle(got[strong] * np.conj(want[strong])))
    weak_err = np.abs(got[~strong] - want[~strong]).max() / scale if (~strong).any() else 0.0
    return (float(amp_err.max()) if amp_err.size else 0.0,
            float(ph_err.max()) if ph_err.size else 0.0,
            float(weak_err))


def assert_spectra(got, want, amp_rtol=AMP_RTOL, phase_atol=PHASE_ATOL, rel_floor=1e-5, what=""):
    a, p, w = compare_spectra(got, want, rel_floor=rel_floor)
    say(what, "amp_rel_err=%.3e phase_err=%.3e weak_abs_rel=%.3e" % (a, p, w))
    assert a <= amp_rtol, (what, a)
    assert p <= phase_atol, (what, p)
    assert w <= rel_floor, (what, w)
    return a, p


def rounded_tables(fs, fo, N, M, prec):
    """The rotator factors a reduced-precision period-fold form multiplies by, rounded here with numpy.

    The fold rotates period position q = m N + b by u[m] v[b], u[m] = exp(-j w_o N m),
    v[b] = exp(-j w_o b) (Eq. 3 with the phase index reduced exactly).  Returns
    (u, v, gain) for oracle.correlate_rotator: MIXED stores each u[m] as two FP16
    terms (the rounded value and its rounded residual) and divides the table's
    mean gain 1 + gamma out, v exact; F16 (the literal single-FP16 form) rounds u
    to one FP16 value, v exact, gain 1; F32 rounds u and v to FP32, gain 1.
    """
    m = np.arange(M, dtype=np.int64)
    b = np.arange(N, dtype=np.int64)
    u = np.exp(-2j * np.pi * ((fo * N * m) % fs) / fs)
    v = np.exp(-2j * np.pi * ((fo * b) % fs) / fs)
    def f16(z):
        return z.real.astype(np.float16).astype(float) + 1j * z.imag.astype(np.float16).astype(float)
    if prec == 1:
        hi = f16(u)
        uh = hi + f16(u - hi)
        gamma = np.mean(np.conj(u) * (uh - u))
        return uh, v, 1.0 / (1.0 + gamma)
    if prec == 3:  # the literal single-FP16 form: rounded rows, no gain correction
        return f16(u), v, 1.0

    def f32(z):
        return z.real.astype(np.float32).astype(float) + 1j * z.imag.astype(np.float32).astype(float)
    return f32(u), f32(v), 1.0
