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
