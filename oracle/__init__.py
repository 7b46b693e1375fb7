"""FP64 CPU oracle for multi-tone phase-calibration extraction.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product library (the HIP path and
its Python binding) never does, and the two share no code.

* :mod:`oracle.core` -- ctypes wrapper over ``pcal_oracle.c``: the plain
  per-tone correlation ``C_k = sum_n x[n] exp(-j 2 pi (k f_comb + f_offset) n / fs)``
  in FP64, the integer fold of Eq. 2, the rotated fold with an integer
  (fixed-point) rotator table (Section 4.8), and the packed-sample decoder.
* :mod:`oracle.fit` -- amplitude, phase and delay from the C_k (numpy, FP64).
* :mod:`oracle.params` -- rotator period (Eq. 4) and phase step (Eq. 5).
* :mod:`oracle.pulse` -- the delay at the power peak of the folded pulse
  (Sections 2-3) from the rotated bins P[b] (``fold_rot``, Eqs. 2-3), the
  band-pass corrected for that group delay (Section 3), and the multi-pass
  refinement of the delay by counter-rotation with the residual phase
  (Section 2).
"""
from .core import (build, correlate, correlate_f64, correlate_rotator, decode, fixed_rotator, fold_int,  # noqa: F401
                   fold_rot, fold_table_int, max_threads)
from .pulse import bandpass, pulse_peak, refine  # noqa: F401
from .fit import delay_fit, in_band, results, tone_freqs  # noqa: F401
from .params import ntones, phase_step, rotator_period  # noqa: F401
