"""Multi-pass delay refinement (pcal_refine, Section 2) on the GPU against the oracle.

The device runs the finalize, the pulse readout (pass 0: the pulse-peak
delay) and the passes that counter-rotate the tone responses by the current
delay and fit the residual phase slope.  The oracle does the same from its
own correlation and rotated fold: after the first pass the delays must agree
to FP64 rounding of the fit (the two start from pulse-peak delays that agree
to the pulse tolerance), the intercept and rms likewise.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_05993_amd import pcal

    pcal.lib()
    return pcal


CASES = [
    # fs, f_offset, nbits, L, t_d, sideband, method
    (64_000_000, 10_000, 2, 1 << 22, 3.7e-9, 1, 1),
    (1_024_000_000, 510_000, 8, 3 * 102_400 + 4093, 125e-9, 1, 1),
    (32_000_000, 250_000, 2, 4 * 300_001, -210e-9, -1, 1),
    (64_000_000, 10_008, 8, 1 << 20, 41e-9, 1, 3),            # recurrence form, rotator period 8e6
]


@pytest.mark.parametrize("fs,fo,nbits,L,td,sb,method", CASES)
def test_refine_matches_oracle(pc, fs, fo, nbits, L, td, sb, method):
    spec = synth.CombSpec(fs, 1_000_000, fo, nbits, amp=0.3 if nbits == 2 else 3.0, t_d=td,
                          sigma=1.0 if nbits == 2 else 20.0, jitter=0.05, seed=(71, fo))
    packed = synth.make_stream(spec, L)
    dev = torch.from_numpy(packed).cuda()
    iters = 3
    with pc.PCal(fs, 1_000_000, fo, nbits, sideband=sb, method=method) as h:
        h.extract(dev, L)
        d, a, rms = h.refine(iters)
        _, pdelay, _, _, _ = h.pulse()
    Co = oracle.correlate(packed, nbits, L, fs, 1_000_000, fo)
    Po = oracle.fold_rot(packed, nbits, L, fs, fo, spec.ntones)
    _, _, t0, _ = oracle.pulse_peak(Po, fs, sideband=sb)
    do, ao, rmso = oracle.refine(Co, fs, 1_000_000, fo, t0, iters, sideband=sb)
    say("refine fs=%d fo=%d: device %s oracle %s (t_d %.3e); a %.6f/%.6f rms %.3e/%.3e"
        % (fs, fo, d, do, td, a, ao, rms, rmso))
    assert d[0] == pdelay
    assert abs(d[0] - do[0]) * fs < 1e-6
    assert np.abs(d[1:] - do[1:]).max() < 1e-16
    assert abs(a - ao) < 1e-9 and abs(rms - rmso) < 1e-9


def test_refine_rejects_bad_pass_count(pc):
    with pc.PCal(64_000_000, 1_000_000, 10_000, 2) as h:
        for bad in (0, 17):
            with pytest.raises(pc.PcalError) as e:
                h.refine(bad)
            assert e.value.code == pc.EINVAL
