"""Fixed-point rotator form (PCAL_PREC_Q17, Section 4.8's integer arithmetic) on the GPU.

The period fold sums the integer samples per period position, multiplies
each position sum by the Q17 rotator (exp(-j w_o r) * 2^17 rounded, r the
position mod R) in integers and adds the products in int64 and in
integer-valued FP64 atomics, so the bins are exact: they must equal the
oracle's integer table fold bit for bit.  The spectrum (FP64 DFT of the
bins, scaled by 2^-17) must equal the DFT of the oracle's bins to FP64
rounding, and is reported against the exact FP64 oracle, where the table
rounding (2^-18 per component) keeps it within the 1e-5 / 1e-4 rad bar on
these streams.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import AMP_RTOL, PHASE_ATOL, assert_spectra, say

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
    # workload spec, samples, chunk split (samples), byte offset
    (synth.WORKLOADS["fold2_64M_10k"]["spec"], 4 * 1_000_003, 4 * 123_457, 3),
    (synth.WORKLOADS["wide8_1024M_510k"]["spec"], 3 * 102_400 + 4093, 100_001, 5),
    (synth.CombSpec(16_000_000, 1_000_000, 250_000, 2, amp=0.3, t_d=12e-9, seed=(81,)), 1 << 22, 4 * 77, 0),
    (synth.WORKLOADS["small_2bit_fo0"]["spec"], 1 << 20, 1 << 19, 8),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fixed_point_bins_exact(pc, case):
    spec, L, split, off = CASES[case]
    say("fixed point: fs=%d fo=%d nbits=%d L=%d" % (spec.fs, spec.f_offset, spec.nbits, L))
    packed = synth.make_stream(spec, L)
    buf = np.zeros(packed.size + 16, np.uint8)
    buf[off:off + packed.size] = packed
    dev = torch.from_numpy(buf).cuda()
    spb = 8 // spec.nbits
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits, precision=pc.PREC_Q17) as h:
        info = h.info()
        assert info["precision"] == pc.PREC_Q17 and info["method"] == pc.METHOD_PERIOD_FOLD
        h.extract(dev, split, byte_offset=off)
        h.extract(dev, L - split, byte_offset=off + split // spb)
        P = h.bins()
        C = h.spectrum()
    T = oracle.fixed_rotator(spec.fs, spec.f_offset)
    re, im = oracle.fold_table_int(packed, spec.nbits, L, spec.ntones, T)
    np.testing.assert_array_equal(P.real * 131072.0, re.astype(np.float64))  # 2^17
    np.testing.assert_array_equal(P.imag * 131072.0, im.astype(np.float64))
    Cq = np.fft.fft((re + 1j * im) / 131072.0)
    assert np.abs(C - Cq).max() <= 1e-12 * np.abs(Cq).max()
    Co = oracle.correlate(packed, spec.nbits, L, spec.fs, spec.f_comb, spec.f_offset)
    assert_spectra(C, Co, amp_rtol=AMP_RTOL, phase_atol=PHASE_ATOL, rel_floor=1e-5, what="fixed point vs FP64")


def test_fixed_point_refused_where_unsupported(pc):
    with pytest.raises(pc.PcalError) as e:
        pc.PCal(64_000_000, 1_000_000, 10_000, 2, method=pc.METHOD_OSC, precision=pc.PREC_Q17)
    assert e.value.code == pc.ENOTSUP
    with pytest.raises(pc.PcalError) as e:
        pc.PCalBatch(4, precision=pc.PREC_Q17)
    assert e.value.code == pc.ENOTSUP
