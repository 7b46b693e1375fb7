"""Per-sample rotation forms (rotator table, Eq. 4; recurrences, Eq. 6-7 and the coupled form) on the GPU.

Every sample is multiplied by a rotator; the table form reads it from one
rotator period, the recurrence forms step a direct-form resonator (method 3)
or a coupled-form oscillator (method 4) per row with exact FP64 restarts
every 64 rows; the magic-circle oscillator (method 5) and the resonator with
truncation-error feedback (method 6) likewise.  The FP64 form (FP64 table or recurrence state, FP64 products
and sums) is checked against the FP64 oracle to 1e-10; the mixed form (table
entries as two FP16 terms, FP32 state, products and run sums, Kahan totals)
and the all-FP32 form to the contract tolerance (1e-5 relative amplitude,
1e-4 rad phase).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import AMP_RTOL, F64_RTOL, PHASE_ATOL, assert_spectra, compare_spectra, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_05993_amd import pcal

    pcal.lib()
    return pcal


def _extract(pc, spec, packed, L, method, prec=0, chunks=None, offset=0):
    buf = np.zeros(packed.size + 32, np.uint8)
    buf[offset:offset + packed.size] = packed
    dev = torch.from_numpy(buf).cuda()
    spb = 8 // spec.nbits
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits, method=method, precision=prec) as h:
        assert h.info()["method"] == method
        if chunks is None:
            h.extract(dev, L, byte_offset=offset)
        else:
            pos = 0
            for c in chunks:
                h.extract(dev, c, byte_offset=offset + pos // spb)
                pos += c
        C = h.spectrum()
        res = h.results()
    return C, res


@pytest.mark.parametrize("method", [2, 3, 4, 5, 6])
def test_wide8_per_sample(pc, method):
    spec = synth.WORKLOADS["wide8_1024M_510k"]["spec"]
    L = (1 << 22) + 4096 + 7
    say("wide8 per-sample method %d L=%d" % (method, L))
    packed = synth.make_stream(spec, L)
    C, (amp, ph, d) = _extract(pc, spec, packed, L, method, offset=5)
    Co = oracle.correlate(packed, 8, L, spec.fs, spec.f_comb, spec.f_offset)
    assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="wide8 method %d" % method)
    ao, po, do = oracle.results(Co, L, spec.fs, spec.f_comb, spec.f_offset)
    assert abs(d - do) < 1e-15


@pytest.mark.parametrize("method", [2, 3, 4, 5, 6])
def test_fold2_per_sample_chunks(pc, method):
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    L = 4 * 700_001
    say("fold2 per-sample method %d L=%d" % (method, L))
    packed = synth.make_stream(spec, L)
    chunks = [4 * 3, 4 * 250_000, 4 * 123_457]
    chunks.append(L - sum(chunks))
    C, _ = _extract(pc, spec, packed, L, method, chunks=chunks, offset=2)
    Co = oracle.correlate(packed, 2, L, spec.fs, spec.f_comb, spec.f_offset)
    assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="fold2 method %d" % method)


def test_long_fold_period_auto(pc):
    """f_offset = 10008 Hz at 64 MHz: an 8e6-sample fold period, the longest class AUTO still folds.
    625 column tiles and 125000 rotator rows (read from global memory in the epilogue, beyond LDS), two
    launches (the second starting mid-period, on a ragged byte count); FP64 against the oracle."""
    spec = synth.CombSpec(64_000_000, 1_000_000, 10_008, 2, amp=0.05, t_d=3.7e-9, seed=(43,))
    L = (1 << 25) + 4 * 333
    packed = synth.make_stream(spec, L)
    dev = torch.from_numpy(packed).cuda()
    cut = 4 * 3_000_001
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 2) as h:
        info = h.info()
        assert info["method"] == pc.METHOD_PERIOD_FOLD and info["fold_period"] == 8_000_000
        h.extract(dev[: cut // 4], cut)
        h.extract(dev[cut // 4:], L - cut)
        C = h.spectrum()
    Co = oracle.correlate(packed, 2, L, spec.fs, spec.f_comb, spec.f_offset)
    assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="8e6-sample fold period")


def test_prime_offset_recurrence(pc):
    """f_offset = 10007 Hz: rotator period = fs, no fold period or table; AUTO takes the recurrence."""
    spec = synth.CombSpec(64_000_000, 2_000_000, 10_007, 8, amp=2.0, t_d=4e-9, sigma=20.0, seed=(41,))
    L = 1 << 21
    packed = synth.make_stream(spec, L)
    dev = torch.from_numpy(packed).cuda()
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 8) as h:
        assert h.info()["method"] == pc.METHOD_OSC
        h.extract(dev[: L // 2], L // 2)
        h.extract(dev[L // 2:], L // 2)
        C = h.spectrum()
    Co = oracle.correlate(packed, 8, L, spec.fs, spec.f_comb, spec.f_offset)
    assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="prime offset")


@pytest.mark.parametrize("method", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("prec", [1, 2])
def test_per_sample_reduced_precision(pc, method, prec):
    spec = synth.WORKLOADS["wide8_1024M_510k"]["spec"]
    L = 1 << 22
    packed = synth.make_stream(spec, L)
    C, _ = _extract(pc, spec, packed, L, method, prec=prec)
    Co = oracle.correlate(packed, 8, L, spec.fs, spec.f_comb, spec.f_offset)
    a, p, w = compare_spectra(C, Co)
    say("wide8 method %d prec %d: amp %.2e phase %.2e" % (method, prec, a, p))
    assert a < AMP_RTOL and p < PHASE_ATOL and w < 1e-5


@pytest.mark.parametrize("fs,fc,fo", [(64_000_000, 1_000_000, 15_650), (256_000_000, 1_000_000, 62_600)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_recurrence_near_zero_row_step(pc, fs, fc, fo, prec):
    """Offsets whose rotator advance per 4096-sample row lies near 0 (mod 2 pi; |sin d| = 0.01
    there): with the resonator coefficient 2 cos d rounded to FP32 the recurrence would drift by
    up to 2e-4 rad over a 64-row run.  The plan picks a row length whose step is far from 0 and
    pi; the resonator then meets the contract in the FP32 forms and FP64 accuracy in the FP64
    form.  (Comb periods of 1.28e6 samples keep the synthetic input quick to build.)"""
    spec = synth.CombSpec(fs, fc, fo, 8, amp=1.0, t_d=7e-9, sigma=20.0, seed=(43, fo))
    L = 1 << 22
    packed = synth.make_stream(spec, L)
    with pc.PCal(fs, fc, fo, 8, method=pc.METHOD_OSC, precision=prec) as h:
        info = h.info()
    dn = info["row_vectors"] * 16
    d = 2 * np.pi * ((fo * dn) % fs) / fs
    say("fs=%d fo=%d prec %d: %d-sample rows, |sin d| = %.3f" % (fs, fo, prec, dn, abs(np.sin(d))))
    assert abs(np.sin(d)) >= 0.2
    C, _ = _extract(pc, spec, packed, L, pc.METHOD_OSC, prec=prec)
    Co = oracle.correlate(packed, 8, L, fs, fc, fo)
    if prec == 0:
        assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="near-zero step F64")
    else:
        assert_spectra(C, Co, what="near-zero step prec %d" % prec)


def test_table_single_fp16_variant(pc):
    """The literal mixed variant of the table form (PCAL_PREC_F16: single FP16 entries, no gain
    correction) runs and reports its form; its table rounding (2^-11 per entry) is what separates it
    from the FP64 oracle, within a few times that rounding."""
    spec = synth.WORKLOADS["wide8_1024M_510k"]["spec"]
    L = 1 << 22
    packed = synth.make_stream(spec, L)
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 8, method=pc.METHOD_LUT, precision=pc.PREC_F16) as h:
        assert h.info()["precision"] == pc.PREC_F16
    C, _ = _extract(pc, spec, packed, L, pc.METHOD_LUT, prec=pc.PREC_F16)
    Co = oracle.correlate(packed, 8, L, spec.fs, spec.f_comb, spec.f_offset)
    a, p, w = compare_spectra(C, Co)
    say("wide8 table single-FP16: amp %.2e phase %.2e" % (a, p))
    assert a < 2e-3 and p < 2e-3
