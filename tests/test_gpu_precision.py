"""Reduced-precision forms on the GPU, through the C ABI.

MIXED: rotator rows as two FP16 terms (the rounded row and its rounded
residual), FP32 products with Kahan-compensated per-workgroup sums, FP64
cross-workgroup reduction and DFT, the table's known gain divided out.  F32:
FP32 rows, plain FP32 sums, FP32 reduction and DFT.  F16: the literal mixed
variant, single FP16 rows and no gain correction (reported, not held to the
contract).

Each form is checked twice: tightly against the oracle's rotator-form
correlation fed with the same rounded tables (rounded here with numpy,
independently of the library), which isolates the kernel's arithmetic; and
against the exact FP64 oracle, whose error is reported and bounded.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import compare_spectra, rounded_tables, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_05993_amd import pcal

    pcal.lib()
    return pcal


@pytest.mark.parametrize("prec", [1, 2, 3])
@pytest.mark.parametrize("s", [0, 3, 4, 8, 9])
def test_precision_form(pc, prec, s):
    spec = synth.batch_specs()[s]
    L = 1 << 22
    say("precision form %d stream %d fs=%d fo=%d" % (prec, s, spec.fs, spec.f_offset))
    packed = synth.make_stream(spec, L)
    dev = torch.from_numpy(packed).cuda()
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 2, precision=prec) as h:
        h.extract(dev, L)
        C = h.spectrum()
        info = h.info()
    u, v, gain = rounded_tables(spec.fs, spec.f_offset, spec.ntones, info["fold_period"] // spec.ntones, prec)
    Cr = oracle.correlate_rotator(packed, 2, L, spec.ntones, u, v) * gain
    scale = np.abs(Cr).max()
    err_kernel = np.abs(C - Cr).max() / scale
    Co = oracle.correlate(packed, 2, L, spec.fs, spec.f_comb, spec.f_offset)
    amp_e, ph_e, weak = compare_spectra(C, Co, rel_floor=1e-6)
    say("  kernel vs rounded-table oracle: %.2e; vs FP64 oracle: amp %.2e phase %.2e rad" % (err_kernel, amp_e, ph_e))
    if prec == 1:
        # FP32 products and Kahan sums over at most M rows per workgroup: a few FP32 ulps
        assert err_kernel < 2e-6
        # two-term FP16 rows (about 22 bits): within the 1e-5 amplitude and
        # 1e-4 rad phase tolerance of the FP64 oracle
        assert amp_e < 1e-5 and ph_e < 1e-4
    elif prec == 3:
        # the literal single-FP16 variant: the kernel is the mixed form's, exact to
        # the same few FP32 ulps against its own (single-term) table; its table
        # rounding (2^-11 relative per row, no gain correction) is what it reports
        # against the FP64 oracle, within a few times the row rounding over sqrt(M)
        assert err_kernel < 2e-6
        assert amp_e < 2e-3 and ph_e < 2e-3
    else:
        # FP32 sums over rows, workgroups (atomics) and the N-point DFT: measured
        # at most 3.8e-6 against the FP64 oracle on the 64-stream mix
        assert err_kernel < 1e-5
        assert amp_e < 1e-5 and ph_e < 1e-5
