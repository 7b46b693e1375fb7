"""The allocation-free entry point (pcal_extract_noalloc) against the handle path on the GPU.

One call of pcal_extract_noalloc is one integration of the period-fold FP64
form with the tables, accumulators and counters in the library's fixed
device array.  Its results must equal pcal_create + pcal_extract +
pcal_results of the same bytes to the FP64 form's tolerance, on consecutive
calls that share the array (the second with a smaller input, so that
anything a call leaves behind would show), and on other parameters; sizes
beyond the array and streams that need a per-sample form are refused.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import F64_RTOL, assert_spectra, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_05993_amd import pcal

    pcal.lib()
    return pcal


def _handle(pc, spec, dev, L):
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits) as h:
        h.extract(dev, L)
        C = h.spectrum()
        amp, ph, d = h.results()
    return C, amp, ph, d


def _noalloc(pc, spec, dev, L, byte_offset=0):
    N = spec.ntones
    out = torch.full((4 * N + 1,), float("nan"), dtype=torch.float64, device="cuda")
    pc.extract_noalloc(spec.fs, spec.f_comb, spec.f_offset, spec.nbits, dev.data_ptr() + byte_offset, L, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return o[2 * N:3 * N] + 1j * o[3 * N:4 * N], o[:N], o[N:2 * N], o[4 * N]


def _check(pc, spec, L, what, byte_offset=0):
    packed = synth.make_stream(spec, L)
    buf = np.zeros(packed.size + 16, np.uint8)
    buf[byte_offset:byte_offset + packed.size] = packed
    dev = torch.from_numpy(buf).cuda()
    say("noalloc %s: fs=%d fo=%d nbits=%d L=%d" % (what, spec.fs, spec.f_offset, spec.nbits, L))
    C0, a0, p0, d0 = _handle(pc, spec, dev[byte_offset:], L)
    C1, a1, p1, d1 = _noalloc(pc, spec, dev, L, byte_offset)
    if L == 0:  # an empty integration: every output zero on both paths
        assert not np.any(C1) and not np.any(C0) and not np.any(a1) and d1 == 0.0 == d0
        return
    assert_spectra(C1, C0, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, rel_floor=1e-6, what="noalloc " + what)
    np.testing.assert_allclose(a1, a0, rtol=1e-10, atol=1e-14)
    assert abs(d1 - d0) < 1e-15


def test_noalloc_two_calls_in_a_row_second_smaller(pc):
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    _check(pc, spec, 4 * 1_000_003, "first call")
    _check(pc, spec, 4 * 250_001, "second, smaller call", byte_offset=3)


def test_noalloc_other_parameters(pc):
    # 8-bit, N = 1024, column tiles; then 2-bit with f_offset = 0 (integer bins), after it
    _check(pc, synth.WORKLOADS["wide8_1024M_510k"]["spec"], 3 * 102_400 + 4093, "wide8")
    _check(pc, synth.WORKLOADS["small_2bit_fo0"]["spec"], 1 << 20, "f_offset 0")
    _check(pc, synth.WORKLOADS["fold2_64M_10k"]["spec"], 0, "empty")


def test_noalloc_refusals(pc):
    out = torch.zeros(4 * 64 + 1, dtype=torch.float64, device="cuda")
    dev = torch.zeros(2048, dtype=torch.uint8, device="cuda")
    # a prime offset needs a per-sample form
    with pytest.raises(pc.PcalError) as e:
        pc.extract_noalloc(64_000_000, 1_000_000, 10_007, 2, dev, 4096, out)
    assert e.value.code == pc.ENOTSUP
    # N = 16 with a 2^22-sample fold period: 4 MiB of rotator rows alone, beyond the array
    out16 = torch.zeros(4 * 16 + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(pc.PcalError) as e:
        pc.extract_noalloc(1 << 24, 1 << 20, 4, 2, dev, 4096, out16)
    assert e.value.code == pc.EINVAL and "scratch" in pc.last_error()
    # nsamples not a multiple of the samples per byte
    with pytest.raises(pc.PcalError) as e:
        pc.extract_noalloc(64_000_000, 1_000_000, 10_000, 2, dev, 4097, out)
    assert e.value.code == pc.EINVAL

