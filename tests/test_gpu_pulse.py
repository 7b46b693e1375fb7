"""Parity of the pulse readout (pcal_pulse, through the C ABI) with the oracle, on the GPU.

The device returns the rotated bins P[b] of Eqs. 2-3 and the delay at the
power peak of the pulse (Sections 2-3).  Small sizes are compared bin by bin
with the oracle's own fold (``oracle.fold_rot``) and its peak estimator
(``oracle.pulse_peak``); the full-size stream, in the launch configuration
the benchmark times, is checked through properties that hold at any size:
the DFT of the pulse is the spectrum, and the device's estimate equals the
oracle estimator applied to the device's own pulse.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import F64_RTOL, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_05993_amd import pcal

    pcal.lib()
    return pcal


def _dev(packed):
    return torch.from_numpy(np.ascontiguousarray(packed)).cuda()


def _pulse(pc, spec, dev, L, chunks=(), **kw):
    spb = 8 // spec.nbits
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits, **kw) as h:
        pos = 0
        for c in (chunks or (L,)):
            h.extract(dev, c, byte_offset=pos // spb)
            pos += c
        assert pos == L
        return h.pulse()


def _check(got, P_want, fs, L, sideband=1, p_rtol=F64_RTOL, d_tol=1e-7, what=""):
    P, delay, b0, off, power = got
    scale = np.abs(P_want).max()
    p_err = np.abs(P - P_want).max() / scale
    wb0, woff, wdelay, wpower = oracle.pulse_peak(P_want, fs, sideband=sideband)
    say(what, "P rel err %.3e  delay %.6e s (oracle %.6e)  b0 %d (oracle %d)" % (p_err, delay, wdelay, b0, wb0))
    assert p_err <= p_rtol, (what, p_err)
    pw = np.abs(P_want) ** 2
    top2 = np.sort(pw)[-2:] if pw.size > 1 else np.array([0.0, pw[0]])
    gap = max(1e-6, 10 * p_rtol)  # peaks closer than this may swap under the path's rounding
    if top2[1] - top2[0] > gap * top2[1]:
        assert b0 == wb0, (what, b0, wb0)
        assert abs(delay - wdelay) * fs <= d_tol, (what, delay, wdelay)
    else:
        assert pw[b0] >= top2[1] * (1 - gap), (what, b0)
    assert abs(power - wpower / float(L) ** 2) <= 3 * p_rtol * wpower / float(L) ** 2, (what, power)
    return delay


def test_pulse_2bit_rotated(pc):
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    L = 1 << 24
    say("pulse fold2_64M_10k L=%d" % L)
    packed = synth.make_stream(spec, L)
    got = _pulse(pc, spec, _dev(packed), L)
    want = oracle.fold_rot(packed, 2, L, spec.fs, spec.f_offset, spec.ntones)
    delay = _check(got, want, spec.fs, L, what="2-bit f_o=10k")
    assert abs(delay - spec.t_d) * spec.fs < 0.1


def test_pulse_8bit_wide_chunked(pc):
    spec = synth.WORKLOADS["wide8_1024M_510k"]["spec"]
    L = 1 << 23
    say("pulse wide8_1024M_510k L=%d in 3 chunks" % L)
    packed = synth.make_stream(spec, L)
    got = _pulse(pc, spec, _dev(packed), L, chunks=(3 * (1 << 20) + 96, 1 << 22, L - 3 * (1 << 20) - 96 - (1 << 22)))
    want = oracle.fold_rot(packed, 8, L, spec.fs, spec.f_offset, spec.ntones)
    _check(got, want, spec.fs, L, what="8-bit N=1024 chunked")


def test_pulse_f0_matches_integer_fold(pc):
    spec = synth.WORKLOADS["small_2bit_fo0"]["spec"]
    L = 1 << 22
    say("pulse small_2bit_fo0 L=%d" % L)
    packed = synth.make_stream(spec, L)
    got = _pulse(pc, spec, _dev(packed), L)
    want = oracle.fold_int(packed, 2, L, spec.ntones).astype(np.float64)
    _check(got, want + 0j, spec.fs, L, what="2-bit f_o=0")
    assert np.abs(got[0] - want).max() <= 1e-12 * np.abs(want).max()


def test_pulse_lower_sideband(pc):
    spec = synth.CombSpec(16_000_000, 1_000_000, 250_000, 2, amp=0.05, t_d=-120e-9, seed=(7, 1, 0))
    L = 1 << 22
    say("pulse lower sideband fs=16M f_o=250k L=%d" % L)
    packed = synth.make_stream(spec, L)
    got = _pulse(pc, spec, _dev(packed), L, sideband=-1)
    want = oracle.fold_rot(packed, 2, L, spec.fs, spec.f_offset, spec.ntones)
    _check(got, want, spec.fs, L, sideband=-1, what="LSB")


@pytest.mark.parametrize("method,prec", [(3, 0), (4, 0), (2, 0), (1, 1), (1, 2)])
def test_pulse_other_forms(pc, method, prec):
    """Per-sample rotator forms (table, recurrences) and the mixed / all-FP32 precision forms."""
    spec = synth.CombSpec(32_000_000, 1_000_000, 10_000, 8, amp=1.0, t_d=20e-9, sigma=20.0, seed=(4, method, prec))
    L = 1 << 22
    say("pulse method=%d precision=%d L=%d" % (method, prec, L))
    packed = synth.make_stream(spec, L)
    got = _pulse(pc, spec, _dev(packed), L, method=method, precision=prec)
    want = oracle.fold_rot(packed, 8, L, spec.fs, spec.f_offset, spec.ntones)
    _check(got, want, spec.fs, L, p_rtol=1e-5, d_tol=1e-3, what="method %d precision %d" % (method, prec))


def test_pulse_empty_integration(pc):
    with pc.PCal(64_000_000, 1_000_000, 10_000, 2) as h:
        P, delay, b0, off, power = h.pulse()
    assert not np.any(P) and (delay, b0, off, power) == (0.0, 0, 0.0, 0.0)


def test_pulse_full_size_properties(pc):
    """2^30 2-bit samples as the benchmark runs them: DFT(pulse) = spectrum; device estimate = oracle estimate."""
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    L = 1 << 30
    say("pulse full size fold2_64M_10k L=%d" % L)
    dev = synth.make_stream_device(spec, L)
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 2) as h:
        h.extract(dev, L)
        P, delay, b0, off, power = h.pulse()
        C = h.spectrum()
    del dev
    torch.cuda.empty_cache()
    assert np.abs(np.fft.fft(P) - C).max() <= 1e-12 * np.abs(C).max()
    wb0, woff, wdelay, wpower = oracle.pulse_peak(P, spec.fs)
    say("full size: delay %.6e s (t_d %.3e), b0 %d, offset %.4f" % (delay, spec.t_d, b0, off))
    assert b0 == wb0 and abs(off - woff) <= 1e-9 and abs(delay - wdelay) * spec.fs <= 1e-9
    assert abs(power - wpower / float(L) ** 2) <= 1e-12 * power
    assert abs(delay - spec.t_d) * spec.fs < 0.1


@pytest.mark.parametrize("name,sideband,L", [("fold2_64M_10k", 1, 1 << 24), ("fold2_64M_10k", -1, 1 << 22),
                                             ("wide8_1024M_510k", 1, 1 << 22)])
def test_bandpass_matches_oracle(pc, name, sideband, L):
    """Band-pass corrected for the pulse's group delay (Section 3) against the oracle's, tone by tone."""
    spec = synth.WORKLOADS[name]["spec"]
    say("bandpass %s sideband %d L=%d" % (name, sideband, L))
    packed = synth.make_stream(spec, L)
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits, sideband=sideband) as h:
        h.extract(_dev(packed), L)
        amp, ph, delay = h.bandpass()
        amp_r, _, _ = h.results()
    C = oracle.correlate(packed, spec.nbits, L, spec.fs, spec.f_comb, spec.f_offset)
    P = oracle.fold_rot(packed, spec.nbits, L, spec.fs, spec.f_offset, spec.ntones)
    _, _, wdelay, _ = oracle.pulse_peak(P, spec.fs, sideband=sideband)
    want = oracle.bandpass(C, spec.fs, spec.f_comb, spec.f_offset, wdelay, sideband=sideband)
    strong = np.abs(C) >= 1e-5 * np.abs(C).max()
    err = np.abs(np.angle(np.exp(1j * (ph - want))))[strong].max()
    say("bandpass phase err %.3e rad, delay %.6e s (oracle %.6e)" % (err, delay, wdelay))
    assert np.array_equal(amp, amp_r)
    assert abs(delay - wdelay) * spec.fs <= 1e-7
    assert err <= 1e-6
