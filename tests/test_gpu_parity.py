"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on the GPU.

Inputs are seeded synthetic streams with the shapes of the evaluation
workloads.  Small sizes are compared tone by tone against the full oracle;
full sizes, in the launch configuration the benchmark times, are compared on
a sample of tones the oracle computes one by one.
"""
import numpy as np
import pytest

import oracle
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


def _dev(packed):
    return torch.from_numpy(np.ascontiguousarray(packed)).cuda()


def _run(pc, spec, dev, nsamples=None, prec=0, sideband=1, chunks=None):
    h = pc.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits, sideband=sideband, precision=prec)
    spb = 8 // spec.nbits
    ns = nsamples if nsamples is not None else dev.numel() * spb
    if chunks is None:
        h.extract(dev, ns)
    else:
        pos = 0
        for c in chunks:
            h.extract(dev, c, byte_offset=pos // spb)
            pos += c
        assert pos == ns
    C = h.spectrum()
    res = h.results()
    ib = h.bins(integer=True)[1] if spec.f_offset == 0 else None
    h.close()
    return C, res, ib


# ------------------------------------------------------------------ small 2-bit, f_offset = 0 (bit-exact)

def test_small_2bit_f0_bit_exact(pc):
    w = synth.WORKLOADS["small_2bit_fo0"]
    spec, L = w["spec"], w["nsamples"]
    say("small_2bit_fo0 L=%d" % L)
    packed = synth.make_stream(spec, L)
    C, (amp, ph, delay), ib = _run(pc, spec, _dev(packed))
    want_bins = oracle.fold_int(packed, 2, L, spec.ntones)
    np.testing.assert_array_equal(ib, want_bins)
    Co = oracle.correlate(packed, 2, L, spec.fs, spec.f_comb, spec.f_offset)
    assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, rel_floor=1e-6, what="small_2bit_fo0")
    ao, po, do = oracle.results(Co, L, spec.fs, spec.f_comb, spec.f_offset)
    np.testing.assert_allclose(amp, ao, rtol=1e-10, atol=1e-12)
    k = oracle.in_band(spec.fs, spec.f_comb, spec.f_offset)
    assert np.max(np.abs(np.angle(np.exp(1j * (ph[k] - po[k]))))) < 1e-9
    assert abs(delay - do) < 1e-15


# ------------------------------------------------------------------ rotated 2-bit, several tiles + ragged tail

@pytest.mark.parametrize("L,offset", [(4 * 1_000_003, 0), (4 * 777_777, 3), (1 << 22, 8)])
def test_rotated_2bit_small(pc, L, offset):
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    say("fold2_64M_10k L=%d offset=%d" % (L, offset))
    packed = synth.make_stream(spec, L)
    buf = np.zeros(packed.size + 16, np.uint8)
    buf[offset:offset + packed.size] = packed
    dev = _dev(buf)
    h = pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 2)
    h.extract(dev, L, byte_offset=offset)
    C = h.spectrum()
    amp, ph, delay = h.results()
    h.close()
    Co = oracle.correlate(packed, 2, L, spec.fs, spec.f_comb, spec.f_offset)
    assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="fold2 small")
    ao, po, do = oracle.results(Co, L, spec.fs, spec.f_comb, spec.f_offset)
    np.testing.assert_allclose(amp, ao, rtol=1e-9)
    assert abs(delay - do) < 1e-13


# ------------------------------------------------------------------ full size, benchmark launch configuration

def test_fold2_full_size_sampled(pc):
    w = synth.WORKLOADS["fold2_64M_10k"]
    spec, L = w["spec"], w["nsamples"]
    say("fold2_64M_10k full L=%d" % L)
    dev = synth.make_stream_device(spec, L)
    h = pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 2)
    h.extract(dev, L)
    C = h.spectrum()
    h.close()
    host = dev.cpu().numpy()
    tones = [0, 1, 2, 17, 31, 32, 45, 63]
    Co = oracle.correlate(host, 2, L, spec.fs, spec.f_comb, spec.f_offset, tones=tones)
    assert_spectra(C[tones], Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="fold2 full (sampled tones)")


# ------------------------------------------------------------------ 8-bit, N = 1024, column tiles, chunk boundary

def test_wide8_chunks_sampled(pc):
    w = synth.WORKLOADS["wide8_1024M_510k"]
    spec = w["spec"]
    chunk = 1 << 24
    L = 2 * chunk
    say("wide8_1024M_510k two chunks of %d" % chunk)
    dev = synth.make_stream_device(spec, L)
    h = pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 8)
    h.extract(dev[:chunk], chunk)
    h.extract(dev[chunk:], chunk)
    C = h.spectrum()
    amp, ph, delay = h.results()
    h.close()
    host = dev.cpu().numpy()
    tones = [0, 1, 100, 255, 511, 512, 777, 1023]
    Co = oracle.correlate(host, 8, L, spec.fs, spec.f_comb, spec.f_offset, tones=tones)
    assert_spectra(C[tones], Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="wide8 (sampled tones)")


@pytest.fixture(scope="module")
def wide8_real_chunks(pc):
    """The 8-bit wide workload at its real chunk size: the first two 2^28-sample chunks
    (one chunk boundary), 8 tones from the oracle."""
    spec = synth.WORKLOADS["wide8_1024M_510k"]["spec"]
    chunk = 1 << 28
    say("wide8_1024M_510k: generating two chunks of 2^28 samples")
    dev = synth.make_stream_device(spec, 2 * chunk)
    tones = [0, 1, 100, 255, 511, 512, 777, 1023]
    Co = oracle.correlate(dev.cpu().numpy(), 8, 2 * chunk, spec.fs, spec.f_comb, spec.f_offset, tones=tones)
    yield spec, chunk, dev, tones, Co
    del dev
    torch.cuda.empty_cache()


@pytest.mark.parametrize("method", [1, 2, 3, 4])
def test_wide8_real_chunks_sampled(pc, wide8_real_chunks, method):
    """Two 2^28-sample chunks, each one pcal_extract in the launch shape the benchmark
    times (the period fold's persistent grid walks many 4-row groups per workgroup;
    the per-sample forms cross a chunk boundary mid-period, 2^28 mod 102400 != 0).
    The period fold (FP64 rotation of exact integer sums) to 1e-10; the per-sample
    forms to the contract tolerance."""
    spec, chunk, dev, tones, Co = wide8_real_chunks
    say("wide8 real chunks, method %d" % method)
    h = pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 8, method=method)
    assert h.info()["method"] == method
    h.extract(dev[:chunk], chunk)
    h.extract(dev[chunk:], chunk)
    C = h.spectrum()
    h.close()
    if method == 1:
        assert_spectra(C[tones], Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="wide8 2x2^28 fold")
    else:
        assert_spectra(C[tones], Co, what="wide8 2x2^28 method %d" % method)


def test_wide8_small_all_tones(pc):
    spec = synth.WORKLOADS["wide8_1024M_510k"]["spec"]
    L = 3 * 102_400 + 4093
    say("wide8 small L=%d" % L)
    packed = synth.make_stream(spec, L)
    C, (amp, ph, delay), _ = _run(pc, spec, _dev(packed))
    Co = oracle.correlate(packed, 8, L, spec.fs, spec.f_comb, spec.f_offset)
    assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="wide8 small")
    ao, po, do = oracle.results(Co, L, spec.fs, spec.f_comb, spec.f_offset)
    np.testing.assert_allclose(amp, ao, rtol=1e-9)
    assert abs(delay - do) < 1e-12


# ------------------------------------------------------------------ stream mix of the precision study (all tones)

@pytest.mark.parametrize("s", range(0, 64, 9))
def test_batch_mix_streams(pc, s):
    spec = synth.batch_specs()[s]
    L = 1 << 20
    say("batch mix stream %d fs=%d fo=%d" % (s, spec.fs, spec.f_offset))
    packed = synth.make_stream(spec, L)
    C, res, ib = _run(pc, spec, _dev(packed))
    Co = oracle.correlate(packed, 2, L, spec.fs, spec.f_comb, spec.f_offset)
    assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, rel_floor=1e-6, what="mix %d" % s)
    if ib is not None:
        np.testing.assert_array_equal(ib, oracle.fold_int(packed, 2, L, spec.ntones))


# ------------------------------------------------------------------ edge cases

def test_chunk_split_invariance_integer(pc):
    """Any split into extract calls (odd sizes, misaligned starts) gives identical integer bins."""
    spec = synth.WORKLOADS["small_2bit_fo0"]["spec"]
    L = 4 * 250_001
    packed = synth.make_stream(spec, L)
    dev = _dev(packed)
    _, _, whole = _run(pc, spec, dev, L)
    _, _, split = _run(pc, spec, dev, L, chunks=[4, 4 * 1001, 60, 4 * 77_777, 4 * 13, L - 4 - 4 * 1001 - 60
                                                  - 4 * 77_777 - 4 * 13])
    np.testing.assert_array_equal(whole, split)
    np.testing.assert_array_equal(whole, oracle.fold_int(packed, 2, L, spec.ntones))


def test_chunk_split_rotated(pc):
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    L = 4 * 300_007
    packed = synth.make_stream(spec, L)
    dev = _dev(packed)
    C1, _, _ = _run(pc, spec, dev, L)
    chunks = [20, 4 * 99_999, 4 * 100_000]
    chunks.append(L - sum(chunks))
    C2, _, _ = _run(pc, spec, dev, L, chunks=chunks)
    Co = oracle.correlate(packed, 2, L, spec.fs, spec.f_comb, spec.f_offset)
    assert_spectra(C1, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="whole")
    assert_spectra(C2, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="split")


@pytest.mark.parametrize("nbits,L", [(2, 4), (2, 60), (2, 64), (2, 68), (8, 1), (8, 15), (8, 17)])
def test_tiny_inputs(pc, nbits, L):
    spec = synth.CombSpec(64_000_000, 1_000_000, 10_000, nbits, amp=0.5, t_d=1e-9,
                          sigma=1.0 if nbits == 2 else 20.0, seed=(5, L))
    packed = synth.make_stream(spec, L + (-L) % (8 // nbits))
    for off in (0, 1, 7):
        buf = np.zeros(packed.size + 32, np.uint8)
        buf[off:off + packed.size] = packed
        h = pc.PCal(spec.fs, spec.f_comb, spec.f_offset, nbits)
        h.extract(_dev(buf), L, byte_offset=off)
        C = h.spectrum()
        h.close()
        Co = oracle.correlate(packed, nbits, L, spec.fs, spec.f_comb, spec.f_offset)
        np.testing.assert_allclose(C, Co, rtol=0, atol=1e-9 * max(1.0, np.abs(Co).max()))


def test_empty_and_reset(pc):
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    L = 4 * 100_000
    packed = synth.make_stream(spec, 2 * L)
    dev = _dev(packed)
    h = pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 2)
    h.extract(dev, 0)
    C0 = h.spectrum()
    assert np.all(C0 == 0)
    amp, ph, d = h.results()
    assert np.all(amp == 0) and d == 0.0
    h.extract(dev, L)
    h.reset()
    h.extract(dev[L // 4:], L)          # second integration continues the global index
    C = h.spectrum()
    assert h.info()["samples_total"] == 2 * L and h.info()["samples_integ"] == L
    h.close()
    Co = oracle.correlate(packed[L // 4:], 2, L, spec.fs, spec.f_comb, spec.f_offset, n0=L)
    assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="after reset")


def test_lower_sideband_conjugates(pc):
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    L = 1 << 20
    dev = _dev(synth.make_stream(spec, L))
    Cu, (au, pu, du), _ = _run(pc, spec, dev, L, sideband=1)
    Cl, (al, pl, dl), _ = _run(pc, spec, dev, L, sideband=-1)
    # workgroups add their bins with FP64 atomics: the summation order (not the terms) varies
    np.testing.assert_allclose(Cl, np.conj(Cu), rtol=1e-13, atol=1e-13 * np.abs(Cu).max())
    np.testing.assert_allclose(al, au, rtol=1e-13)
    assert dl == pytest.approx(-du, rel=1e-12, abs=1e-20)


def test_streams_ordered(pc):
    """Calls on different streams are ordered after each other (shared accumulators)."""
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    L = 1 << 22
    packed = synth.make_stream(spec, L)
    dev = _dev(packed)
    streams = [torch.cuda.Stream() for _ in range(3)]
    h = pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 2)
    q = L // 4
    for i in range(4):
        h.extract(dev[i * q // 4:], q, stream=streams[i % 3])
    C = h.spectrum()
    h.close()
    Co = oracle.correlate(packed, 2, L, spec.fs, spec.f_comb, spec.f_offset)
    assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="streams")


def test_invalid_calls(pc):
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    h = pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 2)
    dev = _dev(np.zeros(64, np.uint8))
    with pytest.raises(pc.PcalError) as e:
        h.extract(dev, 6)                 # not a multiple of 4 samples
    assert e.value.code == pc.EINVAL
    with pytest.raises(pc.PcalError):
        h.bins(integer=True)              # integer bins only exist for f_offset = 0
    h.close()


@pytest.mark.parametrize("case", ["n64_pinned", "n64_pageable", "n256_pinned", "lut_pinned"])
def test_results_async_pipelined(pc, case):
    """Pipelined integrations: results_async(reset) equals synchronous results, and resets.

    With reset the finalize is deferred into the next fold launch (extra
    workgroups, the other accumulator bank); a single-workgroup finalize writes
    mapped pinned host memory directly, otherwise results are copied."""
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    method = pc.METHOD_AUTO
    if case == "n256_pinned":
        spec = synth.CombSpec(256_000_000, 1_000_000, 10_000, 2, amp=0.05, t_d=4e-9, seed=(41, 2))
    if case == "lut_pinned":
        method = pc.METHOD_LUT
    L = 1 << 21
    K = 5  # integrations: the two accumulator banks are each reused
    packed = synth.make_stream(spec, (K + 1) * L)
    dev = _dev(packed)
    N = spec.ntones
    say("results_async pipelined: %s" % case)
    if case == "n64_pageable":
        ring = torch.from_numpy(np.zeros((K, 4 * N + 1)))
    else:
        ring = torch.zeros((K, 4 * N + 1), dtype=torch.float64, pin_memory=True)
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 2, method=method) as h:
        for i in range(K):
            h.extract(dev[i * L // 4:], L // 2)
            h.extract(dev[i * L // 4 + L // 8:], L // 2)
            h.results_async(ring[i], reset=True)
        # a synchronous read of the next integration sees only its own samples
        h.extract(dev[K * L // 4:], L)
        Cn = h.spectrum()
        h.sync()
        assert h.info()["samples_integ"] == L and h.info()["samples_total"] == (K + 1) * L
    # the per-sample table form adds FP32 products per sample: the contract tolerance
    tol = (1e-5, 1e-4, 1e-5, 1e-10) if case == "lut_pinned" else (F64_RTOL, F64_RTOL, 1e-9, 1e-13)
    Co = oracle.correlate(packed[K * L // 4:(K + 1) * L // 4], 2, L, spec.fs, spec.f_comb, spec.f_offset, n0=K * L)
    assert_spectra(Cn, Co, amp_rtol=tol[0], phase_atol=tol[1], what="after async resets")
    for i in range(K):
        r = ring[i].numpy()
        C = r[2 * N:3 * N] + 1j * r[3 * N:4 * N]
        Co = oracle.correlate(packed[i * L // 4:(i + 1) * L // 4], 2, L, spec.fs, spec.f_comb, spec.f_offset,
                              n0=i * L)
        assert_spectra(C, Co, amp_rtol=tol[0], phase_atol=tol[1], what="async %d" % i)
        ao, po, do = oracle.results(Co, L, spec.fs, spec.f_comb, spec.f_offset)
        np.testing.assert_allclose(r[:N], ao, rtol=tol[2])
        assert abs(r[4 * N] - do) < tol[3]


@pytest.mark.parametrize("tones", [64, 256])
def test_flush_delivers_results_without_another_extract(pc, tones):
    """pcal_flush enqueues the finalize that results_async(reset) deferred: once the
    handle's stream has reached it, host_out holds the integration's results, with
    no further extract on the handle; the next integration starts from zero."""
    spec = synth.CombSpec(tones * 1_000_000, 1_000_000, 10_000, 2, amp=0.05, t_d=4e-9, seed=(43, tones))
    L = 1 << 21
    packed = synth.make_stream(spec, 3 * L)
    dev = _dev(packed)
    N = spec.ntones
    st = torch.cuda.Stream()
    ring = torch.zeros((2, 4 * N + 1), dtype=torch.float64, pin_memory=True)
    say("flush: N = %d" % N)
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 2) as h:
        for i in range(2):
            h.extract(dev[i * L // 4:], L, stream=st)
            h.results_async(ring[i], reset=True)
            h.flush()
            h.flush()  # nothing pending: no-op
            st.synchronize()
            r = ring[i].numpy()
            C = r[2 * N:3 * N] + 1j * r[3 * N:4 * N]
            Co = oracle.correlate(packed[i * L // 4:(i + 1) * L // 4], 2, L, spec.fs, spec.f_comb, spec.f_offset,
                                  n0=i * L)
            assert_spectra(C, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="flushed %d" % i)
        # a later extract on another stream is ordered after the flushed finalize (it cleared a bank)
        h.extract(dev[2 * L // 4:], L)
        Cn = h.spectrum()
    Co = oracle.correlate(packed[2 * L // 4:3 * L // 4], 2, L, spec.fs, spec.f_comb, spec.f_offset, n0=2 * L)
    assert_spectra(Cn, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="after flushes")


@pytest.mark.gpu
def test_extract_timed_matches_extract():
    """pcal_extract_timed: the same bins as pcal_extract, and events that bracket the kernel."""
    import torch
    from paper_2501_05993_amd import pcal

    spec = synth.CombSpec(64_000_000, 1_000_000, 10_000, 2, amp=0.3, t_d=5e-9, sigma=1.0, seed=(31, 1))
    ns = 4 * 300_001
    buf = synth.make_stream_device(spec, ns)
    say("extract_timed: 64 MHz / 10 kHz, %d samples" % ns)
    a = pcal.PCal(spec.fs, spec.f_comb, spec.f_offset, 2)
    b = pcal.PCal(spec.fs, spec.f_comb, spec.f_offset, 2)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    e1.record(stream)
    a.extract(buf, ns)
    b.extract(buf, ns, events=(e0, e1))
    torch.cuda.synchronize()
    ra, rb = a.spectrum(), b.spectrum()
    np.testing.assert_array_equal(np.abs(ra - rb) <= 1e-12 * np.abs(ra).max(), True)
    ms = e0.elapsed_time(e1)
    assert 0.0 < ms < 50.0
    a.close()
    b.close()


def test_repeatability(pc):
    """The FP64 bins are summed with hardware atomics (16 slots, added in slot
    order by the finalize), so the order of the additions within a slot varies
    from run to run: repeated extractions agree to FP64 rounding (far below
    the 1e-10 parity bar), and the exact integer bins (f_offset = 0) agree bit
    for bit."""
    spec = synth.WORKLOADS["fold2_64M_10k"]["spec"]
    L = 1 << 26
    packed = synth.make_stream(spec, L)
    dev = _dev(packed)
    runs = []
    for _ in range(3):
        with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, 2) as h:
            h.extract(dev, L)
            runs.append(h.spectrum())
    scale = np.abs(runs[0]).max()
    for C in runs[1:]:
        d = np.abs(C - runs[0]).max() / scale
        say("repeatability: max |dC| / max |C| = %.3e" % d)
        assert d < 1e-13
    s0 = synth.WORKLOADS["small_2bit_fo0"]["spec"]
    p0 = synth.make_stream(s0, 1 << 22)
    d0 = _dev(p0)
    bins = []
    for _ in range(3):
        with pc.PCal(s0.fs, s0.f_comb, 0, 2) as h:
            h.extract(d0, 1 << 22)
            bins.append(h.bins(integer=True)[1])
    for b in bins[1:]:
        np.testing.assert_array_equal(b, bins[0])
