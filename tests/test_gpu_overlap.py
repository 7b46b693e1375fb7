"""Pipelined integrations (pcal_results_async with PCAL_RESET_OVERLAP) on the GPU.

A handle whose integrations end with the overlap reset alternates them
between two lanes (accumulators, pending finalize and stream order of their
own), so integrations fed on two streams in turn run side by side.  Every
integration's results must equal those of the same handle driven the plain
way (one stream, a plain reset per integration) to FP64 rounding (the
accumulators' atomics add in another order), and one of them the oracle.
The mixed sequence checks what the lanes must keep: plain resets between
overlapped ones (which end the alternation), a third stream, a readout of
the new integration before its first extract, results read synchronously
within an integration, results copied from the device into pageable memory,
and the global sample index across lanes.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import F64_RTOL, assert_spectra, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

L = 1 << 24          # samples per integration
NINT = 6             # integrations


@pytest.fixture(scope="module")
def pc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_05993_amd import pcal

    pcal.lib()
    return pcal


def _stream_data(spec, n):
    buf = synth.make_stream_device(spec, n)
    torch.cuda.synchronize()
    return buf


def _spectra(ring, N):
    r = ring.cpu().numpy() if isinstance(ring, torch.Tensor) else ring
    return [row[2 * N:3 * N] + 1j * row[3 * N:4 * N] for row in r]


def _plain(pc, spec, buf, n_int, method=1, prec=0, halves=False):
    """Reference: one stream, a plain reset per integration."""
    N = spec.ntones
    spb = 8 // spec.nbits
    ring = torch.zeros((n_int, 4 * N + 1), dtype=torch.float64, pin_memory=True)
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits, method=method, precision=prec) as h:
        for k in range(n_int):
            c = (L // 2) if halves else (L // 3 // spb * spb)
            h.extract(buf, c, byte_offset=k * L // spb)
            h.extract(buf, L - c, byte_offset=(k * L + c) // spb)
            h.results_async(ring[k], reset=True)
        h.sync()
    return _spectra(ring, N)


@pytest.mark.parametrize("method,prec", [(1, 0), (1, 1), (3, 0)])
def test_overlap_two_streams_equals_plain(pc, method, prec):
    # the per-sample form on a prime offset (rotator period = fs, 16e6 samples)
    spec = (synth.CombSpec(64_000_000, 1_000_000, 10_000, 2, amp=0.3, t_d=4e-9, seed=(97, method, prec))
            if method == 1 else synth.CombSpec(16_000_000, 1_000_000, 10_007, 2, amp=0.3, t_d=4e-9, seed=(97, method)))
    buf = _stream_data(spec, NINT * L)
    want = _plain(pc, spec, buf, NINT, method, prec)
    N = spec.ntones
    spb = 8 // spec.nbits
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ring = torch.zeros((NINT, 4 * N + 1), dtype=torch.float64, pin_memory=True)
    say("overlap: method %d, precision form %d, %d integrations of 2^24 samples on two streams in turn"
        % (method, prec, NINT))
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits, method=method, precision=prec) as h:
        for k in range(NINT):
            st = streams[k % 2]
            c = L // 3 // spb * spb
            h.extract(buf, c, byte_offset=k * L // spb, stream=st)
            h.extract(buf, L - c, byte_offset=(k * L + c) // spb, stream=st)
            h.results_async(ring[k], reset=pc.RESET_OVERLAP)
        assert h.info()["samples_total"] == NINT * L
        h.flush()
        h.sync()
        got = _spectra(ring, N)
    tol = F64_RTOL if prec == 0 else 1e-6
    for k in range(NINT):
        assert_spectra(got[k], want[k], amp_rtol=tol, phase_atol=tol, rel_floor=1e-6,
                       what="overlapped integration %d vs plain" % k)
    if prec == 0:
        host = buf.cpu().numpy()
        k = 3
        Co = oracle.correlate(host[k * L // spb:(k + 1) * L // spb], spec.nbits, L, spec.fs, spec.f_comb,
                              spec.f_offset, n0=k * L)
        assert_spectra(got[k], Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="overlapped integration vs oracle")


def test_overlap_mixed_sequences(pc):
    spec = synth.CombSpec(128_000_000, 1_000_000, 250_000, 2, amp=0.3, t_d=7e-9, seed=(98,))
    n_int = 8
    buf = _stream_data(spec, n_int * L)
    N = spec.ntones
    spb = 8 // spec.nbits
    want = _plain(pc, spec, buf, n_int, halves=True)
    s = [torch.cuda.Stream() for _ in range(3)]
    ring = torch.zeros((n_int, 4 * N + 1), dtype=torch.float64, pin_memory=True)
    pageable = np.zeros((n_int, 4 * N + 1))
    # (stream of integration k, its reset, whether its results go to pageable memory)
    plan = [(0, "overlap", False), (1, "overlap", True), (0, "plain", False), (2, "overlap", False),
            (0, "overlap", False), (0, "overlap", True), (1, "plain", False), (2, "overlap", False)]
    say("overlap: mixed sequence over %d integrations, three streams" % n_int)
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits) as h:
        for k, (si, how, page) in enumerate(plan):
            if k in (1, 5):
                # a readout of the new integration before its first extract: its bins start at zero
                assert np.all(h.bins() == 0.0), "integration %d starts cleared" % k
            h.extract(buf, L // 2, byte_offset=k * L // spb, stream=s[si])
            if k == 4:
                # results so far, synchronously, inside an integration (no reset)
                half = h.spectrum()
                Co = oracle.correlate(buf[k * L // spb:(k * L + L // 2) // spb].cpu().numpy(), spec.nbits, L // 2,
                                      spec.fs, spec.f_comb, spec.f_offset, n0=k * L)
                assert_spectra(half, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="half integration 4")
            h.extract(buf, L // 2, byte_offset=(k * L + L // 2) // spb, stream=s[si])
            out = pageable[k] if page else ring[k]
            h.results_async(out, reset=pc.RESET_OVERLAP if how == "overlap" else True)
        assert h.info()["samples_total"] == n_int * L
        h.sync()  # runs and waits for both lanes' pending finalizes
    got = _spectra(ring, N)
    for k, (si, how, page) in enumerate(plan):
        g = (pageable[k][2 * N:3 * N] + 1j * pageable[k][3 * N:4 * N]) if page else got[k]
        assert_spectra(g, want[k], amp_rtol=F64_RTOL, phase_atol=F64_RTOL, rel_floor=1e-6,
                       what="integration %d (stream %d, %s reset)" % (k, si, how))


def test_overlap_refused_for_batch_members(pc):
    """A batch folds its members in one lane: the overlap reset on a member handle is PCAL_ENOTSUP
    (the plain reset stays available)."""
    import ctypes

    with pc.PCalBatch(2) as b:
        i = b.add(64_000_000, 1_000_000, 10_000, 2)
        h = ctypes.c_void_p()
        assert pc.lib().pcal_batch_handle(b._b, i, ctypes.byref(h)) == pc.OK
        out = torch.zeros(4 * 64 + 1, dtype=torch.float64, pin_memory=True)
        assert pc.lib().pcal_results_async(h, ctypes.c_void_p(out.data_ptr()), pc.RESET_OVERLAP) == pc.ENOTSUP
        assert pc.lib().pcal_results_async(h, ctypes.c_void_p(out.data_ptr()), 1) == pc.OK
        assert pc.lib().pcal_sync(h) == pc.OK


@pytest.mark.parametrize("seed", [3, 4])
def test_overlap_random_sequences(pc, seed):
    """Seeded random sequences: each integration in one to three chunks on one of three streams,
    ended by an overlapped or a plain reset, with synchronous readouts of the integration so far
    between chunks now and then; every integration equals the plain one-stream sequence's."""
    rng = np.random.default_rng(seed)
    spec = synth.CombSpec(32_000_000, 1_000_000, 10_000, 2, amp=0.3, t_d=3e-9, seed=(99, seed))
    n_int = 10
    Li = 1 << 22
    buf = _stream_data(spec, n_int * Li)
    N = spec.ntones
    spb = 8 // spec.nbits
    ref = torch.zeros((n_int, 4 * N + 1), dtype=torch.float64, pin_memory=True)
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits) as h:
        for k in range(n_int):
            h.extract(buf, Li, byte_offset=k * Li // spb)
            h.results_async(ref[k], reset=True)
        h.sync()
    want = _spectra(ref, N)
    s = [torch.cuda.Stream() for _ in range(3)]
    ring = torch.zeros((n_int, 4 * N + 1), dtype=torch.float64, pin_memory=True)
    say("overlap: random sequence, seed %d" % seed)
    with pc.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits) as h:
        for k in range(n_int):
            cuts = sorted(set(int(c) * spb for c in rng.integers(1, Li // spb, size=int(rng.integers(0, 3)))))
            edges = [0] + cuts + [Li]
            st = s[int(rng.integers(0, 3))]
            for a, b in zip(edges[:-1], edges[1:]):
                h.extract(buf, b - a, byte_offset=(k * Li + a) // spb, stream=st)
                if rng.random() < 0.2:
                    part = h.spectrum()
                    Co = oracle.correlate(buf[k * Li // spb:(k * Li + b) // spb].cpu().numpy(), spec.nbits, b,
                                          spec.fs, spec.f_comb, spec.f_offset, n0=k * Li)
                    assert_spectra(part, Co, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, rel_floor=1e-6,
                                   what="integration %d so far" % k)
            h.results_async(ring[k], reset=pc.RESET_OVERLAP if rng.random() < 0.7 else True)
        h.sync()
    got = _spectra(ring, N)
    for k in range(n_int):
        assert_spectra(got[k], want[k], amp_rtol=F64_RTOL, phase_atol=F64_RTOL, rel_floor=1e-6,
                       what="random sequence %d, integration %d" % (seed, k))
