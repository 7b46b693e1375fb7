"""Served form (pcal_server_*): continuous batching of many live streams.

Each integration a server reports must equal the plain one-stream extraction
of the same samples (same handle semantics: the global sample index runs on
across integrations), whatever mix of other streams shared its launches and
however its chunks straddled integration boundaries; one stream is also
checked against the oracle.  Admission by memory budget: a stream that does
not fit is refused with PCAL_EAGAIN and admitted once budget is released.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import AMP_RTOL, F64_RTOL, PHASE_ATOL, assert_spectra, say

pytestmark = pytest.mark.gpu

STREAMS = [
    # fs, f_comb, f_offset, nbits, integration samples
    (64_000_000, 1_000_000, 10_000, 2, 600_000),
    (32_000_000, 1_000_000, 0, 2, 400_000),
    (16_000_000, 1_000_000, 250_000, 2, 333_332),
    (128_000_000, 1_000_000, 510_000, 8, 500_001),
    (256_000_000, 2_000_000, 10_000, 2, 1_000_000),
]
TOTAL = 2_000_000  # samples per stream (several integrations, the last one partial)


def _chunks(rng, total, spb):
    """Random chunk sizes (multiples of the samples per byte) covering total."""
    out, n = [], 0
    while n < total:
        c = int(rng.integers(1, 300_000)) * spb
        c = min(c, total - n)
        out.append(c)
        n += c
    return out


def _streams_on_device():
    import torch

    data = []
    for i, (fs, fc, fo, nbits, integ) in enumerate(STREAMS):
        spec = synth.CombSpec(fs, fc, fo, nbits, amp=0.3 if nbits == 2 else 4.0, t_d=5e-9,
                              sigma=1.0 if nbits == 2 else 20.0, seed=(61, i))
        data.append(synth.make_stream_device(spec, TOTAL))
    torch.cuda.synchronize()
    return data


def _plain_integrations(buf, fs, fc, fo, nbits, integ, prec=0):
    """Spectra of the complete integrations with one plain handle, extract + reset per integration."""
    from paper_2501_05993_amd import pcal

    spb = 8 // nbits
    out = []
    with pcal.PCal(fs, fc, fo, nbits, method=pcal.METHOD_PERIOD_FOLD, precision=prec) as h:
        for k in range(TOTAL // integ):
            h.extract(buf, integ, byte_offset=k * integ // spb)
            out.append(h.spectrum())
            h.reset()
    return out


# alone (one plain handle) vs in the served mix: the FP64 form to its rounding, the
# reduced forms to the reordering of their FP32 sums (atomics, Kahan compensation)
ALONE_TOL = {0: F64_RTOL, 1: 1e-6, 2: 1e-5}


@pytest.mark.parametrize("prec,resident,task_kib", [(0, False, None), (1, False, None), (2, False, None),
                                                    (0, True, None), (1, True, None), (0, True, 8),
                                                    (0, True, "backlog")])
def test_served_matches_plain_per_integration(prec, resident, task_kib, monkeypatch):
    """Host-step form, and the device-resident form (one persistent kernel fed through the work
    ring: 24 workgroups, fewer than a chunk's 32 task indices, so chunks also run one task after
    another; with 8 KiB per fold task, most tasks of a chunk read the descriptor's device copy;
    "backlog": 8 KiB per task, 64 KiB whenever the chunk before has not ended, so the chunks of
    one integration come with task counts of both sizes)."""
    import time

    from paper_2501_05993_amd import pcal

    bufs = _streams_on_device()
    rng = np.random.default_rng(5)
    srv = pcal.PCalServer(mem_budget_bytes=1 << 30, max_streams=len(STREAMS), precision=prec)
    sids = []
    for fs, fc, fo, nbits, integ in STREAMS:
        sids.append(srv.open(fs, fc, fo, nbits, integ))
    if resident:
        if task_kib == "backlog":
            monkeypatch.setenv("PCAL_SERVED_TASK_KIB", "8")
            monkeypatch.setenv("PCAL_SERVED_BACKLOG", "1")
            monkeypatch.setenv("PCAL_SERVED_BACKLOG_TASK_KIB", "64")
        elif task_kib is not None:  # many fold tasks per chunk: most read the descriptor's device copy
            monkeypatch.setenv("PCAL_SERVED_TASK_KIB", str(task_kib))
        srv.start(workgroups=24)
    # interleave the streams' chunks in a random order of arrival
    queue = []
    for i, (fs, fc, fo, nbits, integ) in enumerate(STREAMS):
        spb = 8 // nbits
        off = 0
        for c in _chunks(rng, TOTAL, spb):
            queue.append((i, off, c))
            off += c
    order = np.argsort(rng.random(len(queue)), kind="stable")
    # keep per-stream order: sort by (arrival rank) but within a stream by offset
    per = {i: [q for q in queue if q[0] == i] for i in range(len(STREAMS))}
    arrivals, pos = [], {i: 0 for i in per}
    for j in order:
        i = queue[j][0]
        arrivals.append(per[i][pos[i]])
        pos[i] += 1
    say("served (precision form %d, resident %s): %d streams, %d chunks" % (prec, resident, len(STREAMS),
                                                                          len(arrivals)))
    got = {}
    k = 0
    while k < len(arrivals) or srv.stats()["queued_samples"] > 0:
        burst = arrivals[k:k + int(rng.integers(1, 8))]
        k += len(burst)
        if burst:
            srv.submit([sids[i] for i, _, _ in burst],
                       [bufs[i].data_ptr() + off // (8 // STREAMS[i][3]) for i, off, _ in burst],
                       [c for _, _, c in burst])
        srv.step()
        for sid, integ in srv.poll():
            got[(sid, integ)] = srv.spectrum(sid, integ)
    import torch

    if resident:
        t_end = time.time() + 60.0
        while time.time() < t_end:
            srv.step()
            for sid, integ in srv.poll():
                got[(sid, integ)] = srv.spectrum(sid, integ)
            st = srv.stats()
            if st["queued_samples"] == 0 and st["inflight_finalizes"] == 0:
                break
        srv.stop()
        for sid, integ in srv.poll():
            got[(sid, integ)] = srv.spectrum(sid, integ)
        loop = srv.loop_stats()
        say("loop counters: %s" % loop)
        assert loop["tasks_run"] == loop["tasks_published"]
    torch.cuda.synchronize()
    for _ in range(100):
        for sid, integ in srv.poll():
            got[(sid, integ)] = srv.spectrum(sid, integ)
        if srv.stats()["inflight_finalizes"] == 0:
            break
    bad = []
    for i, (fs, fc, fo, nbits, integ) in enumerate(STREAMS):
        want = _plain_integrations(bufs[i], fs, fc, fo, nbits, integ, prec)
        assert len(want) == TOTAL // integ
        for k2, w in enumerate(want):
            assert (sids[i], k2) in got, "integration %d of stream %d not reported" % (k2, i)
            try:
                assert_spectra(got[(sids[i], k2)], w, amp_rtol=ALONE_TOL[prec], phase_atol=ALONE_TOL[prec],
                               rel_floor=1e-6, what="stream %d integration %d" % (i, k2))
            except AssertionError as err:  # report every integration before failing
                bad.append(str(err))
    assert not bad, bad
    # one stream against the oracle: its second integration (global index continues)
    fs, fc, fo, nbits, integ = STREAMS[0]
    host = bufs[0].cpu().numpy()
    sub = host[integ // 4:2 * integ // 4]
    want = oracle.correlate(sub, nbits, integ, fs, fc, fo, n0=integ)
    if prec == 0:
        assert_spectra(got[(sids[0], 1)], want, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, what="served vs oracle")
    else:
        assert_spectra(got[(sids[0], 1)], want, amp_rtol=AMP_RTOL, phase_atol=PHASE_ATOL, rel_floor=1e-6,
                       what="served form %d vs oracle" % prec)
    srv.close()


def test_served_admission_by_memory_budget():
    from paper_2501_05993_amd import pcal

    probe = pcal.PCalServer(mem_budget_bytes=1 << 30, max_streams=1)
    a = probe.open(64_000_000, 1_000_000, 10_000, 2, 1 << 20)
    need = probe.stats()["device_bytes"]
    probe.close()
    assert need > 0
    say("served admission: %d device bytes per stream" % need)
    srv = pcal.PCalServer(mem_budget_bytes=need + need // 2, max_streams=4)
    a = srv.open(64_000_000, 1_000_000, 10_000, 2, 1 << 20)
    with pytest.raises(pcal.PcalError) as e:
        srv.open(64_000_000, 1_000_000, 10_000, 2, 1 << 20)
    assert e.value.code == pcal.EAGAIN
    assert srv.stats()["device_bytes"] == need
    srv.close_stream(a)
    assert srv.stats()["device_bytes"] == 0
    b = srv.open(64_000_000, 1_000_000, 10_000, 2, 1 << 20)
    assert b >= 0
    # the planner's device bytes (no allocation) are what the stream takes
    assert pcal.plan(64_000_000, 1_000_000, 10_000, 2, method=pcal.METHOD_PERIOD_FOLD)["device_bytes"] == need
    with pytest.raises(pcal.PcalError) as e:
        srv.submit([b], [0], [3])  # not a multiple of the samples per byte
    assert e.value.code == pcal.EINVAL
    srv.close()


def test_served_admission_refuses_before_allocating():
    """A budget below one stream's device bytes: the open is refused with PCAL_EAGAIN from the plan
    alone, nothing is allocated (no device bytes in use, the free device memory unchanged), and a
    stream that fits is admitted afterwards."""
    import torch
    from paper_2501_05993_amd import pcal

    need = pcal.plan(128_000_000, 1_000_000, 250_000, 8, method=pcal.METHOD_PERIOD_FOLD,
                     precision=pcal.PREC_MIXED)["device_bytes"]
    small = pcal.plan(32_000_000, 1_000_000, 0, 2, method=pcal.METHOD_PERIOD_FOLD,
                      precision=pcal.PREC_MIXED)["device_bytes"]
    assert small < need
    srv = pcal.PCalServer(mem_budget_bytes=need - 1, max_streams=2, precision=pcal.PREC_MIXED)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    with pytest.raises(pcal.PcalError) as e:
        srv.open(128_000_000, 1_000_000, 250_000, 8, 1 << 20)
    assert e.value.code == pcal.EAGAIN
    assert srv.stats()["device_bytes"] == 0
    assert torch.cuda.mem_get_info()[0] == free0
    a = srv.open(32_000_000, 1_000_000, 0, 2, 1 << 20)
    assert srv.stats()["device_bytes"] == small
    srv.close_stream(a)
    srv.close()


def test_served_resident_states_and_limits():
    """Start twice / stop when not started: PCAL_ESTATE; a stream of more than 1792 tones is refused in the
    device-resident form (PCAL_ENOTSUP) but admitted by the host-step form; a started loop with no work
    stops at once and every workgroup leaves."""
    from paper_2501_05993_amd import pcal

    srv = pcal.PCalServer(mem_budget_bytes=1 << 30, max_streams=4)
    with pytest.raises(pcal.PcalError) as e:
        srv.stop()
    assert e.value.code == pcal.ESTATE
    srv.start(workgroups=8)
    with pytest.raises(pcal.PcalError) as e:
        srv.start(workgroups=8)
    assert e.value.code == pcal.ESTATE
    with pytest.raises(pcal.PcalError) as e:
        srv.open(4_096_000_000, 1_000_000, 0, 2, 1 << 20)  # N = 4096
    assert e.value.code == pcal.ENOTSUP
    srv.stop()
    a = srv.open(4_096_000_000, 1_000_000, 0, 2, 1 << 20)
    with pytest.raises(pcal.PcalError) as e:
        srv.start(workgroups=8)  # an open stream does not fit the resident form
    assert e.value.code == pcal.ENOTSUP
    srv.close_stream(a)
    srv.close()


PER_SAMPLE_MIX = [
    # fs, f_comb, f_offset, nbits, integration samples: one fold stream, two no fold period fits
    (64_000_000, 1_000_000, 10_000, 2, 600_000),
    (128_000_000, 2_000_000, 10_007, 2, 500_000),
    (64_000_000, 2_000_000, 10_007, 8, 400_000),
]


@pytest.mark.parametrize("prec", [0, 1])
def test_served_host_step_per_sample_streams(prec):
    """Streams whose rotator has no fold period that fits (prime f_offset) are admitted by the host-step
    form, which runs them in per-sample launches beside the batched fold: every integration of each
    stream, arriving in random chunks, equals a plain AUTO handle's; the resident form refuses them
    (PCAL_ENOTSUP), both at open on a started server and at start with one open."""
    import torch

    from paper_2501_05993_amd import pcal

    bufs = []
    for i, (fs, fc, fo, nbits, integ) in enumerate(PER_SAMPLE_MIX):
        spec = synth.CombSpec(fs, fc, fo, nbits, amp=0.3 if nbits == 2 else 4.0, t_d=5e-9,
                              sigma=1.0 if nbits == 2 else 20.0, seed=(71, i))
        bufs.append(synth.make_stream_device(spec, TOTAL))
    torch.cuda.synchronize()
    srv = pcal.PCalServer(mem_budget_bytes=1 << 30, max_streams=4, precision=prec)
    srv.start(workgroups=8)
    with pytest.raises(pcal.PcalError) as e:
        srv.open(*PER_SAMPLE_MIX[1])
    assert e.value.code == pcal.ENOTSUP
    srv.stop()
    sids = [srv.open(*m) for m in PER_SAMPLE_MIX]
    with pytest.raises(pcal.PcalError) as e:
        srv.start(workgroups=8)
    assert e.value.code == pcal.ENOTSUP
    rng = np.random.default_rng(17)
    arrivals = []
    for i, (fs, fc, fo, nbits, integ) in enumerate(PER_SAMPLE_MIX):
        off = 0
        for c in _chunks(rng, TOTAL, 8 // nbits):
            arrivals.append((rng.random(), i, off, c))
            off += c
    # a random arrival order across streams, each stream's chunks in order
    arrivals.sort(key=lambda a: a[0])
    nxt = {i: 0 for i in range(len(PER_SAMPLE_MIX))}
    per = {i: sorted([a for a in arrivals if a[1] == i], key=lambda a: a[2]) for i in nxt}
    order = []
    for a in arrivals:
        order.append(per[a[1]][nxt[a[1]]])
        nxt[a[1]] += 1
    say("served host-step with per-sample streams (precision form %d): %d chunks" % (prec, len(order)))
    got = {}
    k = 0
    while k < len(order) or srv.stats()["queued_samples"] > 0:
        burst = order[k:k + int(rng.integers(1, 6))]
        k += len(burst)
        if burst:
            srv.submit([sids[i] for _, i, _, _ in burst],
                       [bufs[i].data_ptr() + off // (8 // PER_SAMPLE_MIX[i][3]) for _, i, off, _ in burst],
                       [c for _, _, _, c in burst])
        srv.step()
        for sid, integ in srv.poll():
            got[(sid, integ)] = srv.spectrum(sid, integ)
    torch.cuda.synchronize()
    for _ in range(100):
        for sid, integ in srv.poll():
            got[(sid, integ)] = srv.spectrum(sid, integ)
        if srv.stats()["inflight_finalizes"] == 0:
            break
    bad = []
    for i, (fs, fc, fo, nbits, integ) in enumerate(PER_SAMPLE_MIX):
        spb = 8 // nbits
        with pcal.PCal(fs, fc, fo, nbits, precision=prec) as h:
            if i:
                assert h.info()["method"] != pcal.METHOD_PERIOD_FOLD
            for k2 in range(TOTAL // integ):
                h.extract(bufs[i], integ, byte_offset=k2 * integ // spb)
                w = h.spectrum()
                h.reset()
                assert (sids[i], k2) in got, "integration %d of stream %d not reported" % (k2, i)
                # a per-sample form in FP32 restarts its rotator recurrence at every launch: chunked
                # and whole extraction differ by that FP32 recurrence error, within the contract
                at, pt = (ALONE_TOL[prec],) * 2 if i == 0 or prec == 0 else (AMP_RTOL, PHASE_ATOL)
                try:
                    assert_spectra(got[(sids[i], k2)], w, amp_rtol=at, phase_atol=pt,
                                   rel_floor=1e-6, what="stream %d integration %d" % (i, k2))
                except AssertionError as err:
                    bad.append(str(err))
    assert not bad, bad
    # a per-sample stream against the oracle: its second integration
    fs, fc, fo, nbits, integ = PER_SAMPLE_MIX[2]
    host = bufs[2].cpu().numpy()
    want = oracle.correlate(host[integ:2 * integ], nbits, integ, fs, fc, fo, n0=integ)
    if prec == 0:
        assert_spectra(got[(sids[2], 1)], want, amp_rtol=F64_RTOL, phase_atol=F64_RTOL, rel_floor=1e-6,
                       what="per-sample stream vs oracle")
    else:
        assert_spectra(got[(sids[2], 1)], want, amp_rtol=AMP_RTOL, phase_atol=PHASE_ATOL, rel_floor=1e-6,
                       what="per-sample stream, form %d, vs oracle" % prec)
    srv.close()


def test_served_resident_relaunch_after_idle(monkeypatch):
    """The device-resident loop leaves once idle for its limit (200 ms here) and the next step launches
    it again where it stopped: integrations served before and after equal plain extraction, and the
    loop counters add up (one relaunch at least, every fold task counted, one finalize per integration)."""
    import time

    from paper_2501_05993_amd import pcal

    monkeypatch.setenv("PCAL_SERVED_IDLE_MS", "200")
    bufs = _streams_on_device()
    fs, fc, fo, nbits, integ = STREAMS[0]
    spb = 8 // nbits
    want = _plain_integrations(bufs[0], fs, fc, fo, nbits, integ, 0)
    srv = pcal.PCalServer(mem_budget_bytes=1 << 30, max_streams=2, precision=0)
    sid = srv.open(fs, fc, fo, nbits, integ)
    srv.start(workgroups=16)
    got = {}

    def serve(k):
        # integration k in three chunks of whole bytes, then wait (bounded) for its report
        cuts = [k * integ, k * integ + integ // 3 // spb * spb, k * integ + 2 * integ // 3 // spb * spb,
                (k + 1) * integ]
        for a, b in zip(cuts[:-1], cuts[1:]):
            srv.submit([sid], [bufs[0].data_ptr() + a // spb], [b - a])
        t_end = time.time() + 30.0
        while (sid, k) not in got and time.time() < t_end:
            srv.step()
            for s_, k_ in srv.poll():
                got[(s_, k_)] = srv.spectrum(s_, k_)
        assert (sid, k) in got, "integration %d not reported" % k

    say("resident loop: integration 0, 1 s idle, integration 1")
    serve(0)
    time.sleep(1.0)  # every workgroup leaves after 200 ms without work
    serve(1)
    srv.stop()
    st = srv.loop_stats()
    say("loop counters: %s" % st)
    assert st["relaunches"] >= 1
    assert st["finalizes"] == 2
    assert st["tasks_run"] == st["tasks_published"] >= st["chunks_published"] == 6
    assert st["descriptor_reads_from_host"] == 6  # the scheduler's copies, one per chunk
    for k in range(2):
        assert_spectra(got[(sid, k)], want[k], amp_rtol=F64_RTOL, phase_atol=F64_RTOL,
                       what="integration %d around a relaunch" % k)
    with pytest.raises(pcal.PcalError) as e:
        srv.start(workgroups=1)  # the scheduler needs at least one worker
    assert e.value.code == pcal.EINVAL
    srv.close()


@pytest.mark.parametrize("prec", [0, 2])
def test_served_resident_wide_stream(prec):
    """A stream of 1536 tones (twiddles beyond the served finalize's LDS share) through the device-
    resident loop, FP64 and FP32 forms: each integration equals plain extraction.  In the FP32 form the
    two differ by the order of their FP32 sums, an error of about FP32 rounding times the strongest
    tone: tones more than 40 dB below it are compared by their absolute error against it."""
    import time

    import torch

    from paper_2501_05993_amd import pcal

    fs, fc, fo, nbits = 1_536_000_000, 1_000_000, 10_000, 2
    integ, n_integ, spb = 1_536_000, 2, 4
    spec = synth.CombSpec(fs, fc, fo, nbits, amp=0.3, t_d=5e-9, sigma=1.0, seed=(67, prec))
    buf = synth.make_stream_device(spec, integ * n_integ)
    torch.cuda.synchronize()
    want = []
    with pcal.PCal(fs, fc, fo, nbits, method=pcal.METHOD_PERIOD_FOLD, precision=prec) as h:
        for k in range(n_integ):
            h.extract(buf, integ, byte_offset=k * integ // spb)
            want.append(h.spectrum())
            h.reset()
    srv = pcal.PCalServer(mem_budget_bytes=1 << 30, max_streams=1, precision=prec)
    sid = srv.open(fs, fc, fo, nbits, integ)
    srv.start(workgroups=32)
    cuts = [0, 400_000, 1_536_000, 2_000_000, integ * n_integ]
    for a, b in zip(cuts[:-1], cuts[1:]):
        srv.submit([sid], [buf.data_ptr() + a // spb], [b - a])
    got = {}
    t_end = time.time() + 30.0
    while len(got) < n_integ and time.time() < t_end:
        srv.step()
        for s_, k_ in srv.poll():
            got[k_] = srv.spectrum(s_, k_)
    srv.stop()
    for k in range(n_integ):
        assert k in got, "integration %d not reported" % k
        assert_spectra(got[k], want[k], amp_rtol=ALONE_TOL[prec], phase_atol=ALONE_TOL[prec],
                       rel_floor=1e-6 if prec == 0 else 1e-2, what="1536 tones, form %d, integration %d" % (prec, k))
    srv.close()


def test_served_resident_idle_workers_stay(monkeypatch):
    """Workers that wait longer than their own time limit (150 ms here) stay while the scheduler's
    heartbeat moves: after 1 s of idling (the loop itself stays, its idle limit being 4 s), a burst of
    small chunks spread over many workers is served completely and equals plain extraction; no relaunch."""
    import time

    from paper_2501_05993_amd import pcal

    monkeypatch.setenv("PCAL_SERVED_WORKER_MS", "150")
    monkeypatch.setenv("PCAL_SERVED_TASK_KIB", "4")
    bufs = _streams_on_device()
    fs, fc, fo, nbits, integ = STREAMS[0]
    spb = 8 // nbits
    want = _plain_integrations(bufs[0], fs, fc, fo, nbits, integ, 0)
    srv = pcal.PCalServer(mem_budget_bytes=1 << 30, max_streams=2, precision=0)
    sid = srv.open(fs, fc, fo, nbits, integ)
    srv.start(workgroups=64)
    got = {}
    for k in range(2):
        if k:
            time.sleep(1.0)  # every worker waits far past 150 ms; the heartbeat keeps them
        srv.submit([sid], [bufs[0].data_ptr() + k * integ // spb], [integ])
        t_end = time.time() + 30.0
        while (sid, k) not in got and time.time() < t_end:
            srv.step()
            for s_, k_ in srv.poll():
                got[(s_, k_)] = srv.spectrum(s_, k_)
        assert (sid, k) in got, "integration %d not reported" % k
    srv.stop()
    st = srv.loop_stats()
    say("loop counters: %s" % st)
    assert st["relaunches"] == 0 and st["tasks_run"] == st["tasks_published"] and st["finalizes"] == 2
    for k in range(2):
        assert_spectra(got[(sid, k)], want[k], amp_rtol=F64_RTOL, phase_atol=F64_RTOL,
                       what="integration %d after idle workers" % k)
    srv.close()
