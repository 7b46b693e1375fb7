"""Benchmark of the PCal extraction hot path on one MI355X.

A step is one whole integration of the 2-bit workload fs = 64 MHz,
f_comb = 1 MHz (N = 64 tones), f_offset = 10 kHz (rotator period 6400),
2^30 samples (256 MiB packed): the fused unpack-rotate-fold kernel with its
cross-workgroup reduction, the FP64 DFT/amplitude/phase/delay finalize
(which also clears the bins for the next integration), and the copy of the
results to pinned host memory.  Steps are enqueued back to back; latency
per integration is measured separately with synchronised calls.  Inputs are resident in
HBM before timing starts and rotate over four distinct 256 MiB buffers so
the 256 MB last-level cache cannot serve them.

Prints one JSON line (see the keys below).  ``--gpus N`` with N > 1 exits
with a message: the benchmark runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gsamples/s and % HBM peak, 2-bit fold @1e-4 rad; p99 latency per integration"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "fold2_64M_10k"
STAMPED_STEPS = 30  # kernel-stamped steps after the timed region (the kernel's duration)
# the fold kernel's source: its body (pcal_fold.h) and its kernels and launchers (pcal_kernels.hip)
KERNEL_SRCS = [os.path.join(ROOT, "paper_2501_05993_amd", "csrc", f) for f in ("pcal_fold.h", "pcal_kernels.hip")]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "fold_kernel_fold2_64M_10k_pmc.md")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic():
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it matches this kernel source."""
    try:
        with open(PMC_SUMMARY) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("|") and "=" not in line:
            continue
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(host_bytes, spec, target_s=12.0):
    """The FP64 oracle timed on this host on a bounded prefix of the same stream."""
    import oracle

    threads = oracle.max_threads()
    n1 = 1 << 23  # the same work on one core (run first: every call below sets its own thread count)
    t0 = time.perf_counter()
    oracle.correlate(host_bytes[: n1 // 4], 2, n1, spec.fs, spec.f_comb, spec.f_offset, nthreads=1)
    dt1 = time.perf_counter() - t0
    n = 1 << 20
    t0 = time.perf_counter()
    oracle.correlate(host_bytes[: n // 4], 2, n, spec.fs, spec.f_comb, spec.f_offset, nthreads=threads)
    dt = time.perf_counter() - t0
    n2 = int(min(len(host_bytes) * 4, max(n, n * target_s / max(dt, 1e-6))))
    n2 -= n2 % (1 << 20)
    t0 = time.perf_counter()
    oracle.correlate(host_bytes[: n2 // 4], 2, n2, spec.fs, spec.f_comb, spec.f_offset, nthreads=threads)
    dt2 = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(n2 / dt2 / 1e9, 6), "unit": "Gsamples/s", "cores": threads, "kind": "oracle",
            "sample": "first %d samples (2^%.1f) of the bench's 2-bit input buffers, all %d tones, FP64 "
                      "per-tone correlation, %.1f s" % (n2, np.log2(n2), spec.ntones, dt2),
            "one_core": {"value": round(n1 / dt1 / 1e9, 6), "sample": "first 2^23 samples, %.1f s" % dt1},
            "cpu_model": model, "cost": "N x L complex multiply-adds (N = %d tones)" % spec.ntones}


def cpu_baseline_configs(torch, synth, target_s=4.0):
    """The oracle on the host cores on the other single-stream, batched and served workloads, each on a
    bounded sample sized for about target_s of work: the small 2-bit f_offset = 0 stream in full, a prefix
    of the 8-bit wide stream, a prefix of every stream of the 64-stream batch and of 32 integrations of
    the serving mix."""
    import oracle

    threads = oracle.max_threads()
    out = {}

    def timed(packed, nbits, n, sp):
        t0 = time.perf_counter()
        oracle.correlate(packed, nbits, n, sp.fs, sp.f_comb, sp.f_offset, nthreads=threads)
        return time.perf_counter() - t0

    w = synth.WORKLOADS["small_2bit_fo0"]
    sp, L = w["spec"], w["nsamples"]
    packed = synth.make_stream(sp, L)
    dt = timed(packed, 2, L, sp)
    out["small_2bit_fo0"] = {"value": round(L / dt / 1e9, 6), "unit": "Gsamples/s",
                             "sample": "the whole stream: 2^24 samples, N = 32 tones, %.2f s" % dt}
    w = synth.WORKLOADS["wide8_1024M_510k"]
    sp = w["spec"]
    n = 1 << 20
    dev = synth.make_stream_device(sp, 1 << 26)
    host = dev.cpu().numpy()
    del dev
    dt = timed(host, 8, n, sp)
    n2 = int(min(1 << 26, max(n, n * target_s / max(dt, 1e-6)))) & ~((1 << 20) - 1)
    dt2 = timed(host, 8, n2, sp)
    out["wide8_1024M_510k"] = {"value": round(n2 / dt2 / 1e9, 6), "unit": "Gsamples/s",
                               "sample": "first %d samples (2^%.1f) of the 8-bit stream, N = 1024 tones, %.1f s; "
                                         "a prefix, not the 2^33-sample integration" % (n2, np.log2(n2), dt2)}
    specs = synth.batch_specs()
    per = 1 << 18
    packs = [synth.make_stream(s_, per) for s_ in specs]
    t0 = time.perf_counter()
    for s_, pk in zip(specs, packs):
        oracle.correlate(pk, 2, per, s_.fs, s_.f_comb, s_.f_offset, nthreads=threads)
    dt = time.perf_counter() - t0
    out["batch64"] = {"value": round(len(specs) * per / dt / 1e9, 6), "unit": "Gsamples/s",
                      "sample": "first 2^18 samples of each of the 64 streams (N = 16-512 tones), %.1f s" % dt}
    # the serving mix: 32 of its streams, stratified over (fs, sample width), one integration's first
    # 2^19 samples each
    served = synth.served_specs(256)
    classes = {}
    for s_ in served:
        classes.setdefault((s_.fs, s_.nbits), []).append(s_)
    keys = sorted(classes)
    pick = []
    while len(pick) < 32:
        for k in keys:
            if classes[k] and len(pick) < 32:
                pick.append(classes[k].pop(0))
    per = 1 << 19
    packs = [synth.make_stream(s_, per) for s_ in pick]
    t0 = time.perf_counter()
    for s_, pk in zip(pick, packs):
        oracle.correlate(pk, s_.nbits, per, s_.fs, s_.f_comb, s_.f_offset, nthreads=threads)
    dt = time.perf_counter() - t0
    out["served32"] = {"value": round(len(pick) * per / dt / 1e9, 6), "unit": "Gsamples/s",
                       "sample": "first 2^19 samples of one integration of 32 streams of the serving mix, "
                                 "stratified over (fs, sample width) (N = 32-512 tones), %.1f s; prefixes, not "
                                 "whole 1 s integrations" % dt}
    out["cores"] = threads
    return out


SERVED_POOL = 1 << 25  # samples of the pre-staged device pool per stream configuration (~0.8 GB in all)


def _served_setup(torch, synth, seconds):
    """Stream mix, arrival trace and device-resident chunk pools of the serving study."""
    specs = synth.served_specs(256)
    t, sid, ns = synth.served_trace(len(specs), seconds)
    pools = {}
    for sp in specs:
        key = (sp.fs, sp.f_offset, sp.nbits)
        if key not in pools:
            pools[key] = synth.make_stream_device(sp, SERVED_POOL)
    torch.cuda.synchronize()
    return specs, (t, sid, ns), pools


def _pieces(sp, pool, pos, n):
    """Device (address, samples) pieces of the stream samples [pos, pos + n), taken cyclically from the pool."""
    spb = 8 // sp.nbits
    out = []
    while n > 0:
        off = pos % SERVED_POOL
        take = min(n, SERVED_POOL - off)
        out.append((pool.data_ptr() + off // spb, take))
        pos += take
        n -= take
    return out


def served_run(pcal, torch, setup, mode, drain_s=5.0, flat_out=False, prec=None, workgroups=256):
    """Replay the arrival trace through the served form (mode "served": host-stepped; "resident": the
    device-resident loop of `workgroups` workgroups) or through plain per-chunk extraction ("plain"),
    all in precision form `prec` (default: mixed).

    Latency of an integration = host time its results are seen - arrival time of its last chunk.
    flat_out: every chunk is available at once (capacity: the sustained rate is the result; latencies
    then measure queueing and are not reported); the served forms then get all pieces in one submit,
    listed before the clock starts (the plain form's per-chunk calls are its own cost and stay timed).
    """
    from collections import deque

    specs, (t, sid, ns), pools = setup
    if prec is None:
        prec = pcal.PREC_MIXED
    if flat_out:
        t = np.zeros_like(t)
        drain_s = 120.0
    S = len(specs)
    pos = [0] * S
    last_arrival = {}
    lat = []
    done_samples = 0
    served = mode in ("served", "resident")
    queued = 0
    if served:
        srv = pcal.PCalServer(mem_budget_bytes=16 << 30, max_streams=S, precision=prec)
        ids = [srv.open(sp.fs, sp.f_comb, sp.f_offset, sp.nbits, sp.fs) for sp in specs]
        rev = {v: k for k, v in enumerate(ids)}
    else:
        K = 4
        hs = [pcal.PCal(sp.fs, sp.f_comb, sp.f_offset, sp.nbits, method=pcal.METHOD_PERIOD_FOLD, precision=prec)
              for sp in specs]
        streams = [torch.cuda.Stream() for _ in range(K)]
        slots = [torch.zeros((8, 4 * sp.ntones + 1), dtype=torch.float64, pin_memory=True) for sp in specs]
        in_integ = [0] * S
        integ_no = [0] * S
        pending = deque()
    torch.cuda.synchronize()
    # the host-step form launches on the caller's stream: named once here rather than looked up per step
    # (the device-resident loop runs on a stream of its own and takes none)
    step_stream = torch.cuda.current_stream() if mode == "served" else None
    n_arr = len(t)
    pre = None
    if flat_out and served:
        pre_s, pre_p, pre_n = [], [], []
        for a in range(n_arr):
            s_, n_ = int(sid[a]), int(ns[a])
            sp = specs[s_]
            p0 = pos[s_]
            for k in range(p0 // sp.fs, (p0 + n_) // sp.fs):
                last_arrival[(s_, k)] = 0.0
            for ptr, m in _pieces(sp, pools[(sp.fs, sp.f_offset, sp.nbits)], p0, n_):
                pre_s.append(ids[s_])
                pre_p.append(ptr)
                pre_n.append(m)
            pos[s_] += n_
        pre = (np.asarray(pre_s, dtype=np.int32), np.asarray(pre_p, dtype=np.uint64),
               np.asarray(pre_n, dtype=np.int64))
    if mode == "resident":  # after the device-wide synchronisation: that would wait for the persistent kernel
        srv.start(workgroups=workgroups)
    t0 = time.perf_counter()
    i = 0
    while True:
        now = time.perf_counter() - t0
        j = int(np.searchsorted(t, now, side="right"))
        if pre is not None and j > i:
            srv.submit(*pre)
            queued += int(pre[2].sum())
            i = j
        if j > i:
            sub_s, sub_p, sub_n = [], [], []
            for a in range(i, j):
                s_, n_ = int(sid[a]), int(ns[a])
                sp = specs[s_]
                p0 = pos[s_]
                for k in range(p0 // sp.fs, (p0 + n_) // sp.fs):
                    last_arrival[(s_, k)] = t[a]
                for ptr, m in _pieces(sp, pools[(sp.fs, sp.f_offset, sp.nbits)], p0, n_):
                    if served:
                        sub_s.append(ids[s_])
                        sub_p.append(ptr)
                        sub_n.append(m)
                    else:
                        h, st = hs[s_], streams[s_ % K]
                        spb = 8 // sp.nbits
                        while m > 0:
                            take = min(m, sp.fs - in_integ[s_])
                            h.extract(ptr, take, stream=st)
                            ptr += take // spb
                            m -= take
                            in_integ[s_] += take
                            if in_integ[s_] == sp.fs:
                                k = integ_no[s_]
                                h.results_async(slots[s_][k % 8], reset=True)
                                h.flush()  # finalize now, not with this stream's next chunk
                                ev = torch.cuda.Event()
                                ev.record(st)
                                pending.append((ev, s_, k))
                                integ_no[s_] += 1
                                in_integ[s_] = 0
                pos[s_] += n_
            if served:
                srv.submit(sub_s, np.asarray(sub_p, dtype=np.uint64), sub_n)
                queued += sum(sub_n)
            i = j
        if served:
            # step only with work queued: a piece held back (ring full, or its stream's previous
            # integration not yet reported) stays queued until a later step takes it
            if queued > 0:
                queued -= srv.step(step_stream)
            for sv, k in srv.poll():
                s_ = rev[sv]
                lat.append(time.perf_counter() - t0 - last_arrival[(s_, k)])
                done_samples += specs[s_].fs
            idle = False
            if i >= n_arr:  # every chunk submitted: has all of it been reported?
                st_ = srv.stats()
                idle = st_["queued_samples"] == 0 and st_["inflight_finalizes"] == 0
        else:
            while pending and pending[0][0].query():
                _, s_, k = pending.popleft()
                lat.append(time.perf_counter() - t0 - last_arrival[(s_, k)])
                done_samples += specs[s_].fs
            idle = not pending
        if i >= n_arr and (idle or now > t[-1] + drain_s):
            break
    wall = time.perf_counter() - t0
    loop = None
    if mode == "resident":
        srv.stop()
        loop = srv.loop_stats()
    torch.cuda.synchronize()
    if served:
        srv.close()
    else:
        for h in hs:
            h.close()
    offered = float(ns.sum())
    if flat_out:
        r = {"samples": offered, "sustained_gsps": round(offered / wall / 1e9, 1), "wall_s": round(wall, 3),
             "integrations": len(lat)}
        if loop:
            r["loop"] = loop
        return r
    r = {"integrations": len(lat),
            "latency_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 3) if lat else None,
            "latency_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 3) if lat else None,
            "sustained_gsps": round(offered / wall / 1e9, 2),
            "completed_integration_gsps": round(done_samples / wall / 1e9, 2),
            "wall_s": round(wall, 2)}
    if loop:
        r["loop"] = loop
    return r


def pipelined_steps(pcal, torch, bufs, spec, L, steps, warmup, check):
    """The headline's steps pipelined: one handle whose integrations end with the overlap reset
    (pcal_results_async with PCAL_RESET_OVERLAP) fed on two streams in turn, so consecutive
    integrations run side by side (each lane's finalize inside its own next fold).  Same work per
    step as the headline (2^30 samples, fold + FP64 finalize + results to pinned host memory); the
    last integration checked against the oracle on two tones."""
    N = spec.ntones
    h = pcal.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ring = torch.zeros((8, 4 * N + 1), dtype=torch.float64, pin_memory=True)

    def step(i):
        h.extract(bufs[i % 4], L, stream=streams[i % 2])
        h.results_async(ring[i % 8], reset=pcal.RESET_OVERLAP)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, warmup + steps):
        step(i)
    h.flush()  # both lanes' last finalizes
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    out = {"streams": 2, "ms_per_step": round(ms, 5), "gsamples_per_s": round(L / (ms * 1e-3) / 1e9, 1),
           "hbm_frac_per_step": round(L * spec.nbits / 8 / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
           "note": "the headline's steps with pcal_results_async(PCAL_RESET_OVERLAP) on two streams in turn "
                   "(two lanes of one handle); per-step figure: two fold kernels overlap, so no per-kernel "
                   "roofline applies"}
    if check:
        import oracle

        k = warmup + steps - 1
        last = ring[k % 8].numpy().copy()
        C = last[2 * N:3 * N] + 1j * last[3 * N:4 * N]
        tones = [1, 31]
        Co = oracle.correlate(bufs[k % 4].cpu().numpy(), spec.nbits, L, spec.fs, spec.f_comb, spec.f_offset,
                              n0=k * L, tones=tones)
        out["accuracy_vs_oracle"] = {
            "tones": tones,
            "amp_rel_err_max": float(np.max(np.abs(np.abs(C[tones]) - np.abs(Co)) / np.abs(Co))),
            "phase_err_rad_max": float(np.max(np.abs(np.angle(C[tones] * np.conj(Co))))),
        }
    h.close()
    return out


def precision_report(pcal, torch, synth, oracle=None):
    """Config-4 precision study: 64 streams (fs 16-512 MHz, f_offset 0-510 kHz, 2-bit, 2^26 samples each)
    through the batched form in each precision form -- mixed (two-term FP16 table, Kahan FP32, FP64
    reduce/DFT), all-FP32, and the literal single-FP16 mixed variant -- against the FP64 form, per stream;
    the FP64 form itself against the FP64 oracle on two tones per stream."""
    specs = synth.batch_specs()
    L = 1 << 26
    print("[bench] precision study: 64 streams x 2^26 samples in 4 precision forms", file=sys.stderr, flush=True)
    devs = [synth.make_stream_device(sp, L) for sp in specs]
    torch.cuda.synchronize()
    forms = (("f64", pcal.PREC_F64), ("mixed", pcal.PREC_MIXED), ("f32", pcal.PREC_F32),
             ("f16_single", pcal.PREC_F16))
    res = {}
    for name, prec in forms:
        b = pcal.PCalBatch(len(specs), precision=prec)
        ids = [b.add(sp.fs, sp.f_comb, sp.f_offset, 2) for sp in specs]
        b.extract(ids, devs, [L] * len(ids))
        C = b.spectra(ids)
        b.reset(ids)
        b.extract(ids, devs, [L] * len(ids))
        amp, ph, d = b.results(ids)
        K = 5
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            b.reset(ids)
            b.extract(ids, devs, [L] * len(ids))
            b.results(ids)
        dt = (time.perf_counter() - t0) / K
        res[name] = (C, d, dt)
        b.close()
    C64, d64, t64 = res["f64"]
    out = {"workload": "64 streams, fs 16-512 MHz, f_offset {0,10,250,510} kHz, 2-bit, 2^26 samples each",
           "streams": [[sp.fs // 1_000_000, sp.f_offset] for sp in specs],
           "stream_key": "[fs MHz, f_offset Hz] per stream, in the order of the per-stream lists",
           "bar": {"amp_rel": 1e-5, "phase_rad": 1e-4},
           "batched_step_ms": {"f64": round(t64 * 1e3, 3)}}
    if oracle is not None:
        errs = []
        for sp, dv, c64 in zip(specs, devs, C64):
            tones = [1, sp.ntones // 3]
            Co = oracle.correlate(dv.cpu().numpy(), 2, L, sp.fs, sp.f_comb, sp.f_offset, tones=tones)
            errs.append(float(np.abs(c64[tones] - Co).max() / np.abs(Co).max()))
        out["f64_vs_oracle"] = {"rel_err_max": max(errs), "tones": "1 and N/3 of every stream"}
    for name, _ in forms[1:]:
        C, d, dt = res[name]
        amp_e, ph_e = [], []
        for c, c64 in zip(C, C64):
            strong = np.abs(c64) >= 1e-5 * np.abs(c64).max()
            amp_e.append(float(np.max(np.abs(np.abs(c[strong]) - np.abs(c64[strong])) / np.abs(c64[strong]))))
            ph_e.append(float(np.max(np.abs(np.angle(c[strong] * np.conj(c64[strong]))))))
        del_e = np.abs(np.asarray(d) - np.asarray(d64))
        out[name] = {"amp_rel_err_max": max(amp_e), "amp_rel_err_median": float(np.median(amp_e)),
                     "phase_err_rad_max": max(ph_e), "phase_err_rad_median": float(np.median(ph_e)),
                     "delay_err_s_max": float(del_e.max()), "delay_err_s_median": float(np.median(del_e)),
                     "streams_within_bar": int(sum(a <= 1e-5 and p <= 1e-4 for a, p in zip(amp_e, ph_e))),
                     "per_stream": {"amp_rel_err": [float("%.3g" % a) for a in amp_e],
                                    "phase_err_rad": [float("%.3g" % p) for p in ph_e],
                                    "delay_err_s": [float("%.3g" % x) for x in del_e]}}
        out["batched_step_ms"][name] = round(dt * 1e3, 3)
    del devs
    torch.cuda.empty_cache()
    return out


READ_PROBE_SHAPES = ((1024, 256), (1024, 512), (2048, 256), (512, 1024))


def read_ceiling(pcal, torch, bufs, launches=20):
    """Measured streaming-read ceiling: pcal_read_probe (16-byte non-temporal loads, nothing else) over the
    same input buffers as the fold, stamped like the fold's launches; the fastest of a few launch shapes."""
    nbytes = bufs[0].numel()
    stream = torch.cuda.current_stream()
    out = torch.empty(max(b * t // 64 for b, t in READ_PROBE_SHAPES), dtype=torch.int64, device="cuda")
    best = None
    for blocks, threads in READ_PROBE_SHAPES:
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(launches)]
        for a, b in evs:
            a.record(stream)
            b.record(stream)
        for i in range(4):
            pcal.read_probe(bufs[i % len(bufs)], out, blocks, threads)
        for i, ev in enumerate(evs):
            pcal.read_probe(bufs[i % len(bufs)], out, blocks, threads, events=ev)
        torch.cuda.synchronize()
        us = float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e3
        if best is None or us < best[0]:
            best = (us, blocks, threads)
    us, blocks, threads = best
    gbs = nbytes / (us * 1e-6) / 1e9
    return {"kernel": "read_probe_kernel", "bytes_per_launch": nbytes, "avg_us": round(us, 2),
            "achieved": round(gbs, 1), "unit": "GB/s", "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "launch": "%d x %d threads" % (blocks, threads),
            "note": "one pass of 16-byte non-temporal loads over the same buffers, fastest of %d launch shapes"
                    % len(READ_PROBE_SHAPES)}


def batched_study(pcal, torch, synth):
    """Batched form on the 64-stream mix (fs 16-512 MHz, f_offset {0,10,250,510} kHz, 2-bit, 2^26 samples
    each: 1 GiB): one batched fold call (one launch per sample width over the work-list of all 64 streams,
    the work-list copy included) timed back to back with events, with its HBM roofline fraction (0.25 B per
    sample read once); and one synchronised integration of all 64 streams (reset, batched fold, batched
    finalize, results) against one handle per stream doing the same one stream after another."""
    specs = synth.batch_specs()
    L = 1 << 26
    print("[bench] batched study: 64 streams x 2^26 2-bit samples", file=sys.stderr, flush=True)
    devs = [synth.make_stream_device(sp, L) for sp in specs]
    torch.cuda.synchronize()
    nbytes = len(specs) * L // 4
    stream = torch.cuda.current_stream()
    b = pcal.PCalBatch(len(specs))
    ids = [b.add(sp.fs, sp.f_comb, sp.f_offset, 2) for sp in specs]
    ns = [L] * len(ids)
    for _ in range(3):
        b.extract(ids, devs, ns)
    torch.cuda.synchronize()
    K = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(K):
        b.extract(ids, devs, ns)
    e1.record(stream)
    torch.cuda.synchronize()
    t_fold = e0.elapsed_time(e1) * 1e-3 / K
    integ = []
    for _ in range(10):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        b.reset(ids)
        b.extract(ids, devs, ns)
        b.results(ids)
        integ.append(time.perf_counter() - ts)
    b.close()
    hs = [pcal.PCal(sp.fs, sp.f_comb, sp.f_offset, 2) for sp in specs]
    for h, d in zip(hs, devs):
        h.extract(d, L)
        h.results()
    single = []
    for _ in range(5):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for h, d in zip(hs, devs):
            h.reset()
            h.extract(d, L)
            h.results()
        single.append(time.perf_counter() - ts)
    for h in hs:
        h.close()
    del devs
    torch.cuda.empty_cache()
    gbs = nbytes / t_fold / 1e9
    return {"workload": "64 streams, fs 16-512 MHz, f_offset {0,10,250,510} kHz, 2-bit, 2^26 samples each",
            "fold_call_us": round(t_fold * 1e6, 1),
            "gsamples_per_s": round(len(specs) * L / t_fold / 1e9, 1),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "kernel": "fold_batch_kernel<2,0>",
                         "algorithmic_bytes_per_call": nbytes},
            "integration_ms_p50": round(float(np.median(integ)) * 1e3, 3),
            "one_handle_per_stream_integration_ms_p50": round(float(np.median(single)) * 1e3, 3)}


def precision_single(pcal, torch, synth):
    """Precision of the mixed and all-FP32 forms against the FP64 form on the single-stream workloads: the
    2-bit fs 64 MHz / 10 kHz stream (2^30 samples, one launch) and the 8-bit fs 1024 MHz / 510 kHz stream
    (2^33 samples in 2^28-sample launches, the global index running on), period fold."""
    out = {}
    for name in ("fold2_64M_10k", "wide8_1024M_510k"):
        w = synth.WORKLOADS[name]
        spec, L = w["spec"], w["nsamples"]
        chunk = w.get("chunk", L)
        print("[bench] precision study: %s" % name, file=sys.stderr, flush=True)
        buf = synth.make_stream_device(spec, L)
        torch.cuda.synchronize()
        res = {}
        for prec in (pcal.PREC_F64, pcal.PREC_MIXED, pcal.PREC_F32):
            with pcal.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits, precision=prec) as h:
                for k in range(L // chunk):
                    h.extract(buf, chunk, byte_offset=k * chunk * spec.nbits // 8)
                C = h.spectrum()
                _, _, d = h.results()
            res[prec] = (C, d)
        del buf
        torch.cuda.empty_cache()
        C64, d64 = res[pcal.PREC_F64]
        strong = np.abs(C64) >= 1e-5 * np.abs(C64).max()
        entry = {}
        for label, prec in (("mixed", pcal.PREC_MIXED), ("f32", pcal.PREC_F32)):
            C, d = res[prec]
            entry[label] = {
                "amp_rel_err_max": float(np.max(np.abs(np.abs(C[strong]) - np.abs(C64[strong])) / np.abs(C64[strong]))),
                "phase_err_rad_max": float(np.max(np.abs(np.angle(C[strong] * np.conj(C64[strong]))))),
                "delay_err_s": float(abs(d - d64))}
        out[name] = entry
    return out


def per_sample_2bit_study(pcal, torch, synth, oracle=None):
    """2-bit stream with a long rotator period (fs = 64 MHz, f_offset = 10008 Hz: the rotator repeats only
    after 8e6 samples, near the longest fold period AUTO folds): one 2^30-sample integration through AUTO's
    choice (the period fold) and the per-sample forms, timed with events, HBM roofline at 0.25 B per
    sample, and each form's spectrum against the oracle on two tones."""
    w = synth.WORKLOADS["osc2_64M_10008"]
    spec, L = w["spec"], w["nsamples"]
    print("[bench] per-sample 2-bit study (f_offset 10008 Hz)", file=sys.stderr, flush=True)
    buf = synth.make_stream_device(spec, L)
    torch.cuda.synchronize()
    tones = [1, 21]
    Co = None
    if oracle is not None:
        Co = oracle.correlate(buf.cpu().numpy(), 2, L, spec.fs, spec.f_comb, spec.f_offset, tones=tones)
    stream = torch.cuda.current_stream()
    forms = (("auto_f64", pcal.METHOD_AUTO, pcal.PREC_F64), ("recurrence_f64", pcal.METHOD_OSC, pcal.PREC_F64),
             ("recurrence_mixed", pcal.METHOD_OSC, pcal.PREC_MIXED),
             ("coupled_form_mixed", pcal.METHOD_CFO, pcal.PREC_MIXED), ("recurrence_f32", pcal.METHOD_OSC,
                                                                         pcal.PREC_F32))
    out = {}
    for name, method, prec in forms:
        h = pcal.PCal(spec.fs, spec.f_comb, spec.f_offset, 2, method=method, precision=prec)
        chosen = h.info()["method"]
        h.extract(buf, L)  # the integration compared with the oracle (global index from 0)
        C = h.spectrum()
        K = 5
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        for a, b in evs:
            a.record(stream)
            b.record(stream)
        for k in range(K):
            h.extract(buf, L, events=evs[k])
        torch.cuda.synchronize()
        us = float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e3
        h.close()
        gbs = L / 4 / (us * 1e-6) / 1e9
        entry = {"method": {1: "period_fold", 2: "table", 3: "recurrence", 4: "coupled_form", 5: "magic_circle",
                            6: "error_feedback_dfr"}[chosen],
                 "kernel_us": round(us, 1), "gsamples_per_s": round(L / (us * 1e-6) / 1e9, 1),
                 "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(gbs / HBM_PEAK_GBS, 4)}}
        if Co is not None:
            entry["vs_oracle"] = {
                "tones": tones,
                "amp_rel_err_max": float(np.max(np.abs(np.abs(C[tones]) - np.abs(Co)) / np.abs(Co))),
                "phase_err_rad_max": float(np.max(np.abs(np.angle(C[tones] * np.conj(Co)))))}
        out[name] = entry
    del buf
    torch.cuda.empty_cache()
    return {"workload": "2-bit, fs 64 MHz, f_comb 1 MHz (N = 64), f_offset 10008 Hz (rotator period 8e6 = the "
                        "fold period), 2^30 samples, one launch per form (kernel-stamped); AUTO folds",
            **out}


def rotator_study(pcal, torch, synth):
    """8-bit wide workload (fs = 1024 MHz, f_offset = 510 kHz, N = 1024, rotator period 102400): one
    integration of 2^33 samples streamed in 2^28-sample chunks (the global sample index runs on across
    chunks) through each rotator form -- the period fold (FP64 rotation, and the fixed-point Q17 rotator),
    the per-sample rotator table, the direct-form resonator (Eq. 7), the coupled-form and magic-circle
    oscillators and the resonator with error feedback, in the FP64 and mixed precision forms -- timed with
    events around the 32 launches, with each form's HBM roofline fraction (1 B per sample read once) and its
    spectrum's spread against the FP64 period fold's (tones with signal)."""
    w = synth.WORKLOADS["wide8_1024M_510k"]
    spec, L, chunk = w["spec"], w["nsamples"], w["chunk"]
    print("[bench] rotator study: generating %d GiB of 8-bit samples" % (L >> 30), file=sys.stderr, flush=True)
    buf = synth.make_stream_device(spec, L)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    P64, PMX = pcal.PREC_F64, pcal.PREC_MIXED
    forms = (("period_fold", pcal.METHOD_PERIOD_FOLD, P64), ("period_fold_q17", pcal.METHOD_PERIOD_FOLD, pcal.PREC_Q17),
             ("table", pcal.METHOD_LUT, P64), ("table_mixed", pcal.METHOD_LUT, PMX),
             ("recurrence", pcal.METHOD_OSC, P64), ("recurrence_mixed", pcal.METHOD_OSC, PMX),
             ("coupled_form", pcal.METHOD_CFO, P64), ("coupled_form_mixed", pcal.METHOD_CFO, PMX),
             ("magic_circle_mixed", pcal.METHOD_MCO, PMX), ("error_feedback_dfr_mixed", pcal.METHOD_DFR_EF, PMX))
    out, spectra = {}, {}
    for name, method, prec in forms:
        h = pcal.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits, method=method, precision=prec)
        h.extract(buf, chunk)  # warm-up chunk, then a fresh integration (global index continues)
        torch.cuda.synchronize()
        h.reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(L // chunk):
            h.extract(buf, chunk, byte_offset=k * chunk)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        spectra[name] = h.spectrum()
        gbs = L / t / 1e9  # 1 B per sample
        out[name] = {"ms_per_integration": round(t * 1e3, 3), "gsamples_per_s": round(L / t / 1e9, 1),
                     "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(gbs / HBM_PEAK_GBS, 4)}}
        h.close()
    ref = spectra["period_fold"]
    strong = np.abs(ref) >= 1e-3 * np.abs(ref).max()
    for name, _, _ in forms[1:]:
        c = spectra[name]
        out[name]["vs_period_fold"] = {
            "amp_rel_err_max": float(np.max(np.abs(np.abs(c[strong]) - np.abs(ref[strong])) / np.abs(ref[strong]))),
            "phase_err_rad_max": float(np.max(np.abs(np.angle(c[strong] * np.conj(ref[strong]))))),
        }
    del buf
    torch.cuda.empty_cache()
    return {"workload": "8-bit, fs 1024 MHz, f_comb 1 MHz (N = 1024), f_offset 510 kHz, 2^33 samples in "
                        "2^28-sample chunks, one integration per form", **out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--precision-report", action="store_true",
                    help="only run the 64-stream precision study (mixed and FP32 forms against FP64)")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the 64-stream per-stream precision report of the precision forms")
    ap.add_argument("--no-per-sample-study", action="store_true",
                    help="skip the 2-bit long-period (f_offset 10008 Hz) study of AUTO and the per-sample forms")
    ap.add_argument("--no-batched-study", action="store_true",
                    help="skip the 64-stream batched-form measurement")
    ap.add_argument("--no-pipelined", action="store_true",
                    help="skip the pipelined (two-stream) run of the headline's steps")
    ap.add_argument("--no-rotator-study", action="store_true",
                    help="skip the 8-bit wide-workload comparison of the rotator forms")
    ap.add_argument("--served-seconds", type=float, default=30.0,
                    help="length of the serving-study arrival trace (0: skip the serving study)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 256 MiB (10 times): the known-size reference that "
                         "scales rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the extraction of one stream does not span GPUs, and more than "
              "one is not supported", file=sys.stderr)
        sys.exit(2)

    global np
    import numpy as np
    import torch

    import synth
    from paper_2501_05993_amd import pcal

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 256 << 20, "copies": 10}), flush=True)
        return
    if args.precision_report:
        import oracle

        print(json.dumps({"precision_report": precision_report(pcal, torch, synth, oracle),
                          "precision_single_stream": precision_single(pcal, torch, synth)}), flush=True)
        return
    w = synth.WORKLOADS[WORKLOAD]
    spec, L = w["spec"], w["nsamples"]
    nbytes = L * spec.nbits // 8
    print("[bench] generating 4 x %d MiB input buffers" % (nbytes >> 20), file=sys.stderr, flush=True)
    bufs = []
    for i in range(4):
        s = synth.CombSpec(spec.fs, spec.f_comb, spec.f_offset, spec.nbits, amp=spec.amp, t_d=spec.t_d,
                           sigma=spec.sigma, jitter=spec.jitter, seed=tuple(spec.seed) + (i,))
        bufs.append(synth.make_stream_device(s, L))
    torch.cuda.synchronize()

    h = pcal.PCal(spec.fs, spec.f_comb, spec.f_offset, spec.nbits)
    stream = torch.cuda.current_stream()
    N = spec.ntones
    ring = torch.zeros((8, 4 * N + 1), dtype=torch.float64, pin_memory=True)

    # One step = one integration: fused unpack-rotate-fold over the 2^30 samples,
    # then the FP64 finalize (DFT, amplitude, phase, delay) which also clears the
    # bins for the next integration, and the copy of the results to pinned host
    # memory.  Steps are enqueued back to back (no host round trip per step).
    # The kernel's own duration comes from events that hipExtLaunchKernel stamps
    # at the fold kernel's start and end (pcal_extract_timed): no launch gaps.
    def step(i, ev=None):
        h.extract(bufs[i % 4], L, events=ev)
        h.results_async(ring[i % 8], reset=True)

    h.reset()
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    h.flush()  # the last integration's finalize, enqueued now (no later fold to carry it)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    last = ring[(args.steps - 1) % 8].numpy().copy()
    n_last = h.info()["samples_total"] - L   # global index of the last integration's first sample
    # The kernel's own duration: a separate pass of the same steps after the
    # timed region, every fold launch stamped at its start and end (a stamped
    # launch costs the stream a few us more, so none is taken inside the timed
    # region).
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(STAMPED_STEPS)]
    for a, b in evs:  # torch creates an event at its first record
        a.record(stream)
        b.record(stream)
    for i, ev in enumerate(evs):
        step(args.steps + i, ev)
    h.sync()
    torch.cuda.synchronize()
    kern_ms = [a.elapsed_time(b) for a, b in evs]

    # Latency per integration: extract then results, synchronised, one at a time.
    h.reset()
    lat = []
    for i in range(max(20, min(args.steps, 50))):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        h.extract(bufs[i % 4], L)
        h.results()
        lat.append(time.perf_counter() - ts)
        h.reset()

    pipelined = None if args.no_pipelined else pipelined_steps(pcal, torch, bufs, spec, L, args.steps, args.warmup,
                                                               not args.no_accuracy)
    ceiling = read_ceiling(pcal, torch, bufs)
    ms_per_step = elapsed * 1e3 / args.steps
    value = L / (ms_per_step * 1e-3) / 1e9
    kavg_s = float(np.mean(kern_ms)) * 1e-3
    achieved = nbytes / kavg_s / 1e9
    traffic = pmc_traffic()
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u2->i32 fold, f64 rotate/DFT", "data": "synthetic",
        "config": {"workload": WORKLOAD, "fs_hz": spec.fs, "f_comb_hz": spec.f_comb,
                   "f_offset_hz": spec.f_offset, "nbits": spec.nbits, "nsamples": L, "ntones": spec.ntones,
                   "rotator_period": 6400, "input_buffers": 4, "method": "period_fold", "precision": "f64"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "fold_kernel<2,0>",
                     "kernel_note": "each launch also runs the previous integration's finalize in 1 of its "
                                    "256 workgroups (pcal_results_async with reset defers it into the next fold)",
                     "kernel_avg_us": round(kavg_s * 1e6, 2),
                     "kernel_stamped_launches": len(kern_ms),
                     "kernel_us_p10_p50_p90": [round(float(np.percentile(kern_ms, q)) * 1e3, 2) for q in (10, 50, 90)],
                     "read_ceiling": ceiling,
                     "frac_of_read_ceiling": round(achieved / ceiling["achieved"], 4),
                     "algorithmic_bytes_per_launch": nbytes},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 4),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 4),
                       "per": "integration of 2^30 samples, extract + results, synchronised"},
    }
    if pipelined:
        out["pipelined"] = pipelined
    if not args.no_accuracy:
        import oracle

        C = last[2 * N:3 * N] + 1j * last[3 * N:4 * N]
        host = bufs[(args.steps - 1) % 4].cpu().numpy()
        tones = [1, 31]
        Co = oracle.correlate(host, 2, L, spec.fs, spec.f_comb, spec.f_offset, n0=n_last, tones=tones)
        out["accuracy_vs_oracle"] = {
            "tones": tones,
            "amp_rel_err_max": float(np.max(np.abs(np.abs(C[tones]) - np.abs(Co)) / np.abs(Co))),
            "phase_err_rad_max": float(np.max(np.abs(np.angle(C[tones] * np.conj(Co))))),
        }
    if not args.no_cpu_baseline:
        # two of the input buffers back to back: room for ~12 s of oracle work
        host = torch.cat([bufs[0], bufs[1]]).cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(host, spec)
    h.close()
    bufs.clear()
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"]["other_workloads"] = cpu_baseline_configs(torch, synth)
    if not args.no_precision:
        import oracle

        out["precision"] = precision_report(pcal, torch, synth, oracle)
    if not args.no_per_sample_study:
        import oracle

        out["per_sample_2bit"] = per_sample_2bit_study(pcal, torch, synth, oracle)
    if not args.no_batched_study:
        out["batched"] = batched_study(pcal, torch, synth)
    if not args.no_rotator_study:
        out["rotator_study"] = rotator_study(pcal, torch, synth)
    if args.served_seconds > 0:
        print("[bench] serving study: %.0f s trace, 256 streams" % args.served_seconds, file=sys.stderr, flush=True)
        setup = _served_setup(torch, synth, args.served_seconds)
        pool_bytes = sum(int(v.numel()) for v in setup[2].values())
        resident = served_run(pcal, torch, setup, "resident")
        print("[bench] device-resident served form done", file=sys.stderr, flush=True)
        served = served_run(pcal, torch, setup, "served")
        print("[bench] host-step served form done", file=sys.stderr, flush=True)
        plain = served_run(pcal, torch, setup, "plain")
        print("[bench] serving capacity: the same trace with every chunk available at once",
              file=sys.stderr, flush=True)
        cap_res = served_run(pcal, torch, setup, "resident", flat_out=True)
        cap_served = served_run(pcal, torch, setup, "served", flat_out=True)
        cap_plain = served_run(pcal, torch, setup, "plain", flat_out=True)
        # bytes per sample of the mix (2-bit 0.25 B, 8-bit 1 B), for the HBM fraction of the capacity
        specs, (tt, sid_, ns_), _ = setup
        bps = float(np.sum(ns_ * np.array([specs[int(k)].nbits / 8.0 for k in sid_])) / np.sum(ns_))
        for c in (cap_res, cap_served, cap_plain):
            c["hbm_frac"] = round(c["sustained_gsps"] * 1e9 * bps / (HBM_PEAK_GBS * 1e9), 4)
        out["served"] = {"workload": "256 streams (2-/8-bit, fs 32-512 MHz, f_offset 0-510 kHz), Poisson "
                                     "chunks of 2^20-2^24 samples at 200 Gsamples/s offered, 1 s integrations, "
                                     "%.0f s trace, mixed precision form; chunks drawn from device pools of "
                                     "%.0f MB in all" % (args.served_seconds, pool_bytes / 1e6),
                         "resident": resident, "served": served, "plain_per_chunk": plain,
                         "notes": "resident: one persistent kernel of 256 workgroups fed through a work ring; "
                                  "served: host-stepped batched launches; plain: one pcal_extract per chunk "
                                  "on 4 HIP streams",
                         "capacity": {"note": "the same trace with every chunk available at once; sustained "
                                              "Gsamples/s until every integration's results are in; "
                                              "hbm_frac at %.3f B per sample" % bps,
                                      "resident": cap_res, "served": cap_served, "plain_per_chunk": cap_plain}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
