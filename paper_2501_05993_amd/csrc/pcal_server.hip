// Served form of libpcal: many live streams under one device-memory budget,
// continuously batched.  Chunks queue per stream on the host.  In the
// host-step form every step folds the oldest queued piece of each stream with
// one launch of the batched fused kernel, and finalizes (reads and clears)
// with one batched launch every stream whose integration that step completed.
// In the device-resident form (pcal_server_start) one persistent kernel runs
// the loop: a step only publishes the queued pieces as descriptors in a work
// ring in coherent host memory, the kernel's workgroups claim them, fold them
// into the streams' accumulator banks and finalize each integration as its
// last task ends, and report it in a completion ring.  Results reach pinned
// host memory asynchronously and are picked up by polling.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <new>
#include <vector>

#include "pcal_host.h"

using namespace pcal;
using namespace pcal::host;

namespace {

constexpr int kResultDepth = 8;  // integrations kept per stream for pcal_server_result

struct Piece {
    const uint8_t *ptr;
    int64_t n;  // samples
};

struct SrvStream {
    bool open = false;
    int bid = -1;                    // member id in the batch
    int spb = 4;                     // samples per byte
    int N = 0;
    int64_t integ_samples = 0;       // samples per integration
    int64_t integ = 0;               // index of the integration being accumulated
    int64_t in_integ = 0;            // its samples dispatched so far
    int64_t device_bytes = 0;
    std::deque<Piece> queue;
    int64_t queued = 0;              // samples in queue
    double *slots = nullptr;         // pinned [kResultDepth][4N + 1]
    double *slots_dev = nullptr;     // the same memory's device address (the finalize writes it)
    int64_t slot_integ[kResultDepth];  // integration held by each slot (-1: none)
    bool slot_ready[kResultDepth];
    // device-resident form
    int64_t integ_tasks = 0;         // fold tasks published in the current integration
    bool fin_inflight = false;       // an integration's last chunk is published, its completion not yet seen
};

struct Done {
    int sid;
    int64_t integ;
};

struct Inflight {
    hipEvent_t ev;
    std::vector<Done> items;
    size_t next = 0;  // items already reported
};

}  // namespace

struct pcal_server_ctx {
    pcal_batch_t batch = nullptr;
    int64_t budget = 0;
    int64_t used = 0;
    int prec = PCAL_PREC_F64;
    int max_streams = 0;
    std::vector<SrvStream> streams;
    std::deque<Inflight> inflight;
    std::vector<hipEvent_t> spare_events;
    // scratch of one step
    std::vector<int> ids, done_bids;
    std::vector<double *> done_outs;
    std::vector<const void *> ptrs;
    std::vector<int64_t> ns;
    std::vector<Done> done;
    int rr = 0;  // first stream served next step (round robin)
    // device-resident loop (pcal_server_start)
    bool resident = false;
    hipStream_t rstream = nullptr;
    int rgrid = 0, tasks = 0, cap = 0, done_cap = 0;
    int64_t task_bytes = 0;   // chunk bytes per fold task
    int64_t backlog_task_bytes = 0;  // the same under a backlog of backlog_chunks chunks
    int backlog_chunks = 0;
    size_t mail_bytes = 0;    // both mailbox arrays (cleared before a relaunch)
    unsigned long long tasks_published = 0;  // fold tasks of the chunks published
    hipStream_t sstream = nullptr;           // reads of the loop counters while the kernel runs
    unsigned long long last_stat[kServedStats] = {};  // the loop counters at the last stop
    bool have_stat = false;
    ServedDesc *ring = nullptr;              // coherent host memory, written by the host
    unsigned long long *slot_free = nullptr;  // coherent host memory, written by the device
    ServedDone *dn = nullptr;
    int *ctl = nullptr;                      // [0] quit, [1] workgroups that left, [2] 1 if they left when idle
    unsigned long long *pub = nullptr;       // tasks published (coherent host memory, read by the device)
    int relaunches = 0;                      // kernels launched again after every workgroup had left
    ServedArgs args{};
    void *dmem = nullptr;                    // device counters
    unsigned long long published = 0;        // chunks published
    unsigned long long done_next = 0;        // next completion record to read
    std::deque<Done> ready;                  // completions read while waiting, not yet polled
};

namespace {

int take_event(pcal_server_ctx *s, hipEvent_t *ev) {
    if (!s->spare_events.empty()) {
        *ev = s->spare_events.back();
        s->spare_events.pop_back();
        return PCAL_OK;
    }
    PCAL_HIP(hipEventCreateWithFlags(ev, hipEventDisableTiming));
    return PCAL_OK;
}

bool valid_sid(const pcal_server_ctx *s, int sid) {
    return sid >= 0 && sid < static_cast<int>(s->streams.size()) && s->streams[sid].open;
}

constexpr int kRingSlots = 512;        // chunks in the work ring
constexpr int kDoneSlots = 4096;       // completion records
constexpr int kTasksPerChunk = 32;     // largest number of fold tasks per chunk (PCAL_SERVED_TASKS)
static_assert(kRingSlots <= kServedMaxRing, "the scheduler looks ahead over the whole ring");
// Time without work before the loop leaves (PCAL_SERVED_IDLE_MS), so that the
// kernel ends even if the host never sets quit (the host launches it again
// when work comes: keep_alive); a waiting worker leaves on its own only once
// the scheduler's heartbeat has stood still for kWorkerSeconds
// (PCAL_SERVED_WORKER_MS): the scheduler always tells it to leave first.
constexpr int kIdleMs = 4000;
constexpr double kWorkerSeconds = 60.0;  // a frozen scheduler heartbeat for this long: a waiting worker leaves
constexpr double kQuitSeconds = 1.0;     // after quit, the scheduler waits this long for pending work
// Bytes of a chunk per fold task of the resident loop (PCAL_SERVED_TASK_KIB):
// a chunk gets ceil(bytes / this) tasks, at least its column tiles, at most
// the tasks per chunk.
constexpr int kTaskKib = 128;
// Under a backlog -- the chunk published kBacklogChunks chunks before this one
// has not ended (PCAL_SERVED_BACKLOG) -- every worker is busy and a new chunk
// waits for its turn anyway: its tasks then take kBacklogTaskKib of the chunk
// each (PCAL_SERVED_BACKLOG_TASK_KIB), fewer hand-outs for the scheduler at no
// cost in latency.
constexpr int kBacklogChunks = 32;
constexpr int kBacklogTaskKib = 2048;

template <class T>
int coherent_alloc(T **host, size_t count) {
    const hipError_t e = hipHostMalloc(reinterpret_cast<void **>(host), sizeof(T) * count,
                                       hipHostMallocCoherent | hipHostMallocMapped);
    if (e != hipSuccess) {
        set_error("hipHostMalloc(coherent)", e);
        *host = nullptr;
        return e == hipErrorOutOfMemory ? PCAL_ENOMEM : PCAL_EHIP;
    }
    memset(*host, 0, sizeof(T) * count);
    return PCAL_OK;
}

template <class T>
int device_address(T *host, T **dev) {
    const hipError_t e = hipHostGetDevicePointer(reinterpret_cast<void **>(dev), host, 0);
    if (e != hipSuccess) {
        set_error("hipHostGetDevicePointer", e);
        return PCAL_EHIP;
    }
    return PCAL_OK;
}

// Resident form: move finished integrations from the completion ring to `ready`.
void drain_done(pcal_server_ctx *s) {
    for (;;) {
        ServedDone *r = s->dn + s->done_next % static_cast<unsigned>(s->done_cap);
        if (__atomic_load_n(&r->seq, __ATOMIC_ACQUIRE) != s->done_next + 1) return;
        const Done d{r->sid, r->integ};
        s->done_next += 1;
        if (valid_sid(s, d.sid)) {
            SrvStream &st = s->streams[d.sid];
            const int k = static_cast<int>(d.integ % kResultDepth);
            if (st.slot_integ[k] == d.integ) st.slot_ready[k] = true;
            st.fin_inflight = false;
        }
        s->ready.push_back(d);
    }
}

// Resident form: when every workgroup of the loop has left (they leave
// together, about 4 s after the last work), launch it again with clear
// mailboxes; the loop leaves only with every handed-out task ended, and the
// next chunk to hand out is kept in device memory, so the new launch continues
// where the old one stopped.
int keep_alive(pcal_server_ctx *s) {
    if (__atomic_load_n(s->ctl + 1, __ATOMIC_ACQUIRE) < s->rgrid) return PCAL_OK;
    PCAL_HIP(hipStreamSynchronize(s->rstream));
    __atomic_store_n(s->ctl + 1, 0, __ATOMIC_RELAXED);
    __atomic_store_n(s->ctl + 2, 0, __ATOMIC_RELAXED);
    launch_zero(s->args.mail_assigned, s->mail_bytes, s->rstream);
    launch_served(s->args, kernel_prec(s->prec), s->rgrid, kServedThreads, kServedLds, s->rstream);
    PCAL_HIP(hipGetLastError());
    s->relaunches += 1;
    return PCAL_OK;
}

// Resident form: every published chunk's tasks have ended.
bool ring_idle(const pcal_server_ctx *s) {
    const unsigned long long lo = s->published > static_cast<unsigned long long>(s->cap)
                                      ? s->published - static_cast<unsigned long long>(s->cap) : 0ull;
    for (unsigned long long c = lo; c < s->published; ++c)
        if (__atomic_load_n(s->slot_free + c % static_cast<unsigned>(s->cap), __ATOMIC_ACQUIRE) < c + 1) return false;
    return true;
}

// Resident form: wait (bounded) until every published chunk has ended and every
// published finalize has been reported.
int wait_idle(pcal_server_ctx *s, double seconds) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const int rc = keep_alive(s);
        if (rc) return rc;
        drain_done(s);
        bool fin = false;
        for (const SrvStream &st : s->streams) fin = fin || (st.open && st.fin_inflight);
        if (!fin && ring_idle(s)) return PCAL_OK;
        if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > seconds) {
            set_message("served loop: published work did not finish in time");
            return PCAL_EHIP;
        }
    }
}

void free_resident(pcal_server_ctx *s) {
    if (s->rstream) {
        (void)hipStreamSynchronize(s->rstream);
        (void)hipStreamDestroy(s->rstream);
        s->rstream = nullptr;
    }
    if (s->sstream) {
        (void)hipStreamDestroy(s->sstream);
        s->sstream = nullptr;
    }
    if (s->dmem && s->args.stat &&
        hipMemcpy(s->last_stat, s->args.stat, sizeof(s->last_stat), hipMemcpyDeviceToHost) == hipSuccess)
        s->have_stat = true;
    (void)hipGetLastError();
    s->args.stat = nullptr;
    if (s->ring) (void)hipHostFree(s->ring);
    if (s->slot_free) (void)hipHostFree(s->slot_free);
    if (s->dn) (void)hipHostFree(s->dn);
    if (s->ctl) (void)hipHostFree(s->ctl);
    if (s->pub) (void)hipHostFree(s->pub);
    if (s->dmem) (void)hipFree(s->dmem);
    s->pub = nullptr;
    s->ring = nullptr;
    s->slot_free = nullptr;
    s->dn = nullptr;
    s->ctl = nullptr;
    s->dmem = nullptr;
    s->resident = false;
}

// Resident form: whether a stream's plan fits the persistent kernel.
bool resident_fits(const pcal_server_ctx *s, const Plan &p) {
    return p.method == PCAL_METHOD_PERIOD_FOLD && p.N <= kServedMaxTones && p.geom.col_tiles <= s->tasks;
}

// Resident form: publish queued pieces as long as the ring has room; a piece
// that completes an integration waits while the stream's previous finalize
// is still in flight (the two would share the finalize's scratch).
int publish(pcal_server_ctx *s, int64_t *samples) {
    const int M = s->max_streams;
    bool progress = true;
    while (progress) {
        progress = false;
        for (int j = 0; j < M; ++j) {
            const int sid = (s->rr + j) % M;
            SrvStream &st = s->streams[sid];
            if (!st.open || st.queue.empty()) continue;
            const unsigned long long c = s->published;
            const int slot = static_cast<int>(c % static_cast<unsigned>(s->cap));
            if (c >= static_cast<unsigned long long>(s->cap) &&
                __atomic_load_n(s->slot_free + slot, __ATOMIC_ACQUIRE) < c - static_cast<unsigned>(s->cap) + 1)
                return PCAL_OK;  // ring full
            Piece &pc = st.queue.front();
            const int64_t take = std::min(pc.n, st.integ_samples - st.in_integ);
            const bool completes = st.in_integ + take == st.integ_samples;
            if (completes && st.fin_inflight) continue;
            pcal_t h = nullptr;
            int rc = pcal_batch_handle(s->batch, st.bid, &h);
            if (rc) return rc;
            const Plan &p = h->plan;
            const int bank = static_cast<int>(st.integ & 1);
            const size_t NS = static_cast<size_t>(kAccSlots) * static_cast<size_t>(p.N);
            ServedDesc &d = s->ring[slot];
            const unsigned long long back = static_cast<unsigned>(s->backlog_chunks);
            const bool backlog =
                back > 0 && c >= back &&
                __atomic_load_n(s->slot_free + (c - back) % static_cast<unsigned>(s->cap), __ATOMIC_RELAXED) <
                    c - back + 1;
            const int64_t tb = backlog ? s->backlog_task_bytes : s->task_bytes;
            const int64_t want = (take / st.spb + tb - 1) / tb;
            const int target = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, s->tasks)));
            const pcal_launch_t L = plan_launch(p, reinterpret_cast<uintptr_t>(pc.ptr), h->n_total, take, target);
            d.fold = fold_args(h, L, pc.ptr);
            d.fold.acc = h->acc_mem + bank * NS;
            d.fold.acc_int = h->acc_int_mem + bank * NS;
            d.fold.accf = h->accf_mem + bank * NS;
            d.sid = sid;
            d.bank = bank;
            d.ntasks = static_cast<int>(L.grid);
            d.integ = st.integ;
            d.fin_total = 0;
            if (completes) {
                const int k = static_cast<int>(st.integ % kResultDepth);
                FinArgs f = fin_args(h, st.slots_dev + static_cast<size_t>(k) * (4 * st.N + 1));
                f.acc = d.fold.acc;
                f.accf = d.fold.accf;
                // clear only the accumulators the form adds into (the others stay zero)
                const bool f32 = p.prec == PCAL_PREC_F32;
                f.acc_clear = f32 ? nullptr : d.fold.acc;
                f.accf_clear = f32 ? d.fold.accf : nullptr;
                f.acc_int_clear = d.fold.int_bins ? d.fold.acc_int : nullptr;
                f.counter = h->counters + bank;
                f.inv_L = 1.0 / static_cast<double>(st.integ_samples);
                f.clear = 1;
                d.fin = f;
                d.fin_total = static_cast<int>(st.integ_tasks + d.ntasks);
                st.slot_integ[k] = st.integ;
                st.slot_ready[k] = false;
                st.fin_inflight = true;
            }
            s->published = c + 1;
            // the descriptor is complete: publish its tasks
            __atomic_store_n(s->pub, s->published * static_cast<unsigned long long>(s->tasks), __ATOMIC_RELEASE);
            if (samples) *samples += take;
            h->n_total += take;
            pc.ptr += take / st.spb;
            pc.n -= take;
            st.queued -= take;
            if (pc.n == 0) st.queue.pop_front();
            st.in_integ += take;
            st.integ_tasks += d.ntasks;
            s->tasks_published += static_cast<unsigned long long>(d.ntasks);
            if (completes) {
                st.integ += 1;
                st.in_integ = 0;
                st.integ_tasks = 0;
            }
            progress = true;
        }
        s->rr = M > 0 ? (s->rr + 1) % M : 0;
    }
    return PCAL_OK;
}

}  // namespace

extern "C" {

int pcal_server_create(int64_t mem_budget_bytes, int max_streams, int precision, pcal_server_t *out) {
    if (!out || mem_budget_bytes <= 0 || max_streams <= 0) return PCAL_EINVAL;
    *out = nullptr;
    pcal_server_ctx *s = new (std::nothrow) pcal_server_ctx();
    if (!s) return PCAL_ENOMEM;
    const int rc = pcal_batch_create(max_streams, precision, &s->batch);
    if (rc) {
        delete s;
        return rc;
    }
    s->budget = mem_budget_bytes;
    s->prec = precision;
    s->max_streams = max_streams;
    s->streams.resize(max_streams);
    *out = s;
    return PCAL_OK;
}

int pcal_server_open(pcal_server_t s, int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int sideband,
                     int64_t integration_samples, int *sid) {
    if (!s || !sid) return PCAL_EINVAL;
    if (nbits != 2 && nbits != 8) return PCAL_EINVAL;
    const int spb = 8 / nbits;
    if (integration_samples <= 0 || integration_samples % spb) return PCAL_EINVAL;
    int slot = -1;
    for (int i = 0; i < s->max_streams; ++i)
        if (!s->streams[i].open) {
            slot = i;
            break;
        }
    if (slot < 0) return PCAL_EAGAIN;
    // admission, before anything is allocated: the device memory of the
    // stream's tables and accumulators, from its plan, must fit the budget left
    // (the plan the batch will make: the period fold, else AUTO's per-sample form)
    Plan plan{};
    int rc = make_plan(fs_hz, f_comb_hz, f_offset_hz, nbits, sideband, PCAL_METHOD_PERIOD_FOLD, s->prec, &plan,
                       batch_threads(s->batch));
    if (rc == PCAL_ENOTSUP)
        rc = make_plan(fs_hz, f_comb_hz, f_offset_hz, nbits, sideband, PCAL_METHOD_AUTO, s->prec, &plan, 0);
    if (rc) return rc;
    if (s->resident && !resident_fits(s, plan)) return PCAL_ENOTSUP;
    if (s->used + plan_device_bytes(plan) > s->budget) return PCAL_EAGAIN;
    int bid = -1;
    rc = pcal_batch_add(s->batch, fs_hz, f_comb_hz, f_offset_hz, nbits, sideband, &bid);
    if (rc) return rc;
    pcal_t h = nullptr;
    if ((rc = pcal_batch_handle(s->batch, bid, &h))) return rc;
    const int N = static_cast<int>(h->plan.N);
    const int64_t slots_bytes = static_cast<int64_t>(sizeof(double)) * kResultDepth * (4 * N + 1);
    SrvStream &st = s->streams[slot];
    {
        // coherent: the device-resident loop's finalize writes here while its kernel runs on
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&st.slots), static_cast<size_t>(slots_bytes),
                                     hipHostMallocCoherent | hipHostMallocMapped);
        if (e != hipSuccess) {
            set_error("hipHostMalloc", e);
            (void)batch_release(s->batch, bid);
            st.slots = nullptr;
            return e == hipErrorOutOfMemory ? PCAL_ENOMEM : PCAL_EHIP;
        }
        e = hipHostGetDevicePointer(reinterpret_cast<void **>(&st.slots_dev), st.slots, 0);
        if (e != hipSuccess) {
            set_error("hipHostGetDevicePointer", e);
            (void)batch_release(s->batch, bid);
            (void)hipHostFree(st.slots);
            st.slots = nullptr;
            return PCAL_EHIP;
        }
    }
    st.open = true;
    st.bid = bid;
    st.spb = spb;
    st.N = N;
    st.integ_samples = integration_samples;
    st.integ = 0;
    st.in_integ = 0;
    st.device_bytes = h->device_bytes;
    st.queue.clear();
    st.queued = 0;
    st.integ_tasks = 0;
    st.fin_inflight = false;
    for (int i = 0; i < kResultDepth; ++i) {
        st.slot_integ[i] = -1;
        st.slot_ready[i] = false;
    }
    s->used += h->device_bytes;
    *sid = slot;
    return PCAL_OK;
}

int pcal_server_close(pcal_server_t s, int sid) {
    if (!s || !valid_sid(s, sid)) return PCAL_EINVAL;
    SrvStream &st = s->streams[sid];
    // its work and any results still in flight end before its memory goes
    for (Inflight &f : s->inflight) PCAL_HIP(hipEventSynchronize(f.ev));
    if (s->resident) {
        const int rc = wait_idle(s, 30.0);
        if (rc) return rc;
    }
    const int rc = batch_release(s->batch, st.bid);
    if (st.slots) (void)hipHostFree(st.slots);
    st.slots = nullptr;
    st.slots_dev = nullptr;
    st.open = false;
    st.queue.clear();
    st.queued = 0;
    s->used -= st.device_bytes;
    return rc;
}

int pcal_server_submit(pcal_server_t s, int count, const int *sids, const void *const *dev_ptrs,
                       const int64_t *nsamples) {
    if (!s || count < 0 || (count > 0 && (!sids || !dev_ptrs || !nsamples))) return PCAL_EINVAL;
    for (int i = 0; i < count; ++i) {
        if (!valid_sid(s, sids[i])) return PCAL_EINVAL;
        const SrvStream &st = s->streams[sids[i]];
        if (nsamples[i] < 0 || nsamples[i] % st.spb || (nsamples[i] > 0 && !dev_ptrs[i])) return PCAL_EINVAL;
    }
    for (int i = 0; i < count; ++i)
        if (nsamples[i] > 0) {
            SrvStream &st = s->streams[sids[i]];
            st.queue.push_back(Piece{static_cast<const uint8_t *>(dev_ptrs[i]), nsamples[i]});
            st.queued += nsamples[i];
        }
    return PCAL_OK;
}

int pcal_server_step(pcal_server_t s, pcal_stream_t stream, int64_t *samples_dispatched) {
    if (!s) return PCAL_EINVAL;
    if (samples_dispatched) *samples_dispatched = 0;
    if (s->resident) {
        const int rc = keep_alive(s);
        if (rc) return rc;
        drain_done(s);
        return publish(s, samples_dispatched);
    }
    hipStream_t hs = static_cast<hipStream_t>(stream);
    s->ids.clear();
    s->ptrs.clear();
    s->ns.clear();
    s->done.clear();
    s->done_bids.clear();
    s->done_outs.clear();
    int64_t total = 0;
    const int M = s->max_streams;
    for (int j = 0; j < M; ++j) {
        const int sid = (s->rr + j) % M;
        SrvStream &st = s->streams[sid];
        if (!st.open || st.queue.empty()) continue;
        Piece &pc = st.queue.front();
        const int64_t take = std::min(pc.n, st.integ_samples - st.in_integ);
        s->ids.push_back(st.bid);
        s->ptrs.push_back(pc.ptr);
        s->ns.push_back(take);
        total += take;
        pc.ptr += take / st.spb;
        pc.n -= take;
        st.queued -= take;
        if (pc.n == 0) st.queue.pop_front();
        st.in_integ += take;
        if (st.in_integ == st.integ_samples) {
            s->done.push_back(Done{sid, st.integ});
            s->done_bids.push_back(st.bid);
            s->done_outs.push_back(st.slots_dev + static_cast<size_t>(st.integ % kResultDepth) * (4 * st.N + 1));
        }
    }
    s->rr = M > 0 ? (s->rr + 1) % M : 0;
    if (s->ids.empty()) return PCAL_OK;
    int rc = pcal_batch_extract(s->batch, static_cast<int>(s->ids.size()), s->ids.data(), s->ptrs.data(),
                                s->ns.data(), stream);
    if (rc) return rc;
    if (samples_dispatched) *samples_dispatched = total;
    if (s->done.empty()) return PCAL_OK;
    // The finalize writes each finished integration's results straight into
    // its stream's pinned result slot (no copies).
    for (const Done &d : s->done) {
        SrvStream &st = s->streams[d.sid];
        const int k = static_cast<int>(d.integ % kResultDepth);
        st.slot_integ[k] = d.integ;
        st.slot_ready[k] = false;
        st.integ += 1;
        st.in_integ = 0;
    }
    if ((rc = batch_finalize_async(s->batch, static_cast<int>(s->done_bids.size()), s->done_bids.data(),
                                   s->done_outs.data(), hs)))
        return rc;
    Inflight f;
    if ((rc = take_event(s, &f.ev))) return rc;
    PCAL_HIP(hipEventRecord(f.ev, hs));
    f.items = s->done;
    s->inflight.push_back(std::move(f));
    return PCAL_OK;
}

int pcal_server_poll(pcal_server_t s, int max, int *sids, int64_t *integrations, int *n) {
    if (!s || !n || max < 0 || (max > 0 && (!sids || !integrations))) return PCAL_EINVAL;
    *n = 0;
    if (s->resident) drain_done(s);
    while (!s->ready.empty() && *n < max) {
        sids[*n] = s->ready.front().sid;
        integrations[*n] = s->ready.front().integ;
        s->ready.pop_front();
        ++*n;
    }
    while (!s->inflight.empty() && *n < max) {
        Inflight &f = s->inflight.front();
        const hipError_t q = hipEventQuery(f.ev);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
            set_error("hipEventQuery", q);
            return PCAL_EHIP;
        }
        while (f.next < f.items.size() && *n < max) {
            const Done &d = f.items[f.next++];
            if (valid_sid(s, d.sid)) {
                SrvStream &st = s->streams[d.sid];
                const int k = static_cast<int>(d.integ % kResultDepth);
                if (st.slot_integ[k] == d.integ) st.slot_ready[k] = true;
            }
            sids[*n] = d.sid;
            integrations[*n] = d.integ;
            ++*n;
        }
        if (f.next == f.items.size()) {
            s->spare_events.push_back(f.ev);
            s->inflight.pop_front();
        }
    }
    return PCAL_OK;
}

int pcal_server_result(pcal_server_t s, int sid, int64_t integration, double *amp, double *phase, double *delay) {
    if (!s || !valid_sid(s, sid) || integration < 0) return PCAL_EINVAL;
    const SrvStream &st = s->streams[sid];
    const int k = static_cast<int>(integration % kResultDepth);
    if (st.slot_integ[k] != integration || !st.slot_ready[k]) return PCAL_ESTATE;
    const double *r = st.slots + static_cast<size_t>(k) * (4 * st.N + 1);
    const size_t N = static_cast<size_t>(st.N);
    if (amp) memcpy(amp, r, sizeof(double) * N);
    if (phase) memcpy(phase, r + N, sizeof(double) * N);
    if (delay) *delay = r[4 * N];
    return PCAL_OK;
}

int pcal_server_spectrum(pcal_server_t s, int sid, int64_t integration, double *re, double *im) {
    if (!s || !valid_sid(s, sid) || integration < 0) return PCAL_EINVAL;
    const SrvStream &st = s->streams[sid];
    const int k = static_cast<int>(integration % kResultDepth);
    if (st.slot_integ[k] != integration || !st.slot_ready[k]) return PCAL_ESTATE;
    const double *r = st.slots + static_cast<size_t>(k) * (4 * st.N + 1);
    const size_t N = static_cast<size_t>(st.N);
    if (re) memcpy(re, r + 2 * N, sizeof(double) * N);
    if (im) memcpy(im, r + 3 * N, sizeof(double) * N);
    return PCAL_OK;
}

int pcal_server_stats(pcal_server_t s, int64_t *queued_samples, int *inflight_finalizes, int64_t *device_bytes) {
    if (!s) return PCAL_EINVAL;
    if (queued_samples) {
        int64_t q = 0;
        for (const SrvStream &st : s->streams)
            if (st.open) q += st.queued;
        *queued_samples = q;
    }
    if (inflight_finalizes) {
        int f = static_cast<int>(s->inflight.size());
        for (const SrvStream &st : s->streams) f += (st.open && st.fin_inflight) ? 1 : 0;
        *inflight_finalizes = f;
    }
    if (device_bytes) *device_bytes = s->used;
    return PCAL_OK;
}

int pcal_server_start(pcal_server_t s, int workgroups, pcal_stream_t stream) {
    if (!s || workgroups < 2 || workgroups > kServedMaxWorkgroups) return PCAL_EINVAL;
    if (s->resident) return PCAL_ESTATE;
    if (batch_threads(s->batch) != kServedThreads) return PCAL_ENOTSUP;
    s->args = ServedArgs{};
    s->tasks = std::max(1, env_int("PCAL_SERVED_TASKS", kTasksPerChunk));
    s->task_bytes = static_cast<int64_t>(std::max(1, env_int("PCAL_SERVED_TASK_KIB", kTaskKib))) << 10;
    s->backlog_task_bytes =
        static_cast<int64_t>(std::max(1, env_int("PCAL_SERVED_BACKLOG_TASK_KIB", kBacklogTaskKib))) << 10;
    s->backlog_chunks = std::min(kRingSlots - 1, std::max(0, env_int("PCAL_SERVED_BACKLOG", kBacklogChunks)));
    for (int i = 0; i < s->max_streams; ++i) {
        if (!s->streams[i].open) continue;
        pcal_t h = nullptr;
        int rc = pcal_batch_handle(s->batch, s->streams[i].bid, &h);
        if (rc) return rc;
        if (!resident_fits(s, h->plan)) return PCAL_ENOTSUP;
    }
    // the host-step form's work ends first: its results are reported by later polls
    for (Inflight &f : s->inflight) PCAL_HIP(hipEventSynchronize(f.ev));
    int rc;
    s->cap = kRingSlots;
    s->done_cap = kDoneSlots;
    if ((rc = coherent_alloc(&s->ring, s->cap)) || (rc = coherent_alloc(&s->slot_free, s->cap)) ||
        (rc = coherent_alloc(&s->dn, s->done_cap)) || (rc = coherent_alloc(&s->ctl, 4)) ||
        (rc = coherent_alloc(&s->pub, 1))) {
        free_resident(s);
        return rc;
    }
    // Device memory of the loop: the scheduler's state, the completion cursor,
    // the loop counters and the heartbeat, each on a line of its own (256 B), then the
    // per-slot and per-bank counters, the per-bank finalize arguments, the
    // mailboxes (one 256-byte line per workgroup each way) and the device
    // copies of the descriptors.
    const size_t nsb = 2 * static_cast<size_t>(s->max_streams);
    const size_t cap = static_cast<size_t>(s->cap);
    const size_t o_cnt = 4 * 256;
    const size_t o_done = (o_cnt + 4 * cap + 7) & ~static_cast<size_t>(7);
    const size_t o_fin = (o_done + 8 * nsb + 255) & ~static_cast<size_t>(255);
    const size_t o_mail = (o_fin + sizeof(FinArgs) * nsb + 255) & ~static_cast<size_t>(255);
    const size_t mail = 8 * kMailStride * static_cast<size_t>(workgroups);
    const size_t o_ring = o_mail + 2 * mail;
    const size_t dbytes = o_ring + sizeof(ServedDesc) * cap;
    {
        const hipError_t e = hipMalloc(&s->dmem, dbytes);
        if (e != hipSuccess) {
            set_error("hipMalloc", e);
            free_resident(s);
            return e == hipErrorOutOfMemory ? PCAL_ENOMEM : PCAL_EHIP;
        }
    }
    // The loop runs on a stream of its own that does not synchronise with the
    // null stream (default priority): synchronous copies elsewhere (tables of
    // streams opened later) must not wait for the persistent kernel.  It
    // starts after the work already enqueued on the caller's stream.
    hipStream_t hs = nullptr;
    {
        hipError_t e = hipStreamCreateWithFlags(&hs, hipStreamNonBlocking);
        if (e != hipSuccess) {
            set_error("hipStreamCreateWithFlags", e);
            free_resident(s);
            return PCAL_EHIP;
        }
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, static_cast<hipStream_t>(stream));
        if (e == hipSuccess) e = hipStreamWaitEvent(hs, ev, 0);
        if (ev) (void)hipEventDestroy(ev);
        if (e != hipSuccess) {
            set_error("ordering the served loop after the caller's stream", e);
            (void)hipStreamDestroy(hs);
            free_resident(s);
            return PCAL_EHIP;
        }
    }
    s->rstream = hs;
    launch_zero(s->dmem, dbytes, hs);
    ServedArgs &a = s->args;
    a = ServedArgs{};
    unsigned char *dm = static_cast<unsigned char *>(s->dmem);
    a.sched = reinterpret_cast<unsigned long long *>(dm);
    a.done_cursor = reinterpret_cast<unsigned long long *>(dm + 256);
    a.stat = reinterpret_cast<unsigned long long *>(dm + 2 * 256);
    a.heartbeat = reinterpret_cast<unsigned long long *>(dm + 3 * 256);
    static_assert(kServedStats * 8 <= 256, "loop counters fit their line");
    a.slot_cnt = reinterpret_cast<unsigned *>(dm + o_cnt);
    a.task_done = reinterpret_cast<unsigned long long *>(dm + o_done);
    a.fin_args = reinterpret_cast<FinArgs *>(dm + o_fin);
    a.mail_assigned = reinterpret_cast<unsigned long long *>(dm + o_mail);
    a.mail_done = reinterpret_cast<unsigned long long *>(dm + o_mail + mail);
    a.dring = reinterpret_cast<ServedDesc *>(dm + o_ring);
    s->mail_bytes = 2 * mail;
    if ((rc = device_address(s->ring, const_cast<ServedDesc **>(&a.ring))) ||
        (rc = device_address(s->slot_free, &a.slot_free)) || (rc = device_address(s->dn, &a.done)) ||
        (rc = device_address(s->ctl, &a.status)) ||
        (rc = device_address(s->pub, const_cast<unsigned long long **>(&a.published)))) {
        free_resident(s);
        return rc;
    }
    a.quit = a.status;   // ctl[0]
    a.status = a.status + 1;  // ctl[1], ctl[2]
    a.cap = s->cap;
    a.done_cap = s->done_cap;
    a.tasks = s->tasks;
    a.grid = workgroups;
    {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            khz = 100000;  // the documented 100 MHz
        (void)hipGetLastError();
        const int idle_ms = std::max(1, env_int("PCAL_SERVED_IDLE_MS", kIdleMs));
        a.idle_ticks = static_cast<unsigned long long>(idle_ms) * static_cast<unsigned long long>(khz);
        const int worker_ms = std::max(1, env_int("PCAL_SERVED_WORKER_MS", static_cast<int>(kWorkerSeconds * 1e3)));
        a.worker_ticks = static_cast<unsigned long long>(worker_ms) * static_cast<unsigned long long>(khz);
        a.check_ticks = static_cast<unsigned long long>(khz);  // 1 ms
        a.quit_ticks = static_cast<unsigned long long>(kQuitSeconds * 1e3 * static_cast<double>(khz));
    }
    s->published = 0;
    s->tasks_published = 0;
    s->done_next = 0;
    s->relaunches = 0;
    s->have_stat = false;
    s->rgrid = workgroups;
    launch_served(a, kernel_prec(s->prec), workgroups, kServedThreads, kServedLds, hs);
    {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("launch of the served loop", e);
            (void)hipStreamSynchronize(hs);
            free_resident(s);
            return PCAL_EHIP;
        }
    }
    for (SrvStream &st : s->streams) {
        st.integ_tasks = 0;
        st.fin_inflight = false;
    }
    s->resident = true;
    return PCAL_OK;
}

int pcal_server_stop(pcal_server_t s) {
    if (!s) return PCAL_EINVAL;
    if (!s->resident) return PCAL_ESTATE;
    const int idle = wait_idle(s, 30.0);
    __atomic_store_n(s->ctl, 1, __ATOMIC_RELEASE);  // quit: every workgroup leaves at its next empty poll
    PCAL_HIP(hipStreamSynchronize(s->rstream));
    const int left = __atomic_load_n(s->ctl + 1, __ATOMIC_ACQUIRE);
    free_resident(s);
    if (idle) return idle;
    if (left != s->rgrid) {
        set_message("served loop: not every workgroup left at quit");
        return PCAL_EHIP;
    }
    return PCAL_OK;
}

int pcal_server_loop_stats(pcal_server_t s, int64_t *out, int n) {
    if (!s || !out || n < 0) return PCAL_EINVAL;
    if (!s->have_stat && !s->resident) return PCAL_ESTATE;
    unsigned long long dev[kServedStats] = {};
    if (s->resident) {
        // while the kernel runs: a copy on a non-blocking stream of our own,
        // which does not wait for the persistent kernel's stream
        if (!s->sstream) PCAL_HIP(hipStreamCreateWithFlags(&s->sstream, hipStreamNonBlocking));
        PCAL_HIP(hipMemcpyAsync(dev, s->args.stat, sizeof(dev), hipMemcpyDeviceToHost, s->sstream));
        PCAL_HIP(hipStreamSynchronize(s->sstream));
    } else {
        memcpy(dev, s->last_stat, sizeof(dev));
    }
    int khz = 0, devno = 0;
    PCAL_HIP(hipGetDevice(&devno));
    PCAL_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, devno));
    const double ns_per_tick = khz > 0 ? 1e6 / khz : 10.0;
    int64_t v[PCAL_LOOP_STATS];
    v[0] = static_cast<int64_t>(s->published);
    for (int k = 1; k < 8; ++k) v[k] = static_cast<int64_t>(dev[k]);
    v[2] = static_cast<int64_t>(s->tasks_published);
    v[6] = s->relaunches;
    for (int k = 8; k < 13; ++k) v[k] = static_cast<int64_t>(static_cast<double>(dev[k]) * ns_per_tick);
    for (int k = 0; k < n && k < PCAL_LOOP_STATS; ++k) out[k] = v[k];
    return PCAL_OK;
}

int pcal_server_destroy(pcal_server_t s) {
    if (!s) return PCAL_EINVAL;
    if (s->resident) (void)pcal_server_stop(s);
    for (Inflight &f : s->inflight) {
        (void)hipEventSynchronize(f.ev);
        (void)hipEventDestroy(f.ev);
    }
    for (hipEvent_t e : s->spare_events) (void)hipEventDestroy(e);
    for (SrvStream &st : s->streams)
        if (st.slots) (void)hipHostFree(st.slots);
    const int rc = pcal_batch_destroy(s->batch);
    delete s;
    return rc;
}

}  // extern "C"
