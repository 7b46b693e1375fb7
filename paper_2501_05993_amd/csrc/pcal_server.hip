// Served form of libpcal: many live streams under one device-memory budget,
// continuously batched.  Chunks queue per stream on the host; every step folds
// the oldest queued piece of each stream with one launch of the batched fused
// kernel, and finalizes (reads and clears) with one batched launch every
// stream whose integration that step completed.  Results reach pinned host
// memory asynchronously and are picked up by polling.
#include <string.h>

#include <algorithm>
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
    double *slots = nullptr;         // pinned [kResultDepth][4N + 1]
    double *slots_dev = nullptr;     // the same memory's device address (the finalize writes it)
    int64_t slot_integ[kResultDepth];  // integration held by each slot (-1: none)
    bool slot_ready[kResultDepth];
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
    Plan plan{};
    int rc = make_plan(fs_hz, f_comb_hz, f_offset_hz, nbits, sideband, PCAL_METHOD_PERIOD_FOLD, s->prec, &plan);
    if (rc) return rc;
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
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&st.slots), static_cast<size_t>(slots_bytes),
                                     hipHostMallocDefault);
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
    const int rc = batch_release(s->batch, st.bid);
    if (st.slots) (void)hipHostFree(st.slots);
    st.slots = nullptr;
    st.slots_dev = nullptr;
    st.open = false;
    st.queue.clear();
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
        if (nsamples[i] > 0)
            s->streams[sids[i]].queue.push_back(Piece{static_cast<const uint8_t *>(dev_ptrs[i]), nsamples[i]});
    return PCAL_OK;
}

int pcal_server_step(pcal_server_t s, pcal_stream_t stream, int64_t *samples_dispatched) {
    if (!s) return PCAL_EINVAL;
    if (samples_dispatched) *samples_dispatched = 0;
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
            if (st.open)
                for (const Piece &p : st.queue) q += p.n;
        *queued_samples = q;
    }
    if (inflight_finalizes) *inflight_finalizes = static_cast<int>(s->inflight.size());
    if (device_bytes) *device_bytes = s->used;
    return PCAL_OK;
}

int pcal_server_destroy(pcal_server_t s) {
    if (!s) return PCAL_EINVAL;
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
