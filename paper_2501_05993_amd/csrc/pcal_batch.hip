// Batched multi-stream form of libpcal: many streams (each its own fs,
// f_offset, sample format, tables and accumulators) extracted by one launch of
// the fused kernel over a work-list, finalized by one launch, results copied
// by one transfer.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "pcal_host.h"

using namespace pcal;
using namespace pcal::host;

namespace {

constexpr int kBatchThreads = 512;        // workgroup size members are planned for (PCAL_BATCH_THREADS)
constexpr int kBatchTargetBlocks = 2048;  // workgroups per batched launch, split by bytes (PCAL_BATCH_BLOCKS)
constexpr int kStages = 4;                // pinned staging buffers in flight

// Host staging of one launch's work-list (pinned) and its device copy: one
// block holding first[] (the first workgroup of each item, then the total),
// then the items (FoldArgs, FinArgs or ZeroItem: one kind per use), so that a
// work-list goes to the device in one copy.
struct Stage {
    unsigned char *h_buf = nullptr;
    unsigned char *d_buf = nullptr;
    size_t off_items = 0;       // byte offset of the items in both blocks
    int *h_first = nullptr;
    FoldArgs *h_items = nullptr;
    FinArgs *h_fin = nullptr;
    ZeroItem *h_zero = nullptr;
    hipEvent_t done = nullptr;  // the launch that read this stage has been enqueued past this event
    hipEvent_t copied = nullptr;  // the copy of this stage's work-list (on the copy stream) is past this event
    bool pending = false;
    const int *d_first() const { return reinterpret_cast<const int *>(d_buf); }
    template <class T>
    const T *d_items() const { return reinterpret_cast<const T *>(d_buf + off_items); }
    // Copy first[0..nfirst) and items [0, item_bytes) to the device in one
    // transfer on the copy stream `up`, and make s wait for it.  On s itself
    // the copy would stall the stream between two launches (~15 us measured
    // for a 24 KiB work-list); on its own stream it runs while s still works
    // on earlier launches, and the wait costs s nothing once the copy is done.
    hipError_t upload(int nfirst, size_t item_bytes, hipStream_t up, hipStream_t s) const {
        const size_t bytes = item_bytes ? off_items + item_bytes : sizeof(int) * nfirst;
        hipError_t e = hipMemcpyAsync(d_buf, h_buf, bytes, hipMemcpyHostToDevice, up);
        if (e == hipSuccess) e = hipEventRecord(copied, up);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, copied, 0);
        return e;
    }
};

}  // namespace

struct pcal_batch_ctx {
    int prec = PCAL_PREC_F64;
    int max_streams = 0;
    int threads = kBatchThreads;        // workgroup size members are planned for
    int target_blocks = kBatchTargetBlocks;
    std::vector<pcal_ctx *> members;
    Stage stage[kStages];
    int next = 0;
    double *d_out = nullptr;   // results of a batched finalize
    double *h_out = nullptr;   // pinned copy
    size_t out_cap = 0;        // doubles
    hipStream_t last_stream = nullptr;
    bool dirty = false;        // a batched call has enqueued work on last_stream
    hipEvent_t ev = nullptr;   // recorded on last_stream when the batch is destroyed
    hipStream_t up = nullptr;  // copy stream of the staged work-lists (default priority)
    std::vector<unsigned> seen;  // per member id: the call stamp that last listed it
    unsigned stamp = 0;
};

namespace {

int stage_alloc(Stage &st, int n) {
    st.off_items = (sizeof(int) * (n + 1) + 255) & ~static_cast<size_t>(255);
    const size_t item_cap = std::max(std::max(sizeof(FoldArgs), sizeof(FinArgs)), 3 * sizeof(ZeroItem)) * n;
    const size_t bytes = st.off_items + item_cap;
    PCAL_HIP(hipHostMalloc(reinterpret_cast<void **>(&st.h_buf), bytes, hipHostMallocDefault));
    PCAL_HIP(hipMalloc(reinterpret_cast<void **>(&st.d_buf), bytes));
    st.h_first = reinterpret_cast<int *>(st.h_buf);
    st.h_items = reinterpret_cast<FoldArgs *>(st.h_buf + st.off_items);
    st.h_fin = reinterpret_cast<FinArgs *>(st.h_buf + st.off_items);
    st.h_zero = reinterpret_cast<ZeroItem *>(st.h_buf + st.off_items);
    PCAL_HIP(hipEventCreateWithFlags(&st.done, hipEventDisableTiming));
    PCAL_HIP(hipEventCreateWithFlags(&st.copied, hipEventDisableTiming));
    return PCAL_OK;
}

void stage_free(Stage &st) {
    if (st.h_buf) (void)hipHostFree(st.h_buf);
    if (st.d_buf) (void)hipFree(st.d_buf);
    if (st.done) (void)hipEventDestroy(st.done);
    if (st.copied) (void)hipEventDestroy(st.copied);
}

// A staging buffer whose previous use has been consumed by the GPU.
int take_stage(pcal_batch_ctx *b, Stage **out) {
    Stage &st = b->stage[b->next];
    b->next = (b->next + 1) % kStages;
    if (st.pending) PCAL_HIP(hipEventSynchronize(st.done));
    st.pending = false;
    *out = &st;
    return PCAL_OK;
}

int check_ids(const pcal_batch_ctx *b, int count, const int *ids) {
    if (count < 0 || (count > 0 && !ids) || count > b->max_streams) return PCAL_EINVAL;
    for (int i = 0; i < count; ++i)
        if (ids[i] < 0 || ids[i] >= static_cast<int>(b->members.size()) || !b->members[ids[i]]) return PCAL_EINVAL;
    return PCAL_OK;
}

// Order `s` after every listed member's previous work.
int order_members(pcal_batch_ctx *b, int count, const int *ids, hipStream_t s) {
    for (int i = 0; i < count; ++i) {
        const int rc = order_on(b->members[ids[i]], s);
        if (rc) return rc;
    }
    return PCAL_OK;
}

// Note the call's work on s as every listed member's last work (events are
// recorded only when a member moves to another stream or is synchronised).
int mark_members(pcal_batch_ctx *b, int count, const int *ids, hipStream_t s) {
    for (int i = 0; i < count; ++i) mark(b->members[ids[i]], s);
    b->last_stream = s;
    b->dirty = true;
    return PCAL_OK;
}

}  // namespace

namespace pcal {
namespace host {

// Batched finalize of members ids[0..count) that reads and clears their bins
// (the next integration starts at zero); each member's results land in its
// own device buffer h->out.  Asynchronous on s.
int batch_finalize_async(pcal_batch_ctx *b, int count, const int *ids, double *const *outs, hipStream_t s) {
    int rc = check_ids(b, count, ids);
    if (rc || count == 0) return rc;
    DeviceGuard guard(b->members[ids[0]]->device);
    if ((rc = order_members(b, count, ids, s))) return rc;
    // a short list travels in the kernel arguments; a longer one is staged
    FinListInline il;
    Stage *st = nullptr;
    const bool inl = count <= kInlineFinItems;
    if (!inl && (rc = take_stage(b, &st))) return rc;
    FinArgs *items = inl ? il.items : st->h_fin;
    int *first = inl ? il.first : st->h_first;
    int grid = 0;
    size_t lds = 0;
    for (int i = 0; i < count; ++i) {
        pcal_ctx *h = b->members[ids[i]];
        items[i] = fin_args(h, outs && outs[i] ? outs[i] : h->out);
        items[i].clear = 1;
        first[i] = grid;
        grid += static_cast<int>((h->plan.N + 63) / 64);
        lds = std::max(lds, finalize_lds_bytes(static_cast<int>(h->plan.N)));
        h->n_integ = 0;
    }
    first[count] = grid;
    if (inl) {
        il.n = count;
        launch_finalize_batch(il, grid, lds, s);
        PCAL_HIP(hipGetLastError());
    } else {
        PCAL_HIP(st->upload(count + 1, sizeof(FinArgs) * count, b->up, s));
        launch_finalize_batch(DeviceList<FinArgs>{st->d_items<FinArgs>(), st->d_first(), count}, grid, lds, s);
        PCAL_HIP(hipGetLastError());
        PCAL_HIP(hipEventRecord(st->done, s));
        st->pending = true;
    }
    return mark_members(b, count, ids, s);
}

int batch_threads(const pcal_batch_ctx *b) { return b->threads; }

// Destroy member id (after its work) and free its slot for reuse.
int batch_release(pcal_batch_ctx *b, int id) {
    if (!b || id < 0 || id >= static_cast<int>(b->members.size()) || !b->members[id]) return PCAL_EINVAL;
    const int rc = pcal_destroy(b->members[id]);
    b->members[id] = nullptr;
    return rc;
}

}  // namespace host
}  // namespace pcal

extern "C" {

int pcal_batch_create(int max_streams, int precision, pcal_batch_t *out) {
    if (!out || max_streams <= 0 || precision < PCAL_PREC_F64 || precision > PCAL_PREC_Q17) return PCAL_EINVAL;
    if (precision == PCAL_PREC_Q17) return PCAL_ENOTSUP;  // the fixed-point form runs on single handles
    *out = nullptr;
    pcal_batch_ctx *b = new (std::nothrow) pcal_batch_ctx();
    if (!b) return PCAL_ENOMEM;
    b->prec = precision;
    b->max_streams = max_streams;
    b->threads = env_int("PCAL_BATCH_THREADS", kBatchThreads);
    if (b->threads < 64 || b->threads > kMaxFoldThreads || b->threads % 64) b->threads = kBatchThreads;
    b->target_blocks = env_int("PCAL_BATCH_BLOCKS", kBatchTargetBlocks);
    if (b->target_blocks < 1) b->target_blocks = kBatchTargetBlocks;
    {
        hipError_t e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            set_error("hipEventCreateWithFlags", e);
            delete b;
            return PCAL_EHIP;
        }
        e = hipStreamCreateWithFlags(&b->up, hipStreamNonBlocking);
        if (e != hipSuccess) {
            set_error("hipStreamCreateWithFlags", e);
            b->up = nullptr;
            pcal_batch_destroy(b);
            return PCAL_EHIP;
        }
    }
    for (int i = 0; i < kStages; ++i) {
        const int rc = stage_alloc(b->stage[i], max_streams);
        if (rc) {
            pcal_batch_destroy(b);
            return rc;
        }
    }
    *out = b;
    return PCAL_OK;
}

int pcal_batch_add(pcal_batch_t b, int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int sideband,
                   int *id) {
    if (!b || !id) return PCAL_EINVAL;
    // a released slot is reused first
    int slot = -1;
    for (int i = 0; i < static_cast<int>(b->members.size()); ++i)
        if (!b->members[i]) {
            slot = i;
            break;
        }
    if (slot < 0 && static_cast<int>(b->members.size()) >= b->max_streams) return PCAL_EAGAIN;
    // the period fold at the batch's workgroup size; a stream no fold period
    // fits takes a per-sample form (AUTO's), run in launches of its own
    pcal_ctx *h = nullptr;
    int rc = create(fs_hz, f_comb_hz, f_offset_hz, nbits, sideband, PCAL_METHOD_PERIOD_FOLD, b->prec, b->threads, &h);
    if (rc == PCAL_ENOTSUP) rc = create(fs_hz, f_comb_hz, f_offset_hz, nbits, sideband, PCAL_METHOD_AUTO, b->prec, 0, &h);
    if (rc) return rc;
    h->batch_member = true;
    if (slot < 0) {
        b->members.push_back(h);
        slot = static_cast<int>(b->members.size()) - 1;
    } else {
        b->members[slot] = h;
    }
    *id = slot;
    return PCAL_OK;
}

int pcal_batch_handle(pcal_batch_t b, int id, pcal_t *h) {
    if (!b || !h || id < 0 || id >= static_cast<int>(b->members.size()) || !b->members[id]) return PCAL_EINVAL;
    *h = b->members[id];
    return PCAL_OK;
}

int pcal_batch_extract(pcal_batch_t b, int count, const int *ids, const void *const *dev_ptrs,
                       const int64_t *nsamples, pcal_stream_t stream) {
    if (!b) return PCAL_EINVAL;
    int rc = check_ids(b, count, ids);
    if (rc) return rc;
    if (count > 0 && (!dev_ptrs || !nsamples)) return PCAL_EINVAL;
    int64_t total_bytes = 0;
    // one chunk per stream and call: each id at most once (stamped, linear time)
    if (b->seen.size() < b->members.size()) b->seen.resize(b->members.size(), 0u);
    if (++b->stamp == 0) {
        std::fill(b->seen.begin(), b->seen.end(), 0u);
        b->stamp = 1;
    }
    bool any = false;
    for (int i = 0; i < count; ++i) {
        const Plan &p = b->members[ids[i]]->plan;
        if (nsamples[i] < 0 || nsamples[i] % (8 / p.nbits) || (nsamples[i] > 0 && !dev_ptrs[i])) return PCAL_EINVAL;
        if (b->seen[ids[i]] == b->stamp) return PCAL_EINVAL;
        b->seen[ids[i]] = b->stamp;
        any = any || nsamples[i] > 0;
        if (p.method == PCAL_METHOD_PERIOD_FOLD) total_bytes += nsamples[i] * p.nbits / 8;  // the fold work-list
    }
    if (!any) return PCAL_OK;
    DeviceGuard guard(b->members[ids[0]]->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = order_members(b, count, ids, s))) return rc;
    // The work-list holds the 2-bit items first, then the 8-bit ones (one fold
    // launch per sample width).  A short list travels in the kernel
    // arguments; a longer one is staged and copied.
    int n = 0, grid = 0, grid2 = 0, threads = 64, used = 0;
    auto folded = [&](int i) { return nsamples[i] > 0 && b->members[ids[i]]->plan.method == PCAL_METHOD_PERIOD_FOLD; };
    for (int i = 0; i < count; ++i)
        if (folded(i)) {
            threads = std::max(threads, b->members[ids[i]]->plan.geom.threads);
            ++used;
        }
    FoldListInline il;
    Stage *st = nullptr;
    const bool inl = used <= kInlineFoldItems;
    if (used > 0 && !inl && (rc = take_stage(b, &st))) return rc;
    FoldArgs *items = inl ? il.items : st->h_items;
    int *first = inl ? il.first : st->h_first;
    size_t lds[2] = {0, 0};
    for (int pass = 0; pass < 2; ++pass) {
        const int width = pass == 0 ? 2 : 8;
        for (int i = 0; i < count; ++i) {
            if (!folded(i) || b->members[ids[i]]->plan.nbits != width) continue;
            pcal_ctx *h = b->members[ids[i]];
            const Plan &p = h->plan;
            const int64_t bytes = nsamples[i] * p.nbits / 8;
            const int target = static_cast<int>(std::max<int64_t>(
                p.geom.col_tiles, (b->target_blocks * bytes + total_bytes - 1) / total_bytes));
            const pcal_launch_t L =
                plan_launch(p, reinterpret_cast<uintptr_t>(dev_ptrs[i]), h->n_total, nsamples[i], target);
            items[n] = fold_args(h, L, dev_ptrs[i]);
            first[n] = grid;
            grid += static_cast<int>(L.grid);
            const FoldArgs &a = items[n];
            lds[pass] = std::max(lds[pass], fold_lds_bytes(a.npos, p.geom.spv, threads, a.M));
            ++n;
        }
        if (pass == 0) grid2 = grid;
    }
    first[n] = grid;
    if (used == 0) {
        // no fold member in this call
    } else if (inl) {
        il.n = n;
        launch_fold_batch(il, kernel_prec(b->prec), grid2, grid - grid2, threads, lds[0], lds[1], s);
        PCAL_HIP(hipGetLastError());
    } else {
        PCAL_HIP(st->upload(n + 1, sizeof(FoldArgs) * n, b->up, s));
        launch_fold_batch(DeviceList<FoldArgs>{st->d_items<FoldArgs>(), st->d_first(), n}, kernel_prec(b->prec), grid2,
                          grid - grid2, threads, lds[0], lds[1], s);
        PCAL_HIP(hipGetLastError());
        PCAL_HIP(hipEventRecord(st->done, s));
        st->pending = true;
    }
    for (int i = 0; i < count; ++i) {
        pcal_ctx *h = b->members[ids[i]];
        if (h->plan.method == PCAL_METHOD_PERIOD_FOLD) {
            h->n_total += nsamples[i];
            h->n_integ += nsamples[i];
        } else if (nsamples[i] > 0) {
            // a per-sample member: its own launch, after the fold's on the same stream
            if ((rc = pcal_extract(h, dev_ptrs[i], nsamples[i], stream))) return rc;
        }
    }
    return mark_members(b, count, ids, s);
}

int pcal_batch_results(pcal_batch_t b, int count, const int *ids, double *amp, double *phase, double *delay) {
    if (!b) return PCAL_EINVAL;
    int rc = check_ids(b, count, ids);
    if (rc || count == 0) return rc;
    DeviceGuard guard(b->members[ids[0]]->device);
    hipStream_t s = b->members[ids[0]]->last_stream;
    if ((rc = order_members(b, count, ids, s))) return rc;
    size_t need = 0;
    for (int i = 0; i < count; ++i) need += 4 * static_cast<size_t>(b->members[ids[i]]->plan.N) + 1;
    if (need > b->out_cap) {
        if (b->d_out) (void)hipFree(b->d_out);
        if (b->h_out) (void)hipHostFree(b->h_out);
        b->d_out = nullptr;
        b->h_out = nullptr;
        b->out_cap = 0;
        PCAL_HIP(hipMalloc(reinterpret_cast<void **>(&b->d_out), sizeof(double) * need));
        PCAL_HIP(hipHostMalloc(reinterpret_cast<void **>(&b->h_out), sizeof(double) * need, hipHostMallocDefault));
        b->out_cap = need;
    }
    Stage *st = nullptr;
    if ((rc = take_stage(b, &st))) return rc;
    size_t off = 0;
    int grid = 0;
    size_t lds = 0;
    for (int i = 0; i < count; ++i) {
        const pcal_ctx *h = b->members[ids[i]];
        st->h_fin[i] = fin_args(h, b->d_out + off);
        st->h_first[i] = grid;
        grid += static_cast<int>((h->plan.N + 63) / 64);
        lds = std::max(lds, finalize_lds_bytes(static_cast<int>(h->plan.N)));
        off += 4 * static_cast<size_t>(h->plan.N) + 1;
    }
    st->h_first[count] = grid;
    PCAL_HIP(st->upload(count + 1, sizeof(FinArgs) * count, b->up, s));
    launch_finalize_batch(DeviceList<FinArgs>{st->d_items<FinArgs>(), st->d_first(), count}, grid, lds, s);
    PCAL_HIP(hipGetLastError());
    PCAL_HIP(hipEventRecord(st->done, s));
    st->pending = true;
    PCAL_HIP(hipMemcpyAsync(b->h_out, b->d_out, sizeof(double) * off, hipMemcpyDeviceToHost, s));
    PCAL_HIP(hipStreamSynchronize(s));
    if ((rc = mark_members(b, count, ids, s))) return rc;
    off = 0;
    size_t ao = 0;
    for (int i = 0; i < count; ++i) {
        const size_t N = static_cast<size_t>(b->members[ids[i]]->plan.N);
        if (amp) memcpy(amp + ao, b->h_out + off, sizeof(double) * N);
        if (phase) memcpy(phase + ao, b->h_out + off + N, sizeof(double) * N);
        if (delay) delay[i] = b->h_out[off + 4 * N];
        ao += N;
        off += 4 * N + 1;
    }
    return PCAL_OK;
}

int pcal_batch_spectra(pcal_batch_t b, int count, const int *ids, double *re, double *im) {
    // C_k of each listed stream, concatenated (runs the batched finalize)
    if (!b) return PCAL_EINVAL;
    int rc = pcal_batch_results(b, count, ids, nullptr, nullptr, nullptr);
    if (rc || count == 0) return rc;
    size_t off = 0, ao = 0;
    for (int i = 0; i < count; ++i) {
        const size_t N = static_cast<size_t>(b->members[ids[i]]->plan.N);
        if (re) memcpy(re + ao, b->h_out + off + 2 * N, sizeof(double) * N);
        if (im) memcpy(im + ao, b->h_out + off + 3 * N, sizeof(double) * N);
        ao += N;
        off += 4 * N + 1;
    }
    return PCAL_OK;
}

int pcal_batch_reset(pcal_batch_t b, int count, const int *ids) {
    if (!b) return PCAL_EINVAL;
    int rc = check_ids(b, count, ids);
    if (rc || count == 0) return rc;
    DeviceGuard guard(b->members[ids[0]]->device);
    hipStream_t s = b->members[ids[0]]->last_stream;
    if ((rc = order_members(b, count, ids, s))) return rc;
    Stage *st = nullptr;
    if ((rc = take_stage(b, &st))) return rc;
    int n = 0;
    for (int i = 0; i < count; ++i) {
        pcal_ctx *h = b->members[ids[i]];
        const size_t N = static_cast<size_t>(h->plan.N) * kAccSlots;
        st->h_zero[n++] = ZeroItem{h->acc, sizeof(double2) * N};
        st->h_zero[n++] = ZeroItem{h->accf, sizeof(float2) * N};
        st->h_zero[n++] = ZeroItem{h->acc_int, sizeof(long long) * N};
        h->n_integ = 0;
    }
    PCAL_HIP(hipMemcpyAsync(st->d_buf + st->off_items, st->h_zero, sizeof(ZeroItem) * n, hipMemcpyHostToDevice, b->up));
    PCAL_HIP(hipEventRecord(st->copied, b->up));
    PCAL_HIP(hipStreamWaitEvent(s, st->copied, 0));
    launch_zero_list(st->d_items<ZeroItem>(), n, s);
    PCAL_HIP(hipGetLastError());
    PCAL_HIP(hipEventRecord(st->done, s));
    st->pending = true;
    return mark_members(b, count, ids, s);
}

int pcal_batch_size(pcal_batch_t b, int *n) {
    if (!b || !n) return PCAL_EINVAL;
    *n = static_cast<int>(b->members.size());
    return PCAL_OK;
}

int pcal_batch_destroy(pcal_batch_t b) {
    if (!b) return PCAL_EINVAL;
    if (b->ev && b->dirty && hipEventRecord(b->ev, b->last_stream) == hipSuccess) (void)hipEventSynchronize(b->ev);
    for (pcal_ctx *h : b->members)
        if (h) pcal_destroy(h);
    if (b->up) (void)hipStreamSynchronize(b->up);  // no copy still reads a stage
    for (int i = 0; i < kStages; ++i) {
        if (b->stage[i].pending) (void)hipEventSynchronize(b->stage[i].done);
        stage_free(b->stage[i]);
    }
    if (b->d_out) (void)hipFree(b->d_out);
    if (b->h_out) (void)hipHostFree(b->h_out);
    if (b->ev) (void)hipEventDestroy(b->ev);
    if (b->up) (void)hipStreamDestroy(b->up);
    delete b;
    return PCAL_OK;
}

}  // extern "C"
