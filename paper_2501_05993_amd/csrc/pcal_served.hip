// The device-resident served loop (pcal_server_start): one persistent kernel
// whose workgroup 0 schedules and whose other workgroups fold published chunk
// tasks with the fold body of pcal_fold.h, each integration finalized by the
// task that completes it.
#include <stddef.h>

#include "pcal_fold.h"

namespace pcal {
namespace {

// Memory ordering.  An acquire or release at agent or system scope makes
// gfx950 invalidate or write back a whole L2 (one per XCD), so the loop keeps
// them out of everything done per poll or per task: it polls, hands out and
// counts with relaxed atomics, which are coherent per location, and orders
// them by waiting for its outstanding memory operations (s_waitcnt) where one
// must be complete before the next is issued.  Host memory is read with
// system-scope loads, which no GPU cache keeps; the device copies of the
// descriptors are written and read with agent-scope atomics.  The one acquire
// (before a finalize reads the bank that other workgroups' atomics filled)
// and the one release (after it clears that bank with plain stores) come once
// per integration: without them the finalized spectra moved by 1e-7 from the
// one-stream extraction's.

__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_stat(const ServedArgs &sa, int k, unsigned long long v) {
    if (v) __hip_atomic_fetch_add(sa.stat + k, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

constexpr int kWords = static_cast<int>(sizeof(ServedDesc) / 4);
constexpr int kFinWords = static_cast<int>(sizeof(FinArgs) / 4);
static_assert(sizeof(FinArgs) % 4 == 0, "finalize arguments are copied as words");
constexpr int kNtasksWord = static_cast<int>(offsetof(ServedDesc, ntasks) / 4);
constexpr int kScanEvery = 16;  // scheduler rounds with nothing pending between reads of the mailboxes
constexpr unsigned long long kLeave = 1ull;  // mailbox value: leave the loop (tasks are handed out as task + 2)

// Workgroup 0: hand the published tasks out, chunk after chunk and in task
// order within a chunk, to the workers whose mailbox shows them idle.  Each
// round: read the host's count of published tasks and its quit flag; copy the
// descriptors of newly published chunks into device memory (complete before
// any of their tasks is handed out); read every worker's mailbox; give the
// k-th idle worker (in worker order) the k-th pending task; and rewrite its
// heartbeat.  It leaves, and tells every worker to leave, after idle_ticks
// without work, or on quit, in both cases with no task pending and no worker
// busy -- or, on quit, once quit_ticks have passed (the host sets quit only
// after the published work ended: a pending task then is a fault, and the
// kernel still ends; busy workers finish their task first).
//
// The host publishes chunk c only after chunk c - cap has ended, so at most
// cap chunks are pending and a slot's descriptor is replaced only after every
// task of its previous chunk has read it.
__device__ void schedule(const ServedArgs &sa, unsigned char *lds) {
    const int t = static_cast<int>(threadIdx.x), nt = static_cast<int>(blockDim.x);
    const int lane = t & 63, wave = t >> 6, nwaves = (nt + 63) / 64;
    const int G = sa.grid;
    unsigned long long *s_assigned = reinterpret_cast<unsigned long long *>(lds);  // [G]: last value handed out
    int *s_ntasks = reinterpret_cast<int *>(s_assigned + kServedMaxWorkgroups);      // [kServedMaxRing]
    int *s_pref = s_ntasks + kServedMaxRing;  // [kServedMaxRing + 1]: exclusive prefix of the pending tasks
    int *s_wave = s_pref + kServedMaxRing + 1;  // [16]: per-wave totals
    __shared__ unsigned long long s_chunks, s_copied, s_next;
    __shared__ int s_next_wg, s_quit, s_pending, s_busy, s_handed, s_skip;
    for (int w = t; w < G; w += nt) s_assigned[w] = 1ull;  // a started, idle worker's mailbox reads 1
    if (t == 0) {
        // every chunk before s_next was handed out, and has ended, in an earlier launch
        s_next = ld_agent(sa.sched);
        s_copied = s_next;
        s_next_wg = 0;
        s_skip = 0;
        s_busy = 0;
        s_pending = 0;
    }
    __syncthreads();
    unsigned long long polls = 0, rounds_idle = 0, copies = 0;
    unsigned long long t_work = wall_clock64(), t_quit = 0;
    for (;;) {
        if (t == 0) {
            const unsigned long long pub =
                __hip_atomic_load(sa.published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            s_quit = __hip_atomic_load(sa.quit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            s_chunks = pub / static_cast<unsigned>(sa.tasks);
            ++polls;
            st_agent(sa.heartbeat, polls);
        }
        __syncthreads();
        // every shared value thread 0 rewrites at the top of a round is read
        // here, between that round's first and last barriers
        const unsigned long long chunks = s_chunks, copied = s_copied, next = s_next;
        const bool quit = s_quit != 0;
        // copy the new descriptors (the host wrote each before raising the
        // count): word w of chunk copied + c, all threads
        const int ncopy = static_cast<int>(chunks - copied);
        for (int i = t; i < ncopy * kWords; i += nt) {
            const int c = i / kWords, w = i - c * kWords;
            const int slot = static_cast<int>((copied + c) % static_cast<unsigned>(sa.cap));
            const uint32_t v = __hip_atomic_load(reinterpret_cast<const uint32_t *>(sa.ring + slot) + w,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(reinterpret_cast<uint32_t *>(sa.dring + slot) + w, v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            if (w == kNtasksWord) s_ntasks[slot] = static_cast<int>(v);
        }
        wait_memory();  // the copies are complete before any of their tasks is handed out
        copies += static_cast<unsigned long long>(ncopy);
        __syncthreads();
        if (t == 0) s_copied = chunks;
        // pending tasks: chunks [next, chunks), the first one from task s_next_wg
        const int P = static_cast<int>(chunks - next);  // <= cap <= kServedMaxRing <= nt
        // with nothing pending a round only watches the host's count: the
        // workers' mailboxes are read again every kScanEvery such rounds (the
        // busy count the idle exit needs)
        const bool scan = P > 0 || s_skip >= kScanEvery;
        int nh = 0;
        if (scan) {
            int rem = 0;
            if (t < P) {
                const int slot = static_cast<int>((next + t) % static_cast<unsigned>(sa.cap));
                rem = s_ntasks[slot] - (t == 0 ? s_next_wg : 0);
            }
            int incl = rem;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int o = __shfl_up(incl, d, 64);
                if (lane >= d) incl += o;
            }
            if (lane == 63) s_wave[wave] = incl;
            __syncthreads();
            int before = 0, total = 0;
            for (int w = 0; w < nwaves; ++w) {
                if (w < wave) before += s_wave[w];
                total += s_wave[w];
            }
            if (t < P) s_pref[t + 1] = before + incl;
            if (t == 0) s_pref[0] = 0;
            __syncthreads();
            // idle workers ranked in worker order: the k-th gets pending task k
            int rank_base = 0, busy = 0, handed = 0;
            for (int w0 = 1; w0 < G; w0 += nt) {
                const int w = w0 + t;
                bool idle = false;
                if (w < G) {
                    const unsigned long long dv = ld_agent(sa.mail_done + static_cast<size_t>(w) * kMailStride);
                    idle = dv == s_assigned[w];
                    // not started yet (its mailbox still zero, nothing handed to it): neither idle nor busy
                    busy += (idle || (dv == 0ull && s_assigned[w] == 1ull)) ? 0 : 1;
                }
                const unsigned long long mask = __ballot(idle);
                __syncthreads();  // every read of s_wave above is done
                if (lane == 0) s_wave[wave] = __popcll(mask);
                __syncthreads();
                int wb = 0, wt = 0;
                for (int v = 0; v < nwaves; ++v) {
                    wt += s_wave[v];
                    if (v < wave) wb += s_wave[v];
                }
                const int r = rank_base + wb + __popcll(mask & ((1ull << lane) - 1ull));
                if (idle && r < total) {
                    // pending task r: chunk j with s_pref[j] <= r < s_pref[j + 1]
                    int lo = 0, hi = P - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pref[mid] <= r)
                            lo = mid;
                        else
                            hi = mid - 1;
                    }
                    const int wg = (lo == 0 ? s_next_wg : 0) + (r - s_pref[lo]);
                    const unsigned long long task = (next + lo) * static_cast<unsigned>(sa.tasks) + wg;
                    s_assigned[w] = task + 2;
                    st_agent(sa.mail_assigned + static_cast<size_t>(w) * kMailStride, task + 2);
                    ++handed;
                }
                rank_base += wt;
            }
            // tasks handed out and workers busy, summed over the workgroup
            int h = handed, b = busy;
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) {
                h += __shfl_xor(h, d, 64);
                b += __shfl_xor(b, d, 64);
            }
            if (t == 0) {
                s_handed = 0;
                s_busy = 0;
            }
            __syncthreads();
            if (lane == 0) {
                atomicAdd(&s_handed, h);
                atomicAdd(&s_busy, b);
            }
            __syncthreads();
            nh = s_handed;
            if (t == 0) {
                // move past the tasks handed out
                if (nh >= total) {
                    s_next = chunks;
                    s_next_wg = 0;
                } else if (nh > 0) {
                    int lo = 0, hi = P - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (s_pref[mid] <= nh)
                            lo = mid;
                        else
                            hi = mid - 1;
                    }
                    s_next_wg = (lo == 0 ? s_next_wg : 0) + (nh - s_pref[lo]);
                    s_next = next + lo;
                }
                s_pending = total - nh;
            }
        }
        __syncthreads();
        const bool quiet = s_pending == 0 && s_busy == 0 && nh == 0;
        if (t == 0) s_skip = scan ? 0 : s_skip + 1;
        const unsigned long long now = wall_clock64();
        if (!quiet) t_work = now;
        if (quit && t_quit == 0) t_quit = now;
        if ((quiet && (quit || now - t_work > sa.idle_ticks)) || (quit && now - t_quit > sa.quit_ticks)) {
            for (int w = 1 + t; w < G; w += nt)
                st_agent(sa.mail_assigned + static_cast<size_t>(w) * kMailStride, kLeave);
            if (t == 0) {
                st_agent(sa.sched, s_next);
                add_stat(sa, 3, copies);
                add_stat(sa, 4, polls);
                add_stat(sa, 7, rounds_idle);
                wait_memory();
                __hip_atomic_fetch_add(sa.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                if (!quit) __hip_atomic_fetch_add(sa.status + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            return;
        }
        if (nh == 0) {
            ++rounds_idle;
            __builtin_amdgcn_s_sleep(4);
        }
    }
}

// The finalize of one integration in one workgroup (the served loop's worker),
// every tone of the integration at once and the phases kept in LDS.  The
// N-point DFT of the bins: for N a power of two, in the FP64 forms, a radix-2
// FFT (decimation in time, bins loaded in bit-reversed order, twiddles from
// the exact table: stage with half-length h uses tw[j N / 2h]), which needs
// O(N log N) operations where the direct sum needs N^2 -- one workgroup's FP64
// units take about 7 us for the direct sum at N = 512; otherwise the direct
// sum as finalize_body computes it (four partial sums over the quarters of the
// bins, added in quarter order), which also keeps the FP32 form's arithmetic
// that of the other paths.  Slot sums, unwrap and least-squares delay are
// finalize_body's.
__device__ void finalize_wg(const FinArgs &a, unsigned char *lds) {
    const int N = a.N, t = static_cast<int>(threadIdx.x), nt = static_cast<int>(blockDim.x);
    const int lane = t & 63, wave = t >> 6;
    const bool tw_lds = N <= kServedTwLdsTones;
    double2 *P = reinterpret_cast<double2 *>(lds);
    double2 *TW = tw_lds ? P + N : nullptr;
    // with the twiddles in LDS the results wait there too, for one pass of
    // writes to the (host) output at the end: one wait for their acknowledgement
    double2 *C = tw_lds ? P + 2 * N : nullptr;
    double *ph = reinterpret_cast<double *>(P + (tw_lds ? 3 * N : N));  // [N] phases
    double *sh = ph + N;  // [4] wave totals of the scan, [4] of the products
    const bool f32 = a.prec == 2;
    const bool fft = !f32 && tw_lds && N >= 2 && (N & (N - 1)) == 0;
    const int log2n = fft ? __builtin_ctz(static_cast<unsigned>(N)) : 0;
    {
        const double2 *acc = a.acc, *tw = a.tw;
        const float2 *accf = a.accf;
        for (int i = t; i < N; i += nt) {
            const int at = fft ? static_cast<int>(__brev(static_cast<unsigned>(i)) >> (32 - log2n)) : i;
            const double2 w = tw[i];  // issued with the slot loads
            P[at] = slot_sum(acc, accf, f32, N, i);
            if (tw_lds) TW[i] = w;
        }
    }
    __syncthreads();
    if (fft) {
        for (int h = 1; h < N; h <<= 1) {
            const int tw_step = N / (2 * h);
            for (int q = t; q < N / 2; q += nt) {
                const int j = q & (h - 1);
                const int i0 = ((q - j) << 1) + j, i1 = i0 + h;
                const double2 w = TW[j * tw_step];
                const double2 u = P[i0], v = P[i1];
                const double vr = v.x * w.x - v.y * w.y, vi = v.x * w.y + v.y * w.x;
                P[i0] = make_double2(u.x + vr, u.y + vi);
                P[i1] = make_double2(u.x - vr, u.y - vi);
            }
            __syncthreads();
        }
    }
    const int qn = (N + 3) / 4;
    for (int k = t; k < N; k += nt) {
        double part_re[4], part_im[4];
        if (fft) {  // the transform is in P: C_k = P[k] (partials unused)
            part_re[0] = P[k].x;
            part_im[0] = P[k].y;
            part_re[1] = part_re[2] = part_re[3] = 0.0;
            part_im[1] = part_im[2] = part_im[3] = 0.0;
        } else
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int bb = w * qn;
            const int be = (bb + qn) < N ? (bb + qn) : N;
            double re = 0.0, im = 0.0;
            if (bb < be) {
                int idx = static_cast<int>((static_cast<int64_t>(k) * bb) % N);
                if (f32) {
                    float fr = 0.f, fi = 0.f;
                    for (int b = bb; b < be; ++b) {
                        const double2 p = P[b];
                        const double2 w2 = tw_lds ? TW[idx] : a.tw[idx];
                        const float pr = static_cast<float>(p.x), pi = static_cast<float>(p.y);
                        const float wr = static_cast<float>(w2.x), wi = static_cast<float>(w2.y);
                        fr += pr * wr - pi * wi;
                        fi += pr * wi + pi * wr;
                        idx += k;
                        if (idx >= N) idx -= N;
                    }
                    re = fr;
                    im = fi;
                } else {
                    for (int b = bb; b < be; ++b) {
                        const double2 p = P[b];
                        const double2 w2 = tw_lds ? TW[idx] : a.tw[idx];
                        re += p.x * w2.x - p.y * w2.y;
                        im += p.x * w2.y + p.y * w2.x;
                        idx += k;
                        if (idx >= N) idx -= N;
                    }
                }
            }
            part_re[w] = re;
            part_im[w] = im;
        }
        double cr = 0.0, ci = 0.0;
        float fr = 0.f, fi = 0.f;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            if (f32) {
                fr += static_cast<float>(part_re[w]);
                fi += static_cast<float>(part_im[w]);
            } else {
                cr += part_re[w];
                ci += part_im[w];
            }
        }
        if (f32) {
            cr = fr;
            ci = fi;
        }
        {  // known gain of a rounded rotator table, divided out
            const double gr = cr * a.gain_re - ci * a.gain_im;
            ci = cr * a.gain_im + ci * a.gain_re;
            cr = gr;
        }
        if (a.sideband < 0) ci = -ci;
        const double phase = atan2(ci, cr);
        if (C) {
            C[k] = make_double2(cr, ci);
        } else {
            a.out[k] = sqrt(cr * cr + ci * ci) * a.inv_L;
            a.out[N + k] = phase;
            a.out[2 * N + k] = cr;
            a.out[3 * N + k] = ci;
        }
        ph[k] = phase;
    }
    __syncthreads();
    // delay: unwrap the in-band phases [k_lo, k_hi), fit phase = a + 2 pi t_d f
    // (the first 256 threads, as finalize_body)
    const bool me = t < 256;
    const int n = a.k_hi - a.k_lo;
    const double *php = ph + a.k_lo;
    const int seg = (n + 255) / 256;
    const int s0 = t * seg;
    const int s1 = (s0 + seg) < n ? (s0 + seg) : n;
    const double two_pi = 6.283185307179586476925286766559;
    double dsum = 0.0;
    for (int i = s0; me && i < s1; ++i) {
        if (i == 0) continue;
        const double d = php[i] - php[i - 1];
        dsum += d - two_pi * rint(d / two_pi);
    }
    double incl = dsum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (me && lane == 63) sh[wave] = incl;
    __syncthreads();
    double before = 0.0;
    for (int w = 0; w < wave && w < 4; ++w) before += sh[w];
    const double excl = before + incl - dsum;
    const double kbar = 0.5 * static_cast<double>(n - 1);
    double unw = (n > 0 ? php[0] : 0.0) + excl;
    double sxu = 0.0;
    for (int i = s0; me && i < s1; ++i) {
        if (i > 0) {
            const double d = php[i] - php[i - 1];
            unw += d - two_pi * rint(d / two_pi);
        }
        sxu += (static_cast<double>(i) - kbar) * unw;
    }
    // the sum of the products: a fixed shuffle tree in each of the four waves,
    // then the wave totals in wave order (sh[0..3] still hold the scan's)
    double v = me ? sxu : 0.0;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
    if (me && lane == 0) sh[4 + wave] = v;
    __syncthreads();
    if (t == 0) {
        double delay = 0.0;
        if (n >= 2) {
            const double dn = static_cast<double>(n);
            const double sxx = dn * (dn * dn - 1.0) / 12.0;
            const double sum = ((sh[4] + sh[5]) + sh[6]) + sh[7];
            delay = sum / sxx / a.f_comb / two_pi;
        }
        a.out[4 * N] = delay;
    }
    if (C) {  // each thread writes the tones it computed
        for (int k = t; k < N; k += nt) {
            const double2 c = C[k];
            a.out[k] = sqrt(c.x * c.x + c.y * c.y) * a.inv_L;
            a.out[N + k] = ph[k];
            a.out[2 * N + k] = c.x;
            a.out[3 * N + k] = c.y;
        }
    }
    if (a.clear) {
        // start the next integration in this bank: the accumulators the form
        // adds into (null: not used, still zero)
        for (int i = t; i < kAccSlots * N; i += nt) {
            if (a.acc_clear) a.acc_clear[i] = make_double2(0.0, 0.0);
            if (a.accf_clear) a.accf_clear[i] = make_float2(0.f, 0.f);
            if (a.acc_int_clear) a.acc_int_clear[i] = 0;
        }
    }
}

// Workgroups 1 .. grid - 1: wait on the own mailbox for a task (or the word to
// leave), fold the task into the stream's accumulator bank and count it; the
// task whose count completes an integration finalizes it and writes its
// completion record.  That task may belong to any chunk of the integration,
// and only the last chunk's descriptor carries the finalize: its tasks leave
// a copy per stream and bank in device memory before they count.  A worker
// may wait for a task as long as the scheduler lives (a worker of high index
// can stay idle long under partial load, and must still be there when handed
// a task); the scheduler always sends the word to leave before it ends, and a
// worker leaves on its own only once the scheduler's heartbeat has not moved
// for worker_ticks, so every wait is bounded.
template <int PREC>
__device__ void work(const ServedArgs &sa, unsigned char *lds) {
    __shared__ __align__(16) ServedDesc d;
    __shared__ __align__(16) FinArgs fa;
    __shared__ unsigned long long s_val, s_rec;
    __shared__ int s_fin;
    const int t = static_cast<int>(threadIdx.x);
    const size_t me = static_cast<size_t>(blockIdx.x) * kMailStride;
    unsigned long long last = 0ull, t_prev = wall_clock64();
    if (t == 0) st_agent(sa.mail_done + me, 1ull);  // started and idle
    for (;;) {
        if (t == 0) {
            unsigned long long v = ld_agent(sa.mail_assigned + me);
            unsigned long long t_beat = wall_clock64(), t_look = t_beat, beat = ld_agent(sa.heartbeat);
            while (v == last || v == 0ull) {
                const unsigned long long now = wall_clock64();
                if (now - t_look > sa.check_ticks) {
                    t_look = now;
                    const unsigned long long b = ld_agent(sa.heartbeat);
                    if (b != beat) {
                        beat = b;
                        t_beat = now;
                    } else if (now - t_beat > sa.worker_ticks) {
                        v = kLeave;  // no scheduler round for worker_ticks
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(8);
                v = ld_agent(sa.mail_assigned + me);
            }
            s_val = v;
        }
        __syncthreads();
        const unsigned long long val = s_val;
        if (val == kLeave) {
            if (t == 0) __hip_atomic_fetch_add(sa.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            return;
        }
        const unsigned long long t_claim = wall_clock64();
        const unsigned long long task = val - 2;
        const unsigned long long chunk = task / static_cast<unsigned>(sa.tasks);
        const int wg = static_cast<int>(task % static_cast<unsigned>(sa.tasks));
        const int slot = static_cast<int>(chunk % static_cast<unsigned>(sa.cap));
        uint32_t *dw = reinterpret_cast<uint32_t *>(&d);
        const uint32_t *src = reinterpret_cast<const uint32_t *>(sa.dring + slot);
        for (int i = t; i < kWords; i += static_cast<int>(blockDim.x))
            dw[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const unsigned long long t_desc = wall_clock64();
        if (d.fold.nbits == 2)
            fold_body<2, PREC>(d.fold, wg, lds);
        else
            fold_body<8, PREC>(d.fold, wg, lds);
        const int bank_ix = 2 * d.sid + d.bank;
        if (d.fin_total > 0) {  // the integration's last chunk: its finalize, for whichever task completes it
            uint32_t *dst = reinterpret_cast<uint32_t *>(sa.fin_args + bank_ix);
            const uint32_t *fw = reinterpret_cast<const uint32_t *>(&d.fin);
            for (int i = t; i < kFinWords; i += static_cast<int>(blockDim.x))
                __hip_atomic_store(dst + i, fw[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // every wave's atomics (and the copy above) are acknowledged before the task is counted
        wait_memory();
        __syncthreads();
        const unsigned long long t_fold = wall_clock64();
        if (t == 0) {
            // one atomic counts the task (low 32 bits) and, from the first
            // task of the integration's last chunk, brings the integration's
            // task total (high 32 bits): the task whose count makes the two
            // equal finalizes (the total is there by then: that first task has
            // counted).  The ring slot's count goes out beside it: the slot is
            // free for the host once every task of its chunk ended (their
            // reads of the slot are complete: the waits above).
            const unsigned long long add =
                1ull + (d.fin_total > 0 && wg == 0 ? static_cast<unsigned long long>(d.fin_total) << 32 : 0ull);
            const unsigned long long v =
                __hip_atomic_fetch_add(sa.task_done + bank_ix, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + add;
            const unsigned c = __hip_atomic_fetch_add(sa.slot_cnt + slot, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT) + 1u;
            const unsigned long long want = v >> 32;
            s_fin = (want != 0ull && (v & 0xffffffffull) == want) ? 1 : 0;
            // the finalizing task's completion record, claimed now
            unsigned long long rec = 0ull;
            if (s_fin) rec = atomicAdd(sa.done_cursor, 1ull);
            s_rec = rec;
            if (c == static_cast<unsigned>(d.ntasks)) {
                __hip_atomic_store(sa.slot_cnt + slot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                wait_memory();
                __hip_atomic_store(sa.slot_free + slot, chunk + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();
        if (s_fin) {
            // the whole integration is in the bank: finalize it here, every
            // part in turn (read, DFT, results into the stream's pinned slot,
            // clear the bank), then report it
            {
                const uint32_t *src_f = reinterpret_cast<const uint32_t *>(sa.fin_args + bank_ix);
                uint32_t *fw = reinterpret_cast<uint32_t *>(&fa);
                for (int i = t; i < kFinWords; i += static_cast<int>(blockDim.x))
                    fw[i] = __hip_atomic_load(src_f + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __syncthreads();
            const unsigned long long t_f0 = wall_clock64();
            finalize_wg(fa, lds);
            __syncthreads();
            wait_memory();
            __syncthreads();
            if (t == 0) {
                __hip_atomic_store(sa.task_done + bank_ix, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long k = s_rec;
                ServedDone *r = sa.done + k % static_cast<unsigned>(sa.done_cap);
                __hip_atomic_store(&r->sid, d.sid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&r->integ, d.integ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                // one release for all of it (results, cleared bank, counters,
                // the record's fields): the host reads seq, then the rest
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
                __hip_atomic_store(&r->seq, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                add_stat(sa, 5, 1ull);
                add_stat(sa, 12, wall_clock64() - t_f0);
            }
            __syncthreads();
        }
        if (t == 0) {
            wait_memory();
            st_agent(sa.mail_done + me, val);  // idle again
            const unsigned long long t_end = wall_clock64();
            add_stat(sa, 1, 1ull);
            add_stat(sa, 8, t_claim - t_prev);
            add_stat(sa, 9, t_desc - t_claim);
            add_stat(sa, 10, t_fold - t_desc);
            add_stat(sa, 11, t_end - t_fold);
            t_prev = t_end;
        }
        last = val;
    }
}

template <int PREC>
__global__ void __launch_bounds__(kServedThreads) served_kernel(ServedArgs sa) {
    extern __shared__ __align__(16) unsigned char lds[];
    if (blockIdx.x == 0)
        schedule(sa, lds);
    else
        work<PREC>(sa, lds);
}

}  // namespace

void launch_served(const ServedArgs &a, int prec, int grid, int threads, size_t lds, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL(served_kernel<0>, dim3(grid), dim3(threads), lds, s, a);
    else if (prec == 1)
        hipLaunchKernelGGL(served_kernel<1>, dim3(grid), dim3(threads), lds, s, a);
    else
        hipLaunchKernelGGL(served_kernel<2>, dim3(grid), dim3(threads), lds, s, a);
}

}  // namespace pcal
