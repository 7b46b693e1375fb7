// Host side of libpcal: parameter checks, planning of the fold geometry,
// FP64 rotator tables, device memory, stream ordering and the C ABI of pcal.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "pcal_host.h"

namespace pcal {
namespace host {

thread_local char g_last_error[256] = "";

void set_error(const char *what, hipError_t e) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
}

void set_message(const char *what) { snprintf(g_last_error, sizeof(g_last_error), "%s", what); }


int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a < 0 ? -a : a;
}

// lcm, or -1 on overflow past limit
int64_t lcm_capped(int64_t a, int64_t b, int64_t limit) {
    const int64_t g = gcd64(a, b);
    const int64_t q = a / g;
    if (q > limit / b) return -1;
    return q * b;
}

// exp(-j 2 pi num / den) for 0 <= num < den.  The angle a = 2 pi num / den is
// split exactly in integers as a = k pi/2 + x with |x| <= pi/4 (k the nearest
// quarter turn: 8 num = q den + r gives the octant q and the remainder r), so
// libm sees only |x| <= pi/4, quarter turns come out exact, and cos a, sin a
// follow from cos x, sin x by the quadrant k mod 4.
void phasor(int64_t num, int64_t den, double *re, double *im) {
    const unsigned __int128 n8 = static_cast<unsigned __int128>(num) * 8u;
    const int q = static_cast<int>(n8 / static_cast<uint64_t>(den));
    const int64_t r = static_cast<int64_t>(n8 % static_cast<uint64_t>(den));
    const double quarter_pi = 0.78539816339744830961566084581988;
    const double x = (q & 1) ? -quarter_pi * (static_cast<double>(den - r) / static_cast<double>(den))
                             : quarter_pi * (static_cast<double>(r) / static_cast<double>(den));
    const double cx = cos(x), sx = sin(x);
    double ca, sa;
    switch (((q + 1) / 2) & 3) {
        case 0: ca = cx; sa = sx; break;
        case 1: ca = -sx; sa = cx; break;
        case 2: ca = -cx; sa = -sx; break;
        default: ca = sx; sa = -cx; break;
    }
    *re = ca;
    *im = -sa;
}

// Tuning knobs (defaults chosen by measurement; environment overrides for sweeps).
int env_int(const char *name, int dflt) {
    const char *s = getenv(name);
    return (s && *s) ? atoi(s) : dflt;
}

int check_params(int64_t fs, int64_t fc, int64_t fo, int nbits, int sideband) {
    if (fs <= 0 || fc <= 0 || fs % fc) return PCAL_EINVAL;
    if (fo < 0 || fo >= fs) return PCAL_EINVAL;
    if (fs / fc > kMaxTones) return PCAL_EINVAL;
    if (nbits != 2 && nbits != 8) return PCAL_EINVAL;
    if (sideband != 1 && sideband != -1) return PCAL_EINVAL;
    return PCAL_OK;
}

// Fold geometry.  One tile holds the whole period when it fits the LDS
// position budget: then a row is k periods long and the workgroup size is
// picked to waste the fewest lanes.  Otherwise a row is one period, split
// into equal column tiles of at most the budget.  Among workgroup sizes that
// waste equally few lanes, the one nearest aim_threads is taken (0: the
// smallest); sizes below min_threads are not considered unless none fits.
FoldGeom plan_geom(int64_t Sp, int spv, int64_t max_positions, int max_threads, int force_threads,
                   int min_threads, int aim_threads) {
    FoldGeom g{};
    g.spv = spv;
    const int64_t W = Sp / g.spv;  // vectors per period
    g.period_vecs = static_cast<int>(W);
    const int pref = force_threads ? force_threads : env_int("PCAL_FOLD_THREADS", 0);
    // columns of one period per workgroup: the whole period when it fits the
    // LDS position budget and the workgroup, else equal tiles within both
    // (split tiles are whole 128-byte lines wide: 8 vectors)
    int64_t tile = W;
    if (Sp > max_positions || W > max_threads) {
        const int64_t tile_max = std::min<int64_t>(max_threads, max_positions / g.spv) / 8 * 8;
        const int64_t tiles = (W + tile_max - 1) / tile_max;
        tile = ((W + tiles - 1) / tiles + 7) / 8 * 8;
    }
    g.tile_vecs = static_cast<int>(tile);
    g.col_tiles = static_cast<int>((W + tile - 1) / tile);
    g.pos_cols = g.tile_vecs;
    g.npos = static_cast<int>(tile * g.spv);
    // workgroup size: k sub-rows of one tile each, wasting the fewest lanes
    int best_t = 0;
    double best = -1.0;
    for (int t = pref ? pref : std::min(min_threads, max_threads) / 64 * 64; t <= max_threads; t += 64) {
        if (pref && t != pref) continue;
        const int64_t k = t / tile;
        if (k < 1) continue;
        const double eff = static_cast<double>(k * tile) / t;
        const bool nearer = aim_threads > 0 && std::abs(t - aim_threads) < std::abs(best_t - aim_threads);
        if (eff > best + 1e-9 || (eff > best - 1e-9 && nearer)) {
            best = eff;
            best_t = t;
        }
    }
    if (best_t == 0) best_t = static_cast<int>(((tile + 63) / 64) * 64);
    const int64_t k = std::max<int64_t>(1, best_t / tile);
    g.threads = best_t;
    g.row_vecs = static_cast<int>(k * W);
    return g;
}

int make_plan(int64_t fs, int64_t fc, int64_t fo, int nbits, int sideband, int method, int prec, Plan *p,
              int force_threads) {
    int rc = check_params(fs, fc, fo, nbits, sideband);
    if (rc) return rc;
    if (method < PCAL_METHOD_AUTO || method > PCAL_METHOD_DFR_EF) return PCAL_EINVAL;
    if (prec < PCAL_PREC_F64 || prec > PCAL_PREC_Q17) return PCAL_EINVAL;
    p->fs = fs;
    p->fc = fc;
    p->fo = fo;
    p->nbits = nbits;
    p->sideband = sideband;
    p->prec = kernel_prec(prec);
    p->prec_api = prec;
    p->N = fs / fc;
    p->R = fs / gcd64(fs, fo);  // Eq. 4 (gcd(fs, 0) = fs gives R = 1)
    p->S = lcm_capped(p->N, p->R, kMaxFoldPeriod);
    p->Sp = p->S > 0 ? lcm_capped(p->S, spv_of(nbits), kMaxFoldPeriod) : -1;
    // A fold period of fewer than 64 vectors puts several lanes of a wave on
    // the same period positions, and their flushes to LDS collide (64 lanes on
    // one address at one vector per period).  Any multiple of the period folds
    // the same (rotator and bins repeat with it), so a short period is widened
    // to the first multiple of at least 64 vectors.
    if (p->Sp > 0 && p->Sp < 64 * spv_of(nbits)) {
        const int64_t W = p->Sp / spv_of(nbits);
        p->Sp *= (64 + W - 1) / W;
    }
    p->M = p->Sp > 0 ? p->Sp / p->N : -1;
    p->tab_rows = prec == PCAL_PREC_Q17 ? p->R : p->M;
    const bool fold_ok = p->Sp > 0 && p->M <= kMaxTableRows;
    const bool osc_ok = fs < (int64_t(1) << 32);
    // The fold pays off while a launch spans many fold periods; for long periods
    // (offsets sharing few factors with fs, Section 6) AUTO takes the recurrence.
    const bool auto_method = method == PCAL_METHOD_AUTO;
    if (auto_method)
        method = (fold_ok && p->Sp <= kAutoFoldPeriod) ? PCAL_METHOD_PERIOD_FOLD : PCAL_METHOD_OSC;
    // the fixed-point form is a period-fold form (any fold period that fits)
    if (prec == PCAL_PREC_Q17) {
        if (auto_method) method = PCAL_METHOD_PERIOD_FOLD;
        if (method != PCAL_METHOD_PERIOD_FOLD) return PCAL_ENOTSUP;
    }
    if (method == PCAL_METHOD_PERIOD_FOLD && !fold_ok) return PCAL_ENOTSUP;
    if (method == PCAL_METHOD_LUT && (p->R > kMaxLutPeriod || !osc_ok)) return PCAL_ENOTSUP;
    const bool recurrence = method == PCAL_METHOD_OSC || method == PCAL_METHOD_CFO || method == PCAL_METHOD_MCO ||
                            method == PCAL_METHOD_DFR_EF;
    if (recurrence && !osc_ok) return PCAL_ENOTSUP;
    p->method = method;
    if (method == PCAL_METHOD_PERIOD_FOLD) {
        p->geom = plan_geom(p->Sp, spv_of(nbits), kMaxLdsPositions, kMaxFoldThreads, force_threads,
                            kMinFoldThreads, kAimFoldThreads);
        if (p->geom.col_tiles > kSmallTileWgTiles && !force_threads && env_int("PCAL_FOLD_THREADS", 0) == 0) {
            // More column tiles than the larger workgroups have resident slots
            // (one per compute unit): one row of a tile per workgroup (the
            // smallest workgroup that covers a tile), so that all tiles, each
            // ending with an epilogue of its own, run at once (measured at
            // 2-bit, fold period 8e6, 625 tiles of 200 vectors: 256 threads 53
            // us per 2^30 samples against 62 us with 640; period 64e6, 5000
            // tiles: 104 against 160 us).  With fewer tiles the larger
            // workgroups win (2-8 tiles: 48-50 us against 52-71 us): the
            // smaller ones split each tile over more workgroups, each adding
            // an epilogue over the whole tile.
            p->geom = plan_geom(p->Sp, spv_of(nbits), kMaxLdsPositions, kMaxFoldThreads,
                                (p->geom.tile_vecs + 63) / 64 * 64, kMinFoldThreads, kAimFoldThreads);
        }
    } else {
        // rows of a multiple of lcm(N, 16) samples: every lane keeps its bin
        const int64_t per = p->N / gcd64(p->N, kRotLanes) * kRotLanes;
        p->geom = plan_geom(per, kRotLanes, INT64_MAX, kMaxRotThreads, force_threads, 256, 0);
        if (recurrence && !force_threads && env_int("PCAL_FOLD_THREADS", 0) == 0) {
            // The resonator steps once per row by d = w_o * (samples per row) with
            // the coefficient 2 cos d rounded to the form's precision; the
            // frequency that rounding leaves is off by about delta / (2 |sin d|),
            // so a d near 0 or pi makes the recurrence drift (Section 2.2 notes the
            // resonator's loss of accuracy at low steps); the magic circle's
            // read-out divides by cos(d / 2), small near d = pi.  Every recurrence
            // form takes the same row choice.  Rows hold k periods of
            // lcm(N, 16) samples, k the workgroup's sub-rows: among the workgroup
            // sizes that waste no more lanes, take the k whose d is farthest from
            // 0 and pi (|sin d| >= 0.2 counts as far enough: the FP32 coefficient
            // then moves the frequency by at most 1.5e-7 rad per row, 1e-5 rad over
            // a 64-row run between exact re-seeds), then the smallest workgroup.
            const FoldGeom &g0 = p->geom;
            int best_t = g0.threads;
            double best_s = -1.0, best_eff = -1.0;
            for (int t = 256; t <= kMaxRotThreads; t += 64) {
                const int64_t k = t / g0.tile_vecs;
                if (k < 1) continue;
                const double eff = static_cast<double>(k * g0.tile_vecs) / t;
                const int64_t di = static_cast<int64_t>((static_cast<unsigned __int128>(fo) * (k * per)) % fs);
                double c, sn;
                phasor(di, fs, &c, &sn);
                const double sc = std::min(std::fabs(sn), 0.2);
                if (sc > best_s + 1e-12 || (sc > best_s - 1e-12 && eff > best_eff + 1e-9)) {
                    best_s = sc;
                    best_eff = eff;
                    best_t = t;
                }
            }
            p->geom.threads = best_t;
            p->geom.row_vecs = static_cast<int>((best_t / g0.tile_vecs) * g0.period_vecs);
            p->osc_sin = best_s;
            // Even the best row length leaves d near 0 or pi: AUTO takes the
            // coupled form instead, whose rounding does not depend on d, unless
            // the recurrence runs in FP64 (its coefficient error is 2^-29 of FP32's).
            if (auto_method && best_s < 0.1 && prec != PCAL_PREC_F64) method = PCAL_METHOD_CFO;
            p->method = method;
        }
    }
    {
        const int sp = env_int("PCAL_SYNC_PAIRS", kSyncPairs);  // power of two or 0
        p->sync_pairs = (sp > 0 && (sp & (sp - 1)) == 0) ? sp : 0;
    }
    p->target_blocks = env_int("PCAL_TARGET_BLOCKS", 0);
    p->target_from_env = p->target_blocks > 0;
    if (!p->target_from_env)
        p->target_blocks = (method == PCAL_METHOD_PERIOD_FOLD || nbits == 2) ? kTargetBlocks
                           : method == PCAL_METHOD_LUT                    ? kLutTargetBlocks8
                                                                          : kRotTargetBlocks8;
    p->max_blocks = std::max(p->geom.col_tiles, p->target_blocks) + p->geom.col_tiles;
    return PCAL_OK;
}

// Launch geometry of one extract call.
pcal_launch_t plan_launch(const Plan &p, uint64_t addr, int64_t n_before, int64_t nsamples, int target_blocks) {
    const FoldGeom &g = p.geom;
    const int spb = 8 / p.nbits;
    pcal_launch_t L{};
    const int64_t nbytes = nsamples / spb;
    const int64_t vb = static_cast<int64_t>(g.spv) / spb;  // bytes per thread-vector (16 or 4)
    int64_t head = static_cast<int64_t>((vb - static_cast<int64_t>(addr % vb)) % vb);
    if (head > nbytes) head = nbytes;
    L.head_bytes = head;
    L.nvec = (nbytes - head) / vb;
    L.tail_bytes = nbytes - head - vb * L.nvec;
    const int64_t g0 = n_before + head * spb;  // global index of the first full-vector sample
    L.rows_total = (L.nvec + g.row_vecs - 1) / g.row_vecs;
    const int64_t groups_want = std::max<int64_t>(1, (target_blocks ? target_blocks : p.target_blocks) / g.col_tiles);
    const int64_t groups = std::max<int64_t>(1, std::min<int64_t>(groups_want, L.rows_total));
    if (p.method == PCAL_METHOD_PERIOD_FOLD) {
        // The full rows in groups of whole walker groups (5 rows at 2-bit, 4 at
        // 8-bit), split as evenly as groups allow over the workgroups of a tile;
        // the rows after the last group go to the first workgroup of each tile.
        const int64_t unit = p.nbits == 2 ? 5 : 4;
        const int64_t wgroups = L.nvec / g.row_vecs / unit;  // whole walker groups of full rows
        const int64_t fgroups = std::max<int64_t>(1, std::min<int64_t>(groups, wgroups));
        L.grid = fgroups * g.col_tiles;
        L.groups_per_wg = wgroups / fgroups;
        L.extra_groups = wgroups % fgroups;
        L.odd_start = wgroups * unit;
        L.rows_per_group = unit * (L.groups_per_wg + (L.extra_groups ? 1 : 0));
    } else {
        L.rows_per_group = L.rows_total > 0 ? (L.rows_total + groups - 1) / groups : 1;
        const int64_t ngroups = L.rows_total > 0 ? (L.rows_total + L.rows_per_group - 1) / L.rows_per_group : 1;
        L.grid = ngroups * g.col_tiles;
        L.groups_per_wg = 0;
        L.extra_groups = 0;
        L.odd_start = L.rows_total;
    }
    L.threads = g.threads;
    if (p.method == PCAL_METHOD_PERIOD_FOLD) {
        L.lds_bytes = static_cast<int64_t>(fold_lds_bytes(g.npos, g.spv, g.threads, p.tab_rows));
        L.q0 = g0 % p.Sp;
        L.head_q = n_before % p.Sp;
        L.tail_q = (g0 + L.nvec * g.spv) % p.Sp;
    } else {
        L.lds_bytes = static_cast<int64_t>(sizeof(double2)) * p.N;
        L.q0 = g0;
        L.head_q = n_before;
        L.tail_q = g0 + L.nvec * g.spv;
    }
    return L;
}

// Device bytes a handle of this plan allocates (build() below), computed
// without allocating: what admission under a memory budget compares.
int64_t plan_device_bytes(const Plan &p) {
    const bool fold = p.method == PCAL_METHOD_PERIOD_FOLD;
    const int64_t N = p.N, M = fold ? p.M : 1, NS = 2 * kAccSlots * N;
    auto b = [](int64_t size, int64_t count) { return size * (count ? count : 1); };
    int64_t bytes = b(16, M) + b(8, M) + b(4, 2 * M)          // u64, u32, u16 (two terms)
                    + b(16, N) + b(16, N)                     // v, tw
                    + b(16, NS) + b(8, NS) + b(8, NS)         // acc, acc_int, accf (two banks)
                    + b(4, 2) + b(8, 2 * (4 * N + 1))         // counters, out
                    + b(8, N) + b(8, 3 * N + 4) + b(8, N)     // phases, pulse, pulse_int
                    + b(8, kMaxRefinePasses + 3);             // refine_out
    if (fold && p.prec_api == PCAL_PREC_Q17) bytes += b(8, p.R);  // Q17 rotator
    if (!fold) {
        bytes += b(16, kRotLanes);                            // lane factors
        if (p.method == PCAL_METHOD_LUT)
            bytes += p.prec == PCAL_PREC_F64 ? b(16, p.R) : p.prec == PCAL_PREC_MIXED ? b(4, 2 * p.R) : b(8, p.R);
    }
    return bytes;
}

void fill_info(const Plan &p, pcal_info_t *info) {
    memset(info, 0, sizeof(*info));
    info->ntones = p.N;
    info->rotator_period = p.R;
    info->joint_period = p.S;
    info->fold_period = p.Sp;
    info->method = p.method;
    info->precision = p.prec_api;
    info->block_threads = p.geom.threads;
    info->row_vectors = p.geom.row_vecs;
    info->col_tiles = p.geom.col_tiles;
    info->lds_positions = p.geom.npos;
    info->period_vectors = p.geom.period_vecs;
    info->tile_vectors = p.geom.tile_vecs;
    info->target_blocks = p.target_blocks;
    info->device_bytes = plan_device_bytes(p);
}


template <typename T>
int dalloc(pcal_ctx *h, T **p, size_t count) {
    const size_t bytes = sizeof(T) * (count ? count : 1);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), bytes);
    if (e != hipSuccess) {
        set_error("hipMalloc", e);
        return e == hipErrorOutOfMemory ? PCAL_ENOMEM : PCAL_EHIP;
    }
    h->device_bytes += bytes;
    return PCAL_OK;
}

void release(pcal_ctx *h) {
    if (h->twin) release(h->twin);
    void *lane[] = {h->acc_mem, h->acc_int_mem, h->accf_mem, h->counters, h->out, h->phases, h->pulse, h->pulse_int,
                    h->refine_out};
    for (void *p : lane)
        if (p) (void)hipFree(p);
    if (!h->shares_tables) {
        void *tables[] = {h->u64, h->u32, h->u16, h->v, h->tw, h->rot64, h->rot32, h->rot16, h->w, h->uq};
        for (void *p : tables)
            if (p) (void)hipFree(p);
    }
    if (h->host_out) (void)hipHostFree(h->host_out);
    if (h->ev) (void)hipEventDestroy(h->ev);
    delete h;
}

void set_bank(pcal_ctx *h, int b) {
    const size_t NS = static_cast<size_t>(kAccSlots) * static_cast<size_t>(h->plan.N);
    h->bank = b;
    h->acc = h->acc_mem + b * NS;
    h->acc_int = h->acc_int_mem + b * NS;
    h->accf = h->accf_mem + b * NS;
}

int flush_pending(pcal_ctx *h, hipStream_t s) {
    if (!h->fin_pending) return PCAL_OK;
    h->fin_pending = false;
    launch_finalize(h->fin, s);
    PCAL_HIP(hipGetLastError());
    if (h->fin_dev)
        PCAL_HIP(hipMemcpyAsync(h->fin_host, h->fin_dev, sizeof(double) * (4 * h->plan.N + 1),
                                hipMemcpyDeviceToHost, s));
    return PCAL_OK;
}

// Device address of a host result buffer the finalize may write directly
// (pinned, mapped host memory of 4N + 1 doubles), or null.  Queried on every
// call (once per integration): a cached answer could outlive the buffer, and a
// pageable buffer later at the same address must not be written by the GPU.
double *mapped_results(pcal_ctx *h, double *host) {
    (void)h;
    void *dev = nullptr;
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, host) != hipSuccess || at.type != hipMemoryTypeHost ||
        hipHostGetDevicePointer(&dev, host, 0) != hipSuccess)
        dev = nullptr;
    (void)hipGetLastError();  // a refused query leaves no error behind
    return static_cast<double *>(dev);
}

// Mean rounding gain gamma = mean over k of conj(t[k]) * (t_rounded[k] - t[k]) of a
// rotator table: every tone's response is scaled by 1 + gamma when the table is
// used rounded, so 1 / (1 + gamma) restores it (returned as re, im).
double2 from_half2(__half2 h) {
    _Float16 hx, hy;
    memcpy(&hx, reinterpret_cast<const char *>(&h), 2);
    memcpy(&hy, reinterpret_cast<const char *>(&h) + 2, 2);
    return make_double2(static_cast<double>(hx), static_cast<double>(hy));
}

void table_gain(const std::vector<double2> &t, const std::vector<double2> &tr, double *re, double *im) {
    double gr = 0.0, gi = 0.0;
    for (size_t m = 0; m < t.size(); ++m) {
        const double dr = tr[m].x - t[m].x, di = tr[m].y - t[m].y;
        gr += t[m].x * dr + t[m].y * di;
        gi += t[m].x * di - t[m].y * dr;
    }
    gr /= static_cast<double>(t.size());
    gi /= static_cast<double>(t.size());
    const double den = (1.0 + gr) * (1.0 + gr) + gi * gi;
    *re = (1.0 + gr) / den;
    *im = -gi / den;
}

__half2 to_half2(double2 v) {
    __half2 r;
    const _Float16 hx = static_cast<_Float16>(v.x), hy = static_cast<_Float16>(v.y);
    memcpy(reinterpret_cast<char *>(&r), &hx, 2);
    memcpy(reinterpret_cast<char *>(&r) + 2, &hy, 2);
    return r;
}

int build(pcal_ctx *h) {
    const Plan &p = h->plan;
    const bool fold = p.method == PCAL_METHOD_PERIOD_FOLD;
    const int64_t N = p.N, M = fold ? p.M : 1;
    int rc;
    if (!fold) {
        // per-sample forms: lane factors, recurrence step, rotator table
        const int64_t dn = static_cast<int64_t>(p.geom.row_vecs) * p.geom.spv;  // samples per row
        std::vector<double2> w(kRotLanes);
        for (int i = 0; i < kRotLanes; ++i)
            phasor(static_cast<int64_t>((static_cast<unsigned __int128>(p.fo) * i) % p.fs), p.fs, &w[i].x, &w[i].y);
        double br, bi;
        const int64_t di = static_cast<int64_t>((static_cast<unsigned __int128>(p.fo) * dn) % p.fs);
        phasor(di, p.fs, &br, &bi);
        h->back = make_double2(br, -bi);
        h->c2 = 2.0 * br;
        // half the row step (rows are an even number of samples), for the magic circle
        double hr, hi;
        phasor(static_cast<int64_t>((static_cast<unsigned __int128>(p.fo) * (dn / 2)) % p.fs), p.fs, &hr, &hi);
        h->half_cos = hr;
        h->half_sin = -hi;
        if ((rc = dalloc(h, &h->w, kRotLanes))) return rc;
        PCAL_HIP(hipMemcpy(h->w, w.data(), sizeof(double2) * kRotLanes, hipMemcpyHostToDevice));
        if (p.method == PCAL_METHOD_LUT) {
            // One rotator period from exact integer phase indices (Eq. 4-5), in
            // FP64, then in the form's storage: FP64, two FP16 terms (hi = the
            // rounded entry, lo = the rounded rest; hi + lo is exact in FP32,
            // about 22 bits) or FP32.
            const int64_t R = p.R;
            std::vector<double2> t(R);
            int64_t idx = 0;
            for (int64_t n = 0; n < R; ++n) {
                phasor(idx, p.fs, &t[n].x, &t[n].y);
                idx += p.fo;
                if (idx >= p.fs) idx -= p.fs;
            }
            // de-interleaved by D (the largest power of two <= 16 dividing R):
            // entry n at (n mod D) * (R / D) + n / D, so that the lookups of
            // lanes 16 entries apart fall on neighbouring addresses
            int shift = 0;
            while (shift < 4 && R % (int64_t(2) << shift) == 0) ++shift;
            h->lut_shift = shift;
            h->lut_rows = R >> shift;
            auto slot = [&](int64_t n) { return (n & ((int64_t(1) << shift) - 1)) * h->lut_rows + (n >> shift); };
            if (p.prec == PCAL_PREC_F64) {
                std::vector<double2> td(R);
                for (int64_t n = 0; n < R; ++n) td[slot(n)] = t[n];
                if ((rc = dalloc(h, &h->rot64, R))) return rc;
                PCAL_HIP(hipMemcpy(h->rot64, td.data(), sizeof(double2) * R, hipMemcpyHostToDevice));
            } else if (p.prec == PCAL_PREC_MIXED) {
                // (the single-FP16 form keeps only the rounded entry, lo = 0, and
                // divides no gain out)
                const bool single16 = p.prec_api == PCAL_PREC_F16;
                std::vector<__half2> thd(2 * R);
                std::vector<double2> tr(R);
                for (int64_t n = 0; n < R; ++n) {
                    const __half2 hi = to_half2(t[n]);
                    const double2 h0 = from_half2(hi);
                    const __half2 lo = to_half2(single16 ? make_double2(0.0, 0.0)
                                                         : make_double2(t[n].x - h0.x, t[n].y - h0.y));
                    const double2 l0 = from_half2(lo);
                    tr[n] = make_double2(h0.x + l0.x, h0.y + l0.y);
                    thd[2 * slot(n)] = hi;
                    thd[2 * slot(n) + 1] = lo;
                }
                if (!single16) table_gain(t, tr, &h->gain_re, &h->gain_im);
                if ((rc = dalloc(h, &h->rot16, 2 * R))) return rc;
                PCAL_HIP(hipMemcpy(h->rot16, thd.data(), sizeof(__half2) * 2 * R, hipMemcpyHostToDevice));
            } else {
                std::vector<float2> tfd(R);
                for (int64_t n = 0; n < R; ++n)
                    tfd[slot(n)] = make_float2(static_cast<float>(t[n].x), static_cast<float>(t[n].y));
                if ((rc = dalloc(h, &h->rot32, R))) return rc;
                PCAL_HIP(hipMemcpy(h->rot32, tfd.data(), sizeof(float2) * R, hipMemcpyHostToDevice));
            }
        }
    }
    if ((rc = dalloc(h, &h->u64, M)) || (rc = dalloc(h, &h->u32, M)) || (rc = dalloc(h, &h->u16, 2 * M)) ||
        (rc = dalloc(h, &h->v, N)) || (rc = dalloc(h, &h->tw, N)) || (rc = alloc_lane(h)))
        return rc;
    // Rotator factors from exact integer phase indices, in FP64 (Eq. 3-5):
    //   u[m] = exp(-j 2 pi (f_o N m mod fs) / fs),  v[b] = exp(-j 2 pi (f_o b mod fs) / fs),
    //   tw[j] = exp(-j 2 pi j / N)  (DFT twiddles).
    std::vector<double2> u(M), v(N), tw(N);
    std::vector<float2> uf(M);
    std::vector<__half2> uh(2 * M);  // two-term FP16 rows: u ~ hi + lo
    std::vector<double2> ur(M);        // hi + lo, exactly
    const int64_t step_u = static_cast<int64_t>((static_cast<unsigned __int128>(p.fo) * N) % p.fs);
    int64_t idx = 0;
    for (int64_t m = 0; m < M; ++m) {
        phasor(idx, p.fs, &u[m].x, &u[m].y);
        uf[m] = make_float2(static_cast<float>(u[m].x), static_cast<float>(u[m].y));
        uh[2 * m] = to_half2(u[m]);
        const double2 hi = from_half2(uh[2 * m]);
        uh[2 * m + 1] = to_half2(p.prec_api == PCAL_PREC_F16 ? make_double2(0.0, 0.0)
                                                             : make_double2(u[m].x - hi.x, u[m].y - hi.y));
        const double2 lo = from_half2(uh[2 * m + 1]);
        ur[m] = make_double2(hi.x + lo.x, hi.y + lo.y);
        idx += step_u;
        if (idx >= p.fs) idx -= p.fs;
    }
    idx = 0;
    for (int64_t b = 0; b < N; ++b) {
        phasor(idx, p.fs, &v[b].x, &v[b].y);
        idx += p.fo;
        if (idx >= p.fs) idx -= p.fs;
        phasor(b, N, &tw[b].x, &tw[b].y);
    }
    // Mixed form: each row is stored as two FP16 terms hi + lo (hi = u rounded,
    // lo = the rest rounded; their sum is exact in FP32, about 22 bits).  The
    // rounded rows change every tone's response by the same known complex gain
    // 1 + gamma, gamma = mean over m of conj(u[m]) * (u16[m] - u[m]) (the rows
    // sum against conj(u[m]) for every tone); the FP64 finalize divides it out.
    // The single-FP16 form (PCAL_PREC_F16) keeps hi alone and divides no gain out.
    if (fold && p.prec_api == PCAL_PREC_MIXED) table_gain(u, ur, &h->gain_re, &h->gain_im);
    if (fold && p.prec_api == PCAL_PREC_Q17) {
        // fixed-point rotator of one period: exp(-j 2 pi (f_o r mod fs) / fs) * 2^17,
        // each part rounded to the nearest integer (ties to even); the bins then
        // hold integers times 2^17, which the finalize scales back
        std::vector<int2> q(p.R);
        int64_t iq = 0;
        for (int64_t r = 0; r < p.R; ++r) {
            double re, im;
            phasor(iq, p.fs, &re, &im);
            q[r] = make_int2(static_cast<int>(nearbyint(kFixedScale * re)), static_cast<int>(nearbyint(kFixedScale * im)));
            iq += p.fo;
            if (iq >= p.fs) iq -= p.fs;
        }
        if ((rc = dalloc(h, &h->uq, p.R))) return rc;
        PCAL_HIP(hipMemcpy(h->uq, q.data(), sizeof(int2) * p.R, hipMemcpyHostToDevice));
        h->gain_re = 1.0 / kFixedScale;
        h->gain_im = 0.0;
    }
    PCAL_HIP(hipMemcpy(h->u64, u.data(), sizeof(double2) * M, hipMemcpyHostToDevice));
    PCAL_HIP(hipMemcpy(h->u32, uf.data(), sizeof(float2) * M, hipMemcpyHostToDevice));
    PCAL_HIP(hipMemcpy(h->u16, uh.data(), sizeof(__half2) * 2 * M, hipMemcpyHostToDevice));
    PCAL_HIP(hipMemcpy(h->v, v.data(), sizeof(double2) * N, hipMemcpyHostToDevice));
    PCAL_HIP(hipMemcpy(h->tw, tw.data(), sizeof(double2) * N, hipMemcpyHostToDevice));
    return clear_lane(h);
}

// A lane's own device memory: the accumulators of its two banks, finalize
// counters and results, readout buffers, and its pinned result copy.
int alloc_lane(pcal_ctx *h) {
    const int64_t N = h->plan.N;
    int rc;
    if ((rc = dalloc(h, &h->acc_mem, 2 * kAccSlots * N)) || (rc = dalloc(h, &h->acc_int_mem, 2 * kAccSlots * N)) ||
        (rc = dalloc(h, &h->accf_mem, 2 * kAccSlots * N)) || (rc = dalloc(h, &h->counters, 2)) ||
        (rc = dalloc(h, &h->out, 2 * (4 * N + 1))) || (rc = dalloc(h, &h->phases, N)) ||
        (rc = dalloc(h, &h->pulse, 3 * N + 4)) || (rc = dalloc(h, &h->pulse_int, N)) ||
        (rc = dalloc(h, &h->refine_out, kMaxRefinePasses + 3)))
        return rc;
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&h->host_out), sizeof(double) * (4 * N + 1),
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
        set_error("hipHostMalloc", e);
        return PCAL_ENOMEM;
    }
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, h->host_out, 0) == hipSuccess)
        h->host_out_dev = static_cast<double *>(d);
    else
        (void)hipGetLastError();  // not mapped: results go through a device copy
    return PCAL_OK;
}

// Zeroed accumulators and counters, bank 0, and the lane's event.
int clear_lane(pcal_ctx *h) {
    const size_t N = static_cast<size_t>(h->plan.N);
    PCAL_HIP(hipMemset(h->acc_mem, 0, sizeof(double2) * 2 * kAccSlots * N));
    PCAL_HIP(hipMemset(h->acc_int_mem, 0, sizeof(long long) * 2 * kAccSlots * N));
    PCAL_HIP(hipMemset(h->accf_mem, 0, sizeof(float2) * 2 * kAccSlots * N));
    PCAL_HIP(hipMemset(h->counters, 0, 2 * sizeof(unsigned)));
    set_bank(h, 0);
    PCAL_HIP(hipEventCreateWithFlags(&h->ev, hipEventDisableTiming));
    return PCAL_OK;
}

// The second lane of a handle (pipelined integrations): a copy of the
// primary's plan, tables and scalars with lane state of its own.
int make_twin(pcal_ctx *h) {
    pcal_ctx *t = new (std::nothrow) pcal_ctx();
    if (!t) return PCAL_ENOMEM;
    *t = *h;
    t->acc_mem = nullptr;
    t->acc_int_mem = nullptr;
    t->accf_mem = nullptr;
    t->acc = nullptr;
    t->acc_int = nullptr;
    t->accf = nullptr;
    t->counters = nullptr;
    t->out = nullptr;
    t->phases = nullptr;
    t->pulse = nullptr;
    t->pulse_int = nullptr;
    t->refine_out = nullptr;
    t->host_out = nullptr;
    t->host_out_dev = nullptr;
    t->ev = nullptr;
    t->wait_ev = nullptr;
    t->have_ev = false;
    t->dirty = false;
    t->last_stream = nullptr;
    t->fin_pending = false;
    t->n_integ = 0;
    t->device_bytes = 0;
    t->twin = nullptr;
    t->on_twin = false;
    t->shares_tables = true;
    int rc = alloc_lane(t);
    if (!rc) rc = clear_lane(t);
    if (rc) {
        release(t);
        return rc;
    }
    h->device_bytes += t->device_bytes;
    h->twin = t;
    return PCAL_OK;
}

// An event for the handle's last work: recorded now on its last stream when
// work was enqueued there since the previous record.  Recorded only when
// needed (a switch of stream, a synchronisation), because an event record
// between two dependent launches costs the stream ~3-4 us.
int settle(pcal_ctx *h) {
    if (!h->dirty) return PCAL_OK;
    PCAL_HIP(hipEventRecord(h->ev, h->last_stream));
    h->wait_ev = h->ev;
    h->have_ev = true;
    h->dirty = false;
    return PCAL_OK;
}

// Order work on `s` after the handle's previous work (possibly on another stream).
int order_on(pcal_ctx *h, hipStream_t s, bool flush) {
    if (s != h->last_stream && (h->dirty || h->have_ev)) {
        const int rc = settle(h);
        if (rc) return rc;
        PCAL_HIP(hipStreamWaitEvent(s, h->wait_ev, 0));
    }
    return flush ? flush_pending(h, s) : PCAL_OK;
}

int mark(pcal_ctx *h, hipStream_t s) {
    h->last_stream = s;
    h->dirty = true;
    return PCAL_OK;
}



FinArgs fin_args(const pcal_ctx *h, double *out) {
    const Plan &p = h->plan;
    const int N = static_cast<int>(p.N);
    FinArgs f{};
    f.acc = h->acc;
    f.accf = h->accf;
    f.tw = h->tw;
    f.N = N;
    f.prec = p.prec;
    f.sideband = p.sideband;
    f.inv_L = h->n_integ > 0 ? 1.0 / static_cast<double>(h->n_integ) : 0.0;
    // in-band tones 0 < f_o + k f_c < fs / 2
    int k_lo = N, k_hi = 0;
    for (int k = 0; k < N; ++k) {
        const int64_t fk = p.fo + int64_t(k) * p.fc;
        if (fk > 0 && 2 * fk < p.fs) {
            k_lo = std::min(k_lo, k);
            k_hi = std::max(k_hi, k + 1);
        }
    }
    if (k_hi <= k_lo) k_lo = k_hi = 0;
    f.k_lo = k_lo;
    f.k_hi = k_hi;
    f.f_comb = static_cast<double>(p.fc);
    f.gain_re = h->gain_re;
    f.gain_im = h->gain_im;
    f.out = out;
    f.phases = h->phases;
    f.counter = h->counters;
    f.clear = 0;
    f.acc_clear = h->acc;
    f.accf_clear = h->accf;
    f.acc_int_clear = h->acc_int;
    return f;
}

int run_finalize(pcal_ctx *h, bool device_results) {
    const Plan &p = h->plan;
    hipStream_t s = h->last_stream;
    int rc = flush_pending(h, s);
    if (rc) return rc;
    if (!device_results && h->host_out_dev) {
        // results for the host only: the finalize writes the pinned copy
        // itself (no device-to-host copy after it)
        launch_finalize(fin_args(h, h->host_out_dev), s);
        PCAL_HIP(hipGetLastError());
        PCAL_HIP(hipStreamSynchronize(s));
        return PCAL_OK;
    }
    launch_finalize(fin_args(h, h->out), s);
    PCAL_HIP(hipGetLastError());
    PCAL_HIP(hipMemcpyAsync(h->host_out, h->out, sizeof(double) * (4 * p.N + 1), hipMemcpyDeviceToHost, s));
    PCAL_HIP(hipStreamSynchronize(s));
    return PCAL_OK;
}

FoldArgs fold_args(pcal_ctx *h, const pcal_launch_t &L, const void *dev_ptr) {
    const Plan &p = h->plan;
    const FoldGeom &g = p.geom;
    FoldArgs a{};
    a.data = reinterpret_cast<const uint4 *>(static_cast<const uint8_t *>(dev_ptr) + L.head_bytes);
    a.nvec = L.nvec;
    a.rows_total = L.rows_total;
    a.rows_per_group = L.rows_per_group;
    a.row_vecs = g.row_vecs;
    a.tile_vecs = g.tile_vecs;
    a.col_tiles = g.col_tiles;
    a.pos_cols = g.pos_cols;
    a.npos = g.npos;
    a.period_vecs = g.period_vecs;
    a.N = static_cast<int>(p.N);
    a.nbits = p.nbits;
    a.prec = p.prec;
    a.int_bins = p.fo == 0 ? 1 : 0;
    a.Sp = p.Sp;
    a.M = p.tab_rows;
    a.q0 = L.q0;
    a.u64 = h->u64;
    a.u32 = h->u32;
    a.u16 = h->u16;
    a.v = h->v;
    a.uq = h->uq;
    a.head = static_cast<const uint8_t *>(dev_ptr);
    a.head_bytes = static_cast<int>(L.head_bytes);
    a.head_q = L.head_q;
    a.tail = static_cast<const uint8_t *>(dev_ptr) + L.head_bytes + 16 * L.nvec;
    a.tail_bytes = static_cast<int>(L.tail_bytes);
    a.tail_q = L.tail_q;
    a.acc = h->acc;
    a.acc_int = h->acc_int;
    a.accf = h->accf;
    a.groups_per_wg = L.groups_per_wg;
    a.extra_groups = L.extra_groups;
    a.odd_start = L.odd_start;
    a.sync_pairs = p.sync_pairs;
    a.fold_wgs = static_cast<int>(L.grid);
    a.fin_wgs = 0;
    return a;
}

int create(int64_t fs, int64_t fc, int64_t fo, int nbits, int sideband, int method, int prec, int force_threads,
           pcal_ctx **out) {
    *out = nullptr;
    Plan p{};
    int rc = make_plan(fs, fc, fo, nbits, sideband, method, prec, &p, force_threads);
    if (rc) return rc;
    pcal_ctx *h = new (std::nothrow) pcal_ctx();
    if (!h) return PCAL_ENOMEM;
    h->plan = p;
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        set_error("hipGetDevice", e);
        delete h;
        return PCAL_EHIP;
    }
    if (p.method == PCAL_METHOD_PERIOD_FOLD && !p.target_from_env) {
        // persistent grid: every workgroup resident at once, and as few per
        // compute unit as keep kMinResidentWaves waves there (each workgroup
        // adds an epilogue and N atomics of its own)
        int cus = 0;
        const int per_cu = fold_blocks_per_cu(p.nbits, p.prec, p.geom.threads,
                                              fold_lds_bytes(p.geom.npos, p.geom.spv, p.geom.threads, p.tab_rows));
        const int waves = (p.geom.threads + 63) / 64;
        const int use = std::min(per_cu, std::max(1, (kMinResidentWaves + waves - 1) / waves));
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
            per_cu > 0 && cus > 0) {
            h->plan.target_blocks = std::max(use * cus, h->plan.geom.col_tiles);
            h->plan.max_blocks = std::max(h->plan.geom.col_tiles, h->plan.target_blocks) + h->plan.geom.col_tiles;
        }
    }
    rc = build(h);
    if (rc) {
        release(h);
        return rc;
    }
    *out = h;
    return PCAL_OK;
}

}  // namespace host
}  // namespace pcal

using namespace pcal;
using namespace pcal::host;

extern "C" {

int pcal_plan(int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int method, int precision,
              pcal_info_t *info) {
    if (!info) return PCAL_EINVAL;
    Plan p{};
    const int rc = make_plan(fs_hz, f_comb_hz, f_offset_hz, nbits, 1, method, precision, &p);
    if (rc) return rc;
    fill_info(p, info);
    return PCAL_OK;
}

int pcal_plan_launch(int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int method,
                     int precision, uint64_t addr_low, int64_t samples_before, int64_t nsamples,
                     pcal_launch_t *out) {
    if (!out || samples_before < 0 || nsamples < 0) return PCAL_EINVAL;
    Plan p{};
    const int rc = make_plan(fs_hz, f_comb_hz, f_offset_hz, nbits, 1, method, precision, &p);
    if (rc) return rc;
    if (nsamples % (8 / nbits)) return PCAL_EINVAL;
    *out = plan_launch(p, addr_low, samples_before, nsamples);
    return PCAL_OK;
}

int pcal_create_ex(int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int sideband, int method,
                   int precision, pcal_t *out) {
    if (!out) return PCAL_EINVAL;
    return create(fs_hz, f_comb_hz, f_offset_hz, nbits, sideband, method, precision, 0, out);
}

int pcal_create(int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int sideband, pcal_t *out) {
    return pcal_create_ex(fs_hz, f_comb_hz, f_offset_hz, nbits, sideband, PCAL_METHOD_AUTO, PCAL_PREC_F64, out);
}

int pcal_extract(pcal_t h, const void *dev_ptr, int64_t nsamples, pcal_stream_t stream) {
    return pcal_extract_timed(h, dev_ptr, nsamples, stream, nullptr, nullptr);
}

static int extract_lane(pcal_ctx *h, const void *dev_ptr, int64_t nsamples, pcal_stream_t stream, void *start_event,
                        void *stop_event) {
    if (!h || nsamples < 0) return PCAL_EINVAL;
    hipEvent_t t0 = static_cast<hipEvent_t>(start_event), t1 = static_cast<hipEvent_t>(stop_event);
    const Plan &p = h->plan;
    const int spb = 8 / p.nbits;
    if (nsamples % spb) return PCAL_EINVAL;
    if (nsamples == 0) return PCAL_OK;
    if (!dev_ptr) return PCAL_EINVAL;
    DeviceGuard guard(h->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool fold = p.method == PCAL_METHOD_PERIOD_FOLD;
    int rc = order_on(h, s, !fold);
    if (rc) return rc;

    const FoldGeom &g = p.geom;
    // A pending finalize takes fin_wgs of the launch's resident workgroups, so
    // that every workgroup starts at once: the fold gets the rest.
    const int fin_wgs = (fold && h->fin_pending) ? static_cast<int>((p.N + 63) / 64) : 0;
    const int target = fin_wgs ? std::max(g.col_tiles, p.target_blocks - fin_wgs) : 0;
    const pcal_launch_t L = plan_launch(p, reinterpret_cast<uintptr_t>(dev_ptr), h->n_total, nsamples, target);
    if (L.grid > p.max_blocks) return PCAL_EINVAL;  // cannot happen by construction

    if (fold) {
        FoldArgs a = fold_args(h, L, dev_ptr);
        size_t lds = static_cast<size_t>(L.lds_bytes);
        if (fin_wgs) {  // the previous integration's finalize rides along in extra workgroups
            a.fin = h->fin;
            a.fin_wgs = fin_wgs;
            lds = std::max(lds, finalize_lds_bytes(static_cast<int>(p.N)));
        }
        launch_fold(a, p.nbits, static_cast<int>(L.grid) + a.fin_wgs, g.threads, lds, s, t0, t1);
        if (h->fin_pending) {
            h->fin_pending = false;
            if (h->fin_dev)
                PCAL_HIP(hipMemcpyAsync(h->fin_host, h->fin_dev, sizeof(double) * (4 * p.N + 1),
                                        hipMemcpyDeviceToHost, s));
        }
    } else {
        const int64_t vb = static_cast<int64_t>(g.spv) * p.nbits / 8;  // bytes per thread-vector
        RotArgs a{};
        a.data = static_cast<const uint8_t *>(dev_ptr) + L.head_bytes;
        a.nvec = L.nvec;
        a.rows_total = L.rows_total;
        a.rows_per_group = L.rows_per_group;
        a.row_vecs = g.row_vecs;
        a.tile_vecs = g.tile_vecs;
        a.col_tiles = g.col_tiles;
        a.period_vecs = g.period_vecs;
        a.N = static_cast<int>(p.N);
        a.nbits = p.nbits;
        a.prec = p.prec;
        a.method = p.method;
        a.g0 = L.q0;
        a.fs = p.fs;
        a.fo = p.fo;
        a.R = p.R;
        a.rot64 = h->rot64;
        a.rot16 = h->rot16;
        a.rot32 = h->rot32;
        a.lut_shift = h->lut_shift;
        a.lut_rows = h->lut_rows;
        a.w = h->w;
        a.back = h->back;
        a.c2 = h->c2;
        a.half_sin = h->half_sin;
        a.half_cos = h->half_cos;
        a.head = static_cast<const uint8_t *>(dev_ptr);
        a.head_bytes = static_cast<int>(L.head_bytes);
        a.head_n = L.head_q;
        a.tail = static_cast<const uint8_t *>(dev_ptr) + L.head_bytes + vb * L.nvec;
        a.tail_bytes = static_cast<int>(L.tail_bytes);
        a.tail_n = L.tail_q;
        a.acc = h->acc;
        a.accf = h->accf;
        launch_rotate(a, static_cast<int>(L.grid), g.threads, static_cast<size_t>(L.lds_bytes), s, t0, t1);
    }
    PCAL_HIP(hipGetLastError());
    h->n_total += nsamples;
    h->n_integ += nsamples;
    return mark(h, s);
}

static int results_lane(pcal_ctx *h, double *amp, double *phase, double *delay) {
    if (!h) return PCAL_EINVAL;
    DeviceGuard guard(h->device);
    int rc = run_finalize(h, false);
    if (rc) return rc;
    const size_t N = static_cast<size_t>(h->plan.N);
    if (amp) memcpy(amp, h->host_out, sizeof(double) * N);
    if (phase) memcpy(phase, h->host_out + N, sizeof(double) * N);
    if (delay) *delay = h->host_out[4 * N];
    return PCAL_OK;
}

static int results_async_lane(pcal_ctx *h, double *host_out, int reset) {
    if (!h || !host_out) return PCAL_EINVAL;
    DeviceGuard guard(h->device);
    const Plan &p = h->plan;
    hipStream_t s = h->last_stream;
    int rc = flush_pending(h, s);
    if (rc) return rc;
    if (!reset) {
        launch_finalize(fin_args(h, h->out), s);
        PCAL_HIP(hipGetLastError());
        PCAL_HIP(hipMemcpyAsync(host_out, h->out, sizeof(double) * (4 * p.N + 1), hipMemcpyDeviceToHost, s));
        return mark(h, s);
    }
    // Finish the integration: its finalize (reading and clearing the current
    // bank) is left pending for the next fold launch, and the handle moves on
    // to the other bank.  The finalize writes the results straight into
    // host_out when that is pinned host memory mapped for the device;
    // otherwise into a device buffer that is then copied.
    const int b = h->bank;
    double *dev_host = mapped_results(h, host_out);
    double *out = dev_host ? dev_host : h->out + static_cast<size_t>(b) * (4 * p.N + 1);
    h->fin = fin_args(h, out);
    h->fin.counter = h->counters + b;
    h->fin.clear = 1;
    h->fin_host = host_out;
    h->fin_dev = dev_host ? nullptr : out;
    h->fin_pending = true;
    set_bank(h, b ^ 1);
    h->n_integ = 0;
    if (p.method != PCAL_METHOD_PERIOD_FOLD) return flush_pending(h, s);
    return PCAL_OK;
}

static int flush_lane(pcal_ctx *h) {
    if (!h->fin_pending) return PCAL_OK;
    DeviceGuard guard(h->device);
    const int rc = flush_pending(h, h->last_stream);
    // later calls on other streams order after the finalize (it clears a bank)
    return rc ? rc : mark(h, h->last_stream);
}

static int sync_lane(pcal_ctx *h) {
    DeviceGuard guard(h->device);
    if (h->fin_pending) {
        const int rc = flush_pending(h, h->last_stream);
        if (rc) return rc;
        PCAL_HIP(hipStreamSynchronize(h->last_stream));
    }
    const int rc = settle(h);
    if (rc) return rc;
    if (h->have_ev) PCAL_HIP(hipEventSynchronize(h->wait_ev));
    return PCAL_OK;
}

static int spectrum_lane(pcal_ctx *h, double *re, double *im) {
    if (!h) return PCAL_EINVAL;
    DeviceGuard guard(h->device);
    int rc = run_finalize(h, false);
    if (rc) return rc;
    const size_t N = static_cast<size_t>(h->plan.N);
    if (re) memcpy(re, h->host_out + 2 * N, sizeof(double) * N);
    if (im) memcpy(im, h->host_out + 3 * N, sizeof(double) * N);
    return PCAL_OK;
}

// Run the pulse readout kernel on the handle's last stream and copy its
// results (2N + 4 doubles, 3N + 4 with the band-pass of spec, and the integer
// bins when host_int is set) to the host.
static PulseArgs pulse_args(pcal_ctx *h, bool ints, const double *spec) {
    const Plan &p = h->plan;
    PulseArgs a{};
    a.acc = h->acc;
    a.accf = h->accf;
    a.acc_int = ints ? h->acc_int : nullptr;
    a.N = static_cast<int>(p.N);
    a.prec = p.prec;
    a.sideband = p.sideband;
    a.fs = static_cast<double>(p.fs);
    a.inv_L = h->n_integ > 0 ? 1.0 / static_cast<double>(h->n_integ) : 0.0;
    a.gain_re = h->gain_re;
    a.gain_im = h->gain_im;
    a.out = h->pulse;
    a.out_int = ints ? h->pulse_int : nullptr;
    a.spec = spec;
    a.f_offset = static_cast<double>(p.fo);
    a.f_comb = static_cast<double>(p.fc);
    return a;
}

static int read_pulse(pcal_ctx *h, double *host, long long *host_int, const double *spec = nullptr) {
    const size_t N = static_cast<size_t>(h->plan.N);
    hipStream_t s = h->last_stream;
    launch_pulse(pulse_args(h, host_int != nullptr, spec), s);
    PCAL_HIP(hipGetLastError());
    PCAL_HIP(hipMemcpyAsync(host, h->pulse, sizeof(double) * ((spec ? 3 : 2) * N + 4), hipMemcpyDeviceToHost, s));
    if (host_int) PCAL_HIP(hipMemcpyAsync(host_int, h->pulse_int, sizeof(long long) * N, hipMemcpyDeviceToHost, s));
    PCAL_HIP(hipStreamSynchronize(s));
    return PCAL_OK;
}

static int bins_lane(pcal_ctx *h, double *re, double *im, int64_t *int_bins) {
    if (!h) return PCAL_EINVAL;
    if (int_bins && (h->plan.fo != 0 || h->plan.method != PCAL_METHOD_PERIOD_FOLD)) return PCAL_ESTATE;
    DeviceGuard guard(h->device);
    const size_t N = static_cast<size_t>(h->plan.N);
    std::vector<double> out(2 * N + 4);
    std::vector<long long> ib(int_bins ? N : 0);
    const int rc = read_pulse(h, out.data(), int_bins ? ib.data() : nullptr);
    if (rc) return rc;
    if (re) memcpy(re, out.data(), sizeof(double) * N);
    if (im) memcpy(im, out.data() + N, sizeof(double) * N);
    for (size_t i = 0; int_bins && i < N; ++i) int_bins[i] = ib[i];
    return PCAL_OK;
}

static int pulse_lane(pcal_ctx *h, double *re, double *im, double *delay, double *peak) {
    if (!h) return PCAL_EINVAL;
    DeviceGuard guard(h->device);
    const size_t N = static_cast<size_t>(h->plan.N);
    std::vector<double> out(2 * N + 4);
    const int rc = read_pulse(h, out.data(), nullptr);
    if (rc) return rc;
    if (re) memcpy(re, out.data(), sizeof(double) * N);
    if (im) memcpy(im, out.data() + N, sizeof(double) * N);
    if (delay) *delay = out[2 * N];
    if (peak) memcpy(peak, out.data() + 2 * N + 1, sizeof(double) * 3);
    return PCAL_OK;
}

static int bandpass_lane(pcal_ctx *h, double *amp, double *phase, double *delay) {
    if (!h) return PCAL_EINVAL;
    DeviceGuard guard(h->device);
    // the finalize leaves amp, phase, re, im and the slope delay in h->out
    int rc = run_finalize(h, true);
    if (rc) return rc;
    const size_t N = static_cast<size_t>(h->plan.N);
    std::vector<double> out(3 * N + 4);
    if ((rc = read_pulse(h, out.data(), nullptr, h->out + 2 * N))) return rc;
    if (amp) memcpy(amp, h->host_out, sizeof(double) * N);
    if (phase) memcpy(phase, out.data() + 2 * N + 4, sizeof(double) * N);
    if (delay) *delay = out[2 * N];
    return PCAL_OK;
}

static int refine_lane(pcal_ctx *h, int iters, double *delays, double *resid) {
    if (!h || iters < 1 || iters > kMaxRefinePasses) return PCAL_EINVAL;
    DeviceGuard guard(h->device);
    // the finalize leaves the reported spectrum in h->out, the pulse readout its peak delay in h->pulse
    int rc = run_finalize(h, true);
    if (rc) return rc;
    hipStream_t s = h->last_stream;
    launch_pulse(pulse_args(h, false, nullptr), s);
    PCAL_HIP(hipGetLastError());
    const FinArgs f = fin_args(h, h->out);
    RefineArgs r{};
    r.spec = h->out + 2 * h->plan.N;
    r.t0 = h->pulse + 2 * h->plan.N;
    r.N = static_cast<int>(h->plan.N);
    r.k_lo = f.k_lo;
    r.k_hi = f.k_hi;
    r.iters = iters;
    r.f_offset = static_cast<double>(h->plan.fo);
    r.f_comb = static_cast<double>(h->plan.fc);
    r.out = h->refine_out;
    launch_refine(r, s);
    PCAL_HIP(hipGetLastError());
    double out[kMaxRefinePasses + 3];
    PCAL_HIP(hipMemcpyAsync(out, h->refine_out, sizeof(double) * (iters + 3), hipMemcpyDeviceToHost, s));
    PCAL_HIP(hipStreamSynchronize(s));
    if (delays) memcpy(delays, out, sizeof(double) * (iters + 1));
    if (resid) memcpy(resid, out + iters + 1, sizeof(double) * 2);
    return PCAL_OK;
}

static int reset_lane(pcal_ctx *h) {
    if (!h) return PCAL_EINVAL;
    DeviceGuard guard(h->device);
    hipStream_t s = h->last_stream;
    launch_zero(h->acc, sizeof(double2) * kAccSlots * h->plan.N, s);
    launch_zero(h->acc_int, sizeof(long long) * kAccSlots * h->plan.N, s);
    launch_zero(h->accf, sizeof(float2) * kAccSlots * h->plan.N, s);
    PCAL_HIP(hipGetLastError());
    h->n_integ = 0;
    return mark(h, s);
}

static void drain_lane(pcal_ctx *h) {
    if (h->fin_pending && flush_pending(h, h->last_stream) == PCAL_OK) (void)hipStreamSynchronize(h->last_stream);
    if (settle(h) == PCAL_OK && h->have_ev) (void)hipEventSynchronize(h->wait_ev);
}

// The lane of the current integration, and the other one (null without a twin).
static pcal_ctx *cur_lane(pcal_ctx *h) { return h->on_twin ? h->twin : h; }
static pcal_ctx *other_lane(pcal_ctx *h) { return h->twin ? (h->on_twin ? h : h->twin) : nullptr; }

int pcal_extract_timed(pcal_t h, const void *dev_ptr, int64_t nsamples, pcal_stream_t stream, void *start_event,
                       void *stop_event) {
    if (!h) return PCAL_EINVAL;
    pcal_ctx *L = cur_lane(h);
    if (L == h) return extract_lane(h, dev_ptr, nsamples, stream, start_event, stop_event);
    L->n_total = h->n_total;  // the global sample index runs on across lanes
    const int rc = extract_lane(L, dev_ptr, nsamples, stream, start_event, stop_event);
    h->n_total = L->n_total;
    return rc;
}

int pcal_results(pcal_t h, double *amp, double *phase, double *delay) {
    return h ? results_lane(cur_lane(h), amp, phase, delay) : PCAL_EINVAL;
}

int pcal_results_async(pcal_t h, double *host_out, int reset) {
    if (!h || !host_out) return PCAL_EINVAL;
    pcal_ctx *L = cur_lane(h);
    if (reset != PCAL_RESET_OVERLAP) {
        int rc = results_async_lane(L, host_out, reset);
        pcal_ctx *O = other_lane(h);
        // a plain reset ends the pipelining: the other lane's pending finalize runs now
        if (!rc && reset && O) rc = flush_lane(O);
        return rc;
    }
    if (h->batch_member) return PCAL_ENOTSUP;  // the batch folds its members in one lane
    int rc = PCAL_OK;
    if (!h->twin) {  // the second lane first: a failure leaves the integration going on
        DeviceGuard guard(h->device);
        if ((rc = make_twin(h))) return rc;
    }
    // finish this integration on its lane (its finalize rides in that lane's
    // next fold) and take the next one on the other lane
    if ((rc = results_async_lane(L, host_out, 1))) return rc;
    h->on_twin = !h->on_twin;
    return PCAL_OK;
}

int pcal_flush(pcal_t h) {
    if (!h) return PCAL_EINVAL;
    int rc = flush_lane(h);
    if (!rc && h->twin) rc = flush_lane(h->twin);
    return rc;
}

int pcal_sync(pcal_t h) {
    if (!h) return PCAL_EINVAL;
    int rc = sync_lane(h);
    if (!rc && h->twin) rc = sync_lane(h->twin);
    return rc;
}

int pcal_spectrum(pcal_t h, double *re, double *im) { return h ? spectrum_lane(cur_lane(h), re, im) : PCAL_EINVAL; }

int pcal_bins(pcal_t h, double *re, double *im, int64_t *int_bins) {
    return h ? bins_lane(cur_lane(h), re, im, int_bins) : PCAL_EINVAL;
}

int pcal_pulse(pcal_t h, double *re, double *im, double *delay, double *peak) {
    return h ? pulse_lane(cur_lane(h), re, im, delay, peak) : PCAL_EINVAL;
}

int pcal_bandpass(pcal_t h, double *amp, double *phase, double *delay) {
    return h ? bandpass_lane(cur_lane(h), amp, phase, delay) : PCAL_EINVAL;
}

int pcal_refine(pcal_t h, int iters, double *delays, double *resid) {
    return h ? refine_lane(cur_lane(h), iters, delays, resid) : PCAL_EINVAL;
}

int pcal_reset(pcal_t h) { return h ? reset_lane(cur_lane(h)) : PCAL_EINVAL; }

int pcal_destroy(pcal_t h) {
    if (!h) return PCAL_EINVAL;
    {
        DeviceGuard guard(h->device);
        drain_lane(h);
        if (h->twin) drain_lane(h->twin);
        release(h);
    }
    return PCAL_OK;
}

int pcal_num_tones(pcal_t h, int *n) {
    if (!h || !n) return PCAL_EINVAL;
    *n = static_cast<int>(h->plan.N);
    return PCAL_OK;
}

int pcal_info(pcal_t h, pcal_info_t *info) {
    if (!h || !info) return PCAL_EINVAL;
    fill_info(h->plan, info);
    info->samples_total = h->n_total;
    info->samples_integ = cur_lane(h)->n_integ;
    info->device_bytes = static_cast<int64_t>(h->device_bytes);
    return PCAL_OK;
}

const char *pcal_strerror(int code) {
    switch (code) {
        case PCAL_OK: return "ok";
        case PCAL_EINVAL: return "invalid argument";
        case PCAL_ENOMEM: return "out of memory";
        case PCAL_EHIP: return "HIP runtime error";
        case PCAL_EAGAIN: return "resources busy, try again";
        case PCAL_ESTATE: return "invalid state for this call";
        case PCAL_ENOTSUP: return "parameters not supported by any kernel form";
        default: return "unknown status";
    }
}

const char *pcal_last_error(void) { return g_last_error; }

}  // extern "C"
