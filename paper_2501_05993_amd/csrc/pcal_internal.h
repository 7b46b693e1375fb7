// Internal definitions shared by the libpcal host code and its gfx950 kernels.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace pcal {

// Samples per 16-byte vector load for each sample format.
constexpr int spv_of(int nbits) { return nbits == 2 ? 64 : 16; }

// Largest number of period positions a fold workgroup keeps in LDS (int32 each):
// 200 vectors of 2-bit samples, with the skew, the spare column and a 512-row
// FP64 table under 64 KiB.
constexpr int kMaxLdsPositions = 12800;
// Column tiles beyond which a tiled fold period gets one tile row per
// workgroup (the compute units of the device: one larger fold workgroup is
// resident on each).
constexpr int kSmallTileWgTiles = 256;
// Rotator rows (u table) kept in LDS by the fold kernel when the table is at most this long.
constexpr int kLdsTableRows = 512;
// Per-thread LDS scratch of the fold epilogue (a partial bin sum in every precision).
constexpr int kEpilogueScratch = 40;
// Copies of the integration bins that fold workgroups add into (workgroup mod
// kAccSlots), summed by the finalize: spreads same-address atomics.
constexpr int kAccSlots = 16;

// Bin i of [kAccSlots][N] accumulators, the slots added in slot order (FP32
// sums for the FP32 form, FP64 otherwise).  Every slot is loaded before the
// first add, with no branch between the loads, so the kAccSlots reads are in
// flight together rather than one memory round trip after another.
__device__ __forceinline__ double2 slot_sum(const double2 *acc, const float2 *accf, bool f32, int N, int i) {
    if (f32) {
        float2 v[kAccSlots];
#pragma unroll
        for (int k = 0; k < kAccSlots; ++k) v[k] = accf[k * N + i];
        float fr = 0.f, fi = 0.f;
#pragma unroll
        for (int k = 0; k < kAccSlots; ++k) {
            fr += v[k].x;
            fi += v[k].y;
        }
        return make_double2(fr, fi);
    }
    double2 v[kAccSlots];
#pragma unroll
    for (int k = 0; k < kAccSlots; ++k) v[k] = acc[k * N + i];
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int k = 0; k < kAccSlots; ++k) {
        re += v[k].x;
        im += v[k].y;
    }
    return make_double2(re, im);
}
// Largest workgroup of the fold kernel.
constexpr int kMaxFoldThreads = 768;
// Largest workgroup of the per-sample rotation kernels (they keep 16 complex lanes
// and their totals in registers).
constexpr int kMaxRotThreads = 512;
// Largest number of tones (bins) supported.
constexpr int kMaxTones = 4096;

// Geometry of the period-fold kernel for one handle (host-computed at create time).
//
// The packed stream is viewed as rows of `row_vecs` 16-byte vectors; row_vecs is a
// multiple of the fold period S' expressed in vectors, so a thread that always reads
// the same column of successive rows always meets the same period positions and can
// keep one integer counter per position in registers.  A row is split into
// `col_tiles` tiles of `tile_vecs` columns, one thread per column.
//
// Thread t of a workgroup on column tile c reads column c*tile_vecs + t%tile_vecs
// of period t/tile_vecs of every row: a row holds row_vecs/period_vecs periods
// (sub-rows), so tiles narrower than the workgroup still use all its threads.
struct FoldGeom {
    int spv;          // samples per vector (64 at 2-bit fold, 16 otherwise)
    int period_vecs;  // vectors per fold period (S'/spv)
    int row_vecs;     // vectors per row (a multiple of period_vecs)
    int tile_vecs;    // columns of one period per workgroup
    int col_tiles;    // workgroups across a period
    int pos_cols;     // = tile_vecs: columns with distinct period positions
    int npos;         // period positions held per workgroup = tile_vecs * spv
    int threads;      // workgroup size (multiple of 64, >= tile_vecs)
};

// Dynamic LDS of the fold kernel.  In front (fold_front_bytes): the skewed
// position sums (one pad word per vector) and one spare column of spv + 1
// words (the sink of the lanes that walk no column), reused by the epilogue
// as scratch of kEpilogueScratch bytes per thread.  Behind it
// (fold_lds_bytes): the rotator rows, when there are at most kLdsTableRows.
__host__ __device__ constexpr size_t fold_front_bytes(int npos, int spv, int threads) {
    return ((static_cast<size_t>(npos + npos / spv + spv + 1) * 4 > static_cast<size_t>(threads) * kEpilogueScratch
                 ? static_cast<size_t>(npos + npos / spv + spv + 1) * 4
                 : static_cast<size_t>(threads) * kEpilogueScratch) +
            15) & ~static_cast<size_t>(15);
}
__host__ __device__ constexpr size_t fold_lds_bytes(int npos, int spv, int threads, int64_t M) {
    return fold_front_bytes(npos, spv, threads) + (M <= kLdsTableRows ? static_cast<size_t>(M) * 16 : 0);
}

// Arguments of the FP64 finalize (DFT, amplitude, phase, delay).
struct FinArgs {
    const double2 *acc;      // [kAccSlots][N] bins (FP64 forms)
    const float2 *accf;      // [kAccSlots][N] bins (FP32 form)
    const double2 *tw;       // [N] exp(-j 2 pi j / N)
    int N;
    int prec;
    int sideband;
    double inv_L;            // 1 / samples in the integration (0 if none)
    int k_lo, k_hi;          // in-band tones [k_lo, k_hi): 0 < f_k < fs/2
    double f_comb;           // Hz
    double gain_re, gain_im; // C_k is multiplied by this (1 / (1 + gamma) in the mixed form, else 1)
    double *out;             // [4N + 1]: amp, phase, re, im, delay (device or mapped host memory)
    double *phases;          // [N] device copy of the phases, read back by the last of several workgroups
    unsigned *counter;
    int clear;               // zero the accumulators afterwards (next integration)
    double2 *acc_clear;      // the accumulators to zero ([kAccSlots][N] each)
    float2 *accf_clear;
    long long *acc_int_clear;
};

// Arguments of the pulse readout (one workgroup): the bins P[b] of the current
// integration and the delay at the power peak of the pulse.
struct PulseArgs {
    const double2 *acc;        // [kAccSlots][N] bins (FP64 forms)
    const float2 *accf;        // [kAccSlots][N] bins (FP32 form)
    const long long *acc_int;  // [kAccSlots][N] exact integer bins (f_offset == 0), read when out_int is set
    int N;
    int prec;
    int sideband;
    double fs;                 // Hz
    double inv_L;              // 1 / samples in the integration (0 if none)
    double gain_re, gain_im;   // known gain of the rotator table (identity unless the mixed form)
    double *out;               // [2N + 4] (3N + 4 with spec): re[N], im[N], delay (s), peak bin,
                               // offset (bins), peak power, then the corrected phases [N]
    long long *out_int;        // [N] integer bins, or null
    const double *spec;        // [2N] reported spectrum (re[N], im[N]) to correct by the delay, or null
    double f_offset, f_comb;   // Hz: tone k is at f_offset + k f_comb
};

// Arguments of the multi-pass delay refinement (one workgroup): the reported
// spectrum of the integration and the pulse-peak delay it starts from.
struct RefineArgs {
    const double *spec;        // [2N] device: Re C[N], Im C[N] as reported
    const double *t0;          // device address of the starting delay (s)
    int N, k_lo, k_hi;         // tones; in-band tones [k_lo, k_hi): 0 < f_k < fs/2
    int iters;                 // passes, >= 1
    double f_offset, f_comb;   // Hz: tone k is at f_offset + k f_comb
    double *out;               // [iters + 3]: delays t_0 .. t_iters (s), intercept (rad), rms residual (rad)
};

// Arguments of the fused unpack-rotate-fold kernel (one launch per pcal_extract).
struct FoldArgs {
    const uint4 *data;       // 16-byte aligned start of the full vectors
    int64_t nvec;            // number of full vectors at data
    int64_t rows_total;      // ceil(nvec / row_vecs)
    int64_t rows_per_group;  // rows per workgroup (per-sample forms)
    int row_vecs, tile_vecs, col_tiles, pos_cols, npos;
    int period_vecs;         // vectors per fold period
    int N;                   // tones = bins
    int nbits;               // 2 or 8
    int prec;                // enum pcal_precision
    int int_bins;            // f_offset == 0: also keep exact int64 bins
    int64_t Sp;              // fold period S' (samples)
    int64_t M;               // S' / N rows of the factorised rotator table
    int64_t q0;              // period coordinate (global index mod S') of data[0], sample 0
    const double2 *u64;      // u[m] = exp(-j w_o N m), m < M  (FP64)
    const float2 *u32;       // same, rounded to FP32
    const __half2 *u16;      // [2M]: u[m] ~ u16[2m] + u16[2m+1] (FP16 rounded, then its residual)
    const double2 *v;        // v[b] = exp(-j w_o b), b < N  (FP64)
    const int2 *uq;          // fixed-point form: exp(-j w_o r) * 2^17 rounded, r < R (then M = R)
    // Samples outside the full vectors (misaligned head, short tail), <= 15 bytes each.
    const uint8_t *head;
    int head_bytes;
    int64_t head_q;          // period coordinate of the first head sample
    const uint8_t *tail;
    int tail_bytes;
    int64_t tail_q;
    // Row layout of the fold walk: the full rows form groups of 5 (2-bit) or 4
    // (8-bit) rows; workgroup g of a column tile walks groups_per_wg groups from
    // row R*(g*groups_per_wg + min(g, extra_groups)), one more if g <
    // extra_groups.  Rows [odd_start, rows_total) go to the first workgroup of
    // each tile.
    int64_t groups_per_wg, extra_groups, odd_start;
    int sync_pairs;          // a workgroup barrier every sync_pairs pairs of groups (power of 2; 0: none)
    // Fused finalize of the previous integration: workgroups [fold_wgs,
    // fold_wgs + fin_wgs) of the launch run the finalize of `fin` (another
    // accumulator bank) instead of folding; fin_wgs = 0: none.
    int fold_wgs, fin_wgs;
    FinArgs fin;
    // Integration accumulators of the handle (each workgroup adds its bins atomically).
    double2 *acc;            // [kAccSlots][N] rotated, folded bins P[b], FP64
    float2 *accf;            // [kAccSlots][N] the same in FP32 (PREC_F32 form)
    long long *acc_int;      // [kAccSlots][N] integer bins of Eq. 2 (int_bins only)
};

// Arguments of the per-sample rotation kernels (table or recurrence rotator).
struct RotArgs {
    const void *data;        // aligned start of the full thread-vectors (16 samples each)
    int64_t nvec, rows_total, rows_per_group;
    int row_vecs, tile_vecs, col_tiles;
    int period_vecs;
    int N, nbits, prec, method;
    int64_t g0;              // global index of the first full-vector sample
    int64_t fs, fo, R;       // Hz, Hz, rotator period (Eq. 4)
    // Rotator table of one period (table method), in the handle's precision form:
    // FP64 entries (F64), two FP16 terms per entry, the rounded value and its
    // rounded residual, stored as neighbours (MIXED), or FP32 entries (F32).
    // Entries de-interleaved as described below.
    const double2 *rot64;    // [R]
    const __half2 *rot16;    // [2R]: entry k = rot16[2k] + rot16[2k + 1]
    const float2 *rot32;     // [R]
    // Entry n of the table is stored at (n mod D) * (R / D) + n / D, D = 2^lut_shift
    // the largest power of two <= 16 dividing R: the lanes of a wave look up
    // entries 16 apart, which this places next to each other.
    int lut_shift;
    int64_t lut_rows;        // R / D
    const double2 *w;        // [16] lane factors exp(-j w_o i)
    double2 back;            // exp(+j w_o * samples per row): one row back, FP64
    double c2;               // 2 cos(w_o * samples per row), recurrence coefficient (FP32 forms round it)
    double half_sin, half_cos;  // sin and cos of half the row step (magic circle)
    const uint8_t *head;
    int head_bytes;
    int64_t head_n;          // global index of the first head sample
    const uint8_t *tail;
    int tail_bytes;
    int64_t tail_n;
    double2 *acc;            // [kAccSlots][N]
    float2 *accf;            // [kAccSlots][N] (F32 form)
};


// t0 / t1: optional events stamped with the kernel's start and end (null: a plain launch)
void launch_fold(const FoldArgs &a, int nbits, int grid, int threads, size_t lds, hipStream_t s,
                 hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// Fold workgroups of the given shape resident at once on one compute unit (0 on error).
int fold_blocks_per_cu(int nbits, int prec, int threads, size_t lds);
// ---- Device-resident served loop (pcal_server_start) ----------------------
//
// One chunk of a served stream as the host publishes it in the work ring
// (pinned, coherent host memory): the chunk's fold, planned for at most
// `tasks` workgroups, and, when the chunk completes an integration, that
// integration's finalize.  The host then raises the count of published tasks.
struct ServedDesc {
    FoldArgs fold;
    FinArgs fin;
    int sid;          // stream slot of the server
    int bank;         // accumulator bank of the integration
    int ntasks;       // fold tasks of the chunk (1 <= ntasks <= the task indices per chunk)
    int fin_total;    // fold tasks of the whole integration if this chunk completes it, else 0
    long long integ;  // integration index (completion record)
};

// A finished integration, written by the device into the completion ring;
// seq = record index + 1, written last.
struct ServedDone {
    int sid;
    int pad;
    long long integ;
    unsigned long long seq;
};

// Arguments of the persistent served kernel.  Workgroup 0 schedules, the
// others fold.  The scheduler alone reads host memory: the count of published
// tasks, the quit flag and each new chunk's descriptor, which it copies into
// device memory (dring).  It hands tasks to idle workers through per-worker
// mailbox lines (mail_assigned, written by the scheduler; mail_done, written
// by the worker), so that no line in device memory is polled by more than two
// workgroups: lines that many workgroups poll with coherent loads serialise at
// the memory.
struct ServedArgs {
    const ServedDesc *ring;      // [cap] work ring (host memory, device address)
    unsigned long long *slot_free;  // [cap] host memory: chunk index + 1 of the last chunk whose tasks all ended
    ServedDone *done;            // [done_cap] completion ring (host memory)
    const unsigned long long *published;  // host memory: tasks published (chunks published x tasks)
    const int *quit;             // host memory: nonzero asks the loop to leave once every published task ended
    int *status;                 // host memory: [0] workgroups that left, [1] of them after the idle limit
    unsigned long long *sched;   // device: [0] next chunk to hand out (kept across launches)
    unsigned long long *heartbeat;  // device: the scheduler's round count, rewritten every round
    unsigned long long *done_cursor;  // device: next completion record
    unsigned *slot_cnt;          // device [cap]: tasks of the chunk in the slot that ended
    unsigned long long *task_done;  // device [streams][2]: tasks of the integration in the bank that ended (low
                                    // 32 bits) and its task total once its last chunk has counted (high 32 bits)
    FinArgs *fin_args;           // device [streams][2]: that integration's finalize, from its last chunk
    ServedDesc *dring;           // device [cap]: the scheduler's copy of each slot's descriptor
    unsigned long long *mail_assigned;  // device [grid][kMailStride]: task + 2 handed to the worker; 1: leave
    unsigned long long *mail_done;      // device [grid][kMailStride]: task + 2 the worker finished; 1: started
    int cap, done_cap, tasks;    // ring slots, completion records, task indices per chunk
    int grid;                    // workgroups of the launch (the scheduler and grid - 1 workers)
    unsigned long long idle_ticks;    // wall-clock ticks without work before the loop leaves
    unsigned long long worker_ticks;  // ticks of a frozen heartbeat after which a waiting worker leaves
    unsigned long long check_ticks;   // ticks between a waiting worker's looks at the heartbeat
    unsigned long long quit_ticks;    // ticks after quit the scheduler still waits for pending work
    unsigned long long *stat;    // device [kServedStats]: loop counters (pcal_server_loop_stats order from [1])
};
constexpr int kServedStats = 13;
constexpr int kMailStride = 32;            // u64 words per mailbox (256 B: a line of its own)
constexpr int kServedMaxWorkgroups = 2048;
constexpr int kServedMaxRing = 512;        // ring slots the scheduler can look ahead over (<= its threads)

void launch_served(const ServedArgs &a, int prec, int grid, int threads, size_t lds, hipStream_t s);
constexpr int kServedThreads = 512;          // the batched form's member workgroup size
constexpr size_t kServedLds = 61440;         // fold geometries up to 12800 positions, finalize up to 1792 tones
static_assert(kServedLds >= 8 * kServedMaxWorkgroups + 4 * (2 * kServedMaxRing + 17), "scheduler state");
static_assert(kServedMaxRing <= kServedThreads, "one scheduler thread per pending chunk");
constexpr int kServedMaxTones = 1792;
// The served loop's one-workgroup finalize keeps the bins, the phases and 256
// scratch words in LDS, and the twiddles and the tone results too up to this
// many tones.
constexpr int kServedTwLdsTones = 1024;
static_assert(kServedLds >= 56 * kServedTwLdsTones + 8 * 256 && kServedLds >= 24 * kServedMaxTones + 8 * 256,
              "served finalize");

// Work-lists of the batched kernels: item i owns workgroups [first[i],
// first[i + 1]).  A list in device memory (copied there before the launch),
// or a short one carried in the kernel arguments (no copy).
template <class T>
struct DeviceList {
    const T *items;
    const int *first;
    int n;
};
template <class T, int CAP>
struct InlineList {
    static constexpr int kCap = CAP;
    int n;
    int first[CAP + 1];
    T items[CAP];
};
constexpr int kInlineFoldItems = 8;   // 8 x 376 B of FoldArgs: within 4 KiB of kernel arguments
constexpr int kInlineFinItems = 16;
using FoldListInline = InlineList<FoldArgs, kInlineFoldItems>;
using FinListInline = InlineList<FinArgs, kInlineFinItems>;

// Work-list items [0, n2) are 2-bit and own workgroups [0, grid2); the rest
// are 8-bit and own the next grid8 workgroups.  One launch per width.
void launch_fold_batch(const DeviceList<FoldArgs> &list, int prec, int grid2, int grid8, int threads, size_t lds2,
                       size_t lds8, hipStream_t s);
void launch_fold_batch(const FoldListInline &list, int prec, int grid2, int grid8, int threads, size_t lds2,
                       size_t lds8, hipStream_t s);
void launch_rotate(const RotArgs &a, int grid, int threads, size_t lds, hipStream_t s,
                   hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
void launch_finalize(const FinArgs &a, hipStream_t s);
void launch_pulse(const PulseArgs &a, hipStream_t s);
void launch_refine(const RefineArgs &a, hipStream_t s);
constexpr int kMaxRefinePasses = 16;
size_t finalize_lds_bytes(int N);
void launch_finalize_batch(const DeviceList<FinArgs> &list, int grid, size_t lds, hipStream_t s);
void launch_finalize_batch(const FinListInline &list, int grid, size_t lds, hipStream_t s);
struct ZeroItem {
    void *ptr;
    size_t bytes;  // multiple of 4
};
void launch_zero_list(const ZeroItem *items, int n, hipStream_t s);
void launch_zero(void *p, size_t bytes, hipStream_t s);

}  // namespace pcal
