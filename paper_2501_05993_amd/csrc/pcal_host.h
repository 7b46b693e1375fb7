// Private host-side definitions of libpcal shared by its C ABI translation
// units (single-stream API, batched and served forms).
#pragma once

#include <stdint.h>

#include <vector>

#include "pcal.h"
#include "pcal_internal.h"

namespace pcal {
namespace host {

void set_error(const char *what, hipError_t e);
// A library error text for pcal_last_error() (no HIP status involved).
void set_message(const char *what);

#define PCAL_HIP(call)                      \
    do {                                    \
        hipError_t e_ = (call);             \
        if (e_ != hipSuccess) {             \
            set_error(#call, e_);           \
            return PCAL_EHIP;               \
        }                                   \
    } while (0)

int64_t gcd64(int64_t a, int64_t b);
// Kernel arithmetic of a precision form: the single-FP16 form is the mixed
// form's arithmetic with single-term table entries.
// Fixed-point rotator scale: 17 fractional bits (PCAL_PREC_Q17).
constexpr double kFixedScale = 131072.0;
inline int kernel_prec(int prec) { return prec == PCAL_PREC_F16 ? PCAL_PREC_MIXED : prec == PCAL_PREC_Q17 ? 3 : prec; }
void phasor(int64_t num, int64_t den, double *re, double *im);

struct Plan {
    int64_t fs, fc, fo;
    int nbits, sideband, method;
    int prec;      // arithmetic of the kernels (F64, MIXED or F32; the single-FP16 form runs MIXED's)
    int prec_api;  // enum pcal_precision as requested
    int64_t N, R, S, Sp, M;
    int64_t tab_rows;  // entries of the fold's rotator table: M (factorised forms) or R (fixed-point form)
    FoldGeom geom;
    int target_blocks;
    int sync_pairs;   // fold walk: workgroup barrier every sync_pairs pairs of groups (0: none)
    bool target_from_env;  // PCAL_TARGET_BLOCKS set: keep it on every device
    int max_blocks;
    double osc_sin = 1.0;  // resonator: |sin d| of the row step d (capped at 0.2 by the row choice)
};

constexpr int kSyncPairs = 1;  // fold walk: a workgroup barrier after every pair of groups (PCAL_SYNC_PAIRS)
constexpr int64_t kMaxFoldPeriod = int64_t(1) << 26;  // S' samples
// Fold workgroup size: at least kMinFoldThreads (7 waves) and, among the sizes
// that waste equally few lanes, the one nearest kAimFoldThreads (measured on
// 2^30-sample 2-bit launches: 256-thread workgroups of a 64-vector period ran
// at 54 % of the HBM peak, 576-640 at 73 %).
constexpr int kMinFoldThreads = 448;
constexpr int kAimFoldThreads = 640;
// Waves per compute unit the persistent fold grid aims for with the fewest
// workgroups (2^28-sample 8-bit launches, N = 1024: one 768-thread workgroup
// per compute unit ran at 73.5 % of the HBM peak, two at 70 %; the 8-bit
// 6400-sample period: two 448-thread workgroups 76.8 %, three 75.4 %).
constexpr int kMinResidentWaves = 10;
constexpr int64_t kMaxTableRows = int64_t(1) << 20;   // u table entries
constexpr int64_t kMaxLutPeriod = int64_t(1) << 24;   // rotator table entries (table method)
constexpr int kRotLanes = 16;                          // samples per thread-row, per-sample forms
// Workgroups per launch before the period fold's persistent grid replaces it
// (PCAL_TARGET_BLOCKS overrides).  The 8-bit per-sample forms (256-thread
// workgroups) run best with fewer (256 MiB launches, N = 64 and 1024): the
// recurrences at 512 workgroups reach 56-62 % of the HBM peak against 42-51 %
// at 1024 and 42-47 % at 768; the table, whose row reads want more waves in
// flight, 39-40 % at 768 against 35-36 % at 512 and 30-34 % at 1024.  At
// 2 bits 512-2048 measure alike.
constexpr int kTargetBlocks = 1024;
constexpr int kRotTargetBlocks8 = 512;
constexpr int kLutTargetBlocks8 = 768;
// Longest fold period AUTO folds.  The fold's cost is the walk (HBM-bound)
// plus an epilogue per period position; a per-sample recurrence costs VALU per
// sample.  Measured on 2-bit fs = 64 MHz streams (one MI355X): an 8e6-sample
// fold period folds 2^30 samples in 62 us (54 % of the HBM peak) against
// 201 us for the FP64 recurrence, and wins at every launch length down to one
// period (20 us against 33 us at 2^23 samples); a 64e6-sample period wins only
// from about 2^29 samples per launch, so longer periods keep the recurrence.
constexpr int64_t kAutoFoldPeriod = int64_t(1) << 23;

int make_plan(int64_t fs, int64_t fc, int64_t fo, int nbits, int sideband, int method, int prec, Plan *p,
              int force_threads = 0);
// Launch geometry of one extract call; target_blocks = 0 takes the plan's.
pcal_launch_t plan_launch(const Plan &p, uint64_t addr, int64_t n_before, int64_t nsamples,
                          int target_blocks = 0);
void fill_info(const Plan &p, pcal_info_t *info);
// Device bytes a handle of this plan allocates (no allocation made).
int64_t plan_device_bytes(const Plan &p);

}  // namespace host
}  // namespace pcal

struct pcal_ctx {
    pcal::host::Plan plan;
    int device = 0;
    double2 *u64 = nullptr;
    float2 *u32 = nullptr;
    __half2 *u16 = nullptr;
    int2 *uq = nullptr;            // fixed-point form: Q17 rotator of one period [R]
    double2 *v = nullptr;
    double2 *tw = nullptr;
    // Integration accumulators in two banks; acc / acc_int / accf point at the
    // current one.  pcal_results_async with reset leaves the current bank's
    // finalize pending and switches banks; the next fold launch runs that
    // finalize in extra workgroups (flush_pending runs it alone otherwise).
    double2 *acc_mem = nullptr;     // [2][kAccSlots][N]
    long long *acc_int_mem = nullptr;
    float2 *accf_mem = nullptr;
    double2 *acc = nullptr;
    long long *acc_int = nullptr;
    float2 *accf = nullptr;
    int bank = 0;
    bool fin_pending = false;
    pcal::FinArgs fin;              // the pending finalize (clearing the other bank)
    double *fin_host = nullptr;     // where its results go
    const double *fin_dev = nullptr;  // device results to copy to fin_host (null: written there directly)
    int lut_shift = 0;            // rotator table layout (RotArgs::lut_shift)
    int64_t lut_rows = 0;
    double *phases = nullptr;      // [N] phases the last finalize workgroup reads back
    double *pulse = nullptr;       // [2N + 4] pulse readout (PulseArgs::out)
    long long *pulse_int = nullptr;  // [N] integer bins of the readout
    double *refine_out = nullptr;  // [kMaxRefinePasses + 3] delay refinement (RefineArgs::out)
    unsigned *counters = nullptr;  // [0] finalize of bank 0's pending form / plain, [1] bank 1
    double *out = nullptr;         // device results [2][4N + 1]
    double *host_out = nullptr;    // pinned copy
    double *host_out_dev = nullptr;  // its device address (the finalize of pcal_results writes it directly)
    double2 *rot64 = nullptr;      // rotator table of the table method, in the precision form's
    __half2 *rot16 = nullptr;      // arithmetic (RotArgs): only the one the form reads is allocated
    float2 *rot32 = nullptr;
    double2 *w = nullptr;          // [16] lane factors (per-sample forms)
    double2 back = {1.0, 0.0};     // exp(+j w_o * samples per row)
    double c2 = 2.0;               // 2 cos(w_o * samples per row)
    double half_sin = 0.0, half_cos = 1.0;  // sin, cos of half that row step (magic circle)
    double gain_re = 1.0, gain_im = 0.0;  // 1 / (1 + gamma) of the FP16 table (mixed form)
    int64_t n_total = 0;
    int64_t n_integ = 0;
    hipStream_t last_stream = nullptr;
    bool dirty = false;            // work enqueued on last_stream since ev was last recorded
    hipEvent_t ev = nullptr;       // recorded on last_stream when another stream or a sync needs it (settle)
    hipEvent_t wait_ev = nullptr;  // the recorded event marking the handle's last work
    bool have_ev = false;
    size_t device_bytes = 0;
    // Pipelined integrations (pcal_results_async with PCAL_RESET_OVERLAP): a
    // second lane with its own accumulators, result buffers, pending finalize
    // and stream bookkeeping, and the primary's read-only tables, takes every
    // other integration, so that consecutive integrations fed on two streams
    // run side by side (each lane's finalize rides in its own next fold).
    pcal_ctx *twin = nullptr;
    bool on_twin = false;         // the current integration is the twin's
    bool shares_tables = false;   // this is a twin: its tables are the primary's
    bool batch_member = false;    // folded by a batch (pcal_batch_*), which uses its one lane
};

namespace pcal {
namespace host {

int build(pcal_ctx *h);
// A lane's own device memory (accumulators, counters, results, readouts) and
// its zeroed state; the second lane of pipelined integrations.
int alloc_lane(pcal_ctx *h);
int clear_lane(pcal_ctx *h);
int make_twin(pcal_ctx *h);
// Point acc / acc_int / accf at bank b.
void set_bank(pcal_ctx *h, int b);
// Run a pending finalize on its own (on s).
int flush_pending(pcal_ctx *h, hipStream_t s);
void release(pcal_ctx *h);
int create(int64_t fs, int64_t fc, int64_t fo, int nbits, int sideband, int method, int prec, int force_threads,
           pcal_ctx **out);
// Order s after the handle's last work (a pending finalize runs first unless flush is false).
int order_on(pcal_ctx *h, hipStream_t s, bool flush = true);
// Note work just enqueued on s as the handle's last work (no event is recorded here).
int mark(pcal_ctx *h, hipStream_t s);
// Record the handle's event on its last stream if work was enqueued there since the last record.
int settle(pcal_ctx *h);
// Kernel arguments of one extract call of a period-fold handle (advances the
// handle's chunk-counter base past the launch).
FoldArgs fold_args(pcal_ctx *h, const pcal_launch_t &L, const void *dev_ptr);
// Finalize arguments writing to `out` (4N + 1 doubles).
FinArgs fin_args(const pcal_ctx *h, double *out);

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Integer from the environment (tuning knobs), dflt when unset.
int env_int(const char *name, int dflt);

// Batched read-and-clear finalize and member release (pcal_batch.hip), for the
// served form.
// outs: per member, the device address its results go to (mapped pinned host
// memory allowed), or null for h->out; outs itself may be null.
int batch_finalize_async(pcal_batch_ctx *b, int count, const int *ids, double *const *outs, hipStream_t s);
int batch_release(pcal_batch_ctx *b, int id);
// Workgroup size the batch plans its members for.
int batch_threads(const pcal_batch_ctx *b);

}  // namespace host
}  // namespace pcal
