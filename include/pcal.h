/*
 * pcal.h -- C ABI of libpcal, a gfx950 (MI355X) implementation of fast
 * multi-tone phase-calibration (PCal) extraction (Wagner & Pogrebenko,
 * "Fast Multi-tone Phase Calibration Signal Extraction", arXiv:2501.05993).
 *
 * Method (Section 2 of the paper).  A real baseband stream x[n] sampled at fs
 * carries a comb of N = fs / f_comb tones at k*f_comb + f_offset (Eq. 1).
 * Rotating by exp(-j*w_offset*n) (Eq. 3, w_offset = 2*pi*f_offset/fs, Eq. 5)
 * moves every tone onto a multiple of f_comb; folding the rotated samples
 * into N bins by n mod N (Eq. 2) and taking one N-point DFT of the bins
 * (Section 2, DFT(P)) gives each tone's complex response
 *
 *     C_k = sum_n x[n] * exp(-j * 2*pi * (k*f_comb + f_offset) * n / fs).
 *
 * The sampled rotator repeats after fs / gcd(fs, f_offset) samples (Eq. 4).
 *
 * Conventions shared by every entry point:
 *   - Frequencies are integer Hz (Eq. 4 needs integers).
 *   - Samples: nbits = 2 -> offset-binary codes 0..3 meaning levels
 *     -3,-1,+1,+3, four per byte, sample 4j+q in bits [2q, 2q+1] of byte j;
 *     nbits = 8 -> two's-complement int8.
 *   - Sample indices are global: each pcal_extract continues where the
 *     previous call on the handle stopped, so splitting a stream into calls
 *     does not change the result (phase continuity).
 *   - Every function returns a status code (enum pcal_status); nothing
 *     throws across the ABI.  A HIP failure returns PCAL_EHIP and its text
 *     is kept for pcal_last_error().
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Device pointers are HIP device (or managed) addresses; host pointers
 *     are ordinary process memory.
 */
#ifndef PCAL_H
#define PCAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pcal_ctx *pcal_t; /* opaque handle, owned by the library */
typedef void *pcal_stream_t;     /* a hipStream_t; NULL means the null stream */

enum pcal_status {
    PCAL_OK = 0,
    PCAL_EINVAL = -1,  /* an argument is out of range or inconsistent */
    PCAL_ENOMEM = -2,  /* device or host allocation failed */
    PCAL_EHIP = -3,    /* a HIP runtime call failed; see pcal_last_error() */
    PCAL_EAGAIN = -4,  /* admission refused for now (memory budget); retry later */
    PCAL_ESTATE = -5,  /* call not valid in the handle's current state */
    PCAL_ENOTSUP = -6  /* parameters valid but no kernel form supports them */
};

/* How the rotation of Eq. 3 is carried out.
 *  PERIOD_FOLD: fold integer samples over the joint period S = lcm(N, R)
 *      (R from Eq. 4) and rotate each of the S positions once; by
 *      distributivity this is the precomputed-rotator method with the rotation
 *      moved after the accumulation (Section 4.1 proposes accumulating over a
 *      rotator period and folding into the bins after the sample loop).
 *  LUT: multiply every sample by a precomputed rotator table value (Eq. 4
 *      table, Section 4.1), accumulate in the precision form's arithmetic.
 *  OSC: multiply every sample by a recurrence sinewave generator (Eq. 6-7
 *      direct-form resonator), re-seeded exactly at intervals.  The
 *      generator steps once per row of samples by d = w_offset * (row length);
 *      the row length is chosen so that d stays away from 0 and pi, where the
 *      rounded coefficient 2 cos d would detune it (Section 2.2).
 *  CFO: as OSC with the coupled-form oscillator of Section 2.2 (the rotator
 *      times exp(-j d) per step, d the rotator advance of one step), for
 *      comparison with the direct-form resonator.
 *  MCO: as OSC with the magic-circle oscillator of Section 2.2 (x += e y,
 *      then y -= e x with the new x, e = 2 sin(d/2)); its state is not in
 *      quadrature, so each step's rotator is read out as x - j sin(a) with
 *      -sin(a) = (y + x sin(d/2)) / cos(d/2).
 *  DFR_EF: the direct-form resonator with truncation-error feedback (a remedy
 *      Section 2.2 names): state and coefficient in two terms each, every
 *      step's rounding error carried into the next.
 *  AUTO: PERIOD_FOLD when the joint period fits (at most 2^23 samples), else
 *      OSC; CFO instead of OSC in the FP32-state forms (MIXED, F32) when no
 *      row length keeps |sin d| >= 0.1.
 * The recurrence forms (OSC, CFO, MCO, DFR_EF) share one row choice. */
enum pcal_method {
    PCAL_METHOD_AUTO = 0,
    PCAL_METHOD_PERIOD_FOLD = 1,
    PCAL_METHOD_LUT = 2,
    PCAL_METHOD_OSC = 3,
    PCAL_METHOD_CFO = 4,
    PCAL_METHOD_MCO = 5,
    PCAL_METHOD_DFR_EF = 6
};

/* Arithmetic of the rotation and the per-block fold.  The cross-block
 * reduction, the N-point DFT and the delay fit always run in FP64 except in
 * PCAL_PREC_F32, the all-FP32 comparison form.
 *  F64:   rotator in FP64 (table entries, recurrence state), products and
 *         per-block sums in FP64.  The period fold sums integer samples
 *         exactly and rotates each period position once with an FP64 entry.
 *  MIXED: rotator table entries as two FP16 terms, the rounded value and its
 *         rounded residual (about 22 bits together; the recurrences keep FP32
 *         state), FP32 products, Kahan-compensated FP32 per-block sums; FP64
 *         from the cross-block reduction on, with the table's known mean
 *         gain divided out.
 *  F32:   FP32 table or recurrence state, plain FP32 sums, FP32 reduction
 *         and DFT.
 *  F16:   the literal mixed form, for comparison: MIXED's arithmetic with each
 *         table entry a single FP16 value (the rounded rotator) and no gain
 *         correction.  Its rounding leaves errors of order 1e-5 in amplitude,
 *         at or above the 1e-5 bar MIXED meets.
 *  Q17:   fixed-point rotator (the integer arithmetic of Section 4.8's FPGA
 *         design, whose 18-bit multiplier operands hold a rotator value with
 *         17 fractional bits): each rotator value exp(-j w_offset n) over one
 *         period (Eq. 4) scaled by 2^17 and rounded to an integer (int32
 *         entries, so +1 itself is exact), integer products with the integer
 *         samples and exact integer sums; the bins P[b] (times 2^17) are
 *         integers, exact while each bin's sum of |x| * 2^17 stays below
 *         2^53, and the FP64 DFT scales them by 2^-17.  Period fold only (PCAL_ENOTSUP for
 *         the per-sample forms and for batches). */
enum pcal_precision {
    PCAL_PREC_F64 = 0,
    PCAL_PREC_MIXED = 1,
    PCAL_PREC_F32 = 2,
    PCAL_PREC_F16 = 3,
    PCAL_PREC_Q17 = 4
};

/* Create a handle for one stream.
 *   fs_hz > 0, f_comb_hz > 0, fs_hz % f_comb_hz == 0 (N integer, Section 2),
 *   0 <= f_offset_hz < fs_hz, N <= 4096, nbits in {2, 8},
 *   sideband = +1 (upper) or -1 (lower: results are complex-conjugated, so
 *   phases and delay change sign).
 * Allocates the handle's tables and accumulators on the current HIP device.
 * Returns PCAL_EINVAL without touching the GPU when a parameter is invalid. */
int pcal_create(int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int sideband,
                pcal_t *out);

/* As pcal_create with an explicit kernel form and precision. */
int pcal_create_ex(int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int sideband,
                   int method, int precision, pcal_t *out);

/* Enqueue the unpack-rotate-fold of nsamples packed samples at dev_ptr on
 * stream.  nsamples must be a multiple of the samples per byte (4 at 2-bit);
 * dev_ptr needs no particular alignment (a misaligned head is handled
 * separately).  Asynchronous: dev_ptr must stay valid until the stream has
 * passed the enqueued work.  Work on a stream other than the previous call's
 * is ordered after it.  nsamples == 0 is a no-op. */
int pcal_extract(pcal_t h, const void *dev_ptr, int64_t nsamples, pcal_stream_t stream);

/* pcal_extract, with the extraction kernel launched between two events the
 * caller created (hipEvent_t, passed as void*; either may be NULL).  The
 * events take the kernel's own start and end time stamps (hipExtLaunchKernel),
 * so hipEventElapsedTime(start, stop) is the kernel's duration, free of launch
 * gaps: the figure a throughput-versus-bandwidth comparison needs.  Every other
 * behaviour, argument and error is that of pcal_extract. */
int pcal_extract_timed(pcal_t h, const void *dev_ptr, int64_t nsamples, pcal_stream_t stream,
                       void *start_event, void *stop_event);

/* Finish the current integration: FP64 N-point DFT of the bins, then for
 * every tone k (k = 0..N-1, tone frequency f_offset + k*f_comb)
 *   amp[k]   = |C_k| / L  (L = samples since the last reset),
 *   phase[k] = arg C_k in (-pi, pi] (radians),
 * and delay[0] = slope / (2*pi) of the least-squares line through the
 * phases unwrapped along increasing frequency over the tones with
 * 0 < f_k < fs/2 (seconds).  Any output pointer may be NULL.  Synchronises
 * the handle's last stream; does not reset the accumulators. */
int pcal_results(pcal_t h, double *amp, double *phase, double *delay);

/* Asynchronous form of pcal_results for pipelined integrations.  host_out
 * (4N + 1 doubles) receives amp[0..N), phase[N..2N), Re C[2N..3N),
 * Im C[3N..4N), delay[4N]; it must stay valid until pcal_sync returns.
 * reset == 0: enqueues the FP64 finalize and a copy to host_out on the
 *   handle's last stream; the integration goes on.
 * reset != 0: finishes the integration and starts the next one.  The handle
 *   keeps its bins in two banks: the finalize of the current bank (which also
 *   clears it) is left pending and the handle switches banks, so the next
 *   pcal_extract runs that finalize inside its own launch, in one of its
 *   workgroups (period fold; the per-sample forms run it at once).  The calls
 *   that finalize (pcal_results, pcal_spectrum, pcal_bandpass, another
 *   pcal_results_async) and pcal_flush run a pending finalize on its own
 *   first, pcal_sync runs it and waits; pcal_bins, pcal_pulse and pcal_reset
 *   work on the new integration's bank and leave it pending.  With host_out
 *   in pinned host memory (hipHostMalloc)
 *   the finalize writes host_out directly; otherwise a device copy is
 *   enqueued after it.
 * reset == PCAL_RESET_OVERLAP: pipelined integrations on two streams.  The
 *   integration finishes as with reset != 0, and the handle takes the next
 *   one in a second lane: accumulators, result buffers, pending finalize and
 *   stream order of its own (allocated at the first such call, about
 *   1.1 KB per tone of device memory more; the rotator tables are shared).  Integrations then
 *   alternate between the lanes, each lane's calls ordered after that lane's
 *   previous work only, so a caller that feeds them on two streams in turn has
 *   consecutive integrations run side by side on the GPU; each lane's finalize
 *   runs inside that lane's next fold launch (pcal_flush runs both lanes'
 *   at once; pcal_sync and pcal_destroy wait for both).  The global sample
 *   index runs on across the lanes in call order.  A reset other than
 *   PCAL_RESET_OVERLAP ends the alternation: the other lane's pending
 *   finalize runs at once and the next integration stays in the current lane.
 *   The calls that read the current integration (pcal_results,
 *   pcal_spectrum, pcal_bins, pcal_pulse, pcal_bandpass, pcal_refine,
 *   pcal_reset) act on the lane of the current integration.  PCAL_ENOTSUP
 *   for a member of a batch (pcal_batch_handle), which the batch folds in its
 *   one lane. */
#define PCAL_RESET_OVERLAP 2
int pcal_results_async(pcal_t h, double *host_out, int reset);

/* Run any pending finalize and wait until all work enqueued on the handle has
 * finished (both lanes' after PCAL_RESET_OVERLAP). */
int pcal_sync(pcal_t h);

/* Enqueue a finalize left pending by pcal_results_async(reset != 0) now, on
 * the handle's last stream (with two lanes, each lane's on that lane's last
 * stream), instead of inside the next pcal_extract; returns
 * at once (host_out is complete when that stream reaches this point).  For
 * callers that want each integration's results without waiting for the next
 * chunk.  No-op when nothing is pending.  Errors: PCAL_EINVAL (null handle),
 * PCAL_EHIP. */
int pcal_flush(pcal_t h);

/* The raw C_k (k = 0..N-1) of the current integration, FP64 real and imaginary
 * parts (after the sideband convention).  Synchronises. */
int pcal_spectrum(pcal_t h, double *re, double *im);

/* The rotated, folded bins P[b] (b = 0..N-1) of Eq. 2-3 in FP64, with the
 * precision form's known gain taken out (the mixed form's table gain, the
 * fixed-point form's 2^17 scale: a power of two, so its bins stay exact), so
 * that their DFT is the upper-sideband C_k.  When
 * f_offset == 0 and int_bins != NULL, also the exact integer bins of Eq. 2
 * (int64); PCAL_ESTATE when int_bins is requested for any other handle.
 * Computed on the device (the accumulator slots added in slot order) on the
 * handle's last stream; synchronises. */
int pcal_bins(pcal_t h, double *re, double *im, int64_t *int_bins);

/* The time-domain pulse of the current integration and the delay at its power
 * peak (Section 2: bin b of the fold stands for a delay of b / fs, refined by
 * a fit over the neighbours of the largest bin; Section 3: the group delay is
 * taken at the position of maximum power).
 *   re, im  [N] or NULL: the pulse P[b], as pcal_bins returns it.
 *   delay   [1] or NULL: seconds, in the sign convention of pcal_results'
 *           phase-slope delay (a comb delayed by t_d gives t_d), in
 *           (-N/(2 fs), N/(2 fs)].  The peak bin b0 is the first bin of
 *           largest |P[b]|^2; the offset d in [0, 1/2] towards the larger
 *           neighbour b0 + s (s = +-1) fits the periodic-hyperbola envelope
 *           c / |sin(pi (b - x0) / N)| of an N-tone pulse through the two
 *           amplitudes: tan(pi d / N) = a_s sin(pi / N) / (a_0 + a_s cos(pi / N));
 *           equal neighbours give d = 0.  Upper sideband: delay = -(b0 + s d) / fs;
 *           lower sideband: +(b0 + s d) / fs.
 *   peak    [3] or NULL: b0, the signed offset s d (bins), and the peak power
 *           |P[b0]|^2 / L^2 (L = samples in the integration).
 * An integration with no samples gives b0 = 0 and delay 0.  Computed by one
 * device workgroup on the handle's last stream; synchronises.  Errors:
 * PCAL_EINVAL (null handle), PCAL_EHIP. */
int pcal_pulse(pcal_t h, double *re, double *im, double *delay, double *peak);

/* The band-pass of the current integration corrected for the group delay at
 * the pulse's power peak (Section 3): amp[N] as pcal_results gives it,
 * phase[N] = arg(C_k exp(-j 2 pi f_k t_g)) in (-pi, pi] with C_k the reported
 * spectrum (pcal_spectrum), f_k = f_offset + k f_comb and t_g the delay of
 * pcal_pulse, which is returned in delay[1].  A comb whose tone phases grow
 * as 2 pi f_k t_g comes out flat.  Any output may be NULL.  Runs the finalize
 * and the pulse readout on the device (the handle's last stream);
 * synchronises.  Errors: PCAL_EINVAL (null handle), PCAL_EHIP. */
int pcal_bandpass(pcal_t h, double *amp, double *phase, double *delay);

/* Multi-pass refinement of the delay of the current integration (Section 2:
 * the delay read coarsely off the pulse peak, then refined by passes that
 * counter-rotate by the current estimate and measure the residual phase).
 * The counter-rotation by a delay t turns tone k by exp(-j 2 pi f_k t),
 * f_k = f_offset + k f_comb, which is what counter-rotating the input by that
 * delay does to the tone responses.  Pass 0 is the pulse-peak delay of
 * pcal_pulse, t_0.  Pass i = 1..iters takes the residual phases
 * psi_k = arg(C_k exp(-j 2 pi f_k t_{i-1})) of the tones with 0 < f_k < fs/2
 * (C_k as pcal_spectrum reports it), unwraps them along increasing f_k, fits
 * the least-squares line psi = a + 2 pi f t_res and sets t_i = t_{i-1} + t_res.
 *   iters   1 .. 16.
 *   delays  [iters + 1] or NULL: t_0 .. t_iters (seconds).
 *   resid   [2] or NULL: the last pass's intercept a (rad, the line's phase
 *           at f = 0) and the rms of its phase residuals about the line (rad).
 * Fewer than two in-band tones leave the delay at t_0 (resid 0, 0).  Runs the
 * finalize, the pulse readout and the passes on the device (one workgroup, the
 * handle's last stream); synchronises.  Errors: PCAL_EINVAL (null handle,
 * iters out of range), PCAL_EHIP. */
int pcal_refine(pcal_t h, int iters, double *delays, double *resid);

/* Start a new integration: zero the accumulators; the global sample index
 * keeps counting (rotator phase stays continuous).  Ordered on the handle's
 * last stream. */
int pcal_reset(pcal_t h);

/* Release the handle and everything it owns (synchronises first). */
int pcal_destroy(pcal_t h);

/* Number of tones N of the handle. */
int pcal_num_tones(pcal_t h, int *n);

/* Derived quantities of a handle, for reporting and tests. */
typedef struct {
    int64_t ntones;          /* N = fs / f_comb */
    int64_t rotator_period;  /* R = fs / gcd(fs, f_offset), Eq. 4 */
    int64_t joint_period;    /* S = lcm(N, R) */
    int64_t fold_period;     /* S' = lcm(S, samples per 16-byte vector) */
    int64_t method;          /* enum pcal_method actually used */
    int64_t precision;       /* enum pcal_precision */
    int64_t samples_total;   /* global samples consumed so far */
    int64_t samples_integ;   /* samples in the current integration */
    int64_t block_threads;   /* fold kernel workgroup size */
    int64_t row_vectors;     /* 16-byte vectors per fold row */
    int64_t col_tiles;       /* workgroups across one fold row */
    int64_t lds_positions;   /* period positions held per workgroup */
    int64_t device_bytes;    /* device memory owned by the handle */
    int64_t period_vectors;  /* thread-vectors per fold period */
    int64_t tile_vectors;    /* columns of one period per workgroup */
    int64_t target_blocks;   /* workgroups one launch aims at: for a fold handle the number of fold
                                workgroups resident at once on its device (one wave of workgroups,
                                each walking one block of rows); 1024 from pcal_plan; the
                                environment variable PCAL_TARGET_BLOCKS overrides both */
} pcal_info_t;

int pcal_info(pcal_t h, pcal_info_t *info);

/* Host-only planning (no GPU call): fills info for the given parameters as
 * pcal_create_ex would, without allocating.  For tests and admission. */
int pcal_plan(int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int method,
              int precision, pcal_info_t *info);

/* Launch geometry of one pcal_extract call (host-only, no GPU call): the
 * numbers the fused kernel is launched with for nsamples samples at a device
 * address whose low bits are addr_low (only addr_low mod 16 matters) when
 * samples_before samples were consumed earlier.  For tests and tools that
 * check the kernel's index arithmetic on the CPU. */
typedef struct {
    int64_t grid;            /* workgroups */
    int64_t threads;         /* threads per workgroup */
    int64_t lds_bytes;       /* dynamic LDS per workgroup */
    int64_t head_bytes;      /* bytes before the first 16-byte aligned vector */
    int64_t nvec;            /* full 16-byte vectors */
    int64_t tail_bytes;      /* bytes after the last full vector */
    int64_t rows_total;      /* rows of row_vectors vectors (last may be partial) */
    int64_t rows_per_group;  /* rows walked by one workgroup (period fold: at most) */
    int64_t q0;              /* global index of the first vector sample, mod fold_period */
    int64_t head_q;          /* global index of the first head sample, mod fold_period */
    int64_t tail_q;          /* global index of the first tail sample, mod fold_period */
    /* Period fold only: the full rows form groups of 5 (2-bit) or 4 (8-bit)
     * rows; workgroup g of a column tile walks groups_per_wg groups (one more
     * if g < extra_groups) from group g*groups_per_wg + min(g, extra_groups).
     * Rows [odd_start, rows_total) go to the first workgroup of each tile. */
    int64_t groups_per_wg;
    int64_t extra_groups;
    int64_t odd_start;
} pcal_launch_t;

int pcal_plan_launch(int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int method,
                     int precision, uint64_t addr_low, int64_t samples_before, int64_t nsamples,
                     pcal_launch_t *out);

/* ---------------------------------------------------------------------------
 * Batched form: many streams, one launch.
 *
 * A batch owns member handles (each with its own fs, f_offset, sample format,
 * tables and accumulators, planned for the batch's workgroup size and the
 * batch's precision form).  pcal_batch_extract folds one chunk for each of
 * `count` members in a single launch of the fused kernel over a work-list;
 * pcal_batch_results finalizes `count` members in a single launch and one
 * device-to-host transfer.  Members are ordinary handles otherwise
 * (pcal_batch_handle): pcal_extract/pcal_results on them still work.  The
 * sample index of every member stays global, exactly as for pcal_extract.
 * ------------------------------------------------------------------------- */
typedef struct pcal_batch_ctx *pcal_batch_t;

/* Create an empty batch of at most max_streams members; precision is the
 * enum pcal_precision every member uses. */
int pcal_batch_create(int max_streams, int precision, pcal_batch_t *out);

/* Add a member stream (parameters as pcal_create).  *id is its index.  The
 * member takes the period fold, planned for the batch's workgroup size and
 * folded in the batch's launches, whenever a fold period fits (at most 2^26
 * samples and 2^20 rotator rows); else AUTO's per-sample form, which
 * pcal_batch_extract runs in a launch of its own after the fold launches.
 * PCAL_EAGAIN when the batch is full. */
int pcal_batch_add(pcal_batch_t b, int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int sideband,
                   int *id);

/* The member handle with index id (owned by the batch). */
int pcal_batch_handle(pcal_batch_t b, int id, pcal_t *h);

/* One launch per sample width for the fold members: for i < count,
 * nsamples[i] samples of member ids[i] at device address dev_ptrs[i] (each
 * id at most once); then one launch per per-sample member.  Asynchronous on
 * stream, ordered after each member's previous work. */
int pcal_batch_extract(pcal_batch_t b, int count, const int *ids, const void *const *dev_ptrs,
                       const int64_t *nsamples, pcal_stream_t stream);

/* Finalize members ids[0..count): amp and phase receive N_id values per member,
 * concatenated in the order of ids (either may be NULL); delay[i] per member.
 * One launch and one transfer; synchronises. */
int pcal_batch_results(pcal_batch_t b, int count, const int *ids, double *amp, double *phase, double *delay);

/* The C_k of members ids[0..count), concatenated as in pcal_batch_results. */
int pcal_batch_spectra(pcal_batch_t b, int count, const int *ids, double *re, double *im);

/* Start a new integration for the listed members (one launch). */
int pcal_batch_reset(pcal_batch_t b, int count, const int *ids);

/* Number of members. */
int pcal_batch_size(pcal_batch_t b, int *n);

/* Release the batch and its member handles (synchronises). */
int pcal_batch_destroy(pcal_batch_t b);

/* ---- Served form: many live streams under one memory budget -------------
 *
 * The spec serving configuration (continuous batching of many
 * independent streams; the paper extracts one stream at a time).  A server
 * holds up to max_streams live streams of any (fs, f_comb, f_offset, nbits,
 * sideband), all in one precision form (enum pcal_precision).
 *
 * pcal_server_open admits a stream only if the device memory of its tables
 * and accumulators fits what is left of mem_budget_bytes, else it returns
 * PCAL_EAGAIN and keeps nothing.  integration_samples (a multiple of the
 * samples per byte) is the length of one integration: its results are one
 * Eq. 1 extraction over exactly those samples, and the global sample index
 * (rotator phase) continues across integrations.
 *
 * pcal_server_submit queues chunks on the host, in order per stream (same
 * rules as pcal_extract: nsamples a multiple of the samples per byte; device
 * memory the caller keeps valid until a pcal_server_step that dispatched the
 * chunk's last samples has completed on its stream).  It never blocks.
 *
 * pcal_server_step dispatches, with one launch of the batched fused kernel
 * per sample width, the oldest queued piece of every stream that has one (a
 * chunk crossing an integration boundary is split there; a stream no fold
 * period fits runs its piece in a per-sample launch of its own, see
 * pcal_batch_add), then one batched finalize for the
 * streams whose integration it completed: it reads and clears their bins and
 * copies their results (amplitude, phase, C_k, delay) to pinned host memory.
 * All of it is asynchronous on `stream`; *samples_dispatched (may be NULL)
 * gets the samples dispatched.  Call it repeatedly while samples are queued.
 *
 * pcal_server_poll reports, without blocking, up to `max` integrations whose
 * results have reached the host (stream id and integration index, in order of
 * completion); pcal_server_result / pcal_server_spectrum copy one out (the
 * last 8 integrations of each stream are kept; an older or unfinished one
 * gives PCAL_ESTATE).  Output arrays hold N doubles.
 *
 * pcal_server_close waits for work in flight and frees the stream's memory
 * (its budget returns); pcal_server_stats reports queued samples, finalizes
 * in flight and the device bytes of open streams.  A server is not
 * thread-safe. */
typedef struct pcal_server_ctx *pcal_server_t;
int pcal_server_create(int64_t mem_budget_bytes, int max_streams, int precision, pcal_server_t *out);
int pcal_server_open(pcal_server_t s, int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits,
                     int sideband, int64_t integration_samples, int *sid);
int pcal_server_close(pcal_server_t s, int sid);
int pcal_server_submit(pcal_server_t s, int count, const int *sids, const void *const *dev_ptrs,
                       const int64_t *nsamples);
int pcal_server_step(pcal_server_t s, pcal_stream_t stream, int64_t *samples_dispatched);
int pcal_server_poll(pcal_server_t s, int max, int *sids, int64_t *integrations, int *n);
int pcal_server_result(pcal_server_t s, int sid, int64_t integration, double *amp, double *phase, double *delay);
int pcal_server_spectrum(pcal_server_t s, int sid, int64_t integration, double *re, double *im);
int pcal_server_stats(pcal_server_t s, int64_t *queued_samples, int *inflight_finalizes, int64_t *device_bytes);
int pcal_server_destroy(pcal_server_t s);

/* Device-resident form of the served loop.  pcal_server_start launches one
 * persistent kernel of `workgroups` workgroups (2 to 2048; at most as many as
 * are resident at once on the device is the useful range) on `stream`; from
 * then on pcal_server_step launches nothing: it publishes the queued pieces
 * (split at integration boundaries, every queued piece that fits, not one per
 * stream) as descriptors in a work ring of 512 chunks in pinned, coherent
 * host memory and returns.  Workgroup 0 of the kernel schedules: it reads the
 * count of published chunks, copies each new descriptor into device memory
 * and hands the chunks' fold tasks (one per 128 KiB of the chunk,
 * PCAL_SERVED_TASK_KIB, or per 2 MiB, PCAL_SERVED_BACKLOG_TASK_KIB, when
 * the chunk published 32 chunks earlier, PCAL_SERVED_BACKLOG, has not yet
 * ended; at least its column tiles, at most 32, PCAL_SERVED_TASKS) in
 * order to idle workgroups through per-workgroup
 * mailboxes in device memory.  The other workgroups fold their task into the
 * stream's accumulator bank in HBM (two banks per stream, alternating by
 * integration); the task that completes an integration runs its FP64
 * finalize, writes the results into the stream's pinned result slot and
 * appends a completion record that pcal_server_poll reads.  A piece that
 * completes an integration is published only after the stream's previous
 * integration has been reported.  The loop leaves when pcal_server_stop sets
 * the quit flag, or about 4 s after its last work (PCAL_SERVED_IDLE_MS),
 * each time with every published task ended (on quit, at most 1 s later
 * even if not: pcal_server_stop sets quit only after the published work
 * ended or its wait ran out, which it reports), so the kernel always ends;
 * pcal_server_step launches it again when every workgroup has left and work
 * comes.  The kernel runs on a non-blocking stream of the server's own (after
 * the work already enqueued on `stream`): a device-wide synchronisation
 * (hipDeviceSynchronize) waits for it, so call pcal_server_stop first.
 * pcal_server_stop waits (up to 30 s) for the published work, sets the quit
 * flag and waits for the kernel; the server continues in the host-step form.
 * pcal_server_close and pcal_server_destroy wait for published work first.
 * Streams need the period fold, at most 1792 tones and a fold period of at
 * most 32 column tiles in this form (PCAL_ENOTSUP otherwise, at start or
 * open), and the
 * batch workgroup size of 512 threads (PCAL_BATCH_THREADS unset).
 * Errors: PCAL_EINVAL (workgroups outside 2..2048), PCAL_ESTATE (already
 * started / not started), PCAL_ENOTSUP, PCAL_ENOMEM, PCAL_EHIP (a launch
 * failed, or the published work did not end in time). */
int pcal_server_start(pcal_server_t s, int workgroups, pcal_stream_t stream);
int pcal_server_stop(pcal_server_t s);

/* Counters of the device-resident loop since pcal_server_start (observability
 * of the loop, not part of the extraction).  Writes min(n, PCAL_LOOP_STATS)
 * values to out (host memory of the caller), in this order:
 *   [0] chunks published, [1] fold tasks run, [2] fold tasks published
 *   (equal to [1] once the published work has ended), [3] descriptors
 *   the scheduler copied into device memory, [4] scheduler rounds (each reads
 *   the host's count once), [5] integrations finalized, [6] relaunches of the
 *   kernel, [7] scheduler rounds that handed out nothing, then worker time
 *   summed over tasks, in ns: [8] waiting for the task (from the end of the
 *   previous one), [9] reading the descriptor, [10] folding, [11] counting
 *   and finalizing, [12] of that, finalizing (summed over integrations).
 * The scheduler adds its counts ([3], [4], [7]) when the loop leaves; the
 * others are read while the kernel runs, each value on its own, so the set is
 * a consistent snapshot only after pcal_server_stop; it is kept until the
 * next pcal_server_start.
 * Errors: PCAL_EINVAL (null s or out, n < 0), PCAL_ESTATE (never started). */
#define PCAL_LOOP_STATS 13
int pcal_server_loop_stats(pcal_server_t s, int64_t *out, int n);

/* Streaming-read reference (not part of the extraction): reads `bytes`
 * bytes at dev_ptr once with 16-byte non-temporal loads, as the fold kernel
 * reads its input, in `blocks` workgroups of `threads` threads, each
 * workgroup owning a contiguous slice, and writes the XOR of the 64-bit words
 * each wave read to out[wave] (device memory owned by the caller, at least
 * blocks * threads / 64 words).  Its duration, taken with start_event /
 * stop_event as in pcal_extract_timed, is the measured ceiling the
 * bandwidth-bound kernels are compared with.  Asynchronous on stream.
 * Errors: PCAL_EINVAL for a null or misaligned (16-byte) pointer, bytes not a
 * positive multiple of 16, threads not a multiple of 64 in [64, 1024], or
 * blocks < 1; PCAL_EHIP. */
int pcal_read_probe(const void *dev_ptr, int64_t bytes, int blocks, int threads, uint64_t *out,
                    pcal_stream_t stream, void *start_event, void *stop_event);

/* ---- Allocation-free extraction -------------------------------------------
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  One call is
 * one integration of the period-fold FP64 form, what pcal_create +
 * pcal_extract + pcal_results_async + pcal_destroy compute for the same
 * arguments, with no allocation and no host-to-device copy: the rotator
 * tables, accumulators and counters live in a fixed device array of
 * PCAL_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from its first
 * use on that GPU until the process ends, and the tables are computed on the
 * device.
 *   Parameters as pcal_create; the global sample index of dev_ptr's first
 *   sample is 0.  nsamples as pcal_extract (0 gives an empty integration).
 *   dev_out: device memory of 4N + 1 doubles, owned by the caller, that
 *   receives amp[0..N), phase[N..2N), Re C[2N..3N), Im C[3N..4N), delay[4N]
 *   (the layout of pcal_results_async's host_out).
 * Asynchronous on stream: dev_ptr and dev_out must stay valid until the
 * stream has passed the call.  Every call on one GPU uses that GPU's one
 * array and leaves its contents there (each call clears what must start at
 * zero): calls that overlap on one GPU (on different streams or from several
 * host threads) race and give wrong results; calls ordered on one stream do
 * not.
 * Errors: PCAL_EINVAL (parameters as pcal_create; null dev_out; nsamples
 * negative or not a multiple of the samples per byte; tables and
 * accumulators larger than the array, with the sizes in pcal_last_error()),
 * PCAL_ENOTSUP (the stream needs a per-sample form: fold period over 2^23
 * samples, or fs >= 2^32 Hz), PCAL_EHIP. */
#define PCAL_NOALLOC_SCRATCH_BYTES (4 << 20)
int pcal_extract_noalloc(int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int sideband,
                         const void *dev_ptr, int64_t nsamples, double *dev_out, pcal_stream_t stream);

/* Text of a status code. */
const char *pcal_strerror(int code);

/* Text of the last HIP error seen by the library in this thread ("" if none). */
const char *pcal_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PCAL_H */
