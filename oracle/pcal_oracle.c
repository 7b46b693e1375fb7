/*
 * pcal_oracle.c -- plain, slow, FP64 reference for multi-tone phase-calibration
 * extraction.  TEST INFRASTRUCTURE ONLY: it is built and called by the tests,
 * by the smoke check and by the benchmark's CPU-baseline leg.  The product
 * library never links, loads or calls it, and it shares no code with it.
 *
 * What it computes
 * ----------------
 * The extraction method (Section 2: rotate by exp(-j*w_offset*n), Eq. 3; fold
 * by n mod N, Eq. 2; one DFT of the N bins) reaches, up to rounding order, the
 * plain per-tone correlation
 *
 *     C_k = sum_{n} x[n] * exp(-j * 2*pi * (k*f_comb + f_offset) * n / fs),
 *     k = 0 .. N-1,   N = fs / f_comb,
 *
 * because exp(-j*2*pi*k*(n mod N)/N) = exp(-j*2*pi*k*n/N).  This file writes
 * that definition out directly, tone by tone and sample by sample, with no
 * folding, no rotator table of the method and no transform:
 *
 *   * the phase of sample n for tone k is reduced exactly in integers:
 *     with g = gcd(fs, f_comb, f_offset), P = fs/g and a_k = (k*f_comb+f_offset)/g,
 *     the angle is 2*pi*((a_k*n) mod P)/P;
 *   * exp(-j*2*pi*m/P) comes from libm cos/sin of an argument reduced to
 *     |angle| <= pi (a table of P entries when P is small, direct calls otherwise);
 *   * sums run in FP64 with Neumaier compensation per block of samples, and the
 *     block sums are added pairwise in block order (deterministic).
 *
 * It also provides the integer fold of Eq. 2 (bins P[b] = sum of x[n] with
 * n = b mod N, exact in int64), the rotated fold of Eqs. 2-3 (the pulse
 * P[b] = sum of x[n] exp(-j*w_offset*n), with the same exact phase index),
 * and its own decoder of the packed samples
 * (2-bit offset-binary LSB-first codes -> levels {-3,-1,+1,+3}; 8-bit two's
 * complement), written independently of the library's unpacking.
 *
 * Global sample index: every entry point takes n0, the index of the first
 * sample passed, so a stream split into chunks gives the same result as one
 * long call (phase continuity across calls).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

#define ORC_BLOCK 65536          /* samples per compensated partial sum */
#define ORC_TABLE_MAX (1 << 22)  /* largest phasor table built (64 MiB) */

static const double ORC_TWO_PI = 6.283185307179586476925286766559;

static int64_t orc_gcd(int64_t a, int64_t b)
{
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

/* Decoded level of sample i of a packed stream. */
static inline int orc_level(const uint8_t *packed, int nbits, int64_t i)
{
    if (nbits == 2) {
        int code = (packed[i >> 2] >> (2 * (int)(i & 3))) & 3;
        return 2 * code - 3;
    }
    return (int)(int8_t)packed[i];
}

int orc_decode(const uint8_t *packed, int nbits, int64_t nsamples, int8_t *out)
{
    if (!packed || !out || nsamples < 0 || (nbits != 2 && nbits != 8)) return ORC_EINVAL;
    for (int64_t i = 0; i < nsamples; i++) out[i] = (int8_t)orc_level(packed, nbits, i);
    return ORC_OK;
}

/* exp(-j*2*pi*m/P) for 0 <= m < P, with the argument reduced to [-pi, pi]. */
static inline void orc_phasor(int64_t m, int64_t P, double *c, double *s)
{
    double ang;
    if (2 * m <= P)
        ang = ORC_TWO_PI * (double)m / (double)P;
    else
        ang = -ORC_TWO_PI * (double)(P - m) / (double)P;
    *c = cos(ang);
    *s = -sin(ang);
}

/* Neumaier-compensated accumulator. */
typedef struct {
    double s, c;
} orc_acc;

static inline void orc_add(orc_acc *a, double y)
{
    double t = a->s + y;
    if (fabs(a->s) >= fabs(y))
        a->c += (a->s - t) + y;
    else
        a->c += (y - t) + a->s;
    a->s = t;
}

/* Pairwise sum of v[0..n) (in index order). */
static double orc_pairwise(const double *v, int64_t n)
{
    if (n <= 0) return 0.0;
    if (n == 1) return v[0];
    int64_t h = n / 2;
    return orc_pairwise(v, h) + orc_pairwise(v + h, n - h);
}

typedef struct {
    const uint8_t *packed; /* one of packed / samples is set */
    const double *samples;
    int nbits;
} orc_src;

static inline double orc_sample(const orc_src *src, int64_t i)
{
    if (src->samples) return src->samples[i];
    return (double)orc_level(src->packed, src->nbits, i);
}

static int orc_correlate(const orc_src *src, int64_t nsamples, int64_t n0, int64_t fs, int64_t fc,
                         int64_t fo, int ntones, const int32_t *tones, int nthreads, double *re,
                         double *im)
{
    if (nsamples < 0 || n0 < 0 || fs <= 0 || fc <= 0 || fo < 0 || fo >= fs || fs % fc) return ORC_EINVAL;
    if (ntones < 0 || (ntones && (!tones || !re || !im))) return ORC_EINVAL;
    const int64_t N = fs / fc;
    for (int t = 0; t < ntones; t++)
        if (tones[t] < 0 || tones[t] >= N) return ORC_EINVAL;

    const int64_t g = orc_gcd(orc_gcd(fs, fc), fo);
    const int64_t P = fs / g;
    double *tab = NULL;
    if (P <= ORC_TABLE_MAX) {
        tab = (double *)malloc(sizeof(double) * 2 * (size_t)P);
        if (!tab) return ORC_ENOMEM;
        for (int64_t m = 0; m < P; m++) orc_phasor(m, P, &tab[2 * m], &tab[2 * m + 1]);
    }
    const int64_t nblk = (nsamples + ORC_BLOCK - 1) / ORC_BLOCK;
    const int64_t ntask = nblk * (int64_t)ntones;
    double *pre = (double *)malloc(sizeof(double) * (size_t)(ntask > 0 ? ntask : 1));
    double *pim = (double *)malloc(sizeof(double) * (size_t)(ntask > 0 ? ntask : 1));
    if (!pre || !pim) {
        free(tab);
        free(pre);
        free(pim);
        return ORC_ENOMEM;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t task = 0; task < ntask; task++) {
        const int64_t b = task / ntones;
        const int t = (int)(task % ntones);
        const int64_t k = tones[t];
        const int64_t a = ((k * fc + fo) / g) % P; /* phase index step per sample */
        const int64_t i0 = b * ORC_BLOCK;
        const int64_t i1 = (i0 + ORC_BLOCK < nsamples) ? i0 + ORC_BLOCK : nsamples;
        /* exact phase index of the first sample of the block: (a * (n0 + i0)) mod P */
        int64_t m = (int64_t)(((unsigned __int128)(uint64_t)a * (uint64_t)((n0 + i0) % P)) % (uint64_t)P);
        orc_acc sr = {0.0, 0.0}, si = {0.0, 0.0};
        for (int64_t i = i0; i < i1; i++) {
            double c, s;
            if (tab) {
                c = tab[2 * m];
                s = tab[2 * m + 1];
            } else {
                orc_phasor(m, P, &c, &s);
            }
            const double x = orc_sample(src, i);
            orc_add(&sr, x * c);
            orc_add(&si, x * s);
            m += a;
            if (m >= P) m -= P;
        }
        pre[t * nblk + b] = sr.s + sr.c;
        pim[t * nblk + b] = si.s + si.c;
    }
    for (int t = 0; t < ntones; t++) {
        re[t] = orc_pairwise(pre + t * nblk, nblk);
        im[t] = orc_pairwise(pim + t * nblk, nblk);
    }
    free(tab);
    free(pre);
    free(pim);
    return ORC_OK;
}

int orc_correlate_packed(const uint8_t *packed, int nbits, int64_t nsamples, int64_t n0, int64_t fs,
                         int64_t fc, int64_t fo, int ntones, const int32_t *tones, int nthreads,
                         double *re, double *im)
{
    if ((!packed && nsamples > 0) || (nbits != 2 && nbits != 8)) return ORC_EINVAL;
    orc_src src = {packed, NULL, nbits};
    return orc_correlate(&src, nsamples, n0, fs, fc, fo, ntones, tones, nthreads, re, im);
}

int orc_correlate_f64(const double *samples, int64_t nsamples, int64_t n0, int64_t fs, int64_t fc,
                      int64_t fo, int ntones, const int32_t *tones, int nthreads, double *re, double *im)
{
    if (!samples && nsamples > 0) return ORC_EINVAL;
    orc_src src = {NULL, samples, 0};
    return orc_correlate(&src, nsamples, n0, fs, fc, fo, ntones, tones, nthreads, re, im);
}

/* Per-tone correlation with a supplied rotator in place of exp(-j w_o n):
 *
 *     C_k = sum_n x[n] * U[m(n)] * V[n mod N] * exp(-j 2 pi k (n mod N) / N),
 *     m(n) = (n mod (M*N)) div N,
 *
 * i.e. Eq. 3 with the rotator read from a table that repeats every M*N
 * samples and is split into a row factor U (M entries) and a column factor
 * V (N entries).  With the exact U[m] = exp(-j w_o N m), V[b] = exp(-j w_o b)
 * this equals the plain C_k above; with rounded tables it is the exact-
 * arithmetic value of an extraction that rotates by those rounded values
 * (used to check reduced-precision forms).  Sums as in orc_correlate. */
int orc_correlate_rotator(const uint8_t *packed, int nbits, int64_t nsamples, int64_t n0, int64_t nbins,
                          int64_t rows, const double *u_re, const double *u_im, const double *v_re,
                          const double *v_im, int ntones, const int32_t *tones, int nthreads, double *re,
                          double *im)
{
    if ((!packed && nsamples > 0) || (nbits != 2 && nbits != 8) || nsamples < 0 || n0 < 0 || nbins <= 0 ||
        rows <= 0 || !u_re || !u_im || !v_re || !v_im || ntones < 0 || (ntones && (!tones || !re || !im)))
        return ORC_EINVAL;
    for (int t = 0; t < ntones; t++)
        if (tones[t] < 0 || tones[t] >= nbins) return ORC_EINVAL;
    const int64_t period = rows * nbins;
    double *tw = (double *)malloc(sizeof(double) * 2 * (size_t)nbins);
    const int64_t nblk = (nsamples + ORC_BLOCK - 1) / ORC_BLOCK;
    const int64_t ntask = nblk * (int64_t)ntones;
    double *pre = (double *)malloc(sizeof(double) * (size_t)(ntask > 0 ? ntask : 1));
    double *pim = (double *)malloc(sizeof(double) * (size_t)(ntask > 0 ? ntask : 1));
    if (!tw || !pre || !pim) {
        free(tw);
        free(pre);
        free(pim);
        return ORC_ENOMEM;
    }
    for (int64_t j = 0; j < nbins; j++) orc_phasor(j, nbins, &tw[2 * j], &tw[2 * j + 1]);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t task = 0; task < ntask; task++) {
        const int64_t b = task / ntones;
        const int t = (int)(task % ntones);
        const int64_t k = tones[t];
        const int64_t i0 = b * ORC_BLOCK;
        const int64_t i1 = (i0 + ORC_BLOCK < nsamples) ? i0 + ORC_BLOCK : nsamples;
        int64_t q = (n0 + i0) % period; /* position in the rotator period */
        orc_acc sr = {0.0, 0.0}, si = {0.0, 0.0};
        for (int64_t i = i0; i < i1; i++) {
            const int64_t col = q % nbins, row = q / nbins;
            /* rotator U[row] * V[col], then the tone's twiddle exp(-j 2 pi k col / N) */
            const double rr = u_re[row] * v_re[col] - u_im[row] * v_im[col];
            const double ri = u_re[row] * v_im[col] + u_im[row] * v_re[col];
            const int64_t w = (k * col) % nbins;
            const double cr = rr * tw[2 * w] - ri * tw[2 * w + 1];
            const double ci = rr * tw[2 * w + 1] + ri * tw[2 * w];
            const double x = (double)orc_level(packed, nbits, i);
            orc_add(&sr, x * cr);
            orc_add(&si, x * ci);
            if (++q == period) q = 0;
        }
        pre[t * nblk + b] = sr.s + sr.c;
        pim[t * nblk + b] = si.s + si.c;
    }
    for (int t = 0; t < ntones; t++) {
        re[t] = orc_pairwise(pre + t * nblk, nblk);
        im[t] = orc_pairwise(pim + t * nblk, nblk);
    }
    free(tw);
    free(pre);
    free(pim);
    return ORC_OK;
}

/* Eq. 2: P[b] = sum of x[n] over n = b (mod N), n = n0 .. n0+nsamples-1, exact in int64. */
int orc_fold_int(const uint8_t *packed, int nbits, int64_t nsamples, int64_t n0, int64_t nbins,
                 int64_t *bins)
{
    if ((!packed && nsamples > 0) || !bins || nbins <= 0 || n0 < 0 || nsamples < 0 ||
        (nbits != 2 && nbits != 8))
        return ORC_EINVAL;
    memset(bins, 0, sizeof(int64_t) * (size_t)nbins);
    int64_t b = n0 % nbins;
    for (int64_t i = 0; i < nsamples; i++) {
        bins[b] += orc_level(packed, nbits, i);
        if (++b == nbins) b = 0;
    }
    return ORC_OK;
}

/* Eqs. 2-3 (Section 2): the rotated, folded bins
 *   P[b] = sum of x[n] exp(-j 2 pi f_o n / fs) over n = b (mod N),
 * n = n0 .. n0+nsamples-1, N = nbins.  The phase index (f_o n) mod fs is kept
 * exact in integers (reduced by g = gcd(fs, f_o)); each bin is one compensated
 * sum over its samples in increasing n.  The plain definition of the pulse
 * whose DFT is C_k (Section 2). */
int orc_fold_rot(const uint8_t *packed, int nbits, int64_t nsamples, int64_t n0, int64_t fs, int64_t fo,
                 int64_t nbins, int nthreads, double *re, double *im)
{
    if ((!packed && nsamples > 0) || (nbits != 2 && nbits != 8) || nsamples < 0 || n0 < 0 || fs <= 0 ||
        fo < 0 || fo >= fs || nbins <= 0 || !re || !im)
        return ORC_EINVAL;
    const int64_t g = orc_gcd(fs, fo);
    const int64_t P = fs / g;
    const int64_t a = (fo / g) % P; /* phase index step per sample */
    /* phase index step between consecutive samples of one bin: (a * N) mod P */
    const int64_t da = (int64_t)(((unsigned __int128)(uint64_t)a * (uint64_t)(nbins % P)) % (uint64_t)P);
    double *tab = NULL;
    if (P <= ORC_TABLE_MAX) {
        tab = (double *)malloc(sizeof(double) * 2 * (size_t)P);
        if (!tab) return ORC_ENOMEM;
        for (int64_t m = 0; m < P; m++) orc_phasor(m, P, &tab[2 * m], &tab[2 * m + 1]);
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nbins; b++) {
        /* first sample i >= 0 with (n0 + i) = b (mod N) */
        const int64_t i0 = ((b - n0 % nbins) % nbins + nbins) % nbins;
        int64_t m = (int64_t)(((unsigned __int128)(uint64_t)a * (uint64_t)((n0 + i0) % P)) % (uint64_t)P);
        orc_acc sr = {0.0, 0.0}, si = {0.0, 0.0};
        for (int64_t i = i0; i < nsamples; i += nbins) {
            double c, s;
            if (tab) {
                c = tab[2 * m];
                s = tab[2 * m + 1];
            } else {
                orc_phasor(m, P, &c, &s);
            }
            const double x = (double)orc_level(packed, nbits, i);
            orc_add(&sr, x * c);
            orc_add(&si, x * s);
            m += da;
            if (m >= P) m -= P;
        }
        re[b] = sr.s + sr.c;
        im[b] = si.s + si.c;
    }
    free(tab);
    return ORC_OK;
}

/* Eqs. 2-3 with the rotator given as a table of integers (the fixed-point
 * rotator of Section 4.8: each rotator value scaled and rounded to an integer,
 * products and sums in integers):
 *   P[b] = sum of x[n] * T[n mod R] over n = b (mod N), n = n0 .. n0+nsamples-1,
 * T[r] = t_re[r] + j t_im[r], exact in int64 (no rounding anywhere). */
int orc_fold_table_int(const uint8_t *packed, int nbits, int64_t nsamples, int64_t n0, int64_t nbins, int64_t R,
                       const int32_t *t_re, const int32_t *t_im, int64_t *re, int64_t *im)
{
    if ((!packed && nsamples > 0) || (nbits != 2 && nbits != 8) || nsamples < 0 || n0 < 0 || nbins <= 0 ||
        R <= 0 || !t_re || !t_im || !re || !im)
        return ORC_EINVAL;
    memset(re, 0, sizeof(int64_t) * (size_t)nbins);
    memset(im, 0, sizeof(int64_t) * (size_t)nbins);
    int64_t b = n0 % nbins, r = n0 % R;
    for (int64_t i = 0; i < nsamples; i++) {
        const int64_t x = orc_level(packed, nbits, i);
        re[b] += x * t_re[r];
        im[b] += x * t_im[r];
        if (++b == nbins) b = 0;
        if (++r == R) r = 0;
    }
    return ORC_OK;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
