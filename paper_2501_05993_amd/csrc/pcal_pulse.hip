// Time-domain pulse of an integration (Section 2): the rotated, folded bins
// P[b] of Eqs. 2-3, read out of the accumulator slots, and the delay at the
// power peak of that pulse (Section 2's interpolation near the largest bin,
// Section 3's group delay at maximum power).  One workgroup, launched once per
// readout; it reads N x kAccSlots bins and writes 2N + 4 doubles.
//
// Delay estimate.  The peak bin b0 is the first bin of largest power.  The
// pulse of N equal tones is a periodic sinc whose amplitude envelope is
// c / |sin(pi (b - x0) / N)| (a hyperbola near the peak, made periodic);
// fitted through the amplitudes of b0 and of its larger neighbour b0 + s it
// gives the offset d in [0, 1/2] from tan(u d) = a_s sin u / (a_0 + a_s cos u),
// u = pi / N, exact for an equal-amplitude comb at any delay.  Equal
// neighbours give d = 0.  The position b0 + s d, taken in (-N/2, N/2], is
// turned into a delay in the convention of the phase-slope delay: -pos / fs
// for an upper sideband, +pos / fs for a lower one.
//
// Multi-pass refinement (refine_kernel, below): passes over the tone responses
// that counter-rotate by the current delay and fit the residual phase slope.
//
// Delay-corrected band-pass (Section 3): given the reported spectrum C_k, the
// phases arg(C_k exp(-j 2 pi f_k t)) with t that delay, f_k = f_offset +
// k f_comb: flat for a comb whose phases grow as 2 pi f_k t.
#include "pcal.h"
#include "pcal_internal.h"

namespace pcal {
namespace {

constexpr int kPulseThreads = 256;

// Bin i with the accumulator slots added in slot order (as the finalize adds them).
__device__ __forceinline__ double2 pulse_bin(const PulseArgs &a, int i) {
    return slot_sum(a.acc, a.accf, a.prec == PCAL_PREC_F32, a.N, i);
}

// Bin i times the form's known gain (the mixed form's table gain, the
// fixed-point form's 2^-17; 1 otherwise): the P[b] whose DFT is the reported C_k.
__device__ __forceinline__ double2 pulse_val(const PulseArgs &a, int i) {
    const double2 p = pulse_bin(a, i);
    return make_double2(p.x * a.gain_re - p.y * a.gain_im, p.x * a.gain_im + p.y * a.gain_re);
}

// |p|^2 with both products rounded before the add (no fused multiply-add), so
// the peak is chosen on the same values a plain FP64 evaluation gives.
__device__ __forceinline__ double power_of(double2 p) {
    return __dadd_rn(__dmul_rn(p.x, p.x), __dmul_rn(p.y, p.y));
}

// Offset and delay of the pulse peak at bin b0 of power p0; writes
// out[2N .. 2N + 3] and returns the delay.
__device__ double peak_delay(const PulseArgs &a, int b0, double p0) {
    const int N = a.N;
    const double a0 = sqrt(p0);
    const double am = sqrt(power_of(pulse_val(a, b0 == 0 ? N - 1 : b0 - 1)));
    const double ap = sqrt(power_of(pulse_val(a, b0 == N - 1 ? 0 : b0 + 1)));
    int s = 0;
    double as = 0.0;
    if (ap > am) {
        s = 1;
        as = ap;
    } else if (am > ap) {
        s = -1;
        as = am;
    }
    const double u = M_PI / N;
    const double d = s ? atan2(as * sin(u), a0 + as * cos(u)) / u : 0.0;
    double pos = b0 + s * d;
    if (pos > 0.5 * N) pos -= N;
    const double delay = (a.sideband > 0 ? -pos : pos) / a.fs;
    a.out[2 * N] = delay;
    a.out[2 * N + 1] = b0;
    a.out[2 * N + 2] = s * d;
    a.out[2 * N + 3] = p0 * a.inv_L * a.inv_L;
    return delay;
}

__global__ void __launch_bounds__(kPulseThreads) pulse_kernel(PulseArgs a) {
    __shared__ double s_pw[kPulseThreads];
    __shared__ int s_ix[kPulseThreads];
    __shared__ double s_delay;
    const int N = a.N, t = static_cast<int>(threadIdx.x);
    double best = -1.0;  // below any power: a thread without bins never wins
    int bi = 0;
    for (int i = t; i < N; i += kPulseThreads) {
        const double2 p = pulse_val(a, i);
        a.out[i] = p.x;
        a.out[N + i] = p.y;
        if (a.out_int) {
            long long s = 0;
            for (int k = 0; k < kAccSlots; ++k) s += a.acc_int[k * N + i];
            a.out_int[i] = s;
        }
        const double pw = power_of(p);
        if (pw > best) {  // bins visited in increasing order: ties keep the first
            best = pw;
            bi = i;
        }
    }
    s_pw[t] = best;
    s_ix[t] = bi;
    __syncthreads();
    for (int w = kPulseThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            const double o = s_pw[t + w];
            const int oi = s_ix[t + w];
            if (o > s_pw[t] || (o == s_pw[t] && oi < s_ix[t])) {
                s_pw[t] = o;
                s_ix[t] = oi;
            }
        }
        __syncthreads();
    }
    if (t == 0) s_delay = peak_delay(a, s_ix[0], s_pw[0]);
    if (!a.spec) return;
    __syncthreads();
    const double delay = s_delay;
    for (int k = t; k < N; k += kPulseThreads) {
        const double th = 2.0 * M_PI * (a.f_offset + k * a.f_comb) * delay;
        const double c = cos(th), sn = sin(th);
        const double re = a.spec[k], im = a.spec[N + k];
        a.out[2 * N + 4 + k] = atan2(im * c - re * sn, re * c + im * sn);
    }
}

// Sum of v over the workgroup (every thread gets it).
__device__ double block_sum(double v, double *red) {
    const int t = static_cast<int>(threadIdx.x);
    red[t] = v;
    __syncthreads();
    for (int w = kPulseThreads / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Multi-pass refinement of the delay (Section 2: a coarse delay off the pulse,
// then passes that counter-rotate by the current estimate and measure the
// residual phase).  The counter-rotation by a delay t turns tone k by
// exp(-j 2 pi f_k t); each pass takes the residual phases psi of the in-band
// tones, unwraps them along increasing frequency (wrapped neighbour
// differences, prefix-summed: per-thread runs of consecutive tones, their
// totals scanned by one thread) and fits the least-squares line
// psi = a + 2 pi f t_res with the frequencies centred on their mean (their
// spread is the closed form f_comb^2 n (n^2 - 1) / 12); the estimate moves to
// t + t_res.
__global__ void __launch_bounds__(kPulseThreads) refine_kernel(RefineArgs a) {
    extern __shared__ double sh[];
    __shared__ double part[kPulseThreads];
    __shared__ double red[kPulseThreads];
    __shared__ double s_t;
    const int n = a.k_hi - a.k_lo, t = static_cast<int>(threadIdx.x), nt = kPulseThreads;
    double *psi = sh;
    if (t == 0) {
        s_t = *a.t0;
        a.out[0] = s_t;
    }
    __syncthreads();
    if (n < 2) {  // no line to fit: the estimate stays
        if (t == 0) {
            for (int i = 1; i <= a.iters; ++i) a.out[i] = s_t;
            a.out[a.iters + 1] = 0.0;
            a.out[a.iters + 2] = 0.0;
        }
        return;
    }
    const double two_pi = 6.283185307179586476925286766559;
    const int per = (n + nt - 1) / nt;
    const int c0 = min(n, t * per), c1 = min(n, c0 + per);
    const double fm = a.f_offset + a.f_comb * (a.k_lo + 0.5 * (n - 1));
    const double sff = a.f_comb * a.f_comb * static_cast<double>(n) * (static_cast<double>(n) * n - 1.0) / 12.0;
    for (int pass = 1; pass <= a.iters; ++pass) {
        const double tc = s_t;
        for (int i = c0; i < c1; ++i) {
            const int k = a.k_lo + i;
            const double f = a.f_offset + static_cast<double>(k) * a.f_comb;
            double sn, c;
            sincos(two_pi * f * tc, &sn, &c);
            const double re = a.spec[k], im = a.spec[a.N + k];
            psi[i] = atan2(im * c - re * sn, re * c + im * sn);  // arg(C_k exp(-j 2 pi f_k t))
        }
        __syncthreads();
        double run = 0.0;
        for (int i = c0 > 0 ? c0 : 1; i < c1; ++i) {
            const double d = psi[i] - psi[i - 1];
            run += d - two_pi * rint(d / two_pi);
        }
        part[t] = run;
        __syncthreads();
        if (t == 0) {
            double acc = 0.0;
            for (int j = 0; j < nt; ++j) {
                const double v = part[j];
                part[j] = acc;
                acc += v;
            }
        }
        __syncthreads();
        // unwrapped phases of this thread's run, kept in registers across the sums
        double su = 0.0, sfu = 0.0;
        {
            double u = psi[0] + part[t];
            for (int i = c0; i < c1; ++i) {
                if (i > 0) {
                    const double d = psi[i] - psi[i - 1];
                    u += d - two_pi * rint(d / two_pi);
                }
                const double fc = a.f_comb * (static_cast<double>(i) - 0.5 * (n - 1));  // f_i - fm
                su += u;
                sfu += fc * u;
            }
        }
        const double um = block_sum(su, red) / n;
        const double slope = block_sum(sfu, red) / sff;
        double sr = 0.0;
        {
            double u = psi[0] + part[t];
            for (int i = c0; i < c1; ++i) {
                if (i > 0) {
                    const double d = psi[i] - psi[i - 1];
                    u += d - two_pi * rint(d / two_pi);
                }
                const double r = u - um - slope * a.f_comb * (static_cast<double>(i) - 0.5 * (n - 1));
                sr += r * r;
            }
        }
        const double rss = block_sum(sr, red);
        if (t == 0) {
            s_t = tc + slope / two_pi;
            a.out[pass] = s_t;
            if (pass == a.iters) {
                a.out[a.iters + 1] = um - slope * fm;
                a.out[a.iters + 2] = sqrt(rss / n);
            }
        }
        __syncthreads();
    }
}

}  // namespace

void launch_pulse(const PulseArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(pulse_kernel, dim3(1), dim3(kPulseThreads), 0, s, a);
}

void launch_refine(const RefineArgs &a, hipStream_t s) {
    const size_t lds = sizeof(double) * static_cast<size_t>(a.k_hi > a.k_lo ? a.k_hi - a.k_lo : 1);
    hipLaunchKernelGGL(refine_kernel, dim3(1), dim3(kPulseThreads), lds, s, a);
}

}  // namespace pcal
