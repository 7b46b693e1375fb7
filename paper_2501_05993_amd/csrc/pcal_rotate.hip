// Per-sample rotation forms of libpcal: every sample is multiplied by the
// rotator exp(-j w_o n) of Eq. 3 before it is folded into bin n mod N (Eq. 2).
// The rotator comes either from a precomputed table of one rotator period
// (Eq. 4, the precomputed method of Section 4.1), from the direct-form
// resonator recurrence y[r+1] = 2 cos(d) y[r] - y[r-1] (Eq. 6-7, the
// oscillator method), from the coupled-form oscillator z[r+1] = z[r]
// exp(-j d) or the magic-circle oscillator (the first two recursions Section
// 2.2 lists), or from the resonator with truncation-error feedback (one of the
// remedies Section 2.2 names for the resonator's rounding); every recurrence is
// re-seeded exactly at fixed intervals.
//
// Layout.  A thread owns 16 consecutive samples of every row (one 16-byte
// load at 8-bit, one 4-byte load at 2-bit); rows are a multiple of N samples,
// so each of the thread's 16 lanes always lands in the same bin.  Sample n of
// lane i in row r is n = n_r + i with n_r the row's first sample of the
// thread, and exp(-j w_o n) = exp(-j w_o n_r) exp(-j w_o i): the row factor
// z_r is produced once per row (table read or one recurrence step), every
// sample costs two FMAs against it, and the fixed lane factor exp(-j w_o i)
// is applied once per lane at the end, in FP64.
//
// Arithmetic by precision form.  F64: FP64 table entries or FP64 recurrence
// state, FP64 products, run sums and totals.  MIXED: table entries as two
// FP16 terms summed in FP32 (or FP32 recurrence state), FP32 products and run
// sums, Kahan-compensated FP32 totals.  F32: FP32 throughout up to the lane
// totals.  Workgroup bins and the cross-workgroup sums are FP64 except in F32.
#include <type_traits>

#include "pcal_internal.h"

namespace pcal {
namespace {

constexpr int kLanes = 16;   // samples per thread and row
constexpr int kRun = 64;     // rows per run: run sums, then folded into the lane totals
// rows loaded ahead: 8 in the FP32 forms, 4 in the FP64 form (twice the
// registers per lane sum)
template <int PREC>
constexpr int unroll_of() { return PREC == 0 ? 4 : 8; }

// Arithmetic type of the products and run sums of a precision form.
template <int PREC>
using real_t = typename std::conditional<PREC == 0, double, float>::type;

__device__ __forceinline__ float mad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double mad(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class T>
struct cplx {
    T x, y;
};

__device__ __forceinline__ int edge_level(const uint8_t *p, int nbits, int i) {
    if (nbits == 2) return 2 * ((p[i >> 2] >> (2 * (i & 3))) & 3) - 3;
    return static_cast<int>(static_cast<int8_t>(p[i]));
}

// exp(-j 2 pi (f_o n mod fs) / fs) in FP64 from an exact integer phase index (fs < 2^32).
__device__ __forceinline__ double2 exact_rotator(int64_t n, int64_t fs, int64_t fo) {
    const uint64_t nm = static_cast<uint64_t>(n % fs);
    int64_t idx = static_cast<int64_t>((static_cast<uint64_t>(fo) * nm) % static_cast<uint64_t>(fs));
    if (2 * idx > fs) idx -= fs;  // reduce the angle to (-pi, pi]
    const double ang = 6.283185307179586476925286766559 * static_cast<double>(idx) / static_cast<double>(fs);
    double s, c;
    sincos(ang, &s, &c);
    return make_double2(c, -s);
}

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// The 16 sample values of one thread-row: biased bytes x + 128
// (8-bit) or offset-binary codes c (2-bit), lane i = sample i.
template <int NBITS>
struct RowVec;

template <>
struct RowVec<8> {
    uint4 v;
    __device__ __forceinline__ void load(const void *base, int64_t idx) {
        const u32x4_t x = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(base) + idx);
        v = make_uint4(x.x ^ 0x80808080u, x.y ^ 0x80808080u, x.z ^ 0x80808080u, x.w ^ 0x80808080u);
    }
    template <class T>
    __device__ __forceinline__ T get(int i) const {
        const uint32_t w = i < 4 ? v.x : i < 8 ? v.y : i < 12 ? v.z : v.w;
        return static_cast<T>((w >> (8 * (i & 3))) & 0xFFu);
    }
};

template <>
struct RowVec<2> {
    uint32_t q[4];  // q[j]: byte lanes hold the codes of samples 4*lane + j
    __device__ __forceinline__ void load(const void *base, int64_t idx) {
        const uint32_t d = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(base) + idx);
#pragma unroll
        for (int j = 0; j < 4; ++j) q[j] = (d >> (2 * j)) & 0x03030303u;
    }
    template <class T>
    __device__ __forceinline__ T get(int i) const {
        uint32_t w = q[i & 3];
        if constexpr (std::is_same<T, float>::value) {
            // An empty statement the optimiser cannot see through: knowing that
            // every byte of w is below 4, it would extract the code with a
            // bit-field extract before a byte-0 conversion (two instructions)
            // instead of the one conversion of byte b (v_cvt_f32_ubyte<b>).
            // (The FP64 forms convert through integers either way.)
            __asm__("" : "+v"(w));
        }
        return static_cast<T>((w >> (8 * (i >> 2))) & 0xFFu);
    }
};

// Lane totals in the arithmetic of the precision form: FP64 (0), Kahan FP32 (1), FP32 (2).
template <int PREC>
struct LaneTot {
    double r[kLanes], i[kLanes];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < kLanes; ++k) r[k] = i[k] = 0.0;
    }
    __device__ __forceinline__ void add(int k, double a, double b) {
        r[k] += a;
        i[k] += b;
    }
    __device__ __forceinline__ double2 get(int k) const { return make_double2(r[k], i[k]); }
};

template <>
struct LaneTot<1> {
    float r[kLanes], i[kLanes], cr[kLanes], ci[kLanes];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < kLanes; ++k) r[k] = i[k] = cr[k] = ci[k] = 0.f;
    }
    __device__ __forceinline__ static void kahan(float y, float &s, float &c) {
        const float yc = y - c;
        const float t = s + yc;
        c = (t - s) - yc;
        s = t;
    }
    __device__ __forceinline__ void add(int k, float a, float b) {
        kahan(a, r[k], cr[k]);
        kahan(b, i[k], ci[k]);
    }
    __device__ __forceinline__ double2 get(int k) const {
        return make_double2(static_cast<double>(r[k]) - cr[k], static_cast<double>(i[k]) - ci[k]);
    }
};

template <>
struct LaneTot<2> {
    float r[kLanes], i[kLanes];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int k = 0; k < kLanes; ++k) r[k] = i[k] = 0.f;
    }
    __device__ __forceinline__ void add(int k, float a, float b) {
        r[k] += a;
        i[k] += b;
    }
    __device__ __forceinline__ double2 get(int k) const { return make_double2(r[k], i[k]); }
};

// Exact sum s + e of two values (Knuth's two-sum): s = fl(a + b).
template <class T>
__device__ __forceinline__ void two_sum(T a, T b, T &s, T &e) {
    s = a + b;
    const T bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Row rotator source: table (METHOD 2), direct-form resonator (METHOD 3),
// coupled-form oscillator (METHOD 4), magic-circle oscillator (METHOD 5) or
// the direct-form resonator with error feedback (METHOD 6), in the arithmetic
// of the precision form.
template <int METHOD, int PREC>
struct RowRot {
    using T = real_t<PREC>;
    // table state
    int64_t idx = 0, step = 0, R = 1;
    // recurrence state: the DFR runs the same two-term recurrence on the real
    // and imaginary parts (c2 = 2 cos d); the CFO multiplies the rotator by
    // m = exp(-j d) each row (d = w_o times the samples per row).  The MCO
    // keeps x = cos a and y = -sin(a + d/2) of the row angle a in zr, pr
    // (and zi unused) and steps x += eps y, y -= eps x with eps = 2 sin(d/2)
    // (the second update uses the new x); the rotator is x - j sin a with
    // -sin a = (y + x sin(d/2)) / cos(d/2).  The error-feedback DFR keeps each
    // state value as an unevaluated sum hi + lo (zr + zlr, pr + plr, ...) and
    // the coefficient as c2 + c2l: every step's rounding error, taken exactly
    // by error-free transformations, is fed back into the next step.
    T zr = 0, zi = 0, pr = 0, pi = 0, c2 = 0, mr = 0, mi = 0;
    T zlr = 0, zli = 0, plr = 0, pli = 0, c2l = 0;  // error-feedback parts
    T eps = 0, hs = 0, ihc = 0;                      // magic circle: 2 sin(d/2), sin(d/2), 1 / cos(d/2)
    int64_t n = 0, dn = 0;  // global index of the row's first lane sample, row stride in samples

    __device__ __forceinline__ cplx<T> table(const RotArgs &a, int64_t n) const {
        const int64_t k = (n & ((int64_t(1) << a.lut_shift) - 1)) * a.lut_rows + (n >> a.lut_shift);
        if constexpr (PREC == 0) {
            const double2 e = a.rot64[k];
            return {e.x, e.y};
        } else if constexpr (PREC == 1) {
            // two FP16 terms in one 8-byte load; their FP32 sum is exact
            const uint2 w = reinterpret_cast<const uint2 *>(a.rot16)[k];
            __half2 hi, lo;
            __builtin_memcpy(&hi, &w.x, 4);
            __builtin_memcpy(&lo, &w.y, 4);
            const float2 h = __half22float2(hi), l = __half22float2(lo);
            return {h.x + l.x, h.y + l.y};
        } else {
            const float2 e = a.rot32[k];
            return {e.x, e.y};
        }
    }
    // exact seed at global sample n (recurrence): z(n) and z(n - dn) in FP64, rounded once
    // (the magic circle: cos a and -sin(a + d/2), the rotator at n + dn / 2)
    __device__ __forceinline__ void seed(const RotArgs &a) {
        const double2 z = exact_rotator(n, a.fs, a.fo);
        if constexpr (METHOD == 5) {
            const double2 zh = exact_rotator(n + dn / 2, a.fs, a.fo);
            zr = static_cast<T>(z.x);
            pr = static_cast<T>(zh.y);
            return;
        }
        const double2 zp = make_double2(z.x * a.back.x - z.y * a.back.y, z.x * a.back.y + z.y * a.back.x);
        zr = static_cast<T>(z.x);
        zi = static_cast<T>(z.y);
        pr = static_cast<T>(zp.x);
        pi = static_cast<T>(zp.y);
        if constexpr (METHOD == 6) {
            zlr = static_cast<T>(z.x - static_cast<double>(zr));
            zli = static_cast<T>(z.y - static_cast<double>(zi));
            plr = static_cast<T>(zp.x - static_cast<double>(pr));
            pli = static_cast<T>(zp.y - static_cast<double>(pi));
        }
    }
    // one error-feedback resonator step on one component: (y, yl) <- c2 (y, yl) - (yp, ypl)
    __device__ __forceinline__ void ef_step(T &y, T &yl, T &yp, T &ypl) const {
        const T ph = c2 * y;
        T pl = mad(c2, y, -ph);                    // exact low part of the product c2 * y
        pl = mad(c2, yl, mad(c2l, y, pl));         // + the small cross terms
        T sh, sl;
        two_sum(ph, -yp, sh, sl);                  // exact sum of the large parts
        const T low = sl + (pl - ypl);
        const T hi = sh + low;                     // renormalise: the rounding error stays in lo
        const T lo = low - (hi - sh);
        yp = y;
        ypl = yl;
        y = hi;
        yl = lo;
    }
    // rotators of the next U rows, then move U rows on
    template <int U>
    __device__ __forceinline__ void fetch(const RotArgs &a, cplx<T> (&z)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if constexpr (METHOD == 2) {
                z[u] = table(a, idx);
                idx += step;
                if (idx >= R) idx -= R;
            } else if constexpr (METHOD == 3) {
                z[u] = {zr, zi};
                // Eq. 7: one FMA per component and row
                const T nr = mad(c2, zr, -pr), ni = mad(c2, zi, -pi);
                pr = zr;
                pi = zi;
                zr = nr;
                zi = ni;
            } else if constexpr (METHOD == 4) {
                z[u] = {zr, zi};
                // coupled form: a complex multiply by exp(-j d) per row
                const T nr = mad(zr, mr, -zi * mi), ni = mad(zr, mi, zi * mr);
                zr = nr;
                zi = ni;
            } else if constexpr (METHOD == 5) {
                // magic circle (Section 2.2's modified coupled form): x = zr, y = pr
                z[u] = {zr, mad(zr, hs, pr) * ihc};
                zr = mad(eps, pr, zr);
                pr = mad(-eps, zr, pr);
            } else {
                z[u] = {zr + zlr, zi + zli};
                ef_step(zr, zlr, pr, plr);
                ef_step(zi, zli, pi, pli);
            }
        }
        n += U * dn;
    }
};

template <int NBITS, int METHOD, int PREC>
__global__ void __launch_bounds__(kMaxRotThreads) rot_kernel(RotArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    double2 *bins = reinterpret_cast<double2 *>(lds);  // [N] workgroup bins (FP64)
    const int t = threadIdx.x, nt = blockDim.x, N = a.N;
    for (int b = t; b < N; b += nt) bins[b] = make_double2(0.0, 0.0);
    __syncthreads();

    const int c = static_cast<int>(blockIdx.x % a.col_tiles);
    const int64_t g = blockIdx.x / a.col_tiles;
    const int tc = t % a.tile_vecs, sub = t / a.tile_vecs;
    const int colp = c * a.tile_vecs + tc;
    const int colr = colp + sub * a.period_vecs;
    const int64_t r0 = g * a.rows_per_group;
    const int64_t r1 = (r0 + a.rows_per_group) < a.rows_total ? (r0 + a.rows_per_group) : a.rows_total;
    if (colp < a.period_vecs && colr < a.row_vecs && r0 < r1) {
        const int64_t stride = a.row_vecs;
        const int64_t rfull = a.nvec / stride;
        const bool last_ok = colr < a.nvec - rfull * stride;
        const int64_t rend = r1 < rfull ? r1 : (r1 > rfull && last_ok ? r1 : rfull);
        using T = real_t<PREC>;
        RowRot<METHOD, PREC> rot;
        rot.n = a.g0 + (r0 * stride + colr) * kLanes;
        rot.dn = stride * kLanes;
        if constexpr (METHOD == 2) {
            rot.R = a.R;
            rot.step = (stride * kLanes) % a.R;
            rot.idx = rot.n % a.R;
        } else {
            rot.c2 = static_cast<T>(a.c2);
            rot.c2l = static_cast<T>(a.c2 - static_cast<double>(rot.c2));
            rot.mr = static_cast<T>(a.back.x);   // exp(-j d) = conj(exp(+j d))
            rot.mi = static_cast<T>(-a.back.y);
            rot.eps = static_cast<T>(2.0 * a.half_sin);
            rot.hs = static_cast<T>(a.half_sin);
            rot.ihc = static_cast<T>(1.0 / a.half_cos);
            rot.seed(a);
        }
        LaneTot<PREC> tot;
        tot.zero();
        int64_t r = r0;
        while (r < rend) {
            const int64_t run_end = (r + kRun) < rend ? (r + kRun) : rend;
            T ar[kLanes], ai[kLanes];
#pragma unroll
            for (int k = 0; k < kLanes; ++k) ar[k] = ai[k] = T(0);
            T sr = 0, si = 0;  // sum of the row rotators of the run (bias term)
            constexpr int kUnroll = unroll_of<PREC>();
            for (; r + kUnroll <= run_end; r += kUnroll) {
                cplx<T> z[kUnroll];
                rot.fetch(a, z);  // table reads are issued with the sample loads
                RowVec<NBITS> x[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) x[u].load(a.data, (r + u) * stride + colr);
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
                    for (int k = 0; k < kLanes; ++k) {
                        const T xv = x[u].template get<T>(k);
                        ar[k] = mad(xv, z[u].x, ar[k]);
                        ai[k] = mad(xv, z[u].y, ai[k]);
                    }
                    sr += z[u].x;
                    si += z[u].y;
                }
            }
            for (; r < run_end; ++r) {
                cplx<T> z[1];
                rot.fetch(a, z);
                RowVec<NBITS> x;
                x.load(a.data, r * stride + colr);
#pragma unroll
                for (int k = 0; k < kLanes; ++k) {
                    const T xv = x.template get<T>(k);
                    ar[k] = mad(xv, z[0].x, ar[k]);
                    ai[k] = mad(xv, z[0].y, ai[k]);
                }
                sr += z[0].x;
                si += z[0].y;
            }
            // undo the affine sample map: 8-bit x = u - 128, 2-bit level = 2c - 3
#pragma unroll
            for (int k = 0; k < kLanes; ++k) {
                if constexpr (NBITS == 8)
                    tot.add(k, ar[k] - T(128) * sr, ai[k] - T(128) * si);
                else
                    tot.add(k, T(2) * ar[k] - T(3) * sr, T(2) * ai[k] - T(3) * si);
            }
            if constexpr (METHOD != 2) rot.seed(a);  // exact restart of the recurrence
        }
        // lane factor exp(-j w_o i) in FP64, then into the workgroup's bins
        const int bbase = static_cast<int>((a.g0 + static_cast<int64_t>(colr) * kLanes) % N);
#pragma unroll
        for (int k = 0; k < kLanes; ++k) {
            const double2 v = tot.get(k);
            const double2 w = a.w[k];
            const int b = (bbase + k) % N;
            atomicAdd(&bins[b].x, v.x * w.x - v.y * w.y);
            atomicAdd(&bins[b].y, v.x * w.y + v.y * w.x);
        }
    }
    // samples outside the full vectors: exact FP64 rotator per sample
    if (blockIdx.x == 0) {
        for (int part = 0; part < 2; ++part) {
            const uint8_t *src = part ? a.tail : a.head;
            const int ns = (part ? a.tail_bytes : a.head_bytes) * (8 / a.nbits);
            const int64_t n0 = part ? a.tail_n : a.head_n;
            for (int i = t; i < ns; i += nt) {
                const double2 z = exact_rotator(n0 + i, a.fs, a.fo);
                const int x = edge_level(src, a.nbits, i);
                const int b = static_cast<int>((n0 + i) % N);
                atomicAdd(&bins[b].x, x * z.x);
                atomicAdd(&bins[b].y, x * z.y);
            }
        }
    }
    __syncthreads();
    const size_t slot = static_cast<size_t>(blockIdx.x % kAccSlots) * N;
    for (int b = t; b < N; b += nt) {
        const double2 v = bins[b];
        if (v.x == 0.0 && v.y == 0.0) continue;
        if constexpr (PREC == 2) {
            unsafeAtomicAdd(&a.accf[slot + b].x, static_cast<float>(v.x));
            unsafeAtomicAdd(&a.accf[slot + b].y, static_cast<float>(v.y));
        } else {
            unsafeAtomicAdd(&a.acc[slot + b].x, v.x);
            unsafeAtomicAdd(&a.acc[slot + b].y, v.y);
        }
    }
}

}  // namespace

void launch_rotate(const RotArgs &a, int grid, int threads, size_t lds, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
    const dim3 gd(grid), bd(threads);
#define PCAL_ROT(NB, ME, PR)                                                                 \
    do {                                                                                     \
        if (t0 || t1)                                                                        \
            hipExtLaunchKernelGGL((rot_kernel<NB, ME, PR>), gd, bd, lds, s, t0, t1, 0, a);   \
        else                                                                                 \
            hipLaunchKernelGGL((rot_kernel<NB, ME, PR>), gd, bd, lds, s, a);                 \
    } while (0)
#define PCAL_ROT_P(NB, ME)                                  \
    do {                                                    \
        if (a.prec == 0) PCAL_ROT(NB, ME, 0);               \
        else if (a.prec == 1) PCAL_ROT(NB, ME, 1);          \
        else PCAL_ROT(NB, ME, 2);                           \
    } while (0)
#define PCAL_ROT_M(NB)                                      \
    do {                                                    \
        if (a.method == 2) PCAL_ROT_P(NB, 2);               \
        else if (a.method == 3) PCAL_ROT_P(NB, 3);          \
        else if (a.method == 4) PCAL_ROT_P(NB, 4);          \
        else if (a.method == 5) PCAL_ROT_P(NB, 5);          \
        else PCAL_ROT_P(NB, 6);                             \
    } while (0)
    if (a.nbits == 2)
        PCAL_ROT_M(2);
    else
        PCAL_ROT_M(8);
#undef PCAL_ROT_M
#undef PCAL_ROT_P
#undef PCAL_ROT
}

}  // namespace pcal
