// Device code shared by the fold kernels (pcal_kernels.hip) and the served loop
// (pcal_served.hip): the fused unpack -> rotate -> fold body with its
// per-workgroup epilogue and cross-workgroup commit, and the FP64 finalize
// (N-point DFT, amplitude, phase, delay).
//
// Period fold.  With R = fs / gcd(fs, f_offset) the rotator exp(-j w_o n) of
// Eq. 3 repeats every R samples (Eq. 4) and the fold index n mod N (Eq. 2)
// every N, so both repeat every S' (a multiple of lcm(N, R) and of the samples
// in one 16-byte load).  The sum over the stream of x[n] * rot[n] into bin
// n mod N therefore equals, by distributivity, first summing the integer
// samples that share a period position q = n mod S' and then rotating each of
// the S' position sums once.  Section 4.1 suggests accumulating over one
// rotator period and folding into the bins after the sample loop; here the
// samples are summed before any rotation, which carries that idea to its end.  The rotator
// is factorised as rot[q] = u[q / N] * v[q mod N] with u[m] = exp(-j w_o N m)
// and v[b] = exp(-j w_o b); a workgroup applies u to its position sums and
// folds them to N bins, and v is applied once per bin in the final reduction.
//
// Each thread owns one column of the row view of the stream (rows are a
// multiple of S' long), so it meets the same period positions on every row
// and sums the 2-bit codes (or biased 8-bit values) of its 64 (16) positions
// in SWAR lanes of ordinary registers: the inner loop is a few integer
// operations per 32-bit word, well under the HBM time of the data it reads.
#pragma once

#include <type_traits>

#include "pcal_internal.h"

namespace pcal {

namespace {

constexpr uint32_t kM33 = 0x33333333u;
constexpr uint32_t kM0F = 0x0F0F0F0Fu;
constexpr uint32_t kM00FF = 0x00FF00FFu;
// Finalize keeps the twiddles in LDS up to this many tones (bins + twiddles + 4 KiB <= 64 KiB).
constexpr int kTwLdsMaxTones = 1792;

// The packed stream is read once: non-temporal 16-byte loads keep it from
// displacing reusable lines in the caches.
//
// Every device read goes through a pointer in the global address space.  The
// batched kernel takes its pointers from memory, where the compiler cannot
// tell global memory from LDS and would emit flat loads; a flat load counts on
// both wait counters, and with one pending the compiler's waits for the
// stream's loads all become waits for every load.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef const u32x4_t __attribute__((address_space(1))) *global_u32x4_ptr;
__device__ __forceinline__ uint4 load_stream(const uint4 *p) {
    const u32x4_t v = __builtin_nontemporal_load((global_u32x4_ptr)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}
// (A struct is loaded as a raw vector of its size: its copy constructor would
// take the address back to the generic space.)
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
template <int B> struct RawOf;
template <> struct RawOf<1> { using T = uint8_t; };
template <> struct RawOf<4> { using T = uint32_t; };
template <> struct RawOf<8> { using T = u32x2_t; };
template <> struct RawOf<16> { using T = u32x4_t; };
template <class T>
__device__ __forceinline__ T load_global(const T *p) {
    using V = typename RawOf<sizeof(T)>::T;
    const V v = *(const __attribute__((address_space(1))) V *)p;
    T r;
    __builtin_memcpy(&r, &v, sizeof(T));
    return r;
}

__device__ __forceinline__ int level_of(const uint8_t *p, int nbits, int i) {
    if (nbits == 2) return 2 * ((load_global(p + (i >> 2)) >> (2 * (i & 3))) & 3) - 3;
    return static_cast<int>(static_cast<int8_t>(load_global(p + i)));
}

// True in every thread of the workgroup that finishes last (all workgroups
// call it once, after their global stores).  Self-resetting counter.
__device__ __forceinline__ bool last_workgroup_done(unsigned *counter, unsigned total) {
    __shared__ unsigned s_last;
    // every wave's global stores are complete (acknowledged by L2) before the
    // barrier, so the single write-back below covers the whole workgroup
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool last = prev == total - 1;
        if (last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_last = last ? 1u : 0u;
    }
    __syncthreads();
    return s_last != 0u;
}

// ---------------------------------------------------------------- 2-bit rows

// Spread the two nibble-lane sums of one 32-bit word into the four byte-lane
// code sums.  lo holds codes q=0 (even nibbles) and q=2 (odd nibbles) of each
// byte, hi holds q=1 and q=3.
__device__ __forceinline__ void nibbles_to_bytes(uint32_t lo, uint32_t hi, uint32_t (&bq)[4]) {
    bq[0] += lo & kM0F;
    bq[2] += (lo >> 4) & kM0F;
    bq[1] += hi & kM0F;
    bq[3] += (hi >> 4) & kM0F;
}

// Add the byte-lane code sums of a thread to the workgroup's position sums as
// levels: sum of (2c - 3) over cnt rows = 2 * sum(c) - 3 * cnt.
__device__ __forceinline__ void flush2(uint32_t (&bq)[4][4], int cnt, int *Fp) {
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int s = 16 * w + 4 * j + q;
                const int val = 2 * static_cast<int>((bq[w][q] >> (8 * j)) & 0xFFu) - 3 * cnt;
                atomicAdd(&Fp[s], val);
                bq[w][q] = (j == 3) ? 0u : bq[w][q];
            }
}

__device__ __forceinline__ void add_codes(uint4 x, uint32_t (&lo)[4], uint32_t (&hi)[4]) {
    lo[0] += x.x & kM33;
    hi[0] += (x.x >> 2) & kM33;
    lo[1] += x.y & kM33;
    hi[1] += (x.y >> 2) & kM33;
    lo[2] += x.z & kM33;
    hi[2] += (x.z >> 2) & kM33;
    lo[3] += x.w & kM33;
    hi[3] += (x.w >> 2) & kM33;
}

struct Walk2 {
    const uint4 *col;
    int64_t stride, rfull;
    bool last_ok;
    int *Fp;
    uint32_t bq[4][4];
    int cnt, spreads;

    static constexpr int kRows = 5;  // rows of one group
    struct Buf {
        uint4 v[5];
    };

    __device__ __forceinline__ void init(const FoldArgs &a, int colr, int *fp) {
        col = a.data + colr;
        stride = a.row_vecs;
        rfull = a.nvec / stride;
        last_ok = colr < a.nvec - rfull * stride;
        Fp = fp;
#pragma unroll
        for (int w = 0; w < 4; ++w)
#pragma unroll
            for (int q = 0; q < 4; ++q) bq[w][q] = 0u;
        cnt = spreads = 0;
    }
    __device__ __forceinline__ void spread(const uint32_t (&lo)[4], const uint32_t (&hi)[4]) {
        if (spreads == 17) {
            flush2(bq, cnt, Fp);
            cnt = 0;
            spreads = 0;
        }
#pragma unroll
        for (int w = 0; w < 4; ++w) nibbles_to_bytes(lo[w], hi[w], bq[w]);
        ++spreads;
    }
    // loads of the five full rows [r, r + 5)
    __device__ __forceinline__ void load_group(Buf &b, int64_t r) const {
#pragma unroll
        for (int u = 0; u < 5; ++u) b.v[u] = load_stream(col + (r + u) * stride);
    }
    __device__ __forceinline__ void take(const Buf &b) {
        uint32_t lo[4] = {0u, 0u, 0u, 0u}, hi[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int u = 0; u < 5; ++u) add_codes(b.v[u], lo, hi);
        spread(lo, hi);
        cnt += 5;
    }
    // rows [r0, r1) of this column, one at a time (the last row of the stream
    // may be partial): the odd rows around the grouped walk
    __device__ void rows(int64_t r0, int64_t r1) {
        uint32_t lo[4] = {0u, 0u, 0u, 0u}, hi[4] = {0u, 0u, 0u, 0u};
        int nib = 0;
        for (int64_t r = r0; r < r1; ++r) {
            if (r < rfull || (r == rfull && last_ok)) {
                add_codes(load_stream(col + r * stride), lo, hi);
                if (++nib == 5) {
                    spread(lo, hi);
                    cnt += 5;
                    nib = 0;
#pragma unroll
                    for (int w = 0; w < 4; ++w) lo[w] = hi[w] = 0u;
                }
            }
        }
        if (nib) {
            spread(lo, hi);
            cnt += nib;
        }
    }
    __device__ __forceinline__ void finish() {
        if (cnt) flush2(bq, cnt, Fp);
    }
};

// ---------------------------------------------------------------- 8-bit rows

// Biased values u = x + 128 (0..255) of bytes 0,2 / 1,3 of each word go to the
// 16-bit lanes of e / o; 256 rows fit before a lane can overflow.
__device__ __forceinline__ void add_bytes(uint4 x, uint32_t (&e)[4], uint32_t (&o)[4]) {
    const uint32_t b0 = x.x ^ 0x80808080u, b1 = x.y ^ 0x80808080u;
    const uint32_t b2 = x.z ^ 0x80808080u, b3 = x.w ^ 0x80808080u;
    e[0] += b0 & kM00FF;
    o[0] += (b0 >> 8) & kM00FF;
    e[1] += b1 & kM00FF;
    o[1] += (b1 >> 8) & kM00FF;
    e[2] += b2 & kM00FF;
    o[2] += (b2 >> 8) & kM00FF;
    e[3] += b3 & kM00FF;
    o[3] += (b3 >> 8) & kM00FF;
}

__device__ __forceinline__ void flush8(uint32_t (&e)[4], uint32_t (&o)[4], int cnt, int *Fp) {
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        atomicAdd(&Fp[4 * w + 0], static_cast<int>(e[w] & 0xFFFFu) - 128 * cnt);
        atomicAdd(&Fp[4 * w + 1], static_cast<int>(o[w] & 0xFFFFu) - 128 * cnt);
        atomicAdd(&Fp[4 * w + 2], static_cast<int>(e[w] >> 16) - 128 * cnt);
        atomicAdd(&Fp[4 * w + 3], static_cast<int>(o[w] >> 16) - 128 * cnt);
        e[w] = 0u;
        o[w] = 0u;
    }
}

// One thread's column walk over 8-bit rows: biased sums of its 16 positions in
// 16-bit lanes, 256 rows per flush to LDS.
constexpr int kGroup8 = 4;  // rows loaded together

struct Walk8 {
    const uint4 *col;
    int64_t stride, rfull;
    bool last_ok;
    int *Fp;
    uint32_t e[4], o[4];
    int cnt;

    static constexpr int kRows = kGroup8;
    struct Buf {
        uint4 v[kGroup8];
    };

    __device__ __forceinline__ void init(const FoldArgs &a, int colr, int *fp) {
        col = a.data + colr;
        stride = a.row_vecs;
        rfull = a.nvec / stride;
        last_ok = colr < a.nvec - rfull * stride;
        Fp = fp;
#pragma unroll
        for (int w = 0; w < 4; ++w) e[w] = o[w] = 0u;
        cnt = 0;
    }
    __device__ __forceinline__ void add(const uint4 &x) {
        if (cnt == 256) {
            flush8(e, o, cnt, Fp);
            cnt = 0;
        }
        add_bytes(x, e, o);
        ++cnt;
    }
    __device__ __forceinline__ void load_group(Buf &b, int64_t r) const {
#pragma unroll
        for (int u = 0; u < kGroup8; ++u) b.v[u] = load_stream(col + (r + u) * stride);
    }
    __device__ __forceinline__ void take(const Buf &b) {
#pragma unroll
        for (int u = 0; u < kGroup8; ++u) add(b.v[u]);
    }
    __device__ void rows(int64_t r0, int64_t r1) {
        for (int64_t r = r0; r < r1; ++r)
            if (r < rfull || (r == rfull && last_ok)) add(load_stream(col + r * stride));
    }
    __device__ __forceinline__ void finish() {
        if (cnt) flush8(e, o, cnt, Fp);
    }
};

// ---------------------------------------------------------------- per-workgroup bins

// A partial bin sum in the arithmetic of one precision form (the kernels'
// form: enum pcal_precision, with PCAL_PREC_F16 run as 1 and PCAL_PREC_Q17 as 3):
//   0 (F64):   FP64 table, FP64 products and sums;
//   1 (MIXED): two-term FP16 table (hi + lo, held as FP32), FP32 products, Kahan-compensated FP32 sums;
//   2 (F32):   FP32 table, plain FP32 products and sums;
//   3 (Q17):   integer full-period table, integer products, int64 sums.
// si carries the exact integer sum (the Eq. 2 bin when f_offset = 0).
template <int PREC>
struct BinAcc;

template <>
struct BinAcc<0> {
    using Tab = double2;
    double re = 0.0, im = 0.0;
    long long si = 0;
    __device__ __forceinline__ void add(int f, Tab u) {
        re += f * u.x;
        im += f * u.y;
        si += f;
    }
    __device__ __forceinline__ void merge(const BinAcc &o) {
        re += o.re;
        im += o.im;
        si += o.si;
    }
    __device__ __forceinline__ double2 value() const { return make_double2(re, im); }
};

template <>
struct BinAcc<1> {
    using Tab = float2;
    float sr = 0.f, cr = 0.f, sm = 0.f, cm = 0.f;
    long long si = 0;
    __device__ __forceinline__ void kahan(float y, float &s, float &c) {
        const float yc = y - c;
        const float t = s + yc;
        c = (t - s) - yc;
        s = t;
    }
    __device__ __forceinline__ void add(int f, Tab u) {
        kahan(static_cast<float>(f) * u.x, sr, cr);
        kahan(static_cast<float>(f) * u.y, sm, cm);
        si += f;
    }
    __device__ __forceinline__ void merge(const BinAcc &o) {
        kahan(o.sr - o.cr, sr, cr);
        kahan(o.sm - o.cm, sm, cm);
        si += o.si;
    }
    __device__ __forceinline__ double2 value() const {
        return make_double2(static_cast<double>(sr) - static_cast<double>(cr),
                            static_cast<double>(sm) - static_cast<double>(cm));
    }
};

template <>
struct BinAcc<2> {
    using Tab = float2;
    float sr = 0.f, sm = 0.f;
    long long si = 0;
    __device__ __forceinline__ void add(int f, Tab u) {
        sr += static_cast<float>(f) * u.x;
        sm += static_cast<float>(f) * u.y;
        si += f;
    }
    __device__ __forceinline__ void merge(const BinAcc &o) {
        sr += o.sr;
        sm += o.sm;
        si += o.si;
    }
    __device__ __forceinline__ double2 value() const { return make_double2(sr, sm); }
};

// Fixed-point form (3): the full-period rotator table in Q17 integers
// (Section 4.8's integer rotator), integer products and exact int64 sums.
// value() is the integer bin sum, exact in FP64 below 2^53; the finalize
// scales it by 2^-17.
template <>
struct BinAcc<3> {
    using Tab = int2;
    long long sr = 0, sm = 0, si = 0;
    __device__ __forceinline__ void add(int f, Tab u) {
        sr += static_cast<long long>(f) * u.x;
        sm += static_cast<long long>(f) * u.y;
        si += f;
    }
    __device__ __forceinline__ void merge(const BinAcc &o) {
        sr += o.sr;
        sm += o.sm;
        si += o.si;
    }
    __device__ __forceinline__ double2 value() const {
        return make_double2(static_cast<double>(sr), static_cast<double>(sm));
    }
};

template <int PREC>
__device__ __forceinline__ typename BinAcc<PREC>::Tab table_row(const FoldArgs &a, int m) {
    if constexpr (PREC == 3)
        return load_global(a.uq + m);
    else if constexpr (PREC == 0)
        return load_global(a.u64 + m);
    else if constexpr (PREC == 1) {
        // two FP16 terms; their FP32 sum is exact
        const float2 hi = __half22float2(load_global(a.u16 + 2 * m));
        const float2 lo = __half22float2(load_global(a.u16 + 2 * m + 1));
        return make_float2(hi.x + lo.x, hi.y + lo.y);
    }
    else
        return load_global(a.u32 + m);
}

// Add one workgroup's bin b (before v) to the integration accumulators:
// acc[slot][b] += v[b] * Q  (FP64 atomics; FP32 atomics into accf in the F32
// form), acc_int[slot][b] += exact integer sum.  Workgroups spread over
// kAccSlots copies of the bins so that few atomics meet on one address; the
// finalize adds the slots.
template <int PREC>
__device__ __forceinline__ void commit_bin(const FoldArgs &a, int wg, int b, const BinAcc<PREC> &q, double2 v) {
    const double2 Q = q.value();
    const size_t k = static_cast<size_t>(wg % kAccSlots) * a.N + b;
    if constexpr (PREC == 2) {
        const float qr = static_cast<float>(Q.x), qi = static_cast<float>(Q.y);
        const float vr = static_cast<float>(v.x), vi = static_cast<float>(v.y);
        unsafeAtomicAdd(&a.accf[k].x, qr * vr - qi * vi);
        unsafeAtomicAdd(&a.accf[k].y, qr * vi + qi * vr);
    } else if constexpr (PREC == 3) {
        // the table holds the whole rotator: no column factor; integer-valued
        // FP64 adds stay exact below 2^53, in any order
        (void)v;
        unsafeAtomicAdd(&a.acc[k].x, Q.x);
        unsafeAtomicAdd(&a.acc[k].y, Q.y);
    } else {
        unsafeAtomicAdd(&a.acc[k].x, Q.x * v.x - Q.y * v.y);
        unsafeAtomicAdd(&a.acc[k].y, Q.x * v.y + Q.y * v.x);
    }
    if (a.int_bins)
        atomicAdd(reinterpret_cast<unsigned long long *>(&a.acc_int[k]), static_cast<unsigned long long>(q.si));
}

// Sum F[p] * u[m] over the positions p = p, p + step_p, ... < npos of one bin
// (skewed LDS position sums), the rotator row m advancing by step_m mod M;
// tab(m) gives u[m].  The table's source (LDS or global) is chosen outside the
// loop: a choice inside it made the compiler wait on every load in turn.
template <int SPV, class Acc, class Tab>
__device__ __forceinline__ void rotate_bin(Acc &acc, const int *F, int p, int m, int step_p, int step_m, int npos,
                                           int M, const Tab &tab) {
#pragma unroll 4
    for (; p < npos; p += step_p) {
        acc.add(F[p + p / SPV], tab(m));
        m += step_m;
        if (m >= M) m -= M;
    }
}

// Samples of the misaligned head and short tail of bin b (workgroup 0 only).
template <int PREC, typename Tab>
__device__ void add_edges(const FoldArgs &a, int b, BinAcc<PREC> &q, const Tab *UL, bool u_lds) {
    for (int part = 0; part < 2; ++part) {
        const uint8_t *src = part ? a.tail : a.head;
        const int ns = (part ? a.tail_bytes : a.head_bytes) * (8 / a.nbits);
        int64_t qq = part ? a.tail_q : a.head_q;
        int qb = static_cast<int>(qq % a.N);
        for (int i = 0; i < ns; ++i) {
            if (qb == b) {
                const int m = static_cast<int>(PREC == 3 ? qq % a.M : qq / a.N);
                q.add(level_of(src, a.nbits, i), u_lds ? UL[m] : table_row<PREC>(a, m));
            }
            if (++qq == a.Sp) qq = 0;
            if (++qb == a.N) qb = 0;
        }
    }
}

// ---------------------------------------------------------------- the fused kernel

// The fused kernel's work for workgroup `wg` of one stream's launch geometry.
template <int NBITS, int PREC>
__device__ __forceinline__ void fold_body(const FoldArgs &a, const int wg, unsigned char *lds) {
    using Acc = BinAcc<PREC>;
    using Tab = typename Acc::Tab;
    static_assert(sizeof(Acc) <= kEpilogueScratch, "epilogue scratch");
    // Start the walk with no memory operation outstanding.  Code that may run
    // before it in the same kernel (the fused finalize's stores, whose path
    // the compiler joins to this one) would otherwise leave mixed kinds of
    // operations pending in the compiler's wait accounting, which then waits
    // for every load in the walk instead of keeping two groups in flight.
    __builtin_amdgcn_s_waitcnt(0);
    constexpr int SPV = NBITS == 2 ? 64 : 16;
    constexpr int kPre = 4;  // rotator rows prefetched per thread
    const int t = threadIdx.x, nt = blockDim.x;
    const int npos_sk = a.npos + a.npos / SPV;
    int *F = reinterpret_cast<int *>(lds);
    Tab *UL = reinterpret_cast<Tab *>(lds + fold_front_bytes(a.npos, SPV, nt));
    const bool u_lds = a.M <= kLdsTableRows;
    const int M = static_cast<int>(a.M);

    // v[b] of the bin this thread commits (group form), loaded now.
    const double2 vb = (a.N < nt && t < a.N) ? load_global(a.v + t) : make_double2(0.0, 0.0);
    // Rotator rows: loads issued now, stored to LDS after the walk.
    Tab upre[kPre];
#pragma unroll
    for (int j = 0; j < kPre; ++j)
        if (u_lds && t + j * nt < M) upre[j] = table_row<PREC>(a, t + j * nt);

    const int c = wg % a.col_tiles;
    const int64_t g = wg / a.col_tiles;
    const int tc = t % a.tile_vecs, sub = t / a.tile_vecs;
    const int colp = c * a.tile_vecs + tc;                 // column within the period
    const int colr = colp + sub * a.period_vecs;           // column within the row
    const bool active = colp < a.period_vecs && colr < a.row_vecs;
    // Workgroup g of the tile walks its block of whole groups of rows; the rows
    // after the last whole group (with the partial last row) go to the first
    // workgroup of each tile.  Each wave keeps two groups of rows in flight
    // throughout (buffers A and B in turn): the loads of the next group are
    // issued before the current one is added.
    using W = typename std::conditional<NBITS == 2, Walk2, Walk8>::type;
    constexpr int R = W::kRows;
    const int64_t r0 = R * (g * a.groups_per_wg + (g < a.extra_groups ? g : a.extra_groups));
    const int64_t r1 = r0 + R * (a.groups_per_wg + (g < a.extra_groups ? 1 : 0));
    // Lanes that walk no column load column 0 and add into a spare LDS column,
    // so that the walk has no divergent branch: the compiler's wait counting
    // then keeps both groups in flight.
    W walk;
    walk.init(a, active ? colr : 0, active ? F + tc * (SPV + 1) : F + npos_sk);
    typename W::Buf A, B;
    const int64_t ngr = (r1 - r0) / R;  // groups of this workgroup
    if (ngr > 0) walk.load_group(A, r0);
    for (int j = t; j < npos_sk; j += nt) F[j] = 0;
    __syncthreads();
    if (g == 0 && active) walk.rows(a.odd_start, a.rows_total);
    // group i in A, i + 1 in B; past the last group the loads repeat one (never
    // added).  A barrier every few pairs keeps the waves in step: waves that
    // ran ahead would otherwise leave the last stretch to a few waves with few
    // loads in flight.  (A bare s_barrier: no fence, so no wait on the loads.)
    const int sync_mask = a.sync_pairs > 0 ? a.sync_pairs - 1 : -1;
    for (int64_t i = 0; i + 1 < ngr; i += 2) {
        const int64_t q = r0 + i * R;
        walk.load_group(B, q + R);
        walk.take(A);
        walk.load_group(A, i + 2 < ngr ? q + 2 * R : q + R);
        walk.take(B);
        if (sync_mask >= 0 && ((i >> 1) & sync_mask) == sync_mask) __builtin_amdgcn_s_barrier();
    }
    if (ngr & 1) walk.take(A);
    if (active) walk.finish();
    if (u_lds) {
#pragma unroll
        for (int j = 0; j < kPre; ++j)
            if (t + j * nt < M) UL[t + j * nt] = upre[j];
        for (int i = t + kPre * nt; i < M; i += nt) UL[i] = table_row<PREC>(a, i);
    }
    __syncthreads();

    // Rotate this workgroup's position sums by u and fold them onto the N bins.
    // Local position p has period coordinate (qb + p) mod S', rotator row
    // ((qb + p) mod S') / N and bin (qb + p) mod N.
    const int N = a.N;
    const int Sp = static_cast<int>(a.Sp);
    const int qb = static_cast<int>((a.q0 + static_cast<int64_t>(c) * a.tile_vecs * SPV) % a.Sp);
    const int qbN = qb % N;
    const bool edges = wg == 0 && (a.head_bytes > 0 || a.tail_bytes > 0);
    if (N >= nt) {
        for (int b = t; b < N; b += nt) {
            int p = b >= qbN ? b - qbN : b - qbN + N;
            int q = qb + p;
            if (q >= Sp) q -= Sp;
            // table entry of position q: the rotator row q / N (factorised
            // forms) or the rotator itself at q mod R (fixed-point form)
            int m = PREC == 3 ? q % M : q / N;
            const int step_m = PREC == 3 ? N % M : 1;
            Acc acc;
            if (u_lds)
                rotate_bin<SPV>(acc, F, p, m, N, step_m, a.npos, M, [&](int mm) { return UL[mm]; });
            else
                rotate_bin<SPV>(acc, F, p, m, N, step_m, a.npos, M, [&](int mm) { return table_row<PREC>(a, mm); });
            if (edges) add_edges<PREC>(a, b, acc, UL, u_lds);
            commit_bin<PREC>(a, wg, b, acc, load_global(a.v + b));
        }
    } else {
        // G groups of N threads split the positions of every bin; the group
        // partials are merged in group order (deterministic within the workgroup).
        const int G = nt / N;
        const int gi = t / N, b = t % N;
        Acc acc;
        if (gi < G) {
            int p = (b >= qbN ? b - qbN : b - qbN + N) + N * gi;
            int q = qb + p;
            if (q >= Sp) q -= Sp;
            int m = PREC == 3 ? q % M : q / N;
            const int step_p = N * G, step_m = PREC == 3 ? step_p % M : G % M;
            if (u_lds)
                rotate_bin<SPV>(acc, F, p, m, step_p, step_m, a.npos, M, [&](int mm) { return UL[mm]; });
            else
                rotate_bin<SPV>(acc, F, p, m, step_p, step_m, a.npos, M,
                                [&](int mm) { return table_row<PREC>(a, mm); });
        }
        __syncthreads();  // every read of F is done: reuse its space
        Acc *scr = reinterpret_cast<Acc *>(lds);
        if (gi < G) scr[t] = acc;
        __syncthreads();
        if (t < N) {
            Acc tot = scr[b];
            for (int k = 1; k < G; ++k) tot.merge(scr[k * N + b]);
            if (edges) add_edges<PREC>(a, b, tot, UL, u_lds);
            commit_bin<PREC>(a, wg, b, tot, vb);
        }
    }
}


// Index of the work item that owns workgroup `wg`: the last i with first[i] <= wg.
__device__ __forceinline__ int owner_of(const int *first, int nitems, int wg) {
    // first[] increases strictly (every item owns a workgroup): the owner is the
    // number of items starting at or before wg, less one.  One wave-wide load
    // per 64 items instead of a chain of dependent loads.
    const int lane = static_cast<int>(threadIdx.x) & 63;
    int count = 0;
    for (int j0 = 0; j0 < nitems; j0 += 64) {
        const int j = j0 + lane;
        const bool at_or_before = j < nitems && load_global(first + j) <= wg;
        count += __popcll(__ballot(at_or_before));
    }
    return count - 1;
}

// Item i of a work-list and its first workgroup, for both list forms.
template <class T>
__device__ __forceinline__ int list_owner(const DeviceList<T> &l, int wg) {
    return __builtin_amdgcn_readfirstlane(owner_of(l.first, l.n, wg));
}
template <class T, int CAP>
__device__ __forceinline__ int list_owner(const InlineList<T, CAP> &l, int wg) {
    int i = 0;  // a short list in the kernel arguments: a scalar scan
    while (i + 1 < l.n && l.first[i + 1] <= wg) ++i;
    return i;
}
template <class T>
__device__ __forceinline__ int list_first(const DeviceList<T> &l, int i) { return load_global(l.first + i); }
template <class T, int CAP>
__device__ __forceinline__ int list_first(const InlineList<T, CAP> &l, int i) { return l.first[i]; }
template <class T>
__device__ __forceinline__ T list_item(const DeviceList<T> &l, int i) { return l.items[i]; }
template <class T, int CAP>
__device__ __forceinline__ T list_item(const InlineList<T, CAP> &l, int i) { return l.items[i]; }

// One launch over the work items of many streams of one sample width (each
// item: one stream's launch geometry, tables and accumulators).  Workgroup
// blockIdx.x is workgroup wg0 + blockIdx.x of the work-list, so that the
// 2-bit and 8-bit items of one work-list (2-bit first) go to two launches:
// with both bodies in one kernel, the compiler's wait accounting carries the
// pending operations of one body into the other.
template <int NBITS, int PREC, class List>
__global__ void __launch_bounds__(kMaxFoldThreads) fold_batch_kernel(const List list, int wg0) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int wg = wg0 + static_cast<int>(blockIdx.x);
    const int i = list_owner(list, wg);
    const FoldArgs a = list_item(list, i);
    fold_body<NBITS, PREC>(a, wg - list_first(list, i), lds);
}

// ---------------------------------------------------------------- finalize

// One workgroup per 64 tones, the first 256 threads working (more may be
// present when it runs inside the fold kernel; they only meet the barriers):
// lane -> tone, four waves split the N-term DFT sum, twiddles indexed exactly
// by (k*b) mod N.  The last workgroup unwraps the in-band phases (prefix sum
// of wrapped differences) and fits the delay by least squares.
__device__ __forceinline__ void finalize_body(const FinArgs &a, const int wg, const int nwg, unsigned char *lds) {
    const int N = a.N, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const bool me = t < 256;
    __shared__ double s_ph[64];  // phases of a single-workgroup finalize
    double2 *P = reinterpret_cast<double2 *>(lds);
    const bool tw_lds = N <= kTwLdsMaxTones;
    double2 *TW = tw_lds ? P + N : nullptr;
    double2 *red = P + (tw_lds ? 2 * N : N);
    const bool f32 = a.prec == 2;
    {
        const double2 *acc = a.acc, *tw = a.tw;
        const float2 *accf = a.accf;
        for (int i = t; me && i < N; i += 256) {
            const double2 w = tw[i];  // issued with the slot loads
            P[i] = slot_sum(acc, accf, f32, N, i);
            if (tw_lds) TW[i] = w;
        }
    }
    __syncthreads();
    const int k = wg * 64 + lane;
    const int qn = (N + 3) / 4;
    const int bb = wave * qn;
    const int be = (bb + qn) < N ? (bb + qn) : N;
    double re = 0.0, im = 0.0;
    if (me && k < N && bb < be) {
        int idx = static_cast<int>((static_cast<int64_t>(k) * bb) % N);
        if (f32) {
            float fr = 0.f, fi = 0.f;
            for (int b = bb; b < be; ++b) {
                const double2 p = P[b];
                const double2 w = tw_lds ? TW[idx] : a.tw[idx];
                const float pr = static_cast<float>(p.x), pi = static_cast<float>(p.y);
                const float wr = static_cast<float>(w.x), wi = static_cast<float>(w.y);
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
                const double2 w = tw_lds ? TW[idx] : a.tw[idx];
                re += p.x * w.x - p.y * w.y;
                im += p.x * w.y + p.y * w.x;
                idx += k;
                if (idx >= N) idx -= N;
            }
        }
    }
    if (me) red[wave * 64 + lane] = make_double2(re, im);
    __syncthreads();
    if (wave == 0 && k < N) {
        double cr = 0.0, ci = 0.0;
        float fr = 0.f, fi = 0.f;
        for (int w = 0; w < 4; ++w) {
            const double2 p = red[w * 64 + lane];
            if (f32) {
                fr += static_cast<float>(p.x);
                fi += static_cast<float>(p.y);
            } else {
                cr += p.x;
                ci += p.y;
            }
        }
        if (f32) {
            cr = fr;
            ci = fi;
        }
        {  // known gain of a rounded rotator table, divided out (identity unless the mixed form)
            const double gr = cr * a.gain_re - ci * a.gain_im;
            ci = cr * a.gain_im + ci * a.gain_re;
            cr = gr;
        }
        if (a.sideband < 0) ci = -ci;
        const double phase = atan2(ci, cr);
        a.out[k] = sqrt(cr * cr + ci * ci) * a.inv_L;
        a.out[N + k] = phase;
        a.out[2 * N + k] = cr;
        a.out[3 * N + k] = ci;
        if (nwg == 1)
            s_ph[k] = phase;
        else
            a.phases[k] = phase;
    }

    // One workgroup (N <= 64) has every phase in LDS; several meet at a counter
    // and the last one reads the phases back from device memory (out may be
    // mapped host memory).
    if (nwg == 1)
        __syncthreads();
    else if (!last_workgroup_done(a.counter, static_cast<unsigned>(nwg)))
        return;

    // Delay: unwrap phases over tones [k_lo, k_hi) and fit phase = a + 2 pi t_d f.
    const int n = a.k_hi - a.k_lo;
    double *sh = reinterpret_cast<double *>(lds);  // reuse: [4] wave totals of the scan, [4] of the products
    const double *ph = (nwg == 1 ? s_ph : a.phases) + a.k_lo;
    const int seg = (n + 255) / 256;
    const int s0 = t * seg;
    const int s1 = (s0 + seg) < n ? (s0 + seg) : n;
    const double two_pi = 6.283185307179586476925286766559;
    double dsum = 0.0;
    for (int i = s0; i < s1; ++i) {
        if (i == 0) continue;
        const double d = ph[i] - ph[i - 1];
        dsum += d - two_pi * rint(d / two_pi);
    }
    // exclusive prefix of the segment sums: scan inside each wave, then add the
    // totals of the waves before (fixed order: deterministic)
    double incl = dsum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (me && lane == 63) sh[wave] = incl;
    __syncthreads();
    double before = 0.0;
    for (int w = 0; w < wave; ++w) before += sh[w];
    const double excl = before + incl - dsum;
    const double kbar = 0.5 * static_cast<double>(n - 1);
    double unw = (n > 0 ? ph[0] : 0.0) + excl;
    double sxu = 0.0;
    for (int i = s0; i < s1; ++i) {
        if (i > 0) {
            const double d = ph[i] - ph[i - 1];
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
    if (a.clear) {
        // start the next integration: every workgroup has read the bins
        for (int i = t; me && i < kAccSlots * N; i += 256) {
            a.acc_clear[i] = make_double2(0.0, 0.0);
            a.accf_clear[i] = make_float2(0.f, 0.f);
            a.acc_int_clear[i] = 0;
        }
    }
}

template <int NBITS, int PREC>
__global__ void __launch_bounds__(kMaxFoldThreads) fold_kernel(FoldArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int wg = static_cast<int>(blockIdx.x);
    if (wg >= a.fold_wgs) {  // the previous integration's finalize, fused into this launch
        finalize_body(a.fin, wg - a.fold_wgs, a.fin_wgs, lds);
        return;
    }
    fold_body<NBITS, PREC>(a, wg, lds);
}

__global__ void __launch_bounds__(256) finalize_kernel(FinArgs a) {
    extern __shared__ __align__(16) unsigned char lds[];
    finalize_body(a, static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x), lds);
}

// Finalize of many streams in one launch: item i owns workgroups
// [first[i], first[i + 1]), ceil(N_i / 64) of them.
template <class List>
__global__ void __launch_bounds__(256) finalize_batch_kernel(const List list) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int wg = static_cast<int>(blockIdx.x);
    const int i = list_owner(list, wg);
    const FinArgs a = list_item(list, i);
    finalize_body(a, wg - list_first(list, i), (a.N + 63) / 64, lds);
}

}  // namespace
}  // namespace pcal
