// Allocation-free extraction (pcal_extract_noalloc): the period-fold FP64 path
// of pcal_create + pcal_extract + pcal_results_async for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  The rotator tables, the integration
// accumulators, the finalize's phases and its counter live in one fixed
// device array per GPU instead of handle memory; the tables are computed on
// the device, so a call makes no host-to-device copy either.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "pcal_host.h"

using namespace pcal;
using namespace pcal::host;

namespace {

constexpr int kMaxDevices = 64;

// The library's scratch for the allocation-free entry point, one copy per GPU.
// Host code never uses this name as an address: the device address comes
// from hipGetSymbolAddress, once per device (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[PCAL_NOALLOC_SCRATCH_BYTES];

std::mutex g_init_mu;
std::atomic<void *> g_scratch_dev[kMaxDevices];

// Device address of this device's copy of the scratch array (null on error).
void *scratch_ptr(int dev) {
    void *p = g_scratch_dev[dev].load(std::memory_order_acquire);
    if (p) return p;
    std::lock_guard<std::mutex> lock(g_init_mu);
    p = g_scratch_dev[dev].load(std::memory_order_relaxed);
    if (p) return p;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        set_error("hipGetSymbolAddress(scratch)", e);
        return nullptr;
    }
    g_scratch_dev[dev].store(p, std::memory_order_release);
    return p;
}

// Byte offsets of the pieces of one call inside the scratch array (256-byte aligned).
struct Layout {
    size_t u64, v, tw, acc, acc_int, accf, phases, counters, end;
};

size_t up256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

Layout layout_of(int64_t N, int64_t M) {
    Layout l{};
    size_t o = 0;
    l.u64 = o;     o = up256(o + 16 * static_cast<size_t>(M));
    l.v = o;       o = up256(o + 16 * static_cast<size_t>(N));
    l.tw = o;      o = up256(o + 16 * static_cast<size_t>(N));
    l.acc = o;     o = up256(o + 16 * static_cast<size_t>(kAccSlots * N));
    l.acc_int = o; o = up256(o + 8 * static_cast<size_t>(kAccSlots * N));
    l.accf = o;    o = up256(o + 8 * static_cast<size_t>(kAccSlots * N));
    l.phases = o;  o = up256(o + 8 * static_cast<size_t>(N));
    l.counters = o; o = up256(o + 8);
    l.end = o;
    return l;
}

// exp(-j 2 pi idx / fs) for 0 <= idx < fs, the angle reduced to [-pi, pi].
__device__ double2 phasor_dev(uint64_t idx, uint64_t fs) {
    const double two_pi = 6.283185307179586476925286766559;
    const double ang = (2 * idx <= fs) ? two_pi * static_cast<double>(idx) / static_cast<double>(fs)
                                       : -two_pi * static_cast<double>(fs - idx) / static_cast<double>(fs);
    double s, c;
    sincos(ang, &s, &c);
    return make_double2(c, -s);
}

// Per call: the FP64 rotator factors of the period fold from exact integer
// phase indices (Eq. 3-5), u[m] = exp(-j w_o N m), v[b] = exp(-j w_o b), the
// DFT twiddles tw[j] = exp(-j 2 pi j / N), and zeroed accumulators and counters
// (the previous call's are still in the array).  fs < 2^32 and M <= 2^20, so
// every index product fits 64 bits.
__global__ void noalloc_setup_kernel(unsigned char *base, Layout l, uint64_t fs, uint64_t step_u, uint64_t fo,
                                     int N, int M) {
    double2 *u = reinterpret_cast<double2 *>(base + l.u64);
    double2 *v = reinterpret_cast<double2 *>(base + l.v);
    double2 *tw = reinterpret_cast<double2 *>(base + l.tw);
    uint32_t *zero = reinterpret_cast<uint32_t *>(base + l.acc);
    const size_t nzero = (l.end - l.acc) / 4;  // accumulators, phases, counters
    const size_t i0 = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = i0; i < static_cast<size_t>(M); i += stride) u[i] = phasor_dev((step_u * i) % fs, fs);
    for (size_t i = i0; i < static_cast<size_t>(N); i += stride) {
        v[i] = phasor_dev((fo * i) % fs, fs);
        tw[i] = phasor_dev(i, static_cast<uint64_t>(N));
    }
    for (size_t i = i0; i < nzero; i += stride) zero[i] = 0u;
}

}  // namespace

extern "C" {

int pcal_extract_noalloc(int64_t fs_hz, int64_t f_comb_hz, int64_t f_offset_hz, int nbits, int sideband,
                         const void *dev_ptr, int64_t nsamples, double *dev_out, pcal_stream_t stream) {
    if (!dev_out || nsamples < 0 || (nsamples > 0 && !dev_ptr)) return PCAL_EINVAL;
    Plan p{};
    int rc = make_plan(fs_hz, f_comb_hz, f_offset_hz, nbits, sideband, PCAL_METHOD_AUTO, PCAL_PREC_F64, &p);
    if (rc) return rc;
    if (nsamples % (8 / nbits)) return PCAL_EINVAL;
    if (p.method != PCAL_METHOD_PERIOD_FOLD || fs_hz >= (int64_t(1) << 32)) {
        set_message("pcal_extract_noalloc: the stream needs a per-sample form; only the period fold runs "
                    "without allocating");
        return PCAL_ENOTSUP;
    }
    const Layout l = layout_of(p.N, p.M);
    if (l.end > static_cast<size_t>(PCAL_NOALLOC_SCRATCH_BYTES)) {
        char msg[160];
        snprintf(msg, sizeof(msg), "pcal_extract_noalloc: needs %zu bytes of scratch, the array holds %d",
                 l.end, PCAL_NOALLOC_SCRATCH_BYTES);
        set_message(msg);
        return PCAL_EINVAL;
    }
    int dev = 0;
    PCAL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return PCAL_EINVAL;
    unsigned char *base = static_cast<unsigned char *>(scratch_ptr(dev));
    if (!base) return PCAL_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);

    // The handle that pcal_create would build, on the stack, pointing into the array.
    pcal_ctx h;
    h.plan = p;
    h.device = dev;
    h.u64 = reinterpret_cast<double2 *>(base + l.u64);
    h.v = reinterpret_cast<double2 *>(base + l.v);
    h.tw = reinterpret_cast<double2 *>(base + l.tw);
    h.acc = reinterpret_cast<double2 *>(base + l.acc);
    h.acc_int = reinterpret_cast<long long *>(base + l.acc_int);
    h.accf = reinterpret_cast<float2 *>(base + l.accf);
    h.phases = reinterpret_cast<double *>(base + l.phases);
    h.counters = reinterpret_cast<unsigned *>(base + l.counters);
    h.n_integ = nsamples;
    // the persistent fold grid of this device, as pcal_create plans it
    if (!p.target_from_env) {
        int cus = 0;
        const int per_cu = fold_blocks_per_cu(p.nbits, p.prec, p.geom.threads,
                                              fold_lds_bytes(p.geom.npos, p.geom.spv, p.geom.threads, p.M));
        const int waves = (p.geom.threads + 63) / 64;
        const int use = std::min(per_cu, std::max(1, (kMinResidentWaves + waves - 1) / waves));
        PCAL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        if (per_cu > 0 && cus > 0) h.plan.target_blocks = std::max(use * cus, p.geom.col_tiles);
    }

    const uint64_t fs = static_cast<uint64_t>(fs_hz), fo = static_cast<uint64_t>(f_offset_hz);
    const uint64_t step_u = (fo * static_cast<uint64_t>(p.N)) % fs;
    const int nset = static_cast<int>(std::max<size_t>({static_cast<size_t>(p.M), static_cast<size_t>(p.N),
                                                       (l.end - l.acc) / 4}));
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3(std::min(1024, (nset + 255) / 256)), dim3(256), 0, s, base, l, fs,
                       step_u, fo, static_cast<int>(p.N), static_cast<int>(p.M));
    PCAL_HIP(hipGetLastError());
    if (nsamples > 0) {
        const pcal_launch_t L = plan_launch(h.plan, reinterpret_cast<uintptr_t>(dev_ptr), 0, nsamples, 0);
        const FoldArgs a = fold_args(&h, L, dev_ptr);
        launch_fold(a, p.nbits, static_cast<int>(L.grid), p.geom.threads, static_cast<size_t>(L.lds_bytes), s);
        PCAL_HIP(hipGetLastError());
    }
    launch_finalize(fin_args(&h, dev_out), s);
    PCAL_HIP(hipGetLastError());
    return PCAL_OK;
}

}  // extern "C"
