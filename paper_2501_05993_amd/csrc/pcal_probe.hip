// Streaming-read reference: one pass over a device buffer with 16-byte
// non-temporal loads, the way the fold kernel reads its input, and nothing
// else.  Its duration is the measured ceiling that the bandwidth-bound fold is
// compared with (start-up and drain of a launch included); it is not part of
// the extraction.  Each workgroup owns a contiguous slice; each wave writes the
// XOR of the 64-bit words it read, so the loads cannot be dropped and the pass
// can be checked.
#include "pcal.h"
#include "pcal_host.h"

namespace pcal {
namespace {

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef const u32x4_t __attribute__((address_space(1))) *global_u32x4_ptr;

__device__ __forceinline__ uint64_t xor_of(const uint4 *p) {
    const u32x4_t v = __builtin_nontemporal_load((global_u32x4_ptr)p);
    return (static_cast<uint64_t>(v.y) << 32 | v.x) ^ (static_cast<uint64_t>(v.w) << 32 | v.z);
}

constexpr int kProbeUnroll = 8;  // loads in flight per thread

__global__ void __launch_bounds__(1024) read_probe_kernel(const uint4 *p, int64_t nvec, int64_t per_block,
                                                          uint64_t *out) {
    const int64_t bd = blockDim.x;
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * per_block;
    const int64_t b1 = b0 + per_block < nvec ? b0 + per_block : nvec;
    uint64_t acc = 0;
    int64_t i = b0 + threadIdx.x;
    for (; i + (kProbeUnroll - 1) * bd < b1; i += kProbeUnroll * bd) {
        uint64_t x[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) x[u] = xor_of(p + i + u * bd);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) acc ^= x[u];
    }
    for (; i < b1; i += bd) acc ^= xor_of(p + i);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) out[(static_cast<int64_t>(blockIdx.x) * bd + threadIdx.x) >> 6] = acc;
}

}  // namespace
}  // namespace pcal

extern "C" int pcal_read_probe(const void *dev_ptr, int64_t bytes, int blocks, int threads, uint64_t *out,
                               pcal_stream_t stream, void *start_event, void *stop_event) {
    if (!dev_ptr || !out || bytes <= 0 || bytes % 16 || reinterpret_cast<uintptr_t>(dev_ptr) % 16 || blocks < 1 ||
        threads < 64 || threads > 1024 || threads % 64)
        return PCAL_EINVAL;
    const int64_t nvec = bytes / 16;
    const int64_t per_block = (nvec + blocks - 1) / blocks;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t t0 = static_cast<hipEvent_t>(start_event), t1 = static_cast<hipEvent_t>(stop_event);
    const uint4 *p = static_cast<const uint4 *>(dev_ptr);
    if (t0 || t1)
        hipExtLaunchKernelGGL(pcal::read_probe_kernel, dim3(blocks), dim3(threads), 0, s, t0, t1, 0, p, nvec,
                              per_block, out);
    else
        hipLaunchKernelGGL(pcal::read_probe_kernel, dim3(blocks), dim3(threads), 0, s, p, nvec, per_block, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        pcal::host::set_error("read_probe_kernel", e);
        return PCAL_EHIP;
    }
    return PCAL_OK;
}
