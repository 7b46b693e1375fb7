// gfx950 kernels of libpcal: the fused unpack-rotate-fold kernel (one stream per
// launch, and the batched form over a work-list), the FP64 finalize kernels and
// their launchers.  The fold body and the finalize body live in pcal_fold.h.
#include "pcal_fold.h"

namespace pcal {
namespace {

// Zero a list of buffers (one workgroup per buffer, grid-stride inside).
__global__ void zero_list_kernel(const ZeroItem *items, int n) {
    for (int j = blockIdx.x; j < n; j += gridDim.x) {
        uint32_t *p = static_cast<uint32_t *>(items[j].ptr);
        const size_t w = items[j].bytes / 4;
        for (size_t i = threadIdx.x; i < w; i += blockDim.x) p[i] = 0u;
    }
}

__global__ void zero_kernel(uint32_t *p, size_t n) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

}  // namespace

void launch_fold(const FoldArgs &a, int nbits, int grid, int threads, size_t lds, hipStream_t s, hipEvent_t t0,
                 hipEvent_t t1) {
    const dim3 gd(grid), bd(threads);
    // with events: hipExtLaunchKernel stamps them with the kernel's own start and end
#define PCAL_FOLD(NB, PR)                                                                   \
    do {                                                                                    \
        if (t0 || t1)                                                                       \
            hipExtLaunchKernelGGL((fold_kernel<NB, PR>), gd, bd, lds, s, t0, t1, 0, a);     \
        else                                                                                \
            hipLaunchKernelGGL((fold_kernel<NB, PR>), gd, bd, lds, s, a);                   \
    } while (0)
    if (nbits == 2) {
        if (a.prec == 0) PCAL_FOLD(2, 0);
        else if (a.prec == 1) PCAL_FOLD(2, 1);
        else if (a.prec == 2) PCAL_FOLD(2, 2);
        else PCAL_FOLD(2, 3);
    } else {
        if (a.prec == 0) PCAL_FOLD(8, 0);
        else if (a.prec == 1) PCAL_FOLD(8, 1);
        else if (a.prec == 2) PCAL_FOLD(8, 2);
        else PCAL_FOLD(8, 3);
    }
#undef PCAL_FOLD
}

int fold_blocks_per_cu(int nbits, int prec, int threads, size_t lds) {
    const void *f = nullptr;
    if (nbits == 2)
        f = prec == 0   ? reinterpret_cast<const void *>(&fold_kernel<2, 0>)
            : prec == 1 ? reinterpret_cast<const void *>(&fold_kernel<2, 1>)
            : prec == 2 ? reinterpret_cast<const void *>(&fold_kernel<2, 2>)
                        : reinterpret_cast<const void *>(&fold_kernel<2, 3>);
    else
        f = prec == 0   ? reinterpret_cast<const void *>(&fold_kernel<8, 0>)
            : prec == 1 ? reinterpret_cast<const void *>(&fold_kernel<8, 1>)
            : prec == 2 ? reinterpret_cast<const void *>(&fold_kernel<8, 2>)
                        : reinterpret_cast<const void *>(&fold_kernel<8, 3>);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, threads, lds) != hipSuccess) return 0;
    return n;
}

template <class List>
void launch_fold_batch_list(const List &list, int prec, int grid2, int grid8, int threads, size_t lds2, size_t lds8,
                            hipStream_t s) {
    const dim3 bd(threads);
#define PCAL_BATCH_LAUNCH(NB, PR, G, L, W0) \
    hipLaunchKernelGGL((fold_batch_kernel<NB, PR, List>), dim3(G), bd, L, s, list, W0)
    if (grid2 > 0) {
        if (prec == 0)
            PCAL_BATCH_LAUNCH(2, 0, grid2, lds2, 0);
        else if (prec == 1)
            PCAL_BATCH_LAUNCH(2, 1, grid2, lds2, 0);
        else
            PCAL_BATCH_LAUNCH(2, 2, grid2, lds2, 0);
    }
    if (grid8 > 0) {
        if (prec == 0)
            PCAL_BATCH_LAUNCH(8, 0, grid8, lds8, grid2);
        else if (prec == 1)
            PCAL_BATCH_LAUNCH(8, 1, grid8, lds8, grid2);
        else
            PCAL_BATCH_LAUNCH(8, 2, grid8, lds8, grid2);
    }
#undef PCAL_BATCH_LAUNCH
}


void launch_fold_batch(const DeviceList<FoldArgs> &list, int prec, int grid2, int grid8, int threads, size_t lds2,
                       size_t lds8, hipStream_t s) {
    launch_fold_batch_list(list, prec, grid2, grid8, threads, lds2, lds8, s);
}

void launch_fold_batch(const FoldListInline &list, int prec, int grid2, int grid8, int threads, size_t lds2,
                       size_t lds8, hipStream_t s) {
    launch_fold_batch_list(list, prec, grid2, grid8, threads, lds2, lds8, s);
}

void launch_finalize(const FinArgs &a, hipStream_t s) {
    const int grid = (a.N + 63) / 64;
    const size_t lds = finalize_lds_bytes(a.N);
    hipLaunchKernelGGL(finalize_kernel, dim3(grid), dim3(256), lds, s, a);
}

size_t finalize_lds_bytes(int N) { return sizeof(double2) * ((N <= kTwLdsMaxTones ? 2 * N : N) + 256); }

void launch_finalize_batch(const DeviceList<FinArgs> &list, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((finalize_batch_kernel<DeviceList<FinArgs>>), dim3(grid), dim3(256), lds, s, list);
}

void launch_finalize_batch(const FinListInline &list, int grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((finalize_batch_kernel<FinListInline>), dim3(grid), dim3(256), lds, s, list);
}

void launch_zero_list(const ZeroItem *items, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_list_kernel, dim3(n < 1024 ? n : 1024), dim3(256), 0, s, items, n);
}

void launch_zero(void *p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 4;
    const int grid = static_cast<int>((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    hipLaunchKernelGGL(zero_kernel, dim3(grid > 0 ? grid : 1), dim3(256), 0, s,
                       static_cast<uint32_t *>(p), n);
}

}  // namespace pcal
