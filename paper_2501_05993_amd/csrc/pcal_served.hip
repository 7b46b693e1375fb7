// The device-resident served loop (pcal_server_start): one persistent kernel
// that claims published chunk tasks, folds them with the fold body of
// pcal_fold.h and finalizes each integration in the task that completes it.
#include "pcal_fold.h"

namespace pcal {
namespace {

// ---------------------------------------------------------------- served loop

// Copy n 32-bit words from coherent host memory with system-scope loads (the
// host may have written them after this kernel started).
__device__ __forceinline__ void copy_from_host(uint32_t *dst, const uint32_t *src, int n) {
    for (int i = static_cast<int>(threadIdx.x); i < n; i += blockDim.x)
        dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Persistent kernel of the served form: every workgroup claims published
// tasks in increasing order (task t is workgroup t mod tasks of chunk
// t / tasks; a task is claimed only once the host has published it, by a
// compare-and-swap on the claim cursor, so a workgroup never holds a claim on
// unpublished work), runs its share of the chunk's fold into the stream's
// accumulator bank, and counts the task.  The task that completes an
// integration (its count reaches the integration's total, which the
// integration's last chunk records before counting) runs that integration's
// finalize alone, then writes a completion record.  No workgroup ever waits
// for another: a wait is only for the host to publish, and it ends when the
// host sets quit or after spin_limit idle polls (the host relaunches the
// kernel when every workgroup has left and work is published).
template <int PREC>
__global__ void __launch_bounds__(kServedThreads) served_kernel(ServedArgs sa) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ __align__(16) ServedDesc d;
    __shared__ unsigned long long s_task;
    __shared__ int s_go, s_fin;
    const int t = static_cast<int>(threadIdx.x);
    for (;;) {
        if (t == 0) {
            int go = 0;
            unsigned long long task = 0;
            for (unsigned long long idle = 0; idle < sa.spin_limit;) {
                const unsigned long long pub =
                    __hip_atomic_load(sa.published, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                unsigned long long c = __hip_atomic_load(sa.cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (c < pub) {
                    if (__hip_atomic_compare_exchange_strong(sa.cursor, &c, c + 1, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) {
                        task = c;
                        go = 1;
                        break;
                    }
                    continue;  // another workgroup took it: look again at once
                }
                if (__hip_atomic_load(sa.quit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
                    go = -1;
                    break;
                }
                __builtin_amdgcn_s_sleep(32);
                ++idle;
            }
            s_task = task;
            s_go = go;
        }
        __syncthreads();
        if (s_go != 1) {
            if (t == 0) {
                __hip_atomic_fetch_add(sa.status, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
                if (s_go == 0) __hip_atomic_fetch_add(sa.status + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            return;
        }
        const unsigned long long task = s_task;
        const unsigned long long chunk = task / static_cast<unsigned>(sa.tasks);
        const int wg = static_cast<int>(task % static_cast<unsigned>(sa.tasks));
        const int slot = static_cast<int>(chunk % static_cast<unsigned>(sa.cap));
        copy_from_host(reinterpret_cast<uint32_t *>(&d), reinterpret_cast<const uint32_t *>(sa.ring + slot),
                       static_cast<int>(sizeof(ServedDesc) / 4));
        __syncthreads();
        if (wg < d.ntasks) {
            if (d.fold.nbits == 2)
                fold_body<2, PREC>(d.fold, wg, lds);
            else
                fold_body<8, PREC>(d.fold, wg, lds);
        }
        // every wave's atomics are acknowledged before the task is counted
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (t == 0) {
            unsigned *done = sa.task_done + 2 * d.sid + d.bank;
            unsigned *total = sa.fin_total + 2 * d.sid + d.bank;
            if (d.fin_total > 0) __hip_atomic_store(total, static_cast<unsigned>(d.fin_total), __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
            const unsigned v = __hip_atomic_fetch_add(done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
            const unsigned want = __hip_atomic_load(total, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            s_fin = (want != 0u && v == want) ? 1 : 0;
            // the ring slot is free for the host once every task of its chunk ended
            const unsigned c = __hip_atomic_fetch_add(sa.slot_cnt + slot, 1u, __ATOMIC_ACQ_REL,
                                                      __HIP_MEMORY_SCOPE_AGENT) + 1u;
            if (c == static_cast<unsigned>(sa.tasks)) {
                __hip_atomic_store(sa.slot_cnt + slot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(sa.slot_free + slot, chunk + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();
        if (s_fin) {
            // the whole integration is in the bank: finalize it here, every
            // part in turn (read, DFT, results into the stream's pinned slot,
            // clear the bank), then report it
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int nwg = (d.fin.N + 63) / 64;
            for (int part = 0; part < nwg; ++part) {
                finalize_body(d.fin, part, nwg, lds);
                __syncthreads();
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            if (t == 0) {
                __hip_atomic_store(sa.task_done + 2 * d.sid + d.bank, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(sa.fin_total + 2 * d.sid + d.bank, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
                const unsigned long long k = atomicAdd(sa.done_cursor, 1ull);
                ServedDone *r = sa.done + k % static_cast<unsigned>(sa.done_cap);
                __hip_atomic_store(&r->sid, d.sid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&r->integ, d.integ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&r->seq, k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            __syncthreads();
        }
    }
}

}  // namespace

void launch_served(const ServedArgs &a, int prec, int grid, int threads, size_t lds, hipStream_t s) {
    if (prec == 0)
        hipLaunchKernelGGL(served_kernel<0>, dim3(grid), dim3(threads), lds, s, a);
    else if (prec == 1)
        hipLaunchKernelGGL(served_kernel<1>, dim3(grid), dim3(threads), lds, s, a);
    else
        hipLaunchKernelGGL(served_kernel<2>, dim3(grid), dim3(threads), lds, s, a);
}

}  // namespace pcal
