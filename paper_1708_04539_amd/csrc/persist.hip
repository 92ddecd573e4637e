// persist.hip -- persistent, dependency-driven level sweep.
//
// Algorithm 1 needs, before supernode K is processed, every supernode of
// C_L(K) and C_U(K) finished; the paper's scheduler (section on
// inter-supernode parallelism) launches tasks by a priority list and adds no
// synchronisation beyond these data dependencies.  This kernel does the same
// on one GPU: a fixed grid of workgroups takes tasks in queue order from an
// atomic counter.  The queue holds, level by level from the root, the gather
// tiles, the tiles of the step-3/5 products and the tiles of the step-4
// product of every supernode.  Per-supernode counters carry the
// dependencies:
//   gather tile of K   waits until the parent P of K is complete (every tile
//                      of its step-3/5/4 products done).  For the
//                      structurally symmetric pattern, C(K) minus P lies in
//                      C(P), so by induction all of C(K) is then complete;
//   step-3/5 tile of K waits for all gather tiles of K;
//   step-4 tile of K   waits for all tiles of the step-3 product of K.
// Every task waits only on tasks earlier in the queue, and tasks are taken in
// queue order, so the earliest unfinished task can always run: no deadlock.
// Waits are bounded (SPIN_LIMIT); a wait that runs out sets an error flag and
// the task proceeds, so that every workgroup still reaches the end of the
// queue and the grid drains.  Writes are published with a device-scope
// release before a counter increment and observed with a device-scope
// acquire, which also makes them visible across the XCDs.
#include <hip/hip_runtime.h>

#include "device_types.hpp"
#include "kernels.hpp"
#include "tiles.hpp"

namespace selinv {

// about 2^26 polls of ~64 cycles: seconds, far beyond any legitimate wait
constexpr long SPIN_LIMIT = 1L << 26;

// Poll with relaxed device-scope loads (coherent across the XCDs without
// touching the caches) and acquire once, after the wait succeeded: an acquire
// invalidates the L2 of the XCD, which must not happen on every poll.
__device__ inline void wait_geq(const int32_t *p, int32_t target, int32_t *err) {
    if (target <= 0) return;
    for (long i = 0; i < SPIN_LIMIT; i++) {
        if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int MODE>
__global__ __launch_bounds__(256) void sweep_kernel(const PersistArgs a) {
    typedef typename Mode<MODE>::T T;
    union Shared {
        Smem<MODE, 64, 64> g;
        GatherSmem<T> t;
    };
    __shared__ Shared sm;
    __shared__ int32_t task;
    for (;;) {
        __syncthreads();  // the previous task is done with LDS and `task`
        if (threadIdx.x == 0) task = __hip_atomic_fetch_add(a.head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int32_t t = task;
        if (t >= a.ntasks) break;
        const PTask tk = a.tasks[t];
        if (threadIdx.x == 0) {
            const PSn me = a.sn[tk.gid];
            if (tk.type == PT_GATHER) {
                if (me.parent >= 0) wait_geq(&a.cnt[3 * me.parent + 2], a.sn[me.parent].n_all, a.err);
            } else if (tk.type == PT_STEP35) {
                wait_geq(&a.cnt[3 * tk.gid + 0], me.n_gather, a.err);
            } else {
                wait_geq(&a.cnt[3 * tk.gid + 1], me.n_zu, a.err);
            }
        }
        __syncthreads();
        if (tk.type == PT_GATHER)
            gather_tile<T>(a.mats[tk.mat], tk.K, tk.i0, tk.i1, sm.t);
        else if (tk.type == PT_STEP35)
            gemm_tile<MODE, 64, 64, T, T, false>(a.probs[tk.prob], tk.i0, tk.i1, sm.g);
        else
            gemm_tile<MODE, 64, 64, T, double, true>(a.probs[tk.prob], tk.i0, tk.i1, sm.g);
        __syncthreads();  // every thread's stores of this task are complete
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (tk.type == PT_GATHER) {
                atomicAdd(&a.cnt[3 * tk.gid + 0], 1);
            } else {
                if (tk.is_zu) atomicAdd(&a.cnt[3 * tk.gid + 1], 1);
                atomicAdd(&a.cnt[3 * tk.gid + 2], 1);
            }
        }
    }
}

// Small supernodes (c_L, c_U, s <= 64): one workgroup does the whole of
// Algorithm 1 steps 3-5 for one supernode -- gather G_K (one tile), then the
// step-3 and step-5 products, then the step-4 product -- so that the deep
// levels of the tree cost one launch instead of three.  G_K and the step-3
// result are written to global memory and read back by the same workgroup
// after a barrier (workgroup-scope ordering suffices).
template <int MODE>
__global__ __launch_bounds__(256) void small_kernel(const MatDev *__restrict__ mats, const GemmProb *__restrict__ probs,
                                                    const SmallItem *__restrict__ items) {
    typedef typename Mode<MODE>::T T;
    union Shared {
        Smem<MODE, 64, 64> g;
        GatherSmem<T> t;
    };
    __shared__ Shared sm;
    const SmallItem it = items[blockIdx.x];
    const SELINV_GLOBAL SnRec *sn = gptr(mats[it.mat].sn);
    if (sn[it.K].cl > 0 && sn[it.K].cu > 0) gather_tile<T>(mats[it.mat], it.K, 0, 0, sm.t);
    __syncthreads();
    if (it.pzu >= 0) gemm_tile<MODE, 64, 64, T, T, false>(probs[it.pzu], 0, 0, sm.g);
    if (it.pzl >= 0) gemm_tile<MODE, 64, 64, T, T, false>(probs[it.pzl], 0, 0, sm.g);
    __syncthreads();
    if (it.pg4 >= 0) gemm_tile<MODE, 64, 64, T, double, true>(probs[it.pg4], 0, 0, sm.g);
}

hipError_t launch_small(int mode, const MatDev *mats, const GemmProb *probs, const SmallItem *items, int count,
                        hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (mode == CMP_F64)
        hipLaunchKernelGGL(small_kernel<CMP_F64>, dim3(count), dim3(256), 0, st, mats, probs, items);
    else if (mode == CMP_F32)
        hipLaunchKernelGGL(small_kernel<CMP_F32>, dim3(count), dim3(256), 0, st, mats, probs, items);
    else
        hipLaunchKernelGGL(small_kernel<CMP_BF16X3>, dim3(count), dim3(256), 0, st, mats, probs, items);
    return hipGetLastError();
}

// zero the counters, the queue head and the error flag (a kernel rather than a
// memset, so that the sweep can be recorded into a HIP graph)
__global__ void sweep_reset_kernel(int32_t *cnt, int64_t n, int32_t *head, int32_t *err) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) cnt[i] = 0;
    if (i == 0) {
        *head = 0;
        *err = 0;
    }
}

int persist_grid(int mode) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e;
    if (mode == CMP_F64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, sweep_kernel<CMP_F64>, 256, 0);
    else if (mode == CMP_F32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, sweep_kernel<CMP_F32>, 256, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, sweep_kernel<CMP_BF16X3>, 256, 0);
    if (e != hipSuccess || per <= 0) per = 1;
    return cus * per;
}

hipError_t launch_persist(int mode, const PersistArgs &a, int64_t ncnt, int grid, hipStream_t st) {
    const int64_t nb = (std::max<int64_t>(ncnt, 1) + 255) / 256;
    hipLaunchKernelGGL(sweep_reset_kernel, dim3((unsigned)nb), dim3(256), 0, st, a.cnt, ncnt, a.head, a.err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.ntasks <= 0 || grid <= 0) return hipSuccess;
    if (mode == CMP_F64)
        hipLaunchKernelGGL(sweep_kernel<CMP_F64>, dim3(grid), dim3(256), 0, st, a);
    else if (mode == CMP_F32)
        hipLaunchKernelGGL(sweep_kernel<CMP_F32>, dim3(grid), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(sweep_kernel<CMP_BF16X3>, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace selinv
