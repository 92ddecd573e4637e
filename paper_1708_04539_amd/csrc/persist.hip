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
//   gather tile of K   waits until every supernode its gather reads is
//                      complete (every tile of its step-3/5/4 products
//                      done): with the exact analysis every supernode that
//                      R_L(K) u R_U(K) meets; with the symmetrized one the
//                      parent P alone, since C(K) minus P lies in C(P) and by
//                      induction all of C(K) is then complete;
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
                for (int d = 0; d < me.ndep; d++) {
                    const int32_t P = a.deps[me.dep_off + d];
                    wait_geq(&a.cnt[3 * P + 2], a.sn[P].n_all, a.err);
                }
            } else if (tk.type == PT_STEP35) {
                wait_geq(&a.cnt[3 * tk.gid + 0], me.n_gather, a.err);
            } else {
                wait_geq(&a.cnt[3 * tk.gid + 1], me.n_zu, a.err);
            }
        }
        __syncthreads();
        if (tk.type == PT_GATHER)
            gather_tile<T>(a.mats[tk.mat], gather_desc(a.mats[tk.mat], tk.mat, tk.K, tk.i0, tk.i1), sm.t);
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
// Algorithm 1 steps 3-5 for one supernode, so that a level of them costs one
// launch instead of three.
//   0. each wavefront owns one block of 16 columns (of the s columns of the
//      three results) and loads its columns of Lhat and Uhat straight from
//      global memory into registers, before anything else: those loads are
//      in flight during the gather;
//   1. gather G_K (one tile) into LDS; it never goes to global memory;
//   2. the step-3 product -G^T Lhat and the step-5 product -G Uhat^T, 16x16
//      output tiles, op(A) from the LDS copy of G; the step-3 result is also
//      kept in LDS;
//   3. the step-4 product from that LDS copy and the Uhat registers.
// When s < 49 several wavefronts share a column block and split its row
// blocks.  Products run with the k order, operand roles and operand split of
// the grouped GEMM (v_mfma_f64/f32_16x16x4; split-BF16: per 32-wide k chunk
// B_lo A_hi, B_hi A_lo, B_hi A_hi on v_mfma_f32_16x16x32_bf16), so that the
// results are bitwise those of the per-phase launches in every form.
template <typename T>
struct SmallSmem {
    // G_K while steps 3 and 5 read it, then A^{-T}(K, R_U)^T for step 4
    // (zu[b][j]); one tile, so that four workgroups fit on a compute unit
    GatherSmem<T> g;
};

template <typename T>
struct SmallMfma;
template <>
struct SmallMfma<double> {
    typedef v4d Acc;
    static __device__ __forceinline__ Acc step(double b, double a, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c, 0, 0, 0);
    }
    // column of the 16x16 result held in item v of lane l
    static __device__ __forceinline__ int col(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct SmallMfma<float> {
    typedef v4f Acc;
    static __device__ __forceinline__ Acc step(float b, float a, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(b, a, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int col(int l, int v) { return 4 * (l >> 4) + v; }
};

// op(B)(k, n0 + lane % 16) for k = 4 q + lane / 16, q < 16, from a K x N
// column-major operand (clamped addresses; zero outside)
template <typename T>
__device__ __forceinline__ void small_loadB(T (&bv)[16], const T *Bp, int64_t ldb, int N, int K, int n0) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    if (!Bp || K <= 0) {
#pragma unroll
        for (int q = 0; q < 16; q++) bv[q] = (T)0;
        return;
    }
    const SELINV_GLOBAL T *B = gptr(Bp);
    const int n = n0 + li;
    const int64_t nc = min(n, N - 1);
#pragma unroll
    for (int q = 0; q < 16; q++) bv[q] = B[min(4 * q + lk, K - 1) + nc * ldb];
#pragma unroll
    for (int q = 0; q < 16; q++) bv[q] = (n < N && 4 * q + lk < K) ? bv[q] : (T)0;
}

// One 16x16 tile (rows m0..) of op(A) op(B): op(A)(m, k) from getA (LDS),
// op(B) from the registers of small_loadB, k < K <= 64.
template <typename T, typename GetA>
__device__ __forceinline__ typename SmallMfma<T>::Acc small_tile(GetA getA, const T (&bv)[16], int M, int K,
                                                                 int m0) {
    typedef typename SmallMfma<T>::Acc Acc;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    Acc acc = {0, 0, 0, 0};
    const int m = m0 + li;
#pragma unroll
    for (int q = 0; q < 16; q++) {
        if (4 * q >= K) break;
        const int k = 4 * q + lk;
        const T a = (m < M && k < K) ? getA(m, k) : (T)0;
        acc = SmallMfma<T>::step(bv[q], a, acc);
    }
    return acc;
}

// Split-BF16 operands of the small products, as the grouped GEMM splits
// them: x = hi + lo, hi = bf16(x), lo = bf16(x - hi).  Lane l holds k =
// 32 c + 8 (l / 16) + e, e < 8, of chunk c (K <= 64: two chunks).
struct SplitB {
    v8bf h[2], l[2];
};

__device__ __forceinline__ void split_bf16(float v, __bf16 &h, __bf16 &l) {
    h = (__bf16)v;
    l = (__bf16)(v - (float)h);
}

// op(B)(k, n0 + lane % 16) of a K x N column-major FP32 operand, split
__device__ __forceinline__ void small_loadB_split(SplitB &b, const float *Bp, int64_t ldb, int N, int K, int n0) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    float v[2][8];
    if (!Bp || K <= 0) {
#pragma unroll
        for (int c = 0; c < 2; c++)
#pragma unroll
            for (int e = 0; e < 8; e++) v[c][e] = 0.0f;
    } else {
        const SELINV_GLOBAL float *B = gptr(Bp);
        const int n = n0 + li;
        const int64_t nc = min(n, N - 1);
#pragma unroll
        for (int c = 0; c < 2; c++)
#pragma unroll
            for (int e = 0; e < 8; e++) v[c][e] = B[min(32 * c + 8 * lk + e, K - 1) + nc * ldb];
#pragma unroll
        for (int c = 0; c < 2; c++)
#pragma unroll
            for (int e = 0; e < 8; e++) v[c][e] = (n < N && 32 * c + 8 * lk + e < K) ? v[c][e] : 0.0f;
    }
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int e = 0; e < 8; e++) {
            __bf16 h, l;
            split_bf16(v[c][e], h, l);
            b.h[c][e] = h;
            b.l[c][e] = l;
        }
}

// One 16x16 tile (rows m0..) of op(A) op(B) in split-BF16: op(A)(m, k) from
// getA (LDS), op(B) split in registers, k < K <= 64.
template <typename GetA>
__device__ __forceinline__ v4f small_tile_split(GetA getA, const SplitB &b, int M, int K, int m0) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    v4f acc = {0, 0, 0, 0};
    const int m = m0 + li;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        if (32 * c >= K) break;
        v8bf ah, al;
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int k = 32 * c + 8 * lk + e;
            const float a = (m < M && k < K) ? getA(m, k) : 0.0f;
            __bf16 h, l;
            split_bf16(a, h, l);
            ah[e] = h;
            al[e] = l;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b.l[c], ah, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b.h[c], al, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b.h[c], ah, acc, 0, 0, 0);
    }
    return acc;
}

// op(B) registers of one wavefront's column block, in the form's arithmetic
template <int MODE>
struct SmallB {
    typedef typename Mode<MODE>::T T;
    T v[16];
    __device__ __forceinline__ void load(const T *Bp, int64_t ldb, int N, int K, int n0) {
        small_loadB<T>(v, Bp, ldb, N, K, n0);
    }
    template <typename GetA>
    __device__ __forceinline__ typename SmallMfma<T>::Acc tile(GetA getA, int M, int K, int m0) const {
        return small_tile<T>(getA, v, M, K, m0);
    }
};
template <>
struct SmallB<CMP_BF16X3> {
    SplitB v;
    __device__ __forceinline__ void load(const float *Bp, int64_t ldb, int N, int K, int n0) {
        small_loadB_split(v, Bp, ldb, N, K, n0);
    }
    template <typename GetA>
    __device__ __forceinline__ v4f tile(GetA getA, int M, int K, int m0) const {
        return small_tile_split(getA, v, M, K, m0);
    }
};

// G_K of a small supernode (c_L, c_U <= 64) into tileS[b][a] from its source
// codes.  The threads walk the codes in storage order (both code arrays are
// laid out in the order their side reads the panels), CH entries per thread
// and round (every load of a round in flight together): 4 in FP64, so that
// the kernel stays within the registers of four workgroups per compute unit
// (one round up to 1024 entries), 8 in FP32 (up to 2048).
template <typename T>
__device__ __forceinline__ void gather_small_codes(const MatDev &M, int cl, int cu, int64_t c_off,
                                                   T (&tileS)[64][65]) {
    constexpr int CH = sizeof(T) == sizeof(double) ? 4 : 8;
    const int tid = threadIdx.x, n = cl * cu;
    const SELINV_GLOBAL uint32_t *cL = gptr(M.gcL) + c_off;
    const SELINV_GLOBAL uint32_t *cU = gptr(M.gcU) + c_off;
    const SELINV_GLOBAL T *ZL = gptr((const T *)M.ZL);
    const SELINV_GLOBAL T *ZU = gptr((const T *)M.ZU);
    const SELINV_GLOBAL double *Zd = gptr(M.Zd);
    for (int base = 0; base < n; base += 256 * CH) {
        uint32_t kl[CH], ku[CH];
#pragma unroll
        for (int t = 0; t < CH; t++) {
            const int e = base + tid + 256 * t, i = e < n ? e : 0;
            kl[t] = cL[i];
            ku[t] = cU[i];
        }
        T vl[CH], vu[CH];
#pragma unroll
        for (int t = 0; t < CH; t++) {
            const uint32_t k = kl[t] >> GCODE_SHIFT, off = kl[t] & GCODE_MASK;
            if constexpr (sizeof(T) == sizeof(double)) {
                // one load: the diagonal blocks and the L panels hold the same type
                vl[t] = (k == 1 ? (const SELINV_GLOBAL T *)Zd : ZL)[k >= 1 && k <= 2 ? off : 0];
            } else {
                const double vd = Zd[k == 1 ? off : 0];
                const T v = ZL[k == 2 ? off : 0];
                vl[t] = k == 1 ? (T)vd : v;
            }
            const uint32_t k3 = ku[t] >> GCODE_SHIFT, off3 = ku[t] & GCODE_MASK;
            vu[t] = ZU[k3 == 3 ? off3 : 0];
        }
#pragma unroll
        for (int t = 0; t < CH; t++) {
            const int e = base + tid + 256 * t;
            if (e >= n) continue;
            const uint32_t k = kl[t] >> GCODE_SHIFT;
            if (k == 1 || k == 2) tileS[e / cl][e % cl] = vl[t];
            if ((ku[t] >> GCODE_SHIFT) == 3) tileS[e % cu][e / cu] = vu[t];
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(256, 4) void small_kernel(const MatDev *__restrict__ mats, const GemmProb *__restrict__ probs,
                                                    const SmallItem *__restrict__ items) {
    typedef typename Mode<MODE>::T T;
    typedef SmallMfma<T> MF;
    __shared__ SmallSmem<T> sm;
    const SmallItem it = items[blockIdx.x];
    const int s = it.s, cl = it.cl, cu = it.cu;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15;
    // column block of this wavefront, and its share of the row blocks
    const int ns = (s + 15) / 16, per = 4 / ns;  // wavefronts per column block
    const bool active = wave < ns * per;
    const int n0 = 16 * (wave % ns), mfirst = wave / ns;
    const GemmProb *pzu = it.pzu >= 0 ? &probs[it.pzu] : nullptr;
    const GemmProb *pzl = it.pzl >= 0 ? &probs[it.pzl] : nullptr;
    const GemmProb *pg4 = it.pg4 >= 0 ? &probs[it.pg4] : nullptr;
    SmallB<MODE> bL, bU;
    bL.load(pzu ? (const T *)pzu->B : nullptr, pzu ? pzu->ldb : 1, s, cl, n0);
    const GemmProb *pu = pzl ? pzl : pg4;  // Uhat: op(B) of steps 5 and 4
    bU.load(pu ? (const T *)pu->B : nullptr, pu ? pu->ldb : 1, s, cu, n0);

    // (a small supernode with a non-empty G_K always has source codes)
    if (cl > 0 && cu > 0) gather_small_codes<T>(mats[it.mat], cl, cu, it.c_off, sm.g.tileS);
    __syncthreads();
    T(&G)[64][65] = sm.g.tileS;  // G[b][a] = G_K(a, b), later zu[b][j]
    // step 3: A^{-T}(K,R_U)^T = -G^T Lhat (cu x s); the wavefront's tiles stay
    // in registers until every wavefront has finished reading G
    typename MF::Acc zacc[4];
    if (active) {
        if (pzu) {
            SELINV_GLOBAL T *C = gptr_w((T *)pzu->C);
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int mb = mfirst + i * per;
                if (16 * mb >= cu) break;
                zacc[i] = bL.tile([&](int m, int k) { return G[m][k]; }, cu, cl, 16 * mb);
                const int m = 16 * mb + li;
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int c = n0 + MF::col(lane, v);
                    zacc[i][v] = (T)(pzu->alpha * (double)zacc[i][v]);
                    if (m < cu && c < s) C[m + (int64_t)c * pzu->ldc] = zacc[i][v];
                }
            }
        }
        // step 5: A^{-T}(R_L,K) = -G Uhat^T (cl x s)
        if (pzl) {
            SELINV_GLOBAL T *C = gptr_w((T *)pzl->C);
            for (int mb = mfirst; 16 * mb < cl; mb += per) {
                const typename MF::Acc acc = bU.tile([&](int m, int k) { return G[k][m]; }, cl, cu, 16 * mb);
                const int m = 16 * mb + li;
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int c = n0 + MF::col(lane, v);
                    if (m >= cl || c >= s) continue;
                    C[m + (int64_t)c * pzl->ldc] = (T)(pzl->alpha * (double)acc[v]);
                }
            }
        }
    }
    __syncthreads();
    // A^{-T}(K,R_U)^T into LDS over G
    if (active && pzu) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int mb = mfirst + i * per;
            if (16 * mb >= cu) break;
            const int m = 16 * mb + li;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int c = n0 + MF::col(lane, v);
                if (m < cu && c < s) G[m][c] = zacc[i][v];
            }
        }
    }
    __syncthreads();
    // step 4: A^{-T}(K,K) -= A^{-T}(K,R_U) Uhat^T (FP64 accumulation)
    if (active && pg4) {
        SELINV_GLOBAL double *C = gptr_w((double *)pg4->C);
        // the initial A^{-T}(K,K) of all of this wavefront's row blocks in
        // flight together (clamped addresses), then the products
        double cin[4][4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int m = min(16 * (mfirst + i * per) + li, s - 1);
#pragma unroll
            for (int v = 0; v < 4; v++) cin[i][v] = C[m + (int64_t)min(n0 + MF::col(lane, v), s - 1) * pg4->ldc];
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int mb = mfirst + i * per;
            if (16 * mb >= s) break;
            const typename MF::Acc acc = bU.tile([&](int m, int k) { return G[k][m]; }, s, cu, 16 * mb);
            const int m = 16 * mb + li;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int c = n0 + MF::col(lane, v);
                if (m >= s || c >= s) continue;
                double r = pg4->alpha * (double)acc[v];
                r += pg4->beta * cin[i][v];
                C[m + (int64_t)c * pg4->ldc] = r;
            }
        }
    }
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
