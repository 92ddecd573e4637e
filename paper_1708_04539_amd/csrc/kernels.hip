// kernels.hip -- gfx950 kernels of supernodal selected inversion
// (arXiv:1708.04539, Algorithm 1).
//
//   tri_base_kernel  diagonal 64x64 sub-blocks of (L_KK)^{-1} and (U_KK)^{-1}
//                    in FP64 (step 2 / step 4 initialisation); the rest of the
//                    triangular inverses comes from GEMM rounds.
//   (the grouped MFMA GEMM of steps 2-5 lives in gemm.hip)
//   gather_kernel    G_K = A^{-T}(R_L(K), R_U(K)) from the diagonal blocks and
//                    panels of the ancestors (Theorem 1), one 64x64 tile per
//                    workgroup with the tile's index metadata staged in LDS;
//                    entries from U-side panels are read along their
//                    contiguous dimension and transposed through LDS.
//   extract_kernel   step 6: the selected entries, one per entry of A.
#include <hip/hip_runtime.h>

#include "device_types.hpp"
#include "kernels.hpp"
#include "tiles.hpp"

namespace selinv {


// ---------------------------------------------------------------------------
// triangular inversion, diagonal 64x64 blocks
// ---------------------------------------------------------------------------
// One workgroup (4 wavefronts) inverts both triangles of the 64x64 (16 NB
// wide) diagonal sub-block that starts at row/column o of one supernode's packed
// L_KK \ U_KK (column-major, s x s; L unit lower, U upper).  A ragged
// sub-block (s - o < 64) is padded with the identity, whose inverse stays the
// identity and is not stored.  Blocked by 16:
//   1. the 16x16 diagonal blocks, by substitution: wavefront w takes block w;
//      lane c < 16 forms column c of (L_ww)^{-1} and lane 16 + c column c of
//      (U_ww^T)^{-1} = row c of (U_ww)^{-1}, the same forward recurrence for
//      both (the L diagonal is 1; U's diagonal enters through reciprocals
//      formed once per block);
//   2. the off-diagonal 16x16 blocks by distance d = 1, 2, 3 from the
//      diagonal, on v_mfma_f64_16x16x4 (X = L^{-1}, Y = U^{-1}):
//        X_ij = -X_ii (sum_{k=j}^{i-1} L_ik X_kj)      (i = j + d)
//        Y_ij = -Y_ii (sum_{k=i+1}^{j} U_ik Y_kj)      (j = i + d)
//      every block of one distance in parallel, one per wavefront.
// Both results live packed in one LDS tile (strict lower part: L^{-1}; upper
// part with the diagonal: U^{-1}) and are written out with coalesced stores,
// together with the zeros of L^{-1} above the sub-block and of U^{-1} left of
// it.  The off-diagonal 64x64 blocks of the inverses come from the GEMM rounds
// of the recursive doubling (X21 = -B^{-1} C A^{-1} for L,
// X12 = -A^{-1} C B^{-1} for U).
// NB = 4 handles every 64-wide sub-block; NB = 1 and 2 (16- and 32-wide
// blocks, far less LDS) serve the supernodes of at most 16 or 32 columns
// whose normalisation runs in the same workgroup.
template <int NB>
struct TriSmem {
    static constexpr int W = 16 * NB;
    double Ds[W][65];        // Ds[c][r] = D(o + r, o + c), identity-padded; later a panel (64 rows)
    double Xs[W][W + 1];     // Xs[c][r]: r > c: L^{-1}(r, c); r <= c: U^{-1}(r, c)
    double Ts[4][16][17];    // per-wavefront 16x16 intermediate
    double rd[W];            // 1 / U(c, c)
};

typedef double v4d_t __attribute__((ext_vector_type(4)));

// L^{-1}(r, c) and U^{-1}(r, c) read from the packed tile (zero outside the
// triangle; the unit diagonal of L^{-1} is implicit)
template <class SM>
__device__ __forceinline__ double linv_at(const SM &sm, int r, int c) {
    return r > c ? sm.Xs[c][r] : (r == c ? 1.0 : 0.0);
}
template <class SM>
__device__ __forceinline__ double uinv_at(const SM &sm, int r, int c) { return r <= c ? sm.Xs[c][r] : 0.0; }

// One off-diagonal block at distance D, computed by the calling wavefront.
// The lanes feed the MFMA with A(i = lane % 16, k = lane / 16) and
// B(k = lane / 16, j = lane % 16); the result row is lane / 16 + 4 v, its
// column lane % 16 (register v of the accumulator).
template <int NB, int D>
__device__ __forceinline__ void tri_offdiag(TriSmem<NB> &sm, int t, int lane, int wave) {
    const bool upper = t >= NB - D;
    const int i = upper ? t - (NB - D) : t + D;  // row block of the result
    const int j = upper ? i + D : t;             // column block
    const int kb = upper ? 16 * (i + 1) : 16 * j;  // contraction range [kb, kb + 16 D)
    const int li = lane & 15, lk = lane >> 4;
    v4d_t acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16 * D; kk += 4) {
        const int k = kb + kk + lk;
        // factor entry L(16 i + li, k) or U(16 i + li, k): strictly off the diagonal
        const double a = sm.Ds[k][16 * i + li];
        const double bv = upper ? uinv_at(sm, k, 16 * j + li) : linv_at(sm, k, 16 * j + li);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; v++) sm.Ts[wave][lk + 4 * v][li] = acc[v];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    v4d_t out = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
        const int r = 16 * i + li, c = 16 * i + kk + lk;
        const double a = upper ? uinv_at(sm, r, c) : linv_at(sm, r, c);
        out = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sm.Ts[wave][kk + lk][li], out, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; v++) sm.Xs[16 * j + li][16 * i + lk + 4 * v] = -out[v];
    // the wavefront's next task overwrites Ts
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int NB, int D>
__device__ __forceinline__ void tri_round(TriSmem<NB> &sm, int lane, int wave) {
    __syncthreads();
    for (int t = wave; t < 2 * (NB - D); t += 4) tri_offdiag<NB, D>(sm, t, lane, wave);
}

// Normalisation and diagonal initialisation of a supernode with s, c_L,
// c_U <= 64, after its inverses are complete in sm.Xs (FP64 arithmetic on
// v_mfma_f64_16x16x4, results in the storage precision).  Every product is
// formed transposed (the MFMA takes the inverse as its first operand), so
// that a lane's results run down a column of the output and the stores are
// coalesced.  The panels are staged through sm.Ds, free after the rounds.
template <int NB>
__device__ __forceinline__ void tri_fused_epilogue(TriSmem<NB> &sm, const TriItem &it, int lane, int wave) {
    const int s = it.s, li = lane & 15, lk = lane >> 4;
    const int nbs = (s + 15) / 16;
    auto stage = [&](const double *pan, int rows) {
        // Ds[k][m] = pan(m, k), zero outside rows x s
        const SELINV_GLOBAL double *P = gptr(pan);
        const int r = lane, rr = min(r, rows - 1);
        double v[4 * NB];
#pragma unroll
        for (int q = 0; q < 4 * NB; q++) {
            const int c = wave + 4 * q;
            v[q] = P[(int64_t)rr + (int64_t)min(c, s - 1) * rows];
        }
#pragma unroll
        for (int q = 0; q < 4 * NB; q++) {
            const int c = wave + 4 * q;
            sm.Ds[c][r] = (r < rows && c < s) ? v[q] : 0.0;
        }
    };
    auto put = [&](void *out, int64_t idx, double v) {
        if (it.f32out)
            gptr_w((float *)out)[idx] = (float)v;
        else
            gptr_w((double *)out)[idx] = v;
    };
    // panel products: out(m, n) = sum_k pan(m, k) inv(k, n), inv(k, n) =
    // Linv(k, n) (L side) or Uinv(n, k) (U side)
    auto panel = [&](const double *pan, int rows, void *out, bool upper) {
        __syncthreads();  // Ds free (rounds done / previous panel read)
        stage(pan, rows);
        __syncthreads();
        const int mbs = (rows + 15) / 16;
        for (int t = wave; t < mbs * nbs; t += 4) {
            const int mb = t % mbs, nb = t / mbs;
            v4d_t acc = {0, 0, 0, 0};
            for (int kk = 0; kk < s; kk += 4) {
                const int k = kk + lk;
                const double a = upper ? uinv_at(sm, 16 * nb + li, k) : linv_at(sm, k, 16 * nb + li);
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sm.Ds[k][16 * mb + li], acc, 0, 0, 0);
            }
            // acc[v] = out(16 mb + li, 16 nb + lk + 4 v)
            const int m = 16 * mb + li;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int n = 16 * nb + lk + 4 * v;
                if (m < rows && n < s) put(out, m + (int64_t)n * rows, acc[v]);
            }
        }
    };
    if (it.lpan) panel(it.lpan, it.cl, it.Lh, false);
    if (it.upan) panel(it.upan, it.cu, it.Uh, true);
    // A^{-T}(K,K) := Linv^T Uinv^T:  Zd(m, n) = sum_k Linv(k, m) Uinv(n, k)
    SELINV_GLOBAL double *Zd = gptr_w(it.Zd);
    for (int t = wave; t < nbs * nbs; t += 4) {
        const int mb = t % nbs, nb = t / nbs;
        v4d_t acc = {0, 0, 0, 0};
        for (int kk = 0; kk < s; kk += 4) {
            const int k = kk + lk;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(uinv_at(sm, 16 * nb + li, k), linv_at(sm, k, 16 * mb + li),
                                                       acc, 0, 0, 0);
        }
        const int m = 16 * mb + li;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int n = 16 * nb + lk + 4 * v;
            if (m < s && n < s) Zd[m + (int64_t)n * s] = acc[v];
        }
    }
}

template <int NB>
__device__ __forceinline__ void tri_base_item(const TriItem &it, TriSmem<NB> &sm) {
    constexpr int W = 16 * NB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int s = it.s, o = it.j0, b = min(W, s - o);
    {
        // all loads of a thread in flight at once; addresses clamped into
        // the block, the identity padding selected afterwards
        constexpr int PER = W * W / 256 > 0 ? W * W / 256 : 1;
        double v[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int e = tid + 256 * q, r = e % W, c = e / W;
            v[q] = gptr(it.D)[(int64_t)(o + min(r, b - 1)) + (int64_t)(o + min(c, b - 1)) * s];
        }
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int e = tid + 256 * q, r = e % W, c = e / W;
            if (e >= W * W) continue;
            const double d = (r < b && c < b) ? v[q] : (r == c ? 1.0 : 0.0);
            sm.Ds[c][r] = d;
            if (r == c) sm.rd[c] = 1.0 / d;
        }
    }
    __syncthreads();
    if (wave < NB) {
        const int base = 16 * wave, c = lane & 15;
        const bool up = (lane & 16) != 0;  // lanes 32..63 repeat lanes 0..31 and store nothing
        double x[16];
#pragma unroll
        for (int r = 0; r < 16; r++) x[r] = r == c ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (up) x[k] = x[k] * sm.rd[base + k];
#pragma unroll
            for (int r = k + 1; r < 16; r++)
                x[r] = fma(-(up ? sm.Ds[base + r][base + k] : sm.Ds[base + k][base + r]), x[k], x[r]);
        }
        if (lane < 32) {
#pragma unroll
            for (int r = 0; r < 16; r++) {
                if (!up && r > c) sm.Xs[base + c][base + r] = x[r];  // L^{-1}(r, c)
                if (up && r >= c) sm.Xs[base + r][base + c] = x[r];  // U^{-1}(c, r)
            }
        }
    }
    if constexpr (NB >= 2) tri_round<NB, 1>(sm, lane, wave);
    if constexpr (NB >= 3) tri_round<NB, 2>(sm, lane, wave);
    if constexpr (NB >= 4) tri_round<NB, 3>(sm, lane, wave);
    __syncthreads();
    if (it.fused) {
        tri_fused_epilogue<NB>(sm, it, lane, wave);
        return;
    }
    if constexpr (NB == 4) {
        SELINV_GLOBAL double *Linv = gptr_w(it.Linv), *Uinv = gptr_w(it.Uinv);
        {
            const int r = lane;
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int c = wave + 4 * q;
                if (r < b && c < b) {
                    const int64_t g = (int64_t)(o + r) + (int64_t)(o + c) * s;
                    Linv[g] = linv_at(sm, r, c);
                    Uinv[g] = uinv_at(sm, r, c);
                }
            }
        }
        // zeros of L^{-1} above the sub-block and of U^{-1} left of it
        for (int c = wave; c < b; c += 4)
            for (int r = lane; r < o; r += 64) Linv[r + (int64_t)(o + c) * s] = 0.0;
        if (lane < b)
            for (int c = wave; c < o; c += 4) Uinv[(o + lane) + (int64_t)c * s] = 0.0;
    }
}

// One item per workgroup.
template <int NB>
__global__ __launch_bounds__(256) void tri_base_kernel(const TriItem *__restrict__ items) {
    __shared__ TriSmem<NB> sm;
    tri_base_item<NB>(items[blockIdx.x], sm);
}

// Items [0, count), item b + q gridDim.x to workgroup b: a launch with fewer
// workgroups than items keeps at most that many resident (the side-stream
// inversion of the leaves, beside the level chain: one 64-wide workgroup takes
// half the LDS of a compute unit).  The item is a call: inlined into the
// loop, the item's per-lane LDS addresses are hoisted out of it and held
// across iterations, which more than triples the kernel's registers.
template <int NB>
__device__ __attribute__((noinline)) void tri_base_item_call(const TriItem *__restrict__ items, int b,
                                                             TriSmem<NB> &sm) {
    tri_base_item<NB>(items[b], sm);
}

template <int NB>
__global__ __launch_bounds__(256) void tri_base_loop_kernel(const TriItem *__restrict__ items, int count) {
    __shared__ TriSmem<NB> sm;
    for (int b = blockIdx.x; b < count; b += gridDim.x) {
        tri_base_item_call<NB>(items, b, sm);
        __syncthreads();  // LDS free for the next item
    }
}

// ---------------------------------------------------------------------------
// gather
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(const MatDev *__restrict__ mats,
                                                     const GatherTile *__restrict__ tiles) {
    __shared__ GatherSmem<T> sm;
    const GatherTile tl = tiles[blockIdx.x];
    gather_tile<T>(mats[tl.mat], tl, sm);
}

// ---------------------------------------------------------------------------
// split-K reduction of the step-4 products
// ---------------------------------------------------------------------------
// blockIdx.y = item; each thread one entry of C; the partial products are
// added in a fixed order, so the result does not depend on the schedule.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const ReduceItem *__restrict__ items,
                                                            const MatDev *__restrict__ mats) {
    const ReduceItem it = items[blockIdx.y];
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, mn = (int64_t)it.M * it.N;
    if (e >= mn) return;
    const int m = (int)(e % it.M), n = (int)(e / it.M);
    // complex blocks: column n of the parts is column 2n of C, which gives
    // entry (m ^ 1, 2n + 1)
    const int nc = it.cpx ? 2 * n : n;
    SELINV_GLOBAL double *C = gptr_w(it.C) + m + (int64_t)nc * it.ldc;
    const SELINV_GLOBAL double *P = gptr(it.P) + e;
    double acc = *C;
    for (int p = 0; p < it.nparts; p++) acc += P[p * it.pstride];
    *C = acc;
    const double csign = (m & 1) ? -1.0 : 1.0;
    if (it.cpx) gptr_w(it.C)[(m ^ 1) + (int64_t)(nc + 1) * it.ldc] = csign * acc;
    if (it.push_sn < 0) return;
    // the final entry (m, n) of A^{-T}(P,P) into G_K of every child K of P
    // (the children's gathers skip these entries)
    const MatDev &Md = mats[it.push_mat];
    const SELINV_GLOBAL SnRec *sn = gptr(Md.sn);
    const SELINV_GLOBAL int32_t *kp = gptr(Md.kids_ptr);
    const SELINV_GLOBAL int32_t *kids = gptr(Md.kids);
    const int Pa = it.push_sn, sP = it.M;
    for (int q = kp[Pa]; q < kp[Pa + 1]; q++) {
        const int32_t K = kids[q];
        const SELINV_GLOBAL int32_t *posL = gptr(Md.push_pos) + gptr(Md.push_off)[K];
        for (int h = 0; h < (it.cpx ? 2 : 1); h++) {
            // h = 1: the odd-column entry that this one gives
            const int a = posL[h ? (m ^ 1) : m], b = posL[sP + nc + h];
            if (a < 0 || b < 0) continue;
            const double v = h ? csign * acc : acc;
            const int64_t g = sn[K].g_off + a + (int64_t)b * sn[K].cl;
            if (it.g_f32)
                gptr_w((float *)Md.G)[g] = (float)v;
            else
                gptr_w((double *)Md.G)[g] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// extraction
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void extract_kernel(ExtractArgs a) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= a.nnz) return;
    const int64_t loc = gptr(a.loc)[p];
    const int64_t kind = loc >> 60, off = loc & ((int64_t(1) << 60) - 1);
    double v;
    if (kind == 0)
        v = gptr(a.Zd)[off];
    else if (kind == 1)
        v = (double)gptr((const T *)a.ZL)[off];
    else
        v = (double)gptr((const T *)a.ZU)[off];
    gptr_w(a.out)[p] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_tri_base(const TriItem *items, int count, int nb, hipStream_t st, int max_groups) {
    if (count <= 0) return hipSuccess;
    if (nb != 1 && nb != 2 && nb != 4) return hipErrorInvalidValue;
    if (max_groups > 0 && max_groups < count) {
        const dim3 g(max_groups);
        if (nb == 1)
            hipLaunchKernelGGL(tri_base_loop_kernel<1>, g, dim3(256), 0, st, items, count);
        else if (nb == 2)
            hipLaunchKernelGGL(tri_base_loop_kernel<2>, g, dim3(256), 0, st, items, count);
        else
            hipLaunchKernelGGL(tri_base_loop_kernel<4>, g, dim3(256), 0, st, items, count);
    } else if (nb == 1) {
        hipLaunchKernelGGL(tri_base_kernel<1>, dim3(count), dim3(256), 0, st, items);
    } else if (nb == 2) {
        hipLaunchKernelGGL(tri_base_kernel<2>, dim3(count), dim3(256), 0, st, items);
    } else {
        hipLaunchKernelGGL(tri_base_kernel<4>, dim3(count), dim3(256), 0, st, items);
    }
    return hipGetLastError();
}

hipError_t launch_gather(int f64, const MatDev *mats, const GatherTile *tiles, int ntiles, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(gather_kernel<double>, dim3(ntiles), dim3(256), 0, st, mats, tiles);
    else
        hipLaunchKernelGGL(gather_kernel<float>, dim3(ntiles), dim3(256), 0, st, mats, tiles);
    return hipGetLastError();
}

hipError_t launch_splitk_reduce(const ReduceItem *items, int count, int64_t max_mn, const MatDev *mats,
                                hipStream_t st) {
    if (count <= 0 || max_mn <= 0) return hipSuccess;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((max_mn + 255) / 256), count), dim3(256), 0, st, items,
                       mats);
    return hipGetLastError();
}

hipError_t launch_extract(int f64, const ExtractArgs &a, hipStream_t st) {
    if (a.nnz <= 0) return hipSuccess;
    const int64_t blocks = (a.nnz + 255) / 256;
    if (f64)
        hipLaunchKernelGGL(extract_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(extract_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace selinv
