// kernels.hip -- gfx950 kernels of supernodal selected inversion
// (arXiv:1708.04539, Algorithm 1).
//
//   tri_inv_kernel   (L_KK)^{-1} and (U_KK)^{-1} in FP64 (step 2 / step 4
//                    initialisation), one wavefront per column.
//   gemm_kernel      grouped GEMM C = alpha op(A) op(B) + beta Cin over a list
//                    of 64x64 output tiles of many problems, on MFMA:
//                    FP64 (v_mfma_f64_16x16x4), FP32 (v_mfma_f32_16x16x4) or a
//                    two-term bfloat16 split of both operands with three
//                    products (v_mfma_f32_16x16x32_bf16).  Used for the
//                    normalisation of step 2, and steps 3, 4 and 5.
//   gather_kernel    G_K = A^{-T}(R_L(K), R_U(K)) from the diagonal blocks and
//                    panels of the ancestors (Theorem 1), one 64x64 tile per
//                    workgroup with the tile's index metadata staged in LDS;
//                    entries from U-side panels are read along their
//                    contiguous dimension and transposed through LDS.
//   extract_kernel   step 6: the selected entries, one per entry of A.
#include <hip/hip_runtime.h>

#include "device_types.hpp"
#include "kernels.hpp"

namespace selinv {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// triangular inversion
// ---------------------------------------------------------------------------
// Row i of a column is held by lane (i mod 64) in register x[i / 64]; the
// substitution broadcasts the finished entry with a lane shuffle and updates
// the remaining rows with coalesced loads of one column of the factor.
constexpr int TRI_MAXM = TRI_MAX_S / 64;

__global__ __launch_bounds__(256) void tri_inv_kernel(const TriItem *__restrict__ items) {
    const TriItem it = items[blockIdx.x];
    const int lane = threadIdx.x & 63;
    const int j = it.j0 + (threadIdx.x >> 6);
    const int s = it.s;
    if (j >= s) return;
    const double *D = it.D;
    double x[TRI_MAXM];

    // (L_KK)^{-1} e_j, L unit lower: forward substitution
#pragma unroll
    for (int m = 0; m < TRI_MAXM; m++) x[m] = (64 * m + lane == j) ? 1.0 : 0.0;
#pragma unroll
    for (int m = 0; m < TRI_MAXM; m++) {
        if (64 * m >= s) break;
        for (int kk = 0; kk < 64; kk++) {
            const int k = 64 * m + kk;
            if (k >= s) break;
            if (k < j) continue;
            const double xk = __shfl(x[m], kk, 64);
            const double *col = D + (int64_t)k * s;
#pragma unroll
            for (int m2 = m; m2 < TRI_MAXM; m2++) {
                const int i = 64 * m2 + lane;
                if (i > k && i < s) x[m2] -= col[i] * xk;
            }
        }
    }
#pragma unroll
    for (int m = 0; m < TRI_MAXM; m++) {
        const int i = 64 * m + lane;
        if (i < s) it.Linv[i + (int64_t)j * s] = x[m];
    }

    // (U_KK)^{-1} e_j, U upper: back substitution
#pragma unroll
    for (int m = 0; m < TRI_MAXM; m++) x[m] = (64 * m + lane == j) ? 1.0 : 0.0;
#pragma unroll
    for (int m = TRI_MAXM - 1; m >= 0; m--) {
        if (64 * m > j) continue;
        for (int kk = 63; kk >= 0; kk--) {
            const int k = 64 * m + kk;
            if (k > j) continue;
            const double *col = D + (int64_t)k * s;
            if (lane == kk) x[m] = x[m] / col[k];
            const double xk = __shfl(x[m], kk, 64);
#pragma unroll
            for (int m2 = 0; m2 <= m; m2++) {
                const int i = 64 * m2 + lane;
                if (i < k) x[m2] -= col[i] * xk;
            }
        }
    }
#pragma unroll
    for (int m = 0; m < TRI_MAXM; m++) {
        const int i = 64 * m + lane;
        if (i < s) it.Uinv[i + (int64_t)j * s] = x[m];
    }
}

// ---------------------------------------------------------------------------
// grouped GEMM on MFMA
// ---------------------------------------------------------------------------
// Tile 64x64, 256 threads = 4 wavefronts in a 2x2 arrangement, each owning a
// 32x32 quarter as 2x2 MFMA 16x16 blocks.  The MFMA is fed with op(B) as its
// first operand and op(A) as its second, i.e. it computes the transposed
// product; a lane then holds four n-columns of one m-row, and the 16 lanes of
// a row group store 16 consecutive rows of one column of the column-major C
// (coalesced).
constexpr int GBM = 64, GBN = 64;

template <int MODE>
struct GemmCfg;
template <>
struct GemmCfg<CMP_F64> {
    typedef double T;
    static constexpr int BK = 16;
    typedef v4d Acc;
};
template <>
struct GemmCfg<CMP_F32> {
    typedef float T;
    static constexpr int BK = 16;
    typedef v4f Acc;
};
template <>
struct GemmCfg<CMP_BF16X3> {
    typedef float T;
    static constexpr int BK = 32;
    typedef v4f Acc;
};

__device__ inline void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

template <typename TA, typename TC, int MODE>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmProb *__restrict__ probs,
                                                   const GemmTile *__restrict__ tiles) {
    typedef typename GemmCfg<MODE>::T T;
    typedef typename GemmCfg<MODE>::Acc Acc;
    constexpr int BK = GemmCfg<MODE>::BK;
    __shared__ T As[BK][GBM + 1];
    __shared__ T Bs[BK][GBN + 1];

    const GemmTile tl = tiles[blockIdx.x];
    const GemmProb p = probs[tl.prob];
    const TA *__restrict__ A = (const TA *)p.A;
    const TA *__restrict__ B = (const TA *)p.B;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = tl.m0, n0 = tl.n0;
    const int M = p.M, N = p.N, K = p.K;

    Acc acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = Acc{0, 0, 0, 0};

    for (int k0 = 0; k0 < K; k0 += BK) {
        // stage op(A)(m0.., k0..) into As[k][m] and op(B)(k0.., n0..) into Bs[k][n]
#pragma unroll
        for (int e = tid; e < GBM * BK; e += 256) {
            int i, k;
            if (p.opA == 0) {
                i = e % GBM;
                k = e / GBM;
            } else {
                k = e % BK;
                i = e / BK;
            }
            const int gi = m0 + i, gk = k0 + k;
            T v = 0;
            if (gi < M && gk < K)
                v = (T)(p.opA == 0 ? A[gi + (int64_t)gk * p.lda] : A[gk + (int64_t)gi * p.lda]);
            As[k][i] = v;
        }
#pragma unroll
        for (int e = tid; e < GBN * BK; e += 256) {
            int jn, k;
            if (p.opB == 0) {
                k = e % BK;
                jn = e / BK;
            } else {
                jn = e % GBN;
                k = e / GBN;
            }
            const int gj = n0 + jn, gk = k0 + k;
            T v = 0;
            if (gj < N && gk < K)
                v = (T)(p.opB == 0 ? B[gk + (int64_t)gj * p.ldb] : B[gj + (int64_t)gk * p.ldb]);
            Bs[k][jn] = v;
        }
        __syncthreads();
        if constexpr (MODE == CMP_F64 || MODE == CMP_F32) {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                const int kr = kk + (lane >> 4);
                T av[2], bv[2];
#pragma unroll
                for (int t = 0; t < 2; t++) {
                    av[t] = As[kr][wm * 32 + t * 16 + (lane & 15)];
                    bv[t] = Bs[kr][wn * 32 + t * 16 + (lane & 15)];
                }
#pragma unroll
                for (int si = 0; si < 2; si++)
#pragma unroll
                    for (int sj = 0; sj < 2; sj++) {
                        if constexpr (MODE == CMP_F64)
                            acc[si][sj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[sj], av[si], acc[si][sj], 0, 0, 0);
                        else
                            acc[si][sj] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[sj], av[si], acc[si][sj], 0, 0, 0);
                    }
            }
        } else {
            // two-term bfloat16 split: x = hi + lo; products hi*hi + hi*lo + lo*hi
            const int kb = 8 * (lane >> 4);
            v8bf ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int t = 0; t < 2; t++) {
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    __bf16 h, l;
                    split_bf16(As[kb + e][wm * 32 + t * 16 + (lane & 15)], h, l);
                    ah[t][e] = h;
                    al[t][e] = l;
                    split_bf16(Bs[kb + e][wn * 32 + t * 16 + (lane & 15)], h, l);
                    bh[t][e] = h;
                    bl[t][e] = l;
                }
            }
#pragma unroll
            for (int si = 0; si < 2; si++)
#pragma unroll
                for (int sj = 0; sj < 2; sj++) {
                    acc[si][sj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[sj], ah[si], acc[si][sj], 0, 0, 0);
                    acc[si][sj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[sj], al[si], acc[si][sj], 0, 0, 0);
                    acc[si][sj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[sj], ah[si], acc[si][sj], 0, 0, 0);
                }
        }
        __syncthreads();
    }

    TC *__restrict__ C = (TC *)p.C;
    const TC *__restrict__ Cin = (const TC *)p.Cin;
#pragma unroll
    for (int si = 0; si < 2; si++)
#pragma unroll
        for (int sj = 0; sj < 2; sj++) {
            const int gm = m0 + wm * 32 + si * 16 + (lane & 15);
            if (gm >= M) continue;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                // result rows held by this lane: v_mfma_f64_16x16x4 interleaves the
                // four row groups (row = lane/16 + 4v); the f32 and bf16 forms keep
                // them contiguous (row = 4 (lane/16) + v)
                const int nr = (MODE == CMP_F64) ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
                const int gn = n0 + wn * 32 + sj * 16 + nr;
                if (gn >= N) continue;
                double r = p.alpha * (double)acc[si][sj][v];
                if (Cin) r += p.beta * (double)Cin[gm + (int64_t)gn * p.ldcin];
                C[gm + (int64_t)gn * p.ldc] = (TC)r;
            }
        }
}

// ---------------------------------------------------------------------------
// gather
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(const MatDev *__restrict__ mats,
                                                     const GatherTile *__restrict__ tiles) {
    const GatherTile tl = tiles[blockIdx.x];
    const MatDev M = mats[tl.mat];
    const SnRec sk = M.sn[tl.K];
    __shared__ T tileS[64][65];  // [b][a]
    __shared__ int32_t rowR[64], rowI[64], colJ[64];
    __shared__ int64_t rowUp[64], rowUoff[64], colDiag[64], colLow[64], colLoff[64];
    const int tid = threadIdx.x;
    const int na = min(64, sk.cl - tl.a0), nb = min(64, sk.cu - tl.b0);
    if (tid < 64) {
        if (tid < na) {
            const int64_t a = sk.rl_off + tl.a0 + tid;
            const int32_t r = M.rl[a];
            const int32_t I = M.supof[r];
            const SnRec si = M.sn[I];
            rowR[tid] = r;
            rowI[tid] = I;
            rowUp[tid] = si.off_u + (int64_t)(r - si.f) * si.cu;
            rowUoff[tid] = M.u_rowoff[a] + tl.b0;
        }
    } else if (tid < 128) {
        const int t = tid - 64;
        if (t < nb) {
            const int64_t b = sk.ru_off + tl.b0 + t;
            const int32_t c = M.ru[b];
            const int32_t J = M.supof[c];
            const SnRec sj = M.sn[J];
            colJ[t] = J;
            colDiag[t] = sj.off_d + (int64_t)(c - sj.f) * sj.s - sj.f;
            colLow[t] = sj.off_l + (int64_t)(c - sj.f) * sj.cl;
            colLoff[t] = M.l_coloff[b] + tl.a0;
        }
    }
    __syncthreads();
    const T *ZL = (const T *)M.ZL;
    const T *ZU = (const T *)M.ZU;
    // diagonal and L-side sources: contiguous along the rows of G
    for (int e = tid; e < 64 * 64; e += 256) {
        const int ia = e & 63, ib = e >> 6;
        if (ia < na && ib < nb) {
            const int32_t I = rowI[ia], J = colJ[ib];
            if (I == J)
                tileS[ib][ia] = (T)M.Zd[colDiag[ib] + rowR[ia]];
            else if (I > J)
                tileS[ib][ia] = ZL[colLow[ib] + M.mapL[colLoff[ib] + ia]];
        }
    }
    // U-side sources: contiguous along the columns of G
    for (int e = tid; e < 64 * 64; e += 256) {
        const int ib = e & 63, ia = e >> 6;
        if (ia < na && ib < nb && rowI[ia] < colJ[ib]) tileS[ib][ia] = ZU[rowUp[ia] + M.mapU[rowUoff[ia] + ib]];
    }
    __syncthreads();
    T *G = (T *)M.G + sk.g_off;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int ia = e & 63, ib = e >> 6;
        if (ia < na && ib < nb) G[(tl.a0 + ia) + (int64_t)(tl.b0 + ib) * sk.cl] = tileS[ib][ia];
    }
}

// ---------------------------------------------------------------------------
// extraction
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void extract_kernel(ExtractArgs a) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= a.nnz) return;
    const int64_t loc = a.loc[p];
    const int64_t kind = loc >> 60, off = loc & ((int64_t(1) << 60) - 1);
    double v;
    if (kind == 0)
        v = a.Zd[off];
    else if (kind == 1)
        v = (double)((const T *)a.ZL)[off];
    else
        v = (double)((const T *)a.ZU)[off];
    a.out[p] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_tri_inv(const TriItem *items, int count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(tri_inv_kernel, dim3(count), dim3(256), 0, st, items);
    return hipGetLastError();
}

hipError_t launch_gemm(int in_f64, int out_f64, int mode, const GemmProb *probs, const GemmTile *tiles,
                       int ntiles, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    dim3 g(ntiles), b(256);
    if (mode == CMP_F64) {
        if (!in_f64) return hipErrorInvalidValue;
        if (out_f64)
            hipLaunchKernelGGL((gemm_kernel<double, double, CMP_F64>), g, b, 0, st, probs, tiles);
        else
            hipLaunchKernelGGL((gemm_kernel<double, float, CMP_F64>), g, b, 0, st, probs, tiles);
    } else if (mode == CMP_F32) {
        if (in_f64) return hipErrorInvalidValue;
        if (out_f64)
            hipLaunchKernelGGL((gemm_kernel<float, double, CMP_F32>), g, b, 0, st, probs, tiles);
        else
            hipLaunchKernelGGL((gemm_kernel<float, float, CMP_F32>), g, b, 0, st, probs, tiles);
    } else {
        if (in_f64) return hipErrorInvalidValue;
        if (out_f64)
            hipLaunchKernelGGL((gemm_kernel<float, double, CMP_BF16X3>), g, b, 0, st, probs, tiles);
        else
            hipLaunchKernelGGL((gemm_kernel<float, float, CMP_BF16X3>), g, b, 0, st, probs, tiles);
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
