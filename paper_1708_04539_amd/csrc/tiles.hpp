// tiles.hpp -- device building blocks shared by the per-level kernels and the
// persistent sweep: one output tile of the grouped MFMA GEMM and one tile of
// the gather.
#pragma once

#include <hip/hip_runtime.h>

#include "device_types.hpp"

namespace selinv {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int MODE>
struct Mode;
template <>
struct Mode<CMP_F64> {
    typedef double T;
    typedef v4d Acc;
    static constexpr int BK = 16;
};
template <>
struct Mode<CMP_F32> {
    typedef float T;
    typedef v4f Acc;
    static constexpr int BK = 16;
};
template <>
struct Mode<CMP_BF16X3> {
    typedef float T;
    typedef v4f Acc;
    static constexpr int BK = 32;
};

// LDS layouts.  F64/F32: [k][m] (m contiguous: the 16 lanes of a row group
// read 16 consecutive m of one k).  BF16X3: [m][k] (k contiguous: a lane reads
// its 8 consecutive k of one m with one 16-byte load).
template <int MODE, int BM, int BN, int BK = Mode<MODE>::BK>
struct Smem {
    typedef typename Mode<MODE>::T T;
    T a[2][BK][BM + 2];
    T b[2][BK][BN + 2];
};
template <int BM, int BN, int BK>
struct Smem<CMP_BF16X3, BM, BN, BK> {
    static constexpr int P = BK + 8;
    __bf16 ah[2][BM][P], al[2][BM][P];
    __bf16 bh[2][BN][P], bl[2][BN][P];
};

// One BM x BN output tile of C = alpha op(A) op(B) + beta Cin, computed by
// the 256 threads of the calling workgroup (see gemm.hip for the design).
template <int MODE, int BM, int BN, typename TA, typename TC, int BK = Mode<MODE>::BK>
__device__ __forceinline__ void gemm_tile(const GemmProb &p, const int m0, const int n0,
                                          Smem<MODE, BM, BN, BK> &sm) {
    typedef typename Mode<MODE>::T T;
    typedef typename Mode<MODE>::Acc Acc;
    static_assert(MODE != CMP_BF16X3 || BK % 32 == 0, "split-BF16 chunks are multiples of 32");
    constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
    constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
    const TA *__restrict__ A = (const TA *)p.A;
    const TA *__restrict__ B = (const TA *)p.B;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int M = p.M, N = p.N, K = p.K;
    const int opA = p.opA, opB = p.opB;
    const int64_t lda = p.lda, ldb = p.ldb;

    Acc acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++) acc[i][j] = Acc{0, 0, 0, 0};

    T ra[LA], rb[LB];
    // element t of this thread's share of a chunk: (row in tile, k in chunk)
    auto a_idx = [&](int t, int &i, int &k) {
        const int e = tid + 256 * t;
        if (opA == 0) {
            i = e % BM;
            k = e / BM;
        } else {
            k = e % BK;
            i = e / BK;
        }
    };
    auto b_idx = [&](int t, int &j, int &k) {
        const int e = tid + 256 * t;
        if (opB == 0) {
            k = e % BK;
            j = e / BK;
        } else {
            j = e % BN;
            k = e / BN;
        }
    };
    auto gload = [&](int k0) {
#pragma unroll
        for (int t = 0; t < LA; t++) {
            int i, k;
            a_idx(t, i, k);
            const int gi = m0 + i, gk = k0 + k;
            T v = 0;
            if (gi < M && gk < K) v = (T)(opA == 0 ? A[gi + gk * lda] : A[gk + gi * lda]);
            ra[t] = v;
        }
#pragma unroll
        for (int t = 0; t < LB; t++) {
            int j, k;
            b_idx(t, j, k);
            const int gj = n0 + j, gk = k0 + k;
            T v = 0;
            if (gj < N && gk < K) v = (T)(opB == 0 ? B[gk + gj * ldb] : B[gj + gk * ldb]);
            rb[t] = v;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int t = 0; t < LA; t++) {
            int i, k;
            a_idx(t, i, k);
            if constexpr (MODE == CMP_BF16X3) {
                const __bf16 h = (__bf16)ra[t];
                sm.ah[buf][i][k] = h;
                sm.al[buf][i][k] = (__bf16)(ra[t] - (float)h);
            } else {
                sm.a[buf][k][i] = ra[t];
            }
        }
#pragma unroll
        for (int t = 0; t < LB; t++) {
            int j, k;
            b_idx(t, j, k);
            if constexpr (MODE == CMP_BF16X3) {
                const __bf16 h = (__bf16)rb[t];
                sm.bh[buf][j][k] = h;
                sm.bl[buf][j][k] = (__bf16)(rb[t] - (float)h);
            } else {
                sm.b[buf][k][j] = rb[t];
            }
        }
    };
    auto compute = [&](int buf) {
        if constexpr (MODE == CMP_BF16X3) {
#pragma unroll
            for (int kq = 0; kq < BK; kq += 32) {
                const int kb = kq + 8 * (lane >> 4);
                v8bf ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
                for (int i = 0; i < TM; i++) {
                    const int r = wm * WM + i * 16 + (lane & 15);
                    ah[i] = *(const v8bf *)&sm.ah[buf][r][kb];
                    al[i] = *(const v8bf *)&sm.al[buf][r][kb];
                }
#pragma unroll
                for (int j = 0; j < TN; j++) {
                    const int c = wn * WN + j * 16 + (lane & 15);
                    bh[j] = *(const v8bf *)&sm.bh[buf][c][kb];
                    bl[j] = *(const v8bf *)&sm.bl[buf][c][kb];
                }
#pragma unroll
                for (int i = 0; i < TM; i++)
#pragma unroll
                    for (int j = 0; j < TN; j++) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[j], ah[i], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], al[i], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], ah[i], acc[i][j], 0, 0, 0);
                    }
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                const int kr = kk + (lane >> 4);
                T av[TM], bv[TN];
#pragma unroll
                for (int i = 0; i < TM; i++) av[i] = sm.a[buf][kr][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < TN; j++) bv[j] = sm.b[buf][kr][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < TM; i++)
#pragma unroll
                    for (int j = 0; j < TN; j++) {
                        if constexpr (MODE == CMP_F64)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[j], av[i], acc[i][j], 0, 0, 0);
                        else
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[j], av[i], acc[i][j], 0, 0, 0);
                    }
            }
        }
    };

    gload(0);
    sstore(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += BK) {
        const bool more = k0 + BK < K;
        if (more) gload(k0 + BK);
        compute(buf);
        if (more) sstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    TC *__restrict__ C = (TC *)p.C;
    const TC *__restrict__ Cin = (const TC *)p.Cin;
    const int64_t ldc = p.ldc, ldcin = p.ldcin;
    const double alpha = p.alpha, beta = p.beta;
#pragma unroll
    for (int i = 0; i < TM; i++)
#pragma unroll
        for (int j = 0; j < TN; j++) {
            const int gm = m0 + wm * WM + i * 16 + (lane & 15);
            if (gm >= M) continue;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                // rows of the 16x16 result held by this lane: v_mfma_f64_16x16x4
                // interleaves the four row groups (row = lane/16 + 4v); the f32
                // and bf16 forms keep them contiguous (row = 4 (lane/16) + v)
                const int nr = (MODE == CMP_F64) ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
                const int gn = n0 + wn * WN + j * 16 + nr;
                if (gn >= N) continue;
                double r = alpha * (double)acc[i][j][v];
                if (Cin) r += beta * (double)Cin[gm + gn * ldcin];
                C[gm + gn * ldc] = (TC)r;
            }
        }
}

// LDS of one gather tile
template <typename T>
struct GatherSmem {
    T tileS[64][65];  // [b][a]
    int32_t rowR[64], rowI[64], colJ[64];
    int64_t rowUp[64], rowUoff[64], colDiag[64], colLow[64], colLoff[64];
};

// One 64x64 tile (rows a0.., columns b0..) of G_K = A^{-T}(R_L(K), R_U(K)),
// gathered by the 256 threads of the calling workgroup (see kernels.hip).
template <typename T>
__device__ __forceinline__ void gather_tile(const MatDev &M, const int K, const int a0, const int b0,
                                            GatherSmem<T> &sm) {
    const SnRec sk = M.sn[K];
    T(&tileS)[64][65] = sm.tileS;
    int32_t *rowR = sm.rowR, *rowI = sm.rowI, *colJ = sm.colJ;
    int64_t *rowUp = sm.rowUp, *rowUoff = sm.rowUoff, *colDiag = sm.colDiag, *colLow = sm.colLow,
            *colLoff = sm.colLoff;
    const int tid = threadIdx.x;
    const int na = min(64, sk.cl - a0), nb = min(64, sk.cu - b0);
    if (tid < 64) {
        if (tid < na) {
            const int64_t a = sk.rl_off + a0 + tid;
            const int32_t r = M.rl[a];
            const int32_t I = M.supof[r];
            const SnRec si = M.sn[I];
            rowR[tid] = r;
            rowI[tid] = I;
            rowUp[tid] = si.off_u + (int64_t)(r - si.f) * si.cu;
            rowUoff[tid] = M.u_rowoff[a] + b0;
        }
    } else if (tid < 128) {
        const int t = tid - 64;
        if (t < nb) {
            const int64_t b = sk.ru_off + b0 + t;
            const int32_t c = M.ru[b];
            const int32_t J = M.supof[c];
            const SnRec sj = M.sn[J];
            colJ[t] = J;
            colDiag[t] = sj.off_d + (int64_t)(c - sj.f) * sj.s - sj.f;
            colLow[t] = sj.off_l + (int64_t)(c - sj.f) * sj.cl;
            colLoff[t] = M.l_coloff[b] + a0;
        }
    }
    __syncthreads();
    const T *ZL = (const T *)M.ZL;
    const T *ZU = (const T *)M.ZU;
    // Each thread owns 16 entries of the tile.  Loads are batched: first every
    // relative index, then every source value, so that a thread waits for two
    // memory round trips rather than two per entry.
    constexpr int PER = 64 * 64 / 256;
    {
        // diagonal and L-side sources, threads along the rows of G (contiguous)
        int kind[PER];
        int32_t mi[PER];
        T val[PER];
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ia = e & 63, ib = e >> 6;
            kind[t] = 0;
            if (ia < na && ib < nb) {
                const int32_t I = rowI[ia], J = colJ[ib];
                kind[t] = I == J ? 1 : (I > J ? 2 : 0);
            }
        }
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ia = e & 63, ib = e >> 6;
            mi[t] = kind[t] == 2 ? M.mapL[colLoff[ib] + ia] : 0;
        }
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ia = e & 63, ib = e >> 6;
            val[t] = kind[t] == 1 ? (T)M.Zd[colDiag[ib] + rowR[ia]] : kind[t] == 2 ? ZL[colLow[ib] + mi[t]] : (T)0;
        }
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ia = e & 63, ib = e >> 6;
            if (kind[t]) tileS[ib][ia] = val[t];
        }
    }
    {
        // U-side sources, threads along the columns of G (contiguous in ZU)
        bool up[PER];
        int32_t mi[PER];
        T val[PER];
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ib = e & 63, ia = e >> 6;
            up[t] = ia < na && ib < nb && rowI[ia] < colJ[ib];
        }
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ib = e & 63, ia = e >> 6;
            mi[t] = up[t] ? M.mapU[rowUoff[ia] + ib] : 0;
        }
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ia = e >> 6;
            val[t] = up[t] ? ZU[rowUp[ia] + mi[t]] : (T)0;
        }
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ib = e & 63, ia = e >> 6;
            if (up[t]) tileS[ib][ia] = val[t];
        }
    }
    __syncthreads();
    T *G = (T *)M.G + sk.g_off;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int ia = e & 63, ib = e >> 6;
        if (ia < na && ib < nb) G[(a0 + ia) + (int64_t)(b0 + ib) * sk.cl] = tileS[ib][ia];
    }
}

}  // namespace selinv
