// gemm.hip -- grouped GEMM on gfx950 matrix cores for the dense supernode
// products of selected inversion (arXiv:1708.04539, Algorithm 1: the
// normalisation of step 2 and the products of steps 3, 4 and 5).
//
//   C = alpha * op(A) op(B) + beta * Cin       (column-major, op = N or T)
//
// One launch covers a list of output tiles drawn from many problems of
// different shapes (all supernodes of one level, of every matrix of a batch).
// Tile BM x BN (128x128 or 64x64) per workgroup of 256 threads = 4 wavefronts
// in a 2x2 arrangement, each wavefront owning a (BM/2)x(BN/2) block made of
// 16x16 MFMA tiles.  The k loop is software pipelined: the next k-chunk is
// loaded from global memory into registers while the current one is consumed
// from LDS, and LDS is double buffered (one barrier per chunk).
//
// Arithmetic modes
//   CMP_F64     v_mfma_f64_16x16x4, FP64 operands and accumulation.
//   CMP_F32     v_mfma_f32_16x16x4, FP32 operands and accumulation.
//   CMP_BF16X3  both operands split once, when staged into LDS, into
//               x = hi + lo with hi = bf16(x) and lo = bf16(x - hi); the
//               product is hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16
//               with FP32 accumulation (the lo*lo term is dropped).
// The MFMA is fed with op(B) as its first operand and op(A) as its second,
// i.e. it computes the transposed product, so that the 16 lanes of a row
// group hold 16 consecutive rows of one column of the column-major C and the
// stores are coalesced.
#include <hip/hip_runtime.h>

#include "device_types.hpp"
#include "kernels.hpp"

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
template <int MODE, int BM, int BN>
struct Smem {
    typedef typename Mode<MODE>::T T;
    static constexpr int BK = Mode<MODE>::BK;
    T a[2][BK][BM + 2];
    T b[2][BK][BN + 2];
};
template <int BM, int BN>
struct Smem<CMP_BF16X3, BM, BN> {
    static constexpr int BK = 32, P = BK + 8;
    __bf16 ah[2][BM][P], al[2][BM][P];
    __bf16 bh[2][BN][P], bl[2][BN][P];
};

// ROLE only names the launch site in profiles (0: triangular inversion,
// normalisation and diagonal initialisation; 1: products of steps 3 and 5;
// 2: product of step 4); the code is the same.
template <int MODE, int BM, int BN, typename TA, typename TC, int ROLE>
__global__ __launch_bounds__(256) void gemm_v2(const GemmProb *__restrict__ probs,
                                               const GemmTile *__restrict__ tiles) {
    typedef typename Mode<MODE>::T T;
    typedef typename Mode<MODE>::Acc Acc;
    constexpr int BK = Mode<MODE>::BK;
    constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
    constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
    __shared__ Smem<MODE, BM, BN> sm;

    const GemmTile tl = tiles[blockIdx.x];
    const GemmProb p = probs[tl.prob];
    const TA *__restrict__ A = (const TA *)p.A;
    const TA *__restrict__ B = (const TA *)p.B;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = tl.m0, n0 = tl.n0, M = p.M, N = p.N, K = p.K;
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
            const int kb = 8 * (lane >> 4);
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

template <int MODE, typename TA, typename TC, int ROLE>
static void launch_mode(int tile, const GemmProb *probs, const GemmTile *tiles, int ntiles, hipStream_t st) {
    if (tile == GEMM_TILE_128)
        hipLaunchKernelGGL((gemm_v2<MODE, 128, 128, TA, TC, ROLE>), dim3(ntiles), dim3(256), 0, st, probs, tiles);
    else
        hipLaunchKernelGGL((gemm_v2<MODE, 64, 64, TA, TC, ROLE>), dim3(ntiles), dim3(256), 0, st, probs, tiles);
}

hipError_t launch_gemm(int role, int mode, int tile, const GemmProb *probs, const GemmTile *tiles, int ntiles,
                       hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (tile != GEMM_TILE_64 && tile != GEMM_TILE_128) return hipErrorInvalidValue;
    switch (role) {
        case GEMM_PRO_F64:  // FP64 in and out
            launch_mode<CMP_F64, double, double, 0>(tile, probs, tiles, ntiles, st);
            break;
        case GEMM_PRO_F32OUT:  // FP64 in, FP32 out (normalised panels of the mixed forms)
            launch_mode<CMP_F64, double, float, 0>(tile, probs, tiles, ntiles, st);
            break;
        case GEMM_STEP35:  // operands and results in the run's storage precision
            if (mode == CMP_F64)
                launch_mode<CMP_F64, double, double, 1>(tile, probs, tiles, ntiles, st);
            else if (mode == CMP_F32)
                launch_mode<CMP_F32, float, float, 1>(tile, probs, tiles, ntiles, st);
            else if (mode == CMP_BF16X3)
                launch_mode<CMP_BF16X3, float, float, 1>(tile, probs, tiles, ntiles, st);
            else
                return hipErrorInvalidValue;
            break;
        case GEMM_STEP4:  // FP64 accumulation into the diagonal block
            if (mode == CMP_F64)
                launch_mode<CMP_F64, double, double, 2>(tile, probs, tiles, ntiles, st);
            else if (mode == CMP_F32)
                launch_mode<CMP_F32, float, double, 2>(tile, probs, tiles, ntiles, st);
            else if (mode == CMP_BF16X3)
                launch_mode<CMP_BF16X3, float, double, 2>(tile, probs, tiles, ntiles, st);
            else
                return hipErrorInvalidValue;
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace selinv
