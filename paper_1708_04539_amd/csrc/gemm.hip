// gemm.hip -- grouped GEMM on gfx950 matrix cores for the dense supernode
// products of selected inversion (arXiv:1708.04539, Algorithm 1: the
// normalisation of step 2 and the products of steps 3, 4 and 5).
//
//   C = alpha * op(A) op(B) + beta * Cin       (column-major, op = N or T)
//
// One launch covers a list of output tiles drawn from many problems of
// different shapes (all supernodes of one level, of every matrix of a batch).
// Tile BM x BN (128x128, 64x64 or 32x32) per workgroup of 256 threads = 4
// wavefronts in a 2x2 arrangement, each wavefront owning a (BM/2)x(BN/2)
// block made of 16x16 MFMA tiles.  The k loop is software pipelined: the next k-chunk is
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
#include "tiles.hpp"

namespace selinv {

// ROLE only names the launch site in profiles (0: triangular inversion,
// normalisation and diagonal initialisation; 1: products of steps 3 and 5;
// 2: product of step 4); the code is the same.
// Workgroups are dispatched to the 8 XCDs round robin (workgroup b to XCD
// b mod 8), and each XCD has its own L2.  The tile list is ordered row-block
// major, so tiles that share a strip of op(A) are neighbours; the remap gives
// each XCD one contiguous range of the list, so that such tiles run on the
// same XCD at about the same time and share the strip in its L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    constexpr int X = 8;
    const int q = n / X, r = n % X, x = b % X, i = b / X;
    return x * q + min(x, r) + i;
}

// Occupancy: four workgroups per compute unit for the 32- and 64-wide tiles
// (their LDS allows four; at most 128 VGPRs, which the two chunks in flight
// of the FP64 64-wide tile would otherwise exceed), two for the 128-wide ones.
template <int MODE, int BM, int BN, typename TA, typename TC, int ROLE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BM == 128 ? 2 : 4))) void gemm_v2(const GemmProb *__restrict__ probs,
                                               const GemmTile *__restrict__ tiles) {
    __shared__ Smem<MODE, BM, BN> sm;
    const GemmTile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    // only the step-4 product accumulates into an input matrix
    gemm_tile<MODE, BM, BN, TA, TC, ROLE == 2>(probs[tl.prob], tl.m0, tl.n0, sm);
    if (tl.n1 > 0) {
        __syncthreads();  // LDS free for the second tile
        gemm_tile<MODE, BM, BN, TA, TC, ROLE == 2>(probs[tl.prob], tl.m0, tl.n1 - 1, sm);
    }
}

// Steps 3 and 5 of a level whose G_K are not stored: op(A) is read from the
// ancestors' blocks through the source codes (see gemm_tile_g35).
template <int MODE, int BM, int BN, typename TA>
__global__ __launch_bounds__(256) void gemm_g35(const GemmProb *__restrict__ probs,
                                                const GemmTile *__restrict__ tiles,
                                                const MatDev *__restrict__ mats) {
    __shared__ Smem<MODE, BM, BN> sm;
    const GemmTile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    gemm_tile_g35<MODE, BM, BN, TA>(probs[tl.prob], tl.m0, tl.n0, sm, mats);
}

template <int MODE, typename TA>
static void launch_g35_mode(int tile, const GemmProb *probs, const GemmTile *tiles, int ntiles, const MatDev *mats,
                            hipStream_t st) {
    if (tile == GEMM_TILE_128)
        hipLaunchKernelGGL((gemm_g35<MODE, 128, 128, TA>), dim3(ntiles), dim3(256), 0, st, probs, tiles, mats);
    else if (tile == GEMM_TILE_64)
        hipLaunchKernelGGL((gemm_g35<MODE, 64, 64, TA>), dim3(ntiles), dim3(256), 0, st, probs, tiles, mats);
    else
        hipLaunchKernelGGL((gemm_g35<MODE, 32, 32, TA>), dim3(ntiles), dim3(256), 0, st, probs, tiles, mats);
}

hipError_t launch_gemm_g35(int mode, int tile, const GemmProb *probs, const GemmTile *tiles, int ntiles,
                           const MatDev *mats, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (tile != GEMM_TILE_32 && tile != GEMM_TILE_64 && tile != GEMM_TILE_128) return hipErrorInvalidValue;
    if (mode == CMP_F64)
        launch_g35_mode<CMP_F64, double>(tile, probs, tiles, ntiles, mats, st);
    else if (mode == CMP_F32)
        launch_g35_mode<CMP_F32, float>(tile, probs, tiles, ntiles, mats, st);
    else if (mode == CMP_BF16X3)
        launch_g35_mode<CMP_BF16X3, float>(tile, probs, tiles, ntiles, mats, st);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int MODE, typename TA, typename TC, int ROLE>
static void launch_mode(int tile, const GemmProb *probs, const GemmTile *tiles, int ntiles, hipStream_t st) {
    if (tile == GEMM_TILE_128)
        hipLaunchKernelGGL((gemm_v2<MODE, 128, 128, TA, TC, ROLE>), dim3(ntiles), dim3(256), 0, st, probs, tiles);
    else if (tile == GEMM_TILE_64)
        hipLaunchKernelGGL((gemm_v2<MODE, 64, 64, TA, TC, ROLE>), dim3(ntiles), dim3(256), 0, st, probs, tiles);
    else
        hipLaunchKernelGGL((gemm_v2<MODE, 32, 32, TA, TC, ROLE>), dim3(ntiles), dim3(256), 0, st, probs, tiles);
}

// Step-4 products of one level (pushing A^{-T}(P,P) into the children's G)
// and, in the same launch, the gather tiles of the next level (which skip
// those entries): workgroups [0, ntiles) run product tiles, the rest gather
// tiles.  The two sets write disjoint entries of G.
template <int MODE, int BM, int BN, typename TA>
__global__ __launch_bounds__(256) void step4_gather(const GemmProb *__restrict__ probs,
                                                    const GemmTile *__restrict__ tiles, int ntiles,
                                                    const MatDev *__restrict__ mats,
                                                    const GatherTile *__restrict__ gtiles) {
    union Shared {
        Smem<MODE, BM, BN> g;
        GatherSmem<TA> t;
    };
    __shared__ Shared sm;
    const int b = blockIdx.x;
    if (b < ntiles) {
        const GemmTile tl = tiles[xcd_tile(b, ntiles)];
        gemm_tile<MODE, BM, BN, TA, double, true, true>(probs[tl.prob], tl.m0, tl.n0, sm.g, mats);
    } else {
        const GatherTile gt = gtiles[b - ntiles];
        gather_tile<TA>(mats[gt.mat], gt, sm.t);
    }
}

template <int MODE, typename TA>
static void launch_s4g(int tile, const GemmProb *probs, const GemmTile *tiles, int ntiles, const MatDev *mats,
                       const GatherTile *gtiles, int ngtiles, hipStream_t st) {
    const dim3 grid(ntiles + ngtiles);
    if (tile == GEMM_TILE_128)
        hipLaunchKernelGGL((step4_gather<MODE, 128, 128, TA>), grid, dim3(256), 0, st, probs, tiles, ntiles, mats,
                           gtiles);
    else if (tile == GEMM_TILE_64)
        hipLaunchKernelGGL((step4_gather<MODE, 64, 64, TA>), grid, dim3(256), 0, st, probs, tiles, ntiles, mats,
                           gtiles);
    else
        hipLaunchKernelGGL((step4_gather<MODE, 32, 32, TA>), grid, dim3(256), 0, st, probs, tiles, ntiles, mats,
                           gtiles);
}

hipError_t launch_step4_gather(int mode, int tile, const GemmProb *probs, const GemmTile *tiles, int ntiles,
                               const MatDev *mats, const GatherTile *gtiles, int ngtiles, hipStream_t st) {
    if (ntiles + ngtiles <= 0) return hipSuccess;
    if (tile != GEMM_TILE_32 && tile != GEMM_TILE_64 && tile != GEMM_TILE_128) return hipErrorInvalidValue;
    if (mode == CMP_F64)
        launch_s4g<CMP_F64, double>(tile, probs, tiles, ntiles, mats, gtiles, ngtiles, st);
    else if (mode == CMP_F32)
        launch_s4g<CMP_F32, float>(tile, probs, tiles, ntiles, mats, gtiles, ngtiles, st);
    else if (mode == CMP_BF16X3)
        launch_s4g<CMP_BF16X3, float>(tile, probs, tiles, ntiles, mats, gtiles, ngtiles, st);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_gemm(int role, int mode, int tile, const GemmProb *probs, const GemmTile *tiles, int ntiles,
                       hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (tile != GEMM_TILE_32 && tile != GEMM_TILE_64 && tile != GEMM_TILE_128) return hipErrorInvalidValue;
    switch (role) {
        case GEMM_PRO_F64:  // FP64 in and out
            launch_mode<CMP_F64, double, double, 0>(tile, probs, tiles, ntiles, st);
            break;
        case GEMM_PRO_MIXED:  // FP64 operands rounded when staged, FP32 or split-BF16 products, FP32 out
            if (mode == CMP_F32)
                launch_mode<CMP_F32, double, float, 0>(tile, probs, tiles, ntiles, st);
            else if (mode == CMP_BF16X3)
                launch_mode<CMP_BF16X3, double, float, 0>(tile, probs, tiles, ntiles, st);
            else
                return hipErrorInvalidValue;
            break;
        case GEMM_PRO_F32OUT:  // FP64 in, FP32 out, FP64 arithmetic
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
