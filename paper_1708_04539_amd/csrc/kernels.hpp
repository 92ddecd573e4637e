// kernels.hpp -- host-callable launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device_types.hpp"

namespace selinv {

// widest diagonal block (supernode) the library accepts
constexpr int TRI_MAX_S = 1024;

// diagonal 64x64 sub-blocks of the triangular inverses, one item per sub-block
// (TriItem.j0 = first row/column of the sub-block); nb = 1 or 2: 16- or
// 32-wide blocks, for fused items of at most that many columns only
// max_groups > 0: at most that many workgroups, each looping over items
hipError_t launch_tri_base(const TriItem *items, int count, int nb, hipStream_t st, int max_groups = 0);
// output tile of the grouped GEMM
enum : int { GEMM_TILE_32 = 32, GEMM_TILE_64 = 64, GEMM_TILE_128 = 128 };

// launch sites of the grouped GEMM (each is its own kernel symbol in profiles)
enum : int {
    GEMM_PRO_F64 = 0,     // FP64 -> FP64 (triangular rounds, normalisation, diag init)
    GEMM_PRO_F32OUT = 1,  // FP64 -> FP32 in FP64 arithmetic
    GEMM_PRO_MIXED = 4,   // FP64 operands -> FP32, in the mode's arithmetic (normalisation of the mixed forms)
    GEMM_STEP35 = 2,      // steps 3 and 5, operands/results in the storage precision
    GEMM_STEP4 = 3        // step 4, accumulated into the FP64 diagonal block
};

// mode: arithmetic for GEMM_STEP35 / GEMM_STEP4 (CMP_*); tile: GEMM_TILE_32,
// GEMM_TILE_64 or GEMM_TILE_128 (the tile list must use the same size)
hipError_t launch_gemm(int role, int mode, int tile, const GemmProb *probs, const GemmTile *tiles, int ntiles,
                       hipStream_t st);
hipError_t launch_gather(int f64, const MatDev *mats, const GatherTile *tiles, int ntiles, hipStream_t st);
// steps 3 and 5 with G_K read from its sources through the codes of
// mats[p.gmat].gcA (every problem has gcode >= 0 and opB = 0), results in the
// storage precision of the mode (gemm.hip)
hipError_t launch_gemm_g35(int mode, int tile, const GemmProb *probs, const GemmTile *tiles, int ntiles,
                           const MatDev *mats, hipStream_t st);
// step-4 product tiles of one level (pushing into the children's G) and the
// next level's gather tiles in one launch (gemm.hip)
hipError_t launch_step4_gather(int mode, int tile, const GemmProb *probs, const GemmTile *tiles, int ntiles,
                               const MatDev *mats, const GatherTile *gtiles, int ngtiles, hipStream_t st);
// gather + steps 3/5 + step 4 of small supernodes, one workgroup each (persist.hip)
hipError_t launch_small(int mode, const MatDev *mats, const GemmProb *probs, const SmallItem *items, int count,
                        hipStream_t st);
hipError_t launch_extract(int f64, const ExtractArgs &a, hipStream_t st);
// C += sum of the split-K partial products, for `count` items (count <= 65535),
// pushing the results into the children's G where an item asks for it
hipError_t launch_splitk_reduce(const ReduceItem *items, int count, int64_t max_mn, const MatDev *mats,
                                hipStream_t st);

// device LU (lu_device.hip): entries of A into the block storage (emb:
// complex source map or null); LU of 64x64 diagonal tiles (a zero or
// non-finite pivot lowers *bad to its permuted column); the Schur complement
// updates W_K (tiles: K, a0, b0, cl, cu, g_off into W) added to the
// ancestors' blocks of `mat`
hipError_t launch_scatter_values(const int64_t *loc, const double *vals, const int64_t *emb, int64_t nnz,
                                 double *diag, double *lpan, double *upan, hipStream_t st);
hipError_t launch_lu_tiles(const LuTile *items, int count, int32_t *bad, hipStream_t st);
hipError_t launch_scatter_update(const MatDev *mat, const GatherTile *tiles, int count, const double *W,
                                 double *diag, double *lpan, double *upan, hipStream_t st);

// persistent sweep (64x64 product tiles): resets the ncnt counters, the queue
// head and the error flag, then runs the task queue on `grid` workgroups
hipError_t launch_persist(int mode, const PersistArgs &a, int64_t ncnt, int grid, hipStream_t st);
// workgroups of the persistent sweep that fit on the device at once
int persist_grid(int mode);

}  // namespace selinv
