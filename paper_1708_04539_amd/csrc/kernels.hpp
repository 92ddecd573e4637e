// kernels.hpp -- host-callable launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device_types.hpp"

namespace selinv {

// widest diagonal block (supernode) the library accepts
constexpr int TRI_MAX_S = 1024;

// diagonal 64x64 sub-blocks of the triangular inverses, one item per sub-block
// (TriItem.j0 = first row/column of the sub-block)
hipError_t launch_tri_base(const TriItem *items, int count, hipStream_t st);
// output tile of the grouped GEMM
enum : int { GEMM_TILE_64 = 64, GEMM_TILE_128 = 128 };

// in_f64: operands in FP64 (else FP32); out_f64: C / Cin in FP64 (else FP32);
// tile: GEMM_TILE_64 or GEMM_TILE_128 (the tile list must use the same size)
hipError_t launch_gemm(int in_f64, int out_f64, int mode, int tile, const GemmProb *probs,
                       const GemmTile *tiles, int ntiles, hipStream_t st);
hipError_t launch_gather(int f64, const MatDev *mats, const GatherTile *tiles, int ntiles, hipStream_t st);
hipError_t launch_extract(int f64, const ExtractArgs &a, hipStream_t st);

}  // namespace selinv
