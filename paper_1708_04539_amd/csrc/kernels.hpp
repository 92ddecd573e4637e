// kernels.hpp -- host-callable launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device_types.hpp"

namespace selinv {

// widest diagonal block the triangular-inversion kernel handles
constexpr int TRI_MAX_S = 1024;

hipError_t launch_tri_inv(const TriItem *items, int count, hipStream_t st);
// in_f64: operands in FP64 (else FP32); out_f64: C / Cin in FP64 (else FP32)
hipError_t launch_gemm(int in_f64, int out_f64, int mode, const GemmProb *probs, const GemmTile *tiles,
                       int ntiles, hipStream_t st);
hipError_t launch_gather(int f64, const MatDev *mats, const GatherTile *tiles, int ntiles, hipStream_t st);
hipError_t launch_extract(int f64, const ExtractArgs &a, hipStream_t st);

}  // namespace selinv
