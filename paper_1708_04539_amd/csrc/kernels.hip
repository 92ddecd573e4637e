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

namespace selinv {


// ---------------------------------------------------------------------------
// triangular inversion, diagonal 64x64 blocks
// ---------------------------------------------------------------------------
// One wavefront handles the 64x64 diagonal sub-block that starts at
// row/column o of one supernode's packed L_KK \ U_KK (column-major, s x s);
// ragged sub-blocks (s - o < 64) are padded with the identity.
//   UPPER = false: column l of (L_oo)^{-1} (forward substitution, unit
//                  diagonal);
//   UPPER = true:  column l of (U_oo^T)^{-1} = row l of (U_oo)^{-1} (forward
//                  substitution on the transpose, dividing by the diagonal),
//                  so that the stores of a row are coalesced across lanes.
// Lane l keeps its 64 entries in registers; the substitution is fully
// unrolled and every factor entry it uses is the same for all lanes (an LDS
// broadcast).  The kernel also writes the zeros of L^{-1} above the sub-block
// and of U^{-1} left of it; the off-diagonal blocks come from the GEMM rounds
// of the recursive doubling (X21 = -B^{-1} C A^{-1} for L,
// X12 = -A^{-1} C B^{-1} for U).
template <bool UPPER>
__global__ __launch_bounds__(64) void tri_base_kernel(const TriItem *__restrict__ items) {
    const TriItem it = items[blockIdx.x];
    const int l = threadIdx.x;
    const int s = it.s, o = it.j0;
    const int b = min(64, s - o);
    // Ds[c][r] = D(o + r, o + c); reused for the result after the substitution
    __shared__ double Ds[64][65];
    for (int c = 0; c < 64; c++)
        Ds[c][l] = (l < b && c < b) ? it.D[(int64_t)(o + l) + (int64_t)(o + c) * s] : (l == c ? 1.0 : 0.0);
    __syncthreads();
    double x[64];
#pragma unroll
    for (int r = 0; r < 64; r++) x[r] = (r == l) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < 64; k++) {
        if constexpr (UPPER) x[k] = x[k] / Ds[k][k];
        const double xk = x[k];
#pragma unroll
        for (int r = k + 1; r < 64; r++) x[r] -= (UPPER ? Ds[r][k] : Ds[k][r]) * xk;
    }
    // Through LDS to global memory: x goes to row l of the tile (all 64
    // entries, unconditionally), then each column of the result is written
    // with the lanes along its rows (coalesced).  Lane l's x is column l of
    // (L_oo)^{-1}, or row l of (U_oo)^{-1}.
    __syncthreads();
    double(&Xs)[64][65] = Ds;
#pragma unroll
    for (int r = 0; r < 64; r++) Xs[l][r] = x[r];
    __syncthreads();
    double *out = UPPER ? it.Uinv : it.Linv;
    for (int c = 0; c < b; c++) {
        double *col = out + (int64_t)(o + c) * s;
        if (l < b) col[o + l] = UPPER ? Xs[l][c] : Xs[c][l];
        // zeros of L^{-1} above the sub-block
        if (!UPPER)
            for (int r = l; r < o; r += 64) col[r] = 0.0;
    }
    // zeros of U^{-1} left of the sub-block (rows o .. o+b-1)
    if (UPPER && l < b)
        for (int c = 0; c < o; c++) out[(o + l) + (int64_t)c * s] = 0.0;
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
hipError_t launch_tri_base(const TriItem *items, int count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(tri_base_kernel<false>, dim3(count), dim3(64), 0, st, items);
    hipLaunchKernelGGL(tri_base_kernel<true>, dim3(count), dim3(64), 0, st, items);
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
