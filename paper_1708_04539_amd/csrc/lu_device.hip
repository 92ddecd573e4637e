// lu_device.hip -- kernels of the supernodal LU without pivoting on the GPU:
// the factorisation At = L U (eq. LU) that Algorithm 1 of arXiv:1708.04539
// starts from, in the block storage the selected inversion reads (the s x s
// diagonal block holding L_KK \ U_KK, the c_L x s panel L(R_L, K) and the
// c_U x s panel U(K, R_U)^T of every supernode K).
//
// The host orchestration (runtime.hip) runs the levels of the supernodal
// dependency graph from the deepest up.  Per level, in 64-column steps j0 of
// every supernode's diagonal block:
//   lu_tile_kernel   LU of the 64 x 64 tile at (j0, j0), one wave;
//   tri_base_kernel  the inverses of the tile's unit L and of its U
//                    (kernels.hip);
//   grouped GEMM     the solves against the tile as products with those
//                    inverses, in place: the rows of D below the tile and of
//                    the L panel times U11^{-1}, L11^{-1} times the columns of
//                    D right of the tile, the rows of the U panel times
//                    L11^{-T};
//   grouped GEMM     the trailing updates of the block and the panels;
// then the Schur complement product W_K = -L(R_L, K) U(K, R_U) (grouped GEMM)
// and scatter_update_kernel, which adds W_K to the blocks of the ancestors.
#include <hip/hip_runtime.h>

#include <climits>

#include "device_types.hpp"
#include "kernels.hpp"
#include "tiles.hpp"

namespace selinv {

// vals[p] (emb == nullptr), or for complex handles the entry of the real form
// taken from the interleaved complex values: emb[p] = source << 1 | negate
__global__ __launch_bounds__(256) void scatter_values_kernel(const int64_t *__restrict__ loc,
                                                             const double *__restrict__ vals,
                                                             const int64_t *__restrict__ emb, int64_t nnz,
                                                             double *diag, double *lpan, double *upan) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    const int64_t l = gptr(loc)[p];
    const int64_t kind = l >> 60, off = l & ((int64_t(1) << 60) - 1);
    double v;
    if (emb) {
        const int64_t e = gptr(emb)[p];
        v = gptr(vals)[e >> 1];
        if (e & 1) v = -v;
    } else {
        v = gptr(vals)[p];
    }
    double *dst = kind == 0 ? diag : kind == 1 ? lpan : upan;
    gptr_w(dst)[off] = v;
}

// Right-looking elimination of the b x b tile (b = min(64, s - j0)) at
// (j0, j0) of the column-major s x s block D, one wave per tile: lane i holds
// row i of the tile in registers.  At step k lane k publishes its row (the
// pivot row U(k, k:)) in LDS; every lane below it scales its entry of column
// k by the pivot's reciprocal and takes the rank-one update of the rest of its
// row.  A zero or non-finite pivot lowers *bad to its permuted column
// f + j0 + k (the arithmetic goes on; the host reports the failure).
__global__ __launch_bounds__(64) void lu_tile_kernel(const LuTile *__restrict__ items, int32_t *bad) {
    __shared__ double urow[2][64];  // pivot rows of even / odd steps
    const LuTile it = items[blockIdx.x];
    const int i = threadIdx.x;
    const int s = it.s, j0 = it.j0, b = min(64, s - j0);
    SELINV_GLOBAL double *D = gptr_w(it.D) + j0 + (int64_t)j0 * s;
    double a[64];
#pragma unroll
    for (int c = 0; c < 64; c++) a[c] = (i < b && c < b) ? D[i + (int64_t)c * s] : (i == c ? 1.0 : 0.0);
#pragma unroll
    for (int k = 0; k < 64; k++) {
        if (k < b) {
            double *u = urow[k & 1];
            if (i == k) {
#pragma unroll
                for (int c = k; c < 64; c++) u[c] = a[c];
            }
            __syncthreads();
            const double p = u[k];
            if (i == 0 && !(p != 0.0 && isfinite(p))) atomicMin(bad, it.f + j0 + k);
            if (i > k) {
                double ur[64];  // the pivot row, all reads in flight before the update
#pragma unroll
                for (int c = k + 1; c < 64; c++) ur[c] = u[c];
                const double l = a[k] * (1.0 / p);
                a[k] = l;
#pragma unroll
                for (int c = k + 1; c < 64; c++) a[c] = fma(-l, ur[c], a[c]);
            }
        }
    }
    if (i < b) {
#pragma unroll
        for (int c = 0; c < 64; c++)
            if (c < b) D[i + (int64_t)c * s] = a[c];
    }
}

// One 64 x 64 tile of W_K (c_L x c_U column-major at W + g_off) per
// workgroup.  W_K(a, b) belongs to entry (R_L(K)[a], R_U(K)[b]) of At, which
// lies in the diagonal block of J (I = J), the L panel of J (I > J) or the U
// panel of I (I < J), I and J the supernodes of its row and column; the
// relative-index maps give its place there.  As in the gather of the
// selected inversion (the same positions, read there), the tile's row and
// column records go to LDS first; the tile itself is staged in LDS, then the
// diagonal and L-side entries are added with the threads along the rows
// (contiguous in the L panels) and the U-side entries along the columns
// (contiguous in the U panels).  Supernodes of one level update the same
// entries of their common ancestors, hence the atomic adds.
__global__ __launch_bounds__(256) void scatter_update_kernel(const MatDev *__restrict__ mat,
                                                             const GatherTile *__restrict__ tiles,
                                                             const double *__restrict__ W, double *diag,
                                                             double *lpan, double *upan) {
    __shared__ double tileS[64][65];  // [b][a]
    __shared__ int32_t rowR[64], rowI[64], colJ[64];
    __shared__ int64_t rowUp[64], rowUoff[64], colDiag[64], colLow[64], colLoff[64];
    const GatherTile gt = tiles[blockIdx.x];
    const MatDev &M = *mat;
    const SELINV_GLOBAL SnRec *sn = gptr(M.sn);
    const SELINV_GLOBAL int32_t *supof = gptr(M.supof);
    const int K = gt.K, a0 = gt.a0, b0 = gt.b0, cl = gt.cl, cu = gt.cu;
    const int64_t rl_off = sn[K].rl_off, ru_off = sn[K].ru_off;
    const int tid = threadIdx.x;
    const int na = min(64, cl - a0), nb = min(64, cu - b0);  // both >= 1
    if (tid < 64) {
        const int t = min(tid, na - 1);
        const int64_t a = rl_off + a0 + t;
        const int32_t r = gptr(M.rl)[a];
        const int64_t uo = gptr(M.u_rowoff)[a];
        const int32_t I = supof[r];
        if (tid < na) {
            rowR[tid] = r;
            rowI[tid] = I;
            rowUp[tid] = sn[I].off_u + (int64_t)(r - sn[I].f) * sn[I].cu;
            rowUoff[tid] = uo + b0;
        }
    } else if (tid < 128) {
        const int t = min(tid - 64, nb - 1);
        const int64_t bb = ru_off + b0 + t;
        const int32_t c = gptr(M.ru)[bb];
        const int64_t lo = gptr(M.l_coloff)[bb];
        const int32_t J = supof[c];
        if (tid - 64 < nb) {
            colJ[t] = J;
            colDiag[t] = sn[J].off_d + (int64_t)(c - sn[J].f) * sn[J].s - sn[J].f;
            colLow[t] = sn[J].off_l + (int64_t)(c - sn[J].f) * sn[J].cl;
            colLoff[t] = lo + a0;
        }
    }
    const SELINV_GLOBAL double *Wk = gptr(W) + gt.g_off;
    constexpr int PER = 64 * 64 / 256;
#pragma unroll
    for (int t = 0; t < PER; t++) {
        const int e = tid + 256 * t, ia = e & 63, ib = e >> 6;
        if (ia < na && ib < nb) tileS[ib][ia] = Wk[(a0 + ia) + (int64_t)(b0 + ib) * cl];
    }
    __syncthreads();
    const SELINV_GLOBAL int32_t *mapL = gptr(M.mapL);
    const SELINV_GLOBAL int32_t *mapU = gptr(M.mapU);
    {
        int kind[PER];  // 0 none, 1 diagonal block, 2 L panel
        int32_t mi[PER];
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
            mi[t] = mapL[kind[t] == 2 ? colLoff[ib] + ia : 0];
        }
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ia = e & 63, ib = e >> 6;
            if (kind[t] == 1)
                atomicAdd(diag + colDiag[ib] + rowR[ia], tileS[ib][ia]);
            else if (kind[t] == 2)
                atomicAdd(lpan + colLow[ib] + mi[t], tileS[ib][ia]);
        }
    }
    {
        bool up[PER];
        int32_t mi[PER];
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ib = e & 63, ia = e >> 6;
            up[t] = ia < na && ib < nb && rowI[ia] < colJ[ib];
        }
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ib = e & 63, ia = e >> 6;
            mi[t] = mapU[up[t] ? rowUoff[ia] + ib : 0];
        }
#pragma unroll
        for (int t = 0; t < PER; t++) {
            const int e = tid + 256 * t, ib = e & 63, ia = e >> 6;
            if (up[t]) atomicAdd(upan + rowUp[ia] + mi[t], tileS[ib][ia]);
        }
    }
}

hipError_t launch_scatter_values(const int64_t *loc, const double *vals, const int64_t *emb, int64_t nnz,
                                 double *diag, double *lpan, double *upan, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_values_kernel, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st, loc, vals, emb,
                       nnz, diag, lpan, upan);
    return hipGetLastError();
}

hipError_t launch_lu_tiles(const LuTile *items, int count, int32_t *bad, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(lu_tile_kernel, dim3(count), dim3(64), 0, st, items, bad);
    return hipGetLastError();
}

hipError_t launch_scatter_update(const MatDev *mat, const GatherTile *tiles, int count, const double *W,
                                 double *diag, double *lpan, double *upan, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_update_kernel, dim3(count), dim3(256), 0, st, mat, tiles, W, diag, lpan, upan);
    return hipGetLastError();
}

}  // namespace selinv
