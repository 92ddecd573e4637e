// lu_device.hip -- kernels of the supernodal LU without pivoting on the GPU:
// the factorisation At = L U (eq. LU) that Algorithm 1 of arXiv:1708.04539
// starts from, in the block storage the selected inversion reads (the s x s
// diagonal block holding L_KK \ U_KK, the c_L x s panel L(R_L, K) and the
// c_U x s panel U(K, R_U)^T of every supernode K).
//
// The host orchestration (runtime.hip) runs the levels of the supernodal
// dependency graph from the deepest up.  Per level, in 64-column steps j0 of
// every supernode's diagonal block:
//   lu_tile_kernel   LU of the 64 x 64 tile at (j0, j0), in LDS;
//   trsm_tile_kernel the rows of [D(j0+64:, j0 block); L panel] solved with
//                    the tile's U, and the rows of [D(j0 block, j0+64:)^T;
//                    U panel] with its unit L transposed (right solves);
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
// (j0, j0) of the column-major s x s block D: for every k the column below the
// pivot is scaled by the pivot's reciprocal, then the rest of the tile takes
// the rank-one update.  A zero or non-finite pivot lowers *bad to its permuted
// column f + j0 + k (the arithmetic goes on; the host reports the failure).
__global__ __launch_bounds__(256) void lu_tile_kernel(const LuTile *__restrict__ items, int32_t *bad) {
    __shared__ double T[64][65];  // T[c][r] = D(j0 + r, j0 + c)
    const LuTile it = items[blockIdx.x];
    const int tid = threadIdx.x;
    const int s = it.s, j0 = it.j0, b = min(64, s - j0);
    SELINV_GLOBAL double *D = gptr_w(it.D);
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        T[c][r] = (r < b && c < b) ? D[(int64_t)(j0 + r) + (int64_t)(j0 + c) * s] : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int k = 0; k < b; k++) {
        const double p = T[k][k];
        if (tid == 0 && !(p != 0.0 && isfinite(p))) atomicMin(bad, it.f + j0 + k);
        const double inv = 1.0 / p;
        if (tid > k && tid < b) T[k][tid] *= inv;
        __syncthreads();
        const int w = b - k - 1;  // trailing columns k+1 .. b-1, all 64 rows (rows <= k skipped)
        for (int e = tid; e < w * 64; e += 256) {
            const int r = e & 63, c = k + 1 + (e >> 6);
            if (r > k && r < b) T[c][r] -= T[k][r] * T[c][k];
        }
        __syncthreads();
    }
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (r < b && c < b) D[(int64_t)(j0 + r) + (int64_t)(j0 + c) * s] = T[c][r];
    }
}

// X T = B for the rows of one item: X(i, t) = X[i rs + t cs] (i < rows <= 64,
// t < b <= 64), overwritten in place; T(u, t) = T[u tu + t tt] upper
// triangular (u <= t), unit diagonal when `unit`.  Column t of X is final once
// the columns before it have been subtracted; then it is divided by T(t, t)
// and taken off the columns after it.
__global__ __launch_bounds__(256) void trsm_tile_kernel(const TrsmItem *__restrict__ items) {
    __shared__ double Ts[64][65];  // Ts[t][u] = T(u, t)
    __shared__ double Xs[64][65];  // Xs[t][i] = X(i, t)
    const TrsmItem it = items[blockIdx.x];
    const int tid = threadIdx.x, rows = it.rows, b = it.b;
    SELINV_GLOBAL double *X = gptr_w(it.X);
    const SELINV_GLOBAL double *Tg = gptr(it.T);
    const bool xrow = it.rs == 1, trow = it.tu == 1;  // which index is contiguous in memory
    for (int e = tid; e < 64 * 64; e += 256) {
        const int lo = e & 63, hi = e >> 6;
        const int i = xrow ? lo : hi, t = xrow ? hi : lo;
        Xs[t][i] = (i < rows && t < b) ? X[i * it.rs + t * it.cs] : 0.0;
        const int u = trow ? lo : hi, v = trow ? hi : lo;
        Ts[v][u] = (u < b && v < b && u <= v) ? (u == v && it.unit ? 1.0 : Tg[u * it.tu + v * it.tt]) : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < b; t++) {
        if (!it.unit && tid < 64) Xs[t][tid] = Xs[t][tid] / Ts[t][t];
        __syncthreads();
        const int w = b - t - 1;
        for (int e = tid; e < w * 64; e += 256) {
            const int i = e & 63, c = t + 1 + (e >> 6);
            Xs[c][i] -= Xs[t][i] * Ts[c][t];
        }
        __syncthreads();
    }
    for (int e = tid; e < 64 * 64; e += 256) {
        const int lo = e & 63, hi = e >> 6;
        const int i = xrow ? lo : hi, t = xrow ? hi : lo;
        if (i < rows && t < b) X[i * it.rs + t * it.cs] = Xs[t][i];
    }
}

// One 64 x 64 tile of W_K (c_L x c_U column-major at W + g_off) per
// workgroup.  W_K(a, b) belongs to entry (R_L(K)[a], R_U(K)[b]) of At, which
// lies in the diagonal block of J (I = J), the L panel of J (I > J) or the U
// panel of I (I < J), I and J the supernodes of its row and column; the
// relative-index maps give its place there.  Supernodes of one level update
// the same entries of their common ancestors, hence the atomic adds.
__global__ __launch_bounds__(256) void scatter_update_kernel(const MatDev *__restrict__ mat,
                                                             const GatherTile *__restrict__ tiles,
                                                             const double *__restrict__ W, double *diag,
                                                             double *lpan, double *upan) {
    const GatherTile gt = tiles[blockIdx.x];
    const MatDev &M = *mat;
    const SELINV_GLOBAL SnRec *sn = gptr(M.sn);
    const int64_t rl_off = sn[gt.K].rl_off, ru_off = sn[gt.K].ru_off;
    const int cl = gt.cl, cu = gt.cu;
    const SELINV_GLOBAL double *Wk = gptr(W) + gt.g_off;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int a = gt.a0 + (e & 63), b = gt.b0 + (e >> 6);
        if (a >= cl || b >= cu) continue;
        const int32_t r = gptr(M.rl)[rl_off + a], c = gptr(M.ru)[ru_off + b];
        const int32_t I = gptr(M.supof)[r], J = gptr(M.supof)[c];
        const double w = Wk[a + (int64_t)b * cl];
        double *dst;
        if (I == J) {
            const int32_t f = sn[J].f;
            dst = diag + sn[J].off_d + (int64_t)(c - f) * sn[J].s + (r - f);
        } else if (I > J) {
            const int64_t m = gptr(M.l_coloff)[ru_off + b] + a;
            dst = lpan + sn[J].off_l + (int64_t)(c - sn[J].f) * sn[J].cl + gptr(M.mapL)[m];
        } else {
            const int64_t m = gptr(M.u_rowoff)[rl_off + a] + b;
            dst = upan + sn[I].off_u + (int64_t)(r - sn[I].f) * sn[I].cu + gptr(M.mapU)[m];
        }
        atomicAdd(dst, w);
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
    hipLaunchKernelGGL(lu_tile_kernel, dim3(count), dim3(256), 0, st, items, bad);
    return hipGetLastError();
}

hipError_t launch_trsm_tiles(const TrsmItem *items, int count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(trsm_tile_kernel, dim3(count), dim3(256), 0, st, items);
    return hipGetLastError();
}

hipError_t launch_scatter_update(const MatDev *mat, const GatherTile *tiles, int count, const double *W,
                                 double *diag, double *lpan, double *upan, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_update_kernel, dim3(count), dim3(256), 0, st, mat, tiles, W, diag, lpan, upan);
    return hipGetLastError();
}

}  // namespace selinv
