// device_types.hpp -- records shared by the host runtime and the HIP kernels.
#pragma once

#include <cstdint>

namespace selinv {

// One supernode, as the kernels see it.  Offsets are in elements of the
// owning array (diag/Zd: off_d; lpan/ZL/Lh: off_l; upan/ZU/Uh: off_u).
struct SnRec {
    int32_t f, s, cl, cu;
    int64_t off_d, off_l, off_u;
    int64_t rl_off, ru_off;  // into rl / u_rowoff and ru / l_coloff
    int64_t g_off;           // G_K inside the gather workspace of its level
    int64_t c_off;           // source codes of G_K in gcL / gcU (-1: none, the maps serve)
};

// Source code of one entry of G_K: array << 30 | element offset, array 1 = Zd,
// 2 = ZL, 3 = ZU, 0 = none (the entry comes from the other code array).
constexpr uint32_t GCODE_SHIFT = 30;
constexpr uint32_t GCODE_MASK = (1u << GCODE_SHIFT) - 1;

// One matrix (handle) on the device; every pointer is a device address.
struct MatDev {
    const SnRec *sn;
    const int32_t *supof;
    const int32_t *rl, *ru;
    const int64_t *l_coloff, *u_rowoff;
    const int32_t *mapL, *mapU;
    const double *Zd;  // A^{-T} diagonal blocks (FP64 in every form)
    const void *ZL;    // A^{-T}(R_L, K) panels, FP64 or FP32
    const void *ZU;    // A^{-T}(K, R_U)^T panels, FP64 or FP32
    void *G;           // gather workspace, FP64 or FP32
    // children of every supernode (kids[kids_ptr[P] .. kids_ptr[P+1])), and
    // for a child K of P the positions of P's columns in R_L(K) and R_U(K):
    // push_pos[push_off[K] + r] = a with R_L(K)[a] = first(P) + r (or -1),
    // push_pos[push_off[K] + s_P + c] = b with R_U(K)[b] = first(P) + c (or -1)
    const int32_t *kids_ptr, *kids;
    const int64_t *push_off;
    const int32_t *push_pos;
    // precomputed source codes of the gather (supernodes with c_off >= 0):
    // gcL[c_off + a + b cl] for the diagonal-block and L-side entries,
    // gcU[c_off + b + a cu] for the U-side entries of G_K(a, b)
    const uint32_t *gcL, *gcU;
    // source codes of every entry of G_K in the layout of G_K itself (all
    // three arrays, gcA[ca_off(K) + a + b c_L]), read by the step-3/5 products
    // that take G_K from its sources instead of a stored G (GemmProb::gcode)
    const uint32_t *gcA;
    // where the rows and columns of every G_K come from, per entry of rl / ru
    // (index rl_off(K) + a, ru_off(K) + b).  Row r: its supernode I (row_I)
    // and the start of row r of U(I, R_U(I)) in ZU (row_up).  Column c: its
    // supernode J (col_J), the start of column c of the diagonal block of J
    // less first(J), so that col_diag + r addresses row r (col_diag), and the
    // start of column c of the L panel of J (col_low)
    const int32_t *row_I, *col_J;
    const int64_t *row_up, *col_diag, *col_low;
};

// gather: tile of G_K rows [a0, a0+64) x columns [b0, b0+64); entries from
// the diagonal block of supernode `skip` (the parent, when its step-4 product
// pushes them, see GemmProb) are left to that product; -1: none skipped.
// The supernode's sizes and offsets ride along, so that the tile starts its
// loads without reading the supernode record first.
struct GatherTile {
    int32_t mat, K, a0, b0;
    int32_t skip, cl, cu, pad;
    int64_t g_off, c_off;       // as in SnRec
    int64_t skip_lo, skip_hi;   // elements of Zd holding the skipped diagonal block
    int64_t rl_off, ru_off;     // as in SnRec
};

// C = alpha * op(A) op(B) + beta * Cin, column-major, op = N (0) or T (1)
struct GemmProb {
    const void *A;
    const void *B;
    void *C;
    const void *Cin;
    int32_t M, N, K;
    int32_t lda, ldb, ldc, ldcin;
    int32_t opA, opB;
    // step-4 product of supernode push_sn of matrix push_mat (-1: none): the
    // final entries of A^{-T}(P,P) are also written into G of P's children,
    // whose gather skips them
    int32_t push_sn, push_mat;
    // zero structure of the operands: bit 0 op(B)(k, n) = 0 for k < n, bit 1
    // op(A)(m, k) = 0 for k < m (products with the triangular inverses); a
    // tile then starts its k loop at the chunk holding max(n0, m0) (the
    // skipped chunks would add exact zeros)
    int32_t ktri;
    // cpx != 0: a product of a complex matrix in its real form whose result
    // is made of 2x2 blocks of one complex entry (rows 2i, 2i+1, columns 2j,
    // 2j+1), [[x, -y], [y, x]] or its transpose.  The problem lists only the
    // even columns (N halved, ldb, ldc and ldcin doubled); every stored entry
    // (m, 2j) also gives the entry (m ^ 1, 2j + 1), at ldc / 2 past it: the
    // same value for even m, its negative for odd m (in either orientation)
    int32_t cpx;
    // gcode >= 0: op(A) is G_K of matrix gmat, not read from A: its entry
    // (a, b) is the value that the code gcA[gcode + a + b lda] names (A is then
    // unused; a step-3 or step-5 product, op(B) = B)
    int32_t gmat;
    int64_t gcode;
    double alpha, beta;
};

// n1: 0, or 1 + the first column of a second output tile of the same rows
// that the workgroup forms after the first (gemm_v2; the normalisation pairs
// tiles of long and short triangular k ranges)
struct GemmTile {
    int32_t prob, m0, n0, n1;
};

// triangular inversion: one 64x64 diagonal sub-block of one supernode
struct TriItem {
    const double *D;  // packed L\U, s x s column-major
    double *Linv, *Uinv;
    int32_t s, j0;
    // a supernode with s, c_L, c_U <= 64 (lpan or upan non-null, j0 = 0):
    // the same workgroup forms Lhat = L(R_L,K) L_KK^{-1} (c_L x s),
    // Uhat = U(K,R_U)^T U_KK^{-T} (c_U x s) and A^{-T}(K,K) := L_KK^{-T}
    // U_KK^{-T} from the inverses in LDS; Linv / Uinv are then not stored
    const double *lpan, *upan;
    void *Lh, *Uh;  // FP64, or FP32 when f32out
    double *Zd;
    int32_t cl, cu, f32out, fused;
};

// fused step 3/4/5 of one small supernode (every product a single 64x64
// tile): problem indices of its step-3, step-5 and step-4 products (-1: none)
struct SmallItem {
    int32_t mat, K;
    int32_t pzu, pzl, pg4;
    int32_t s, cl, cu;
    int64_t g_off, c_off;
};

// split-K of a step-4 product: C(M x N, ld ldc) += sum of nparts partial
// products P[p * pstride + m + n M], added in order p = 0, 1, ...; with
// push_sn >= 0 the final entries also go into G of that supernode's children
// (as the push of an unsplit step-4 product, see GemmProb), G in FP32 when
// g_f32
struct ReduceItem {
    double *C;
    const double *P;
    int32_t M, N, ldc, nparts;
    int64_t pstride;
    int32_t push_sn, push_mat, g_f32;
    // cpx != 0: the parts hold the even columns of a complex block (N of
    // them); column n of the sum is column 2n of C, and column 2n + 1 follows
    // from it as for GemmProb::cpx
    int32_t cpx;
};

// device LU: one 64x64 diagonal tile (rows / columns j0 ..) of the s x s
// block D of the supernode whose first column is f
struct LuTile {
    double *D;
    int32_t s, j0, f, pad;
};

// extraction of the selected entries
struct ExtractArgs {
    const int64_t *loc;  // kind << 60 | offset per entry of A
    const double *Zd;
    const void *ZL, *ZU;
    double *out;
    int64_t nnz;
};

enum Compute : int { CMP_F64 = 0, CMP_F32 = 1, CMP_BF16X3 = 2 };

// persistent sweep: task kinds, per-supernode dependency record, arguments
enum : int32_t { PT_GATHER = 0, PT_STEP35 = 1, PT_STEP4 = 2 };

struct PTask {
    int32_t type;   // PT_*
    int32_t gid;    // supernode id over all matrices of the sweep
    int32_t mat, K; // matrix and local supernode (gather tiles)
    int32_t i0, i1; // gather: a0, b0; products: m0, n0
    int32_t prob;   // product problem index
    int32_t is_zu;  // the tile belongs to the step-3 product (A^{-T}(K, R_U))
};

struct PSn {
    // supernodes whose results the gather of this one reads (gids):
    // deps[dep_off .. dep_off + ndep) of PersistArgs
    int32_t dep_off, ndep;
    int32_t n_gather;  // gather tiles of this supernode
    int32_t n_zu;      // tiles of its step-3 product
    int32_t n_all;     // tiles of its step-3, step-5 and step-4 products
};

struct PersistArgs {
    const PTask *tasks;
    int32_t ntasks;
    const PSn *sn;
    const int32_t *deps;
    int32_t *cnt;  // 3 per supernode: gather tiles, step-3 tiles, all product tiles done
    int32_t *head; // next task
    int32_t *err;  // set when a dependency wait ran out
    const MatDev *mats;
    const GemmProb *probs;
};

}  // namespace selinv
