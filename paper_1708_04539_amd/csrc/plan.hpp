// plan.hpp -- host-side structures of the selected-inversion library.
//
// The analysis output ("plan") describes the supernodal block pattern of L+U
// that Algorithm 1 of arXiv:1708.04539 walks, and where every block lives in
// the flat device arrays:
//   diag[K]  s x s, column-major     : L_KK \ U_KK  ->  A^{-T}(K,K)
//   lpan[K]  cL x s, column-major    : L(R_L,K)     ->  A^{-T}(R_L,K)
//   upan[K]  cU x s, column-major    : U(K,R_U)^T   ->  A^{-T}(K,R_U)^T
// (section "Distributed data layout and structure": diagonal blocks dense,
// off-diagonal blocks dense with non-contiguous row (L) / column (U) index
// lists).  Both panels are stored with the long dimension contiguous, so that
// the gather and the products read them in long coalesced runs.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/selinv.h"

namespace selinv {

// kind of a storage location, kept in the top bits of a 64-bit location code
enum : int64_t { LOC_DIAG = 0, LOC_L = 1, LOC_U = 2 };
constexpr int LOC_SHIFT = 60;
constexpr int64_t LOC_MASK = (int64_t(1) << LOC_SHIFT) - 1;

struct Plan {
    int64_t n = 0, nnz_a = 0;
    std::vector<int64_t> a_colptr;
    std::vector<int32_t> a_rowind;
    std::vector<int32_t> p, q;  // p: new -> old, q: old -> new
    int32_t ns = 0;
    std::vector<int32_t> xsup, supof;
    std::vector<int64_t> rl_ptr, ru_ptr;
    std::vector<int32_t> rl, ru;
    int32_t symbolic = SELINV_SYMBOLIC_SYMMETRIZED;
    // level(K) = 1 + the deepest level among the supernodes touched by
    // R_L(K) u R_U(K) (0 when both are empty); sparent(K) = the first of those
    // supernodes on level(K) - 1 (-1 on level 0).  With the symmetrized
    // analysis this is the supernodal elimination tree.
    std::vector<int32_t> sparent;
    std::vector<int32_t> level;
    // one_top[K]: sparent(K) is the only supernode on level(K) - 1 that
    // R_L(K) u R_U(K) touches (always true with the symmetrized analysis)
    std::vector<char> one_top;
    int32_t nlevels = 0;
    std::vector<std::vector<int32_t>> levels;
    std::vector<int64_t> off_d, off_l, off_u;  // element offsets
    int64_t tot_d = 0, tot_l = 0, tot_u = 0;
    // gather maps: for column b of G_K with J = sup(R_U(K)[b]) and a row a
    // with sup(R_L(K)[a]) > J, the row position of R_L(K)[a] inside R_L(J) is
    // mapL[l_coloff[ru_ptr[K] + b] + a]; symmetrically for the U side.
    std::vector<int32_t> mapL, mapU;
    std::vector<int64_t> l_coloff, u_rowoff;
    std::vector<int64_t> a_loc;  // storage location of every entry of A
    // accounting
    double flops = 0, flops_gemm = 0, bytes64 = 0, bytes32 = 0;
    double max_gemm_flops = 0;
    int32_t max_gemm_m = 0, max_gemm_n = 0, max_gemm_k = 0;
    int32_t max_s = 0, max_c = 0;

    int32_t first(int32_t K) const { return xsup[K]; }
    int32_t width(int32_t K) const { return xsup[K + 1] - xsup[K]; }
    int64_t cl(int32_t K) const { return rl_ptr[K + 1] - rl_ptr[K]; }
    int64_t cu(int32_t K) const { return ru_ptr[K + 1] - ru_ptr[K]; }
    // location of the permuted entry (r, c) in the block pattern, -1 if absent
    int64_t locate(int32_t r, int32_t c) const;
};

selinv_status analyze(Plan &P, int64_t n, const int64_t *colptr, const int32_t *rowind,
                      const int32_t *perm, int32_t max_super, int32_t relax, int32_t pad_pct,
                      int32_t symbolic, std::string &err);

struct HostFactors {
    std::vector<double> d, l, u;
};

selinv_status factor_host(const Plan &P, const double *values, HostFactors &F, std::string &err);

int64_t check_gather_maps(const Plan &P, std::string &err);

}  // namespace selinv
