// factor.cpp -- host supernodal LU without pivoting (setup for the device run).
//
// At = L U with L unit lower and U upper (eq. LU), on the block pattern of the
// analysis, written straight into the device layout (diag / lpan / upan, see
// plan.hpp).  Left-looking: supernode K first pulls the updates
// -L(., D) U(D, .) of every descendant D whose block rows or columns meet K,
// then factors its diagonal block and solves for its panels.  Supernodes on
// one level of the tree are independent; the deep levels run one supernode per
// thread, the top levels (few, wide supernodes) split each product over the
// threads.  Summation order is fixed, so the factors do not depend on the
// thread count.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "plan.hpp"

namespace selinv {
namespace {

// C(m x n) -= A(m x k) * op(B),  op(B)(t, j) = transB ? B[j + t*ldb] : B[t + j*ldb].
// All column-major.  Register block 8 x 4, cache block over k.
void gemm_sub(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B,
              int64_t ldb, bool transB, double *C, int64_t ldc, bool par) {
    if (m <= 0 || n <= 0 || k <= 0) return;
    const int64_t MR = 8, NR = 4, KC = 256, MC = 128;
    int64_t nib = (m + MC - 1) / MC, njb = (n + NR - 1) / NR;
    int64_t ntiles = nib * njb;
#pragma omp parallel for schedule(dynamic, 4) if (par && ntiles > 1)
    for (int64_t tile = 0; tile < ntiles; tile++) {
        int64_t ib = tile % nib, jb = tile / nib;
        int64_t i0 = ib * MC, i1 = std::min(m, i0 + MC);
        int64_t j0 = jb * NR, nj = std::min<int64_t>(NR, n - j0);
        for (int64_t k0 = 0; k0 < k; k0 += KC) {
            int64_t k1 = std::min(k, k0 + KC);
            for (int64_t i = i0; i < i1; i += MR) {
                int64_t ni = std::min<int64_t>(MR, i1 - i);
                if (ni == MR && nj == NR) {
                    double c[NR][MR] = {};
                    for (int64_t t = k0; t < k1; t++) {
                        const double *a = A + i + t * lda;
                        double b[NR];
                        for (int64_t j = 0; j < NR; j++)
                            b[j] = transB ? B[(j0 + j) + t * ldb] : B[t + (j0 + j) * ldb];
                        for (int64_t j = 0; j < NR; j++)
#pragma omp simd
                            for (int64_t r = 0; r < MR; r++) c[j][r] += a[r] * b[j];
                    }
                    for (int64_t j = 0; j < NR; j++)
                        for (int64_t r = 0; r < MR; r++) C[(i + r) + (j0 + j) * ldc] -= c[j][r];
                } else {
                    for (int64_t j = 0; j < nj; j++)
                        for (int64_t r = 0; r < ni; r++) {
                            double acc = 0.0;
                            for (int64_t t = k0; t < k1; t++)
                                acc += A[(i + r) + t * lda] *
                                       (transB ? B[(j0 + j) + t * ldb] : B[t + (j0 + j) * ldb]);
                            C[(i + r) + (j0 + j) * ldc] -= acc;
                        }
                }
            }
        }
    }
}

// X := X * T^{-1} in place, X m x s column-major (ld m), T s x s given by
// T(u, t) = upper ? d[u + t*s] : d[t + u*s] (the transpose of the lower part),
// unit diagonal when `unit`.  Blocked by 64 columns.
void trsm_right(int64_t m, int64_t s, const double *d, bool upper, bool unit, double *X, bool par) {
    if (m <= 0) return;
    const int64_t NB = 64;
    auto T = [&](int64_t u, int64_t t) { return upper ? d[u + t * s] : d[t + u * s]; };
    for (int64_t t0 = 0; t0 < s; t0 += NB) {
        int64_t t1 = std::min(s, t0 + NB);
        // X(:, t0:t1) -= X(:, 0:t0) * T(0:t0, t0:t1)
        if (t0 > 0) {
            if (upper)
                gemm_sub(m, t1 - t0, t0, X, m, d + t0 * s, s, false, X + t0 * m, m, par);
            else
                gemm_sub(m, t1 - t0, t0, X, m, d + t0, s, true, X + t0 * m, m, par);
        }
#pragma omp parallel for schedule(static) if (par && m > 256)
        for (int64_t i0 = 0; i0 < m; i0 += 64) {
            int64_t i1 = std::min(m, i0 + 64);
            for (int64_t t = t0; t < t1; t++) {
                double *xt = X + t * m;
                for (int64_t u = t0; u < t; u++) {
                    double tv = T(u, t);
                    const double *xu = X + u * m;
                    for (int64_t i = i0; i < i1; i++) xt[i] -= xu[i] * tv;
                }
                if (!unit) {
                    double inv = T(t, t);
                    for (int64_t i = i0; i < i1; i++) xt[i] /= inv;
                }
            }
        }
    }
}

}  // namespace

selinv_status factor_host(const Plan &P, const double *values, HostFactors &F, std::string &err) {
    const int32_t ns = P.ns;
    F.d.assign(P.tot_d, 0.0);
    F.l.assign(P.tot_l, 0.0);
    F.u.assign(P.tot_u, 0.0);
    for (int64_t k = 0; k < P.nnz_a; k++) {
        int64_t loc = P.a_loc[k];
        int64_t kind = loc >> LOC_SHIFT, off = loc & LOC_MASK;
        (kind == LOC_DIAG ? F.d : kind == LOC_L ? F.l : F.u)[off] = values[k];
    }
    // descendants whose block rows or columns meet K
    std::vector<std::vector<int32_t>> upd(ns);
    {
        std::vector<int32_t> last(ns, -1);
        for (int32_t D = 0; D < ns; D++) {
            for (int64_t t = P.rl_ptr[D]; t < P.rl_ptr[D + 1]; t++) {
                int32_t K = P.supof[P.rl[t]];
                if (last[K] != D) {
                    last[K] = D;
                    upd[K].push_back(D);
                }
            }
            for (int64_t t = P.ru_ptr[D]; t < P.ru_ptr[D + 1]; t++) {
                int32_t K = P.supof[P.ru[t]];
                if (last[K] != D) {
                    last[K] = D;
                    upd[K].push_back(D);
                }
            }
        }
    }
    int nthreads = omp_get_max_threads();
    std::vector<int32_t> bad(ns, -1);

    auto process = [&](int32_t K, bool par) {
        const int32_t f = P.xsup[K], l = P.xsup[K + 1] - 1;
        const int64_t s = P.width(K), clK = P.cl(K), cuK = P.cu(K);
        double *dK = F.d.data() + P.off_d[K];
        double *lK = F.l.data() + P.off_l[K];
        double *uK = F.u.data() + P.off_u[K];
        const int32_t *RLK = P.rl.data() + P.rl_ptr[K], *RUK = P.ru.data() + P.ru_ptr[K];
        std::vector<double> T;
        std::vector<int64_t> rowpos, colpos;
        for (int32_t D : upd[K]) {
            const int64_t sD = P.width(D), clD = P.cl(D), cuD = P.cu(D);
            const int32_t *RL = P.rl.data() + P.rl_ptr[D], *RU = P.ru.data() + P.ru_ptr[D];
            const double *lD = F.l.data() + P.off_l[D];
            const double *uD = F.u.data() + P.off_u[D];
            int64_t a0 = std::lower_bound(RL, RL + clD, f) - RL;
            int64_t a1 = std::upper_bound(RL, RL + clD, l) - RL;
            int64_t b0 = std::lower_bound(RU, RU + cuD, f) - RU;
            int64_t b1 = std::upper_bound(RU, RU + cuD, l) - RU;
            // rows a >= a0 of L(., D) against columns of U(D, .) inside K
            int64_t mr = clD - a0, nc = b1 - b0;
            if (mr > 0 && nc > 0) {
                T.assign(mr * nc, 0.0);
                gemm_sub(mr, nc, sD, lD + a0, clD, uD + b0, cuD, true, T.data(), mr, par);
                rowpos.resize(mr);
                int64_t t = 0;
                for (int64_t a = a0; a < clD; a++) {
                    int32_t r = RL[a];
                    if (r <= l) {
                        rowpos[a - a0] = -1 - (r - f);
                    } else {
                        while (t < clK && RLK[t] < r) t++;
                        rowpos[a - a0] = t;  // closure: RLK[t] == r
                    }
                }
                for (int64_t b = 0; b < nc; b++) {
                    int64_t cc = RU[b0 + b] - f;
                    const double *tb = T.data() + b * mr;
                    for (int64_t a = 0; a < mr; a++) {
                        int64_t rp = rowpos[a];
                        if (rp < 0)
                            dK[(-1 - rp) + cc * s] += tb[a];  // T holds -L U
                        else
                            lK[rp + cc * clK] += tb[a];
                    }
                }
            }
            // rows inside K against columns of U(D, .) beyond K
            int64_t mi = a1 - a0, nb = cuD - b1;
            if (mi > 0 && nb > 0) {
                T.assign(mi * nb, 0.0);
                gemm_sub(mi, nb, sD, lD + a0, clD, uD + b1, cuD, true, T.data(), mi, par);
                colpos.resize(nb);
                int64_t t = 0;
                for (int64_t b = b1; b < cuD; b++) {
                    while (t < cuK && RUK[t] < RU[b]) t++;
                    colpos[b - b1] = t;
                }
                for (int64_t b = 0; b < nb; b++) {
                    int64_t cp = colpos[b];
                    const double *tb = T.data() + b * mi;
                    for (int64_t a = 0; a < mi; a++) {
                        int64_t rr = RL[a0 + a] - f;
                        uK[cp + rr * cuK] += tb[a];
                    }
                }
            }
        }
        // dense LU of the diagonal block, no pivoting
        for (int64_t t = 0; t < s; t++) {
            double piv = dK[t + t * s];
            if (piv == 0.0 || !std::isfinite(piv)) {
                bad[K] = f + (int32_t)t;
                return;
            }
            double inv = 1.0 / piv;
            for (int64_t r = t + 1; r < s; r++) dK[r + t * s] *= inv;
            for (int64_t c = t + 1; c < s; c++) {
                double ucv = dK[t + c * s];
                if (ucv == 0.0) continue;
                double *col = dK + c * s;
                const double *lt = dK + t * s;
                for (int64_t r = t + 1; r < s; r++) col[r] -= lt[r] * ucv;
            }
        }
        // L(R_L, K) := A(R_L, K) U_KK^{-1};  U(K, R_U)^T := A(K, R_U)^T L_KK^{-T}
        trsm_right(clK, s, dK, true, false, lK, par);
        trsm_right(cuK, s, dK, false, true, uK, par);
    };

    for (int32_t lev = P.nlevels - 1; lev >= 0; lev--) {
        const std::vector<int32_t> &Ks = P.levels[lev];
        if ((int)Ks.size() >= nthreads) {
#pragma omp parallel for schedule(dynamic, 1)
            for (size_t i = 0; i < Ks.size(); i++) process(Ks[i], false);
        } else {
            for (int32_t K : Ks) process(K, true);
        }
        for (int32_t K : Ks)
            if (bad[K] >= 0) {
                err = "zero or non-finite pivot at permuted column " + std::to_string(bad[K]) +
                      " (original column " + std::to_string(P.p[bad[K]]) + ")";
                return SELINV_E_ZERO_PIVOT;
            }
    }
    return SELINV_OK;
}

}  // namespace selinv
