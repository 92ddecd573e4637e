// Host-only driver for the sanitizer test (tests/test_host_sanitize.py): the
// symbolic analysis in both forms, the host check of every gather and
// extraction index, and the host LU, on one matrix read from a binary file
// (n, nnz, colptr, rowind, perm, values, max_super, relax, pad_pct).
#include <cstdio>
#include <vector>
#include <string>
#include "plan.hpp"
using namespace selinv;
int main(int argc, char **argv) {
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n = 0, nnz = 0;
    bool ok = fread(&n, 8, 1, f) == 1 && fread(&nnz, 8, 1, f) == 1;
    if (!ok || n < 1 || nnz < n) return 2;
    std::vector<int64_t> cp(n + 1);
    std::vector<int32_t> ri(nnz), perm(n);
    std::vector<double> v(nnz);
    int32_t cap = 0, relax = 0, pad = 0;
    ok = fread(cp.data(), 8, n + 1, f) == (size_t)(n + 1) && fread(ri.data(), 4, nnz, f) == (size_t)nnz &&
         fread(perm.data(), 4, n, f) == (size_t)n && fread(v.data(), 8, nnz, f) == (size_t)nnz &&
         fread(&cap, 4, 1, f) == 1 && fread(&relax, 4, 1, f) == 1 && fread(&pad, 4, 1, f) == 1;
    fclose(f);
    if (!ok) return 2;
    for (int sym = 0; sym < 2; sym++) {
        Plan P; std::string err;
        selinv_status st = analyze(P, n, cp.data(), ri.data(), perm.data(), cap, relax, pad, sym, err);
        if (st) { printf("analyze(%d) failed: %s\n", sym, err.c_str()); return 1; }
        int64_t bad = check_gather_maps(P, err);
        HostFactors F;
        st = factor_host(P, v.data(), F, err);
        printf("%s sym=%d ns=%d levels=%d bad=%lld factor=%d\n", argv[1], sym, P.ns, P.nlevels, (long long)bad, (int)st);
        if (bad || st) return 1;
    }
    return 0;
}
