// runtime.hip -- C ABI of the selected-inversion library (include/selinv.h):
// handle life cycle, device buffers, per-level work lists and the level sweep.
//
// One run (selinv_run) is
//   tri_base + gemm      (L_KK)^{-1}, (U_KK)^{-1} for every supernode (64x64
//                        diagonal sub-blocks, then recursive-doubling rounds)
//   gemm [F64]           Lhat = L(R_L,K) (L_KK)^{-1},  Uhat^T = U(K,R_U)^T (U_KK)^{-T}
//   gemm [F64]           A^{-T}(K,K) := (L_KK)^{-T} (U_KK)^{-T}
//   for level = 0 .. depth-1 (root first; Algorithm 1 walks K = N..1 and a
//   level depends only on shallower levels):
//     gather             G_K = A^{-T}(R_L(K), R_U(K))           (all K of the level)
//     gemm               step 3: A^{-T}(K,R_U)^T = -G_K^T Lhat;  step 5: A^{-T}(R_L,K) = -G_K Uhat^T
//     gemm               step 4: A^{-T}(K,K) -= A^{-T}(K,R_U) Uhat^T   (FP64 accumulation)
// All supernodes of a level (and of every matrix of a batch) share one launch
// per kernel; the work lists are built once per (handle set, precision).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "device_types.hpp"
#include "kernels.hpp"
#include "plan.hpp"

using namespace selinv;

namespace {

// Source of device memory (selinv_set_allocator): hipMalloc / hipFree, or the
// caller's hook.  Each handle and batch keeps the source in effect when it was
// created and returns every allocation to it.  Memory handed back to a hook
// may be given out again at once, so the device is drained before the hook
// sees a pointer again.
struct DevAlloc {
    selinv_alloc_fn alloc = nullptr;
    selinv_free_fn dealloc = nullptr;
    void *ctx = nullptr;
    hipError_t get(void **p, size_t bytes) const {
        bytes = std::max<size_t>(bytes, 16);
        if (!alloc) return hipMalloc(p, bytes);
        *p = alloc(bytes, ctx);
        if (!*p) return hipErrorOutOfMemory;
        if ((uintptr_t)*p % 256) {  // the kernels' vector loads assume this alignment
            (void)hipDeviceSynchronize();
            dealloc(*p, ctx);
            *p = nullptr;
            return hipErrorInvalidValue;
        }
        return hipSuccess;
    }
    void put(void *p) const {
        if (!p) return;
        if (!alloc) {
            (void)hipFree(p);
            return;
        }
        (void)hipDeviceSynchronize();
        dealloc(p, ctx);
    }
};

std::mutex g_alloc_mu;
DevAlloc g_alloc;  // the source new handles and batches take

DevAlloc current_alloc() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

struct PrecBufs {
    bool ready = false;
    double *Zd = nullptr;
    void *ZL = nullptr, *ZU = nullptr, *Lh = nullptr, *Uh = nullptr, *G = nullptr;
};

struct Range {
    int64_t off = 0;
    int count = 0;
    int tile = GEMM_TILE_64;
};

struct Sweep {
    int prec = 0;
    MatDev *d_mats = nullptr;
    TriItem *d_tri = nullptr;
    GemmProb *d_probs = nullptr;
    GemmTile *d_tiles = nullptr;
    GatherTile *d_gt = nullptr;
    // Diagonal-block inversion, normalisation and diagonal initialisation, in
    // parts by level: part i covers the supernodes of levels [pro_level[i],
    // pro_level[i + 1]).  In an unprofiled run part 0 runs on the run's
    // stream before the sweep and parts 1.. on a side stream forked from it,
    // in order, each joined (ev_part[i]) before the sweep reaches its first
    // level, so that they overlap the sweep of the levels above, which leave
    // most of the device idle.  Two parts split at level `split` (the first
    // wide level), or one part per level above it plus the rest (tuning), or
    // one part (split = 0).
    struct Prologue {
        Range tri, norm, dt;
        Range tri1, tri2;  // fused items of at most 16 / 32 columns (16- / 32-wide kernel)
        std::vector<Range> tri_rounds;  // pairs (T products, X products) per doubling round
    };
    std::vector<Prologue> pro;
    std::vector<int> pro_level;
    int split = 0;
    hipStream_t side = nullptr;
    // tile-inversion workgroups on the side stream (0: one per item).  A
    // launch that fills every compute unit leaves the upper levels' launches
    // waiting for slots until it drains; with fewer workgroups than items,
    // each looping over items, the side stream keeps compute units free.
    int side_chunk = 0;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_part;  // [i]: part i done (i >= 1)
    std::vector<Range> small, gat, g35, g4;
    // split-K step 4: per level the reduction items (red4[d].count of them,
    // red4_mn[d] the largest M N), the partial products in ws4
    std::vector<Range> red4;
    std::vector<int64_t> red4_mn;
    ReduceItem *d_red = nullptr;
    double *d_ws4 = nullptr;
    // gather tiles of level d + 1 launched with the step-4 products of level
    // d (fused[d + 1]); those products push A^{-T}(P,P) into the children's G
    std::vector<Range> g4gat;
    std::vector<char> fused;
    // levels whose steps 3/5 read G_K from its sources (launch_gemm_g35); they
    // have no gather tiles and their parents push nothing
    std::vector<char> vg;
    SmallItem *d_small = nullptr;
    std::vector<double> lev_flops35, lev_flops4, lev_gather_elems;  // launches of the large supernodes
    std::vector<double> lev_small_flops, lev_small_elems;          // the fused small-supernode launch
    std::vector<int> lev_nsup, lev_maxs;
    // algorithmic HBM bytes per launch (every operand read once, every result
    // written once; a materialised G is not counted, its sources are):
    // steps 3+5, step 4 (with the sources of the next level's gather when that
    // runs in the same launch), the standalone gather, the small-supernode
    // launch; and the largest single step-3/5 product of the level (flops)
    std::vector<double> lev_bytes35, lev_bytes4, lev_bytes_gather, lev_bytes_small, lev_max_prod;
    // prologue phases (0 inversion, 1 normalisation, 2 diagonal initialisation
    // of the mixed forms): algorithmic flops and bytes
    double pro_flops[3] = {0, 0, 0}, pro_bytes[3] = {0, 0, 0};
    // persistent sweep (used instead of the per-level launches when `persistent`)
    bool persistent = false;
    PTask *d_ptasks = nullptr;
    int32_t ntasks = 0;
    PSn *d_psn = nullptr;
    int32_t *d_deps = nullptr;
    int32_t *d_cnt = nullptr;  // 3 counters per supernode, then head, then error flag
    int64_t ncnt = 0;
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t graph_stream = nullptr;
    DevAlloc al;  // source of the work lists' device memory
    ~Sweep() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        for (auto q : ev_part)
            if (q) (void)hipEventDestroy(q);
        if (side) (void)hipStreamDestroy(side);
        for (void *q : {(void *)d_mats, (void *)d_tri, (void *)d_probs, (void *)d_tiles, (void *)d_gt,
                        (void *)d_small, (void *)d_red, (void *)d_ws4, (void *)d_ptasks, (void *)d_psn,
                        (void *)d_deps, (void *)d_cnt})
            al.put(q);
    }
};

enum : int { SWEEP_AUTO = 0, SWEEP_LEVELS = 1, SWEEP_PERSISTENT = 2 };

// Measured launch choices of one handle for one precision (selinv_tune): the
// tile edge of every launch class of grouped GEMMs (0: the size policy of
// emit_launch), per level whether a level made only of small supernodes
// keeps the fused small-supernode launch, and the sweep form.
struct Tuning {
    bool set = false;
    int tri = 0, norm = 0, dt = 0;  // prologue: doubling rounds, normalisation, diagonal init
    std::vector<int> t35, t4;       // per level: steps 3+5, step 4 (+ the next level's gather)
    std::vector<char> no_small;     // per level: 1 = per-phase launches for its small supernodes
    std::vector<char> vg;           // per level: 1 = steps 3/5 read G_K from its sources (no stored G)
    int sweep = SWEEP_AUTO;         // SWEEP_LEVELS / SWEEP_PERSISTENT, or the handle's own mode
    int no_fork = 0;                // 1: the whole prologue before the sweep, no side stream;
                                    // 2: one side-stream part per level above the split
    int side_chunk = 0;             // tile-inversion workgroups on the side stream (0: one per item)
};

constexpr int NPREC = 3;

// What one level sweep runs over: a handle alone, or the handles of a batch
// with their levels aligned at the roots.  Per precision the work lists (and
// the HIP graph recorded from them) and the tuning table; the events of the
// last profiled eager run.
struct Runner {
    DevAlloc al;
    std::vector<selinv_handle> hs;
    std::unique_ptr<Sweep> sweep[3];
    Tuning tune[3];
    int sweep_mode = 0;
    // where G_K comes from: 0 the tuning's choice per level (stored without
    // one), 1 always a stored G, 2 its sources inside the step-3/5 products
    // on every level that allows it
    int gather_form = 0;
    bool profiling = false;
    std::vector<hipEvent_t> events;
    hipStream_t own_stream = nullptr;
    int last_prec = -1;          // precision of the last run through this runner
    bool last_profiled = false;  // that run recorded its phase events
    int depth() const;
    ~Runner() {
        for (int p = 0; p < 3; p++) sweep[p].reset();
        for (auto e : events) (void)hipEventDestroy(e);
        if (own_stream) (void)hipStreamDestroy(own_stream);
    }
};

// Work lists of the device LU (selinv_factor_device), built once per handle:
// per level (deepest first) and per 64-column step of the diagonal blocks one
// launch each of tile LUs, tile inverses, solves (products with the
// inverses) and trailing updates, then the Schur complement products W_K and
// their scatter into the ancestors.
struct LuPlan {
    enum : int { L_TILES = 0, L_TRI = 1, L_SOLVE = 2, L_UPDATE = 3, L_SCHUR = 4, L_SCATTER = 5 };
    struct Launch {
        int kind;
        int64_t first;
        int count;
    };
    std::vector<Launch> launches;
    LuTile *d_lu = nullptr;
    TriItem *d_tri = nullptr;
    GemmProb *d_probs = nullptr;
    GemmTile *d_tiles = nullptr;
    GatherTile *d_sc = nullptr;
    MatDev *d_mat = nullptr;
    double *d_W = nullptr;  // W_K of one level
    int32_t *d_bad = nullptr;
    int64_t *d_emb = nullptr;  // complex handles: source of every entry of the real form
    DevAlloc al;
    ~LuPlan() {
        for (void *q : {(void *)d_lu, (void *)d_tri, (void *)d_probs, (void *)d_tiles, (void *)d_sc, (void *)d_mat,
                        (void *)d_W, (void *)d_bad, (void *)d_emb})
            al.put(q);
    }
};

inline int elem_bytes(int prec) { return prec == SELINV_FP64 ? 8 : 4; }
inline int mode_of(int prec) {
    return prec == SELINV_FP64 ? CMP_F64 : prec == SELINV_MIXED_FP32 ? CMP_F32 : CMP_BF16X3;
}

}  // namespace

struct selinv_handle_s {
    DevAlloc al;  // source of all of the handle's device memory
    Plan P;
    std::string err;
    int state = 0;  // 0 analyzed, 1 factored, 2 ran
    int device = -1;
    std::vector<SnRec> sn;
    int64_t g_elems = 0;
    double *d_diag = nullptr, *d_lpan = nullptr, *d_upan = nullptr, *d_Linv = nullptr, *d_Uinv = nullptr;
    double *d_tl = nullptr, *d_tu = nullptr;  // scratch of the triangular-inversion rounds
    SnRec *d_sn = nullptr;
    int32_t *d_supof = nullptr, *d_rl = nullptr, *d_ru = nullptr, *d_mapL = nullptr, *d_mapU = nullptr;
    int64_t *d_lcol = nullptr, *d_urow = nullptr, *d_aloc = nullptr;
    // complex matrices, held in the real-equivalent form of order 2 n_c:
    // the pattern of A (n_c, colptr_c) and, per entry p of A, the
    // locations of Re and Im of A^{-1}(j, i) (aloc_c[2p], aloc_c[2p + 1])
    bool cplx = false;
    // the supernodes and the block row / column sets of the real form come in
    // node pairs (2i, 2i + 1): the products of steps 3-5 then form only the
    // even columns of their results (GemmProb::cpx)
    bool cpx_ok = false;
    int64_t n_c = 0, nnz_c = 0;
    std::vector<int64_t> colptr_c, aloc_c;
    int64_t *d_aloc_c = nullptr;
    // children lists and positions of the parent's columns in each child's
    // R_L / R_U (see MatDev), for the push of A^{-T}(P,P) into the children's G
    std::vector<int32_t> kids_ptr, kids, push_pos;
    std::vector<int64_t> push_off;
    int32_t *d_kids_ptr = nullptr, *d_kids = nullptr, *d_push_pos = nullptr;
    // source codes of the gather (see MatDev)
    std::vector<uint32_t> gcL, gcU;
    uint32_t *d_gcL = nullptr, *d_gcU = nullptr;
    // codes of every G_K in the layout of G_K (MatDev::gcA) for the products
    // that read G_K from its sources: built on first use (ca_state 0 not yet,
    // 1 built, -1 unavailable: offsets beyond the code's 30 bits); ca_off[K]
    // its first code (-1: c_L or c_U is 0), ca_total the code count
    std::vector<int64_t> ca_off;
    int64_t ca_total = 0;
    uint32_t *d_gcA = nullptr;
    int ca_state = 0;
    // row and column source records of the gather (MatDev::row_I ...)
    int32_t *d_row_I = nullptr, *d_col_J = nullptr;
    int64_t *d_row_up = nullptr, *d_col_diag = nullptr, *d_col_low = nullptr;
    int64_t *d_push_off = nullptr;
    PrecBufs pb[NPREC];
    Runner run;  // the handle's own sweeps (hs = {this})
    int last_prec = -1;
    hipStream_t last_stream = nullptr;
    const Sweep *last_sweep = nullptr;  // sweep of the last run (own or a batch's)
    bool last_profiled = false;         // the last run was a profiled eager run of that sweep
    std::unique_ptr<LuPlan> lu;
};

int Runner::depth() const {
    int d = 0;
    for (auto h : hs) d = std::max(d, h->P.nlevels);
    return d;
}

struct selinv_batch_s {
    Runner run;
    std::string err;
};

namespace {

selinv_status dev_fail(std::string &err, hipError_t e, const char *what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? SELINV_E_NOMEM : SELINV_E_DEVICE;
}

#define HIPCHK(err, call, what)                                   \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return dev_fail((err), e_, (what)); \
    } while (0)

template <class T>
hipError_t upload(const DevAlloc &al, T **dptr, const std::vector<T> &v) {
    size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
    hipError_t e = al.get((void **)dptr, bytes);
    if (e != hipSuccess) return e;
    if (!v.empty()) e = hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

hipError_t alloc_bytes(const DevAlloc &al, void **p, size_t bytes) { return al.get(p, bytes); }

selinv_status ensure_prec(selinv_handle h, int prec) {
    PrecBufs &b = h->pb[prec];
    if (b.ready) return SELINV_OK;
    const Plan &P = h->P;
    const size_t e = elem_bytes(prec);
    HIPCHK(h->err, alloc_bytes(h->al, (void **)&b.Zd, P.tot_d * 8), "alloc Zd");
    HIPCHK(h->err, alloc_bytes(h->al, &b.ZL, P.tot_l * e), "alloc ZL");
    HIPCHK(h->err, alloc_bytes(h->al, &b.ZU, P.tot_u * e), "alloc ZU");
    HIPCHK(h->err, alloc_bytes(h->al, &b.Lh, P.tot_l * e), "alloc Lh");
    HIPCHK(h->err, alloc_bytes(h->al, &b.Uh, P.tot_u * e), "alloc Uh");
    HIPCHK(h->err, alloc_bytes(h->al, &b.G, h->g_elems * e), "alloc G");
    b.ready = true;
    return SELINV_OK;
}

// launches with fewer 64x64 tiles than this use 32x32 tiles; with at least
// kTile128From 128x128 tiles, 128x128 (measured on MI355X: the FP64 and FP32
// products run faster on 64x64 tiles at every size of these workloads, the
// split-BF16 products on 128x128 tiles once a launch has a few waves of them)
constexpr double kTile32Below = 512;
// levels at least this wide (in supernodes) start the part of the prologue
// that runs beside the sweep of the levels above
constexpr int kSplitWidth = 64;
// split-K of step 4: levels whose step-4 launch has fewer 64x64 tiles than
// this cut the k range of their products (k >= 2 kSplitKMin) into parts of at
// least kSplitKMin, up to 8, aiming at about 1024 tiles
constexpr double kSplitKBelow = 512;
constexpr int kSplitKMin = 512;
constexpr double kTile128From = 192;

// row-block major: the tiles of one strip of op(A) are neighbours in the
// list (the GEMM kernel keeps neighbours on one XCD).  pair: a product whose
// op(B) is lower triangular (GemmProb::ktri == 1: the normalisation) pairs
// column block j with block J - 1 - j of the same strip in one workgroup
// (GemmTile::n1), so that every workgroup runs about s + T of k and reads the
// strip's rows once from HBM.
void add_tiles(std::vector<GemmTile> &tiles, int prob, int M, int N, int T, bool pair = false) {
    const int J = (N + T - 1) / T;
    for (int m0 = 0; m0 < M; m0 += T) {
        if (!pair) {
            for (int n0 = 0; n0 < N; n0 += T) tiles.push_back(GemmTile{prob, m0, n0, 0});
            continue;
        }
        for (int j = 0; 2 * j < J; j++) {
            const int j2 = J - 1 - j;
            tiles.push_back(GemmTile{prob, m0, j * T, j2 > j ? j2 * T + 1 : 0});
        }
    }
}

// A launch with triangular operands (GemmProb::ktri: the normalisation and
// the diagonal initialisation) has tiles of very different k ranges (a tile
// of output columns n0.. runs k from n0).  Longest first, dealt round robin
// over the 8 per-XCD ranges of the list (gemm.hip, xcd_tile): every XCD gets
// the same mix of lengths, and runs its share longest first.  Paired tiles
// (GemmTile::n1) are dealt in runs of 4 list neighbours, which keeps the
// pairs of one strip on one XCD.
void order_by_k_length(const std::vector<GemmProb> &probs, std::vector<GemmTile> &tiles, const Range &r) {
    bool tri = false, paired = false;
    for (int i = 0; i < r.count; i++) {
        tri = tri || probs[tiles[r.off + i].prob].ktri != 0;
        paired = paired || tiles[r.off + i].n1 > 0;
    }
    if (!tri || r.count < 2) return;
    auto len1 = [&](const GemmProb &p, int m0, int n0) {
        const int klo = std::max((p.ktri & 1) ? (p.cpx ? 2 * n0 : n0) : 0, (p.ktri & 2) ? m0 : 0);
        return std::max(p.K - klo, 0);
    };
    auto len = [&](const GemmTile &t) {
        const GemmProb &p = probs[t.prob];
        return len1(p, t.m0, t.n0) + (t.n1 > 0 ? len1(p, t.m0, t.n1 - 1) : 0);
    };
    std::vector<GemmTile> sorted(tiles.begin() + r.off, tiles.begin() + r.off + r.count);
    std::stable_sort(sorted.begin(), sorted.end(),
                     [&](const GemmTile &a, const GemmTile &b) { return len(a) > len(b); });
    const int n = r.count, q = n / 8, rem = n % 8, run = paired ? 4 : 1;
    int fill[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int x = 0;
    for (int j = 0; j < n; j++) {
        if (j > 0 && j % run == 0) x = (x + 1) % 8;
        while (fill[x] >= q + (x < rem ? 1 : 0)) x = (x + 1) % 8;  // range of XCD x full
        tiles[r.off + x * q + std::min(x, rem) + fill[x]++] = sorted[j];
    }
}

// Tiles of one GEMM launch over problems [first, probs.size()).  The output
// tile is the largest that still gives the launch about two workgroups per
// compute unit: a workgroup runs the whole k range of its tile, so a launch
// with few tiles is bound by the length of that chain, and smaller tiles
// spread it over more compute units.  128x128 tiles (allow128) only for
// launches large enough to fill the device a few times over and wasting
// little of their area.
void emit_launch(const std::vector<GemmProb> &probs, size_t first, std::vector<GemmTile> &tiles, Range &r,
                 bool allow128 = false, int forced = 0, bool pair_lower = false) {
    double area = 0, t128 = 0, t64 = 0;
    for (size_t q = first; q < probs.size(); q++) {
        const double M = probs[q].M, N = probs[q].N;
        area += M * N;
        t128 += std::ceil(M / 128) * std::ceil(N / 128);
        t64 += std::ceil(M / 64) * std::ceil(N / 64);
    }
    r.tile = GEMM_TILE_64;
    if (forced == GEMM_TILE_32 || forced == GEMM_TILE_64 || forced == GEMM_TILE_128)
        r.tile = forced;  // a measured choice (selinv_tune)
    else if (t64 < kTile32Below)
        r.tile = GEMM_TILE_32;
    else if (allow128 && t128 >= kTile128From && area / (t128 * 128 * 128) >= 0.75 * area / (t64 * 64 * 64))
        r.tile = GEMM_TILE_128;
    r.off = tiles.size();
    for (size_t q = first; q < probs.size(); q++)
        add_tiles(tiles, (int)q, probs[q].M, probs[q].N, r.tile, pair_lower && probs[q].ktri == 1);
    r.count = (int)(tiles.size() - r.off);
    order_by_k_length(probs, tiles, r);
}

// As emit_launch, over the problems listed in `idx` (in that order).
void emit_launch_list(const std::vector<GemmProb> &probs, const std::vector<int> &idx, std::vector<GemmTile> &tiles,
                      Range &r, bool allow128 = false, int forced = 0) {
    std::vector<GemmProb> sub;
    sub.reserve(idx.size());
    for (int q : idx) sub.push_back(probs[q]);
    Range tmp;
    std::vector<GemmTile> t2;
    emit_launch(sub, 0, t2, tmp, allow128, forced);
    r.tile = tmp.tile;
    r.off = tiles.size();
    for (const GemmTile &t : t2) tiles.push_back(GemmTile{idx[t.prob], t.m0, t.n0, 0});
    r.count = (int)(tiles.size() - r.off);
}

// Device allocations a work list may touch: [base, base + bytes).
struct Extents {
    std::vector<std::pair<const char *, size_t>> allocs;
    int64_t violations = 0;
    void add(const void *p, size_t bytes) { allocs.push_back({(const char *)p, bytes}); }
    // the element range [first, last] of a column-major operand lies inside one allocation
    void check(const void *p, int64_t rows, int64_t cols, int64_t ld, int esize) {
        if (rows <= 0 || cols <= 0) return;
        const char *lo = (const char *)p;
        const char *hi = lo + ((rows - 1) + (cols - 1) * ld + 1) * esize;
        for (auto &a : allocs)
            if (lo >= a.first && hi <= a.first + a.second) return;
        violations++;
    }
};

int add_prob(std::vector<GemmProb> &probs, const void *A, int opA, int lda,
             const void *B, int opB, int ldb, void *C, int ldc, const void *Cin, int ldcin, int M, int N, int K,
             double alpha, double beta, Extents *ext = nullptr, int ein = 8, int eout = 8, int ktri = 0) {
    if (M <= 0 || N <= 0) return 0;
    if (ext) {
        if (K > 0) {
            if (opA == 0) ext->check(A, M, K, lda, ein); else ext->check(A, K, M, lda, ein);
            if (opB == 0) ext->check(B, K, N, ldb, ein); else ext->check(B, N, K, ldb, ein);
        }
        if (K < 0) ext->violations++;
        ext->check(C, M, N, ldc, eout);
        if (Cin) ext->check(Cin, M, N, ldcin, eout);
        if (lda < (opA == 0 ? M : K) || ldb < (opB == 0 ? K : N) || ldc < M) ext->violations++;
    }
    GemmProb p;
    p.A = A;
    p.B = B;
    p.C = C;
    p.Cin = Cin;
    p.M = M;
    p.N = N;
    p.K = K;
    p.lda = std::max(lda, 1);
    p.ldb = std::max(ldb, 1);
    p.ldc = std::max(ldc, 1);
    p.ldcin = std::max(ldcin, 1);
    p.opA = opA;
    p.opB = opB;
    p.push_sn = -1;
    p.push_mat = -1;
    p.ktri = ktri;
    p.cpx = 0;
    p.gmat = -1;
    p.gcode = -1;
    p.alpha = alpha;
    p.beta = beta;
    probs.push_back(p);
    return 1;
}

// The persistent sweep pays off when the levels are too small to fill the
// device on their own (launch latency dominates): use it when the average
// level carries less than about two waves of 64x64 product tiles.
bool persist_auto(const std::vector<selinv_handle> &hs) {
    double tiles = 0;
    int depth = 0;
    for (auto h : hs) {
        depth = std::max(depth, h->P.nlevels);
        for (const SnRec &r : h->sn)
            tiles += std::ceil(r.s / 64.0) * (std::ceil(r.cl / 64.0) + 2 * std::ceil(r.cu / 64.0));
    }
    return depth > 0 && tiles / depth < 512;
}

GatherTile gather_tile_of(selinv_handle h, int32_t mi, int32_t K, int a0, int b0, int32_t skip);
selinv_status ensure_codes_all(selinv_handle h);

// A supernode whose diagonal block, R_L and R_U all fit one 64-wide tile has
// its normalisation and diagonal initialisation done by the workgroup that
// inverts its diagonal block (tri_base_kernel), from the inverses in LDS.
inline bool fused_prologue(const SnRec &r) { return r.s <= 64 && r.cl <= 64 && r.cu <= 64; }

// Build the work lists of one sweep over a set of factored handles.
selinv_status build_sweep(std::vector<selinv_handle> &hs, const DevAlloc &al, int prec, int sweep_mode,
                          std::unique_ptr<Sweep> &out, std::string &err, const Tuning *tn = nullptr,
                          int gather_form = 0) {
    if (tn && !tn->set) tn = nullptr;
    auto t35_of = [&](int d) { return tn && d < (int)tn->t35.size() ? tn->t35[d] : 0; };
    auto t4_of = [&](int d) { return tn && d < (int)tn->t4.size() ? tn->t4[d] : 0; };
    if (tn && sweep_mode == SWEEP_AUTO && tn->sweep != SWEEP_AUTO) sweep_mode = tn->sweep;
    // Levels whose steps 3/5 read G_K from its sources (no stored G): those
    // the gather form asks for (2 every level, 1 none, 0 the tuning's
    // choice), in a level sweep only (the persistent sweep gathers), and
    // never a level of the fused small-supernode launch (decided below).
    bool vg_ok = sweep_mode == SWEEP_LEVELS || (sweep_mode == SWEEP_AUTO && !persist_auto(hs));
    auto vg_wanted = [&](int d) {
        return gather_form == 2 || (gather_form == 0 && tn && d < (int)tn->vg.size() && tn->vg[d]);
    };
    {
        int dmax = 0;
        for (auto h : hs) dmax = std::max(dmax, h->P.nlevels);
        bool any = false;
        for (int d = 0; vg_ok && d < dmax; d++) any |= vg_wanted(d);
        vg_ok = vg_ok && any;
        for (auto h : hs) {
            if (!vg_ok) break;
            selinv_status st = ensure_codes_all(h);
            if (st) {
                err = h->err;
                return st;
            }
            vg_ok = h->ca_state == 1;
        }
    }
    std::unique_ptr<Sweep> S(new Sweep());
    S->al = al;
    S->prec = prec;
    const int e = elem_bytes(prec);
    std::vector<MatDev> mats;
    std::vector<TriItem> tri;
    std::vector<GemmProb> probs;
    std::vector<GemmTile> tiles;
    std::vector<GatherTile> gts;
    int depth = 0;
    Extents X;
    // a product of a complex handle's real form that forms only the even
    // columns of its result C (rows x cols) and derives the odd ones from the
    // 2x2 complex blocks (GemmProb::cpx)
    auto halve = [&](int pi, const void *C, int64_t rows, int64_t cols, int esz) {
        if (pi < 0) return;
        GemmProb &q = probs[pi];
        q.N /= 2;
        q.ldb *= 2;
        q.ldc *= 2;
        if (q.Cin) q.ldcin *= 2;
        q.cpx = 1;
        X.check(C, rows, cols, q.ldc / 2, esz);
    };
    for (auto h : hs) {
        selinv_status st = ensure_prec(h, prec);
        if (st) {
            err = h->err;
            return st;
        }
        const PrecBufs &b = h->pb[prec];
        const Plan &P = h->P;
        X.add(h->d_lpan, P.tot_l * 8);
        X.add(h->d_upan, P.tot_u * 8);
        X.add(h->d_Linv, P.tot_d * 8);
        X.add(h->d_Uinv, P.tot_d * 8);
        X.add(h->d_tl, P.tot_d * 8);
        X.add(h->d_tu, P.tot_d * 8);
        X.add(h->d_diag, P.tot_d * 8);
        X.add(b.Zd, P.tot_d * 8);
        X.add(b.ZL, P.tot_l * e);
        X.add(b.ZU, P.tot_u * e);
        X.add(b.Lh, P.tot_l * e);
        X.add(b.Uh, P.tot_u * e);
        X.add(b.G, h->g_elems * e);
        MatDev m;
        m.sn = h->d_sn;
        m.supof = h->d_supof;
        m.rl = h->d_rl;
        m.ru = h->d_ru;
        m.l_coloff = h->d_lcol;
        m.u_rowoff = h->d_urow;
        m.mapL = h->d_mapL;
        m.mapU = h->d_mapU;
        m.kids_ptr = h->d_kids_ptr;
        m.kids = h->d_kids;
        m.push_off = h->d_push_off;
        m.push_pos = h->d_push_pos;
        m.gcL = h->d_gcL;
        m.gcU = h->d_gcU;
        m.gcA = h->d_gcA;
        m.row_I = h->d_row_I;
        m.row_up = h->d_row_up;
        m.col_J = h->d_col_J;
        m.col_diag = h->d_col_diag;
        m.col_low = h->d_col_low;
        m.Zd = b.Zd;
        m.ZL = b.ZL;
        m.ZU = b.ZU;
        m.G = b.G;
        mats.push_back(m);
        depth = std::max(depth, h->P.nlevels);
    }
    // Split of the prologue: the first level (below the root) that holds at
    // least kSplitWidth supernodes over the batch starts pro[1].
    {
        std::vector<int> width(depth, 0);
        for (auto h : hs)
            for (int d = 0; d < h->P.nlevels; d++) width[d] += (int)h->P.levels[d].size();
        S->split = 0;
        for (int d = 1; d < depth; d++)
            if (width[d] >= kSplitWidth) {
                S->split = d;
                break;
            }
        if (tn && tn->no_fork == 1) S->split = 0;
        if (tn) S->side_chunk = tn->side_chunk;
        // part of each level
        S->pro_level.assign(1, 0);
        if (S->split > 0) {
            if (tn && tn->no_fork == 2)
                for (int d = 1; d < S->split; d++) S->pro_level.push_back(d);
            S->pro_level.push_back(S->split);
        }
        S->pro.resize(S->pro_level.size());
    }
    const int npro = (int)S->pro.size();
    std::vector<int> part_of_level(depth, 0);
    for (int d = 0; d < depth; d++)
        for (int i = 0; i < npro; i++)
            if (d >= S->pro_level[i]) part_of_level[d] = i;
    std::vector<std::vector<int>> part(hs.size());
    for (size_t mi = 0; mi < hs.size(); mi++) {
        part[mi].assign(hs[mi]->P.ns, 0);
        for (int d = 0; d < hs[mi]->P.nlevels; d++)
            for (int32_t K : hs[mi]->P.levels[d]) part[mi][K] = part_of_level[d];
    }
    for (int pp = 0; pp < npro; pp++) {
        Sweep::Prologue &PR = S->pro[pp];
        // diagonal-block inversion: 64x64 diagonal sub-blocks, then recursive
        // doubling.  Round h joins neighbouring inverted blocks A (h x h, at o)
        // and B (h' x h', at o + h) of every supernode wider than h:
        //   L: X21 = -B^{-1} (C A^{-1}),   C = L(o+h.., o..)
        //   U: X12 = -A^{-1} (C B^{-1}),   C = U(o.., o+h..)
        // the inner products go to scratch (tl / tu) in a first launch, the
        // outer ones into L^{-1} / U^{-1} in a second.
        std::vector<TriItem> by_nb[3];  // 64-wide, 16-wide, 32-wide
        for (size_t mi = 0; mi < hs.size(); mi++) {
            selinv_handle h = hs[mi];
            const PrecBufs &b = h->pb[prec];
            for (int32_t K = 0; K < h->P.ns; K++) {
                if (part[mi][K] != pp) continue;
                const SnRec &r = h->sn[K];
                {
                    const double s3 = (double)r.s * r.s * r.s, s2 = (double)r.s * r.s, pc = (double)r.s * (r.cl + r.cu);
                    S->pro_flops[0] += 2.0 * s3 / 3;  // both triangular inverses
                    S->pro_bytes[0] += 16.0 * s2;
                    if (fused_prologue(r)) {  // normalisation and diagonal initialisation in the same workgroup
                        S->pro_flops[0] += (double)r.s * pc + 2.0 * s3 / 3;
                        S->pro_bytes[0] += 8.0 * pc + e * pc + 8.0 * s2;
                    } else {
                        S->pro_flops[1] += (double)r.s * pc;
                        S->pro_bytes[1] += 8.0 * pc + 8.0 * s2 + e * pc;
                        const int ph = prec == SELINV_FP64 ? 1 : 2;  // FP64: one launch for both
                        S->pro_flops[ph] += 2.0 * s3 / 3;
                        S->pro_bytes[ph] += 16.0 * s2;
                    }
                }
                for (int j0 = 0; j0 < r.s; j0 += 64) {
                    TriItem t{};
                    t.D = h->d_diag + r.off_d;
                    t.Linv = h->d_Linv + r.off_d;
                    t.Uinv = h->d_Uinv + r.off_d;
                    t.s = r.s;
                    t.j0 = j0;
                    if (fused_prologue(r)) {
                        // normalisation and diagonal initialisation in the same workgroup
                        t.fused = 1;
                        t.lpan = r.cl > 0 ? h->d_lpan + r.off_l : nullptr;
                        t.upan = r.cu > 0 ? h->d_upan + r.off_u : nullptr;
                        t.Lh = (char *)b.Lh + r.off_l * e;
                        t.Uh = (char *)b.Uh + r.off_u * e;
                        t.Zd = b.Zd + r.off_d;
                        t.cl = r.cl;
                        t.cu = r.cu;
                        t.f32out = e == 4;
                        X.check(t.D, r.s, r.s, r.s, 8);
                        X.check(t.Zd, r.s, r.s, r.s, 8);
                        if (t.lpan) X.check(t.lpan, r.cl, r.s, r.cl, 8), X.check(t.Lh, r.cl, r.s, r.cl, e);
                        if (t.upan) X.check(t.upan, r.cu, r.s, r.cu, 8), X.check(t.Uh, r.cu, r.s, r.cu, e);
                    }
                    by_nb[!t.fused ? 0 : r.s <= 16 ? 1 : r.s <= 32 ? 2 : 0].push_back(t);
                }
            }
        }
        Range *rg[3] = {&PR.tri, &PR.tri1, &PR.tri2};
        for (int c = 0; c < 3; c++) {
            rg[c]->off = tri.size();
            tri.insert(tri.end(), by_nb[c].begin(), by_nb[c].end());
            rg[c]->count = (int)by_nb[c].size();
        }
        for (int hb = 64;; hb *= 2) {
            bool any = false;
            for (size_t mi = 0; mi < hs.size(); mi++)
                for (int32_t K = 0; K < hs[mi]->P.ns; K++) any |= part[mi][K] == pp && hs[mi]->sn[K].s > hb;
            if (!any) break;
            for (int half = 0; half < 2; half++) {
                size_t first0 = probs.size();
                for (size_t mi = 0; mi < hs.size(); mi++) {
                    selinv_handle h = hs[mi];
                    for (int32_t K = 0; K < h->P.ns; K++) {
                        const SnRec &r = h->sn[K];
                        if (part[mi][K] != pp || r.s <= hb) continue;
                        const int64_t s_ = r.s;
                        const double *D = h->d_diag + r.off_d;
                        double *Li = h->d_Linv + r.off_d, *Ui = h->d_Uinv + r.off_d;
                        for (int o = 0; o + hb < r.s; o += 2 * hb) {
                            const int hp = std::min(hb, r.s - o - hb);
                            double *TL = h->d_tl + r.off_d + (int64_t)o * hb;
                            double *TU = h->d_tu + r.off_d + (int64_t)o * hb;
                            const int64_t oo = o + (int64_t)o * s_, ob = (o + hb) + (int64_t)(o + hb) * s_;
                            const int64_t lo_off = (o + hb) + (int64_t)o * s_, up_off = o + (int64_t)(o + hb) * s_;
                            if (half == 0) {
                                add_prob(probs, D + lo_off, 0, r.s, Li + oo, 0, r.s, TL, hp, nullptr, 1, hp, hb, hb,
                                         1.0, 0.0, &X, 8, 8);
                                add_prob(probs, D + up_off, 0, r.s, Ui + ob, 0, r.s, TU, hb, nullptr, 1, hb, hp, hp,
                                         1.0, 0.0, &X, 8, 8);
                            } else {
                                add_prob(probs, Li + ob, 0, r.s, TL, 0, hp, Li + lo_off, r.s, nullptr, 1, hp, hb, hp,
                                         -1.0, 0.0, &X, 8, 8);
                                add_prob(probs, Ui + oo, 0, r.s, TU, 0, hb, Ui + up_off, r.s, nullptr, 1, hb, hp, hb,
                                         -1.0, 0.0, &X, 8, 8);
                            }
                        }
                    }
                }
                Range rr;
                emit_launch(probs, first0, tiles, rr, false, tn ? tn->tri : 0);
                PR.tri_rounds.push_back(rr);
            }
        }
        // normalisation (FP64 arithmetic in the FP64 form, the bulk arithmetic of
        // the mixed forms; output in the run's precision)
        size_t first = probs.size();
        for (size_t mi = 0; mi < hs.size(); mi++) {
            selinv_handle h = hs[mi];
            const PrecBufs &b = h->pb[prec];
            for (int32_t K = 0; K < h->P.ns; K++) {
                if (part[mi][K] != pp || fused_prologue(h->sn[K])) continue;
                const SnRec &r = h->sn[K];
                char *Lh = (char *)b.Lh + r.off_l * e;
                char *Uh = (char *)b.Uh + r.off_u * e;
                // op(B) = (L_KK)^{-1} and (U_KK)^{-T} are lower triangular: a
                // tile of output columns n0.. needs k >= n0 only
                // Complex handles: Lhat = A(R_L,K) A_KK^{-1} is made of 2x2
                // complex blocks, so its even columns are formed and the odd
                // ones derived (op(B) = L_KK^{-1} is taken column by column;
                // (U_KK)^{-T} as op(B) is not, so Uhat is formed whole)
                if (add_prob(probs, h->d_lpan + r.off_l, 0, r.cl, h->d_Linv + r.off_d, 0, r.s, Lh, r.cl, nullptr, 1,
                             r.cl, r.s, r.s, 1.0, 0.0, &X, 8, e, 1) &&
                    h->cpx_ok)
                    halve((int)probs.size() - 1, Lh, r.cl, r.s, e);
                add_prob(probs, h->d_upan + r.off_u, 0, r.cu, h->d_Uinv + r.off_d, 1, r.s, Uh, r.cu, nullptr, 1, r.cu,
                         r.s, r.s, 1.0, 0.0, &X, 8, e, 1);
            }
        }
        // In the FP64 form the normalisation and the diagonal initialisation
        // run on the same kernel and share one launch; the mixed forms write
        // FP32 normalised panels and need a second kernel for the FP64
        // diagonal.
        if (prec != SELINV_FP64) {
            emit_launch(probs, first, tiles, PR.norm, false, tn ? tn->norm : 0, true);
            first = probs.size();
        }
        for (size_t mi = 0; mi < hs.size(); mi++) {
            selinv_handle h = hs[mi];
            const PrecBufs &b = h->pb[prec];
            for (int32_t K = 0; K < h->P.ns; K++) {
                if (part[mi][K] != pp || fused_prologue(h->sn[K])) continue;
                const SnRec &r = h->sn[K];
                // op(A) = (L_KK)^{-T} upper, op(B) = (U_KK)^{-T} lower: k >= max(m0, n0)
                add_prob(probs, h->d_Linv + r.off_d, 1, r.s, h->d_Uinv + r.off_d, 1, r.s, b.Zd + r.off_d, r.s,
                         nullptr, 1, r.s, r.s, r.s, 1.0, 0.0, &X, 8, 8, 3);
            }
        }
        if (prec == SELINV_FP64)
            emit_launch(probs, first, tiles, PR.norm, false, tn ? tn->norm : 0, true);
        else
            emit_launch(probs, first, tiles, PR.dt, false, tn ? tn->dt : 0);
    }
    if (npro > 1) {
        HIPCHK(err, hipStreamCreateWithFlags(&S->side, hipStreamNonBlocking), "create side stream");
        HIPCHK(err, hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming), "create event");
        S->ev_part.assign(npro, nullptr);
        for (int i = 1; i < npro; i++)
            HIPCHK(err, hipEventCreateWithFlags(&S->ev_part[i], hipEventDisableTiming), "create event");
    }
    size_t first = probs.size();
    // supernode ids over the whole batch, and the product problems of each
    std::vector<int32_t> gbase(hs.size() + 1, 0);
    for (size_t mi = 0; mi < hs.size(); mi++) gbase[mi + 1] = gbase[mi] + hs[mi]->P.ns;
    const int32_t nsn = gbase[hs.size()];
    std::vector<int> prob_zu(nsn, -1), prob_zl(nsn, -1), prob_g4(nsn, -1);
    std::vector<SmallItem> smalls;
    S->small.resize(depth);
    S->gat.resize(depth);
    S->g35.resize(depth);
    S->g4.resize(depth);
    S->lev_flops35.assign(depth, 0);
    S->lev_flops4.assign(depth, 0);
    S->lev_gather_elems.assign(depth, 0);
    S->lev_small_flops.assign(depth, 0);
    S->lev_small_elems.assign(depth, 0);
    S->lev_nsup.assign(depth, 0);
    S->lev_maxs.assign(depth, 0);
    S->lev_bytes35.assign(depth, 0);
    S->lev_bytes4.assign(depth, 0);
    S->lev_bytes_gather.assign(depth, 0);
    S->lev_bytes_small.assign(depth, 0);
    S->lev_max_prod.assign(depth, 0);
    // A supernode whose gather and three products are single 64x64 tiles is
    // handled whole by one workgroup of the fused small-supernode kernel, on
    // the levels where every supernode is of that kind: the fused launch then
    // replaces the three per-phase launches of the level.
    // (the fused kernel gathers through the source codes only)
    auto small_dims = [](const SnRec &r) {
        return r.s <= 64 && r.cl <= 64 && r.cu <= 64 && (r.cl == 0 || r.cu == 0 || r.c_off >= 0);
    };
    std::vector<char> level_small(depth, 1);
    for (size_t mi = 0; mi < hs.size(); mi++)
        for (int d = 0; d < hs[mi]->P.nlevels; d++)
            for (int32_t K : hs[mi]->P.levels[d])
                if (!small_dims(hs[mi]->sn[K])) level_small[d] = 0;
    if (tn)
        for (int d = 0; d < depth && d < (int)tn->no_small.size(); d++)
            if (tn->no_small[d]) level_small[d] = 0;
    int cur_level = 0;
    auto is_small = [&](const SnRec &r) { return level_small[cur_level] && small_dims(r); };
    // The gather of a level runs in the step-4 launch of the level above when
    // both use the per-phase launches: the parent's step-4 product writes its
    // final diagonal block into the children's G, the gather tiles fill the
    // rest.  One launch fewer per level.
    // Only where the parent is the one supernode of the level above that a
    // child's sets meet (always so for the symmetrized analysis).
    S->fused.assign(depth, 0);
    for (int d = 1; d < depth; d++) S->fused[d] = !level_small[d - 1] && !level_small[d];
    for (size_t mi = 0; mi < hs.size(); mi++)
        for (int d = 1; d < hs[mi]->P.nlevels; d++)
            for (int32_t K : hs[mi]->P.levels[d])
                if (!hs[mi]->P.one_top[K]) S->fused[d] = 0;
    S->vg.assign(depth, 0);
    for (int d = 0; d < depth; d++) {
        S->vg[d] = vg_ok && !level_small[d] && vg_wanted(d);
        if (S->vg[d]) S->fused[d] = 0;
    }
    // Split-K of the step-4 products (s x s, k = c_U) on levels whose step-4
    // launch cannot fill the device: the parts write FP64 partial products
    // that a reduction launch adds to A^{-T}(K,K) in a fixed order.  The next
    // level's gather still runs in the step-4 launch (skipping the parent's
    // diagonal block); the reduction pushes that block into the children's G.
    std::vector<int> parts4(nsn, 1);
    std::vector<int64_t> ws_off4(nsn, -1);
    std::vector<char> split4(depth, 0);
    int64_t ws_elems = 0;
    for (int d = 0; d < depth; d++) {
        cur_level = d;
        double t64 = 0;
        for (size_t mi = 0; mi < hs.size(); mi++) {
            if (d >= hs[mi]->P.nlevels) continue;
            for (int32_t K : hs[mi]->P.levels[d]) {
                const SnRec &r = hs[mi]->sn[K];
                if (!is_small(r) && r.cu > 0) t64 += std::ceil(r.s / 64.0) * std::ceil(r.s / 64.0);
            }
        }
        if (t64 <= 0 || t64 >= kSplitKBelow) continue;
        const int lvl_parts = std::min(8, (int)std::ceil(1024.0 / t64));
        for (size_t mi = 0; mi < hs.size(); mi++) {
            if (d >= hs[mi]->P.nlevels) continue;
            for (int32_t K : hs[mi]->P.levels[d]) {
                const SnRec &r = hs[mi]->sn[K];
                const int sp = std::min(lvl_parts, r.cu / kSplitKMin);
                if (is_small(r) || sp < 2) continue;
                const int32_t gid = gbase[mi] + K;
                parts4[gid] = sp;
                ws_off4[gid] = ws_elems;
                ws_elems += (int64_t)sp * r.s * r.s;
                split4[d] = 1;
            }
        }
    }
    std::vector<int> red_of(nsn, -1);  // reduction item of a split supernode
    if (ws_elems) {
        HIPCHK(err, alloc_bytes(S->al, (void **)&S->d_ws4, ws_elems * 8), "alloc split-K workspace");
        X.add(S->d_ws4, ws_elems * 8);
    }
    std::vector<ReduceItem> reds;
    S->red4.assign(depth, Range());
    S->red4_mn.assign(depth, 0);
    S->g4gat.resize(depth);
    for (int d = 0; d < depth; d++) {
        cur_level = d;
        S->gat[d].off = gts.size();
        for (size_t mi = 0; mi < hs.size(); mi++) {
            selinv_handle h = hs[mi];
            if (d >= h->P.nlevels) continue;
            for (int32_t K : h->P.levels[d]) {
                const SnRec &r = h->sn[K];
                if (!is_small(r)) {
                    if (!S->fused[d] && !S->vg[d])
                        for (int b0 = 0; b0 < r.cu; b0 += 64)
                            for (int a0 = 0; a0 < r.cl; a0 += 64)
                                gts.push_back(gather_tile_of(h, (int32_t)mi, K, a0, b0, -1));
                    S->lev_gather_elems[d] += (double)r.cl * r.cu;
                } else {
                    S->lev_small_elems[d] += (double)r.cl * r.cu;
                }
                S->lev_nsup[d]++;
                S->lev_maxs[d] = std::max(S->lev_maxs[d], r.s);
            }
        }
        S->gat[d].count = (int)(gts.size() - S->gat[d].off);
        // steps 3 and 5: the large supernodes' problems first (one launch), then
        // those of the small supernodes (run by the fused kernel)
        for (int pass = 0; pass < 2; pass++) {
            first = probs.size();
            for (size_t mi = 0; mi < hs.size(); mi++) {
                selinv_handle h = hs[mi];
                if (d >= h->P.nlevels) continue;
                const PrecBufs &b = h->pb[prec];
                for (int32_t K : h->P.levels[d]) {
                    const SnRec &r = h->sn[K];
                    if (is_small(r) != (pass == 1)) continue;
                    const int32_t gid = gbase[mi] + K;
                    const char *G = (const char *)b.G + r.g_off * e;
                    char *Lh = (char *)b.Lh + r.off_l * e, *Uh = (char *)b.Uh + r.off_u * e;
                    char *ZL = (char *)b.ZL + r.off_l * e, *ZU = (char *)b.ZU + r.off_u * e;
                    // step 3 (stored transposed): A^{-T}(K,R_U)^T = -G^T Lhat
                    prob_zu[gid] = add_prob(probs, G, 1, r.cl, Lh, 0, r.cl, ZU, r.cu, nullptr, 1, r.cu, r.s, r.cl,
                                            -1.0, 0.0, &X, e, e)
                                       ? (int)probs.size() - 1
                                       : -1;
                    // step 5: A^{-T}(R_L,K) = -G Uhat^T
                    prob_zl[gid] = add_prob(probs, G, 0, r.cl, Uh, 0, r.cu, ZL, r.cl, nullptr, 1, r.cl, r.s, r.cu,
                                            -1.0, 0.0, &X, e, e)
                                       ? (int)probs.size() - 1
                                       : -1;
                    // complex handles: the even columns of both results
                    const bool half = pass == 0 && h->cpx_ok;
                    if (half) {
                        halve(prob_zu[gid], ZU, r.cu, r.s, e);
                        halve(prob_zl[gid], ZL, r.cl, r.s, e);
                    }
                    if (S->vg[d]) {
                        // op(A) = G_K from its sources: gcA[ca_off(K) + a + b c_L]
                        const int64_t co = h->ca_off.empty() ? -1 : h->ca_off[K];
                        if (is_small(r) || (co >= 0 && co + (int64_t)r.cl * r.cu > h->ca_total)) X.violations++;
                        for (int pi : {prob_zu[gid], prob_zl[gid]}) {
                            if (pi < 0) continue;
                            GemmProb &q = probs[pi];
                            if (q.opB != 0 || q.lda != std::max(r.cl, 1) || (co < 0 && q.K > 0)) X.violations++;
                            q.gmat = (int32_t)mi;
                            q.gcode = co >= 0 ? co : 0;
                        }
                        S->lev_bytes35[d] += 4.0 * r.cl * (double)r.cu;  // the codes
                    }
                    (pass == 0 ? S->lev_flops35[d] : S->lev_small_flops[d]) +=
                        4.0 * r.s * (double)r.cl * r.cu / (half ? 2 : 1);
                    (pass == 0 ? S->lev_bytes35[d] : S->lev_bytes_small[d]) +=
                        e * ((double)r.cl * r.cu + 2.0 * r.s * ((double)r.cl + r.cu));
                    if (pass == 0) S->lev_max_prod[d] = std::max(S->lev_max_prod[d], 2.0 * r.s * (double)r.cl * r.cu);
                }
            }
            if (pass == 0) emit_launch(probs, first, tiles, S->g35[d], mode_of(prec) == CMP_BF16X3, t35_of(d));
        }
        // step 4
        for (int pass = 0; pass < 2; pass++) {
            first = probs.size();
            std::vector<int> lst;  // problems of the step-4 launch
            if (pass == 0) S->red4[d].off = reds.size();
            for (size_t mi = 0; mi < hs.size(); mi++) {
                selinv_handle h = hs[mi];
                if (d >= h->P.nlevels) continue;
                const PrecBufs &b = h->pb[prec];
                for (int32_t K : h->P.levels[d]) {
                    const SnRec &r = h->sn[K];
                    if (is_small(r) != (pass == 1)) continue;
                    const int32_t gid = gbase[mi] + K;
                    if (r.cu == 0) continue;
                    char *Uh = (char *)b.Uh + r.off_u * e, *ZU = (char *)b.ZU + r.off_u * e;
                    // step 4: A^{-T}(K,K) = (L_KK)^{-T}(U_KK)^{-T} - A^{-T}(K,R_U) Uhat^T
                    prob_g4[gid] = add_prob(probs, ZU, 1, r.cu, Uh, 0, r.cu, b.Zd + r.off_d, r.s, b.Zd + r.off_d,
                                            r.s, r.s, r.s, r.cu, -1.0, 1.0, &X, e, 8)
                                       ? (int)probs.size() - 1
                                       : -1;
                    const bool half = pass == 0 && h->cpx_ok;
                    if (half && prob_g4[gid] >= 0 && parts4[gid] < 2) halve(prob_g4[gid], b.Zd + r.off_d, r.s, r.s, 8);
                    (pass == 0 ? S->lev_flops4[d] : S->lev_small_flops[d]) +=
                        2.0 * r.s * (double)r.s * r.cu / (half ? 2 : 1);
                    if (pass == 0)
                        S->lev_bytes4[d] += 2.0 * e * r.s * (double)r.cu + 16.0 * r.s * (double)r.s;
                    else
                        S->lev_bytes_small[d] += 16.0 * r.s * (double)r.s;
                    if (pass != 0 || prob_g4[gid] < 0) continue;
                    if (parts4[gid] < 2) {
                        lst.push_back(prob_g4[gid]);
                        continue;
                    }
                    // split-K: parts of kc (a multiple of 64) columns of k
                    const int sp = parts4[gid];
                    const int kc = ((r.cu + sp - 1) / sp + 63) / 64 * 64;
                    double *P0 = S->d_ws4 + ws_off4[gid];
                    int np = 0;
                    for (int k0 = 0; k0 < r.cu; k0 += kc, np++) {
                        add_prob(probs, ZU + (int64_t)k0 * e, 1, r.cu, Uh + (int64_t)k0 * e, 0, r.cu,
                                 P0 + (int64_t)np * r.s * r.s, r.s, nullptr, 1, r.s, r.s, std::min(kc, r.cu - k0),
                                 -1.0, 0.0, &X, e, 8);
                        if (half) {  // the even columns only, packed s x s/2; the reduction gives the rest
                            GemmProb &q = probs.back();
                            q.N /= 2;
                            q.ldb *= 2;
                        }
                        lst.push_back((int)probs.size() - 1);
                    }
                    X.check(b.Zd + r.off_d, r.s, r.s, r.s, 8);
                    X.check(P0, (int64_t)r.s * r.s, np, (int64_t)r.s * r.s, 8);
                    red_of[gid] = (int)reds.size();
                    reds.push_back(ReduceItem{b.Zd + r.off_d, P0, r.s, half ? r.s / 2 : r.s, r.s, np,
                                              (int64_t)r.s * r.s, -1, -1, e == 4, half ? 1 : 0});
                    S->red4_mn[d] = std::max<int64_t>(S->red4_mn[d], (int64_t)r.s * r.s);
                }
            }
            if (pass == 0) {
                S->red4[d].count = (int)(reds.size() - S->red4[d].off);
                emit_launch_list(probs, lst, tiles, S->g4[d], mode_of(prec) == CMP_BF16X3, t4_of(d));
            }
        }
        // A step-4 launch of 128-wide tiles runs two workgroups per compute
        // unit, too few for the gather's dependent loads: the next level's
        // gather then gets a launch of its own (split-BF16 on C4: 0.05-0.12 ms
        // less per level)
        if (d + 1 < depth && S->g4[d].count > 0 && S->g4[d].tile == GEMM_TILE_128) S->fused[d + 1] = 0;
        S->g4gat[d].off = gts.size();
        if (d + 1 < depth && S->fused[d + 1]) {
            for (size_t mi = 0; mi < hs.size(); mi++) {
                selinv_handle h = hs[mi];
                if (d + 1 >= h->P.nlevels) continue;
                for (int32_t K : h->P.levels[d + 1]) {
                    const SnRec &r = h->sn[K];
                    const int32_t Pa = h->P.sparent[K];
                    const int pg = Pa >= 0 ? prob_g4[gbase[mi] + Pa] : -1;
                    // a parent without a step-4 product keeps its initial
                    // diagonal block, which the gather reads as usual
                    int32_t skip = -1;
                    if (pg >= 0) {
                        probs[pg].push_sn = Pa;
                        probs[pg].push_mat = (int32_t)mi;
                        skip = Pa;
                        // a split product is pushed by its reduction
                        const int ri = red_of[gbase[mi] + Pa];
                        if (ri >= 0) {
                            reds[ri].push_sn = Pa;
                            reds[ri].push_mat = (int32_t)mi;
                        }
                    }
                    for (int b0 = 0; b0 < r.cu; b0 += 64)
                        for (int a0 = 0; a0 < r.cl; a0 += 64)
                            gts.push_back(gather_tile_of(h, (int32_t)mi, K, a0, b0, skip));
                }
            }
        }
        S->g4gat[d].count = (int)(gts.size() - S->g4gat[d].off);
        S->small[d].off = smalls.size();
        for (size_t mi = 0; mi < hs.size(); mi++) {
            selinv_handle h = hs[mi];
            if (d >= h->P.nlevels) continue;
            for (int32_t K : h->P.levels[d]) {
                const SnRec &r = h->sn[K];
                const int32_t gid = gbase[mi] + K;
                if (!is_small(r) || (prob_zu[gid] < 0 && prob_zl[gid] < 0 && prob_g4[gid] < 0)) continue;
                smalls.push_back(SmallItem{(int32_t)mi, K, prob_zu[gid], prob_zl[gid], prob_g4[gid], r.s, r.cl, r.cu,
                                           r.g_off, r.c_off});
            }
        }
        S->small[d].count = (int)(smalls.size() - S->small[d].off);
    }
    for (int d = 0; d < depth; d++) {
        const double src = e * S->lev_gather_elems[d];
        if (S->vg[d]) continue;  // the sources are the G operand of the level's steps 3/5
        if (d > 0 && S->fused[d])
            S->lev_bytes4[d - 1] += src;
        else
            S->lev_bytes_gather[d] += src;
    }
    // persistent task queue: level by level from the root; per level all
    // gather tiles, then the step-3 tiles, the step-5 tiles, the step-4 tiles
    {
        std::vector<PTask> pt;
        std::vector<PSn> psn(nsn);
        std::vector<int32_t> deps;
        auto tiles64 = [](int M, int N) { return ((M + 63) / 64) * ((N + 63) / 64); };
        for (size_t mi = 0; mi < hs.size(); mi++) {
            selinv_handle h = hs[mi];
            for (int32_t K = 0; K < h->P.ns; K++) {
                const int32_t gid = gbase[mi] + K;
                const SnRec &r = h->sn[K];
                PSn &q = psn[gid];
                // symmetrized sets: the parent carries every dependency on;
                // exact sets: every supernode that R_L(K) u R_U(K) meets
                q.dep_off = (int32_t)deps.size();
                const Plan &P = h->P;
                if (P.symbolic == SELINV_SYMBOLIC_SYMMETRIZED) {
                    if (P.sparent[K] >= 0) deps.push_back(gbase[mi] + P.sparent[K]);
                } else {
                    std::vector<int32_t> blk;
                    for (int64_t x = P.rl_ptr[K]; x < P.rl_ptr[K + 1]; x++) blk.push_back(P.supof[P.rl[x]]);
                    for (int64_t x = P.ru_ptr[K]; x < P.ru_ptr[K + 1]; x++) blk.push_back(P.supof[P.ru[x]]);
                    std::sort(blk.begin(), blk.end());
                    blk.erase(std::unique(blk.begin(), blk.end()), blk.end());
                    for (int32_t J : blk) deps.push_back(gbase[mi] + J);
                }
                q.ndep = (int32_t)deps.size() - q.dep_off;
                q.n_gather = tiles64(r.cl, r.cu);
                q.n_zu = prob_zu[gid] >= 0 ? tiles64(probs[prob_zu[gid]].M, probs[prob_zu[gid]].N) : 0;
                q.n_all = q.n_zu;
                if (prob_zl[gid] >= 0) q.n_all += tiles64(probs[prob_zl[gid]].M, probs[prob_zl[gid]].N);
                if (prob_g4[gid] >= 0) q.n_all += tiles64(probs[prob_g4[gid]].M, probs[prob_g4[gid]].N);
            }
        }
        auto push_prob = [&](int type, int32_t gid, int mat, int32_t K, int prob, int is_zu) {
            if (prob < 0) return;
            const GemmProb &p = probs[prob];
            for (int n0 = 0; n0 < p.N; n0 += 64)
                for (int m0 = 0; m0 < p.M; m0 += 64) pt.push_back(PTask{type, gid, mat, K, m0, n0, prob, is_zu});
        };
        for (int d = 0; d < depth; d++) {
            for (size_t mi = 0; mi < hs.size(); mi++) {
                selinv_handle h = hs[mi];
                if (d >= h->P.nlevels) continue;
                for (int32_t K : h->P.levels[d]) {
                    const SnRec &r = h->sn[K];
                    for (int b0 = 0; b0 < r.cu; b0 += 64)
                        for (int a0 = 0; a0 < r.cl; a0 += 64)
                            pt.push_back(PTask{PT_GATHER, gbase[mi] + K, (int32_t)mi, K, a0, b0, -1, 0});
                }
            }
            for (int pass = 0; pass < 3; pass++)
                for (size_t mi = 0; mi < hs.size(); mi++) {
                    selinv_handle h = hs[mi];
                    if (d >= h->P.nlevels) continue;
                    for (int32_t K : h->P.levels[d]) {
                        const int32_t gid = gbase[mi] + K;
                        if (pass == 0) push_prob(PT_STEP35, gid, (int)mi, K, prob_zu[gid], 1);
                        if (pass == 1) push_prob(PT_STEP35, gid, (int)mi, K, prob_zl[gid], 0);
                        if (pass == 2) push_prob(PT_STEP4, gid, (int)mi, K, prob_g4[gid], 0);
                    }
                }
        }
        // a task may only wait for tasks earlier in the queue
        std::vector<int64_t> last_gather(nsn, -1), last_zu(nsn, -1), last_all(nsn, -1), first_any(nsn, INT64_MAX);
        for (int64_t t = 0; t < (int64_t)pt.size(); t++) {
            const PTask &k = pt[t];
            first_any[k.gid] = std::min(first_any[k.gid], t);
            if (k.type == PT_GATHER) last_gather[k.gid] = t;
            if (k.type != PT_GATHER) last_all[k.gid] = t;
            if (k.is_zu) last_zu[k.gid] = t;
        }
        for (int32_t g = 0; g < nsn; g++)
            for (int32_t d = 0; d < psn[g].ndep; d++) {
                const int32_t P = deps[psn[g].dep_off + d];
                if (P < 0 || P >= nsn || P == g) X.violations++;
                else if (first_any[g] != INT64_MAX && last_all[P] >= first_any[g]) X.violations++;
            }
        for (int64_t t = 0; t < (int64_t)pt.size(); t++) {
            const PTask &k = pt[t];
            if (k.type == PT_STEP35 && last_gather[k.gid] > t) X.violations++;
            if (k.type == PT_STEP4 && last_zu[k.gid] > t) X.violations++;
        }
        const bool small = pt.size() <= 400000;
        S->persistent = sweep_mode == SWEEP_PERSISTENT || (sweep_mode == SWEEP_AUTO && small && persist_auto(hs));
        if (S->persistent) {
            if (pt.size() >= (size_t)INT32_MAX) {
                err = "persistent task queue too long";
                return SELINV_E_INVALID_ARG;
            }
            S->ntasks = (int32_t)pt.size();
            S->ncnt = 3 * (int64_t)nsn;
            std::vector<int32_t> zero(S->ncnt + 2, 0);
            HIPCHK(err, upload(S->al, &S->d_ptasks, pt), "upload tasks");
            HIPCHK(err, upload(S->al, &S->d_psn, psn), "upload task deps");
            HIPCHK(err, upload(S->al, &S->d_deps, deps), "upload task deps");
            HIPCHK(err, upload(S->al, &S->d_cnt, zero), "upload counters");
            S->grid = persist_grid(mode_of(prec));
            if (S->grid <= 0) {
                err = "could not size the persistent grid";
                return SELINV_E_DEVICE;
            }
        }
    }
    // gather tiles stay inside their supernode's G block
    for (const GatherTile &t : gts) {
        const SnRec &r = hs[t.mat]->sn[t.K];
        if (t.a0 < 0 || t.b0 < 0 || t.a0 >= r.cl || t.b0 >= r.cu ||
            r.g_off + (int64_t)r.cl * r.cu > hs[t.mat]->g_elems)
            X.violations++;
    }
    // a small item's products are single tiles of problems in the list
    for (const SmallItem &it : smalls) {
        const SnRec &r = hs[it.mat]->sn[it.K];
        if (r.s > 64 || r.cl > 64 || r.cu > 64) X.violations++;
        for (int32_t p : {it.pzu, it.pzl, it.pg4})
            if (p >= (int32_t)probs.size() || (p >= 0 && (probs[p].M > 64 || probs[p].N > 64))) X.violations++;
    }
    for (auto h : hs)
        for (const SnRec &r : h->sn)
            if (r.s > TRI_MAX_S || r.off_d + (int64_t)r.s * r.s > h->P.tot_d) X.violations++;
    // every level's reduction items lie inside the uploaded list
    for (int d = 0; d < depth; d++)
        if (S->red4[d].off < 0 || S->red4[d].count < 0 ||
            S->red4[d].off + S->red4[d].count > (int64_t)reds.size())
            X.violations++;
    if (X.violations) {
        err = "internal error: " + std::to_string(X.violations) + " work-list entries outside their buffers";
        return SELINV_E_INVALID_ARG;
    }
    HIPCHK(err, upload(S->al, &S->d_mats, mats), "upload mats");
    HIPCHK(err, upload(S->al, &S->d_tri, tri), "upload tri");
    HIPCHK(err, upload(S->al, &S->d_probs, probs), "upload probs");
    HIPCHK(err, upload(S->al, &S->d_tiles, tiles), "upload tiles");
    HIPCHK(err, upload(S->al, &S->d_gt, gts), "upload gather tiles");
    HIPCHK(err, upload(S->al, &S->d_small, smalls), "upload small supernodes");
    HIPCHK(err, upload(S->al, &S->d_red, reds), "upload split-K reductions");
    out = std::move(S);
    return SELINV_OK;
}

// Launch a sweep; `ev` (optional) receives one event after each phase.
hipError_t launch_sweep(const Sweep &S, hipStream_t st, std::vector<hipEvent_t> *ev) {
    const int prec = S.prec, mode = mode_of(prec);
    const int f64 = prec == SELINV_FP64;
    hipError_t e;
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord((*ev)[i], st);
    };
    // prologue parts: diagonal-block inversion (base blocks and doubling
    // rounds), normalisation, diagonal initialisation
    // on the side stream, at most side_chunk inversion workgroups resident
    // (each loops over items), so that the level chain finds free compute units
    auto tri_launch = [&](const Range &r, int nb, hipStream_t s) -> hipError_t {
        return launch_tri_base(S.d_tri + r.off, r.count, nb, s, s == S.side ? S.side_chunk : 0);
    };
    auto tri_part = [&](const Sweep::Prologue &P, hipStream_t s) -> hipError_t {
        hipError_t e2;
        if ((e2 = tri_launch(P.tri, 4, s))) return e2;
        if ((e2 = tri_launch(P.tri1, 1, s))) return e2;
        if ((e2 = tri_launch(P.tri2, 2, s))) return e2;
        for (const Range &r : P.tri_rounds)
            if ((e2 = launch_gemm(GEMM_PRO_F64, CMP_F64, r.tile, S.d_probs, S.d_tiles + r.off, r.count, s)))
                return e2;
        return hipSuccess;
    };
    auto norm_part = [&](const Sweep::Prologue &P, hipStream_t s) -> hipError_t {
        // the mixed forms run the normalisation in their bulk arithmetic (FP32
        // or split-BF16 from the FP64 factors); FP64 stays for the diagonal
        // inversions and the diagonal blocks of A^{-T}
        return launch_gemm(f64 ? GEMM_PRO_F64 : GEMM_PRO_MIXED, f64 ? CMP_F64 : mode, P.norm.tile, S.d_probs,
                           S.d_tiles + P.norm.off, P.norm.count, s);
    };
    auto dt_part = [&](const Sweep::Prologue &P, hipStream_t s) -> hipError_t {
        return launch_gemm(GEMM_PRO_F64, CMP_F64, P.dt.tile, S.d_probs, S.d_tiles + P.dt.off, P.dt.count, s);
    };
    // The side parts are forked after the main part, so that the main part
    // (needed first) does not share the device with them.  A profiled run
    // runs every part on the run's stream, phase by phase.  The side parts
    // are issued after the first level's launches: a graph captured from
    // this order keeps the level chain, which is the critical path, on the
    // queue that ran the main part, and the side branch takes the cross-queue
    // wait of the fork (tens of microseconds when a graph branch starts on
    // another queue).  Every side part is first needed at level 1 or later.
    const int npro = (int)S.pro.size();
    const bool fork = npro > 1 && ev == nullptr;
    const int nmain = fork ? 1 : npro;
    mark(0);
    for (int q = 0; q < nmain; q++)
        if ((e = tri_part(S.pro[q], st))) return e;
    mark(1);
    for (int q = 0; q < nmain; q++)
        if ((e = norm_part(S.pro[q], st))) return e;
    mark(2);
    for (int q = 0; q < nmain; q++)
        if ((e = dt_part(S.pro[q], st))) return e;
    mark(3);
    if (fork && (e = hipEventRecord(S.ev_fork, st))) return e;
    bool side_due = fork;
    auto side_parts = [&]() -> hipError_t {
        side_due = false;
        hipError_t e2;
        if ((e2 = hipStreamWaitEvent(S.side, S.ev_fork, 0))) return e2;
        for (int q = 1; q < npro; q++) {
            if ((e2 = tri_part(S.pro[q], S.side))) return e2;
            if ((e2 = norm_part(S.pro[q], S.side))) return e2;
            if ((e2 = dt_part(S.pro[q], S.side))) return e2;
            if ((e2 = hipEventRecord(S.ev_part[q], S.side))) return e2;
        }
        return hipSuccess;
    };
    if (S.persistent) {
        PersistArgs a;
        a.tasks = S.d_ptasks;
        a.ntasks = S.ntasks;
        a.sn = S.d_psn;
        a.deps = S.d_deps;
        a.cnt = S.d_cnt;
        a.head = S.d_cnt + S.ncnt;
        a.err = S.d_cnt + S.ncnt + 1;
        a.mats = S.d_mats;
        a.probs = S.d_probs;
        if (side_due && (e = side_parts())) return e;
        if (fork && (e = hipStreamWaitEvent(st, S.ev_part[npro - 1], 0))) return e;
        if ((e = launch_persist(mode, a, S.ncnt, S.grid, st))) return e;
        for (size_t d = 0; d < 4 * S.gat.size(); d++) mark(4 + d);
        return hipSuccess;
    }
    for (size_t d = 0; d < S.gat.size(); d++) {
        if (side_due && d > 0 && (e = side_parts())) return e;
        if (fork)
            for (int q = 1; q < npro; q++)
                if (S.pro_level[q] == (int)d && (e = hipStreamWaitEvent(st, S.ev_part[q], 0))) return e;
        if ((e = launch_small(mode, S.d_mats, S.d_probs, S.d_small + S.small[d].off, S.small[d].count, st)))
            return e;
        mark(4 + 4 * d);
        if ((e = launch_gather(f64, S.d_mats, S.d_gt + S.gat[d].off, S.gat[d].count, st))) return e;
        mark(5 + 4 * d);
        if (S.vg[d]) {
            if ((e = launch_gemm_g35(mode, S.g35[d].tile, S.d_probs, S.d_tiles + S.g35[d].off, S.g35[d].count,
                                     S.d_mats, st)))
                return e;
        } else if ((e = launch_gemm(GEMM_STEP35, mode, S.g35[d].tile, S.d_probs, S.d_tiles + S.g35[d].off,
                                    S.g35[d].count, st))) {
            return e;
        }
        mark(6 + 4 * d);
        if ((e = launch_step4_gather(mode, S.g4[d].tile, S.d_probs, S.d_tiles + S.g4[d].off, S.g4[d].count,
                                     S.d_mats, S.d_gt + S.g4gat[d].off, S.g4gat[d].count, st)))
            return e;
        if ((e = launch_splitk_reduce(S.d_red + S.red4[d].off, S.red4[d].count, S.red4_mn[d], S.d_mats, st)))
            return e;
        mark(7 + 4 * d);
    }
    if (side_due) {  // a sweep with no level past the first: join the side parts here
        if ((e = side_parts())) return e;
        for (int q = 1; q < npro; q++)
            if ((e = hipStreamWaitEvent(st, S.ev_part[q], 0))) return e;
    }
    return hipSuccess;
}

bool valid_prec(int p) { return p >= 0 && p < NPREC; }

// Real-equivalent form of a complex matrix: the entry a = x + i y of A at
// (i, j) becomes the block [[x, -y], [y, x]] at rows 2i, 2i+1 and columns 2j,
// 2j+1, so that M = [[Re A, -Im A], [Im A, Re A]] up to the interleaving and
// M^{-1} holds A^{-1} in the same way.  The pattern of column 2j and of column
// 2j+1 lists rows 2i, 2i+1 for every row i of column j; the ordering keeps
// the two rows and columns of a node together (perm2[2k + h] = 2 perm[k] + h).
selinv_status complex_embedding(int64_t n, const int64_t *colptr, const int32_t *rowind, const int32_t *perm,
                                std::vector<int64_t> &cp2, std::vector<int32_t> &ri2, std::vector<int32_t> &pm2,
                                std::string &err) {
    if (n < 1 || !colptr || !rowind) {
        err = "n must be >= 1 and colptr/rowind non-null";
        return SELINV_E_INVALID_ARG;
    }
    if (2 * n >= (int64_t(1) << 31) - 1) {
        err = "2 n exceeds the int32 index range (complex matrices take the real form of order 2 n)";
        return SELINV_E_INVALID_ARG;
    }
    if (colptr[0] != 0) {
        err = "colptr[0] != 0";
        return SELINV_E_BAD_PATTERN;
    }
    for (int64_t j = 0; j < n; j++)
        if (colptr[j + 1] < colptr[j]) {
            err = "colptr decreases";
            return SELINV_E_BAD_PATTERN;
        }
    cp2.assign(2 * n + 1, 0);
    ri2.resize(4 * colptr[n]);
    int64_t at = 0;
    for (int64_t j = 0; j < n; j++)
        for (int h = 0; h < 2; h++) {
            for (int64_t k = colptr[j]; k < colptr[j + 1]; k++) {
                const int32_t i = rowind[k];
                if (i < 0 || i >= n) {
                    err = "row index out of range in column " + std::to_string(j);
                    return SELINV_E_BAD_PATTERN;
                }
                ri2[at++] = 2 * i;
                ri2[at++] = 2 * i + 1;
            }
            cp2[2 * j + h + 1] = at;
        }
    pm2.resize(2 * n);
    for (int64_t k = 0; k < n; k++) {
        const int32_t v = perm ? perm[k] : (int32_t)k;
        if (v < 0 || v >= n) {
            err = "perm is not a permutation";
            return SELINV_E_BAD_PERM;
        }
        pm2[2 * k] = 2 * v;
        pm2[2 * k + 1] = 2 * v + 1;
    }
    return SELINV_OK;
}

// Source codes of the gather (MatDev::gcL / gcU): for every supernode K that
// gets them, the location of A^{-T}(R_L(K)[a], R_U(K)[b]) as array << 30 |
// element offset, found through the relative-index maps as the map-based
// gather finds it.  Every supernode gets codes while their total stays within
// kCodeBudget entries; otherwise only those with G_K of at most 64 x 64 (the
// latency-bound ones), in order, while the budget lasts.  Offsets must fit 30
// bits, else no codes at all.
constexpr int64_t kCodeBudget = int64_t(1) << 26;

// Source code of entry (a, b) of G_K, where column b of R_U(K) is node c of
// supernode J (first node fJ): array << 30 | element offset.
inline uint32_t gcode_of(const Plan &P, int32_t K, int64_t a, int64_t b, int32_t c, int32_t J, int32_t fJ) {
    const int32_t r = P.rl[P.rl_ptr[K] + a], I = P.supof[r];
    if (I == J)  // diagonal block of J
        return (1u << GCODE_SHIFT) | (uint32_t)(P.off_d[J] + int64_t(c - fJ) * P.width(J) + (r - fJ));
    if (I > J)  // row r in the L panel of J
        return (2u << GCODE_SHIFT) |
               (uint32_t)(P.off_l[J] + int64_t(c - fJ) * P.cl(J) + P.mapL[P.l_coloff[P.ru_ptr[K] + b] + a]);
    // column c in the U panel of I
    return (3u << GCODE_SHIFT) |
           (uint32_t)(P.off_u[I] + int64_t(r - P.xsup[I]) * P.cu(I) + P.mapU[P.u_rowoff[P.rl_ptr[K] + a] + b]);
}

void build_gather_codes(const Plan &P, std::vector<SnRec> &sn, std::vector<uint32_t> &gcL,
                        std::vector<uint32_t> &gcU, int64_t budget) {
    gcL.clear();
    gcU.clear();
    for (SnRec &r : sn) r.c_off = -1;
    const int64_t lim = int64_t(GCODE_MASK) + 1;
    if (P.tot_d > lim || P.tot_l > lim || P.tot_u > lim) return;
    int64_t total = 0;
    for (int32_t K = 0; K < P.ns; K++) total += P.cl(K) * P.cu(K);
    const bool all = total <= budget;
    int64_t used = 0;
    for (int32_t K = 0; K < P.ns; K++) {
        const int64_t cl = P.cl(K), cu = P.cu(K);
        if (cl == 0 || cu == 0 || (!all && (cl > 64 || cu > 64)) || used + cl * cu > budget) continue;
        sn[K].c_off = used;
        used += cl * cu;
    }
    gcL.assign(used, 0);
    gcU.assign(used, 0);
    for (int32_t K = 0; K < P.ns; K++) {
        const int64_t co = sn[K].c_off, cl = P.cl(K), cu = P.cu(K);
        if (co < 0) continue;
        for (int64_t b = 0; b < cu; b++) {
            const int32_t c = P.ru[P.ru_ptr[K] + b], J = P.supof[c], fJ = P.xsup[J];
            for (int64_t a = 0; a < cl; a++) {
                const uint32_t code = gcode_of(P, K, a, b, c, J, fJ);
                if ((code >> GCODE_SHIFT) == 3)
                    gcU[co + b + a * cu] = code;
                else
                    gcL[co + a + b * cl] = code;
            }
        }
    }
}

// The codes of every G_K in its own layout (MatDev::gcA), built once per
// handle on first use: filled by up to 16 host threads over the supernodes,
// uploaded, and the host copy released.
selinv_status ensure_codes_all(selinv_handle h) {
    if (h->ca_state != 0) return SELINV_OK;
    const Plan &P = h->P;
    const int64_t lim = int64_t(GCODE_MASK) + 1;
    if (P.tot_d > lim || P.tot_l > lim || P.tot_u > lim) {
        h->ca_state = -1;
        return SELINV_OK;
    }
    h->ca_off.assign(P.ns, -1);
    int64_t used = 0;
    for (int32_t K = 0; K < P.ns; K++) {
        const int64_t cl = P.cl(K), cu = P.cu(K);
        if (cl == 0 || cu == 0) continue;
        h->ca_off[K] = used;
        used += cl * cu;
    }
    std::vector<uint32_t> codes;
    try {
        codes.resize(std::max<int64_t>(used, 1));
    } catch (const std::bad_alloc &) {
        h->err = "host allocation failed for the gather codes";
        return SELINV_E_NOMEM;
    }
    std::atomic<int32_t> next{0};
    auto work = [&]() {
        for (int32_t K; (K = next.fetch_add(1)) < P.ns;) {
            const int64_t co = h->ca_off[K], cl = P.cl(K), cu = P.cu(K);
            if (co < 0) continue;
            for (int64_t b = 0; b < cu; b++) {
                const int32_t c = P.ru[P.ru_ptr[K] + b], J = P.supof[c], fJ = P.xsup[J];
                uint32_t *col = codes.data() + co + b * cl;
                for (int64_t a = 0; a < cl; a++) col[a] = gcode_of(P, K, a, b, c, J, fJ);
            }
        }
    };
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nt; t++) pool.emplace_back(work);
    work();
    for (auto &t : pool) t.join();
    HIPCHK(h->err, upload(h->al, &h->d_gcA, codes), "upload gather codes");
    h->ca_total = used;
    h->ca_state = 1;
    return SELINV_OK;
}

// Gather tile of supernode K of handle h (matrix mi of the sweep); skip: the
// supernode whose diagonal block the tile leaves to that supernode's step-4
// product (-1: none).
GatherTile gather_tile_of(selinv_handle h, int32_t mi, int32_t K, int a0, int b0, int32_t skip) {
    const SnRec &r = h->sn[K];
    GatherTile g;
    g.mat = mi;
    g.K = K;
    g.a0 = a0;
    g.b0 = b0;
    g.skip = skip;
    g.cl = r.cl;
    g.cu = r.cu;
    g.pad = 0;
    g.g_off = r.g_off;
    g.c_off = r.c_off;
    g.skip_lo = g.skip_hi = 0;
    g.rl_off = r.rl_off;
    g.ru_off = r.ru_off;
    if (skip >= 0) {
        g.skip_lo = h->sn[skip].off_d;
        g.skip_hi = g.skip_lo + (int64_t)h->sn[skip].s * h->sn[skip].s;
    }
    return g;
}

// Children of every supernode, and for each child K of P the positions of
// P's columns first(P) + r in R_L(K) and R_U(K) (-1 where absent).  Both
// lists are sorted, so one merge walk each.
void build_push_maps(const Plan &P, std::vector<int32_t> &kids_ptr, std::vector<int32_t> &kids,
                     std::vector<int64_t> &push_off, std::vector<int32_t> &push_pos) {
    kids_ptr.assign(P.ns + 1, 0);
    for (int32_t K = 0; K < P.ns; K++)
        if (P.sparent[K] >= 0) kids_ptr[P.sparent[K] + 1]++;
    for (int32_t K = 0; K < P.ns; K++) kids_ptr[K + 1] += kids_ptr[K];
    kids.assign(kids_ptr[P.ns], 0);
    std::vector<int32_t> fill(kids_ptr.begin(), kids_ptr.end() - 1);
    for (int32_t K = 0; K < P.ns; K++)
        if (P.sparent[K] >= 0) kids[fill[P.sparent[K]]++] = K;
    push_off.assign(P.ns, -1);
    int64_t tot = 0;
    for (int32_t K = 0; K < P.ns; K++)
        if (P.sparent[K] >= 0) {
            push_off[K] = tot;
            tot += 2 * (int64_t)P.width(P.sparent[K]);
        }
    push_pos.assign(tot, -1);
    for (int32_t K = 0; K < P.ns; K++) {
        const int32_t Pa = P.sparent[K];
        if (Pa < 0) continue;
        const int32_t f = P.xsup[Pa], sP = P.width(Pa);
        int32_t *posL = push_pos.data() + push_off[K], *posU = posL + sP;
        for (int64_t a = P.rl_ptr[K]; a < P.rl_ptr[K + 1]; a++) {
            const int32_t r = P.rl[a] - f;
            if (r >= 0 && r < sP) posL[r] = (int32_t)(a - P.rl_ptr[K]);
        }
        for (int64_t b = P.ru_ptr[K]; b < P.ru_ptr[K + 1]; b++) {
            const int32_t c = P.ru[b] - f;
            if (c >= 0 && c < sP) posU[c] = (int32_t)(b - P.ru_ptr[K]);
        }
    }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *selinv_status_string(selinv_status s) {
    switch (s) {
        case SELINV_OK: return "OK";
        case SELINV_E_INVALID_ARG: return "INVALID_ARG";
        case SELINV_E_BAD_PATTERN: return "BAD_PATTERN";
        case SELINV_E_BAD_PERM: return "BAD_PERM";
        case SELINV_E_ZERO_PIVOT: return "ZERO_PIVOT";
        case SELINV_E_NOT_SELECTED: return "NOT_SELECTED";
        case SELINV_E_STATE: return "STATE";
        case SELINV_E_NOMEM: return "NOMEM";
        case SELINV_E_DEVICE: return "DEVICE";
    }
    return "UNKNOWN";
}

// message of the last failed selinv_analyze on this thread
static thread_local std::string g_analyze_err;

const char *selinv_last_error(selinv_handle h) { return h ? h->err.c_str() : g_analyze_err.c_str(); }

selinv_status selinv_analyze(int64_t n, const int64_t *colptr, const int32_t *rowind, const int32_t *perm,
                             const selinv_analyze_opts *opts, selinv_handle *out) {
    if (!out) return SELINV_E_INVALID_ARG;
    *out = nullptr;
    selinv_handle h = new (std::nothrow) selinv_handle_s();
    if (!h) return SELINV_E_NOMEM;
    h->al = current_alloc();
    h->run.al = h->al;
    h->run.hs.assign(1, h);
    const int32_t symbolic = opts ? opts->symbolic : SELINV_SYMBOLIC_SYMMETRIZED;
    if (symbolic != SELINV_SYMBOLIC_SYMMETRIZED && symbolic != SELINV_SYMBOLIC_EXACT) {
        g_analyze_err = "opts->symbolic must be SELINV_SYMBOLIC_SYMMETRIZED or SELINV_SYMBOLIC_EXACT";
        delete h;
        return SELINV_E_INVALID_ARG;
    }
    int32_t cap = opts ? opts->max_super : 0;
    int32_t relax = opts ? std::max<int32_t>(0, opts->relax) : 0;
    int32_t pad = opts ? std::min<int32_t>(100, std::max<int32_t>(0, opts->pad_pct)) : 0;
    if (cap <= 0 || cap > TRI_MAX_S) cap = TRI_MAX_S;
    const bool cplx = opts && opts->complex_values;
    selinv_status st;
    try {
        if (cplx) {
            std::vector<int64_t> cp2;
            std::vector<int32_t> ri2, pm2;
            st = complex_embedding(n, colptr, rowind, perm, cp2, ri2, pm2, h->err);
            if (!st)
                st = analyze(h->P, 2 * n, cp2.data(), ri2.data(), pm2.data(), cap, relax, pad, symbolic, h->err);
            if (!st) {
                h->cplx = true;
                h->n_c = n;
                h->nnz_c = colptr[n];
                h->colptr_c.assign(colptr, colptr + n + 1);
                // entry p = k of column j (row i): Re A^{-1}(j,i) = M^{-1}(2j, 2i) is
                // the selected value of the real-form entry (2i, 2j), Im A^{-1}(j,i)
                // = M^{-1}(2j+1, 2i) that of the entry (2i, 2j+1)
                h->aloc_c.resize(2 * h->nnz_c);
                for (int64_t j = 0; j < n; j++)
                    for (int64_t k = colptr[j]; k < colptr[j + 1]; k++) {
                        const int64_t t = k - colptr[j];
                        h->aloc_c[2 * k] = h->P.a_loc[cp2[2 * j] + 2 * t];
                        h->aloc_c[2 * k + 1] = h->P.a_loc[cp2[2 * j + 1] + 2 * t];
                    }
            }
        } else {
            st = analyze(h->P, n, colptr, rowind, perm, cap, relax, pad, symbolic, h->err);
        }
    } catch (const std::bad_alloc &) {
        st = SELINV_E_NOMEM;
        h->err = "host allocation failed in analyze";
    }
    if (st) {
        g_analyze_err = h->err;
        delete h;
        return st;
    }
    const Plan &P = h->P;
    h->sn.resize(P.ns);
    h->g_elems = 0;
    for (int32_t K = 0; K < P.ns; K++) {
        SnRec &r = h->sn[K];
        r.f = P.xsup[K];
        r.s = P.width(K);
        r.cl = (int32_t)P.cl(K);
        r.cu = (int32_t)P.cu(K);
        r.off_d = P.off_d[K];
        r.off_l = P.off_l[K];
        r.off_u = P.off_u[K];
        r.rl_off = P.rl_ptr[K];
        r.ru_off = P.ru_ptr[K];
        // every supernode has its own G block: the persistent sweep overlaps
        // levels, so blocks are not reused from one level to the next
        r.g_off = h->g_elems;
        h->g_elems += (int64_t)r.cl * r.cu;
    }
    if (h->cplx) {
        bool ok = true;
        for (int32_t K = 0; K <= P.ns && ok; K++) ok = P.xsup[K] % 2 == 0;
        auto pairs = [&](const std::vector<int64_t> &ptr, const std::vector<int32_t> &idx) {
            for (int32_t K = 0; K < P.ns; K++) {
                if ((ptr[K + 1] - ptr[K]) % 2) return false;
                for (int64_t x = ptr[K]; x < ptr[K + 1]; x += 2)
                    if (idx[x] % 2 || idx[x + 1] != idx[x] + 1) return false;
            }
            return true;
        };
        h->cpx_ok = ok && pairs(P.rl_ptr, P.rl) && pairs(P.ru_ptr, P.ru);
    }
    try {
        build_push_maps(P, h->kids_ptr, h->kids, h->push_off, h->push_pos);
        build_gather_codes(P, h->sn, h->gcL, h->gcU, kCodeBudget);
    } catch (const std::bad_alloc &) {
        g_analyze_err = "host allocation failed in analyze";
        delete h;
        return SELINV_E_NOMEM;
    }
    *out = h;
    return SELINV_OK;
}

static selinv_status ensure_device(selinv_handle h);

selinv_status selinv_factor(selinv_handle h, const double *values) {
    if (!h || !values) return SELINV_E_INVALID_ARG;
    if (h->state < 0) return SELINV_E_STATE;
    HostFactors F;
    selinv_status st;
    try {
        std::vector<double> v2;
        if (h->cplx) {
            // values of the real-equivalent form: a = x + i y becomes
            // [[x, -y], [y, x]] at rows 2i, 2i+1 of columns 2j, 2j+1
            const Plan &P = h->P;
            v2.resize(P.nnz_a);
            for (int64_t j = 0; j < h->n_c; j++)
                for (int64_t k = h->colptr_c[j]; k < h->colptr_c[j + 1]; k++) {
                    const int64_t t = k - h->colptr_c[j];
                    const double x = values[2 * k], y = values[2 * k + 1];
                    const int64_t e0 = P.a_colptr[2 * j] + 2 * t, e1 = P.a_colptr[2 * j + 1] + 2 * t;
                    v2[e0] = x;
                    v2[e0 + 1] = y;
                    v2[e1] = -y;
                    v2[e1 + 1] = x;
                }
        }
        st = factor_host(h->P, h->cplx ? v2.data() : values, F, h->err);
    } catch (const std::bad_alloc &) {
        h->err = "host allocation failed in factor";
        return SELINV_E_NOMEM;
    }
    if (st) return st;
    if ((st = ensure_device(h))) return st;
    const Plan &P = h->P;
    if (P.tot_d) HIPCHK(h->err, hipMemcpy(h->d_diag, F.d.data(), P.tot_d * 8, hipMemcpyHostToDevice), "H2D diag");
    if (P.tot_l) HIPCHK(h->err, hipMemcpy(h->d_lpan, F.l.data(), P.tot_l * 8, hipMemcpyHostToDevice), "H2D lpan");
    if (P.tot_u) HIPCHK(h->err, hipMemcpy(h->d_upan, F.u.data(), P.tot_u * 8, hipMemcpyHostToDevice), "H2D upan");
    h->state = 1;
    return SELINV_OK;
}

// Factor storage and plan metadata on the current device (first factor call).
static selinv_status ensure_device(selinv_handle h) {
    int dev = 0;
    HIPCHK(h->err, hipGetDevice(&dev), "hipGetDevice");
    if (h->device >= 0 && h->device != dev) {
        h->err = "factor called on a different device than before";
        return SELINV_E_STATE;
    }
    h->device = dev;
    const Plan &P = h->P;
    if (!h->d_diag) {
        HIPCHK(h->err, alloc_bytes(h->al, (void **)&h->d_diag, P.tot_d * 8), "alloc diag");
        HIPCHK(h->err, alloc_bytes(h->al, (void **)&h->d_lpan, P.tot_l * 8), "alloc lpan");
        HIPCHK(h->err, alloc_bytes(h->al, (void **)&h->d_upan, P.tot_u * 8), "alloc upan");
        HIPCHK(h->err, alloc_bytes(h->al, (void **)&h->d_Linv, P.tot_d * 8), "alloc Linv");
        HIPCHK(h->err, alloc_bytes(h->al, (void **)&h->d_Uinv, P.tot_d * 8), "alloc Uinv");
        HIPCHK(h->err, alloc_bytes(h->al, (void **)&h->d_tl, P.tot_d * 8), "alloc tri scratch");
        HIPCHK(h->err, alloc_bytes(h->al, (void **)&h->d_tu, P.tot_d * 8), "alloc tri scratch");
        HIPCHK(h->err, upload(h->al, &h->d_sn, h->sn), "upload sn");
        HIPCHK(h->err, upload(h->al, &h->d_supof, P.supof), "upload supof");
        HIPCHK(h->err, upload(h->al, &h->d_rl, P.rl), "upload rl");
        HIPCHK(h->err, upload(h->al, &h->d_ru, P.ru), "upload ru");
        HIPCHK(h->err, upload(h->al, &h->d_mapL, P.mapL), "upload mapL");
        HIPCHK(h->err, upload(h->al, &h->d_mapU, P.mapU), "upload mapU");
        HIPCHK(h->err, upload(h->al, &h->d_lcol, P.l_coloff), "upload l_coloff");
        HIPCHK(h->err, upload(h->al, &h->d_urow, P.u_rowoff), "upload u_rowoff");
        HIPCHK(h->err, upload(h->al, &h->d_aloc, P.a_loc), "upload a_loc");
        if (h->cplx) HIPCHK(h->err, upload(h->al, &h->d_aloc_c, h->aloc_c), "upload complex locations");
        HIPCHK(h->err, upload(h->al, &h->d_kids_ptr, h->kids_ptr), "upload children");
        HIPCHK(h->err, upload(h->al, &h->d_kids, h->kids), "upload children");
        HIPCHK(h->err, upload(h->al, &h->d_push_off, h->push_off), "upload push maps");
        HIPCHK(h->err, upload(h->al, &h->d_push_pos, h->push_pos), "upload push maps");
        HIPCHK(h->err, upload(h->al, &h->d_gcL, h->gcL), "upload gather codes");
        HIPCHK(h->err, upload(h->al, &h->d_gcU, h->gcU), "upload gather codes");
        {
            // row and column source records of the gather tiles (see MatDev)
            std::vector<int32_t> rI(P.rl.size()), cJ(P.ru.size());
            std::vector<int64_t> rUp(P.rl.size()), cD(P.ru.size()), cLw(P.ru.size());
            for (size_t x = 0; x < P.rl.size(); x++) {
                const int32_t r = P.rl[x], I = P.supof[r];
                const SnRec &q = h->sn[I];
                rI[x] = I;
                rUp[x] = q.off_u + (int64_t)(r - q.f) * q.cu;
            }
            for (size_t y = 0; y < P.ru.size(); y++) {
                const int32_t c = P.ru[y], J = P.supof[c];
                const SnRec &q = h->sn[J];
                cJ[y] = J;
                cD[y] = q.off_d + (int64_t)(c - q.f) * q.s - q.f;
                cLw[y] = q.off_l + (int64_t)(c - q.f) * q.cl;
            }
            HIPCHK(h->err, upload(h->al, &h->d_row_I, rI), "upload gather records");
            HIPCHK(h->err, upload(h->al, &h->d_row_up, rUp), "upload gather records");
            HIPCHK(h->err, upload(h->al, &h->d_col_J, cJ), "upload gather records");
            HIPCHK(h->err, upload(h->al, &h->d_col_diag, cD), "upload gather records");
            HIPCHK(h->err, upload(h->al, &h->d_col_low, cLw), "upload gather records");
        }
    }
    return SELINV_OK;
}

// Work lists of the device LU.  Every operand range of a tile LU, tile
// inverse or product is checked on the host against its supernode's segment of
// the factor storage, and every destination of a Schur complement entry
// against the segment and the level of the supernode that holds it, before
// anything is uploaded.
static selinv_status build_lu(selinv_handle h) {
    const Plan &P = h->P;
    auto L = std::make_unique<LuPlan>();
    L->al = h->al;
    std::vector<LuTile> lus;
    std::vector<TriItem> tris;
    std::vector<GemmProb> probs;
    std::vector<GemmTile> tiles;
    std::vector<GatherTile> scs;
    bool ok = true;
    // elements [off, off + last] inside [seg, seg + len)
    auto inside = [&](int64_t off, int64_t last, int64_t seg, int64_t len) {
        if (off < seg || last < 0 || off + last >= seg + len) ok = false;
    };
    // W_K of one level, packed: the largest level decides the buffer
    int64_t w_max = 0;
    for (int32_t lev = 0; lev < P.nlevels; lev++) {
        int64_t w = 0;
        for (int32_t K : P.levels[lev]) w += (int64_t)h->sn[K].cl * h->sn[K].cu;
        w_max = std::max(w_max, w);
    }
    HIPCHK(h->err, alloc_bytes(L->al, (void **)&L->d_W, w_max * 8), "alloc Schur complement buffer");
    double *D0 = h->d_diag, *L0 = h->d_lpan, *U0 = h->d_upan, *W0 = L->d_W;
    double *Li0 = h->d_Linv, *Ui0 = h->d_Uinv;  // the tile inverses (the run recomputes them)
    // C = alpha op(A) op(B) + beta C
    auto gemm = [&](const double *A, int64_t lda, int opA, const double *B, int64_t ldb, int opB, double *C,
                    int64_t ldc, int M, int N, int K, double alpha, double beta) {
        GemmProb g{};
        g.A = A;
        g.B = B;
        g.C = C;
        g.Cin = beta != 0.0 ? C : nullptr;
        g.M = M;
        g.N = N;
        g.K = K;
        g.lda = (int32_t)lda;
        g.ldb = (int32_t)ldb;
        g.ldc = g.ldcin = (int32_t)ldc;
        g.opA = opA;
        g.opB = opB;
        g.push_sn = g.push_mat = -1;
        g.alpha = alpha;
        g.beta = beta;
        add_tiles(tiles, (int)probs.size(), M, N, GEMM_TILE_64);
        probs.push_back(g);
    };
    auto mark = [&](int kind, size_t first, size_t end) {
        if (end > first) L->launches.push_back({kind, (int64_t)first, (int)(end - first)});
    };
    for (int32_t lev = P.nlevels - 1; lev >= 0; lev--) {
        const std::vector<int32_t> &Ks = P.levels[lev];
        int smax = 0;
        for (int32_t K : Ks) smax = std::max(smax, h->sn[K].s);
        for (int j0 = 0; j0 < smax; j0 += 64) {
            // solves first (launch L_SOLVE), trailing updates after them
            const size_t l0 = lus.size(), t0 = tris.size(), g0 = tiles.size();
            struct Upd {
                const double *A;
                int64_t lda;
                int opA;
                const double *B;
                int64_t ldb;
                int opB;
                double *C;
                int64_t ldc;
                int M, N, K;
            };
            std::vector<Upd> upd;
            for (int32_t K : Ks) {
                const SnRec &r = h->sn[K];
                const int s = r.s, cl = r.cl, cu = r.cu;
                if (s <= j0) continue;
                const int b = std::min(64, s - j0), rest = s - j0 - b;
                const int64_t ss = (int64_t)s * s, ld = s;
                double *D = D0 + r.off_d;
                const int64_t tile = j0 + j0 * ld;
                inside(r.off_d + tile, (b - 1) + (b - 1) * ld, r.off_d, ss);
                lus.push_back(LuTile{D, s, j0, r.f, 0});
                TriItem ti{};
                ti.D = D;
                ti.Linv = Li0 + r.off_d;
                ti.Uinv = Ui0 + r.off_d;
                ti.s = s;
                ti.j0 = j0;
                tris.push_back(ti);
                const double *Lt = Li0 + r.off_d + tile, *Ut = Ui0 + r.off_d + tile;
                // solves, in place: every product has one 64-wide tile along
                // the solved dimension, so each workgroup reads only the rows
                // (columns) it writes
                if (rest > 0) {
                    const int64_t l21 = (j0 + b) + j0 * ld, u12 = j0 + (j0 + b) * ld, c22 = (j0 + b) * (1 + ld);
                    inside(r.off_d + l21, (rest - 1) + (b - 1) * ld, r.off_d, ss);
                    inside(r.off_d + u12, (b - 1) + (rest - 1) * ld, r.off_d, ss);
                    inside(r.off_d + c22, (rest - 1) + (rest - 1) * ld, r.off_d, ss);
                    gemm(D + l21, ld, 0, Ut, ld, 0, D + l21, ld, rest, b, b, 1.0, 0.0);  // L21 = A21 U11^{-1}
                    gemm(Lt, ld, 0, D + u12, ld, 0, D + u12, ld, b, rest, b, 1.0, 0.0);  // U12 = L11^{-1} A12
                    upd.push_back({D + l21, ld, 0, D + u12, ld, 0, D + c22, ld, rest, rest, b});
                }
                if (cl > 0) {  // L(R_L, K) columns of the tile: A U11^{-1}; later columns -= them U12
                    const int64_t a = r.off_l + (int64_t)j0 * cl;
                    inside(a, (cl - 1) + (int64_t)(b - 1) * cl, r.off_l, (int64_t)cl * s);
                    gemm(L0 + a, cl, 0, Ut, ld, 0, L0 + a, cl, cl, b, b, 1.0, 0.0);
                    if (rest > 0) {
                        const int64_t c = r.off_l + (int64_t)(j0 + b) * cl;
                        inside(c, (cl - 1) + (int64_t)(rest - 1) * cl, r.off_l, (int64_t)cl * s);
                        upd.push_back({L0 + a, cl, 0, D + j0 + (j0 + b) * ld, ld, 0, L0 + c, cl, cl, rest, b});
                    }
                }
                if (cu > 0) {  // U(K, R_U)^T columns of the tile: A L11^{-T}; later columns -= them L21^T
                    const int64_t a = r.off_u + (int64_t)j0 * cu;
                    inside(a, (cu - 1) + (int64_t)(b - 1) * cu, r.off_u, (int64_t)cu * s);
                    gemm(U0 + a, cu, 0, Lt, ld, 1, U0 + a, cu, cu, b, b, 1.0, 0.0);
                    if (rest > 0) {
                        const int64_t c = r.off_u + (int64_t)(j0 + b) * cu;
                        inside(c, (cu - 1) + (int64_t)(rest - 1) * cu, r.off_u, (int64_t)cu * s);
                        upd.push_back({U0 + a, cu, 0, D + (j0 + b) + j0 * ld, ld, 1, U0 + c, cu, cu, rest, b});
                    }
                }
            }
            mark(LuPlan::L_TILES, l0, lus.size());
            mark(LuPlan::L_TRI, t0, tris.size());
            mark(LuPlan::L_SOLVE, g0, tiles.size());
            const size_t g1 = tiles.size();
            for (const Upd &u : upd) gemm(u.A, u.lda, u.opA, u.B, u.ldb, u.opB, u.C, u.ldc, u.M, u.N, u.K, -1.0, 1.0);
            mark(LuPlan::L_UPDATE, g1, tiles.size());
        }
        // W_K = -L(R_L, K) U(K, R_U) and its scatter into the ancestors
        const size_t g0 = tiles.size(), c0 = scs.size();
        int64_t w = 0;
        for (int32_t K : Ks) {
            const SnRec &r = h->sn[K];
            const int s = r.s, cl = r.cl, cu = r.cu;
            if (cl == 0 || cu == 0) continue;
            inside(w, (int64_t)cl * cu - 1, 0, w_max);
            gemm(L0 + r.off_l, cl, 0, U0 + r.off_u, cu, 1, W0 + w, cl, cl, cu, s, -1.0, 0.0);
            for (int a0 = 0; a0 < cl; a0 += 64)
                for (int b0 = 0; b0 < cu; b0 += 64) scs.push_back(GatherTile{0, K, a0, b0, -1, cl, cu, 0, w, -1, 0, 0, 0, 0});
            // destinations of every entry of W_K
            const int32_t *RL = P.rl.data() + P.rl_ptr[K], *RU = P.ru.data() + P.ru_ptr[K];
            for (int b2 = 0; b2 < cu && ok; b2++) {
                const int32_t c = RU[b2], J = P.supof[c];
                for (int a = 0; a < cl; a++) {
                    const int32_t rr = RL[a], I = P.supof[rr];
                    const int32_t Q = std::min(I, J);
                    if (P.level[Q] >= lev) ok = false;
                    if (I == J) {
                        if (c < P.xsup[J] || c >= P.xsup[J + 1] || rr < P.xsup[J] || rr >= P.xsup[J + 1]) ok = false;
                    } else if (I > J) {
                        const int64_t m = P.l_coloff[P.ru_ptr[K] + b2] + a;
                        if (m < 0 || m >= (int64_t)P.mapL.size() || P.mapL[m] < 0 || P.mapL[m] >= P.cl(J)) ok = false;
                    } else {
                        const int64_t m = P.u_rowoff[P.rl_ptr[K] + a] + b2;
                        if (m < 0 || m >= (int64_t)P.mapU.size() || P.mapU[m] < 0 || P.mapU[m] >= P.cu(I)) ok = false;
                    }
                }
            }
            w += (int64_t)cl * cu;
        }
        mark(LuPlan::L_SCHUR, g0, tiles.size());
        mark(LuPlan::L_SCATTER, c0, scs.size());
    }
    if (!ok) {
        h->err = "device LU: work list outside the factor storage (inconsistent analysis)";
        return SELINV_E_STATE;
    }
    HIPCHK(h->err, upload(L->al, &L->d_lu, lus), "upload LU tiles");
    HIPCHK(h->err, upload(L->al, &L->d_tri, tris), "upload tile inverses");
    HIPCHK(h->err, upload(L->al, &L->d_probs, probs), "upload LU products");
    HIPCHK(h->err, upload(L->al, &L->d_tiles, tiles), "upload LU product tiles");
    HIPCHK(h->err, upload(L->al, &L->d_sc, scs), "upload scatter tiles");
    MatDev m{};
    m.sn = h->d_sn;
    m.supof = h->d_supof;
    m.rl = h->d_rl;
    m.ru = h->d_ru;
    m.l_coloff = h->d_lcol;
    m.u_rowoff = h->d_urow;
    m.mapL = h->d_mapL;
    m.mapU = h->d_mapU;
    HIPCHK(h->err, upload(L->al, &L->d_mat, std::vector<MatDev>{m}), "upload LU matrix record");
    HIPCHK(h->err, alloc_bytes(L->al, (void **)&L->d_bad, sizeof(int32_t)), "alloc pivot flag");
    if (h->cplx) {
        // entry e of the real form: +-(Re or Im) of complex entry k, as in selinv_factor
        std::vector<int64_t> emb(P.nnz_a, 0);
        for (int64_t j = 0; j < h->n_c; j++)
            for (int64_t k = h->colptr_c[j]; k < h->colptr_c[j + 1]; k++) {
                const int64_t t = k - h->colptr_c[j];
                const int64_t e0 = P.a_colptr[2 * j] + 2 * t, e1 = P.a_colptr[2 * j + 1] + 2 * t;
                emb[e0] = (2 * k) << 1;
                emb[e0 + 1] = (2 * k + 1) << 1;
                emb[e1] = ((2 * k + 1) << 1) | 1;
                emb[e1 + 1] = (2 * k) << 1;
            }
        HIPCHK(h->err, upload(L->al, &L->d_emb, emb), "upload complex entry map");
    }
    h->lu = std::move(L);
    return SELINV_OK;
}

selinv_status selinv_factor_device(selinv_handle h, const double *values, void *stream) {
    if (!h || !values) return SELINV_E_INVALID_ARG;
    if (h->state < 0) return SELINV_E_STATE;
    selinv_status st;
    if ((st = ensure_device(h))) return st;
    {
        hipPointerAttribute_t attr;
        const hipError_t e = hipPointerGetAttributes(&attr, values);
        if (e != hipSuccess || (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) ||
            attr.device != h->device) {
            (void)hipGetLastError();
            h->err = "factor_device: values is not device memory of the handle's device";
            return SELINV_E_INVALID_ARG;
        }
    }
    try {
        if (!h->lu && (st = build_lu(h))) return st;
    } catch (const std::bad_alloc &) {
        h->err = "host allocation failed in factor_device";
        return SELINV_E_NOMEM;
    }
    const Plan &P = h->P;
    LuPlan &L = *h->lu;
    hipStream_t s = (hipStream_t)stream;
    h->state = 0;  // the factor storage is rewritten from here on
    HIPCHK(h->err, hipMemsetAsync(h->d_diag, 0, P.tot_d * 8, s), "clear diag");
    HIPCHK(h->err, hipMemsetAsync(h->d_lpan, 0, P.tot_l * 8, s), "clear lpan");
    HIPCHK(h->err, hipMemsetAsync(h->d_upan, 0, P.tot_u * 8, s), "clear upan");
    HIPCHK(h->err, hipMemsetAsync(L.d_bad, 0x7f, sizeof(int32_t), s), "clear pivot flag");
    HIPCHK(h->err, launch_scatter_values(h->d_aloc, values, L.d_emb, P.nnz_a, h->d_diag, h->d_lpan, h->d_upan, s),
           "scatter values");
    for (const LuPlan::Launch &l : L.launches) {
        hipError_t e = hipSuccess;
        switch (l.kind) {
            case LuPlan::L_TILES: e = launch_lu_tiles(L.d_lu + l.first, l.count, L.d_bad, s); break;
            case LuPlan::L_TRI: e = launch_tri_base(L.d_tri + l.first, l.count, 4, s); break;
            case LuPlan::L_SOLVE:
                e = launch_gemm(GEMM_PRO_F64, CMP_F64, GEMM_TILE_64, L.d_probs, L.d_tiles + l.first, l.count, s);
                break;
            case LuPlan::L_UPDATE:
                e = launch_gemm(GEMM_STEP4, CMP_F64, GEMM_TILE_64, L.d_probs, L.d_tiles + l.first, l.count, s);
                break;
            case LuPlan::L_SCHUR:
                e = launch_gemm(GEMM_PRO_F64, CMP_F64, GEMM_TILE_64, L.d_probs, L.d_tiles + l.first, l.count, s);
                break;
            default:
                e = launch_scatter_update(L.d_mat, L.d_sc + l.first, l.count, L.d_W, h->d_diag, h->d_lpan,
                                          h->d_upan, s);
        }
        HIPCHK(h->err, e, "device LU launch");
    }
    int32_t bad = 0;
    HIPCHK(h->err, hipMemcpyAsync(&bad, L.d_bad, sizeof(bad), hipMemcpyDeviceToHost, s), "pivot flag");
    HIPCHK(h->err, hipStreamSynchronize(s), "device LU");
    if (bad != 0x7f7f7f7f) {
        h->err = "zero or non-finite pivot at permuted column " + std::to_string(bad) + " (original column " +
                 std::to_string(bad >= 0 && bad < (int32_t)P.p.size() ? P.p[bad] : -1) + ")";
        return SELINV_E_ZERO_PIVOT;
    }
    h->state = 1;
    return SELINV_OK;
}

static selinv_status check_run(selinv_handle h, int prec) {
    if (!h || !valid_prec(prec)) return SELINV_E_INVALID_ARG;
    if (h->state < 1) {
        h->err = "run before factor";
        return SELINV_E_STATE;
    }
    int dev = 0;
    HIPCHK(h->err, hipGetDevice(&dev), "hipGetDevice");
    if (dev != h->device) {
        h->err = "run on a different device than factor";
        return SELINV_E_STATE;
    }
    return SELINV_OK;
}

// ---------------------------------------------------------------------------
// runs over a Runner (one handle, or a batch)
// ---------------------------------------------------------------------------
static selinv_status runner_ensure(Runner &R, int prec, std::string &err) {
    if (R.sweep[prec]) return SELINV_OK;
    return build_sweep(R.hs, R.al, prec, R.sweep_mode, R.sweep[prec], err, &R.tune[prec], R.gather_form);
}

static void runner_drop(Runner &R, int prec) {
    for (auto h : R.hs)
        if (h->last_sweep == R.sweep[prec].get()) h->last_sweep = nullptr;
    R.sweep[prec].reset();
    if (R.last_prec == prec) R.last_profiled = false;
}

// One sweep of `prec` on stream s: eager launches (with one event after each
// phase while profiling is on) or a replay of the HIP graph recorded from
// them at the first graph run.
static selinv_status runner_launch(Runner &R, int prec, hipStream_t s, bool graph, std::string &err) {
    selinv_status st = runner_ensure(R, prec, err);
    if (st) return st;
    Sweep &S = *R.sweep[prec];
    bool profiled = false;
    if (graph) {
        if (!s) {  // graphs are not captured on the legacy null stream
            if (!R.own_stream) HIPCHK(err, hipStreamCreateWithFlags(&R.own_stream, hipStreamNonBlocking), "stream");
            s = R.own_stream;
        }
        if (!S.gexec) {
            HIPCHK(err, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
            hipError_t e = launch_sweep(S, s, nullptr);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(s, &g);
            if (e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return dev_fail(err, e, "capture launch");
            }
            if (e2 != hipSuccess) return dev_fail(err, e2, "end capture");
            S.graph = g;
            HIPCHK(err, hipGraphInstantiate(&S.gexec, g, nullptr, nullptr, 0), "graph instantiate");
        }
        HIPCHK(err, hipGraphLaunch(S.gexec, s), "graph launch");
    } else {
        std::vector<hipEvent_t> *ev = nullptr;
        if (R.profiling) {
            const size_t need = 4 + 4 * S.gat.size();
            while (R.events.size() < need) {
                hipEvent_t e;
                HIPCHK(err, hipEventCreate(&e), "hipEventCreate");
                R.events.push_back(e);
            }
            ev = &R.events;
            profiled = true;
        }
        hipError_t e = launch_sweep(S, s, ev);
        if (e != hipSuccess) return dev_fail(err, e, "kernel launch");
    }
    for (auto h : R.hs) {
        h->last_sweep = &S;
        h->last_prec = prec;
        h->last_stream = s;
        h->last_profiled = profiled && R.hs.size() == 1;
        h->state = 2;
    }
    R.last_prec = prec;
    R.last_profiled = profiled;
    return SELINV_OK;
}

// Event intervals of the runner's last profiled run (see selinv_timings).
static selinv_status runner_timings(Runner &R, double *ms, int32_t count, std::string &err) {
    if (R.last_prec < 0 || !R.last_profiled || !R.sweep[R.last_prec]) {
        err = "no profiled run";
        return SELINV_E_STATE;
    }
    const Sweep &S = *R.sweep[R.last_prec];
    size_t nev = 4 + 4 * S.gat.size();
    if (R.events.size() < nev) return SELINV_E_STATE;
    HIPCHK(err, hipEventSynchronize(R.events[nev - 1]), "event sync");
    for (int32_t i = 0; i < count; i++) {
        if ((size_t)i + 1 >= nev) {
            ms[i] = 0;
            continue;
        }
        float t = 0;
        HIPCHK(err, hipEventElapsedTime(&t, R.events[i], R.events[i + 1]), "elapsed");
        ms[i] = t;
    }
    return SELINV_OK;
}

static void level_stats_of(const Sweep &S, int32_t level, double *stats) {
    stats[0] = S.lev_nsup[level];
    stats[1] = S.lev_maxs[level];
    stats[2] = S.lev_flops35[level];
    stats[3] = S.lev_flops4[level];
    stats[4] = S.lev_gather_elems[level];
    stats[5] = S.gat[level].count;
    stats[6] = S.g35[level].count;
    stats[7] = S.g4[level].count;
    stats[8] = S.g35[level].tile;
    stats[9] = S.g4[level].tile;
    stats[10] = S.small[level].count;
    stats[11] = S.lev_small_flops[level];
    stats[12] = S.lev_small_elems[level];
    stats[13] = S.vg[level] ? 2 : S.fused[level];
    stats[14] = S.lev_bytes35[level];
    stats[15] = S.lev_bytes4[level];
    stats[16] = S.lev_bytes_gather[level];
    stats[17] = S.lev_bytes_small[level];
    stats[18] = S.lev_max_prod[level];
}

static selinv_status sweep_level_stats(const Sweep &S, int32_t level, double *stats) {
    if (level == -1) {
        for (int k = 0; k < 19; k++) stats[k] = 0;
        for (int k = 0; k < 3; k++) {
            stats[2 * k] = S.pro_flops[k];
            stats[2 * k + 1] = S.pro_bytes[k];
        }
        return SELINV_OK;
    }
    if (level < 0 || level >= (int32_t)S.gat.size()) return SELINV_E_INVALID_ARG;
    level_stats_of(S, level, stats);
    return SELINV_OK;
}

// Runs the sweep of `prec` reps + 1 times (the first untimed) under the
// runner's current tuning.  total: fastest run in ms (HIP events on `s`
// around a replay of the sweep's HIP graph, or around the eager launches of a
// profiled run); phase (profiled runs): fastest time of every event interval
// of the profiled sweep.
static selinv_status tune_measure(Runner &R, int prec, hipStream_t s, int reps, bool profiled, double &total,
                                  std::vector<double> *phase, std::string &err) {
    runner_drop(R, prec);
    selinv_status st = runner_ensure(R, prec, err);
    if (st) return st;
    const bool was = R.profiling;
    R.profiling = profiled;
    hipEvent_t a = nullptr, b = nullptr;
    auto done = [&](selinv_status r) {
        R.profiling = was;
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        return r;
    };
    hipError_t ec = hipEventCreate(&a);
    if (ec == hipSuccess) ec = hipEventCreate(&b);
    if (ec != hipSuccess) return done(dev_fail(err, ec, "hipEventCreate"));
    const int nint = 3 + 4 * (int)R.sweep[prec]->gat.size();
    total = 1e300;
    if (phase) phase->assign(nint, 1e300);
    std::vector<double> t(nint);
    hipError_t e;
    for (int r = 0; r <= reps; r++) {
        if ((e = hipEventRecord(a, s)) != hipSuccess) return done(dev_fail(err, e, "event record"));
        if ((st = runner_launch(R, prec, s, !profiled, err))) return done(st);
        if ((e = hipEventRecord(b, s)) != hipSuccess) return done(dev_fail(err, e, "event record"));
        if ((e = hipEventSynchronize(b)) != hipSuccess) return done(dev_fail(err, e, "event sync"));
        if (r == 0) continue;
        float ms = 0;
        if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) return done(dev_fail(err, e, "elapsed"));
        total = std::min(total, (double)ms);
        if (phase) {
            if ((st = runner_timings(R, t.data(), nint, err))) return done(st);
            for (int i = 0; i < nint; i++) (*phase)[i] = std::min((*phase)[i], t[i]);
        }
    }
    return done(SELINV_OK);
}

// The autotuner (selinv_tune / selinv_batch_tune); stream s is not the null stream.
static selinv_status runner_tune(Runner &R, int prec, int32_t reps, hipStream_t s, double *ms_policy,
                                 double *ms_tuned, std::string &err) {
    if (reps < 1 || reps > 100) {
        err = "reps must be in 1..100";
        return SELINV_E_INVALID_ARG;
    }
    selinv_status st;
    const int L = R.depth();
    const bool can_persist = R.sweep_mode == SWEEP_AUTO;
    // the size policy, in the runner's own sweep form
    R.tune[prec] = Tuning();
    double t_policy = 0, t = 0;
    if ((st = tune_measure(R, prec, s, reps, false, t_policy, nullptr, err))) return st;

    // 1. tile edge of every launch class: the whole level sweep profiled once
    //    per candidate edge, every class keeps its fastest edge
    Tuning best;
    best.set = true;
    best.t35.assign(L, 0);
    best.t4.assign(L, 0);
    best.no_small.assign(L, 0);
    best.vg.assign(L, 0);
    best.sweep = R.sweep_mode == SWEEP_AUTO ? SWEEP_LEVELS : SWEEP_AUTO;
    const int cand[3] = {GEMM_TILE_32, GEMM_TILE_64, GEMM_TILE_128};
    std::vector<double> bt(3 + 2 * L, 1e300);
    std::vector<double> ph;
    for (int c : cand) {
        Tuning tn = best;
        tn.tri = tn.norm = tn.dt = c;
        std::fill(tn.t35.begin(), tn.t35.end(), c);
        std::fill(tn.t4.begin(), tn.t4.end(), c);
        tn.sweep = SWEEP_LEVELS;
        R.tune[prec] = tn;
        if ((st = tune_measure(R, prec, s, reps, true, t, &ph, err))) return st;
        auto keep = [&](int k, double v, int &slot) {
            if (v < bt[k]) {
                bt[k] = v;
                slot = c;
            }
        };
        // event intervals: tri, norm, dt, then per level small, gather, steps 3+5,
        // step 4.  A step-4 edge counts with the next level's gather, which
        // runs in the step-4 launch or (after 128-wide tiles) in its own.
        keep(0, ph[0], best.tri);
        keep(1, ph[1], best.norm);
        keep(2, ph[2], best.dt);
        for (int d = 0; d < L; d++) {
            keep(3 + 2 * d, ph[3 + 4 * d + 2], best.t35[d]);
            keep(4 + 2 * d, ph[3 + 4 * d + 3] + (d + 1 < L ? ph[3 + 4 * (d + 1) + 1] : 0.0), best.t4[d]);
        }
    }
    // 2. levels made only of small supernodes: the fused small-supernode
    //    launch or the per-phase launches, compared on the level's own
    //    intervals plus the step-4 launch above it (which takes over the
    //    level's gather when both levels use the per-phase launches)
    {
        Tuning on = best, off = best;
        on.sweep = off.sweep = SWEEP_LEVELS;
        std::fill(off.no_small.begin(), off.no_small.end(), 1);
        std::vector<double> pon, poff;
        R.tune[prec] = on;
        if ((st = tune_measure(R, prec, s, reps, true, t, &pon, err))) return st;
        R.tune[prec] = off;
        if ((st = tune_measure(R, prec, s, reps, true, t, &poff, err))) return st;
        for (int d = 0; d < L; d++) {
            auto lev = [&](const std::vector<double> &p) {
                double v = 0;
                for (int i = 0; i < 4; i++) v += p[3 + 4 * d + i];
                if (d > 0) v += p[3 + 4 * (d - 1) + 3];
                return v;
            };
            best.no_small[d] = lev(poff) < 0.97 * lev(pon);
        }
    }
    // 2b. levels of large supernodes: a stored G (gather launch or the gather
    //     tiles in the step-4 launch above) or G_K read from its sources by
    //     the step-3/5 products, compared as in 2.  Only under the tuning's
    //     own choice of gather form, and only for a level sweep.
    if (R.gather_form == 0 && R.sweep_mode != SWEEP_PERSISTENT) {
        Tuning on = best, off = best;
        on.sweep = off.sweep = SWEEP_LEVELS;
        std::fill(on.vg.begin(), on.vg.end(), 1);
        std::vector<double> pon, poff;
        R.tune[prec] = on;
        if ((st = tune_measure(R, prec, s, reps, true, t, &pon, err))) return st;
        R.tune[prec] = off;
        if ((st = tune_measure(R, prec, s, reps, true, t, &poff, err))) return st;
        for (int d = 0; d < L; d++) {
            auto lev = [&](const std::vector<double> &p) {
                double v = 0;
                for (int i = 0; i < 4; i++) v += p[3 + 4 * d + i];
                if (d > 0) v += p[3 + 4 * (d - 1) + 3];
                return v;
            };
            best.vg[d] = lev(pon) < 0.97 * lev(poff);
        }
    }
    // 3. the sweep form, where the persistent sweep is available
    R.tune[prec] = best;
    double t_best = 0;
    if ((st = tune_measure(R, prec, s, reps, false, t_best, nullptr, err))) return st;
    if (can_persist) {
        Tuning pe = best;
        pe.sweep = SWEEP_PERSISTENT;
        R.tune[prec] = pe;
        if ((st = tune_measure(R, prec, s, reps, false, t, nullptr, err))) return st;
        if (t < t_best) {
            best = pe;
            t_best = t;
        }
    }
    // 4. the prologue of the lower levels beside the upper levels (side
    //    stream), also cut into one part per upper level, or entirely before
    //    the sweep
    for (int nf_form : {2, 1}) {
        Tuning nf = best;
        nf.no_fork = nf_form;
        R.tune[prec] = nf;
        if ((st = tune_measure(R, prec, s, reps, false, t, nullptr, err))) return st;
        if (t < t_best) {
            best = nf;
            t_best = t;
        }
    }
    // 5. with a side stream: its tile inversions on a number of workgroups
    //    that is a multiple of the compute-unit count (from a quarter of it,
    //    which leaves compute units free for the upper levels' launches, to
    //    three times), or one workgroup per item
    if (best.no_fork != 1) {
        R.tune[prec] = best;
        runner_drop(R, prec);
        if ((st = runner_ensure(R, prec, err))) return st;
        int cus = 0;
        HIPCHK(err, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, R.hs[0]->device),
               "device attribute");
        if (R.sweep[prec]->split > 0 && cus > 0) {
            for (int q : {1, 2, 3, 4, 5, 6, 7, 8, 10, 12}) {
                Tuning ch = best;
                ch.side_chunk = q * cus / 4;
                R.tune[prec] = ch;
                if ((st = tune_measure(R, prec, s, reps, false, t, nullptr, err))) return st;
                if (t < t_best) {
                    best = ch;
                    t_best = t;
                }
            }
        }
    }
    // 6. keep the size policy when the measured choices are no faster
    if (t_best > t_policy) {
        Tuning pol;
        pol.set = true;
        pol.t35.assign(L, 0);
        pol.t4.assign(L, 0);
        pol.no_small.assign(L, 0);
        pol.vg.assign(L, 0);
        best = pol;
        t_best = t_policy;
    }
    R.tune[prec] = best;
    runner_drop(R, prec);
    if (ms_policy) *ms_policy = t_policy;
    if (ms_tuned) *ms_tuned = t_best;
    return SELINV_OK;
}

// flat form: [4, nlevels, sweep, tri, norm, dt, no_fork, side_chunk, then per
// level: t35, t4, no_small, vg] (tables of the earlier layouts are still
// accepted: 3 without vg, 2 without side_chunk as well, 1 without no_fork)
static selinv_status runner_get_tuning(const Runner &R, int prec, int32_t *out, int32_t cap, int32_t *count,
                                       std::string &err) {
    const Tuning &tn = R.tune[prec];
    const int L = R.depth();
    *count = tn.set ? 8 + 4 * L : 0;
    if (!tn.set || !out) return SELINV_OK;
    if (cap < *count) {
        err = "tuning buffer too small";
        return SELINV_E_INVALID_ARG;
    }
    int32_t *o = out;
    *o++ = 4;
    *o++ = L;
    *o++ = tn.sweep;
    *o++ = tn.tri;
    *o++ = tn.norm;
    *o++ = tn.dt;
    *o++ = tn.no_fork;
    *o++ = tn.side_chunk;
    for (int d = 0; d < L; d++) {
        *o++ = tn.t35[d];
        *o++ = tn.t4[d];
        *o++ = tn.no_small[d];
        *o++ = d < (int)tn.vg.size() ? tn.vg[d] : 0;
    }
    return SELINV_OK;
}

static selinv_status runner_set_tuning(Runner &R, int prec, const int32_t *in, int32_t count, std::string &err) {
    if (count == 0) {  // back to the size policy
        R.tune[prec] = Tuning();
        runner_drop(R, prec);
        return SELINV_OK;
    }
    const int L = R.depth();
    auto tile_ok = [](int v) { return v == 0 || v == GEMM_TILE_32 || v == GEMM_TILE_64 || v == GEMM_TILE_128; };
    const int ver = in && count > 0 ? in[0] : 0, hd = ver >= 3 ? 8 : ver == 2 ? 7 : 6, pl = ver == 4 ? 4 : 3;
    bool ok = in && ver >= 1 && ver <= 4 && count == hd + pl * L && in[1] == L && in[2] >= SWEEP_AUTO &&
              in[2] <= SWEEP_PERSISTENT && tile_ok(in[3]) && tile_ok(in[4]) && tile_ok(in[5]) &&
              (ver == 1 || in[6] == 0 || in[6] == 1 || (ver == 4 && in[6] == 2)) &&
              (ver < 3 || (in[7] >= 0 && in[7] <= (1 << 20)));
    for (int d = 0; ok && d < L; d++)
        ok = tile_ok(in[hd + pl * d]) && tile_ok(in[hd + 1 + pl * d]) &&
             (in[hd + 2 + pl * d] == 0 || in[hd + 2 + pl * d] == 1) &&
             (pl == 3 || in[hd + 3 + pl * d] == 0 || in[hd + 3 + pl * d] == 1);
    if (!ok) {
        err = "tuning table does not fit (layout, level count, tile edges or sweep form)";
        return SELINV_E_INVALID_ARG;
    }
    Tuning tn;
    tn.set = true;
    tn.sweep = in[2];
    tn.tri = in[3];
    tn.norm = in[4];
    tn.dt = in[5];
    tn.no_fork = ver >= 2 ? in[6] : 0;
    tn.side_chunk = ver >= 3 ? in[7] : 0;
    for (int d = 0; d < L; d++) {
        tn.t35.push_back(in[hd + pl * d]);
        tn.t4.push_back(in[hd + 1 + pl * d]);
        tn.no_small.push_back((char)in[hd + 2 + pl * d]);
        tn.vg.push_back(pl == 4 ? (char)in[hd + 3 + pl * d] : 0);
    }
    R.tune[prec] = tn;
    runner_drop(R, prec);
    return SELINV_OK;
}

static selinv_status runner_set_gather_form(Runner &R, int32_t form) {
    if (form < 0 || form > 2) return SELINV_E_INVALID_ARG;
    if (form != R.gather_form) {
        R.gather_form = form;
        for (int p = 0; p < NPREC; p++) runner_drop(R, p);
    }
    return SELINV_OK;
}

static selinv_status runner_set_mode(Runner &R, int32_t mode) {
    if (mode < SWEEP_AUTO || mode > SWEEP_PERSISTENT) return SELINV_E_INVALID_ARG;
    if (mode != R.sweep_mode) {
        R.sweep_mode = mode;
        for (int p = 0; p < NPREC; p++) runner_drop(R, p);
    }
    return SELINV_OK;
}

// ---------------------------------------------------------------------------
// C ABI: runs of one handle
// ---------------------------------------------------------------------------
selinv_status selinv_run(selinv_handle h, selinv_precision prec, void *stream) {
    selinv_status st = check_run(h, prec);
    if (st) return st;
    return runner_launch(h->run, prec, (hipStream_t)stream, false, h->err);
}

selinv_status selinv_run_graph(selinv_handle h, selinv_precision prec, void *stream) {
    selinv_status st = check_run(h, prec);
    if (st) return st;
    return runner_launch(h->run, prec, (hipStream_t)stream, true, h->err);
}

selinv_status selinv_set_sweep_mode(selinv_handle h, int32_t mode) {
    if (!h) return SELINV_E_INVALID_ARG;
    return runner_set_mode(h->run, mode);
}

selinv_status selinv_set_gather_form(selinv_handle h, int32_t form) {
    if (!h) return SELINV_E_INVALID_ARG;
    return runner_set_gather_form(h->run, form);
}

int32_t selinv_sweep_is_persistent(selinv_handle h, selinv_precision prec) {
    if (!h || !valid_prec(prec) || !h->run.sweep[prec]) return -1;
    return h->run.sweep[prec]->persistent ? 1 : 0;
}

selinv_status selinv_set_profiling(selinv_handle h, int32_t on) {
    if (!h) return SELINV_E_INVALID_ARG;
    h->run.profiling = on != 0;
    return SELINV_OK;
}

selinv_status selinv_timings(selinv_handle h, double *ms, int32_t count) {
    if (!h || !ms) return SELINV_E_INVALID_ARG;
    // the events belong to the last run only if it was this handle's own
    // profiled run and its sweep still exists
    if (h->state < 2 || h->last_prec < 0 || !h->last_profiled || !h->last_sweep ||
        h->last_sweep != h->run.sweep[h->last_prec].get())
        return SELINV_E_STATE;
    return runner_timings(h->run, ms, count, h->err);
}

selinv_status selinv_tune(selinv_handle h, selinv_precision prec, int32_t reps, void *stream, double *ms_policy,
                          double *ms_tuned) {
    selinv_status st = check_run(h, prec);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!s) {  // graphs are not captured on the legacy null stream
        if (!h->run.own_stream)
            HIPCHK(h->err, hipStreamCreateWithFlags(&h->run.own_stream, hipStreamNonBlocking), "stream");
        s = h->run.own_stream;
    }
    return runner_tune(h->run, prec, reps, s, ms_policy, ms_tuned, h->err);
}

selinv_status selinv_get_tuning(selinv_handle h, selinv_precision prec, int32_t *out, int32_t cap,
                                int32_t *count) {
    if (!h || !valid_prec(prec) || !count) return SELINV_E_INVALID_ARG;
    return runner_get_tuning(h->run, prec, out, cap, count, h->err);
}

selinv_status selinv_set_tuning(selinv_handle h, selinv_precision prec, const int32_t *in, int32_t count) {
    if (!h || !valid_prec(prec)) return SELINV_E_INVALID_ARG;
    return runner_set_tuning(h->run, prec, in, count, h->err);
}

selinv_status selinv_level_stats(selinv_handle h, int32_t level, double *stats) {
    if (!h || !stats) return SELINV_E_INVALID_ARG;
    if (!h->last_sweep) return SELINV_E_STATE;  // no run yet, or its sweep was dropped
    return sweep_level_stats(*h->last_sweep, level, stats);
}

static selinv_status check_sweep_error(std::string &err, const Sweep *S) {
    if (!S || !S->persistent) return SELINV_OK;
    int32_t flag = 0;
    HIPCHK(err, hipMemcpy(&flag, S->d_cnt + S->ncnt + 1, 4, hipMemcpyDeviceToHost), "read sweep flag");
    if (flag) {
        err = "persistent sweep: a dependency wait ran out (results invalid)";
        return SELINV_E_DEVICE;
    }
    return SELINV_OK;
}

static selinv_status sync_last(selinv_handle h) {
    if (h->state < 2 || h->last_prec < 0) {
        h->err = "no completed run";
        return SELINV_E_STATE;
    }
    HIPCHK(h->err, hipStreamSynchronize(h->last_stream), "stream sync");
    return check_sweep_error(h->err, h->last_sweep);
}

static selinv_status get_real(selinv_handle h, int64_t i, int64_t j, double *out);

selinv_status selinv_get(selinv_handle h, int64_t i, int64_t j, double *out) {
    if (!h || !out) return SELINV_E_INVALID_ARG;
    if (h->state < 0) return SELINV_E_STATE;
    if (!h->cplx) return get_real(h, i, j, out);
    // A^{-1}(i, j) = M^{-1}(2i, 2j) + i M^{-1}(2i+1, 2j)
    if (i < 0 || j < 0 || i >= h->n_c || j >= h->n_c) return SELINV_E_INVALID_ARG;
    selinv_status st = get_real(h, 2 * i, 2 * j, out);
    if (!st) st = get_real(h, 2 * i + 1, 2 * j, out + 1);
    return st;
}

static selinv_status get_real(selinv_handle h, int64_t i, int64_t j, double *out) {
    const Plan &P = h->P;
    if (i < 0 || j < 0 || i >= P.n || j >= P.n) return SELINV_E_INVALID_ARG;
    selinv_status st = sync_last(h);
    if (st) return st;
    int64_t loc = P.locate(P.q[j], P.q[i]);
    if (loc < 0) return SELINV_E_NOT_SELECTED;
    const PrecBufs &b = h->pb[h->last_prec];
    int64_t kind = loc >> LOC_SHIFT, off = loc & LOC_MASK;
    if (kind == LOC_DIAG) {
        HIPCHK(h->err, hipMemcpy(out, b.Zd + off, 8, hipMemcpyDeviceToHost), "D2H");
    } else {
        const void *base = kind == LOC_L ? b.ZL : b.ZU;
        if (h->last_prec == SELINV_FP64) {
            HIPCHK(h->err, hipMemcpy(out, (const double *)base + off, 8, hipMemcpyDeviceToHost), "D2H");
        } else {
            float f = 0;
            HIPCHK(h->err, hipMemcpy(&f, (const float *)base + off, 4, hipMemcpyDeviceToHost), "D2H");
            *out = f;
        }
    }
    return SELINV_OK;
}

selinv_status selinv_set_allocator(selinv_alloc_fn alloc, selinv_free_fn dealloc, void *ctx) {
    if ((alloc == nullptr) != (dealloc == nullptr)) return SELINV_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.dealloc = dealloc;
    g_alloc.ctx = alloc ? ctx : nullptr;
    return SELINV_OK;
}

selinv_status selinv_get_many(selinv_handle h, int64_t count, const int64_t *i, const int64_t *j, double *out) {
    if (!h || count < 0 || (count > 0 && (!i || !j || !out))) return SELINV_E_INVALID_ARG;
    if (h->state < 0) return SELINV_E_STATE;
    if (count == 0) return SELINV_OK;
    const Plan &P = h->P;
    const int64_t nn = h->cplx ? h->n_c : P.n;
    const int64_t per = h->cplx ? 2 : 1;
    std::vector<int64_t> loc;
    try {
        loc.resize(count * per);
    } catch (const std::bad_alloc &) {
        h->err = "host allocation failed in get_many";
        return SELINV_E_NOMEM;
    }
    for (int64_t k = 0; k < count; k++) {
        if (i[k] < 0 || j[k] < 0 || i[k] >= nn || j[k] >= nn) {
            h->err = "get_many: position " + std::to_string(k) + " outside the matrix";
            return SELINV_E_INVALID_ARG;
        }
        // A^{-1}(i, j) = At^{-T}(q[j], q[i]); complex: the real form's (2i, 2j) and (2i + 1, 2j)
        for (int64_t c = 0; c < per; c++) {
            const int64_t ii = h->cplx ? 2 * i[k] + c : i[k], jj = h->cplx ? 2 * j[k] : j[k];
            const int64_t l = P.locate(P.q[jj], P.q[ii]);
            if (l < 0) {
                h->err = "get_many: position " + std::to_string(k) + " outside the computed set";
                return SELINV_E_NOT_SELECTED;
            }
            loc[k * per + c] = l;
        }
    }
    selinv_status st = sync_last(h);
    if (st) return st;
    const int64_t m = count * per;
    int64_t *d_loc = nullptr;
    double *d_out = nullptr;
    hipError_t e = upload(h->al, &d_loc, loc);
    if (e == hipSuccess) e = alloc_bytes(h->al, (void **)&d_out, m * 8);
    if (e == hipSuccess) {
        const PrecBufs &b = h->pb[h->last_prec];
        ExtractArgs a{d_loc, b.Zd, b.ZL, b.ZU, d_out, m};
        e = launch_extract(h->last_prec == SELINV_FP64, a, h->last_stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->last_stream);
    if (e == hipSuccess) e = hipMemcpy(out, d_out, m * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) st = dev_fail(h->err, e, "get_many");
    h->al.put(d_loc);
    h->al.put(d_out);
    return st;
}

selinv_status selinv_set_gather_code_budget(selinv_handle h, int64_t entries) {
    if (!h) return SELINV_E_INVALID_ARG;
    if (h->d_diag) {
        h->err = "the gather code budget must be set before the first factor call";
        return SELINV_E_STATE;
    }
    try {
        build_gather_codes(h->P, h->sn, h->gcL, h->gcU, entries < 0 ? kCodeBudget : entries);
    } catch (const std::bad_alloc &) {
        h->err = "host allocation failed in set_gather_code_budget";
        return SELINV_E_NOMEM;
    }
    return SELINV_OK;
}

selinv_status selinv_get_selected_device(selinv_handle h, double *out, void *stream) {
    if (!h || !out) return SELINV_E_INVALID_ARG;
    if (h->state < 2 || h->last_prec < 0) return SELINV_E_STATE;
    const PrecBufs &b = h->pb[h->last_prec];
    ExtractArgs a{h->cplx ? h->d_aloc_c : h->d_aloc, b.Zd, b.ZL, b.ZU, out, h->cplx ? 2 * h->nnz_c : h->P.nnz_a};
    hipError_t e = launch_extract(h->last_prec == SELINV_FP64, a, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail(h->err, e, "extract launch");
    return SELINV_OK;
}

// Staging of selinv_get_selected_noalloc: the extraction writes one chunk of
// the selected entries here and the host copy reads it back.  A file-scope
// device array: each device the library runs on holds its own copy until the
// process ends.  Host code never passes its name to a kernel or a copy (on
// the host it only stands for the symbol): the array's device address comes
// from hipGetSymbolAddress, once per device, with that device current.
constexpr int64_t kScratchEntries = int64_t(1) << 20;  // 8 MiB of doubles
static __device__ __align__(256) double scratch[kScratchEntries];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

static selinv_status scratch_of_device(int dev, double **out, std::string &err) {
    if (dev < 0 || dev >= kMaxDevices) {
        err = "device ordinal beyond the staging table";
        return SELINV_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return dev_fail(err, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                   "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return SELINV_OK;
}

selinv_status selinv_get_selected_noalloc(selinv_handle h, double *out) {
    if (!h || !out) return SELINV_E_INVALID_ARG;
    selinv_status st = sync_last(h);
    if (st) return st;
    int dev = 0;
    HIPCHK(h->err, hipGetDevice(&dev), "hipGetDevice");
    if (dev != h->device) {
        h->err = "get_selected_noalloc on a different device than factor";
        return SELINV_E_STATE;
    }
    double *buf = nullptr;
    if ((st = scratch_of_device(dev, &buf, h->err))) return st;
    const PrecBufs &b = h->pb[h->last_prec];
    const int64_t cnt = h->cplx ? 2 * h->nnz_c : h->P.nnz_a;
    const int64_t *loc = h->cplx ? h->d_aloc_c : h->d_aloc;
    hipStream_t s = h->last_stream;
    // chunks of at most kScratchEntries: extraction into the array, copy to
    // the host, and the stream drained before the next chunk reuses it
    for (int64_t p0 = 0; p0 < cnt; p0 += kScratchEntries) {
        const int64_t m = std::min(kScratchEntries, cnt - p0);
        ExtractArgs a{loc + p0, b.Zd, b.ZL, b.ZU, buf, m};
        HIPCHK(h->err, launch_extract(h->last_prec == SELINV_FP64, a, s), "extract launch");
        HIPCHK(h->err, hipMemcpyAsync(out + p0, buf, m * 8, hipMemcpyDeviceToHost, s), "extract copy");
        HIPCHK(h->err, hipStreamSynchronize(s), "extract copy");
    }
    return SELINV_OK;
}

selinv_status selinv_get_selected(selinv_handle h, double *out) {
    if (!h || !out) return SELINV_E_INVALID_ARG;
    selinv_status st = sync_last(h);
    if (st) return st;
    double *d = nullptr;
    const int64_t cnt = h->cplx ? 2 * h->nnz_c : h->P.nnz_a;
    HIPCHK(h->err, alloc_bytes(h->al, (void **)&d, cnt * 8), "alloc extract");
    st = selinv_get_selected_device(h, d, h->last_stream);
    if (!st) {
        hipError_t e = hipStreamSynchronize(h->last_stream);
        if (e == hipSuccess) e = hipMemcpy(out, d, cnt * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = dev_fail(h->err, e, "extract copy");
    }
    h->al.put(d);
    return st;
}

selinv_status selinv_export(selinv_handle h, int32_t *row, int32_t *col, double *val) {
    if (!h || !row || !col || !val) return SELINV_E_INVALID_ARG;
    selinv_status st = sync_last(h);
    if (st) return st;
    const Plan &P = h->P;
    const PrecBufs &b = h->pb[h->last_prec];
    std::vector<double> zd(P.tot_d), zl(P.tot_l), zu(P.tot_u);
    if (P.tot_d) HIPCHK(h->err, hipMemcpy(zd.data(), b.Zd, P.tot_d * 8, hipMemcpyDeviceToHost), "D2H Zd");
    if (h->last_prec == SELINV_FP64) {
        if (P.tot_l) HIPCHK(h->err, hipMemcpy(zl.data(), b.ZL, P.tot_l * 8, hipMemcpyDeviceToHost), "D2H ZL");
        if (P.tot_u) HIPCHK(h->err, hipMemcpy(zu.data(), b.ZU, P.tot_u * 8, hipMemcpyDeviceToHost), "D2H ZU");
    } else {
        std::vector<float> tl(P.tot_l), tu(P.tot_u);
        if (P.tot_l) HIPCHK(h->err, hipMemcpy(tl.data(), b.ZL, P.tot_l * 4, hipMemcpyDeviceToHost), "D2H ZL");
        if (P.tot_u) HIPCHK(h->err, hipMemcpy(tu.data(), b.ZU, P.tot_u * 4, hipMemcpyDeviceToHost), "D2H ZU");
        std::copy(tl.begin(), tl.end(), zl.begin());
        std::copy(tu.begin(), tu.end(), zu.begin());
    }
    int64_t k = 0;
    // A^{-T}(r, c) (permuted) = A^{-1}(p[c], p[r])
    for (int32_t K = 0; K < P.ns; K++) {
        const int32_t f = P.xsup[K], s = P.width(K);
        const int64_t cl = P.cl(K), cu = P.cu(K);
        const int32_t *RL = P.rl.data() + P.rl_ptr[K], *RU = P.ru.data() + P.ru_ptr[K];
        for (int32_t c = 0; c < s; c++)
            for (int32_t r = 0; r < s; r++, k++) {
                row[k] = P.p[f + c];
                col[k] = P.p[f + r];
                val[k] = zd[P.off_d[K] + r + (int64_t)c * s];
            }
        for (int32_t t = 0; t < s; t++)
            for (int64_t a = 0; a < cl; a++, k++) {
                row[k] = P.p[f + t];
                col[k] = P.p[RL[a]];
                val[k] = zl[P.off_l[K] + a + t * cl];
            }
        for (int32_t t = 0; t < s; t++)
            for (int64_t bb = 0; bb < cu; bb++, k++) {
                row[k] = P.p[RU[bb]];
                col[k] = P.p[f + t];
                val[k] = zu[P.off_u[K] + bb + t * cu];
            }
    }
    return SELINV_OK;
}

selinv_status selinv_structure(selinv_handle h, int32_t *perm_out, int32_t *xsup, int64_t *rl_ptr, int32_t *rl,
                               int64_t *ru_ptr, int32_t *ru, int32_t *level) {
    if (!h || h->state < 0) return SELINV_E_INVALID_ARG;
    const Plan &P = h->P;
    if (perm_out) std::copy(P.p.begin(), P.p.end(), perm_out);
    if (xsup) std::copy(P.xsup.begin(), P.xsup.end(), xsup);
    if (rl_ptr) std::copy(P.rl_ptr.begin(), P.rl_ptr.end(), rl_ptr);
    if (rl) std::copy(P.rl.begin(), P.rl.end(), rl);
    if (ru_ptr) std::copy(P.ru_ptr.begin(), P.ru_ptr.end(), ru_ptr);
    if (ru) std::copy(P.ru.begin(), P.ru.end(), ru);
    if (level) std::copy(P.level.begin(), P.level.end(), level);
    return SELINV_OK;
}

selinv_status selinv_check_plan(selinv_handle h, int64_t *mismatches) {
    if (!h || !mismatches) return SELINV_E_INVALID_ARG;
    *mismatches = check_gather_maps(h->P, h->err);
    // push maps: every position of a parent column found in a child's R_L /
    // R_U holds that column, and every such column has a position
    const Plan &P = h->P;
    int64_t bad = 0;
    for (int32_t K = 0; K < P.ns; K++) {
        const int32_t Pa = P.sparent[K];
        if (Pa < 0) continue;
        const int32_t f = P.xsup[Pa], sP = P.width(Pa);
        const int32_t *posL = h->push_pos.data() + h->push_off[K], *posU = posL + sP;
        int64_t inL = 0, inU = 0;
        for (int64_t a = P.rl_ptr[K]; a < P.rl_ptr[K + 1]; a++) inL += P.rl[a] >= f && P.rl[a] < f + sP;
        for (int64_t b = P.ru_ptr[K]; b < P.ru_ptr[K + 1]; b++) inU += P.ru[b] >= f && P.ru[b] < f + sP;
        for (int32_t r = 0; r < sP; r++) {
            if (posL[r] >= 0) {
                inL--;
                bad += posL[r] >= P.cl(K) || P.rl[P.rl_ptr[K] + posL[r]] != f + r;
            }
            if (posU[r] >= 0) {
                inU--;
                bad += posU[r] >= P.cu(K) || P.ru[P.ru_ptr[K] + posU[r]] != f + r;
            }
        }
        bad += (inL != 0) + (inU != 0);
    }
    for (int32_t Q = 0; Q < P.ns; Q++)
        for (int32_t q = h->kids_ptr[Q]; q < h->kids_ptr[Q + 1]; q++) bad += P.sparent[h->kids[q]] != Q;
    bad += h->kids_ptr[P.ns] != (int32_t)std::count_if(P.sparent.begin(), P.sparent.end(), [](int32_t x) { return x >= 0; });
    // levels: every supernode met by R_L(K) u R_U(K) lies on a shallower
    // level, sparent(K) on level(K) - 1, and with one_top(K) no other
    // supernode met lies there
    for (int32_t K = 0; K < P.ns; K++) {
        const int32_t lev = P.level[K], Pa = P.sparent[K];
        bad += (Pa >= 0) ? P.level[Pa] != lev - 1 : lev != 0;
        auto visit = [&](int32_t x) {
            const int32_t J = P.supof[x];
            bad += P.level[J] >= lev;
            bad += P.one_top[K] && P.level[J] == lev - 1 && J != Pa;
        };
        for (int64_t a = P.rl_ptr[K]; a < P.rl_ptr[K + 1]; a++) visit(P.rl[a]);
        for (int64_t b = P.ru_ptr[K]; b < P.ru_ptr[K + 1]; b++) visit(P.ru[b]);
    }
    // gather codes: each names the location that an independent binary
    // search finds for the same entry, in the array of its kind
    for (int32_t K = 0; K < P.ns; K++) {
        const int64_t co = h->sn[K].c_off, cl = P.cl(K), cu = P.cu(K);
        if (co < 0) continue;
        if (co + cl * cu > (int64_t)h->gcL.size()) {
            bad++;
            continue;
        }
        for (int64_t b = 0; b < cu; b++)
            for (int64_t a = 0; a < cl; a++) {
                const int64_t loc = P.locate(P.rl[P.rl_ptr[K] + a], P.ru[P.ru_ptr[K] + b]);
                const int64_t kind = loc >> LOC_SHIFT, off = loc & LOC_MASK;
                const uint32_t want = (uint32_t)((kind == LOC_DIAG ? 1 : kind == LOC_L ? 2 : 3) << GCODE_SHIFT) |
                                      (uint32_t)off;
                const uint32_t l = h->gcL[co + a + b * cl], u = h->gcU[co + b + a * cu];
                bad += loc < 0 || (kind == LOC_U ? (u != want || l != 0) : (l != want || u != 0));
            }
    }
    if (bad && h->err.empty()) h->err = "push maps, levels or gather codes inconsistent with R_L / R_U";
    *mismatches += bad;
    return SELINV_OK;
}

selinv_status selinv_query(selinv_handle h, selinv_info *info) {
    if (!h || !info || h->state < 0) return SELINV_E_INVALID_ARG;
    const Plan &P = h->P;
    info->n = P.n;
    info->nnz_a = P.nnz_a;
    info->nnz_lu = P.tot_d + P.tot_l + P.tot_u;
    info->nsuper = P.ns;
    info->nlevels = P.nlevels;
    info->max_s = P.max_s;
    info->max_c = P.max_c;
    info->flops = P.flops;
    info->flops_gemm = P.flops_gemm;
    info->bytes_min_fp64 = P.bytes64;
    info->bytes_min_fp32 = P.bytes32;
    info->max_gemm_flops = P.max_gemm_flops;
    info->max_gemm_m = P.max_gemm_m;
    info->max_gemm_n = P.max_gemm_n;
    info->max_gemm_k = P.max_gemm_k;
    info->symbolic = P.symbolic;
    info->nnz_l = P.tot_l;
    info->nnz_u = P.tot_u;
    info->complex_values = h->cplx ? 1 : 0;
    return SELINV_OK;
}

void selinv_destroy(selinv_handle h) {
    if (!h) return;
    for (int p = 0; p < NPREC; p++) {
        h->run.sweep[p].reset();
        PrecBufs &b = h->pb[p];
        for (void *q : {(void *)b.Zd, b.ZL, b.ZU, b.Lh, b.Uh, b.G}) h->al.put(q);
    }
    h->lu.reset();
    for (void *q : {(void *)h->d_diag, (void *)h->d_lpan, (void *)h->d_upan, (void *)h->d_Linv, (void *)h->d_Uinv,
                    (void *)h->d_tl, (void *)h->d_tu,
                    (void *)h->d_sn, (void *)h->d_supof, (void *)h->d_rl, (void *)h->d_ru, (void *)h->d_mapL,
                    (void *)h->d_mapU, (void *)h->d_lcol, (void *)h->d_urow, (void *)h->d_aloc, (void *)h->d_aloc_c,
                    (void *)h->d_kids_ptr, (void *)h->d_kids, (void *)h->d_push_off, (void *)h->d_push_pos,
                    (void *)h->d_gcL, (void *)h->d_gcU, (void *)h->d_gcA, (void *)h->d_row_I, (void *)h->d_row_up,
                    (void *)h->d_col_J, (void *)h->d_col_diag, (void *)h->d_col_low})
        h->al.put(q);
    delete h;
}

selinv_status selinv_batch_create(selinv_handle *hs, int32_t count, selinv_batch *out) {
    if (!hs || count <= 0 || !out) return SELINV_E_INVALID_ARG;
    *out = nullptr;
    for (int32_t i = 0; i < count; i++)
        if (!hs[i] || hs[i]->state < 1) return SELINV_E_STATE;
    for (int32_t i = 0; i < count; i++)
        for (int32_t k = 0; k < i; k++)
            if (hs[k] == hs[i]) return SELINV_E_INVALID_ARG;  // a matrix appears once
    selinv_batch b = new (std::nothrow) selinv_batch_s();
    if (!b) return SELINV_E_NOMEM;
    b->run.al = current_alloc();
    b->run.hs.assign(hs, hs + count);
    *out = b;
    return SELINV_OK;
}

static selinv_status check_batch(selinv_batch b, int prec) {
    if (!b || !valid_prec(prec)) return SELINV_E_INVALID_ARG;
    for (auto h : b->run.hs) {
        selinv_status st = check_run(h, prec);
        if (st) {
            b->err = h->err;
            return st;
        }
    }
    return SELINV_OK;
}

selinv_status selinv_batch_run(selinv_batch b, selinv_precision prec, void *stream) {
    selinv_status st = check_batch(b, prec);
    if (st) return st;
    return runner_launch(b->run, prec, (hipStream_t)stream, false, b->err);
}

selinv_status selinv_batch_run_graph(selinv_batch b, selinv_precision prec, void *stream) {
    selinv_status st = check_batch(b, prec);
    if (st) return st;
    return runner_launch(b->run, prec, (hipStream_t)stream, true, b->err);
}

selinv_status selinv_batch_set_gather_form(selinv_batch b, int32_t form) {
    if (!b) return SELINV_E_INVALID_ARG;
    return runner_set_gather_form(b->run, form);
}

selinv_status selinv_batch_set_sweep_mode(selinv_batch b, int32_t mode) {
    if (!b) return SELINV_E_INVALID_ARG;
    return runner_set_mode(b->run, mode);
}

selinv_status selinv_batch_tune(selinv_batch b, selinv_precision prec, int32_t reps, void *stream,
                                double *ms_policy, double *ms_tuned) {
    selinv_status st = check_batch(b, prec);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!s) {
        if (!b->run.own_stream)
            HIPCHK(b->err, hipStreamCreateWithFlags(&b->run.own_stream, hipStreamNonBlocking), "stream");
        s = b->run.own_stream;
    }
    return runner_tune(b->run, prec, reps, s, ms_policy, ms_tuned, b->err);
}

selinv_status selinv_batch_get_tuning(selinv_batch b, selinv_precision prec, int32_t *out, int32_t cap,
                                      int32_t *count) {
    if (!b || !valid_prec(prec) || !count) return SELINV_E_INVALID_ARG;
    return runner_get_tuning(b->run, prec, out, cap, count, b->err);
}

selinv_status selinv_batch_set_tuning(selinv_batch b, selinv_precision prec, const int32_t *in, int32_t count) {
    if (!b || !valid_prec(prec)) return SELINV_E_INVALID_ARG;
    return runner_set_tuning(b->run, prec, in, count, b->err);
}

selinv_status selinv_batch_set_profiling(selinv_batch b, int32_t on) {
    if (!b) return SELINV_E_INVALID_ARG;
    b->run.profiling = on != 0;
    return SELINV_OK;
}

selinv_status selinv_batch_timings(selinv_batch b, double *ms, int32_t count) {
    if (!b || !ms) return SELINV_E_INVALID_ARG;
    return runner_timings(b->run, ms, count, b->err);
}

selinv_status selinv_batch_level_stats(selinv_batch b, int32_t level, double *stats) {
    if (!b || !stats) return SELINV_E_INVALID_ARG;
    const Runner &R = b->run;
    if (R.last_prec < 0 || !R.sweep[R.last_prec]) return SELINV_E_STATE;
    return sweep_level_stats(*R.sweep[R.last_prec], level, stats);
}

selinv_status selinv_batch_query(selinv_batch b, int32_t *count, int32_t *nlevels, double *flops) {
    if (!b) return SELINV_E_INVALID_ARG;
    if (count) *count = (int32_t)b->run.hs.size();
    if (nlevels) *nlevels = b->run.depth();
    if (flops) {
        double f = 0;
        for (auto h : b->run.hs) f += h->P.flops;
        *flops = f;
    }
    return SELINV_OK;
}

const char *selinv_batch_last_error(selinv_batch b) { return b ? b->err.c_str() : ""; }

void selinv_batch_destroy(selinv_batch b) {
    if (!b) return;
    for (int p = 0; p < NPREC; p++) runner_drop(b->run, p);
    delete b;
}

}  // extern "C"
