/*
 * selinv.h -- C ABI of the MI355X (gfx950) selected-inversion library.
 *
 * Method: supernodal selected inversion of a non-symmetric sparse matrix from
 * its LU factors (Jacquelin, Lin, Yang, arXiv:1708.04539), Algorithm 1
 * ("Selected inversion algorithm for a general sparse matrix").  Given a
 * sparse A and a fill-reducing ordering P, the library factors
 * At = P A P^T = L U (unpivoted; eq. permuteLU with Q = P^T) and computes every
 * entry of A^{-1} whose transposed position lies in the block pattern of L+U
 * (Theorems 1 and 2).  This superset contains the selected set
 * { A^{-1}(i,j) : A(j,i) != 0 } (eq. sel_entries).
 *
 * Call order: selinv_analyze -> selinv_factor -> selinv_run (repeatable) ->
 * selinv_get / selinv_get_selected / selinv_export.  Out-of-order calls
 * return SELINV_E_STATE.  No call aborts or exits; every failure is a status
 * code, and selinv_last_error() gives a message for the handle.
 *
 * Conventions
 *   * Indices are 0-based.  CSC input: colptr[n+1] (int64), rowind[nnz]
 *     (int32) sorted and unique inside each column, with every diagonal entry
 *     structurally present; otherwise SELINV_E_BAD_PATTERN.
 *   * perm[new] = old (perm = NULL means the natural order); the permuted
 *     matrix is At[a][b] = A[perm[a]][perm[b]].  Not a permutation:
 *     SELINV_E_BAD_PERM.  The symmetrized analysis may replace perm by a
 *     postorder of the elimination tree of At + At^T; this changes neither
 *     the fill nor any result.  The exact analysis keeps perm as given.
 *   * Every input array is copied; the caller may free it on return.  The
 *     handle owns all host and device memory until selinv_destroy().
 *   * Device memory comes from hipMalloc, or from the hook installed with
 *     selinv_set_allocator(), on the device that is current when
 *     selinv_factor() is called; later calls must use the same device.
 *   * Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  selinv_run() is asynchronous on that stream; the get/export
 *     calls synchronise it.
 */
#ifndef SELINV_H
#define SELINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct selinv_handle_s *selinv_handle;
typedef struct selinv_batch_s *selinv_batch;

typedef enum {
    SELINV_OK = 0,
    SELINV_E_INVALID_ARG = 1,  /* null pointer, size or index out of range        */
    SELINV_E_BAD_PATTERN = 2,  /* CSC not sorted/unique, or missing diagonal      */
    SELINV_E_BAD_PERM = 3,     /* perm is not a permutation of 0..n-1             */
    SELINV_E_ZERO_PIVOT = 4,   /* exact zero or non-finite pivot (no pivoting)    */
    SELINV_E_NOT_SELECTED = 5, /* (i,j) outside the computed superset             */
    SELINV_E_STATE = 6,        /* call out of order                               */
    SELINV_E_NOMEM = 7,        /* host or device allocation failed                */
    SELINV_E_DEVICE = 8        /* HIP runtime error                               */
} selinv_status;

/* Arithmetic of the run.  Every form keeps the factors, the diagonal-block
 * inversions (L_KK^{-1}, U_KK^{-1}), the normalisation of step 2 and the
 * accumulation of the diagonal blocks of step 4 in FP64.
 *   SELINV_FP64         : all of Algorithm 1 in FP64 (FP64 MFMA).
 *   SELINV_MIXED_FP32   : off-diagonal blocks of A^{-T} stored in FP32; the
 *                         products of steps 3-5 on FP32 MFMA.
 *   SELINV_MIXED_BF16X3 : as MIXED_FP32, but each product is formed from a
 *                         two-term bfloat16 split of both operands
 *                         (hi*hi + hi*lo + lo*hi) on BF16 MFMA with FP32
 *                         accumulation.                                       */
typedef enum {
    SELINV_FP64 = 0,
    SELINV_MIXED_FP32 = 1,
    SELINV_MIXED_BF16X3 = 2
} selinv_precision;

/* Symbolic analysis forms (section 2: the method needs no structural
 * symmetrization; its block row and column sets R_L(K) and R_U(K) may differ).
 *   SELINV_SYMBOLIC_SYMMETRIZED : pattern of At + At^T (R_L = R_U), elimination
 *       tree postorder, relaxed supernodes (relax, pad_pct below).
 *   SELINV_SYMBOLIC_EXACT : the exact pattern of the unpivoted L and U of At,
 *       no symmetrization: supernodes are runs of consecutive columns of L
 *       with L(j, j-1) != 0 and equal structure below row j (fundamental
 *       supernodes of L), cut every max_super columns; R_L(K) and R_U(K) are
 *       the row set of L(:, K) and the column set of U(K, :) beyond K, closed
 *       under the block fill R_L(K) x R_U(K) of every earlier supernode, so
 *       that Theorem 1 holds blockwise.  The ordering is used as given.
 *       relax > 0: every maximal subtree of the elimination tree of
 *       At + At^T with at most relax columns that occupies a contiguous
 *       column range becomes one supernode; pad_pct > 0: outside those, a
 *       column also joins the run before it when it has that run's last
 *       column as its only child and the padding estimate of the exact
 *       counts stays within pad_pct percent (as for the symmetrized form,
 *       with the rows of L and the columns of U counted separately).
 *       relax = pad_pct = 0: the fundamental supernodes alone. */
typedef enum {
    SELINV_SYMBOLIC_SYMMETRIZED = 0,
    SELINV_SYMBOLIC_EXACT = 1
} selinv_symbolic;

/* Supernode partition rules (paper section 2, paragraph on supernodes:
 * relaxed supernodes with a maximal width).
 *   max_super : widest supernode; wider ones are cut into consecutive pieces
 *               of max_super columns (<= 0 or above 1024: 1024, the widest
 *               block the diagonal-inversion kernel handles).
 *   relax     : every maximal elimination subtree with at most `relax`
 *               columns becomes one supernode.
 *   pad_pct   : outside those subtrees, column j joins the supernode [f, j-1]
 *               of its only child j-1 while the padding estimate
 *               Z = s cnt(j) - sum_{t=f..j} cnt(t) + s(s-1)/2  (s = j-f+1,
 *               cnt = off-diagonal count of a column of L) stays at most
 *               pad_pct percent of s (cnt(j) + s).  0 gives fundamental
 *               supernodes; values are clamped to [0, 100].
 *   symbolic  : a selinv_symbolic value (other values: SELINV_E_INVALID_ARG).
 *   complex_values : nonzero for a complex A (the paper's experiments are
 *               complex, e.g. H - zS).  The library then works on the real
 *               form M of order 2n: the entry a = x + i y at (i, j) becomes
 *               [[x, -y], [y, x]] at rows 2i, 2i+1 and columns 2j, 2j+1, and
 *               M^{-1} holds A^{-1} the same way.  Every kernel, precision and
 *               sweep form applies unchanged, at twice the flops and storage
 *               of native complex arithmetic.  The unpivoted LU of M needs a
 *               nonzero real part at every pivot of its 2 x 2 node blocks
 *               (true for matrices whose diagonal dominates in its real part);
 *               else SELINV_E_ZERO_PIVOT.  selinv_factor takes 2 nnz doubles
 *               (re, im per entry of A); selinv_get writes 2 doubles (re, im);
 *               selinv_get_selected(_device) writes 2 nnz doubles;
 *               selinv_structure, selinv_export, selinv_query (n, nnz_a, ...)
 *               and the supernode sizes (max_super, relax) refer to M.
 * Padded entries are stored explicitly; their values are still exact entries
 * of A^{-1}.  opts = NULL: all fields 0. */
typedef struct {
    int32_t max_super;
    int32_t relax;
    int32_t pad_pct;
    int32_t symbolic;
    int32_t complex_values;
} selinv_analyze_opts;

typedef struct {
    int64_t n;          /* matrix order                                          */
    int64_t nnz_a;      /* stored entries of A                                    */
    int64_t nnz_lu;     /* entries of the block pattern of L+U (= computed set)  */
    int32_t nsuper;     /* supernodes                                            */
    int32_t nlevels;    /* depth of the supernodal elimination tree (+1)         */
    int32_t max_s;      /* widest supernode                                      */
    int32_t max_c;      /* largest |R_L(K)| or |R_U(K)|                          */
    double flops;       /* algorithmic flops of steps 2-5        */
    double flops_gemm;  /* of which in the products of steps 3-5                 */
    double bytes_min_fp64; /* algorithmic HBM bytes of one run, FP64 form        */
    double bytes_min_fp32; /* same with FP32 off-diagonal blocks                 */
    double max_gemm_flops;  /* flops of the largest single supernode product    */
    int32_t max_gemm_m, max_gemm_n, max_gemm_k; /* its shape                    */
    int32_t symbolic;   /* selinv_symbolic form of the analysis                  */
    int64_t nnz_l, nnz_u; /* stored entries of the off-diagonal blocks of L, U   */
    int32_t complex_values; /* 1: a complex A in its real form (n, nnz_a of M)  */
} selinv_info;

/* Source of device memory (Algorithm 1 takes the factors and returns the
 * selected blocks; the paper's implementation keeps them in its own
 * distributed objects, section "Distributed data layout and structure").
 * alloc(bytes, ctx) returns device memory of the current device, aligned to
 * 256 bytes, or NULL when it has none (the calling library function then
 * returns SELINV_E_NOMEM; a pointer that is not 256-byte aligned is handed
 * back and gives SELINV_E_DEVICE); dealloc(ptr, ctx) takes back a pointer
 * that alloc returned.  Both are called on the thread that called the
 * library, never from a kernel or a stream callback.  Before a pointer is
 * handed back, the library waits for the device to finish its work
 * (hipDeviceSynchronize), so the hook may reuse the memory at once.
 * alloc = dealloc = NULL restores hipMalloc / hipFree (the default); one of
 * them NULL gives SELINV_E_INVALID_ARG.  The setting is process-wide; each
 * handle and batch keeps the one in effect when it was created
 * (selinv_analyze, selinv_batch_create) for all of its memory, so changing it
 * later affects only new handles and batches.  Thread-safe. */
typedef void *(*selinv_alloc_fn)(size_t bytes, void *ctx);
typedef void (*selinv_free_fn)(void *ptr, void *ctx);
selinv_status selinv_set_allocator(selinv_alloc_fn alloc, selinv_free_fn dealloc, void *ctx);

/* Symbolic analysis (host only).  Builds the supernode partition, the block
 * row/column sets R_L(K), R_U(K) of Algorithm 1 (from At + At^T or from the
 * exact pattern, see selinv_symbolic), the level sets of the supernodal
 * dependency graph (level(K) = 0 if R_L(K) and R_U(K) are empty, else one
 * more than the deepest supernode they touch; roots at level 0) and the
 * relative-index maps used by the gather. */
selinv_status selinv_analyze(int64_t n, const int64_t *colptr, const int32_t *rowind,
                             const int32_t *perm, const selinv_analyze_opts *opts,
                             selinv_handle *out);

/* Numerical factorization At = L U without pivoting, FP64, on the host
 * (setup; OpenMP).  values[] is aligned with rowind[] of selinv_analyze.
 * The factors are then copied to the current device (one host->device copy).
 * An exact zero or non-finite pivot gives SELINV_E_ZERO_PIVOT. */
selinv_status selinv_factor(selinv_handle h, const double *values);

/* The same factorization on the device, asynchronous on `stream` until its
 * end, where the call waits for the stream to read the pivot check.
 * values: DEVICE memory of the current device, aligned with rowind[] of
 * selinv_analyze (nnz doubles; 2 nnz interleaved re, im for a complex
 * handle), owned by the caller and only read; a host pointer gives
 * SELINV_E_INVALID_ARG, a shorter buffer is undefined behaviour.  The
 * entries are scattered into the block storage, then the levels of the
 * dependency graph run from the deepest up: per level, 64-column steps of the
 * diagonal blocks (LU of the 64x64 tile in one wave, the inverses of its
 * triangular factors, the solves of the block and panel rows as products
 * with them, trailing GEMM updates), then W_K = -L(R_L,K) U(K,R_U) for every
 * supernode of the level and its atomic scatter-add into the blocks of the
 * ancestors (right-looking supernodal LU; supernodes of one level are
 * independent).  FP64 throughout; rounding differs from selinv_factor (the
 * solves multiply by tile inverses, sums run in another order).  The first
 * call builds and uploads its work lists (host range checks included).  A
 * zero or non-finite pivot gives SELINV_E_ZERO_PIVOT (the smallest permuted
 * column with such a pivot) and leaves the handle unfactored.  Earlier work
 * of the handle on other streams must be complete before the call. */
selinv_status selinv_factor_device(selinv_handle h, const double *values, void *stream);

/* Steps 2-5 of Algorithm 1 on the device, asynchronous on `stream`:
 * diagonal-block inversion and normalisation of every supernode, then one
 * level of the supernodal tree after another (root first): gather of
 * A^{-T}(R_L, R_U), the products of steps 3 and 5, and the diagonal block of
 * step 4.  The factors are left intact, so the call may be repeated. */
selinv_status selinv_run(selinv_handle h, selinv_precision prec, void *stream);

/* Same as selinv_run for the last completed run, but the sweep is recorded
 * once into a HIP graph per (handle, precision) and replayed. */
selinv_status selinv_run_graph(selinv_handle h, selinv_precision prec, void *stream);

/* How the level sweep is launched.
 *   0 (auto, default): persistent when the levels are too small to fill the
 *     device on their own, per-level launches otherwise;
 *   1: one launch per kernel class per level (gather, steps 3+5, step 4);
 *   2: one persistent, dependency-driven launch for the whole sweep
 *     (section on inter-supernode parallelism: tasks start as soon as their
 *     data dependencies are met).  A dependency wait that runs out of its
 *     bound makes the next synchronising call return SELINV_E_DEVICE.
 * Changing the mode drops the cached work lists (and HIP graph) of the
 * handle.  selinv_sweep_is_persistent() tells which form the last built sweep
 * of that precision uses (-1: none built yet). */
selinv_status selinv_set_sweep_mode(selinv_handle h, int32_t mode);

/* Where the level sweep takes G_K = At^{-T}(R_L(K), R_U(K)) from (Fig. 3:
 * the supernode's products need only those rows and columns of the blocks
 * computed before it; Theorem 1 names the blocks they lie in).
 *   0 (default): the tuning's choice per level (selinv_tune), a stored G
 *     without a tuning;
 *   1: a stored G: gather tiles copy G_K into a workspace that the products
 *     of steps 3 and 5 then read;
 *   2: no stored G on any level of large supernodes: the products of steps
 *     3 and 5 read every entry of G_K from the diagonal block, L panel or U
 *     panel that holds it, through a 32-bit source code per entry (built on
 *     the first such run, c_L c_U codes per supernode, 4 bytes each, in
 *     device memory from the handle's allocator; SELINV_E_NOMEM when that
 *     fails).  Levels run by the fused small-supernode launch keep G_K in
 *     LDS, and the persistent sweep always gathers into G.
 * The results of forms 1 and 2 are equal bit for bit (the same values in the
 * same order).  form outside 0..2: SELINV_E_INVALID_ARG.  Changing the form
 * drops the cached work lists (and HIP graphs) of the handle. */
selinv_status selinv_set_gather_form(selinv_handle h, int32_t form);

/* Autotuner (the section on inter-supernode parallelism leaves the schedule
 * of a level's supernodes to the implementation).  Measures the launch
 * choices of the level sweep of one precision on the current device and on
 * `stream`, and keeps the fastest for this handle:
 *   - the output tile edge (32, 64 or 128) of every grouped-GEMM launch class:
 *     the diagonal-block inversion rounds, the normalisation, the diagonal
 *     initialisation, and per level the step-3/5 launch and the step-4
 *     launch.  Each candidate edge runs over the whole sweep with per-launch
 *     HIP events; every class keeps its fastest edge;
 *   - per level made only of small supernodes, the fused small-supernode
 *     launch or the per-phase launches;
 *   - with gather form 0 and a level sweep, per level of large supernodes a
 *     stored G or G_K read from its sources by the products (see
 *     selinv_set_gather_form);
 *   - with sweep mode 0, the level sweep or the persistent sweep;
 *   - the prologue of the wide lower levels on a side stream beside the
 *     upper levels (also with one part per upper level), or all of the
 *     prologue before the sweep;
 *   - with the side stream, its tile inversions on one workgroup per item
 *     or on 1/4, 1/2, 3/4, 1, 5/4, 3/2, 7/4, 2, 5/2 or 3 times the
 *     compute-unit count of workgroups, each looping over items (a launch
 *     that fills the device holds the upper levels' launches back until it
 *     drains).
 * Each configuration runs reps + 1 times (the first untimed; 1 <= reps <=
 * 100) and counts its fastest run: per-launch times from eager runs with
 * events, whole-sweep comparisons from replays of the sweep's HIP graph.  When the measured choices are not faster
 * than the built-in size policy, the policy is kept.  ms_policy and ms_tuned
 * (nullable) receive the two sweep times.  Needs a factored handle; the runs
 * leave the results of an ordinary run behind.  Batches have their own
 * tables (selinv_batch_tune). */
selinv_status selinv_tune(selinv_handle h, selinv_precision prec, int32_t reps, void *stream,
                          double *ms_policy, double *ms_tuned);

/* The tuning table of `prec` as int32 values:
 *   [4, nlevels, sweep form (0: the handle's mode, 1: levels, 2: persistent),
 *    tile of the inversion rounds, of the normalisation, of the diagonal
 *    initialisation, prologue placement (0: the levels from the first wide
 *    one on a side stream beside the sweep of the levels above; 1: the whole
 *    prologue before the sweep, no side stream; 2: as 0, and every level
 *    above the first wide one its own part on the side stream, joined just
 *    before the sweep reaches that level), tile-inversion workgroups on the
 *    side stream, each looping over items (0: one workgroup per item; at
 *    most 2^20), then for every level
 *    d = 0 .. nlevels-1: tile of
 *    steps 3+5, tile of step 4, 1 if the level's small supernodes use the
 *    per-phase launches, 1 if its steps 3/5 read G_K from its sources
 *    (gather form 0)],
 * tile 0 meaning the size policy.  *count receives 8 + 4 nlevels (0 when the
 * handle is untuned; nothing written); out = NULL queries the count;
 * cap < count gives SELINV_E_INVALID_ARG.  selinv_set_tuning also takes the
 * earlier layouts, all with a stored G: [3, ... as above, per level the first
 * three values] (8 + 3 nlevels values), [2, nlevels, sweep, tri, norm, dt,
 * no_fork, per level ...] (7 + 3 nlevels values, one workgroup per side
 * inversion item) and [1,
 * nlevels, sweep, tri, norm, dt, per level ...] (6 + 3 nlevels values, side
 * stream kept). */
selinv_status selinv_get_tuning(selinv_handle h, selinv_precision prec, int32_t *out, int32_t cap,
                                int32_t *count);

/* Installs a table of that layout (a cached one, say); count = 0 returns to
 * the size policy.  A table that does not fit the handle (layout, level
 * count or tile edges) gives
 * SELINV_E_INVALID_ARG and changes nothing.  The work lists of `prec` are
 * rebuilt at the next run. */
selinv_status selinv_set_tuning(selinv_handle h, selinv_precision prec, const int32_t *in, int32_t count);
int32_t selinv_sweep_is_persistent(selinv_handle h, selinv_precision prec);

/* Batches: several factored handles processed by one level sweep, levels
 * aligned at the roots (section on inter-supernode parallelism: supernodes
 * with the same priority run together, here those of every matrix).  Every
 * launch of the sweep covers the supernodes of one level of all matrices.
 * The batch keeps pointers to the handles (each may appear once; else
 * SELINV_E_INVALID_ARG; unfactored: SELINV_E_STATE); destroy the batch before
 * its handles.  Its device memory (work lists) comes from the allocator in
 * effect at selinv_batch_create.  Results land in each handle's own buffers
 * and are read with the handle's get/export calls, as after selinv_run; the
 * FP64 results equal those of single runs bit for bit.
 *   selinv_batch_run         eager launches on `stream`;
 *   selinv_batch_run_graph   the sweep recorded once into a HIP graph per
 *                            (batch, precision) and replayed;
 *   selinv_batch_set_sweep_mode, selinv_batch_set_gather_form,
 *   selinv_batch_tune, selinv_batch_get_tuning,
 *   selinv_batch_set_tuning  as for a handle (selinv_set_sweep_mode,
 *                            selinv_set_gather_form, selinv_tune, ...),
 *                            over the batch's aligned
 *                            levels (nlevels = the deepest matrix's);
 *   selinv_batch_set_profiling, selinv_batch_timings, selinv_batch_level_stats
 *                            as for a handle, for the batch's last eager run;
 *   selinv_batch_query       matrices, aligned levels and the total
 *                            algorithmic flops (any pointer may be NULL). */
selinv_status selinv_batch_create(selinv_handle *hs, int32_t count, selinv_batch *out);
selinv_status selinv_batch_run(selinv_batch b, selinv_precision prec, void *stream);
selinv_status selinv_batch_run_graph(selinv_batch b, selinv_precision prec, void *stream);
selinv_status selinv_batch_set_sweep_mode(selinv_batch b, int32_t mode);
selinv_status selinv_batch_set_gather_form(selinv_batch b, int32_t form);
selinv_status selinv_batch_tune(selinv_batch b, selinv_precision prec, int32_t reps, void *stream,
                                double *ms_policy, double *ms_tuned);
selinv_status selinv_batch_get_tuning(selinv_batch b, selinv_precision prec, int32_t *out, int32_t cap,
                                      int32_t *count);
selinv_status selinv_batch_set_tuning(selinv_batch b, selinv_precision prec, const int32_t *in, int32_t count);
selinv_status selinv_batch_set_profiling(selinv_batch b, int32_t on);
selinv_status selinv_batch_timings(selinv_batch b, double *ms, int32_t count);
selinv_status selinv_batch_level_stats(selinv_batch b, int32_t level, double *stats);
selinv_status selinv_batch_query(selinv_batch b, int32_t *count, int32_t *nlevels, double *flops);
const char *selinv_batch_last_error(selinv_batch b);
void selinv_batch_destroy(selinv_batch b);

/* A^{-1}(i, j) = At^{-T}(q[j], q[i]), q = perm^{-1} (step 6; eq. unpermute).
 * Synchronises the run's stream; SELINV_E_NOT_SELECTED when (i, j) is
 * outside the computed set. */
selinv_status selinv_get(selinv_handle h, int64_t i, int64_t j, double *out);

/* Many entries at once (step 6 for a list of positions; eq. unpermute):
 * out[k] = A^{-1}(i[k], j[k]) for k < count (host arrays; a complex handle
 * writes re, im pairs, 2 count doubles).  Every position is checked on the
 * host first: an index outside [0, n) gives SELINV_E_INVALID_ARG, a position
 * outside the computed set SELINV_E_NOT_SELECTED, and then nothing is
 * written.  The values are gathered on the device (one launch) from the last
 * run's results, after the run's stream is synchronised; count = 0 does
 * nothing. */
selinv_status selinv_get_many(selinv_handle h, int64_t count, const int64_t *i, const int64_t *j, double *out);

/* out[p] = A^{-1}(j, i) for the p-th stored entry (i, j) of A (host buffer of
 * nnz(A) doubles).  Tr[B A^{-1}] = sum_p B_p out[p] for any B on A's pattern. */
selinv_status selinv_get_selected(selinv_handle h, double *out);

/* selinv_get_selected without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and result as
 * selinv_get_selected; the entries are staged through a fixed device array of
 * 2^20 doubles (8 MiB, one per device, held until the process ends) in chunks
 * of at most that many, so any nnz(A) is served; the call makes no hipMalloc,
 * hipFree or allocator-hook call.  It synchronises the run's stream once per
 * chunk.  Calls that overlap on one device (other threads, or another handle
 * on the same device) share that array and race: serialise them. */
selinv_status selinv_get_selected_noalloc(selinv_handle h, double *out);

/* Device version: `out` is a device buffer of nnz(A) doubles; the extraction
 * kernel runs asynchronously on `stream`. */
selinv_status selinv_get_selected_device(selinv_handle h, double *out, void *stream);

/* Every computed entry: row[k], col[k], val[k] = A^{-1}(row, col), for k <
 * info.nnz_lu, in storage order (host buffers). */
selinv_status selinv_export(selinv_handle h, int32_t *row, int32_t *col, double *val);

/* Structure of the analysis (host buffers; any pointer may be NULL):
 * perm_out[n] (final ordering, new -> old), xsup[nsuper+1], rl_ptr/ru_ptr
 * [nsuper+1] (int64), rl/ru (block rows/columns, permuted indices),
 * level[nsuper]. */
selinv_status selinv_structure(selinv_handle h, int32_t *perm_out, int32_t *xsup, int64_t *rl_ptr,
                               int32_t *rl, int64_t *ru_ptr, int32_t *ru, int32_t *level);

selinv_status selinv_query(selinv_handle h, selinv_info *info);

/* Budget of the gather's precomputed source codes, in entries of G (one
 * 32-bit code per entry and side): while the total of |R_L(K)| |R_U(K)| over
 * all supernodes stays within it, every supernode gets codes; otherwise only
 * supernodes whose G_K fits one 64 x 64 tile, in order, while the budget
 * lasts.  Supernodes without codes gather through the relative-index maps
 * (Theorem 1: the positions of R_L(K) inside R_L(J) and of R_U(K) inside
 * R_U(I)), and supernodes of at most 64 columns without codes take the
 * per-phase launches instead of the fused small-supernode kernel.  entries < 0
 * restores the default (2^26); 0 turns the codes off.  Only before the first
 * factor call of the handle (SELINV_E_STATE afterwards). */
selinv_status selinv_set_gather_code_budget(selinv_handle h, int64_t entries);

/* Host-only consistency check of the analysis: recomputes the source location
 * of every entry of every G_K from the relative-index maps (as the gather
 * kernel does) and compares it with a direct search of the block pattern, and
 * checks every storage location of A's entries against its array.
 * *mismatches = 0 when all agree.  Costs O(sum_K |R_L(K)| |R_U(K)|). */
selinv_status selinv_check_plan(selinv_handle h, int64_t *mismatches);

/* Device-side timing of the last selinv_run, from HIP events recorded on the
 * run's stream while profiling is on (selinv_set_profiling; not recorded by
 * selinv_run_graph or batches).  ms[0] diagonal-block inversion, ms[1]
 * normalisation (and, in the FP64 form, the diagonal initialisation), ms[2]
 * diagonal initialisation of the mixed forms, then for every level d
 * ms[3+4d] fused steps 3-5 of the level's small supernodes (s, |R_L|,
 * |R_U| <= 64), ms[4+4d] gather of the others (0 when it runs in the step-4
 * launch of level d-1), ms[5+4d] their products of steps 3 and 5, ms[6+4d]
 * their product of step 4 together with the gather of level d+1 when that is
 * fused into it.  count = number of doubles the caller provides (3 + 4 *
 * nlevels covers all). */
selinv_status selinv_set_profiling(selinv_handle h, int32_t on);
selinv_status selinv_timings(selinv_handle h, double *ms, int32_t count);

/* Work of one level of the last run's sweep (stats: 19 doubles): [0]
 * supernodes, [1] widest supernode; for the launches of the large supernodes
 * [2] flops of steps 3+5, [3] flops of step 4, [4] entries of G gathered, [5]
 * gather tiles, [6] product tiles of steps 3+5, [7] of step 4, [8] and [9] the
 * output tile edge (32, 64 or 128) of those two product launches; for the fused
 * small-supernode launch [10] supernodes, [11] flops of steps 3-5, [12]
 * entries of G gathered; [13] 1 when the level's gather tiles run in the
 * step-4 launch of the level above (the parent's step-4 product then writes
 * its diagonal block into the children's G), 2 when the level's step-3/5
 * products read G_K from its sources (no stored G); [5] is 0 in both cases.  Algorithmic
 * HBM bytes (every operand read once, every result written once, e bytes per
 * element of the run's storage precision, 8 for diagonal blocks; a
 * materialised G is not counted, the sources it is gathered from are):
 * [14] of the steps-3+5 launch, e (c_L c_U + 2 s (c_L + c_U)) per supernode,
 * plus 4 c_L c_U (the source codes) when [13] is 2;
 * [15] of the step-4 launch, 2 e s c_U + 16 s^2 per supernode, plus
 * e c_L c_U for each supernode of the next level whose gather runs in it;
 * [16] of the standalone gather, e c_L c_U per supernode; [17] of the
 * small-supernode launch; [18] flops of the largest single step-3/5 product
 * (2 s c_L c_U) of the level.  level = -1: the prologue, [0]/[1] flops/bytes
 * of the diagonal-block inversion (with the normalisation and diagonal
 * initialisation of the supernodes it does whole), [2]/[3] of the
 * normalisation (in the FP64 form with the diagonal initialisation, which
 * shares its launch), [4]/[5] of the diagonal initialisation of the mixed
 * forms; the rest 0. */
selinv_status selinv_level_stats(selinv_handle h, int32_t level, double *stats);

/* Message of the last failure on handle h; with h == NULL, of the last failed
 * selinv_analyze on the calling thread (which then returns *out = NULL). */
const char *selinv_last_error(selinv_handle h);
const char *selinv_status_string(selinv_status s);
void selinv_destroy(selinv_handle h);

#ifdef __cplusplus
}
#endif

#endif /* SELINV_H */
