/*
 * selinv_oracle.c -- plain, slow, FP64 reference for supernodal selected
 * inversion of a non-symmetric sparse matrix (Jacquelin, Lin, Yang,
 * "PSelInv -- A distributed memory parallel algorithm for selected
 * inversion: the non-symmetric case", arXiv:1708.04539).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or helper with
 * the HIP library.
 *
 * What it computes (section "Selected inversion algorithm for non-symmetric
 * matrices"):
 *   * Permuted matrix  At = P A P^T,  At[a][b] = A[p[a]][p[b]]  (eq. permuteLU
 *     with Q = P^T; symmetric fill-reducing ordering, no row pivoting).
 *   * Unpivoted LU  At = L U, L unit lower, U upper (eq. LU).
 *   * Supernodal partition of the columns (relaxed and capped, section
 *     "Selected inversion ...", paragraph on supernodes), applied to rows too.
 *   * Algorithm 1 ("Selected inversion algorithm for a general sparse
 *     matrix"): step 2 normalised factors for every supernode, then for
 *     K = last ... first: step 3 (off-diagonal row block of A^{-T}), step 4
 *     (diagonal block), step 5 (off-diagonal column block), and step 6
 *     (undo the permutation and transpose).
 *   * A^{-T} is kept on the block pattern of L+U (Fig. "selinv_entries" (b)):
 *     the U(K, R_U) slot holds A^{-T}(K, R_U), the L(R_L, K) slot holds
 *     A^{-T}(R_L, K), the diagonal block holds A^{-T}(K, K).
 *
 * Everything is stored in one hash map keyed by (row, column) of the permuted
 * matrix, so every read of an already computed entry of A^{-T} is a direct
 * lookup by position (Theorem 1 guarantees that the lookup exists; a missing
 * key is reported as an error instead of being read as zero).
 *
 * Symbolic structure, two modes:
 *   mode 0 ("sym"): pattern of At + At^T (structurally symmetric factors).
 *     Elimination tree parent(j) = min{ i > j : L(i,j) != 0 }; the ordering is
 *     replaced by a postorder of that tree (children visited in increasing
 *     index order), which changes neither fill nor results.  Supernodes:
 *       - relaxed: every maximal subtree with at most `relax` nodes (a node v
 *         with size(v) <= relax whose parent has size > relax, or is a root)
 *         is one supernode;
 *       - chains: otherwise j joins the supernode [f, j-1] when
 *         parent(j-1) = j, j has exactly one child, and the columns are nearly
 *         identical: the padding estimate Z of [f, j] (see partition_sym) is at
 *         most pad_pct percent of its stored entries (pad_pct = 0 gives the
 *         fundamental supernodes, colcount(j-1) = colcount(j) + 1);
 *       - cap: each supernode is cut into consecutive pieces of at most
 *         `max_super` columns.
 *   mode 1 ("exact"): exact non-symmetric elimination structure from a dense
 *     boolean simulation (small n only); supernodes are maximal runs of
 *     columns with identical L structure below the block and a dense lower
 *     triangle (the paper's definition), no relaxation, then the cap.
 * In both modes the block rows/columns R_L(K), R_U(K) come from simulating
 * block elimination on the pattern: R_L(K) = rows r > last(K) with an entry
 * in a column of K, R_U(K) = columns c > last(K) with an entry in a row of K,
 * and every (r, c) in R_L(K) x R_U(K) becomes structurally nonzero.
 *
 * Arithmetic: FP64, built with -O2 -ffp-contract=off, every dot product summed
 * in a fixed sequential order inside one thread.  OpenMP only splits loops
 * over independent output entries, so results do not depend on the number of
 * threads.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

enum {
    OR_OK = 0,
    OR_E_INVALID_ARG = 1,
    OR_E_BAD_PATTERN = 2,
    OR_E_BAD_PERM = 3,
    OR_E_ZERO_PIVOT = 4,
    OR_E_NOT_SELECTED = 5,
    OR_E_STATE = 6,
    OR_E_NOMEM = 7,
    OR_E_CLOSURE = 8,
};

/* ------------------------------------------------------------------------ */
/* hash map: int64 key -> int64 slot index                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t *keys; /* -1 = empty */
    int64_t *idx;
    int64_t cap;   /* power of two */
    int64_t count;
} hmap;

static uint64_t hmix(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

static int hmap_init(hmap *h, int64_t expected) {
    int64_t cap = 16;
    while (cap < 2 * expected + 16) cap <<= 1;
    h->keys = (int64_t *)malloc(sizeof(int64_t) * cap);
    h->idx = (int64_t *)malloc(sizeof(int64_t) * cap);
    if (!h->keys || !h->idx) return OR_E_NOMEM;
    for (int64_t i = 0; i < cap; i++) h->keys[i] = -1;
    h->cap = cap;
    h->count = 0;
    return OR_OK;
}

static void hmap_free(hmap *h) {
    free(h->keys);
    free(h->idx);
    h->keys = h->idx = NULL;
    h->cap = h->count = 0;
}

static int64_t hmap_find(const hmap *h, int64_t key) {
    uint64_t m = (uint64_t)h->cap - 1;
    uint64_t s = hmix((uint64_t)key) & m;
    for (;;) {
        int64_t k = h->keys[s];
        if (k == key) return h->idx[s];
        if (k < 0) return -1;
        s = (s + 1) & m;
    }
}

static int hmap_grow(hmap *h) {
    hmap g;
    if (hmap_init(&g, h->cap) != OR_OK) return OR_E_NOMEM;
    uint64_t m = (uint64_t)g.cap - 1;
    for (int64_t i = 0; i < h->cap; i++) {
        if (h->keys[i] < 0) continue;
        uint64_t s = hmix((uint64_t)h->keys[i]) & m;
        while (g.keys[s] >= 0) s = (s + 1) & m;
        g.keys[s] = h->keys[i];
        g.idx[s] = h->idx[i];
    }
    g.count = h->count;
    hmap_free(h);
    *h = g;
    return OR_OK;
}

/* Insert `key` if absent.  Returns its slot index; *inserted tells whether it
 * was new.  Slot indices are assigned 0, 1, 2, ... in insertion order. */
static int64_t hmap_insert(hmap *h, int64_t key, int *inserted) {
    if (2 * (h->count + 1) > h->cap) {
        if (hmap_grow(h) != OR_OK) return -1;
    }
    uint64_t m = (uint64_t)h->cap - 1;
    uint64_t s = hmix((uint64_t)key) & m;
    for (;;) {
        int64_t k = h->keys[s];
        if (k == key) {
            if (inserted) *inserted = 0;
            return h->idx[s];
        }
        if (k < 0) {
            h->keys[s] = key;
            h->idx[s] = h->count++;
            if (inserted) *inserted = 1;
            return h->idx[s];
        }
        s = (s + 1) & m;
    }
}

/* ------------------------------------------------------------------------ */
/* growable int32 list                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t *v;
    int64_t n, cap;
} ilist;

static int ilist_push(ilist *l, int32_t x) {
    if (l->n == l->cap) {
        int64_t c = l->cap ? 2 * l->cap : 4;
        int32_t *nv = (int32_t *)realloc(l->v, sizeof(int32_t) * c);
        if (!nv) return OR_E_NOMEM;
        l->v = nv;
        l->cap = c;
    }
    l->v[l->n++] = x;
    return OR_OK;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* sort + unique in place, returns new length */
static int64_t sort_unique(int32_t *v, int64_t n) {
    if (n <= 1) return n;
    qsort(v, (size_t)n, sizeof(int32_t), cmp_i32);
    int64_t w = 1;
    for (int64_t i = 1; i < n; i++)
        if (v[i] != v[w - 1]) v[w++] = v[i];
    return w;
}

/* ------------------------------------------------------------------------ */
/* oracle object                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n, nnz_a;
    int64_t *a_colptr;
    int32_t *a_rowind;
    int32_t *p; /* new -> old */
    int32_t *q; /* old -> new */
    int32_t nsup;
    int32_t *xsup;   /* nsup+1 */
    int32_t *supof;  /* column -> supernode */
    int64_t *rl_ptr; /* nsup+1 */
    int32_t *rl;
    int64_t *ru_ptr;
    int32_t *ru;
    hmap pos;   /* (r*n + c) -> slot, permuted indices, block pattern of L+U */
    double *lu; /* factor values per slot */
    double *z;  /* A^{-T} values per slot */
    int state;  /* 0 analyzed, 1 factored, 2 inverted */
    double diag_alt_maxdiff, diag_alt_maxabs;
    char err[256];
} oracle_t;

static void set_err(oracle_t *o, const char *msg) {
    if (o) snprintf(o->err, sizeof(o->err), "%s", msg);
}

void oracle_free(oracle_t *o) {
    if (!o) return;
    free(o->a_colptr);
    free(o->a_rowind);
    free(o->p);
    free(o->q);
    free(o->xsup);
    free(o->supof);
    free(o->rl_ptr);
    free(o->rl);
    free(o->ru_ptr);
    free(o->ru);
    hmap_free(&o->pos);
    free(o->lu);
    free(o->z);
    free(o);
}

const char *oracle_last_error(oracle_t *o) { return o ? o->err : "null handle"; }

void oracle_set_threads(int t) {
    if (t > 0) omp_set_num_threads(t);
}

int oracle_get_threads(void) { return omp_get_max_threads(); }

static int validate_csc(int64_t n, const int64_t *colptr, const int32_t *rowind) {
    if (n < 0 || !colptr || (n > 0 && !rowind)) return OR_E_INVALID_ARG;
    if (colptr[0] != 0) return OR_E_BAD_PATTERN;
    for (int64_t j = 0; j < n; j++) {
        if (colptr[j + 1] < colptr[j]) return OR_E_BAD_PATTERN;
        int diag = 0;
        for (int64_t k = colptr[j]; k < colptr[j + 1]; k++) {
            int32_t r = rowind[k];
            if (r < 0 || r >= n) return OR_E_BAD_PATTERN;
            if (k > colptr[j] && rowind[k - 1] >= r) return OR_E_BAD_PATTERN;
            if (r == j) diag = 1;
        }
        if (!diag) return OR_E_BAD_PATTERN;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* symbolic, mode 0: column structures of L for the pattern of At + At^T     */
/* ------------------------------------------------------------------------ */

/* Computes, for the ordering p, the strict-lower column structures of the
 * Cholesky-like factor of pattern(At + At^T):
 *    struct(j) = { i > j : B(i,j) != 0 }  U  union over children c of
 *                (struct(c) minus {j}),   parent(j) = min struct(j).
 * Returns lists in `cols` (one ilist per column) and parent[]. */
static int sym_column_structs(int64_t n, const int64_t *colptr, const int32_t *rowind,
                              const int32_t *q, ilist **cols_out, int32_t *parent) {
    ilist *low = (ilist *)calloc((size_t)n, sizeof(ilist));
    ilist *cols = (ilist *)calloc((size_t)n, sizeof(ilist));
    ilist *kids = (ilist *)calloc((size_t)n, sizeof(ilist));
    if (!low || !cols || !kids) return OR_E_NOMEM;
    for (int64_t j = 0; j < n; j++) {
        for (int64_t k = colptr[j]; k < colptr[j + 1]; k++) {
            int32_t a = q[rowind[k]], b = q[j];
            if (a == b) continue;
            int32_t hi = a > b ? a : b, lo = a > b ? b : a;
            if (ilist_push(&low[lo], hi)) return OR_E_NOMEM;
        }
    }
    for (int64_t j = 0; j < n; j++) {
        ilist *c = &cols[j];
        for (int64_t t = 0; t < low[j].n; t++)
            if (ilist_push(c, low[j].v[t])) return OR_E_NOMEM;
        for (int64_t t = 0; t < kids[j].n; t++) {
            ilist *kc = &cols[kids[j].v[t]];
            for (int64_t u = 0; u < kc->n; u++)
                if (kc->v[u] != j && ilist_push(c, kc->v[u])) return OR_E_NOMEM;
        }
        c->n = sort_unique(c->v, c->n);
        parent[j] = c->n ? c->v[0] : -1;
        if (parent[j] >= 0 && ilist_push(&kids[parent[j]], (int32_t)j)) return OR_E_NOMEM;
    }
    for (int64_t j = 0; j < n; j++) {
        free(low[j].v);
        free(kids[j].v);
    }
    free(low);
    free(kids);
    *cols_out = cols;
    return OR_OK;
}

static void free_cols(ilist *cols, int64_t n) {
    if (!cols) return;
    for (int64_t j = 0; j < n; j++) free(cols[j].v);
    free(cols);
}

/* postorder of the forest given by parent[], children in increasing order.
 * post[k] = node visited k-th. */
static int postorder(int64_t n, const int32_t *parent, int32_t *post) {
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *cursor = (int32_t *)malloc(sizeof(int32_t) * n);
    if (!head || !next || !stack || !cursor) return OR_E_NOMEM;
    for (int64_t j = 0; j < n; j++) head[j] = -1;
    /* build child lists in increasing order: insert from the largest down */
    for (int64_t j = n - 1; j >= 0; j--) {
        if (parent[j] >= 0) {
            next[j] = head[parent[j]];
            head[parent[j]] = (int32_t)j;
        }
    }
    int64_t k = 0;
    for (int64_t r = 0; r < n; r++) {
        if (parent[r] >= 0) continue;
        int64_t top = 0;
        stack[top] = (int32_t)r;
        cursor[r] = head[r];
        while (top >= 0) {
            int32_t v = stack[top];
            int32_t c = cursor[v];
            if (c >= 0) {
                cursor[v] = next[c];
                stack[++top] = c;
                cursor[c] = head[c];
            } else {
                post[k++] = v;
                top--;
            }
        }
    }
    free(head);
    free(next);
    free(stack);
    free(cursor);
    return k == n ? OR_OK : OR_E_INVALID_ARG;
}

/* ------------------------------------------------------------------------ */
/* partition                                                                */
/* ------------------------------------------------------------------------ */

/* Cut supernodes [first, last] (given by flag `start[j]`) at the cap and
 * write xsup. */
static int make_xsup(oracle_t *o, const char *start, int32_t max_super) {
    int64_t n = o->n;
    int32_t *xs = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    if (!xs) return OR_E_NOMEM;
    int32_t ns = 0;
    int64_t j = 0;
    while (j < n) {
        int64_t e = j + 1;
        while (e < n && !start[e]) e++;
        for (int64_t f = j; f < e; f += (max_super > 0 ? max_super : (e - j))) xs[ns++] = (int32_t)f;
        j = e;
    }
    xs[ns] = (int32_t)n;
    o->nsup = ns;
    o->xsup = xs;
    o->supof = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    if (!o->supof) return OR_E_NOMEM;
    for (int32_t K = 0; K < ns; K++)
        for (int32_t c = xs[K]; c < xs[K + 1]; c++) o->supof[c] = K;
    return OR_OK;
}

static int partition_sym(oracle_t *o, ilist *cols, const int32_t *parent, int32_t max_super,
                         int32_t relax, int32_t pad_pct) {
    int64_t n = o->n;
    int32_t *nkids = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int64_t *size = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    int32_t *relroot = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    char *start = (char *)calloc((size_t)n + 1, 1);
    if (!nkids || !size || !relroot || !start) return OR_E_NOMEM;
    for (int64_t j = 0; j < n; j++) size[j] = 1;
    for (int64_t j = 0; j < n; j++) { /* children precede parents */
        if (parent[j] >= 0) {
            nkids[parent[j]]++;
            size[parent[j]] += size[j];
        }
    }
    for (int64_t j = 0; j < n; j++) relroot[j] = -1;
    for (int64_t v = 0; v < n; v++) {
        if (size[v] <= relax && (parent[v] < 0 || size[parent[v]] > relax)) {
            for (int64_t u = v - size[v] + 1; u <= v; u++) relroot[u] = (int32_t)v;
        }
    }
    /* chain merge: j joins the supernode [f, j-1] when j-1's parent is j, j has
     * no other child, and the padding estimate of [f, j] stays within pad_pct
     * percent of its stored entries:  with s = j - f + 1 and cnt(t) the number
     * of off-diagonal entries of column t,
     *     Z = s cnt(j) - sum_{t=f..j} cnt(t) + s (s - 1) / 2,
     *     join  iff  100 Z <= pad_pct s (cnt(j) + s).
     * For identical structures (cnt(t) = cnt(j) + j - t) Z = 0. */
    int64_t f = 0, sumcnt = 0;
    for (int64_t j = 0; j < n; j++) {
        int join = 0;
        if (j > 0) {
            if (relroot[j] >= 0 || relroot[j - 1] >= 0) {
                join = relroot[j] >= 0 && relroot[j] == relroot[j - 1];
            } else if (parent[j - 1] == j && nkids[j] == 1) {
                int64_t sz = j - f + 1, cj = cols[j].n;
                int64_t Z = sz * cj - (sumcnt + cj) + sz * (sz - 1) / 2;
                join = 100 * Z <= (int64_t)pad_pct * sz * (cj + sz);
            }
        }
        start[j] = !join;
        if (!join) {
            f = j;
            sumcnt = 0;
        }
        sumcnt += cols[j].n;
    }
    int rc = make_xsup(o, start, max_super);
    free(nkids);
    free(size);
    free(relroot);
    free(start);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* block symbolic simulation, mode 0 (symmetric pattern)                    */
/* ------------------------------------------------------------------------ */
static int block_symbolic_sym(oracle_t *o) {
    int64_t n = o->n;
    int32_t ns = o->nsup;
    hmap lowset;
    ilist *rows = (ilist *)calloc((size_t)n + 1, sizeof(ilist)); /* rows r > c of column c */
    if (!rows) return OR_E_NOMEM;
    if (hmap_init(&lowset, o->nnz_a) != OR_OK) return OR_E_NOMEM;
    for (int64_t j = 0; j < n; j++) {
        for (int64_t k = o->a_colptr[j]; k < o->a_colptr[j + 1]; k++) {
            int32_t a = o->q[o->a_rowind[k]], b = o->q[j];
            if (a == b) continue;
            int32_t hi = a > b ? a : b, lo = a > b ? b : a;
            int ins;
            if (hmap_insert(&lowset, (int64_t)hi * n + lo, &ins) < 0) return OR_E_NOMEM;
            if (ins && ilist_push(&rows[lo], hi)) return OR_E_NOMEM;
        }
    }
    o->rl_ptr = (int64_t *)malloc(sizeof(int64_t) * (ns + 1));
    ilist R = {0};
    ilist all = {0};
    o->rl_ptr[0] = 0;
    for (int32_t K = 0; K < ns; K++) {
        int32_t f = o->xsup[K], l = o->xsup[K + 1] - 1;
        R.n = 0;
        for (int32_t c = f; c <= l; c++)
            for (int64_t t = 0; t < rows[c].n; t++)
                if (rows[c].v[t] > l && ilist_push(&R, rows[c].v[t])) return OR_E_NOMEM;
        R.n = sort_unique(R.v, R.n);
        /* fill: every pair (r1 > r2) of R becomes nonzero */
        for (int64_t a = 0; a < R.n; a++) {
            for (int64_t b = 0; b < a; b++) {
                int32_t r1 = R.v[a], r2 = R.v[b];
                int ins;
                if (hmap_insert(&lowset, (int64_t)r1 * n + r2, &ins) < 0) return OR_E_NOMEM;
                if (ins && ilist_push(&rows[r2], r1)) return OR_E_NOMEM;
            }
        }
        for (int64_t a = 0; a < R.n; a++)
            if (ilist_push(&all, R.v[a])) return OR_E_NOMEM;
        o->rl_ptr[K + 1] = all.n;
    }
    o->rl = all.v ? all.v : (int32_t *)malloc(4);
    o->ru_ptr = (int64_t *)malloc(sizeof(int64_t) * (ns + 1));
    o->ru = (int32_t *)malloc(sizeof(int32_t) * (all.n + 1));
    memcpy(o->ru_ptr, o->rl_ptr, sizeof(int64_t) * (ns + 1));
    if (all.n) memcpy(o->ru, o->rl, sizeof(int32_t) * all.n);
    free(R.v);
    for (int64_t j = 0; j < n; j++) free(rows[j].v);
    free(rows);
    hmap_free(&lowset);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* mode 1: exact non-symmetric structure (dense boolean, small n)            */
/* ------------------------------------------------------------------------ */
static int symbolic_exact(oracle_t *o, int32_t max_super) {
    int64_t n = o->n;
    if (n > 6000) {
        set_err(o, "exact mode is limited to n <= 6000");
        return OR_E_INVALID_ARG;
    }
    unsigned char *M = (unsigned char *)calloc((size_t)(n * n + 1), 1); /* M[r*n + c] */
    if (!M) return OR_E_NOMEM;
    for (int64_t j = 0; j < n; j++)
        for (int64_t k = o->a_colptr[j]; k < o->a_colptr[j + 1]; k++)
            M[(int64_t)o->q[o->a_rowind[k]] * n + o->q[j]] = 1;
    /* scalar elimination: L(i,k) != 0 and U(k,j) != 0 make (i,j) nonzero */
    for (int64_t k = 0; k < n; k++)
        for (int64_t i = k + 1; i < n; i++)
            if (M[i * n + k])
                for (int64_t j = k + 1; j < n; j++)
                    if (M[k * n + j]) M[i * n + j] = 1;
    /* fundamental supernodes: j joins j-1 when L(j,j-1) != 0 and the column
     * structures of j-1 and j agree strictly below row j */
    char *start = (char *)calloc((size_t)n + 1, 1);
    for (int64_t j = 0; j < n; j++) {
        int join = 0;
        if (j > 0 && M[j * n + (j - 1)]) {
            join = 1;
            for (int64_t i = j + 1; i < n && join; i++)
                if (M[i * n + (j - 1)] != M[i * n + j]) join = 0;
        }
        start[j] = !join;
    }
    int rc = make_xsup(o, start, max_super);
    free(start);
    if (rc) return rc;
    int32_t ns = o->nsup;
    ilist L = {0}, U = {0};
    o->rl_ptr = (int64_t *)malloc(sizeof(int64_t) * (ns + 1));
    o->ru_ptr = (int64_t *)malloc(sizeof(int64_t) * (ns + 1));
    o->rl_ptr[0] = o->ru_ptr[0] = 0;
    for (int32_t K = 0; K < ns; K++) {
        int64_t f = o->xsup[K], l = o->xsup[K + 1] - 1;
        int64_t l0 = L.n, u0 = U.n;
        for (int64_t r = l + 1; r < n; r++) {
            int hit = 0;
            for (int64_t t = f; t <= l && !hit; t++) hit = M[r * n + t];
            if (hit && ilist_push(&L, (int32_t)r)) return OR_E_NOMEM;
        }
        for (int64_t c = l + 1; c < n; c++) {
            int hit = 0;
            for (int64_t t = f; t <= l && !hit; t++) hit = M[t * n + c];
            if (hit && ilist_push(&U, (int32_t)c)) return OR_E_NOMEM;
        }
        for (int64_t a = l0; a < L.n; a++)
            for (int64_t b = u0; b < U.n; b++) M[(int64_t)L.v[a] * n + U.v[b]] = 1;
        o->rl_ptr[K + 1] = L.n;
        o->ru_ptr[K + 1] = U.n;
    }
    o->rl = L.v ? L.v : (int32_t *)malloc(4);
    o->ru = U.v ? U.v : (int32_t *)malloc(4);
    free(M);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* position set of the block pattern of L+U                                 */
/* ------------------------------------------------------------------------ */
static int build_positions(oracle_t *o) {
    int64_t n = o->n, total = 0;
    for (int32_t K = 0; K < o->nsup; K++) {
        int64_t s = o->xsup[K + 1] - o->xsup[K];
        total += s * s + s * (o->rl_ptr[K + 1] - o->rl_ptr[K]) + s * (o->ru_ptr[K + 1] - o->ru_ptr[K]);
    }
    if (hmap_init(&o->pos, total) != OR_OK) return OR_E_NOMEM;
    for (int32_t K = 0; K < o->nsup; K++) {
        int32_t f = o->xsup[K], l = o->xsup[K + 1] - 1;
        for (int32_t c = f; c <= l; c++)
            for (int32_t r = f; r <= l; r++)
                if (hmap_insert(&o->pos, (int64_t)r * n + c, NULL) < 0) return OR_E_NOMEM;
        for (int64_t a = o->rl_ptr[K]; a < o->rl_ptr[K + 1]; a++)
            for (int32_t c = f; c <= l; c++)
                if (hmap_insert(&o->pos, (int64_t)o->rl[a] * n + c, NULL) < 0) return OR_E_NOMEM;
        for (int64_t b = o->ru_ptr[K]; b < o->ru_ptr[K + 1]; b++)
            for (int32_t r = f; r <= l; r++)
                if (hmap_insert(&o->pos, (int64_t)r * n + o->ru[b], NULL) < 0) return OR_E_NOMEM;
    }
    o->lu = (double *)calloc((size_t)o->pos.count + 1, sizeof(double));
    o->z = (double *)calloc((size_t)o->pos.count + 1, sizeof(double));
    if (!o->lu || !o->z) return OR_E_NOMEM;
    return OR_OK;
}

static int64_t slot(const oracle_t *o, int64_t r, int64_t c) { return hmap_find(&o->pos, r * o->n + c); }

/* ------------------------------------------------------------------------ */
/* analyze                                                                  */
/* ------------------------------------------------------------------------ */
int oracle_analyze(int64_t n, const int64_t *colptr, const int32_t *rowind, const int32_t *perm,
                   int32_t max_super, int32_t relax, int32_t pad_pct, int32_t mode, oracle_t **out) {
    if (!out) return OR_E_INVALID_ARG;
    *out = NULL;
    oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
    if (!o) return OR_E_NOMEM;
    int rc = validate_csc(n, colptr, rowind);
    if (rc) {
        set_err(o, "bad CSC pattern");
        oracle_free(o);
        return rc;
    }
    o->n = n;
    o->nnz_a = colptr[n];
    o->a_colptr = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    o->a_rowind = (int32_t *)malloc(sizeof(int32_t) * (o->nnz_a + 1));
    o->p = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    o->q = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
    memcpy(o->a_colptr, colptr, sizeof(int64_t) * (n + 1));
    if (o->nnz_a) memcpy(o->a_rowind, rowind, sizeof(int32_t) * o->nnz_a);
    for (int64_t i = 0; i < n; i++) o->q[i] = -1;
    for (int64_t i = 0; i < n; i++) {
        int32_t v = perm ? perm[i] : (int32_t)i;
        if (v < 0 || v >= n || o->q[v] >= 0) {
            set_err(o, "perm is not a permutation");
            oracle_free(o);
            return OR_E_BAD_PERM;
        }
        o->p[i] = v;
        o->q[v] = (int32_t)i;
    }
    if (mode == 0) {
        int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
        int32_t *post = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
        ilist *cols = NULL;
        for (int pass = 0; pass < 2; pass++) {
            rc = sym_column_structs(n, colptr, rowind, o->q, &cols, parent);
            if (rc) break;
            rc = postorder(n, parent, post);
            if (rc) break;
            int identity = 1;
            for (int64_t k = 0; k < n; k++) identity &= post[k] == k;
            if (identity) break;
            if (pass == 1) {
                set_err(o, "postorder did not converge");
                rc = OR_E_INVALID_ARG;
                break;
            }
            /* relabel: new position k holds old position post[k] */
            int32_t *np = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
            for (int64_t k = 0; k < n; k++) np[k] = o->p[post[k]];
            memcpy(o->p, np, sizeof(int32_t) * n);
            for (int64_t k = 0; k < n; k++) o->q[o->p[k]] = (int32_t)k;
            free(np);
            free_cols(cols, n);
            cols = NULL;
        }
        if (!rc) rc = partition_sym(o, cols, parent, max_super, relax, pad_pct);
        free_cols(cols, n);
        free(parent);
        free(post);
        if (!rc) rc = block_symbolic_sym(o);
    } else if (mode == 1) {
        rc = symbolic_exact(o, max_super);
    } else {
        rc = OR_E_INVALID_ARG;
    }
    if (!rc) rc = build_positions(o);
    if (rc) {
        if (!o->err[0]) set_err(o, "analyze failed");
        oracle_free(o);
        return rc;
    }
    *out = o;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* factor: unpivoted supernodal LU, right-looking, on the block pattern      */
/* ------------------------------------------------------------------------ */
int oracle_factor(oracle_t *o, const double *values) {
    if (!o || !values) return OR_E_INVALID_ARG;
    int64_t n = o->n;
    for (int64_t i = 0; i < o->pos.count; i++) o->lu[i] = 0.0;
    for (int64_t j = 0; j < n; j++) {
        for (int64_t k = o->a_colptr[j]; k < o->a_colptr[j + 1]; k++) {
            int64_t s = slot(o, o->q[o->a_rowind[k]], o->q[j]);
            if (s < 0) {
                set_err(o, "entry of A outside the symbolic pattern");
                return OR_E_CLOSURE;
            }
            o->lu[s] = values[k];
        }
    }
    for (int32_t K = 0; K < o->nsup; K++) {
        int32_t f = o->xsup[K];
        int64_t s = o->xsup[K + 1] - f;
        int64_t cl = o->rl_ptr[K + 1] - o->rl_ptr[K], cu = o->ru_ptr[K + 1] - o->ru_ptr[K];
        const int32_t *RL = o->rl + o->rl_ptr[K], *RU = o->ru + o->ru_ptr[K];
        double *D = (double *)malloc(sizeof(double) * (s * s + 1));   /* D[r*s + c] */
        double *Lp = (double *)malloc(sizeof(double) * (cl * s + 1)); /* Lp[a*s + t] */
        double *Up = (double *)malloc(sizeof(double) * (s * cu + 1)); /* Up[t*cu + b] */
        if (!D || !Lp || !Up) return OR_E_NOMEM;
        for (int64_t r = 0; r < s; r++)
            for (int64_t c = 0; c < s; c++) D[r * s + c] = o->lu[slot(o, f + r, f + c)];
        /* dense LU without pivoting of the diagonal block */
        for (int64_t t = 0; t < s; t++) {
            double piv = D[t * s + t];
            if (piv == 0.0 || !isfinite(piv)) {
                snprintf(o->err, sizeof(o->err), "zero or non-finite pivot at permuted column %lld",
                         (long long)(f + t));
                free(D);
                free(Lp);
                free(Up);
                return OR_E_ZERO_PIVOT;
            }
            for (int64_t r = t + 1; r < s; r++) D[r * s + t] /= piv;
            for (int64_t r = t + 1; r < s; r++)
                for (int64_t c = t + 1; c < s; c++) D[r * s + c] -= D[r * s + t] * D[t * s + c];
        }
        /* L(R_L, K) = A(R_L, K) U_KK^{-1}: row by row, x U = a */
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < cl; a++) {
            double *x = Lp + a * s;
            for (int64_t t = 0; t < s; t++) x[t] = o->lu[slot(o, RL[a], f + t)];
            for (int64_t t = 0; t < s; t++) {
                double acc = x[t];
                for (int64_t u = 0; u < t; u++) acc -= x[u] * D[u * s + t];
                x[t] = acc / D[t * s + t];
            }
        }
        /* U(K, R_U) = L_KK^{-1} A(K, R_U): column by column, L y = a */
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < cu; b++) {
            for (int64_t t = 0; t < s; t++) Up[t * cu + b] = o->lu[slot(o, f + t, RU[b])];
            for (int64_t t = 0; t < s; t++) {
                double acc = Up[t * cu + b];
                for (int64_t u = 0; u < t; u++) acc -= D[t * s + u] * Up[u * cu + b];
                Up[t * cu + b] = acc;
            }
        }
        for (int64_t r = 0; r < s; r++)
            for (int64_t c = 0; c < s; c++) o->lu[slot(o, f + r, f + c)] = D[r * s + c];
        for (int64_t a = 0; a < cl; a++)
            for (int64_t t = 0; t < s; t++) o->lu[slot(o, RL[a], f + t)] = Lp[a * s + t];
        for (int64_t t = 0; t < s; t++)
            for (int64_t b = 0; b < cu; b++) o->lu[slot(o, f + t, RU[b])] = Up[t * cu + b];
        /* Schur complement update of the trailing matrix */
        int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
        for (int64_t a = 0; a < cl; a++) {
            for (int64_t b = 0; b < cu; b++) {
                double acc = 0.0;
                for (int64_t t = 0; t < s; t++) acc += Lp[a * s + t] * Up[t * cu + b];
                int64_t sl = slot(o, RL[a], RU[b]);
                if (sl < 0) {
                    bad = 1;
                    continue;
                }
                o->lu[sl] -= acc;
            }
        }
        free(D);
        free(Lp);
        free(Up);
        if (bad) {
            set_err(o, "Schur update outside the block pattern");
            return OR_E_CLOSURE;
        }
    }
    o->state = 1;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* selected inversion: Algorithm 1, steps 2-5                               */
/* ------------------------------------------------------------------------ */
int oracle_selinv(oracle_t *o) {
    if (!o) return OR_E_INVALID_ARG;
    if (o->state < 1) {
        set_err(o, "selinv before factor");
        return OR_E_STATE;
    }
    int32_t ns = o->nsup;
    double **Lh = (double **)calloc((size_t)ns + 1, sizeof(double *)); /* Lh[K][a*s+t] */
    double **Uh = (double **)calloc((size_t)ns + 1, sizeof(double *)); /* Uh[K][t*cu+b] */
    double **Dt = (double **)calloc((size_t)ns + 1, sizeof(double *)); /* (L^-T U^-T)[t*s+t2] */
    if (!Lh || !Uh || !Dt) return OR_E_NOMEM;
    int nomem = 0;
    /* step 2, for every supernode */
#pragma omp parallel for schedule(dynamic, 1) reduction(| : nomem)
    for (int32_t K = 0; K < ns; K++) {
        int32_t f = o->xsup[K];
        int64_t s = o->xsup[K + 1] - f;
        int64_t cl = o->rl_ptr[K + 1] - o->rl_ptr[K], cu = o->ru_ptr[K + 1] - o->ru_ptr[K];
        const int32_t *RL = o->rl + o->rl_ptr[K], *RU = o->ru + o->ru_ptr[K];
        double *D = (double *)malloc(sizeof(double) * (s * s + 1));
        double *Li = (double *)calloc((size_t)(s * s + 1), sizeof(double)); /* Li[r*s+c] */
        double *Ui = (double *)calloc((size_t)(s * s + 1), sizeof(double));
        Lh[K] = (double *)malloc(sizeof(double) * (cl * s + 1));
        Uh[K] = (double *)malloc(sizeof(double) * (s * cu + 1));
        Dt[K] = (double *)malloc(sizeof(double) * (s * s + 1));
        if (!D || !Li || !Ui || !Lh[K] || !Uh[K] || !Dt[K]) {
            nomem = 1;
            continue;
        }
        for (int64_t r = 0; r < s; r++)
            for (int64_t c = 0; c < s; c++) D[r * s + c] = o->lu[slot(o, f + r, f + c)];
        /* (L_KK)^{-1}: unit lower; column c solves L x = e_c */
        for (int64_t c = 0; c < s; c++) {
            Li[c * s + c] = 1.0;
            for (int64_t r = c + 1; r < s; r++) {
                double acc = 0.0;
                for (int64_t k = c; k < r; k++) acc += D[r * s + k] * Li[k * s + c];
                Li[r * s + c] = -acc;
            }
        }
        /* (U_KK)^{-1}: upper; column c solves U x = e_c by back substitution */
        for (int64_t c = 0; c < s; c++) {
            for (int64_t r = c; r >= 0; r--) {
                double acc = (r == c) ? 1.0 : 0.0;
                for (int64_t k = r + 1; k <= c; k++) acc -= D[r * s + k] * Ui[k * s + c];
                Ui[r * s + c] = acc / D[r * s + r];
            }
        }
        /* Lhat(R_L, K) = L(R_L, K) (L_KK)^{-1}  (row a of L(R_L, K) looked up once) */
        double *lrow = (double *)malloc(sizeof(double) * (s + 1));
        if (!lrow) {
            nomem = 1;
            continue;
        }
        for (int64_t a = 0; a < cl; a++) {
            for (int64_t k = 0; k < s; k++) lrow[k] = o->lu[slot(o, RL[a], f + k)];
            for (int64_t t = 0; t < s; t++) {
                double acc = 0.0;
                for (int64_t k = 0; k < s; k++) acc += lrow[k] * Li[k * s + t];
                Lh[K][a * s + t] = acc;
            }
        }
        /* Uhat(K, R_U) = (U_KK)^{-1} U(K, R_U)  (column b of U(K, R_U) looked up once) */
        double *ucol = lrow;
        for (int64_t b = 0; b < cu; b++) {
            for (int64_t k = 0; k < s; k++) ucol[k] = o->lu[slot(o, f + k, RU[b])];
            for (int64_t t = 0; t < s; t++) {
                double acc = 0.0;
                for (int64_t k = 0; k < s; k++) acc += Ui[t * s + k] * ucol[k];
                Uh[K][t * cu + b] = acc;
            }
        }
        free(lrow);
        /* (L_KK)^{-T} (U_KK)^{-T}, entry (t, t2) = sum_k Li(k, t) Ui(t2, k) */
        for (int64_t t = 0; t < s; t++)
            for (int64_t t2 = 0; t2 < s; t2++) {
                double acc = 0.0;
                for (int64_t k = 0; k < s; k++) acc += Li[k * s + t] * Ui[t2 * s + k];
                Dt[K][t * s + t2] = acc;
            }
        free(D);
        free(Li);
        free(Ui);
    }
    if (nomem) return OR_E_NOMEM;

    double altdiff = 0.0, altabs = 0.0;
    int missing = 0;
    for (int32_t K = ns - 1; K >= 0; K--) {
        int32_t f = o->xsup[K];
        int64_t s = o->xsup[K + 1] - f;
        int64_t cl = o->rl_ptr[K + 1] - o->rl_ptr[K], cu = o->ru_ptr[K + 1] - o->ru_ptr[K];
        const int32_t *RL = o->rl + o->rl_ptr[K], *RU = o->ru + o->ru_ptr[K];
        double *G = (double *)malloc(sizeof(double) * (cl * cu + 1)); /* G[a*cu + b] */
        double *X = (double *)malloc(sizeof(double) * (s * cu + 1));  /* X[t*cu + b] */
        double *Y = (double *)malloc(sizeof(double) * (cl * s + 1));  /* Y[a*s + t] */
        double *Z = (double *)malloc(sizeof(double) * (s * s + 1));   /* Z[t*s + t2] */
        if (!G || !X || !Y || !Z) return OR_E_NOMEM;
        /* gather G = A^{-T}(R_L, R_U) from entries computed earlier in the loop */
#pragma omp parallel for schedule(static) reduction(| : missing)
        for (int64_t a = 0; a < cl; a++)
            for (int64_t b = 0; b < cu; b++) {
                int64_t sl = slot(o, RL[a], RU[b]);
                if (sl < 0) {
                    missing = 1;
                    G[a * cu + b] = 0.0;
                } else {
                    G[a * cu + b] = o->z[sl];
                }
            }
        if (missing) {
            free(G);
            free(X);
            free(Y);
            free(Z);
            set_err(o, "an entry of A^{-T}(R_L, R_U) is outside the block pattern");
            return OR_E_CLOSURE;
        }
        /* step 3: X = A^{-T}(K, R_U) = -Lhat(R_L, K)^T G.  Every entry X(t, b)
         * sums its terms in increasing a; the sums of one row t advance
         * together so that the inner loop runs along a row of G. */
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < s; t++) {
            double *acc = X + t * cu;
            for (int64_t b = 0; b < cu; b++) acc[b] = 0.0;
            for (int64_t a = 0; a < cl; a++) {
                const double l = Lh[K][a * s + t];
                const double *g = G + a * cu;
                for (int64_t b = 0; b < cu; b++) acc[b] += l * g[b];
            }
            for (int64_t b = 0; b < cu; b++) acc[b] = -acc[b];
        }
        /* step 4: Z = (L_KK)^{-T}(U_KK)^{-T} - X Uhat(K, R_U)^T */
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < s; t++)
            for (int64_t t2 = 0; t2 < s; t2++) {
                double acc = 0.0;
                for (int64_t b = 0; b < cu; b++) acc += X[t * cu + b] * Uh[K][t2 * cu + b];
                Z[t * s + t2] = Dt[K][t * s + t2] - acc;
            }
        /* step 5: Y = A^{-T}(R_L, K) = -G Uhat(K, R_U)^T */
#pragma omp parallel for schedule(static)
        for (int64_t a = 0; a < cl; a++)
            for (int64_t t = 0; t < s; t++) {
                double acc = 0.0;
                for (int64_t b = 0; b < cu; b++) acc += G[a * cu + b] * Uh[K][t * cu + b];
                Y[a * s + t] = -acc;
            }
        /* the other diagonal formula, (L_KK)^{-T}(U_KK)^{-T} - Lhat^T Y, as a check
         * (each sum in increasing a, the sums of one row t together) */
#pragma omp parallel for schedule(static) reduction(max : altdiff, altabs)
        for (int64_t t = 0; t < s; t++) {
            double *acc = (double *)calloc((size_t)s + 1, sizeof(double));
            if (!acc) {
                altdiff = INFINITY;
                continue;
            }
            for (int64_t a = 0; a < cl; a++) {
                const double l = Lh[K][a * s + t];
                const double *y = Y + a * s;
                for (int64_t t2 = 0; t2 < s; t2++) acc[t2] += l * y[t2];
            }
            for (int64_t t2 = 0; t2 < s; t2++) {
                double alt = Dt[K][t * s + t2] - acc[t2];
                double d = fabs(alt - Z[t * s + t2]);
                if (d > altdiff) altdiff = d;
                if (fabs(Z[t * s + t2]) > altabs) altabs = fabs(Z[t * s + t2]);
            }
            free(acc);
        }
        for (int64_t t = 0; t < s; t++)
            for (int64_t b = 0; b < cu; b++) o->z[slot(o, f + t, RU[b])] = X[t * cu + b];
        for (int64_t t = 0; t < s; t++)
            for (int64_t t2 = 0; t2 < s; t2++) o->z[slot(o, f + t, f + t2)] = Z[t * s + t2];
        for (int64_t a = 0; a < cl; a++)
            for (int64_t t = 0; t < s; t++) o->z[slot(o, RL[a], f + t)] = Y[a * s + t];
        free(G);
        free(X);
        free(Y);
        free(Z);
    }
    for (int32_t K = 0; K < ns; K++) {
        free(Lh[K]);
        free(Uh[K]);
        free(Dt[K]);
    }
    free(Lh);
    free(Uh);
    free(Dt);
    o->diag_alt_maxdiff = altdiff;
    o->diag_alt_maxabs = altabs;
    o->state = 2;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* step 6: extraction (undo the permutation and transpose)                   */
/* ------------------------------------------------------------------------ */

/* A^{-1}(i, j) = At^{-T}(q[j], q[i])   (eq. unpermute with Q = P^T) */
int oracle_get(oracle_t *o, int64_t i, int64_t j, double *out) {
    if (!o || !out || i < 0 || j < 0 || i >= o->n || j >= o->n) return OR_E_INVALID_ARG;
    if (o->state < 2) return OR_E_STATE;
    int64_t sl = slot(o, o->q[j], o->q[i]);
    if (sl < 0) return OR_E_NOT_SELECTED;
    *out = o->z[sl];
    return OR_OK;
}

/* out[p] = A^{-1}(j, i) for the p-th stored entry (i, j) of A */
int oracle_get_selected(oracle_t *o, double *out) {
    if (!o || !out) return OR_E_INVALID_ARG;
    if (o->state < 2) return OR_E_STATE;
    for (int64_t j = 0; j < o->n; j++)
        for (int64_t k = o->a_colptr[j]; k < o->a_colptr[j + 1]; k++) {
            int64_t sl = slot(o, o->q[o->a_rowind[k]], o->q[j]);
            if (sl < 0) return OR_E_NOT_SELECTED;
            out[k] = o->z[sl];
        }
    return OR_OK;
}

int64_t oracle_superset_nnz(oracle_t *o) { return o ? o->pos.count : -1; }

/* Every computed entry as A^{-1}(row, col) in original indices. */
int oracle_export(oracle_t *o, int32_t *row, int32_t *col, double *val) {
    if (!o || !row || !col || !val) return OR_E_INVALID_ARG;
    if (o->state < 2) return OR_E_STATE;
    int64_t k = 0;
    for (int64_t s = 0; s < o->pos.cap; s++) {
        int64_t key = o->pos.keys[s];
        if (key < 0) continue;
        int64_t r = key / o->n, c = key % o->n; /* At^{-T}(r, c) = A^{-1}(p[c], p[r]) */
        row[k] = o->p[c];
        col[k] = o->p[r];
        val[k] = o->z[o->pos.idx[s]];
        k++;
    }
    return k == o->pos.count ? OR_OK : OR_E_INVALID_ARG;
}

/* structure queries (for comparing partitions exactly) */
int32_t oracle_nsuper(oracle_t *o) { return o ? o->nsup : -1; }
int64_t oracle_rl_total(oracle_t *o) { return o ? o->rl_ptr[o->nsup] : -1; }
int64_t oracle_ru_total(oracle_t *o) { return o ? o->ru_ptr[o->nsup] : -1; }

int oracle_structure(oracle_t *o, int32_t *perm_out, int32_t *xsup, int64_t *rl_ptr, int32_t *rl,
                     int64_t *ru_ptr, int32_t *ru) {
    if (!o) return OR_E_INVALID_ARG;
    if (perm_out) memcpy(perm_out, o->p, sizeof(int32_t) * o->n);
    if (xsup) memcpy(xsup, o->xsup, sizeof(int32_t) * (o->nsup + 1));
    if (rl_ptr) memcpy(rl_ptr, o->rl_ptr, sizeof(int64_t) * (o->nsup + 1));
    if (rl) memcpy(rl, o->rl, sizeof(int32_t) * o->rl_ptr[o->nsup]);
    if (ru_ptr) memcpy(ru_ptr, o->ru_ptr, sizeof(int64_t) * (o->nsup + 1));
    if (ru) memcpy(ru, o->ru, sizeof(int32_t) * o->ru_ptr[o->nsup]);
    return OR_OK;
}

void oracle_diag_alt(oracle_t *o, double *maxdiff, double *maxabs) {
    if (!o) return;
    if (maxdiff) *maxdiff = o->diag_alt_maxdiff;
    if (maxabs) *maxabs = o->diag_alt_maxabs;
}

/* ------------------------------------------------------------------------ */
/* entry from given factors (for block-structure fixtures)                   */
/* ------------------------------------------------------------------------ */
/* Supernodal structure and dense factors of an already permuted matrix:
 * xsup (nsup+1), rl_ptr/rl and ru_ptr/ru (sorted block rows/columns), and the
 * n x n column-major arrays L (unit lower; its diagonal is ignored) and U
 * (upper).  Entries of L/U outside the block pattern must be zero; this is
 * checked.  The permutation is the identity. */
int oracle_from_factors(int64_t n, int32_t nsup, const int32_t *xsup, const int64_t *rl_ptr,
                        const int32_t *rl, const int64_t *ru_ptr, const int32_t *ru,
                        const double *L, const double *U, oracle_t **out) {
    if (!out || n <= 0 || nsup <= 0) return OR_E_INVALID_ARG;
    *out = NULL;
    oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
    if (!o) return OR_E_NOMEM;
    o->n = n;
    o->nsup = nsup;
    o->p = (int32_t *)malloc(sizeof(int32_t) * n);
    o->q = (int32_t *)malloc(sizeof(int32_t) * n);
    for (int64_t i = 0; i < n; i++) o->p[i] = o->q[i] = (int32_t)i;
    o->xsup = (int32_t *)malloc(sizeof(int32_t) * (nsup + 1));
    memcpy(o->xsup, xsup, sizeof(int32_t) * (nsup + 1));
    o->supof = (int32_t *)malloc(sizeof(int32_t) * n);
    for (int32_t K = 0; K < nsup; K++)
        for (int32_t c = xsup[K]; c < xsup[K + 1]; c++) o->supof[c] = K;
    o->rl_ptr = (int64_t *)malloc(sizeof(int64_t) * (nsup + 1));
    o->ru_ptr = (int64_t *)malloc(sizeof(int64_t) * (nsup + 1));
    memcpy(o->rl_ptr, rl_ptr, sizeof(int64_t) * (nsup + 1));
    memcpy(o->ru_ptr, ru_ptr, sizeof(int64_t) * (nsup + 1));
    o->rl = (int32_t *)malloc(sizeof(int32_t) * (rl_ptr[nsup] + 1));
    o->ru = (int32_t *)malloc(sizeof(int32_t) * (ru_ptr[nsup] + 1));
    if (rl_ptr[nsup]) memcpy(o->rl, rl, sizeof(int32_t) * rl_ptr[nsup]);
    if (ru_ptr[nsup]) memcpy(o->ru, ru, sizeof(int32_t) * ru_ptr[nsup]);
    int rc = build_positions(o);
    if (rc) {
        oracle_free(o);
        return rc;
    }
    for (int64_t c = 0; c < n; c++)
        for (int64_t r = 0; r < n; r++) {
            double v = r > c ? L[c * n + r] : U[c * n + r];
            int64_t sl = slot(o, r, c);
            if (sl < 0) {
                if (v != 0.0) {
                    set_err(o, "factor entry outside the given block pattern");
                    oracle_free(o);
                    return OR_E_BAD_PATTERN;
                }
                continue;
            }
            o->lu[sl] = v;
        }
    o->state = 1;
    *out = o;
    return OR_OK;
}
