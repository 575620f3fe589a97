/*
 * dls_oracle.c -- plain CPU oracle for counting diagonal Latin squares.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  The product path
 * (the HIP library under paper_1709_02599_amd/) never calls it, and the two
 * share no code, headers, tables or helpers.
 *
 * Everything here follows Kochemazov, Vatutin, Zaikin, "Fast Algorithm for
 * Enumerating Diagonal Latin Squares of Small Order" (arXiv:1709.02599), and
 * is written to be checked against the paper by eye, not to be fast:
 *
 *  - the object counted is the definition of Sec. 1: an N x N array over
 *    {0..N-1} whose rows, columns, main diagonal and main antidiagonal each
 *    hold every value once; "vertically symmetric" (VS) additionally asks
 *    a[i][j] + a[i][N-1-j] = N-1 (Sec. 1 and the formula of Sec. 5.4);
 *  - the search is the nested-loop scheme of Algorithms 1 and 2 (Sec. 2.2):
 *    boolean occupancy arrays Rows[N][N], Columns[N][N], MD[N], AD[N]; each
 *    cell tries the values 0..N-1 in turn, skips occupied ones, marks,
 *    descends, unmarks.  The cell order is a fixed simple one (main diagonal
 *    top-down, then antidiagonal top-down, then every other cell row-major);
 *    Sec. 2.3 makes the point that the order changes speed, never the count;
 *  - VS is checked as a plain constraint once both cells of a mirror pair
 *    hold values (not by filling half the square as Sec. 5.4 does);
 *  - symmetry breaking follows Sec. 4: the M-transformations of Sec. 4.1
 *    acting on hourglass designs (Sec. 4.2), renormalised so that row 0 is
 *    0..N-1, canonical form = lexicographically least image in row-major
 *    order of the known cells, class power = number of distinct images
 *    (Algorithm 5, Corollary 1).  The transformation group is built here by
 *    closing a small generator set under composition -- a different
 *    construction from a product of transformation tables.
 *
 * Cells are uint8 in row-major order, 0xFF meaning "not assigned".
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define OR_MAXN 16
#define OR_EMPTY 0xFF

/* ------------------------------------------------------------------------ */
/* Counting completions of a partial square (Sec. 1 definition, Alg. 1/2).  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n;
    int vs;                              /* 1: enforce vertical symmetry     */
    int ls[OR_MAXN][OR_MAXN];            /* LS[i][j], -1 = empty             */
    unsigned char rows[OR_MAXN][OR_MAXN];/* Rows[i][v] = 1: v used in row i  */
    unsigned char cols[OR_MAXN][OR_MAXN];/* Columns[j][v]                    */
    unsigned char md[OR_MAXN];           /* MD[v]                            */
    unsigned char ad[OR_MAXN];           /* AD[v]                            */
    int order[OR_MAXN * OR_MAXN];        /* cells still to fill, as i*n+j    */
    int norder;
    uint64_t count;                      /* SquaresCnt                       */
} or_state;

/* Can value v go into cell (i,j) given everything assigned so far? */
static int or_allowed(const or_state *s, int i, int j, int v)
{
    int n = s->n;
    if (s->rows[i][v] || s->cols[j][v]) return 0;
    if (i == j && s->md[v]) return 0;
    if (i + j == n - 1 && s->ad[v]) return 0;
    if (s->vs) {
        int pj = n - 1 - j;              /* mirror cell (i, n-1-j)           */
        if (pj == j) {
            if (v + v != n - 1) return 0;
        } else if (s->ls[i][pj] >= 0 && s->ls[i][pj] + v != n - 1) {
            return 0;
        }
    }
    return 1;
}

static void or_mark(or_state *s, int i, int j, int v, int on)
{
    int n = s->n;
    s->rows[i][v] = (unsigned char)on;
    s->cols[j][v] = (unsigned char)on;
    if (i == j) s->md[v] = (unsigned char)on;
    if (i + j == n - 1) s->ad[v] = (unsigned char)on;
    s->ls[i][j] = on ? v : -1;
}

/* Load the fixed cells.  Returns 0 if they already break a constraint. */
static int or_load(or_state *s, int n, int vs, const uint8_t *cells)
{
    memset(s, 0, sizeof(*s));
    s->n = n;
    s->vs = vs;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) s->ls[i][j] = -1;
    for (int c = 0; c < n * n; c++) {
        int v = cells[c];
        if (v == OR_EMPTY) continue;
        int i = c / n, j = c % n;
        if (!or_allowed(s, i, j, v)) return 0;
        or_mark(s, i, j, v, 1);
    }
    return 1;
}

/* The oracle's fixed fill order: main diagonal top-down, antidiagonal
 * top-down, then every remaining cell row-major; assigned cells skipped. */
static void or_make_order(or_state *s)
{
    int n = s->n;
    unsigned char taken[OR_MAXN * OR_MAXN];
    memset(taken, 0, sizeof(taken));
    s->norder = 0;
    for (int i = 0; i < n; i++) {
        int c = i * n + i;
        if (!taken[c] && s->ls[i][i] < 0) s->order[s->norder++] = c;
        taken[c] = 1;
    }
    for (int i = 0; i < n; i++) {
        int c = i * n + (n - 1 - i);
        if (!taken[c] && s->ls[i][n - 1 - i] < 0) s->order[s->norder++] = c;
        taken[c] = 1;
    }
    for (int c = 0; c < n * n; c++) {
        if (!taken[c] && s->ls[c / n][c % n] < 0) s->order[s->norder++] = c;
        taken[c] = 1;
    }
}

/* One nested loop of Algorithm 2, written as recursion over the order. */
static void or_recurse(or_state *s, int k)
{
    if (k == s->norder) {                /* every cell filled: one square    */
        s->count++;
        return;
    }
    int n = s->n;
    int c = s->order[k], i = c / n, j = c % n;
    for (int v = 0; v < n; v++) {
        if (!or_allowed(s, i, j, v)) continue;
        or_mark(s, i, j, v, 1);
        or_recurse(s, k + 1);
        or_mark(s, i, j, v, 0);
    }
}

static int or_check_args(int n, const uint8_t *cells)
{
    if (n < 1 || n > OR_MAXN) return 0;
    for (int c = 0; c < n * n; c++)
        if (cells[c] != OR_EMPTY && cells[c] >= n) return 0;
    return 1;
}

/* Number of DLS (VS-DLS if vs) of order n agreeing with the assigned cells.
 * Returns -1 on invalid arguments. */
int64_t oracle_count(int n, int vs, const uint8_t *cells)
{
    if (!or_check_args(n, cells)) return -1;
    or_state *s = (or_state *)malloc(sizeof(or_state));
    if (!s) return -1;
    int64_t result = 0;
    if (or_load(s, n, vs, cells)) {
        or_make_order(s);
        or_recurse(s, 0);
        result = (int64_t)s->count;
    }
    free(s);
    return result;
}

/* ---- one completion: the same nested loops, stopping at the first square.
 * Used to build complete squares of larger orders as test inputs (the
 * near-complete prefixes that pin the counts of orders 11-16).  Value k of
 * cell c is tried in the order given by value_order[c*n + k] (a permutation
 * of 0..n-1 per cell, drawn by the caller; NULL = 0..n-1). */

typedef struct {
    or_state st;
    const uint8_t *value_order;
    int64_t nodes, limit;
} or_first;

static int or_first_rec(or_first *f, int k)
{
    or_state *s = &f->st;
    if (k == s->norder) return 1;
    if (++f->nodes > f->limit) return -1;
    int n = s->n;
    int c = s->order[k], i = c / n, j = c % n;
    for (int t = 0; t < n; t++) {
        int v = f->value_order ? f->value_order[c * n + t] : t;
        if (!or_allowed(s, i, j, v)) continue;
        or_mark(s, i, j, v, 1);
        int r = or_first_rec(f, k + 1);
        if (r) return r;                 /* found (cells stay marked) or limit */
        or_mark(s, i, j, v, 0);
    }
    return 0;
}

/* 1: out (n*n) holds a square agreeing with cells; 0: none exists;
 * -1: invalid arguments or more than node_limit cells entered. */
int oracle_first(int n, int vs, const uint8_t *cells, const uint8_t *value_order,
                 int64_t node_limit, uint8_t *out)
{
    if (!or_check_args(n, cells)) return -1;
    if (value_order)
        for (int c = 0; c < n * n; c++) {
            int seen = 0;
            for (int t = 0; t < n; t++) {
                int v = value_order[c * n + t];
                if (v >= n || (seen >> v) & 1) return -1;
                seen |= 1 << v;
            }
        }
    or_first *f = (or_first *)malloc(sizeof(or_first));
    if (!f) return -1;
    f->value_order = value_order;
    f->nodes = 0;
    f->limit = node_limit;
    int r = 0;
    if (or_load(&f->st, n, vs, cells)) {
        or_make_order(&f->st);
        r = or_first_rec(f, 0);
        if (r == 1)
            for (int c = 0; c < n * n; c++) out[c] = (uint8_t)f->st.ls[c / n][c % n];
    }
    free(f);
    return r;
}

/* ---- many prefixes on a pool of threads (independent subproblems, Sec. 5.2) */

typedef struct {
    int n, vs;
    const uint8_t *prefixes;
    int64_t num;
    uint64_t *counts;
    int64_t next;                        /* shared work index                */
    pthread_mutex_t lock;
    int bad;
} or_pool;

static void *or_pool_worker(void *arg)
{
    or_pool *pl = (or_pool *)arg;
    for (;;) {
        pthread_mutex_lock(&pl->lock);
        int64_t k = pl->next++;
        pthread_mutex_unlock(&pl->lock);
        if (k >= pl->num) break;
        int64_t r = oracle_count(pl->n, pl->vs, pl->prefixes + k * pl->n * pl->n);
        if (r < 0) { pl->bad = 1; r = 0; }
        pl->counts[k] = (uint64_t)r;
    }
    return NULL;
}

int oracle_count_many(int n, int vs, const uint8_t *prefixes, int64_t num,
                      uint64_t *counts, int threads)
{
    if (n < 1 || n > OR_MAXN || num < 0) return -1;
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    or_pool pl;
    pl.n = n; pl.vs = vs; pl.prefixes = prefixes; pl.num = num;
    pl.counts = counts; pl.next = 0; pl.bad = 0;
    pthread_mutex_init(&pl.lock, NULL);
    pthread_t th[256];
    for (int t = 0; t < threads; t++) pthread_create(&th[t], NULL, or_pool_worker, &pl);
    for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&pl.lock);
    return pl.bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Assignments of a given list of cells (the workunits of Sec. 5.2).        */
/* ------------------------------------------------------------------------ */

typedef struct {
    or_state st;
    const int *cells;
    int k;
    uint8_t *out;
    int64_t cap, found;
} or_enum;

static void or_enum_rec(or_enum *e, int t)
{
    or_state *s = &e->st;
    int n = s->n;
    if (t == e->k) {
        if (e->out && e->found < e->cap) {
            uint8_t *dst = e->out + e->found * n * n;
            for (int c = 0; c < n * n; c++) {
                int v = s->ls[c / n][c % n];
                dst[c] = (uint8_t)(v < 0 ? OR_EMPTY : v);
            }
        }
        e->found++;
        return;
    }
    int c = e->cells[t], i = c / n, j = c % n;
    for (int v = 0; v < n; v++) {
        if (!or_allowed(s, i, j, v)) continue;
        or_mark(s, i, j, v, 1);
        or_enum_rec(e, t + 1);
        or_mark(s, i, j, v, 0);
    }
}

/* Every assignment of the listed (empty) cells that keeps all constraints
 * among assigned cells, each written as a full square.  Returns how many
 * exist (writes at most cap of them), or -1 on invalid input. */
int64_t oracle_assignments(int n, int vs, const uint8_t *base, const int *cells,
                           int k, uint8_t *out, int64_t cap)
{
    if (!or_check_args(n, base) || k < 0 || k > n * n) return -1;
    for (int t = 0; t < k; t++) {
        if (cells[t] < 0 || cells[t] >= n * n || base[cells[t]] != OR_EMPTY) return -1;
        for (int u = 0; u < t; u++) if (cells[u] == cells[t]) return -1;
    }
    or_enum *e = (or_enum *)malloc(sizeof(or_enum));
    if (!e) return -1;
    int64_t r = 0;
    if (or_load(&e->st, n, vs, base)) {
        e->cells = cells; e->k = k; e->out = out; e->cap = cap; e->found = 0;
        or_enum_rec(e, 0);
        r = e->found;
    }
    free(e);
    return r;
}

/* ------------------------------------------------------------------------ */
/* M-transformations (Sec. 4.1) as pairs (p, q): T[i][j] = H[p(i)][q(j)].   */
/* ------------------------------------------------------------------------ */

#define OR_MAXG 4096

typedef struct { signed char p[OR_MAXN], q[OR_MAXN]; } or_perm2;

static int or_same(const or_perm2 *a, const or_perm2 *b, int n)
{
    return memcmp(a->p, b->p, (size_t)n) == 0 && memcmp(a->q, b->q, (size_t)n) == 0;
}

/* (a o b)(x) = a(b(x)) on both coordinates. */
static or_perm2 or_compose(const or_perm2 *a, const or_perm2 *b, int n)
{
    or_perm2 r;
    memset(&r, 0, sizeof(r));
    for (int x = 0; x < n; x++) {
        r.p[x] = a->p[(int)b->p[x]];
        r.q[x] = a->q[(int)b->q[x]];
    }
    return r;
}

/* The transformations that map hourglass designs to hourglass designs
 * (Sec. 4.2): generated by the vertical mirror (type 1), the swap of one
 * symmetric row pair together with the matching column pair (type 2), and
 * the exchange of two neighbouring symmetric pairs k, k+1 with k >= 1 (type 3
 * restricted to pairs other than the pair of the first and last rows, which
 * must stay rows 0 and N-1).  Closed under composition by breadth-first
 * search.  Writes the elements into g (capacity cap); returns their number,
 * or -1. */
int oracle_hourglass_group(int n, signed char *p_out, signed char *q_out, int cap)
{
    if (n < 1 || n > OR_MAXN) return -1;
    int m = n / 2;
    or_perm2 gens[2 * OR_MAXN + 1];
    int ng = 0;
    or_perm2 id;
    memset(&id, 0, sizeof(id));
    for (int x = 0; x < n; x++) { id.p[x] = (signed char)x; id.q[x] = (signed char)x; }
    /* vertical mirror: columns reversed, rows kept */
    gens[ng] = id;
    for (int x = 0; x < n; x++) gens[ng].q[x] = (signed char)(n - 1 - x);
    ng++;
    /* swap rows k <-> n-1-k and columns k <-> n-1-k */
    for (int k = 0; k < m; k++) {
        gens[ng] = id;
        gens[ng].p[k] = gens[ng].q[k] = (signed char)(n - 1 - k);
        gens[ng].p[n - 1 - k] = gens[ng].q[n - 1 - k] = (signed char)k;
        ng++;
    }
    /* exchange pair k with pair k+1 (k >= 1), rows and columns alike */
    for (int k = 1; k + 1 < m; k++) {
        gens[ng] = id;
        gens[ng].p[k] = gens[ng].q[k] = (signed char)(k + 1);
        gens[ng].p[k + 1] = gens[ng].q[k + 1] = (signed char)k;
        gens[ng].p[n - 1 - k] = gens[ng].q[n - 1 - k] = (signed char)(n - 2 - k);
        gens[ng].p[n - 2 - k] = gens[ng].q[n - 2 - k] = (signed char)(n - 1 - k);
        ng++;
    }
    or_perm2 *grp = (or_perm2 *)malloc(sizeof(or_perm2) * OR_MAXG);
    if (!grp) return -1;
    int size = 0;
    grp[size++] = id;
    for (int head = 0; head < size; head++) {
        for (int t = 0; t < ng; t++) {
            or_perm2 e = or_compose(&grp[head], &gens[t], n);
            int seen = 0;
            for (int u = 0; u < size && !seen; u++) seen = or_same(&grp[u], &e, n);
            if (!seen) {
                if (size >= OR_MAXG) { free(grp); return -1; }
                grp[size++] = e;
            }
        }
    }
    int w = size < cap ? size : cap;
    for (int u = 0; u < w; u++) {
        memcpy(p_out + u * n, grp[u].p, (size_t)n);
        memcpy(q_out + u * n, grp[u].q, (size_t)n);
    }
    free(grp);
    return size;
}

/* Apply (p,q) to the known cells of h, then rename values so that row 0
 * reads 0..N-1 (the normalisation of Sec. 4.1).  Empty cells stay empty. */
static void or_transform(int n, const uint8_t *h, const signed char *p,
                         const signed char *q, uint8_t *out)
{
    uint8_t t[OR_MAXN * OR_MAXN];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) t[i * n + j] = h[p[i] * n + q[j]];
    uint8_t rename[OR_MAXN];
    for (int j = 0; j < n; j++) rename[t[j]] = (uint8_t)j;
    for (int c = 0; c < n * n; c++) out[c] = t[c] == OR_EMPTY ? OR_EMPTY : rename[t[c]];
}

/* Row-major lexicographic comparison of two designs with the same known
 * cells (empty cells compare equal to each other). */
static int or_lexcmp(int n, const uint8_t *a, const uint8_t *b)
{
    for (int c = 0; c < n * n; c++)
        if (a[c] != b[c]) return a[c] < b[c] ? -1 : 1;
    return 0;
}

static int or_cmp_bytes(const void *x, const void *y, void *nn)
{
    return memcmp(x, y, (size_t)(*(int *)nn));
}

/* Canonicity test of Algorithm 5: 0 if some image of h is lexicographically
 * smaller, otherwise the number of distinct images (the class power).
 * imgs: scratch of at least gsize * n*n bytes. */
static int or_canon(int n, const uint8_t *h, int gsize, const signed char *gp,
                    const signed char *gq, uint8_t *imgs)
{
    int nn = n * n;
    for (int g = 0; g < gsize; g++) {
        uint8_t *img = imgs + (size_t)g * nn;
        or_transform(n, h, gp + g * n, gq + g * n, img);
        if (or_lexcmp(n, img, h) < 0) return 0;
    }
    qsort_r(imgs, (size_t)gsize, (size_t)nn, or_cmp_bytes, &nn);
    int distinct = 1;
    for (int g = 1; g < gsize; g++)
        if (memcmp(imgs + (size_t)g * nn, imgs + (size_t)(g - 1) * nn, (size_t)nn) != 0)
            distinct++;
    return distinct;
}

/* Canonicity test of one design (exposed for property tests). */
int oracle_canon(int n, const uint8_t *h)
{
    if (!or_check_args(n, h)) return -1;
    signed char gp[OR_MAXG * OR_MAXN], gq[OR_MAXG * OR_MAXN];
    int gsize = oracle_hourglass_group(n, gp, gq, OR_MAXG);
    if (gsize <= 0) return -1;
    uint8_t *imgs = (uint8_t *)malloc((size_t)gsize * n * n);
    if (!imgs) return -1;
    int r = or_canon(n, h, gsize, gp, gq, imgs);
    free(imgs);
    return r;
}

/* Apply group element g (index into the closure order) to h, renormalised. */
int oracle_apply(int n, int g, const uint8_t *h, uint8_t *out)
{
    if (!or_check_args(n, h)) return -1;
    signed char gp[OR_MAXG * OR_MAXN], gq[OR_MAXG * OR_MAXN];
    int gsize = oracle_hourglass_group(n, gp, gq, OR_MAXG);
    if (g < 0 || g >= gsize) return -1;
    or_transform(n, h, gp + g * n, gq + g * n, out);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Hourglass designs (Sec. 4.2) and their classes (Corollary 1).            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n, vs;
    int gsize;
    const signed char *gp, *gq;
    int hc[4 * OR_MAXN];                 /* hourglass cells beyond row 0    */
    int nhc;
    /* work list: assignments of the first `split` hourglass cells */
    const uint8_t *seeds;
    int64_t nseeds;
    int split;
    int64_t next;
    pthread_mutex_t lock;
    /* results */
    uint8_t *reps;                       /* canonical designs               */
    uint32_t *mult;
    int64_t cap, nreps;
    uint64_t nhourglass;
    int overflow;
} or_hg;

typedef struct {
    or_hg *hg;
    or_state st;
    uint8_t *imgs;
    uint64_t nh;
} or_hg_worker;

static void or_hg_leaf(or_hg_worker *w)
{
    or_hg *hg = w->hg;
    int n = hg->n;
    uint8_t h[OR_MAXN * OR_MAXN];
    for (int c = 0; c < n * n; c++) {
        int v = w->st.ls[c / n][c % n];
        h[c] = (uint8_t)(v < 0 ? OR_EMPTY : v);
    }
    w->nh++;
    int mult = or_canon(n, h, hg->gsize, hg->gp, hg->gq, w->imgs);
    if (mult > 0) {
        pthread_mutex_lock(&hg->lock);
        if (hg->nreps < hg->cap) {
            memcpy(hg->reps + hg->nreps * n * n, h, (size_t)(n * n));
            hg->mult[hg->nreps] = (uint32_t)mult;
        } else if (hg->reps) {
            hg->overflow = 1;
        }
        hg->nreps++;
        pthread_mutex_unlock(&hg->lock);
    }
}

static void or_hg_rec(or_hg_worker *w, int t)
{
    or_hg *hg = w->hg;
    if (t == hg->nhc) { or_hg_leaf(w); return; }
    or_state *s = &w->st;
    int n = hg->n;
    int c = hg->hc[t], i = c / n, j = c % n;
    for (int v = 0; v < n; v++) {
        if (!or_allowed(s, i, j, v)) continue;
        or_mark(s, i, j, v, 1);
        or_hg_rec(w, t + 1);
        or_mark(s, i, j, v, 0);
    }
}

static void *or_hg_thread(void *arg)
{
    or_hg_worker *w = (or_hg_worker *)arg;
    or_hg *hg = w->hg;
    int n = hg->n;
    for (;;) {
        pthread_mutex_lock(&hg->lock);
        int64_t k = hg->next++;
        pthread_mutex_unlock(&hg->lock);
        if (k >= hg->nseeds) break;
        if (!or_load(&w->st, n, hg->vs, hg->seeds + k * n * n)) continue;
        or_hg_rec(w, hg->split);
    }
    return NULL;
}

/* Enumerate every hourglass design of order n (row 0 = 0..n-1; rows 0 and
 * n-1, main diagonal and antidiagonal assigned, all constraints among them
 * kept; VS designs only if vs), test each for canonicity, and return the
 * canonical ones with their class powers.  *n_hourglass gets the number of
 * designs.  Returns the number of classes (reps/mult written up to cap;
 * reps may be NULL to count only), or -1. */
int64_t oracle_hourglass_classes(int n, int vs, uint8_t *reps, uint32_t *mult,
                                 int64_t cap, uint64_t *n_hourglass, int threads)
{
    if (n < 2 || n > OR_MAXN) return -1;
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    or_hg *hg = (or_hg *)calloc(1, sizeof(or_hg));
    if (!hg) return -1;
    static signed char gp[OR_MAXG * OR_MAXN], gq[OR_MAXG * OR_MAXN];
    static pthread_mutex_t glock = PTHREAD_MUTEX_INITIALIZER;
    pthread_mutex_lock(&glock);
    int gsize = oracle_hourglass_group(n, gp, gq, OR_MAXG);
    hg->n = n; hg->vs = vs; hg->gsize = gsize; hg->gp = gp; hg->gq = gq;
    hg->reps = reps; hg->mult = mult; hg->cap = reps ? cap : 0;
    pthread_mutex_init(&hg->lock, NULL);
    /* hourglass cells in the oracle's order: main diagonal top-down,
     * antidiagonal top-down, then the last row left to right */
    unsigned char in[OR_MAXN * OR_MAXN];
    memset(in, 0, sizeof(in));
    for (int j = 0; j < n; j++) in[j] = 1;
    for (int i = 1; i < n; i++) {
        int c = i * n + i;
        if (!in[c]) { in[c] = 1; hg->hc[hg->nhc++] = c; }
    }
    for (int i = 1; i < n; i++) {
        int c = i * n + (n - 1 - i);
        if (!in[c]) { in[c] = 1; hg->hc[hg->nhc++] = c; }
    }
    for (int j = 0; j < n; j++) {
        int c = (n - 1) * n + j;
        if (!in[c]) { in[c] = 1; hg->hc[hg->nhc++] = c; }
    }
    /* seeds: all consistent assignments of the main-diagonal cells */
    uint8_t base[OR_MAXN * OR_MAXN];
    memset(base, OR_EMPTY, sizeof(base));
    for (int j = 0; j < n; j++) base[j] = (uint8_t)j;
    hg->split = n - 1 < hg->nhc ? n - 1 : hg->nhc;
    int64_t ns = oracle_assignments(n, vs, base, hg->hc, hg->split, NULL, 0);
    uint8_t *seeds = (uint8_t *)malloc((size_t)(ns > 0 ? ns : 1) * n * n);
    int64_t result = -1;
    if (seeds && ns >= 0) {
        oracle_assignments(n, vs, base, hg->hc, hg->split, seeds, ns);
        hg->seeds = seeds; hg->nseeds = ns;
        or_hg_worker *ws = (or_hg_worker *)calloc((size_t)threads, sizeof(or_hg_worker));
        pthread_t th[256];
        int ok = ws != NULL;
        for (int t = 0; ok && t < threads; t++) {
            ws[t].hg = hg;
            ws[t].imgs = (uint8_t *)malloc((size_t)gsize * n * n);
            if (!ws[t].imgs) ok = 0;
        }
        if (ok) {
            for (int t = 0; t < threads; t++) pthread_create(&th[t], NULL, or_hg_thread, &ws[t]);
            for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
            uint64_t total = 0;
            for (int t = 0; t < threads; t++) total += ws[t].nh;
            if (n_hourglass) *n_hourglass = total;
            result = hg->overflow ? -1 : hg->nreps;
        }
        if (ws) {
            for (int t = 0; t < threads; t++) free(ws[t].imgs);
            free(ws);
        }
    }
    free(seeds);
    pthread_mutex_destroy(&hg->lock);
    pthread_mutex_unlock(&glock);
    free(hg);
    return result;
}

/* ------------------------------------------------------------------------ */
/* Workunits at chosen positions of the depth-first enumeration.            */
/* ------------------------------------------------------------------------ */

typedef struct {
    or_state st;
    const int *cells;
    int k;
    const int64_t *pos;   /* increasing positions wanted */
    int64_t npos, next;   /* next index into pos          */
    int64_t seen;         /* assignments enumerated so far */
    uint8_t *out;
} or_select;

static void or_select_rec(or_select *e, int t)
{
    or_state *s = &e->st;
    int n = s->n;
    if (e->next >= e->npos) return;            /* all found: stop early */
    if (t == e->k) {
        if (e->seen == e->pos[e->next]) {
            uint8_t *dst = e->out + e->next * n * n;
            for (int c = 0; c < n * n; c++) {
                int v = s->ls[c / n][c % n];
                dst[c] = (uint8_t)(v < 0 ? OR_EMPTY : v);
            }
            e->next++;
        }
        e->seen++;
        return;
    }
    int c = e->cells[t], i = c / n, j = c % n;
    for (int v = 0; v < n; v++) {
        if (!or_allowed(s, i, j, v)) continue;
        or_mark(s, i, j, v, 1);
        or_select_rec(e, t + 1);
        or_mark(s, i, j, v, 0);
    }
}

/* The assignments that oracle_assignments(n, vs, base, cells, k) would list
 * at the given increasing positions, written in order; returns the total
 * number of assignments enumerated (all of them if the last position is
 * beyond the end), or -1 on invalid input. */
int64_t oracle_assignments_at(int n, int vs, const uint8_t *base, const int *cells, int k,
                              const int64_t *pos, int64_t npos, uint8_t *out)
{
    if (!or_check_args(n, base) || k < 0 || k > n * n || npos < 0) return -1;
    for (int64_t t = 1; t < npos; t++) if (pos[t] <= pos[t - 1]) return -1;
    or_select *e = (or_select *)malloc(sizeof(or_select));
    if (!e) return -1;
    int64_t r = 0;
    if (or_load(&e->st, n, vs, base)) {
        e->cells = cells; e->k = k; e->pos = pos; e->npos = npos; e->next = 0;
        e->seen = 0; e->out = out;
        or_select_rec(e, 0);
        r = e->seen;
    }
    free(e);
    return r;
}
