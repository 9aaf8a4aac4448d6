/*
 * CPU oracle for butterfly counting in bipartite graphs.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header, table or helper with the HIP library.
 *
 * Everything here works from the raw edge list (l[i], r[i]), i < m, with
 * 0 <= l[i] < nl and 0 <= r[i] < nr, and builds its own adjacency lists.
 * Integer results are exact (uint64); floating point is IEEE binary64.
 *
 * Paper sections followed (Sanei-Mehri, Sariyuce, Tirthapura, "Butterfly
 * Counting in Bipartite Networks"):
 *   - butterfly, per-vertex and per-edge counts: Sec. 2 (Preliminaries);
 *   - exact count: Lemma 1, Eq. (1)-(4), Algorithm ExactBFC (Sec. 4) with the
 *     side-choice rule and the ordering that counts each same-side pair once;
 *   - per-vertex count: Algorithm vBFC (Sec. 4.2, local counting);
 *   - per-edge count: Algorithm eBFC (Sec. 4.2) with the fold read as
 *     sum(C[x]-1) (the printed fold sum(C(C[x],2)) overcounts; see the
 *     notes on readings of the paper);
 *   - vertex sampling VSamp and edge sampling ESamp (Sec. 5.1, 5.2);
 *   - edge sparsification ESpar (Sec. 6.1) and colourful sparsification
 *     ClrSpar (Sec. 6.2).
 *
 * Random decisions use Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 * keyed by the 64-bit seed, with counters fixed per decision; the layout of
 * counters is given next to each estimator below.
 *
 * Parity pins: brute force over 2x2 quadruples, complete bipartite closed
 * forms, counting from either side, sums of local counts (2B per side, 4B over
 * edges), Philox known-answer vectors, estimator special cases (p = 1, N = 1,
 * proposal proportional to the local count).  The tests hold them.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_RANGE (-2)
#define ORC_E_DUP (-3)
#define ORC_E_NOMEM (-4)
#define ORC_E_PROBS (-5)
#define ORC_E_OVERFLOW (-6)

/* ------------------------------------------------------------------ */
/* Adjacency lists of one side: row v holds the neighbours of v, in    */
/* ascending id order, with the input index of each edge alongside.   */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t n;
    uint64_t *off;  /* n+1 */
    uint32_t *nbr;  /* m */
    uint64_t *eid;  /* m */
} adj_t;

static void adj_free(adj_t *a) {
    free(a->off); free(a->nbr); free(a->eid);
    memset(a, 0, sizeof(*a));
}

/* Rows are sorted by neighbour id with qsort on (neighbour, edge index)
 * pairs; the oracle favours plainness over speed. */
typedef struct { uint32_t nbr; uint64_t eid; } pair_t;
static int pair_cmp(const void *a, const void *b) {
    const pair_t *x = (const pair_t *)a, *y = (const pair_t *)b;
    return (x->nbr > y->nbr) - (x->nbr < y->nbr);
}

/* Build the rows of side `src` (ids src[i] < n) pointing at dst[i]. */
static int adj_build(adj_t *a, uint32_t n, uint64_t m, const uint32_t *src,
                     const uint32_t *dst) {
    memset(a, 0, sizeof(*a));
    a->n = n;
    a->off = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    a->nbr = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    a->eid = (uint64_t *)malloc((m ? m : 1) * sizeof(uint64_t));
    if (!a->off || !a->nbr || !a->eid) { adj_free(a); return ORC_E_NOMEM; }
    for (uint64_t i = 0; i < m; i++) a->off[src[i] + 1]++;
    for (uint32_t v = 0; v < n; v++) a->off[v + 1] += a->off[v];
    uint64_t *fill = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    if (!fill) { adj_free(a); return ORC_E_NOMEM; }
    memcpy(fill, a->off, ((size_t)n + 1) * sizeof(uint64_t));
    for (uint64_t i = 0; i < m; i++) {
        uint64_t k = fill[src[i]]++;
        a->nbr[k] = dst[i];
        a->eid[k] = i;
    }
    free(fill);
    pair_t *tmp = NULL;
    size_t tmp_cap = 0;
    for (uint32_t v = 0; v < n; v++) {
        uint64_t b = a->off[v], e = a->off[v + 1], len = e - b;
        if (len < 2) continue;
        if (len > tmp_cap) {
            free(tmp);
            tmp_cap = len;
            tmp = (pair_t *)malloc(len * sizeof(pair_t));
            if (!tmp) { adj_free(a); return ORC_E_NOMEM; }
        }
        for (uint64_t k = 0; k < len; k++) { tmp[k].nbr = a->nbr[b + k]; tmp[k].eid = a->eid[b + k]; }
        qsort(tmp, len, sizeof(pair_t), pair_cmp);
        for (uint64_t k = 0; k < len; k++) { a->nbr[b + k] = tmp[k].nbr; a->eid[b + k] = tmp[k].eid; }
    }
    free(tmp);
    return ORC_OK;
}

/* The paper assumes a simple bipartite graph (Sec. 2): ids in range and no
 * repeated edge.  Rows are sorted, so a repeat shows as equal neighbours. */
static int check_input(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l,
                       const uint32_t *r) {
    if (m && (!l || !r)) return ORC_E_ARG;
    for (uint64_t i = 0; i < m; i++)
        if (l[i] >= nl || r[i] >= nr) return ORC_E_RANGE;
    return ORC_OK;
}

static int has_dup(const adj_t *a) {
    for (uint32_t v = 0; v < a->n; v++)
        for (uint64_t k = a->off[v] + 1; k < a->off[v + 1]; k++)
            if (a->nbr[k] == a->nbr[k - 1]) return 1;
    return 0;
}

typedef struct { adj_t L, R; } graph_t;

static void graph_free(graph_t *g) { adj_free(&g->L); adj_free(&g->R); }

static int graph_build(graph_t *g, uint32_t nl, uint32_t nr, uint64_t m,
                       const uint32_t *l, const uint32_t *r) {
    memset(g, 0, sizeof(*g));
    int rc = check_input(nl, nr, m, l, r);
    if (rc) return rc;
    rc = adj_build(&g->L, nl, m, l, r);
    if (rc) return rc;
    rc = adj_build(&g->R, nr, m, r, l);
    if (rc) { graph_free(g); return rc; }
    if (has_dup(&g->L)) { graph_free(g); return ORC_E_DUP; }
    return ORC_OK;
}

static inline uint64_t choose2(uint64_t c) { return c < 2 ? 0 : c * (c - 1) / 2; }

/* ------------------------------------------------------------------ */
/* Threads over start vertices.  The counts of different starts are     */
/* independent (each start has its own counter array), so the starts of */
/* a loop may be handed to several threads in chunks; integer sums do   */
/* not depend on the order in which chunks finish.  One thread (the     */
/* default) runs the loop in order on the calling thread.               */
/* ------------------------------------------------------------------ */
static int g_threads = 1;

void orc_set_threads(int n) { g_threads = n < 1 ? 1 : (n > 256 ? 256 : n); }
int orc_get_threads(void) { return g_threads; }

typedef void (*range_fn)(void *ctx, int worker, uint64_t lo, uint64_t hi);

typedef struct {
    range_fn fn;
    void *ctx;
    uint64_t next, end, chunk;
    int worker;
} pool_t;

static void *pool_main(void *arg) {
    pool_t *p = ((pool_t **)arg)[0];
    int worker = (int)(intptr_t)((void **)arg)[1];
    for (;;) {
        uint64_t lo = __atomic_fetch_add(&p->next, p->chunk, __ATOMIC_RELAXED);
        if (lo >= p->end) break;
        uint64_t hi = lo + p->chunk < p->end ? lo + p->chunk : p->end;
        p->fn(p->ctx, worker, lo, hi);
    }
    return NULL;
}

/* Run fn over [lo, hi) in chunks on `workers` threads (worker ids 0 ..
 * workers-1 index per-thread scratch).  Returns the number of workers used. */
static int parallel_range(range_fn fn, void *ctx, uint64_t lo, uint64_t hi, int workers,
                          uint64_t chunk) {
    if (workers <= 1 || hi - lo <= chunk) {
        if (lo < hi) fn(ctx, 0, lo, hi);
        return 1;
    }
    pool_t p = {fn, ctx, lo, hi, chunk, 0};
    pthread_t th[256];
    void *args[256][2];
    int started = 0;
    for (int t = 1; t < workers; t++) {
        args[t][0] = &p;
        args[t][1] = (void *)(intptr_t)t;
        if (pthread_create(&th[t], NULL, pool_main, args[t]) != 0) break;
        started = t;
    }
    args[0][0] = &p;
    args[0][1] = (void *)(intptr_t)0;
    pool_main(args[0]);
    for (int t = 1; t <= started; t++) pthread_join(th[t], NULL);
    return started + 1;
}

/* ------------------------------------------------------------------ */
/* Exact count: ExactBFC (Sec. 4).                                      */
/*                                                                      */
/* Side choice: start from L unless sum_{L} d^2 < sum_{R} d^2, in which */
/* case start from R (the red lines of ExactBFC).  For every start v,   */
/* every neighbour u of v and every neighbour w of u with w before v in */
/* the order (here: smaller id), C[w] is incremented; the count adds    */
/* C(C[w],2) over the touched w.  The order makes every unordered pair  */
/* {v, w} of same-side vertices count once, so no final halving.        */
/* `side`: 0 = the paper's rule, 1 = start from L, 2 = start from R.    */
/* `wedges` receives the number of (v,u,w) triples visited.            */
/* ------------------------------------------------------------------ */
/* Per-thread counter arrays of one loop over starts (zeroed, n + 1 each). */
typedef struct {
    int workers;
    uint32_t *C[256], *T[256];
    uint64_t sum[256], visits[256];
} scratch_t;

static void scratch_free(scratch_t *s) {
    for (int t = 0; t < s->workers; t++) { free(s->C[t]); free(s->T[t]); }
    memset(s, 0, sizeof(*s));
}

static int scratch_init(scratch_t *s, uint64_t n) {
    memset(s, 0, sizeof(*s));
    s->workers = g_threads;
    for (int t = 0; t < s->workers; t++) {
        s->C[t] = (uint32_t *)calloc((size_t)n + 1, sizeof(uint32_t));
        s->T[t] = (uint32_t *)malloc(((size_t)n + 1) * sizeof(uint32_t));
        if (!s->C[t] || !s->T[t]) { scratch_free(s); return ORC_E_NOMEM; }
    }
    return ORC_OK;
}

typedef struct {
    const adj_t *A, *B;
    scratch_t *sc;
} exact_ctx;

/* ExactBFC's loop body for the starts v in [lo, hi). */
static void exact_starts(void *vctx, int worker, uint64_t lo, uint64_t hi) {
    exact_ctx *x = (exact_ctx *)vctx;
    const adj_t *A = x->A, *B = x->B;
    uint32_t *C = x->sc->C[worker], *touched = x->sc->T[worker];
    uint64_t sum = 0, visits = 0;
    for (uint64_t v = lo; v < hi; v++) {
        uint32_t nt = 0;
        for (uint64_t k = A->off[v]; k < A->off[v + 1]; k++) {
            uint32_t u = A->nbr[k];
            for (uint64_t j = B->off[u]; j < B->off[u + 1]; j++) {
                uint32_t w = B->nbr[j];
                if (!(w < v)) continue;           /* w precedes v */
                visits++;
                if (C[w] == 0) touched[nt++] = w;
                C[w]++;
            }
        }
        for (uint32_t t = 0; t < nt; t++) {
            sum += choose2(C[touched[t]]);
            C[touched[t]] = 0;
        }
    }
    x->sc->sum[worker] += sum;
    x->sc->visits[worker] += visits;
}

static int exact_on(const graph_t *g, int side, uint64_t start_lo, uint64_t start_hi,
                    uint64_t *total, uint64_t *wedges, int *side_used) {
    uint64_t sl = 0, sr = 0;
    for (uint32_t v = 0; v < g->L.n; v++) { uint64_t d = g->L.off[v + 1] - g->L.off[v]; sl += d * d; }
    for (uint32_t v = 0; v < g->R.n; v++) { uint64_t d = g->R.off[v + 1] - g->R.off[v]; sr += d * d; }
    int start_r;
    if (side == 1) start_r = 0;
    else if (side == 2) start_r = 1;
    else start_r = (sl < sr);
    exact_ctx x;
    x.A = start_r ? &g->R : &g->L;   /* starts and end points */
    x.B = start_r ? &g->L : &g->R;   /* midpoints */
    scratch_t sc;
    if (scratch_init(&sc, x.A->n)) return ORC_E_NOMEM;
    x.sc = &sc;
    if (start_hi > x.A->n) start_hi = x.A->n;
    if (start_lo < start_hi) parallel_range(exact_starts, &x, start_lo, start_hi, sc.workers, 256);
    uint64_t sum = 0, visits = 0;
    for (int t = 0; t < sc.workers; t++) { sum += sc.sum[t]; visits += sc.visits[t]; }
    scratch_free(&sc);
    *total = sum;
    if (wedges) *wedges = visits;
    if (side_used) *side_used = start_r ? 2 : 1;
    return ORC_OK;
}

int orc_exact(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
              int side, uint64_t *total, uint64_t *wedges, int *side_used) {
    if (!total || side < 0 || side > 2) return ORC_E_ARG;
    graph_t g;
    int rc = graph_build(&g, nl, nr, m, l, r);
    if (rc) return rc;
    rc = exact_on(&g, side, 0, UINT64_MAX, total, wedges, side_used);
    graph_free(&g);
    return rc;
}

/* ExactBFC restricted to the starts v in [start_lo, start_hi) of the chosen
 * side: the partial sum of Eq. (3) over those starts (used to time the
 * oracle on a bounded slice of a large graph). */
int orc_exact_range(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
                    int side, uint64_t start_lo, uint64_t start_hi, uint64_t *total,
                    uint64_t *wedges, int *side_used) {
    if (!total || side < 0 || side > 2) return ORC_E_ARG;
    graph_t g;
    int rc = graph_build(&g, nl, nr, m, l, r);
    if (rc) return rc;
    rc = exact_on(&g, side, start_lo, start_hi, total, wedges, side_used);
    graph_free(&g);
    return rc;
}

/* Degree-square sums of both sides (the quantities of the side choice and
 * of the paper's dataset table). */
int orc_degree_stats(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l,
                     const uint32_t *r, uint64_t *sumsq_l, uint64_t *sumsq_r,
                     uint64_t *maxdeg_l, uint64_t *maxdeg_r) {
    int rc = check_input(nl, nr, m, l, r);
    if (rc) return rc;
    uint64_t *dl = (uint64_t *)calloc((size_t)nl + 1, 8), *dr = (uint64_t *)calloc((size_t)nr + 1, 8);
    if (!dl || !dr) { free(dl); free(dr); return ORC_E_NOMEM; }
    for (uint64_t i = 0; i < m; i++) { dl[l[i]]++; dr[r[i]]++; }
    uint64_t a = 0, b = 0, ma = 0, mb = 0;
    for (uint32_t v = 0; v < nl; v++) { a += dl[v] * dl[v]; if (dl[v] > ma) ma = dl[v]; }
    for (uint32_t v = 0; v < nr; v++) { b += dr[v] * dr[v]; if (dr[v] > mb) mb = dr[v]; }
    *sumsq_l = a; *sumsq_r = b; *maxdeg_l = ma; *maxdeg_r = mb;
    free(dl); free(dr);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Per-vertex counts, Eq. (2): B_v = sum over same-side w != v of       */
/* C(|N(v) & N(w)|, 2).  vBFC (Sec. 4.2): count paths v-u-w with w != v */
/* in a zeroed counter array, then add C(C[w],2).  Every vertex of both */
/* sides is done this way.                                              */
/* ------------------------------------------------------------------ */
static void vbfc_side(const adj_t *A, const adj_t *B, uint32_t v, uint32_t *C,
                      uint32_t *touched, uint64_t *out) {
    uint32_t nt = 0;
    for (uint64_t k = A->off[v]; k < A->off[v + 1]; k++) {
        uint32_t u = A->nbr[k];
        for (uint64_t j = B->off[u]; j < B->off[u + 1]; j++) {
            uint32_t w = B->nbr[j];
            if (w == v) continue;
            if (C[w] == 0) touched[nt++] = w;
            C[w]++;
        }
    }
    uint64_t s = 0;
    for (uint32_t t = 0; t < nt; t++) { s += choose2(C[touched[t]]); C[touched[t]] = 0; }
    *out = s;
}

typedef struct {
    const adj_t *A, *B;
    scratch_t *sc;
    uint64_t *out;
} vbfc_ctx;

static void vbfc_range(void *vctx, int worker, uint64_t lo, uint64_t hi) {
    vbfc_ctx *x = (vbfc_ctx *)vctx;
    for (uint64_t v = lo; v < hi; v++)
        vbfc_side(x->A, x->B, (uint32_t)v, x->sc->C[worker], x->sc->T[worker], &x->out[v]);
}

int orc_per_vertex(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
                   uint64_t *cnt_l, uint64_t *cnt_r) {
    if ((nl && !cnt_l) || (nr && !cnt_r)) return ORC_E_ARG;
    graph_t g;
    int rc = graph_build(&g, nl, nr, m, l, r);
    if (rc) return rc;
    uint32_t n = nl > nr ? nl : nr;
    scratch_t sc;
    if (scratch_init(&sc, n)) { graph_free(&g); return ORC_E_NOMEM; }
    vbfc_ctx xl = {&g.L, &g.R, &sc, cnt_l}, xr = {&g.R, &g.L, &sc, cnt_r};
    parallel_range(vbfc_range, &xl, 0, nl, sc.workers, 256);
    parallel_range(vbfc_range, &xr, 0, nr, sc.workers, 256);
    scratch_free(&sc); graph_free(&g);
    return ORC_OK;
}

/* Single-vertex vBFC; side 0 = L id, 1 = R id. */
int orc_vbfc(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
             int side, uint32_t v, uint64_t *out) {
    if (!out || side < 0 || side > 1) return ORC_E_ARG;
    if ((side == 0 && v >= nl) || (side == 1 && v >= nr)) return ORC_E_RANGE;
    graph_t g;
    int rc = graph_build(&g, nl, nr, m, l, r);
    if (rc) return rc;
    uint32_t n = nl > nr ? nl : nr;
    uint32_t *C = (uint32_t *)calloc((size_t)n + 1, 4), *T = (uint32_t *)malloc(((size_t)n + 1) * 4);
    if (!C || !T) { free(C); free(T); graph_free(&g); return ORC_E_NOMEM; }
    if (side == 0) vbfc_side(&g.L, &g.R, v, C, T, out);
    else vbfc_side(&g.R, &g.L, v, C, T, out);
    free(C); free(T); graph_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Per-edge counts.  A butterfly contains edge (a, x) (a in L, x in R)  */
/* iff it is {a, b} x {x, y} with b in N(x) \ {a} and y a common        */
/* neighbour of a and b other than x.  So                               */
/*     B_(a,x) = sum_{b in N(x), b != a} (|N(a) & N(b)| - 1).           */
/* eBFC (Sec. 4.2) computes C[b] = |N(a) & N(b)| for b in N(x) \ {a} by */
/* walking N(a) then N(w); its fold is read as sum(C[b] - 1).  Here the */
/* counters of start a are built once (walk a-u-b, b != a) and every    */
/* edge (a, x) of a is folded from them, which is eBFC for all edges of */
/* a at once.                                                           */
/* ------------------------------------------------------------------ */
typedef struct {
    const graph_t *g;
    scratch_t *sc;
    uint64_t *cnt_e;
} edge_ctx;

/* The edges of the L vertices a in [lo, hi). */
static void edge_range(void *vctx, int worker, uint64_t lo, uint64_t hi) {
    edge_ctx *x = (edge_ctx *)vctx;
    const graph_t *g = x->g;
    uint32_t *C = x->sc->C[worker], *T = x->sc->T[worker];
    for (uint64_t a = lo; a < hi; a++) {
        uint32_t nt = 0;
        for (uint64_t k = g->L.off[a]; k < g->L.off[a + 1]; k++) {
            uint32_t u = g->L.nbr[k];
            for (uint64_t j = g->R.off[u]; j < g->R.off[u + 1]; j++) {
                uint32_t b = g->R.nbr[j];
                if (b == a) continue;
                if (C[b] == 0) T[nt++] = b;
                C[b]++;
            }
        }
        for (uint64_t k = g->L.off[a]; k < g->L.off[a + 1]; k++) {
            uint32_t x2 = g->L.nbr[k];
            uint64_t s = 0;
            for (uint64_t j = g->R.off[x2]; j < g->R.off[x2 + 1]; j++) {
                uint32_t b = g->R.nbr[j];
                if (b == a) continue;
                s += (uint64_t)C[b] - 1;   /* C[b] >= 1: x2 is common */
            }
            x->cnt_e[g->L.eid[k]] = s;
        }
        for (uint32_t t = 0; t < nt; t++) C[T[t]] = 0;
    }
}

int orc_per_edge(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
                 uint64_t *cnt_e) {
    if (m && !cnt_e) return ORC_E_ARG;
    graph_t g;
    int rc = graph_build(&g, nl, nr, m, l, r);
    if (rc) return rc;
    scratch_t sc;
    if (scratch_init(&sc, nl)) { graph_free(&g); return ORC_E_NOMEM; }
    edge_ctx x = {&g, &sc, cnt_e};
    parallel_range(edge_range, &x, 0, nl, sc.workers, 256);
    scratch_free(&sc); graph_free(&g);
    return ORC_OK;
}

/* Literal eBFC for one edge (index e of the input list), with the corrected
 * fold: for w in N(a), for b in N(w): if b in N(x) \ {a}: C[b]++; return
 * sum(C[b] - 1) over the b that were counted. */
int orc_ebfc(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
             uint64_t e, uint64_t *out) {
    if (!out) return ORC_E_ARG;
    if (e >= m) return ORC_E_RANGE;
    graph_t g;
    int rc = graph_build(&g, nl, nr, m, l, r);
    if (rc) return rc;
    uint32_t a = l[e], x = r[e];
    uint8_t *inx = (uint8_t *)calloc((size_t)nl + 1, 1);
    uint32_t *C = (uint32_t *)calloc((size_t)nl + 1, 4);
    if (!inx || !C) { free(inx); free(C); graph_free(&g); return ORC_E_NOMEM; }
    for (uint64_t j = g.R.off[x]; j < g.R.off[x + 1]; j++) inx[g.R.nbr[j]] = 1;
    inx[a] = 0;
    for (uint64_t k = g.L.off[a]; k < g.L.off[a + 1]; k++) {
        uint32_t w = g.L.nbr[k];
        for (uint64_t j = g.R.off[w]; j < g.R.off[w + 1]; j++) {
            uint32_t b = g.R.nbr[j];
            if (inx[b]) C[b]++;
        }
    }
    uint64_t s = 0;
    for (uint64_t j = g.R.off[x]; j < g.R.off[x + 1]; j++) {
        uint32_t b = g.R.nbr[j];
        if (b != a && C[b] > 0) s += (uint64_t)C[b] - 1;
    }
    *out = s;
    free(inx); free(C); graph_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Philox-4x32-10 (Salmon et al., SC'11): a 4x32-bit counter, a 2x32-bit */
/* key, ten rounds.  A round multiplies words 0 and 2 by two 32-bit      */
/* constants into 64-bit products and mixes the halves with words 1, 3   */
/* and the key; the key is bumped by two Weyl constants between rounds. */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter tags (word 2 of the Philox counter) per kind of decision. */
#define TAG_ESPAR 0x45535052u   /* keep decision of an edge */
#define TAG_COLOR 0x434c5253u   /* colour of a vertex */
#define TAG_VDRAW 0x56445257u   /* vertex draw */
#define TAG_EDRAW 0x45445257u   /* edge draw */

static void seed_key(uint64_t seed, uint32_t key[2]) {
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
}

/* Uniform integer in [0, n) from the stream (a, b, tag, attempt): 64-bit
 * words out0 | out1 << 32, rejected while >= 2^64 - (2^64 mod n). */
static uint64_t uniform_below(uint64_t seed, uint32_t a, uint32_t b, uint32_t tag, uint64_t n) {
    uint32_t key[2], ctr[4], out[4];
    seed_key(seed, key);
    uint64_t rem = (0 - n) % n;       /* 2^64 mod n */
    for (uint32_t attempt = 0;; attempt++) {
        ctr[0] = a; ctr[1] = b; ctr[2] = tag; ctr[3] = attempt;
        orc_philox4x32_10(ctr, key, out);
        uint64_t x = (uint64_t)out[0] | ((uint64_t)out[1] << 32);
        if (rem == 0 || x < (uint64_t)(0 - rem)) return x % n;
    }
}

/* ------------------------------------------------------------------ */
/* ESpar (Sec. 6.1): keep each edge independently with probability p,  */
/* count the butterflies beta of the kept graph with ExactBFC, return   */
/* beta * p^-4.  Keep decision of edge (l, r): Philox counter           */
/* (l, r, TAG_ESPAR, 0), x = out0 | out1 << 32, kept iff x < T with     */
/* T = floor(p * 2^64) (p = 1 keeps every edge).                        */
/* The estimate is (double)beta / ((p*p)*(p*p)).                        */
/* ------------------------------------------------------------------ */
int orc_espar(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
              double p, uint64_t seed, uint64_t *beta, double *est, uint64_t *kept) {
    if (!beta || !est || !(p > 0.0) || !(p <= 1.0)) return ORC_E_ARG;
    int rc = check_input(nl, nr, m, l, r);
    if (rc) return rc;
    uint64_t T = (p >= 1.0) ? 0 : (uint64_t)ldexp(p, 64);
    uint32_t *kl = (uint32_t *)malloc((m ? m : 1) * 4), *kr = (uint32_t *)malloc((m ? m : 1) * 4);
    if (!kl || !kr) { free(kl); free(kr); return ORC_E_NOMEM; }
    uint32_t key[2], ctr[4], out[4];
    seed_key(seed, key);
    uint64_t mk = 0;
    for (uint64_t i = 0; i < m; i++) {
        int keep = 1;
        if (p < 1.0) {
            ctr[0] = l[i]; ctr[1] = r[i]; ctr[2] = TAG_ESPAR; ctr[3] = 0;
            orc_philox4x32_10(ctr, key, out);
            uint64_t x = (uint64_t)out[0] | ((uint64_t)out[1] << 32);
            keep = x < T;
        }
        if (keep) { kl[mk] = l[i]; kr[mk] = r[i]; mk++; }
    }
    rc = orc_exact(nl, nr, mk, kl, kr, 0, beta, NULL, NULL);
    free(kl); free(kr);
    if (rc) return rc;
    *est = (double)(*beta) / ((p * p) * (p * p));
    if (kept) *kept = mk;
    return ORC_OK;
}

/* Colour of vertex v of side s (0 = L, 1 = R) among N colours: Philox     */
/* counter (v, s, TAG_COLOR, attempt), x = out0, rejected while            */
/* x >= 2^32 - (2^32 mod N); colour = x mod N.                             */
uint32_t orc_color(uint64_t seed, uint32_t side, uint32_t v, uint32_t N) {
    uint32_t key[2], ctr[4], out[4];
    seed_key(seed, key);
    uint64_t lim = (0x100000000ull / N) * N;
    for (uint32_t attempt = 0;; attempt++) {
        ctr[0] = v; ctr[1] = side; ctr[2] = TAG_COLOR; ctr[3] = attempt;
        orc_philox4x32_10(ctr, key, out);
        if ((uint64_t)out[0] < lim) return out[0] % N;
    }
}

/* ------------------------------------------------------------------ */
/* ClrSpar (Sec. 6.2): colour every vertex uniformly with one of N      */
/* colours, keep the monochromatic edges, count their butterflies beta  */
/* with ExactBFC and return beta * N^3 (p = 1/N, estimate beta p^-3).   */
/* The estimate is (double)beta * ((double)N * (double)N * (double)N).  */
/* ------------------------------------------------------------------ */
int orc_clrspar(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
                uint32_t N, uint64_t seed, uint64_t *beta, double *est, uint64_t *kept) {
    if (!beta || !est || N == 0) return ORC_E_ARG;
    int rc = check_input(nl, nr, m, l, r);
    if (rc) return rc;
    uint32_t *kl = (uint32_t *)malloc((m ? m : 1) * 4), *kr = (uint32_t *)malloc((m ? m : 1) * 4);
    if (!kl || !kr) { free(kl); free(kr); return ORC_E_NOMEM; }
    uint64_t mk = 0;
    for (uint64_t i = 0; i < m; i++) {
        if (N == 1 || orc_color(seed, 0, l[i], N) == orc_color(seed, 1, r[i], N)) {
            kl[mk] = l[i]; kr[mk] = r[i]; mk++;
        }
    }
    rc = orc_exact(nl, nr, mk, kl, kr, 0, beta, NULL, NULL);
    free(kl); free(kr);
    if (rc) return rc;
    *est = (double)(*beta) * ((double)N * (double)N * (double)N);
    if (kept) *kept = mk;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Sampling with replacement, shared by VSamp and ESamp.                */
/*                                                                      */
/* Uniform (probs == NULL): draw i picks uniform_below(n) from the       */
/* stream (i lo, i hi, tag, attempt).                                    */
/* Weighted: integer weights q_j = probs_j > 0 ?                         */
/*   max(1, floor(probs_j / max(probs) * (2^32 - 1))) : 0, total Q; draw */
/* i takes t = uniform_below(Q) from the same stream and picks the first */
/* j whose inclusive prefix sum of q exceeds t.                          */
/* ------------------------------------------------------------------ */
static int quantise(const double *probs, uint64_t n, uint32_t *q, uint64_t *total) {
    double mx = 0.0;
    for (uint64_t j = 0; j < n; j++) {
        double p = probs[j];
        if (!(p >= 0.0) || isinf(p)) return ORC_E_PROBS;   /* NaN, negative, inf */
        if (p > mx) mx = p;
    }
    if (!(mx > 0.0)) return ORC_E_PROBS;
    uint64_t t = 0;
    for (uint64_t j = 0; j < n; j++) {
        double p = probs[j];
        if (p > 0.0) {
            double s = floor(p / mx * 4294967295.0);
            uint32_t w = (uint32_t)s;
            q[j] = w < 1 ? 1 : w;
        } else {
            q[j] = 0;
        }
        t += q[j];
    }
    *total = t;
    return ORC_OK;
}

static uint64_t pick_weighted(const uint64_t *prefix_incl, uint64_t n, uint64_t t) {
    uint64_t lo = 0, hi = n;          /* first j with prefix_incl[j] > t */
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (prefix_incl[mid] > t) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* Estimate combine shared by both samplers.  Uniform: (double)sum(counts)
 * * (double)n / (4.0 * (double)k), the sum exact in uint64.  Weighted:
 * term_i = (double)count_i * ((double)Q / (4.0 * (double)q_i)); the terms are
 * summed left to right inside consecutive blocks of 1024 draws, the block
 * sums left to right, and the total divided by (double)k. */
#define COMBINE_BLOCK 1024
static int combine(uint64_t n, uint64_t k, const uint64_t *counts, const uint32_t *qdraw,
                   uint64_t Q, int weighted, double *est) {
    if (!weighted) {
        uint64_t s = 0;
        for (uint64_t i = 0; i < k; i++) {
            if (s + counts[i] < s) return ORC_E_OVERFLOW;
            s += counts[i];
        }
        *est = ((double)s * (double)n) / (4.0 * (double)k);
        return ORC_OK;
    }
    double total = 0.0;
    for (uint64_t b = 0; b < k; b += COMBINE_BLOCK) {
        double part = 0.0;
        uint64_t e = b + COMBINE_BLOCK < k ? b + COMBINE_BLOCK : k;
        for (uint64_t i = b; i < e; i++)
            part += (double)counts[i] * ((double)Q / (4.0 * (double)qdraw[i]));
        total += part;
    }
    *est = total / (double)k;
    return ORC_OK;
}

/* VSamp (Sec. 5.1): ids are global (L ids, then nl + R id); count_i is the
 * vBFC count of the drawn vertex; the estimate is combine() above (for the
 * uniform case: mean of B_v * n / 4, Alg. VSamp averaged over k draws). */
int orc_vsamp(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
              const double *probs, uint64_t k, uint64_t seed, uint32_t *ids, uint64_t *counts,
              double *est) {
    if (k == 0 || !ids || !counts || !est) return ORC_E_ARG;
    uint64_t n = (uint64_t)nl + nr;
    if (n == 0) return ORC_E_ARG;
    graph_t g;
    int rc = graph_build(&g, nl, nr, m, l, r);
    if (rc) return rc;
    uint32_t *q = NULL, *qd = NULL;
    uint64_t *pre = NULL, Q = 0;
    if (probs) {
        q = (uint32_t *)malloc(n * 4); pre = (uint64_t *)malloc(n * 8); qd = (uint32_t *)malloc(k * 4);
        if (!q || !pre || !qd) { rc = ORC_E_NOMEM; goto done; }
        rc = quantise(probs, n, q, &Q);
        if (rc) goto done;
        uint64_t run = 0;
        for (uint64_t j = 0; j < n; j++) { run += q[j]; pre[j] = run; }
    }
    for (uint64_t i = 0; i < k; i++) {
        uint64_t v;
        if (probs) {
            uint64_t t = uniform_below(seed, (uint32_t)i, (uint32_t)(i >> 32), TAG_VDRAW, Q);
            v = pick_weighted(pre, n, t);
            qd[i] = q[v];
        } else {
            v = uniform_below(seed, (uint32_t)i, (uint32_t)(i >> 32), TAG_VDRAW, n);
        }
        ids[i] = (uint32_t)v;
    }
    {
        uint32_t nmax = nl > nr ? nl : nr;
        uint32_t *C = (uint32_t *)calloc((size_t)nmax + 1, 4), *T = (uint32_t *)malloc(((size_t)nmax + 1) * 4);
        if (!C || !T) { free(C); free(T); rc = ORC_E_NOMEM; goto done; }
        for (uint64_t i = 0; i < k; i++) {
            uint32_t v = ids[i];
            if (v < nl) vbfc_side(&g.L, &g.R, v, C, T, &counts[i]);
            else vbfc_side(&g.R, &g.L, v - nl, C, T, &counts[i]);
        }
        free(C); free(T);
    }
    rc = combine(n, k, counts, qd, Q, probs != NULL, est);
done:
    free(q); free(pre); free(qd); graph_free(&g);
    return rc;
}

/* ESamp (Sec. 5.2): draws edge indices of the input list (uniform or
 * weighted as above), count_i is the eBFC count of the drawn edge, the
 * estimate is combine() with n = m (uniform: mean of B_e * m / 4). */
int orc_esamp(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
              const double *probs, uint64_t k, uint64_t seed, uint64_t *eids, uint64_t *counts,
              double *est) {
    if (k == 0 || !eids || !counts || !est || m == 0) return ORC_E_ARG;
    uint64_t *all = (uint64_t *)malloc(m * 8);
    uint32_t *q = NULL, *qd = NULL;
    uint64_t *pre = NULL, Q = 0;
    int rc = ORC_OK;
    if (!all) return ORC_E_NOMEM;
    rc = orc_per_edge(nl, nr, m, l, r, all);
    if (rc) goto done;
    if (probs) {
        q = (uint32_t *)malloc(m * 4); pre = (uint64_t *)malloc(m * 8); qd = (uint32_t *)malloc(k * 4);
        if (!q || !pre || !qd) { rc = ORC_E_NOMEM; goto done; }
        rc = quantise(probs, m, q, &Q);
        if (rc) goto done;
        uint64_t run = 0;
        for (uint64_t j = 0; j < m; j++) { run += q[j]; pre[j] = run; }
    }
    for (uint64_t i = 0; i < k; i++) {
        uint64_t e;
        if (probs) {
            uint64_t t = uniform_below(seed, (uint32_t)i, (uint32_t)(i >> 32), TAG_EDRAW, Q);
            e = pick_weighted(pre, m, t);
            qd[i] = q[e];
        } else {
            e = uniform_below(seed, (uint32_t)i, (uint32_t)(i >> 32), TAG_EDRAW, m);
        }
        eids[i] = e;
        counts[i] = all[e];
    }
    rc = combine(m, k, counts, qd, Q, probs != NULL, est);
done:
    free(all); free(q); free(pre); free(qd);
    return rc;
}

/* ------------------------------------------------------------------ */
/* ESamp with Fast-eBFC (Sec. 5.5): the drawn edge's count is not       */
/* counted but estimated.  One trial for edge e = (a, x), a in L, x in R: */
/* pick b uniformly from the neighbours of x and y uniformly from the    */
/* neighbours of a; the trial hits iff b != a, y != x and (b, y) is an   */
/* edge, i.e. {a, b} x {x, y} is a butterfly.  hit * d_a * d_x has mean  */
/* B_e (the lemma of Sec. 5.5), since exactly B_e of the d_a * d_x pairs */
/* (b, y) hit.  Picking from the whole neighbourhood (b = a or y = x is  */
/* simply a miss) keeps that scale exact.                                */
/*                                                                      */
/* Draw i picks the edge exactly as ESamp above (same stream, same ids). */
/* Trial j of draw i (i < 2^32) uses the Philox counter                  */
/* (i, j, TAG_FAST, attempt): x1 = out0 | out1 << 32, x2 = out2 | out3   */
/* << 32; the attempt is kept iff x1 < 2^64 - 2^64 mod d_x and x2 <      */
/* 2^64 - 2^64 mod d_a, then b is neighbour x1 mod d_x of x and y is     */
/* neighbour x2 mod d_a of a.  Neighbours are listed in ascending order   */
/* of (degree, id) on their side.                                        */
/*                                                                      */
/* hits_i = number of hits among alpha trials.  Estimate: term_i =       */
/* ((double)hits_i * (double)(d_a * d_x)) * s_i with s_i = (double)m / 4 */
/* (uniform) or (double)Q / (4.0 * (double)q_i) (weighted), summed left  */
/* to right in blocks of 1024 draws and the block sums left to right,    */
/* divided by ((double)k * (double)alpha).                               */
/* ------------------------------------------------------------------ */
#define TAG_FAST 0x46454243u    /* neighbour pair of a Fast-eBFC trial */

static const uint64_t *fast_deg_key;    /* degrees of the side being sorted */
static int deg_id_cmp(const void *pa, const void *pb) {
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    uint64_t da = fast_deg_key[a], db = fast_deg_key[b];
    if (da != db) return da < db ? -1 : 1;
    return (a > b) - (a < b);
}

/* Neighbours of v (row v of A, ids of the other side) in (degree, id)
 * order of the other side, whose degrees are deg. */
static void list_by_degree(const adj_t *A, uint32_t v, const uint64_t *deg, uint32_t *out) {
    uint64_t b = A->off[v], d = A->off[v + 1] - b;
    for (uint64_t k = 0; k < d; k++) out[k] = A->nbr[b + k];
    fast_deg_key = deg;
    qsort(out, d, sizeof(uint32_t), deg_id_cmp);
}

static int has_edge(const adj_t *L, uint32_t b, uint32_t y) {
    uint64_t lo = L->off[b], hi = L->off[b + 1];    /* row b sorted by id */
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (L->nbr[mid] == y) return 1;
        if (L->nbr[mid] < y) lo = mid + 1; else hi = mid;
    }
    return 0;
}

/* The trial's test on picked neighbours b (of x) and y (of a). */
static int fast_hit(const graph_t *g, uint32_t a, uint32_t x, uint32_t b, uint32_t y) {
    return b != a && y != x && has_edge(&g->L, b, y);
}

typedef struct { uint64_t *deg_l, *deg_r; uint32_t *nb_x, *nb_a; } fast_tmp_t;

static void fast_tmp_free(fast_tmp_t *t) {
    free(t->deg_l); free(t->deg_r); free(t->nb_x); free(t->nb_a);
}

static int fast_tmp_init(fast_tmp_t *t, const graph_t *g) {
    uint32_t maxd = 1;
    t->deg_l = (uint64_t *)malloc(((size_t)g->L.n + 1) * 8);
    t->deg_r = (uint64_t *)malloc(((size_t)g->R.n + 1) * 8);
    for (uint32_t v = 0; t->deg_l && v < g->L.n; v++) {
        t->deg_l[v] = g->L.off[v + 1] - g->L.off[v];
        if (t->deg_l[v] > maxd) maxd = (uint32_t)t->deg_l[v];
    }
    for (uint32_t v = 0; t->deg_r && v < g->R.n; v++) {
        t->deg_r[v] = g->R.off[v + 1] - g->R.off[v];
        if (t->deg_r[v] > maxd) maxd = (uint32_t)t->deg_r[v];
    }
    t->nb_x = (uint32_t *)malloc((size_t)maxd * 4);
    t->nb_a = (uint32_t *)malloc((size_t)maxd * 4);
    if (!t->deg_l || !t->deg_r || !t->nb_x || !t->nb_a) { fast_tmp_free(t); return ORC_E_NOMEM; }
    return ORC_OK;
}

/* alpha trials on edge (a, x) for draw i. */
static uint32_t fast_trials(const graph_t *g, fast_tmp_t *t, uint32_t a, uint32_t x, uint32_t i,
                            uint32_t alpha, uint64_t seed) {
    uint64_t da = g->L.off[a + 1] - g->L.off[a];
    uint64_t dx = g->R.off[x + 1] - g->R.off[x];
    list_by_degree(&g->R, x, t->deg_l, t->nb_x);    /* neighbours of x: L ids */
    list_by_degree(&g->L, a, t->deg_r, t->nb_a);    /* neighbours of a: R ids */
    uint64_t rem_x = (0 - dx) % dx, rem_a = (0 - da) % da;
    uint32_t key[2], ctr[4], out[4], hits = 0;
    seed_key(seed, key);
    for (uint32_t j = 0; j < alpha; j++) {
        uint64_t x1, x2;
        for (uint32_t attempt = 0;; attempt++) {
            ctr[0] = i; ctr[1] = j; ctr[2] = TAG_FAST; ctr[3] = attempt;
            orc_philox4x32_10(ctr, key, out);
            x1 = (uint64_t)out[0] | ((uint64_t)out[1] << 32);
            x2 = (uint64_t)out[2] | ((uint64_t)out[3] << 32);
            if ((rem_x == 0 || x1 < (uint64_t)(0 - rem_x)) &&
                (rem_a == 0 || x2 < (uint64_t)(0 - rem_a)))
                break;
        }
        hits += (uint32_t)fast_hit(g, a, x, t->nb_x[x1 % dx], t->nb_a[x2 % da]);
    }
    return hits;
}

int orc_esamp_fast(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
                   const double *probs, uint64_t k, uint32_t alpha, uint64_t seed,
                   uint64_t *eids, uint32_t *hits, double *est) {
    if (k == 0 || k > 0xFFFFFFFFull || alpha == 0 || !eids || !hits || !est || m == 0)
        return ORC_E_ARG;
    graph_t g;
    fast_tmp_t t;
    uint32_t *q = NULL, *qd = NULL;
    uint64_t *pre = NULL, Q = 0;
    double total = 0.0, part = 0.0;
    int rc = graph_build(&g, nl, nr, m, l, r);
    if (rc) return rc;
    rc = fast_tmp_init(&t, &g);
    if (rc) { graph_free(&g); return rc; }
    if (probs) {
        q = (uint32_t *)malloc(m * 4); pre = (uint64_t *)malloc(m * 8); qd = (uint32_t *)malloc(k * 4);
        if (!q || !pre || !qd) { rc = ORC_E_NOMEM; goto done; }
        rc = quantise(probs, m, q, &Q);
        if (rc) goto done;
        uint64_t run = 0;
        for (uint64_t j = 0; j < m; j++) { run += q[j]; pre[j] = run; }
    }
    for (uint64_t i = 0; i < k; i++) {
        uint64_t e;
        if (probs) {
            uint64_t u = uniform_below(seed, (uint32_t)i, (uint32_t)(i >> 32), TAG_EDRAW, Q);
            e = pick_weighted(pre, m, u);
            qd[i] = q[e];
        } else {
            e = uniform_below(seed, (uint32_t)i, (uint32_t)(i >> 32), TAG_EDRAW, m);
        }
        eids[i] = e;
        uint32_t a = l[e], x = r[e];
        hits[i] = fast_trials(&g, &t, a, x, (uint32_t)i, alpha, seed);
        uint64_t dd = (g.L.off[a + 1] - g.L.off[a]) * (g.R.off[x + 1] - g.R.off[x]);
        double s = probs ? (double)Q / (4.0 * (double)qd[i]) : (double)m / 4.0;
        part += ((double)hits[i] * (double)dd) * s;
        if ((i + 1) % COMBINE_BLOCK == 0 || i + 1 == k) { total += part; part = 0.0; }
    }
    *est = total / ((double)k * (double)alpha);
done:
    free(q); free(pre); free(qd); fast_tmp_free(&t); graph_free(&g);
    return rc;
}

/* Number of hitting (b, y) pairs over every pick of the two neighbours of
 * input edge e: the lemma of Sec. 5.5 says it is B_e. */
int orc_fast_ebfc_pairs(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l,
                        const uint32_t *r, uint64_t e, uint64_t *pairs) {
    if (!pairs || e >= m) return ORC_E_ARG;
    graph_t g;
    fast_tmp_t t;
    int rc = graph_build(&g, nl, nr, m, l, r);
    if (rc) return rc;
    rc = fast_tmp_init(&t, &g);
    if (rc) { graph_free(&g); return rc; }
    uint32_t a = l[e], x = r[e];
    uint64_t da = g.L.off[a + 1] - g.L.off[a], dx = g.R.off[x + 1] - g.R.off[x], s = 0;
    list_by_degree(&g.R, x, t.deg_l, t.nb_x);
    list_by_degree(&g.L, a, t.deg_r, t.nb_a);
    for (uint64_t jb = 0; jb < dx; jb++)
        for (uint64_t jy = 0; jy < da; jy++) s += (uint64_t)fast_hit(&g, a, x, t.nb_x[jb], t.nb_a[jy]);
    *pairs = s;
    fast_tmp_free(&t);
    graph_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* WSamp (Sec. 5.3): draw a wedge uniformly (its midpoint u with        */
/* probability C(d_u,2) / W, then two distinct neighbours), count the   */
/* butterflies through it, |G_v n G_w| - 1, and return beta * W / 4.    */
/*                                                                      */
/* Wedges are numbered 0 .. W-1: vertices in global order (L ids, then   */
/* n_left + R id) take consecutive ranges of C(d_u,2) numbers; inside    */
/* u's range, number p is the pair (j1, j2), j1 < j2, of positions in u's */
/* neighbour list (ascending (degree, id) order of the other side) with  */
/* p = C(j2,2) + j1 (pairs (0,1), (0,2), (1,2), (0,3), ...).  A uniform  */
/* number is a uniform wedge, which is the lemma of Sec. 5.3.            */
/* Draw i takes t = uniform_below(W) from the stream (i lo, i hi,        */
/* TAG_WDRAW, attempt).  Estimate: ((double)sum beta * (double)W) /      */
/* (4.0 * (double)k), the sum exact in uint64.                           */
/* ------------------------------------------------------------------ */
#define TAG_WDRAW 0x57445257u   /* wedge draw */

typedef struct {
    graph_t g;
    fast_tmp_t t;
    uint64_t n, W;
    uint64_t *pre;      /* inclusive prefix sums of C(d,2) in global order */
} wedges_t;

static void wedges_free(wedges_t *w) {
    free(w->pre); fast_tmp_free(&w->t); graph_free(&w->g);
}

static int wedges_init(wedges_t *w, uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l,
                       const uint32_t *r) {
    memset(w, 0, sizeof(*w));
    int rc = graph_build(&w->g, nl, nr, m, l, r);
    if (rc) return rc;
    rc = fast_tmp_init(&w->t, &w->g);
    if (rc) { graph_free(&w->g); return rc; }
    w->n = (uint64_t)nl + nr;
    w->pre = (uint64_t *)malloc((w->n ? w->n : 1) * 8);
    if (!w->pre) { wedges_free(w); return ORC_E_NOMEM; }
    uint64_t run = 0;
    for (uint64_t v = 0; v < w->n; v++) {
        uint64_t d = v < nl ? w->t.deg_l[v] : w->t.deg_r[v - nl];
        run += choose2(d);
        w->pre[v] = run;
    }
    w->W = run;
    return ORC_OK;
}

static uint64_t common_neighbours(const adj_t *A, uint32_t v, uint32_t w) {
    uint64_t i = A->off[v], ie = A->off[v + 1], j = A->off[w], je = A->off[w + 1], c = 0;
    while (i < ie && j < je) {       /* merge of two id-sorted rows */
        if (A->nbr[i] == A->nbr[j]) { c++; i++; j++; }
        else if (A->nbr[i] < A->nbr[j]) i++;
        else j++;
    }
    return c;
}

/* Wedge number t: midpoint (global id), endpoints (global ids, j1 then
 * j2) and the butterflies through it. */
static void wedge_of(wedges_t *w, uint64_t t, uint32_t *mid, uint32_t *e1, uint32_t *e2,
                     uint64_t *beta) {
    uint32_t nl = w->g.L.n;
    uint64_t u = pick_weighted(w->pre, w->n, t);
    uint64_t p = t - (u ? w->pre[u - 1] : 0);
    uint64_t j2 = 1;
    while (choose2(j2 + 1) <= p) j2++;
    uint64_t j1 = p - choose2(j2);
    *mid = (uint32_t)u;
    if (u < nl) {                                   /* midpoint in L, ends in R */
        list_by_degree(&w->g.L, (uint32_t)u, w->t.deg_r, w->t.nb_a);
        uint32_t v = w->t.nb_a[j1], x = w->t.nb_a[j2];
        *e1 = nl + v; *e2 = nl + x;
        *beta = common_neighbours(&w->g.R, v, x) - 1;
    } else {                                        /* midpoint in R, ends in L */
        list_by_degree(&w->g.R, (uint32_t)(u - nl), w->t.deg_l, w->t.nb_a);
        uint32_t v = w->t.nb_a[j1], x = w->t.nb_a[j2];
        *e1 = v; *e2 = x;
        *beta = common_neighbours(&w->g.L, v, x) - 1;
    }
}

int orc_wsamp(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
              uint64_t k, uint64_t seed, uint32_t *mids, uint32_t *ends, uint64_t *counts,
              double *est) {
    if (k == 0 || !mids || !ends || !counts || !est) return ORC_E_ARG;
    wedges_t w;
    int rc = wedges_init(&w, nl, nr, m, l, r);
    if (rc) return rc;
    if (w.W == 0) { wedges_free(&w); return ORC_E_ARG; }
    uint64_t s = 0;
    for (uint64_t i = 0; i < k; i++) {
        uint64_t t = uniform_below(seed, (uint32_t)i, (uint32_t)(i >> 32), TAG_WDRAW, w.W);
        wedge_of(&w, t, &mids[i], &ends[2 * i], &ends[2 * i + 1], &counts[i]);
        s += counts[i];
    }
    *est = ((double)s * (double)w.W) / (4.0 * (double)k);
    wedges_free(&w);
    return ORC_OK;
}

/* Decode wedge numbers t[0..cnt) (for tests that enumerate every wedge);
 * *W receives the number of wedges. */
int orc_wedges(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *l, const uint32_t *r,
               const uint64_t *t, uint64_t cnt, uint32_t *mids, uint32_t *ends, uint64_t *counts,
               uint64_t *W) {
    if (!W || (cnt && (!t || !mids || !ends || !counts))) return ORC_E_ARG;
    wedges_t w;
    int rc = wedges_init(&w, nl, nr, m, l, r);
    if (rc) return rc;
    *W = w.W;
    for (uint64_t i = 0; i < cnt; i++) {
        if (t[i] >= w.W) { wedges_free(&w); return ORC_E_ARG; }
        wedge_of(&w, t[i], &mids[i], &ends[2 * i], &ends[2 * i + 1], &counts[i]);
    }
    wedges_free(&w);
    return ORC_OK;
}

/* Raw draws only (for statistics tests that do not need the counts). */
int orc_uniform_below(uint64_t seed, uint32_t a, uint32_t b, uint32_t tag, uint64_t n,
                      uint64_t *out) {
    if (!out || n == 0) return ORC_E_ARG;
    *out = uniform_below(seed, a, b, tag, n);
    return ORC_OK;
}
