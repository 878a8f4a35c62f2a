/*
 * CPU oracle for delta-temporal motif counting.  TEST INFRASTRUCTURE ONLY:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this library.  It shares no code with the HIP path.
 *
 * What it computes (paper, section 2.1, "A delta-Temporal Motif" and
 * "Temporal Motif Mining"): for a motif M = ((u_1,v_1),...,(u_k,v_k)) and a
 * window delta, the number of edge-index sequences (i_1,...,i_k) with
 *   t_{i_1} < t_{i_2} < ... < t_{i_k}            (strict temporal order)
 *   t_{i_k} - t_{i_1} <= delta                   (window, inclusive)
 *   an injective phi: V_M -> V with phi(u_j) = src_{i_j}, phi(v_j) = dst_{i_j}.
 *
 * How (paper, Algorithm 1, "Temporal Motif Mining"): depth-first matching of
 * the motif edges in order.  The candidates for motif edge j are the
 * out-edges of phi(u_j) when u_j is bound, else the in-edges of phi(v_j) when
 * v_j is bound, else every edge (the paper takes all edges whenever u_j is
 * unbound; the choice of list cannot change the count).  A candidate must
 * satisfy t_prev < t <= t_first + delta and the structural test: a bound
 * endpoint must equal its image, an unbound one must be a vertex not yet in
 * the image of phi (injectivity).  Lists are time-sorted, so the temporal
 * filter is applied by starting at the first entry past t_prev (bisection)
 * and stopping at the first entry past t_first + delta; that skips exactly
 * the candidates the filter would reject.  The "incnt" bookkeeping of the
 * paper is not needed: each level records the vertices it bound and unbinds
 * them on return.
 *
 * Readings of the paper (each listed in the design notes):
 *  - equal timestamps never appear in one match (strict order), although the
 *    pseudocode only skips t < t_prev;
 *  - the window is measured from the first matched edge, inclusive;
 *  - injectivity is enforced for new vertices as well as bound ones;
 *  - graph self-loops never match (motif edges have u != v, phi injective).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_K 16
#define OR_MAX_V 32

/* Planted mistakes, compiled only into separate test libraries to show that
 * the pins catch them: 1 admits equal timestamps, 2 drops injectivity for new
 * vertices, 3 makes the window exclusive, 4 measures the window from the
 * previous edge, 5 logs window entries only when they pass the structural
 * filter, 6 logs a partial match before its structural filter.  0 (the
 * default) is the oracle. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

typedef struct {
    int64_t n;          /* edges */
    int32_t nv;         /* vertices */
    const int32_t *src, *dst;
    const int64_t *t;   /* sorted ascending (stable) */
    int64_t *out_off;   /* nv+1 */
    int64_t *out_e;     /* edge ids, time order */
    int64_t *in_off;
    int64_t *in_e;
} or_graph;

typedef struct {
    int k;
    int nmv;                 /* distinct motif vertices */
    int u[OR_MAX_K], v[OR_MAX_K];
} or_motif;

typedef struct {
    const or_graph *g;
    const or_motif *m;
    int64_t delta;
    int32_t m2g[OR_MAX_V];
    int64_t t_first;
    uint64_t count;
    uint64_t *level;  /* k entries or NULL */
    uint64_t *win;    /* k entries or NULL: window entries scanned per edge */
} or_ctx;

/* first position p in [lo,hi) of the edge-id list ids with t[ids[p]] > tv */
static int64_t first_after(const int64_t *t, const int64_t *ids, int64_t lo,
                           int64_t hi, int64_t tv) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int64_t e = ids ? ids[mid] : mid;
        if (t[e] > tv) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static int in_image(const or_ctx *c, int32_t x) {
    for (int i = 0; i < c->m->nmv; i++)
        if (c->m2g[i] == x) return 1;
    return 0;
}

static void match_edge(or_ctx *c, int j, int64_t t_prev) {
    const or_motif *m = c->m;
    const or_graph *g = c->g;
    if (j == m->k) { c->count++; return; }
    int um = m->u[j], vm = m->v[j];
    int32_t ug = c->m2g[um], vg = c->m2g[vm];
    const int64_t *ids; int64_t lo, hi;
    if (ug >= 0) { ids = g->out_e; lo = g->out_off[ug]; hi = g->out_off[ug + 1]; }
    else if (vg >= 0) { ids = g->in_e; lo = g->in_off[vg]; hi = g->in_off[vg + 1]; }
    else { ids = NULL; lo = 0; hi = g->n; }
    int64_t t0 = (ORACLE_MUTANT == 4) ? t_prev : c->t_first;
    int64_t tmax = (t0 > INT64_MAX - c->delta) ? INT64_MAX : t0 + c->delta;
    int64_t tstart = (ORACLE_MUTANT == 1) ? t_prev - 1 : t_prev;
    for (int64_t p = first_after(g->t, ids, lo, hi, tstart); p < hi; p++) {
        int64_t e = ids ? ids[p] : p;
        int64_t te = g->t[e];
        if (te > tmax || (ORACLE_MUTANT == 3 && te == tmax)) break;  /* window */
        if (c->win && ORACLE_MUTANT != 5) c->win[j]++;
        if (c->level && ORACLE_MUTANT == 6) c->level[j]++;
        int32_t s = g->src[e], d = g->dst[e];
        /* structural filter */
        if (ug >= 0 && s != ug) continue;
        if (vg >= 0 && d != vg) continue;
        if (ORACLE_MUTANT != 2 && ug < 0 && in_image(c, s)) continue;
        if (ORACLE_MUTANT != 2 && vg < 0 && in_image(c, d)) continue;
        if (ug < 0 && vg < 0 && s == d) continue;
        int new_u = (ug < 0), new_v = (vg < 0);
        if (new_u) c->m2g[um] = s;
        if (new_v) c->m2g[vm] = d;
        if (c->win && ORACLE_MUTANT == 5) c->win[j]++;
        if (c->level && ORACLE_MUTANT != 6) c->level[j]++;
        match_edge(c, j + 1, te);
        if (new_u) c->m2g[um] = -1;
        if (new_v) c->m2g[vm] = -1;
    }
}

/* one root: the root edge is the candidate for motif edge 1 */
static uint64_t count_root(const or_graph *g, const or_motif *m, int64_t delta,
                           int64_t r, uint64_t *level, uint64_t *win) {
    or_ctx c;
    c.g = g; c.m = m; c.delta = delta; c.count = 0; c.level = level; c.win = win;
    for (int i = 0; i < OR_MAX_V; i++) c.m2g[i] = -1;
    int32_t s = g->src[r], d = g->dst[r];
    if (s == d) return 0;                     /* injectivity */
    c.m2g[m->u[0]] = s;
    c.m2g[m->v[0]] = d;
    c.t_first = g->t[r];
    if (level) level[0]++;
    match_edge(&c, 1, g->t[r]);
    return c.count;
}

typedef struct { int64_t t, i; } or_key;
static int key_cmp(const void *a, const void *b) {
    const or_key *x = a, *y = b;
    if (x->t != y->t) return x->t < y->t ? -1 : 1;
    return x->i < y->i ? -1 : (x->i > y->i);
}

/* Stable sort by t, then per-vertex out/in lists in time order. */
static int build(or_graph *g, int64_t n, const int32_t *src, const int32_t *dst,
                 const int64_t *t, int32_t nv, int32_t **s2, int32_t **d2,
                 int64_t **t2) {
    or_key *k = malloc(sizeof(or_key) * (n ? n : 1));
    *s2 = malloc(sizeof(int32_t) * (n ? n : 1));
    *d2 = malloc(sizeof(int32_t) * (n ? n : 1));
    *t2 = malloc(sizeof(int64_t) * (n ? n : 1));
    g->out_off = calloc(nv + 1, sizeof(int64_t));
    g->in_off = calloc(nv + 1, sizeof(int64_t));
    g->out_e = malloc(sizeof(int64_t) * (n ? n : 1));
    g->in_e = malloc(sizeof(int64_t) * (n ? n : 1));
    if (!k || !*s2 || !*d2 || !*t2 || !g->out_off || !g->in_off || !g->out_e || !g->in_e)
        return -2;
    for (int64_t i = 0; i < n; i++) { k[i].t = t[i]; k[i].i = i; }
    qsort(k, n, sizeof(or_key), key_cmp);
    for (int64_t i = 0; i < n; i++) {
        (*s2)[i] = src[k[i].i]; (*d2)[i] = dst[k[i].i]; (*t2)[i] = t[k[i].i];
    }
    free(k);
    for (int64_t i = 0; i < n; i++) { g->out_off[(*s2)[i] + 1]++; g->in_off[(*d2)[i] + 1]++; }
    for (int32_t v = 0; v < nv; v++) {
        g->out_off[v + 1] += g->out_off[v];
        g->in_off[v + 1] += g->in_off[v];
    }
    int64_t *po = malloc(sizeof(int64_t) * (nv ? nv : 1));
    int64_t *pi = malloc(sizeof(int64_t) * (nv ? nv : 1));
    if (!po || !pi) return -2;
    memcpy(po, g->out_off, sizeof(int64_t) * nv);
    memcpy(pi, g->in_off, sizeof(int64_t) * nv);
    for (int64_t i = 0; i < n; i++) {
        g->out_e[po[(*s2)[i]]++] = i;
        g->in_e[pi[(*d2)[i]]++] = i;
    }
    free(po); free(pi);
    g->n = n; g->nv = nv; g->src = *s2; g->dst = *d2; g->t = *t2;
    return 0;
}

static void release(or_graph *g, int32_t *s2, int32_t *d2, int64_t *t2) {
    free(g->out_off); free(g->in_off); free(g->out_e); free(g->in_e);
    free(s2); free(d2); free(t2);
}

static int load_motif(or_motif *m, int k, const int32_t *uv) {
    int32_t labels[OR_MAX_V]; int nl = 0;
    if (k < 1 || k > OR_MAX_K) return -1;
    m->k = k;
    for (int j = 0; j < 2 * k; j++) {
        int32_t x = uv[j], id = -1;
        if (x < 0) return -1;
        for (int i = 0; i < nl; i++) if (labels[i] == x) id = i;
        if (id < 0) { if (nl == OR_MAX_V) return -1; labels[nl] = x; id = nl++; }
        if (j & 1) m->v[j / 2] = id; else m->u[j / 2] = id;
    }
    for (int j = 0; j < k; j++) if (m->u[j] == m->v[j]) return -1;
    m->nmv = nl;
    return 0;
}

typedef struct {
    or_graph g;
    int32_t *s2, *d2;
    int64_t *t2;
} oracle_graph;

/*
 * Load a graph: src,dst,t are n_edges edges in any order; they are copied and
 * stably sorted by t.  Returns NULL on a bad argument or when out of memory.
 */
oracle_graph *oracle_graph_new(int64_t n_edges, const int32_t *src, const int32_t *dst,
                               const int64_t *t, int32_t n_nodes) {
    if (n_edges < 0 || n_nodes < 0) return NULL;
    for (int64_t i = 0; i < n_edges; i++)
        if (src[i] < 0 || src[i] >= n_nodes || dst[i] < 0 || dst[i] >= n_nodes) return NULL;
    oracle_graph *h = calloc(1, sizeof(oracle_graph));
    if (!h) return NULL;
    if (build(&h->g, n_edges, src, dst, t, n_nodes, &h->s2, &h->d2, &h->t2)) {
        release(&h->g, h->s2, h->d2, h->t2);
        free(h);
        return NULL;
    }
    return h;
}

void oracle_graph_free(oracle_graph *h) {
    if (!h) return;
    release(&h->g, h->s2, h->d2, h->t2);
    free(h);
}

/*
 * Count one motif in a loaded graph.
 *   motif_uv  : 2k vertex labels, edge j = (motif_uv[2j], motif_uv[2j+1])
 *   roots     : positions in the stably time-sorted edge list to use as the
 *               first edge; NULL means every edge
 *   per_root  : NULL or n_roots counts (matches that start at each root)
 *   level     : NULL or n_roots*k: entry [r*k + j] = partial matches of the
 *               first j+1 motif edges that start at root r
 *   win       : NULL or k totals: window entries scanned for motif edge j
 *               (entry 0 stays 0: the first edge has no window)
 *   win_root  : NULL or n_roots*k: the same per root, entry [r*k + j]
 *   threads   : OpenMP threads (<=0: library default)
 *   total     : out, the count over the chosen roots
 * Returns 0, -1 on a bad argument.
 */
int oracle_graph_count(const oracle_graph *h, int32_t k, const int32_t *motif_uv,
                       int64_t delta, const int64_t *roots, int64_t n_roots,
                       uint64_t *per_root, uint64_t *level, uint64_t *win,
                       uint64_t *win_root, int32_t threads, uint64_t *total) {
    or_motif m;
    if (!h || delta < 0 || !total) return -1;
    if (load_motif(&m, k, motif_uv)) return -1;
    const or_graph *g = &h->g;
    if (!roots) n_roots = g->n;
    for (int64_t r = 0; roots && r < n_roots; r++)
        if (roots[r] < 0 || roots[r] >= g->n) return -1;
    if (level) memset(level, 0, sizeof(uint64_t) * (size_t)n_roots * (size_t)k);
    uint64_t sum = 0;
    uint64_t wsum[OR_MAX_K] = {0};
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#endif
    #pragma omp parallel
    {
        uint64_t wl[OR_MAX_K] = {0};
        uint64_t wr[OR_MAX_K];
        #pragma omp for schedule(dynamic, 64) reduction(+ : sum)
        for (int64_t r = 0; r < n_roots; r++) {
            int64_t e = roots ? roots[r] : r;
            for (int j = 0; j < k; j++) wr[j] = 0;
            uint64_t c = count_root(g, &m, delta, e, level ? level + (size_t)r * k : NULL,
                                    (win || win_root) ? wr : NULL);
            if (per_root) per_root[r] = c;
            sum += c;
            for (int j = 0; j < k; j++) {
                wl[j] += wr[j];
                if (win_root) win_root[(size_t)r * k + j] = wr[j];
            }
        }
        if (win) {
            #pragma omp critical
            for (int j = 0; j < k; j++) wsum[j] += wl[j];
        }
    }
    if (win) for (int j = 0; j < k; j++) win[j] = wsum[j];
    *total = sum;
    return 0;
}

/* One-shot form of oracle_graph_new + oracle_graph_count + oracle_graph_free. */
int oracle_count(int64_t n_edges, const int32_t *src, const int32_t *dst,
                 const int64_t *t, int32_t n_nodes, int32_t k,
                 const int32_t *motif_uv, int64_t delta, const int64_t *roots,
                 int64_t n_roots, uint64_t *per_root, uint64_t *level,
                 int32_t threads, uint64_t *total) {
    oracle_graph *h = oracle_graph_new(n_edges, src, dst, t, n_nodes);
    if (!h) return -1;
    int rc = oracle_graph_count(h, k, motif_uv, delta, roots, n_roots, per_root, level,
                                NULL, NULL, threads, total);
    oracle_graph_free(h);
    return rc;
}

/* Threads an OpenMP parallel region would use. */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
