/*
 * mayura.h -- C ABI of the MI355X (gfx950) temporal-motif co-mining library.
 *
 * The library counts delta-temporal motifs (paper, section 2.1): for every
 * motif M = ((u_1,v_1),...,(u_k,v_k)) of a motif group and a window delta it
 * returns the number of edge sequences with strictly increasing timestamps,
 * last minus first <= delta, whose endpoints follow M under an injective
 * vertex map.  Motifs that share a prefix share one search path through the
 * Motif-Group Tree (paper, section 4.3 and Algorithm 2); the search is the
 * co-mining recursion of Algorithm 3 run by HIP kernels on the GPU.
 *
 * Conventions for every entry point:
 *  - The return value is an mg_status.  On any error the outputs are left
 *    untouched and mg_last_error() describes the failure.  No C++ exception
 *    crosses this boundary.
 *  - Host arrays passed in are copied; the caller keeps ownership.
 *  - Handles are owned by the caller and released by the matching destroy
 *    function (NULL is accepted there).
 *  - "stream" arguments are hipStream_t values passed as void* (NULL = the
 *    null stream).  All device work of a call is queued on that stream and the
 *    call returns after its results are on the host.
 *  - One handle must not be used by two threads at once.
 */
#ifndef MAYURA_H
#define MAYURA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MG_OK = 0,
    MG_EINVAL = -1,        /* bad argument (ids out of range, delta < 0, ...) */
    MG_ENOMEM = -2,        /* host or device allocation failed */
    MG_EDEVICE = -3,       /* a HIP call failed */
    MG_EUNSUPPORTED = -4,  /* valid input beyond the compiled limits */
    MG_EINTERNAL = -5
} mg_status;

/* compiled limits */
#define MG_MAX_EDGES_PER_MOTIF 5   /* k <= 5 */
#define MG_MAX_MOTIF_VERTICES 6    /* distinct motif vertices <= 6 */
#define MG_MAX_QUERIES 4096        /* distinct motifs per tree */

/* mg_graph_create flags */
#define MG_SORTED_BY_T 1u          /* caller promises t is non-decreasing */

typedef struct mg_graph mg_graph;  /* opaque */
typedef struct mg_tree mg_tree;    /* opaque */

/*
 * Optional device allocator (e.g. a framework's caching allocator).  alloc
 * returns a device pointer of at least `bytes` usable on `stream` (NULL on
 * failure); release frees it.  Passing NULL for both restores hipMalloc /
 * hipFree.  Affects allocations made after the call.
 */
typedef void *(*mg_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*mg_release_fn)(void *ptr, void *stream, void *ctx);
int mg_set_allocator(mg_alloc_fn alloc, mg_release_fn release, void *ctx);

/*
 * Load a temporal graph (paper, section 2.1 "A Temporal Graph"; data loading
 * into a time-sorted adjacency, section 4.2).
 *   src, dst : n_edges vertex ids in [0, n_nodes), host memory
 *   t        : n_edges timestamps, host memory, any order unless
 *              MG_SORTED_BY_T is given (then it must be non-decreasing)
 * The edges are stably sorted by t; edge i of the graph is position i of that
 * order and is the i-th root edge.  Self-loops are kept as roots but never
 * match (a motif edge has two distinct vertices and the vertex map is
 * injective).  The time-sorted edge list plus out- and in-adjacency (each
 * list ascending in t) are built on the host and copied to the device.
 * Limits: n_edges < 2^31; max(t) - min(t) < 2^63.
 */
int mg_graph_create(const int32_t *src, const int32_t *dst, const int64_t *t,
                    int64_t n_edges, int32_t n_nodes, uint32_t flags,
                    void *stream, mg_graph **out);

typedef struct {
    int64_t n_edges;
    int32_t n_nodes;
    int64_t self_loops;
    int64_t t_min, t_max;
    int32_t time_bytes;      /* 4: times stored as uint32 offsets, else 8 */
    int64_t device_bytes;    /* device memory held by the graph */
} mg_graph_info_t;
int mg_graph_info(const mg_graph *g, mg_graph_info_t *out);
void mg_graph_destroy(mg_graph *g);

/*
 * Build the MG-Tree of a motif group for a window delta (paper, section 4.3,
 * Algorithm 2).
 *   motif_uv : for motif i, motif_k[i] pairs (u, v) of vertex labels >= 0,
 *              motifs concatenated; the order of the pairs is the temporal
 *              order of the motif edges
 *   motif_k  : n_motifs edge counts, each in [1, MG_MAX_EDGES_PER_MOTIF]
 *   delta    : window, >= 0 (same unit as t)
 * Each motif is relabelled by first appearance (source before destination),
 * which makes equal prefixes under different labels the same node.
 * Duplicate motifs are allowed and receive identical counts.
 * Errors: MG_EINVAL for a label < 0, u == v, k < 1, delta < 0, n_motifs < 1;
 * MG_EUNSUPPORTED beyond the compiled limits.
 */
int mg_tree_create(const int32_t *motif_uv, const int32_t *motif_k,
                   int32_t n_motifs, int64_t delta, mg_tree **out);

typedef struct {
    int32_t n_motifs;        /* as given */
    int32_t n_distinct;      /* after relabelling and de-duplication */
    int32_t n_prefixes;      /* distinct non-empty prefixes (search levels) */
    int32_t n_nodes;         /* MG-Tree nodes (prefixes that branch or are queries, plus the root) */
    int32_t depth;           /* longest motif, in edges */
    int32_t root_edges;      /* |C_root|, edges common to every motif */
    double similarity;       /* SM, paper section 5: 1 - n_prefixes / sum of motif edges */
    int64_t delta;
} mg_tree_info_t;
int mg_tree_info(const mg_tree *tr, mg_tree_info_t *out);
void mg_tree_destroy(mg_tree *tr);

/* count modes */
#define MG_MODE_COMINE 0      /* one search over the whole MG-Tree (Algorithm 3) */
#define MG_MODE_PER_MOTIF 1   /* one search per distinct motif (Algorithm 1 per motif) */

typedef struct {
    int32_t mode;             /* MG_MODE_* */
    int32_t blocks;           /* persistent workgroups; 0 = fill the device */
    int32_t chunk;            /* roots claimed per queue grab, multiple of 64; 0 = default */
    int32_t queues;           /* root queues: 0 = one per XCD (8), else 1..8 */
    void *stream;             /* hipStream_t */
    const int64_t *roots;     /* host: root positions to search from; NULL = all */
    int64_t n_roots;
    float *elapsed_ms;        /* optional out: device time of the search kernel(s) */
    uint64_t *stats;          /* optional out, MG_NSTATS entries: search statistics
                                 (runs an instrumented kernel; not for timing) */
    uint64_t *root_cost;      /* optional out, n_edges entries indexed by root edge:
                                 1 + the candidate edges examined (window entries)
                                 in the search below that root, 0 for roots not
                                 searched; summed over motifs in per-motif mode.
                                 Runs an instrumented kernel; exclusive with stats. */
} mg_count_opts;

/* mg_count_opts.stats entries; every one is independent of the schedule */
#define MG_STAT_WIN_LIST 0   /* windows read from a per-vertex adjacency list */
#define MG_STAT_WIN_ALL 1    /* windows read from the whole time-ordered edge list */
#define MG_STAT_ENT_LIST 2   /* entries in per-vertex windows */
#define MG_STAT_ENT_ALL 3    /* entries in whole-list windows */
#define MG_STAT_PUSH 4       /* partial matches kept for a deeper level */
#define MG_STAT_CREDIT 5     /* prefix matches found below the first edge */
#define MG_STAT_ROOTS 6      /* root edges searched (self-loops excluded) */
#define MG_NSTATS 7

/* Fill opts with the defaults (co-mining, all roots, null stream). */
void mg_count_opts_init(mg_count_opts *opts);

/*
 * Count every motif of the tree in the graph (paper, Algorithm 3).
 *   opts   : NULL = defaults
 *   counts : host, n_motifs entries in the caller's motif order
 * The result is exact and independent of every scheduling option.
 */
int mg_count(const mg_graph *g, const mg_tree *tr, const mg_count_opts *opts,
             uint64_t *counts);

/* Thread-local description of the last failure on this thread. */
const char *mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MAYURA_H */
