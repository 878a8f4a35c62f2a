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
#define MG_MAX_QUERIES 4096        /* counters per tree: distinct motifs x windows */
#define MG_MAX_DELTAS 8            /* windows counted in one search */

/* mg_graph_create flags */
#define MG_SORTED_BY_T 1u          /* caller promises t is non-decreasing */
#define MG_DEVICE_INPUT 2u         /* src, dst and t are device pointers (current
                                      device); they are read on `stream` */
#define MG_HOST_ONLY 4u            /* keep the graph on the host only, for the CPU
                                      backend (mg_count_cpu); no device is needed and
                                      the GPU entry points refuse the graph */

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
 *   src, dst : n_edges vertex ids in [0, n_nodes), host memory (device
 *              memory with MG_DEVICE_INPUT)
 *   t        : n_edges timestamps, same memory as src, any order unless
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

/*
 * One tree for several windows at once (the window sweep of the paper's
 * evaluation, "Effect of delta", and its appendix table of delta/4 against
 * 4 delta).  The search runs once, at the largest window; a match whose span
 * (last time minus first time) is s counts for every window >= s, which is
 * exact because a match within a window is also within every larger one.
 *   deltas   : n_deltas windows, each >= 0, any order (duplicates allowed)
 * mg_count then returns n_deltas * n_motifs counts, window-major:
 * counts[i * n_motifs + m] is motif m at deltas[i].  mg_tree_create is the
 * case n_deltas = 1.  Errors as mg_tree_create; MG_EUNSUPPORTED beyond
 * MG_MAX_DELTAS windows or MG_MAX_QUERIES counters.
 */
int mg_tree_create_multi(const int32_t *motif_uv, const int32_t *motif_k,
                         int32_t n_motifs, const int64_t *deltas, int32_t n_deltas,
                         mg_tree **out);

typedef struct {
    int32_t n_motifs;        /* as given */
    int32_t n_distinct;      /* after relabelling and de-duplication */
    int32_t n_prefixes;      /* distinct non-empty prefixes (search levels) */
    int32_t n_nodes;         /* MG-Tree nodes (prefixes that branch or are queries, plus the root) */
    int32_t depth;           /* longest motif, in edges */
    int32_t root_edges;      /* |C_root|, edges common to every motif */
    double similarity;       /* SM, paper section 5: 1 - n_prefixes / sum of motif edges */
    int64_t delta;           /* the largest window */
    int32_t n_deltas;        /* windows as given */
} mg_tree_info_t;
int mg_tree_info(const mg_tree *tr, mg_tree_info_t *out);
void mg_tree_destroy(mg_tree *tr);

/* count modes */
#define MG_MODE_COMINE 0      /* one search over the whole MG-Tree (Algorithm 3) */
#define MG_MODE_PER_MOTIF 1   /* one search per distinct motif (Algorithm 1 per motif) */
#define MG_MODE_AUTO 2        /* mg_count only: co-mining or per-motif mining as the
                                 paper's heuristic advises for the GPU
                                 (mg_comine_advice) */

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
    int32_t sched;            /* MG_SCHED_PLAIN (default) or MG_SCHED_LEARNED */
    int32_t leaf_scan;        /* windows whose children all end a motif are
                                 counted without the candidate expansion, one
                                 equality count per bound vertex: by the window's
                                 own lane when at most this long, by the whole
                                 wave (one ballot per bound vertex) when longer.
                                 0 = default (256), < 0 = never (every window goes
                                 through the candidate expansion).  In trees of
                                 three edges, a window on a later vertex's out-list
                                 whose edges can only close on the root's vertices
                                 may instead be counted, by its lane, in those
                                 vertices' in-lists when they are shorter. */
    const struct mg_model *model;   /* cost model for MG_SCHED_LEARNED */
    uint64_t *root_cost;      /* optional out, n_edges entries indexed by root edge:
                                 1 + the candidate edges examined (window entries)
                                 in the search below that root, 0 for roots not
                                 searched; summed over motifs in per-motif mode.
                                 Runs an instrumented kernel; exclusive with stats. */
    int32_t sample;           /* MG_SCHED_LEARNED: the model scores one root in
                                 `sample` of every 64-root segment (a power of
                                 two, 1..64; 0 = default 1) */
    /* Stopping and resuming (the counterpart of the paper's epoch contexts,
     * section 4.5, which let a search be suspended and picked up again).
     * Every wave reads `stop` and takes a claim from the budget before it
     * claims a chunk of roots; a chunk once claimed is searched to the end.
     * So a launch that stops has searched a prefix of every root queue, and
     * `cursor` records those prefixes.  Supported with MG_MODE_COMINE and
     * MG_SCHED_PLAIN only. */
    const int32_t *stop;      /* NULL, or a flag in host-pinned (hipHostMalloc)
                                 or device memory: non-zero = claim no more
                                 chunks.  The caller may set it while the call
                                 runs. */
    int64_t max_chunks;       /* 0 = no limit, else claim at most this many chunks
                                 in this call (and at least one while roots are
                                 left, unless stopped by the flag) */
    struct mg_cursor *cursor; /* NULL, or in/out resume point (below) */
    uint64_t *wave_clock;     /* optional out (co-mining only), wave_clock_len
                                 entries: entries 2w and 2w + 1 get the start and
                                 end of wave w's search in ticks of the device's
                                 constant real-time clock (its rate is
                                 hipDeviceAttributeWallClockRate, kHz); entries of
                                 waves not launched are 0.  For measuring how
                                 evenly a schedule ends; counts are unchanged. */
    int64_t wave_clock_len;
    /* Epochs (paper, section 4.5: inter-warp load balancing).  With
     * epoch_idle > 0, a launch ends its epoch once that percentage of its
     * waves has run out of work: the waves still searching write what is left
     * of their root-level windows as contexts (root edge, group, a range of
     * at most 64 candidates), finish the deeper work they already hold and
     * exit.  The next launch spreads those contexts over all of its waves, and
     * so on until no context is left; the last of max_epochs launches runs to
     * the end.  A context's candidates are never searched twice, so counts
     * are exact.  MG_MODE_COMINE with MG_SCHED_PLAIN only, and not with stop,
     * max_chunks, cursor, stats, root_cost or wave_clock (MG_EINVAL). */
    int32_t epoch_idle;       /* 0 = off, else 1..100 (percent of the waves) */
    int32_t max_epochs;       /* launches at most; 0 = default (16) */
    int64_t *epoch_contexts;  /* optional out, max_epochs entries: contexts
                                 carried out of each launch (0 from the last
                                 one on) */
} mg_count_opts;

/* Resume point of a stopped count.  Initialise with mg_cursor_init; pass the
 * same cursor, graph, tree, roots, chunk and queues to every call of one
 * count.  Each call's counts are those of the roots it searched, so the sum
 * over the calls until `done` is the full count (and likewise stats and
 * root_cost). */
#define MG_CURSOR_QUEUES 8
typedef struct mg_cursor {
    uint64_t head[MG_CURSOR_QUEUES]; /* roots already searched from each root queue */
    int64_t n_roots;          /* roots of the count the cursor belongs to */
    int32_t chunk, queues;    /* the settings it was made with (resolved defaults) */
    int32_t started;          /* 0 = fresh: start from the first root */
    int32_t done;             /* out: 1 once every root has been searched */
} mg_cursor;
void mg_cursor_init(mg_cursor *c);

/* mg_count_opts.stats entries; every one is independent of the schedule */
#define MG_STAT_WIN_LIST 0   /* windows read from a per-vertex adjacency list */
#define MG_STAT_WIN_ALL 1    /* windows read from the whole time-ordered edge list */
#define MG_STAT_ENT_LIST 2   /* entries in per-vertex windows */
#define MG_STAT_ENT_ALL 3    /* entries in whole-list windows */
#define MG_STAT_PUSH 4       /* partial matches kept for a deeper level */
#define MG_STAT_CREDIT 5     /* prefix matches found below the first edge */
#define MG_STAT_ROOTS 6      /* root edges searched (self-loops excluded) */
#define MG_NSTATS 7

/* schedules (what runs where; never what is counted) */
#define MG_SCHED_PLAIN 0      /* roots in time order, 64-root chunks from XCD queues */
#define MG_SCHED_LEARNED 1    /* an MLP predicts the cost of every 64-root
                                 segment; segments above 8x the mean run first,
                                 heaviest first (the costliest split into single
                                 roots, a root still above 1/32768 of the total
                                 into up to 16 parts of its first-level
                                 candidates), then the rest in time order from
                                 the root queues in 64-root chunks (ignores
                                 chunk) */

/* Fill opts with the defaults (co-mining, all roots, null stream). */
void mg_count_opts_init(mg_count_opts *opts);

/*
 * Count every motif of the tree in the graph (paper, Algorithm 3).
 *   opts   : NULL = defaults
 *   counts : host, n_deltas * n_motifs entries: for each window in the
 *            caller's order, the motifs in the caller's motif order
 * The result is exact and independent of every scheduling option.
 */
int mg_count(const mg_graph *g, const mg_tree *tr, const mg_count_opts *opts,
             uint64_t *counts);

/*
 * Enumeration: every match itself, not only the counts (paper, section 2.1:
 * a match is a sequence of edges; the matcher of Algorithm 1 records each one
 * it completes).  The count sizes the output, then the same search writes one
 * record per match -- the motif and its edges in the motif's order -- in no
 * particular order.
 *   out       : host, capacity records; with NULL or a capacity below the
 *               number of matches nothing is written and *n_matches tells how
 *               many records are needed
 *   motif     : the caller's motif index (for duplicate motifs, the first one
 *               with that edge sequence; the others have the same matches)
 *   edges     : the caller's edge indices (the input order of
 *               mg_graph_create), -1 past the motif's length
 * MG_EUNSUPPORTED for a tree with several windows.
 */
typedef struct {
    int32_t motif;
    int32_t edges[MG_MAX_EDGES_PER_MOTIF];
} mg_match;
int mg_enumerate(const mg_graph *g, const mg_tree *tr, void *stream, mg_match *out,
                 int64_t capacity, int64_t *n_matches);

/*
 * mg_count for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same search, with its queue heads, counters and statistics in a static
 * device array of MG_NOALLOC_SCRATCH_BYTES per GPU (held until the process
 * ends) instead of memory allocated per call.  Nothing is allocated: no
 * hipMalloc, hipFree, events or allocator callbacks.
 *   opts : NULL = defaults.  Accepted: blocks, chunk, queues, stream,
 *          leaf_scan, stats, stop, max_chunks.  MG_EINVAL for anything that
 *          needs memory of its own: per-motif mode, the learned schedule,
 *          roots, root_cost, elapsed_ms, cursor, wave_clock.
 * The tree's device tables must already exist on the current device (any
 * earlier mg_count of the tree there creates them), else MG_EINVAL.
 * MG_EUNSUPPORTED when the tree has more distinct motifs than the array
 * holds (MG_MAX_QUERIES).  Every call on one GPU shares that GPU's array, so
 * calls that overlap on one GPU (two threads, or two streams in flight) race
 * and must be serialised by the caller; each call clears what it uses before
 * its search and returns after its counts are on the host.
 */
#define MG_NOALLOC_SCRATCH_BYTES ((160 + MG_MAX_QUERIES + 8) * 8)   /* 34,112 */
int mg_count_noalloc(const mg_graph *g, const mg_tree *tr, const mg_count_opts *opts,
                     uint64_t *counts);

/*
 * CPU backend (paper, section 5.1.1 "CPU code-generation" and its appendix
 * listing of the generated nested loops): the search of the tree is emitted
 * as C++ with one loop nest per level of the prefix trie, compiled by the
 * host compiler (MG_CXX, else c++; once per tree), loaded and run over the
 * root edges on the host's cores with dynamic chunks of roots.  codegen = 0
 * interprets the trie instead (the recursion of the paper's CPU baseline).
 * The graph may be MG_HOST_ONLY; a device graph is read back once.  Counts
 * as mg_count (exact, every window of the tree).
 */
typedef struct {
    int32_t mode;             /* MG_MODE_COMINE or MG_MODE_PER_MOTIF */
    int32_t threads;          /* 0 = every host core */
    int32_t codegen;          /* 1 = generated and compiled search (default), 0 = interpreted */
    int32_t reserved;
    const int64_t *roots;     /* host: root positions; NULL = all */
    int64_t n_roots;
    double *elapsed_ms;       /* optional out: wall time of the searches (code
                                 generation and compilation not included) */
} mg_cpu_opts;
void mg_cpu_opts_init(mg_cpu_opts *opts);
int mg_count_cpu(const mg_graph *g, const mg_tree *tr, const mg_cpu_opts *opts,
                 uint64_t *counts);

/*
 * The paper's heuristic for whether co-mining pays (section 7, "Heuristic
 * for Co-Mining"): on a bipartite graph (edges taken as undirected) always;
 * on the GPU not when the group's similarity SM is below 0.44 (the paper's
 * measured break-even); otherwise yes (a smaller window helps further).
 */
#define MG_PLATFORM_GPU 0
#define MG_PLATFORM_CPU 1
#define MG_GPU_SM_THRESHOLD 0.44
typedef struct {
    int32_t co_mine;          /* 1 = co-mine, 0 = mine each motif on its own */
    int32_t bipartite;        /* the graph is bipartite */
    double similarity;        /* the tree's SM */
    double threshold;         /* the SM the platform needs (0 on the CPU) */
} mg_advice;
int mg_comine_advice(const mg_graph *g, const mg_tree *tr, int32_t platform, mg_advice *out);

/*
 * Autotuner (not in the paper): picks the launch settings of mg_count for a
 * (graph, tree, device) by timing plain co-mining counts: the leaf-count
 * limit (leaf_scan), roots per chunk, root queues and workgroups, one at a
 * time from the defaults (coordinate descent, two sweeps at most, a setting
 * kept only when it is more than 2 % faster).  Counts never depend on these
 * settings.
 *   cache_path : NULL, or a file of one JSON object per line keyed by the
 *                graph's and tree's statistics and the device: a cached entry
 *                is returned without timing; a new result is appended
 *   out        : the chosen settings (copy them into mg_count_opts), their
 *                time and that of the defaults
 */
typedef struct {
    int32_t blocks, chunk, queues, leaf_scan;   /* the settings */
    float ms;                 /* median search time with them */
    float default_ms;         /* the same with the defaults */
    int32_t from_cache;       /* 1 when read from the cache */
    int32_t trials;           /* settings timed (0 from the cache) */
} mg_tune_result;
int mg_tune(const mg_graph *g, const mg_tree *tr, const char *cache_path, void *stream,
            mg_tune_result *out);

/*
 * Learned root-cost model (not in the paper): a 4-layer MLP, 16 -> 64 -> 64 ->
 * 64 -> 1 with ReLU, BF16 weights and activations, FP32 accumulation (MFMA),
 * that predicts log(1 + candidate edges examined below a root) -- the label
 * mg_count_opts.root_cost logs.  Parameters are an FP32 master copy of
 * MG_MODEL_PARAMS floats laid out as W1[32][64] (rows 16..31 zero), b1[64],
 * W2[64][64], b2[64], W3[64][64], b3[64], W4[64], b4 (row-major [in][out]).
 * All model calls run on the null stream and return when done.
 */
#define MG_NFEATURES 16
#define MG_MODEL_PARAMS 10497
typedef struct mg_model mg_model;  /* opaque */
/* He-initialised weights from a seeded generator, zero biases. */
int mg_model_create(uint64_t seed, mg_model **out);
int mg_model_get_weights(const mg_model *m, float *w /* MG_MODEL_PARAMS */);
int mg_model_set_weights(mg_model *m, const float *w /* MG_MODEL_PARAMS */);
/* Adam's first and second moments (MG_MODEL_PARAMS floats each, host; either
 * may be NULL), in the parameter layout above.  After one step from fresh
 * moments (mg_model_create or mg_model_set_weights), m1 = (1 - 0.9) * g and
 * m2 = (1 - 0.999) * g^2 for the minibatch gradient g of the mean squared
 * error, so the backward pass can be read back exactly. */
int mg_model_get_moments(const mg_model *m, float *m1, float *m2);
void mg_model_destroy(mg_model *m);
/* Features of roots (positions in time order; NULL = all n_edges roots) into
 * feats (host, n x MG_NFEATURES): scaled log1p of the out/in degrees of both
 * endpoints, of the entries of out(a), out(b), in(a), in(b) and of the whole
 * edge list in the root's window (t, t + delta], the tree depth and the
 * number of distinct motifs, and a constant 1 (all zero for self-loops). */
int mg_root_features(const mg_graph *g, const mg_tree *tr, const int64_t *roots, int64_t n,
                     float *feats);
/* Forward pass on host features (n x MG_NFEATURES) -> out[n] (host). */
int mg_model_predict(const mg_model *m, const float *feats, int64_t n, float *out);
/* Adam (lr, betas 0.9/0.999) on mean squared error, minibatches of 32 in a
 * seeded shuffled order; loss (optional, host) gets the mean loss per epoch. */
int mg_model_train(mg_model *m, const float *feats, const float *labels, int64_t n,
                   int32_t epochs, float lr, uint64_t seed, float *loss);

/*
 * Batches: many (graph, tree) jobs of uneven size counted by one persistent
 * kernel launch.  The work queue holds root ranges ("items") of every job,
 * largest graphs first; each step zeroes the counters with a fill kernel,
 * runs the batched kernel and copies the counts back, and after the first
 * step that sequence is replayed as one captured HIP graph.
 *
 *   graphs, trees : n jobs (the same graph may appear in several jobs); all
 *                   graphs must live on the current device and use the same
 *                   time width (mg_graph_info_t.time_bytes)
 *   opts          : NULL = defaults (autotuned item size, graph replay)
 * The handles must outlive the batch.  Counts are exact and independent of
 * every option.
 */
typedef struct mg_batch mg_batch;  /* opaque */
typedef struct {
    int32_t blocks;           /* persistent workgroups; 0 = fill the device */
    int32_t item_roots;       /* roots per work item (multiple of 64); 0 = autotune */
    int32_t use_graph;        /* 1 = capture the step and replay it (default), 0 = plain launches */
    int32_t reserved;
    void *stream;             /* hipStream_t the steps run on (NULL = null stream) */
    const struct mg_model *model;  /* optional: the model predicts every job's
                                      64-root segments at creation; segments above
                                      8x the mean run first, heaviest first (the
                                      costliest as one item per root, a root above
                                      1/(128 x CUs) of the total in up to 16 parts
                                      of its first-level candidates), then every
                                      other segment in job order (largest graph
                                      first) and time order (item_roots is then
                                      ignored) */
} mg_batch_opts;
void mg_batch_opts_init(mg_batch_opts *opts);
int mg_batch_create(const mg_graph *const *graphs, const mg_tree *const *trees, int32_t n,
                    const mg_batch_opts *opts, mg_batch **out);

/* One step.  counts: host, sum of the trees' n_deltas * n_motifs,
 * concatenated in job order, each tree laid out as mg_count lays it out.  elapsed_ms (optional): device
 * time of the step from events on the batch's stream. */
int mg_batch_count(mg_batch *b, uint64_t *counts, float *elapsed_ms);

typedef struct {
    int32_t n_jobs;
    int32_t total_motifs;     /* length of the counts output */
    int64_t total_roots;
    int64_t n_items;
    int32_t item_roots;       /* chosen (or given) item size */
    int32_t blocks;           /* 0 = filled the device */
    int32_t graph_captured;   /* 1 once a HIP graph replays the step */
    int32_t depth;            /* depth of the search kernel: the deepest tree's
                                 edges, or 4 for a three-edge tree with a two-edge
                                 prefix on four vertices */
    float tuned_ms;           /* best step time seen by the autotuner (0 if none) */
    int32_t learned;          /* 1 when items come from the cost model */
    float predict_ms;         /* wall time of the cost model at creation: features,
                                 MLP and ordering of the items (0 without a model) */
} mg_batch_info_t;
int mg_batch_info(const mg_batch *b, mg_batch_info_t *out);
void mg_batch_destroy(mg_batch *b);

/*
 * One-shot batch: mg_batch_create, one mg_batch_count and mg_batch_destroy
 * in one call, for a set of jobs counted once.  A plan that is counted once
 * gains nothing from a captured graph or from autotuning (which times
 * several steps), so use_graph is ignored and item_roots 0 means 64.
 * counts: as mg_batch_count.
 */
int mg_count_batch(const mg_graph *const *graphs, const mg_tree *const *trees, int32_t n,
                   const mg_batch_opts *opts, uint64_t *counts);

/* Thread-local description of the last failure on this thread. */
const char *mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MAYURA_H */
