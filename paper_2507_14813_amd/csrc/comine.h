// Internal interface between the host code (host.cpp) and the HIP kernels
// (comine.hip).  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace mg {

constexpr int kVMax = 6;        // motif vertices
constexpr int kKMax = 5;        // motif edges
constexpr int kWave = 64;
constexpr int kMaxDeltas = 8;   // windows counted in one search
constexpr int kWavesPerBlock = 4;
constexpr int kQueues = 8;      // root queues, one per XCD
constexpr int kQueueStride = 16;  // u64 words between queue heads (own cache line)
// queue words: kQueues root-queue heads, the work-item queue head, the claim
// counter of a chunk budget, each kQueueStride words apart
constexpr int kItemSlot = kQueues;
constexpr int kBudgetSlot = kQueues + 1;
constexpr int kQueueSlots = kQueues + 2;
constexpr int kQueueWords = kQueueSlots * kQueueStride;

// Root queue q of n_queues over n_roots roots holds positions [begin, end):
// boundaries on multiples of 64 roots, so that 64-root chunks are the
// scheduler's segments.  Host and device use this one definition.
__host__ __device__ inline uint32_t queue_begin(uint32_t n_roots, uint32_t n_queues, uint32_t q) {
    const uint64_t b = ((uint64_t)n_roots * q) / n_queues + 63;
    const uint32_t r = (uint32_t)(b & ~(uint64_t)63);
    return r < n_roots ? r : n_roots;
}
__host__ __device__ inline uint32_t queue_end(uint32_t n_roots, uint32_t n_queues, uint32_t q) {
    return q + 1 == n_queues ? n_roots : queue_begin(n_roots, n_queues, q + 1);
}
constexpr uint32_t kLeafScanDefault = 256;   // lane-counted leaf window limit

// fields of an internal-node word (see below)
__host__ __device__ inline uint32_t node_groups(uint32_t w) { return (w >> 20) & 31u; }
__host__ __device__ inline uint32_t node_near(uint32_t w) { return (w >> 25) & 31u; }
constexpr uint32_t kLeafParent = 1u << 30;
static_assert(2 * kVMax + 1 < 32, "groups of a node fit 5 bits");

// group direction: which adjacency list holds the candidates
enum : int { kDirOut = 0, kDirIn = 1, kDirAll = 2 };

// Search tables, as uploaded to the device.
//   inode[i]  internal (non-leaf) trie node i: first group | group count << 20
//             | count of the leading groups on a list of motif vertex 0 or 1 << 25
//             | leaf_parent << 30 (every child a leaf reached through a list
//             of a bound vertex: all groups leaf_only)
//   grp[2g], grp[2g+1]: eight words of group g:
//     w0 = dir | anchor << 4 | nv << 8 | leaf_only << 12 | last_end << 13
//          (nv: vertices bound at the owning node; leaf_only: a per-vertex
//          list whose children all end a motif; last_end: the anchor is the
//          source (1) or destination (2) of the owning node's last edge, 0
//          otherwise)
//     w1..w6 = child reached when the scanned endpoint is bound motif vertex 0..5
//     w7 = child reached when the scanned endpoint(s) are new vertices
//   A child word is 0 when there is no such child, else
//     internal index (bits 0-15, if internal) | (query + 1) << 16 | internal << 31.
// Counters: n_d per distinct motif, counter q * n_d + j holding the matches
// of motif q whose span (last time - first time) fits window j but not
// window j - 1 (windows ascending); the count at window j is the sum of
// slots 0..j.
struct DevTree {
    const uint32_t *inode;
    const uint4 *grp;
    int32_t n_q;        // distinct motifs
    int32_t root_q;     // query id of the one-edge prefix, -1 if none
    int32_t depth;      // longest motif in edges
    int32_t kdepth;     // kernel instantiation that searches it: depth, or 4
                        // for a depth-3 tree with a buffered two-edge prefix
                        // on four vertices (depth-3 kernels keep three)
    int32_t n_d;        // windows (1..kMaxDeltas), counter slots per motif
};
__host__ __device__ inline int32_t counter_slots(const DevTree &t) { return t.n_q * t.n_d; }

// One adjacency entry: the other endpoint and the edge time, side by side so
// that the bisection that finds a window also brings its entries into cache.
// Both layouts are two TT-sized words: entry i's time is ((TT *)list)[2i + 1]
// and its endpoint is ((int32_t *)list)[i * sizeof(Entry) / 4].
template <typename TT> struct Entry;
template <> struct Entry<uint32_t> { int32_t v; uint32_t t; };
template <> struct Entry<uint64_t> { int32_t v; int32_t pad; uint64_t t; };

template <typename TT>
struct DevGraph {
    const int32_t *gsrc, *gdst;   // time-sorted edge list (all edges)
    const TT *gt;
    const uint4 *gx;              // per edge u -> v at t: the first index with a later
                                  // time in out(u), in(u), out(v), in(v) (self-loops:
                                  // unused)
    const uint32_t *out_eid;      // edge id of every out_adj entry
    const uint32_t *in_eid;       // edge id of every in_adj entry
    const uint32_t *out_off;      // V+1
    const Entry<TT> *out_adj;     // out-lists: destination, time
    const uint32_t *in_off;
    const Entry<TT> *in_adj;      // in-lists: source, time
    uint32_t n_edges;
};

// A piece of search left over when an epoch ends: the candidates of one
// root-level window, entries [e0, e1) of the list of group g of the root
// a -> b at time t_lo | t_hi << 32, with the root's windows in out(a), in(a),
// out(b), in(b) as far as it had found them (first entry and length, as the
// per-wave root windows keep them).  The root itself was credited when it was
// started.
struct EpochCtx {
    int32_t a, b;
    uint32_t t_lo, t_hi;
    uint32_t g, e0, e1, pad;
    uint32_t hlo[4];
    uint16_t hlen[4];
    uint32_t pad2[2];
};
static_assert(sizeof(EpochCtx) == 64, "context record");
constexpr uint32_t kCtxPiece = 64;   // candidates per context at most

template <typename TT>
struct KParams {
    DevGraph<TT> g;
    DevTree tree;
    TT delta_sat;                 // the largest window, clamped to the TT range
    TT dlo[kMaxDeltas - 1];       // the smaller windows, ascending (tree.n_d - 1 of them)
    const uint32_t *roots;        // NULL: roots are 0..n_roots-1
    uint32_t n_roots;
    uint32_t chunk;               // roots per queue grab (multiple of 64)
    uint32_t n_queues;            // 1..kQueues root queues
    unsigned long long *queues;   // kQueueWords: queue heads (zeroed, or a resume
                                  // point) and the claim counter (zeroed)
    const int32_t *stop;          // NULL, or a flag (host-pinned or device memory)
                                  // read before every chunk claim: non-zero = claim
                                  // no more chunks
    uint32_t max_chunks;          // 0, or the launch claims at most this many chunks
    unsigned long long *counts;   // counter_slots(tree), zeroed before launch
    unsigned long long *stats;    // NULL, or kStats totals (zeroed before launch)
    unsigned long long *root_cost;  // NULL, or per root edge id: 1 + window entries
                                    // examined below that root (zeroed before launch)
    const uint2 *items;           // NULL, or work items searched before the queues:
                                  // {first, end} of root positions, or, with
                                  // kItemSplit set in .y, {root, kItemSplit |
                                  // part << 15 | nparts} (part < nparts < 2^15;
                                  // p.roots NULL): one part of one root's search
    const uint32_t *n_items;      // device count of items (with items)
    const uint8_t *skip;          // NULL, or per 64-root segment: 1 = covered by the
                                  // items (needs 64-root chunks and roots NULL)
    int32_t *enum_out;            // NULL, or enumeration: records of 1 + kKMax words
                                  // (distinct motif, edge ids, -1 past the motif's
                                  // length), enum_cap of them, at slots taken from
                                  // *enum_cursor (zeroed); needs leaf_scan 0
    unsigned long long *enum_cursor;
    unsigned long long enum_cap;
    unsigned long long *wave_clock;  // NULL, or per wave: start and end of its search
                                     // (device real-time clock ticks)
    uint32_t n_wave_clock;           // waves that wave_clock holds
    // epochs (the kernels' MODE 5 and 6, MODE 0 and 3 with epochs): ctx_out
    // and ctx_in NULL = off.  A wave that finds no work
    // left adds one to *idle; once *idle reaches idle_pct percent of the
    // launch's waves, the waves still searching stop expanding root-level
    // candidates, write what is left of their root-level windows as contexts,
    // finish what they already hold and exit.  The next launch searches the
    // contexts (ctx_in) instead of the root queues, claiming them through the
    // item slot of `queues`.
    EpochCtx *ctx_out;            // contexts written (ctx_cap at most; each wave at
                                  // most its share, ctx_cap / waves)
    unsigned long long *ctx_count;  // contexts written so far (zeroed)
    unsigned long long ctx_cap;
    uint32_t *idle;               // idle waves (zeroed)
    uint32_t idle_pct;            // the epoch ends once this percentage of the
                                  // launch's waves is idle (1..100)
    const EpochCtx *ctx_in;       // NULL, or the contexts this launch searches
    uint32_t n_ctx_in;
    uint32_t leaf_scan;           // windows whose children are all leaves are counted
                                  // without the candidate expansion: by one lane up
                                  // to this long, by the whole wave when longer
                                  // (0: never)
};

constexpr uint32_t kItemSplit = 0x80000000u;

// search statistics (schedule independent), filled when KParams::stats is set
enum : int {
    kStatWinList = 0,   // windows on a per-vertex list
    kStatWinAll,        // windows on the whole time-ordered edge list
    kStatEntList,       // entries scanned in per-vertex windows
    kStatEntAll,        // entries scanned in whole-list windows
    kStatPush,          // partial matches buffered for a deeper level
    kStatCredit,        // trie nodes reached below the root (prefix matches)
    kStatRoots,         // roots searched (non-self-loop)
    kStats
};

// Launch the persistent co-mining kernel.  `blocks` <= 0 fills the device.
// Returns a hipError_t value.
template <typename TT>
hipError_t launch_comine(const KParams<TT> &p, int blocks, hipStream_t stream);

// ---- batches: many (graph, tree) jobs in one launch
template <typename TT>
struct BatchJob {
    KParams<TT> p;                // the job's search (roots: every edge, in order)
    uint32_t count_off;           // first counter of this job in BatchParams::counts
};
struct BatchItem {
    uint32_t job, begin, end;   // roots [begin, end) of one job
    uint32_t part;              // 0, or kItemSplit | part << 15 | nparts: that part
                                // of the search from root `begin` (end = begin + 1)
};
template <typename TT>
struct BatchParams {
    const BatchJob<TT> *jobs;
    const BatchItem *items;
    uint32_t n_items;
    uint32_t n_q_max;             // largest tree's counter_slots
    unsigned long long *cursor;   // item queue head, zeroed before launch
    unsigned long long *counts;   // every job's counters, zeroed before launch
    uint32_t multi;               // 1 when some job's tree has several windows
};

// `depth` = the deepest tree of the batch.
template <typename TT>
hipError_t launch_batch(const BatchParams<TT> &bp, int depth, int blocks, hipStream_t stream);

// The same for one tree depth D (search.h; instantiated in search_d<D>_t<bits>.hip).
// MODE 0 is the plain search, 3 the search of trees with several windows.
template <typename TT, int D>
hipError_t launch_d(const KParams<TT> &p, int blocks, hipStream_t stream);
template <typename TT, int D, int MODE>
hipError_t launch_batch_d(const BatchParams<TT> &bp, int blocks, hipStream_t stream);

// Device scratch of the count that allocates nothing: queue words, then
// kMaxQueries counters, then kStats statistics.  One array per device, held
// until the process ends; *ptr is its address on the current device.
constexpr int kMaxQueries = 4096;
constexpr size_t kStaticWords = (size_t)kQueueWords + kMaxQueries + 8;
hipError_t static_scratch(unsigned long long **ptr);

// p[0..n) = v with a kernel (safe to record into a captured graph)
hipError_t launch_fill_u64(unsigned long long *p, uint32_t n, unsigned long long v,
                           hipStream_t stream);

}  // namespace mg
