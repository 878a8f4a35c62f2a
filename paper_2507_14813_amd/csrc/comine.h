// Internal interface between the host code (host.cpp) and the HIP kernels
// (comine.hip).  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace mg {

constexpr int kVMax = 6;        // motif vertices
constexpr int kKMax = 5;        // motif edges
constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;

// group direction: which adjacency list holds the candidates
enum : int { kDirOut = 0, kDirIn = 1, kDirAll = 2 };

// Trie ("search level") tables, as uploaded to the device.
//   node[n] = {query id or -1, first group, group count, nv | internal << 8}
//   grp[2g], grp[2g+1] = {dir | anchor << 4, child_new, tgt0..tgt5}
struct DevTree {
    const int4 *node;
    const int4 *grp;
    int32_t n_q;        // distinct motifs (counter slots)
    int32_t root_q;     // query id of the one-edge prefix, -1 if none
    int32_t depth;      // longest motif in edges
};

template <typename TT>
struct DevGraph {
    const int32_t *gsrc, *gdst;   // time-sorted edge list (all edges)
    const TT *gt;
    const uint32_t *out_off;      // V+1
    const int32_t *out_nbr;       // destination of each out-entry
    const TT *out_t;
    const uint32_t *in_off;
    const int32_t *in_nbr;        // source of each in-entry
    const TT *in_t;
    uint32_t n_edges;
};

template <typename TT>
struct KParams {
    DevGraph<TT> g;
    DevTree tree;
    TT delta_sat;                 // delta clamped to the TT range
    const uint32_t *roots;        // NULL: roots are 0..n_roots-1
    uint32_t n_roots;
    uint32_t chunk;               // roots per queue grab
    uint32_t *cursor;             // queue head, zeroed before launch
    unsigned long long *counts;   // n_q, zeroed before launch
    unsigned long long *stats;    // NULL, or kStats totals (zeroed before launch)
};

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

// Blocks that fill the device for this tree depth and counter count.
template <typename TT>
int comine_fill_blocks(int depth, int n_q);

}  // namespace mg
