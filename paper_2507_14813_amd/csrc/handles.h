// Internal definitions shared by the host files of the library (host.cpp:
// the C ABI and the GPU path; cpu.cpp: the CPU co-mining backend).  Not part
// of the public C ABI.
#pragma once
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mayura.h"

namespace mgh {

// Records a failure for mg_last_error and returns `code`.
int fail(int code, const char *fmt, ...);

// A device allocation (the registered allocator, or hipMalloc).
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    void *stream = nullptr;
    bool custom = false;
    mg_release_fn release = nullptr;
    void *ctx = nullptr;
};
int dev_alloc(DevBuf &b, size_t bytes, void *stream);
void dev_free(DevBuf &b);

// Host copy of a graph for the CPU backend: the time-sorted edge list and
// the out- and in-lists (self-loops left out), each list ascending in time.
struct HostAdj {
    std::vector<int32_t> src, dst;
    std::vector<int64_t> t;
    std::vector<uint32_t> out_off, in_off;
    std::vector<int32_t> out_v, in_v;
    std::vector<int64_t> out_t, in_t;
};

// A prefix of the motif group: one node of the search trie.
struct TrieNode {
    int parent = -1;
    int u = 0, v = 0;      // edge that extends the parent (canonical labels)
    int depth = 0;         // edges in the prefix
    int nv = 0;            // vertices bound after the prefix
    std::vector<int> kids;
    int q = -1;            // distinct motif whose edge sequence is this prefix
};

using Motif = std::vector<std::pair<int, int>>;

}  // namespace mgh

struct mg_graph {
    int64_t E = 0;
    int32_t V = 0;
    int64_t self_loops = 0;
    int64_t t_min = 0, t_max = 0;
    int time_bytes = 4;
    int device = 0;
    bool host_only = false;             // no device copy (MG_HOST_ONLY)
    std::vector<int64_t> input_index;   // caller's index of each edge (empty: the same)
    mgh::DevBuf gsrc, gdst, gt, gx, out_eid, in_eid, out_off, out_adj, in_off, in_adj;
    int64_t device_bytes = 0;
    std::unique_ptr<mgh::HostAdj> host;   // for the CPU backend, built on first use
    int8_t bipartite = -1;              // -1 unknown, else whether the undirected graph is
    ~mg_graph();
};

struct mg_tree {
    int32_t n_motifs = 0;
    int64_t delta = 0;                  // the largest window
    std::vector<int64_t> deltas;        // distinct windows, ascending
    std::vector<int32_t> delta_slot;    // caller's window i -> index in deltas
    std::vector<int32_t> motif_q;       // caller motif -> distinct id
    std::vector<mgh::Motif> distinct;
    std::vector<mgh::TrieNode> nodes;   // node 0 = prefix ((0,1))
    std::vector<int32_t> node_tab;      // one word per internal node
    std::vector<int32_t> grp_tab;       // 8 words per group
    int32_t depth = 0, root_q = -1;
    int32_t kdepth = 0;    // depth of the kernel that searches it (DevTree::kdepth)
    mg_tree_info_t info{};
    // device copies
    int device = -1;
    mgh::DevBuf d_node, d_grp;
    // per-motif chain trees (built on first per-motif count)
    std::vector<std::unique_ptr<mg_tree>> singles;
    // CPU backend: the generated and compiled search of this tree
    void *cpu_lib = nullptr;
    void *cpu_fn = nullptr;
    std::string cpu_error;              // why generation failed, if it did
    ~mg_tree();
};

namespace mgh {
// releases the CPU backend's compiled code of a tree (cpu.cpp)
void release_cpu_code(mg_tree *tr);
// the host copy of a graph from its time-sorted edge list (cpu.cpp)
void build_host(mg_graph *g, std::vector<int32_t> s, std::vector<int32_t> d, std::vector<int64_t> t);
// the per-motif chain trees of a tree, built once (host.cpp)
int chain_trees(mg_tree *tr);
}  // namespace mgh
