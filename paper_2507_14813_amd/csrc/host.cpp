// Host side of the C ABI declared in include/mayura.h: graph ingest into
// time-sorted adjacency, motif relabelling, MG-Tree / search-trie
// construction and flattening, and the count dispatch.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mayura.h"
#include "comine.h"
#include "handles.h"
#include "sched.h"

using mg::kVMax;
using mg::kKMax;
// the learned schedule predicts the cost of one root in this many per segment
constexpr uint32_t kSampleDefault = 1;
// most items one root's search is split into by the learned schedule
constexpr uint32_t kRootParts = 16;
// queue heads (root queues, work items, chunk budget)
constexpr size_t kQueueBytes = sizeof(unsigned long long) * mg::kQueueWords;
static_assert(MG_CURSOR_QUEUES == mg::kQueues, "cursor layout");
static_assert(MG_MAX_QUERIES == mg::kMaxQueries, "query limit");
static_assert(MG_MAX_DELTAS == mg::kMaxDeltas, "window limit");
static_assert(MG_NOALLOC_SCRATCH_BYTES == 8 * mg::kStaticWords, "static scratch size");

namespace mgh {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return fail(MG_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- allocator
mg_alloc_fn g_alloc = nullptr;
mg_release_fn g_release = nullptr;
void *g_alloc_ctx = nullptr;

int dev_alloc(DevBuf &b, size_t bytes, void *stream) {
    b.bytes = bytes;
    b.stream = stream;
    if (bytes == 0) bytes = 16;
    if (g_alloc) {
        b.ptr = g_alloc(bytes, stream, g_alloc_ctx);
        b.custom = true;
        b.release = g_release;
        b.ctx = g_alloc_ctx;
        if (!b.ptr) return fail(MG_ENOMEM, "device allocator returned NULL for %zu bytes", bytes);
        return MG_OK;
    }
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        return fail(MG_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    return MG_OK;
}

void dev_free(DevBuf &b) {
    if (!b.ptr) return;
    if (b.custom) {
        if (b.release) b.release(b.ptr, b.stream, b.ctx);
    } else {
        (void)hipFree(b.ptr);
    }
    b.ptr = nullptr;
}

}  // namespace mgh

using namespace mgh;

mg_graph::~mg_graph() {
    for (DevBuf *b : {&gsrc, &gdst, &gt, &gx, &out_eid, &in_eid, &out_off, &out_adj, &in_off,
                      &in_adj})
        dev_free(*b);
}

namespace {

// f(begin, end) over [0, n) in contiguous pieces on the host's cores
template <typename F>
void parallel_for(int64_t n, F f) {
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(std::thread::hardware_concurrency(),
                                                                n / 65536 + 1));
    std::vector<std::thread> th;
    for (int64_t k = 0; k < nt; ++k)
        th.emplace_back([&, k] { f(n * k / nt, n * (k + 1) / nt); });
    for (auto &x : th) x.join();
}

template <typename TT>
int upload_graph(mg_graph *g, const std::vector<int32_t> &s, const std::vector<int32_t> &d,
                 const std::vector<int64_t> &t, hipStream_t st) {
    const int64_t E = g->E;
    const int32_t V = g->V;
    std::vector<TT> rt(E);
    for (int64_t i = 0; i < E; ++i) rt[i] = (TT)(uint64_t)(t[i] - g->t_min);

    // out/in adjacency (self-loops excluded), each list in time order:
    // a counting sort by vertex over the time-ordered edge list is stable.
    std::vector<uint32_t> oo(V + 1, 0), io(V + 1, 0);
    for (int64_t i = 0; i < E; ++i)
        if (s[i] != d[i]) { oo[s[i] + 1]++; io[d[i] + 1]++; }
    for (int32_t v = 0; v < V; ++v) { oo[v + 1] += oo[v]; io[v + 1] += io[v]; }
    const uint32_t A = oo[V];
    std::vector<mg::Entry<TT>> oadj(A), iadj(A);
    std::vector<uint32_t> oeid(A), ieid(A);   // edge id of every list entry
    {
        std::vector<uint32_t> po(oo.begin(), oo.end() - 1), pi(io.begin(), io.end() - 1);
        for (int64_t i = 0; i < E; ++i) {
            if (s[i] == d[i]) continue;
            oeid[po[s[i]]] = (uint32_t)i;
            ieid[pi[d[i]]] = (uint32_t)i;
            mg::Entry<TT> &x = oadj[po[s[i]]++];
            std::memset(&x, 0, sizeof x);
            x.v = d[i]; x.t = rt[i];
            mg::Entry<TT> &y = iadj[pi[d[i]]++];
            std::memset(&y, 0, sizeof y);
            y.v = s[i]; y.t = rt[i];
        }
    }
    // per edge (u -> v at t): where the entries after time t start in out(u),
    // in(u), out(v) and in(v) -- the first index with a later time
    std::vector<uint32_t> gx(4 * (size_t)E, 0);
    parallel_for(E, [&](int64_t i0, int64_t i1) {
        auto after = [&](const std::vector<mg::Entry<TT>> &adj, const std::vector<uint32_t> &off,
                         int32_t v, TT t) {
            uint32_t lo = off[v], n = off[v + 1] - off[v];
            while (n > 0) {
                const uint32_t h = n >> 1;
                if (adj[lo + h].t <= t) { lo += h + 1; n -= h + 1; }
                else n = h;
            }
            return lo;
        };
        for (int64_t i = i0; i < i1; ++i) {
            if (s[i] == d[i]) continue;
            gx[4 * i + 0] = after(oadj, oo, s[i], rt[i]);
            gx[4 * i + 1] = after(iadj, io, s[i], rt[i]);
            gx[4 * i + 2] = after(oadj, oo, d[i], rt[i]);
            gx[4 * i + 3] = after(iadj, io, d[i], rt[i]);
        }
    });
    struct Up { DevBuf *b; const void *h; size_t n; };
    Up ups[] = {
        {&g->gsrc, s.data(), sizeof(int32_t) * E}, {&g->gdst, d.data(), sizeof(int32_t) * E},
        {&g->gt, rt.data(), sizeof(TT) * E},
        {&g->gx, gx.data(), sizeof(uint32_t) * 4 * E},
        {&g->out_eid, oeid.data(), sizeof(uint32_t) * A},
        {&g->in_eid, ieid.data(), sizeof(uint32_t) * A},
        {&g->out_off, oo.data(), sizeof(uint32_t) * (V + 1)},
        {&g->out_adj, oadj.data(), sizeof(mg::Entry<TT>) * A},
        {&g->in_off, io.data(), sizeof(uint32_t) * (V + 1)},
        {&g->in_adj, iadj.data(), sizeof(mg::Entry<TT>) * A},
    };
    g->device_bytes = 0;
    for (auto &u : ups) {
        int rc = dev_alloc(*u.b, u.n, (void *)st);
        if (rc) return rc;
        if (u.n) HIP_TRY(hipMemcpyAsync(u.b->ptr, u.h, u.n, hipMemcpyHostToDevice, st));
        g->device_bytes += (int64_t)u.n;
    }
    HIP_TRY(hipStreamSynchronize(st));
    return MG_OK;
}

}  // namespace

// ---------------------------------------------------------------- tree
mg_tree::~mg_tree() {
    dev_free(d_node);
    dev_free(d_grp);
    release_cpu_code(this);
}

namespace {

// First-appearance relabelling: vertices are numbered in the order they are
// first seen, source before destination.  Two motifs are the same ordered
// edge sequence up to relabelling iff their relabelled forms are equal.
int canonical(const int32_t *uv, int k, Motif &out) {
    std::vector<std::pair<int32_t, int>> seen;
    auto id = [&](int32_t x) {
        for (auto &p : seen) if (p.first == x) return p.second;
        seen.push_back({x, (int)seen.size()});
        return (int)seen.size() - 1;
    };
    out.clear();
    for (int j = 0; j < k; ++j) {
        int32_t a = uv[2 * j], b = uv[2 * j + 1];
        if (a < 0 || b < 0) return fail(MG_EINVAL, "motif vertex label < 0");
        if (a == b) return fail(MG_EINVAL, "motif edge %d is a self-loop", j);
        int ia = id(a), ib = id(b);
        out.push_back({ia, ib});
    }
    if ((int)seen.size() > kVMax)
        return fail(MG_EUNSUPPORTED, "motif has %d vertices (limit %d)", (int)seen.size(), kVMax);
    return MG_OK;
}

// Build the prefix trie, then the flat tables the kernel reads.
int build_tree(mg_tree *tr) {
    tr->nodes.clear();
    TrieNode root;
    root.u = 0; root.v = 1; root.depth = 1; root.nv = 2;
    tr->nodes.push_back(root);
    for (size_t q = 0; q < tr->distinct.size(); ++q) {
        const Motif &m = tr->distinct[q];
        int cur = 0;
        for (size_t j = 1; j < m.size(); ++j) {
            int found = -1;
            for (int c : tr->nodes[cur].kids)
                if (tr->nodes[c].u == m[j].first && tr->nodes[c].v == m[j].second) found = c;
            if (found < 0) {
                TrieNode n;
                n.parent = cur;
                n.u = m[j].first; n.v = m[j].second;
                n.depth = tr->nodes[cur].depth + 1;
                int hi = std::max(n.u, n.v);
                n.nv = std::max(tr->nodes[cur].nv, hi + 1);
                found = (int)tr->nodes.size();
                tr->nodes.push_back(n);
                tr->nodes[cur].kids.push_back(found);
            }
            cur = found;
        }
        tr->nodes[cur].q = (int)q;
    }
    // flat tables (see comine.h): internal nodes get dense indices, the
    // root (node 0) being internal index 0 whenever it has children
    const int N = (int)tr->nodes.size();
    std::vector<int> iidx(N, -1);
    int n_int = 0;
    for (int n = 0; n < N; ++n)
        if (!tr->nodes[n].kids.empty()) iidx[n] = n_int++;
    if (n_int > 0xffff) return fail(MG_EUNSUPPORTED, "%d internal search nodes (limit 65535)", n_int);
    auto child_word = [&](int c) -> int32_t {
        const TrieNode &ch = tr->nodes[c];
        uint32_t w = ((uint32_t)(ch.q + 1) & 0x7fffu) << 16;
        if (iidx[c] >= 0) w |= (uint32_t)iidx[c] | 0x80000000u;
        return (int32_t)w;
    };
    tr->node_tab.assign(n_int > 0 ? n_int : 1, 0);
    tr->grp_tab.clear();
    tr->depth = 0;
    bool wide2 = false;   // an internal two-edge prefix on four vertices
    for (int n = 0; n < N; ++n) {
        const TrieNode &nd = tr->nodes[n];
        tr->depth = std::max(tr->depth, nd.depth);
        if (nd.depth == 2 && nd.nv > 3 && !nd.kids.empty()) wide2 = true;
        if (nd.kids.empty()) continue;
        // group the children by the list they scan
        std::map<std::pair<int, int>, std::vector<int>> groups;
        for (int c : nd.kids) {
            const TrieNode &ch = tr->nodes[c];
            int dir, anc;
            if (ch.u < nd.nv) { dir = mg::kDirOut; anc = ch.u; }
            else if (ch.v < nd.nv) { dir = mg::kDirIn; anc = ch.v; }
            else { dir = mg::kDirAll; anc = 0; }
            groups[{dir, anc}].push_back(c);
        }
        const int g0 = (int)tr->grp_tab.size() / 8;
        if (g0 + (int)groups.size() > (1 << 20))
            return fail(MG_EUNSUPPORTED, "too many child groups");
        // groups on a list of motif vertex 0 or 1 first: below the first
        // level the search finds their windows inside the root's windows
        std::vector<std::pair<std::pair<int, int>, std::vector<int>>> ordered;
        for (int cls = 0; cls < 2; ++cls)
            for (auto &kv : groups) {
                const bool near = kv.first.first != mg::kDirAll && kv.first.second < 2;
                if (near == (cls == 0)) ordered.push_back(kv);
            }
        int n_near = 0;
        for (auto &kv : ordered)
            n_near += (kv.first.first != mg::kDirAll && kv.first.second < 2) ? 1 : 0;
        for (auto &kv : ordered) {
            bool leaf_only = kv.first.first != mg::kDirAll;
            for (int c : kv.second) leaf_only = leaf_only && tr->nodes[c].kids.empty();
            // the anchor is the source (1) or destination (2) of the node's
            // own last edge: the window then starts where that edge's time
            // ends in the anchor's list, known per edge
            const int anc = kv.first.second;
            const int last_end = kv.first.first == mg::kDirAll ? 0
                                 : anc == nd.u ? 1 : anc == nd.v ? 2 : 0;
            int32_t rec[8] = {kv.first.first | (anc << 4) | (nd.nv << 8) |
                                  ((leaf_only ? 1 : 0) << 12) | (last_end << 13),
                              0, 0, 0, 0, 0, 0, 0};
            for (int c : kv.second) {
                const TrieNode &ch = tr->nodes[c];
                // out-group: the scanned endpoint is the destination; a bound
                // destination selects word 1+v, a new one word 7.  In- and
                // whole-list groups only ever reach new vertices (word 7).
                if (kv.first.first == mg::kDirOut && ch.v < nd.nv) rec[1 + ch.v] = child_word(c);
                else rec[7] = child_word(c);
            }
            tr->grp_tab.insert(tr->grp_tab.end(), rec, rec + 8);
        }
        // a leaf parent: every match below it is one more edge on a list of
        // a bound vertex
        bool leaf_parent = true;
        for (int c : nd.kids) {
            const TrieNode &ch = tr->nodes[c];
            leaf_parent = leaf_parent && ch.kids.empty() && (ch.u < nd.nv || ch.v < nd.nv);
        }
        tr->node_tab[iidx[n]] = (int32_t)((uint32_t)g0 | ((uint32_t)groups.size() << 20) |
                                          ((uint32_t)n_near << 25) |
                                          (leaf_parent ? mg::kLeafParent : 0u));
    }
    if (tr->grp_tab.empty()) tr->grp_tab.assign(8, 0);
    tr->root_q = tr->nodes[0].q;
    tr->kdepth = (tr->depth == 3 && wide2) ? 4 : tr->depth;

    // MG-Tree view: the root is the longest prefix shared by every motif;
    // below it a node exists where a prefix is a query or branches.
    int r = 0;
    while (tr->nodes[r].q < 0 && tr->nodes[r].kids.size() == 1) r = tr->nodes[r].kids[0];
    int mg_nodes = 0;
    std::vector<int> stack{r};
    while (!stack.empty()) {
        int n = stack.back();
        stack.pop_back();
        const TrieNode &nd = tr->nodes[n];
        if (n == r || nd.q >= 0 || nd.kids.size() != 1) mg_nodes++;
        for (int c : nd.kids) stack.push_back(c);
    }
    long total_edges = 0;
    for (auto &m : tr->distinct) total_edges += (long)m.size();
    mg_tree_info_t &in = tr->info;
    in.n_motifs = tr->n_motifs;
    in.n_distinct = (int32_t)tr->distinct.size();
    in.n_prefixes = N;
    in.n_nodes = mg_nodes;
    in.depth = tr->depth;
    in.root_edges = tr->nodes[r].depth;
    in.similarity = total_edges ? 1.0 - (double)N / (double)total_edges : 0.0;
    in.delta = tr->delta;
    in.n_deltas = (int32_t)tr->delta_slot.size();
    return MG_OK;
}

int make_tree(const std::vector<Motif> &canon, const std::vector<int64_t> &windows,
              mg_tree **out) {
    std::unique_ptr<mg_tree> tr(new (std::nothrow) mg_tree);
    if (!tr) return fail(MG_ENOMEM, "out of host memory");
    tr->n_motifs = (int32_t)canon.size();
    tr->deltas = windows;
    std::sort(tr->deltas.begin(), tr->deltas.end());
    tr->deltas.erase(std::unique(tr->deltas.begin(), tr->deltas.end()), tr->deltas.end());
    for (int64_t w : windows)
        tr->delta_slot.push_back(
            (int32_t)(std::lower_bound(tr->deltas.begin(), tr->deltas.end(), w) - tr->deltas.begin()));
    tr->delta = tr->deltas.back();
    std::map<Motif, int> ids;
    for (const Motif &m : canon) {
        auto it = ids.find(m);
        int q;
        if (it == ids.end()) {
            q = (int)tr->distinct.size();
            ids[m] = q;
            tr->distinct.push_back(m);
        } else {
            q = it->second;
        }
        tr->motif_q.push_back(q);
    }
    if ((int)tr->distinct.size() > MG_MAX_QUERIES)
        return fail(MG_EUNSUPPORTED, "%d distinct motifs (limit %d)", (int)tr->distinct.size(),
                    MG_MAX_QUERIES);
    if (tr->distinct.size() * tr->deltas.size() > (size_t)MG_MAX_QUERIES)
        return fail(MG_EUNSUPPORTED, "%d distinct motifs x %d windows exceed %d counters",
                    (int)tr->distinct.size(), (int)tr->deltas.size(), MG_MAX_QUERIES);
    int rc = build_tree(tr.get());
    if (rc) return rc;
    *out = tr.release();
    return MG_OK;
}

// Caller-visible counts of one tree from its counters (n_d slots per
// distinct motif; slot j holds the matches whose span fits window j but not
// window j - 1): out[i * n_motifs + m] for the caller's window i and motif m.
void map_counts(const mg_tree *tr, const uint64_t *slots, uint64_t *out) {
    const size_t nd = tr->deltas.size();
    for (size_t i = 0; i < tr->delta_slot.size(); ++i)
        for (int32_t m = 0; m < tr->n_motifs; ++m) {
            const uint64_t *c = slots + (size_t)tr->motif_q[m] * nd;
            uint64_t sum = 0;
            for (int32_t j = 0; j <= tr->delta_slot[i]; ++j) sum += c[j];
            out[i * (size_t)tr->n_motifs + m] = sum;
        }
}

size_t n_slots(const mg_tree *tr) { return tr->distinct.size() * tr->deltas.size(); }

int upload_tree(mg_tree *tr, int device, hipStream_t st) {
    if (tr->device == device && tr->d_node.ptr) return MG_OK;
    dev_free(tr->d_node);
    dev_free(tr->d_grp);
    int rc = dev_alloc(tr->d_node, tr->node_tab.size() * 4, (void *)st);
    if (rc) return rc;
    rc = dev_alloc(tr->d_grp, tr->grp_tab.size() * 4, (void *)st);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(tr->d_node.ptr, tr->node_tab.data(), tr->node_tab.size() * 4,
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(tr->d_grp.ptr, tr->grp_tab.data(), tr->grp_tab.size() * 4,
                           hipMemcpyHostToDevice, st));
    tr->device = device;
    return MG_OK;
}

// One launch of the co-mining kernel over a tree; counts land in d_counts.
template <typename TT>
int learned_search(const mg_graph *g, mg_tree *tr, const mg_model *model,
                   const mg::KParams<TT> &base, int blocks, uint32_t stride, hipStream_t st);

template <typename TT>
mg::DevGraph<TT> dev_graph(const mg_graph *g);
mg::DevTree dev_tree(const mg_tree *tr);
template <typename TT>
TT delta_sat(int64_t delta);

// Kernel parameters of a count over every root of g (the caller may then
// restrict the roots).
template <typename TT>
void fill_params(mg::KParams<TT> &p, const mg_graph *g, const mg_tree *tr, const mg_count_opts &o,
                 unsigned long long *d_queues, unsigned long long *d_counts,
                 unsigned long long *d_stats, unsigned long long *d_cost) {
    p.g = dev_graph<TT>(g);
    p.tree = dev_tree(tr);
    p.delta_sat = delta_sat<TT>(tr->delta);
    for (size_t i = 0; i + 1 < tr->deltas.size(); ++i) p.dlo[i] = delta_sat<TT>(tr->deltas[i]);
    p.roots = nullptr;
    p.n_roots = (uint32_t)g->E;
    p.chunk = (uint32_t)(o.chunk > 0 ? o.chunk : 64);
    p.n_queues = (uint32_t)(o.queues > 0 ? o.queues : mg::kQueues);
    p.leaf_scan = o.leaf_scan < 0 ? 0u : (o.leaf_scan == 0 ? mg::kLeafScanDefault
                                                           : (uint32_t)o.leaf_scan);
    p.queues = d_queues;
    p.counts = d_counts;
    p.stats = d_stats;
    p.root_cost = d_cost;
    p.stop = o.stop;
    p.max_chunks = (uint32_t)o.max_chunks;
}

// Epochs (paper, section 4.5): launch after launch, each ending once
// o.epoch_idle percent of its waves are idle; the root-level candidates the
// busy waves had not reached yet come back as contexts, which the next launch
// spreads over all of its waves.  The last of max_epochs launches runs to the
// end.  Counts accumulate in p.counts; p.queues is cleared before each launch.
constexpr uint64_t kCtxCap = 1u << 20;   // contexts one epoch can hand on (64 MB)

template <typename TT>
int epoch_search(mg::KParams<TT> p, const mg_count_opts &o, hipStream_t st) {
    const int max_epochs = o.max_epochs > 0 ? o.max_epochs : 16;
    struct Free {
        DevBuf *b;
        ~Free() { dev_free(b[0]); dev_free(b[1]); dev_free(b[2]); }
    };
    DevBuf all[3];
    Free fr{all};
    for (int i = 0; i < 2; ++i) {
        int rc = dev_alloc(all[i], sizeof(mg::EpochCtx) * kCtxCap, (void *)st);
        if (rc) return rc;
    }
    int rc = dev_alloc(all[2], 16, (void *)st);
    if (rc) return rc;
    p.ctx_count = (unsigned long long *)all[2].ptr;
    p.idle = (uint32_t *)((char *)all[2].ptr + 8);
    p.ctx_cap = kCtxCap;
    p.idle_pct = (uint32_t)o.epoch_idle;
    for (int ep = 0; ep < max_epochs; ++ep) {
        const bool last = ep + 1 == max_epochs;
        p.ctx_out = last ? nullptr : (mg::EpochCtx *)all[ep & 1].ptr;
        HIP_TRY(hipMemsetAsync(all[2].ptr, 0, 16, st));
        if (ep > 0) HIP_TRY(hipMemsetAsync(p.queues, 0, kQueueBytes, st));
        // (the first launch with neither contexts in nor out is the plain search)
        hipError_t e = mg::launch_comine<TT>(p, o.blocks, st);
        if (e != hipSuccess)
            return fail(MG_EDEVICE, "co-mining launch failed: %s", hipGetErrorString(e));
        unsigned long long n = 0;
        if (p.ctx_out) {
            HIP_TRY(hipMemcpyAsync(&n, p.ctx_count, sizeof n, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        if (o.epoch_contexts) o.epoch_contexts[ep] = (int64_t)n;
        if (n == 0) {
            for (int k = ep + 1; o.epoch_contexts && k < max_epochs; ++k) o.epoch_contexts[k] = 0;
            break;
        }
        p.ctx_in = (const mg::EpochCtx *)all[ep & 1].ptr;
        p.n_ctx_in = (uint32_t)n;
    }
    return MG_OK;
}

template <typename TT>
int launch_tree(const mg_graph *g, mg_tree *tr, const uint32_t *d_roots, uint32_t n_roots,
                unsigned long long *d_queues, unsigned long long *d_counts,
                unsigned long long *d_stats, unsigned long long *d_cost,
                unsigned long long *d_clock, const mg_count_opts &o, hipStream_t st, float *ms) {
    mg::KParams<TT> p{};
    fill_params<TT>(p, g, tr, o, d_queues, d_counts, d_stats, d_cost);
    p.roots = d_roots;
    p.n_roots = n_roots;
    p.wave_clock = d_clock;
    p.n_wave_clock = d_clock ? (uint32_t)std::min<int64_t>(o.wave_clock_len / 2, 0x7fffffff) : 0u;

    if (o.cursor && o.cursor->started) {
        // resume: every root queue starts where the last call stopped
        std::vector<unsigned long long> q(mg::kQueueWords, 0ull);
        for (int i = 0; i < mg::kQueues; ++i) q[(size_t)i * mg::kQueueStride] = o.cursor->head[i];
        HIP_TRY(hipMemcpyAsync(d_queues, q.data(), kQueueBytes, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));   // q is released on return
    }
    const uint32_t n_counts = (uint32_t)mg::counter_slots(p.tree);
    if (!(o.cursor && o.cursor->started) && d_counts == d_queues + mg::kQueueWords) {
        // queue heads and counters side by side: one fill kernel clears both
        // (cheaper on the host than two memsets, and no memset node when the
        // caller captures the stream)
        HIP_TRY(mg::launch_fill_u64(d_queues, (uint32_t)mg::kQueueWords + n_counts, 0ull, st));
    } else {
        if (!(o.cursor && o.cursor->started)) HIP_TRY(hipMemsetAsync(d_queues, 0, kQueueBytes, st));
        HIP_TRY(hipMemsetAsync(d_counts, 0, sizeof(unsigned long long) * n_counts, st));
    }
    if (d_stats) HIP_TRY(hipMemsetAsync(d_stats, 0, sizeof(unsigned long long) * mg::kStats, st));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms) {
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        HIP_TRY(hipEventRecord(e0, st));
    }
    if (n_roots > 0 && o.sched == MG_SCHED_LEARNED) {
        int rc = learned_search<TT>(g, tr, o.model, p, o.blocks,
                                    o.sample > 0 ? (uint32_t)o.sample : kSampleDefault, st);
        if (rc) return rc;
    } else if (n_roots > 0 && o.epoch_idle > 0) {
        int rc = epoch_search<TT>(p, o, st);
        if (rc) return rc;
    } else if (n_roots > 0) {
        hipError_t e = mg::launch_comine<TT>(p, o.blocks, st);
        if (e != hipSuccess)
            return fail(MG_EDEVICE, "co-mining launch failed: %s", hipGetErrorString(e));
    }
    if (ms) {
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return MG_OK;
}

}  // namespace

int mgh::chain_trees(mg_tree *tr) {
    if (!tr->singles.empty()) return MG_OK;
    for (const Motif &m : tr->distinct) {
        mg_tree *one = nullptr;
        int rc = make_tree({m}, tr->deltas, &one);
        if (rc) return rc;
        tr->singles.emplace_back(one);
    }
    return MG_OK;
}


// ---------------------------------------------------------------- cost model
static_assert(mg::kParams == MG_MODEL_PARAMS, "parameter layout");
static_assert(mg::kFeat == MG_NFEATURES, "feature count");

struct mg_model {
    int device = 0;
    DevBuf params, adam_m, adam_v;
    ~mg_model() {
        dev_free(params);
        dev_free(adam_m);
        dev_free(adam_v);
    }
};

namespace {

uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
double uniform01(uint64_t &s) { return ((splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
double normal(uint64_t &s) {   // Box-Muller
    const double u = uniform01(s), v = uniform01(s);
    return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
}

template <typename TT>
mg::DevGraph<TT> dev_graph(const mg_graph *g) {
    mg::DevGraph<TT> d{};
    d.gsrc = (const int32_t *)g->gsrc.ptr;
    d.gdst = (const int32_t *)g->gdst.ptr;
    d.gt = (const TT *)g->gt.ptr;
    d.gx = (const uint4 *)g->gx.ptr;
    d.out_eid = (const uint32_t *)g->out_eid.ptr;
    d.in_eid = (const uint32_t *)g->in_eid.ptr;
    d.out_off = (const uint32_t *)g->out_off.ptr;
    d.out_adj = (const mg::Entry<TT> *)g->out_adj.ptr;
    d.in_off = (const uint32_t *)g->in_off.ptr;
    d.in_adj = (const mg::Entry<TT> *)g->in_adj.ptr;
    d.n_edges = (uint32_t)g->E;
    return d;
}

mg::DevTree dev_tree(const mg_tree *tr) {
    mg::DevTree t{};
    t.inode = (const uint32_t *)tr->d_node.ptr;
    t.grp = (const uint4 *)tr->d_grp.ptr;
    t.n_q = (int32_t)tr->distinct.size();
    t.root_q = tr->root_q;
    t.depth = tr->depth;
    t.kdepth = tr->kdepth;
    t.n_d = (int32_t)tr->deltas.size();
    return t;
}

template <typename TT>
TT delta_sat(int64_t delta) {
    return sizeof(TT) == 4 ? (TT)std::min<uint64_t>((uint64_t)delta, 0xffffffffull)
                           : (TT)(uint64_t)delta;
}

// Learned schedule + search on stream st: predicted segment costs -> items ->
// item-driven search kernel.
template <typename TT>
int learned_search(const mg_graph *g, mg_tree *tr, const mg_model *model,
                   const mg::KParams<TT> &base, int blocks, uint32_t stride, hipStream_t st) {
    const uint32_t E = (uint32_t)g->E;
    const uint32_t n_seg = (E + mg::kSeg - 1) / mg::kSeg;
    DevBuf d;
    const size_t off_total = 4 * (size_t)n_seg;
    const size_t off_work = off_total + 16;
    const size_t off_nitems = off_work + 4 * (size_t)mg::kBinWords;
    const size_t off_items = (off_nitems + 16 + 15) & ~(size_t)15;
    const size_t off_feat = (off_items + 8 * (size_t)std::max<uint32_t>(E, 1) + 15) & ~(size_t)15;
    const size_t off_skip = off_feat + 32 * (size_t)std::max<uint32_t>((E + stride - 1) / stride, 1);
    int rc = dev_alloc(d, off_skip + n_seg + 16, (void *)st);
    if (rc) return rc;
    struct G { DevBuf *b; ~G() { dev_free(*b); } } guard{&d};
    char *p0 = (char *)d.ptr;
    float *seg_cost = (float *)p0, *total = (float *)(p0 + off_total);
    uint32_t *work = (uint32_t *)(p0 + off_work), *n_items = (uint32_t *)(p0 + off_nitems);
    uint2 *items = (uint2 *)(p0 + off_items);
    uint4 *feat = (uint4 *)(p0 + off_feat);
    uint8_t *skip = (uint8_t *)(p0 + off_skip);
    hipError_t e = mg::launch_fill_f32_zero(total, 1, st);
    if (e == hipSuccess)
        e = mg::launch_predict_roots<TT>(base.g, base.tree, base.delta_sat,
                                         (const float *)model->params.ptr, stride, seg_cost, total,
                                         feat, st);
    // segments predicted at more than 8x the mean go first (one root per item
    // above ~1/(4 * resident waves) of the total, heavy roots in up to
    // kRootParts parts); the rest keep time order
    if (e == hipSuccess)
        e = mg::launch_bin(seg_cost, n_seg, E, total, 8.0f, 1.0f / 32768.0f, kRootParts, work,
                           items, std::max<uint32_t>(E, 1), n_items, skip, st);
    if (e != hipSuccess) return fail(MG_EDEVICE, "learned schedule failed: %s", hipGetErrorString(e));
    mg::KParams<TT> p = base;
    p.items = items;
    p.n_items = n_items;
    p.skip = skip;
    p.roots = nullptr;
    p.chunk = mg::kSeg;      // one chunk is one segment
    e = mg::launch_comine<TT>(p, blocks, st);
    if (e != hipSuccess) return fail(MG_EDEVICE, "co-mining launch failed: %s", hipGetErrorString(e));
    // the buffer is released after the caller synchronises the stream
    HIP_TRY(hipStreamSynchronize(st));
    return MG_OK;
}

}  // namespace

// ---------------------------------------------------------------- batches
struct mg_batch {
    std::vector<const mg_graph *> graphs;
    std::vector<mg_tree *> trees;
    int time_bytes = 4;
    int device = 0;
    int depth = 1;
    uint32_t n_q_max = 1;
    uint32_t total_q = 0;         // device counters (distinct motifs per job)
    int32_t total_motifs = 0;     // caller-visible counts
    int64_t total_roots = 0;
    std::vector<uint32_t> count_off;
    mg_batch_opts opts{};
    int32_t item_roots = 0;
    float tuned_ms = 0.f;
    float predict_ms = 0.f;       // features + MLP + ordering at plan creation
    bool learned = false;
    std::vector<mg::BatchItem> items;
    DevBuf d_jobs, d_items, d_work;   // d_work: cursor (16 B) + counters
    uint64_t *h_counts = nullptr;     // pinned
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
    ~mg_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (h_counts) (void)hipHostFree(h_counts);
        dev_free(d_jobs);
        dev_free(d_items);
        dev_free(d_work);
    }
};

namespace {

template <typename TT>
int upload_jobs(mg_batch *b, hipStream_t st) {
    std::vector<mg::BatchJob<TT>> jobs(b->graphs.size());
    mg_count_opts o;
    mg_count_opts_init(&o);
    for (size_t j = 0; j < jobs.size(); ++j) {
        mg::BatchJob<TT> &J = jobs[j];
        std::memset(&J, 0, sizeof J);
        fill_params<TT>(J.p, b->graphs[j], b->trees[j], o, nullptr, nullptr, nullptr, nullptr);
        J.count_off = b->count_off[j];
    }
    int rc = dev_alloc(b->d_jobs, sizeof(mg::BatchJob<TT>) * jobs.size(), (void *)st);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(b->d_jobs.ptr, jobs.data(), sizeof(mg::BatchJob<TT>) * jobs.size(),
                           hipMemcpyHostToDevice, st));
    return MG_OK;
}

// Work items: root ranges of item_roots roots, largest graphs first.
int make_items(mg_batch *b, int32_t item_roots, hipStream_t st) {
    std::vector<uint32_t> order(b->graphs.size());
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        return b->graphs[x]->E > b->graphs[y]->E;
    });
    b->items.clear();
    for (uint32_t j : order) {
        const uint32_t E = (uint32_t)b->graphs[j]->E;
        for (uint32_t r = 0; r < E; r += (uint32_t)item_roots)
            b->items.push_back({j, r, std::min<uint32_t>(E, r + (uint32_t)item_roots), 0u});
    }
    dev_free(b->d_items);
    int rc = dev_alloc(b->d_items, sizeof(mg::BatchItem) * std::max<size_t>(1, b->items.size()),
                       (void *)st);
    if (rc) return rc;
    if (!b->items.empty())
        HIP_TRY(hipMemcpyAsync(b->d_items.ptr, b->items.data(),
                               sizeof(mg::BatchItem) * b->items.size(), hipMemcpyHostToDevice, st));
    b->item_roots = item_roots;
    return MG_OK;
}

// Predicted segment costs of one job (learned_items orders the items).
template <typename TT>
int predict_job_segments(const mg_graph *g, mg_tree *tr, const mg_model *m, float *d_seg,
                         float *d_total, uint4 *d_feat, hipStream_t st) {
    hipError_t e = mg::launch_fill_f32_zero(d_total, 1, st);
    if (e == hipSuccess)
        e = mg::launch_predict_roots<TT>(dev_graph<TT>(g), dev_tree(tr), delta_sat<TT>(tr->delta),
                                         (const float *)m->params.ptr, kSampleDefault, d_seg,
                                         d_total, d_feat, st);
    if (e != hipSuccess) return fail(MG_EDEVICE, "cost prediction failed: %s", hipGetErrorString(e));
    return MG_OK;
}

int learned_items(mg_batch *b, const mg_model *m, hipStream_t st) {
    const auto t0 = std::chrono::steady_clock::now();
    struct Seg { float cost; uint32_t job, first, end; };
    std::vector<Seg> segs;
    double total = 0.0;
    for (size_t j = 0; j < b->graphs.size(); ++j) {
        const mg_graph *g = b->graphs[j];
        const uint32_t E = (uint32_t)g->E, n_seg = (E + mg::kSeg - 1) / mg::kSeg;
        if (!n_seg) continue;
        DevBuf d;
        const size_t off_feat = (4 * (size_t)n_seg + 16 + 15) & ~(size_t)15;
        int rc = dev_alloc(d, off_feat + 32 * (size_t)((E + kSampleDefault - 1) / kSampleDefault),
                           (void *)st);
        if (rc) return rc;
        struct G { DevBuf *b; ~G() { dev_free(*b); } } guard{&d};
        float *d_seg = (float *)d.ptr, *d_total = d_seg + n_seg;
        uint4 *d_feat = (uint4 *)((char *)d.ptr + off_feat);
        rc = b->time_bytes == 4
                 ? predict_job_segments<uint32_t>(g, b->trees[j], m, d_seg, d_total, d_feat, st)
                 : predict_job_segments<uint64_t>(g, b->trees[j], m, d_seg, d_total, d_feat, st);
        if (rc) return rc;
        std::vector<float> h(n_seg);
        HIP_TRY(hipMemcpyAsync(h.data(), d_seg, 4 * (size_t)n_seg, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (uint32_t sg = 0; sg < n_seg; ++sg) {
            const uint32_t r0 = sg * mg::kSeg;
            segs.push_back({h[sg], (uint32_t)j, r0, std::min<uint32_t>(E, r0 + mg::kSeg)});
            total += h[sg];
        }
    }
    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // heavy segments (above 8x the mean) first, heaviest first; one root per
    // item above a quarter of one wave's fair share (~32 resident waves per
    // CU), a root still above that in up to kRootParts parts of its
    // first-level candidates; then every other segment in job order (largest
    // graph first) and time order, as the plain schedule runs them
    const double split = total / (4.0 * 32.0 * std::max(ncu, 1));
    const double heavy = segs.empty() ? 0.0 : 8.0 * total / (double)segs.size();
    std::vector<std::pair<float, mg::BatchItem>> it;
    std::vector<uint8_t> is_heavy(segs.size(), 0);
    for (size_t i = 0; i < segs.size(); ++i) {
        const Seg &sg = segs[i];
        if (!(total > 0.0 && sg.cost > heavy)) continue;
        is_heavy[i] = 1;
        const uint32_t nr = sg.end - sg.first;
        if (sg.cost > split && nr > 1) {
            const double c = (double)sg.cost / nr;
            const uint32_t k =
                (uint32_t)std::min<double>(kRootParts, std::max(1.0, std::ceil(c / split)));
            for (uint32_t r = sg.first; r < sg.end; ++r)
                for (uint32_t q = 0; q < k; ++q)
                    it.push_back({(float)(c / k), {sg.job, r, r + 1,
                                                   k > 1 ? (mg::kItemSplit | (q << 15) | k) : 0u}});
        } else {
            it.push_back({sg.cost, {sg.job, sg.first, sg.end, 0u}});
        }
    }
    std::stable_sort(it.begin(), it.end(),
                     [](const auto &x, const auto &y) { return x.first > y.first; });
    std::vector<uint32_t> order(b->graphs.size());
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        return b->graphs[x]->E > b->graphs[y]->E;
    });
    std::vector<size_t> seg0(b->graphs.size() + 1, 0);   // first segment of each job
    for (const Seg &sg : segs) seg0[sg.job + 1]++;
    for (size_t j = 0; j < b->graphs.size(); ++j) seg0[j + 1] += seg0[j];
    for (uint32_t j : order)
        for (size_t i = seg0[j]; i < seg0[j + 1]; ++i)
            if (!is_heavy[i]) it.push_back({0.f, {j, segs[i].first, segs[i].end, 0u}});
    b->items.clear();
    for (auto &x : it) b->items.push_back(x.second);
    dev_free(b->d_items);
    int rc = dev_alloc(b->d_items, sizeof(mg::BatchItem) * std::max<size_t>(1, b->items.size()),
                       (void *)st);
    if (rc) return rc;
    if (!b->items.empty())
        HIP_TRY(hipMemcpyAsync(b->d_items.ptr, b->items.data(),
                               sizeof(mg::BatchItem) * b->items.size(), hipMemcpyHostToDevice, st));
    b->item_roots = mg::kSeg;
    b->learned = true;
    HIP_TRY(hipStreamSynchronize(st));
    b->predict_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return MG_OK;
}

// Enqueue one step on st: zero, search, copy the counters to pinned memory.
template <typename TT>
int enqueue_step(mg_batch *b, hipStream_t st) {
    mg::BatchParams<TT> bp{};
    bp.jobs = (const mg::BatchJob<TT> *)b->d_jobs.ptr;
    bp.items = (const mg::BatchItem *)b->d_items.ptr;
    bp.n_items = (uint32_t)b->items.size();
    bp.n_q_max = b->n_q_max;
    bp.cursor = (unsigned long long *)b->d_work.ptr;
    bp.counts = (unsigned long long *)((char *)b->d_work.ptr + 16);
    bp.multi = 0;
    for (const mg_tree *tr : b->trees) bp.multi |= tr->deltas.size() > 1 ? 1u : 0u;
    hipError_t e = mg::launch_fill_u64(bp.cursor, 2 + b->total_q, 0ull, st);
    if (e != hipSuccess) return fail(MG_EDEVICE, "fill launch failed: %s", hipGetErrorString(e));
    if (bp.n_items) {
        e = mg::launch_batch<TT>(bp, b->depth, b->opts.blocks, st);
        if (e != hipSuccess) return fail(MG_EDEVICE, "batch launch failed: %s", hipGetErrorString(e));
    }
    HIP_TRY(hipMemcpyAsync(b->h_counts, bp.counts, 8 * (size_t)std::max<uint32_t>(1, b->total_q),
                           hipMemcpyDeviceToHost, st));
    return MG_OK;
}

int run_step(mg_batch *b, hipStream_t st, float *ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms) {
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        HIP_TRY(hipEventRecord(e0, st));
    }
    int rc;
    if (b->exec) {
        HIP_TRY(hipGraphLaunch(b->exec, st));
        rc = MG_OK;
    } else {
        rc = b->time_bytes == 4 ? enqueue_step<uint32_t>(b, st) : enqueue_step<uint64_t>(b, st);
    }
    if (rc) return rc;
    if (ms) {
        HIP_TRY(hipEventRecord(e1, st));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    HIP_TRY(hipStreamSynchronize(st));
    return MG_OK;
}

int capture(mg_batch *b) {
    if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = b->time_bytes == 4 ? enqueue_step<uint32_t>(b, b->cap_stream)
                                : enqueue_step<uint64_t>(b, b->cap_stream);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &gr);
    if (rc) { if (gr) (void)hipGraphDestroy(gr); return rc; }
    if (e != hipSuccess) return fail(MG_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    b->graph = gr;
    HIP_TRY(hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0));
    return MG_OK;
}

}  // namespace

// ---------------------------------------------------------------- C ABI
extern "C" {

int mg_set_allocator(mg_alloc_fn alloc, mg_release_fn release, void *ctx) {
    if ((alloc == nullptr) != (release == nullptr))
        return fail(MG_EINVAL, "alloc and release must both be set or both be NULL");
    g_alloc = alloc;
    g_release = release;
    g_alloc_ctx = ctx;
    return MG_OK;
}

const char *mg_last_error(void) { return g_err.c_str(); }

int mg_model_create(uint64_t seed, mg_model **out) {
    try {
        if (!out) return fail(MG_EINVAL, "out is NULL");
        std::unique_ptr<mg_model> m(new (std::nothrow) mg_model);
        if (!m) return fail(MG_ENOMEM, "out of host memory");
        HIP_TRY(hipGetDevice(&m->device));
        std::vector<float> w(mg::kParams, 0.f);
        uint64_t s = seed;
        auto he = [&](int off, int fan_in, int rows, int cols) {
            const double sd = std::sqrt(2.0 / fan_in);
            for (int i = 0; i < rows * cols; ++i) w[off + i] = (float)(normal(s) * sd);
        };
        he(mg::kOffW1, mg::kFeat, mg::kFeat, mg::kHid);    // rows 16..31 stay zero
        he(mg::kOffW2, mg::kHid, mg::kHid, mg::kHid);
        he(mg::kOffW3, mg::kHid, mg::kHid, mg::kHid);
        he(mg::kOffW4, mg::kHid, 1, mg::kHid);
        for (DevBuf *b : {&m->params, &m->adam_m, &m->adam_v}) {
            int rc = dev_alloc(*b, sizeof(float) * mg::kParams, nullptr);
            if (rc) return rc;
        }
        HIP_TRY(hipMemcpy(m->params.ptr, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemset(m->adam_m.ptr, 0, sizeof(float) * mg::kParams));
        HIP_TRY(hipMemset(m->adam_v.ptr, 0, sizeof(float) * mg::kParams));
        *out = m.release();
        return MG_OK;
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

int mg_model_get_weights(const mg_model *m, float *w) {
    if (!m || !w) return fail(MG_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpy(w, m->params.ptr, sizeof(float) * mg::kParams, hipMemcpyDeviceToHost));
    return MG_OK;
}

int mg_model_set_weights(mg_model *m, const float *w) {
    if (!m || !w) return fail(MG_EINVAL, "NULL argument");
    for (int i = 0; i < mg::kParams; ++i)
        if (!std::isfinite(w[i])) return fail(MG_EINVAL, "weight %d is not finite", i);
    for (int r = mg::kFeat; r < 32; ++r)
        for (int c = 0; c < mg::kHid; ++c)
            if (w[mg::kOffW1 + r * mg::kHid + c] != 0.f)
                return fail(MG_EINVAL, "W1 rows %d..31 must be zero", mg::kFeat);
    HIP_TRY(hipMemcpy(m->params.ptr, w, sizeof(float) * mg::kParams, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(m->adam_m.ptr, 0, sizeof(float) * mg::kParams));
    HIP_TRY(hipMemset(m->adam_v.ptr, 0, sizeof(float) * mg::kParams));
    return MG_OK;
}

int mg_model_get_moments(const mg_model *m, float *m1, float *m2) {
    if (!m) return fail(MG_EINVAL, "NULL model");
    if (m1) HIP_TRY(hipMemcpy(m1, m->adam_m.ptr, sizeof(float) * mg::kParams, hipMemcpyDeviceToHost));
    if (m2) HIP_TRY(hipMemcpy(m2, m->adam_v.ptr, sizeof(float) * mg::kParams, hipMemcpyDeviceToHost));
    return MG_OK;
}

void mg_model_destroy(mg_model *m) { delete m; }

int mg_root_features(const mg_graph *g, const mg_tree *tr_c, const int64_t *roots, int64_t n,
                     float *feats) {
    try {
        if (!g || !tr_c || !feats || n < 0) return fail(MG_EINVAL, "bad argument");
        if (g->host_only) return fail(MG_EINVAL, "the graph is on the host only (MG_HOST_ONLY)");
        if (!roots && n != g->E) return fail(MG_EINVAL, "without roots, n must be n_edges");
        mg_tree *tr = const_cast<mg_tree *>(tr_c);
        int rc = upload_tree(tr, g->device, nullptr);
        if (rc) return rc;
        std::vector<uint32_t> r;
        if (roots) {
            r.resize(n);
            for (int64_t i = 0; i < n; ++i) {
                if (roots[i] < 0 || roots[i] >= g->E) return fail(MG_EINVAL, "root out of range");
                r[i] = (uint32_t)roots[i];
            }
        }
        DevBuf d_r, d_f;
        struct G { DevBuf *a, *b; ~G() { dev_free(*a); dev_free(*b); } } guard{&d_r, &d_f};
        if (roots) {
            rc = dev_alloc(d_r, 4 * std::max<size_t>(1, r.size()), nullptr);
            if (rc) return rc;
            if (n) HIP_TRY(hipMemcpy(d_r.ptr, r.data(), 4 * r.size(), hipMemcpyHostToDevice));
        }
        rc = dev_alloc(d_f, sizeof(float) * mg::kFeat * std::max<int64_t>(1, n), nullptr);
        if (rc) return rc;
        hipError_t e = g->time_bytes == 4
            ? mg::launch_features<uint32_t>(dev_graph<uint32_t>(g), dev_tree(tr),
                                            delta_sat<uint32_t>(tr->delta),
                                            (const uint32_t *)d_r.ptr, (uint32_t)n,
                                            (float *)d_f.ptr, nullptr)
            : mg::launch_features<uint64_t>(dev_graph<uint64_t>(g), dev_tree(tr),
                                            delta_sat<uint64_t>(tr->delta),
                                            (const uint32_t *)d_r.ptr, (uint32_t)n,
                                            (float *)d_f.ptr, nullptr);
        if (e != hipSuccess) return fail(MG_EDEVICE, "features launch failed: %s", hipGetErrorString(e));
        if (n) HIP_TRY(hipMemcpy(feats, d_f.ptr, sizeof(float) * mg::kFeat * n, hipMemcpyDeviceToHost));
        return MG_OK;
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

int mg_model_predict(const mg_model *m, const float *feats, int64_t n, float *out) {
    try {
        if (!m || !feats || !out || n < 0 || n >= (int64_t)1 << 31)
            return fail(MG_EINVAL, "bad argument");
        DevBuf d_f, d_o;
        struct G { DevBuf *a, *b; ~G() { dev_free(*a); dev_free(*b); } } guard{&d_f, &d_o};
        int rc = dev_alloc(d_f, sizeof(float) * mg::kFeat * std::max<int64_t>(1, n), nullptr);
        if (rc) return rc;
        rc = dev_alloc(d_o, sizeof(float) * std::max<int64_t>(1, n), nullptr);
        if (rc) return rc;
        if (n) HIP_TRY(hipMemcpy(d_f.ptr, feats, sizeof(float) * mg::kFeat * n, hipMemcpyHostToDevice));
        hipError_t e = mg::launch_predict_feats((const float *)m->params.ptr, (const float *)d_f.ptr,
                                                (uint32_t)n, (float *)d_o.ptr, nullptr);
        if (e != hipSuccess) return fail(MG_EDEVICE, "predict launch failed: %s", hipGetErrorString(e));
        if (n) HIP_TRY(hipMemcpy(out, d_o.ptr, sizeof(float) * n, hipMemcpyDeviceToHost));
        return MG_OK;
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

int mg_model_train(mg_model *m, const float *feats, const float *labels, int64_t n,
                   int32_t epochs, float lr, uint64_t seed, float *loss) {
    try {
        if (!m || !feats || !labels || n < 0 || n >= (int64_t)1 << 31 || epochs < 0 ||
            !(lr > 0.f))
            return fail(MG_EINVAL, "bad argument");
        std::vector<uint32_t> perm(n);
        std::iota(perm.begin(), perm.end(), 0u);
        uint64_t s = seed;
        for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[splitmix(s) % (uint64_t)(i + 1)]);
        DevBuf d_f, d_y, d_p, d_l;
        struct G {
            DevBuf *a, *b, *c, *d;
            ~G() { dev_free(*a); dev_free(*b); dev_free(*c); dev_free(*d); }
        } guard{&d_f, &d_y, &d_p, &d_l};
        int rc = dev_alloc(d_f, sizeof(float) * mg::kFeat * std::max<int64_t>(1, n), nullptr);
        if (!rc) rc = dev_alloc(d_y, sizeof(float) * std::max<int64_t>(1, n), nullptr);
        if (!rc) rc = dev_alloc(d_p, sizeof(uint32_t) * std::max<int64_t>(1, n), nullptr);
        if (!rc) rc = dev_alloc(d_l, sizeof(float) * std::max(1, epochs), nullptr);
        if (rc) return rc;
        if (n) {
            HIP_TRY(hipMemcpy(d_f.ptr, feats, sizeof(float) * mg::kFeat * n, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(d_y.ptr, labels, sizeof(float) * n, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(d_p.ptr, perm.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice));
        }
        hipError_t e = mg::launch_train((float *)m->params.ptr, (float *)m->adam_m.ptr,
                                        (float *)m->adam_v.ptr, (const float *)d_f.ptr,
                                        (const float *)d_y.ptr, (uint32_t)n,
                                        (const uint32_t *)d_p.ptr, (uint32_t)epochs, lr,
                                        (float *)d_l.ptr, nullptr);
        if (e != hipSuccess) return fail(MG_EDEVICE, "train launch failed: %s", hipGetErrorString(e));
        HIP_TRY(hipDeviceSynchronize());
        if (loss && epochs)
            HIP_TRY(hipMemcpy(loss, d_l.ptr, sizeof(float) * epochs, hipMemcpyDeviceToHost));
        return MG_OK;
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

void mg_batch_opts_init(mg_batch_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->use_graph = 1;
}

int mg_batch_create(const mg_graph *const *graphs, const mg_tree *const *trees, int32_t n,
                    const mg_batch_opts *opts, mg_batch **out) {
    try {
        if (!out || !graphs || !trees || n < 1) return fail(MG_EINVAL, "empty batch");
        mg_batch_opts o;
        mg_batch_opts_init(&o);
        if (opts) o = *opts;
        if (o.item_roots < 0 || o.item_roots % 64 || o.item_roots > (1 << 24))
            return fail(MG_EINVAL, "item_roots must be a multiple of 64 in [0, 2^24]");
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        if (o.model && o.model->device != dev) return fail(MG_EINVAL, "model on another device");
        std::unique_ptr<mg_batch> b(new (std::nothrow) mg_batch);
        if (!b) return fail(MG_ENOMEM, "out of host memory");
        b->opts = o;
        b->device = dev;
        hipStream_t st = (hipStream_t)o.stream;
        for (int32_t j = 0; j < n; ++j) {
            if (!graphs[j] || !trees[j]) return fail(MG_EINVAL, "job %d has a NULL handle", j);
            if (graphs[j]->host_only) return fail(MG_EINVAL, "job %d: graph on the host only", j);
            if (graphs[j]->device != dev) return fail(MG_EINVAL, "job %d: graph on another device", j);
            if (j && graphs[j]->time_bytes != graphs[0]->time_bytes)
                return fail(MG_EUNSUPPORTED, "graphs of one batch must share the time width");
            mg_tree *tr = const_cast<mg_tree *>(trees[j]);
            int rc = upload_tree(tr, dev, st);
            if (rc) return rc;
            b->graphs.push_back(graphs[j]);
            b->trees.push_back(tr);
            b->count_off.push_back(b->total_q);
            b->total_q += (uint32_t)n_slots(tr);
            b->total_motifs += tr->n_motifs * (int32_t)tr->delta_slot.size();
            b->total_roots += graphs[j]->E;
            b->n_q_max = std::max<uint32_t>(b->n_q_max, (uint32_t)n_slots(tr));
            b->depth = std::max(b->depth, tr->kdepth);
        }
        b->time_bytes = graphs[0]->time_bytes;
        int rc = b->time_bytes == 4 ? upload_jobs<uint32_t>(b.get(), st)
                                    : upload_jobs<uint64_t>(b.get(), st);
        if (rc) return rc;
        rc = dev_alloc(b->d_work, 16 + 8 * (size_t)std::max<uint32_t>(1, b->total_q), (void *)st);
        if (rc) return rc;
        HIP_TRY(hipHostMalloc((void **)&b->h_counts, 8 * (size_t)std::max<uint32_t>(1, b->total_q),
                              hipHostMallocDefault));
        if (o.model) {
            rc = learned_items(b.get(), o.model, st);
            if (rc) return rc;
        } else if (o.item_roots > 0) {
            rc = make_items(b.get(), o.item_roots, st);
            if (rc) return rc;
        } else {
            // autotune the item size: one timed step per candidate, from small
            // to large, stopping at the first one that is clearly slower
            float best = -1.f;
            int32_t best_ir = 64;
            bool warm = false;
            for (int32_t ir : {64, 128, 256, 512, 1024}) {
                rc = make_items(b.get(), ir, st);
                if (rc) return rc;
                if (!warm) {
                    rc = run_step(b.get(), st, nullptr);
                    if (rc) return rc;
                    warm = true;
                }
                float ms = 0.f;
                rc = run_step(b.get(), st, &ms);
                if (rc) return rc;
                if (best < 0.f || ms < best) { best = ms; best_ir = ir; }
                else if (ms > 1.05f * best) break;
            }
            b->tuned_ms = best;
            if (b->item_roots != best_ir) {
                rc = make_items(b.get(), best_ir, st);
                if (rc) return rc;
            }
        }
        HIP_TRY(hipStreamSynchronize(st));
        *out = b.release();
        return MG_OK;
    } catch (const std::bad_alloc &) {
        return fail(MG_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

int mg_batch_count(mg_batch *b, uint64_t *counts, float *elapsed_ms) {
    try {
        if (!b || !counts) return fail(MG_EINVAL, "NULL argument");
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        if (dev != b->device) return fail(MG_EINVAL, "batch lives on device %d", b->device);
        hipStream_t st = (hipStream_t)b->opts.stream;
        int rc;
        if (b->opts.use_graph && !b->exec) {
            rc = capture(b);
            if (rc) return rc;
        }
        rc = run_step(b, st, elapsed_ms);
        if (rc) return rc;
        size_t k = 0;
        for (size_t j = 0; j < b->trees.size(); ++j) {
            const mg_tree *tr = b->trees[j];
            map_counts(tr, b->h_counts + b->count_off[j], counts + k);
            k += (size_t)tr->n_motifs * tr->delta_slot.size();
        }
        return MG_OK;
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

int mg_batch_info(const mg_batch *b, mg_batch_info_t *out) {
    if (!b || !out) return fail(MG_EINVAL, "NULL argument");
    out->n_jobs = (int32_t)b->trees.size();
    out->total_motifs = b->total_motifs;
    out->total_roots = b->total_roots;
    out->n_items = (int64_t)b->items.size();
    out->item_roots = b->item_roots;
    out->blocks = b->opts.blocks;
    out->graph_captured = b->exec ? 1 : 0;
    out->depth = b->depth;
    out->tuned_ms = b->tuned_ms;
    out->learned = b->learned ? 1 : 0;
    out->predict_ms = b->predict_ms;
    return MG_OK;
}

void mg_batch_destroy(mg_batch *b) { delete b; }

int mg_count_batch(const mg_graph *const *graphs, const mg_tree *const *trees, int32_t n,
                   const mg_batch_opts *opts, uint64_t *counts) {
    if (!counts) return fail(MG_EINVAL, "NULL counts");
    mg_batch_opts o;
    mg_batch_opts_init(&o);
    if (opts) o = *opts;
    o.use_graph = 0;
    if (o.item_roots == 0) o.item_roots = 64;
    mg_batch *b = nullptr;
    int rc = mg_batch_create(graphs, trees, n, &o, &b);
    if (rc) return rc;
    rc = mg_batch_count(b, counts, nullptr);
    mg_batch_destroy(b);
    return rc;
}

int mg_graph_create(const int32_t *src, const int32_t *dst, const int64_t *t, int64_t n_edges,
                    int32_t n_nodes, uint32_t flags, void *stream, mg_graph **out) {
    try {
        if (!out) return fail(MG_EINVAL, "out is NULL");
        if (n_edges < 0 || n_nodes < 0) return fail(MG_EINVAL, "negative size");
        if (n_edges > 0 && (!src || !dst || !t)) return fail(MG_EINVAL, "NULL edge array");
        if (n_edges >= (int64_t)1 << 31)
            return fail(MG_EUNSUPPORTED, "n_edges %lld >= 2^31", (long long)n_edges);
        if (n_nodes >= INT32_MAX) return fail(MG_EUNSUPPORTED, "n_nodes too large");
        if (flags & ~(MG_SORTED_BY_T | MG_DEVICE_INPUT | MG_HOST_ONLY))
            return fail(MG_EINVAL, "unknown flags");
        if ((flags & MG_DEVICE_INPUT) && (flags & MG_HOST_ONLY))
            return fail(MG_EINVAL, "MG_DEVICE_INPUT and MG_HOST_ONLY exclude each other");
        std::vector<int32_t> hs, hd;
        std::vector<int64_t> ht;
        if ((flags & MG_DEVICE_INPUT) && n_edges > 0) {
            // device arrays: brought to the host, where the adjacency is built
            hs.resize(n_edges);
            hd.resize(n_edges);
            ht.resize(n_edges);
            hipStream_t st = (hipStream_t)stream;
            HIP_TRY(hipMemcpyAsync(hs.data(), src, 4 * (size_t)n_edges, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(hd.data(), dst, 4 * (size_t)n_edges, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(ht.data(), t, 8 * (size_t)n_edges, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            src = hs.data();
            dst = hd.data();
            t = ht.data();
        }
        for (int64_t i = 0; i < n_edges; ++i)
            if (src[i] < 0 || src[i] >= n_nodes || dst[i] < 0 || dst[i] >= n_nodes)
                return fail(MG_EINVAL, "edge %lld has a vertex outside [0, %d)", (long long)i,
                            n_nodes);
        bool sorted = true;
        for (int64_t i = 1; i < n_edges; ++i)
            if (t[i] < t[i - 1]) { sorted = false; break; }
        if ((flags & MG_SORTED_BY_T) && !sorted)
            return fail(MG_EINVAL, "MG_SORTED_BY_T given but t is not non-decreasing");
        std::unique_ptr<mg_graph> g(new (std::nothrow) mg_graph);
        if (!g) return fail(MG_ENOMEM, "out of host memory");
        g->E = n_edges;
        g->V = n_nodes;
        std::vector<int32_t> s(n_edges), d(n_edges);
        std::vector<int64_t> tt(n_edges);
        if (sorted) {
            std::copy(src, src + n_edges, s.begin());
            std::copy(dst, dst + n_edges, d.begin());
            std::copy(t, t + n_edges, tt.begin());
        } else {
            std::vector<int64_t> ord(n_edges);
            std::iota(ord.begin(), ord.end(), 0);
            std::stable_sort(ord.begin(), ord.end(),
                             [&](int64_t a, int64_t b) { return t[a] < t[b]; });
            for (int64_t i = 0; i < n_edges; ++i) {
                s[i] = src[ord[i]]; d[i] = dst[ord[i]]; tt[i] = t[ord[i]];
            }
            g->input_index = std::move(ord);
        }
        for (int64_t i = 0; i < n_edges; ++i) g->self_loops += (s[i] == d[i]);
        g->t_min = n_edges ? tt[0] : 0;
        g->t_max = n_edges ? tt[n_edges - 1] : 0;
        if (n_edges && g->t_max - g->t_min < 0) return fail(MG_EUNSUPPORTED, "time span >= 2^63");
        const uint64_t span = n_edges ? (uint64_t)(g->t_max - g->t_min) : 0;
        g->time_bytes = span < 0xffffffffull ? 4 : 8;
        if (flags & MG_HOST_ONLY) {
            g->host_only = true;
            g->device = -1;
            build_host(g.get(), std::move(s), std::move(d), std::move(tt));
            *out = g.release();
            return MG_OK;
        }
        HIP_TRY(hipGetDevice(&g->device));
        hipStream_t st = (hipStream_t)stream;
        int rc = g->time_bytes == 4 ? upload_graph<uint32_t>(g.get(), s, d, tt, st)
                                    : upload_graph<uint64_t>(g.get(), s, d, tt, st);
        if (rc) return rc;
        *out = g.release();
        return MG_OK;
    } catch (const std::bad_alloc &) {
        return fail(MG_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

int mg_graph_info(const mg_graph *g, mg_graph_info_t *out) {
    if (!g || !out) return fail(MG_EINVAL, "NULL argument");
    out->n_edges = g->E;
    out->n_nodes = g->V;
    out->self_loops = g->self_loops;
    out->t_min = g->t_min;
    out->t_max = g->t_max;
    out->time_bytes = g->time_bytes;
    out->device_bytes = g->device_bytes;
    return MG_OK;
}

void mg_graph_destroy(mg_graph *g) { delete g; }

int mg_tree_create(const int32_t *motif_uv, const int32_t *motif_k, int32_t n_motifs,
                   int64_t delta, mg_tree **out) {
    return mg_tree_create_multi(motif_uv, motif_k, n_motifs, &delta, 1, out);
}

int mg_tree_create_multi(const int32_t *motif_uv, const int32_t *motif_k, int32_t n_motifs,
                         const int64_t *deltas, int32_t n_deltas, mg_tree **out) {
    try {
        if (!out) return fail(MG_EINVAL, "out is NULL");
        if (n_motifs < 1 || !motif_uv || !motif_k) return fail(MG_EINVAL, "no motifs");
        if (!deltas || n_deltas < 1) return fail(MG_EINVAL, "no window");
        if (n_deltas > MG_MAX_DELTAS)
            return fail(MG_EUNSUPPORTED, "%d windows (limit %d)", n_deltas, MG_MAX_DELTAS);
        for (int32_t i = 0; i < n_deltas; ++i)
            if (deltas[i] < 0) return fail(MG_EINVAL, "delta < 0");
        std::vector<Motif> canon(n_motifs);
        int64_t off = 0;
        for (int32_t i = 0; i < n_motifs; ++i) {
            const int k = motif_k[i];
            if (k < 1) return fail(MG_EINVAL, "motif %d has %d edges", i, k);
            if (k > kKMax)
                return fail(MG_EUNSUPPORTED, "motif %d has %d edges (limit %d)", i, k, kKMax);
            int rc = canonical(motif_uv + 2 * off, k, canon[i]);
            if (rc) return rc;
            off += k;
        }
        return make_tree(canon, std::vector<int64_t>(deltas, deltas + n_deltas), out);
    } catch (const std::bad_alloc &) {
        return fail(MG_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

int mg_tree_info(const mg_tree *tr, mg_tree_info_t *out) {
    if (!tr || !out) return fail(MG_EINVAL, "NULL argument");
    *out = tr->info;
    return MG_OK;
}

void mg_tree_destroy(mg_tree *tr) { delete tr; }

int mg_enumerate(const mg_graph *g, const mg_tree *tr_c, void *stream, mg_match *out,
                 int64_t capacity, int64_t *n_matches) {
    try {
        if (!g || !tr_c || !n_matches || capacity < 0) return fail(MG_EINVAL, "bad argument");
        if (g->host_only) return fail(MG_EINVAL, "the graph is on the host only (MG_HOST_ONLY)");
        mg_tree *tr = const_cast<mg_tree *>(tr_c);
        if (tr->deltas.size() != 1)
            return fail(MG_EUNSUPPORTED, "enumeration takes a tree with one window");
        static_assert(sizeof(mg_match) == 4 * (1 + mg::kKMax), "record layout");
        // the count sizes the output
        mg_count_opts o;
        mg_count_opts_init(&o);
        o.stream = stream;
        std::vector<uint64_t> cnt(tr->n_motifs);
        int rc = mg_count(g, tr, &o, cnt.data());
        if (rc) return rc;
        std::vector<int32_t> first(tr->distinct.size(), -1);   // first caller motif per distinct one
        for (int32_t m = 0; m < tr->n_motifs; ++m)
            if (first[tr->motif_q[m]] < 0) first[tr->motif_q[m]] = m;
        uint64_t total = 0;
        for (size_t q = 0; q < first.size(); ++q) total += cnt[first[q]];
        if (!out || (uint64_t)capacity < total) {
            *n_matches = (int64_t)total;
            return MG_OK;
        }
        hipStream_t st = (hipStream_t)stream;
        DevBuf d_work, d_rec;
        struct G { DevBuf *a, *b; ~G() { dev_free(*a); dev_free(*b); } } guard{&d_work, &d_rec};
        const size_t cnt_off = kQueueBytes, cur_off = cnt_off + 8 * n_slots(tr);
        rc = dev_alloc(d_work, cur_off + 8, (void *)st);
        if (!rc) rc = dev_alloc(d_rec, sizeof(mg_match) * std::max<uint64_t>(total, 1), (void *)st);
        if (rc) return rc;
        HIP_TRY(hipMemsetAsync(d_work.ptr, 0, cur_off + 8, st));
        unsigned long long *w = (unsigned long long *)d_work.ptr;
        o.leaf_scan = -1;   // every match goes through the candidate expansion
        hipError_t e = hipSuccess;
        if (g->E > 0) {
            if (g->time_bytes == 4) {
                mg::KParams<uint32_t> p{};
                fill_params<uint32_t>(p, g, tr, o, w, w + cnt_off / 8, nullptr, nullptr);
                p.enum_out = (int32_t *)d_rec.ptr;
                p.enum_cursor = w + cur_off / 8;
                p.enum_cap = total;
                e = mg::launch_comine<uint32_t>(p, 0, st);
            } else {
                mg::KParams<uint64_t> p{};
                fill_params<uint64_t>(p, g, tr, o, w, w + cnt_off / 8, nullptr, nullptr);
                p.enum_out = (int32_t *)d_rec.ptr;
                p.enum_cursor = w + cur_off / 8;
                p.enum_cap = total;
                e = mg::launch_comine<uint64_t>(p, 0, st);
            }
        }
        if (e != hipSuccess) return fail(MG_EDEVICE, "enumeration launch failed: %s", hipGetErrorString(e));
        uint64_t written = 0;
        HIP_TRY(hipMemcpyAsync(&written, w + cur_off / 8, 8, hipMemcpyDeviceToHost, st));
        if (total) HIP_TRY(hipMemcpyAsync(out, d_rec.ptr, sizeof(mg_match) * total, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (written != total)
            return fail(MG_EINTERNAL, "enumeration wrote %llu matches, the count is %llu",
                        (unsigned long long)written, (unsigned long long)total);
        // motifs in the caller's numbering (a duplicate's first occurrence),
        // edges in the caller's input order
        for (uint64_t i = 0; i < total; ++i) {
            mg_match &m = out[i];
            m.motif = first[m.motif];
            if (!g->input_index.empty())
                for (int j = 0; j < mg::kKMax && m.edges[j] >= 0; ++j)
                    m.edges[j] = (int32_t)g->input_index[m.edges[j]];
        }
        *n_matches = (int64_t)total;
        return MG_OK;
    } catch (const std::bad_alloc &) {
        return fail(MG_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

int mg_count_noalloc(const mg_graph *g, const mg_tree *tr, const mg_count_opts *opts,
                     uint64_t *counts) {
    try {
        if (!g || !tr || !counts) return fail(MG_EINVAL, "NULL argument");
        if (g->host_only) return fail(MG_EINVAL, "the graph is on the host only (MG_HOST_ONLY)");
        mg_count_opts o;
        mg_count_opts_init(&o);
        if (opts) o = *opts;
        if (o.mode != MG_MODE_COMINE || o.sched != MG_SCHED_PLAIN || o.roots || o.root_cost ||
            o.elapsed_ms || o.cursor || o.wave_clock || o.epoch_idle)
            return fail(MG_EINVAL, "mg_count_noalloc takes co-mining with the plain schedule over "
                                   "every root; roots, root_cost, elapsed_ms, cursor and epochs "
                                   "need memory");
        if (o.chunk < 0 || (o.chunk % 64) != 0 || o.chunk > (1 << 16))
            return fail(MG_EINVAL, "chunk must be a multiple of 64 in [0, 65536]");
        if (o.queues < 0 || o.queues > mg::kQueues)
            return fail(MG_EINVAL, "queues must be in [0, %d]", mg::kQueues);
        if (o.max_chunks < 0 || o.max_chunks > 0xffffffffll)
            return fail(MG_EINVAL, "max_chunks must be in [0, 2^32)");
        const size_t nq = n_slots(tr);
        if (nq > (size_t)mg::kMaxQueries)
            return fail(MG_EUNSUPPORTED, "%zu counters; the static array holds %d", nq,
                        mg::kMaxQueries);
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        if (dev != g->device) return fail(MG_EINVAL, "graph lives on device %d, current is %d",
                                          g->device, dev);
        if (tr->device != dev || !tr->d_node.ptr)
            return fail(MG_EINVAL, "the tree has no device tables on device %d yet (count it "
                                   "with mg_count there once)", dev);
        unsigned long long *scr = nullptr;
        HIP_TRY(mg::static_scratch(&scr));
        unsigned long long *d_queues = scr;
        unsigned long long *d_counts = scr + mg::kQueueWords;
        unsigned long long *d_stats = o.stats ? d_counts + mg::kMaxQueries : nullptr;
        hipStream_t st = (hipStream_t)o.stream;
        // queue heads, claim counter, counters and statistics start at zero
        // (a fill kernel, no memset node if the caller captures the stream)
        HIP_TRY(mg::launch_fill_u64(scr, (uint32_t)mg::kStaticWords, 0ull, st));
        const uint32_t n_roots = (uint32_t)g->E;
        if (n_roots > 0) {
            hipError_t e;
            if (g->time_bytes == 4) {
                mg::KParams<uint32_t> p{};
                fill_params<uint32_t>(p, g, tr, o, d_queues, d_counts, d_stats, nullptr);
                e = mg::launch_comine<uint32_t>(p, o.blocks, st);
            } else {
                mg::KParams<uint64_t> p{};
                fill_params<uint64_t>(p, g, tr, o, d_queues, d_counts, d_stats, nullptr);
                e = mg::launch_comine<uint64_t>(p, o.blocks, st);
            }
            if (e != hipSuccess)
                return fail(MG_EDEVICE, "co-mining launch failed: %s", hipGetErrorString(e));
        }
        uint64_t h[mg::kMaxQueries];
        uint64_t hs[mg::kStats];
        if (nq) HIP_TRY(hipMemcpyAsync(h, d_counts, 8 * nq, hipMemcpyDeviceToHost, st));
        if (d_stats) HIP_TRY(hipMemcpyAsync(hs, d_stats, sizeof hs, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        map_counts(tr, h, counts);
        if (o.stats) std::copy(hs, hs + mg::kStats, o.stats);
        return MG_OK;
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

void mg_cursor_init(mg_cursor *c) {
    if (c) std::memset(c, 0, sizeof *c);
}

void mg_count_opts_init(mg_count_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->mode = MG_MODE_COMINE;
}

int mg_count(const mg_graph *g, const mg_tree *tr_c, const mg_count_opts *opts,
             uint64_t *counts) {
    try {
        if (!g || !tr_c || !counts) return fail(MG_EINVAL, "NULL argument");
        if (g->host_only) return fail(MG_EINVAL, "the graph is on the host only (MG_HOST_ONLY)");
        mg_tree *tr = const_cast<mg_tree *>(tr_c);   // device copy is a cache
        mg_count_opts o;
        mg_count_opts_init(&o);
        if (opts) o = *opts;
        if (o.mode == MG_MODE_AUTO) {
            mg_advice a{};
            int rc = mg_comine_advice(g, tr, MG_PLATFORM_GPU, &a);
            if (rc) return rc;
            o.mode = a.co_mine ? MG_MODE_COMINE : MG_MODE_PER_MOTIF;
        }
        if (o.mode != MG_MODE_COMINE && o.mode != MG_MODE_PER_MOTIF)
            return fail(MG_EINVAL, "unknown mode %d", o.mode);
        if (o.chunk < 0 || (o.chunk % 64) != 0 || o.chunk > (1 << 16))
            return fail(MG_EINVAL, "chunk must be a multiple of 64 in [0, 65536]");
        if (o.roots && o.n_roots < 0) return fail(MG_EINVAL, "n_roots < 0");
        if (o.queues < 0 || o.queues > mg::kQueues)
            return fail(MG_EINVAL, "queues must be in [0, %d]", mg::kQueues);
        if (o.stats && o.root_cost)
            return fail(MG_EINVAL, "stats and root_cost are exclusive");
        if (o.wave_clock && (o.mode != MG_MODE_COMINE || o.wave_clock_len < 0))
            return fail(MG_EINVAL, "wave_clock needs co-mining and a length >= 0");
        if (o.sched != MG_SCHED_PLAIN && o.sched != MG_SCHED_LEARNED)
            return fail(MG_EINVAL, "unknown schedule %d", o.sched);
        if (o.max_chunks < 0 || o.max_chunks > 0xffffffffll)
            return fail(MG_EINVAL, "max_chunks must be in [0, 2^32)");
        const bool stoppable = o.stop || o.max_chunks || o.cursor;
        if (stoppable && (o.mode != MG_MODE_COMINE || o.sched != MG_SCHED_PLAIN))
            return fail(MG_EINVAL, "stop, max_chunks and cursor need co-mining with the plain schedule");
        if (o.epoch_idle < 0 || o.epoch_idle > 100 || o.max_epochs < 0)
            return fail(MG_EINVAL, "epoch_idle must be in [0, 100] and max_epochs >= 0");
        if (o.epoch_idle && (o.mode != MG_MODE_COMINE || o.sched != MG_SCHED_PLAIN || stoppable ||
                             o.stats || o.root_cost || o.wave_clock))
            return fail(MG_EINVAL, "epochs need co-mining with the plain schedule, without stop, "
                                   "max_chunks, cursor, stats, root_cost or wave_clock");
        if (o.cursor && o.cursor->started) {
            const int32_t ch = o.chunk > 0 ? o.chunk : 64, nq = o.queues > 0 ? o.queues : mg::kQueues;
            const int64_t nr = o.roots ? o.n_roots : g->E;
            if (o.cursor->n_roots != nr || o.cursor->chunk != ch || o.cursor->queues != nq)
                return fail(MG_EINVAL, "the cursor belongs to a count with other roots, chunk or queues");
            for (int q = 0; q < nq; ++q) {
                const uint32_t len = mg::queue_end((uint32_t)nr, (uint32_t)nq, (uint32_t)q) -
                                     mg::queue_begin((uint32_t)nr, (uint32_t)nq, (uint32_t)q);
                if (o.cursor->head[q] > len) return fail(MG_EINVAL, "cursor head %d past its queue", q);
            }
        }
        if (o.sched == MG_SCHED_LEARNED) {
            if (!o.model) return fail(MG_EINVAL, "the learned schedule needs a model");
            if (o.roots) return fail(MG_EINVAL, "the learned schedule searches every root");
            if (o.sample < 0 || o.sample > mg::kSeg || (o.sample & (o.sample - 1)))
                return fail(MG_EINVAL, "sample must be 0 or a power of two up to %d", mg::kSeg);
            if (o.model->device != g->device) return fail(MG_EINVAL, "model on another device");
        }
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        if (dev != g->device) return fail(MG_EINVAL, "graph lives on device %d, current is %d",
                                          g->device, dev);
        hipStream_t st = (hipStream_t)o.stream;

        // roots
        DevBuf d_roots;
        uint32_t n_roots = (uint32_t)g->E;
        if (o.roots) {
            std::vector<uint32_t> r(o.n_roots);
            for (int64_t i = 0; i < o.n_roots; ++i) {
                if (o.roots[i] < 0 || o.roots[i] >= g->E)
                    return fail(MG_EINVAL, "root %lld outside [0, %lld)", (long long)o.roots[i],
                                (long long)g->E);
                r[i] = (uint32_t)o.roots[i];
            }
            n_roots = (uint32_t)o.n_roots;
            int rc = dev_alloc(d_roots, sizeof(uint32_t) * r.size(), (void *)st);
            if (rc) return rc;
            if (!r.empty())
                HIP_TRY(hipMemcpyAsync(d_roots.ptr, r.data(), sizeof(uint32_t) * r.size(),
                                       hipMemcpyHostToDevice, st));
        }
        struct Guard { DevBuf *b; ~Guard() { dev_free(*b); } } gr{&d_roots};

        // trees to run: the whole group, or one chain per distinct motif
        std::vector<mg_tree *> runs;
        if (o.mode == MG_MODE_COMINE) {
            runs.push_back(tr);
        } else {
            int rc = chain_trees(tr);
            if (rc) return rc;
            for (auto &u : tr->singles) runs.push_back(u.get());
        }
        size_t maxq = 1;
        for (mg_tree *t : runs) maxq = std::max(maxq, n_slots(t));
        static_assert(mg::kStats == MG_NSTATS, "stats layout");
        DevBuf d_work;
        const size_t stats_off = kQueueBytes + 8 * maxq;
        int rc = dev_alloc(d_work, stats_off + 8 * mg::kStats, (void *)st);
        if (rc) return rc;
        struct Guard2 { DevBuf *b; ~Guard2() { dev_free(*b); } } gw{&d_work};
        unsigned long long *d_queues = (unsigned long long *)d_work.ptr;
        unsigned long long *d_counts = (unsigned long long *)((char *)d_work.ptr + kQueueBytes);
        unsigned long long *d_stats =
            o.stats ? (unsigned long long *)((char *)d_work.ptr + stats_off) : nullptr;
        std::vector<uint64_t> stats_sum(mg::kStats, 0);
        DevBuf d_cost;
        if (o.root_cost) {
            rc = dev_alloc(d_cost, sizeof(uint64_t) * (size_t)g->E, (void *)st);
            if (rc) return rc;
            if (g->E) HIP_TRY(hipMemsetAsync(d_cost.ptr, 0, sizeof(uint64_t) * (size_t)g->E, st));
        }
        struct Guard3 { DevBuf *b; ~Guard3() { dev_free(*b); } } gc{&d_cost};
        DevBuf d_clock;
        if (o.wave_clock && o.wave_clock_len >= 2) {
            rc = dev_alloc(d_clock, 8 * (size_t)o.wave_clock_len, (void *)st);
            if (rc) return rc;
            HIP_TRY(hipMemsetAsync(d_clock.ptr, 0, 8 * (size_t)o.wave_clock_len, st));
        }
        struct Guard4 { DevBuf *b; ~Guard4() { dev_free(*b); } } gk{&d_clock};

        std::vector<uint64_t> qcount(n_slots(tr), 0);
        float total_ms = 0.f;
        mg_cursor cur{};
        for (size_t ri = 0; ri < runs.size(); ++ri) {
            mg_tree *t = runs[ri];
            rc = upload_tree(t, dev, st);
            if (rc) return rc;
            float ms = 0.f;
            rc = g->time_bytes == 4
                     ? launch_tree<uint32_t>(g, t, (const uint32_t *)d_roots.ptr, n_roots,
                                             d_queues, d_counts, d_stats,
                                             (unsigned long long *)d_cost.ptr,
                                             (unsigned long long *)d_clock.ptr, o, st,
                                             o.elapsed_ms ? &ms : nullptr)
                     : launch_tree<uint64_t>(g, t, (const uint32_t *)d_roots.ptr, n_roots,
                                             d_queues, d_counts, d_stats,
                                             (unsigned long long *)d_cost.ptr,
                                             (unsigned long long *)d_clock.ptr, o, st,
                                             o.elapsed_ms ? &ms : nullptr);
            if (rc) return rc;
            total_ms += ms;
            if (o.cursor) {
                std::vector<unsigned long long> q(mg::kQueueWords);
                HIP_TRY(hipMemcpyAsync(q.data(), d_queues, kQueueBytes, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                const uint32_t nq = o.queues > 0 ? (uint32_t)o.queues : (uint32_t)mg::kQueues;
                cur.n_roots = n_roots;
                cur.chunk = o.chunk > 0 ? o.chunk : 64;
                cur.queues = (int32_t)nq;
                cur.started = 1;
                cur.done = 1;
                for (uint32_t i = 0; i < (uint32_t)mg::kQueues; ++i) {
                    const uint64_t len = i < nq ? mg::queue_end(n_roots, nq, i) -
                                                      mg::queue_begin(n_roots, nq, i)
                                                : 0;
                    cur.head[i] = std::min<uint64_t>(q[(size_t)i * mg::kQueueStride], len);
                    if (cur.head[i] < len) cur.done = 0;
                }
            }
            std::vector<uint64_t> h(n_slots(t));
            HIP_TRY(hipMemcpyAsync(h.data(), d_counts, 8 * h.size(), hipMemcpyDeviceToHost, st));
            std::vector<uint64_t> hs(mg::kStats, 0);
            if (d_stats)
                HIP_TRY(hipMemcpyAsync(hs.data(), d_stats, 8 * hs.size(), hipMemcpyDeviceToHost,
                                       st));
            HIP_TRY(hipStreamSynchronize(st));
            for (int i = 0; i < mg::kStats; ++i) stats_sum[i] += hs[i];
            if (o.mode == MG_MODE_COMINE) qcount = h;
            else std::copy(h.begin(), h.end(), qcount.begin() + ri * h.size());
        }
        map_counts(tr, qcount.data(), counts);
        if (o.root_cost && g->E) {
            HIP_TRY(hipMemcpyAsync(o.root_cost, d_cost.ptr, sizeof(uint64_t) * (size_t)g->E,
                                   hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        if (d_clock.ptr) {
            HIP_TRY(hipMemcpyAsync(o.wave_clock, d_clock.ptr, 8 * (size_t)o.wave_clock_len,
                                   hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        if (o.elapsed_ms) *o.elapsed_ms = total_ms;
        if (o.stats) std::copy(stats_sum.begin(), stats_sum.end(), o.stats);
        if (o.cursor) *o.cursor = cur;
        return MG_OK;
    } catch (const std::bad_alloc &) {
        return fail(MG_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}


}  // extern "C"

// ---------------------------------------------------------------- autotuner
namespace {

// Identity of a (graph, tree, device) for the tuning cache: the graph's and
// tree's statistics and the device's name and compute-unit count.
std::string tune_key(const mg_graph *g, const mg_tree *tr) {
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, g->device) != hipSuccess) prop.name[0] = 0;
    uint64_t h = 1469598103934665603ull;   // FNV-1a over the relabelled motifs
    auto mix = [&](uint64_t x) { h = (h ^ x) * 1099511628211ull; };
    for (const Motif &m : tr->distinct) {
        mix(m.size());
        for (auto &e : m) mix((uint64_t)e.first << 8 | (uint64_t)e.second);
    }
    for (int64_t w : tr->deltas) mix((uint64_t)w);
    char buf[512];
    snprintf(buf, sizeof buf, "%s/%d|E=%lld|V=%d|span=%lld|tb=%d|loops=%lld|motifs=%zu|depth=%d|"
             "prefixes=%d|trees=%016llx", prop.name, prop.multiProcessorCount, (long long)g->E,
             g->V, (long long)(g->t_max - g->t_min), g->time_bytes, (long long)g->self_loops,
             tr->distinct.size(), tr->depth, tr->info.n_prefixes, (unsigned long long)h);
    std::string k(buf);
    for (char &c : k)
        if (c == '"' || c == '\\' || c == '\n') c = '_';
    return k;
}

// One cache line: {"key": "...", "blocks": b, "chunk": c, "queues": q, "leaf_scan": l, "ms": t}
bool cache_lookup(const char *path, const std::string &key, mg_tune_result *r) {
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    const std::string want = "{\"key\": \"" + key + "\"";
    while (fgets(line, sizeof line, f)) {
        if (strncmp(line, want.c_str(), want.size()) != 0 || line[want.size()] != ',') continue;
        mg_tune_result t{};
        if (sscanf(line + want.size(),
                   ", \"blocks\": %d, \"chunk\": %d, \"queues\": %d, \"leaf_scan\": %d, "
                   "\"ms\": %f, \"default_ms\": %f",
                   &t.blocks, &t.chunk, &t.queues, &t.leaf_scan, &t.ms, &t.default_ms) == 6) {
            *r = t;
            found = true;   // the last entry for a key wins
        }
    }
    fclose(f);
    return found;
}

int cache_store(const char *path, const std::string &key, const mg_tune_result &r) {
    FILE *f = fopen(path, "a");
    if (!f) return fail(MG_EINVAL, "cannot append to the tuning cache %s", path);
    fprintf(f,
            "{\"key\": \"%s\", \"blocks\": %d, \"chunk\": %d, \"queues\": %d, \"leaf_scan\": %d, "
            "\"ms\": %.4f, \"default_ms\": %.4f}\n",
            key.c_str(), r.blocks, r.chunk, r.queues, r.leaf_scan, r.ms, r.default_ms);
    fclose(f);
    return MG_OK;
}

}  // namespace

extern "C" {

int mg_tune(const mg_graph *g, const mg_tree *tr, const char *cache_path, void *stream,
            mg_tune_result *out) {
    try {
        if (!g || !tr || !out) return fail(MG_EINVAL, "NULL argument");
        if (g->host_only) return fail(MG_EINVAL, "the graph is on the host only (MG_HOST_ONLY)");
        const std::string key = tune_key(g, tr);
        mg_tune_result best{};
        if (cache_path && cache_lookup(cache_path, key, &best)) {
            best.from_cache = 1;
            *out = best;
            return MG_OK;
        }
        int dev = 0, ncu = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        // median of three timed counts after one untimed one
        int32_t trials = 0;
        auto time_of = [&](const mg_tune_result &c, float *ms) -> int {
            mg_count_opts o;
            mg_count_opts_init(&o);
            o.blocks = c.blocks;
            o.chunk = c.chunk;
            o.queues = c.queues;
            o.leaf_scan = c.leaf_scan;
            o.stream = stream;
            std::vector<uint64_t> cnt((size_t)tr->n_motifs * tr->delta_slot.size());
            int rc = mg_count(g, tr, &o, cnt.data());
            if (rc) return rc;
            float t[3];
            o.elapsed_ms = nullptr;
            for (float &x : t) {
                o.elapsed_ms = &x;
                rc = mg_count(g, tr, &o, cnt.data());
                if (rc) return rc;
            }
            std::sort(t, t + 3);
            *ms = t[1];
            ++trials;
            return MG_OK;
        };
        // coordinate descent from the defaults, one setting at a time
        mg_tune_result cur{};
        cur.blocks = 0;
        cur.chunk = 64;
        cur.queues = mg::kQueues;
        cur.leaf_scan = (int32_t)mg::kLeafScanDefault;
        int rc = time_of(cur, &cur.ms);
        if (rc) return rc;
        cur.default_ms = cur.ms;
        const std::vector<int32_t> chunks = {64, 128, 256}, queues = {8, 4, 2, 1},
                                   scans = {64, 128, 256, 512, 1024},
                                   blocks = {0, ncu * 4, ncu * 6};
        for (int sweep = 0; sweep < 2; ++sweep) {
            bool moved = false;
            for (int dim = 0; dim < 4; ++dim) {
                const std::vector<int32_t> &vals =
                    dim == 0 ? scans : dim == 1 ? chunks : dim == 2 ? queues : blocks;
                for (int32_t v : vals) {
                    mg_tune_result c = cur;
                    int32_t &field = dim == 0 ? c.leaf_scan : dim == 1 ? c.chunk
                                     : dim == 2 ? c.queues : c.blocks;
                    if (field == v) continue;
                    field = v;
                    rc = time_of(c, &c.ms);
                    if (rc) return rc;
                    // a new setting must win by more than the noise of one timing
                    if (c.ms < 0.98f * cur.ms) {
                        cur = c;
                        moved = true;
                    }
                }
            }
            if (!moved) break;
        }
        cur.trials = trials;
        if (cache_path) {
            rc = cache_store(cache_path, key, cur);
            if (rc) return rc;
        }
        *out = cur;
        return MG_OK;
    } catch (const std::bad_alloc &) {
        return fail(MG_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

}  // extern "C"
