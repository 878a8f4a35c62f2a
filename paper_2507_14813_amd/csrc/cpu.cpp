// CPU co-mining backend (the paper's second backend, section 5.1.1 "CPU
// code-generation", and its nested-loop listing in the appendix): the search
// of a motif group is emitted as C++ with one loop nest per level of the
// group's prefix trie -- every trie node a block, every child group a loop
// over one time window, the graph vertices bound so far as local variables
// -- compiled by the host compiler, loaded, and run over the root edges on
// every host core.  Without a compiler the same search is interpreted from
// the trie tables.  Also here: the paper's heuristic for whether co-mining
// pays (section 7, "Heuristic for Co-Mining").
#include <dlfcn.h>
#include <spawn.h>
#include <sys/wait.h>
#include <unistd.h>

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <thread>
#include <vector>

#include "../../include/mayura.h"
#include "handles.h"

extern char **environ;

namespace mgh {
namespace {

// The compiled search: roots [r0, r1) of the graph, counters n_d per
// distinct motif (slot j: the matches whose span fits window j but not
// window j - 1; dlo: the windows below the largest).
struct GenGraph {
    const int32_t *src, *dst;
    const int64_t *t;
    const uint32_t *oo, *io;
    const int32_t *ov, *iv;
    const int64_t *ot, *it;
    int64_t n;
};
using GenFn = void (*)(const GenGraph *g, int64_t r0, int64_t r1, int64_t delta, const int64_t *dlo,
                       int32_t nd, uint64_t *cnt);

// ---------------------------------------------------------------- host copy
void build_lists(HostAdj &h, int32_t V) {
    const int64_t E = (int64_t)h.src.size();
    h.out_off.assign(V + 1, 0);
    h.in_off.assign(V + 1, 0);
    for (int64_t i = 0; i < E; ++i)
        if (h.src[i] != h.dst[i]) { h.out_off[h.src[i] + 1]++; h.in_off[h.dst[i] + 1]++; }
    for (int32_t v = 0; v < V; ++v) {
        h.out_off[v + 1] += h.out_off[v];
        h.in_off[v + 1] += h.in_off[v];
    }
    const uint32_t A = h.out_off[V];
    h.out_v.resize(A);
    h.in_v.resize(A);
    h.out_t.resize(A);
    h.in_t.resize(A);
    std::vector<uint32_t> po(h.out_off.begin(), h.out_off.end() - 1),
        pi(h.in_off.begin(), h.in_off.end() - 1);
    for (int64_t i = 0; i < E; ++i) {   // the edge list is in time order: lists are too
        if (h.src[i] == h.dst[i]) continue;
        const uint32_t a = po[h.src[i]]++, b = pi[h.dst[i]]++;
        h.out_v[a] = h.dst[i];
        h.out_t[a] = h.t[i];
        h.in_v[b] = h.src[i];
        h.in_t[b] = h.t[i];
    }
}

// The host copy of a graph that lives on the device: its edge list read
// back, the lists rebuilt.
int ensure_host(mg_graph *g) {
    if (g->host) return MG_OK;
    std::unique_ptr<HostAdj> h(new HostAdj);
    const int64_t E = g->E;
    h->src.resize(E);
    h->dst.resize(E);
    h->t.resize(E);
    if (E) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(g->device) != hipSuccess)
            return fail(MG_EDEVICE, "cannot select device %d", g->device);
        bool ok = hipMemcpy(h->src.data(), g->gsrc.ptr, 4 * (size_t)E, hipMemcpyDeviceToHost) ==
                      hipSuccess &&
                  hipMemcpy(h->dst.data(), g->gdst.ptr, 4 * (size_t)E, hipMemcpyDeviceToHost) ==
                      hipSuccess;
        if (ok && g->time_bytes == 4) {
            std::vector<uint32_t> rt(E);
            ok = hipMemcpy(rt.data(), g->gt.ptr, 4 * (size_t)E, hipMemcpyDeviceToHost) == hipSuccess;
            for (int64_t i = 0; i < E; ++i) h->t[i] = g->t_min + (int64_t)rt[i];
        } else if (ok) {
            std::vector<uint64_t> rt(E);
            ok = hipMemcpy(rt.data(), g->gt.ptr, 8 * (size_t)E, hipMemcpyDeviceToHost) == hipSuccess;
            for (int64_t i = 0; i < E; ++i) h->t[i] = g->t_min + (int64_t)rt[i];
        }
        (void)hipSetDevice(cur);
        if (!ok) return fail(MG_EDEVICE, "reading the graph back from the device failed");
    }
    build_lists(*h, g->V);
    g->host = std::move(h);
    return MG_OK;
}

// ---------------------------------------------------------------- code generation
struct Gen {
    const mg_tree *tr;
    std::ostringstream o;
    int tmp = 0;

    static std::string ind(int d) { return std::string(2 * d + 2, ' '); }

    // the code of the subtree under trie node n: vars[k] holds the graph
    // vertex of motif vertex k (the first nv are bound), tp the time of the
    // last matched edge
    void node(int n, std::vector<std::string> vars, const std::string &tp, int d) {
        const TrieNode &nd = tr->nodes[n];
        // the children by the list they scan, as the GPU tables group them
        std::map<std::pair<int, int>, std::vector<int>> groups;
        for (int c : nd.kids) {
            const TrieNode &ch = tr->nodes[c];
            int dir, anc;
            if (ch.u < nd.nv) { dir = 0; anc = ch.u; }
            else if (ch.v < nd.nv) { dir = 1; anc = ch.v; }
            else { dir = 2; anc = 0; }
            groups[{dir, anc}].push_back(c);
        }
        for (auto &kv : groups) {
            const int dir = kv.first.first, anc = kv.first.second, k = tmp++;
            const std::string i = "i" + std::to_string(k), e = "e" + std::to_string(k),
                              w = "w" + std::to_string(k), x = "x" + std::to_string(k),
                              t = "t" + std::to_string(k);
            if (dir == 2) {
                // every edge of the window: both endpoints new
                o << ind(d) << "for (int64_t " << i << " = after(g->t, (int64_t)0, g->n, " << tp << "), " << e
                  << " = after(g->t, " << i << ", g->n, thi); " << i << " < " << e << "; ++" << i
                  << ") {\n";
                o << ind(d + 1) << "const int32_t " << x << " = g->src[" << i << "], " << w
                  << " = g->dst[" << i << "];\n";
                o << ind(d + 1) << "const int64_t " << t << " = g->t[" << i << "];\n";
                o << ind(d + 1) << "if (" << x << " == " << w;
                for (int b = 0; b < nd.nv; ++b)
                    o << " || " << x << " == " << vars[b] << " || " << w << " == " << vars[b];
                o << ") continue;\n";
                for (int c : kv.second) {
                    const TrieNode &ch = tr->nodes[c];
                    std::vector<std::string> nv = vars;
                    nv.resize(std::max<size_t>(nv.size(), ch.nv));
                    nv[ch.u] = x;
                    nv[ch.v] = w;
                    child(c, nv, t, d + 1);
                }
                o << ind(d) << "}\n";
                continue;
            }
            const std::string off = dir == 0 ? "g->oo" : "g->io", ts = dir == 0 ? "g->ot" : "g->it",
                              vs = dir == 0 ? "g->ov" : "g->iv", a = vars[anc];
            o << ind(d) << "for (uint32_t " << i << " = after(" << ts << ", " << off << "[" << a
              << "], " << off << "[" << a << " + 1], " << tp << "), " << e << " = after(" << ts
              << ", " << i << ", " << off << "[" << a << " + 1], thi); " << i << " < " << e
              << "; ++" << i << ") {\n";
            o << ind(d + 1) << "const int32_t " << w << " = " << vs << "[" << i << "];\n";
            o << ind(d + 1) << "const int64_t " << t << " = " << ts << "[" << i << "];\n";
            // a bound endpoint selects its child; a new one must differ from
            // every bound vertex
            bool first = true;
            int newc = -1;
            for (int c : kv.second) {
                const TrieNode &ch = tr->nodes[c];
                const int far = dir == 0 ? ch.v : ch.u;
                if (far >= nd.nv) { newc = c; continue; }
                o << ind(d + 1) << (first ? "if (" : "else if (") << w << " == " << vars[far]
                  << ") {\n";
                child(c, vars, t, d + 2);
                o << ind(d + 1) << "}\n";
                first = false;
            }
            if (newc >= 0) {
                const TrieNode &ch = tr->nodes[newc];
                o << ind(d + 1) << (first ? "if (" : "else if (");
                for (int b = 0; b < nd.nv; ++b) o << (b ? " && " : "") << w << " != " << vars[b];
                o << ") {\n";
                std::vector<std::string> nv = vars;
                nv.resize(std::max<size_t>(nv.size(), ch.nv));
                nv[dir == 0 ? ch.v : ch.u] = w;
                child(newc, nv, t, d + 2);
                o << ind(d + 1) << "}\n";
            }
            o << ind(d) << "}\n";
        }
    }

    void child(int c, const std::vector<std::string> &vars, const std::string &t, int d) {
        const TrieNode &ch = tr->nodes[c];
        if (ch.q >= 0) o << ind(d) << "++cnt[" << ch.q << " * nd + slot(tf, " << t << ", dlo, nd)];\n";
        if (!ch.kids.empty()) node(c, vars, t, d);
    }

    std::string source() {
        o << "// generated: the search of one motif group, one loop nest per trie level\n"
             "#include <stdint.h>\n"
             "struct G { const int32_t *src, *dst; const int64_t *t; const uint32_t *oo, *io;\n"
             "           const int32_t *ov, *iv; const int64_t *ot, *it; int64_t n; };\n"
             "template <typename I> static inline I after(const int64_t *ts, I lo, I hi, int64_t v) {\n"
             "  I n = hi - lo;\n"
             "  while (n > 0) { I h = n / 2; if (ts[lo + h] <= v) { lo += h + 1; n -= h + 1; } else n = h; }\n"
             "  return lo;\n"
             "}\n"
             "static inline int64_t slot(int64_t tf, int64_t t, const int64_t *dlo, int32_t nd) {\n"
             "  int64_t j = 0;\n"
             "  for (int32_t i = 0; i + 1 < nd; ++i) j += t - tf > dlo[i];\n"
             "  return j;\n"
             "}\n"
             "extern \"C\" void mg_gen_search(const G *g, int64_t r0, int64_t r1, int64_t delta,\n"
             "                              const int64_t *dlo, int32_t nd, uint64_t *cnt) {\n"
             "  for (int64_t r = r0; r < r1; ++r) {\n"
             "    const int32_t v0 = g->src[r], v1 = g->dst[r];\n"
             "    if (v0 == v1) continue;\n"
             "    const int64_t tf = g->t[r];\n"
             "    const int64_t thi = tf > INT64_MAX - delta ? INT64_MAX : tf + delta;\n"
             "    (void)thi;\n";
        if (tr->root_q >= 0) o << "    ++cnt[" << tr->root_q << " * nd];\n";
        node(0, {"v0", "v1"}, "tf", 1);
        o << "  }\n}\n";
        return o.str();
    }
};

// Compiled searches by their source text: trees with the same motifs (any
// windows: they are arguments) share one, loaded for the life of the process.
std::mutex g_code_mu;
std::map<std::string, void *> g_code;

// Generates, compiles and loads the search of tr (once per tree; a tree is
// not used by two threads at once).
bool load_generated(mg_tree *tr) {
    if (tr->cpu_fn) return true;
    if (!tr->cpu_error.empty()) return false;
    Gen gen{tr, {}, 0};
    const std::string src = gen.source();
    {
        std::lock_guard<std::mutex> lock(g_code_mu);
        auto it = g_code.find(src);
        if (it != g_code.end()) {
            tr->cpu_fn = it->second;
            return true;
        }
    }
    const char *tmp = getenv("TMPDIR");
    std::string dir = std::string(tmp && *tmp ? tmp : "/tmp") + "/mayura_cpu_XXXXXX";
    std::vector<char> dbuf(dir.begin(), dir.end());
    dbuf.push_back(0);
    if (!mkdtemp(dbuf.data())) { tr->cpu_error = "mkdtemp failed"; return false; }
    dir = dbuf.data();
    const std::string cpp = dir + "/search.cpp", so = dir + "/search.so";
    { std::ofstream f(cpp); f << src; }
    const char *cxx_env = getenv("MG_CXX");
    const std::string cxx = cxx_env && *cxx_env ? cxx_env : "c++";
    std::vector<std::string> args = {cxx, "-O3", "-march=native", "-std=c++17", "-shared", "-fPIC",
                                     "-o", so, cpp};
    std::vector<char *> argv;
    for (auto &a : args) argv.push_back(const_cast<char *>(a.c_str()));
    argv.push_back(nullptr);
    pid_t pid = 0;
    int status = -1;
    if (posix_spawnp(&pid, cxx.c_str(), nullptr, nullptr, argv.data(), environ) != 0 ||
        waitpid(pid, &status, 0) != pid || !WIFEXITED(status) || WEXITSTATUS(status) != 0) {
        tr->cpu_error = "compiling the generated search with " + cxx + " failed";
    } else {
        void *lib = dlopen(so.c_str(), RTLD_NOW | RTLD_LOCAL);
        void *fn = lib ? dlsym(lib, "mg_gen_search") : nullptr;
        if (!fn) {
            tr->cpu_error = "loading the generated search failed";
            if (lib) dlclose(lib);
        } else {
            tr->cpu_fn = fn;
            std::lock_guard<std::mutex> lock(g_code_mu);
            g_code.emplace(src, fn);   // the library stays loaded
        }
    }
    unlink(so.c_str());
    unlink(cpp.c_str());
    rmdir(dir.c_str());
    return tr->cpu_fn != nullptr;
}

// ---------------------------------------------------------------- interpreter
// The same search read from the trie: no code generated (the recursion the
// paper's CPU baseline runs).
struct Interp {
    const HostAdj &h;
    const mg_tree *tr;
    int64_t tf, thi;
    const int64_t *dlo;
    int32_t nd;
    uint64_t *cnt;
    int32_t vars[MG_MAX_MOTIF_VERTICES];

    static uint32_t after(const int64_t *ts, uint32_t lo, uint32_t hi, int64_t v) {
        uint32_t n = hi - lo;
        while (n > 0) {
            const uint32_t m = n / 2;
            if (ts[lo + m] <= v) { lo += m + 1; n -= m + 1; }
            else n = m;
        }
        return lo;
    }
    int64_t slot(int64_t t) const {
        int64_t j = 0;
        for (int32_t i = 0; i + 1 < nd; ++i) j += t - tf > dlo[i];
        return j;
    }
    bool bound(int32_t x, int nv) const {
        for (int b = 0; b < nv; ++b)
            if (vars[b] == x) return true;
        return false;
    }
    void reach(int c, int64_t t) {
        const TrieNode &ch = tr->nodes[c];
        if (ch.q >= 0) ++cnt[ch.q * nd + slot(t)];
        if (!ch.kids.empty()) node(c, t);
    }
    void node(int n, int64_t tp) {
        const TrieNode &nd_ = tr->nodes[n];
        for (int c : nd_.kids) {
            const TrieNode &ch = tr->nodes[c];
            const int nv = nd_.nv;
            if (ch.u < nv) {   // out-list of the bound source
                const int32_t a = vars[ch.u];
                const uint32_t b0 = after(h.out_t.data(), h.out_off[a], h.out_off[a + 1], tp);
                const uint32_t e = after(h.out_t.data(), b0, h.out_off[a + 1], thi);
                for (uint32_t i = b0; i < e; ++i) {
                    const int32_t w = h.out_v[i];
                    if (ch.v < nv ? w != vars[ch.v] : bound(w, nv)) continue;
                    if (ch.v >= nv) vars[ch.v] = w;
                    reach(c, h.out_t[i]);
                }
            } else if (ch.v < nv) {   // in-list of the bound destination, new source
                const int32_t a = vars[ch.v];
                const uint32_t b0 = after(h.in_t.data(), h.in_off[a], h.in_off[a + 1], tp);
                const uint32_t e = after(h.in_t.data(), b0, h.in_off[a + 1], thi);
                for (uint32_t i = b0; i < e; ++i) {
                    const int32_t w = h.in_v[i];
                    if (bound(w, nv)) continue;
                    vars[ch.u] = w;
                    reach(c, h.in_t[i]);
                }
            } else {   // every edge of the window, both endpoints new
                const int64_t n_ = (int64_t)h.t.size();
                int64_t lo = 0, cntn = n_;
                while (cntn > 0) {
                    const int64_t m = cntn / 2;
                    if (h.t[lo + m] <= tp) { lo += m + 1; cntn -= m + 1; }
                    else cntn = m;
                }
                for (int64_t i = lo; i < n_ && h.t[i] <= thi; ++i) {
                    const int32_t s = h.src[i], d = h.dst[i];
                    if (s == d || bound(s, nv) || bound(d, nv)) continue;
                    vars[ch.u] = s;
                    vars[ch.v] = d;
                    reach(c, h.t[i]);
                }
            }
        }
    }
};

// ---------------------------------------------------------------- run
int count_tree(mg_graph *g, mg_tree *tr, const std::vector<int64_t> &roots, bool use_roots,
               int32_t threads, bool codegen, std::vector<uint64_t> &slots) {
    const HostAdj &h = *g->host;
    const size_t nd = tr->deltas.size();
    slots.assign(tr->distinct.size() * nd, 0);
    std::vector<int64_t> dlo(tr->deltas.begin(), tr->deltas.end());
    GenFn fn = nullptr;
    if (codegen) {
        if (!load_generated(tr)) return fail(MG_EUNSUPPORTED, "%s", tr->cpu_error.c_str());
        fn = (GenFn)tr->cpu_fn;
    }
    GenGraph gg{h.src.data(), h.dst.data(), h.t.data(), h.out_off.data(), h.in_off.data(),
                h.out_v.data(), h.in_v.data(), h.out_t.data(), h.in_t.data(),
                (int64_t)h.src.size()};
    const int64_t n = use_roots ? (int64_t)roots.size() : g->E;
    const int64_t chunk = 1024;
    std::atomic<int64_t> next{0};
    std::mutex mu;
    auto work = [&]() {
        std::vector<uint64_t> local(slots.size(), 0);
        Interp in{h, tr, 0, 0, dlo.data(), (int32_t)nd, local.data(), {}};
        for (;;) {
            const int64_t b = next.fetch_add(chunk);
            if (b >= n) break;
            const int64_t e = std::min(n, b + chunk);
            // root positions: a contiguous range, or one call per listed root
            for (int64_t k = b; k < e;) {
                int64_t r0 = use_roots ? roots[k] : k, r1 = r0 + 1;
                int64_t k1 = k + 1;
                if (!use_roots) { r1 = e; k1 = e; }
                if (fn) {
                    fn(&gg, r0, r1, tr->delta, dlo.data(), (int32_t)nd, local.data());
                } else {
                    for (int64_t r = r0; r < r1; ++r) {
                        if (h.src[r] == h.dst[r]) continue;
                        in.tf = h.t[r];
                        in.thi = in.tf > INT64_MAX - tr->delta ? INT64_MAX : in.tf + tr->delta;
                        in.vars[0] = h.src[r];
                        in.vars[1] = h.dst[r];
                        if (tr->root_q >= 0) ++local[tr->root_q * nd];
                        in.node(0, in.tf);
                    }
                }
                k = k1;
            }
        }
        std::lock_guard<std::mutex> lock(mu);
        for (size_t i = 0; i < slots.size(); ++i) slots[i] += local[i];
    };
    const int32_t nt = threads > 0 ? threads : (int32_t)std::max(1u, std::thread::hardware_concurrency());
    std::vector<std::thread> pool;
    for (int32_t k = 1; k < nt; ++k) pool.emplace_back(work);
    work();
    for (auto &t : pool) t.join();
    return MG_OK;
}

// Whether the graph, its edges taken as undirected, has no odd cycle
// (two-colouring by breadth-first search).
bool is_bipartite(const mg_graph *g) {
    const HostAdj &h = *g->host;
    std::vector<int8_t> col(g->V, -1);
    std::vector<int32_t> queue;
    for (int32_t s = 0; s < g->V; ++s) {
        if (col[s] >= 0) continue;
        col[s] = 0;
        queue.assign(1, s);
        for (size_t qi = 0; qi < queue.size(); ++qi) {
            const int32_t x = queue[qi];
            for (int side = 0; side < 2; ++side) {
                const std::vector<uint32_t> &off = side ? h.in_off : h.out_off;
                const std::vector<int32_t> &nb = side ? h.in_v : h.out_v;
                for (uint32_t i = off[x]; i < off[x + 1]; ++i) {
                    const int32_t y = nb[i];
                    if (col[y] < 0) { col[y] = (int8_t)(1 - col[x]); queue.push_back(y); }
                    else if (col[y] == col[x]) return false;
                }
            }
        }
    }
    return true;
}

}  // namespace

void release_cpu_code(mg_tree *tr) {
    // the compiled code is shared through the cache and stays loaded
    tr->cpu_lib = nullptr;
    tr->cpu_fn = nullptr;
}

void build_host(mg_graph *g, std::vector<int32_t> s, std::vector<int32_t> d, std::vector<int64_t> t) {
    std::unique_ptr<HostAdj> h(new HostAdj);
    h->src = std::move(s);
    h->dst = std::move(d);
    h->t = std::move(t);
    build_lists(*h, g->V);
    g->host = std::move(h);
}

}  // namespace mgh

using namespace mgh;

extern "C" {

void mg_cpu_opts_init(mg_cpu_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->codegen = 1;
}

int mg_count_cpu(const mg_graph *g_c, const mg_tree *tr_c, const mg_cpu_opts *opts,
                 uint64_t *counts) {
    try {
        if (!g_c || !tr_c || !counts) return fail(MG_EINVAL, "NULL argument");
        mg_cpu_opts o;
        mg_cpu_opts_init(&o);
        if (opts) o = *opts;
        if (o.mode != MG_MODE_COMINE && o.mode != MG_MODE_PER_MOTIF)
            return fail(MG_EINVAL, "unknown mode %d", o.mode);
        if (o.threads < 0 || (o.roots && o.n_roots < 0)) return fail(MG_EINVAL, "bad argument");
        mg_graph *g = const_cast<mg_graph *>(g_c);   // the host copy is a cache
        mg_tree *tr = const_cast<mg_tree *>(tr_c);
        int rc = ensure_host(g);
        if (rc) return rc;
        std::vector<int64_t> roots;
        if (o.roots) {
            roots.assign(o.roots, o.roots + o.n_roots);
            for (int64_t r : roots)
                if (r < 0 || r >= g->E) return fail(MG_EINVAL, "root %lld out of range", (long long)r);
        }
        std::vector<mg_tree *> runs;
        if (o.mode == MG_MODE_COMINE) {
            runs.push_back(tr);
        } else {
            rc = chain_trees(tr);
            if (rc) return rc;
            for (auto &u : tr->singles) runs.push_back(u.get());
        }
        if (o.codegen) {
            // generate and compile first (in parallel), so that the timing
            // holds the searches only
            std::vector<std::thread> cc;
            std::atomic<size_t> next{0};
            const size_t nt = std::min<size_t>(runs.size(), std::max(1u, std::thread::hardware_concurrency()));
            for (size_t k = 0; k < nt; ++k)
                cc.emplace_back([&] {
                    for (size_t i; (i = next.fetch_add(1)) < runs.size();) load_generated(runs[i]);
                });
            for (auto &t : cc) t.join();
            for (mg_tree *t : runs)
                if (!t->cpu_fn) return fail(MG_EUNSUPPORTED, "%s", t->cpu_error.c_str());
        }
        const auto t0 = std::chrono::steady_clock::now();
        const size_t nd = tr->deltas.size();
        std::vector<uint64_t> slots(tr->distinct.size() * nd, 0), one;
        for (size_t q = 0; q < runs.size(); ++q) {
            rc = count_tree(g, runs[q], roots, o.roots != nullptr, o.threads, o.codegen != 0, one);
            if (rc) return rc;
            if (o.mode == MG_MODE_COMINE) slots = one;
            else std::copy(one.begin(), one.end(), slots.begin() + q * nd);
        }
        if (o.elapsed_ms)
            *o.elapsed_ms = std::chrono::duration<double, std::milli>(
                                std::chrono::steady_clock::now() - t0).count();
        // window slots to counts in the caller's order, as mg_count
        for (size_t i = 0; i < tr->delta_slot.size(); ++i)
            for (int32_t m = 0; m < tr->n_motifs; ++m) {
                uint64_t sum = 0;
                for (int32_t j = 0; j <= tr->delta_slot[i]; ++j) sum += slots[tr->motif_q[m] * nd + j];
                counts[i * (size_t)tr->n_motifs + m] = sum;
            }
        return MG_OK;
    } catch (const std::bad_alloc &) {
        return fail(MG_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

int mg_comine_advice(const mg_graph *g_c, const mg_tree *tr, int32_t platform, mg_advice *out) {
    try {
        if (!g_c || !tr || !out || (platform != MG_PLATFORM_GPU && platform != MG_PLATFORM_CPU))
            return fail(MG_EINVAL, "bad argument");
        mg_graph *g = const_cast<mg_graph *>(g_c);
        if (g->bipartite < 0) {
            int rc = ensure_host(g);
            if (rc) return rc;
            g->bipartite = is_bipartite(g) ? 1 : 0;
        }
        out->bipartite = g->bipartite;
        out->similarity = tr->info.similarity;
        out->threshold = platform == MG_PLATFORM_GPU ? MG_GPU_SM_THRESHOLD : 0.0;
        out->co_mine = g->bipartite || !(platform == MG_PLATFORM_GPU &&
                                         tr->info.similarity < MG_GPU_SM_THRESHOLD);
        return MG_OK;
    } catch (...) {
        return fail(MG_EINTERNAL, "unexpected exception");
    }
}

}  // extern "C"
