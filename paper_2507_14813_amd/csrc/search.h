// Co-mining kernel for gfx950 (CDNA4, wave64).  This header is included once
// per tree depth by search_d<depth>_t<bits>.hip (one translation unit per tree depth and time width).
//
// What runs here is the co-mining recursion of the paper (Algorithm 3, built
// on the per-motif matcher of Algorithm 1): from every root edge, partial
// matches are extended edge by edge along the search levels of the motif
// group's prefix trie; reaching a trie node credits every motif whose edge
// sequence equals that prefix, and the same partial match then continues into
// all of the node's children.
//
// How it is laid out for the hardware (not the paper's warp-per-candidate
// design):
//   * Every wave is an independent worker.  Root edges are split into eight
//     contiguous (time-ordered) queues, one per XCD; a wave grabs chunks from
//     its XCD's queue and steals from the others when it runs dry, so roots
//     that are close in time, and the adjacency they read, share one L2.
//   * Partial matches are buffered per search level in LDS.  For a batch of
//     partial matches at level L, every (partial match, child group) pair is
//     a window of one time-sorted adjacency list: the entries with
//     t_prev < t <= t_first + delta, found by bisection.  Children that read
//     the same list (same direction, same anchor vertex) form one group and
//     share one scan of the window.
//   * Windows are found from other windows where possible: a root's windows
//     in out(a) and in(b) start just past the root edge's own list position,
//     and a deeper window on a list of the root's two vertices lies inside the
//     root's window on that list (kept in LDS), so it needs a short bisection
//     and no search for its end.  Below the first level, the pairs on such
//     lists are taken before the others, so the lanes of one pass run
//     bisections of similar length.
//   * A window whose children all end a motif is counted, not expanded: one
//     equality count per bound vertex (the list's own anchor left out), the
//     new-vertex child taking the rest; a short one by its own lane, a long
//     one by the whole wave with ballots.
//   * A batch whose partial matches all sit at leaf parents (trie nodes
//     whose children all end a motif, reached through lists of bound
//     vertices) is taken one partial match per lane instead: the lane finds
//     and counts the window of each of the node's groups in turn, with no
//     pairing of partial matches and groups across the wave.
//   * The other non-empty windows, up to 64 at a time, are expanded as one
//     flat candidate range: lane i takes candidate c + i, finds its window
//     from a 64-bit mask of window ends (LDS flags + ballot + popcount), reads
//     one adjacency entry, finds which bound motif vertex it hits with
//     predicated compares, picks the reached child from the group record
//     (which also carries the child's motif id), credits LDS counters, and
//     compacts the survivors that still have children into the next level's
//     buffer with ballot + mbcnt.
//   * When the next level's buffer holds 64 or more partial matches it is
//     expanded at once (depth first over batches), so LDS use is bounded by
//     the motif length, not by the size of the search tree.
//   * The level loop nest is unrolled at compile time for the tree depth
//     (1..5 motif edges), one instantiation per depth.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "comine.h"
#include "device_util.h"

namespace mg {
namespace {


constexpr uint32_t kChunkLimit = 0x7fffffffu;   // candidates per window chunk

// child word of a group for scanned-endpoint index y (0..5 bound, else new)
__device__ __forceinline__ uint32_t child_word(const uint4 &a, const uint4 &b, int y) {
    uint32_t r = b.w;             // new vertex
    r = (y == 0) ? a.y : r;
    r = (y == 1) ? a.z : r;
    r = (y == 2) ? a.w : r;
    r = (y == 3) ? b.x : r;
    r = (y == 4) ? b.y : r;
    r = (y == 5) ? b.z : r;
    return r;
}

// The smaller window j of a multi-window tree (selects, so that the
// parameter array is never indexed at run time: a local copy of it would go
// to scratch memory).
template <typename TT>
__device__ __forceinline__ TT window_lo(const KParams<TT> &p, uint32_t j) {
    TT r = p.dlo[0];
#pragma unroll
    for (int i = 1; i < kMaxDeltas - 1; ++i) r = j == (uint32_t)i ? p.dlo[i] : r;
    return r;
}

// Window slot of a match with first time tf and last time tl: the number of
// smaller windows its span exceeds.
template <typename TT>
__device__ __forceinline__ uint32_t window_slot(const KParams<TT> &p, uint32_t nd, TT tf, TT tl) {
    uint32_t j = 0;
#pragma unroll
    for (int i = 0; i < kMaxDeltas - 1; ++i)
        j += ((uint32_t)i + 1 < nd && tl > sat_add(tf, p.dlo[i])) ? 1u : 0u;
    return j;
}

// c matches of the child in `word`, credited to window slot j of its motif
// (nd slots per motif).  With `move`, the c matches were already credited to
// slot j + 1 (they lie in a larger window too) and move down to slot j: slot
// j + 1 loses them.  The counters are summed over slots modulo 2^64, so a
// slot may hold a negative amount in between.
__device__ __forceinline__ uint32_t credit_child(uint32_t word, uint32_t c,
                                                unsigned long long *cnt, uint32_t nd,
                                                uint32_t j, bool move = false) {
    if (!c || !word) return 0;
    const uint32_t q1 = (word >> 16) & 0x7fffu;
    if (q1) {
        atomicAdd(&cnt[(q1 - 1) * nd + j], (unsigned long long)c);
        if (move) atomicAdd(&cnt[(q1 - 1) * nd + j + 1], 0ull - c);
    }
    return move ? 0u : c;
}

// Counts a leaf-only window [l0, l0 + len) of one adjacency list for one
// partial match: each entry reaches the child of the bound vertex it hits, or
// the new-vertex child.  The bound vertices are distinct, so an entry hits at
// most one of them: one equality count per bound vertex, and the new-vertex
// child gets the rest of the window.  The list's own anchor is left out of
// q[] (no entry equals it: lists hold no self-loops); q[0..K) are the other
// bound vertices (-1 for none) and w[0..K) their child words, wn the
// new-vertex child's word.  Credits go to window slot j of each motif (nd
// slots per motif).  Returns the credits.
template <int U, int K, typename TT, int N>
__device__ __forceinline__ uint32_t leaf_count(const Entry<TT> *__restrict__ adj, uint32_t l0,
                                               uint32_t len, const int32_t (&q)[N],
                                               const uint32_t (&w)[N], uint32_t wn,
                                               unsigned long long *cnt, uint32_t nd,
                                               uint32_t j, bool move = false) {
    static_assert(K <= N, "slots");
    uint32_t c[K];
#pragma unroll
    for (int s = 0; s < K; ++s) c[s] = 0;
    // U independent loads per step, the last step included: there an index
    // past the window reloads its last entry (len >= 1) and counts as no hit,
    // so a window of up to U entries costs one memory trip
    const Entry<TT> *e = adj + l0;
    uint32_t i = 0;
    for (; i + U <= len; i += U) {
        int32_t v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = e[i + j].v;
#pragma unroll
        for (int j = 0; j < U; ++j)
#pragma unroll
            for (int s = 0; s < K; ++s) c[s] += v[j] == q[s];
    }
    if (i < len) {
        int32_t v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = e[min(i + j, len - 1)].v;
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int32_t x = i + j < len ? v[j] : -2;   // -2 matches no vertex
#pragma unroll
            for (int s = 0; s < K; ++s) c[s] += x == q[s];
        }
    }
    uint32_t hit = 0, got = 0;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        hit += c[s];
        got += credit_child(w[s], c[s], cnt, nd, j, move);
    }
    return got + credit_child(wn, len - hit, cnt, nd, j, move);
}


// Counts the leaf-only window [l0, l0 + len) of group g for the partial match
// with bound vertices ph[] with the whole wave, 64 entries per pass: one ballot per bound
// vertex counts the entries that hit it, and the new-vertex child gets the
// rest.  All arguments are wave-uniform.  Credits go to window slot j.
// Returns the credits on lane 0 (0 on the other lanes).
template <typename TT, int SA>
__device__ __forceinline__ uint32_t leaf_scan_wave(const KParams<TT> &p, const int32_t (&ph)[SA],
                                                   uint32_t g, uint32_t l0, uint32_t len,
                                                   const int lane, unsigned long long *cnt,
                                                   uint32_t nd, uint32_t j, bool move = false) {
    const uint4 ga = p.tree.grp[2 * g], gb = p.tree.grp[2 * g + 1];
    const uint32_t nvp = (ga.x >> 8) & 15;
    const Entry<TT> *__restrict__ e =
        ((ga.x & 15) == kDirOut ? p.g.out_adj : p.g.in_adj) + l0;
    int32_t q[SA];
    uint32_t c[SA];
#pragma unroll
    for (int s = 0; s < SA; ++s) {
        q[s] = (uint32_t)s < nvp ? ph[s] : -1;
        c[s] = 0;
    }
    uint32_t i = 0;
    for (; i + 4 * kWave <= len; i += 4 * kWave) {
        int32_t v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = e[i + j * kWave + lane].v;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int s = 0; s < SA; ++s) c[s] += (uint32_t)__popcll(__ballot(v[j] == q[s]));
    }
    for (; i < len; i += kWave) {
        const int32_t v = i + lane < len ? e[i + lane].v : -2;   // -2 matches no slot
#pragma unroll
        for (int s = 0; s < SA; ++s) c[s] += (uint32_t)__popcll(__ballot(v == q[s]));
    }
    if (lane != 0) return 0;
    const uint32_t words[6] = {ga.y, ga.z, ga.w, gb.x, gb.y, gb.z};
    uint32_t hit = 0, got = 0;
#pragma unroll
    for (int s = 0; s < SA; ++s) {
        hit += c[s];
        got += credit_child(words[s], c[s], cnt, nd, j, move);
    }
    return got + credit_child(gb.w, len - hit, cnt, nd, j, move);
}

// The same for a tree with several windows: the whole window counts at the
// largest window, and each smaller window, a prefix of it whose length the
// same pass measures (entries with t <= t_first + its delta, one ballot per
// window), moves its matches down one slot with a second, shorter pass.
// tf: the partial match's first time.
template <typename TT, int SA>
__device__ __forceinline__ uint32_t leaf_scan_wave_multi(const KParams<TT> &p,
                                                         const int32_t (&ph)[SA], uint32_t g,
                                                         uint32_t l0, uint32_t len, TT tf,
                                                         const int lane, unsigned long long *cnt,
                                                         uint32_t nd) {
    const uint4 ga = p.tree.grp[2 * g], gb = p.tree.grp[2 * g + 1];
    const uint32_t nvp = (ga.x >> 8) & 15;
    const Entry<TT> *__restrict__ e =
        ((ga.x & 15) == kDirOut ? p.g.out_adj : p.g.in_adj) + l0;
    int32_t q[SA];
    uint32_t c[SA];
#pragma unroll
    for (int s = 0; s < SA; ++s) {
        q[s] = (uint32_t)s < nvp ? ph[s] : -1;
        c[s] = 0;
    }
    TT thr[kMaxDeltas - 1];
    uint32_t pre[kMaxDeltas - 1];
#pragma unroll
    for (int j = 0; j < kMaxDeltas - 1; ++j) {
        thr[j] = sat_add(tf, p.dlo[j]);
        pre[j] = 0;
    }
    // four independent loads per pass while whole, then one at a time
    uint32_t i = 0;
    for (; i + 4 * kWave <= len; i += 4 * kWave) {
        Entry<TT> en[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) en[k] = e[i + k * kWave + lane];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int s = 0; s < SA; ++s) c[s] += (uint32_t)__popcll(__ballot(en[k].v == q[s]));
#pragma unroll
            for (int j = 0; j < kMaxDeltas - 1; ++j)
                if ((uint32_t)j + 1 < nd) pre[j] += (uint32_t)__popcll(__ballot(en[k].t <= thr[j]));
        }
    }
    for (; i < len; i += kWave) {
        const bool in = i + lane < len;
        Entry<TT> en{};
        if (in) en = e[i + lane];
        const int32_t v = in ? en.v : -2;   // -2 matches no slot
#pragma unroll
        for (int s = 0; s < SA; ++s) c[s] += (uint32_t)__popcll(__ballot(v == q[s]));
#pragma unroll
        for (int j = 0; j < kMaxDeltas - 1; ++j)
            if ((uint32_t)j + 1 < nd) pre[j] += (uint32_t)__popcll(__ballot(in && en.t <= thr[j]));
    }
    uint32_t got = 0;
    if (lane == 0) {
        const uint32_t words[6] = {ga.y, ga.z, ga.w, gb.x, gb.y, gb.z};
        uint32_t hit = 0;
#pragma unroll
        for (int s = 0; s < SA; ++s) {
            hit += c[s];
            got += credit_child(words[s], c[s], cnt, nd, nd - 1);
        }
        got += credit_child(gb.w, len - hit, cnt, nd, nd - 1);
    }
#pragma unroll
    for (int j = kMaxDeltas - 2; j >= 0; --j)
        if ((uint32_t)j + 1 < nd && pre[j] > 0)
            leaf_scan_wave<TT, SA>(p, ph, g, l0, pre[j], lane, cnt, nd, (uint32_t)j, true);
    return got;
}

// Partial matches with L motif edges matched.  Level 1 is the root batch:
// every entry is at the trie root and its last edge is its first, so it keeps
// only the two bound vertices and the root time.
// R: 1 = each partial match also keeps its root edge (the per-root cost log),
// 2 = its root edge and the slot of its parent one level up (enumeration,
// which writes out every matched edge).
// V: vertex slots, the most motif vertices bound at this level (vslots).
template <typename TT, int L, int R, int V>
struct LevelBuf {
    static constexpr int S = V;              // vertex slots
    static constexpr int C = 2 * kWave;      // capacity
    // phi[s - 2][i]: graph vertex of motif vertex s >= 2; motif vertices 0 and
    // 1 and t_first are the root's, kept once in the level-1 batch (slot r1)
    int32_t phi[S - 2][C];
    uint32_t eid[C];       // edge id of its last matched edge
    uint16_t node[C];      // internal trie node reached
    uint16_t pincl[C];     // inclusive prefix of child-group counts: groups on
    uint16_t pincl1[C];    // lists of motif vertex 0 or 1, then the others
    uint8_t r1[C];         // slot of its root in the level-1 batch
    uint32_t root[R ? C : 1];
    uint8_t par[R == 2 && L > 2 ? C : 1];   // slot of its parent at level L - 1
};
template <typename TT, int R, int V>
struct LevelBuf<TT, 1, R, V> {
    static constexpr int S = 2;
    static constexpr int C = kWave;
    int32_t phi[2][kWave];
    TT tfirst[kWave];
    uint32_t root[R ? kWave : 1];
};

// Vertex slots at level L of a kernel for trees of depth D: two per edge, at
// most kVMax.  Depth-3 kernels keep three at level 2, which holds for trees
// whose buffered two-edge prefixes share a vertex; the host runs trees with a
// four-vertex two-edge prefix on the depth-4 kernel (DevTree::kdepth).  The
// slot saved is registers the compiler no longer spills.
constexpr int vslots(int D, int L) {
    return (D == 3 && L == 2) ? 3 : (2 * L < kVMax ? 2 * L : kVMax);
}

template <typename TT, int D, int R, int L>
struct LevelChain {
    LevelBuf<TT, L, R, vslots(D, L)> buf;
    LevelChain<TT, D, R, L + 1> next;
};
template <typename TT, int D, int R>
struct LevelChain<TT, D, R, D> {};

// per-wave LDS: level buffers plus small scratch tables.  Its size is a
// multiple of 16 bytes, so that per-wave blocks laid out back to back (with
// 64-bit counters between them) keep those counters 8-byte aligned, as LDS
// 64-bit atomics require.
//
// Root windows: for each root of the level-1 batch, the windows it found in
// out(a), in(a), out(b), in(b) (index anchor * 2 + direction): first entry and
// length, kNoHint as length when not found yet, kLongHint with the window's
// end (not its first entry) when it has 65534 entries or more.  A deeper
// partial match of that root reads a window of the same
// list with t_prev < t <= t_first + delta, t_prev > t_first: it starts inside
// the root's window and ends where it ends, so a bisection over the root's
// window replaces a bisection over the whole list and the search for the end.
template <typename TT, int D, int R>
struct alignas(16) WaveLds {
    static constexpr int H = D > 1 ? 4 : 1;
    uint8_t src[kWave];           // window compaction: lane holding the k-th window
    uint8_t flag[kWave];          // window-end marks of one pass
    uint32_t hlo[H][kWave];       // root windows (used when D > 2)
    uint16_t hlen[H][kWave];
    LevelChain<TT, D, R, 1> lv;
};

static_assert(sizeof(WaveLds<uint32_t, 1, 0>) % 16 == 0, "per-wave LDS block size");
static_assert(sizeof(WaveLds<uint32_t, 3, 0>) % 16 == 0, "per-wave LDS block size");
static_assert(sizeof(WaveLds<uint32_t, 5, 0>) % 16 == 0, "per-wave LDS block size");
static_assert(sizeof(WaveLds<uint64_t, 5, 1>) % 16 == 0, "per-wave LDS block size");

constexpr uint16_t kNoHint = 0xffff;
constexpr uint16_t kLongHint = 0xfffe;

// A new root a -> b in level-1 slot `slot`: its root windows are not found
// yet; their first-entry words hold where they start, the first entries
// after the root's time in out(a), in(a), out(b) and in(b).
template <typename TT, int D, int R>
__device__ __forceinline__ void set_root_slot(WaveLds<TT, D, R> &W, uint32_t slot, uint4 gx) {
    W.hlo[0][slot] = gx.x;
    W.hlo[1][slot] = gx.y;
    W.hlo[2][slot] = gx.z;
    W.hlo[3][slot] = gx.w;
#pragma unroll
    for (int k = 0; k < 4; ++k) W.hlen[k][slot] = kNoHint;
}

template <int L, typename TT, int D, int R, int M>
__device__ __forceinline__ LevelBuf<TT, L, R, vslots(D, L)> &lvl(LevelChain<TT, D, R, M> &c) {
    if constexpr (L == M) return c.buf;
    else return lvl<L>(c.next);
}

// What the level buffers keep per partial match beyond the search itself
// (the R of LevelBuf) in each kernel MODE.
constexpr int keep_of(int mode) { return mode == 2 ? 1 : mode == 4 ? 2 : 0; }
// MODE 5 and 6 are MODE 0 and 3 with epochs (context offload, KParams::ctx_*)
constexpr bool single_of(int mode) { return mode == 0 || mode == 5; }   // one window
constexpr bool plain_of(int mode) { return mode == 0 || mode == 3 || mode == 5 || mode == 6; }
constexpr bool epochs_of(int mode) { return mode == 5 || mode == 6; }

// Enumeration: the edge ids of partial match i at level L, first edge first,
// into e[0..L), following the parent slots up to the root batch.
template <int L, typename TT, int D>
__device__ __forceinline__ void edge_chain(WaveLds<TT, D, 2> &W, uint32_t i, uint32_t (&e)[kKMax]) {
    if constexpr (L == 1) {
        e[0] = lvl<1>(W.lv).root[i];
    } else {
        auto &A = lvl<L>(W.lv);
        e[L - 1] = A.eid[i];
        if constexpr (L == 2) edge_chain<1>(W, A.r1[i], e);
        else edge_chain<L - 1>(W, A.par[i], e);
    }
}

// Enumeration: writes one record per lane with `want` (motif q, then the
// edges e[0..k) and -1 up to kKMax) at consecutive slots of the output, the
// wave taking its slots with one atomic.  Slots past the capacity are
// dropped (the caller sized the output from the count).
template <typename TT>
__device__ __forceinline__ void write_matches(const KParams<TT> &p, bool want, uint32_t q,
                                              const uint32_t (&e)[kKMax], uint32_t k) {
    const uint64_t m = __ballot(want);
    if (!m) return;
    unsigned long long base = 0;
    if ((threadIdx.x & (kWave - 1)) == 0)
        base = atomicAdd(p.enum_cursor, (unsigned long long)__popcll(m));
    base = lane0_u64(base);
    if (!want) return;
    const unsigned long long slot = base + mbcnt(m);
    if (slot >= p.enum_cap) return;
    int32_t *rec = p.enum_out + slot * (1 + kKMax);
    rec[0] = (int32_t)q;
#pragma unroll
    for (int i = 0; i < kKMax; ++i) rec[1 + i] = (uint32_t)i < k ? (int32_t)e[i] : -1;
}

// Counts the leaf-only window [l0, l0 + len) of group g (header word hdr) for
// one partial match by its own lane: ph[] are its bound vertices, tf its
// first time.  nqm is the largest number of bound vertices compared by the
// lanes counting together (the count loop is compiled for it).  Credits go to
// the largest window, and with several windows each smaller one, a prefix of
// this one, moves its matches down one slot.  Returns the credits.
template <typename TT, int D, int MODE, int S>
__device__ __forceinline__ uint32_t count_leaf_window(const KParams<TT> &p, uint32_t g,
                                                      uint32_t hdr, const int32_t (&ph)[S],
                                                      TT tf, uint32_t l0, uint32_t len,
                                                      uint32_t nqm, unsigned long long *cnt,
                                                      uint32_t nd) {
    constexpr int NQ = S - 1;
    const uint32_t anc = (hdr >> 4) & 15;
    const uint32_t nq = ((hdr >> 8) & 15) - 1u;   // bound vertices, the anchor left out
    const uint4 ga = p.tree.grp[2 * g], gb = p.tree.grp[2 * g + 1];
    const uint32_t words[6] = {ga.y, ga.z, ga.w, gb.x, gb.y, gb.z};
    int32_t q[NQ];
    uint32_t w[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        // slot i below the anchor, slot i + 1 from it on
        const bool below = (uint32_t)i < anc, on = (uint32_t)i < nq;
        q[i] = on ? (below ? ph[i] : ph[i + 1]) : -1;
        w[i] = on ? (below ? words[i] : words[i + 1]) : 0u;
    }
    const Entry<TT> *adj = (hdr & 15) == kDirOut ? p.g.out_adj : p.g.in_adj;
    // loads per step (measured: 8 for trees up to depth 4, 4 deeper)
    constexpr int kLU = D <= 4 ? 8 : 4;
    auto count = [&](uint32_t n, uint32_t j, bool move) -> uint32_t {
        uint32_t c = 0;
        if constexpr (NQ >= 1) if (nqm == 1) c = leaf_count<kLU, 1>(adj, l0, n, q, w, gb.w, cnt, nd, j, move);
        if constexpr (NQ >= 2) if (nqm == 2) c = leaf_count<kLU, 2>(adj, l0, n, q, w, gb.w, cnt, nd, j, move);
        if constexpr (NQ >= 3) if (nqm == 3) c = leaf_count<kLU, 3>(adj, l0, n, q, w, gb.w, cnt, nd, j, move);
        if constexpr (NQ >= 4) if (nqm == 4) c = leaf_count<kLU, 4>(adj, l0, n, q, w, gb.w, cnt, nd, j, move);
        if constexpr (NQ >= 5) if (nqm == 5) c = leaf_count<kLU, 5>(adj, l0, n, q, w, gb.w, cnt, nd, j, move);
        return c;
    };
    // the whole window counts at the largest window
    const uint32_t c = count(len, nd - 1, false);
    if constexpr (!single_of(MODE)) {
        // each smaller window is a prefix of this one: its matches move down
        // one slot (usually it is empty)
        const TT *ta = times_of(adj);
        uint32_t e = l0 + len;
        for (uint32_t j = nd - 1; j-- > 0;) {
            e = gallop_greater(ta, 1, l0, e, sat_add(tf, window_lo(p, j)));
            if (e == l0) break;
            count(e - l0, j, true);
        }
    }
    return c;
}

// The number of bound vertices a lane compares in count_leaf_window (0 when it
// counts nothing), maximised over the lanes that run this together.
template <int S>
__device__ __forceinline__ uint32_t leaf_compares(bool counting, uint32_t hdr) {
    const uint32_t nq = counting ? ((hdr >> 8) & 15) - 1u : 0u;
    uint32_t nqm = 0;
#pragma unroll
    for (int k = 1; k < S; ++k) nqm += __ballot(nq >= (uint32_t)k) ? 1u : 0u;
    return nqm;
}

// A partial match at level L whose trie node has leaf children only (every
// match below it is one more edge), counted by the lane that found it, with
// no level buffer: the lane finds and counts the window of each of the node's
// groups in turn.  A window longer than p.leaf_scan entries is left to the
// whole wave, which counts such windows between the lanes' turns.  ph[]: the
// bound vertices, eid and tp: its last edge and that edge's time, tf: its
// first time, r1: its root's slot in the level-1 batch (root windows).
template <typename TT, int D, int MODE, int S>
__device__ __forceinline__ void count_leaf_parent(const KParams<TT> &p,
                                                  WaveLds<TT, D, keep_of(MODE)> &W,
                                                  unsigned long long *cnt, const int lane,
                                                  bool act, uint32_t node,
                                                  const int32_t (&ph)[S], uint32_t eid, TT tp,
                                                  TT tf, uint32_t r1, uint32_t nd) {
    const uint32_t iw = act ? p.tree.inode[node] : 0u;
    uint32_t gi = iw & 0xfffffu;
    const uint32_t gend = gi + (act ? node_groups(iw) : 0u);
    const TT thi = sat_add(tf, p.delta_sat);
    for (;;) {
        bool pend = false;     // a window for the whole wave: group pg, [pl0, pl0 + plen)
        uint32_t pg = 0, pl0 = 0, plen = 0;
        while (gi < gend) {
            const uint32_t g = gi;
            const uint32_t hdr = p.tree.grp[2 * g].x;
            const uint32_t dir = hdr & 15, anc = (hdr >> 4) & 15;
            // The out-list of a later vertex x whose children all end on a root
            // vertex (a or b; no new vertex): the edges x -> a and x -> b in the
            // window are also the entries equal to x in the windows of in(a)
            // and in(b), suffixes of the root's own windows.  Those are
            // counted instead when they are shorter than x's window.
            bool swap = false;
            uint32_t sw_lo[2] = {0, 0}, sw_hi[2] = {0, 0}, sw_word[2] = {0, 0}, sw_len = 0;
            int32_t sw_x = 0;
            if constexpr (single_of(MODE) && D == 3) {   // (measured slower for deeper trees)
                if (dir == kDirOut && anc >= 2) {
                    const uint4 ga = p.tree.grp[2 * g], gb = p.tree.grp[2 * g + 1];
                    if ((gb.w | ga.w | gb.x | gb.y | gb.z) == 0) {
                        const uint32_t hla = W.hlen[1][r1], hlb = W.hlen[3][r1];
                        const bool oka = ga.y == 0 || (hla != kNoHint && hla != kLongHint);
                        const bool okb = ga.z == 0 || (hlb != kNoHint && hlb != kLongHint);
                        if (oka && okb) {
                            swap = true;
#pragma unroll
                            for (int t = 0; t < S; ++t) sw_x |= ph[t] & -(int32_t)(anc == (uint32_t)t);
                            const TT *tin = times_of(p.g.in_adj);
#pragma unroll
                            for (int sv = 0; sv < 2; ++sv) {
                                sw_word[sv] = sv ? ga.z : ga.y;
                                if (!sw_word[sv]) continue;
                                const uint32_t k = 2u * (uint32_t)sv + 1u;   // in(a), in(b)
                                const uint32_t hb = W.hlo[k][r1];
                                sw_hi[sv] = hb + (sv ? hlb : hla);
                                sw_lo[sv] = first_greater(tin, 1, hb, sw_hi[sv], tp);
                                sw_len += sw_hi[sv] - sw_lo[sv];
                            }
                        }
                    }
                }
            }
            auto count_swapped = [&]() {
                constexpr int kLU = D <= 4 ? 8 : 4;
#pragma unroll
                for (int sv = 0; sv < 2; ++sv) {
                    if (sw_hi[sv] > sw_lo[sv]) {
                        const int32_t q1[1] = {sw_x};
                        const uint32_t w1[1] = {sw_word[sv]};
                        leaf_count<kLU, 1>(p.g.in_adj, sw_lo[sv], sw_hi[sv] - sw_lo[sv], q1, w1, 0u,
                                           cnt, 1u, 0u);
                    }
                }
            };
            if (swap && sw_len <= 16u) {   // short enough whatever x's window is
                count_swapped();
                ++gi;
                continue;
            }
            const Entry<TT> *adj = dir == kDirOut ? p.g.out_adj : p.g.in_adj;
            const TT *ta = times_of(adj);
            uint32_t b = 0, e = 0, l0;
            bool hinted = false, whole = true;   // whole: [b, e) is the anchor's list
            if constexpr (D > 2) {
                if (anc < 2) {
                    // a root vertex's list: the window ends where the root's does
                    const uint32_t k = anc * 2u + dir;
                    const uint32_t hl = W.hlen[k][r1];
                    hinted = hl != kNoHint;
                    whole = !hinted || hl == kLongHint;
                    b = W.hlo[k][r1];
                    e = hl == kLongHint ? b : b + hl;
                }
            }
            if (whole) {
                // the anchor's vertex by masks: a select chain over ph[]
                // would be turned into an indexed load from scratch memory
                int32_t a = 0;
#pragma unroll
                for (int t = 0; t < S; ++t) a |= ph[t] & -(int32_t)(anc == (uint32_t)t);
                const uint32_t *off = dir == kDirOut ? p.g.out_off : p.g.in_off;
                const uint32_t end = e;
                b = off[a];
                e = hinted ? end : off[a + 1];
            }
            const uint32_t le = (hdr >> 13) & 3u;
            if (le) {
                // the list of an endpoint of the last edge: its rank is kept
                const uint32_t k = (le == 1 ? 0u : 2u) + (dir == kDirOut ? 0u : 1u);
                l0 = reinterpret_cast<const uint32_t *>(p.g.gx)[4 * (size_t)eid + k];
            } else {
                l0 = first_greater(ta, 1, b, e, tp);
            }
            const uint32_t len = (hinted ? e : gallop_greater(ta, 1, l0, e, thi)) - l0;
            if (swap && sw_len < len) {
                count_swapped();
                ++gi;
                continue;
            }
            if (len > p.leaf_scan) {
                pend = true; pg = g; pl0 = l0; plen = len;
                break;
            }
            const uint32_t nqm = leaf_compares<S>(len > 0, hdr);
            if (len > 0) count_leaf_window<TT, D, MODE>(p, g, hdr, ph, tf, l0, len, nqm, cnt, nd);
            ++gi;
        }
        for (uint64_t cm = __ballot(pend); cm; cm &= cm - 1) {
            const int src = (int)__builtin_ctzll(cm);
            int32_t wph[S];
#pragma unroll
            for (int t = 0; t < S; ++t) wph[t] = (int32_t)__builtin_amdgcn_readlane(ph[t], src);
            const uint32_t wg = __builtin_amdgcn_readlane(pg, src);
            const uint32_t wl0 = __builtin_amdgcn_readlane(pl0, src);
            const uint32_t wlen = __builtin_amdgcn_readlane(plen, src);
            if (nd == 1)
                leaf_scan_wave<TT, S>(p, wph, wg, wl0, wlen, lane, cnt, 1u, 0u);
            else
                leaf_scan_wave_multi<TT, S>(p, wph, wg, wl0, wlen,
                                            lane_time(tf, src), lane, cnt, nd);
        }
        if (pend) ++gi;
        if (!__ballot(gi < gend)) break;
    }
}

// per-lane statistics (only the STATS instantiation touches them)
struct Stats {
    uint64_t v[kStats];
    bool dumped;   // the wave wrote contexts (an epoch ended): claim no more work
};

// MODE: 0 plain search (trees with one window), 1 with search statistics, 2
// with the per-root cost log, 3 plain search of a tree with several windows,
// 4 enumeration (every match written out), 5 and 6: 0 and 3 with epochs
// At level 1 with nparts > 1 (one buffered root), only part `part` of the
// root's candidates is expanded: [T * part / nparts, T * (part + 1) / nparts)
// of its T candidates in window order, so that the parts of one root
// partition its search exactly; windows that a single lane counts, and the
// root's window statistics, belong to part 0.
template <typename TT, int D, int MODE, int L>
__device__ __forceinline__ void run_level(const KParams<TT> &p, WaveLds<TT, D, keep_of(MODE)> &W,
                                          unsigned long long *cnt, const int lane,
                                          const uint32_t nA, Stats &st, const uint32_t part = 0,
                                          const uint32_t nparts = 1,
                                          const EpochCtx *ctx = nullptr) {
    constexpr bool STATS = MODE == 1, LOG = MODE == 2;
    auto &A = lvl<L>(W.lv);
    constexpr int SA = vslots(D, L);
    auto &R1 = lvl<1>(W.lv);
    // graph vertex of motif vertex s, and t_first, of buffered partial match i
    auto vtx = [&](uint32_t s, uint32_t i) -> int32_t {
        if constexpr (L == 1) return A.phi[s][i];
        else return s < 2 ? R1.phi[s][A.r1[i]] : A.phi[s < 2 ? 0 : s - 2][i];
    };
    auto tfirst_of = [&](uint32_t i) -> TT {
        if constexpr (L == 1) return A.tfirst[i];
        else return R1.tfirst[A.r1[i]];
    };
    const uint32_t *__restrict__ inode = p.tree.inode;
    const uint4 *__restrict__ grp = p.tree.grp;
    const uint64_t le_mask = (lane == 63) ? ~0ull : ((2ull << lane) - 1);
    // windows counted at once (MODE 0 serves trees with one window only)
    const uint32_t nd = single_of(MODE) ? 1u : (uint32_t)p.tree.n_d;

    if constexpr (plain_of(MODE) && L > 1 && D <= 4) {
        // a batch of leaf parents only (every match below is one more edge):
        // one lane per partial match finds and counts all of its windows
        // (measured faster for trees of up to four edges, slower for five)
        if (p.leaf_scan != 0) {
            bool mixed = false;
            for (uint32_t x0 = 0; x0 < nA; x0 += kWave) {
                const uint32_t x = x0 + lane;
                if (x < nA) mixed = mixed || (inode[A.node[x]] & kLeafParent) == 0;
            }
            if (!__ballot(mixed)) {
                for (uint32_t x0 = 0; x0 < nA; x0 += kWave) {
                    const uint32_t x = x0 + lane;
                    const bool act = x < nA;
                    int32_t ph[SA];
                    uint32_t node = 0, eid = 0, r1 = 0;
                    TT tp = 0, tf = 0;
#pragma unroll
                    for (int t = 0; t < SA; ++t) ph[t] = act ? vtx(t, x) : -1;
                    if (act) {
                        node = A.node[x];
                        eid = A.eid[x];
                        tp = p.g.gt[eid];
                        tf = tfirst_of(x);
                        r1 = A.r1[x];
                    }
                    count_leaf_parent<TT, D, MODE, SA>(p, W, cnt, lane, act, node, ph, eid, tp, tf,
                                                       r1, nd);
                }
                return;
            }
        }
    }


    // child groups per buffered partial match -> inclusive prefix (at the
    // root level every entry has the root's groups).  Below it the pairs are
    // taken in two classes: groups on a list of motif vertex 0 or 1 (windows
    // found inside the root's windows: short bisections) first, then the
    // others, so that the lanes of one pass do bisections of similar length
    // (pairs are numbered over both classes: the first P0 are of the first, so
    // only the pass across the boundary mixes them).
    uint32_t P = 0, P0 = 0, P1 = 0;
    const uint32_t root_ng = node_groups(inode[0]);
    if constexpr (L == 1) {
        P = ctx ? nA : nA * root_ng;   // a context is one window of its root
    } else {
        for (uint32_t x0 = 0; x0 < nA; x0 += kWave) {
            const uint32_t x = x0 + lane;
            uint32_t n0 = 0, n1 = 0;
            if (x < nA) {
                const uint32_t w = inode[A.node[x]];
                n0 = node_near(w);
                n1 = node_groups(w) - n0;
            }
            const uint32_t i0 = incl_scan32(n0, lane) + P0;
            const uint32_t i1 = incl_scan32(n1, lane) + P1;
            if (x < nA) {
                A.pincl[x] = (uint16_t)i0;
                A.pincl1[x] = (uint16_t)i1;
            }
            P0 = lane_value(i0, kWave - 1);
            P1 = lane_value(i1, kWave - 1);
        }
        P = P0 + P1;
        wave_sync();
    }

    // window chunk: lane w < nw holds non-empty window w
    //   wrec = {entry | group << 8, first list index, exclusive start, inclusive end}
    uint4 wrec = make_uint4(0, 0, 0, 0);
    uint32_t pc = 0, nw = 0, T = 0, cc = 0;
    uint32_t nB = 0;   // partial matches buffered at level L+1
    // epochs: root-level candidates are written out as contexts instead of
    // expanded once enough waves are idle (polled every 16 passes)
    bool dumping = false, room = true;
    uint32_t polls = 0, used = 0;   // contexts this wave wrote (at most its share of ctx_cap)

    for (;;) {
        bool done = false;
        if constexpr (L == 1 && epochs_of(MODE)) {
            // (a wave dumps in one batch at most: the later batches of its
            // chunk search on)
            if (p.ctx_out && room && !dumping && !st.dumped && (++polls & 15u) == 0) {
                uint32_t v = 0;
                if (lane == 0) v = __hip_atomic_load(p.idle, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t waves = gridDim.x * (uint32_t)kWavesPerBlock;
                dumping = (uint64_t)lane_value(v, 0) * 100u >= (uint64_t)p.idle_pct * waves;
            }
        }
        if (cc >= T) {
            if (pc >= P) {
                done = true;
            } else {
                // one (partial match, group) pair per lane -> its window
                const uint32_t pi = pc + lane;
                uint32_t len = 0, x = 0, g = 0, l0 = 0, hdr = 0;
                bool all = false;
                if (pi < P) {
                    uint32_t lo = 0;
                    bool given = false;   // the window comes with a context
                    if constexpr (L == 1) {
                        if (ctx) {
                            const EpochCtx c = ctx[pi];
                            lo = pi;
                            g = c.g;
                            l0 = c.e0;
                            len = c.e1 - c.e0;
                            given = true;
                        } else {
                            lo = pi / root_ng;
                            g = (inode[0] & 0xfffffu) + (pi - lo * root_ng);
                        }
                    } else {
                        const bool c1 = pi >= P0;   // second class
                        const uint32_t pj = c1 ? pi - P0 : pi;
                        const uint16_t *pin = c1 ? A.pincl1 : A.pincl;
                        uint32_t n = nA;
                        while (n > 0) {
                            const uint32_t h = n >> 1;
                            if (pin[lo + h] <= pj) { lo += h + 1; n -= h + 1; }
                            else n = h;
                        }
                        const uint32_t before = lo ? pin[lo - 1] : 0u;
                        const uint32_t w = inode[A.node[lo]];
                        g = (w & 0xfffffu) + (c1 ? node_near(w) : 0u) + (pj - before);
                    }
                    x = lo;
                    hdr = grp[2 * g].x;
                    if (given) {
                        all = (hdr & 15) == kDirAll;
                    } else {
                        const int dir = hdr & 15, anc = (hdr >> 4) & 15;
                        const TT thi = sat_add(tfirst_of(lo), p.delta_sat);
                        uint32_t b, e, sh;
                        const TT *ta;
                        bool hinted = false, known = false;
                        if (dir == kDirAll) {
                            b = 0; e = p.g.n_edges; ta = p.g.gt; sh = 0;
                            all = true;
                            if constexpr (L > 1) {
                                // the whole-list window starts after the last edge
                                // itself (past the entries with its time)
                                b = A.eid[lo] + 1u;
                            }
                        } else {
                            ta = times_of(dir == kDirOut ? p.g.out_adj : p.g.in_adj);
                            sh = 1;
                            bool whole = true;   // [b, e) is the anchor's whole list
                            if constexpr (L > 1 && D > 2) {
                                if (anc < 2) {
                                    const uint32_t k = (uint32_t)anc * 2u + (uint32_t)dir;
                                    const uint32_t r1 = A.r1[lo];
                                    const uint32_t hl = W.hlen[k][r1];
                                    hinted = hl != kNoHint;
                                    whole = !hinted || hl == kLongHint;
                                    b = W.hlo[k][r1];
                                    e = hl == kLongHint ? b : b + hl;
                                }
                            }
                            if (whole) {
                                const int32_t a = vtx((uint32_t)anc, lo);
                                const uint32_t *off = dir == kDirOut ? p.g.out_off : p.g.in_off;
                                const uint32_t end = e;
                                b = off[a];
                                e = hinted ? end : off[a + 1];
                            }
                            if constexpr (L == 1) {
                                // the root edge's own entries: its windows start at
                                // the first entry after its time (set with the root)
                                l0 = W.hlo[(uint32_t)anc * 2u + (uint32_t)dir][lo];
                                known = true;
                            } else {
                                // an anchor on the last matched edge: the window
                                // starts where that edge's time ends in its list
                                const uint32_t le = (hdr >> 13) & 3u;
                                if (le) {
                                    const uint4 gx = p.g.gx[A.eid[lo]];
                                    l0 = le == 1 ? (dir == kDirOut ? gx.x : gx.y)
                                                 : (dir == kDirOut ? gx.z : gx.w);
                                    known = true;
                                }
                            }
                        }
                        if (!known) {
                            TT tp;
                            if constexpr (L == 1) tp = A.tfirst[lo];
                            else tp = p.g.gt[A.eid[lo]];
                            l0 = all && L > 1 ? gallop_greater(ta, sh, b, e, tp)
                                              : first_greater(ta, sh, b, e, tp);
                        }
                        len = (hinted ? e : gallop_greater(ta, sh, l0, e, thi)) - l0;
                        if constexpr (L == 1 && D > 2) {
                            if (!all && anc < 2) {
                                const uint32_t k = (uint32_t)anc * 2u + (uint32_t)dir;
                                // a long window keeps its end, the list's start
                                // then bounds the deeper bisections
                                const bool lng = len >= kLongHint;
                                W.hlo[k][lo] = lng ? l0 + len : l0;
                                W.hlen[k][lo] = lng ? kLongHint : (uint16_t)len;
                            }
                        }
                    }
                }
                // take the longest prefix of pairs whose candidates stay below 2^31
                // (always all of them when every window is under 2^25 entries;
                // 32-bit sums are exact unless some window has 2^26 entries)
                bool take = pi < P;
                if (__ballot(len >= (1u << 25))) {
                    const uint64_t incl64 = __ballot(len >= (1u << 26))
                                                ? incl_scan64((uint64_t)len, lane)
                                                : (uint64_t)incl_scan32(len, lane);
                    take = take && incl64 <= kChunkLimit;
                }
                pc += uniform((uint32_t)__popcll(__ballot(take)));
                const bool own = part == 0;   // this part keeps the per-window work
                if constexpr (STATS) {
                    if (take && own) {
                        st.v[all ? kStatWinAll : kStatWinList] += 1;
                        st.v[all ? kStatEntAll : kStatEntList] += len;
                    }
                }
                if constexpr (LOG) {
                    if (take && own && len > 0)
                        atomicAdd(&p.root_cost[A.root[x]], (unsigned long long)len);
                }
                // a window whose children are all leaves is counted without
                // the candidate expansion: a short one by its own lane, a long
                // one by the whole wave
                const bool leaf = take && len > 0 && p.leaf_scan && ((hdr >> 12) & 1);
                const bool scanned = leaf && len <= p.leaf_scan;
                const bool coop = leaf && len > p.leaf_scan;
                const uint32_t nqm = leaf_compares<SA>(scanned && own, hdr);
                if (scanned && own) {
                    int32_t ph[SA];
#pragma unroll
                    for (int t = 0; t < SA; ++t) ph[t] = vtx(t, x);
                    const uint32_t c = count_leaf_window<TT, D, MODE>(p, g, hdr, ph, tfirst_of(x),
                                                                      l0, len, nqm, cnt, nd);
                    if constexpr (STATS) st.v[kStatCredit] += c;
                }
                for (uint64_t cm = __ballot(coop && own); cm; cm &= cm - 1) {
                    const int src = (int)__builtin_ctzll(cm);
                    const uint32_t wx = __builtin_amdgcn_readlane(x, src);
                    int32_t wph[SA];
#pragma unroll
                    for (int t = 0; t < SA; ++t) wph[t] = (int32_t)uniform((uint32_t)vtx(t, wx));
                    const uint32_t wg = __builtin_amdgcn_readlane(g, src);
                    const uint32_t wl0 = __builtin_amdgcn_readlane(l0, src);
                    const uint32_t wlen = __builtin_amdgcn_readlane(len, src);
                    uint32_t c;
                    if (nd == 1)
                        c = leaf_scan_wave<TT, SA>(p, wph, wg, wl0, wlen, lane, cnt, 1u, 0u);
                    else
                        c = leaf_scan_wave_multi<TT, SA>(p, wph, wg, wl0, wlen, tfirst_of(wx), lane,
                                                         cnt, nd);
                    if constexpr (STATS) st.v[kStatCredit] += c;
                }
                // compact the other non-empty windows into lanes 0..nw-1; their
                // candidate ranges are numbered without the leaf-counted ones
                // (the chunk total stays below the limit checked above)
                const bool keep = take && len > 0 && !leaf;
                const uint64_t km = __ballot(keep);
                nw = uniform((uint32_t)__popcll(km));
                wrec = make_uint4(0, 0, 0, 0);
                T = 0;
                if (nw) {
                    const uint32_t lk = keep ? len : 0u;
                    const uint32_t incl = incl_scan32(lk, lane);
                    if (keep) W.src[mbcnt(km)] = (uint8_t)lane;
                    wave_sync();
                    const int from = (uint32_t)lane < nw ? (int)W.src[lane] : lane;
                    wave_sync();
                    wrec.x = __shfl(x | (g << 8), from);
                    wrec.y = __shfl(l0, from);
                    wrec.z = __shfl(incl - lk, from);
                    wrec.w = __shfl(incl, from);
                    if ((uint32_t)lane >= nw) wrec = make_uint4(0, 0, 0, 0);
                    T = lane_value(wrec.w, nw - 1);
                }
                cc = 0;
                if (L == 1 && nparts > 1) {
                    // one root, so every window fits this one chunk
                    cc = (uint32_t)(((uint64_t)T * part) / nparts);
                    T = (uint32_t)(((uint64_t)T * (part + 1)) / nparts);
                }
            }
        }
        if constexpr (L == 1 && epochs_of(MODE)) {
            if (!done && cc < T && dumping) {
                // write what is left of this chunk's windows as contexts of at
                // most kCtxPiece candidates each (candidates [cc, T) in window
                // order; lane w < nw holds window w)
                uint32_t c_lo = 0, c_hi = 0;
                if ((uint32_t)lane < nw) {
                    c_lo = max(cc, wrec.z);
                    c_hi = wrec.w;
                }
                const uint32_t n = c_hi > c_lo ? (c_hi - c_lo + kCtxPiece - 1) / kCtxPiece : 0u;
                const uint32_t incl = incl_scan32(n, lane);
                const uint32_t tot = lane_value(incl, kWave - 1);
                // every wave may write its share of the buffer, so one atomic
                // add takes the slots and the buffer never overflows
                const uint64_t share = p.ctx_cap / ((uint64_t)gridDim.x * kWavesPerBlock);
                if ((uint64_t)used + tot <= share) {
                    unsigned long long base = 0;
                    if (lane == 0 && tot) base = atomicAdd(p.ctx_count, (unsigned long long)tot);
                    base = lane0_u64(base);
                    used += tot;
                    if (n) {
                        const uint32_t ox = wrec.x & 255, og = wrec.x >> 8;
                        const uint64_t tf = (uint64_t)tfirst_of(ox);
                        EpochCtx c;
                        c.a = vtx(0, ox);
                        c.b = vtx(1, ox);
                        c.t_lo = (uint32_t)tf;
                        c.t_hi = (uint32_t)(tf >> 32);
                        c.g = og;
                        c.pad = 0;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            c.hlo[k] = D > 2 ? W.hlo[k][ox] : 0u;
                            c.hlen[k] = D > 2 ? W.hlen[k][ox] : kNoHint;
                        }
                        c.pad2[0] = c.pad2[1] = 0;
                        const unsigned long long slot = base + (incl - n);
                        for (uint32_t k = 0; k < n; ++k) {
                            const uint32_t c0 = c_lo + k * kCtxPiece;
                            const uint32_t c1 = min(c0 + kCtxPiece, c_hi);
                            c.e0 = wrec.y + (c0 - wrec.z);
                            c.e1 = wrec.y + (c1 - wrec.z);
                            p.ctx_out[slot + k] = c;
                        }
                    }
                    cc = T;
                } else {
                    dumping = false;   // its share is used up: this wave searches on
                    room = false;
                }
            }
        }
        if (!done && cc < T) {
            const uint32_t f = cc + lane;
            // owner window = number of windows that end at or before f
            const uint32_t o0 = (uint32_t)__popcll(__ballot((uint32_t)lane < nw && wrec.w <= cc));
            if ((uint32_t)lane < nw && wrec.w > cc && wrec.w - cc < (uint32_t)kWave)
                W.flag[wrec.w - cc] = 1;
            wave_sync();
            const uint32_t fl = W.flag[lane];
            W.flag[lane] = 0;
            const uint64_t ends = __ballot(fl != 0);
            wave_sync();
            const int oi = (int)((o0 + (uint32_t)__popcll(ends & le_mask)) & 63);
            const uint32_t oxg = __shfl(wrec.x, oi);
            const uint32_t olo = __shfl(wrec.y, oi);
            const uint32_t oex = __shfl(wrec.z, oi);
            const bool valid = f < T;
            const uint32_t ox = oxg & 255, og = oxg >> 8;
            const uint32_t ei = olo + (f - oex);

            uint32_t cw = 0;      // child word reached by this candidate
            TT tn = 0;            // its time
            int dir = 0;
            uint32_t nvp = 0;
            int32_t nv0 = -1, nv1 = -1;
            int32_t ph[SA];
#pragma unroll
            for (int s = 0; s < SA; ++s) ph[s] = 0;
            uint4 ga = make_uint4(0, 0, 0, 0), gb = ga;
            if (valid) {
                ga = grp[2 * og];
                gb = grp[2 * og + 1];
                dir = ga.x & 15;
                nvp = (ga.x >> 8) & 15;
#pragma unroll
                for (int s = 0; s < SA; ++s) ph[s] = vtx(s, ox);
                if (dir != kDirAll) {
                    const Entry<TT> *adj = dir == kDirOut ? p.g.out_adj : p.g.in_adj;
                    const Entry<TT> en = adj[ei];   // one load: vertex and time
                    const int32_t v = en.v;
                    tn = en.t;
                    int y = -1;
#pragma unroll
                    for (int s = 0; s < SA; ++s) y = ((uint32_t)s < nvp && ph[s] == v) ? s : y;
                    // in-groups have no bound-target children, so their words are 0
                    cw = child_word(ga, gb, y);
                    nv0 = v;
                }
            }
            if (__ballot(valid && dir == kDirAll)) {
                if (valid && dir == kDirAll) {
                    const int32_t cs = p.g.gsrc[ei], cd = p.g.gdst[ei];
                    bool hit = cs == cd;
#pragma unroll
                    for (int s = 0; s < SA; ++s)
                        hit |= ((uint32_t)s < nvp && (ph[s] == cs || ph[s] == cd));
                    cw = hit ? 0u : gb.w;
                    nv0 = cs;
                    nv1 = cd;
                    tn = p.g.gt[ei];
                }
            }
            if (cw) {
                const uint32_t q1 = (cw >> 16) & 0x7fffu;
                if (q1) {
                    const uint32_t j = nd > 1 ? window_slot(p, nd, tfirst_of(ox), tn) : 0u;
                    atomicAdd(&cnt[(q1 - 1) * nd + j], 1ull);
                }
                if constexpr (STATS) st.v[kStatCredit] += 1;
            }
            // the edge id of this candidate (pushed along, and written out
            // when enumerating), read only where it is used
            auto cand_eid = [&]() -> uint32_t {
                return dir == kDirAll ? ei : (dir == kDirOut ? p.g.out_eid : p.g.in_eid)[ei];
            };
            if constexpr (MODE == 4) {
                const uint32_t q1 = (cw >> 16) & 0x7fffu;
                uint32_t e[kKMax] = {0, 0, 0, 0, 0};
                edge_chain<L>(W, ox, e);
                e[L] = valid ? cand_eid() : 0u;
                write_matches(p, valid && cw && q1, q1 - 1u, e, L + 1);
            }
            if constexpr (L + 1 < D) {
                auto &B = lvl<L + 1>(W.lv);
                constexpr int SB = vslots(D, L + 1);
                const bool push = (cw >> 31) != 0;
                const uint64_t pm = __ballot(push);
                if (push) {
                    const uint32_t slot = nB + mbcnt(pm);
#pragma unroll
                    for (int s = 2; s < SB; ++s) {
                        int32_t v = (s < SA) ? ph[s < SA ? s : 0] : -1;
                        v = ((uint32_t)s < nvp) ? v
                            : ((uint32_t)s == nvp ? nv0 : ((uint32_t)s == nvp + 1 ? nv1 : -1));
                        B.phi[s - 2][slot] = v;
                    }
                    B.eid[slot] = cand_eid();
                    B.node[slot] = (uint16_t)(cw & 0xffffu);
                    if constexpr (L == 1) B.r1[slot] = (uint8_t)ox;
                    else B.r1[slot] = A.r1[ox];
                    if constexpr (keep_of(MODE) > 0) B.root[slot] = A.root[ox];
                    if constexpr (keep_of(MODE) == 2 && L > 1) B.par[slot] = (uint8_t)ox;
                    if constexpr (STATS) st.v[kStatPush] += 1;
                }
                nB += (uint32_t)__popcll(pm);
            }
            cc += kWave;
        }
        if constexpr (L + 1 < D) {
            if (nB >= kWave || (done && nB > 0)) {
                wave_sync();
                run_level<TT, D, MODE, L + 1>(p, W, cnt, lane, nB, st);
                wave_sync();
                nB = 0;
            }
        }
        if (done) break;
    }
    if constexpr (L == 1) {
        if (dumping) st.dumped = true;
    }
}

// Search from part `part` of `nparts` of the root at position r (an edge id:
// split items come only with p.roots NULL); part 0 credits the root itself.
template <typename TT, int D, int MODE>
__device__ __forceinline__ void process_root_part(const KParams<TT> &p,
                                                  WaveLds<TT, D, keep_of(MODE)> &W,
                                                  unsigned long long *cnt, const int lane,
                                                  const uint32_t r, const uint32_t part,
                                                  const uint32_t nparts, Stats &st) {
    constexpr bool STATS = MODE == 1, LOG = MODE == 2;
    const int32_t s = p.g.gsrc[r], d = p.g.gdst[r];
    if (s == d) return;
    if (part == 0) {
        if (p.tree.root_q >= 0 && lane == 0) atomicAdd(&cnt[p.tree.root_q * p.tree.n_d], 1ull);
        if constexpr (STATS) st.v[kStatRoots] += lane == 0 ? 1 : 0;
        if constexpr (LOG) {
            if (lane == 0) atomicAdd(&p.root_cost[r], 1ull);
        }
    }
    if constexpr (D > 1) {
        auto &A = lvl<1>(W.lv);
        if (lane == 0) {
            A.phi[0][0] = s;
            A.phi[1][0] = d;
            A.tfirst[0] = p.g.gt[r];
            set_root_slot(W, 0, p.g.gx[r]);
            if constexpr (keep_of(MODE) > 0) A.root[0] = r;
        }
        wave_sync();
        run_level<TT, D, MODE, 1>(p, W, cnt, lane, 1u, st, part, nparts);
        wave_sync();
    }
}

// Search from roots [base, end) of the root list (positions, or edge ids when
// p.roots is NULL), 64 at a time.
template <typename TT, int D, int MODE>
__device__ __forceinline__ void process_roots(const KParams<TT> &p,
                                              WaveLds<TT, D, keep_of(MODE)> &W,
                                              unsigned long long *cnt, const int lane,
                                              const uint32_t base, const uint32_t end,
                                              Stats &st) {
    constexpr bool STATS = MODE == 1, LOG = MODE == 2;
    for (uint32_t b = base; b < end; b += kWave) {
        const uint32_t i = b + (uint32_t)lane;
        bool ok = i < end;
        uint32_t r = 0;
        int32_t s = 0, d = 0;
        if (ok) {
            r = p.roots ? p.roots[i] : i;
            s = p.g.gsrc[r];
            d = p.g.gdst[r];
            ok = s != d;
        }
        const uint64_t m = __ballot(ok);
        if (p.tree.root_q >= 0 && lane == 0 && m)
            atomicAdd(&cnt[p.tree.root_q * p.tree.n_d], (unsigned long long)__popcll(m));
        if constexpr (MODE == 4) {
            if (p.tree.root_q >= 0) {
                uint32_t e[kKMax] = {r, 0, 0, 0, 0};
                write_matches(p, ok, (uint32_t)p.tree.root_q, e, 1);
            }
        }
        if constexpr (STATS) st.v[kStatRoots] += ok ? 1 : 0;
        if constexpr (LOG) {
            if (ok) atomicAdd(&p.root_cost[r], 1ull);
        }
        if constexpr (D > 1) {
            auto &A = lvl<1>(W.lv);
            if (ok) {
                const uint32_t slot = mbcnt(m);
                A.phi[0][slot] = s;
                A.phi[1][slot] = d;
                A.tfirst[slot] = p.g.gt[r];
                set_root_slot(W, slot, p.g.gx[r]);
                if constexpr (keep_of(MODE) > 0) A.root[slot] = r;
            }
            const uint32_t n1 = uniform((uint32_t)__popcll(m));
            if (n1 > 0) {
                wave_sync();
                run_level<TT, D, MODE, 1>(p, W, cnt, lane, n1, st);
                wave_sync();
            }
        }
    }
}

// Search contexts [base, end) of p.ctx_in (at most 64): each becomes a
// root in the level-1 batch, with its window and its root windows given.
template <typename TT, int D, int MODE>
__device__ __forceinline__ void process_contexts(const KParams<TT> &p,
                                                 WaveLds<TT, D, keep_of(MODE)> &W,
                                                 unsigned long long *cnt, const int lane,
                                                 const uint32_t base, const uint32_t end,
                                                 Stats &st) {
    if constexpr (D > 1) {
        auto &A = lvl<1>(W.lv);
        const uint32_t i = base + (uint32_t)lane;
        if (i < end) {
            const EpochCtx c = p.ctx_in[i];
            A.phi[0][lane] = c.a;
            A.phi[1][lane] = c.b;
            A.tfirst[lane] = (TT)(((uint64_t)c.t_hi << 32) | c.t_lo);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                W.hlo[k][lane] = c.hlo[k];
                W.hlen[k][lane] = c.hlen[k];
            }
        }
        wave_sync();
        run_level<TT, D, MODE, 1>(p, W, cnt, lane, end - base, st, 0, 1, p.ctx_in + base);
        wave_sync();
    }
}

// Up to depth 3 the plain search (MODE 0) fits 8 waves per SIMD (at most 64
// VGPRs and 96 SGPRs) without spilling in its loops, and the multi-window
// search (MODE 3) is faster there with a few spills than at 6 waves; the
// compiler is asked for that.  Deeper trees and the instrumented modes keep
// the compiler's own allocation.
template <int D, int MODE>
constexpr int min_waves_per_eu() { return D <= 3 && plain_of(MODE) ? 8 : 1; }

template <typename TT, int D, int MODE>
__global__ void __launch_bounds__(kWave * kWavesPerBlock)
__attribute__((amdgpu_waves_per_eu(min_waves_per_eu<D, MODE>(), 8)))
comine_kernel(const KParams<TT> p) {
    constexpr bool STATS = MODE == 1, LOG = MODE == 2;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(smem);
    const int32_t n_slots = counter_slots(p.tree);
    const size_t cnt_bytes = ((size_t)n_slots * 8 + 15) & ~(size_t)15;
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int wave = (int)(threadIdx.x / kWave);
    WaveLds<TT, D, keep_of(MODE)> &W = reinterpret_cast<WaveLds<TT, D, keep_of(MODE)> *>(smem + cnt_bytes)[wave];

    for (int i = (int)threadIdx.x; i < n_slots; i += (int)blockDim.x) cnt[i] = 0;
    W.flag[lane] = 0;
    __syncthreads();
    Stats st;
#pragma unroll
    for (int i = 0; i < kStats; ++i) st.v[i] = 0;
    st.dumped = false;
    // when each wave starts and ends its search (device real-time clock)
    const uint32_t clock_slot = blockIdx.x * kWavesPerBlock + (uint32_t)wave;
    if (p.wave_clock && lane == 0 && clock_slot < p.n_wave_clock)
        p.wave_clock[2 * clock_slot] = __builtin_amdgcn_s_memrealtime();

    if (p.items) {
        // scheduled work items first, claimed in order from their own queue
        const uint32_t n_items = uniform(*p.n_items);
        for (;;) {
            unsigned long long it = 0;
            if (lane == 0) it = atomicAdd(&p.queues[kItemSlot * kQueueStride], 1ull);
            it = lane0_u64(it);
            if (it >= n_items) break;
            const uint2 item = p.items[uniform((uint32_t)it)];
            const uint32_t iy = uniform(item.y);
            if (iy & kItemSplit)
                process_root_part<TT, D, MODE>(p, W, cnt, lane, uniform(item.x),
                                               (iy >> 15) & 0x7fffu, iy & 0x7fffu, st);
            else
                process_roots<TT, D, MODE>(p, W, cnt, lane, uniform(item.x), iy, st);
        }
    }
    bool from_ctx = false;
    if constexpr (epochs_of(MODE)) {
        if (p.ctx_in) {
            // a later epoch: the contexts the last one left, spread over every
            // wave (up to 64 at a time)
            from_ctx = true;
            const uint32_t waves = gridDim.x * (uint32_t)kWavesPerBlock;
            const uint32_t per = min((uint32_t)kWave, max(1u, (p.n_ctx_in + waves - 1) / waves));
            for (;;) {
                unsigned long long it = 0;
                if (lane == 0) it = atomicAdd(&p.queues[kItemSlot * kQueueStride], (unsigned long long)per);
                it = lane0_u64(it);
                if (it >= p.n_ctx_in) break;
                const uint32_t b0 = uniform((uint32_t)it);
                process_contexts<TT, D, MODE>(p, W, cnt, lane, b0, min(b0 + per, p.n_ctx_in), st);
                if (st.dumped) break;
            }
        }
    }
    if (!from_ctx) {
        // workgroups are dispatched to the XCDs round-robin: start on this XCD's
        // share of the roots, then take what is left of the others.  A chunk once
        // claimed is always searched to the end, so after a stop the queue heads
        // (clamped to the queue lengths) mark exactly the roots searched.
        const uint32_t nq = p.n_queues;
        const uint32_t home = blockIdx.x % nq;
        bool stopped = false;
        for (uint32_t qi = 0; qi < nq && !stopped; ++qi) {
            const uint32_t q = (home + qi) % nq;
            const uint32_t qbeg = queue_begin(p.n_roots, nq, q);
            const uint32_t qend = queue_end(p.n_roots, nq, q);
            for (;;) {
                unsigned long long got = 0;
                if (lane == 0) {
                    unsigned long long *head = &p.queues[q * kQueueStride];
                    if (p.stop && __hip_atomic_load(p.stop, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_SYSTEM) != 0) {
                        got = ~0ull;
                    } else if (p.max_chunks) {
                        // the budget is spent only on a queue that still has roots,
                        // so a call makes progress while any root is left: a
                        // budget holder's claim fails only when another holder
                        // took the last chunk
                        const unsigned long long h =
                            __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (h >= (unsigned long long)(qend - qbeg)) got = h;
                        else if (atomicAdd(&p.queues[kBudgetSlot * kQueueStride], 1ull) >= p.max_chunks)
                            got = ~0ull;
                        else got = atomicAdd(head, (unsigned long long)p.chunk);
                    } else {
                        got = atomicAdd(head, (unsigned long long)p.chunk);
                    }
                }
                got = lane0_u64(got);
                if (got == ~0ull) { stopped = true; break; }
                if (got >= (unsigned long long)(qend - qbeg)) break;
                const uint32_t base = uniform(qbeg + (uint32_t)got);
                if (p.skip && p.skip[base / kWave]) continue;   // searched as an item
                process_roots<TT, D, MODE>(p, W, cnt, lane, base, min(base + p.chunk, qend), st);
                if (st.dumped) { stopped = true; break; }   // an epoch ended
            }
        }

    }
    if constexpr (epochs_of(MODE)) {
        // out of work: an idle wave, for the epoch limit
        if (p.ctx_out && !st.dumped && lane == 0) atomicAdd(p.idle, 1u);
    }

    if (p.wave_clock && lane == 0 && clock_slot < p.n_wave_clock)
        p.wave_clock[2 * clock_slot + 1] = __builtin_amdgcn_s_memrealtime();
    if constexpr (STATS) {
#pragma unroll
        for (int i = 0; i < kStats; ++i)
            if (st.v[i]) atomicAdd(&p.stats[i], (unsigned long long)st.v[i]);
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < n_slots; i += (int)blockDim.x)
        if (cnt[i]) atomicAdd(&p.counts[i], cnt[i]);
}

// Many (graph, tree) jobs in one persistent launch.  Waves claim work items
// (root ranges of one job) from one queue; each wave keeps its own LDS
// counters, sized for the largest tree, and flushes them after every item.
template <typename TT, int D, int MODE>
__global__ void __launch_bounds__(kWave * kWavesPerBlock)
batch_kernel(const BatchParams<TT> bp) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int wave = (int)(threadIdx.x / kWave);
    const size_t cnt_bytes = ((size_t)bp.n_q_max * 8 + 15) & ~(size_t)15;
    unsigned char *mine = smem + (size_t)wave * (cnt_bytes + sizeof(WaveLds<TT, D, 0>));
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(mine);
    WaveLds<TT, D, 0> &W = *reinterpret_cast<WaveLds<TT, D, 0> *>(mine + cnt_bytes);
    W.flag[lane] = 0;
    Stats st;
    st.dumped = false;
    for (;;) {
        unsigned long long it = 0;
        if (lane == 0) it = atomicAdd(bp.cursor, 1ull);
        it = lane0_u64(it);
        if (it >= bp.n_items) break;
        const BatchItem item = bp.items[uniform((uint32_t)it)];
        const BatchJob<TT> &job = bp.jobs[uniform(item.job)];
        // the plain search keeps its own copy of the job's parameters (in
        // registers); the multi-window one reads them in place, since its
        // window selection would otherwise put a copy in scratch memory
        auto search = [&](const KParams<TT> &p) {
            const uint32_t ip = uniform(item.part);
            if (ip & kItemSplit)
                process_root_part<TT, D, MODE>(p, W, cnt, lane, uniform(item.begin),
                                               (ip >> 15) & 0x7fffu, ip & 0x7fffu, st);
            else
                process_roots<TT, D, MODE>(p, W, cnt, lane, uniform(item.begin), uniform(item.end),
                                           st);
        };
        const uint32_t nq = (uint32_t)counter_slots(job.p.tree);
        for (uint32_t i = (uint32_t)lane; i < nq; i += kWave) cnt[i] = 0;
        wave_sync();
        if constexpr (MODE == 0) {
            const KParams<TT> p = job.p;
            search(p);
        } else {
            search(job.p);
        }
        wave_sync();
        for (uint32_t i = (uint32_t)lane; i < nq; i += kWave)
            if (cnt[i]) atomicAdd(&bp.counts[job.count_off + i], cnt[i]);
        wave_sync();
    }
}


template <typename TT, int D, int MODE>
size_t smem_bytes(int n_q) {
    return (((size_t)n_q * 8 + 15) & ~(size_t)15) +
           (size_t)kWavesPerBlock * sizeof(WaveLds<TT, D, keep_of(MODE)>);
}

template <typename TT, int D, int MODE>
hipError_t launch_ds(const KParams<TT> &p, int blocks, hipStream_t stream) {
    const size_t sm = smem_bytes<TT, D, MODE>(counter_slots(p.tree));
    auto kern = comine_kernel<TT, D, MODE>;
    if (sm > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        if (e != hipSuccess) return e;
    }
    if (blocks <= 0) {
        int dev = 0, ncu = 0, per = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kWave * kWavesPerBlock, sm);
        if (e != hipSuccess) return e;
        blocks = ncu * (per > 0 ? per : 1);
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kWave * kWavesPerBlock), sm, stream, p);
    return hipGetLastError();
}

}  // namespace

template <typename TT, int D>
hipError_t launch_d(const KParams<TT> &p, int blocks, hipStream_t stream) {
    if (p.ctx_in || p.ctx_out)
        return p.tree.n_d > 1 ? launch_ds<TT, D, 6>(p, blocks, stream) : launch_ds<TT, D, 5>(p, blocks, stream);
    if (p.enum_out) return launch_ds<TT, D, 4>(p, blocks, stream);
    if (p.stats) return launch_ds<TT, D, 1>(p, blocks, stream);
    if (p.root_cost) return launch_ds<TT, D, 2>(p, blocks, stream);
    if (p.tree.n_d > 1) return launch_ds<TT, D, 3>(p, blocks, stream);
    return launch_ds<TT, D, 0>(p, blocks, stream);
}

template <typename TT, int D, int MODE>
hipError_t launch_batch_d(const BatchParams<TT> &bp, int blocks, hipStream_t stream) {
    const size_t sm = (size_t)kWavesPerBlock *
                      ((((size_t)bp.n_q_max * 8 + 15) & ~(size_t)15) + sizeof(WaveLds<TT, D, 0>));
    auto kern = batch_kernel<TT, D, MODE>;
    if (sm > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        if (e != hipSuccess) return e;
    }
    if (blocks <= 0) {
        int dev = 0, ncu = 0, per = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kWave * kWavesPerBlock, sm);
        if (e != hipSuccess) return e;
        blocks = ncu * (per > 0 ? per : 1);
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kWave * kWavesPerBlock), sm, stream, bp);
    return hipGetLastError();
}

}  // namespace mg
