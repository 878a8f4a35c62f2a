// Co-mining kernel for gfx950 (CDNA4, wave64).
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
//   * Every wave is an independent worker.  It grabs a chunk of root edges
//     from a global queue (work stealing), 64 roots per batch.
//   * Partial matches are buffered per search level in LDS.  For a batch of
//     partial matches at level L, every (partial match, child group) pair is
//     a window of one time-sorted adjacency list: the entries with
//     t_prev < t <= t_first + delta, found by bisection.  Children that read
//     the same list (same direction, same anchor vertex) form one group and
//     share one scan of the window.
//   * The wave expands up to 64 windows at a time as one flat candidate range:
//     lane i takes candidate c + i, finds its window by a binary search over
//     the lanes' inclusive prefix sums (cross-lane shuffles), reads one
//     adjacency entry, applies the structural test with predicated compares,
//     credits the reached node's motif in LDS counters, and compacts the
//     survivors that still have children into the next level's buffer with
//     ballot + mbcnt.
//   * When the next level's buffer holds 64 or more partial matches it is
//     expanded at once (depth first over batches), so LDS use is bounded by
//     the motif length, not by the size of the search tree.
//   * The level loop nest is unrolled at compile time for the tree depth
//     (1..5 motif edges), one instantiation per depth.
#include <hip/hip_runtime.h>

#include "comine.h"

namespace mg {
namespace {

constexpr uint32_t kChunkLimit = 0x7fffffffu;   // candidates per window chunk

__device__ __forceinline__ void wave_sync() {
    // Orders this wave's LDS accesses across lanes (LDS executes a wave's
    // operations in order; the fences stop the compiler from moving them).
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t incl_scan32(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = __shfl_up(v, d);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ uint64_t incl_scan64(uint64_t v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t o = __shfl_up(v, d);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t d) {
    uint64_t s = (uint64_t)a + d;
    return s > 0xffffffffull ? 0xffffffffu : (uint32_t)s;
}
__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t d) {
    return a > ~0ull - d ? ~0ull : a + d;
}

// first index in [lo, hi) whose time exceeds v (hi if none)
template <typename TT>
__device__ __forceinline__ uint32_t first_greater(const TT *__restrict__ a, uint32_t lo,
                                                  uint32_t hi, TT v) {
    uint32_t n = hi - lo;
    while (n > 0) {
        uint32_t h = n >> 1;
        if (a[lo + h] <= v) { lo += h + 1; n -= h + 1; }
        else n = h;
    }
    return lo;
}

// same, by exponential probing from lo (windows are short next to their lists)
template <typename TT>
__device__ __forceinline__ uint32_t gallop_greater(const TT *__restrict__ a, uint32_t lo,
                                                   uint32_t hi, TT v) {
    uint64_t step = 1;
    for (;;) {
        uint64_t probe = (uint64_t)lo + step - 1;
        if (probe >= hi) return first_greater(a, lo, hi, v);
        if (a[probe] > v) return first_greater(a, lo, (uint32_t)probe, v);
        lo = (uint32_t)probe + 1;
        step <<= 1;
    }
}

__device__ __forceinline__ int32_t pick6(int y, int32_t a, int32_t b, int32_t c, int32_t d,
                                         int32_t e, int32_t f) {
    int32_t r = a;
    r = (y == 1) ? b : r;
    r = (y == 2) ? c : r;
    r = (y == 3) ? d : r;
    r = (y == 4) ? e : r;
    r = (y == 5) ? f : r;
    return r;
}

// Partial matches with L motif edges matched (L = 1: the root batch).
template <typename TT, int L>
struct LevelBuf {
    static constexpr int S = (2 * L < kVMax) ? 2 * L : kVMax;   // vertex slots
    static constexpr int C = (L == 1) ? kWave : 2 * kWave;       // capacity
    int32_t phi[S][C];     // phi[s][i]: graph vertex of motif vertex s
    TT tfirst[C];
    TT tprev[C];
    int32_t node[C];       // trie node reached
    uint32_t pincl[C];     // inclusive prefix of child-group counts
};

template <typename TT, int D, int L>
struct LevelChain {
    LevelBuf<TT, L> buf;
    LevelChain<TT, D, L + 1> next;
};
template <typename TT, int D>
struct LevelChain<TT, D, D> {};

template <int L, typename TT, int D, int M>
__device__ __forceinline__ LevelBuf<TT, L> &lvl(LevelChain<TT, D, M> &c) {
    if constexpr (L == M) return c.buf;
    else return lvl<L>(c.next);
}

// per-lane statistics (only the STATS instantiation touches them)
struct Stats {
    uint64_t v[kStats];
};

template <typename TT, int D, bool STATS, int L>
__device__ __forceinline__ void run_level(const KParams<TT> &p, LevelChain<TT, D, 1> &W,
                                          unsigned long long *cnt, const int lane,
                                          const uint32_t nA, Stats &st) {
    LevelBuf<TT, L> &A = lvl<L>(W);
    constexpr int SA = LevelBuf<TT, L>::S;
    const int4 *__restrict__ node = p.tree.node;
    const int4 *__restrict__ grp = p.tree.grp;

    // child groups per buffered partial match -> inclusive prefix
    uint32_t P = 0;
    for (uint32_t x0 = 0; x0 < nA; x0 += kWave) {
        const uint32_t x = x0 + lane;
        uint32_t ng = 0;
        if (x < nA) ng = (uint32_t)node[A.node[x]].z;
        const uint32_t incl = incl_scan32(ng, lane) + P;
        if (x < nA) A.pincl[x] = incl;
        P = uniform(__shfl(incl, kWave - 1));
    }
    wave_sync();

    // window chunk state: lane w holds window w of the chunk
    uint32_t wx = 0, wlo = 0, wincl = 0, wexcl = 0;
    int32_t wg = 0;
    uint32_t pc = 0, nw = 0, T = 0, cc = 0;
    uint32_t nB = 0;   // partial matches buffered at level L+1

    for (;;) {
        bool done = false;
        if (cc >= T) {
            if (pc >= P) {
                done = true;
            } else {
                // one (partial match, group) pair per lane -> its window
                const uint32_t pi = pc + lane;
                uint32_t len = 0;
                wx = 0; wlo = 0; wg = 0;
                if (pi < P) {
                    uint32_t lo = 0, n = nA;
                    while (n > 0) {
                        const uint32_t h = n >> 1;
                        if (A.pincl[lo + h] <= pi) { lo += h + 1; n -= h + 1; }
                        else n = h;
                    }
                    wx = lo;
                    const uint32_t before = lo ? A.pincl[lo - 1] : 0u;
                    const int4 nd = node[A.node[lo]];
                    wg = nd.y + (int32_t)(pi - before);
                    const int4 g0 = grp[2 * wg];
                    const int dir = g0.x & 15, anc = g0.x >> 4;
                    const TT tp = A.tprev[lo];
                    const TT thi = sat_add(A.tfirst[lo], p.delta_sat);
                    uint32_t b, e;
                    const TT *ta;
                    if (dir == kDirOut) {
                        const int32_t a = A.phi[anc][lo];
                        b = p.g.out_off[a]; e = p.g.out_off[a + 1]; ta = p.g.out_t;
                    } else if (dir == kDirIn) {
                        const int32_t a = A.phi[anc][lo];
                        b = p.g.in_off[a]; e = p.g.in_off[a + 1]; ta = p.g.in_t;
                    } else {
                        b = 0; e = p.g.n_edges; ta = p.g.gt;
                    }
                    const uint32_t l0 = first_greater(ta, b, e, tp);
                    const uint32_t l1 = gallop_greater(ta, l0, e, thi);
                    wlo = l0;
                    len = l1 - l0;
                }
                // keep the chunk's candidate total below 2^31
                const uint64_t incl64 = incl_scan64((uint64_t)len, lane);
                const bool mine = pi < P && incl64 <= kChunkLimit;
                const uint64_t take = __ballot(mine);
                if constexpr (STATS) {
                    if (mine) {
                        const bool all = (grp[2 * wg].x & 15) == kDirAll;
                        st.v[all ? kStatWinAll : kStatWinList] += 1;
                        st.v[all ? kStatEntAll : kStatEntList] += len;
                    }
                }
                nw = uniform((uint32_t)__popcll(take));
                wincl = (uint32_t)incl64;
                wexcl = wincl - len;
                T = uniform(__shfl(wincl, (int)nw - 1));
                cc = 0;
                pc += nw;
            }
        }
        if (!done && cc < T) {
            const uint32_t f = cc + lane;
            // owner window: number of windows whose inclusive end is <= f
            uint32_t o = 0;
#pragma unroll
            for (uint32_t s = 32; s > 0; s >>= 1) {
                const uint32_t probe = o + s - 1;
                const uint32_t v = __shfl(wincl, (int)(probe & 63));
                if (probe < nw && v <= f) o += s;
            }
            const uint32_t oi = o & 63;
            const uint32_t ox = __shfl(wx, (int)oi);
            const uint32_t olo = __shfl(wlo, (int)oi);
            const uint32_t oex = __shfl(wexcl, (int)oi);
            const int32_t og = __shfl(wg, (int)oi);
            const bool valid = f < T;
            const uint32_t ei = olo + (f - oex);

            int32_t child = -1, nv0 = -1, nv1 = -1;
            int dir = 0;
            uint32_t nvp = 0;
            int32_t ph[SA];
#pragma unroll
            for (int s = 0; s < SA; ++s) ph[s] = 0;
            if (valid) {
                const int4 g0 = grp[2 * og];
                dir = g0.x & 15;
                nvp = (uint32_t)(node[A.node[ox]].w & 255);
#pragma unroll
                for (int s = 0; s < SA; ++s) ph[s] = A.phi[s][ox];
                if (dir == kDirOut) {
                    const int4 g1 = grp[2 * og + 1];
                    const int32_t cd = p.g.out_nbr[ei];
                    int y = -1;
#pragma unroll
                    for (int s = 0; s < SA; ++s) y = ((uint32_t)s < nvp && ph[s] == cd) ? s : y;
                    child = (y < 0) ? g0.y : pick6(y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w);
                    nv0 = cd;
                } else if (dir == kDirIn) {
                    const int32_t cs = p.g.in_nbr[ei];
                    bool hit = false;
#pragma unroll
                    for (int s = 0; s < SA; ++s) hit |= ((uint32_t)s < nvp && ph[s] == cs);
                    child = hit ? -1 : g0.y;
                    nv0 = cs;
                } else {
                    const int32_t cs = p.g.gsrc[ei], cd = p.g.gdst[ei];
                    bool hit = cs == cd;
#pragma unroll
                    for (int s = 0; s < SA; ++s)
                        hit |= ((uint32_t)s < nvp && (ph[s] == cs || ph[s] == cd));
                    child = hit ? -1 : g0.y;
                    nv0 = cs;
                    nv1 = cd;
                }
            }
            int cw = 0;
            if (child >= 0) {
                const int4 cn = node[child];
                cw = cn.w;
                if (cn.x >= 0) atomicAdd(&cnt[cn.x], 1ull);
                if constexpr (STATS) st.v[kStatCredit] += 1;
            }
            if constexpr (L + 1 < D) {
                LevelBuf<TT, L + 1> &B = lvl<L + 1>(W);
                constexpr int SB = LevelBuf<TT, L + 1>::S;
                const bool push = child >= 0 && ((cw >> 8) & 1);
                const uint64_t pm = __ballot(push);
                if (push) {
                    const TT *ta = dir == kDirOut ? p.g.out_t : (dir == kDirIn ? p.g.in_t : p.g.gt);
                    const uint32_t slot = nB + mbcnt(pm);
#pragma unroll
                    for (int s = 0; s < SB; ++s) {
                        int32_t v = (s < SA) ? ph[s < SA ? s : 0] : -1;
                        v = ((uint32_t)s < nvp) ? v
                            : ((uint32_t)s == nvp ? nv0 : ((uint32_t)s == nvp + 1 ? nv1 : -1));
                        B.phi[s][slot] = v;
                    }
                    B.tfirst[slot] = A.tfirst[ox];
                    B.tprev[slot] = ta[ei];
                    B.node[slot] = child;
                    if constexpr (STATS) st.v[kStatPush] += 1;
                }
                nB += (uint32_t)__popcll(pm);
            }
            cc += kWave;
        }
        if constexpr (L + 1 < D) {
            if (nB >= kWave || (done && nB > 0)) {
                wave_sync();
                run_level<TT, D, STATS, L + 1>(p, W, cnt, lane, nB, st);
                wave_sync();
                nB = 0;
            }
        }
        if (done) break;
    }
}

template <typename TT, int D, bool STATS>
__global__ void __launch_bounds__(kWave * kWavesPerBlock)
comine_kernel(const KParams<TT> p) {
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(smem);
    const size_t cnt_bytes = ((size_t)p.tree.n_q * 8 + 15) & ~(size_t)15;
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int wave = (int)(threadIdx.x / kWave);
    LevelChain<TT, D, 1> &W =
        reinterpret_cast<LevelChain<TT, D, 1> *>(smem + cnt_bytes)[wave];

    for (int i = (int)threadIdx.x; i < p.tree.n_q; i += (int)blockDim.x) cnt[i] = 0;
    __syncthreads();
    Stats st;
#pragma unroll
    for (int i = 0; i < kStats; ++i) st.v[i] = 0;

    for (;;) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(p.cursor, p.chunk);
        base = uniform(__shfl(base, 0));
        if (base >= p.n_roots) break;
        const uint32_t end = min(base + p.chunk, p.n_roots);
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
                atomicAdd(&cnt[p.tree.root_q], (unsigned long long)__popcll(m));
            if constexpr (STATS) st.v[kStatRoots] += ok ? 1 : 0;
            if constexpr (D > 1) {
                LevelBuf<TT, 1> &A = lvl<1>(W);
                if (ok) {
                    const uint32_t slot = mbcnt(m);
                    const TT tr = p.g.gt[r];
                    A.phi[0][slot] = s;
                    A.phi[1][slot] = d;
                    A.tfirst[slot] = tr;
                    A.tprev[slot] = tr;
                    A.node[slot] = 0;
                }
                const uint32_t n1 = uniform((uint32_t)__popcll(m));
                if (n1 > 0) {
                    wave_sync();
                    run_level<TT, D, STATS, 1>(p, W, cnt, lane, n1, st);
                    wave_sync();
                }
            }
        }
    }

    if constexpr (STATS) {
#pragma unroll
        for (int i = 0; i < kStats; ++i)
            if (st.v[i]) atomicAdd(&p.stats[i], (unsigned long long)st.v[i]);
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < p.tree.n_q; i += (int)blockDim.x)
        if (cnt[i]) atomicAdd(&p.counts[i], cnt[i]);
}

template <typename TT, int D>
size_t smem_bytes(int n_q) {
    return (((size_t)n_q * 8 + 15) & ~(size_t)15) +
           (size_t)kWavesPerBlock * sizeof(LevelChain<TT, D, 1>);
}

template <typename TT, int D, bool STATS>
hipError_t launch_ds(const KParams<TT> &p, int blocks, hipStream_t stream) {
    const size_t sm = smem_bytes<TT, D>(p.tree.n_q);
    auto kern = comine_kernel<TT, D, STATS>;
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

template <typename TT, int D>
hipError_t launch_d(const KParams<TT> &p, int blocks, hipStream_t stream) {
    return p.stats ? launch_ds<TT, D, true>(p, blocks, stream)
                   : launch_ds<TT, D, false>(p, blocks, stream);
}

template <typename TT, int D>
int fill_d(int n_q) {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, comine_kernel<TT, D, false>,
                                                     kWave * kWavesPerBlock,
                                                     smem_bytes<TT, D>(n_q)) != hipSuccess)
        return 0;
    return ncu * per;
}

}  // namespace

template <typename TT>
hipError_t launch_comine(const KParams<TT> &p, int blocks, hipStream_t stream) {
    switch (p.tree.depth) {
        case 1: return launch_d<TT, 1>(p, blocks, stream);
        case 2: return launch_d<TT, 2>(p, blocks, stream);
        case 3: return launch_d<TT, 3>(p, blocks, stream);
        case 4: return launch_d<TT, 4>(p, blocks, stream);
        case 5: return launch_d<TT, 5>(p, blocks, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename TT>
int comine_fill_blocks(int depth, int n_q) {
    switch (depth) {
        case 1: return fill_d<TT, 1>(n_q);
        case 2: return fill_d<TT, 2>(n_q);
        case 3: return fill_d<TT, 3>(n_q);
        case 4: return fill_d<TT, 4>(n_q);
        case 5: return fill_d<TT, 5>(n_q);
        default: return 0;
    }
}

template hipError_t launch_comine<uint32_t>(const KParams<uint32_t> &, int, hipStream_t);
template hipError_t launch_comine<uint64_t>(const KParams<uint64_t> &, int, hipStream_t);
template int comine_fill_blocks<uint32_t>(int, int);
template int comine_fill_blocks<uint64_t>(int, int);

}  // namespace mg
