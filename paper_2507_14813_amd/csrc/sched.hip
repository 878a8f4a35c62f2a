// Learned root-cost scheduler for gfx950: per-root features, a 4-layer MLP
// (16 -> 64 -> 64 -> 64 -> 1, BF16 weights and activations, FP32
// accumulation on v_mfma_f32_16x16x32_bf16), its training step (forward,
// backward and Adam, all GEMMs on MFMA), and the binning that turns predicted
// costs into work items for the search kernel.  The schedule never changes a
// count: every root is searched exactly once, in whichever item holds it.
//
// MFMA 16x16x32 operand layout used throughout (lane l of the wave):
//   A (16 x 32): row l & 15, k = 8 * (l >> 4) + 0..7   (8 bf16 per lane)
//   B (32 x 16): col l & 15, k = 8 * (l >> 4) + 0..7
//   C (16 x 16): col l & 15, rows 4 * (l >> 4) + 0..3  (4 fp32 per lane)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
#include "sched.h"

namespace mg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16 bits, round to nearest even; NaN stays NaN
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u)
        return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float rbf(float f) { return bf2f(f2bf(f)); }

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {   // 16-byte aligned
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}
__device__ __forceinline__ bf16x8 pack8(const float *x) {
    uint4 v;
    v.x = f2bf(x[0]) | ((uint32_t)f2bf(x[1]) << 16);
    v.y = f2bf(x[2]) | ((uint32_t)f2bf(x[3]) << 16);
    v.z = f2bf(x[4]) | ((uint32_t)f2bf(x[5]) << 16);
    v.w = f2bf(x[6]) | ((uint32_t)f2bf(x[7]) << 16);
    return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ bf16x8 pack8u(const uint16_t *x) {   // from 8 separate values
    uint4 v;
    v.x = x[0] | ((uint32_t)x[1] << 16);
    v.y = x[2] | ((uint32_t)x[3] << 16);
    v.z = x[4] | ((uint32_t)x[5] << 16);
    v.w = x[6] | ((uint32_t)x[7] << 16);
    return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 splat(float x) { return f32x4{x, x, x, x}; }

// ------------------------------------------------------------ features
// Per root edge (a -> b at t), scaled log1p of: out/in degree of a and b,
// the number of entries of out(a), out(b), in(a), in(b) and of the whole edge
// list with time in (t, t + delta] (the windows the first search level
// scans), tree depth, distinct motifs, and a constant.  Self-loops: all 0.
template <typename TT>
__device__ void root_features(const DevGraph<TT> &g, const DevTree &t, TT dsat, uint32_t r,
                              float *f) {
#pragma unroll
    for (int k = 0; k < kFeat; ++k) f[k] = 0.f;
    const int32_t a = g.gsrc[r], b = g.gdst[r];
    if (a == b) return;
    const TT tr = g.gt[r];
    const TT thi = sat_add(tr, dsat);
    const uint32_t oa0 = g.out_off[a], oa1 = g.out_off[a + 1];
    const uint32_t ob0 = g.out_off[b], ob1 = g.out_off[b + 1];
    const uint32_t ia0 = g.in_off[a], ia1 = g.in_off[a + 1];
    const uint32_t ib0 = g.in_off[b], ib1 = g.in_off[b + 1];
    const TT *ot = times_of(g.out_adj), *it = times_of(g.in_adj);
    const float s = 1.f / 16.f;
    f[0] = log1pf((float)(oa1 - oa0)) * s;
    f[1] = log1pf((float)(ia1 - ia0)) * s;
    f[2] = log1pf((float)(ob1 - ob0)) * s;
    f[3] = log1pf((float)(ib1 - ib0)) * s;
    uint32_t l;
    l = first_greater(ot, 1, oa0, oa1, tr);
    f[4] = log1pf((float)(gallop_greater(ot, 1, l, oa1, thi) - l)) * s;
    l = first_greater(ot, 1, ob0, ob1, tr);
    f[5] = log1pf((float)(gallop_greater(ot, 1, l, ob1, thi) - l)) * s;
    l = first_greater(it, 1, ia0, ia1, tr);
    f[6] = log1pf((float)(gallop_greater(it, 1, l, ia1, thi) - l)) * s;
    l = first_greater(it, 1, ib0, ib1, tr);
    f[7] = log1pf((float)(gallop_greater(it, 1, l, ib1, thi) - l)) * s;
    l = gallop_greater(g.gt, 0, r, g.n_edges, tr);   // edges after r with a later time
    f[8] = log1pf((float)(gallop_greater(g.gt, 0, l, g.n_edges, thi) - l)) * s;
    f[9] = (float)t.depth * 0.125f;
    f[10] = log1pf((float)t.n_q) * 0.125f;
    f[11] = 1.f;
}

// ------------------------------------------------------------ MLP forward
struct MlpReg {
    bf16x8 w1[4];          // layer 1 B operands (one k-step), per 16-column tile
    bf16x8 w2[2][4];       // [k-step][column tile]
    bf16x8 w3[2][4];
    float b1[4], b2[4], b3[4], w4[4], b4;
};

__device__ void load_mlp(const float *P, MlpReg &m, int lane) {
    const int c = lane & 15, kq = 8 * (lane >> 4);
    float tmp[8];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
        for (int j = 0; j < 8; ++j) tmp[j] = P[kOffW1 + (kq + j) * kHid + 16 * nt + c];
        m.w1[nt] = pack8(tmp);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
            for (int j = 0; j < 8; ++j) tmp[j] = P[kOffW2 + (32 * ks + kq + j) * kHid + 16 * nt + c];
            m.w2[ks][nt] = pack8(tmp);
#pragma unroll
            for (int j = 0; j < 8; ++j) tmp[j] = P[kOffW3 + (32 * ks + kq + j) * kHid + 16 * nt + c];
            m.w3[ks][nt] = pack8(tmp);
        }
        m.b1[nt] = P[kOffB1 + 16 * nt + c];
        m.b2[nt] = P[kOffB2 + 16 * nt + c];
        m.b3[nt] = P[kOffB3 + 16 * nt + c];
        m.w4[nt] = rbf(P[kOffW4 + 16 * nt + c]);
    }
    m.b4 = P[kOffB4];
}

// One 16-row tile.  X: bf16 rows of 32 (features then zero padding); H: bf16
// scratch [16][64].  Lanes with (lane & 15) == 0 return the outputs of rows
// 4 * (lane >> 4) + r in out[r].
__device__ void mlp_tile(const MlpReg &m, const uint16_t *X, uint16_t *H, int lane,
                         float *out) {
    const int c = lane & 15, q = lane >> 4;
    const bf16x8 a = ld8(X + c * 32 + 8 * q);
    f32x4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma(a, m.w1[nt], splat(m.b1[nt]));
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) H[(4 * q + r) * kHid + 16 * nt + c] = f2bf(fmaxf(acc[nt][r], 0.f));
    wave_sync();
    bf16x8 a0 = ld8(H + c * kHid + 8 * q), a1 = ld8(H + c * kHid + 32 + 8 * q);
    wave_sync();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
        acc[nt] = mfma(a1, m.w2[1][nt], mfma(a0, m.w2[0][nt], splat(m.b2[nt])));
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) H[(4 * q + r) * kHid + 16 * nt + c] = f2bf(fmaxf(acc[nt][r], 0.f));
    wave_sync();
    a0 = ld8(H + c * kHid + 8 * q);
    a1 = ld8(H + c * kHid + 32 + 8 * q);
    wave_sync();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
        acc[nt] = mfma(a1, m.w3[1][nt], mfma(a0, m.w3[0][nt], splat(m.b3[nt])));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float v = 0.f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) v += rbf(fmaxf(acc[nt][r], 0.f)) * m.w4[nt];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        out[r] = v + m.b4;
    }
}

// 64 feature rows (one per lane) -> 64 predictions in pred[] (LDS)
__device__ void mlp_rows64(const MlpReg &m, const float *f, uint16_t *X, uint16_t *H,
                           float *pred, int lane) {
    uint16_t *row = X + lane * 32;
#pragma unroll
    for (int k = 0; k < kFeat; ++k) row[k] = f2bf(f[k]);
#pragma unroll
    for (int k = kFeat; k < 32; ++k) row[k] = 0;
    wave_sync();
    for (int tile = 0; tile < 4; ++tile) {
        float out[4];
        mlp_tile(m, X + tile * 16 * 32, H, lane, out);
        if ((lane & 15) == 0)
#pragma unroll
            for (int r = 0; r < 4; ++r) pred[tile * 16 + 4 * (lane >> 4) + r] = out[r];
        wave_sync();
    }
}

constexpr int kPredWaves = 4;

template <typename TT>
__global__ void __launch_bounds__(kWave * kPredWaves)
features_kernel(const DevGraph<TT> g, const DevTree t, TT dsat, const uint32_t *roots, uint32_t n,
                float *out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        float f[kFeat];
        root_features(g, t, dsat, roots ? roots[i] : i, f);
#pragma unroll
        for (int k = 0; k < kFeat; ++k) out[(size_t)i * kFeat + k] = f[k];
    }
}

__global__ void __launch_bounds__(kWave * kPredWaves)
predict_feats_kernel(const float *P, const float *feats, uint32_t n, float *out) {
    __shared__ __align__(16) uint16_t Xs[kPredWaves][64 * 32];
    __shared__ __align__(16) uint16_t Hs[kPredWaves][16 * kHid];
    __shared__ float Ps[kPredWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    MlpReg m;
    load_mlp(P, m, lane);
    const uint32_t nblk = (n + 63) / 64;
    for (uint32_t blk = blockIdx.x * kPredWaves + w; blk < nblk; blk += gridDim.x * kPredWaves) {
        const uint32_t i = blk * 64 + lane;
        float f[kFeat];
#pragma unroll
        for (int k = 0; k < kFeat; ++k) f[k] = i < n ? feats[(size_t)i * kFeat + k] : 0.f;
        mlp_rows64(m, f, Xs[w], Hs[w], Ps[w], lane);
        if (i < n) out[i] = Ps[w][lane];
        wave_sync();
    }
}

// Features of every stride-th root (roots 0, stride, 2*stride, ...) as 16
// BF16 values, two 16-byte words per sampled root.
template <typename TT>
__global__ void __launch_bounds__(256)
features_pack_kernel(const DevGraph<TT> g, const DevTree t, TT dsat, uint32_t stride,
                     uint4 *out) {
    const uint32_t n_rows = (g.n_edges + stride - 1) / stride;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_rows;
         j += gridDim.x * blockDim.x) {
        float f[kFeat];
        root_features(g, t, dsat, j * stride, f);
        uint4 a, b;
        a.x = f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16);
        a.y = f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16);
        a.z = f2bf(f[4]) | ((uint32_t)f2bf(f[5]) << 16);
        a.w = f2bf(f[6]) | ((uint32_t)f2bf(f[7]) << 16);
        b.x = f2bf(f[8]) | ((uint32_t)f2bf(f[9]) << 16);
        b.y = f2bf(f[10]) | ((uint32_t)f2bf(f[11]) << 16);
        b.z = f2bf(f[12]) | ((uint32_t)f2bf(f[13]) << 16);
        b.w = f2bf(f[14]) | ((uint32_t)f2bf(f[15]) << 16);
        out[2 * (size_t)j] = a;
        out[2 * (size_t)j + 1] = b;
    }
}

// MLP over the packed features of sampled roots, 64 rows per wave step (stride
// segments of 64 / stride rows each): writes each segment's predicted cost,
// stride times the sum of exp(prediction) over its sampled searched roots, and
// adds the segment costs to *total.
__global__ void __launch_bounds__(kWave * kPredWaves)
mlp_segments_kernel(const float *P, const uint4 *feats, uint32_t n_roots, uint32_t stride,
                    float *seg_cost, uint32_t n_seg, float *total) {
    __shared__ __align__(16) uint16_t Xs[kPredWaves][64 * 32];
    __shared__ __align__(16) uint16_t Hs[kPredWaves][16 * kHid];
    __shared__ float Ps[kPredWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t n_rows = (n_roots + stride - 1) / stride;
    const uint32_t n_steps = (n_rows + kWave - 1) / kWave;
    const uint32_t rps = kSeg / stride;            // rows per segment
    MlpReg m;
    load_mlp(P, m, lane);
    float tsum = 0.f;
    for (uint32_t step = blockIdx.x * kPredWaves + w; step < n_steps;
         step += gridDim.x * kPredWaves) {
        const uint32_t j = step * kWave + lane;
        uint4 a = make_uint4(0, 0, 0, 0), b = a;
        if (j < n_rows) {
            a = feats[2 * (size_t)j];
            b = feats[2 * (size_t)j + 1];
        }
        uint4 *row = reinterpret_cast<uint4 *>(Xs[w] + lane * 32);
        row[0] = a;
        row[1] = b;
        row[2] = make_uint4(0, 0, 0, 0);
        row[3] = make_uint4(0, 0, 0, 0);
        wave_sync();
        for (int tile = 0; tile < 4; ++tile) {
            float out[4];
            mlp_tile(m, Xs[w] + tile * 16 * 32, Hs[w], lane, out);
            if ((lane & 15) == 0)
#pragma unroll
                for (int q = 0; q < 4; ++q) Ps[w][tile * 16 + 4 * (lane >> 4) + q] = out[q];
            wave_sync();
        }
        const bool live = (b.y >> 16) != 0;      // feature 11 (constant 1) is 0 for self-loops
        float c = live ? expf(fminf(fmaxf(Ps[w][lane], 0.f), 40.f)) : 0.f;
        for (uint32_t o = rps >> 1; o > 0; o >>= 1) c += __shfl_xor(c, (int)o);
        c *= (float)stride;
        const uint32_t seg = step * stride + (uint32_t)lane / rps;
        if ((uint32_t)lane % rps == 0 && seg < n_seg) {
            seg_cost[seg] = c;
            tsum += c;
        }
        wave_sync();
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tsum += __shfl_xor(tsum, o);
    if (lane == 0 && tsum > 0.f) atomicAdd(total, tsum);
}

// ------------------------------------------------------------ binning
__device__ __forceinline__ int cost_bin(float c) {
    if (!(c >= 1.f)) return 0;
    return min(kBins - 1, 1 + (int)(log2f(c) * 2.f));   // half-octave bins
}

__global__ void fill_u32(uint32_t *p, uint32_t n, uint32_t v) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = v;
}

// work: hist[kBins] | base[kBins] | fill[kBins] | hist1[kBins] | flag
// A segment is heavy when its predicted cost exceeds heavy_mult times the mean
// segment cost; only heavy segments become items (and skip[] marks them), the
// rest stay with the time-ordered queue.  A heavy segment above split_frac of
// the total becomes one item per root, and each of its roots becomes up to
// max_parts items (parts of the root's first-level candidates) when its share
// of the segment is still above split_frac of the total.  If the parts would
// overflow the item capacity, roots are not split (flag set).
__device__ __forceinline__ bool is_heavy(float c, float total, uint32_t n_seg, float heavy_mult) {
    return total > 0.f && c > heavy_mult * (total / (float)n_seg);
}

__device__ __forceinline__ uint32_t root_parts(float c, uint32_t nr, float split,
                                               uint32_t max_parts) {
    const float k = ceilf(c / ((float)nr * split));
    return k >= (float)max_parts ? max_parts : (k < 1.f ? 1u : (uint32_t)k);
}

__global__ void bin_hist_kernel(const float *seg_cost, uint32_t n_seg, uint32_t n_roots,
                                const float *total, float heavy_mult, float split_frac,
                                uint32_t max_parts, uint32_t *work) {
    const float tot = *total, split = tot * split_frac;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n_seg; s += gridDim.x * blockDim.x) {
        const float c = seg_cost[s];
        if (!is_heavy(c, tot, n_seg, heavy_mult)) continue;
        const uint32_t nr = min((uint32_t)kSeg, n_roots - s * kSeg);
        const int b = cost_bin(c);
        if (c > split) {
            atomicAdd(&work[b], nr * root_parts(c, nr, split, max_parts));
            atomicAdd(&work[3 * kBins + b], nr);
        } else {
            atomicAdd(&work[b], 1u);
            atomicAdd(&work[3 * kBins + b], 1u);
        }
    }
}

__global__ void bin_scan_kernel(uint32_t *work, uint32_t cap, uint32_t *n_items) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint64_t all = 0;
        for (int b = 0; b < kBins; ++b) all += work[b];
        const bool whole = all > cap;          // no root parts
        work[4 * kBins] = whole ? 1u : 0u;
        uint32_t run = 0;
        for (int b = kBins - 1; b >= 0; --b) {   // heaviest bin first
            work[kBins + b] = run;
            run += work[(whole ? 3 * kBins : 0) + b];
            work[2 * kBins + b] = 0;
        }
        *n_items = run;
    }
}

__global__ void bin_scatter_kernel(const float *seg_cost, uint32_t n_seg, uint32_t n_roots,
                                   const float *total, float heavy_mult, float split_frac,
                                   uint32_t max_parts, uint32_t *work, uint2 *items,
                                   uint8_t *skip) {
    const float tot = *total, split = tot * split_frac;
    const uint32_t mp = work[4 * kBins] ? 1u : max_parts;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n_seg; s += gridDim.x * blockDim.x) {
        const float c = seg_cost[s];
        const bool heavy = is_heavy(c, tot, n_seg, heavy_mult);
        if (skip) skip[s] = heavy ? 1 : 0;
        if (!heavy) continue;
        const int b = cost_bin(c);
        const uint32_t r0 = s * kSeg, nr = min((uint32_t)kSeg, n_roots - r0);
        if (c > split) {
            const uint32_t k = root_parts(c, nr, split, mp);
            const uint32_t pos = work[kBins + b] + atomicAdd(&work[2 * kBins + b], nr * k);
            for (uint32_t i = 0; i < nr; ++i)
                for (uint32_t j = 0; j < k; ++j)
                    items[pos + i * k + j] =
                        k == 1 ? make_uint2(r0 + i, r0 + i + 1)
                               : make_uint2(r0 + i, kItemSplit | (j << 15) | k);
        } else {
            const uint32_t pos = work[kBins + b] + atomicAdd(&work[2 * kBins + b], 1u);
            items[pos] = make_uint2(r0, r0 + nr);
        }
    }
}

// ------------------------------------------------------------ training
// One wave; minibatches of 32 rows (two 16-row tiles).  LDS keeps bf16 copies
// of the weights in both orientations ([in][out] for the backward products,
// [out][in] for the forward B operands) and the activations of the batch.
constexpr int kTB = 32;

struct TrainLds {
    uint16_t X[kTB * 32];
    uint16_t H1[kTB * kHid], H2[kTB * kHid], H3[kTB * kHid];
    uint16_t G[kTB * kHid], G2[kTB * kHid];          // dZ of two adjacent layers
    uint16_t W1T[kHid * 32];                         // [out][in]
    uint16_t W2[kHid * kHid], W2T[kHid * kHid];
    uint16_t W3[kHid * kHid], W3T[kHid * kHid];
    float B1[kHid], B2[kHid], B3[kHid], W4[kHid], B4;
    float y[kTB], dout[kTB];
};

struct AdamState {
    float *P, *M, *V;
    float lr, c1, c2;      // step size and bias corrections 1/(1-beta^t)
};

__device__ __forceinline__ float adam(AdamState &s, int idx, float g) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float m = b1 * s.M[idx] + (1.f - b1) * g;
    const float v = b2 * s.V[idx] + (1.f - b2) * g * g;
    s.M[idx] = m;
    s.V[idx] = v;
    const float p = s.P[idx] - s.lr * (m * s.c1) / (sqrtf(v * s.c2) + eps);
    s.P[idx] = p;
    return p;
}

__device__ void refresh_lds(const float *P, TrainLds &S, int lane) {
    for (int i = lane; i < kHid * kHid; i += kWave) {
        const int in = i / kHid, out = i % kHid;
        const uint16_t w2 = f2bf(P[kOffW2 + i]), w3 = f2bf(P[kOffW3 + i]);
        S.W2[i] = w2;
        S.W2T[out * kHid + in] = w2;
        S.W3[i] = w3;
        S.W3T[out * kHid + in] = w3;
    }
    for (int i = lane; i < 32 * kHid; i += kWave) {
        const int in = i / kHid, out = i % kHid;
        S.W1T[out * 32 + in] = f2bf(P[kOffW1 + i]);
    }
    for (int i = lane; i < kHid; i += kWave) {
        S.B1[i] = P[kOffB1 + i];
        S.B2[i] = P[kOffB2 + i];
        S.B3[i] = P[kOffB3 + i];
        S.W4[i] = rbf(P[kOffW4 + i]);
    }
    if (lane == 0) S.B4 = P[kOffB4];
}

// D = A(16 x 32k) * B for 16-row tile `tile` of a [kTB][ld] bf16 matrix times
// 4 column tiles of a [out][in] bf16 matrix (contiguous k), nks k-steps.
__device__ void tile_times_T(const uint16_t *A, int ld, int tile, const uint16_t *BT, int ldb,
                             int nks, const float *bias, int lane, f32x4 *acc) {
    const int c = lane & 15, q = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = splat(bias ? bias[16 * nt + c] : 0.f);
    for (int ks = 0; ks < nks; ++ks) {
        const bf16x8 a = ld8(A + (16 * tile + c) * ld + 32 * ks + 8 * q);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            acc[nt] = mfma(a, ld8(BT + (16 * nt + c) * ldb + 32 * ks + 8 * q), acc[nt]);
    }
}

// gradient tile dW[16 mt + i][16 nt + j] = sum_rows Hin[row][16 mt + i] * dZ[row][16 nt + j]
__device__ f32x4 grad_tile(const uint16_t *Hin, int ldh, const uint16_t *dZ, int mt, int nt,
                           int lane) {
    const int c = lane & 15, q = lane >> 4;
    uint16_t av[8], bv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        av[j] = Hin[(8 * q + j) * ldh + 16 * mt + c];
        bv[j] = dZ[(8 * q + j) * kHid + 16 * nt + c];
    }
    return mfma(pack8u(av), pack8u(bv), splat(0.f));
}

__global__ void __launch_bounds__(kWave)
train_kernel(float *P, float *M, float *V, const float *feats, const float *labels, uint32_t n,
             const uint32_t *perm, uint32_t epochs, float lr, float *loss_out) {
    extern __shared__ __align__(16) unsigned char smem[];
    TrainLds &S = *reinterpret_cast<TrainLds *>(smem);
    const int lane = threadIdx.x, c = lane & 15, q = lane >> 4;
    refresh_lds(P, S, lane);
    wave_sync();
    AdamState as{P, M, V, lr, 1.f, 1.f};
    float b1t = 1.f, b2t = 1.f;
    const uint32_t nb = n / kTB;
    for (uint32_t ep = 0; ep < epochs; ++ep) {
        float lsum = 0.f;
        for (uint32_t bi = 0; bi < nb; ++bi) {
            b1t *= 0.9f;
            b2t *= 0.999f;
            as.c1 = 1.f / (1.f - b1t);
            as.c2 = 1.f / (1.f - b2t);
            if (lane < kTB) {
                const uint32_t id = perm[bi * kTB + lane];
#pragma unroll
                for (int k = 0; k < 32; ++k)
                    S.X[lane * 32 + k] = k < kFeat ? f2bf(feats[(size_t)id * kFeat + k]) : 0;
                S.y[lane] = labels[id];
            }
            wave_sync();
            // forward
            f32x4 acc[4];
            for (int tile = 0; tile < 2; ++tile) {
                tile_times_T(S.X, 32, tile, S.W1T, 32, 1, S.B1, lane, acc);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        S.H1[(16 * tile + 4 * q + r) * kHid + 16 * nt + c] = f2bf(fmaxf(acc[nt][r], 0.f));
            }
            wave_sync();
            for (int tile = 0; tile < 2; ++tile) {
                tile_times_T(S.H1, kHid, tile, S.W2T, kHid, 2, S.B2, lane, acc);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        S.H2[(16 * tile + 4 * q + r) * kHid + 16 * nt + c] = f2bf(fmaxf(acc[nt][r], 0.f));
            }
            wave_sync();
            for (int tile = 0; tile < 2; ++tile) {
                tile_times_T(S.H2, kHid, tile, S.W3T, kHid, 2, S.B3, lane, acc);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        S.H3[(16 * tile + 4 * q + r) * kHid + 16 * nt + c] = f2bf(fmaxf(acc[nt][r], 0.f));
            }
            wave_sync();
            // output layer and loss (mean squared error)
            if (lane < kTB) {
                float pr = S.B4;
                for (int j = 0; j < kHid; ++j) pr += bf2f(S.H3[lane * kHid + j]) * S.W4[j];
                const float e = pr - S.y[lane];
                lsum += e * e;
                S.dout[lane] = 2.f * e / (float)kTB;
            }
            wave_sync();
            // layer 4: gradients, and dZ3 = dout * w4 masked by relu (old w4)
            {
                const int j = lane;
                float gw = 0.f;
                for (int row = 0; row < kTB; ++row) {
                    const float h = bf2f(S.H3[row * kHid + j]);
                    gw += h * S.dout[row];
                    S.G[row * kHid + j] = f2bf(h > 0.f ? S.dout[row] * S.W4[j] : 0.f);
                }
                const float w4new = adam(as, kOffW4 + j, gw);
                float gb = lane < kTB ? S.dout[lane] : 0.f;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) gb += __shfl_xor(gb, o);
                wave_sync();
                S.W4[j] = rbf(w4new);
                if (lane == 0) S.B4 = adam(as, kOffB4, gb);
            }
            wave_sync();
            // layer 3: dZ2 = (dZ3 W3^T) * relu'(H2) with the old W3, then W3's update
            for (int tile = 0; tile < 2; ++tile) {
                tile_times_T(S.G, kHid, tile, S.W3, kHid, 2, nullptr, lane, acc);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * tile + 4 * q + r, col = 16 * nt + c;
                        S.G2[row * kHid + col] =
                            f2bf(bf2f(S.H2[row * kHid + col]) > 0.f ? acc[nt][r] : 0.f);
                    }
            }
            wave_sync();
            for (int mt = 0; mt < 4; ++mt)
                for (int nt = 0; nt < 4; ++nt) {
                    const f32x4 gt = grad_tile(S.H2, kHid, S.G, mt, nt, lane);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int in = 16 * mt + 4 * q + r, out = 16 * nt + c;
                        const uint16_t w = f2bf(adam(as, kOffW3 + in * kHid + out, gt[r]));
                        S.W3[in * kHid + out] = w;
                        S.W3T[out * kHid + in] = w;
                    }
                }
            {
                float gb = 0.f;
                for (int row = 0; row < kTB; ++row) gb += bf2f(S.G[row * kHid + lane]);
                S.B3[lane] = adam(as, kOffB3 + lane, gb);
            }
            wave_sync();
            // layer 2: dZ1 = (dZ2 W2^T) * relu'(H1) (into G), then W2's update
            for (int tile = 0; tile < 2; ++tile) {
                tile_times_T(S.G2, kHid, tile, S.W2, kHid, 2, nullptr, lane, acc);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * tile + 4 * q + r, col = 16 * nt + c;
                        S.G[row * kHid + col] =
                            f2bf(bf2f(S.H1[row * kHid + col]) > 0.f ? acc[nt][r] : 0.f);
                    }
            }
            wave_sync();
            for (int mt = 0; mt < 4; ++mt)
                for (int nt = 0; nt < 4; ++nt) {
                    const f32x4 gt = grad_tile(S.H1, kHid, S.G2, mt, nt, lane);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int in = 16 * mt + 4 * q + r, out = 16 * nt + c;
                        const uint16_t w = f2bf(adam(as, kOffW2 + in * kHid + out, gt[r]));
                        S.W2[in * kHid + out] = w;
                        S.W2T[out * kHid + in] = w;
                    }
                }
            {
                float gb = 0.f;
                for (int row = 0; row < kTB; ++row) gb += bf2f(S.G2[row * kHid + lane]);
                S.B2[lane] = adam(as, kOffB2 + lane, gb);
            }
            wave_sync();
            // layer 1 (inputs 0..15 only; the padding rows stay zero)
            for (int nt = 0; nt < 4; ++nt) {
                const f32x4 gt = grad_tile(S.X, 32, S.G, 0, nt, lane);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int in = 4 * q + r, out = 16 * nt + c;
                    S.W1T[out * 32 + in] = f2bf(adam(as, kOffW1 + in * kHid + out, gt[r]));
                }
            }
            {
                float gb = 0.f;
                for (int row = 0; row < kTB; ++row) gb += bf2f(S.G[row * kHid + lane]);
                S.B1[lane] = adam(as, kOffB1 + lane, gb);
            }
            wave_sync();
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
        if (lane == 0 && loss_out) loss_out[ep] = nb ? lsum / (float)(nb * kTB) : 0.f;
    }
}

}  // namespace

template <typename TT>
hipError_t launch_features(const DevGraph<TT> &g, const DevTree &t, TT delta_sat,
                           const uint32_t *roots, uint32_t n, float *feats, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = std::min<uint32_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(features_kernel<TT>, dim3(blocks), dim3(kWave * kPredWaves), 0, st, g, t,
                       delta_sat, roots, n, feats);
    return hipGetLastError();
}

hipError_t launch_predict_feats(const float *params, const float *feats, uint32_t n, float *out,
                                hipStream_t st) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = std::min<uint32_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(predict_feats_kernel, dim3(blocks), dim3(kWave * kPredWaves), 0, st, params,
                       feats, n, out);
    return hipGetLastError();
}

template <typename TT>
hipError_t launch_predict_roots(const DevGraph<TT> &g, const DevTree &t, TT delta_sat,
                                const float *params, uint32_t stride, float *seg_cost,
                                float *total, uint4 *feat_buf, hipStream_t st) {
    const uint32_t n_seg = (g.n_edges + kSeg - 1) / kSeg;
    if (n_seg == 0) return hipSuccess;
    if (stride == 0 || stride > (uint32_t)kSeg || (stride & (stride - 1)))
        return hipErrorInvalidValue;
    const uint32_t n_rows = (g.n_edges + stride - 1) / stride;
    const uint32_t fb = std::min<uint32_t>((n_rows + 255) / 256, 8192);
    hipLaunchKernelGGL(features_pack_kernel<TT>, dim3(fb), dim3(256), 0, st, g, t, delta_sat,
                       stride, feat_buf);
    const uint32_t steps = (n_rows + kWave - 1) / kWave;
    const uint32_t blocks = std::min<uint32_t>((steps + kPredWaves - 1) / kPredWaves, 2048);
    hipLaunchKernelGGL(mlp_segments_kernel, dim3(blocks), dim3(kWave * kPredWaves), 0, st, params,
                       feat_buf, g.n_edges, stride, seg_cost, n_seg, total);
    return hipGetLastError();
}

hipError_t launch_bin(const float *seg_cost, uint32_t n_seg, uint32_t n_roots,
                      const float *total, float heavy_mult, float split_frac, uint32_t max_parts,
                      uint32_t *work, uint2 *items, uint32_t cap, uint32_t *n_items_out,
                      uint8_t *skip, hipStream_t st) {
    if (max_parts < 1 || max_parts >= (1u << 15) || cap < n_roots) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fill_u32, dim3(1), dim3(256), 0, st, work, (uint32_t)kBinWords, 0u);
    const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>((n_seg + 255) / 256, 2048));
    hipLaunchKernelGGL(bin_hist_kernel, dim3(blocks), dim3(256), 0, st, seg_cost, n_seg, n_roots,
                       total, heavy_mult, split_frac, max_parts, work);
    hipLaunchKernelGGL(bin_scan_kernel, dim3(1), dim3(64), 0, st, work, cap, n_items_out);
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(blocks), dim3(256), 0, st, seg_cost, n_seg,
                       n_roots, total, heavy_mult, split_frac, max_parts, work, items, skip);
    return hipGetLastError();
}

hipError_t launch_fill_f32_zero(float *p, uint32_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32, dim3(std::min<uint32_t>((n + 255) / 256, 1024)), dim3(256), 0, st,
                       reinterpret_cast<uint32_t *>(p), n, 0u);
    return hipGetLastError();
}

hipError_t launch_train(float *params, float *adam_m, float *adam_v, const float *feats,
                        const float *labels, uint32_t n, const uint32_t *perm, uint32_t epochs,
                        float lr, float *loss, hipStream_t st) {
    const size_t sm = sizeof(TrainLds);
    if (sm > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)train_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(train_kernel, dim3(1), dim3(kWave), sm, st, params, adam_m, adam_v, feats,
                       labels, n, perm, epochs, lr, loss);
    return hipGetLastError();
}

template hipError_t launch_features<uint32_t>(const DevGraph<uint32_t> &, const DevTree &, uint32_t,
                                              const uint32_t *, uint32_t, float *, hipStream_t);
template hipError_t launch_features<uint64_t>(const DevGraph<uint64_t> &, const DevTree &, uint64_t,
                                              const uint32_t *, uint32_t, float *, hipStream_t);
template hipError_t launch_predict_roots<uint32_t>(const DevGraph<uint32_t> &, const DevTree &,
                                                   uint32_t, const float *, uint32_t, float *,
                                                   float *, uint4 *, hipStream_t);
template hipError_t launch_predict_roots<uint64_t>(const DevGraph<uint64_t> &, const DevTree &,
                                                   uint64_t, const float *, uint32_t, float *,
                                                   float *, uint4 *, hipStream_t);

}  // namespace mg
