// Learned root-cost scheduler: features, MLP (BF16 weights, FP32
// accumulation on MFMA), training, and cost binning.  Internal interface
// between host.cpp and sched.hip.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "comine.h"

namespace mg {

constexpr int kFeat = 16;       // features per root (padded to 32 for MFMA)
constexpr int kHid = 64;        // hidden width
constexpr int kSeg = 64;        // roots per scheduling segment

// Parameter vector (fp32 master copy), row-major [in][out]:
//   W1 [32][64] (rows 16..31 stay zero), b1[64], W2[64][64], b2[64],
//   W3[64][64], b3[64], W4[64], b4[1]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + 32 * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * kHid;
constexpr int kOffW4 = kOffB3 + kHid;
constexpr int kOffB4 = kOffW4 + kHid;
constexpr int kParams = kOffB4 + 1;

// Features of the roots [0, n) of `roots` (or edge ids 0..n-1), fp32 n x 16.
template <typename TT>
hipError_t launch_features(const DevGraph<TT> &g, const DevTree &t, TT delta_sat,
                           const uint32_t *roots, uint32_t n, float *feats, hipStream_t st);

// MLP forward on given fp32 features (n x 16) -> predicted log-cost.
hipError_t launch_predict_feats(const float *params, const float *feats, uint32_t n, float *out,
                                hipStream_t st);

// Features (into feat_buf: 32 bytes per sampled root) then the MLP for one
// root edge in every `stride` (a power of two, 1..64: roots 0, stride, ...);
// per 64-root segment writes stride times the sum of exp(prediction) over its
// sampled roots (predicted cost) to seg_cost[n_edges / 64 rounded up] and adds
// every segment to *total (zeroed by the caller).
template <typename TT>
hipError_t launch_predict_roots(const DevGraph<TT> &g, const DevTree &t, TT delta_sat,
                                const float *params, uint32_t stride, float *seg_cost,
                                float *total, uint4 *feat_buf, hipStream_t st);

// Binning: segments predicted to cost more than heavy_mult times the mean
// segment become work items (root ranges {begin, end}), heaviest cost bin
// first, and are flagged in skip[n_seg] (when skip is not NULL); a heavy
// segment costlier than split_frac * (*total) becomes one item per root, and
// a root of it whose share is still above that becomes up to max_parts
// (1 .. 2^15 - 1) split items {root, kItemSplit | part << 15 | parts}.  When
// the parts would need more than cap (>= n_roots) items, no root is split.
// work: scratch of kBinWords u32 (zeroed here); items: capacity cap;
// n_items_out: device u32.  heavy_mult = 0 makes every segment an item.
constexpr int kBins = 48;
constexpr int kBinWords = 4 * kBins + 4;
hipError_t launch_bin(const float *seg_cost, uint32_t n_seg, uint32_t n_roots, const float *total,
                      float heavy_mult, float split_frac, uint32_t max_parts, uint32_t *work,
                      uint2 *items, uint32_t cap, uint32_t *n_items_out, uint8_t *skip,
                      hipStream_t st);

// p[0..n) = 0 with a kernel
hipError_t launch_fill_f32_zero(float *p, uint32_t n, hipStream_t st);

// Train on (features, label) pairs with Adam; one wave, minibatches of 32.
// params, adam_m, adam_v: kParams fp32 each (device).  loss: per epoch (device).
hipError_t launch_train(float *params, float *adam_m, float *adam_v, const float *feats,
                        const float *labels, uint32_t n, const uint32_t *perm, uint32_t epochs,
                        float lr, float *loss, hipStream_t st);

}  // namespace mg
