// Device helpers shared by the search and scheduler kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include "comine.h"

namespace mg {

static __device__ __forceinline__ void wave_sync() {
    // Orders this wave's LDS accesses across lanes (LDS executes a wave's
    // operations in order; the fences stop the compiler from moving them).
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

static __device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

static __device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Inclusive wave64 prefix sum by DPP: shifts by 1, 2, 4, 8 within each row of
// 16 lanes (lanes shifted in from outside the row read 0), then the total of
// row 0 is added to row 1 and of row 2 to row 3 (row_bcast:15, rows 1 and 3
// written), then the total of rows 0-1 to rows 2 and 3 (row_bcast:31).
static __device__ __forceinline__ uint32_t incl_scan32(uint32_t x, int /*lane*/) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// value of v in lane `src`, which must be the same in every lane
static __device__ __forceinline__ uint32_t lane_value(uint32_t v, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)src);
}
static __device__ __forceinline__ uint32_t lane_time(uint32_t v, int src) {
    return lane_value(v, (uint32_t)src);
}
static __device__ __forceinline__ uint64_t lane_time(uint64_t v, int src) {
    const uint32_t lo = lane_value((uint32_t)v, (uint32_t)src);
    const uint32_t hi = lane_value((uint32_t)(v >> 32), (uint32_t)src);
    return ((uint64_t)hi << 32) | lo;
}
static __device__ __forceinline__ unsigned long long lane0_u64(unsigned long long v) {
    const uint32_t lo = lane_value((uint32_t)v, 0), hi = lane_value((uint32_t)(v >> 32), 0);
    return ((unsigned long long)hi << 32) | lo;
}

static __device__ __forceinline__ uint64_t incl_scan64(uint64_t v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t o = __shfl_up(v, d);
        if (lane >= d) v += o;
    }
    return v;
}

static __device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t d) {
    uint64_t s = (uint64_t)a + d;
    return s > 0xffffffffull ? 0xffffffffu : (uint32_t)s;
}
static __device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t d) {
    return a > ~0ull - d ? ~0ull : a + d;
}

// first index i in [lo, hi) with a[i << sh] > v (hi if none); sh = 1 walks
// the time words of interleaved adjacency entries, sh = 0 a plain array
template <typename TT>
static __device__ __forceinline__ uint32_t first_greater(const TT *__restrict__ a, uint32_t sh,
                                                  uint32_t lo, uint32_t hi, TT v) {
    uint32_t n = hi - lo;
    while (n > 0) {
        uint32_t h = n >> 1;
        if (a[(size_t)(lo + h) << sh] <= v) { lo += h + 1; n -= h + 1; }
        else n = h;
    }
    return lo;
}

// same, by exponential probing from lo (windows are short next to their lists)
template <typename TT>
static __device__ __forceinline__ uint32_t gallop_greater(const TT *__restrict__ a, uint32_t sh,
                                                   uint32_t lo, uint32_t hi, TT v) {
    uint64_t step = 1;
    for (;;) {
        uint64_t probe = (uint64_t)lo + step - 1;
        if (probe >= hi) return first_greater(a, sh, lo, hi, v);
        if (a[(size_t)probe << sh] > v) return first_greater(a, sh, lo, (uint32_t)probe, v);
        lo = (uint32_t)probe + 1;
        step <<= 1;
    }
}

template <typename TT>
static __device__ __forceinline__ const TT *times_of(const Entry<TT> *adj) {
    return reinterpret_cast<const TT *>(adj) + 1;   // word 2i+1 is entry i's time
}

}  // namespace mg
