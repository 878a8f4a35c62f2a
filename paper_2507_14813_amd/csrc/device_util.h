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

static __device__ __forceinline__ uint32_t incl_scan32(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = __shfl_up(v, d);
        if (lane >= d) v += o;
    }
    return v;
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
