// Dispatch of the search kernels by tree depth, the fill kernel and the
// static scratch array of the count that allocates nothing.  The kernels
// themselves are in search.h, instantiated per depth and time width in
// search_d<depth>_t<bits>.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "comine.h"

namespace mg {
namespace {

__global__ void fill_u64(unsigned long long *p, uint32_t n, unsigned long long v) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

template <typename TT>
hipError_t launch_batch(const BatchParams<TT> &bp, int depth, int blocks, hipStream_t stream) {
    if (bp.multi) {
        switch (depth) {
            case 1: return launch_batch_d<TT, 1, 3>(bp, blocks, stream);
            case 2: return launch_batch_d<TT, 2, 3>(bp, blocks, stream);
            case 3: return launch_batch_d<TT, 3, 3>(bp, blocks, stream);
            case 4: return launch_batch_d<TT, 4, 3>(bp, blocks, stream);
            case 5: return launch_batch_d<TT, 5, 3>(bp, blocks, stream);
            default: return hipErrorInvalidValue;
        }
    }
    switch (depth) {
        case 1: return launch_batch_d<TT, 1, 0>(bp, blocks, stream);
        case 2: return launch_batch_d<TT, 2, 0>(bp, blocks, stream);
        case 3: return launch_batch_d<TT, 3, 0>(bp, blocks, stream);
        case 4: return launch_batch_d<TT, 4, 0>(bp, blocks, stream);
        case 5: return launch_batch_d<TT, 5, 0>(bp, blocks, stream);
        default: return hipErrorInvalidValue;
    }
}

// The scratch array itself.  In host code its name is a host-side stand-in,
// never a device address: host code uses only the per-device address that
// hipGetSymbolAddress returns.
static_assert(kStats <= 8, "statistics words");
static __device__ __align__(256) unsigned long long scratch[kStaticWords];

hipError_t static_scratch(unsigned long long **ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static unsigned long long *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<unsigned long long *>(a);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_fill_u64(unsigned long long *p, uint32_t n, unsigned long long v,
                           hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = std::min<uint32_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_u64, dim3(blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

template <typename TT>
hipError_t launch_comine(const KParams<TT> &p, int blocks, hipStream_t stream) {
    switch (p.tree.kdepth) {
        case 1: return launch_d<TT, 1>(p, blocks, stream);
        case 2: return launch_d<TT, 2>(p, blocks, stream);
        case 3: return launch_d<TT, 3>(p, blocks, stream);
        case 4: return launch_d<TT, 4>(p, blocks, stream);
        case 5: return launch_d<TT, 5>(p, blocks, stream);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_comine<uint32_t>(const KParams<uint32_t> &, int, hipStream_t);
template hipError_t launch_comine<uint64_t>(const KParams<uint64_t> &, int, hipStream_t);
template hipError_t launch_batch<uint32_t>(const BatchParams<uint32_t> &, int, int, hipStream_t);
template hipError_t launch_batch<uint64_t>(const BatchParams<uint64_t> &, int, int, hipStream_t);

}  // namespace mg
