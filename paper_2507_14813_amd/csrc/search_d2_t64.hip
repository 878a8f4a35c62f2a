// Search kernels for trees of depth 2 with 64-bit times.
#include "search.h"

namespace mg {
template hipError_t launch_d<uint64_t, 2>(const KParams<uint64_t> &, int, hipStream_t);
template hipError_t launch_batch_d<uint64_t, 2, 0>(const BatchParams<uint64_t> &, int, hipStream_t);
template hipError_t launch_batch_d<uint64_t, 2, 3>(const BatchParams<uint64_t> &, int, hipStream_t);
}  // namespace mg
