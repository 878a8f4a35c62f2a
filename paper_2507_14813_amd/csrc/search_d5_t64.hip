// Search kernels for trees of depth 5 with 64-bit times.
#include "search.h"

namespace mg {
template hipError_t launch_d<uint64_t, 5>(const KParams<uint64_t> &, int, hipStream_t);
template hipError_t launch_batch_d<uint64_t, 5, 0>(const BatchParams<uint64_t> &, int, hipStream_t);
template hipError_t launch_batch_d<uint64_t, 5, 3>(const BatchParams<uint64_t> &, int, hipStream_t);
}  // namespace mg
