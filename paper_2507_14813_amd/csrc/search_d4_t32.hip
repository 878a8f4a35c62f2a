// Search kernels for trees of depth 4 with 32-bit times.
#include "search.h"

namespace mg {
template hipError_t launch_d<uint32_t, 4>(const KParams<uint32_t> &, int, hipStream_t);
template hipError_t launch_batch_d<uint32_t, 4, 0>(const BatchParams<uint32_t> &, int, hipStream_t);
template hipError_t launch_batch_d<uint32_t, 4, 3>(const BatchParams<uint32_t> &, int, hipStream_t);
}  // namespace mg
