// Batched construction kernels for one channel (separate file for a parallel build).
#include "batch_kernels.h"

namespace fdl {
hipError_t batch_launch_c1(const BatchArgs& a, hipStream_t s) { return batch_launch_ct<1>(a, s); }
}  // namespace fdl
