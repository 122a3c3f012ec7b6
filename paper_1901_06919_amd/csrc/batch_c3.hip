// Batched construction kernels for two or three channels (separate file for a parallel build).
#include "batch_kernels.h"

namespace fdl {
hipError_t batch_launch_c3(const BatchArgs& a, hipStream_t s) { return batch_launch_ct<3>(a, s); }
}  // namespace fdl
