// Batched construction kernels for four channels (separate file for a parallel build).
#include "batch_kernels.h"

namespace fdl {
hipError_t batch_launch_c4(const BatchArgs& a, hipStream_t s) { return batch_launch_ct<4>(a, s); }
}  // namespace fdl
