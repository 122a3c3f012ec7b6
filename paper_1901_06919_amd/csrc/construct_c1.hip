// Plain construction kernels for one channel (separate file for a parallel build).
#include "construct_plain.h"

namespace fdl {
hipError_t launch_construct_c1(const ConstructParams& P, hipStream_t s) { return launch_plain_ct<1>(P, s); }
}  // namespace fdl
