// Plain construction kernels for two or three channels (separate file for a parallel build).
#include "construct_plain.h"

namespace fdl {
hipError_t launch_construct_c3(const ConstructParams& P, hipStream_t s) { return launch_plain_ct<3>(P, s); }
}  // namespace fdl
