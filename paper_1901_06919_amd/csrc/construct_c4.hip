// Plain construction kernels for four channels (separate file for a parallel build).
#include "construct_plain.h"

namespace fdl {
hipError_t launch_construct_c4(const ConstructParams& P, hipStream_t s) { return launch_plain_ct<4>(P, s); }
}  // namespace fdl
