// Internal launch interface between the C ABI (host.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdl {

struct ConstructParams {
  const float2* view_spec;   // [m][C][F]
  const float2* u;           // [m]
  const float* d;            // [n]
  float2* layer_spec;        // [n][C][F]
  int* status;               // device counter or null
  int m, n, C, H, W, Wh, F;
  double lambda, eps;
  int reg;
};

struct RenderParams {
  const float2* layer_spec;  // [n][C][F]
  const float* d;            // [n]
  const void* views;         // [V] fdl_view (20 bytes each)
  float2* out_spec;          // [V][C][F]
  int n, C, H, W, Wh, F, V;
};

hipError_t launch_construct(const ConstructParams& P, hipStream_t s);
hipError_t launch_render(const RenderParams& P, hipStream_t s);

}  // namespace fdl
