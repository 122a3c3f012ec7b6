// C ABI of libfdl.so: argument validation, launch-shape choice and status
// mapping.  Every entry point validates on the host, enqueues on the caller's
// stream and returns without synchronising.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "../../include/fdl.h"
#include "fdl_internal.h"

static_assert(sizeof(fdl_c64) == 8, "fdl_c64 must match complex64");
static_assert(sizeof(fdl_view) == 20, "fdl_view layout");

namespace {

int map_hip(hipError_t e) {
  if (e == hipSuccess) return FDL_OK;
  if (std::getenv("FDL_TRACE")) std::fprintf(stderr, "fdl: HIP error %s\n", hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? FDL_ENOMEM : FDL_EHIP;
}

bool is_235(int v) {
  if (v < 1) return false;
  while (v % 2 == 0) v /= 2;
  while (v % 3 == 0) v /= 3;
  return v == 1;
}

void trace(const char* what, int a, int b, int c, int d) {
  if (std::getenv("FDL_TRACE")) std::fprintf(stderr, "fdl: %s %d %d %d %d\n", what, a, b, c, d);
}

}  // namespace

extern "C" {

const char* fdl_status_string(int code) {
  switch (code) {
    case FDL_OK: return "ok";
    case FDL_EINVAL: return "invalid argument";
    case FDL_ESHAPE: return "unsupported shape";
    case FDL_ENOMEM: return "out of memory or workspace too small";
    case FDL_EHIP: return "HIP runtime error";
    case FDL_ENUMERIC: return "numerical failure";
    case FDL_EUNSUPPORTED: return "not supported by this build";
    default: return "unknown status";
  }
}

int fdl_version(void) { return 10000; }

int fdl_construct(const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_dev, int m, int n, int C,
                  int H, int W, float lambda, float eps, int reg, fdl_c64* layer_spec_dev, int32_t* status_dev,
                  void* stream) {
  if (!view_spec_dev || !u_dev || !d_dev || !layer_spec_dev) return FDL_EINVAL;
  if (!(std::isfinite(lambda) && lambda >= 0.f) || !(std::isfinite(eps) && eps >= 0.f)) return FDL_EINVAL;
  if (reg < FDL_REG_VIEW2 || reg > FDL_REG_L2) return FDL_EINVAL;
  if (m < 1 || m > 4096 || n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30)) return FDL_ESHAPE;
  fdl::ConstructParams P;
  P.view_spec = reinterpret_cast<const float2*>(view_spec_dev);
  P.u = reinterpret_cast<const float2*>(u_dev);
  P.d = d_dev;
  P.layer_spec = reinterpret_cast<float2*>(layer_spec_dev);
  P.status = status_dev;
  P.m = m; P.n = n; P.C = C; P.H = H; P.W = W; P.Wh = W / 2 + 1; P.F = (int)F;
  P.lambda = (double)lambda; P.eps = (double)eps; P.reg = reg;
  trace("construct m n C F", m, n, C, (int)F);
  return map_hip(fdl::launch_construct(P, reinterpret_cast<hipStream_t>(stream)));
}

int fdl_render(const fdl_c64* layer_spec_dev, const float* d_dev, int n, int C, int H, int W,
               const fdl_view* views_dev, int V, fdl_c64* out_spec_dev, void* stream) {
  if (!layer_spec_dev || !d_dev || !views_dev || !out_spec_dev) return FDL_EINVAL;
  if (n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS || V < 1) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30) || V > 65535 * 8) return FDL_ESHAPE;
  fdl::RenderParams P;
  P.layer_spec = reinterpret_cast<const float2*>(layer_spec_dev);
  P.d = d_dev;
  P.views = views_dev;
  P.out_spec = reinterpret_cast<float2*>(out_spec_dev);
  P.n = n; P.C = C; P.H = H; P.W = W; P.Wh = W / 2 + 1; P.F = (int)F; P.V = V;
  trace("render n C F V", n, C, (int)F, V);
  return map_hip(fdl::launch_render(P, reinterpret_cast<hipStream_t>(stream)));
}

}  // extern "C"
