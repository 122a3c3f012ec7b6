// Fourier-domain rendering (Sec. IV-B Eq. BsFourier; Sec. VI):
//   B_v(w) = sum_k exp(+2 pi i d_k <u0_v, w>) psi_hat_v((s_v - d_k) w) L_k(w)
// for a batch of V views sharing one pass over the layers.
//
// One thread per half-spectrum bin and a chunk of VB views (grid.y over
// chunks): the layer values of the bin are loaded once per chunk (coalesced
// along the bin index), every view of the chunk accumulates in registers.
// FP32 arithmetic: rendering is a plain weighted sum, no ill-conditioning.
#include "fdl_device.h"
#include "fdl_internal.h"

namespace fdl {

struct ViewRec {   // mirrors fdl_view
  float u, v, focus, radius;
  int shape;
};

// sin(2 pi r), cos(2 pi r) for r in revolutions: exact reduction to
// [-1/2, 1/2] then the hardware transcendental unit (which takes revolutions).
__device__ __forceinline__ void sincos2pi_f(float r, float& s, float& c) {
  r = r - rintf(r);
  s = __builtin_amdgcn_sinf(r);
  c = __builtin_amdgcn_cosf(r);
}

// 2 J1(z) / z for z >= 0.  Polynomial approximations of Abramowitz & Stegun,
// Handbook of Mathematical Functions (1964), 9.4.4 (|x| <= 3, error < 1.3e-8
// in J1(x)/x) and 9.4.6 (x >= 3, J1 = x^-1/2 f1 cos(theta1), errors < 4e-8 in
// f1 and < 9e-8 in theta1).
__device__ __forceinline__ float jinc2(float z) {
  if (z <= 3.0f) {
    const float t = z * (1.0f / 3.0f);
    const float t2 = t * t;
    float p = 0.00001109f;
    p = fmaf(p, t2, -0.00031761f);
    p = fmaf(p, t2, 0.00443319f);
    p = fmaf(p, t2, -0.03954289f);
    p = fmaf(p, t2, 0.21093573f);
    p = fmaf(p, t2, -0.56249985f);
    p = fmaf(p, t2, 0.5f);
    return 2.0f * p;
  }
  const float y = 3.0f / z;
  float f1 = -0.00020033f;
  f1 = fmaf(f1, y, 0.00113653f);
  f1 = fmaf(f1, y, -0.00249511f);
  f1 = fmaf(f1, y, 0.00017105f);
  f1 = fmaf(f1, y, 0.01659667f);
  f1 = fmaf(f1, y, 0.00000156f);
  f1 = fmaf(f1, y, 0.79788456f);
  float th = -0.00029166f;
  th = fmaf(th, y, 0.00079824f);
  th = fmaf(th, y, 0.00074348f);
  th = fmaf(th, y, -0.00637879f);
  th = fmaf(th, y, 0.00005650f);
  th = fmaf(th, y, 0.12499612f);
  th = fmaf(th, y, -2.35619449f);
  // theta1 = z + th; cos via revolutions with the integer part removed
  const float zr = z * (float)(1.0 / kTwoPi);
  const float zi = rintf(zr);
  const float rev = (zr - zi) + th * (float)(1.0 / kTwoPi);
  const float c = __builtin_amdgcn_cosf(rev - rintf(rev));
  const float j1 = f1 * c * rsqrtf(z);
  return 2.0f * j1 / z;
}

// sin(pi t) / (pi t)
__device__ __forceinline__ float sincf(float t) {
  if (fabsf(t) < 1e-4f) {
    const float a = (float)kPi * t;
    return 1.0f - a * a * (1.0f / 6.0f);
  }
  const float h = 0.5f * t;                       // revolutions of pi t
  const float s = __builtin_amdgcn_sinf(h - rintf(h));
  return s / ((float)kPi * t);
}

__device__ __forceinline__ float psi_hat_f(int shape, float rho, float xx, float xy) {
  if (rho == 0.0f) return 1.0f;
  if (shape == 1) {
    const float z = (float)kTwoPi * rho * sqrtf(xx * xx + xy * xy);
    return jinc2(z);
  }
  if (shape == 2) return sincf(2.0f * rho * xx) * sincf(2.0f * rho * xy);
  return 1.0f;
}

template <int VB, int CT>
__global__ __launch_bounds__(256) void k_render(RenderParams P) {
  __shared__ ViewRec s_v[VB];
  const int v0 = blockIdx.y * VB;
  const int nv = min(VB, P.V - v0);
  const ViewRec* views = reinterpret_cast<const ViewRec*>(P.views);
  if (threadIdx.x < VB && (int)threadIdx.x < nv) s_v[threadIdx.x] = views[v0 + threadIdx.x];
  __syncthreads();

  const int f = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (f >= P.F) return;
  double wxd, wyd;
  bin_freq(f, P.Wh, P.H, P.W, wxd, wyd);
  const float wx = (float)wxd, wy = (float)wyd;
  const int C = P.C;
  const size_t F = (size_t)P.F;

  float2 acc[VB][CT];
#pragma unroll
  for (int v = 0; v < VB; ++v)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[v][c] = make_float2(0.f, 0.f);

  for (int k = 0; k < P.n; ++k) {
    const float dk = P.d[k];
    float2 x[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c)
      x[c] = c < C ? P.layer_spec[((size_t)k * C + c) * F + f] : make_float2(0.f, 0.f);
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      if (v < nv) {
        const ViewRec rv = s_v[v];
        float s, co;
        sincos2pi_f(dk * (rv.u * wx + rv.v * wy), s, co);
        const float a = rv.focus - dk;
        const float g = psi_hat_f(rv.shape, rv.radius, a * wx, a * wy);
        const float pr = co * g, pi = s * g;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          acc[v][c].x = fmaf(pr, x[c].x, fmaf(-pi, x[c].y, acc[v][c].x));
          acc[v][c].y = fmaf(pr, x[c].y, fmaf(pi, x[c].x, acc[v][c].y));
        }
      }
    }
  }
#pragma unroll
  for (int v = 0; v < VB; ++v) {
    if (v < nv) {
#pragma unroll
      for (int c = 0; c < CT; ++c)
        if (c < C) P.out_spec[((size_t)(v0 + v) * C + c) * F + f] = acc[v][c];
    }
  }
}

template <int VB, int CT>
static hipError_t launch_render_vc(const RenderParams& P, hipStream_t s) {
  dim3 grid((P.F + 255) / 256, (P.V + VB - 1) / VB);
  hipLaunchKernelGGL((k_render<VB, CT>), grid, dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_render(const RenderParams& P, hipStream_t s) {
  switch (P.C) {
    case 1: return launch_render_vc<32, 1>(P, s);
    case 2: return launch_render_vc<16, 2>(P, s);
    case 3: return launch_render_vc<16, 3>(P, s);
    default: return launch_render_vc<8, 4>(P, s);
  }
}

}  // namespace fdl
