// Fourier-domain rendering (Sec. IV-B Eq. BsFourier; Sec. VI):
//   B_v(w) = sum_k exp(+2 pi i d_k <u0_v, w>) psi_hat_v((s_v - d_k) w) L_k(w)
// for a batch of V views sharing one pass over the layers.
//
// One thread per half-spectrum bin and a chunk of VB views: the layer values
// of the bin are loaded once per chunk (coalesced along the bin index), every
// view of the chunk accumulates in registers; the disk aperture spectrum
// 2 J1(z)/z comes from a per-block LDS table of cubic pieces.  FP32
// arithmetic: rendering is a plain weighted sum, no ill-conditioning.
#include "fdl.h"
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

// sin(pi t) / (pi t) with a hardware reciprocal (about 1 ulp)
__device__ __forceinline__ float sinc_fast(float t) {
  const float a = (float)kPi * t;
  if (fabsf(t) < 1e-4f) return 1.0f - a * a * (1.0f / 6.0f);
  const float h = 0.5f * t;   // revolutions of pi t
  return __builtin_amdgcn_sinf(h - rintf(h)) * __builtin_amdgcn_rcpf(a);
}

// ---- tabulated 2 J1(z) / z --------------------------------------------------
// Cubic pieces on [i h, (i + 1) h], i < kJincN, through the four nodes
// (i-1) h .. (i+2) h (the function is even, so node -h is node h), in the
// local variable t = z / h - i; nodes from jinc2 above.  Interpolation error
// below 1e-6 for h = 1/8 (fourth derivative at most 1/8); beyond kJincN h the
// asymptotic form is evaluated directly.
constexpr int kJincN = 1024;
constexpr float kJincH = 0.125f;

__device__ __forceinline__ void build_jinc_table(float4* tab, float* nodes) {
  for (int i = threadIdx.x; i < kJincN + 3; i += blockDim.x) nodes[i] = jinc2(fabsf((float)(i - 1) * kJincH));
  __syncthreads();
  for (int i = threadIdx.x; i < kJincN; i += blockDim.x) {
    const float fm = nodes[i], f0 = nodes[i + 1], f1 = nodes[i + 2], f2 = nodes[i + 3];
    tab[i] = make_float4(f0, (-2.0f * fm - 3.0f * f0 + 6.0f * f1 - f2) * (1.0f / 6.0f), 0.5f * (fm - 2.0f * f0 + f1),
                         (-fm + 3.0f * f0 - 3.0f * f1 + f2) * (1.0f / 6.0f));
  }
}

__device__ __forceinline__ float jinc_tab(const float4* __restrict__ tab, float z) {
  const float s = z * (1.0f / kJincH);
  if (s >= (float)kJincN) return jinc2(z);
  const float fi = floorf(s);
  const float t = s - fi;
  const float4 c = tab[(int)fi];
  return fmaf(fmaf(fmaf(c.w, t, c.z), t, c.y), t, c.x);
}

// x0 mod N in [0, N) for an integer-valued float x0: the quotient from a
// multiply by 1/N, then one correction step.  Every step is exact in float
// for |x0| < 2^24, so this equals the floored division; the clamp keeps any
// other input inside the table.
__device__ __forceinline__ int wrap_index(float x0, float fN, float invN) {
  float r = x0 - fN * floorf(x0 * invN);
  r = r < 0.0f ? r + fN : (r >= fN ? r - fN : r);
  return min(max((int)r, 0), (int)fN - 1);
}

// psi_hat of a drawn aperture from its table of spectrum samples (N x N,
// rows k_y): bilinear interpolation at the continuous sample index (tx, ty),
// periodic in both directions.  The four samples are buffer loads with
// 32-bit byte offsets (N <= 2048: the table holds at most 2^25 bytes).
__device__ __forceinline__ float2 aperture_tab(__amdgpu_buffer_rsrc_t tab, int N, float fN, float invN, float tx,
                                               float ty) {
  const float x0 = floorf(tx), y0 = floorf(ty);
  const float fx = tx - x0, fy = ty - y0;
  const int ix = wrap_index(x0, fN, invN), iy = wrap_index(y0, fN, invN);
  const int ix1 = ix + 1 == N ? 0 : ix + 1;
  const int iy1 = iy + 1 == N ? 0 : iy + 1;
  const unsigned r0 = (unsigned)(iy * N) * 8u, r1 = (unsigned)(iy1 * N) * 8u;
  const float2 a = buf_load_f2(tab, r0 + (unsigned)ix * 8u, 0), b = buf_load_f2(tab, r0 + (unsigned)ix1 * 8u, 0);
  const float2 c = buf_load_f2(tab, r1 + (unsigned)ix * 8u, 0), e = buf_load_f2(tab, r1 + (unsigned)ix1 * 8u, 0);
  const float w00 = (1.f - fx) * (1.f - fy), w01 = fx * (1.f - fy), w10 = (1.f - fx) * fy, w11 = fx * fy;
  return make_float2(w00 * a.x + w01 * b.x + w10 * c.x + w11 * e.x, w00 * a.y + w01 * b.y + w10 * c.y + w11 * e.y);
}

// TAB: views of shape 3 take their aperture spectrum from the drawn-aperture
// table (complex in general); without it shape 3 renders as a pinhole.
template <int VB, int CT, bool TAB = false>
__global__ __launch_bounds__(256) void k_render(RenderParams P, int nchunks) {
  __shared__ ViewRec s_v[VB];
  __shared__ float4 s_jinc[kJincN];
  __shared__ float s_nodes[kJincN + 3];
  // consecutive (remapped) blocks share a bin range and sit on one XCD, so
  // the layer values of the range are read from HBM once per XCD
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int bin_block = b / nchunks;
  const int v0 = (b - bin_block * nchunks) * VB;
  const int nv = min(VB, P.V - v0);
  const ViewRec* views = reinterpret_cast<const ViewRec*>(P.views);
  if (threadIdx.x < VB && (int)threadIdx.x < nv) s_v[threadIdx.x] = views[v0 + threadIdx.x];
  build_jinc_table(s_jinc, s_nodes);
  __syncthreads();

  const int f = bin_block * 256 + threadIdx.x;
  if (f >= P.F) return;
  double wxd, wyd;
  bin_freq(f, P.Wh, P.H, P.W, wxd, wyd);
  const float wx = (float)wxd, wy = (float)wyd;
  const float wn = sqrtf(wx * wx + wy * wy);
  const int C = P.C;
  const size_t F = (size_t)P.F;
  // drawn-aperture table (TAB kernels only)
  const __amdgpu_buffer_rsrc_t tabr = buf_rsrc(TAB ? (const void*)P.ap_tab : (const void*)P.layer_spec);
  const float apN = (float)P.ap_N, apInv = TAB ? 1.0f / apN : 0.0f;

  // per view: <u0, w>, focus, and the aperture scale of |s - d_k|:
  // disk z = 2 pi rho |w| |s - d|, square arguments 2 rho w_x (s - d), 2 rho w_y (s - d)
  float pv[VB], sv[VB], g1[VB], g2[VB];
  int kind[VB];   // 0 pinhole, 1 disk, 2 square (uniform over the block)
#pragma unroll
  for (int v = 0; v < VB; ++v) {
    const ViewRec rv = s_v[v < nv ? v : 0];
    const int shape = __builtin_amdgcn_readfirstlane(rv.shape);
    const bool open = __builtin_amdgcn_readfirstlane(__float_as_int(rv.radius)) != 0 &&
                      __builtin_amdgcn_readfirstlane(__float_as_int(rv.radius)) != (int)0x80000000;
    kind[v] = open && (shape == 1 || shape == 2 || (TAB && shape == 3)) ? shape : 0;
    pv[v] = rv.u * wx + rv.v * wy;
    sv[v] = rv.focus;
    if (TAB && shape == 3) {   // continuous table index per unit of (s - d)
      g1[v] = rv.radius * wx * P.ap_scale;
      g2[v] = rv.radius * wy * P.ap_scale;
    } else {
      g1[v] = rv.shape == 1 ? (float)kTwoPi * rv.radius * wn : 2.0f * rv.radius * wx;
      g2[v] = 2.0f * rv.radius * wy;
    }
  }

  float2 acc[VB][CT];
#pragma unroll
  for (int v = 0; v < VB; ++v)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[v][c] = make_float2(0.f, 0.f);

  // Layer k + 1 (and d_{k+1}) is loaded while layer k is processed.  Loads
  // are unconditional (channel and layer indices clamped) so that the waits
  // name only the oldest batch; channels c >= C repeat channel C - 1 and are
  // never stored.  d travels as a vector load (lane-varying zero offset):
  // a scalar load would share its wait counter with the LDS table reads.
  int vzero;
  asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
  const float* dp = P.d + vzero;
  const float2* lp = P.layer_spec + f;
  float dn;
  float2 xn[CT];
  auto load_layer = [&](int k) {
    dn = dp[k];
#pragma unroll
    for (int c = 0; c < CT; ++c) xn[c] = lp[((size_t)k * C + (c < C ? c : C - 1)) * F];
  };
  load_layer(0);
  for (int k = 0; k < P.n; ++k) {
    const float dk = dn;
    float2 x[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) x[c] = xn[c];
    load_layer(min(k + 1, P.n - 1));
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      if (v < nv) {
        float s, co;
        sincos2pi_f(dk * pv[v], s, co);
        const float a = sv[v] - dk;
        float g = 1.0f;
        float pr, pi;
        if (TAB && kind[v] == 3) {
          const float2 q = aperture_tab(tabr, P.ap_N, apN, apInv, g1[v] * a, g2[v] * a);
          pr = co * q.x - s * q.y;
          pi = s * q.x + co * q.y;
        } else {
          if (kind[v] == 1) g = jinc_tab(s_jinc, g1[v] * fabsf(a));
          else if (kind[v] == 2) g = sinc_fast(g1[v] * a) * sinc_fast(g2[v] * a);
          pr = co * g;
          pi = s * g;
        }
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
  const int nchunks = (P.V + VB - 1) / VB;
  const int bin_blocks = (P.F + 255) / 256;
  if (P.ap_tab)
    hipLaunchKernelGGL((k_render<VB, CT, true>), dim3(bin_blocks * nchunks), dim3(256), 0, s, P, nchunks);
  else
    hipLaunchKernelGGL((k_render<VB, CT>), dim3(bin_blocks * nchunks), dim3(256), 0, s, P, nchunks);
  return hipGetLastError();
}

// Views per chunk: small chunks keep the accumulators few enough for high
// occupancy, and the layer values re-read by the chunks of one bin range come
// from the L2 of its XCD (sizes from a sweep on the 81-view 512^2 render).
hipError_t launch_render(const RenderParams& P, hipStream_t s) {
  switch (P.C) {
    case 1: return launch_render_vc<8, 1>(P, s);
    case 2: return launch_render_vc<6, 2>(P, s);
    case 3: return launch_render_vc<4, 3>(P, s);
    default: return launch_render_vc<4, 4>(P, s);
  }
}

// ---- drawn apertures (Sec. VI): spectrum samples of an aperture image ----
// table[ky][kx] = sum_{y,x} a[y][x] exp(-2 pi i (x kx + y ky) / N)
//                 * exp(+i pi (S - 1)(kx + ky) / N) / sum a,
// the DFT of the unit-sum S x S image zero-padded to N x N with the origin
// moved to the centre pixel.  One block per table row ky: the column sums
// c[x] = sum_y a[y][x] exp(-2 pi i y ky / N) go to LDS (FP64), then every
// thread finishes entries kx with a table of exp(-2 pi i r / N).
__global__ __launch_bounds__(256) void k_aperture_table(const float* __restrict__ img, int S, int N,
                                                        float2* __restrict__ table) {
  __shared__ double2 s_ph[kApMaxN];      // exp(-2 pi i r / N), r < N
  __shared__ double2 s_col[kApMaxS];
  __shared__ double s_sum[256];
  const int ky = blockIdx.x;
  const int t = threadIdx.x;
  for (int r = t; r < N; r += 256) {
    double sn, cs;
    sincospi(-2.0 * (double)r / (double)N, &sn, &cs);
    s_ph[r] = make_double2(cs, sn);
  }
  __syncthreads();
  double part = 0.0;
  for (int x = t; x < S; x += 256) {
    double re = 0.0, im = 0.0;
    for (int y = 0; y < S; ++y) {
      const double a = (double)img[(size_t)y * S + x];
      const double2 e = s_ph[(int)(((long long)y * ky) % N)];
      re = fma(a, e.x, re);
      im = fma(a, e.y, im);
      part += a;
    }
    s_col[x] = make_double2(re, im);
  }
  s_sum[t] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) s_sum[t] += s_sum[t + w];
    __syncthreads();
  }
  const double inv = 1.0 / s_sum[0];
  for (int kx = t; kx < N; kx += 256) {
    double re = 0.0, im = 0.0;
    for (int x = 0; x < S; ++x) {
      const double2 c = s_col[x];
      const double2 e = s_ph[(int)(((long long)x * kx) % N)];
      re += c.x * e.x - c.y * e.y;
      im += c.x * e.y + c.y * e.x;
    }
    // exp(+i pi (S - 1)(kx + ky) / N) = conj of the table entry at (S - 1)(kx + ky) / 2 mod N
    const long long q = ((long long)(S - 1) / 2 * (long long)(kx + ky)) % N;
    const double2 e = s_ph[(int)q];
    const double pr = re * e.x + im * e.y, pi = im * e.x - re * e.y;
    table[(size_t)ky * N + kx] = make_float2((float)(pr * inv), (float)(pi * inv));
  }
}

hipError_t launch_aperture_table(const float* img, int S, int N, float2* table, hipStream_t s) {
  hipLaunchKernelGGL(k_aperture_table, dim3(N), dim3(256), 0, s, img, S, N, table);
  return hipGetLastError();
}

// ---- relaxed model (Sec. VIII-B): the input views rendered with a free
// shift pair per view and layer, B_j(w) = sum_k exp(2 pi i <P_jk, w>) L_k(w)
// (the denoised output).  Same organisation as k_render: one thread per bin
// and a chunk of VB views; the chunk's shifts sit in LDS and every thread of
// the block reads the same entry (a broadcast).
template <int VB, int CT>
__global__ __launch_bounds__(256) void k_render_relaxed(RenderParams P, int nchunks) {
  __shared__ float2 s_sh[VB][FDL_MAX_LAYERS];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int bin_block = b / nchunks;
  const int v0 = (b - bin_block * nchunks) * VB;
  const int nv = min(VB, P.V - v0);
  const int n = P.n;
  for (int i = threadIdx.x; i < VB * n; i += blockDim.x) {
    const int v = i / n, k = i - v * n;
    s_sh[v][k] = v < nv ? P.shifts[(size_t)(v0 + v) * n + k] : make_float2(0.f, 0.f);
  }
  __syncthreads();

  const int f = bin_block * 256 + threadIdx.x;
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

  // layer k + 1 is loaded while layer k is processed (clamped, unconditional
  // loads; channels c >= C repeat channel C - 1 and are never stored)
  const float2* lp = P.layer_spec + f;
  float2 xn[CT];
  auto load_layer = [&](int k) {
#pragma unroll
    for (int c = 0; c < CT; ++c) xn[c] = lp[((size_t)k * C + (c < C ? c : C - 1)) * F];
  };
  load_layer(0);
  for (int k = 0; k < n; ++k) {
    float2 x[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) x[c] = xn[c];
    load_layer(min(k + 1, n - 1));
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      if (v < nv) {
        const float2 sh = s_sh[v][k];
        float si, co;
        sincos2pi_f(fmaf(sh.x, wx, sh.y * wy), si, co);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          acc[v][c].x = fmaf(co, x[c].x, fmaf(-si, x[c].y, acc[v][c].x));
          acc[v][c].y = fmaf(co, x[c].y, fmaf(si, x[c].x, acc[v][c].y));
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
static hipError_t launch_render_relaxed_vc(const RenderParams& P, hipStream_t s) {
  const int nchunks = (P.V + VB - 1) / VB;
  const int bin_blocks = (P.F + 255) / 256;
  hipLaunchKernelGGL((k_render_relaxed<VB, CT>), dim3(bin_blocks * nchunks), dim3(256), 0, s, P, nchunks);
  return hipGetLastError();
}

hipError_t launch_render_relaxed(const RenderParams& P, hipStream_t s) {
  switch (P.C) {
    case 1: return launch_render_relaxed_vc<8, 1>(P, s);
    case 2: return launch_render_relaxed_vc<6, 2>(P, s);
    case 3: return launch_render_relaxed_vc<4, 3>(P, s);
    default: return launch_render_relaxed_vc<4, 4>(P, s);
  }
}

}  // namespace fdl
