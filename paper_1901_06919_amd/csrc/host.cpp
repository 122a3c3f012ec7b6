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

// Factor N = 4^a 2^b 3^c into Stockham radices; false if N has another factor.
bool make_plan(int N, fdl::FftPlan& plan) {
  plan.N = N;
  plan.nst = 0;
  int v = N;
  while (v % 4 == 0 && plan.nst < 24) { plan.radix[plan.nst++] = 4; v /= 4; }
  while (v % 2 == 0 && plan.nst < 24) { plan.radix[plan.nst++] = 2; v /= 2; }
  while (v % 3 == 0 && plan.nst < 24) { plan.radix[plan.nst++] = 3; v /= 3; }
  return v == 1;
}

int fft_params(int batch, int H, int W, fdl::FftParams& P) {
  if (batch < 1 || H < 1 || H > 4096 || W < 2 || W > 8192 || (W & 1)) return FDL_ESHAPE;
  if (!make_plan(W / 2, P.row_plan) || !make_plan(H, P.col_plan)) return FDL_ESHAPE;
  P.batch = batch;
  P.H = H;
  P.W = W;
  // columns per block: up to 16 (128-byte row segments), within the LDS limit
  const size_t limit = fdl::fft_lds_limit() < 131072 ? fdl::fft_lds_limit() : 131072;
  int tc = 16;
  while (tc > 1 && (size_t)tc * (2 * H + 1) * 8 > limit) tc /= 2;
  P.col_tc = tc;
  return FDL_OK;
}

}  // namespace

namespace fdl_host {
// Classify the disparities: an arithmetic progression up to float rounding
// lets the kernels build A^H A from n Toeplitz moment sums.
void classify(const float* d, int n, fdl::ConstructParams& P) {
  double dmax = 0.0, eta = 0.0;
  for (int k = 0; k < 32; ++k) P.d[k] = k < n ? (double)d[k] : 0.0;
  for (int k = 0; k < n; ++k) dmax = std::fmax(dmax, std::fabs(P.d[k]));
  for (int k1 = 0; k1 < n; ++k1)
    for (int k2 = k1 + 1; k2 < n; ++k2)
      eta = std::fmax(eta, std::fabs((P.d[k2] - P.d[k1]) - (P.d[k2 - k1] - P.d[0])));
  P.eta_max = eta;
  P.toeplitz = eta <= 1e-5 * (1.0 + dmax) ? 1 : 0;
}

}  // namespace fdl_host

extern "C" {

const char* fdl_status_string(int code) {
  switch (code) {
    case FDL_OK: return "ok";
    case FDL_EINVAL: return "invalid argument";
    case FDL_ESHAPE: return "unsupported shape";
    case FDL_ENOMEM: return "out of memory or workspace too small";
    case FDL_EHIP: return "HIP runtime error";
    case FDL_ENUMERIC: return "numerical failure";
    case FDL_EUNSUPPORTED: return "not supported by this library version";
    case FDL_ETIMEOUT: return "timed out";
    default: return "unknown status";
  }
}

int fdl_version(void) { return 20000; }

int fdl_construct(const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_host, int m, int n, int C,
                  int H, int W, float lambda, float eps, int reg, fdl_c64* layer_spec_dev, int32_t* status_dev,
                  void* stream) {
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30)) return FDL_ESHAPE;
  return fdl_construct_bins(view_spec_dev, u_dev, d_host, m, n, C, H, W, lambda, eps, reg, 0, (int)F,
                            layer_spec_dev, status_dev, stream);
}

int fdl_construct_bins(const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_host, int m, int n, int C,
                       int H, int W, float lambda, float eps, int reg, int bin_begin, int bin_count,
                       fdl_c64* layer_spec_dev, int32_t* status_dev, void* stream) {
  if (!view_spec_dev || !u_dev || !d_host || !layer_spec_dev) return FDL_EINVAL;
  if (!(std::isfinite(lambda) && lambda >= 0.f) || !(std::isfinite(eps) && eps >= 0.f)) return FDL_EINVAL;
  if (reg < FDL_REG_VIEW2 || reg > FDL_REG_L2) return FDL_EINVAL;
  if (m < 1 || m > 4096 || n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(d_host[k])) return FDL_EINVAL;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30)) return FDL_ESHAPE;
  fdl::ConstructParams P;
  P.view_spec = reinterpret_cast<const float2*>(view_spec_dev);
  P.u = reinterpret_cast<const float2*>(u_dev);
  P.views = nullptr;
  P.layer_spec = reinterpret_cast<float2*>(layer_spec_dev);
  P.status = status_dev;
  P.m = m; P.n = n; P.C = C; P.H = H; P.W = W; P.Wh = W / 2 + 1; P.F = (int)F;
  P.lambda = (double)lambda; P.eps = (double)eps; P.reg = reg;
  if (bin_begin < 0 || bin_count < 1 || (long long)bin_begin + bin_count > F) return FDL_EINVAL;
  P.f_begin = bin_begin;
  P.f_stop = bin_begin + bin_count;
  fdl_host::classify(d_host, n, P);
  trace("construct m n C F", m, n, C, (int)F);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return map_hip(fdl::launch_construct(P, s));
}

int fdl_construct_views(const fdl_c64* view_spec_dev, const fdl_view* views_dev, const float* d_host, int m, int n,
                        int C, int H, int W, float lambda, float eps, int reg, fdl_c64* layer_spec_dev,
                        int32_t* status_dev, void* stream) {
  if (!view_spec_dev || !views_dev || !d_host || !layer_spec_dev) return FDL_EINVAL;
  if (!(std::isfinite(lambda) && lambda >= 0.f) || !(std::isfinite(eps) && eps >= 0.f)) return FDL_EINVAL;
  if (reg < FDL_REG_VIEW2 || reg > FDL_REG_L2) return FDL_EINVAL;
  if (m < 1 || m > 4096 || n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(d_host[k])) return FDL_EINVAL;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30)) return FDL_ESHAPE;
  fdl::ConstructParams P;
  P.view_spec = reinterpret_cast<const float2*>(view_spec_dev);
  P.u = nullptr;
  P.views = reinterpret_cast<const float*>(views_dev);
  P.layer_spec = reinterpret_cast<float2*>(layer_spec_dev);
  P.status = status_dev;
  P.m = m; P.n = n; P.C = C; P.H = H; P.W = W; P.Wh = W / 2 + 1; P.F = (int)F;
  P.lambda = (double)lambda; P.eps = (double)eps; P.reg = reg;
  fdl_host::classify(d_host, n, P);
  P.toeplitz = 0;   // the apertures scale each A_jk: no Toeplitz Gram
  trace("construct_views m n C F", m, n, C, (int)F);
  return map_hip(fdl::launch_construct_views(P, reinterpret_cast<hipStream_t>(stream)));
}

int fdl_render(const fdl_c64* layer_spec_dev, const float* d_dev, int n, int C, int H, int W,
               const fdl_view* views_dev, int V, fdl_c64* out_spec_dev, void* stream) {
  if (!layer_spec_dev || !d_dev || !views_dev || !out_spec_dev) return FDL_EINVAL;
  if (n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS || V < 1) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  const long long F = (long long)H * (W / 2 + 1);
  // one block per (256 bins, chunk of at least 4 views)
  if (F > (1LL << 30) || (F + 255) / 256 * ((V + 3) / 4) > 0x7fffffffLL) return FDL_ESHAPE;
  fdl::RenderParams P;
  P.layer_spec = reinterpret_cast<const float2*>(layer_spec_dev);
  P.d = d_dev;
  P.views = views_dev;
  P.out_spec = reinterpret_cast<float2*>(out_spec_dev);
  P.n = n; P.C = C; P.H = H; P.W = W; P.Wh = W / 2 + 1; P.F = (int)F; P.V = V;
  trace("render n C F V", n, C, (int)F, V);
  return map_hip(fdl::launch_render(P, reinterpret_cast<hipStream_t>(stream)));
}

int fdl_rfft2(const float* img_dev, fdl_c64* spec_dev, int batch, int H, int W, void* stream) {
  if (!img_dev || !spec_dev) return FDL_EINVAL;
  fdl::FftParams P;
  const int e = fft_params(batch, H, W, P);
  if (e != FDL_OK) return e;
  P.real = const_cast<float*>(img_dev);
  P.cplx = reinterpret_cast<float2*>(spec_dev);
  trace("rfft2 batch H W", batch, H, W, 0);
  return map_hip(fdl::launch_rfft2(P, reinterpret_cast<hipStream_t>(stream)));
}

int fdl_irfft2(fdl_c64* spec_dev, float* img_dev, int batch, int H, int W, void* stream) {
  if (!img_dev || !spec_dev) return FDL_EINVAL;
  fdl::FftParams P;
  const int e = fft_params(batch, H, W, P);
  if (e != FDL_OK) return e;
  P.real = img_dev;
  P.cplx = reinterpret_cast<float2*>(spec_dev);
  trace("irfft2 batch H W", batch, H, W, 0);
  return map_hip(fdl::launch_irfft2(P, reinterpret_cast<hipStream_t>(stream)));
}

size_t fdl_calib_workspace(int m, int n, int Q) {
  if (m < 1 || n < 1 || Q < 1) return 0;
  return (size_t)(Q < fdl::kCalibMaxBlocks ? Q : fdl::kCalibMaxBlocks) * (size_t)(1 + 2 * m + n) * sizeof(double);
}

int fdl_calib_grad(const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_dev, int m, int n, int C, int H,
                   int W, float lambda, float eps, int reg, int mode, const int32_t* freq_idx_dev, int Q,
                   double* loss_dev, double* grad_u_dev, double* grad_d_dev, int32_t* status_dev, void* ws_dev,
                   size_t ws_bytes, void* stream) {
  if (!view_spec_dev || !u_dev || !d_dev || !loss_dev || !grad_u_dev || !grad_d_dev || !ws_dev) return FDL_EINVAL;
  if (!(std::isfinite(lambda) && lambda >= 0.f) || !(std::isfinite(eps) && eps >= 0.f)) return FDL_EINVAL;
  if (reg < FDL_REG_VIEW2 || reg > FDL_REG_L2 || (mode != FDL_LOSS_FIT && mode != FDL_LOSS_LOO)) return FDL_EINVAL;
  if (m < 1 || m > 256 || n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30)) return FDL_ESHAPE;
  if (!freq_idx_dev) Q = (int)F;
  if (Q < 1) return FDL_EINVAL;
  if (ws_bytes < fdl_calib_workspace(m, n, Q)) return FDL_ENOMEM;
  if (fdl::calib_lds_bytes(m, n, C, mode) > fdl::fft_lds_limit()) return FDL_ESHAPE;
  fdl::CalibParams P;
  P.view_spec = reinterpret_cast<const float2*>(view_spec_dev);
  P.u = reinterpret_cast<const float2*>(u_dev);
  P.d = d_dev;
  P.freq_idx = freq_idx_dev;
  P.status = status_dev;
  P.partial = static_cast<double*>(ws_dev);
  P.loss = loss_dev;
  P.grad_u = grad_u_dev;
  P.grad_d = grad_d_dev;
  P.m = m; P.n = n; P.C = C; P.H = H; P.W = W; P.Wh = W / 2 + 1; P.F = (int)F; P.Q = Q;
  P.lambda = (double)lambda; P.eps = (double)eps; P.bscale = 1.0 / std::sqrt((double)H * (double)W);
  P.reg = reg; P.mode = mode; P.stride = 1 + 2 * m + n;
  trace("calib m n Q mode", m, n, Q, mode);
  return map_hip(fdl::launch_calib(P, reinterpret_cast<hipStream_t>(stream)));
}

int fdl_calib_grad_noalloc(const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_dev, int m, int n,
                           int C, int H, int W, float lambda, float eps, int reg, int mode, const int32_t* freq_idx_dev,
                           int Q, double* loss_dev, double* grad_u_dev, double* grad_d_dev, int32_t* status_dev,
                           void* stream) {
  // same checks as fdl_calib_grad, then the partial sums go to the library's
  // static array instead of a caller's workspace (no allocation of any kind)
  if (!view_spec_dev || !u_dev || !d_dev || !loss_dev || !grad_u_dev || !grad_d_dev) return FDL_EINVAL;
  if (m < 1 || m > 256 || n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30)) return FDL_ESHAPE;
  const int Qeff = freq_idx_dev ? Q : (int)F;
  if (Qeff < 1) return FDL_EINVAL;
  const size_t need = fdl_calib_workspace(m, n, Qeff);
  if (need > fdl::kCalibScratchBytes) return FDL_ENOMEM;
  double* scratch_dev = nullptr;
  const int e = map_hip(fdl::calib_scratch(&scratch_dev));
  if (e != FDL_OK) return e;
  return fdl_calib_grad(view_spec_dev, u_dev, d_dev, m, n, C, H, W, lambda, eps, reg, mode, freq_idx_dev, Q, loss_dev,
                        grad_u_dev, grad_d_dev, status_dev, scratch_dev, fdl::kCalibScratchBytes, stream);
}

int fdl_gd_step(fdl_f2* u_dev, float* d_dev, const double* grad_u_dev, const double* grad_d_dev, int m, int n,
                double alpha, double eps_g, void* stream) {
  if (!u_dev || !d_dev || !grad_u_dev || !grad_d_dev) return FDL_EINVAL;
  if (m < 1 || n < 1 || !std::isfinite(alpha) || !(eps_g >= 0.0)) return FDL_EINVAL;
  return map_hip(fdl::launch_gd_step(reinterpret_cast<float2*>(u_dev), d_dev, grad_u_dev, grad_d_dev, m, n, alpha,
                                     eps_g, reinterpret_cast<hipStream_t>(stream)));
}

// ---- finite-region view regulariser (Eq. GTG) ----

int fdl_construct_region(const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_host, int m, int n, int C,
                         int H, int W, float lambda, float eps, float region, fdl_c64* layer_spec_dev,
                         int32_t* status_dev, void* stream) {
  if (!view_spec_dev || !u_dev || !d_host || !layer_spec_dev) return FDL_EINVAL;
  if (!(std::isfinite(lambda) && lambda >= 0.f) || !(std::isfinite(eps) && eps >= 0.f)) return FDL_EINVAL;
  if (!(std::isfinite(region) && region > 0.f)) return FDL_EINVAL;
  if (m < 1 || m > 4096 || n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(d_host[k])) return FDL_EINVAL;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30)) return FDL_ESHAPE;
  fdl::ConstructParams P;
  P.view_spec = reinterpret_cast<const float2*>(view_spec_dev);
  P.u = reinterpret_cast<const float2*>(u_dev);
  P.views = nullptr;
  P.layer_spec = reinterpret_cast<float2*>(layer_spec_dev);
  P.status = status_dev;
  P.m = m; P.n = n; P.C = C; P.H = H; P.W = W; P.Wh = W / 2 + 1; P.F = (int)F;
  P.lambda = (double)lambda; P.eps = (double)eps;
  P.reg = FDL_REG_VIEW2;          // diagonal of the view regulariser; the dense part is added on top
  P.region = (double)region;
  fdl_host::classify(d_host, n, P);
  trace("construct_region m n C F", m, n, C, (int)F);
  return map_hip(fdl::launch_construct_region(P, reinterpret_cast<hipStream_t>(stream)));
}

// ---- drawn apertures (Sec. VI) ----

int fdl_aperture_table(const float* img_dev, int S, int pad, fdl_c64* table_dev, void* stream) {
  if (!img_dev || !table_dev) return FDL_EINVAL;
  if (S < 1 || S > fdl::kApMaxS || !(S & 1) || pad < 1 || (long long)pad * S > fdl::kApMaxN) return FDL_ESHAPE;
  trace("aperture_table S N", S, pad * S, 0, 0);
  return map_hip(fdl::launch_aperture_table(img_dev, S, pad * S, reinterpret_cast<float2*>(table_dev),
                                            reinterpret_cast<hipStream_t>(stream)));
}

int fdl_render_tabulated(const fdl_c64* layer_spec_dev, const float* d_dev, int n, int C, int H, int W,
                         const fdl_view* views_dev, int V, const fdl_c64* table_dev, int N, int S,
                         fdl_c64* out_spec_dev, void* stream) {
  if (!table_dev) return FDL_EINVAL;
  if (S < 1 || S > fdl::kApMaxS || !(S & 1) || N < S || N > fdl::kApMaxN || N % S) return FDL_ESHAPE;
  if (!layer_spec_dev || !d_dev || !views_dev || !out_spec_dev) return FDL_EINVAL;
  if (n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS || V < 1) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30) || (F + 255) / 256 * ((V + 3) / 4) > 0x7fffffffLL) return FDL_ESHAPE;
  fdl::RenderParams P;
  P.layer_spec = reinterpret_cast<const float2*>(layer_spec_dev);
  P.d = d_dev;
  P.views = views_dev;
  P.out_spec = reinterpret_cast<float2*>(out_spec_dev);
  P.n = n; P.C = C; P.H = H; P.W = W; P.Wh = W / 2 + 1; P.F = (int)F; P.V = V;
  P.ap_tab = reinterpret_cast<const float2*>(table_dev);
  P.ap_N = N;
  P.ap_scale = (float)(2.0 * N / S);
  trace("render_tabulated n C F V", n, C, (int)F, V);
  return map_hip(fdl::launch_render(P, reinterpret_cast<hipStream_t>(stream)));
}

// ---- relaxed model (Sec. VIII-B): a free shift pair per view and layer ----

int fdl_construct_relaxed(const fdl_c64* view_spec_dev, const fdl_f2* shifts_dev, int m, int n, int C, int H, int W,
                          float lambda, float eps, int reg, fdl_c64* layer_spec_dev, int32_t* status_dev,
                          void* stream) {
  if (!view_spec_dev || !shifts_dev || !layer_spec_dev) return FDL_EINVAL;
  if (!(std::isfinite(lambda) && lambda >= 0.f) || !(std::isfinite(eps) && eps >= 0.f)) return FDL_EINVAL;
  if (reg != FDL_REG_LAYER2 && reg != FDL_REG_L2) return FDL_EINVAL;   // no disparities: no view regulariser
  if (m < 1 || m > 4096 || n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30)) return FDL_ESHAPE;
  fdl::ConstructParams P;
  P.view_spec = reinterpret_cast<const float2*>(view_spec_dev);
  P.u = nullptr;
  P.views = nullptr;
  P.shifts = reinterpret_cast<const float2*>(shifts_dev);
  P.layer_spec = reinterpret_cast<float2*>(layer_spec_dev);
  P.status = status_dev;
  P.m = m; P.n = n; P.C = C; P.H = H; P.W = W; P.Wh = W / 2 + 1; P.F = (int)F;
  P.lambda = (double)lambda; P.eps = (double)eps; P.reg = reg;
  P.toeplitz = 0;
  P.eta_max = 0.0;
  for (int k = 0; k < 32; ++k) P.d[k] = 0.0;
  trace("construct_relaxed m n C F", m, n, C, (int)F);
  return map_hip(fdl::launch_construct_relaxed(P, reinterpret_cast<hipStream_t>(stream)));
}

int fdl_render_relaxed(const fdl_c64* layer_spec_dev, const fdl_f2* shifts_dev, int n, int C, int H, int W, int V,
                       fdl_c64* out_spec_dev, void* stream) {
  if (!layer_spec_dev || !shifts_dev || !out_spec_dev) return FDL_EINVAL;
  if (n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS || V < 1) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30) || (F + 255) / 256 * ((V + 3) / 4) > 0x7fffffffLL) return FDL_ESHAPE;
  fdl::RenderParams P;
  P.layer_spec = reinterpret_cast<const float2*>(layer_spec_dev);
  P.d = nullptr;
  P.views = nullptr;
  P.shifts = reinterpret_cast<const float2*>(shifts_dev);
  P.out_spec = reinterpret_cast<float2*>(out_spec_dev);
  P.n = n; P.C = C; P.H = H; P.W = W; P.Wh = W / 2 + 1; P.F = (int)F; P.V = V;
  trace("render_relaxed n C F V", n, C, (int)F, V);
  return map_hip(fdl::launch_render_relaxed(P, reinterpret_cast<hipStream_t>(stream)));
}

size_t fdl_calib_relaxed_workspace(int m, int n, int Q) {
  if (m < 1 || n < 1 || Q < 1) return 0;
  return (size_t)(Q < fdl::kCalibMaxBlocks ? Q : fdl::kCalibMaxBlocks) * (size_t)(1 + 2 * m * n) * sizeof(double);
}

int fdl_calib_grad_relaxed(const fdl_c64* view_spec_dev, const fdl_f2* shifts_dev, int m, int n, int C, int H, int W,
                           float lambda, float eps, int reg, int mode, const int32_t* freq_idx_dev, int Q,
                           double* loss_dev, double* grad_shifts_dev, int32_t* status_dev, void* ws_dev,
                           size_t ws_bytes, void* stream) {
  if (!view_spec_dev || !shifts_dev || !loss_dev || !grad_shifts_dev || !ws_dev) return FDL_EINVAL;
  if (!(std::isfinite(lambda) && lambda >= 0.f) || !(std::isfinite(eps) && eps >= 0.f)) return FDL_EINVAL;
  if ((reg != FDL_REG_LAYER2 && reg != FDL_REG_L2) || (mode != FDL_LOSS_FIT && mode != FDL_LOSS_LOO))
    return FDL_EINVAL;
  if (m < 1 || m > 256 || n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS) return FDL_ESHAPE;
  if (H < 1 || W < 2 || (W & 1)) return FDL_ESHAPE;
  const long long F = (long long)H * (W / 2 + 1);
  if (F > (1LL << 30)) return FDL_ESHAPE;
  if (!freq_idx_dev) Q = (int)F;
  if (Q < 1) return FDL_EINVAL;
  if (ws_bytes < fdl_calib_relaxed_workspace(m, n, Q)) return FDL_ENOMEM;
  if (fdl::calib_lds_bytes(m, n, C, mode, true) > fdl::fft_lds_limit()) return FDL_ESHAPE;
  fdl::CalibParams P;
  P.view_spec = reinterpret_cast<const float2*>(view_spec_dev);
  P.u = nullptr;
  P.d = nullptr;
  P.shifts = reinterpret_cast<const float2*>(shifts_dev);
  P.freq_idx = freq_idx_dev;
  P.status = status_dev;
  P.partial = static_cast<double*>(ws_dev);
  P.loss = loss_dev;
  P.grad_u = nullptr;
  P.grad_d = nullptr;
  P.grad_p = grad_shifts_dev;
  P.m = m; P.n = n; P.C = C; P.H = H; P.W = W; P.Wh = W / 2 + 1; P.F = (int)F; P.Q = Q;
  P.lambda = (double)lambda; P.eps = (double)eps; P.bscale = 1.0 / std::sqrt((double)H * (double)W);
  P.reg = reg; P.mode = mode; P.stride = 1 + 2 * m * n;
  trace("calib_relaxed m n Q mode", m, n, Q, mode);
  return map_hip(fdl::launch_calib(P, reinterpret_cast<hipStream_t>(stream)));
}

int fdl_gd_step_relaxed(fdl_f2* shifts_dev, const double* grad_shifts_dev, int m, int n, double alpha, double eps_g,
                        void* stream) {
  if (!shifts_dev || !grad_shifts_dev) return FDL_EINVAL;
  if (m < 1 || n < 1 || (long long)m * n > (1LL << 24) || !std::isfinite(alpha) || !(eps_g >= 0.0))
    return FDL_EINVAL;
  // the shift pairs are updated as one vector of m n positions; no disparities
  return map_hip(fdl::launch_gd_step(reinterpret_cast<float2*>(shifts_dev), nullptr, grad_shifts_dev, nullptr, m * n,
                                     0, alpha, eps_g, reinterpret_cast<hipStream_t>(stream)));
}

}  // extern "C"
