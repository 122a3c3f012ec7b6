// Internal launch interface between the C ABI (host.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdl {

// One light field for the construction kernels.  The disparities travel by
// value (n <= 32), together with the host's classification of them.
struct ConstructParams {
  const float2* view_spec;   // [m][C][F]
  const float2* u;           // [m] positions (sub-aperture inputs)
  const float* views;        // [m][5] fdl_view records (inputs with apertures) or null
  const float2* shifts = nullptr;   // [m][n] shift pairs of the relaxed model or null
  float2* layer_spec;        // [n][C][F]
  int* status;               // device counter or null
  int m, n, C, H, W, Wh, F;
  double lambda, eps;
  int reg;
  int toeplitz;              // 1: d is an arithmetic progression up to rounding
  double eta_max;            // max_k1<k2 |(d_k2-d_k1) - (d_{k2-k1}-d_0)|
  double region = 0.0;       // side of the camera-plane square of the finite-region regulariser
  int f_begin = 0, f_stop = 0;   // bins solved by the plain kernels: [f_begin, f_stop)
  double d[32];
};

struct RenderParams {
  const float2* layer_spec;  // [n][C][F]
  const float* d;            // [n]
  const void* views;         // [V] fdl_view (20 bytes each)
  const float2* shifts = nullptr;   // [V][n] shift pairs of the relaxed model (fdl_render_relaxed)
  const float2* ap_tab = nullptr;   // [N][N] drawn-aperture spectrum samples (shape 3) or null
  int ap_N = 0;
  float ap_scale = 0.f;             // 2N / S: table index per unit of rho (s - d) w
  float2* out_spec;          // [V][C][F]
  int n, C, H, W, Wh, F, V;
};

// Rows factorised by the team solver for n layers: the smallest class that
// holds n (the rows between n and the class are an identity block).  One
// kernel instantiation per class, so that small systems skip the padded work.
constexpr int kSolveRowClasses[] = {8, 16, 20, 24, 28, 30, 32};
inline int solve_rows(int n) {
  for (int c : kSolveRowClasses)
    if (n <= c) return c;
  return 32;
}
// plain construction (one 16-lane team per half-spectrum bin), by channel class
hipError_t launch_construct_c1(const ConstructParams& P, hipStream_t s);   // C == 1
hipError_t launch_construct_c3(const ConstructParams& P, hipStream_t s);   // C <= 3
hipError_t launch_construct_c4(const ConstructParams& P, hipStream_t s);   // C <= 4
inline hipError_t launch_construct(const ConstructParams& P, hipStream_t s) {
  return P.C == 1 ? launch_construct_c1(P, s) : (P.C <= 3 ? launch_construct_c3(P, s) : launch_construct_c4(P, s));
}
hipError_t launch_construct_views(const ConstructParams& P, hipStream_t s);   // inputs with apertures
hipError_t launch_construct_relaxed(const ConstructParams& P, hipStream_t s);   // free shifts per view and layer
hipError_t launch_construct_region(const ConstructParams& P, hipStream_t s);    // finite-region view regulariser
hipError_t launch_render(const RenderParams& P, hipStream_t s);
hipError_t launch_render_relaxed(const RenderParams& P, hipStream_t s);
constexpr int kApMaxS = 255;   // drawn aperture: image side (odd)
constexpr int kApMaxN = 2048;  // and padded table side
hipError_t launch_aperture_table(const float* img, int S, int N, float2* table, hipStream_t s);

// Mixed-radix (4, 2, 3) plan for one FFT length.
struct FftPlan {
  int N;
  int nst;
  int radix[24];
};

struct FftParams {
  float* real;      // [batch][H][W]
  float2* cplx;     // [batch][H][W/2+1]
  int batch, H, W;
  FftPlan row_plan; // length W/2
  FftPlan col_plan; // length H
  int col_tc;       // columns per block in the column pass
};

size_t fft_lds_limit();
hipError_t launch_rfft2(const FftParams& P, hipStream_t s);

struct CalibParams {
  const float2* view_spec;   // [m][C][F]
  const float2* u;           // [m]
  const float* d;            // [n]
  const int* freq_idx;       // [Q] or null (all F bins); clamped into [0, F)
  int* status = nullptr;     // device counter of out-of-range indices, or null
  double* partial;           // workspace [blocks][stride]
  double* loss;              // [1]
  double* grad_u;            // [m][2]
  double* grad_d;            // [n]
  const float2* shifts = nullptr;   // [m][n] relaxed model, or null (rank 1: d_k u_j)
  double* grad_p = nullptr;        // [m][n][2] relaxed model
  int m, n, C, H, W, Wh, F, Q;
  double lambda, eps, bscale;
  int reg, mode, stride;
};

size_t calib_lds_bytes(int m, int n, int C, int mode, bool relaxed = false);
constexpr int kCalibMaxBlocks = 2048;
int calib_blocks(int Q, size_t lds_per_block);
hipError_t launch_calib(const CalibParams& P, hipStream_t s);
// Allocation-free calibration: size of the static partial-sum array and its
// device address on the current device.
constexpr size_t kCalibScratchBytes = size_t(4) << 20;
hipError_t calib_scratch(double** out);
hipError_t launch_gd_step(float2* u, float* d, const double* gu, const double* gd, int m, int n, double alpha,
                          double eps_g, hipStream_t s);
hipError_t launch_irfft2(const FftParams& P, hipStream_t s);

}  // namespace fdl
