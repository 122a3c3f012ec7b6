/*
 * fdl.h -- C ABI of the MI355X Fourier Disparity Layer library (libfdl.so).
 *
 * The library implements the per-frequency hot path of the Fourier Disparity
 * Layer (FDL) representation (Le Pendu, Guillemot, Smolic, "A Fourier
 * Disparity Layer representation for Light Fields"):
 *   - the 2D real DFT of the input views and its inverse (Sec. V-A, Sec. VII),
 *   - layer construction: at every spatial frequency w a regularised least
 *     squares solve x = (A^H A + lambda Gamma^H Gamma + eps I)^-1 A^H b
 *     (Eq. LayerConstructionClosedForm) with A_jk = exp(+2 pi i d_k <u_j, w>)
 *     (Eq. AMatGeneral for sub-aperture inputs),
 *   - rendering: B(w) = sum_k exp(+2 pi i d_k <u0, w>) psi_hat((s - d_k) w) L_k(w)
 *     (Eq. BsFourier),
 *   - the calibration objective and its gradient with respect to the view
 *     positions u_j and disparities d_k (Eqs. CalibrationProb, gradD, gradP),
 *     and a leave-one-out variant with a hand-written adjoint,
 *   - the normalised gradient step on (u, d) (Sec. V-B),
 *   - a batched construction of many uneven light fields in one persistent
 *     launch (a plan object, so the launch can be captured in a HIP graph),
 *   - construction from input views taken with their own apertures
 *     (Eq. AMatGeneral: focal stacks, wide-aperture and mixed inputs),
 *   - the relaxed model of Sec. VIII-B (a free shift per view and layer):
 *     its calibration gradient and update, construction and rendering,
 *   - drawn apertures (Sec. VI): the spectrum of a zero-padded aperture image
 *     and rendering with it,
 *   - the view regulariser over a finite camera-plane region (Eq. GTG).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named *_dev are DEVICE pointers (hipMalloc / torch CUDA tensors),
 *    contiguous, in the layouts stated below.  The caller owns every buffer;
 *    the library keeps no pointer after a call returns (plans excepted, see
 *    there).
 *  - Spectra are complex64 interleaved (re, im), half spectrum of a real
 *    image: [..][H][W/2+1], bin f = ky*(W/2+1) + kx, unnormalised forward DFT
 *    sum_x img(x) exp(-2 pi i <x, w>).  Frequencies are in cycles/pixel:
 *    w_x = kx/W (kx = 0..W/2), w_y = ky/H for ky < H/2 else (ky-H)/H.
 *  - A view position is (u, v) = (horizontal, vertical) in view-grid units;
 *    disparities are pixels per unit of position.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    compute entry points enqueue asynchronously on it and never synchronise.
 *  - Return value: FDL_OK or a negative fdl_status.  Argument and shape errors
 *    are detected on the host before anything is enqueued; HIP launch errors
 *    are returned as FDL_EHIP.  Numerical events detected on the device (a
 *    non-positive Cholesky pivot) are counted into an optional device int32.
 */
#ifndef FDL_H
#define FDL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } fdl_c64;          /* == torch.complex64 element */
typedef struct { float x, y; } fdl_f2;             /* view position (u, v) */

/* One render request: position (u, v), focus disparity s, aperture radius rho
 * (view units; disk radius or square half-side, 0 = pinhole) and shape. */
typedef struct { float u, v, focus, radius; int32_t shape; } fdl_view;

enum fdl_status {
  FDL_OK = 0,
  FDL_EINVAL = -1,        /* null pointer, non-finite or out-of-range scalar */
  FDL_ESHAPE = -2,        /* unsupported size (see each entry point) */
  FDL_ENOMEM = -3,        /* workspace too small / device allocation failed */
  FDL_EHIP = -4,          /* HIP runtime or launch error */
  FDL_ENUMERIC = -5,      /* reserved for numerical failures reported on the host */
  FDL_EUNSUPPORTED = -6,  /* valid request this library version does not implement */
  FDL_ETIMEOUT = -7       /* a wait ended before the work it waited for */
};

enum fdl_reg {
  FDL_REG_VIEW2 = 0,      /* lambda diag(|w|^4 d_k^4): Eq. 2ndOrderView (2D, r -> inf) */
  FDL_REG_LAYER2 = 1,     /* lambda Gamma^T Gamma, Gamma = tridiag(1,-2,1): Eq. 2ndOrderLayer */
  FDL_REG_L2 = 2          /* lambda I (classical l2, Sec. V-C) */
};

enum fdl_loss {
  FDL_LOSS_FIT = 0,       /* Eq. CalibrationProb, gradient by Eqs. gradP/gradD */
  FDL_LOSS_LOO = 1        /* leave-one-out view prediction error, exact adjoint */
};

enum fdl_aperture {
  FDL_AP_PINHOLE = 0,     /* psi = delta, psi_hat = 1 */
  FDL_AP_DISK = 1,        /* unit-integral disk of radius rho: 2 J1(z)/z, z = 2 pi rho |xi| */
  FDL_AP_SQUARE = 2,      /* unit-integral square of half-side rho: sinc(2 rho xi_x) sinc(2 rho xi_y) */
  FDL_AP_IMAGE = 3        /* drawn aperture scaled to half-side rho (fdl_render_tabulated); pinhole elsewhere */
};

/* Limits of the library. */
#define FDL_MAX_LAYERS 32
#define FDL_MAX_CHANNELS 4

/* Human-readable text for a status code (static storage). */
const char* fdl_status_string(int code);

/* Library version: major*10000 + minor*100 + patch. */
int fdl_version(void);

/* ---------------------------------------------------------------------------
 * Real 2D DFT (Sec. V-A: the layers are fitted to the DFT of each input
 * image; Sec. VII: only the Hermitian half of each spectrum is computed).
 *   img_dev  [batch][H][W] float32  ->  spec_dev [batch][H][W/2+1] complex64,
 *   X[ky][kx] = sum_{y,x} img[y][x] exp(-2 pi i (ky y / H + kx x / W)), unnormalised.
 * H and W/2 must be products of powers of 2 and 3 (128, 192, 256, 384, 512,
 * ...); 1 <= H <= 4096, 2 <= W <= 8192, W even.  FDL_ESHAPE otherwise.
 * The buffers must not overlap.
 * ------------------------------------------------------------------------- */
int fdl_rfft2(const float* img_dev, fdl_c64* spec_dev, int batch, int H, int W, void* stream);

/* Inverse of fdl_rfft2 with 1/(H W) normalisation:
 *   spec_dev [batch][H][W/2+1] complex64 -> img_dev [batch][H][W] float32.
 * The half spectrum is extended by Hermitian symmetry; the imaginary parts of
 * the self-conjugate bins of columns kx = 0 and kx = W/2 (after the column
 * transform) do not contribute (numpy irfft2 semantics).  spec_dev is used as
 * scratch: its contents are DESTROYED.  Same size rules as fdl_rfft2. */
int fdl_irfft2(fdl_c64* spec_dev, float* img_dev, int batch, int H, int W, void* stream);

/* ---------------------------------------------------------------------------
 * Layer construction (Sec. V-A, Eq. LayerConstructProb and its closed form
 * Eq. LayerConstructionClosedForm), sub-aperture inputs (psi_j = delta).
 *
 * For every half-spectrum bin w, independently:
 *   A_jk = exp(+2 pi i d_k <u_j, w>)                       (m x n)
 *   M    = A^H A + lambda R(w) + eps I                     (n x n, Hermitian PD)
 *   x_c  = M^-1 A^H b_c  for each channel c                (M shared by channels)
 * with R(w) = diag(|w|^4 d_k^4) (FDL_REG_VIEW2), tridiag(1,-2,1)^T tridiag(1,-2,1)
 * (FDL_REG_LAYER2) or I (FDL_REG_L2); eps is the small diagonal term that makes
 * the DC bin solvable (remark after Eq. 2ndOrderView), added outside lambda.
 *
 *   view_spec_dev  [m][C][H][W/2+1] complex64  (b_j = spectrum of view j)
 *   u_dev          [m] fdl_f2                  view positions (any values).  With
 *                  Toeplitz sums (below) and positions on an exact lattice in
 *                  raster order, u_j = u_0 + a g1 + b g2 for j = a B + b with
 *                  B <= 16 (checked on the device in FP64), the phases are
 *                  stepped from view to view and the moment sums taken in
 *                  closed form; the result is the same up to rounding.
 *   d_host         [n] float32, HOST memory     layer disparities (any values);
 *                  read during the call and passed to the kernels by value.
 *                  When they form an arithmetic progression up to float rounding
 *                  the Gram matrix is built from n Toeplitz moment sums (exact to
 *                  FP64; a bin whose positions make that expansion inexact,
 *                  |2 pi eta p| > 3e-4, is counted in status_dev), otherwise from
 *                  all n(n+1)/2 products.
 *   layer_spec_dev [n][C][H][W/2+1] complex64  output layer spectra
 *   status_dev     int32 device counter or NULL: incremented once per bin whose
 *                  Cholesky factorisation met a non-positive pivot (the pivot
 *                  is then replaced by a tiny positive value and the result is
 *                  not meaningful for that bin) or whose moment expansion was
 *                  out of range (see d_host).
 * Requires 1 <= m <= 4096, 1 <= n <= FDL_MAX_LAYERS, 1 <= C <= FDL_MAX_CHANNELS,
 * H >= 1, W >= 2 even, lambda >= 0, eps >= 0 (eps > 0 needed for a solvable DC
 * bin with the view regulariser).  The solve is carried out in FP64 from the
 * complex64 inputs; outputs are rounded to complex64.
 * ------------------------------------------------------------------------- */
int fdl_construct(const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_host,
                  int m, int n, int C, int H, int W, float lambda, float eps, int reg,
                  fdl_c64* layer_spec_dev, int32_t* status_dev, void* stream);

/* fdl_construct restricted to the bins [bin_begin, bin_begin + bin_count) of
 * the half spectrum (flat index f = ky (W/2+1) + kx): the same per-bin
 * solves, written to the same places of layer_spec_dev; the other bins of
 * the output are not touched.  The bins of a frequency are independent
 * (Eq. LayerConstructionClosedForm holds per w), so a construction may be
 * split into ranges: the request server splits long constructions so that
 * renders can run between the pieces, and a multi-GPU construction would
 * give each device its range.  FDL_EINVAL unless 0 <= bin_begin and
 * 1 <= bin_count <= F - bin_begin; other arguments and errors as
 * fdl_construct. */
int fdl_construct_bins(const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_host,
                       int m, int n, int C, int H, int W, float lambda, float eps, int reg,
                       int bin_begin, int bin_count, fdl_c64* layer_spec_dev, int32_t* status_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Rendering (Sec. IV-B Eq. BsFourier; Sec. VI): for each request v and bin w
 *   B_v(w) = sum_k exp(+2 pi i d_k <(u_v, v_v), w>) psi_hat_v((s_v - d_k) w) L_k(w)
 * with unit-integral apertures (psi_hat(0) = 1; radius 0 is a sub-aperture
 * view for every shape).
 *
 *   layer_spec_dev [n][C][H][W/2+1] complex64
 *   d_dev          [n] float32
 *   views_dev      [V] fdl_view
 *   out_spec_dev   [V][C][H][W/2+1] complex64
 * Requires 1 <= n <= FDL_MAX_LAYERS, 1 <= C <= FDL_MAX_CHANNELS, V >= 1,
 * W >= 2 even.  Shapes outside {PINHOLE, DISK, SQUARE} render as pinhole.
 * ------------------------------------------------------------------------- */
int fdl_render(const fdl_c64* layer_spec_dev, const float* d_dev, int n, int C, int H, int W,
               const fdl_view* views_dev, int V, fdl_c64* out_spec_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Layer construction from input views that carry their own apertures
 * (Eq. AMatGeneral: focal stacks, wide-aperture or mixed inputs, Sec. V-A):
 *   A_jk = exp(2 pi i d_k <u_j, w>) psi_hat_j((s_j - d_k) w),
 * psi_hat_j the unit-integral aperture spectrum of input view j, as in
 * fdl_render (disk of radius rho: 2 J1(z)/z, z = 2 pi rho |xi|; square of
 * half-side rho: sinc(2 rho xi_x) sinc(2 rho xi_y); pinhole or rho = 0: 1),
 * s_j its focus; then M and x exactly as fdl_construct.  The aperture spectra
 * are evaluated in FP64 (power series / Hankel expansion of J1, about 1e-13).
 *   views_dev [m] fdl_view on the device: (u, v) position, focus s, radius,
 *   shape of each INPUT view (the same record as a rendered view);
 *   all other arguments, layouts and errors as fdl_construct.
 * The Toeplitz form of A^H A does not apply (|A_jk| varies), so the cost per
 * bin grows as m n^2 instead of m n. */
int fdl_construct_views(const fdl_c64* view_spec_dev, const fdl_view* views_dev, const float* d_host, int m, int n,
                        int C, int H, int W, float lambda, float eps, int reg, fdl_c64* layer_spec_dev,
                        int32_t* status_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Calibration loss and gradient (Sec. V-B).  Over the Q bins freq_idx_dev
 * (flat half-spectrum indices, or all F = H(W/2+1) bins when freq_idx_dev is
 * NULL), with orthonormal spectra b = view_spec / sqrt(H W):
 *
 * FDL_LOSS_FIT (Eq. CalibrationProb, summed over the sampled bins):
 *   E = sum_q [ ||A x_q - b_q||^2 + lambda ||Gamma x_q||^2 + eps ||x_q||^2 ],
 *   x_q the minimiser; gradient by Eqs. gradP / gradD generalised to 2D:
 *   G_jk = 4 pi Im(conj(x_k) conj(A_jk) r_j), r = A x - b,
 *   grad u_j = sum_q sum_k d_k G_jk w_q, grad d_k = sum_q sum_j G_jk <u_j, w_q>.
 *   Exact when the regulariser does not depend on d (FDL_REG_LAYER2, FDL_REG_L2).
 * FDL_LOSS_LOO (leave-one-out view prediction):
 *   E = sum_q sum_j |r_j / (1 - h_jj)|^2, r = b - A x, h_jj = a_j M^-1 a_j^H,
 *   which equals the error of predicting view j from the layers fitted without
 *   it; the gradient back-propagates through M^-1 (hand-written adjoint).
 *
 *   loss_dev   [1] double, grad_u_dev [m][2] double, grad_d_dev [n] double.
 *   status_dev int32 device counter or NULL: incremented once for every entry
 *   of freq_idx_dev outside [0, F).  Such an index is clamped into [0, F) (the
 *   nearest end) and that bin is used in its place, so no access leaves
 *   view_spec_dev and the outputs stay finite; the result is then that of the
 *   clamped index set.
 *   ws_dev / ws_bytes: device workspace of at least fdl_calib_workspace(m, n, Q)
 *   bytes (per-block partial sums; reduced deterministically on the device).
 * Requires 1 <= m <= 256, 1 <= n <= FDL_MAX_LAYERS, 1 <= C <= FDL_MAX_CHANNELS,
 * Q >= 1 when freq_idx_dev != NULL, and the per-bin system
 * must fit the LDS one block may use on the device (160 KiB on MI355X):
 * 8 * max(2mn + 2n^2 + n + 4mC + 2nC + m + mn, 256) bytes for FIT, plus
 * 8 * (2nm + 4mC + 2nC + m) for LOO (FDL_ESHAPE otherwise; m = 49, n = 16,
 * C = 1 needs 39 KiB in LOO mode, m = 81, n = 30, C = 3 FIT 81 KiB).
 * With FDL_REG_VIEW2 the regulariser depends on d; its derivative is not
 * included (the paper pairs calibration with the layer regulariser).
 * ------------------------------------------------------------------------- */
size_t fdl_calib_workspace(int m, int n, int Q);
int fdl_calib_grad(const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_dev,
                   int m, int n, int C, int H, int W, float lambda, float eps, int reg, int mode,
                   const int32_t* freq_idx_dev, int Q,
                   double* loss_dev, double* grad_u_dev, double* grad_d_dev,
                   int32_t* status_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Allocation-free variant of fdl_calib_grad, for callers that cannot
 * allocate device memory or pass a workspace (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  Same arguments,
 * results (bit for bit), status and errors as fdl_calib_grad, without ws_dev
 * and ws_bytes: the per-block partial sums live in a static 4 MiB array of
 * the library on each GPU (allocated with the library, held until the process
 * ends).  Sizes whose workspace, fdl_calib_workspace(m, n, Q), exceeds 4 MiB
 * are rejected with FDL_ENOMEM before anything is enqueued (m = 49, n = 16
 * needs 1.8 MiB at any Q; m = 256, n = 32 fits for Q <= 961).  Every call on
 * one GPU uses that GPU's array: calls that overlap in time on one GPU (other
 * streams, other host threads) race and must be serialised by the caller.
 * Calls nothing that allocates. */
int fdl_calib_grad_noalloc(const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_dev,
                           int m, int n, int C, int H, int W, float lambda, float eps, int reg, int mode,
                           const int32_t* freq_idx_dev, int Q, double* loss_dev, double* grad_u_dev,
                           double* grad_d_dev, int32_t* status_dev, void* stream);

/* The normalised gradient step of Sec. V-B on the device:
 *   u <- u - alpha grad_u / (eps_g + ||grad_u||^2),  d <- d - alpha grad_d / (eps_g + ||grad_d||^2)
 * (squared norms as printed; alpha = 0.2 in the paper).  Computed in FP64,
 * stored back to the float32 parameters.  u_dev [m] fdl_f2, d_dev [n] float32. */
int fdl_gd_step(fdl_f2* u_dev, float* d_dev, const double* grad_u_dev, const double* grad_d_dev,
                int m, int n, double alpha, double eps_g, void* stream);

/* ---------------------------------------------------------------------------
 * Batched construction of uneven light fields (same mathematics as
 * fdl_construct for each light field) in one launch per channel/disparity
 * class, or one launch per solved-row class within it, as the plan's mode
 * selects (the autotuner picks the mode that measures fastest on the plan's
 * own data).
 *
 * fdl_batch_plan_create reads a HOST array of B descriptors, validates them,
 * chooses the launch shape (defaults, or the autotuner's choice), and
 * uploads the descriptors and a work table to device memory it allocates.
 * The plan keeps the device pointers of the descriptors until it is destroyed:
 * the buffers they point at must stay valid while the plan is executed.
 * fdl_batch_plan_execute only enqueues the kernel (graph-capturable).
 * ------------------------------------------------------------------------- */
typedef struct fdl_lf_desc {
  const fdl_c64* view_spec;   /* device [m][C][H][W/2+1] */
  const fdl_f2* u;            /* device [m] */
  const float* d;             /* device [n] */
  fdl_c64* layer_spec;        /* device [n][C][H][W/2+1] output */
  int32_t* status;            /* device counter or NULL */
  int32_t m, n, C, H, W, reg;
  float lambda, eps;
} fdl_lf_desc;

typedef struct fdl_batch_plan fdl_batch_plan;

/* descs_host: B descriptors in HOST memory (their pointers are device
 * pointers).  Light fields are grouped by channel count and disparity class.
 * mode 0 = flat: one block per 16-bin tile, one launch per solved-row class
 * (the smallest of 8, 16, 20, 24, 28, 30, 32 rows that holds n); mode 1 =
 * persistent: a grid of (blocks per CU x CUs) blocks pulls tiles from an
 * atomic queue, one launch per row-slot class (n <= 16 or n <= 32); mode 2 =
 * flat single: every light field through the n <= 32 solver, so one launch
 * covers all light fields of a channel/disparity class; mode 3 = persistent
 * single: the atomic queue of mode 1 over all light fields of a
 * channel/disparity class through the n <= 32 solver (one launch per class).
 * Launches are ordered largest group first, tiles largest light field first
 * within a launch.  The disparities of each light field are read once
 * (blocking) and classified as fdl_construct does.  Argument errors as
 * fdl_construct. */
int fdl_batch_plan_create(const fdl_lf_desc* descs_host, int B, int mode, fdl_batch_plan** plan_out);
/* Enqueue the plan's launch(es) on `stream`; allocates nothing and issues no
 * memset (each persistent launch's last block resets its queue), so it may be
 * captured in a HIP graph and replayed.  Executions of one plan must not
 * overlap in time (they share the queue counters). */
int fdl_batch_plan_execute(const fdl_batch_plan* plan, void* stream);
/* Totals of the current setting: bins over all light fields, blocks over all
 * launches, launches per execution. */
int fdl_batch_plan_info(const fdl_batch_plan* plan, int64_t* total_bins, int32_t* grid, int32_t* launches);
int fdl_batch_plan_launches(const fdl_batch_plan* plan);
/* Autotuner: times the candidates {flat}, {flat single}, {persistent, chunk 1 or 4 tiles
 * per queue access, 1/2/4 blocks per CU} and {persistent single, chunk 1 or 4, 1/2
 * blocks per CU} on the plan's own data (`reps` timed
 * executions each after a warm-up, synchronising `stream`), keeps the fastest
 * and returns its time in best_ms.  Overwrites the plan's outputs; not
 * capturable. */
int fdl_batch_plan_autotune(fdl_batch_plan* plan, int reps, void* stream, float* best_ms);
int fdl_batch_plan_get_tuning(const fdl_batch_plan* plan, int32_t* mode, int32_t* chunk, int32_t* grid_per_cu);
int fdl_batch_plan_set_tuning(fdl_batch_plan* plan, int32_t mode, int32_t chunk, int32_t grid_per_cu);
int fdl_batch_plan_destroy(fdl_batch_plan* plan);

/* ---------------------------------------------------------------------------
 * Layer construction with the second-order view regulariser restricted to a
 * finite square [-r/2, r/2]^2 of the camera plane (Eq. GTG, divided by the
 * area r^2, in 2D): as fdl_construct, with R(w) the dense real matrix
 *   R_k1k2 = |w|^4 d_k1^2 d_k2^2 sinc(r (d_k1 - d_k2) w_x) sinc(r (d_k1 - d_k2) w_y),
 * sinc(t) = sin(pi t)/(pi t); r -> infinity gives FDL_REG_VIEW2.  region = r
 * (finite, > 0; FDL_EINVAL otherwise).  The off-diagonal entries use the FP32
 * sine (about 1e-7 relative); all other arguments, layouts, status and
 * errors as fdl_construct.
 * ------------------------------------------------------------------------- */
int fdl_construct_region(const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_host, int m, int n, int C,
                         int H, int W, float lambda, float eps, float region, fdl_c64* layer_spec_dev,
                         int32_t* status_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Drawn apertures (Sec. VI: the aperture is drawn as an image, its spectrum
 * taken from the DFT of the zero-padded image and read between the samples
 * by linear interpolation; the view's radius plays the paper's scale f).
 *
 * fdl_aperture_table: img_dev [S][S] float32 on the device, S odd, 1 <= S <=
 *   255; the image tiles the box [-1, 1]^2 of the aperture's own coordinates,
 *   pixel (x, y) centred at ((x - (S-1)/2) 2/S, (y - (S-1)/2) 2/S); values are
 *   weights (a 0/1 mask or grey levels, sum > 0; a zero sum gives non-finite
 *   entries).  Writes table_dev [N][N] complex64, N = pad S <= 2048:
 *     table[ky][kx] = psi_hat(kx S / (2N), ky S / (2N))
 *                   = sum_{x,y} a[y][x] exp(-2 pi i <p_xy, xi>) / sum a,
 *   samples that are N-periodic in kx and ky (FP64 sums, rounded to complex64).
 * fdl_render_tabulated: fdl_render in which views of shape FDL_AP_IMAGE take
 *   psi_hat_rho(xi) = psi_hat(rho xi) from the table (bilinear interpolation in
 *   the sample index rho xi 2N/S, periodic wrap; complex in general), so a
 *   full image renders as the square of half-side rho and an inscribed disk
 *   as the disk of radius rho, up to the drawing and interpolation errors;
 *   the other shapes are rendered as by fdl_render.  table_dev and (N, S) as
 *   produced by fdl_aperture_table (N a multiple of S); other arguments and
 *   errors as fdl_render.
 * ------------------------------------------------------------------------- */
int fdl_aperture_table(const float* img_dev, int S, int pad, fdl_c64* table_dev, void* stream);
int fdl_render_tabulated(const fdl_c64* layer_spec_dev, const float* d_dev, int n, int C, int H, int W,
                         const fdl_view* views_dev, int V, const fdl_c64* table_dev, int N, int S,
                         fdl_c64* out_spec_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Relaxed FDL model (Sec. VIII-B, denoising).  The shift of layer k in input
 * view j is a free pair P_jk = (P^x_jk, P^y_jk) instead of the rank-1 product
 * d_k u_j, so that occlusions and non-Lambertian effects can be absorbed:
 *   A_jk(w) = exp(+2 pi i <P_jk, w>).
 * shifts_dev: [m][n] fdl_f2 on the device (row j: the n shifts of view j);
 * the rank-1 model is P_jk = d_k u_j.  There are no layer disparities, so the
 * regulariser must be FDL_REG_LAYER2 or FDL_REG_L2 (FDL_EINVAL otherwise).
 *
 * fdl_construct_relaxed: layers x = (A^H A + lambda R + eps I)^-1 A^H b per
 *   bin, as fdl_construct (same layouts, status and limits) with A from P;
 *   the Gram matrix is always formed from all n(n+1)/2 products.
 * fdl_render_relaxed: the input views as the model predicts them (the
 *   denoised result): out_j(w) = sum_k exp(2 pi i <P_jk, w>) L_k(w) for the V
 *   rows of shifts_dev ([V][n]); out_spec_dev [V][C][H][W/2+1], FP32 phases.
 * fdl_calib_grad_relaxed: the calibration loss of fdl_calib_grad (FIT or
 *   LOO, same bins, index clamping and status count, scaling and limits) as a
 *   function of P, and its gradient
 *   (Eq. gradP with both components): grad P^x_jk = sum_q T_jk(q) w_x(q),
 *   grad P^y_jk = sum_q T_jk(q) w_y(q), T_jk = dE_q / d<P_jk, w_q>.
 *   grad_shifts_dev [m][n][2] double; loss_dev [1] double; workspace of at
 *   least fdl_calib_relaxed_workspace(m, n, Q) bytes; the per-bin LDS of
 *   fdl_calib_grad (without the max) plus 16 m n + 2048 bytes must fit one
 *   block (FDL_ESHAPE).
 * fdl_gd_step_relaxed: P <- P - alpha grad_P / (eps_g + ||grad_P||^2), the
 *   update of Sec. V-B with the norm over all 2 m n entries, in FP64, stored
 *   back to the float shifts (m n <= 2^24).
 * ------------------------------------------------------------------------- */
int fdl_construct_relaxed(const fdl_c64* view_spec_dev, const fdl_f2* shifts_dev, int m, int n, int C, int H, int W,
                          float lambda, float eps, int reg, fdl_c64* layer_spec_dev, int32_t* status_dev,
                          void* stream);
int fdl_render_relaxed(const fdl_c64* layer_spec_dev, const fdl_f2* shifts_dev, int n, int C, int H, int W, int V,
                       fdl_c64* out_spec_dev, void* stream);
size_t fdl_calib_relaxed_workspace(int m, int n, int Q);
int fdl_calib_grad_relaxed(const fdl_c64* view_spec_dev, const fdl_f2* shifts_dev, int m, int n, int C, int H, int W,
                           float lambda, float eps, int reg, int mode, const int32_t* freq_idx_dev, int Q,
                           double* loss_dev, double* grad_shifts_dev, int32_t* status_dev, void* ws_dev,
                           size_t ws_bytes, void* stream);
int fdl_gd_step_relaxed(fdl_f2* shifts_dev, const double* grad_shifts_dev, int m, int n, double alpha, double eps_g,
                        void* stream);

/* ---------------------------------------------------------------------------
 * Request server (systems pattern over the calls above; no single passage of
 * the paper): construct and render requests against light fields kept
 * resident on the device, served with continuous batching.
 *
 * Everything the server keeps on the device -- the resident layer spectra of
 * every light field and the buffers of the work in flight -- lives in ONE
 * device allocation of hbm_budget bytes made by fdl_server_create, so
 * admission by HBM footprint is exact: a unit of work starts only when its
 * buffer can be placed in it.  A construct re-solves the layers of its light
 * field (fdl_construct) into a new buffer, which replaces the resident layers
 * when it completes (renders already running keep reading the previous
 * layers, which return to the pool when the last of them ends).  A render
 * computes the view's spectrum (fdl_render) and image (fdl_irfft2); renders
 * of one light field that have arrived are launched together (up to
 * max_render_batch views).  A worker thread of the server retires finished
 * work (event polling; the thread spins while work is in flight, so
 * completion is observed within microseconds) and admits arrived requests in
 * arrival order; a request that cannot start yet is skipped by later ones,
 * except that after it has waited 50 ms nothing that arrived later starts
 * before it.  Latency = completion seen by the worker - scheduled arrival.
 * Streams run at the default priority (two for renders, one for constructs).
 * serial = 1 gives the plain baseline: strict arrival order, one unit of
 * work at a time on one stream, one view per render.
 *
 * Footprints: a construct needs n C H (W/2+1) 8 bytes; a rendered view needs
 * its spectrum, image and record (C H (W/2+1) 8 + C H W 4 + 256 bytes,
 * rounded to 256).  A request whose footprint exceeds the budget left beside
 * the resident layers can never start: fdl_server_submit rejects it
 * (FDL_ENOMEM, state FDL_REQ_REJECTED).  A request that cannot be placed
 * while nothing is in flight (fragmented free space) is rejected too, so the
 * server never waits forever.
 * ------------------------------------------------------------------------- */
typedef struct fdl_server fdl_server;

enum fdl_req_kind { FDL_REQ_CONSTRUCT = 0, FDL_REQ_RENDER = 1 };
enum fdl_req_state { FDL_REQ_QUEUED = 0, FDL_REQ_RUNNING = 1, FDL_REQ_DONE = 2, FDL_REQ_REJECTED = 3 };

typedef struct {
  int32_t kind;          /* FDL_REQ_CONSTRUCT or FDL_REQ_RENDER */
  int32_t lf;            /* light field id from fdl_server_add_lightfield */
  fdl_view view;         /* render: position, focus, aperture (as fdl_render) */
  float* image_dev;      /* render: [C][H][W] float32 device buffer of the caller that receives
                          * the image, or NULL (rendered, not copied out) */
  double t_arrival;      /* scheduled arrival on the server clock (seconds since
                          * fdl_server_create; fdl_server_now), < 0: now.  Requests may be
                          * submitted ahead of their arrival; they start no earlier. */
} fdl_request;

typedef struct {
  int64_t submitted, completed, rejected;
  int64_t count[3];               /* completed: all, construct, render */
  double p50_ms[3], p99_ms[3], mean_ms[3];   /* latency percentiles (linear interpolation), same order */
  int64_t render_batches;         /* render launches */
  double mean_render_batch;       /* views per render launch */
  double pool_high_water_bytes;   /* most of the budget ever in use (resident + in flight) */
  double resident_bytes;          /* resident layers of all light fields */
  double first_arrival_s;         /* server clock at the earliest arrival of a completed request */
  double last_completion_s;       /* server clock at the last completion */
} fdl_server_summary;

/* Creates a server on the current device: allocates the hbm_budget pool,
 * pinned staging and streams, and starts its worker thread.  1 <=
 * max_render_batch <= 256, 1 <= max_inflight <= 64 (units of work in flight). */
int fdl_server_create(size_t hbm_budget, int max_render_batch, int max_inflight, int serial, fdl_server** out);
/* Registers a light field: its view spectra, positions and d (HOST array,
 * copied) as fdl_construct takes them; the buffers of view_spec_dev and u_dev
 * must stay valid while the server lives.  Places its layers in the pool and
 * constructs them (blocking).  FDL_ENOMEM if they do not fit. */
int fdl_server_add_lightfield(fdl_server* s, const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_host,
                              int m, int n, int C, int H, int W, float lambda, float eps, int reg, int32_t* lf_out);
/* Queues a request; *id_out identifies it (also when rejected: FDL_ENOMEM).
 * FDL_EINVAL for an unknown kind or light field. */
int fdl_server_submit(fdl_server* s, const fdl_request* req, int64_t* id_out);
/* State of a request (fdl_req_state) and, once done, its latency in ms
 * (else -1).  Returns the first device error the server met, if any. */
int fdl_server_poll(fdl_server* s, int64_t id, int32_t* state, double* latency_ms);
/* Blocks until every accepted request has completed (FDL_ETIMEOUT after
 * timeout_s seconds). */
int fdl_server_drain(fdl_server* s, double timeout_s);
/* The server clock (seconds since creation). */
int fdl_server_now(fdl_server* s, double* t_now);
/* Device address of the current resident layers of a light field
 * ([n][C][H][W/2+1] complex64, valid until the next construct of it ends). */
int fdl_server_layers(fdl_server* s, int32_t lf, const fdl_c64** layer_spec_dev);
int fdl_server_stats(fdl_server* s, fdl_server_summary* out);
/* Serves every accepted request to completion, then frees the server. */
int fdl_server_destroy(fdl_server* s);

/* The server's scheduling policy on a simulated device, without the GPU (for
 * host-side tests and capacity planning): n_lf light fields with the given
 * layer and per-view footprints, fixed service times (a construct takes
 * construct_s, a render of V views V render_s_per_view; streams as the
 * server's, each running its work in order), requests submitted with their
 * arrival times.  out[i]: final state, render launch index (or -1), admission
 * and completion times (simulated seconds). */
typedef struct { double t_arrival; int32_t kind; int32_t lf; } fdl_sim_request;
typedef struct { int32_t state; int32_t batch; double t_admit; double t_done; } fdl_sim_result;
int fdl_server_simulate(size_t hbm_budget, int max_render_batch, int max_inflight, int serial, int n_lf,
                        const size_t* layer_bytes, const size_t* view_bytes, double construct_s,
                        double render_s_per_view, const fdl_sim_request* reqs, int nreq, fdl_sim_result* out,
                        fdl_server_summary* stats);

/* ---------------------------------------------------------------------------
 * Measurement utility (not part of the method): enqueues `blocks` blocks of
 * 256 threads, each thread running 8 independent FP64 multiply-add chains of
 * `iters` steps (16 * iters flops per thread) and writing one double to
 * out_dev[blocks * 256].  Timed by the caller, it gives the achievable FP64
 * VALU throughput against which the kernels above are compared.
 * FDL_EINVAL for a null pointer or non-positive sizes. */
int fdl_fma64_probe(double* out_dev, int blocks, int iters, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FDL_H */
