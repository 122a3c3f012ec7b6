// Real 2D DFT and its inverse for image sizes 2^a 3^b (Sec. V-A: the layer
// model works on the DFT of each input image; Sec. VII: only the Hermitian
// half spectrum [H][W/2+1] is computed and stored).
//
// Forward: (1) rows: each real row of length W is packed as W/2 complex
//   values z[n] = x[2n] + i x[2n+1], transformed by an LDS Stockham FFT and
//   split into the half spectrum X[k] = E[k] + e^{-2 pi i k/W} O[k],
//   E = (Z[k] + conj Z[N-k])/2, O = -i (Z[k] - conj Z[N-k])/2, k = 0..W/2;
//   (2) columns: complex FFT of length H of every column kx, in place.
// Inverse: (1) columns: inverse complex FFT in place (the input buffer is
//   scratch); (2) rows: Z[k] = E[k] + i O[k] with E = (X[k] + conj X[N-k])/2,
//   O = e^{+2 pi i k/W} (X[k] - conj X[N-k])/2 (imaginary parts of X[0], X[N]
//   dropped, numpy semantics), inverse FFT of length W/2, unpacked to 2 reals.
//   Normalisation 1/(H W).
//
// The in-LDS transform is the Stockham autosort formulation (Govindaraju et
// al., "High performance discrete Fourier transforms on graphics processors",
// SC 2008) with radix-4, radix-2 and radix-3 butterflies; twiddles are
// evaluated by the transcendental unit in revolutions after exact range
// reduction.  FP32 throughout.
#include "fdl_device.h"
#include "fdl_internal.h"

namespace fdl {

__device__ __forceinline__ float2 f2add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 f2sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 f2mul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 f2conj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 f2scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// exp(2 pi i r), r in revolutions
__device__ __forceinline__ float2 twiddle(float r) {
  r = r - rintf(r);
  return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
}

// In-place DFT of R = 2, 3 or 4 values (forward sign -, inverse +).
template <int R, bool INV>
__device__ __forceinline__ void butterfly(float2 (&v)[R]) {
  if constexpr (R == 4) {
    const float2 a0 = f2add(v[0], v[2]), a1 = f2sub(v[0], v[2]);
    const float2 a2 = f2add(v[1], v[3]), a3 = rot90<INV>(f2sub(v[1], v[3]));
    v[0] = f2add(a0, a2);
    v[2] = f2sub(a0, a2);
    v[1] = f2add(a1, a3);
    v[3] = f2sub(a1, a3);
  } else if constexpr (R == 2) {
    const float2 a0 = v[0];
    v[0] = f2add(a0, v[1]);
    v[1] = f2sub(a0, v[1]);
  } else {   // R == 3
    const float2 t1 = f2add(v[1], v[2]);
    const float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    const float2 s = f2scale(rot90<INV>(f2sub(v[1], v[2])), 0.86602540378443864676f);
    v[0] = f2add(v[0], t1);
    v[1] = f2add(t2, s);
    v[2] = f2sub(t2, s);
  }
}

// One Stockham stage of radix R over a length-N sequence held in LDS.
template <int R, bool INV>
__device__ __forceinline__ void stockham_stage(const float2* __restrict__ in, float2* __restrict__ out, int N, int Ns,
                                               int t, int G) {
  const int nb = N / R;
  const float sgn = INV ? 1.0f : -1.0f;
  const float inv_span = 1.0f / (float)(Ns * R);
  for (int j = t; j < nb; j += G) {
    const int k = j % Ns;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[j + r * nb];
    if (Ns > 1) {
      const float a = sgn * (float)k * inv_span;
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = f2mul(v[r], twiddle(a * (float)r));
    }
    butterfly<R, INV>(v);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[base + r * Ns] = v[r];
  }
}

// Runs every stage; returns the buffer that holds the result.  All G*groups
// threads of the block call it together (block barriers inside).
template <bool INV>
__device__ __forceinline__ float2* lds_fft(float2* b0, float2* b1, const FftPlan& plan, int t, int G) {
  int Ns = 1;
  float2* in = b0;
  float2* out = b1;
  for (int s = 0; s < plan.nst; ++s) {
    const int R = plan.radix[s];
    if (R == 4) stockham_stage<4, INV>(in, out, plan.N, Ns, t, G);
    else if (R == 2) stockham_stage<2, INV>(in, out, plan.N, Ns, t, G);
    else stockham_stage<3, INV>(in, out, plan.N, Ns, t, G);
    __syncthreads();
    Ns *= R;
    float2* tmp = in;
    in = out;
    out = tmp;
  }
  return in;
}

// ---- register-resident transforms (compile-time length) ---------------------

// cos and sin of 2 pi a / b at compile time (series after reduction to
// [-pi, pi]; converged to double precision).
constexpr double ct_rev_series(long a, long b, bool want_sin) {
  a %= b;
  if (a < 0) a += b;
  if (2 * a > b) a -= b;
  const double x = 6.28318530717958647692 * (double)a / (double)b;
  double term = want_sin ? x : 1.0, sum = term;
  for (int i = 1; i < 40; ++i) {
    const double d = want_sin ? (double)(2 * i) * (2 * i + 1) : (double)(2 * i - 1) * (2 * i);
    term *= -x * x / d;
    sum += term;
  }
  return sum;
}

// Stockham stages over a register array (every index is a compile-time
// constant, so the stages compile to straight-line code).  Radix 4 while it
// divides the remaining length, then 2, then 3; the same stage formula as
// the LDS version above.
template <int N, int Ns, bool INV>
__device__ __forceinline__ void reg_fft_from(float2 (&a)[N]) {
  if constexpr (Ns < N) {
    constexpr int rem = N / Ns;
    constexpr int R = rem % 4 == 0 ? 4 : (rem % 2 == 0 ? 2 : 3);
    static_assert(rem % R == 0, "length must be 2^a 3^b");
    float2 b[N];
    static_for<0, N / R>([&](auto JJ) {
      constexpr int j = decltype(JJ)::value;
      constexpr int k = j % Ns;
      float2 v[R];
      static_for<0, R>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        v[r] = a[j + r * (N / R)];
        if constexpr (k * r != 0) {
          constexpr long num = INV ? (long)k * r : -(long)k * r;
          constexpr float wr = (float)ct_rev_series(num, (long)Ns * R, false);
          constexpr float wi = (float)ct_rev_series(num, (long)Ns * R, true);
          v[r] = f2mul(v[r], make_float2(wr, wi));
        }
      });
      butterfly<R, INV>(v);
      constexpr int base = (j / Ns) * Ns * R + k;
      static_for<0, R>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        b[base + r * Ns] = v[r];
      });
    });
    reg_fft_from<N, Ns * R, INV>(b);
    static_for<0, N>([&](auto II) {
      constexpr int i = decltype(II)::value;
      a[i] = b[i];
    });
  }
}

template <int N, bool INV>
__device__ __forceinline__ void reg_fft(float2 (&a)[N]) {
  reg_fft_from<N, 1, INV>(a);
}

// ---- columns, register four-step version ---------------------------------------
// Length H = P Q with Q a multiple of P; a block transforms TC adjacent
// columns with P threads per column.  With y = t + P q and k = k1 + Q k2,
//   X[k1 + Q k2] = sum_t W_P^{t k2} W_H^{t k1} sum_q x[t + P q] W_Q^{q k1},
// so thread t (1) loads x[t + P q], q < Q, (2) transforms them in registers
// (length Q), (3) multiplies by W_H^{t k1}, (4) passes the Q values through
// LDS, (5) takes Q/P of the k1 rows and transforms each over t in registers
// (length P), (6) stores X[k1 + Q k2].  Loads and stores of a wave cover
// 128-byte row segments (16 columns x 8 bytes); the LDS tile uses padded
// strides (k1 stride P + 1, column stride = 4 mod 32 entries) so that both
// access patterns spread over the banks.
template <int P, int Q, int TC, bool INV>
__global__ __launch_bounds__(TC * P) void k_fft_cols_reg(float2* __restrict__ data, int Wh, int tiles) {
  static_assert(Q % P == 0, "Q must be a multiple of P");
  constexpr int H = P * Q;
  constexpr int KS = P + 1;
  constexpr int CS0 = Q * KS;
  constexpr int CS = CS0 + ((36 - CS0 % 32) % 32);
  __shared__ float2 lds[TC * CS];
  // rows of W/2 + 1 complex values are not 128-byte aligned, so neighbouring
  // tiles share cache lines: keep them on one XCD (one L2)
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int img = b / tiles;
  const int c0 = (b - img * tiles) * TC;
  const int col = threadIdx.x % TC;
  const int t = threadIdx.x / TC;
  const bool live = c0 + col < Wh;
  float2* base = data + (size_t)img * H * Wh + c0 + col;
  float2 v[Q];
  static_for<0, Q>([&](auto QQ) {
    constexpr int q = decltype(QQ)::value;
    v[q] = live ? base[(size_t)(t + P * q) * Wh] : make_float2(0.0f, 0.0f);
  });
  reg_fft<Q, INV>(v);
  const float step = (INV ? 1.0f : -1.0f) * (float)t * (1.0f / (float)H);
  static_for<1, Q>([&](auto KK) {
    constexpr int k1 = decltype(KK)::value;
    v[k1] = f2mul(v[k1], twiddle(step * (float)k1));
  });
  float2* mine = lds + col * CS;
  static_for<0, Q>([&](auto KK) {
    constexpr int k1 = decltype(KK)::value;
    mine[k1 * KS + t] = v[k1];
  });
  __syncthreads();
  static_for<0, Q / P>([&](auto SS) {
    constexpr int s = decltype(SS)::value;
    const int k1 = t + P * s;
    float2 w[P];
    static_for<0, P>([&](auto PP) {
      constexpr int p = decltype(PP)::value;
      w[p] = mine[k1 * KS + p];
    });
    reg_fft<P, INV>(w);
    if (live) {
      static_for<0, P>([&](auto KK) {
        constexpr int k2 = decltype(KK)::value;
        base[(size_t)(k1 + Q * k2) * Wh] = w[k2];
      });
    }
  });
}

template <int P, int Q, int TC, bool INV>
static hipError_t go_cols_reg(float2* data, int batch, int Wh, hipStream_t s) {
  const int tiles = (Wh + TC - 1) / TC;
  hipLaunchKernelGGL((k_fft_cols_reg<P, Q, TC, INV>), dim3(batch * tiles), dim3(TC * P), 0, s, data, Wh, tiles);
  return hipGetLastError();
}

// Register kernel for the column lengths it is instantiated for; false for
// the others (the LDS Stockham kernel below takes them).
template <bool INV>
static bool cols_reg(float2* data, int batch, int H, int Wh, hipStream_t s, hipError_t& err) {
  switch (H) {
    case 64: err = go_cols_reg<8, 8, 16, INV>(data, batch, Wh, s); return true;
    case 128: err = go_cols_reg<8, 16, 16, INV>(data, batch, Wh, s); return true;
    case 256: err = go_cols_reg<16, 16, 16, INV>(data, batch, Wh, s); return true;
    case 384: err = go_cols_reg<8, 48, 16, INV>(data, batch, Wh, s); return true;
    case 512: err = go_cols_reg<16, 32, 16, INV>(data, batch, Wh, s); return true;
    case 768: err = go_cols_reg<16, 48, 8, INV>(data, batch, Wh, s); return true;
    case 1024: err = go_cols_reg<32, 32, 8, INV>(data, batch, Wh, s); return true;
    default: return false;
  }
}

// ---- rows, register four-step versions ---------------------------------------
// Complex length N = W/2 = P Q (Q a multiple of P), P threads per row, 256/P
// rows per block; same decomposition as the column kernel above.  Thread t
// of a row reads z[t + P q] (P threads cover a contiguous P x 8-byte
// segment).  The per-row LDS region holds Y[k1][t] (k1 stride P + 1) and
// then, in the forward kernel, Z in natural order for the real split.
template <int P, int Q>
__global__ __launch_bounds__(256) void k_rfft_rows_reg(const float* __restrict__ img, float2* __restrict__ out,
                                                       int nrows) {
  constexpr int N = P * Q;
  constexpr int RPB = 256 / P;
  constexpr int KS = P + 1;
  constexpr int RS = Q * KS;
  __shared__ float2 lds[RPB * RS];
  const int lr = threadIdx.x / P;
  const int t = threadIdx.x - lr * P;
  const int row = blockIdx.x * RPB + lr;
  const bool live = row < nrows;
  const float2* src = reinterpret_cast<const float2*>(img) + (size_t)row * N + t;
  float2 v[Q];
  static_for<0, Q>([&](auto QQ) {
    constexpr int q = decltype(QQ)::value;
    v[q] = live ? src[P * q] : make_float2(0.0f, 0.0f);
  });
  reg_fft<Q, false>(v);
  const float step = -(float)t * (1.0f / (float)N);
  static_for<1, Q>([&](auto KK) {
    constexpr int k1 = decltype(KK)::value;
    v[k1] = f2mul(v[k1], twiddle(step * (float)k1));
  });
  float2* mine = lds + lr * RS;
  static_for<0, Q>([&](auto KK) {
    constexpr int k1 = decltype(KK)::value;
    mine[k1 * KS + t] = v[k1];
  });
  __syncthreads();
  float2 w[Q / P][P];
  static_for<0, Q / P>([&](auto SS) {
    constexpr int s = decltype(SS)::value;
    const int k1 = t + P * s;
    static_for<0, P>([&](auto PP) {
      constexpr int p = decltype(PP)::value;
      w[s][p] = mine[k1 * KS + p];
    });
    reg_fft<P, false>(w[s]);
  });
  __syncthreads();
  static_for<0, Q / P>([&](auto SS) {
    constexpr int s = decltype(SS)::value;
    static_for<0, P>([&](auto KK) {
      constexpr int k2 = decltype(KK)::value;
      mine[t + P * s + Q * k2] = w[s][k2];
    });
  });
  __syncthreads();
  if (!live) return;
  // X[k] = E[k] + e^{-2 pi i k / W} O[k], k = 0..N
  float2* dst = out + (size_t)row * (N + 1);
  const float invW = 0.5f / (float)N;
  for (int k = t; k <= N; k += P) {
    const float2 zk = mine[k == N ? 0 : k];
    const float2 zn = f2conj(mine[k == 0 ? 0 : N - k]);
    const float2 E = f2scale(f2add(zk, zn), 0.5f);
    const float2 O = f2scale(rot90<false>(f2sub(zk, zn)), 0.5f);
    dst[k] = f2add(E, f2mul(twiddle(-(float)k * invW), O));
  }
}

template <int P, int Q>
__global__ __launch_bounds__(256) void k_irfft_rows_reg(const float2* __restrict__ spec, float* __restrict__ img,
                                                        int nrows, float scale) {
  constexpr int N = P * Q;
  constexpr int RPB = 256 / P;
  constexpr int KS = P + 1;
  constexpr int RS = Q * KS;
  __shared__ float2 lds[RPB * RS];
  const int lr = threadIdx.x / P;
  const int t = threadIdx.x - lr * P;
  const int row = blockIdx.x * RPB + lr;
  const bool live = row < nrows;
  const float2* src = spec + (size_t)row * (N + 1);
  // Z[k] = E[k] + i O[k], E = (X[k] + conj X[N-k]) / 2,
  // O = e^{+2 pi i k / W} (X[k] - conj X[N-k]) / 2 (imaginary parts of X[0], X[N] dropped)
  const float invW = 0.5f / (float)N;
  float2 v[Q];
  static_for<0, Q>([&](auto QQ) {
    constexpr int q = decltype(QQ)::value;
    const int k = t + P * q;
    float2 xk = make_float2(0.0f, 0.0f), xn = make_float2(0.0f, 0.0f);
    if (live) {
      xk = src[k];
      xn = src[N - k];
    }
    if (k == 0) { xk.y = 0.0f; xn.y = 0.0f; }
    xn = f2conj(xn);
    const float2 E = f2scale(f2add(xk, xn), 0.5f);
    const float2 O = f2scale(f2mul(twiddle((float)k * invW), f2sub(xk, xn)), 0.5f);
    v[q] = f2add(E, rot90<true>(O));
  });
  reg_fft<Q, true>(v);
  const float step = (float)t * (1.0f / (float)N);
  static_for<1, Q>([&](auto KK) {
    constexpr int k1 = decltype(KK)::value;
    v[k1] = f2mul(v[k1], twiddle(step * (float)k1));
  });
  float2* mine = lds + lr * RS;
  static_for<0, Q>([&](auto KK) {
    constexpr int k1 = decltype(KK)::value;
    mine[k1 * KS + t] = v[k1];
  });
  __syncthreads();
  if (!live) return;
  float2* dst = reinterpret_cast<float2*>(img + (size_t)row * 2 * N);
  static_for<0, Q / P>([&](auto SS) {
    constexpr int s = decltype(SS)::value;
    const int k1 = t + P * s;
    float2 w[P];
    static_for<0, P>([&](auto PP) {
      constexpr int p = decltype(PP)::value;
      w[p] = mine[k1 * KS + p];
    });
    reg_fft<P, true>(w);
    static_for<0, P>([&](auto KK) {
      constexpr int k2 = decltype(KK)::value;
      dst[k1 + Q * k2] = f2scale(w[k2], scale);
    });
  });
}

template <int P, int Q>
static hipError_t go_rows_reg(const FftParams& F, bool inverse, float scale, hipStream_t s) {
  constexpr int RPB = 256 / P;
  const int nrows = F.batch * F.H;
  const dim3 grid((nrows + RPB - 1) / RPB);
  if (inverse) hipLaunchKernelGGL((k_irfft_rows_reg<P, Q>), grid, dim3(256), 0, s, F.cplx, F.real, nrows, scale);
  else hipLaunchKernelGGL((k_rfft_rows_reg<P, Q>), grid, dim3(256), 0, s, F.real, F.cplx, nrows);
  return hipGetLastError();
}

// Register row kernels for the row lengths they are instantiated for; false
// for the others (the LDS Stockham kernels below take them).
static bool rows_reg(const FftParams& F, bool inverse, float scale, hipStream_t s, hipError_t& err) {
  switch (F.W / 2) {
    case 64: err = go_rows_reg<8, 8>(F, inverse, scale, s); return true;
    case 128: err = go_rows_reg<8, 16>(F, inverse, scale, s); return true;
    case 192: err = go_rows_reg<8, 24>(F, inverse, scale, s); return true;
    case 256: err = go_rows_reg<16, 16>(F, inverse, scale, s); return true;
    case 384: err = go_rows_reg<8, 48>(F, inverse, scale, s); return true;
    case 512: err = go_rows_reg<16, 32>(F, inverse, scale, s); return true;
    case 1024: err = go_rows_reg<32, 32>(F, inverse, scale, s); return true;
    default: return false;
  }
}

// ---- forward rows: real rows -> half spectra --------------------------------
__global__ __launch_bounds__(256) void k_rfft_rows(const float* __restrict__ img, float2* __restrict__ out,
                                                   int nrows, int W, FftPlan plan, int G) {
  extern __shared__ float2 lds[];
  const int N = plan.N;              // W / 2
  const int rpb = blockDim.x / G;
  const int lr = threadIdx.x / G;
  const int t = threadIdx.x - lr * G;
  const int row = blockIdx.x * rpb + lr;
  float2* b0 = lds + (size_t)lr * 2 * N;
  float2* b1 = b0 + N;
  const bool live = row < nrows;
  if (live) {
    const float2* src = reinterpret_cast<const float2*>(img + (size_t)row * W);
    for (int i = t; i < N; i += G) b0[i] = src[i];
  }
  __syncthreads();
  const float2* Z = lds_fft<false>(b0, b1, plan, t, G);
  if (live) {
    float2* dst = out + (size_t)row * (N + 1);
    const float invW = 1.0f / (float)W;
    for (int k = t; k <= N; k += G) {
      const float2 zk = Z[k == N ? 0 : k];
      const float2 zn = f2conj(Z[k == 0 ? 0 : N - k]);
      const float2 E = f2scale(f2add(zk, zn), 0.5f);
      const float2 O = f2scale(rot90<false>(f2sub(zk, zn)), 0.5f);
      dst[k] = f2add(E, f2mul(twiddle(-(float)k * invW), O));
    }
  }
}

// ---- inverse rows: half spectra -> real rows ---------------------------------
__global__ __launch_bounds__(256) void k_irfft_rows(const float2* __restrict__ spec, float* __restrict__ img,
                                                    int nrows, int W, FftPlan plan, int G, float scale) {
  extern __shared__ float2 lds[];
  const int N = plan.N;
  const int rpb = blockDim.x / G;
  const int lr = threadIdx.x / G;
  const int t = threadIdx.x - lr * G;
  const int row = blockIdx.x * rpb + lr;
  float2* b0 = lds + (size_t)lr * 2 * N;
  float2* b1 = b0 + N;
  const bool live = row < nrows;
  if (live) {
    const float2* src = spec + (size_t)row * (N + 1);
    const float invW = 1.0f / (float)W;
    for (int k = t; k < N; k += G) {
      float2 xk = src[k];
      float2 xn = src[N - k];
      if (k == 0) { xk.y = 0.0f; xn.y = 0.0f; }   // self-conjugate bins are real
      xn = f2conj(xn);
      const float2 E = f2scale(f2add(xk, xn), 0.5f);
      const float2 O = f2scale(f2mul(twiddle((float)k * invW), f2sub(xk, xn)), 0.5f);
      b0[k] = f2add(E, rot90<true>(O));
    }
  }
  __syncthreads();
  const float2* z = lds_fft<true>(b0, b1, plan, t, G);
  if (live) {
    float2* dst = reinterpret_cast<float2*>(img + (size_t)row * W);
    for (int i = t; i < N; i += G) dst[i] = f2scale(z[i], scale);
  }
}

// ---- columns: complex FFT of length H over a tile of TC columns, in place ----
template <bool INV>
__global__ __launch_bounds__(256) void k_fft_cols(float2* __restrict__ data, int batch, int H, int Wh, int tiles,
                                                  FftPlan plan, int G, int TC) {
  extern __shared__ float2 lds[];
  const int img = blockIdx.x / tiles;
  const int c0 = (blockIdx.x - img * tiles) * TC;
  const int lc = threadIdx.x / G;
  const int t = threadIdx.x - lc * G;
  float2* base = data + (size_t)img * H * Wh;
  const int CS = 2 * H + 1;   // odd column stride: the transposed accesses spread over the LDS banks
  // transpose-load: lds[c][y]
  for (int q = threadIdx.x; q < H * TC; q += blockDim.x) {
    const int y = q / TC, c = q - y * TC;
    if (c0 + c < Wh) lds[(size_t)c * CS + y] = base[(size_t)y * Wh + c0 + c];
  }
  __syncthreads();
  float2* b0 = lds + (size_t)lc * CS;
  const float2* r = lds_fft<INV>(b0, b0 + H, plan, t, G);
  const size_t roff = (size_t)(r - b0);   // 0 or H: same for every column
  for (int q = threadIdx.x; q < H * TC; q += blockDim.x) {
    const int y = q / TC, c = q - y * TC;
    if (c0 + c < Wh) base[(size_t)y * Wh + c0 + c] = lds[(size_t)c * CS + roff + y];
  }
}

// Largest dynamic LDS a block may request on the current device (queried on
// every call: no process-wide cache, so each device answers for itself).
static size_t max_block_lds() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
    return (size_t)v;
  return 65536;
}

size_t fft_lds_limit() { return max_block_lds(); }

// Dynamic LDS above the 64 KiB default is opted in on every such launch (the
// attribute is per device and the call is cheap; no process-wide state).
template <bool INV>
static void opt_in_lds(size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_cols<INV>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static int pick_threads(int N) {
  int g = 1;
  while (g * 2 <= 256 && g * 2 * 4 <= N) g *= 2;   // about N/4 butterflies per stage
  return g;
}

hipError_t launch_rfft2(const FftParams& P, hipStream_t s) {
  const int N = P.W / 2;
  // rows
  {
    hipError_t e = hipSuccess;
    if (!rows_reg(P, false, 1.0f, s, e)) {
      const int G = pick_threads(N);
      const int rpb = 256 / G;
      const int nrows = P.batch * P.H;
      const size_t lds = (size_t)rpb * 2 * N * sizeof(float2);
      hipLaunchKernelGGL(k_rfft_rows, dim3((nrows + rpb - 1) / rpb), dim3(rpb * G), lds, s, P.real, P.cplx, nrows,
                         P.W, P.row_plan, G);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
  }
  // columns
  {
    const int H = P.H, Wh = N + 1;
    hipError_t e = hipSuccess;
    if (cols_reg<false>(P.cplx, P.batch, H, Wh, s, e)) return e;
    const int TC = P.col_tc;
    const int G = 256 / TC;
    const int tiles = (Wh + TC - 1) / TC;
    const size_t lds = (size_t)TC * (2 * H + 1) * sizeof(float2);
    opt_in_lds<false>(lds);
    hipLaunchKernelGGL(k_fft_cols<false>, dim3(P.batch * tiles), dim3(TC * G), lds, s, P.cplx, P.batch, H, Wh,
                       tiles, P.col_plan, G, TC);
  }
  return hipGetLastError();
}

hipError_t launch_irfft2(const FftParams& P, hipStream_t s) {
  const int N = P.W / 2;
  {
    const int H = P.H, Wh = N + 1;
    hipError_t e = hipSuccess;
    if (!cols_reg<true>(P.cplx, P.batch, H, Wh, s, e)) {
      const int TC = P.col_tc;
      const int G = 256 / TC;
      const int tiles = (Wh + TC - 1) / TC;
      const size_t lds = (size_t)TC * (2 * H + 1) * sizeof(float2);
      opt_in_lds<true>(lds);
      hipLaunchKernelGGL(k_fft_cols<true>, dim3(P.batch * tiles), dim3(TC * G), lds, s, P.cplx, P.batch, H, Wh,
                         tiles, P.col_plan, G, TC);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
  }
  {
    const float scale = 1.0f / ((float)P.H * (float)N);   // E, O above already carry the 1/2
    hipError_t e = hipSuccess;
    if (rows_reg(P, true, scale, s, e)) return e;
    const int G = pick_threads(N);
    const int rpb = 256 / G;
    const int nrows = P.batch * P.H;
    const size_t lds = (size_t)rpb * 2 * N * sizeof(float2);
    hipLaunchKernelGGL(k_irfft_rows, dim3((nrows + rpb - 1) / rpb), dim3(rpb * G), lds, s, P.cplx, P.real, nrows,
                       P.W, P.row_plan, G, scale);
  }
  return hipGetLastError();
}

}  // namespace fdl
