// Calibration objective and gradient with respect to view positions u_j and
// disparities d_k (Sec. V-B, Eqs. CalibrationProb, gradD, gradP), plus the
// leave-one-out (LOO) view-prediction loss with its exact adjoint, and the
// normalised gradient step of Sec. V-B.
//
// One block of 256 threads handles one sampled bin at a time (grid-stride
// over the Q bins); the small dense algebra of the bin lives in LDS in FP64
// and the threads split its loops.  Per bin:
//   A_jk = exp(2 pi i d_k p_j), M = A^H A + lambda Gamma^H Gamma + eps I = L L^H,
//   x = M^-1 A^H b (b orthonormal: DFT / sqrt(HW)).
// FIT:  r = A x - b, E_q = ||r||^2 + x^H (lambda G + eps I) x,
//       T_jk = dE_q/dtheta_jk = 4 pi Im(conj(x_k) conj(A_jk) r_j) (Eq. gradP; the
//       regulariser is frozen at the minimiser, envelope theorem).
// LOO:  r = b - A x, h_j = a_j M^-1 a_j^H = ||L^-1 a_j^H||^2 (PRESS identity),
//       E_q = sum_j |r_j|^2 / (1 - h_j)^2.  With P = L^-1 A^H, G = L^-H P = M^-1 A^H,
//       H = A G, w = r/(1-h)^2, gam = 2|r|^2/(1-h)^3, y = G w, v = w - A y,
//       Wm = A^T diag(gam) G^T, the Wirtinger derivative dE/dA is
//       Psi_jk = sum_c[-conj(v_jc) x_kc - conj(r_jc) y_kc] + gam_j G_kj - (G^T Wm)_jk
//       and T_jk = -4 pi Im(Psi_jk A_jk).
// Both: grad u_j += sum_k d_k T_jk w_q,  grad d_k += sum_j T_jk p_j  (theta_jk =
//       d_k <u_j, w>), summed over the Q sampled bins (Eq. CalibrationProb sums
//       over the frequency components; the sampled subset replaces the full sum).
// Per-block partial sums are reduced in a fixed order by a second kernel, so
// the result is bitwise reproducible.
#include <mutex>

#include "fdl_device.h"
#include "fdl_internal.h"

namespace fdl {

struct CalibLayout {   // offsets (in doubles) into the dynamic LDS of one block
  int A, L, inv, b, x, r, p, T, P, w, y, v, gam, Wm, gP, red;
  int total;
};

__host__ __device__ inline CalibLayout calib_layout(int m, int n, int C, int mode, bool relaxed) {
  CalibLayout o;
  int at = 0;
  o.A = at; at += 2 * m * n;
  o.L = at; at += 2 * n * n;
  o.inv = at; at += n;
  o.b = at; at += 2 * m * C;
  o.x = at; at += 2 * n * C;
  o.r = at; at += 2 * m * C;
  o.p = at; at += m;
  o.T = at; at += m * n;
  if (mode == 1) {
    o.P = at; at += 2 * n * m;
    o.w = at; at += 2 * m * C;
    o.y = at; at += 2 * n * C;
    o.v = at; at += 2 * m * C;
    o.gam = at; at += m;
    o.Wm = o.L;   // L is dead once the sweeps are done, before Wm is formed
  } else {
    o.P = o.w = o.y = o.v = o.gam = o.Wm = 0;
  }
  if (relaxed) {
    o.gP = at;   // relaxed model: running gradient of the shifts, [m][n][2]
    at += 2 * m * n;
    o.red = at;
    at += 256;
  } else {
    // the final block reduction runs after the bin loop, when every other
    // region is dead
    o.gP = 0;
    o.red = 0;
    if (at < 256) at = 256;
  }
  o.total = at;
  return o;
}

size_t calib_lds_bytes(int m, int n, int C, int mode, bool relaxed) {
  return (size_t)calib_layout(m, n, C, mode, relaxed).total * 8;
}

__device__ __forceinline__ cd ldc(const double* s, int i) { return cd{s[2 * i], s[2 * i + 1]}; }
__device__ __forceinline__ void stc(double* s, int i, cd v) { s[2 * i] = v.re; s[2 * i + 1] = v.im; }

__device__ __forceinline__ double reg_entry(int reg, int i, int k, int n, double lambda, double w4, double di) {
  if (reg == 0) return (i == k) ? lambda * w4 * di * di * di * di : 0.0;
  if (reg == 1) {
    double s = 0.0;
    for (int p = i - 1; p <= i + 1; ++p) {
      if (p < 0 || p >= n) continue;
      const int a = p - i, b = p - k;
      if (b < -1 || b > 1) continue;
      s += (a == 0 ? -2.0 : 1.0) * (b == 0 ? -2.0 : 1.0);
    }
    return lambda * s;
  }
  return (i == k) ? lambda : 0.0;
}

// 4 blocks per CU (128 VGPRs): the leave-one-out layout of 49 views and 16
// layers takes 40 KB of LDS, so four bins are in flight per CU.  The grid is
// sized from the LDS, so the register budget must allow as many blocks; 2 and
// 3 blocks per CU measured slower.  Inner loops are unrolled by 4.
// RELAXED: the relaxed model of Sec. VIII-B, phases <P_jk, w> from a free
// shift matrix and the gradient with respect to every shift (Eq. gradP with
// both components) instead of the chain rule to u and d.
// NR > 0 (n <= NR <= 16, leave-one-out loss): the right-hand-side columns of
// the triangular sweeps are swept by the 16-lane teams of the block, one row
// per lane (below); NR = 0: the sweeps run in LDS, or for the paper loss with
// n <= 16 in the teams of wave 0.
// i / d for 0 <= i < 2^24 and d >= 1 without an integer division: the
// float quotient (relative error below 2^-23) is within one of the exact
// one, and one step on the integer remainder corrects it.
struct FastDiv {
  int d;
  float inv;
  __device__ explicit FastDiv(int d_) : d(d_), inv(1.0f / (float)d_) {}
  __device__ int operator()(int i) const {
    int q = (int)((float)i * inv);
    const int r = i - q * d;
    q += r >= d ? 1 : (r < 0 ? -1 : 0);
    return q;
  }
};

template <bool RELAXED, int NR>
__global__ __launch_bounds__(256, 4) void k_calib(CalibParams P) {
  constexpr int NT = 256;
  extern __shared__ double sm[];
  const int m = P.m, n = P.n, C = P.C;
  const CalibLayout o = calib_layout(m, n, C, P.mode, RELAXED);
  const FastDiv div_n(n), div_C(C), div_nn(n * n);
  double* A = sm + o.A;
  double* L = sm + o.L;
  double* b = sm + o.b;
  double* x = sm + o.x;
  double* r = sm + o.r;
  double* pj = sm + o.p;
  double* T = sm + o.T;
  const int t = threadIdx.x;
  const size_t F = (size_t)P.F;

  double gu[2] = {0.0, 0.0};   // view j = t (m <= 256)
  double gd = 0.0;              // layer k = t
  double loss = 0.0;

  // The positions are the same for every bin: thread j keeps u_j.  The
  // spectra of the next bin (m C <= 1024 values, at most 4 per thread) are
  // loaded while the current bin is processed.
  const float2 uj = !RELAXED && t < m ? P.u[t] : make_float2(0.0f, 0.0f);
  double* gP = sm + o.gP;
  if constexpr (RELAXED)
    for (int i = t; i < 2 * m * n; i += NT) gP[i] = 0.0;
  // Bin of sample q.  A caller's index outside [0, F) is clamped into it, so
  // that no access leaves the spectra, and counted in P.status by the block
  // that processes it.
  auto bin_of = [&](int q) -> int {
    const int raw = P.freq_idx ? P.freq_idx[q] : q;
    return min(max(raw, 0), P.F - 1);
  };
  float2 bnext[4];
  auto fetch = [&](int q) {
    if (q >= P.Q) return;
    const int fq = bin_of(q);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = t + s * NT;
      if (i < m * C) bnext[s] = P.view_spec[(size_t)i * F + fq];
    }
  };
  fetch(blockIdx.x);

  for (int q = blockIdx.x; q < P.Q; q += gridDim.x) {
    const int f = bin_of(q);
    if (t == 0 && P.status && P.freq_idx && (unsigned)P.freq_idx[q] >= (unsigned)P.F) atomicAdd(P.status, 1);
    double wx, wy;
    bin_freq(f, P.Wh, P.H, P.W, wx, wy);
    const double w2 = wx * wx + wy * wy, w4 = w2 * w2;

    if (t < m) pj[t] = (double)uj.x * wx + (double)uj.y * wy;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = t + s * NT;
      if (i < m * C) stc(b, i, cd{(double)bnext[s].x * P.bscale, (double)bnext[s].y * P.bscale});
    }
    fetch(q + gridDim.x);
    __syncthreads();
    for (int i = t; i < m * n; i += NT) {
      const int j = div_n(i), k = i - j * n;
      if constexpr (RELAXED) {
        const float2 sh = P.shifts[i];
        stc(A, i, expi2pi(fma((double)sh.x, wx, (double)sh.y * wy)));
      } else {
        stc(A, i, expi2pi((double)P.d[k] * pj[j]));
      }
    }
    __syncthreads();
    // normal matrix (lower triangle, full storage) and right-hand sides
    for (int i = t; i < n * n; i += NT) {
      const int k1 = div_n(i), k2 = i - k1 * n;
      if (k2 > k1) continue;
      cd s = cd{0.0, 0.0};
      #pragma unroll 4
      for (int j = 0; j < m; ++j) cfma_conj(s, ldc(A, j * n + k1), ldc(A, j * n + k2));
      s.re += reg_entry(P.reg, k1, k2, n, P.lambda, w4, RELAXED ? 0.0 : (double)P.d[k1]) + (k1 == k2 ? P.eps : 0.0);
      if (k1 == k2) s.im = 0.0;
      stc(L, i, s);
    }
    for (int i = t; i < n * C; i += NT) {
      const int k = div_C(i), c = i - k * C;
      cd s = cd{0.0, 0.0};
      #pragma unroll 4
      for (int j = 0; j < m; ++j) cfma_conj(s, ldc(A, j * n + k), ldc(b, j * C + c));
      stc(x, i, s);
    }
    __syncthreads();
    // Cholesky (right-looking) in LDS, one barrier per column: step j updates
    // the trailing matrix with the unscaled column j (L_ik -= L_ij conj(L_kj) /
    // piv_j) and scales column j-1, which no thread reads any more.  Only
    // inv[j] = 1 / L_jj is kept: the diagonal itself is read by every thread
    // as the pivot and is never overwritten (nothing later reads it).  Every
    // thread forms 1 / L_jj from the hardware reciprocal square root and two
    // Newton steps, and 1 / piv_j as its square (a few instructions, where a
    // correctly rounded division and square root take dozens).
    double* inv = sm + o.inv;
    for (int j = 0; j < n; ++j) {
      double piv = L[2 * (j * n + j)];
      if (!(piv > 0.0 && isfinite(piv))) piv = 1e-300;
      double rq = __builtin_amdgcn_rsq(piv);
      rq = rq * fma(-0.5 * piv * rq, rq, 1.5);
      rq = rq * fma(-0.5 * piv * rq, rq, 1.5);
      const double ip = rq * rq;
      auto update = [&](int i, int k) {
        cd v = ldc(L, i * n + k);
        cfms_aconjb(v, cscale(ldc(L, i * n + j), ip), ldc(L, k * n + j));
        stc(L, i * n + k, v);
      };
      if (n <= 16) {
        // the trailing block fits a fixed 16 x 16 grid of threads
        const int i = j + 1 + (t >> 4), k = j + 1 + (t & 15);
        if (i < n && k <= i) update(i, k);
      } else {
        const int rem = n - j - 1;
        for (int e = t; e < rem * rem; e += NT) {
          const int i = j + 1 + e / rem, k = j + 1 + e % rem;
          if (k <= i) update(i, k);
        }
      }
      // (leave-one-out kernel) the scaled column j-1 is also mirrored,
      // conjugated, into row j-1 of the upper triangle (unused otherwise),
      // where the team sweeps read it with consecutive lanes on consecutive
      // entries
      if (j > 0)
        for (int i = j + t; i < n; i += NT) {
          const cd v = cscale(ldc(L, i * n + j - 1), inv[j - 1]);
          stc(L, i * n + j - 1, v);
          if constexpr (NR > 0) stc(L, (j - 1) * n + i, cd{v.re, -v.im});
        }
      if (t == 0) inv[j] = rq;
      __syncthreads();
    }

    // Triangular sweeps over a set of right-hand-side columns: the C
    // right-hand sides of x and, for the leave-one-out loss, the m columns of
    // P = conj(A)^T (so that P becomes L^-1 A^H, then G = L^-H P).
    double* Pm = sm + o.P;
    const int ncol = C + (P.mode == 1 ? m : 0);
    auto el = [&](int i, int col) -> double* { return col < C ? x + 2 * (i * C + col) : Pm + 2 * (i * m + col - C); };
    double hj = 0.0;
    if (NR > 0 && ncol >= 32) {
      // Leave-one-out loss, n <= 16: every 16-lane team of the block sweeps
      // four columns at a time, row i in lane i (columns team + 16 r of each
      // group of 64).  Each step broadcasts the final value of row k from lane
      // k (DPP) into the other rows' updates; L comes from LDS, the forward
      // sweep reading its conjugated mirror in the upper triangle.  The
      // leverage h_j = ||P_:j||^2 of a P column is parked in gam[j] (not yet
      // in use) for thread j.
      double* gam = sm + o.gam;
      const int team = t >> 4, l = t & 15;
      const double il = l < n ? inv[l] : 0.0;
      for (int c0 = 0; c0 < ncol; c0 += 64) {
        cd v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = c0 + team + 16 * r, j = col - C;
          v[r] = cd{0.0, 0.0};
          if (col < ncol && l < n) v[r] = col < C ? ldc(x, l * C + col) : cd{A[2 * (j * n + l)], -A[2 * (j * n + l) + 1]};
        }
        // forward: y_k = v_k / L_kk is final at step k; rows i > k subtract L_ik y_k
        static_for<0, 16>([&](auto KK) {
          constexpr int k = decltype(KK)::value;
          if (k + 1 < n) {
            const cd lk = l > k && l < n ? ldc(L, k * n + l) : cd{0.0, 0.0};   // conj(L_lk)
            cd y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) y[r] = cscale(v[r], il);
            dpp_cfms_conja2<k, k>(v[0], lk, y[0], v[1], lk, y[1]);
            dpp_cfms_conja2<k, k>(v[2], lk, y[2], v[3], lk, y[3]);
          }
        });
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          v[r] = cscale(v[r], il);
          const int col = c0 + team + 16 * r;
          const double h = allreduce16(v[r].re * v[r].re + v[r].im * v[r].im);
          if (l == 0 && col >= C && col < ncol) gam[col - C] = h;
        }
        // backward: x_k = w_k / L_kk is final at step k; rows i < k subtract conj(L_ki) x_k
        static_for<0, 16>([&](auto KK) {
          constexpr int k = 15 - decltype(KK)::value;
          if (k >= 1 && k < n) {
            const cd lk = l < k ? ldc(L, k * n + l) : cd{0.0, 0.0};
            cd y[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) y[r] = cscale(v[r], il);
            dpp_cfms_conja2<k, k>(v[0], lk, y[0], v[1], lk, y[1]);
            dpp_cfms_conja2<k, k>(v[2], lk, y[2], v[3], lk, y[3]);
          }
        });
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = c0 + team + 16 * r;
          if (col < ncol && l < n) stc(el(l, col), 0, cscale(v[r], il));
        }
      }
      __syncthreads();
      if (P.mode == 1 && t < m) hj = gam[t];
    } else if (NR == 0 && P.mode == 0 && n <= 16) {
      // Paper loss: the C <= 4 columns of x, one 16-lane team of wave 0 each,
      // row i in lane i.  Each step broadcasts the final value of row k from
      // lane k (DPP) into the updates of the other rows, with L read from
      // LDS; no block barrier until the columns are stored.
      if (t < 64) {
        const int col = t >> 4, l = t & 15;
        const bool live = col < C && l < n;
        cd v = live ? ldc(x, l * C + col) : cd{0.0, 0.0};
        const double il = l < n ? inv[l] : 0.0;
        // forward: x_k = v_k / L_kk is final at step k; rows i > k subtract L_ik x_k
        static_for<0, 16>([&](auto KK) {
          constexpr int k = decltype(KK)::value;
          if (k + 1 < n) {
            const cd y = cscale(v, il);
            const cd lk = l > k && l < n ? ldc(L, l * n + k) : cd{0.0, 0.0};
            dpp_cfms<k>(v, lk, y);
          }
        });
        v = cscale(v, il);
        // backward: x_k = w_k / L_kk is final at step k; rows i < k subtract conj(L_ki) x_k
        static_for<0, 16>([&](auto KK) {
          constexpr int k = 15 - decltype(KK)::value;
          if (k >= 1 && k < n) {
            const cd y = cscale(v, il);
            const cd lk = l < k ? ldc(L, k * n + l) : cd{0.0, 0.0};
            dpp_cfms_conja<k>(v, lk, y);
          }
        });
        v = cscale(v, il);
        if (live) stc(x, l * C + col, v);
      }
      __syncthreads();
    } else {
      // LDS sweeps: each step updates with the final row k and scales the row
      // that became final, one barrier per step.
      if (P.mode == 1) {
        for (int e = t; e < n * m; e += NT) {
          const int k = e / m, j = e - k * m;
          stc(Pm, e, cd{A[2 * (j * n + k)], -A[2 * (j * n + k) + 1]});
        }
        __syncthreads();
      }
      // forward: row 0 scaled, then steps k = 0 .. n-2
      for (int col = t; col < ncol; col += NT) stc(el(0, col), 0, cscale(ldc(el(0, col), 0), inv[0]));
      __syncthreads();
      for (int k = 0; k + 1 < n; ++k) {
        for (int e = t; e < (n - k - 1) * ncol; e += NT) {
          const int i = k + 1 + e / ncol, col = e % ncol;
          cd v = csub(ldc(el(i, col), 0), cmul(ldc(L, i * n + k), ldc(el(k, col), 0)));
          if (i == k + 1) v = cscale(v, inv[i]);
          stc(el(i, col), 0, v);
        }
        __syncthreads();
      }
      if (P.mode == 1 && t < m) {
        for (int k = 0; k < n; ++k) {
          const cd v = ldc(Pm, k * m + t);
          hj += v.re * v.re + v.im * v.im;
        }
      }
      // column t + C of P is read whole above before the thread that owns it
      // (t + C, possibly in another wave) scales its last row below
      __syncthreads();
      // backward: row n-1 scaled, then steps k = n-1 .. 1
      for (int col = t; col < ncol; col += NT) stc(el(n - 1, col), 0, cscale(ldc(el(n - 1, col), 0), inv[n - 1]));
      __syncthreads();
      for (int k = n - 1; k > 0; --k) {
        for (int e = t; e < k * ncol; e += NT) {
          const int i = e / ncol, col = e % ncol;
          cd v = csub(ldc(el(i, col), 0), cmulc(ldc(L, k * n + i), ldc(el(k, col), 0)));
          if (i == k - 1) v = cscale(v, inv[i]);
          stc(el(i, col), 0, v);
        }
        __syncthreads();
      }
    }
    // residual: FIT r = A x - b ; LOO r = b - A x
    const double rs = P.mode == 1 ? -1.0 : 1.0;
    for (int i = t; i < m * C; i += NT) {
      const int j = div_C(i), c = i - j * C;
      cd s = cd{0.0, 0.0};
      #pragma unroll 4
      for (int k = 0; k < n; ++k) cfma(s, ldc(A, j * n + k), ldc(x, k * C + c));
      s = csub(s, ldc(b, i));
      stc(r, i, cscale(s, rs));
    }
    __syncthreads();

    if (P.mode == 0) {
      // loss: ||r||^2 + x^H (lambda G + eps I) x, split over lanes
      for (int i = t; i < m * C; i += NT) { const cd v = ldc(r, i); loss += v.re * v.re + v.im * v.im; }
      for (int i = t; i < n * n * C; i += NT) {
        const int c = div_nn(i), e = i - c * n * n, k1 = div_n(e), k2 = e - k1 * n;
        const double g =
            reg_entry(P.reg, k1, k2, n, P.lambda, w4, RELAXED ? 0.0 : (double)P.d[k1]) + (k1 == k2 ? P.eps : 0.0);
        if (g != 0.0) {
          const cd a = ldc(x, k1 * C + c), bb = ldc(x, k2 * C + c);
          loss += g * (a.re * bb.re + a.im * bb.im);
        }
      }
      for (int i = t; i < m * n; i += NT) {
        const int j = div_n(i), k = i - j * n;
        const cd a = ldc(A, i);
        double s = 0.0;
        for (int c = 0; c < C; ++c) {
          // Im(conj(x) conj(A) r)
          const cd xr = cmulc(ldc(x, k * C + c), ldc(r, j * C + c));
          s += a.re * xr.im - a.im * xr.re;
        }
        T[i] = 4.0 * kPi * s;
      }
    } else {
      double* w = sm + o.w;
      double* y = sm + o.y;
      double* v = sm + o.v;
      double* gam = sm + o.gam;
      double* Wm = sm + o.Wm;
      if (t < m) {
        const double om = 1.0 - hj;
        double rr = 0.0;
        for (int c = 0; c < C; ++c) {
          const cd rv = ldc(r, t * C + c);
          rr += rv.re * rv.re + rv.im * rv.im;
          stc(w, t * C + c, cscale(rv, 1.0 / (om * om)));
        }
        loss += rr / (om * om);
        gam[t] = 2.0 * rr / (om * om * om);
      }
      __syncthreads();
      // y = G w
      for (int i = t; i < n * C; i += NT) {
        const int k = div_C(i), c = i - k * C;
        cd s = cd{0.0, 0.0};
        #pragma unroll 4
        for (int j = 0; j < m; ++j) cfma(s, ldc(Pm, k * m + j), ldc(w, j * C + c));
        stc(y, i, s);
      }
      // Wm[p][k] = sum_i A_ip gam_i G_ki, two entries (p, k) and (p, k + h2)
      // per thread sharing the factor A_ip gam_i
      const int h2 = (n + 1) >> 1;
      const FastDiv div_h2(h2);
      for (int e = t; e < n * h2; e += NT) {
        const int p = div_h2(e), k = e - p * h2;
        const bool two = k + h2 < n;
        const int k1 = two ? k + h2 : k;
        cd s0 = cd{0.0, 0.0}, s1 = cd{0.0, 0.0};
        #pragma unroll 4
        for (int i = 0; i < m; ++i) {
          const cd ag = cscale(ldc(A, i * n + p), gam[i]);
          cfma(s0, ag, ldc(Pm, k * m + i));
          cfma(s1, ag, ldc(Pm, k1 * m + i));
        }
        stc(Wm, p * n + k, s0);
        if (two) stc(Wm, p * n + k1, s1);
      }
      __syncthreads();
      // v = w - A y
      for (int i = t; i < m * C; i += NT) {
        const int j = div_C(i), c = i - j * C;
        cd s = ldc(w, i);
        for (int k = 0; k < n; ++k) s = csub(s, cmul(ldc(A, j * n + k), ldc(y, k * C + c)));
        stc(v, i, s);
      }
      __syncthreads();
      // two entries (j, k) and (j, k + h2) per thread sharing G_pj, v_j and r_j
      for (int e = t; e < m * h2; e += NT) {
        const int j = div_h2(e), k = e - j * h2;
        const bool two = k + h2 < n;
        const int k1 = two ? k + h2 : k;
        cd psi0 = cscale(ldc(Pm, k * m + j), gam[j]);
        cd psi1 = cscale(ldc(Pm, k1 * m + j), gam[j]);
        for (int c = 0; c < C; ++c) {
          const cd vv = ldc(v, j * C + c), rr = ldc(r, j * C + c);
          psi0 = csub(psi0, cmulc(vv, ldc(x, k * C + c)));
          psi0 = csub(psi0, cmulc(rr, ldc(y, k * C + c)));
          psi1 = csub(psi1, cmulc(vv, ldc(x, k1 * C + c)));
          psi1 = csub(psi1, cmulc(rr, ldc(y, k1 * C + c)));
        }
        #pragma unroll 4
        for (int p = 0; p < n; ++p) {
          const cd g = ldc(Pm, p * m + j);
          psi0 = csub(psi0, cmul(g, ldc(Wm, p * n + k)));
          psi1 = csub(psi1, cmul(g, ldc(Wm, p * n + k1)));
        }
        const cd pa0 = cmul(psi0, ldc(A, j * n + k));
        T[j * n + k] = -4.0 * kPi * pa0.im;
        if (two) {
          const cd pa1 = cmul(psi1, ldc(A, j * n + k1));
          T[j * n + k1] = -4.0 * kPi * pa1.im;
        }
      }
    }
    __syncthreads();
    if constexpr (RELAXED) {
      // theta_jk = <P_jk, w>: grad P_jk += T_jk w (each thread keeps the
      // entries it owns, so no barrier is needed between bins)
      for (int i = t; i < m * n; i += NT) {
        gP[2 * i] += T[i] * wx;
        gP[2 * i + 1] += T[i] * wy;
      }
    } else {
      // accumulate the chain rule through theta_jk = d_k <u_j, w>
      if (t < m) {
        double g = 0.0;
        #pragma unroll 4
        for (int k = 0; k < n; ++k) g += (double)P.d[k] * T[t * n + k];
        gu[0] += g * wx;
        gu[1] += g * wy;
      }
      if (t < n) {
        double g = 0.0;
        #pragma unroll 4
        for (int j = 0; j < m; ++j) g += T[j * n + t] * pj[j];
        gd += g;
      }
    }
    __syncthreads();
  }

  // block partials: [loss, grad_u (2m), grad_d (n)], relaxed [loss, grad_P (2mn)]
  double* red = sm + o.red;
  red[t] = loss;
  __syncthreads();
  double* out = P.partial + (size_t)blockIdx.x * P.stride;
  if (t == 0) {
    double s = 0.0;
    for (int i = 0; i < NT; ++i) s += red[i];
    out[0] = s;
  }
  if constexpr (RELAXED) {
    for (int i = t; i < 2 * m * n; i += NT) out[1 + i] = gP[i];
  } else {
    if (t < m) { out[1 + 2 * t] = gu[0]; out[2 + 2 * t] = gu[1]; }
    if (t < n) out[1 + 2 * m + t] = gd;
  }
}

// One block per output value: each thread sums a strided subset of the block
// partials, then a fixed-shape tree in LDS; the order never depends on timing.
__global__ __launch_bounds__(256) void k_calib_reduce(CalibParams P, int nblocks) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int bl = threadIdx.x; bl < nblocks; bl += 256) s += P.partial[(size_t)bl * P.stride + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    s = red[0];
    if (i == 0) P.loss[0] = s;
    else if (P.shifts) P.grad_p[i - 1] = s;
    else if (i <= 2 * P.m) P.grad_u[i - 1] = s;
    else P.grad_d[i - 1 - 2 * P.m] = s;
  }
}

// Blocks resident at once: 256 CUs x (blocks whose LDS fits one CU, at most
// the 4 the register budget of k_calib allows), at most the workspace bound.
// A grid larger than what is resident would leave a tail of late blocks.
int calib_blocks(int Q, size_t lds_per_block) {
  size_t per_cu = lds_per_block ? (size_t)163840 / lds_per_block : 4;
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 4) per_cu = 4;
  size_t nb = 256 * per_cu;
  if (nb > (size_t)kCalibMaxBlocks) nb = kCalibMaxBlocks;
  return Q < (int)nb ? Q : (int)nb;
}

template <bool RELAXED, int NR>
static hipError_t launch_calib_t(const CalibParams& P, hipStream_t s) {
  const size_t lds = calib_lds_bytes(P.m, P.n, P.C, P.mode, RELAXED);
  const int nb = calib_blocks(P.Q, lds);
  // Dynamic LDS beyond 64 KiB needs the kernel attribute on the current
  // device; it is set on every such launch (a host-side call, no stream
  // work), so no process-wide state decides it for another device or thread.
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_calib<RELAXED, NR>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_calib<RELAXED, NR>), dim3(nb), dim3(256), lds, s, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_calib_reduce, dim3(P.stride), dim3(256), 0, s, P, nb);
  return hipGetLastError();
}

hipError_t launch_calib(const CalibParams& P, hipStream_t s) {
  // team sweeps over all waves for the leave-one-out loss (C + m >= 32
  // columns) with at most 16 layers; every other case, the paper loss among
  // them (its C columns swept by the teams of wave 0), runs the kernel
  // without that path, which spills less
  if (P.mode == 1 && P.n <= 16 && P.C + P.m >= 32)
    return P.shifts ? launch_calib_t<true, 16>(P, s) : launch_calib_t<false, 16>(P, s);
  return P.shifts ? launch_calib_t<true, 0>(P, s) : launch_calib_t<false, 0>(P, s);
}

// Partial-sum buffer of the allocation-free calibration entry point: a
// file-scope device array, one copy per GPU, held until the process ends.
// Every block of k_calib overwrites its whole row, so nothing needs clearing
// between calls; calls that overlap in time on one GPU share it and race.
static __device__ __align__(256) double scratch[kCalibScratchBytes / sizeof(double)];

// Device address of `scratch` on the current device.  The name is only a
// host-side stand-in for the array; its address on each device comes from
// the runtime, looked up once per device (under a lock) and kept.
hipError_t calib_scratch(double** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *out = addr[dev];
  return hipSuccess;
}

// Sec. V-B update, u' = u - alpha grad_u / (eps + ||grad_u||^2) (same for d).
__global__ __launch_bounds__(256) void k_gd_step(float2* u, float* d, const double* gu, const double* gd, int m,
                                                 int n, double alpha, double eps_g) {
  __shared__ double su[256], sd[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < 2 * m; i += 256) a += gu[i] * gu[i];
  for (int i = threadIdx.x; i < n; i += 256) b += gd[i] * gd[i];
  su[threadIdx.x] = a;
  sd[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) { su[threadIdx.x] += su[threadIdx.x + w]; sd[threadIdx.x] += sd[threadIdx.x + w]; }
    __syncthreads();
  }
  const double cu = alpha / (eps_g + su[0]);
  const double cdd = alpha / (eps_g + sd[0]);
  for (int j = threadIdx.x; j < m; j += 256) {
    float2 v = u[j];
    v.x = (float)((double)v.x - cu * gu[2 * j]);
    v.y = (float)((double)v.y - cu * gu[2 * j + 1]);
    u[j] = v;
  }
  for (int k = threadIdx.x; k < n; k += 256) d[k] = (float)((double)d[k] - cdd * gd[k]);
}

hipError_t launch_gd_step(float2* u, float* d, const double* gu, const double* gd, int m, int n, double alpha,
                          double eps_g, hipStream_t s) {
  hipLaunchKernelGGL(k_gd_step, dim3(1), dim3(256), 0, s, u, d, gu, gd, m, n, alpha, eps_g);
  return hipGetLastError();
}

}  // namespace fdl
