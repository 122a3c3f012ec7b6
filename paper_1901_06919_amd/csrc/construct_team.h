// Per-bin team solver shared by the plain and the batched construction
// kernels (Sec. V-A, Eq. LayerConstructionClosedForm; regularisers of
// Sec. V-C).
//
// A team is 16 lanes of one wave (one DPP row).  It solves one half-spectrum
// bin w of one light field; lane l owns layers/rows k = l + 16 r (r < R), so
// n <= 16 R.  All arithmetic is FP64.
//
//   1. Views are streamed: each lane forms its own A_jk = exp(2 pi i d_k p_j)
//      (p_j = <u_j, w>) and accumulates c_k = sum_j conj(A_jk) b_j per channel.
//   2. The Gram matrix M = A^H A:
//      TOEP (d an arithmetic progression up to rounding): only the first
//        column's relatives are summed, R_q,t = sum_j p_j^q conj(A_j0) A_jt,
//        q = 0..3, and M_{k,i} = sum_j exp(2 pi i (d_i - d_k) p_j) is
//        recovered exactly from t = i - k and the rounding residue
//        th = 2 pi [(d_i - d_k) - (d_t - d_0)]:
//        M_{k,i} = R0 + i th R1 - th^2/2 R2 - i th^3/6 R3 (remainder
//        (th p)^4/24 < 1e-15 when th |p| <= 3e-4, checked per bin);
//      general: row i accumulates conj(A_ji) A_jk with A_jk broadcast from
//        the lane that owns layer k.
//   3. M += lambda Gamma^H Gamma + eps I.
//   4. Right-looking Cholesky M = L L^H with rows in registers; column j is
//      broadcast with DPP row_newbcast; non-positive pivots are counted.
//   5. Forward substitution (broadcast of y_j) and backward substitution
//      (16-lane DPP reduction per unknown), then the layer values are stored.
#pragma once

#include <type_traits>

#include "fdl_device.h"
#include "fdl_internal.h"

namespace fdl {

template <int I, int N, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (I < N) {
    fn(std::integral_constant<int, I>{});
    static_for<I + 1, N>(fn);
  }
}

// Orders LDS traffic between the lanes of one wave (no block barrier).
__device__ __forceinline__ void team_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// (Gamma^T Gamma)_{ik} for Gamma = tridiag(1,-2,1) of size n (Eq. 2ndOrderLayer).
__device__ __forceinline__ double layer2_gtg(int i, int k, int n) {
  double s = 0.0;
  for (int p = i - 1; p <= i + 1; ++p) {
    if (p < 0 || p >= n) continue;
    const int a = p - i, b = p - k;
    if (b < -1 || b > 1) continue;
    s += (a == 0 ? -2.0 : 1.0) * (b == 0 ? -2.0 : 1.0);
  }
  return s;
}

struct TeamLds {
  double d[32];
  double2 r0[32];
  float4 r12[32];
  float2 r3[32];
};

template <int R>
struct TeamRows {
  cd L0[16];
  cd L1[R > 1 ? 32 : 1];
  template <int r>
  __device__ __forceinline__ cd& at(int k) {
    if constexpr (r == 0) return L0[k];
    else return L1[k];
  }
};

template <int R, int CT, bool TOEP>
__device__ __forceinline__ void team_solve(const ConstructParams& P, TeamLds& T, int f, int lane) {
  constexpr int NMAX = 16 * R;
  const int n = P.n;
  const int C = P.C;

  for (int k = lane; k < NMAX; k += 16) T.d[k] = k < n ? P.d[k] : 0.0;
  team_sync();

  double wx, wy;
  bin_freq(f, P.Wh, P.H, P.W, wx, wy);

  double dk[R];
  cd acc[R][CT];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = lane + 16 * r;
    dk[r] = k < n ? T.d[k] : 0.0;
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[r][c] = cd{0.0, 0.0};
  }
  TeamRows<R> S;
  double pmax = 0.0;

  // ---- 1-2: stream the views ----
  // The next view's position and spectra are loaded one iteration ahead so
  // their latency overlaps the sincos work of the current view.
  const float2* bp = P.view_spec + f;
  const size_t F = (size_t)P.F;
  const int m = P.m;
  float2 un;
  float2 bn[CT];
  auto prefetch = [&](int j) {
    un = P.u[j];
#pragma unroll
    for (int c = 0; c < CT; ++c) bn[c] = bp[((size_t)j * C + (c < C ? c : C - 1)) * F];
  };
  prefetch(0);
  if constexpr (TOEP) {
    cd m0[R], m1[R], m2[R], m3[R];
#pragma unroll
    for (int r = 0; r < R; ++r) m0[r] = m1[r] = m2[r] = m3[r] = cd{0.0, 0.0};
    for (int j = 0; j < m; ++j) {
      const float2 uj = un;
      float2 bc[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) bc[c] = bn[c];
      if (j + 1 < m) prefetch(j + 1);
      const double p = (double)uj.x * wx + (double)uj.y * wy;
      pmax = fmax(pmax, fabs(p));
      cd A[R];
#pragma unroll
      for (int r = 0; r < R; ++r) A[r] = expi2pi(dk[r] * p);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const cd b = c < C ? cd{(double)bc[c].x, (double)bc[c].y} : cd{0.0, 0.0};
#pragma unroll
        for (int r = 0; r < R; ++r) cfma_conj(acc[r][c], A[r], b);
      }
      const cd a0 = bcast16<0>(A[0]);
      const double p2 = p * p, p3 = p2 * p;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const cd g = cmulc(a0, A[r]);
        m0[r] = cadd(m0[r], g);
        m1[r].re = fma(p, g.re, m1[r].re);
        m1[r].im = fma(p, g.im, m1[r].im);
        m2[r].re = fma(p2, g.re, m2[r].re);
        m2[r].im = fma(p2, g.im, m2[r].im);
        m3[r].re = fma(p3, g.re, m3[r].re);
        m3[r].im = fma(p3, g.im, m3[r].im);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int t = lane + 16 * r;
      T.r0[t] = make_double2(m0[r].re, m0[r].im);
      T.r12[t] = make_float4((float)m1[r].re, (float)m1[r].im, (float)m2[r].re, (float)m2[r].im);
      T.r3[t] = make_float2((float)m3[r].re, (float)m3[r].im);
    }
    team_sync();
    const double d0 = T.d[0];
    static_for<0, R>([&](auto RR) {
      constexpr int r = decltype(RR)::value;
      const int i = lane + 16 * r;
      const double di = dk[r];
      static_for<0, 16 * (r + 1)>([&](auto KK) {
        constexpr int k = decltype(KK)::value;
        cd val = cd{0.0, 0.0};
        if (k <= i && i < n) {
          const int t = i - k;
          const double2 q0 = T.r0[t];
          const float4 q12 = T.r12[t];
          const float2 q3 = T.r3[t];
          const double th = kTwoPi * ((di - T.d[k]) - (T.d[t] - d0));
          const double h2 = 0.5 * th * th;
          const double h3 = h2 * th * (1.0 / 3.0);
          const double mre = q0.x - th * (double)q12.y - h2 * (double)q12.z + h3 * (double)q3.y;
          const double mim = q0.y + th * (double)q12.x - h2 * (double)q12.w - h3 * (double)q3.x;
          val = cd{mre, -mim};   // M_{i,k} = conj(M_{k,i})
        }
        S.template at<r>(k) = val;
      });
    });
    if (lane == 0 && P.status && kTwoPi * P.eta_max * pmax > 3e-4) atomicAdd(P.status, 1);
  } else {
    static_for<0, R>([&](auto RR) {
      constexpr int r = decltype(RR)::value;
#pragma unroll
      for (int k = 0; k < 16 * (r + 1); ++k) S.template at<r>(k) = cd{0.0, 0.0};
    });
    for (int j = 0; j < m; ++j) {
      const float2 uj = un;
      float2 bc[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) bc[c] = bn[c];
      if (j + 1 < m) prefetch(j + 1);
      const double p = (double)uj.x * wx + (double)uj.y * wy;
      cd A[R];
#pragma unroll
      for (int r = 0; r < R; ++r) A[r] = expi2pi(dk[r] * p);
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const cd b = c < C ? cd{(double)bc[c].x, (double)bc[c].y} : cd{0.0, 0.0};
#pragma unroll
        for (int r = 0; r < R; ++r) cfma_conj(acc[r][c], A[r], b);
      }
      static_for<0, NMAX>([&](auto KK) {
        constexpr int k = decltype(KK)::value;
        if (k < n) {
          const cd Ak = bcast16<k % 16>(A[k / 16]);
          if constexpr (k < 16) cfma_conj(S.template at<0>(k), A[0], Ak);
          if constexpr (R > 1) cfma_conj(S.template at<1>(k), A[R - 1], Ak);
        }
      });
    }
  }

  // ---- 3: regulariser ----
  {
    const double w2 = wx * wx + wy * wy;
    const double w4 = w2 * w2;
    static_for<0, R>([&](auto RR) {
      constexpr int r = decltype(RR)::value;
      const int i = lane + 16 * r;
      static_for<0, 16 * (r + 1)>([&](auto KK) {
        constexpr int k = decltype(KK)::value;
        if (i < n && k <= i && i - k <= 2) {
          double add = 0.0;
          if (P.reg == 0) {
            if (k == i) { const double d2 = dk[r] * dk[r]; add = P.lambda * w4 * d2 * d2; }
          } else if (P.reg == 1) {
            add = P.lambda * layer2_gtg(i, k, n);
          } else if (k == i) {
            add = P.lambda;
          }
          if (k == i) add += P.eps;
          S.template at<r>(k).re += add;
        }
        if (k == i) S.template at<r>(k).im = 0.0;
      });
    });
  }

  // ---- 4: Cholesky ----
  bool bad = false;
  double invd[R];
#pragma unroll
  for (int r = 0; r < R; ++r) invd[r] = 0.0;
  static_for<0, NMAX>([&](auto JJ) {
    constexpr int j = decltype(JJ)::value;
    if (j < n) {
      constexpr int oj = j % 16, sj = j / 16;
      double piv = bcast16<oj>(S.template at<sj>(j).re);
      if (!(piv > 0.0) || !isfinite(piv)) { bad = true; piv = 1e-300; }
      double y = __builtin_amdgcn_rsq(piv);
      y = y * fma(-0.5 * piv * y, y, 1.5);
      y = y * fma(-0.5 * piv * y, y, 1.5);
      if (lane == oj) invd[sj] = y;
      static_for<0, R>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        if constexpr (j < 16 * (r + 1)) S.template at<r>(j) = cscale(S.template at<r>(j), y);
      });
      static_for<j + 1, NMAX>([&](auto KK) {
        constexpr int k = decltype(KK)::value;
        if (k < n) {
          const cd Lkj = bcast16<k % 16>(S.template at<k / 16>(j));
          static_for<0, R>([&](auto RR) {
            constexpr int r = decltype(RR)::value;
            if constexpr (k < 16 * (r + 1)) cfms_aconjb(S.template at<r>(k), S.template at<r>(j), Lkj);
          });
        }
      });
    }
  });
  if (bad && lane == 0 && P.status) atomicAdd(P.status, 1);

  // strictly lower part only; rows >= n are empty
  static_for<0, R>([&](auto RR) {
    constexpr int r = decltype(RR)::value;
    const int i = lane + 16 * r;
    static_for<0, 16 * (r + 1)>([&](auto KK) {
      constexpr int k = decltype(KK)::value;
      if (k >= i || i >= n) S.template at<r>(k) = cd{0.0, 0.0};
    });
    if (i >= n) {
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[r][c] = cd{0.0, 0.0};
    }
  });

  // ---- 5a: forward substitution L y = c ----
  static_for<0, NMAX>([&](auto JJ) {
    constexpr int j = decltype(JJ)::value;
    if (j < n) {
      constexpr int oj = j % 16, sj = j / 16;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const cd yj = bcast16<oj>(cscale(acc[sj][c], invd[sj]));
        static_for<0, R>([&](auto RR) {
          constexpr int r = decltype(RR)::value;
          if constexpr (j < 16 * (r + 1)) {
            cd t = acc[r][c];
            const cd l = S.template at<r>(j);
            t.re = fma(-l.re, yj.re, t.re);
            t.re = fma(l.im, yj.im, t.re);
            t.im = fma(-l.re, yj.im, t.im);
            t.im = fma(-l.im, yj.re, t.im);
            acc[r][c] = t;
          }
        });
        if (lane == oj) acc[sj][c] = yj;
      }
    }
  });

  // ---- 5b: backward substitution L^H x = y ----
  static_for<0, NMAX>([&](auto II) {
    constexpr int i = NMAX - 1 - decltype(II)::value;
    if (i < n) {
      constexpr int oi = i % 16, si = i / 16;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        cd s = cd{0.0, 0.0};
        static_for<0, R>([&](auto RR) {
          constexpr int r = decltype(RR)::value;
          if constexpr (i < 16 * (r + 1)) cfma_conj(s, S.template at<r>(i), acc[r][c]);
        });
        s.re = allreduce16(s.re);
        s.im = allreduce16(s.im);
        if (lane == oi) acc[si][c] = cscale(csub(acc[si][c], s), invd[si]);
      }
    }
  });

  // ---- store ----
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = lane + 16 * r;
    if (k < n) {
#pragma unroll
      for (int c = 0; c < CT; ++c)
        if (c < C) P.layer_spec[((size_t)k * C + c) * F + f] = make_float2((float)acc[r][c].re, (float)acc[r][c].im);
    }
  }
}

}  // namespace fdl
