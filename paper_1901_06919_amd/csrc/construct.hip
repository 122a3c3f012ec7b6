// Layer construction: per-frequency Tikhonov least squares (Sec. V-A,
// Eq. LayerConstructionClosedForm), sub-aperture inputs (Eq. AMatGeneral with
// psi_j = delta), regularisers of Sec. V-C.
//
// Work decomposition (one CDNA4 wave = 4 teams of 16 lanes = one DPP row each)
//   * one team solves one half-spectrum bin w; lane l of the team owns the
//     rows/layers k = l + 16 r (r < R), so n <= 16 R;
//   * views are streamed (j loop): each lane forms its own A_jk in FP64
//     (sincos2pi), accumulates c_k = sum_j conj(A_jk) b_j for every channel,
//     and the Gram matrix M = A^H A is accumulated either
//       - as Toeplitz moment sums (disparities within 1e-4 rad of an
//         arithmetic progression): M_{k,i} = sum_j exp(2 pi i (d_i-d_k) p_j)
//         = R0_t + i th R1_t - th^2/2 R2_t with t = i-k,
//         R_q,t = sum_j p_j^q conj(A_j0) A_jt, th = 2 pi [(d_i-d_k)-(d_t-d_0)]
//         (the remaining third-order term is below 1e-13 relative), or
//       - directly, row by row, from A_jk broadcast across the team;
//   * the n x n Hermitian system lives in registers (lane = rows), is factored
//     by a right-looking FP64 Cholesky whose column broadcasts are DPP
//     row_newbcast moves, then solved by forward substitution (broadcast of
//     y_j) and backward substitution (16-lane DPP reductions).
// FP64 everywhere: on CDNA4 (packed FP32 disabled) v_fma_f64 issues at the
// same rate as v_fma_f32, and the systems are too ill-conditioned
// (cond(M) up to ~1e6) for an FP32 factorisation.
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

// Gamma^T Gamma for Gamma = tridiag(1,-2,1) of size n (Eq. 2ndOrderLayer).
__device__ __forceinline__ double layer2_gtg(int i, int k, int n) {
  double s = 0.0;
  // (G^T G)_{ik} = sum_p G_{p i} G_{p k}, G_{p q} = -2 (p==q), 1 (|p-q|==1)
  for (int p = i - 1; p <= i + 1; ++p) {
    if (p < 0 || p >= n) continue;
    const int a = p - i, b = p - k;
    const double gi = a == 0 ? -2.0 : 1.0;
    if (b < -1 || b > 1) continue;
    const double gk = b == 0 ? -2.0 : 1.0;
    s += gi * gk;
  }
  return s;
}

template <int R, int CT>
struct TeamSystem {
  // Row storage: slot 0 holds columns 0..15, slot 1 columns 0..31.
  cd L0[16];
  cd L1[R > 1 ? 32 : 1];
  cd acc[R][CT];     // right-hand sides, then y, then x
  double invd[R];    // 1 / L_ii for the owned rows

  template <int r>
  __device__ __forceinline__ cd& at(int k) {
    if constexpr (r == 0) return L0[k];
    else return L1[k];
  }
};

template <int R, int CT>
__global__ __launch_bounds__(256) void k_construct(ConstructParams P) {
  constexpr int NMAX = 16 * R;
  __shared__ double s_d[NMAX];
  __shared__ double2 s_r0[16][NMAX];
  __shared__ float4 s_r12[16][NMAX];
  __shared__ unsigned s_eta_bits, s_p_bits;

  const int tid = threadIdx.x;
  const int lane = tid & 15;
  const int team = tid >> 4;
  const int n = P.n;
  const int C = P.C;

  // ---- block setup: disparities, distance to an arithmetic progression ----
  if (tid < NMAX) s_d[tid] = tid < n ? (double)P.d[tid] : 0.0;
  if (tid == 0) { s_eta_bits = 0u; s_p_bits = 0u; }
  __syncthreads();
  {
    float eta = 0.f;
    for (int q = tid; q < n * n; q += 256) {
      const int k1 = q / n, k2 = q - k1 * n;
      if (k2 > k1) {
        const double e = (s_d[k2] - s_d[k1]) - (s_d[k2 - k1] - s_d[0]);
        eta = fmaxf(eta, (float)fabs(e));
      }
    }
    float pm = 0.f;
    for (int j = tid; j < P.m; j += 256) {
      const float2 uj = P.u[j];
      pm = fmaxf(pm, 0.5f * (fabsf(uj.x) + fabsf(uj.y)));
    }
    atomicMax(&s_eta_bits, __float_as_uint(eta));
    atomicMax(&s_p_bits, __float_as_uint(pm));
  }
  __syncthreads();
  const double eta_max = (double)__uint_as_float(s_eta_bits);
  const double p_max = (double)__uint_as_float(s_p_bits);
  const bool toeplitz = kTwoPi * eta_max * p_max * 1.0000001 <= 1e-4;

  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int f = blk * 16 + team;
  const bool active = f < P.F;

  double wx = 0.0, wy = 0.0;
  if (active) bin_freq(f, P.Wh, P.H, P.W, wx, wy);

  TeamSystem<R, CT> S;
  double dk[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = lane + 16 * r;
    dk[r] = k < n ? s_d[k] : 0.0;
#pragma unroll
    for (int c = 0; c < CT; ++c) S.acc[r][c] = cd{0.0, 0.0};
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) S.L0[k] = cd{0.0, 0.0};
  if constexpr (R > 1) {
#pragma unroll
    for (int k = 0; k < 32; ++k) S.L1[k] = cd{0.0, 0.0};
  }
  cd m0[R], m1[R], m2[R];
#pragma unroll
  for (int r = 0; r < R; ++r) m0[r] = m1[r] = m2[r] = cd{0.0, 0.0};

  // ---- stream the views: A, A^H b, Gram ----
  if (active) {
    const float2* bp = P.view_spec + f;
    const size_t F = (size_t)P.F;
    for (int j = 0; j < P.m; ++j) {
      const float2 uj = P.u[j];
      const double p = (double)uj.x * wx + (double)uj.y * wy;
      cd A[R];
#pragma unroll
      for (int r = 0; r < R; ++r) A[r] = expi2pi(dk[r] * p);
      cd b[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        if (c < C) {
          const float2 v = bp[((size_t)j * C + c) * F];
          b[c] = cd{(double)v.x, (double)v.y};
        } else {
          b[c] = cd{0.0, 0.0};
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) cfma_conj(S.acc[r][c], A[r], b[c]);
      if (toeplitz) {
        const cd a0 = bcast16<0>(A[0]);
        const double p2 = p * p;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const cd g = cmulc(a0, A[r]);
          m0[r] = cadd(m0[r], g);
          m1[r].re = fma(p, g.re, m1[r].re);
          m1[r].im = fma(p, g.im, m1[r].im);
          m2[r].re = fma(p2, g.re, m2[r].re);
          m2[r].im = fma(p2, g.im, m2[r].im);
        }
      } else {
        // M_ik += conj(A_ji) A_jk for the owned rows i, every column k
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
  }

  // ---- Toeplitz assembly through the team's LDS table ----
  if (toeplitz) {
    if (active) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int t = lane + 16 * r;
        if (t < NMAX) {
          s_r0[team][t] = make_double2(m0[r].re, m0[r].im);
          s_r12[team][t] = make_float4((float)m1[r].re, (float)m1[r].im, (float)m2[r].re, (float)m2[r].im);
        }
      }
    }
    __syncthreads();
    if (active) {
      const double d0 = s_d[0];
      static_for<0, R>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        const int i = lane + 16 * r;
        const double di = dk[r];
        static_for<0, 16 * (r + 1)>([&](auto KK) {
          constexpr int k = decltype(KK)::value;
          cd val = cd{0.0, 0.0};
          if (k <= i && i < n) {
            const int t = i - k;
            const double2 q0 = s_r0[team][t];
            const float4 q12 = s_r12[team][t];
            const double th = kTwoPi * ((di - s_d[k]) - (s_d[t] - d0));
            const double h = 0.5 * th * th;
            // M_{k,i} = R0 + i th R1 - h R2 ; store conj(M_{k,i}) = M_{i,k}
            const double mre = q0.x - th * (double)q12.y - h * (double)q12.z;
            const double mim = q0.y + th * (double)q12.x - h * (double)q12.w;
            val = cd{mre, -mim};
          }
          S.template at<r>(k) = val;
        });
      });
    }
  }

  if (!active) return;   // no block-wide barriers below

  // ---- regulariser: lambda Gamma^H Gamma + eps I ----
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
          } else {
            if (k == i) add = P.lambda;
          }
          if (k == i) add += P.eps;
          S.template at<r>(k).re += add;
        }
        if (k == i) S.template at<r>(k).im = 0.0;   // Hermitian diagonal is real
      });
    });
  }

  // ---- Cholesky M = L L^H (right-looking, rows in registers) ----
  bool bad = false;
  static_for<0, NMAX>([&](auto JJ) {
    constexpr int j = decltype(JJ)::value;
    if (j < n) {
      constexpr int oj = j % 16, sj = j / 16;
      double piv = bcast16<oj>(S.template at<sj>(j).re);
      if (!(piv > 0.0) || !isfinite(piv)) { bad = true; piv = 1e-300; }
      double y = __builtin_amdgcn_rsq(piv);
      y = y * fma(-0.5 * piv * y, y, 1.5);
      y = y * fma(-0.5 * piv * y, y, 1.5);
      if (lane == oj) S.invd[sj] = y;
      // scale column j of the owned rows (rows below j become L_ij)
      static_for<0, R>([&](auto RR) {
        constexpr int r = decltype(RR)::value;
        if constexpr (j < 16 * (r + 1)) S.template at<r>(j) = cscale(S.template at<r>(j), y);
      });
      // rank-1 update of the trailing columns
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

  // keep only the strictly lower part (diagonal lives in invd)
  static_for<0, R>([&](auto RR) {
    constexpr int r = decltype(RR)::value;
    const int i = lane + 16 * r;
    static_for<0, 16 * (r + 1)>([&](auto KK) {
      constexpr int k = decltype(KK)::value;
      if (k >= i || i >= n) S.template at<r>(k) = cd{0.0, 0.0};
    });
    if (i >= n) {
#pragma unroll
      for (int c = 0; c < CT; ++c) S.acc[r][c] = cd{0.0, 0.0};
      S.invd[r] = 0.0;
    }
  });

  // ---- forward substitution L y = c ----
  static_for<0, NMAX>([&](auto JJ) {
    constexpr int j = decltype(JJ)::value;
    if (j < n) {
      constexpr int oj = j % 16, sj = j / 16;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const cd own = cscale(S.acc[sj][c], S.invd[sj]);
        const cd yj = bcast16<oj>(own);
        static_for<0, R>([&](auto RR) {
          constexpr int r = decltype(RR)::value;
          if constexpr (j < 16 * (r + 1)) {
            cd t = S.acc[r][c];
            const cd l = S.template at<r>(j);
            t.re = fma(-l.re, yj.re, t.re);
            t.re = fma(l.im, yj.im, t.re);
            t.im = fma(-l.re, yj.im, t.im);
            t.im = fma(-l.im, yj.re, t.im);
            S.acc[r][c] = t;
          }
        });
        if (lane == oj) S.acc[sj][c] = yj;
      }
    }
  });

  // ---- backward substitution L^H x = y ----
  static_for<0, NMAX>([&](auto II) {
    constexpr int i = NMAX - 1 - decltype(II)::value;
    if (i < n) {
      constexpr int oi = i % 16, si = i / 16;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        cd s = cd{0.0, 0.0};
        static_for<0, R>([&](auto RR) {
          constexpr int r = decltype(RR)::value;
          if constexpr (i < 16 * (r + 1)) cfma_conj(s, S.template at<r>(i), S.acc[r][c]);
        });
        s.re = allreduce16(s.re);
        s.im = allreduce16(s.im);
        if (lane == oi) S.acc[si][c] = cscale(csub(S.acc[si][c], s), S.invd[si]);
      }
    }
  });

  // ---- store the layer spectra ----
  const size_t F = (size_t)P.F;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = lane + 16 * r;
    if (k < n) {
#pragma unroll
      for (int c = 0; c < CT; ++c)
        if (c < C) P.layer_spec[((size_t)k * C + c) * F + f] = make_float2((float)S.acc[r][c].re, (float)S.acc[r][c].im);
    }
  }
}

template <int R, int CT>
static hipError_t launch_construct_rc(const ConstructParams& P, hipStream_t s) {
  const int blocks = (P.F + 15) / 16;
  hipLaunchKernelGGL((k_construct<R, CT>), dim3(blocks), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_construct(const ConstructParams& P, hipStream_t s) {
  const bool r1 = P.n <= 16;
  switch (P.C) {
    case 1: return r1 ? launch_construct_rc<1, 1>(P, s) : launch_construct_rc<2, 1>(P, s);
    case 2: return r1 ? launch_construct_rc<1, 2>(P, s) : launch_construct_rc<2, 2>(P, s);
    case 3: return r1 ? launch_construct_rc<1, 3>(P, s) : launch_construct_rc<2, 3>(P, s);
    default: return r1 ? launch_construct_rc<1, 4>(P, s) : launch_construct_rc<2, 4>(P, s);
  }
}

}  // namespace fdl
