// Per-bin team solver shared by the plain and the batched construction
// kernels (Sec. V-A, Eq. LayerConstructionClosedForm; regularisers of
// Sec. V-C).
//
// A team is 16 lanes of one wave (one DPP row).  It solves one half-spectrum
// bin w of one light field; lane l owns layers/rows k = l + 16 r (r < R), so
// n <= 16 R.  All arithmetic is FP64.
//
//   1. Views are streamed: each lane forms its own A_jk = exp(2 pi i d_k p_j)
//      (p_j = <u_j, w>) from a 256-entry table of exp(2 pi i t/256) and a short
//      series for the remainder, and accumulates c_k = sum_j conj(A_jk) b_j
//      per channel.
//   2. The Gram matrix M = A^H A:
//      TOEP (d an arithmetic progression up to rounding): only the first
//        column's relatives are summed, R_q,t = sum_j p_j^q conj(A_j0) A_jt,
//        q = 0..2, and M_{k,i} = sum_j exp(2 pi i (d_i - d_k) p_j) is
//        recovered exactly from t = i - k and the rounding residue
//        th = 2 pi [(d_i - d_k) - (d_t - d_0)]:
//        M_{k,i} = R0 + i th R1 - th^2/2 R2 (relative remainder below
//        (th p)^3/6 < 5e-12 when th |p| <= 3e-4, checked per bin);
//      general: row i accumulates conj(A_ji) A_jk with A_jk broadcast from
//        the lane that owns layer k.
//   3. The diagonal of lambda Gamma^H Gamma + eps I is added to each pivot as
//      the factorisation reaches it (the diagonal registers hold only the
//      Gram part); the off-diagonal bands of the layer regulariser are added
//      to the lower triangle before.
//   4. Right-looking Cholesky M = L L^H with rows in registers; column j is
//      broadcast with DPP row_newbcast; non-positive pivots are counted.
//      Rows n..16R-1 pad the system: their pivots are forced to 1, their
//      unknowns to 0 (1/L_jj := 0) and their rows of L are cleared after the
//      factorisation, so they never reach the live unknowns (the live block
//      of L does not depend on later rows).
//   5. Forward substitution (broadcast of y_j); backward substitution either
//      with a 16-lane DPP reduction per unknown (R = 1) or, for R = 2, after
//      transposing L through LDS so that lane k holds column k of L, with a
//      broadcast of x_i per unknown.  Then the layer values are stored.
#pragma once

#include "fdl_device.h"
#include "fdl_internal.h"

namespace fdl {

// Orders LDS traffic between the lanes of one wave (no block barrier).
__device__ __forceinline__ void team_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- aperture spectra in FP64 (inputs with their own apertures) -------------
// 2 J1(z)/z: its power series sum_k (-1)^k (z/2)^(2k) / (k! (k+1)!) through
// k = 26 for z <= 12 (largest term about 700, so about 1e-13 absolute), and
// for z > 12 the Hankel expansion J1(z) = sqrt(2/(pi z)) (P cos chi - Q sin chi),
// chi = z - 3 pi/4, with P = sum_k (-1)^k a_2k z^-2k, Q = sum_k (-1)^k a_2k+1
// z^-(2k+1), a_k = prod_{i<=k} (4 - (2i-1)^2) / (k! 8^k), through k = 12
// (truncation below 1e-13 at z = 12 and falling fast beyond).
struct JincCoef {
  double s[27], p[13], q[13];
};
constexpr JincCoef make_jinc_coef() {
  JincCoef c{};
  double f = 1.0;   // k! (k+1)!
  for (int k = 0; k <= 26; ++k) {
    if (k > 0) f *= (double)k * (double)(k + 1);
    c.s[k] = (k % 2 ? -1.0 : 1.0) / f;
  }
  double a[26] = {};
  a[0] = 1.0;
  for (int k = 1; k < 26; ++k) a[k] = a[k - 1] * (4.0 - (double)((2 * k - 1) * (2 * k - 1))) / (8.0 * k);
  for (int k = 0; k <= 12; ++k) {
    c.p[k] = (k % 2 ? -1.0 : 1.0) * a[2 * k];
    c.q[k] = (k % 2 ? -1.0 : 1.0) * a[2 * k + 1];
  }
  return c;
}

__device__ __forceinline__ double jinc64(double z) {
  constexpr JincCoef K = make_jinc_coef();
  if (z <= 12.0) {
    const double y = 0.25 * z * z;
    double s = K.s[26];
    static_for<0, 26>([&](auto II) { s = fma(s, y, K.s[25 - decltype(II)::value]); });
    return s;
  }
  const double iz = 1.0 / z, iz2 = iz * iz;
  double p = K.p[12], q = K.q[12];
  static_for<0, 12>([&](auto II) {
    p = fma(p, iz2, K.p[11 - decltype(II)::value]);
    q = fma(q, iz2, K.q[11 - decltype(II)::value]);
  });
  q *= iz;
  double sn, cs;
  sincos2pi(z * (1.0 / kTwoPi) - 0.375, sn, cs);   // chi in turns
  const double j1 = sqrt(2.0 / (kPi * z)) * (p * cs - q * sn);
  return 2.0 * j1 * iz;
}

// sin(pi t) / (pi t)
__device__ __forceinline__ double sinc64(double t) {
  const double a = kPi * t;
  if (fabs(t) < 1e-6) return 1.0 - a * a * (1.0 / 6.0);
  double sn, cs;
  sincos2pi(0.5 * t, sn, cs);
  return sn / a;
}

// psi_hat((s - d) w) of a unit-integral aperture (shape uniform over the
// wave): disk of radius rho 2 J1(z)/z, z = 2 pi rho |s - d| |w|; square of
// half-side rho sinc(2 rho (s - d) w_x) sinc(2 rho (s - d) w_y); else 1.
__device__ __forceinline__ double aperture64(int shape, double rho, double a, double wx, double wy, double wn) {
  if (shape == 1) return jinc64(kTwoPi * rho * fabs(a) * wn);
  if (shape == 2) return sinc64(2.0 * rho * a * wx) * sinc64(2.0 * rho * a * wy);
  return 1.0;
}

// sin(pi x) / (pi x) for the regulariser entries: exact reduction of the
// half-angle in FP64, then the FP32 transcendental unit (about 1e-7).
__device__ __forceinline__ float sinc_pi(double x) {
  if (fabs(x) < 1e-4) {
    const double a = kPi * x;
    return (float)(1.0 - a * a * (1.0 / 6.0));
  }
  const double h = 0.5 * x;
  return __builtin_amdgcn_sinf((float)(h - rint(h))) / (float)(kPi * x);
}

// Per-block table of exp(2 pi i t / kPhaseTab), t = 0..kPhaseTab-1.
constexpr int kPhaseTab = 256;

__device__ __forceinline__ void fill_phase_table(double2* tab) {
  for (int t = threadIdx.x; t < kPhaseTab; t += blockDim.x) {
    double s, c;
    sincos2pi((double)t * (1.0 / kPhaseTab), s, c);
    tab[t] = make_double2(c, s);
  }
}

// exp(2 pi i d p) with dt = kPhaseTab * d: the nearest table entry t = rint(dt p)
// times exp(i x) of the remainder x = 2 pi (dt p - t) / kPhaseTab, |x| <= pi/256,
// summed as Taylor series (sin through x^5, cos through x^6: truncation below
// 1e-17).  dt p - t is formed by one fused multiply-add, so the phase keeps
// full precision for any |d p| < 2^22.
__device__ __forceinline__ cd expi_tab(const double2* __restrict__ tab, double dt, double p) {
  const double t = rint(dt * p);
  const double f = fma(dt, p, -t);
  const double x = f * (kTwoPi / kPhaseTab);
  const double x2 = x * x;
  const double sx = fma(x * x2, fma(x2, 1.0 / 120.0, -1.0 / 6.0), x);
  const double cx = fma(x2, fma(x2, fma(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
  const double2 e = tab[(int)t & (kPhaseTab - 1)];
  return cd{fma(e.x, cx, -e.y * sx), fma(e.y, cx, e.x * sx)};
}

// e_t = d_t - d_0, then either the per-view records of one batch of the
// Toeplitz view loop (at most 16 views x 6 entries) or, after the loop, the
// moments R0, R1, R2 of the Toeplitz Gram (FP64).
constexpr int kViewBatch = 16;
struct TeamMoments {
  double e[32];
  union {
    struct {
      double2 r0[32];
      double2 r1[32];
      double2 r2[32];
    };
    double2 views[kViewBatch * 6];
  };
};

// right-hand sides parked in LDS during the factorisation (lane-major)
struct TeamRhs {
  double2 c[16][8];
};

// 16 x 16 complex tile for the transposition of L (row stride 17 entries so
// that the row-wise writes and the column-wise reads both spread over the
// LDS banks); only the R = 2 solver uses it, after the moments are dead.
constexpr int kTrStride = 17;

// One team's LDS: the view records and moments of the Gram phase, the
// right-hand sides parked during the factorisation and the transposition tile
// of the backward pass are never live together, so they share one area.
template <int R>
union TeamLds {
  TeamMoments m;
  TeamRhs rhs;
  double2 tr[R > 1 ? 16 * kTrStride : 1];
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

// Ends a scheduling region: the unrolled solver is one basic block, and
// without these fences the scheduler hoists loads and broadcasts of later
// steps far enough to exceed the register budget.
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// Pins the computation of v at this point (an empty asm that reads and
// writes it): keeps the compiler from sinking the assembly arithmetic to the
// first use of each entry while its LDS operands stay live in between.
__device__ __forceinline__ void pin(cd& v) { asm volatile("" : "+v"(v.re), "+v"(v.im)); }

// acc -= conj(a) * x
__device__ __forceinline__ void cfms_conja(cd& acc, cd a, cd x) {
  acc.re = fma(-a.re, x.re, acc.re);
  acc.re = fma(-a.im, x.im, acc.re);
  acc.im = fma(-a.re, x.im, acc.im);
  acc.im = fma(a.im, x.re, acc.im);
}

// In-place transposition of the strictly lower factor held by a team
// (R = 2): on entry lane l holds rows l (L0[k] = L_{l,k}, k < 16) and l + 16
// (L1[k] = L_{l+16,k}, k < 32); on exit it holds columns l and l + 16:
//   L_{i,l}    = L0[i] for i < 16, L1[i - 16] for i >= 16,
//   L_{i,l+16} = L1[i] for i >= 16.
// Three 16 x 16 tiles pass through the team's LDS tile in the order
// (0,0), (1,1), (1,0), which frees each register range before it is reused.
template <int R>
__device__ __forceinline__ void team_transpose(TeamRows<R>& S, double2* tr, int lane) {
  auto pass = [&](auto get, auto set) {
    team_sync();
    static_for<0, 16>([&](auto KK) {
      constexpr int k = decltype(KK)::value;
      const cd v = get(std::integral_constant<int, k>{});
      tr[lane * kTrStride + k] = make_double2(v.re, v.im);
    });
    team_sync();
    static_for<0, 16>([&](auto II) {
      constexpr int i = decltype(II)::value;
      const double2 v = tr[i * kTrStride + lane];
      set(std::integral_constant<int, i>{}, cd{v.x, v.y});
    });
  };
  pass([&](auto k) { return S.L0[k]; }, [&](auto i, cd v) { S.L0[i] = v; });
  pass([&](auto k) { return S.L1[16 + k]; }, [&](auto i, cd v) { S.L1[16 + i] = v; });
  pass([&](auto k) { return S.L1[k]; }, [&](auto i, cd v) { S.L1[i] = v; });
  team_sync();
}

// Views on a complete lattice in raster order: u_j = o + a g1 + b g2 for
// j = a B + b, a < A, b < B (a plenoptic camera's sub-aperture views).  Then
// p_j = <u_j, w> = <o, w> + a <g1, w> + b <g2, w>, and each phase of Sec. V-A
// factors as exp(2 pi i e p_j) = exp(2 pi i e <o, w>) U^a V^b with
// U = exp(2 pi i e <g1, w>), V = exp(2 pi i e <g2, w>): the Toeplitz view loop
// steps from one view's phase to the next with one complex product.
struct ViewLattice {
  double ox, oy, g1x, g1y, g2x, g2y;
  int B;
  bool ok;   // the positions satisfy the identity exactly, with B <= 16
};

// Test of the positions by one team (every lane gets the same result; the
// other teams of the wave, if active, test the same positions).  B is the
// first index that leaves the progression u_0 + j (u_1 - u_0); the identity is
// then checked for every view in FP64, where the differences and small
// multiples of float positions are exact, so any mismatch selects the table
// path.  Positions off a lattice usually fail at j = 2 or on m mod B.
__device__ __forceinline__ ViewLattice find_view_lattice(const float2* __restrict__ u, int m, int lane) {
  ViewLattice L;
  const float2 u0 = u[0];
  const float2 u1 = u[m > 1 ? 1 : 0];
  L.ox = u0.x;
  L.oy = u0.y;
  L.g2x = (double)u1.x - L.ox;
  L.g2y = (double)u1.y - L.oy;
  // lane l tests j = l + 2 (2 <= j <= 16)
  bool off = false;
  const int jb = lane + 2;
  if (jb < m && jb <= 16) {
    const float2 v = u[jb];
    off = (double)v.x != fma((double)jb, L.g2x, L.ox) || (double)v.y != fma((double)jb, L.g2y, L.oy);
  }
  const unsigned long long brk = __ballot(off);
  int B = m;
  if (brk != 0)
    B = (__ffsll((long long)brk) - 1) % 16 + 2;   // first break in any active team (all test the same j)
  else if (m > 17)
    B = 17;                                       // no break up to j = 16: a row longer than 16 views
  L.B = B;
  L.ok = false;
  if (B > 16 || m % B != 0) return L;
  const float2 uB = u[B < m ? B : 0];
  L.g1x = (double)uB.x - L.ox;
  L.g1y = (double)uB.y - L.oy;
  // a = floor(j / B) from (j + 1/2) / B, which stays at least 1/32 away from
  // an integer (B <= 16) while its float error is below 1e-3 (j < 2^14)
  const float rb = 1.0f / (float)B;
  bool bad = false;
  for (int j = lane; j < m; j += 16) {
    const int a = (int)(((float)j + 0.5f) * rb);
    const int b = j - a * B;
    const float2 v = u[j];
    bad = bad || (double)v.x != fma((double)a, L.g1x, fma((double)b, L.g2x, L.ox)) ||
          (double)v.y != fma((double)a, L.g1y, fma((double)b, L.g2y, L.oy));
  }
  L.ok = __ballot(bad) == 0;
  return L;
}

// APER: the inputs carry their own apertures (Eq. AMatGeneral):
// A_jk = exp(2 pi i d_k p_j) psi_hat_j((s_j - d_k) w), general Gram path only.
// SHIFTS: the relaxed model (Sec. VIII-B), a free shift pair per view and
// layer: A_jk = exp(2 pi i <P_jk, w>), general Gram path only.
// REGION: the second-order view regulariser over the camera-plane square of
// side P.region (Eq. GTG): the diagonal of the view regulariser plus the dense
// off-diagonal part lambda |w|^4 d_i^2 d_k^2 sinc(r dd w_x) sinc(r dd w_y)
// (P.reg must be 0).
template <int R, int CT, bool TOEP, bool APER = false, bool SHIFTS = false, bool REGION = false, int NF = 16 * R>
__device__ __forceinline__ void team_solve(const ConstructParams& P, TeamLds<R>& T, const double2* __restrict__ tab,
                                           int f, int lane) {
  static_assert(!(TOEP && APER), "apertures break the Toeplitz structure");
  static_assert(!(SHIFTS && (TOEP || APER)), "free shifts use the general Gram path without apertures");
  // The system is padded to NMAX = 16 R unknowns with an identity block
  // (rows and columns >= n), so that every unrolled step below runs without
  // a branch on n: the padded unknowns have zero right-hand sides and solve
  // to zero without touching the others.
  constexpr int NMAX = 16 * R;
  // Rows and columns >= NF (n <= NF <= NMAX) are never touched by the Gram
  // sums, the factorisation or the substitutions: their unknowns are zero.
  static_assert(NF > 16 * (R - 1) && NF <= NMAX, "NF must lie in the last row slot");
  const int n = P.n;
  const int C = P.C;

  // e_k = d_k - d_0 (exact in FP64); padded layers take e = 0 (d = d_0)
  const double d0 = P.d[0];
  for (int k = lane; k < NMAX; k += 16) T.m.e[k] = k < n ? P.d[k] - d0 : 0.0;
  team_sync();

  double wx, wy;
  bin_freq(f, P.Wh, P.H, P.W, wx, wy);

  double dk[R], dt[R];
  cd acc[R][CT];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = lane + 16 * r;
    dk[r] = k < n ? T.m.e[k] + d0 : 0.0;
    dt[r] = dk[r] * kPhaseTab;
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[r][c] = cd{0.0, 0.0};
  }
  TeamRows<R> S;
  double pmax = 0.0;

  // ---- 1-2: stream the views ----
  // The view loop runs at a raised wave priority, the factorisation at the
  // default: with two waves per SIMD, the wave in the view loop (LDS reads,
  // independent accumulators) then takes the issue slots that the other
  // wave's dependent DPP chains leave (measured 2-3.5 % on the 30-row kernel).
  __builtin_amdgcn_s_setprio(1);
  // Channels c >= C (CT > C) read channel C - 1; their sums are never stored.
  const size_t F = (size_t)P.F;
  const int m = P.m;
  // The spectra and positions are read as buffer loads: a uniform base and
  // offsets in SGPRs plus a 32-bit lane offset (bin f), so no 64-bit address
  // arithmetic runs per lane.  Positions (and, with APER, focus, radius and
  // shape) are read through a lane-varying (zero) offset so that they travel
  // as vector loads: a scalar load would share its wait counter with the LDS
  // table reads and stall every one of them.
  unsigned vzero;
  asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
  const unsigned foff = (unsigned)f * 8u;
  const unsigned cstride = (unsigned)P.F * 8u;   // bytes between the channels of one view
  const auto u_rsrc = buf_rsrc(P.u);
  auto at = [](const void* base, unsigned off) -> const char* { return (const char*)base + off; };
  struct ViewIn {
    float2 u;
    float s, rho;
    int shape;
    float2 sh[SHIFTS ? R : 1];
  };
  auto load = [&](int j, ViewIn& v, float2 (&b)[CT]) {
    if constexpr (SHIFTS) {
      // the shifts of this lane's layers (padded layers read layer n - 1;
      // their entries are replaced by the identity block)
#pragma unroll
      for (int r = 0; r < R; ++r)
        v.sh[r] = *(const float2*)at(P.shifts + (size_t)j * n, 8u * (unsigned)min(lane + 16 * r, n - 1));
    } else if constexpr (APER) {
      const float* q = (const float*)at(P.views + 5 * (size_t)j, vzero);
      v.u = make_float2(q[0], q[1]);
      v.s = q[2];
      v.rho = q[3];
      v.shape = __float_as_int(q[4]);
    } else {
      v.u = buf_load_f2(u_rsrc, vzero, 8u * (unsigned)j);
    }
    const auto b_rsrc = buf_rsrc(P.view_spec + (size_t)j * C * F);
#pragma unroll
    for (int c = 0; c < CT; ++c) b[c] = buf_load_f2(b_rsrc, foff, cstride * (unsigned)(c < C ? c : C - 1));
  };
  const double wn = sqrt(wx * wx + wy * wy);
  cd m0[R], m1[R], m2[R];
  if constexpr (TOEP) {
#pragma unroll
    for (int r = 0; r < R; ++r) m0[r] = m1[r] = m2[r] = cd{0.0, 0.0};
  } else {
    // the Gram sums start from the off-diagonal bands of the layer
    // regulariser (zero for the other regularisers)
    const double b1 = P.reg == 1 ? -4.0 * P.lambda : 0.0;
    const double b2 = P.reg == 1 ? P.lambda : 0.0;
    static_for<0, R>([&](auto RR) {
      constexpr int r = decltype(RR)::value;
      const int i = lane + 16 * r;
      static_for<0, 16 * (r + 1)>([&](auto KK) {
        constexpr int k = decltype(KK)::value;
        double band = i - k == 1 ? b1 : 0.0;
        band = i - k == 2 ? b2 : band;
        S.template at<r>(k) = cd{band, 0.0};
      });
    });
  }
  auto view = [&](const ViewIn& vj, const float2 (&bc)[CT]) {
    cd A[R];
    double p = 0.0;
    if constexpr (SHIFTS) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        A[r] = expi_tab(tab, (double)kPhaseTab, fma((double)vj.sh[r].x, wx, (double)vj.sh[r].y * wy));
    } else {
      p = fma((double)vj.u.x, wx, (double)vj.u.y * wy);
#pragma unroll
      for (int r = 0; r < R; ++r) A[r] = expi_tab(tab, dt[r], p);
    }
    if constexpr (APER) {
      // the aperture of view j is the same in every lane of the wave
      const int shape = __builtin_amdgcn_readfirstlane(vj.shape);
      const float rho = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(vj.rho)));
      if (rho != 0.0f && (shape == 1 || shape == 2)) {
        sched_fence();
#pragma unroll
        for (int r = 0; r < R; ++r) {
          A[r] = cscale(A[r], aperture64(shape, (double)rho, (double)vj.s - dk[r], wx, wy, wn));
          sched_fence();
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const cd b = cd{(double)bc[c].x, (double)bc[c].y};
#pragma unroll
      for (int r = 0; r < R; ++r) cfma_conj(acc[r][c], A[r], b);
    }
    // row i accumulates conj(A_ji) A_jk, A_jk broadcast from its lane.  Where
    // only one row of the lane takes part (k >= 16, or R = 1), columns k and
    // k + 1 share one block.
    static_for<0, NF>([&](auto KK) {
      constexpr int k = decltype(KK)::value;
      constexpr int r1 = R - 1, k1 = 16 * (R - 1);   // the single-row range starts at k1
      if constexpr (R > 1 && k < 16)
        dpp_cfma_conj<k % 16>(S.template at<0>(k), A[0], S.template at<1>(k), A[1], A[0]);
      else if constexpr (!SHIFTS && ((k - k1) & 1) == 0 && k + 1 < NF)
        dpp_cfma_conj2<k % 16, (k + 1) % 16>(S.template at<r1>(k), A[r1], A[r1], S.template at<r1>(k + 1), A[r1],
                                             A[r1]);
      else if constexpr (SHIFTS || ((k - k1) & 1) == 0)
        dpp_cfma_conj<k % 16>(S.template at<r1>(k), A[r1], A[r1]);
    });
  };
  if constexpr (TOEP) {
    // Toeplitz path.  Everything the lanes share about view j is formed once,
    // by one lane, for a batch of up to 16 views and staged in LDS:
    //   beta_jc = conj(A_j0) b_jc, Z_j = exp(2 pi i (d_16 - d_0) p_j), p_j, p_j^2.
    // Lane l then needs only W_jt = conj(A_j0) A_jt for its rows t = l, l + 16
    // and accumulates c_t += conj(W_jt) beta_jc (= conj(A_jt) b_jc) and the
    // moments R_q,t = sum_j p_j^q W_jt.  W_jt is formed in one of two ways.
    //
    // Table path (any positions):
    //   W_jl = exp(2 pi i (d_l - d_0) p_j) from the table, and
    //   W_j,l+16 = W_jl Z_j exp(i phi), phi = 2 pi eta_l p_j,
    //   eta_l = (d_{l+16} - d_l) - (d_16 - d_0) (float rounding; |eta_l| <=
    //   eta_max, so |phi| <= 3e-4 when the status check passes, and the series
    //   1 - phi^2/2 + i phi is exact to 5e-12); the moments are summed per view.
    //
    // Lattice path (ViewLattice): the batches are the lattice rows, and
    //   W_jt = E_t U_t^a V_t^b is stepped along a row by V_t and from row to
    //   row by U_t.  The row start is recomputed from the table every 8 rows,
    //   so at most 7 + 15 rounded products separate a phase from a table value
    //   (relative error below 1e-14).  The moments follow in closed form from
    //   sums over the rows and along a row (below), so a view costs only its
    //   right-hand-side products and one step.
    double2* rec = T.m.views;
    constexpr int RS = CT + 2;   // record: beta[CT], Z, (p, p^2)
    const double dt0 = kPhaseTab * d0;
    const ViewLattice lat = find_view_lattice(P.u, m, lane);
    // raw inputs of the next batch (lane l: view j0 + l), loaded one batch ahead
    float2 nu, nb[CT];
    auto fetch = [&](int j0) {
      const int jc = min(j0 + lane, m - 1);
      nu = P.u[jc];
#pragma unroll
      for (int c = 0; c < CT; ++c) nb[c] = P.view_spec[((size_t)jc * C + (c < C ? c : C - 1)) * F + f];
    };
    // stages the records of views j0 .. j0 + nbv - 1 (lane l: view j0 + l)
    // and fetches the next batch; the lattice path needs neither Z nor p
    auto produce = [&](int j0, int nbv, double dtz, bool full) {
      const float2 uu = nu;
      float2 bb[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) bb[c] = nb[c];
      if (j0 + nbv < m) fetch(j0 + nbv);
      const bool valid = lane < nbv && j0 + lane < m;
      const double p = fma((double)uu.x, wx, (double)uu.y * wy);
      const cd a0 = expi_tab(tab, dt0, p);
      cd z = cd{1.0, 0.0};
      if constexpr (R > 1)
        if (full) z = expi_tab(tab, dtz, p);
      pmax = fmax(pmax, valid ? fabs(p) : 0.0);
      team_sync();   // the previous batch's records have been read
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const cd be = valid ? cmulc(a0, cd{(double)bb[c].x, (double)bb[c].y}) : cd{0.0, 0.0};
        rec[lane * RS + c] = make_double2(be.re, be.im);
      }
      if (full) {
        rec[lane * RS + CT] = make_double2(z.re, z.im);
        rec[lane * RS + CT + 1] = make_double2(p, p * p);
      }
      team_sync();
    };
    if (lat.ok) {
      const int B = lat.B;
      const double po = fma(lat.ox, wx, lat.oy * wy);
      const double pg1 = fma(lat.g1x, wx, lat.g1y * wy);
      const double pg2 = fma(lat.g2x, wx, lat.g2y * wy);
      double dte[R];
      cd Srow[R], Ust[R], Vst[R];
      // sums over the lattice rows of a^k E U^a, k = 0, 1, 2
      cd T0[R], T1[R], T2[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        dte[r] = kPhaseTab * T.m.e[lane + 16 * r];
        Srow[r] = expi_tab(tab, dte[r], po);
        Ust[r] = expi_tab(tab, dte[r], pg1);
        Vst[r] = expi_tab(tab, dte[r], pg2);
        T0[r] = T1[r] = T2[r] = cd{0.0, 0.0};
      }
      fetch(0);
      int arow = 0;
      for (int j0 = 0; j0 < m; j0 += B, ++arow) {
        produce(j0, B, 0.0, false);
        const double fa = (double)arow, fa2 = fa * fa;
        cd W[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          W[r] = Srow[r];
          T0[r] = cadd(T0[r], Srow[r]);
          T1[r] = cd{fma(fa, Srow[r].re, T1[r].re), fma(fa, Srow[r].im, T1[r].im)};
          T2[r] = cd{fma(fa2, Srow[r].re, T2[r].re), fma(fa2, Srow[r].im, T2[r].im)};
        }
#pragma unroll 2
        for (int v = 0; v < B; ++v) {
          const double2* q = rec + v * RS;
#pragma unroll
          for (int c = 0; c < CT; ++c) {
            const double2 be = q[c];
#pragma unroll
            for (int r = 0; r < R; ++r) cfma_conj(acc[r][c], W[r], cd{be.x, be.y});
          }
#pragma unroll
          for (int r = 0; r < R; ++r) W[r] = cmul(W[r], Vst[r]);
        }
        // start of the next lattice row
        if (((arow + 1) & 7) == 0) {
          const double pa = fma((double)(arow + 1), pg1, po);
#pragma unroll
          for (int r = 0; r < R; ++r) Srow[r] = expi_tab(tab, dte[r], pa);
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) Srow[r] = cmul(Srow[r], Ust[r]);
        }
      }
      // R_q,t = sum_j p_j^q W_jt with p_j = po + a pg1 + b pg2 and
      // W_jt = E U^a V^b, from T_k and SV_k = sum_b b^k V^b:
      //   R0 = X, R1 = po X + pg1 Y + pg2 Z,
      //   R2 = po (po X + 2 pg1 Y + 2 pg2 Z) + pg1^2 Q + pg2^2 S + 2 pg1 pg2 N,
      // X = T0 SV0, Y = T1 SV0, Z = T0 SV1, Q = T2 SV0, S = T0 SV2, N = T1 SV1.
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cd sv0 = cd{0.0, 0.0}, sv1 = sv0, sv2 = sv0, vb = cd{1.0, 0.0};
        for (int b = 0; b < B; ++b) {
          const double fb = (double)b, fb2 = fb * fb;
          sv0 = cadd(sv0, vb);
          sv1 = cd{fma(fb, vb.re, sv1.re), fma(fb, vb.im, sv1.im)};
          sv2 = cd{fma(fb2, vb.re, sv2.re), fma(fb2, vb.im, sv2.im)};
          vb = cmul(vb, Vst[r]);
        }
        const cd X = cmul(T0[r], sv0), Y = cmul(T1[r], sv0), Z = cmul(T0[r], sv1);
        const cd Q = cmul(T2[r], sv0), S2 = cmul(T0[r], sv2), N = cmul(T1[r], sv1);
        m0[r] = X;
        m1[r] = cd{fma(pg2, Z.re, fma(pg1, Y.re, po * X.re)), fma(pg2, Z.im, fma(pg1, Y.im, po * X.im))};
        const double g1 = 2.0 * pg1, g2 = 2.0 * pg2, g12 = 2.0 * pg1 * pg2;
        const double pg1s = pg1 * pg1, pg2s = pg2 * pg2;
        const double lre = fma(g2, Z.re, fma(g1, Y.re, po * X.re));
        const double lim = fma(g2, Z.im, fma(g1, Y.im, po * X.im));
        m2[r] = cd{fma(g12, N.re, fma(pg2s, S2.re, fma(pg1s, Q.re, po * lre))),
                   fma(g12, N.im, fma(pg2s, S2.im, fma(pg1s, Q.im, po * lim)))};
      }
    } else {
      const double dtl = kPhaseTab * T.m.e[lane];
      double c1 = 0.0, h1 = 0.0, dtz = 0.0;
      if constexpr (R > 1) {
        c1 = kTwoPi * ((T.m.e[lane + 16] - T.m.e[lane]) - T.m.e[16]);
        h1 = -0.5 * c1 * c1;
        dtz = kPhaseTab * T.m.e[16];
      }
      fetch(0);
      for (int j0 = 0; j0 < m; j0 += kViewBatch) {
        produce(j0, kViewBatch, dtz, true);
        const int nv = min(kViewBatch, m - j0);
#pragma unroll 2
        for (int v = 0; v < nv; ++v) {
          const double2* q = rec + v * RS;
          const double2 pp = q[CT + 1];
          const double p = pp.x, p2 = pp.y;
          cd W[R];
          W[0] = expi_tab(tab, dtl, p);
          if constexpr (R > 1) {
            const double2 zz = q[CT];
            const cd Bz = cmul(W[0], cd{zz.x, zz.y});
            const double phi = c1 * p;
            const double a = fma(h1, p2, 1.0);
            W[1] = cd{fma(Bz.re, a, -Bz.im * phi), fma(Bz.im, a, Bz.re * phi)};
          }
#pragma unroll
          for (int c = 0; c < CT; ++c) {
            const double2 be = q[c];
#pragma unroll
            for (int r = 0; r < R; ++r) cfma_conj(acc[r][c], W[r], cd{be.x, be.y});
          }
#pragma unroll
          for (int r = 0; r < R; ++r) {
            m0[r] = cadd(m0[r], W[r]);
            m1[r].re = fma(p, W[r].re, m1[r].re);
            m1[r].im = fma(p, W[r].im, m1[r].im);
            m2[r].re = fma(p2, W[r].re, m2[r].re);
            m2[r].im = fma(p2, W[r].im, m2[r].im);
          }
        }
      }
    }
    team_sync();
    // largest |p_j| over the team (for the status check below)
    pmax = fmax(pmax, dpp_mov<0xB1>(pmax));
    pmax = fmax(pmax, dpp_mov<0x4E>(pmax));
    pmax = fmax(pmax, dpp_mov<0x141>(pmax));
    pmax = fmax(pmax, dpp_mov<0x140>(pmax));
  } else if constexpr (APER) {
    // one view in flight: the aperture spectra already hold many registers
    ViewIn ua;
    float2 ba[CT];
    load(0, ua, ba);
    for (int j = 0; j < m; ++j) {
      const ViewIn uj = ua;
      float2 bj[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) bj[c] = ba[c];
      load(min(j + 1, m - 1), ua, ba);
      view(uj, bj);
    }
  } else {
    // three view buffers in rotation: the loads of a view are issued two
    // views before it is processed.  The prefetch index is clamped instead of
    // guarded, so that every load is unconditional and each wait can name the
    // oldest batch only (a guarded load forces waits for all loads in flight).
    ViewIn ua, ub, uc;
    float2 ba[CT], bb[CT], bc[CT];
    const int last = m - 1;
    load(0, ua, ba);
    load(min(1, last), ub, bb);
    int j = 0;
    for (; j + 3 <= m; j += 3) {
      load(j + 2, uc, bc);
      view(ua, ba);
      load(min(j + 3, last), ua, ba);
      view(ub, bb);
      load(min(j + 4, last), ub, bb);
      view(uc, bc);
    }
    if (j < m) view(ua, ba);
    if (j + 1 < m) view(ub, bb);
  }
  // padded rows get zero right-hand sides
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool live = lane + 16 * r < n;
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[r][c] = live ? acc[r][c] : cd{0.0, 0.0};
  }

  // ---- 3: regulariser (bands of lambda Gamma^H Gamma + eps I) ----
  // diagonal per row: VIEW2 lambda |w|^4 d_i^4, LAYER2 lambda (4 + [i > 0] +
  // [i < n - 1]), L2 lambda; plus eps.  It is added to the pivot in step 4.
  // LAYER2 also has -4 lambda on the first and lambda on the second
  // sub-diagonal (the same in every row): in the Toeplitz path they join the
  // moments R0_1 and R0_2, in the general path they start the Gram sums.
  double diag[R];
  {
    const double w2 = wx * wx + wy * wy;
    const double w4 = w2 * w2;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 16 * r;
      double g;
      if (P.reg == 0) {
        const double d2 = dk[r] * dk[r];
        g = P.lambda * w4 * d2 * d2;
      } else if (P.reg == 1) {
        g = P.lambda * (4.0 + (i > 0 ? 1.0 : 0.0) + (i < n - 1 ? 1.0 : 0.0));
      } else {
        g = P.lambda;
      }
      diag[r] = g + P.eps;
    }
  }

  const double sub1 = P.reg == 1 ? -4.0 * P.lambda : 0.0;
  const double sub2 = P.reg == 1 ? P.lambda : 0.0;
  if constexpr (TOEP) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int t = lane + 16 * r;
      double band = t == 1 ? sub1 : 0.0;
      band = t == 2 ? sub2 : band;
      T.m.r0[t] = make_double2(m0[r].re + band, m0[r].im);
      T.m.r1[t] = make_double2(m1[r].re, m1[r].im);
      T.m.r2[t] = make_double2(m2[r].re, m2[r].im);
    }
    team_sync();
    // Lower-triangle entry (i, k), t = i - k: M_{k,i} = R0_t + i th R1_t -
    // th^2/2 R2_t with th = 2 pi [(d_i - d_k) - (d_t - d_0)] = 2 pi (e_i - e_k -
    // e_t), and M_{i,k} = conj(M_{k,i}).  Entries above the diagonal (and in the
    // padded rows) read some other moment: finite values that no live entry
    // of L ever reads.
    static_for<0, R>([&](auto RR) {
      constexpr int r = decltype(RR)::value;
      const int i = lane + 16 * r;
      const double ei = kTwoPi * T.m.e[i];
      static_for<0, 16 * (r + 1)>([&](auto KK) {
        constexpr int k = decltype(KK)::value;
        if constexpr (k >= NF) {   // column outside the solved rows
          S.template at<r>(k) = cd{0.0, 0.0};
          return;
        }
        const int t = (i - k) & 31;
        const double2 q0 = T.m.r0[t];
        const double2 q1 = T.m.r1[t];
        const double2 q2 = T.m.r2[t];
        const double th = (ei - kTwoPi * T.m.e[k]) - kTwoPi * T.m.e[t];
        const double h2 = (0.5 * th) * th;
        const double mre = fma(-h2, q2.x, fma(-th, q1.y, q0.x));
        const double mim = fma(-h2, q2.y, fma(th, q1.x, q0.y));
        cd e = cd{mre, -mim};
        pin(e);
        S.template at<r>(k) = e;
      });
    });
    if (lane == 0 && P.status && kTwoPi * P.eta_max * pmax > 3e-4) atomicAdd(P.status, 1);
  }
  if constexpr (REGION) {
    // dense part of the finite-region view regulariser (its diagonal is the
    // one of the view regulariser, added at the pivots); padded rows untouched
    sched_fence();
    const double w2 = wx * wx + wy * wy;
    const double lw = P.lambda * w2 * w2;
    const double rx = P.region * wx, ry = P.region * wy;
    static_for<0, R>([&](auto RR) {
      constexpr int r = decltype(RR)::value;
      const int i = lane + 16 * r;
      const double ci = lw * dk[r] * dk[r];
      static_for<0, 16 * (r + 1)>([&](auto KK) {
        constexpr int k = decltype(KK)::value;
        if constexpr (k >= NF) return;
        const double dkk = P.d[k];
        const double dd = dk[r] - dkk;
        const double g = ci * dkk * dkk * (double)(sinc_pi(rx * dd) * sinc_pi(ry * dd));
        S.template at<r>(k).re += (k < i && i < n) ? g : 0.0;
      });
      sched_fence();
    });
  }

  // the right-hand sides wait in LDS while the factorisation holds the registers
  team_sync();
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) T.rhs.c[lane][r * CT + c] = make_double2(acc[r][c].re, acc[r][c].im);

  __builtin_amdgcn_s_setprio(0);
  // ---- 4: Cholesky ----
  bool bad = false;
  double invd[R];
#pragma unroll
  for (int r = 0; r < R; ++r) invd[r] = 0.0;
  static_for<0, NF>([&](auto JJ) {
    constexpr int j = decltype(JJ)::value;
    constexpr int oj = j % 16, sj = j / 16;
    // the diagonal register holds the Gram part; the regulariser's diagonal
    // joins here.  Padded rows (j >= n) take the pivot 1 and 1/L_jj = 0.
    double piv = bcast16<oj>(S.template at<sj>(j).re + diag[sj]);
    if (j >= n) piv = 1.0;
    const bool ok = piv > 0.0 && isfinite(piv);
    bad = bad || !ok;
    piv = ok ? piv : 1e-300;
    double y = __builtin_amdgcn_rsq(piv);
    y = y * fma(-0.5 * piv * y, y, 1.5);
    y = y * fma(-0.5 * piv * y, y, 1.5);
    const double yl = j < n ? y : 0.0;
    invd[sj] = lane == oj ? yl : invd[sj];
    static_for<0, R>([&](auto RR) {
      constexpr int r = decltype(RR)::value;
      if constexpr (j < 16 * (r + 1)) S.template at<r>(j) = cscale(S.template at<r>(j), y);
    });
    // trailing update M_ik -= L_ij conj(L_kj), L_kj broadcast from row k's lane
    // (where only one row of the lane takes part, columns k and k + 1 share
    // one block)
    static_for<j + 1, NF>([&](auto KK) {
      constexpr int k = decltype(KK)::value;
      constexpr int r1 = R - 1;
      constexpr int k1 = j + 1 > 16 * (R - 1) ? j + 1 : 16 * (R - 1);   // first single-row column
      const cd Lk = S.template at<k / 16>(j);
      if constexpr (R > 1 && k < 16)
        dpp_cfms_aconjb<k % 16>(S.template at<0>(k), S.template at<0>(j), S.template at<1>(k), S.template at<1>(j), Lk);
      else if constexpr (((k - k1) & 1) == 0 && k + 1 < NF)
        dpp_cfms_aconjb2<k % 16, (k + 1) % 16>(S.template at<r1>(k), S.template at<r1>(j), Lk,
                                               S.template at<r1>(k + 1), S.template at<r1>(j), Lk);
      else if constexpr (((k - k1) & 1) == 0)
        dpp_cfms_aconjb<k % 16>(S.template at<r1>(k), S.template at<r1>(j), Lk);
    });
    sched_fence();
  });
  if (bad && lane == 0 && P.status) atomicAdd(P.status, 1);

  // keep the strictly lower part of the live rows.  The padded rows are
  // cleared: with their pivots forced to 1, their block is no Cholesky factor
  // and may even overflow, so it must not meet the (zero) padded unknowns in
  // the substitutions.  A select, not a product, so that Inf and NaN vanish.
  static_for<0, R>([&](auto RR) {
    constexpr int r = decltype(RR)::value;
    const int i = lane + 16 * r;
    const bool live = i < n;
    static_for<0, 16 * (r + 1)>([&](auto KK) {
      constexpr int k = decltype(KK)::value;
      const cd v = S.template at<r>(k);
      S.template at<r>(k) = (k < i) & live ? v : cd{0.0, 0.0};
    });
  });

#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const double2 v = T.rhs.c[lane][r * CT + c];
      acc[r][c] = cd{v.x, v.y};
    }

  // ---- 5a: forward substitution L y = c ----
  // acc_j keeps c_j minus the contributions of y_0..y_{j-1}; y_j = acc_j / L_jj
  // is broadcast from its lane and every row i > j subtracts L_ij y_j (the
  // zeroed diagonal and upper entries leave the other rows unchanged).
  static_for<0, NF>([&](auto JJ) {
    constexpr int j = decltype(JJ)::value;
    constexpr int oj = j % 16, sj = j / 16;
    // y_j = acc_j / L_jj in its lane, broadcast into the updates (row j's
    // own sums do not change at this step: its coefficient L_jj was zeroed)
    cd yv[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) yv[c] = cscale(acc[sj][c], invd[sj]);
    if constexpr (R > 1 && j < 16) {
#pragma unroll
      for (int c = 0; c < CT; ++c)
        dpp_cfms<oj>(acc[0][c], S.template at<0>(j), acc[1][c], S.template at<1>(j), yv[c]);
    } else {
      // one row of the lane takes part: two channels per block
      constexpr int r = sj;
#pragma unroll
      for (int c = 0; c + 1 < CT; c += 2)
        dpp_cfms2<oj, oj>(acc[r][c], S.template at<r>(j), yv[c], acc[r][c + 1], S.template at<r>(j), yv[c + 1]);
      if constexpr (CT & 1) dpp_cfms<oj>(acc[r][CT - 1], S.template at<r>(j), yv[CT - 1]);
    }
    sched_fence();
  });
  // y = acc / diag(L)
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[r][c] = cscale(acc[r][c], invd[r]);

  // ---- 5b: backward substitution L^H x = y ----
  if constexpr (R == 1) {
    // row layout: x_i = (y_i - sum_{k>i} conj(L_ki) x_k) / L_ii, the sum over
    // the team's lanes by a DPP reduction
    static_for<0, NF>([&](auto II) {
      constexpr int i = NF - 1 - decltype(II)::value;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        cd s = cd{0.0, 0.0};
        cfma_conj(s, S.L0[i], acc[0][c]);
        s.re = allreduce16(s.re);
        s.im = allreduce16(s.im);
        const cd xi = cscale(csub(acc[0][c], s), invd[0]);
        acc[0][c] = csel(lane == i, xi, acc[0][c]);
      }
      sched_fence();
    });
  } else {
    // column layout: x_i = acc_i / L_ii is broadcast and every row k < i
    // subtracts conj(L_ik) x_i; rows k >= i see zero coefficients
    team_transpose<R>(S, T.tr, lane);
    static_for<0, NF>([&](auto II) {
      constexpr int i = NF - 1 - decltype(II)::value;
      constexpr int oi = i % 16, si = i / 16;
      // x_i = acc_i / L_ii in its lane, broadcast into the updates (row i's own
      // sums do not change: its coefficient is zero)
      cd xv[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) xv[c] = cscale(acc[si][c], invd[si]);
      if constexpr (i < 16) {
        // only the first row of the lane takes part: two channels per block
#pragma unroll
        for (int c = 0; c + 1 < CT; c += 2)
          dpp_cfms_conja2<oi, oi>(acc[0][c], S.L0[i], xv[c], acc[0][c + 1], S.L0[i], xv[c + 1]);
        if constexpr (CT & 1) dpp_cfms_conja<oi>(acc[0][CT - 1], S.L0[i], xv[CT - 1]);
      } else {
#pragma unroll
        for (int c = 0; c < CT; ++c) dpp_cfms_conja<oi>(acc[0][c], S.L1[i - 16], acc[1][c], S.L1[i], xv[c]);
      }
      sched_fence();
    });
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < CT; ++c) acc[r][c] = cscale(acc[r][c], invd[r]);
  }

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
