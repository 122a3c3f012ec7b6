// Device helpers shared by the FDL kernels: FP64 complex arithmetic, an
// FP64 sin/cos of 2*pi*r, 16-lane team communication through DPP, and the
// half-spectrum frequency mapping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace fdl {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;

struct cd {
  double re, im;
};

// Compile-time loop: fn(std::integral_constant<int, i>) for i = I .. N-1.
template <int I, int N, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (I < N) {
    fn(std::integral_constant<int, I>{});
    static_for<I + 1, N>(fn);
  }
}

__device__ __forceinline__ cd cmake(double r, double i) { return cd{r, i}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cmul(cd a, cd b) {
  return cd{fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
// conj(a) * b
__device__ __forceinline__ cd cmulc(cd a, cd b) {
  return cd{fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -a.im * b.re)};
}
__device__ __forceinline__ cd cscale(cd a, double s) { return cd{a.re * s, a.im * s}; }
// c ? a : b per component: a select of the whole struct on a lane-varying
// condition can be lowered through scratch memory instead of two v_cndmask
__device__ __forceinline__ cd csel(bool c, cd a, cd b) { return cd{c ? a.re : b.re, c ? a.im : b.im}; }
// acc += conj(a) * b
__device__ __forceinline__ void cfma_conj(cd& acc, cd a, cd b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
// acc -= a * conj(b)
__device__ __forceinline__ void cfms_aconjb(cd& acc, cd a, cd b) {
  acc.re = fma(-a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(-a.im, b.re, acc.im);
  acc.im = fma(a.re, b.im, acc.im);
}
// acc += a * b
__device__ __forceinline__ void cfma(cd& acc, cd a, cd b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}

// sin(2 pi r), cos(2 pi r) to about 1 ulp of double for any |r| < 2^40.
// Reduction: r - rint(r) in [-1/2, 1/2] (exact), then the nearest quarter
// turn q/4 is removed (exact), leaving |x| = 2 pi |f| <= pi/4 where the
// Taylor series of sin (through x^15) and cos (through x^16) are summed by
// Horner's rule; truncation error < 5e-17.  The quarter turn is restored by
// the identities sin(x + q pi/2), cos(x + q pi/2).
__device__ __forceinline__ void sincos2pi(double r, double& s, double& c) {
  r = r - rint(r);
  const double q = rint(4.0 * r);
  const double f = fma(-0.25, q, r);
  const double x = kTwoPi * f;
  const double x2 = x * x;
  // sin(x) = x (1 - x^2/3! + x^4/5! - ... - x^14/15!)
  double ps = -1.0 / 1307674368000.0;          // -1/15!
  ps = fma(ps, x2, 1.0 / 6227020800.0);        // +1/13!
  ps = fma(ps, x2, -1.0 / 39916800.0);         // -1/11!
  ps = fma(ps, x2, 1.0 / 362880.0);            // +1/9!
  ps = fma(ps, x2, -1.0 / 5040.0);             // -1/7!
  ps = fma(ps, x2, 1.0 / 120.0);               // +1/5!
  ps = fma(ps, x2, -1.0 / 6.0);                // -1/3!
  const double sx = fma(x * x2, ps, x);
  // cos(x) = 1 - x^2/2! + x^4/4! - ... + x^16/16!
  double pc = 1.0 / 20922789888000.0;          // +1/16!
  pc = fma(pc, x2, -1.0 / 87178291200.0);      // -1/14!
  pc = fma(pc, x2, 1.0 / 479001600.0);         // +1/12!
  pc = fma(pc, x2, -1.0 / 3628800.0);          // -1/10!
  pc = fma(pc, x2, 1.0 / 40320.0);             // +1/8!
  pc = fma(pc, x2, -1.0 / 720.0);              // -1/6!
  pc = fma(pc, x2, 1.0 / 24.0);                // +1/4!
  pc = fma(pc, x2, -0.5);                      // -1/2!
  const double cx = fma(x2, pc, 1.0);
  const int qi = ((int)q) & 3;
  const double s1 = (qi & 1) ? cx : sx;
  const double c1 = (qi & 1) ? sx : cx;
  s = (qi & 2) ? -s1 : s1;
  c = ((qi + 1) & 2) ? -c1 : c1;
}

__device__ __forceinline__ cd expi2pi(double r) {
  cd z;
  sincos2pi(r, z.im, z.re);
  return z;
}

// ---- raw buffer loads ----------------------------------------------------------
// A buffer descriptor holds a uniform base address (in SGPRs); a load adds a
// 32-bit per-lane offset and a uniform 32-bit offset in hardware, so per-lane
// 64-bit address arithmetic disappears from the VALU.  The descriptor allows
// offsets below 2 GiB (num_records) with no stride; word 3 selects the 32-bit
// data format that raw (untyped) accesses on CDNA expect.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ float2 buf_load_f2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
}

// ---- 16-lane team communication (one DPP row = one team) -------------------

// Value of `v` in lane SRC of this lane's 16-lane row (row_newbcast).  The
// DPP move has no "old" operand (bound_ctrl), so the compiler needs no copy
// of the source into the destination first; every source lane of a row is
// active wherever these are used, so the result is the same.
template <int SRC>
__device__ __forceinline__ double bcast16(double v) {
  long long x = __double_as_longlong(v);
  x = __builtin_amdgcn_mov_dpp(x, 0x150 + SRC, 0xF, 0xF, true);
  return __longlong_as_double(x);
}
template <int SRC>
__device__ __forceinline__ cd bcast16(cd v) {
  return cd{bcast16<SRC>(v.re), bcast16<SRC>(v.im)};
}

// ---- fused broadcast multiply-adds: v_fmac_f64 with DPP row_newbcast -------
// LLVM does not fold a DPP broadcast into an FP64 multiply-add, so these emit
// v_fmac_f64_dpp directly: the first source is read from lane SRC of the
// lane's 16-lane row, which saves the separate broadcast moves.  A DPP
// instruction needs two wait states after the write of ANY VGPR it reads --
// the broadcast source, the other source and the accumulator alike -- and the
// compiler inserts none for instructions inside inline assembly.  So every
// block starts with s_nop 1 (for the compiler's writes just before it), and
// inside a block the multiply-adds into one accumulator register are at least
// three instructions apart: the two-accumulator blocks interleave their four
// chains, the one-accumulator blocks put an s_nop 0 between the two halves.
// Per accumulator register the operations keep the order of the plain complex
// helpers above (bit-identical results).  `x` below is the broadcast operand.

// acc -= a * conj(x), x from lane SRC
template <int SRC>
__device__ __forceinline__ void dpp_cfms_aconjb(cd& acc, cd a, cd x) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, -%2, %4 row_newbcast:%c6\n\t"
      "v_fmac_f64_dpp %1, -%2, %5 row_newbcast:%c6\n\t"
      "s_nop 0\n\t"
      "v_fmac_f64_dpp %0, -%3, %5 row_newbcast:%c6\n\t"
      "v_fmac_f64_dpp %1, %3, %4 row_newbcast:%c6"
      : "+v"(acc.re), "+v"(acc.im)
      : "v"(x.re), "v"(x.im), "v"(a.re), "v"(a.im), "n"(SRC));
}
// two independent updates in one block: acc0 with (a0, x0 from lane S0)
// and acc1 with (a1, x1 from lane S1)
template <int S0, int S1>
__device__ __forceinline__ void dpp_cfms_aconjb2(cd& acc0, cd a0, cd x0, cd& acc1, cd a1, cd x1) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, -%4, %8 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %1, -%4, %9 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %2, -%6, %10 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %3, -%6, %11 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %0, -%5, %9 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %1, %5, %8 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %2, -%7, %11 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %3, %7, %10 row_newbcast:%c13"
      : "+v"(acc0.re), "+v"(acc0.im), "+v"(acc1.re), "+v"(acc1.im)
      : "v"(x0.re), "v"(x0.im), "v"(x1.re), "v"(x1.im), "v"(a0.re), "v"(a0.im), "v"(a1.re), "v"(a1.im),
        "n"(S0), "n"(S1));
}
// acc and acc1 with the same broadcast x
template <int SRC>
__device__ __forceinline__ void dpp_cfms_aconjb(cd& acc, cd a, cd& acc1, cd a1, cd x) {
  dpp_cfms_aconjb2<SRC, SRC>(acc, a, x, acc1, a1, x);
}

// acc -= l * x, x from lane SRC
template <int SRC>
__device__ __forceinline__ void dpp_cfms(cd& acc, cd l, cd x) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, -%2, %4 row_newbcast:%c6\n\t"
      "v_fmac_f64_dpp %1, -%3, %4 row_newbcast:%c6\n\t"
      "s_nop 0\n\t"
      "v_fmac_f64_dpp %0, %3, %5 row_newbcast:%c6\n\t"
      "v_fmac_f64_dpp %1, -%2, %5 row_newbcast:%c6"
      : "+v"(acc.re), "+v"(acc.im)
      : "v"(x.re), "v"(x.im), "v"(l.re), "v"(l.im), "n"(SRC));
}
// two independent updates in one block: acc0 with (l0, x0 from lane S0)
// and acc1 with (l1, x1 from lane S1)
template <int S0, int S1>
__device__ __forceinline__ void dpp_cfms2(cd& acc0, cd l0, cd x0, cd& acc1, cd l1, cd x1) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, -%4, %8 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %1, -%5, %8 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %2, -%6, %10 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %3, -%7, %10 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %0, %5, %9 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %1, -%4, %9 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %2, %7, %11 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %3, -%6, %11 row_newbcast:%c13"
      : "+v"(acc0.re), "+v"(acc0.im), "+v"(acc1.re), "+v"(acc1.im)
      : "v"(x0.re), "v"(x0.im), "v"(x1.re), "v"(x1.im), "v"(l0.re), "v"(l0.im), "v"(l1.re), "v"(l1.im),
        "n"(S0), "n"(S1));
}
// acc and acc1 with the same broadcast x
template <int SRC>
__device__ __forceinline__ void dpp_cfms(cd& acc, cd l, cd& acc1, cd l1, cd x) {
  dpp_cfms2<SRC, SRC>(acc, l, x, acc1, l1, x);
}

// acc -= conj(a) * x, x from lane SRC
template <int SRC>
__device__ __forceinline__ void dpp_cfms_conja(cd& acc, cd a, cd x) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, -%2, %4 row_newbcast:%c6\n\t"
      "v_fmac_f64_dpp %1, -%3, %4 row_newbcast:%c6\n\t"
      "s_nop 0\n\t"
      "v_fmac_f64_dpp %0, -%3, %5 row_newbcast:%c6\n\t"
      "v_fmac_f64_dpp %1, %2, %5 row_newbcast:%c6"
      : "+v"(acc.re), "+v"(acc.im)
      : "v"(x.re), "v"(x.im), "v"(a.re), "v"(a.im), "n"(SRC));
}
// two independent updates in one block: acc0 with (a0, x0 from lane S0)
// and acc1 with (a1, x1 from lane S1)
template <int S0, int S1>
__device__ __forceinline__ void dpp_cfms_conja2(cd& acc0, cd a0, cd x0, cd& acc1, cd a1, cd x1) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, -%4, %8 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %1, -%5, %8 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %2, -%6, %10 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %3, -%7, %10 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %0, -%5, %9 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %1, %4, %9 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %2, -%7, %11 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %3, %6, %11 row_newbcast:%c13"
      : "+v"(acc0.re), "+v"(acc0.im), "+v"(acc1.re), "+v"(acc1.im)
      : "v"(x0.re), "v"(x0.im), "v"(x1.re), "v"(x1.im), "v"(a0.re), "v"(a0.im), "v"(a1.re), "v"(a1.im),
        "n"(S0), "n"(S1));
}
// acc and acc1 with the same broadcast x
template <int SRC>
__device__ __forceinline__ void dpp_cfms_conja(cd& acc, cd a, cd& acc1, cd a1, cd x) {
  dpp_cfms_conja2<SRC, SRC>(acc, a, x, acc1, a1, x);
}

// acc += conj(a) * x, x from lane SRC
template <int SRC>
__device__ __forceinline__ void dpp_cfma_conj(cd& acc, cd a, cd x) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %2, %4 row_newbcast:%c6\n\t"
      "v_fmac_f64_dpp %1, %3, %4 row_newbcast:%c6\n\t"
      "s_nop 0\n\t"
      "v_fmac_f64_dpp %0, %3, %5 row_newbcast:%c6\n\t"
      "v_fmac_f64_dpp %1, -%2, %5 row_newbcast:%c6"
      : "+v"(acc.re), "+v"(acc.im)
      : "v"(x.re), "v"(x.im), "v"(a.re), "v"(a.im), "n"(SRC));
}
// two independent updates in one block: acc0 with (a0, x0 from lane S0)
// and acc1 with (a1, x1 from lane S1)
template <int S0, int S1>
__device__ __forceinline__ void dpp_cfma_conj2(cd& acc0, cd a0, cd x0, cd& acc1, cd a1, cd x1) {
  asm("s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %4, %8 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %1, %5, %8 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %2, %6, %10 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %3, %7, %10 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %0, %5, %9 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %1, -%4, %9 row_newbcast:%c12\n\t"
      "v_fmac_f64_dpp %2, %7, %11 row_newbcast:%c13\n\t"
      "v_fmac_f64_dpp %3, -%6, %11 row_newbcast:%c13"
      : "+v"(acc0.re), "+v"(acc0.im), "+v"(acc1.re), "+v"(acc1.im)
      : "v"(x0.re), "v"(x0.im), "v"(x1.re), "v"(x1.im), "v"(a0.re), "v"(a0.im), "v"(a1.re), "v"(a1.im),
        "n"(S0), "n"(S1));
}
// acc and acc1 with the same broadcast x
template <int SRC>
__device__ __forceinline__ void dpp_cfma_conj(cd& acc, cd a, cd& acc1, cd a1, cd x) {
  dpp_cfma_conj2<SRC, SRC>(acc, a, x, acc1, a1, x);
}

// Sum of `v` over the 16 lanes of the row, returned to every lane of the row.
// Pair swap, quad swap, half-row mirror, row mirror: every lane adds the same
// operands (in commuted order), so all 16 lanes hold bit-identical sums.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  long long x = __double_as_longlong(v);
  x = __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true);
  return __longlong_as_double(x);
}
__device__ __forceinline__ double allreduce16(double v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  return v;
}

// ---- frequency grid ---------------------------------------------------------

// w_x = kx / W, w_y = ky / H folded to [-1/2, 1/2) (numpy fftfreq / rfftfreq).
__device__ __forceinline__ void bin_freq(int f, int Wh, int H, int W, double& wx, double& wy) {
  const int ky = f / Wh;
  const int kx = f - ky * Wh;
  const int kys = (ky < (H + 1) / 2) ? ky : ky - H;
  wx = (double)kx / (double)W;
  wy = (double)kys / (double)H;
}

// Spread consecutive block indices over the 8 XCDs so that each XCD works on
// a contiguous range of bins (its own L2), instead of the round-robin
// interleave of the hardware dispatcher.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int per = (nblocks + kXcd - 1) / kXcd;
  const int xcd = bid % kXcd;
  const int idx = bid / kXcd;
  const int full = nblocks % kXcd == 0 ? kXcd : nblocks % kXcd;   // XCDs holding `per` blocks
  // blocks of XCDs < full get `per`, the rest `per - 1`
  const int base = xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1);
  return base + idx;
}

}  // namespace fdl
