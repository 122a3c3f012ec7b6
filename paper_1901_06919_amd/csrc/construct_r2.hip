// Plain construction kernels, one 16-lane team per half-spectrum bin,
// instantiations for n <= 32 (R = 2 row slots per lane).
#include "construct_team.h"

namespace fdl {

template <int R, int CT, bool TOEP, int NF>
__global__ __launch_bounds__(256, TOEP ? 2 : 1) void k_construct(ConstructParams P) {
  __shared__ TeamLds<R> s_team[16];
  __shared__ double2 s_tab[kPhaseTab];
  fill_phase_table(s_tab);
  __syncthreads();
  const int lane = threadIdx.x & 15;
  const int team = threadIdx.x >> 4;
  const int f = P.f_begin + xcd_remap(blockIdx.x, gridDim.x) * 16 + team;
  if (f >= P.f_stop) return;
  team_solve<R, CT, TOEP, false, false, false, NF>(P, s_team[team], s_tab, f, lane);
}

// Systems of up to 30 unknowns skip the last two (padded) rows and columns of
// the factorisation and substitutions.
template <int CT, bool TOEP>
static hipError_t go(const ConstructParams& P, hipStream_t s) {
  const int blocks = (P.f_stop - P.f_begin + 15) / 16;
  if (P.n <= 30)
    hipLaunchKernelGGL((k_construct<2, CT, TOEP, 30>), dim3(blocks), dim3(256), 0, s, P);
  else
    hipLaunchKernelGGL((k_construct<2, CT, TOEP, 32>), dim3(blocks), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_construct_r2(const ConstructParams& P, hipStream_t s) {
  const bool t = P.toeplitz != 0;
  if (P.C == 1) return t ? go<1, true>(P, s) : go<1, false>(P, s);
  if (P.C <= 3) return t ? go<3, true>(P, s) : go<3, false>(P, s);
  return t ? go<4, true>(P, s) : go<4, false>(P, s);
}

}  // namespace fdl
