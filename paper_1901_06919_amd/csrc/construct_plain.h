// Plain construction kernels: one 16-lane team per half-spectrum bin, one
// instantiation per (channels, disparity class, solved-row class).
#pragma once
#include "construct_team.h"

namespace fdl {

// NF rows are factorised; R = 1 row slot per lane holds NF <= 16, R = 2 the rest.
template <int CT, bool TOEP, int NF>
__global__ __launch_bounds__(256, TOEP && NF > 16 ? 2 : 1) void k_construct(ConstructParams P) {
  constexpr int R = NF > 16 ? 2 : 1;
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

template <int CT, bool TOEP, int NF>
hipError_t launch_plain(const ConstructParams& P, hipStream_t s) {
  const int blocks = (P.f_stop - P.f_begin + 15) / 16;
  hipLaunchKernelGGL((k_construct<CT, TOEP, NF>), dim3(blocks), dim3(256), 0, s, P);
  return hipGetLastError();
}

template <int CT, bool TOEP>
hipError_t launch_plain_rows(const ConstructParams& P, hipStream_t s) {
  switch (solve_rows(P.n)) {
    case 8: return launch_plain<CT, TOEP, 8>(P, s);
    case 16: return launch_plain<CT, TOEP, 16>(P, s);
    case 20: return launch_plain<CT, TOEP, 20>(P, s);
    case 24: return launch_plain<CT, TOEP, 24>(P, s);
    case 28: return launch_plain<CT, TOEP, 28>(P, s);
    case 30: return launch_plain<CT, TOEP, 30>(P, s);
    default: return launch_plain<CT, TOEP, 32>(P, s);
  }
}

template <int CT>
hipError_t launch_plain_ct(const ConstructParams& P, hipStream_t s) {
  return P.toeplitz ? launch_plain_rows<CT, true>(P, s) : launch_plain_rows<CT, false>(P, s);
}

}  // namespace fdl
