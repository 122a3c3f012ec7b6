// Layer construction for the relaxed model (Sec. VIII-B): the general-Gram
// team solver with a free shift pair per input view and layer.
#include "construct_team.h"

// ---- relaxed model (Sec. VIII-B): a free shift pair P_jk per view and layer ----
// A_jk = exp(2 pi i <P_jk, w>), then the same regularised solve; the general
// Gram path (the entries no longer depend on j - k only).
namespace fdl {

template <int R, int CT>
__global__ __launch_bounds__(256, 2) void k_construct_relaxed(ConstructParams P) {
  __shared__ TeamLds<R> s_team[16];
  __shared__ double2 s_tab[kPhaseTab];
  fill_phase_table(s_tab);
  __syncthreads();
  const int lane = threadIdx.x & 15;
  const int team = threadIdx.x >> 4;
  const int f = xcd_remap(blockIdx.x, gridDim.x) * 16 + team;
  if (f >= P.F) return;
  team_solve<R, CT, false, false, true>(P, s_team[team], s_tab, f, lane);
}

template <int R, int CT>
static hipError_t go_relaxed(const ConstructParams& P, hipStream_t s) {
  const int blocks = (P.F + 15) / 16;
  hipLaunchKernelGGL((k_construct_relaxed<R, CT>), dim3(blocks), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_construct_relaxed(const ConstructParams& P, hipStream_t s) {
  if (P.n <= 16) {
    if (P.C == 1) return go_relaxed<1, 1>(P, s);
    if (P.C <= 3) return go_relaxed<1, 3>(P, s);
    return go_relaxed<1, 4>(P, s);
  }
  if (P.C == 1) return go_relaxed<2, 1>(P, s);
  if (P.C <= 3) return go_relaxed<2, 3>(P, s);
  return go_relaxed<2, 4>(P, s);
}

}  // namespace fdl
