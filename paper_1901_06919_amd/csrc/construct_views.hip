// Construction from input views that carry their own apertures (focal
// stacks, wide-aperture or mixed inputs; Eq. AMatGeneral): the general
// (non-Toeplitz) team solver with A_jk scaled by psi_hat_j((s_j - d_k) w).
#include "construct_team.h"

namespace fdl {

template <int R, int CT>
__global__ __launch_bounds__(256) void k_construct_views(ConstructParams P) {
  __shared__ TeamLds<R> s_team[16];
  __shared__ double2 s_tab[kPhaseTab];
  fill_phase_table(s_tab);
  __syncthreads();
  const int lane = threadIdx.x & 15;
  const int team = threadIdx.x >> 4;
  const int f = xcd_remap(blockIdx.x, gridDim.x) * 16 + team;
  if (f >= P.F) return;
  team_solve<R, CT, false, true>(P, s_team[team], s_tab, f, lane);
}

template <int R, int CT>
static hipError_t go(const ConstructParams& P, hipStream_t s) {
  const int blocks = (P.F + 15) / 16;
  hipLaunchKernelGGL((k_construct_views<R, CT>), dim3(blocks), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_construct_views(const ConstructParams& P, hipStream_t s) {
  if (P.n <= 16) {
    if (P.C == 1) return go<1, 1>(P, s);
    if (P.C <= 3) return go<1, 3>(P, s);
    return go<1, 4>(P, s);
  }
  if (P.C == 1) return go<2, 1>(P, s);
  if (P.C <= 3) return go<2, 3>(P, s);
  return go<2, 4>(P, s);
}

}  // namespace fdl
