// Layer construction with the second-order view regulariser over a finite
// camera-plane region (Eq. GTG): the team solver plus a dense regulariser
// pass, on the Toeplitz and the general Gram paths.
#include "construct_team.h"

// ---- finite-region view regulariser (Eq. GTG): dense regulariser matrix ----
namespace fdl {

template <int R, int CT, bool TOEP>
__global__ __launch_bounds__(256, 2) void k_construct_region(ConstructParams P) {
  __shared__ TeamLds<R> s_team[16];
  __shared__ double2 s_tab[kPhaseTab];
  fill_phase_table(s_tab);
  __syncthreads();
  const int lane = threadIdx.x & 15;
  const int team = threadIdx.x >> 4;
  const int f = xcd_remap(blockIdx.x, gridDim.x) * 16 + team;
  if (f >= P.F) return;
  team_solve<R, CT, TOEP, false, false, true>(P, s_team[team], s_tab, f, lane);
}

template <int R, int CT>
static hipError_t go_region(const ConstructParams& P, hipStream_t s) {
  const int blocks = (P.F + 15) / 16;
  if (P.toeplitz)
    hipLaunchKernelGGL((k_construct_region<R, CT, true>), dim3(blocks), dim3(256), 0, s, P);
  else
    hipLaunchKernelGGL((k_construct_region<R, CT, false>), dim3(blocks), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_construct_region(const ConstructParams& P, hipStream_t s) {
  if (P.n <= 16) {
    if (P.C == 1) return go_region<1, 1>(P, s);
    if (P.C <= 3) return go_region<1, 3>(P, s);
    return go_region<1, 4>(P, s);
  }
  if (P.C == 1) return go_region<2, 1>(P, s);
  if (P.C <= 3) return go_region<2, 3>(P, s);
  return go_region<2, 4>(P, s);
}

}  // namespace fdl
