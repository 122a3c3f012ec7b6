// Batched construction kernels (see batch.hip for the plan and the launch
// modes) and the per-channel-class launch entry points.
#pragma once
#include "construct_team.h"

namespace fdl {

struct Tile {   // 16 bins of one light field (one bin per team)
  int lf;
  int f0;
};

// Opaque copy of the lane index: keeps the lane-dependent predicates of the
// unrolled solver inside loops instead of letting them be hoisted (and held
// in registers) across iterations.  Emits no instruction.
__device__ __forceinline__ int opaque_lane(int lane) {
  asm volatile("" : "+v"(lane));
  return lane;
}

// Flat modes: one block per tile.  R is the row-slot class of the launch and
// NF the solved-row class (NF = 32 also solves every n <= 32, so a single
// launch can cover every light field).
template <int CT, bool TOEP, int R, int NF>
__global__ __launch_bounds__(256, TOEP && R > 1 ? 2 : 1) void k_batched_flat(const ConstructParams* __restrict__ lfs,
                                                      const Tile* __restrict__ tiles) {
  __shared__ TeamLds<R> s_team[16];
  __shared__ double2 s_tab[kPhaseTab];
  fill_phase_table(s_tab);
  __syncthreads();
  const int lane = threadIdx.x & 15;
  const int team = threadIdx.x >> 4;
  // tiles are sorted by light-field cost, so they are NOT remapped to
  // contiguous per-XCD ranges: the dispatcher's round-robin spreads every
  // light field over all XCDs and keeps their loads balanced
  const int t = blockIdx.x;
  const int lf = __builtin_amdgcn_readfirstlane(tiles[t].lf);
  const int f0 = __builtin_amdgcn_readfirstlane(tiles[t].f0);
  const ConstructParams* P = lfs + lf;
  const int f = f0 + team;
  if (f >= P->F) return;
  team_solve<R, CT, TOEP, false, false, false, NF>(*P, s_team[team], s_tab, f, lane);
}

// Persistent mode: a grid sized to the machine pulls `chunk` tiles at a time
// from an atomic queue; one launch per row-slot class R.  The last block out
// resets the queue, so replays need no memset.
template <int CT, bool TOEP, int R>
__global__ __launch_bounds__(256, TOEP && R > 1 ? 2 : 1) void k_batched_persistent(const ConstructParams* __restrict__ lfs,
                                                            const Tile* __restrict__ tiles, int ntiles, int chunk,
                                                            int* counters) {
  __shared__ TeamLds<R> s_team[16];
  __shared__ double2 s_tab[kPhaseTab];
  __shared__ int s_tile;
  fill_phase_table(s_tab);
  const int lane = threadIdx.x & 15;
  const int team = threadIdx.x >> 4;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(&counters[0], chunk);
    __syncthreads();
    const int t0 = __builtin_amdgcn_readfirstlane(s_tile);
    __syncthreads();
    if (t0 >= ntiles) break;
    const int t1 = min(t0 + chunk, ntiles);
    for (int t = t0; t < t1; ++t) {
      const int lf = __builtin_amdgcn_readfirstlane(tiles[t].lf);
      const int f0 = __builtin_amdgcn_readfirstlane(tiles[t].f0);
      const ConstructParams* P = lfs + lf;
      const int f = f0 + team;
      if (f < P->F) team_solve<R, CT, TOEP>(*P, s_team[team], s_tab, f, opaque_lane(lane));
    }
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const int done = atomicAdd(&counters[1], 1);
    if (done == (int)gridDim.x - 1) {
      atomicExch(&counters[0], 0);
      atomicExch(&counters[1], 0);
    }
  }
}

}  // namespace fdl

namespace fdl {

// One launch over a slice of the tile table.
struct BatchArgs {
  const ConstructParams* params;
  const Tile* tiles;
  int ntiles, grid, chunk;
  int* counters;        // persistent mode: 2 ints in device memory
  int toep, r, nf;      // disparity class, row slots and solved rows of the launch
  bool persistent;
};

template <int CT, bool TOEP>
hipError_t batch_launch_t(const BatchArgs& a, hipStream_t s) {
  if (a.persistent) {
    if (a.r == 1)
      hipLaunchKernelGGL((k_batched_persistent<CT, TOEP, 1>), dim3(a.grid), dim3(256), 0, s, a.params, a.tiles,
                         a.ntiles, a.chunk, a.counters);
    else
      hipLaunchKernelGGL((k_batched_persistent<CT, TOEP, 2>), dim3(a.grid), dim3(256), 0, s, a.params, a.tiles,
                         a.ntiles, a.chunk, a.counters);
    return hipGetLastError();
  }
  switch (a.nf) {
#define FDL_FLAT(NFV, RV) \
  case NFV: hipLaunchKernelGGL((k_batched_flat<CT, TOEP, RV, NFV>), dim3(a.grid), dim3(256), 0, s, a.params, a.tiles); break;
    FDL_FLAT(8, 1)
    FDL_FLAT(16, 1)
    FDL_FLAT(20, 2)
    FDL_FLAT(24, 2)
    FDL_FLAT(28, 2)
    FDL_FLAT(30, 2)
    FDL_FLAT(32, 2)
#undef FDL_FLAT
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int CT>
hipError_t batch_launch_ct(const BatchArgs& a, hipStream_t s) {
  return a.toep ? batch_launch_t<CT, true>(a, s) : batch_launch_t<CT, false>(a, s);
}

hipError_t batch_launch_c1(const BatchArgs& a, hipStream_t s);
hipError_t batch_launch_c3(const BatchArgs& a, hipStream_t s);
hipError_t batch_launch_c4(const BatchArgs& a, hipStream_t s);

}  // namespace fdl
