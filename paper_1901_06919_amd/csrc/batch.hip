// Batched construction of many uneven light fields in one persistent launch
// (same mathematics as the plain kernels, Sec. V-A).
//
// A plan holds, in device memory, one ConstructParams per light field and a
// tile table (light field, first bin), ordered largest-work-first; the
// 16 teams of a block solve the tile's 16 bins with the same team solver as
// the plain kernels.  Launch modes: flat (one block per tile, one launch per
// channel/disparity/solved-row class), flat single (every light field through
// the n <= 32 solver: one launch per channel/disparity class), persistent
// (a machine-sized grid pulling tiles from an atomic queue, one launch per
// row-slot class; the last block resets the queue so replays need no memset) and
// persistent single (the queue over every light field of a channel/disparity
// class through the n <= 32 solver: one launch when all share the class).  The
// autotuner times the candidates on the plan's own data and keeps the
// fastest.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/fdl.h"
#include "batch_kernels.h"


struct BatchLaunch {            // one launch over a group of tiles
  int ct, toep, r, nf;          // row slots (1: n <= 16, 2: n <= 32) and solved rows of the launch
  int tile_off, ntiles;         // slice of the device tile table
  int grid;
  int* counters;                // 2 ints in device memory (persistent mode)
};

struct fdl_batch_plan {
  int B = 0;
  int mode = 0;                 // 0 flat per solved-row class, 1 persistent, 2 flat single, 3 persistent single
  int chunk = 1;                // tiles claimed per queue access (persistent)
  int grid_per_cu = 2;          // resident blocks per CU (persistent)
  int64_t total_bins = 0;
  std::vector<fdl::ConstructParams> host_params;
  fdl::ConstructParams* d_params = nullptr;
  fdl::Tile* d_tiles = nullptr;
  int* d_counters = nullptr;    // 2 per launch group
  std::vector<BatchLaunch> launches;
  size_t tiles_capacity = 0;
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? FDL_OK : (e == hipErrorOutOfMemory ? FDL_ENOMEM : FDL_EHIP); }

// compute units of the current device (queried on every plan build: no
// process-wide cache, so plans on different devices size their own grids)
int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return cus;
}

bool persistent_mode(int mode) { return mode == 1 || mode == 3; }

double lf_cost(const fdl::ConstructParams& P) {
  // rough lane instructions per bin: the view loop (phases, right-hand sides
  // and Gram sums of R row slots) plus the factorisation and substitutions of
  // the solved rows
  const int nf = fdl::solve_rows(P.n);
  const double R = nf > 16 ? 2.0 : 1.0;
  return (double)P.F * ((double)P.m * (30.0 + (4.0 * P.C + 6.0) * R) + 2.5 * nf * nf + 8.0 * nf * P.C);
}

// (Re)build the tile table and launch groups for the plan's current settings.
int build_tiles(fdl_batch_plan* p) {
  struct Group { int ct, toep, r, nf; std::vector<int> lfs; double cost = 0.0; };
  std::vector<Group> groups;
  for (int i = 0; i < p->B; ++i) {
    const auto& P = p->host_params[i];
    const int ct = P.C == 1 ? 1 : (P.C <= 3 ? 3 : 4);
    // flat mode: one launch per solved-row class; single modes: every light
    // field through the 32-row solver; persistent: the 16- and 32-row solvers
    int r, nf;
    if (p->mode == 2 || p->mode == 3) {
      r = 2; nf = 32;
    } else if (p->mode == 1) {
      r = P.n <= 16 ? 1 : 2; nf = 16 * r;
    } else {
      nf = fdl::solve_rows(P.n); r = nf > 16 ? 2 : 1;
    }
    bool found = false;
    for (auto& g : groups)
      if (g.ct == ct && g.toep == P.toeplitz && g.nf == nf) { g.lfs.push_back(i); found = true; break; }
    if (!found) groups.push_back(Group{ct, P.toeplitz, r, nf, {i}, 0.0});
  }
  // largest groups first
  for (auto& g : groups) {
    double c = 0.0;
    for (int lf : g.lfs) c += lf_cost(p->host_params[lf]);
    g.cost = c;
  }
  std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) { return a.cost > b.cost; });
  std::vector<fdl::Tile> tiles;
  p->launches.clear();
  int gi = 0;
  for (auto& g : groups) {
    std::sort(g.lfs.begin(), g.lfs.end(), [&](int a, int b) { return lf_cost(p->host_params[a]) > lf_cost(p->host_params[b]); });
    BatchLaunch L;
    L.ct = g.ct; L.toep = g.toep; L.r = g.r; L.nf = g.nf;
    L.tile_off = (int)tiles.size();
    for (int lf : g.lfs)
      for (int f0 = 0; f0 < p->host_params[lf].F; f0 += 16) tiles.push_back(fdl::Tile{lf, f0});
    L.ntiles = (int)tiles.size() - L.tile_off;
    L.grid = persistent_mode(p->mode) ? std::max(1, std::min((L.ntiles + p->chunk - 1) / p->chunk, cu_count() * p->grid_per_cu))
                          : L.ntiles;
    L.counters = p->d_counters + 2 * gi;
    p->launches.push_back(L);
    ++gi;
  }
  if (tiles.size() > p->tiles_capacity) {
    if (p->d_tiles) hipFree(p->d_tiles);
    p->d_tiles = nullptr;
    p->tiles_capacity = 0;
    if (hipMalloc(&p->d_tiles, tiles.size() * sizeof(fdl::Tile)) != hipSuccess) return FDL_ENOMEM;
    p->tiles_capacity = tiles.size();
  }
  if (hipMemcpy(p->d_tiles, tiles.data(), tiles.size() * sizeof(fdl::Tile), hipMemcpyHostToDevice) != hipSuccess)
    return FDL_EHIP;
  return FDL_OK;
}

hipError_t launch_group(const fdl_batch_plan* p, const BatchLaunch& L, hipStream_t s) {
  fdl::BatchArgs a;
  a.params = p->d_params;
  a.tiles = p->d_tiles + L.tile_off;
  a.ntiles = L.ntiles;
  a.grid = L.grid;
  a.chunk = p->chunk;
  a.counters = L.counters;
  a.toep = L.toep;
  a.r = L.r;
  a.nf = L.nf;
  a.persistent = persistent_mode(p->mode);
  if (L.ct == 1) return fdl::batch_launch_c1(a, s);
  if (L.ct == 3) return fdl::batch_launch_c3(a, s);
  return fdl::batch_launch_c4(a, s);
}

}  // namespace

// Defined in host.cpp: disparity classification shared with fdl_construct.
namespace fdl_host {
void classify(const float* d, int n, fdl::ConstructParams& P);
}

extern "C" {

int fdl_batch_plan_create(const fdl_lf_desc* descs_host, int B, int mode, fdl_batch_plan** plan_out) {
  if (!descs_host || !plan_out || B < 1 || mode < 0 || mode > 3) return FDL_EINVAL;
  *plan_out = nullptr;
  auto* p = new fdl_batch_plan();
  p->B = B;
  p->mode = mode;
  p->host_params.resize(B);
  for (int i = 0; i < B; ++i) {
    const fdl_lf_desc& D = descs_host[i];
    if (!D.view_spec || !D.u || !D.d || !D.layer_spec) { delete p; return FDL_EINVAL; }
    if (D.m < 1 || D.m > 4096 || D.n < 1 || D.n > FDL_MAX_LAYERS || D.C < 1 || D.C > FDL_MAX_CHANNELS ||
        D.H < 1 || D.W < 2 || (D.W & 1) || D.reg < 0 || D.reg > 2 || !(D.lambda >= 0.f) || !(D.eps >= 0.f)) {
      delete p;
      return FDL_ESHAPE;
    }
    fdl::ConstructParams& P = p->host_params[i];
    P.view_spec = reinterpret_cast<const float2*>(D.view_spec);
    P.u = reinterpret_cast<const float2*>(D.u);
    P.views = nullptr;
    P.layer_spec = reinterpret_cast<float2*>(D.layer_spec);
    P.status = D.status;
    P.m = D.m; P.n = D.n; P.C = D.C; P.H = D.H; P.W = D.W; P.Wh = D.W / 2 + 1; P.F = D.H * (D.W / 2 + 1);
    P.lambda = D.lambda; P.eps = D.eps; P.reg = D.reg;
    // the disparities live on the device: one blocking read at plan creation
    float dh[FDL_MAX_LAYERS];
    if (hipMemcpy(dh, D.d, sizeof(float) * D.n, hipMemcpyDeviceToHost) != hipSuccess) { delete p; return FDL_EHIP; }
    fdl_host::classify(dh, D.n, P);
    p->total_bins += P.F;
  }
  int e = hip_status(hipMalloc(&p->d_params, sizeof(fdl::ConstructParams) * B));
  if (e == FDL_OK) e = hip_status(hipMalloc(&p->d_counters, sizeof(int) * 2 * 64));
  if (e == FDL_OK) e = hip_status(hipMemcpy(p->d_params, p->host_params.data(), sizeof(fdl::ConstructParams) * B,
                                            hipMemcpyHostToDevice));
  if (e == FDL_OK) e = hip_status(hipMemset(p->d_counters, 0, sizeof(int) * 2 * 64));
  if (e == FDL_OK) e = build_tiles(p);
  if (e != FDL_OK) {
    fdl_batch_plan_destroy(p);
    return e;
  }
  *plan_out = p;
  return FDL_OK;
}

int fdl_batch_plan_execute(const fdl_batch_plan* plan, void* stream) {
  if (!plan) return FDL_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (const auto& L : plan->launches) {
    const hipError_t e = launch_group(plan, L, s);
    if (e != hipSuccess) return hip_status(e);
  }
  return FDL_OK;
}

int fdl_batch_plan_info(const fdl_batch_plan* plan, int64_t* total_bins, int32_t* grid, int32_t* launches) {
  if (!plan) return FDL_EINVAL;
  if (total_bins) *total_bins = plan->total_bins;
  if (grid) {
    int g = 0;
    for (const auto& L : plan->launches) g += L.grid;
    *grid = g;
  }
  if (launches) *launches = (int32_t)plan->launches.size();
  return FDL_OK;
}

int fdl_batch_plan_launches(const fdl_batch_plan* plan) { return plan ? (int)plan->launches.size() : 0; }

int fdl_batch_plan_destroy(fdl_batch_plan* plan) {
  if (!plan) return FDL_EINVAL;
  if (plan->d_params) hipFree(plan->d_params);
  if (plan->d_tiles) hipFree(plan->d_tiles);
  if (plan->d_counters) hipFree(plan->d_counters);
  delete plan;
  return FDL_OK;
}

// Autotuner: times every candidate setting -- flat per class, flat single
// launch, persistent queue (per class or single) with chunk in {1, 4} x
// {1, 2, 4} blocks per CU -- with
// `reps` executions each (after one warm-up) on `stream`, keeps the fastest
// and reports its time.  Synchronises the stream; not for use under capture.
int fdl_batch_plan_autotune(fdl_batch_plan* plan, int reps, void* stream, float* best_ms) {
  if (!plan || reps < 1) return FDL_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  struct Cand { int mode, chunk, grid; };
  const Cand cands[] = {{0, 1, 1}, {2, 1, 1}, {1, 1, 1}, {1, 1, 2}, {1, 1, 4}, {1, 4, 1}, {1, 4, 2}, {1, 4, 4},
                        {3, 1, 1}, {3, 1, 2}, {3, 4, 1}, {3, 4, 2}};
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return FDL_EHIP;
  float best = 1e30f;
  Cand bc{plan->mode, plan->chunk, plan->grid_per_cu};
  for (const Cand& c : cands) {
    plan->mode = c.mode;
    plan->chunk = c.chunk;
    plan->grid_per_cu = c.grid;
    if (build_tiles(plan) != FDL_OK) continue;
    if (fdl_batch_plan_execute(plan, s) != FDL_OK) continue;
    hipEventRecord(a, s);
    for (int r = 0; r < reps; ++r) fdl_batch_plan_execute(plan, s);
    hipEventRecord(b, s);
    hipEventSynchronize(b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, a, b);
    ms /= reps;
    if (std::getenv("FDL_TRACE"))
      std::fprintf(stderr, "fdl: autotune mode=%d chunk=%d grid/cu=%d: %.3f ms\n", c.mode, c.chunk, c.grid, ms);
    if (ms < best) { best = ms; bc = c; }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  plan->mode = bc.mode;
  plan->chunk = bc.chunk;
  plan->grid_per_cu = bc.grid;
  const int e = build_tiles(plan);
  if (best_ms) *best_ms = best;
  return e;
}

int fdl_batch_plan_get_tuning(const fdl_batch_plan* plan, int32_t* mode, int32_t* chunk, int32_t* grid_per_cu) {
  if (!plan) return FDL_EINVAL;
  if (mode) *mode = plan->mode;
  if (chunk) *chunk = plan->chunk;
  if (grid_per_cu) *grid_per_cu = plan->grid_per_cu;
  return FDL_OK;
}

int fdl_batch_plan_set_tuning(fdl_batch_plan* plan, int32_t mode, int32_t chunk, int32_t grid_per_cu) {
  if (!plan || mode < 0 || mode > 3 || chunk < 1 || chunk > 64 || grid_per_cu < 1 || grid_per_cu > 16)
    return FDL_EINVAL;
  plan->mode = mode;
  plan->chunk = chunk;
  plan->grid_per_cu = grid_per_cu;
  return build_tiles(plan);
}

}  // extern "C"
