// Request server of the C ABI (fdl_server_*): continuous batching of
// construct and render requests over resident light fields, admission by
// HBM footprint from one budgeted device pool (policy in serve_core.h), a
// worker thread that retires and launches work, and the same policy on a
// simulated device for host-side tests (fdl_server_simulate).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/fdl.h"
#include "serve_core.h"

namespace {

using fdl_serve::Request;

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  // linear interpolation between closest ranks (numpy's default)
  const double pos = q * (double)(v.size() - 1);
  const size_t i = (size_t)std::floor(pos);
  const size_t j = std::min(i + 1, v.size() - 1);
  return v[i] + (pos - (double)i) * (v[j] - v[i]);
}

void fill_stats(const fdl_serve::Scheduler& S, fdl_server_summary* st) {
  std::memset(st, 0, sizeof(*st));
  std::vector<double> lat[3];
  double last = 0.0, first = -1.0;
  for (const Request& r : S.requests()) {
    if (r.state != fdl_serve::kDone) continue;
    const double ms = (r.t_done - r.t_arrival) * 1e3;
    lat[0].push_back(ms);
    lat[r.kind == fdl_serve::kConstruct ? 1 : 2].push_back(ms);
    last = std::max(last, r.t_done);
    first = first < 0.0 ? r.t_arrival : std::min(first, r.t_arrival);
  }
  for (int k = 0; k < 3; ++k) {
    st->count[k] = (int64_t)lat[k].size();
    st->p50_ms[k] = percentile(lat[k], 0.50);
    st->p99_ms[k] = percentile(lat[k], 0.99);
    double s = 0.0;
    for (double x : lat[k]) s += x;
    st->mean_ms[k] = lat[k].empty() ? 0.0 : s / (double)lat[k].size();
  }
  st->submitted = S.submitted();
  st->completed = S.completed();
  st->rejected = S.rejected();
  st->render_batches = S.render_batches();
  st->mean_render_batch = S.render_batches() ? (double)S.rendered_views() / (double)S.render_batches() : 0.0;
  st->pool_high_water_bytes = (double)S.pool_high_water();
  st->resident_bytes = (double)S.resident_bytes();
  st->first_arrival_s = first < 0.0 ? 0.0 : first;
  st->last_completion_s = last;
}

// ---- the device: launches on HIP streams, completion by events -------------
struct LF {
  const fdl_c64* view_spec;
  const fdl_f2* u;
  float d[FDL_MAX_LAYERS];
  int m, n, C, H, W, reg;
  float lambda, eps;
  float* d_dev;                 // disparities on the device (read by the render kernel)
};

// Bins per construction launch of the server: 2048 blocks of 16 bins, four
// full rounds of the 512 blocks an MI355X holds at once.
constexpr int kSliceBins = 32768;

class HipDevice : public fdl_serve::Device {
 public:
  char* base = nullptr;         // the budgeted pool
  std::vector<LF> lfs;
  std::vector<hipStream_t> render_streams;
  hipStream_t construct_stream = nullptr;
  int rr = 0;
  int max_batch = 1;
  std::vector<hipEvent_t> events;   // token -> event
  std::vector<int> free_tokens;
  float* pinned = nullptr;          // [tokens][max_batch][5] view records in pinned host memory
  std::chrono::steady_clock::time_point t0;
  int error = FDL_OK;

  double now() override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  uint64_t take_token() {
    const int t = free_tokens.back();
    free_tokens.pop_back();
    return (uint64_t)t;
  }
  void note(int e) {
    if (e != FDL_OK && error == FDL_OK) error = e;
  }
  uint64_t construct(int lf, size_t out_off) override {
    const LF& L = lfs[lf];
    const uint64_t tok = take_token();
    // launched in slices of kSliceBins bins: a render issued meanwhile on its
    // own stream gets the device between two slices instead of waiting for
    // the whole construction (4 slices of the 512^2 benchmark light field)
    const int F = L.H * (L.W / 2 + 1);
    for (int b = 0; b < F; b += kSliceBins)
      note(fdl_construct_bins(L.view_spec, L.u, L.d, L.m, L.n, L.C, L.H, L.W, L.lambda, L.eps, L.reg, b,
                              std::min(kSliceBins, F - b), reinterpret_cast<fdl_c64*>(base + out_off), nullptr,
                              construct_stream));
    note(hipEventRecord(events[tok], construct_stream) == hipSuccess ? FDL_OK : FDL_EHIP);
    return tok;
  }
  uint64_t render(int lf, size_t layer_off, const std::vector<const Request*>& group, size_t work_off) override {
    const LF& L = lfs[lf];
    const uint64_t tok = take_token();
    hipStream_t s = render_streams[rr++ % render_streams.size()];
    const int V = (int)group.size();
    const size_t Wh = (size_t)L.W / 2 + 1;
    const size_t spec_bytes = fdl_serve::RangePool::round((size_t)V * L.C * L.H * Wh * 8);
    const size_t img_bytes = fdl_serve::RangePool::round((size_t)V * L.C * L.H * L.W * 4);
    char* spec = base + work_off;
    char* img = spec + spec_bytes;
    char* views = img + img_bytes;
    // view records travel through this token's pinned slot (freed with the token)
    float* host = pinned + (size_t)tok * max_batch * 5;
    for (int v = 0; v < V; ++v) {
      std::memcpy(host + 5 * v, group[v]->view, 4 * sizeof(float));
      const int32_t shape = (int32_t)std::lround(group[v]->view[4]);
      std::memcpy(host + 5 * v + 4, &shape, sizeof(shape));
    }
    if (hipMemcpyAsync(views, host, (size_t)V * 20, hipMemcpyHostToDevice, s) != hipSuccess) note(FDL_EHIP);
    note(fdl_render(reinterpret_cast<const fdl_c64*>(base + layer_off), L.d_dev,
                    L.n, L.C, L.H, L.W, reinterpret_cast<const fdl_view*>(views), V, reinterpret_cast<fdl_c64*>(spec), s));
    note(fdl_irfft2(reinterpret_cast<fdl_c64*>(spec), reinterpret_cast<float*>(img), V * L.C, L.H, L.W, s));
    const size_t one = (size_t)L.C * L.H * L.W * 4;
    for (int v = 0; v < V; ++v)
      if (group[v]->image &&
          hipMemcpyAsync(group[v]->image, img + (size_t)v * one, one, hipMemcpyDeviceToDevice, s) != hipSuccess)
        note(FDL_EHIP);
    note(hipEventRecord(events[tok], s) == hipSuccess ? FDL_OK : FDL_EHIP);
    return tok;
  }
  bool done(uint64_t tok) override {
    const hipError_t e = hipEventQuery(events[tok]);
    if (e == hipErrorNotReady) return false;
    if (e != hipSuccess) note(FDL_EHIP);
    return true;
  }
  void forget(uint64_t tok) override { free_tokens.push_back((int)tok); }
};

// transient bytes of one rendered view: spectrum, image, view record
size_t view_bytes(int C, int H, int W) {
  return fdl_serve::RangePool::round((size_t)C * H * (W / 2 + 1) * 8) +
         fdl_serve::RangePool::round((size_t)C * H * W * 4) + 256;
}

// ---- simulated device (fixed service times, streams run in order) ----------
class SimDevice : public fdl_serve::Device {
 public:
  double t = 0.0;
  double construct_s = 0.0, render_s = 0.0;
  bool serial = false;
  double busy[3] = {0, 0, 0};       // construct stream, two render streams
  int rr = 0;
  std::vector<double> finish;       // token -> completion time
  std::vector<char> active;         // token in use
  std::vector<uint64_t> free_tokens;

  double now() override { return t; }
  uint64_t put(int stream, double service) {
    const double start = std::max(t, busy[stream]);
    busy[stream] = start + service;
    uint64_t tok;
    if (!free_tokens.empty()) {
      tok = free_tokens.back();
      free_tokens.pop_back();
      finish[tok] = busy[stream];
      active[tok] = 1;
    } else {
      tok = finish.size();
      finish.push_back(busy[stream]);
      active.push_back(1);
    }
    return tok;
  }
  uint64_t construct(int, size_t) override { return put(0, construct_s); }
  uint64_t render(int, size_t, const std::vector<const Request*>& g, size_t) override {
    const int s = serial ? 0 : 1 + (rr++ & 1);
    return put(s, render_s * (double)g.size());
  }
  bool done(uint64_t tok) override { return finish[tok] <= t; }
  void forget(uint64_t tok) override {
    active[tok] = 0;
    free_tokens.push_back(tok);
  }
  // earliest completion after the current time among the work in flight
  double next_finish() const {
    double m = -1.0;
    for (size_t k = 0; k < finish.size(); ++k)
      if (active[k] && finish[k] > t && (m < 0.0 || finish[k] < m)) m = finish[k];
    return m;
  }
};

}  // namespace

struct fdl_server {
  fdl_serve::Config cfg;
  HipDevice dev;
  fdl_serve::Scheduler* sched = nullptr;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;

  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!(stop && sched->idle())) {
      const bool progressed = sched->step();
      if (progressed) {
        cv.notify_all();
        continue;
      }
      if (sched->busy()) {
        // work on the device: poll its completion closely (latency is measured here)
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
        continue;
      }
      const double na = sched->next_arrival();
      double wait = 1e-3;
      if (na >= 0.0) wait = std::min(wait, std::max(0.0, na - dev.now()));
      cv.wait_for(lk, std::chrono::duration<double>(wait));
    }
    cv.notify_all();
  }
};

extern "C" {

int fdl_server_create(size_t hbm_budget, int max_render_batch, int max_inflight, int serial, fdl_server** out) {
  if (!out || hbm_budget < 4096 || max_render_batch < 1 || max_render_batch > 256 || max_inflight < 1 ||
      max_inflight > 64)
    return FDL_EINVAL;
  *out = nullptr;
  auto* S = new fdl_server();
  S->cfg.budget = hbm_budget;
  S->cfg.max_render_batch = serial ? 1 : max_render_batch;
  S->cfg.max_inflight = serial ? 1 : max_inflight;
  S->cfg.serial = serial != 0;
  HipDevice& D = S->dev;
  D.max_batch = S->cfg.max_render_batch;
  D.t0 = std::chrono::steady_clock::now();
  int e = hipGetDevice(&S->device) == hipSuccess ? FDL_OK : FDL_EHIP;
  if (e == FDL_OK && hipMalloc(reinterpret_cast<void**>(&D.base), hbm_budget) != hipSuccess) e = FDL_ENOMEM;
  const int ntok = S->cfg.max_inflight + 1;
  if (e == FDL_OK &&
      hipHostMalloc(reinterpret_cast<void**>(&D.pinned), (size_t)ntok * D.max_batch * 5 * sizeof(float)) != hipSuccess)
    e = FDL_ENOMEM;
  for (int t = 0; e == FDL_OK && t < ntok; ++t) {
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) e = FDL_EHIP;
    else {
      D.events.push_back(ev);
      D.free_tokens.push_back(t);
    }
  }
  // streams at the default priority: two for renders, one for constructions
  // (serial mode: one stream for everything, in arrival order)
  const int nrs = serial ? 1 : 2;
  for (int i = 0; e == FDL_OK && i < nrs; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) e = FDL_EHIP;
    else D.render_streams.push_back(s);
  }
  if (e == FDL_OK) {
    if (serial) D.construct_stream = D.render_streams[0];
    else if (hipStreamCreateWithFlags(&D.construct_stream, hipStreamNonBlocking) != hipSuccess) e = FDL_EHIP;
  }
  if (e != FDL_OK) {
    fdl_server_destroy(S);
    return e;
  }
  S->sched = new fdl_serve::Scheduler(S->cfg, &S->dev);
  S->worker = std::thread([S] { S->loop(); });
  *out = S;
  return FDL_OK;
}

int fdl_server_add_lightfield(fdl_server* S, const fdl_c64* view_spec_dev, const fdl_f2* u_dev, const float* d_host,
                              int m, int n, int C, int H, int W, float lambda, float eps, int reg, int32_t* lf_out) {
  if (!S || !view_spec_dev || !u_dev || !d_host || !lf_out) return FDL_EINVAL;
  if (m < 1 || m > 4096 || n < 1 || n > FDL_MAX_LAYERS || C < 1 || C > FDL_MAX_CHANNELS || H < 1 || W < 2 || (W & 1))
    return FDL_ESHAPE;
  if (!(lambda >= 0.f) || !(eps >= 0.f) || reg < FDL_REG_VIEW2 || reg > FDL_REG_L2) return FDL_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  HipDevice& D = S->dev;
  const size_t layer_bytes = (size_t)n * C * H * (W / 2 + 1) * 8;
  // the disparities live beside the pool (FDL_MAX_LAYERS floats per light field)
  float* d_dev = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&d_dev), sizeof(float) * FDL_MAX_LAYERS) != hipSuccess) return FDL_ENOMEM;
  size_t off = 0;
  const int id = S->sched->add_lightfield(layer_bytes, view_bytes(C, H, W), &off);
  if (id < 0) {
    (void)hipFree(d_dev);
    return FDL_ENOMEM;
  }
  LF L;
  L.view_spec = view_spec_dev;
  L.u = u_dev;
  std::memset(L.d, 0, sizeof(L.d));
  std::memcpy(L.d, d_host, sizeof(float) * n);
  L.m = m; L.n = n; L.C = C; L.H = H; L.W = W; L.reg = reg; L.lambda = lambda; L.eps = eps;
  L.d_dev = d_dev;
  D.lfs.push_back(L);
  // initial layers and device disparities, synchronously (set-up, not serving)
  hipStream_t s = D.construct_stream;
  int e = hipMemcpyAsync(d_dev, d_host, sizeof(float) * n, hipMemcpyHostToDevice, s) == hipSuccess ? FDL_OK : FDL_EHIP;
  if (e == FDL_OK)
    e = fdl_construct(view_spec_dev, u_dev, d_host, m, n, C, H, W, lambda, eps, reg,
                      reinterpret_cast<fdl_c64*>(D.base + off), nullptr, s);
  if (e == FDL_OK && hipStreamSynchronize(s) != hipSuccess) e = FDL_EHIP;
  if (e != FDL_OK) return e;
  *lf_out = id;
  return FDL_OK;
}

int fdl_server_submit(fdl_server* S, const fdl_request* req, int64_t* id_out) {
  if (!S || !req || !id_out) return FDL_EINVAL;
  int64_t id = -1;
  int r;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    const double t = req->t_arrival < 0.0 ? S->dev.now() : req->t_arrival;
    const float v[5] = {req->view.u, req->view.v, req->view.focus, req->view.radius, (float)req->view.shape};
    r = S->sched->submit(req->kind, req->lf, v, req->image_dev, t, &id);
  }
  S->cv.notify_all();
  *id_out = id;
  if (r == -2) return FDL_EINVAL;
  if (r == -1) return FDL_ENOMEM;
  return FDL_OK;
}

int fdl_server_poll(fdl_server* S, int64_t id, int32_t* state, double* latency_ms) {
  if (!S || !state) return FDL_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  const Request* r = S->sched->request(id);
  if (!r) return FDL_EINVAL;
  *state = r->state;
  if (latency_ms) *latency_ms = r->state == fdl_serve::kDone ? (r->t_done - r->t_arrival) * 1e3 : -1.0;
  return S->dev.error;
}

int fdl_server_drain(fdl_server* S, double timeout_s) {
  if (!S) return FDL_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  while (!S->sched->idle()) {
    if (S->cv.wait_until(lk, until) == std::cv_status::timeout && !S->sched->idle()) return FDL_ETIMEOUT;
  }
  return S->dev.error;
}

int fdl_server_now(fdl_server* S, double* t) {
  if (!S || !t) return FDL_EINVAL;
  *t = S->dev.now();
  return FDL_OK;
}

int fdl_server_layers(fdl_server* S, int32_t lf, const fdl_c64** layer_spec_dev) {
  if (!S || !layer_spec_dev) return FDL_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  if (lf < 0 || lf >= S->sched->n_lightfields()) return FDL_EINVAL;
  *layer_spec_dev = reinterpret_cast<const fdl_c64*>(S->dev.base + S->sched->resident_off(lf));
  return FDL_OK;
}

int fdl_server_stats(fdl_server* S, fdl_server_summary* st) {
  if (!S || !st) return FDL_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  fill_stats(*S->sched, st);
  return S->dev.error;
}

int fdl_server_destroy(fdl_server* S) {
  if (!S) return FDL_EINVAL;
  if (S->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->cv.notify_all();
    S->worker.join();
  }
  HipDevice& D = S->dev;
  for (hipStream_t s : D.render_streams) {
    (void)hipStreamSynchronize(s);
    if (s != D.construct_stream) (void)hipStreamDestroy(s);
  }
  if (D.construct_stream) {
    (void)hipStreamSynchronize(D.construct_stream);
    (void)hipStreamDestroy(D.construct_stream);
  }
  for (hipEvent_t ev : D.events) (void)hipEventDestroy(ev);
  for (const LF& L : D.lfs) (void)hipFree(L.d_dev);
  if (D.pinned) (void)hipHostFree(D.pinned);
  if (D.base) (void)hipFree(D.base);
  delete S->sched;
  delete S;
  return FDL_OK;
}

int fdl_server_simulate(size_t hbm_budget, int max_render_batch, int max_inflight, int serial, int n_lf,
                        const size_t* layer_bytes, const size_t* view_bytes_per_lf, double construct_s,
                        double render_s_per_view, const fdl_sim_request* reqs, int nreq, fdl_sim_result* out,
                        fdl_server_summary* stats) {
  if (!layer_bytes || !view_bytes_per_lf || (nreq > 0 && (!reqs || !out)) || n_lf < 1 || nreq < 0 ||
      max_render_batch < 1 || max_inflight < 1 || !(construct_s >= 0.0) || !(render_s_per_view >= 0.0))
    return FDL_EINVAL;
  fdl_serve::Config cfg;
  cfg.budget = hbm_budget;
  cfg.max_render_batch = max_render_batch;
  cfg.max_inflight = max_inflight;
  cfg.serial = serial != 0;
  SimDevice D;
  D.construct_s = construct_s;
  D.render_s = render_s_per_view;
  D.serial = cfg.serial;
  fdl_serve::Scheduler S(cfg, &D);
  for (int i = 0; i < n_lf; ++i)
    if (S.add_lightfield(layer_bytes[i], view_bytes_per_lf[i], nullptr) < 0) return FDL_ENOMEM;
  for (int i = 0; i < nreq; ++i) {
    int64_t id;
    if (S.submit(reqs[i].kind, reqs[i].lf, nullptr, nullptr, reqs[i].t_arrival, &id) == -2) return FDL_EINVAL;
  }
  // event-driven clock: run a step at the current time; when nothing moves,
  // jump to the next arrival or completion (each jump passes one of them, so
  // the loop ends)
  for (long guard = 0; !S.idle(); ++guard) {
    if (S.step()) continue;
    double nt = -1.0;
    const double na = S.next_arrival();
    if (na > D.t) nt = na;
    const double nf = D.next_finish();
    if (nf > D.t && (nt < 0.0 || nf < nt)) nt = nf;
    if (nt < 0.0 || guard > 100000000L) return FDL_ENUMERIC;   // no future event: cannot happen
    D.t = nt;
  }
  for (int i = 0; i < nreq; ++i) {
    const Request* r = S.request(i);
    out[i].state = r->state;
    out[i].batch = r->batch;
    out[i].t_admit = r->t_admit;
    out[i].t_done = r->t_done;
  }
  if (stats) fill_stats(S, stats);
  return FDL_OK;
}

}  // extern "C"
