// Scheduling core of the FDL request server (host C++, no HIP calls).
//
// Requests construct the layers of a resident light field again or render one
// view of it.  Everything the server keeps on the device -- the resident layer
// spectra of every light field and the transient buffers of the work in flight
// -- is carved out of ONE device allocation of `budget` bytes, so admission by
// HBM footprint is exact: a unit of work starts only when its buffer can be
// placed.  Resident layer buffers are placed from the top of the pool (best
// fit), transient render buffers from the bottom (first fit), which keeps the
// two apart.
//
// Policy of one scheduling step (`step`):
//   1. retire: every unit of work whose device completion has been observed
//      ends its requests; a render returns its buffer to the pool and drops
//      its hold on the layer buffer it read; a finished construct's output
//      becomes the light field's resident layers, and the previous layers are
//      returned once no render in flight reads them;
//   2. admit: arrived requests in arrival order; a request that cannot start
//      (pool space, one construct per light field at a time, in-flight limit)
//      is skipped and later ones may start, except that once a request has
//      waited longer than `starve_s` nothing that arrived after it starts
//      before it (no starvation).  Renders of one light field that have
//      arrived are grouped into one launch (up to `max_render_batch` views;
//      the group shrinks until its buffer fits).
// Serial mode is the plain baseline: strict arrival order, one unit of work
// at a time, one view per render.
//
// Progress is guaranteed: a request whose footprint can never fit next to the
// resident layers is rejected when it is submitted, and a request that
// cannot be placed while nothing is in flight (only possible if the free
// space is fragmented) is rejected instead of waiting forever.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace fdl_serve {

enum Kind { kConstruct = 0, kRender = 1 };
enum State { kQueued = 0, kRunning = 1, kDone = 2, kRejected = 3 };

// Byte ranges of one allocation (offsets only), 256-byte granules.
class RangePool {
 public:
  static constexpr size_t kNone = ~size_t(0);
  static constexpr size_t kAlign = 256;
  static size_t round(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

  void reset(size_t cap) {
    cap_ = cap / kAlign * kAlign;
    free_.clear();
    if (cap_) free_[0] = cap_;
    used_ = high_ = 0;
  }
  // lowest free range that holds `bytes`
  size_t alloc_low(size_t bytes) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) return take(it, it->first, bytes);
    return kNone;
  }
  // the smallest free range that holds `bytes`, placed at its top end
  size_t alloc_high(size_t bytes) {
    bytes = round(bytes);
    auto best = free_.end();
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes && (best == free_.end() || it->second < best->second ||
                                  (it->second == best->second && it->first > best->first)))
        best = it;
    if (best == free_.end()) return kNone;
    return take(best, best->first + best->second - bytes, bytes);
  }
  void release(size_t off, size_t bytes) {
    bytes = round(bytes);
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t high_water() const { return high_; }

 private:
  size_t take(std::map<size_t, size_t>::iterator it, size_t off, size_t bytes) {
    const size_t r0 = it->first, rn = it->second;
    free_.erase(it);
    if (off > r0) free_[r0] = off - r0;
    if (off + bytes < r0 + rn) free_[off + bytes] = r0 + rn - (off + bytes);
    used_ += bytes;
    high_ = std::max(high_, used_);
    return off;
  }
  size_t cap_ = 0, used_ = 0, high_ = 0;
  std::map<size_t, size_t> free_;   // offset -> length
};

struct Request {
  int64_t id = 0;
  int kind = kRender;
  int lf = 0;
  float view[5] = {0, 0, 0, 0, 0};   // u, v, focus, radius, shape (as fdl_view)
  void* image = nullptr;             // render output [C][H][W] float32 (device) or null
  double t_arrival = 0.0;
  double t_admit = -1.0, t_done = -1.0;
  int state = kQueued;
  int batch = -1;                    // render launch the request joined
};

struct LayerBuf {
  size_t off = 0;
  int readers = 0;                   // renders in flight that read it
  bool retired = false;              // replaced by a newer construction
};

struct LightField {
  size_t layer_bytes = 0;            // n C H (W/2+1) complex64
  size_t view_bytes = 0;             // transient bytes of one rendered view
  int resident = -1;                 // index into the scheduler's layer buffers
  bool constructing = false;
};

struct Work {
  int kind = kRender;
  int lf = 0;
  std::vector<int64_t> ids;
  size_t off = 0, bytes = 0;         // pool range (render: transient; construct: new layers)
  int buf = -1;                      // layer buffer read (render) or written (construct)
  uint64_t token = 0;
};

// What the scheduler needs from the device: launches that return a completion
// token, a completion test, and a clock (seconds).
class Device {
 public:
  virtual ~Device() {}
  virtual double now() = 0;
  virtual uint64_t construct(int lf, size_t out_off) = 0;
  virtual uint64_t render(int lf, size_t layer_off, const std::vector<const Request*>& group, size_t work_off) = 0;
  virtual bool done(uint64_t token) = 0;
  virtual void forget(uint64_t token) = 0;
};

struct Config {
  size_t budget = 0;
  int max_render_batch = 16;
  int max_inflight = 8;
  bool serial = false;
  double starve_s = 0.05;
};

class Scheduler {
 public:
  Scheduler(const Config& c, Device* dev) : cfg_(c), dev_(dev) {
    if (cfg_.serial) {
      cfg_.max_render_batch = 1;
      cfg_.max_inflight = 1;
    }
    if (cfg_.max_render_batch < 1) cfg_.max_render_batch = 1;
    if (cfg_.max_inflight < 1) cfg_.max_inflight = 1;
    pool_.reset(cfg_.budget);
  }

  // Registers a light field and places its resident layers; returns its id,
  // or -1 when the layers do not fit the pool.
  int add_lightfield(size_t layer_bytes, size_t view_bytes, size_t* resident_off) {
    const size_t off = pool_.alloc_high(layer_bytes);
    if (off == RangePool::kNone) return -1;
    LightField L;
    L.layer_bytes = layer_bytes;
    L.view_bytes = view_bytes;
    L.resident = (int)bufs_.size();
    bufs_.push_back(LayerBuf{off, 0, false});
    lfs_.push_back(L);
    resident_total_ += RangePool::round(layer_bytes);
    if (resident_off) *resident_off = off;
    return (int)lfs_.size() - 1;
  }

  // 0: queued (id set); -1: rejected, can never fit; -2: unknown light field
  // or kind.  A rejected request still gets an id (state kRejected).
  int submit(int kind, int lf, const float* view, void* image, double t_arrival, int64_t* id) {
    if (lf < 0 || lf >= (int)lfs_.size() || (kind != kConstruct && kind != kRender)) return -2;
    Request r;
    r.id = (int64_t)reqs_.size();
    r.kind = kind;
    r.lf = lf;
    if (view)
      for (int i = 0; i < 5; ++i) r.view[i] = view[i];
    r.image = image;
    r.t_arrival = t_arrival;
    const size_t need = RangePool::round(kind == kConstruct ? lfs_[lf].layer_bytes : lfs_[lf].view_bytes);
    const bool fits = need <= pool_.capacity() - resident_total_;
    r.state = fits ? kQueued : kRejected;
    reqs_.push_back(r);
    if (id) *id = r.id;
    ++submitted_;
    if (!fits) {
      ++rejected_;
      return -1;
    }
    // not yet arrived: kept in arrival order until its time comes
    auto pos = std::upper_bound(pending_.begin(), pending_.end(), t_arrival,
                                [&](double t, int64_t o) { return t < reqs_[o].t_arrival; });
    pending_.insert(pos, r.id);
    return 0;
  }

  // One scheduling pass; true if anything was retired or admitted.
  bool step() {
    bool progressed = retire();
    progressed = admit() || progressed;
    return progressed;
  }

  bool idle() const { return pending_.empty() && queue_.empty() && inflight_.empty(); }
  bool busy() const { return !inflight_.empty(); }
  // earliest arrival still to come, or a negative value if none
  double next_arrival() const { return pending_.empty() ? -1.0 : reqs_[pending_.front()].t_arrival; }
  const Request* request(int64_t id) const { return id >= 0 && id < (int64_t)reqs_.size() ? &reqs_[id] : nullptr; }
  int64_t submitted() const { return submitted_; }
  int64_t completed() const { return completed_; }
  int64_t rejected() const { return rejected_; }
  int64_t render_batches() const { return render_batches_; }
  int64_t rendered_views() const { return rendered_views_; }
  size_t pool_high_water() const { return pool_.high_water(); }
  size_t resident_bytes() const { return resident_total_; }
  size_t resident_off(int lf) const { return bufs_[lfs_[lf].resident].off; }
  int n_lightfields() const { return (int)lfs_.size(); }
  const std::vector<Request>& requests() const { return reqs_; }

 private:
  bool retire() {
    bool any = false;
    for (size_t w = 0; w < inflight_.size();) {
      Work& W = inflight_[w];
      if (!dev_->done(W.token)) {
        ++w;
        continue;
      }
      const double t = dev_->now();
      for (int64_t id : W.ids) {
        reqs_[id].state = kDone;
        reqs_[id].t_done = t;
        ++completed_;
      }
      LightField& L = lfs_[W.lf];
      if (W.kind == kRender) {
        pool_.release(W.off, W.bytes);
        LayerBuf& B = bufs_[W.buf];
        --B.readers;
        if (B.retired && B.readers == 0) pool_.release(B.off, lfs_[W.lf].layer_bytes);
      } else {
        LayerBuf& old = bufs_[L.resident];
        old.retired = true;
        if (old.readers == 0) pool_.release(old.off, L.layer_bytes);
        L.resident = W.buf;
        L.constructing = false;
      }
      dev_->forget(W.token);
      inflight_.erase(inflight_.begin() + (long)w);
      any = true;
    }
    return any;
  }

  bool admit() {
    bool any = false;
    const double now = dev_->now();
    while (!pending_.empty() && reqs_[pending_.front()].t_arrival <= now) {
      queue_.push_back(pending_.front());
      pending_.pop_front();
    }
    std::vector<bool> taken(queue_.size(), false);
    for (size_t qi = 0; qi < queue_.size(); ++qi) {
      if ((int)inflight_.size() >= cfg_.max_inflight) break;
      if (taken[qi]) continue;
      Request& r = reqs_[queue_[qi]];
      const bool started = r.kind == kConstruct ? start_construct(r) : start_render(qi, taken);
      if (started) {
        taken[qi] = true;
        any = true;
        continue;
      }
      if (inflight_.empty()) {
        // nothing in flight holds memory, yet it cannot be placed: the free
        // space is fragmented; reject instead of waiting forever
        r.state = kRejected;
        ++rejected_;
        taken[qi] = true;
        any = true;
        continue;
      }
      if (cfg_.serial || now - r.t_arrival > cfg_.starve_s) break;   // nothing may overtake it
    }
    if (any) {
      std::deque<int64_t> rest;
      for (size_t qi = 0; qi < queue_.size(); ++qi)
        if (!taken[qi]) rest.push_back(queue_[qi]);
      queue_.swap(rest);
    }
    return any;
  }

  bool start_construct(Request& r) {
    LightField& L = lfs_[r.lf];
    if (L.constructing) return false;   // one construction per light field at a time
    const size_t off = pool_.alloc_high(L.layer_bytes);
    if (off == RangePool::kNone) return false;
    Work W;
    W.kind = kConstruct;
    W.lf = r.lf;
    W.ids.push_back(r.id);
    W.off = off;
    W.bytes = L.layer_bytes;
    W.buf = (int)bufs_.size();
    bufs_.push_back(LayerBuf{off, 0, false});
    L.constructing = true;
    r.state = kRunning;
    r.t_admit = dev_->now();
    W.token = dev_->construct(r.lf, off);
    inflight_.push_back(W);
    return true;
  }

  bool start_render(size_t qi, std::vector<bool>& taken) {
    Request& r = reqs_[queue_[qi]];
    LightField& L = lfs_[r.lf];
    const double now = dev_->now();
    std::vector<size_t> group{qi};
    for (size_t k = qi + 1; k < queue_.size() && (int)group.size() < cfg_.max_render_batch; ++k) {
      const Request& o = reqs_[queue_[k]];
      if (!taken[k] && o.kind == kRender && o.lf == r.lf) group.push_back(k);
    }
    size_t off = RangePool::kNone;
    while (!group.empty()) {
      off = pool_.alloc_low(L.view_bytes * group.size());
      if (off != RangePool::kNone) break;
      group.pop_back();
    }
    if (group.empty()) return false;
    Work W;
    W.kind = kRender;
    W.lf = r.lf;
    W.off = off;
    W.bytes = L.view_bytes * group.size();
    W.buf = L.resident;
    std::vector<const Request*> reqs;
    for (size_t k : group) {
      Request& o = reqs_[queue_[k]];
      o.state = kRunning;
      o.t_admit = now;
      o.batch = (int)render_batches_;
      W.ids.push_back(o.id);
      reqs.push_back(&o);
      taken[k] = true;
    }
    ++bufs_[W.buf].readers;
    ++render_batches_;
    rendered_views_ += (int64_t)group.size();
    W.token = dev_->render(r.lf, bufs_[W.buf].off, reqs, off);
    inflight_.push_back(W);
    return true;
  }

  Config cfg_;
  Device* dev_;
  RangePool pool_;
  std::vector<LightField> lfs_;
  std::vector<LayerBuf> bufs_;
  std::vector<Request> reqs_;
  std::deque<int64_t> pending_;   // submitted, not yet arrived (arrival order)
  std::deque<int64_t> queue_;     // arrived, waiting to start (arrival order)
  std::vector<Work> inflight_;
  size_t resident_total_ = 0;
  int64_t submitted_ = 0, completed_ = 0, rejected_ = 0, render_batches_ = 0, rendered_views_ = 0;
};

}  // namespace fdl_serve
