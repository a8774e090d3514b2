// Serving loop: continuous batching of cross-section requests on one device.
//
// Requests wait in arrival order until room in the serving arena (one device allocation,
// sub-allocated per request) lets them in; an admitted request holds its block until it is
// done. Each admitted request's path is cut into steps (the parameter kernel of a batch of
// P-T points, then the tile kernel over consecutive chunks of its tile order of at least
// step_items work items each, then the batch's reduction), and a server thread keeps a few
// execution lanes (non-blocking HIP streams at the default priority) fed with steps:
// whenever a lane has room, it takes the next step of the admitted request with the least
// estimated remaining work (weighted down by the time the request has waited, so large
// requests are not starved); one lane is kept for requests of a single step. A request's
// steps run in order: its next step goes to the lane of its step still in flight, or to
// any lane once none is. Kernels of different requests therefore share the device at step
// granularity, short requests finish while long ones are in progress, and a finished
// request frees its block at once.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/xsec.h"
#include "kernel_args.h"
#include "runtime_internal.h"

namespace xs {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t round256(size_t b) { return (std::max<size_t>(b, 1) + 255) / 256 * 256; }

// First-fit allocator over [0, size) in 256-byte units; free blocks are kept by offset and
// merged with their neighbours on release.
class Arena {
 public:
  void reset(size_t size) {
    size_ = size / 256 * 256;
    used_ = peak_ = 0;
    free_.clear();
    if (size_) free_[0] = size_;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, next = it->first + bytes;
      free_.erase(it);
      if (rest) free_[next] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t peak() const { return peak_; }

 private:
  size_t size_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct Waiting {
  uint64_t id;
  size_t bytes;
  int bypassed;
};

// Admission rule. Scans the waiting requests in arrival order and admits the first whose
// footprint fits the arena; every request it passes counts one bypass, and a request that
// has been passed max_bypass times (any time, if max_bypass < 0) may not be passed again,
// so the scan stops there. Returns the index admitted (its block in *off) or -1.
int pick_admission(std::deque<Waiting>& q, Arena& a, int max_bypass, size_t* off) {
  for (size_t i = 0; i < q.size(); ++i) {
    if (a.alloc(q[i].bytes, off)) {
      for (size_t j = 0; j < i; ++j) ++q[j].bypassed;
      return (int)i;
    }
    if (max_bypass < 0 || q[i].bypassed >= max_bypass) return -1;
  }
  return -1;
}

enum { kQueued = 0, kRunning = 1, kDone = 2 };

// One step of a request: the parameter kernel of batch [pt0, pt0 + nb) (params), the tile
// kernel over tile-order positions [c0, c1), and the batch's reduction (reduce).
struct Step {
  int pt0, nb;
  int64_t c0, c1;
  bool params, reduce;
  double est;          // estimated line-point visits
};

struct Request {
  uint64_t id = 0;
  int state = kQueued;
  int status = XS_OK;
  std::string err;
  LinesRes* L = nullptr;
  GridRes* G = nullptr;      // the context's grid, or &own for a window request
  bool own_grid = false;
  GridRes own;
  double nu_start = 0.0, step = 0.0;
  xs_opts o{};
  std::vector<double> pt_pairs;   // (P, T) interleaved
  void* out = nullptr;
  bool out_dev = false;
  Plan plan;
  std::vector<Step> steps;
  size_t next = 0;           // next step to enqueue
  int inflight = 0;          // steps enqueued and not yet complete
  int lane = -1;             // lane of the steps in flight
  double remaining = 0.0;    // estimated visits of the steps not yet enqueued
  double total = 0.0;        // estimated visits of all steps
  bool uploaded = false;     // inputs staged to the device
  bool cancel = false;       // stop at the next step boundary
  int fail_rc = XS_OK;
  std::string fail_msg;
  // arena block and its parts (byte offsets inside the block); pinned staging block
  size_t bytes = 0, off = 0;
  size_t o_rec = 0, o_part = 0, o_out = 0, o_grid = 0, o_pts = 0, o_order = 0;
  size_t pin_bytes = 0, pin_off = 0;
  double t_submit = -1.0, t_admit = -1.0, t_done = -1.0;
};

struct InFlight {
  Request* r;
  hipEvent_t ev;
};

struct Lane {
  hipStream_t st = nullptr;
  std::deque<InFlight> q;
};

constexpr int kLaneDepth = 2;          // steps queued per lane
constexpr double kAgeScale = 0.5;      // s: waiting this long halves a request's priority key

}  // namespace

struct Server {
  Ctx* c = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false, paused = false;
  int n_lanes = 4, max_bypass = 8, max_admitted = 32;
  int64_t step_items = 0;
  char* base = nullptr;        // device arena
  size_t mem = 0;
  Arena arena;
  char* pin_base = nullptr;    // pinned staging arena
  size_t pin_mem = 0;
  Arena pin_arena;
  std::vector<Lane> lanes;
  std::vector<hipEvent_t> events;   // free completion events
  std::deque<Waiting> queue;
  std::vector<Request*> admitted;
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t next_id = 1;

  void loop();
  int enqueue_next(Request& r, Lane& ln);
  void finish(Request& r, int status, const std::string& err);
  void build_steps(Request& r) const;
};

// Cut the request's path into steps of at least step_items work items each (tiles x
// points of the batch x split), so that every tile-kernel launch fills the device even
// when the request runs alone; each step's estimated line-point visits (from the sampled
// windows) rank requests.
void Server::build_steps(Request& r) const {
  const Plan& p = r.plan;
  // units of the issue order: tiles, or groups of p.group tiles (one wavefront per tile)
  const double pts_per_unit = (double)(kWave * p.P * p.group);
  for (int pt0 = 0; pt0 < p.npts; pt0 += p.pt_batch) {
    const int nb = std::min(p.pt_batch, p.npts - pt0);
    const int64_t items_per_unit = (int64_t)nb * p.split * p.group;
    int64_t c0 = 0;
    double acc = 0.0;
    bool first = true;
    for (int64_t i = 0; i < p.n_units; ++i) {
      acc += (double)(p.tile_cost[p.tile_order[i]] + 1) * (double)kSampleStride *
             pts_per_unit * nb;
      if ((i + 1 - c0) * items_per_unit >= step_items || i + 1 == p.n_units) {
        r.steps.push_back({pt0, nb, c0, i + 1, first, i + 1 == p.n_units, acc});
        first = false;
        c0 = i + 1;
        acc = 0.0;
      }
    }
  }
  r.remaining = 0.0;
  for (const Step& s : r.steps) r.remaining += s.est;
  r.total = r.remaining;
}

// Drop the request's references and memory; the caller holds mu and no step of the
// request is in flight.
void Server::finish(Request& r, int status, const std::string& err) {
  if (r.state == kRunning) {
    arena.release(r.off, r.bytes);
    pin_arena.release(r.pin_off, r.pin_bytes);
    admitted.erase(std::find(admitted.begin(), admitted.end(), &r));
  }
  r.L->refs.fetch_sub(1);
  if (!r.own_grid) r.G->refs.fetch_sub(1);
  r.status = status;
  r.err = err;
  r.state = kDone;
  r.t_done = now_s();
  cv_done.notify_all();
}

// Enqueue the request's next step on the lane (staging its inputs first if this is its
// first step) and record a completion event. Called by the server thread without mu: the
// request is admitted, so only this thread changes its dispatch state and frees it, and
// other threads only read its timestamps or set its cancel flag under mu.
int Server::enqueue_next(Request& r, Lane& ln) {
  char* blk = base + r.off;
  hipError_t e;
  if (!r.uploaded) {
    const size_t pts_bytes = r.pt_pairs.size() * sizeof(double);
    const size_t ord_bytes = r.plan.tile_order.size() * sizeof(int);
    char* pin = pin_base + r.pin_off;
    memcpy(pin, r.pt_pairs.data(), pts_bytes);
    memcpy(pin + round256(pts_bytes), r.plan.tile_order.data(), ord_bytes);
    e = hipMemcpyAsync(blk + r.o_pts, pin, pts_bytes, hipMemcpyHostToDevice, ln.st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(blk + r.o_order, pin + round256(pts_bytes), ord_bytes,
                         hipMemcpyHostToDevice, ln.st);
    if (e != hipSuccess) return hip_fail(e, "serving upload");
    if (r.own_grid) {
      r.own.d = (double*)(blk + r.o_grid);
      e = launch_fill_uniform(r.own.d, (int64_t)r.own.n, r.nu_start, r.step, ln.st);
      if (e != hipSuccess) return hip_fail(e, "grid fill launch");
    }
    r.uploaded = true;
  }
  const Step& s = r.steps[r.next];
  void* out_dev = r.out_dev ? r.out : (void*)(blk + r.o_out);
  void* part = r.plan.split > 1 ? (void*)(blk + r.o_part) : nullptr;
  int rc = enqueue_step(*r.L, *r.G, r.o, r.plan, (const double*)(blk + r.o_pts),
                        (const int*)(blk + r.o_order), out_dev, blk + r.o_rec, part, ln.st,
                        s.pt0, s.nb, s.c0, s.c1, s.params, s.reduce);
  if (rc) return rc;
  hipEvent_t ev;
  if (events.empty()) {
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  } else {
    ev = events.back();
    events.pop_back();
  }
  e = hipEventRecord(ev, ln.st);
  if (e != hipSuccess) {
    events.push_back(ev);
    return hip_fail(e, "hipEventRecord");
  }
  ln.q.push_back({&r, ev});
  r.remaining -= s.est;
  ++r.next;
  ++r.inflight;
  return XS_OK;
}

void Server::loop() {
  (void)hipSetDevice(c->device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // completed steps
    std::vector<Request*> done;
    for (size_t li = 0; li < lanes.size(); ++li) {
      Lane& ln = lanes[li];
      while (!ln.q.empty()) {
        const hipError_t e = hipEventQuery(ln.q.front().ev);
        if (e == hipErrorNotReady) break;
        Request& r = *ln.q.front().r;
        events.push_back(ln.q.front().ev);
        ln.q.pop_front();
        --r.inflight;
        if (e != hipSuccess && r.fail_rc == XS_OK) {
          hip_fail(e, "serving step");
          r.fail_rc = XS_EDEVICE;
          r.fail_msg = g_last_error;
        }
        if (r.inflight == 0 && (r.next == r.steps.size() || r.cancel || r.fail_rc))
          done.push_back(&r);
      }
    }
    if (!done.empty()) {
      // download host outputs without holding the lock
      std::vector<std::pair<int, std::string>> res(done.size());
      for (size_t k = 0; k < done.size(); ++k) {
        Request& r = *done[k];
        res[k] = r.fail_rc ? std::make_pair(r.fail_rc, r.fail_msg)
                 : r.cancel ? std::make_pair((int)XS_ECANCELLED, std::string("cancelled"))
                            : std::make_pair((int)XS_OK, std::string());
      }
      lk.unlock();
      for (size_t k = 0; k < done.size(); ++k) {
        Request& r = *done[k];
        if (res[k].first != XS_OK || r.out_dev) continue;
        const size_t ob = r.pt_pairs.size() / 2 * r.G->n * out_elem_bytes(r.o);
        const hipError_t e = hipMemcpy(r.out, base + r.off + r.o_out, ob, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
          hip_fail(e, "result download");
          res[k] = {XS_EDEVICE, g_last_error};
        }
      }
      lk.lock();
      for (size_t k = 0; k < done.size(); ++k) finish(*done[k], res[k].first, res[k].second);
    }
    // admissions: arena room (device and pinned staging) and the admitted-set limit
    while (!paused && !stop && (int)admitted.size() < max_admitted && !queue.empty()) {
      size_t off = 0;
      const int i = pick_admission(queue, arena, max_bypass, &off);
      if (i < 0) break;
      Request* r = reqs[queue[i].id];
      size_t pin_off = 0;
      if (!pin_arena.alloc(r->pin_bytes, &pin_off)) {
        arena.release(off, r->bytes);
        break;
      }
      queue.erase(queue.begin() + i);
      r->off = off;
      r->pin_off = pin_off;
      r->state = kRunning;
      r->t_admit = now_s();
      admitted.push_back(r);
    }
    // dispatch: fill every lane with steps of the admitted requests, least remaining work
    // (discounted by waiting time) first. With two lanes or more, lane 0 only takes
    // requests of at most one step's work, so a short request never queues behind a
    // step of a long one.
    const double t = now_s();
    for (size_t li = 0; li < lanes.size(); ++li) {
      Lane& ln = lanes[li];
      const bool express = li == 0 && lanes.size() >= 2;
      while ((int)ln.q.size() < kLaneDepth) {
        Request* best = nullptr;
        double best_key = 0.0;
        for (Request* r : admitted) {
          if (r->cancel || r->fail_rc || r->next == r->steps.size()) continue;
          if (r->inflight > 0 && r->lane != (int)li) continue;
          if (express && r->steps.size() > 1) continue;
          const double key = r->remaining / (1.0 + (t - r->t_submit) / kAgeScale);
          if (!best || key < best_key) {
            best = r;
            best_key = key;
          }
        }
        if (!best) break;
        // the launches can block (a full hardware queue): submitters and pollers must not
        // wait for them
        lk.unlock();
        const int rc = enqueue_next(*best, ln);
        // earlier parts of a failed step may be queued: let them drain first
        if (rc && best->inflight == 0) (void)hipStreamSynchronize(ln.st);
        lk.lock();
        if (rc) {
          best->fail_rc = rc;
          best->fail_msg = g_last_error;
          if (best->inflight == 0) finish(*best, rc, best->fail_msg);
          continue;
        }
        best->lane = (int)li;
      }
    }
    // requests cancelled with nothing in flight
    for (size_t k = 0; k < admitted.size();) {
      Request* r = admitted[k];
      if (r->cancel && r->inflight == 0) {
        finish(*r, XS_ECANCELLED, "cancelled");
        continue;
      }
      ++k;
    }
    if (stop && admitted.empty()) break;
    if (admitted.empty() && (queue.empty() || paused || stop))
      cv_work.wait(lk);
    else
      cv_work.wait_for(lk, std::chrono::microseconds(20));
  }
}

void serve_shutdown(Ctx* c) {
  Server* s = c->server;
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    while (!s->queue.empty()) {
      Request* r = s->reqs[s->queue.front().id];
      s->queue.pop_front();
      s->finish(*r, XS_ECANCELLED, "cancelled at shutdown");
    }
    for (Request* r : s->admitted) r->cancel = true;
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  for (Lane& ln : s->lanes) {
    if (ln.st) (void)hipStreamSynchronize(ln.st);
    if (ln.st) (void)hipStreamDestroy(ln.st);
  }
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  for (auto& kv : s->reqs) delete kv.second;
  if (s->pin_base) (void)hipHostFree(s->pin_base);
  if (s->base) c->dev_free(s->base, s->mem);
  delete s;
  c->server = nullptr;
}

static int serve_start_locked(Ctx* c, const xs_serve_opts* o) {
  xs_serve_opts d{};
  if (!o) o = &d;
  if (o->max_inflight < 0 || o->max_inflight > 64)
    return fail(XS_EINVAL, "max_inflight must be in [0, 64] (got %d)", o->max_inflight);
  if (o->max_admitted < 0 || o->max_admitted > 4096)
    return fail(XS_EINVAL, "max_admitted must be in [0, 4096] (got %d)", o->max_admitted);
  if (o->step_items < 0) return fail(XS_EINVAL, "step_items must be >= 0");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  Server* s = new Server();
  s->c = c;
  s->n_lanes = o->max_inflight ? o->max_inflight : 4;
  s->max_bypass = o->max_bypass == 0 ? 8 : o->max_bypass;
  s->max_admitted = o->max_admitted ? o->max_admitted : 32;
  // default: two rounds of wavefront slots of the device (4 SIMDs x 7 waves per CU)
  s->step_items = o->step_items > 0 ? o->step_items : (int64_t)c->n_cu * 56;
  s->paused = o->start_paused != 0;
  size_t mem = o->mem_bytes;
  if (mem == 0) {
    const size_t used = c->used.load();
    const size_t free_b = c->budget > used ? c->budget - used : 0;
    mem = std::min<size_t>((size_t)64 << 30, free_b / 2);
  }
  mem = mem / 256 * 256;
  if (mem < 4096) {
    delete s;
    return fail(XS_ENOMEM, "serving arena of %zu bytes is too small", mem);
  }
  int rc = c->dev_alloc((void**)&s->base, mem, "serving arena");
  if (rc) {
    delete s;
    return rc;
  }
  s->mem = mem;
  s->arena.reset(mem);
  c->server = s;
  s->pin_mem = (size_t)32 << 20;
  e = hipHostMalloc((void**)&s->pin_base, s->pin_mem, 0);
  if (e != hipSuccess) {
    s->pin_base = nullptr;
    serve_shutdown(c);
    return hip_fail(e, "hipHostMalloc (serving staging)");
  }
  s->pin_arena.reset(s->pin_mem);
  s->lanes.resize(s->n_lanes);
  for (Lane& ln : s->lanes) {
    e = hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking);
    if (e != hipSuccess) {
      ln.st = nullptr;
      serve_shutdown(c);
      return hip_fail(e, "serving stream");
    }
  }
  s->th = std::thread([s] { s->loop(); });
  return XS_OK;
}

static int ensure_server(Ctx* c) {
  std::lock_guard<std::mutex> lk(c->serve_mu);
  if (c->server) return XS_OK;
  return serve_start_locked(c, nullptr);
}

static Request* find_req(Server* s, xs_req_t id) {
  auto it = s->reqs.find(id);
  return it == s->reqs.end() ? nullptr : it->second;
}

// Common part of xs_submit / xs_submit_window: G == nullptr means a window request.
static int submit(Ctx* c, xs_lines_t lh, xs_grid_t gh, bool window, double nu_start,
                  double step, size_t n_points, const xs_pt* pts, size_t npts,
                  const xs_opts* opts, void* sigma_out, int out_on_device, xs_req_t* out) {
  // the request's latency counts from here (planning and queueing included)
  const double t_submit = now_s();
  if (!c || !out || !sigma_out) return fail(XS_EINVAL, "NULL argument");
  int rc = validate_opts(opts);
  if (rc) return rc;
  rc = validate_pts(pts, npts);
  if (rc) return rc;
  if (window) {
    if (n_points == 0 || n_points > ((size_t)1 << 31))
      return fail(XS_EINVAL, "n_points must be in [1, 2^31] (got %zu)", n_points);
    if (!isfinite(nu_start) || !(step > 0.0) || !isfinite(step) ||
        !isfinite(nu_start + step * (double)(n_points - 1)))
      return fail(XS_EINVAL, "window start %g / step %g invalid", nu_start, step);
  }
  rc = ensure_server(c);
  if (rc) return rc;
  Server* s = c->server;
  Request* r = new Request();
  {
    std::lock_guard<std::mutex> lk(c->mu);
    r->L = c->find_lines(lh);
    if (!window) r->G = c->find_grid(gh);
    if (!r->L || (!window && !r->G)) {
      delete r;
      return fail(XS_ENOTFOUND, "unknown line list %llu or grid %llu",
                  (unsigned long long)lh, (unsigned long long)gh);
    }
    r->L->refs.fetch_add(1);
    if (!window) r->G->refs.fetch_add(1);
  }
  if (window) {
    r->own_grid = true;
    r->nu_start = nu_start;
    r->step = step;
    r->own.n = n_points;
    r->own.host.resize(n_points);
    for (size_t j = 0; j < n_points; ++j) r->own.host[j] = nu_start + (double)j * step;
    r->own.first = r->own.host.front();
    r->own.last = r->own.host.back();
    r->own.bytes = n_points * sizeof(double);
    r->G = &r->own;
  }
  r->o = *opts;
  r->pt_pairs.resize(2 * npts);
  for (size_t k = 0; k < npts; ++k) {
    r->pt_pairs[2 * k] = pts[k].P_bar;
    r->pt_pairs[2 * k + 1] = pts[k].T_K;
  }
  r->out = sigma_out;
  r->out_dev = out_on_device != 0;
  r->plan = make_plan(*c, *r->L, *r->G, npts, *opts, s->mem / 4, kServeItemLines);
  const size_t n = r->G->n;
  size_t at = 0;
  auto part = [&](size_t bytes) {
    const size_t o = at;
    at += round256(bytes);
    return o;
  };
  r->o_rec = part(r->plan.rec_bytes());
  r->o_part = part(r->plan.part_bytes(n));
  r->o_out = part(r->out_dev ? 0 : npts * n * out_elem_bytes(*opts));
  r->o_grid = part(window ? n * sizeof(double) : 0);
  r->o_pts = part(npts * 2 * sizeof(double));
  r->o_order = part(r->plan.tile_order.size() * sizeof(int));
  r->bytes = at;
  r->pin_bytes = round256(npts * 2 * sizeof(double)) + r->plan.tile_order.size() * sizeof(int);
  s->build_steps(*r);
  if (r->bytes > s->arena.size() || round256(r->pin_bytes) > s->pin_arena.size()) {
    const size_t b = r->bytes;
    r->L->refs.fetch_sub(1);
    if (!window) r->G->refs.fetch_sub(1);
    delete r;
    return fail(XS_ENOMEM, "request footprint %zu bytes exceeds the serving arena (%zu)", b,
                s->arena.size());
  }
  std::lock_guard<std::mutex> lk(s->mu);
  r->id = s->next_id++;
  r->t_submit = t_submit;
  s->reqs[r->id] = r;
  s->queue.push_back({r->id, r->bytes, 0});
  *out = r->id;
  s->cv_work.notify_all();
  return XS_OK;
}

// Discrete-event run of the admission rule (host only).
static int simulate(size_t n, const double* arrive, const double* dur, const uint64_t* fp,
                    uint64_t mem, int slots, int max_bypass, double* admit, double* done,
                    uint64_t* peak) {
  Arena a;
  a.reset(mem);
  for (size_t i = 0; i < n; ++i) {
    if (round256(fp[i]) > a.size())
      return fail(XS_ENOMEM, "footprint[%zu] = %llu exceeds the arena", i,
                  (unsigned long long)fp[i]);
    if (i && arrive[i] < arrive[i - 1]) return fail(XS_EINVAL, "arrive must be non-decreasing");
  }
  std::deque<Waiting> q;
  std::vector<size_t> offs(n);
  std::multimap<double, size_t> run;   // completion time -> request
  size_t next = 0, finished = 0;
  double t = n ? arrive[0] : 0.0;
  while (finished < n) {
    while (next < n && arrive[next] <= t) {
      q.push_back({next, fp[next], 0});
      ++next;
    }
    while ((int)run.size() < slots && !q.empty()) {
      size_t off = 0;
      const int i = pick_admission(q, a, max_bypass, &off);
      if (i < 0) break;
      const size_t id = q[i].id;
      q.erase(q.begin() + i);
      offs[id] = off;
      admit[id] = t;
      done[id] = t + dur[id];
      run.emplace(done[id], id);
    }
    const double t_arr = next < n ? arrive[next] : INFINITY;
    const double t_fin = run.empty() ? INFINITY : run.begin()->first;
    if (t_fin <= t_arr) {
      t = t_fin;
      while (!run.empty() && run.begin()->first <= t) {
        const size_t id = run.begin()->second;
        run.erase(run.begin());
        a.release(offs[id], fp[id]);
        ++finished;
      }
    } else {
      t = t_arr;
    }
  }
  if (peak) *peak = a.peak();
  return XS_OK;
}

}  // namespace xs

using namespace xs;

int xs_serve_start(xs_ctx* c, const xs_serve_opts* opts) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->serve_mu);
  if (c->server) return fail(XS_EBUSY, "the server is already running");
  return serve_start_locked(c, opts);
}

int xs_serve_pause(xs_ctx* c, int paused) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  int rc = ensure_server(c);
  if (rc) return rc;
  Server* s = c->server;
  std::lock_guard<std::mutex> lk(s->mu);
  s->paused = paused != 0;
  s->cv_work.notify_all();
  return XS_OK;
}

int xs_submit(xs_ctx* c, xs_lines_t lines, xs_grid_t grid, const xs_pt* pts, size_t npts,
              const xs_opts* opts, void* sigma_out, int out_on_device, xs_req_t* out) {
  return submit(c, lines, grid, false, 0.0, 0.0, 0, pts, npts, opts, sigma_out, out_on_device,
                out);
}

int xs_submit_window(xs_ctx* c, xs_lines_t lines, double nu_start, double step,
                     size_t n_points, const xs_pt* pts, size_t npts, const xs_opts* opts,
                     void* sigma_out, int out_on_device, xs_req_t* out) {
  return submit(c, lines, 0, true, nu_start, step, n_points, pts, npts, opts, sigma_out,
                out_on_device, out);
}

int xs_poll(xs_ctx* c, xs_req_t req, int* done) {
  if (!c || !done) return fail(XS_EINVAL, "NULL argument");
  Server* s = c->server;
  if (!s) return fail(XS_ENOTFOUND, "no server");
  std::lock_guard<std::mutex> lk(s->mu);
  Request* r = find_req(s, req);
  if (!r) return fail(XS_ENOTFOUND, "unknown request %llu", (unsigned long long)req);
  *done = r->state == kDone;
  return XS_OK;
}

int xs_wait(xs_ctx* c, xs_req_t req, double timeout_s) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  Server* s = c->server;
  if (!s) return fail(XS_ENOTFOUND, "no server");
  std::unique_lock<std::mutex> lk(s->mu);
  Request* r = find_req(s, req);
  if (!r) return fail(XS_ENOTFOUND, "unknown request %llu", (unsigned long long)req);
  auto ready = [&] { return r->state == kDone; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return fail(XS_ETIMEOUT, "request %llu still pending after %g s", (unsigned long long)req,
                timeout_s);
  }
  if (r->status != XS_OK) return fail(r->status, "%s", r->err.c_str());
  return XS_OK;
}

int xs_cancel(xs_ctx* c, xs_req_t req) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  Server* s = c->server;
  if (!s) return fail(XS_ENOTFOUND, "no server");
  std::lock_guard<std::mutex> lk(s->mu);
  Request* r = find_req(s, req);
  if (!r) return fail(XS_ENOTFOUND, "unknown request %llu", (unsigned long long)req);
  if (r->state == kRunning) {
    // stops at its next step boundary (the server thread finishes it)
    r->cancel = true;
    s->cv_work.notify_all();
    return XS_OK;
  }
  if (r->state == kQueued) {
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
      if (it->id == req) {
        s->queue.erase(it);
        break;
      }
    s->finish(*r, XS_ECANCELLED, "cancelled");
  }
  return XS_OK;
}

int xs_request_times(xs_ctx* c, xs_req_t req, double* t_submit, double* t_admit,
                     double* t_done) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  Server* s = c->server;
  if (!s) return fail(XS_ENOTFOUND, "no server");
  std::lock_guard<std::mutex> lk(s->mu);
  Request* r = find_req(s, req);
  if (!r) return fail(XS_ENOTFOUND, "unknown request %llu", (unsigned long long)req);
  if (t_submit) *t_submit = r->t_submit;
  if (t_admit) *t_admit = r->t_admit;
  if (t_done) *t_done = r->t_done;
  return XS_OK;
}

int xs_release(xs_ctx* c, xs_req_t req) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  Server* s = c->server;
  if (!s) return fail(XS_ENOTFOUND, "no server");
  std::lock_guard<std::mutex> lk(s->mu);
  Request* r = find_req(s, req);
  if (!r) return fail(XS_ENOTFOUND, "unknown request %llu", (unsigned long long)req);
  if (r->state != kDone) return fail(XS_EBUSY, "request %llu is pending", (unsigned long long)req);
  s->reqs.erase(req);
  delete r;
  return XS_OK;
}

int xs_sched_simulate(size_t n, const double* arrive, const double* duration,
                      const uint64_t* footprint, uint64_t mem_bytes, int max_admitted,
                      int max_bypass, double* admit_out, double* done_out,
                      uint64_t* peak_bytes) {
  if (n && (!arrive || !duration || !footprint || !admit_out || !done_out))
    return fail(XS_EINVAL, "NULL argument");
  if (max_admitted < 1) return fail(XS_EINVAL, "max_admitted must be >= 1");
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(arrive[i]) || !(duration[i] >= 0.0) || !isfinite(duration[i]))
      return fail(XS_EINVAL, "arrive/duration[%zu] invalid", i);
  return simulate(n, arrive, duration, footprint, mem_bytes, max_admitted,
                  max_bypass == 0 ? 8 : max_bypass, admit_out, done_out, peak_bytes);
}
