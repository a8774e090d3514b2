// Autotuner: launch shapes (points per lane = tile width, work items per wavefront slot =
// line range of one item, occupancy target) timed on probe blocks of the real workload,
// kept in a process-wide cache per workload class and persisted as JSON.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cctype>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/xsec.h"
#include "kernel_args.h"
#include "runtime_internal.h"

namespace xs {

namespace {

std::mutex g_tune_mu;
std::map<std::string, TuneVal> g_tune;

bool valid_val(const TuneVal& v) {
  return (v.P == 1 || v.P == 2 || v.P == 4 || v.P == 8) && v.W >= 2 && v.W <= 6 &&
         v.ips >= 1 && v.ips <= 64;
}

// ------------------------------------------------------------------ minimal JSON reader
// Enough for the cache file: objects, strings (with \" and \\ escapes), numbers, and
// nested values that are skipped.
struct Json {
  const char* p;
  const char* e;
  bool ok = true;

  void ws() {
    while (p < e && isspace((unsigned char)*p)) ++p;
  }
  bool eat(char c) {
    ws();
    if (p < e && *p == c) {
      ++p;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    ws();
    if (p >= e || *p != '"') return ok = false;
    ++p;
    std::string s;
    while (p < e && *p != '"') {
      if (*p == '\\') {
        ++p;
        if (p >= e) return ok = false;
      }
      s.push_back(*p++);
    }
    if (p >= e) return ok = false;
    ++p;
    if (out) *out = s;
    return true;
  }
  bool num(double* out) {
    ws();
    char* end = nullptr;
    const double v = strtod(p, &end);
    if (end == p || end > e) return ok = false;
    p = end;
    if (out) *out = v;
    return true;
  }
  bool skip() {   // any value
    ws();
    if (p >= e) return ok = false;
    if (*p == '"') return str(nullptr);
    if (*p == '{' || *p == '[') {
      const char close = *p == '{' ? '}' : ']';
      const bool obj = *p == '{';
      ++p;
      if (eat(close)) return true;
      do {
        if (obj && !(str(nullptr) && eat(':'))) return ok = false;
        if (!skip()) return false;
      } while (eat(','));
      return eat(close) || (ok = false);
    }
    if (!strncmp(p, "true", 4) || !strncmp(p, "null", 4)) {
      p += 4;
      return true;
    }
    if (!strncmp(p, "false", 5)) {
      p += 5;
      return true;
    }
    return num(nullptr);
  }
};

// Reads {"version": 1, "entries": {key: {"P": .., "W": .., "items_per_slot": ..,
// "probe_ms": ..}, ...}} into *out.
bool parse_cache(const std::string& text, std::map<std::string, TuneVal>* out) {
  Json j{text.data(), text.data() + text.size()};
  if (!j.eat('{')) return false;
  if (j.eat('}')) return true;
  do {
    std::string k;
    if (!j.str(&k) || !j.eat(':')) return false;
    if (k != "entries") {
      if (!j.skip()) return false;
      continue;
    }
    if (!j.eat('{')) return false;
    if (j.eat('}')) continue;
    do {
      std::string key;
      if (!j.str(&key) || !j.eat(':') || !j.eat('{')) return false;
      TuneVal v;
      bool hasP = false, hasW = false, hasI = false;
      if (!j.eat('}')) {
        do {
          std::string f;
          if (!j.str(&f) || !j.eat(':')) return false;
          double x = 0.0;
          if (f == "P" || f == "W" || f == "items_per_slot" || f == "probe_ms") {
            if (!j.num(&x)) return false;
            if (f == "P") v.P = (int)x, hasP = true;
            // (0 in files of an earlier version: no occupancy target, the option 2)
            if (f == "W") v.W = (int)x == 0 ? 2 : (int)x, hasW = true;
            if (f == "items_per_slot") v.ips = (int)x, hasI = true;
            if (f == "probe_ms") v.probe_ms = x;
          } else if (!j.skip()) {
            return false;
          }
        } while (j.eat(','));
        if (!j.eat('}')) return false;
      }
      if (!hasP || !hasW || !hasI || !valid_val(v)) return false;
      (*out)[key] = v;
    } while (j.eat(','));
    if (!j.eat('}')) return false;
  } while (j.eat(','));
  if (!j.eat('}')) return false;
  j.ws();
  return j.ok && j.p == j.e;
}

std::string escape(const std::string& s) {
  std::string o;
  for (char ch : s) {
    if (ch == '"' || ch == '\\') o.push_back('\\');
    o.push_back(ch);
  }
  return o;
}

}  // namespace

std::string tune_key(const Ctx& c, const LinesRes& L, const GridRes& G, size_t npts,
                     const xs_opts& o) {
  // line density: lines within the largest cut of the grid's middle point
  const double mid = G.host[G.n / 2];
  const std::vector<double>& sm = L.sample;
  const int64_t k = (int64_t)(std::upper_bound(sm.begin(), sm.end(), mid + o.cut_cm1) -
                              std::lower_bound(sm.begin(), sm.end(), mid - o.cut_cm1));
  const int dens = (int)lround(log2(((double)k + 0.5) * (double)kSampleStride));
  const char* pc = npts == 1 ? "p1" : npts <= 16 ? "p16" : "pmany";
  char buf[192];
  snprintf(buf, sizeof buf, "%s|cu%d|%s|%s|d%d|%s%s", c.arch.c_str(), c.n_cu,
           o.precision == XS_FP64 ? "fp64" : "fp32",
           o.cutoff_kind == XS_CUT_FIXED ? "fixed" : "fwhm", dens, pc,
           o.select_eps > 0.0 ? "|sel" : "");
  return buf;
}

bool tune_get(const std::string& key, TuneVal* v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *v = it->second;
  return true;
}

void tune_put(const std::string& key, const TuneVal& v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = v;
}

namespace {

struct Block {
  int64_t j0, j1;          // grid points [j0, j1), multiples of 512 except at the end
  int64_t rec_lo, rec_n;   // lines that can reach them
};

// Time one candidate shape over the probe blocks: per block the parameter kernel (not
// timed) and the tile kernel (timed with events on the launch stream; one warm-up run,
// then the fastest of three). A block too small to fill the device with the plan's split gets a
// larger one (at least one round of wavefront slots), so that every candidate is timed
// at full occupancy.
int time_candidate(Ctx& c, const LinesRes& L, const GridRes& G, const xs_opts& o,
                   const std::vector<Block>& blocks, int nprobe, const Plan& full,
                   KernelTimer& tm, double* ms_out) {
  // units of the order: tiles, or groups of full.group tiles (one workgroup each)
  const int64_t tile = (int64_t)kWave * full.P * full.group;
  const int64_t round_items = (int64_t)c.n_cu * 28 / full.group;
  double total = 0.0;
  for (const Block& b : blocks) {
    Plan p = full;
    p.rec_lo = b.rec_lo;
    p.rec_n = b.rec_n;
    p.npts = nprobe;
    p.pt_batch = nprobe;
    const int64_t t0 = b.j0 / tile, t1 = (b.j1 + tile - 1) / tile;
    const int64_t nt = t1 - t0;
    int64_t sp = std::max<int64_t>(p.split, (round_items + nt * nprobe - 1) / (nt * nprobe));
    const int64_t part_cap = std::max<int64_t>(
        1, (int64_t)((size_t)2 << 30) / ((int64_t)nprobe * (int64_t)G.n * 8));
    sp = std::min<int64_t>(sp, std::min<int64_t>(kMaxSplit, part_cap));
    p.split = (int)std::max<int64_t>(sp, 1);
    std::vector<int> order((size_t)nt);
    for (int64_t t = t0; t < t1; ++t) order[(size_t)(t - t0)] = (int)t;
    int rc = c.scratch(c.rec_buf, p.rec_bytes(), "tuning records");
    if (rc) return rc;
    void* part = nullptr;
    if (p.split > 1) {
      rc = c.scratch(c.part_buf, p.part_bytes(G.n), "tuning partials");
      if (rc) return rc;
      part = c.part_buf.ptr;
    }
    rc = c.scratch(c.out_buf, (size_t)nprobe * G.n * sizeof(double), "tuning output");
    if (rc) return rc;
    rc = c.scratch(c.order_buf, order.size() * sizeof(int), "tuning tile order");
    if (rc) return rc;
    c.order_host.clear();   // the buffer no longer holds a plan's order
    hipError_t e = hipMemcpy(c.order_buf.ptr, order.data(), order.size() * sizeof(int),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "tuning order upload");
    float best = 0.0f;
    for (int rep = 0; rep < 4; ++rep) {
      tm.used = 0;
      rc = enqueue_step(L, G, o, p, (const double*)c.pts_buf.ptr, (const int*)c.order_buf.ptr,
                        (double*)c.out_buf.ptr, c.rec_buf.ptr, part, nullptr, 0, nprobe, 0, nt,
                        true, false, nullptr, &tm);
      if (rc) return rc;
      e = hipEventSynchronize(tm.ev[1]);
      if (e != hipSuccess) return hip_fail(e, "tuning run");
      float ms = 0.0f;
      e = hipEventElapsedTime(&ms, tm.ev[0], tm.ev[1]);
      if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
      if (rep == 1 || (rep > 1 && ms < best)) best = ms;   // run 0 warms up
    }
    total += best;
  }
  *ms_out = total;
  return XS_OK;
}

}  // namespace

}  // namespace xs

using namespace xs;

int xs_tune_key(xs_ctx* c, xs_lines_t lh, xs_grid_t gh, size_t npts, const xs_opts* opts,
                char* key_out, size_t key_len) {
  if (!c || !key_out || key_len == 0) return fail(XS_EINVAL, "NULL argument");
  int rc = validate_opts(opts);
  if (rc) return rc;
  if (npts == 0) return fail(XS_EINVAL, "npts must be >= 1");
  LinesRes* L;
  GridRes* G;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    L = c->find_lines(lh);
    G = c->find_grid(gh);
  }
  if (!L || !G) return fail(XS_ENOTFOUND, "unknown line list or grid");
  const std::string k = tune_key(*c, *L, *G, npts, *opts);
  if (k.size() + 1 > key_len) return fail(XS_EINVAL, "key buffer too small (%zu)", key_len);
  memcpy(key_out, k.c_str(), k.size() + 1);
  return XS_OK;
}

int xs_autotune(xs_ctx* c, xs_lines_t lh, xs_grid_t gh, const xs_pt* pts, size_t npts,
                const xs_opts* opts, xs_tune_result* out) {
  if (!c || !out) return fail(XS_EINVAL, "NULL argument");
  int rc = validate_opts(opts);
  if (rc) return rc;
  rc = validate_pts(pts, npts);
  if (rc) return rc;
  LinesRes* L;
  GridRes* G;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    L = c->find_lines(lh);
    G = c->find_grid(gh);
  }
  if (!L || !G) return fail(XS_ENOTFOUND, "unknown line list or grid");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (c->pts_event_valid) {
    e = hipEventSynchronize(c->pts_event);   // scratch buffers are reused below
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  }
  const std::string key = tune_key(*c, *L, *G, npts, *opts);

  // probe points: up to five, evenly spaced over the batch (the first and last included),
  // so that a table's cheap and expensive points weigh in about as in the whole batch
  // (with three, one high-pressure point outweighed the rest of a pressure table)
  std::vector<xs_pt> pp;
  const size_t np = std::min<size_t>(npts, 5);
  for (size_t q = 0; q < np; ++q) pp.push_back(pts[np == 1 ? 0 : q * (npts - 1) / (np - 1)]);
  const int nprobe = (int)pp.size();
  rc = upload_pts(*c, pp.data(), pp.size(), nullptr);
  if (rc) return rc;

  // probe blocks: about 4e10 line-point visits in total (a few tens of ms), in up to
  // three blocks of whole 512-point units at 1/6, 1/2 and 5/6 of the grid; each block
  // (timed by a launch of its own) at least large enough that the widest tiles (4 x 64
  // points) fill one round of wavefront slots with a split of at most 16, so that no
  // candidate is timed on a starved device or with a split far from the one the whole
  // workload gets
  const double mid = G->host[G->n / 2];
  const std::vector<double>& sm = L->sample;
  const double dens =
      ((double)(std::upper_bound(sm.begin(), sm.end(), mid + opts->cut_cm1) -
                std::lower_bound(sm.begin(), sm.end(), mid - opts->cut_cm1)) +
       0.5) *
      (double)kSampleStride;
  const int64_t n = (int64_t)G->n;
  int64_t want = (int64_t)std::min(4e10 / (dens * nprobe), 9e15);
  const int64_t min_tiles = ((int64_t)c->n_cu * 28 + 16 * nprobe - 1) / (16 * nprobe);
  want = std::max<int64_t>(want, 3 * std::max<int64_t>(min_tiles * 4 * kWave, 512));
  std::vector<Block> blocks;
  if (2 * want >= n) {
    blocks.push_back({0, n, 0, 0});
  } else {
    const int64_t bl = (want / 3 + 511) / 512 * 512;
    for (double f : {1.0 / 6.0, 0.5, 5.0 / 6.0}) {
      int64_t j0 = ((int64_t)(f * (double)n) - bl / 2) / 512 * 512;
      j0 = std::max<int64_t>(0, std::min<int64_t>(j0, (n - bl) / 512 * 512));
      const int64_t j1 = std::min<int64_t>(n, j0 + bl);
      if (!blocks.empty() && j0 < blocks.back().j1) j0 = blocks.back().j1;
      if (j0 < j1) blocks.push_back({j0, j1, 0, 0});
    }
  }
  for (Block& b : blocks) {
    int64_t hi = 0;
    line_range_nu(*L, G->host[b.j0], G->host[b.j1 - 1], opts->cut_cm1, &b.rec_lo, &hi);
    b.rec_n = hi - b.rec_lo;
  }

  KernelTimer tm;
  auto cleanup = [&]() {
    for (hipEvent_t ev : tm.ev) (void)hipEventDestroy(ev);
  };
  struct Cand {
    int P, ips, W;   // W: option value (2..6)
    double ms;
  };
  // times (P, ips) with occupancy option W (0: the automatic one) and records it
  std::vector<Cand> tried;
  auto run = [&](int P, int ips, int W) -> int {
    xs_opts o = *opts;
    o.pts_per_lane = P;
    o.split = 0;
    o.waves_per_simd = W;
    const Plan full = make_plan(*c, *L, *G, npts, o, 0, 0, ips);
    double ms = 0.0;
    const int r = time_candidate(*c, *L, *G, o, blocks, nprobe, full, tm, &ms);
    if (r == XS_OK) tried.push_back({P, ips, waves_option(full.W), ms});
    return r;
  };
  rc = run(2, 4, 0);   // the untuned default
  if (rc) {
    cleanup();
    return rc;
  }
  const double def_ms = tried.front().ms;
  for (int P : {1, 2, 4})
    for (int ips : {1, 2, 4, 8, 16}) {
      if (P == 2 && ips == 4) continue;
      rc = run(P, ips, 0);
      if (rc) {
        cleanup();
        return rc;
      }
    }
  // the other occupancy options for the two fastest (P, items per slot)
  std::vector<Cand> top = tried;
  std::sort(top.begin(), top.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
  top.resize(std::min<size_t>(2, top.size()));
  for (const Cand& t : top)
    for (int W : {2, 3, 4, 5, 6}) {
      if (W == t.W) continue;
      rc = run(t.P, t.ips, W);
      if (rc) {
        cleanup();
        return rc;
      }
    }
  Cand best = tried.front();
  for (const Cand& t : tried)
    if (t.ms < best.ms) best = t;
  // keep the default unless a shape is clearly faster (probe timings vary by ~2 %)
  if (best.ms > 0.97 * def_ms) best = tried.front();
  cleanup();
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "tuning");
  TuneVal v;
  v.P = best.P;
  v.W = best.W;
  v.ips = best.ips;
  v.probe_ms = best.ms;
  tune_put(key, v);
  // the shape this workload now gets
  xs_opts o = *opts;
  o.pts_per_lane = 0;
  o.split = 0;
  o.waves_per_simd = 0;
  const Plan p = make_plan(*c, *L, *G, npts, o);
  memset(out, 0, sizeof *out);
  out->pts_per_lane = p.P;
  out->split = p.split;
  out->waves_per_simd = waves_option(p.W);
  out->items_per_slot = v.ips;
  out->probe_ms = best.ms;
  out->default_probe_ms = def_ms;
  out->candidates = (int)tried.size();
  snprintf(out->key, sizeof out->key, "%s", key.c_str());
  return XS_OK;
}

int xs_tune_cache_put(const char* key, int P, int W, int ips, double probe_ms) {
  if (!key || !*key) return fail(XS_EINVAL, "empty key");
  TuneVal v;
  v.P = P;
  v.W = W;
  v.ips = ips;
  v.probe_ms = probe_ms;
  if (!valid_val(v))
    return fail(XS_EINVAL, "invalid shape P=%d W=%d items_per_slot=%d", P, W, ips);
  tune_put(key, v);
  return XS_OK;
}

int xs_tune_cache_get(const char* key, int* P, int* W, int* ips, double* probe_ms) {
  if (!key) return fail(XS_EINVAL, "NULL key");
  TuneVal v;
  if (!tune_get(key, &v)) return fail(XS_ENOTFOUND, "no tuned shape for '%s'", key);
  if (P) *P = v.P;
  if (W) *W = v.W;
  if (ips) *ips = v.ips;
  if (probe_ms) *probe_ms = v.probe_ms;
  return XS_OK;
}

int xs_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return XS_OK;
}

int xs_tune_cache_size(size_t* n) {
  if (!n) return fail(XS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  *n = g_tune.size();
  return XS_OK;
}

int xs_tune_cache_load(const char* path) {
  if (!path) return fail(XS_EINVAL, "NULL path");
  FILE* f = fopen(path, "rb");
  if (!f) return fail(XS_ENOTFOUND, "cannot open %s", path);
  std::string text;
  char buf[4096];
  size_t r;
  while ((r = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, r);
  fclose(f);
  std::map<std::string, TuneVal> m;
  if (!parse_cache(text, &m)) return fail(XS_EINVAL, "%s is not a valid tuning cache", path);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& kv : m) g_tune[kv.first] = kv.second;
  return XS_OK;
}

int xs_tune_cache_save(const char* path) {
  if (!path) return fail(XS_EINVAL, "NULL path");
  std::string o = "{\n  \"version\": 1,\n  \"entries\": {";
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    bool first = true;
    for (auto& kv : g_tune) {
      char val[160];
      snprintf(val, sizeof val,
               "{\"P\": %d, \"W\": %d, \"items_per_slot\": %d, \"probe_ms\": %.6g}",
               kv.second.P, kv.second.W, kv.second.ips, kv.second.probe_ms);
      o += first ? "\n    \"" : ",\n    \"";
      o += escape(kv.first) + "\": " + val;
      first = false;
    }
  }
  o += "\n  }\n}\n";
  FILE* f = fopen(path, "wb");
  if (!f) return fail(XS_EINVAL, "cannot write %s", path);
  const bool ok = fwrite(o.data(), 1, o.size(), f) == o.size();
  if (fclose(f) != 0 || !ok) return fail(XS_EINVAL, "write to %s failed", path);
  return XS_OK;
}
