// Internal state of a context (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <set>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/xsec.h"
#include "kernel_args.h"

namespace xs {

struct Scratch {
  void* ptr = nullptr;
  size_t cap = 0;
};

struct LinesRes {
  LinesDev dev{};
  SpeciesDev sp{};
  void* base = nullptr;     // one device allocation holding every array
  size_t bytes = 0;
  size_t n = 0;
  std::atomic<int> refs{0}; // pending serving requests and live graphs
  std::vector<double> q_T_host, q_val_host;
  std::vector<double> sample;   // nu0 of every kSampleStride-th line (host index)
};

constexpr int64_t kSampleStride = 1024;
// Longest line range of one work item of a served request (its default split keeps items
// at or under it, so that a new request's kernels find free wavefront slots quickly).
constexpr int64_t kServeItemLines = 4096;

struct GridRes {
  double* d = nullptr;
  size_t n = 0;
  size_t bytes = 0;
  double first = 0.0, last = 0.0;   // host copies of the end points
  std::vector<double> host;         // host copy of the grid
  std::atomic<int> refs{0};         // pending serving requests and live graphs
};

struct Plan {
  int P = 4;               // grid points per lane (tile = 64 P points)
  int split = 1;           // line splits per tile
  int W = 0;               // occupancy target of the tile kernel (0, 3 or 4 waves/SIMD)
  int64_t n_tiles = 0;
  int group = 1;           // tiles per work item (kGroup: grouped far field)
  int64_t n_units = 0;     // units of the issue order: tiles, or groups of `group` tiles
  int64_t rec_lo = 0;      // lines [rec_lo, rec_lo + rec_n) can reach the grid
  int64_t rec_n = 0;
  int npts = 0;
  int pt_batch = 1;        // (P, T) points per parameter/tile launch pair
  std::vector<int> tile_order;   // units by decreasing estimated work
  std::vector<int64_t> tile_cost;  // sampled line count in each unit's window (x 1024)
  bool tuned = false;              // launch shape from the tuning cache
  double select_eps = 0.0;         // main-contributor selection (0: off)
  // line records [pt_batch][rec_n] (32 B), then with selection the thresholds of the
  // groups of kSelGroup tiles [pt_batch][n_groups()] (8 B)
  int64_t n_groups() const { return (n_tiles + kSelGroup - 1) / kSelGroup; }
  size_t tau_offset() const { return (size_t)rec_n * pt_batch * 32; }
  size_t rec_bytes() const {
    return tau_offset() + (select_eps > 0.0 ? (size_t)pt_batch * n_groups() * 8 : 0);
  }
  size_t part_bytes(size_t n_grid) const {
    return split > 1 ? (size_t)pt_batch * split * n_grid * sizeof(double) : 0;
  }
};

struct Server;  // serving loop (serve.hip)

// HIP event pairs around tile-kernel launches (events are reused across periods).
struct KernelTimer {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  int record(hipStream_t st);   // records the next event on st
};

}  // namespace xs

struct xs_ctx {
  int device = 0;
  size_t budget = 0;
  std::atomic<size_t> used{0};
  int n_cu = 0;
  size_t lds = 0;
  std::string arch;
  std::mutex mu;
  uint64_t next_handle = 1;
  std::unordered_map<uint64_t, xs::LinesRes*> lines;
  std::unordered_map<uint64_t, xs::GridRes*> grids;
  // scratch of xs_compute / xs_count_evals (single caller thread)
  xs::Scratch pts_buf, part_buf, out_buf, count_buf, rec_buf, order_buf;
  std::vector<int> order_host;           // content of order_buf
  void* pts_pinned = nullptr;
  size_t pts_pinned_cap = 0;
  std::vector<double> pts_host;          // content of pts_buf
  hipEvent_t pts_event = nullptr;        // recorded after the last launch reading scratch
  bool pts_event_valid = false;
  hipStream_t last_stream = nullptr;
  xs::Server* server = nullptr;
  std::mutex serve_mu;                   // guards starting the server
  xs::KernelTimer* timer = nullptr;      // non-null while kernel timing is enabled
  std::set<xs_graph*> graphs;            // live graphs (guarded by mu)
  void* noalloc_scratch = nullptr;       // this device's allocation-free scratch array
  std::string noalloc_error;             // why it is missing (nullptr above)

  bool reserve(size_t bytes);
  void release(size_t bytes);
  int dev_alloc(void** p, size_t bytes, const char* what);
  void dev_free(void* p, size_t bytes);
  int scratch(xs::Scratch& s, size_t bytes, const char* what);
  xs::LinesRes* find_lines(xs_lines_t h);
  xs::GridRes* find_grid(xs_grid_t h);
};

namespace xs {
using Ctx = xs_ctx;

extern thread_local std::string g_last_error;   // message of this thread's last failure
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int validate_opts(const xs_opts* o);
int validate_pts(const xs_pt* pts, size_t npts);
// Launch plan; cap_bytes bounds the records and partials of one batch of (P, T) points
// (0: min(64 GiB, a third of the free budget)); max_item_lines > 0 caps the line range
// of a work item when the split is automatic. The launch shape (P, split) depends only on
// the inputs, the options and max_item_lines, never on the memory left.
// items_per_slot > 0 sets the work items per resident wavefront slot of the automatic
// split (default 4). With pts_per_lane, split and waves_per_simd all 0 the shape comes
// from the tuning cache when it holds the workload's class.
Plan make_plan(Ctx& c, const LinesRes& L, const GridRes& G, size_t npts, const xs_opts& o,
               size_t cap_bytes = 0, int64_t max_item_lines = 0, int items_per_slot = 0);

// Lines [lo, hi) that can reach [first, last] within cut (from the sampled index; the
// range errs on the inclusive side).
void line_range_nu(const LinesRes& L, double first, double last, double cut, int64_t* lo,
                   int64_t* hi);
int upload_pts(Ctx& c, const xs_pt* pts, size_t npts, hipStream_t st);

// Tuning cache (tune.hip): launch shapes per workload class, process-wide.
// Occupancy target of the tile kernel for the option value w (0 automatic, 2 the
// compiler's own choice, 3..6 waves per SIMD); the returned 0 means no target. The
// automatic value is 5 on the FP32 path with up to 2 points per lane (measured fastest
// untuned on the mid and table workloads: 96 VGPRs with few spills; 6 waves cap the
// kernel at 80 VGPRs and spill in the far-line code) and the compiler's choice otherwise.
inline int waves_target(int w, int P, bool f64) {
  if (w == 0) return (!f64 && P <= 2) ? 5 : 0;
  return w == 2 ? 0 : w;
}
// The option value of a target (2 for none).
inline int waves_option(int target) { return target == 0 ? 2 : target; }

// A cached launch shape; W is an option value (2..6).
struct TuneVal {
  int P = 2, W = 5, ips = 4;
  double probe_ms = 0.0;
};
std::string tune_key(const Ctx& c, const LinesRes& L, const GridRes& G, size_t npts,
                     const xs_opts& o);
bool tune_get(const std::string& key, TuneVal* v);
void tune_put(const std::string& key, const TuneVal& v);
// Enqueue the whole path on `st`: per batch of (P, T) points the parameter kernel, the
// tile kernel and (split > 1) the fixed-order reduction; with counts != nullptr the count
// kernel instead of tile + reduction. out_dev holds rows of o.out_dtype elements.
int enqueue_path(const LinesRes& L, const GridRes& G, const xs_opts& o, const Plan& p,
                 const double* pts_dev, const int* order_dev, void* out_dev, void* rec_dev,
                 void* part_dev, hipStream_t st, unsigned long long* counts = nullptr,
                 KernelTimer* tm = nullptr);
// One step of the path for the batch of points [pt0, pt0 + nb): the parameter kernel
// (with_params), the tile kernel over positions [c0, c1) of the tile order (order_dev is
// required), and the fixed-order reduction of the batch (with_reduce, split > 1). The
// steps of one batch must run in this order.
int enqueue_step(const LinesRes& L, const GridRes& G, const xs_opts& o, const Plan& p,
                 const double* pts_dev, const int* order_dev, void* out_dev, void* rec_dev,
                 void* part_dev, hipStream_t st, int pt0, int nb, int64_t c0, int64_t c1,
                 bool with_params, bool with_reduce, unsigned long long* counts = nullptr,
                 KernelTimer* tm = nullptr);
// Upload the plan's tile order into the context buffer (skipped when unchanged).
int upload_order(Ctx& c, const Plan& p, hipStream_t st);

// Bytes of one sigma element for the output type of the options.
inline size_t out_elem_bytes(const xs_opts& o) {
  return o.out_dtype == XS_F32 ? sizeof(float) : sizeof(double);
}

inline void free_lines_res(Ctx& c, LinesRes* L) {
  c.dev_free(L->base, L->bytes);
  delete L;
}

void serve_shutdown(Ctx* c);
// Release the device resources of every graph of the context (xs_destroy).
void graphs_release_all(Ctx* c);

}  // namespace xs
