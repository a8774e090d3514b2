// Internal state of a context (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
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
  std::atomic<int> refs{0}; // pending serving requests
  std::vector<double> q_T_host, q_val_host;
};

struct GridRes {
  double* d = nullptr;
  size_t n = 0;
  size_t bytes = 0;
  std::atomic<int> refs{0};
};

struct Plan {
  int P = 4;               // grid points per lane (tile = 64 P points)
  int split = 1;           // line splits per tile
  int64_t n_tiles = 0;
  int64_t n_items = 0;
  int64_t n_wg = 0;
  int64_t per_xcd = 0;
  int64_t phys_wg = 0;
};

struct Server;  // serving loop (serve.hip)

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
  double* wc = nullptr;                  // Weideman coefficients on the device
  // scratch of xs_compute / xs_count_evals (single caller thread)
  xs::Scratch pts_buf, part_buf, out_buf, count_buf;
  void* pts_pinned = nullptr;
  size_t pts_pinned_cap = 0;
  std::vector<double> pts_host;          // content of pts_buf
  hipEvent_t pts_event = nullptr;        // recorded after the last launch reading scratch
  bool pts_event_valid = false;
  hipStream_t last_stream = nullptr;
  xs::Server* server = nullptr;

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

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
const double* host_weideman();
int validate_opts(const xs_opts* o);
int validate_pts(const xs_pt* pts, size_t npts);
Plan make_plan(const Ctx& c, size_t n_grid, size_t npts, const xs_opts& o, int64_t n_lines);
TileArgs make_args(const Ctx& c, const LinesRes& L, const GridRes& G, const xs_opts& o,
                   const Plan& p, const double* pts_dev, int npts);
int enqueue_compute(Ctx& c, const TileArgs& A0, const Plan& p, bool f64, double* out_dev,
                    double* part_dev, hipStream_t st);

inline void free_lines_res(Ctx& c, LinesRes* L) {
  c.dev_free(L->base, L->bytes);
  delete L;
}

void serve_shutdown(Ctx* c);

}  // namespace xs
