// Host runtime behind the C ABI of include/xsec.h: contexts, HBM budget, resident line
// lists and grids, argument validation, work planning, launches and hipGraph capture.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/xsec.h"
#include "kernel_args.h"
#include "runtime_internal.h"
#include "voigt.h"

namespace xs {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(XS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace xs

using xs::fail;

bool xs_ctx::reserve(size_t bytes) {
  size_t cur = used.load();
  do {
    if (cur + bytes > budget) return false;
  } while (!used.compare_exchange_weak(cur, cur + bytes));
  return true;
}

void xs_ctx::release(size_t bytes) { used.fetch_sub(bytes); }

int xs_ctx::dev_alloc(void** p, size_t bytes, const char* what) {
  if (bytes == 0) bytes = 256;
  if (!reserve(bytes))
    return fail(XS_ENOMEM, "%s: %zu bytes exceed the HBM budget (%zu of %zu in use)", what,
                bytes, used.load(), budget);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    release(bytes);
    (void)hipGetLastError();
    return fail(XS_ENOMEM, "%s: hipMalloc(%zu) failed: %s", what, bytes, hipGetErrorString(e));
  }
  return XS_OK;
}

void xs_ctx::dev_free(void* p, size_t bytes) {
  if (!p) return;
  if (bytes == 0) bytes = 256;
  (void)hipFree(p);
  release(bytes);
}

// Grow-only device scratch buffer.
int xs_ctx::scratch(xs::Scratch& s, size_t bytes, const char* what) {
  if (s.cap >= bytes && s.ptr) return XS_OK;
  if (s.ptr) dev_free(s.ptr, s.cap);
  s.ptr = nullptr;
  s.cap = 0;
  size_t want = std::max(bytes, (size_t)4096);
  int rc = dev_alloc(&s.ptr, want, what);
  if (rc) return rc;
  s.cap = want;
  return XS_OK;
}

xs::LinesRes* xs_ctx::find_lines(xs_lines_t h) {
  auto it = lines.find(h);
  return it == lines.end() ? nullptr : it->second;
}

xs::GridRes* xs_ctx::find_grid(xs_grid_t h) {
  auto it = grids.find(h);
  return it == grids.end() ? nullptr : it->second;
}

namespace xs {

// The error budget of a tolerance argument: kTolDefault for 0, else tol itself, which must
// lie in [kTolDefault, kTolMax].
static int tol_budget(double tol, float* eps) {
  if (tol == 0.0) {
    *eps = kTolDefault;
    return XS_OK;
  }
  const float t = (float)tol;   // the budget is compared in FP32, as the kernels use it
  if (!(t >= kTolDefault && t <= kTolMax))
    return fail(XS_EINVAL, "tol must be 0 or in [%g, %g] (got %g)", (double)kTolDefault,
                (double)kTolMax, tol);
  *eps = t;
  return XS_OK;
}

float opts_eps(const xs_opts& o) { return o.tol == 0.0 ? kTolDefault : (float)o.tol; }

int validate_opts(const xs_opts* o) {
  if (!o) return fail(XS_EINVAL, "opts is NULL");
  float eps;
  if (int rc = tol_budget(o->tol, &eps)) return rc;
  if (o->cutoff_kind != XS_CUT_FIXED && o->cutoff_kind != XS_CUT_MIN_FWHM)
    return fail(XS_EINVAL, "unknown cutoff_kind %d", o->cutoff_kind);
  if (!(o->cut_cm1 > 0.0) || !isfinite(o->cut_cm1))
    return fail(XS_EINVAL, "cut_cm1 must be finite and > 0 (got %g)", o->cut_cm1);
  if (o->cutoff_kind == XS_CUT_MIN_FWHM && (!(o->fwhm_mult > 0.0) || !isfinite(o->fwhm_mult)))
    return fail(XS_EINVAL, "fwhm_mult must be finite and > 0 (got %g)", o->fwhm_mult);
  if (o->precision != XS_FP32_KAHAN && o->precision != XS_FP64)
    return fail(XS_EINVAL, "unknown precision %d", o->precision);
  const int P = o->pts_per_lane;
  if (P != 0 && P != 1 && P != 2 && P != 4 && P != 8)
    return fail(XS_EINVAL, "pts_per_lane must be 0, 1, 2, 4 or 8 (got %d)", P);
  if (o->split < 0 || o->split > kMaxSplit)
    return fail(XS_EINVAL, "split must be in [0, %d] (got %d)", kMaxSplit, o->split);
  if (o->waves_per_simd != 0 && (o->waves_per_simd < 2 || o->waves_per_simd > 6))
    return fail(XS_EINVAL, "waves_per_simd must be 0 or 2..6 (got %d)", o->waves_per_simd);
  if (!(o->select_eps >= 0.0 && o->select_eps < 1.0))
    return fail(XS_EINVAL, "select_eps must be in [0, 1) (got %g)", o->select_eps);
  if (o->out_dtype != XS_F64 && o->out_dtype != XS_F32)
    return fail(XS_EINVAL, "unknown out_dtype %d", o->out_dtype);
  if (o->tile_group != 0 && o->tile_group != 1 && o->tile_group != kGroup)
    return fail(XS_EINVAL, "tile_group must be 0, 1 or %d (got %d)", kGroup, o->tile_group);
  if (o->tile_group == kGroup &&
      (o->precision != XS_FP32_KAHAN || o->cutoff_kind != XS_CUT_FIXED || o->select_eps > 0.0 ||
       o->pts_per_lane > 2))
    return fail(XS_EINVAL, "tile_group %d needs the FP32 path, a fixed cut, no selection and "
                           "at most 2 points per lane", kGroup);
  return XS_OK;
}

int validate_pts(const xs_pt* pts, size_t npts) {
  if (npts == 0) return fail(XS_EINVAL, "npts must be >= 1");
  if (!pts) return fail(XS_EINVAL, "pts is NULL");
  if (npts > (size_t)1 << 20) return fail(XS_EINVAL, "npts %zu too large", npts);
  for (size_t k = 0; k < npts; ++k) {
    if (!(pts[k].P_bar > 0.0) || !isfinite(pts[k].P_bar) || !(pts[k].T_K > 0.0) ||
        !isfinite(pts[k].T_K))
      return fail(XS_EINVAL, "pts[%zu] = (P %g bar, T %g K): both must be finite and > 0", k,
                  pts[k].P_bar, pts[k].T_K);
  }
  return XS_OK;
}

// Lines that can reach the grid: nu0 within the largest possible cut of its ends. The
// host index holds every kSampleStride-th centre, so the range is found to within a block
// and errs on the inclusive side.
void line_range_nu(const LinesRes& L, double first, double last, double cut, int64_t* lo,
                   int64_t* hi) {
  const int64_t n = (int64_t)L.n;
  const double reach = cut * (1.0 + 1e-9);
  const double klo = first - reach - fabs(first) * 1e-12;
  const double khi = last + reach + fabs(last) * 1e-12;
  const std::vector<double>& sm = L.sample;
  // largest sample index k with sm[k] < klo: lines before k * stride are all < klo
  int64_t k0 = (int64_t)(std::lower_bound(sm.begin(), sm.end(), klo) - sm.begin()) - 1;
  int64_t k1 = (int64_t)(std::upper_bound(sm.begin(), sm.end(), khi) - sm.begin());
  *lo = k0 < 0 ? 0 : std::min(n, k0 * kSampleStride);
  *hi = k1 >= (int64_t)sm.size() ? n : std::min(n, k1 * kSampleStride);
  if (*hi < *lo) *hi = *lo;
}

static void line_range(const LinesRes& L, const GridRes& G, const xs_opts& o, int64_t* lo,
                       int64_t* hi) {
  line_range_nu(L, G.first, G.last, o.cut_cm1, lo, hi);
}

Plan make_plan(Ctx& c, const LinesRes& L, const GridRes& G, size_t npts, const xs_opts& o,
               size_t cap_bytes, int64_t max_item_lines, int items_per_slot) {
  Plan p;
  p.P = o.pts_per_lane ? o.pts_per_lane : 2;
  p.select_eps = o.select_eps;
  const bool f64 = o.precision == XS_FP64;
  p.W = waves_target(o.waves_per_simd, p.P, f64);
  int ips = items_per_slot > 0 ? items_per_slot : 4;
  if (o.pts_per_lane == 0 && o.split == 0 && o.waves_per_simd == 0) {
    // fully automatic launch shape: the tuned one of this workload class, if any
    TuneVal tv;
    if (tune_get(tune_key(c, L, G, npts, o), &tv)) {
      p.P = tv.P;
      p.W = waves_target(tv.W, tv.P, f64);
      ips = tv.ips;
      p.tuned = true;
    }
  }
  const int64_t tile = (int64_t)kWave * p.P;
  p.n_tiles = ((int64_t)G.n + tile - 1) / tile;
  p.npts = (int)npts;
  // grouped far field: explicit, or automatic where lines far from a whole group of
  // kGroup tiles make up most of a tile's window (the cut spans at least 15 half-widths
  // of a group at the grid's middle)
  const bool can_group = !f64 && o.cutoff_kind == XS_CUT_FIXED && o.select_eps == 0.0 &&
                         p.P <= 2;
  if (o.tile_group == kGroup) {
    p.group = kGroup;
  } else if (o.tile_group == 0 && can_group && G.n >= 2) {
    const size_t m = std::min<size_t>(G.n / 2, G.n - 2);
    const double hv = 0.5 * (double)(kGroup * tile) * (G.host[m + 1] - G.host[m]);
    p.group = o.cut_cm1 >= 3.0 * (double)far_kappa(opts_eps(o)) * hv ? kGroup : 1;
  }
  const int64_t unit = tile * p.group;
  p.n_units = ((int64_t)G.n + unit - 1) / unit;
  int64_t hi = 0;
  line_range(L, G, o, &p.rec_lo, &hi);
  p.rec_n = hi - p.rec_lo;
  // line windows of the units (from the sampled index, within the largest cut)
  const std::vector<double>& sm = L.sample;
  std::vector<int64_t>& cost = p.tile_cost;
  cost.assign(p.n_units, 0);
  int64_t max_cost = 0;
  for (int64_t t = 0; t < p.n_units; ++t) {
    const int64_t j0 = t * unit, j1 = std::min<int64_t>(j0 + unit, (int64_t)G.n) - 1;
    const double lo = G.host[j0] - o.cut_cm1, hi = G.host[j1] + o.cut_cm1;
    cost[t] = (int64_t)(std::upper_bound(sm.begin(), sm.end(), hi) -
                        std::lower_bound(sm.begin(), sm.end(), lo));
    max_cost = std::max(max_cost, cost[t]);
  }
  const int64_t max_window = (max_cost + 1) * kSampleStride;   // lines, upper estimate
  if (o.split) {
    p.split = o.split;
  } else {
    // a few work items per resident wavefront slot (4 SIMDs x 7 waves per CU; 4 by
    // default, or the tuned count), so the last round of waves is short; a grouped item
    // occupies kGroup slots
    const int64_t base = p.n_units * (int64_t)npts;
    const int64_t target = (int64_t)c.n_cu * 28 * ips / p.group;
    int64_t sp = (target + base - 1) / base;
    sp = std::max<int64_t>(1, std::min<int64_t>(sp, 64));
    // and, if asked, no item longer than max_item_lines lines, so that no wave holds its
    // slot for long (kernels of other requests get slots quickly)
    if (max_item_lines > 0)
      sp = std::max<int64_t>(sp, (max_window + max_item_lines - 1) / max_item_lines);
    // no point in splits much shorter than one 64-line chunk per tile window
    sp = std::min<int64_t>(sp, std::max<int64_t>(1, max_window / 64));
    p.split = (int)std::min<int64_t>(sp, kMaxSplit);
  }
  // (P, T) points per batch: the records of a batch (32 B per line and point) and its
  // partials stay under a third of the free budget and 64 GiB (fewer, longer launches:
  // the tail of each tile launch, where the last work items run alone, is paid once
  // per batch)
  size_t cap = cap_bytes;
  if (cap == 0) {
    const size_t used = c.used.load();
    const size_t free_b = c.budget > used ? c.budget - used : 0;
    cap = std::min<size_t>((size_t)64 << 30, free_b / 3);
  }
  const size_t per_pt = std::max<size_t>(
      1, (size_t)p.rec_n * 32 + (p.split > 1 ? (size_t)p.split * G.n * 8 : 0) +
             (p.select_eps > 0.0 ? (size_t)p.n_groups() * 8 : 0));
  p.pt_batch = (int)std::max<size_t>(1, std::min<size_t>(npts, cap / per_pt));
  // issue order: tiles by decreasing number of lines within the largest cut, so the most
  // expensive work items start first
  // coarse cost classes (ratio 2^(1/4)) keep neighbouring tiles of similar cost together,
  // so that they still share their line windows in one XCD's L2
  std::vector<int> cls(p.n_units);
  for (int64_t t = 0; t < p.n_units; ++t)
    cls[t] = (int)std::floor(4.0 * std::log2(1.0 + (double)cost[t]));
  p.tile_order.resize(p.n_units);
  std::iota(p.tile_order.begin(), p.tile_order.end(), 0);
  std::stable_sort(p.tile_order.begin(), p.tile_order.end(),
                   [&](int a, int b) { return cls[a] > cls[b]; });
  return p;
}

int KernelTimer::record(hipStream_t st) {
  if (used == ev.size()) {
    hipEvent_t e = nullptr;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return hip_fail(r, "hipEventCreate");
    ev.push_back(e);
  }
  hipError_t r = hipEventRecord(ev[used], st);
  if (r != hipSuccess) return hip_fail(r, "hipEventRecord");
  ++used;
  return XS_OK;
}

int upload_order(Ctx& c, const Plan& p, hipStream_t st) {
  const size_t bytes = p.tile_order.size() * sizeof(int);
  if (c.order_host == p.tile_order && c.order_buf.ptr) return XS_OK;
  if (c.pts_event_valid) {
    hipError_t e = hipEventSynchronize(c.pts_event);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  }
  int rc = c.scratch(c.order_buf, bytes, "tile order");
  if (rc) return rc;
  hipError_t e = hipMemcpy(c.order_buf.ptr, p.tile_order.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "tile order upload");
  c.order_host = p.tile_order;
  (void)st;
  return XS_OK;
}

int enqueue_step(const LinesRes& L, const GridRes& G, const xs_opts& o, const Plan& p,
                 const double* pts_dev, const int* order_dev, void* out_dev, void* rec_dev,
                 void* part_dev, hipStream_t st, int pt0, int nb, int64_t c0, int64_t c1,
                 bool with_params, bool with_reduce, unsigned long long* counts,
                 KernelTimer* tm) {
  const bool f64 = o.precision == XS_FP64;
  CutDev cut;
  cut.kind = o.cutoff_kind == XS_CUT_FIXED ? kCutFixed : kCutMinFwhm;
  cut.cut = o.cut_cm1;
  cut.mult = o.fwhm_mult;
  hipError_t e;
  if (with_params) {
    ParamArgs PA;
    memset(&PA, 0, sizeof PA);
    PA.L = L.dev;
    PA.sp = L.sp;
    PA.cut = cut;
    PA.pts = pts_dev;
    PA.pt0 = pt0;
    PA.n_pt = nb;
    PA.lo = p.rec_lo;
    PA.n = p.rec_n;
    PA.out = (LineRec*)rec_dev;
    e = launch_params(PA, st);
    if (e != hipSuccess) return hip_fail(e, "parameter kernel launch");
    if (p.select_eps > 0.0) {
      // main-contributor selection: the thresholds of every tile group of the grid
      // (the tile launches of the batch, whatever their tile range, read them)
      TileArgs S;
      memset(&S, 0, sizeof S);
      S.L = L.dev;
      S.sp = L.sp;
      S.cut = cut;
      S.grid = G.d;
      S.n_grid = (int64_t)G.n;
      S.pts = pts_dev;
      S.pt0 = pt0;
      S.n_pt = nb;
      S.n_tiles = p.n_groups();
      S.recs = (const LineRec*)rec_dev;
      S.rec_lo = p.rec_lo;
      S.rec_n = p.rec_n;
      S.tau = (double*)((char*)rec_dev + p.tau_offset());
      S.tau_stride = p.n_groups();
      S.select_eps = p.select_eps;
      e = launch_select(S, p.P, st);
      if (e != hipSuccess) return hip_fail(e, "select kernel launch");
    }
  }
  if (c1 > c0) {
    TileArgs A;
    memset(&A, 0, sizeof A);
    A.L = L.dev;
    A.sp = L.sp;
    A.cut = cut;
    A.grid = G.d;
    A.n_grid = (int64_t)G.n;
    A.pts = pts_dev;
    A.pt0 = pt0;
    A.n_pt = nb;
    A.split = counts ? 1 : p.split;
    A.group = p.group;
    A.n_tiles = c1 - c0;
    A.n_items = A.n_tiles * nb * A.split;
    A.n_wg = p.group > 1 ? A.n_items : (A.n_items + kWavesPerWG - 1) / kWavesPerWG;
    A.tile_order = order_dev + c0;
    A.recs = (const LineRec*)rec_dev;
    A.rec_lo = p.rec_lo;
    A.rec_n = p.rec_n;
    A.l1_eps = opts_eps(o);
    A.far_kappa = far_kappa(A.l1_eps);
    if (p.select_eps > 0.0) {
      // main-contributor selection: the kernels drop the lines below their group's
      // threshold
      A.tau = (double*)((char*)rec_dev + p.tau_offset());
      A.tau_stride = p.n_groups();
    }
    const int64_t phys = phys_workgroups(A.n_wg);
    int rc = tm ? tm->record(st) : XS_OK;
    if (rc) return rc;
    if (counts) {
      A.counts = counts;
      e = launch_count(A, p.P, st, phys);
      if (e != hipSuccess) return hip_fail(e, "count kernel launch");
    } else {
      A.out = (A.split == 1) ? (double*)out_dev : (double*)part_dev;
      A.out_f32 = A.split == 1 && o.out_dtype == XS_F32;
      e = launch_tile(A, p.P, f64, p.W, st, phys);
      if (e != hipSuccess) return hip_fail(e, "tile kernel launch");
    }
    rc = tm ? tm->record(st) : XS_OK;
    if (rc) return rc;
  }
  if (with_reduce && !counts && p.split > 1) {
    e = launch_reduce((const double*)part_dev,
                      (char*)out_dev + (size_t)pt0 * G.n * out_elem_bytes(o),
                      o.out_dtype == XS_F32, (int64_t)G.n, nb, p.split, st);
    if (e != hipSuccess) return hip_fail(e, "reduce kernel launch");
  }
  return XS_OK;
}

int enqueue_path(const LinesRes& L, const GridRes& G, const xs_opts& o, const Plan& p,
                 const double* pts_dev, const int* order_dev, void* out_dev, void* rec_dev,
                 void* part_dev, hipStream_t st, unsigned long long* counts,
                 KernelTimer* tm) {
  for (int pt0 = 0; pt0 < p.npts; pt0 += p.pt_batch) {
    const int nb = std::min(p.pt_batch, p.npts - pt0);
    const int rc = enqueue_step(L, G, o, p, pts_dev, order_dev, out_dev, rec_dev, part_dev, st,
                                pt0, nb, 0, p.n_units, true, true, counts, tm);
    if (rc) return rc;
  }
  return XS_OK;
}

// Upload the (P, T) table into the context's device buffer, waiting first for the last
// launch that read it unless the content is unchanged.
int upload_pts(Ctx& c, const xs_pt* pts, size_t npts, hipStream_t st) {
  const size_t bytes = npts * 2 * sizeof(double);
  std::vector<double> h(2 * npts);
  for (size_t k = 0; k < npts; ++k) {
    h[2 * k] = pts[k].P_bar;
    h[2 * k + 1] = pts[k].T_K;
  }
  if (c.pts_host == h && c.pts_buf.ptr && c.pts_buf.cap >= bytes) return XS_OK;
  if (c.pts_event_valid) {
    hipError_t e = hipEventSynchronize(c.pts_event);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  }
  int rc = c.scratch(c.pts_buf, bytes, "point table");
  if (rc) return rc;
  if (c.pts_pinned_cap < bytes) {
    if (c.pts_pinned) (void)hipHostFree(c.pts_pinned);
    c.pts_pinned = nullptr;
    hipError_t e = hipHostMalloc(&c.pts_pinned, std::max(bytes, (size_t)4096), 0);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
    c.pts_pinned_cap = std::max(bytes, (size_t)4096);
  }
  memcpy(c.pts_pinned, h.data(), bytes);
  hipError_t e = hipMemcpyAsync(c.pts_buf.ptr, c.pts_pinned, bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "point table upload");
  c.pts_host = std::move(h);
  return XS_OK;
}

// Address of the allocation-free scratch array on `device` (the current device), taken
// once per device and kept for the process.
int noalloc_scratch_for(int device, void** out) {
  static std::mutex mu;
  static std::unordered_map<int, void*> addr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(device);
  if (it == addr.end()) {
    void* p = nullptr;
    const hipError_t e = noalloc_scratch_address(&p);
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    it = addr.emplace(device, p).first;
  }
  *out = it->second;
  return XS_OK;
}

}  // namespace xs

using namespace xs;

static_assert(XS_NOALLOC_SCRATCH_BYTES == kNoAllocScratchBytes,
              "allocation-free scratch size of the ABI and the kernels");

extern "C" {

int xs_abi_version(void) { return XS_ABI_VERSION; }

const char* xs_last_error(const xs_ctx*) { return g_last_error.c_str(); }

int xs_create(int device, size_t hbm_budget_bytes, xs_ctx** out) {
  if (!out) return fail(XS_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(XS_EDEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(XS_EINVAL, "device %d out of range", device);
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  size_t free_b = 0, total_b = 0;
  e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) return hip_fail(e, "hipMemGetInfo");
  Ctx* c = new Ctx();
  c->device = device;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
  c->n_cu = prop.multiProcessorCount;
  c->lds = prop.sharedMemPerBlock;
  c->arch = prop.gcnArchName;
  e = hipEventCreateWithFlags(&c->pts_event, hipEventDisableTiming);
  if (e != hipSuccess) {
    xs_destroy(c);
    return hip_fail(e, "hipEventCreate");
  }
  // the allocation-free entry point's scratch on this device (on failure only that entry
  // point is unavailable; it reports the reason)
  if (noalloc_scratch_for(device, &c->noalloc_scratch) != XS_OK) {
    c->noalloc_error = g_last_error;
    g_last_error.clear();
  }
  *out = c;
  return XS_OK;
}

void xs_destroy(xs_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  serve_shutdown(c);
  (void)hipDeviceSynchronize();
  graphs_release_all(c);
  for (auto& kv : c->lines) free_lines_res(*c, kv.second);
  for (auto& kv : c->grids) {
    c->dev_free(kv.second->d, kv.second->bytes);
    delete kv.second;
  }
  for (Scratch* s : {&c->pts_buf, &c->part_buf, &c->out_buf, &c->count_buf, &c->rec_buf,
                     &c->order_buf})
    if (s->ptr) c->dev_free(s->ptr, s->cap);
  if (c->pts_pinned) (void)hipHostFree(c->pts_pinned);
  if (c->pts_event) (void)hipEventDestroy(c->pts_event);
  if (c->timer) {
    for (hipEvent_t e : c->timer->ev) (void)hipEventDestroy(e);
    delete c->timer;
  }
  delete c;
}

int xs_set_kernel_timing(xs_ctx* c, int enable) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  if (enable && !c->timer) c->timer = new KernelTimer();
  if (c->timer) c->timer->used = 0;
  if (!enable && c->timer) {
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    for (hipEvent_t ev : c->timer->ev) {
      (void)hipEventSynchronize(ev);
      (void)hipEventDestroy(ev);
    }
    delete c->timer;
    c->timer = nullptr;
  }
  return XS_OK;
}

int xs_kernel_time(xs_ctx* c, double* ms_sum, int* n_launches) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  if (!c->timer) return fail(XS_EINVAL, "kernel timing is not enabled");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  KernelTimer& t = *c->timer;
  double sum = 0.0;
  for (size_t k = 0; k + 1 < t.used; k += 2) {
    e = hipEventSynchronize(t.ev[k + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, t.ev[k], t.ev[k + 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    sum += ms;
  }
  if (ms_sum) *ms_sum = sum;
  if (n_launches) *n_launches = (int)(t.used / 2);
  t.used = 0;
  return XS_OK;
}

int xs_device_info(xs_ctx* c, int* n_cu, size_t* lds_bytes, char* arch, size_t arch_len) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  if (n_cu) *n_cu = c->n_cu;
  if (lds_bytes) *lds_bytes = c->lds;
  if (arch && arch_len) {
    strncpy(arch, c->arch.c_str(), arch_len - 1);
    arch[arch_len - 1] = 0;
  }
  return XS_OK;
}

int xs_memory_used(xs_ctx* c, size_t* used, size_t* budget) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  if (used) *used = c->used.load();
  if (budget) *budget = c->budget;
  return XS_OK;
}

int xs_load_lines(xs_ctx* c, const xs_lines_desc* d, const xs_species_desc* sp, xs_lines_t* out) {
  if (!c || !d || !sp || !out) return fail(XS_EINVAL, "NULL argument");
  const size_t n = d->n;
  if (n > 0 && (!d->nu0 || !d->A_or_Sref || !d->E_low || !d->gamma_ref || !d->n_T || !d->g_up))
    return fail(XS_EINVAL, "line arrays must be non-NULL when n > 0");
  if (sp->strength_form != XS_EINSTEIN_A && sp->strength_form != XS_REF_STRENGTH)
    return fail(XS_EINVAL, "unknown strength_form %d", sp->strength_form);
  if (!(sp->mass_amu > 0.0) || !isfinite(sp->mass_amu))
    return fail(XS_EINVAL, "mass_amu must be finite and > 0");
  const double T_ref = sp->T_ref > 0 ? sp->T_ref : 296.0;
  const double P_ref = sp->P_ref > 0 ? sp->P_ref : 1.0;
  if (!isfinite(T_ref) || !isfinite(P_ref)) return fail(XS_EINVAL, "T_ref/P_ref not finite");
  if (sp->q_kind == XS_Q_POWER) {
    if (!(sp->q_a > 0.0) || !isfinite(sp->q_a) || !isfinite(sp->q_b))
      return fail(XS_EINVAL, "Q(T) = a T^b needs finite a > 0 and finite b");
  } else if (sp->q_kind == XS_Q_TABLE) {
    if (!sp->q_T || !sp->q_val || sp->q_n < 1)
      return fail(XS_EINVAL, "Q table needs q_T, q_val and q_n >= 1");
    for (size_t k = 0; k < sp->q_n; ++k) {
      if (!isfinite(sp->q_T[k]) || !(sp->q_val[k] > 0.0) || !isfinite(sp->q_val[k]))
        return fail(XS_EINVAL, "Q table node %zu invalid", k);
      if (k && !(sp->q_T[k] > sp->q_T[k - 1]))
        return fail(XS_EINVAL, "Q table temperatures must increase");
    }
  } else {
    return fail(XS_EINVAL, "unknown q_kind %d", sp->q_kind);
  }
  // broadening partners: mixing ratios and tables over J
  const int nb = sp->n_broad;
  const size_t nj = nb > 0 ? sp->broad_nj : 0;
  double bg_max = 0.0, bn_min = 0.0, bn_max = 0.0;
  if (nb < 0 || nb > 8) return fail(XS_EINVAL, "n_broad must be in [0, 8] (got %d)", nb);
  if (nb > 0) {
    if (nj < 1 || nj > 4096 || !sp->broad_vmr || !sp->broad_gamma || !sp->broad_n)
      return fail(XS_EINVAL, "broadening needs broad_vmr, broad_gamma, broad_n and "
                             "1 <= broad_nj <= 4096");
    for (int b = 0; b < nb; ++b) {
      if (!(sp->broad_vmr[b] >= 0.0) || !isfinite(sp->broad_vmr[b]))
        return fail(XS_EINVAL, "broad_vmr[%d] invalid", b);
      double gb = 0.0;
      for (size_t j = 0; j < nj; ++j) {
        const double g = sp->broad_gamma[b * nj + j], nn = sp->broad_n[b * nj + j];
        if (!(g >= 0.0) || !isfinite(g) || !isfinite(nn))
          return fail(XS_EINVAL, "broadening table %d entry %zu invalid", b, j);
        gb = std::max(gb, g);
        if (b == 0 && j == 0) bn_min = bn_max = nn;
        bn_min = std::min(bn_min, nn);
        bn_max = std::max(bn_max, nn);
      }
      bg_max += sp->broad_vmr[b] * gb;
    }
  }
  // validate records; find whether they are sorted
  bool sorted = true;
  double gmax = 0.0, nmin = 0.0, nmax = 0.0;
  for (size_t i = 0; i < n; ++i) {
    const double nu = d->nu0[i];
    const float A = d->A_or_Sref[i], E = d->E_low[i], g = d->gamma_ref[i], nt = d->n_T[i];
    if (!(nu > 0.0) || !isfinite(nu)) return fail(XS_EINVAL, "nu0[%zu] = %g invalid", i, nu);
    if (!(A >= 0.0f) || !isfinite(A)) return fail(XS_EINVAL, "A_or_Sref[%zu] invalid", i);
    if (!(E >= 0.0f) || !isfinite(E)) return fail(XS_EINVAL, "E_low[%zu] invalid", i);
    if (!(g >= 0.0f) || !isfinite(g)) return fail(XS_EINVAL, "gamma_ref[%zu] invalid", i);
    if (!isfinite(nt)) return fail(XS_EINVAL, "n_T[%zu] invalid", i);
    if (sp->strength_form == XS_EINSTEIN_A && d->g_up[i] == 0)
      return fail(XS_EINVAL, "g_up[%zu] = 0", i);
    if (i && nu < d->nu0[i - 1]) sorted = false;
    gmax = std::max(gmax, (double)g);
    if (i == 0) nmin = nmax = nt;
    nmin = std::min(nmin, (double)nt);
    nmax = std::max(nmax, (double)nt);
  }
  std::vector<size_t> order;
  if (!sorted) {
    order.resize(n);
    std::iota(order.begin(), order.end(), (size_t)0);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return d->nu0[a] < d->nu0[b]; });
  }
  LinesRes* L = new LinesRes();
  L->n = n;
  // one allocation, 256-byte aligned sub-arrays
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t b_nu = al(n * 8), b_f = al(n * 4), b_g = al(n * 2);
  const size_t qn = sp->q_kind == XS_Q_TABLE ? sp->q_n : 0;
  const size_t b_q = al(qn * 8);
  const bool has_j = nb > 0 && d->J_low;
  const size_t b_j = has_j ? b_g : 0;
  const size_t b_bv = al((size_t)nb * 8), b_bt = al((size_t)nb * nj * 8);
  L->bytes = b_nu + 4 * b_f + b_g + 2 * b_q + b_j + b_bv + 2 * b_bt;
  int rc = c->dev_alloc(&L->base, L->bytes, "line list");
  if (rc) {
    delete L;
    return rc;
  }
  char* p = (char*)L->base;
  double* nu_d = (double*)p; p += b_nu;
  float* A_d = (float*)p; p += b_f;
  float* E_d = (float*)p; p += b_f;
  float* g_d = (float*)p; p += b_f;
  float* n_d = (float*)p; p += b_f;
  uint16_t* u_d = (uint16_t*)p; p += b_g;
  double* qT_d = (double*)p; p += b_q;
  double* qV_d = (double*)p; p += b_q;
  uint16_t* j_d = (uint16_t*)p; p += b_j;
  double* bv_d = (double*)p; p += b_bv;
  double* bg_d = (double*)p; p += b_bt;
  double* bn_d = (double*)p;
  auto put = [&](void* dst, const void* src, size_t esz) -> hipError_t {
    if (n == 0) return hipSuccess;
    if (sorted) return hipMemcpy(dst, src, n * esz, hipMemcpyHostToDevice);
    std::vector<char> tmp(n * esz);
    const char* s = (const char*)src;
    for (size_t i = 0; i < n; ++i) memcpy(&tmp[i * esz], s + order[i] * esz, esz);
    return hipMemcpy(dst, tmp.data(), n * esz, hipMemcpyHostToDevice);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = put(nu_d, d->nu0, 8);
  if (e == hipSuccess) e = put(A_d, d->A_or_Sref, 4);
  if (e == hipSuccess) e = put(E_d, d->E_low, 4);
  if (e == hipSuccess) e = put(g_d, d->gamma_ref, 4);
  if (e == hipSuccess) e = put(n_d, d->n_T, 4);
  if (e == hipSuccess) e = put(u_d, d->g_up, 2);
  if (e == hipSuccess && qn) e = hipMemcpy(qT_d, sp->q_T, qn * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && qn) e = hipMemcpy(qV_d, sp->q_val, qn * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && has_j) e = put(j_d, d->J_low, 2);
  if (e == hipSuccess && nb > 0) {
    e = hipMemcpy(bv_d, sp->broad_vmr, (size_t)nb * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bg_d, sp->broad_gamma, nb * nj * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bn_d, sp->broad_n, nb * nj * 8, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    c->dev_free(L->base, L->bytes);
    delete L;
    return hip_fail(e, "line list upload");
  }
  L->dev.nu0 = nu_d;
  L->dev.A = A_d;
  L->dev.E = E_d;
  L->dev.gam = g_d;
  L->dev.nT = n_d;
  L->dev.g = u_d;
  L->dev.J = has_j ? j_d : nullptr;
  L->dev.n = (int64_t)n;
  L->sp.form = sp->strength_form == XS_EINSTEIN_A ? kEinstein : kReference;
  L->sp.q_kind = sp->q_kind == XS_Q_POWER ? kQPower : kQTable;
  L->sp.mass_amu = sp->mass_amu;
  L->sp.T_ref = T_ref;
  L->sp.P_ref = P_ref;
  L->sp.q_a = sp->q_a;
  L->sp.q_b = sp->q_b;
  L->sp.q_T = qn ? qT_d : nullptr;
  L->sp.q_val = qn ? qV_d : nullptr;
  L->sp.q_n = (int)qn;
  L->sp.n_broad = nb;
  L->sp.broad_nj = (int)nj;
  L->sp.broad_vmr = nb > 0 ? bv_d : nullptr;
  L->sp.broad_gam = nb > 0 ? bg_d : nullptr;
  L->sp.broad_n = nb > 0 ? bn_d : nullptr;
  // bounds of gamma_L for the per-tile cutoff bound: the lines' own gamma_ref and n_T, or
  // with partners sum_b vmr_b max_j gamma_b and the tables' range of n
  L->sp.gam_max = nb > 0 ? bg_max : gmax;
  L->sp.n_min = nb > 0 ? bn_min : nmin;
  L->sp.n_max = nb > 0 ? bn_max : nmax;
  // host index: every kSampleStride-th centre of the sorted list
  for (size_t i = 0; i < n; i += (size_t)kSampleStride)
    L->sample.push_back(sorted ? d->nu0[i] : d->nu0[order[i]]);
  // host copy of the species for host-side Q evaluation (tables on the host)
  L->q_T_host.assign(sp->q_T ? sp->q_T : nullptr, sp->q_T ? sp->q_T + qn : nullptr);
  L->q_val_host.assign(sp->q_val ? sp->q_val : nullptr, sp->q_val ? sp->q_val + qn : nullptr);
  std::lock_guard<std::mutex> lk(c->mu);
  const uint64_t h = c->next_handle++;
  c->lines[h] = L;
  *out = h;
  return XS_OK;
}

int xs_unload_lines(xs_ctx* c, xs_lines_t h) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  LinesRes* L = c->find_lines(h);
  if (!L) return fail(XS_ENOTFOUND, "unknown line list %llu", (unsigned long long)h);
  if (L->refs.load() > 0)
    return fail(XS_EBUSY, "line list %llu is referenced by %d pending request(s) or graph(s)",
                (unsigned long long)h, L->refs.load());
  c->lines.erase(h);
  (void)hipDeviceSynchronize();
  free_lines_res(*c, L);
  return XS_OK;
}

int xs_lines_info(xs_ctx* c, xs_lines_t h, size_t* n, size_t* bytes) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  LinesRes* L = c->find_lines(h);
  if (!L) return fail(XS_ENOTFOUND, "unknown line list %llu", (unsigned long long)h);
  if (n) *n = L->n;
  if (bytes) *bytes = L->bytes;
  return XS_OK;
}

int xs_set_grid(xs_ctx* c, const double* nu, size_t n, xs_grid_t* out) {
  if (!c || !out) return fail(XS_EINVAL, "NULL argument");
  if (n == 0 || !nu) return fail(XS_EINVAL, "grid needs n >= 1 points");
  if ((int64_t)n < 0) return fail(XS_EINVAL, "grid too large");
  for (size_t j = 0; j < n; ++j) {
    if (!isfinite(nu[j])) return fail(XS_EUNSORTED, "grid[%zu] is not finite", j);
    if (j && !(nu[j] > nu[j - 1]))
      return fail(XS_EUNSORTED, "grid is not strictly increasing at %zu", j);
  }
  GridRes* G = new GridRes();
  G->n = n;
  G->bytes = n * sizeof(double);
  G->first = nu[0];
  G->last = nu[n - 1];
  G->host.assign(nu, nu + n);
  int rc = c->dev_alloc((void**)&G->d, G->bytes, "grid");
  if (rc) {
    delete G;
    return rc;
  }
  hipError_t e = hipMemcpy(G->d, nu, G->bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    c->dev_free(G->d, G->bytes);
    delete G;
    return hip_fail(e, "grid upload");
  }
  std::lock_guard<std::mutex> lk(c->mu);
  const uint64_t h = c->next_handle++;
  c->grids[h] = G;
  *out = h;
  return XS_OK;
}

int xs_wavelength_grid_host(double lmin, double lmax, double R, double* nu_out, size_t cap,
                            size_t* n_out) {
  if (!n_out) return fail(XS_EINVAL, "NULL argument");
  if (!(lmin > 0.0) || !(lmax >= lmin) || !(R > 0.0) || !isfinite(lmax) || !isfinite(R))
    return fail(XS_EINVAL, "need 0 < lambda_min <= lambda_max and R > 0 (got %g, %g, %g)",
                lmin, lmax, R);
  // lambda_k = lambda_min exp(k log(1 + 1/R)): the last k with lambda_k <= lambda_max
  const double step = log1p(1.0 / R);
  const double kmax = floor(log(lmax / lmin) / step);
  if (!(kmax < 2147483647.0)) return fail(XS_EINVAL, "more than 2^31 grid points");
  size_t n = (size_t)kmax + 1;
  // rounding of the logarithms: keep exactly the points with lambda_k <= lambda_max
  while (n > 1 && lmin * exp((double)(n - 1) * step) > lmax) --n;
  while (lmin * exp((double)n * step) <= lmax) ++n;
  *n_out = n;
  if (!nu_out) return XS_OK;
  if (cap < n) return fail(XS_EINVAL, "nu_out holds %zu points, the grid has %zu", cap, n);
  for (size_t k = 0; k < n; ++k) nu_out[n - 1 - k] = 1e4 / (lmin * exp((double)k * step));
  return XS_OK;
}

int xs_set_grid_wavelength(xs_ctx* c, double lmin, double lmax, double R, xs_grid_t* out,
                           size_t* n_out) {
  if (!c || !out || !n_out) return fail(XS_EINVAL, "NULL argument");
  size_t n = 0;
  int rc = xs_wavelength_grid_host(lmin, lmax, R, nullptr, 0, &n);
  if (rc) return rc;
  std::vector<double> nu(n);
  rc = xs_wavelength_grid_host(lmin, lmax, R, nu.data(), n, &n);
  if (rc) return rc;
  rc = xs_set_grid(c, nu.data(), n, out);
  if (rc == XS_OK) *n_out = n;
  return rc;
}

int xs_free_grid(xs_ctx* c, xs_grid_t h) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  GridRes* G = c->find_grid(h);
  if (!G) return fail(XS_ENOTFOUND, "unknown grid %llu", (unsigned long long)h);
  if (G->refs.load() > 0)
    return fail(XS_EBUSY, "grid %llu is referenced by pending requests or graphs",
                (unsigned long long)h);
  c->grids.erase(h);
  (void)hipDeviceSynchronize();
  c->dev_free(G->d, G->bytes);
  delete G;
  return XS_OK;
}

int xs_grid_info(xs_ctx* c, xs_grid_t h, size_t* n) {
  if (!c || !n) return fail(XS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(c->mu);
  GridRes* G = c->find_grid(h);
  if (!G) return fail(XS_ENOTFOUND, "unknown grid %llu", (unsigned long long)h);
  *n = G->n;
  return XS_OK;
}

int xs_compute(xs_ctx* c, xs_lines_t lh, xs_grid_t gh, const xs_pt* pts, size_t npts,
               const xs_opts* opts, void* sigma_out, int out_on_device, void* stream) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  if (!sigma_out) return fail(XS_EINVAL, "sigma_out is NULL");
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
  if (!L) return fail(XS_ENOTFOUND, "unknown line list %llu", (unsigned long long)lh);
  if (!G) return fail(XS_ENOTFOUND, "unknown grid %llu", (unsigned long long)gh);
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (c->pts_event_valid && st != c->last_stream) {
    // scratch buffers are reused: order this call after the previous one
    e = hipEventSynchronize(c->pts_event);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  }
  const Plan p = make_plan(*c, *L, *G, npts, *opts);
  rc = upload_pts(*c, pts, npts, st);
  if (rc) return rc;
  const size_t out_bytes = npts * G->n * out_elem_bytes(*opts);
  rc = c->scratch(c->rec_buf, p.rec_bytes(), "line records");
  if (rc) return rc;
  void* part = nullptr;
  if (p.split > 1) {
    rc = c->scratch(c->part_buf, p.part_bytes(G->n), "split partials");
    if (rc) return rc;
    part = c->part_buf.ptr;
  }
  void* out_dev = sigma_out;
  if (!out_on_device) {
    rc = c->scratch(c->out_buf, out_bytes, "output staging");
    if (rc) return rc;
    out_dev = c->out_buf.ptr;
  }
  rc = upload_order(*c, p, st);
  if (rc) return rc;
  rc = enqueue_path(*L, *G, *opts, p, (const double*)c->pts_buf.ptr,
                    (const int*)c->order_buf.ptr, out_dev, c->rec_buf.ptr, part, st, nullptr,
                    c->timer);
  if (rc) return rc;
  e = hipEventRecord(c->pts_event, st);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  c->pts_event_valid = true;
  c->last_stream = st;
  if (!out_on_device) {
    e = hipMemcpyAsync(sigma_out, out_dev, out_bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "result download");
  }
  return XS_OK;
}

int xs_compute_noalloc(xs_ctx* c, xs_lines_t lh, xs_grid_t gh, const xs_pt* pts, size_t npts,
                       const xs_opts* opts, void* sigma_dev, void* stream) {
  if (!c) return fail(XS_EINVAL, "ctx is NULL");
  if (!sigma_dev) return fail(XS_EINVAL, "sigma_dev is NULL");
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
  if (!L) return fail(XS_ENOTFOUND, "unknown line list %llu", (unsigned long long)lh);
  if (!G) return fail(XS_ENOTFOUND, "unknown grid %llu", (unsigned long long)gh);
  if (!c->noalloc_scratch)
    return fail(XS_EDEVICE, "no scratch array on this device: %s", c->noalloc_error.c_str());
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  // scratch layout: point table | line records (and selection thresholds) | partials
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t pts_area = al(npts * 2 * sizeof(double));
  if (pts_area >= kNoAllocScratchBytes)
    return fail(XS_ENOMEM, "%zu P-T points exceed the scratch of %zu bytes", npts,
                kNoAllocScratchBytes);
  const Plan p = make_plan(*c, *L, *G, npts, *opts, kNoAllocScratchBytes - pts_area);
  const size_t rec_area = al(p.rec_bytes());
  const size_t need = pts_area + rec_area + p.part_bytes(G->n);
  if (need > kNoAllocScratchBytes)
    return fail(XS_ENOMEM,
                "one P-T point needs %zu bytes of scratch (records of %lld lines, %d split "
                "partials of %zu grid points), more than the %zu bytes of the "
                "allocation-free scratch", need, (long long)p.rec_n, p.split, G->n,
                kNoAllocScratchBytes);
  char* base = (char*)c->noalloc_scratch;
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> pairs(2 * npts);
  for (size_t k = 0; k < npts; ++k) {
    pairs[2 * k] = pts[k].P_bar;
    pairs[2 * k + 1] = pts[k].T_K;
  }
  e = launch_fill_pts((double*)base, pairs.data(), (int64_t)npts, st);
  if (e != hipSuccess) return hip_fail(e, "point table fill");
  // tiles in ascending order (no order table to upload; results do not depend on it)
  return enqueue_path(*L, *G, *opts, p, (const double*)base, nullptr, sigma_dev,
                      base + pts_area, p.split > 1 ? base + pts_area + rec_area : nullptr, st);
}

static_assert(XS_N_EVAL_TIERS == kNEvalTiers, "evaluation tiers of the ABI and the kernels");

int xs_count_evals(xs_ctx* c, xs_lines_t lh, xs_grid_t gh, const xs_pt* pts, size_t npts,
                   const xs_opts* opts, uint64_t* counts_out) {
  if (!counts_out) return fail(XS_EINVAL, "NULL argument");
  std::vector<uint64_t> t(npts * kNEvalTiers);
  const int rc = xs_count_evals_by_tier(c, lh, gh, pts, npts, opts, t.data());
  if (rc) return rc;
  for (size_t k = 0; k < npts; ++k) {
    uint64_t sum = 0;
    for (int j = 0; j < kNEvalTiers; ++j) sum += t[k * kNEvalTiers + j];
    counts_out[k] = sum;
  }
  return XS_OK;
}

int xs_count_evals_by_tier(xs_ctx* c, xs_lines_t lh, xs_grid_t gh, const xs_pt* pts,
                           size_t npts, const xs_opts* opts, uint64_t* counts_out) {
  if (!c || !counts_out) return fail(XS_EINVAL, "NULL argument");
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
  hipStream_t st = nullptr;
  if (c->pts_event_valid) {
    e = hipEventSynchronize(c->pts_event);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  }
  xs_opts o = *opts;
  o.split = 1;
  o.tile_group = 1;   // the count kernel walks single tiles
  const Plan p = make_plan(*c, *L, *G, npts, o);
  rc = upload_pts(*c, pts, npts, st);
  if (rc) return rc;
  const size_t ncnt = npts * kNEvalTiers;
  rc = c->scratch(c->count_buf, ncnt * sizeof(uint64_t), "counters");
  if (rc) return rc;
  rc = c->scratch(c->rec_buf, p.rec_bytes(), "line records");
  if (rc) return rc;
  e = launch_fill_u64((unsigned long long*)c->count_buf.ptr, (int64_t)ncnt, st);
  if (e != hipSuccess) return hip_fail(e, "counter clear");
  rc = upload_order(*c, p, st);
  if (rc) return rc;
  rc = enqueue_path(*L, *G, o, p, (const double*)c->pts_buf.ptr,
                    (const int*)c->order_buf.ptr, nullptr, c->rec_buf.ptr, nullptr, st,
                    (unsigned long long*)c->count_buf.ptr, c->timer);
  if (rc) return rc;
  e = hipMemcpyAsync(counts_out, c->count_buf.ptr, ncnt * sizeof(uint64_t),
                     hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "count download");
  e = hipEventRecord(c->pts_event, st);
  c->pts_event_valid = (e == hipSuccess);
  c->last_stream = st;
  return XS_OK;
}

struct xs_graph {
  xs_ctx* ctx = nullptr;       // nullptr once the context has been destroyed
  LinesRes* L = nullptr;       // referenced while the graph exists
  GridRes* G = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* pts = nullptr;
  size_t pts_bytes = 0;
  void* part = nullptr;
  size_t part_bytes = 0;
  void* rec = nullptr;
  size_t rec_bytes = 0;
  void* order = nullptr;
  size_t order_bytes = 0;
};

}  // extern "C"

namespace xs {
// Device resources of a graph (the struct itself stays with the caller's handle).
void graph_release(xs_graph* g) {
  xs_ctx* c = g->ctx;
  if (!c) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
  if (g->pts) c->dev_free(g->pts, g->pts_bytes);
  if (g->part) c->dev_free(g->part, g->part_bytes);
  if (g->rec) c->dev_free(g->rec, g->rec_bytes);
  if (g->order) c->dev_free(g->order, g->order_bytes);
  g->pts = g->part = g->rec = g->order = nullptr;
  if (g->L) g->L->refs.fetch_sub(1);
  if (g->G) g->G->refs.fetch_sub(1);
  g->L = nullptr;
  g->G = nullptr;
}

// xs_destroy: release every graph still alive; their handles only accept destroy.
void graphs_release_all(xs_ctx* c) {
  std::vector<xs_graph*> gs;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    gs.assign(c->graphs.begin(), c->graphs.end());
    c->graphs.clear();
  }
  for (xs_graph* g : gs) {
    graph_release(g);
    g->ctx = nullptr;
  }
}
}  // namespace xs

extern "C" {

int xs_graph_create(xs_ctx* c, xs_lines_t lh, xs_grid_t gh, const xs_pt* pts, size_t npts,
                    const xs_opts* opts, void* sigma_dev, xs_graph** out) {
  if (!c || !out || !sigma_dev) return fail(XS_EINVAL, "NULL argument");
  *out = nullptr;
  int rc = validate_opts(opts);
  if (rc) return rc;
  rc = validate_pts(pts, npts);
  if (rc) return rc;
  xs_graph* g = new xs_graph();
  g->ctx = c;
  {
    // the line list and grid stay referenced while the graph exists
    std::lock_guard<std::mutex> lk(c->mu);
    g->L = c->find_lines(lh);
    g->G = c->find_grid(gh);
    if (!g->L || !g->G) {
      delete g;
      return fail(XS_ENOTFOUND, "unknown line list or grid");
    }
    g->L->refs.fetch_add(1);
    g->G->refs.fetch_add(1);
  }
  LinesRes* L = g->L;
  GridRes* G = g->G;
  auto give_up = [&](int code) {
    graph_release(g);
    delete g;
    return code;
  };
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return give_up(hip_fail(e, "hipSetDevice"));
  const Plan p = make_plan(*c, *L, *G, npts, *opts);
  g->pts_bytes = npts * 2 * sizeof(double);
  rc = c->dev_alloc(&g->pts, g->pts_bytes, "graph point table");
  if (rc) return give_up(rc);
  std::vector<double> h(2 * npts);
  for (size_t k = 0; k < npts; ++k) {
    h[2 * k] = pts[k].P_bar;
    h[2 * k + 1] = pts[k].T_K;
  }
  e = hipMemcpy(g->pts, h.data(), g->pts_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return give_up(hip_fail(e, "graph point table upload"));
  if (p.split > 1) {
    g->part_bytes = p.part_bytes(G->n);
    rc = c->dev_alloc(&g->part, g->part_bytes, "graph partials");
    if (rc) return give_up(rc);
  }
  g->rec_bytes = p.rec_bytes();
  rc = c->dev_alloc(&g->rec, g->rec_bytes, "graph line records");
  if (rc) return give_up(rc);
  g->order_bytes = p.tile_order.size() * sizeof(int);
  rc = c->dev_alloc(&g->order, g->order_bytes, "graph tile order");
  if (rc) return give_up(rc);
  e = hipMemcpy(g->order, p.tile_order.data(), g->order_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return give_up(hip_fail(e, "graph tile order upload"));
  hipStream_t cs = nullptr;
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return give_up(hip_fail(e, "hipStreamCreate"));
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = enqueue_path(*L, *G, *opts, p, (const double*)g->pts, (const int*)g->order, sigma_dev,
                      g->rec, g->part, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
    if (rc == XS_OK && e2 != hipSuccess) rc = hip_fail(e2, "hipStreamEndCapture");
  } else {
    rc = hip_fail(e, "hipStreamBeginCapture");
  }
  (void)hipStreamDestroy(cs);
  if (rc == XS_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
  }
  if (rc) return give_up(rc);
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->graphs.insert(g);
  }
  *out = g;
  return XS_OK;
}

int xs_graph_launch(xs_graph* g, void* stream) {
  if (!g) return fail(XS_EINVAL, "graph is NULL");
  if (!g->ctx || !g->exec) return fail(XS_EINVAL, "the graph's context has been destroyed");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return XS_OK;
}

void xs_graph_destroy(xs_graph* g) {
  if (!g) return;
  if (xs_ctx* c = g->ctx) {
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    {
      std::lock_guard<std::mutex> lk(c->mu);
      c->graphs.erase(g);
    }
    graph_release(g);
  }
  delete g;
}

int xs_cia_regrid(xs_ctx* c, xs_grid_t gh, const size_t* off, size_t nb, const double* nu,
                  const double* alpha, double* out) {
  if (!c || !off || !out) return fail(XS_EINVAL, "NULL argument");
  if (nb == 0 || nb > (1u << 20)) return fail(XS_EINVAL, "n_blocks must be in [1, 2^20]");
  if (off[0] != 0) return fail(XS_EINVAL, "offsets[0] must be 0");
  for (size_t k = 0; k < nb; ++k)
    if (off[k + 1] < off[k]) return fail(XS_EINVAL, "offsets must not decrease (block %zu)", k);
  const size_t n_nodes = off[nb];
  if (n_nodes && (!nu || !alpha)) return fail(XS_EINVAL, "NULL node arrays");
  for (size_t k = 0; k < nb; ++k)
    for (size_t i = off[k]; i < off[k + 1]; ++i) {
      if (!isfinite(nu[i]) || !isfinite(alpha[i]))
        return fail(XS_EINVAL, "node %zu of block %zu not finite", i, k);
      if (i > off[k] && !(nu[i] > nu[i - 1]))
        return fail(XS_EINVAL, "block %zu: wavenumbers not increasing at node %zu", k, i);
    }
  GridRes* G;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    G = c->find_grid(gh);
  }
  if (!G) return fail(XS_ENOTFOUND, "unknown grid");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  const size_t b_off = ((nb + 1) * 8 + 255) & ~(size_t)255;
  const size_t b_nodes = (n_nodes * 8 + 255) & ~(size_t)255;
  const size_t b_out = (size_t)nb * G->n * 8;
  const size_t total = b_off + 2 * b_nodes + b_out;
  void* buf = nullptr;
  int rc = c->dev_alloc(&buf, total, "CIA buffers");
  if (rc) return rc;
  char* p = (char*)buf;
  int64_t* d_off = (int64_t*)p;
  double* d_nu = (double*)(p + b_off);
  double* d_al = (double*)(p + b_off + b_nodes);
  double* d_out = (double*)(p + b_off + 2 * b_nodes);
  std::vector<int64_t> o64(nb + 1);
  for (size_t k = 0; k <= nb; ++k) o64[k] = (int64_t)off[k];
  e = hipMemcpy(d_off, o64.data(), (nb + 1) * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && n_nodes) e = hipMemcpy(d_nu, nu, n_nodes * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && n_nodes) e = hipMemcpy(d_al, alpha, n_nodes * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = launch_cia(G->d, (int64_t)G->n, d_off, (int)nb, d_nu, d_al, d_out, nullptr);
  if (e == hipSuccess) e = hipMemcpy(out, d_out, b_out, hipMemcpyDeviceToHost);
  c->dev_free(buf, total);
  if (e != hipSuccess) return hip_fail(e, "CIA regrid");
  return XS_OK;
}

int xs_eval_voigt(xs_ctx* c, const double* x, const double* y, size_t n, int precision,
                  double* K_out) {
  if (!c || (n && (!x || !y || !K_out))) return fail(XS_EINVAL, "NULL argument");
  if (precision != XS_FP32_KAHAN && precision != XS_FP64)
    return fail(XS_EINVAL, "unknown precision %d", precision);
  if (n == 0) return XS_OK;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  void* buf = nullptr;
  const size_t b = n * sizeof(double);
  int rc = c->dev_alloc(&buf, 3 * b, "voigt evaluation buffers");
  if (rc) return rc;
  double* dx = (double*)buf;
  double* dy = dx + n;
  double* dk = dy + n;
  e = hipMemcpy(dx, x, b, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dy, y, b, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_eval_voigt(dx, dy, (int64_t)n, precision == XS_FP64, dk, nullptr);
  if (e == hipSuccess) e = hipMemcpy(K_out, dk, b, hipMemcpyDeviceToHost);
  c->dev_free(buf, 3 * b);
  if (e != hipSuccess) return hip_fail(e, "voigt evaluation");
  return XS_OK;
}

int xs_eval_voigt_host(const double* x, const double* y, size_t n, int precision, double* K_out) {
  if (n && (!x || !y || !K_out)) return fail(XS_EINVAL, "NULL argument");
  if (precision != XS_FP32_KAHAN && precision != XS_FP64)
    return fail(XS_EINVAL, "unknown precision %d", precision);
  for (size_t i = 0; i < n; ++i)
    K_out[i] = precision == XS_FP64 ? voigt_k64(x[i], y[i])
                                    : (double)voigt_k32(x[i], (float)y[i]);
  return XS_OK;
}

int xs_eval_bounds_host(const double* x, const double* y, size_t n, double* K_lo,
                        double* K_hi) {
  if (n && (!x || !y)) return fail(XS_EINVAL, "NULL argument");
  for (size_t i = 0; i < n; ++i) {
    if (!(y[i] > 0.0)) return fail(XS_EINVAL, "point %zu: y must be > 0 (got %g)", i, y[i]);
    if (K_lo) K_lo[i] = (double)voigt_lower((float)x[i], (float)y[i]);
    if (K_hi) K_hi[i] = (double)voigt_upper((float)x[i], (float)y[i]);
  }
  return XS_OK;
}

int xs_eval_series_host(const double* x, const double* y, size_t n, int variant, double tol,
                        double* K_out, int* variant_out) {
  if (n && (!x || !y || !K_out)) return fail(XS_EINVAL, "NULL argument");
  if (variant < -1 || variant >= kNVar) return fail(XS_EINVAL, "unknown variant %d", variant);
  float eps;
  if (int rc = tol_budget(tol, &eps)) return rc;
  for (size_t i = 0; i < n; ++i) {
    const float xf = (float)x[i], yf = (float)y[i];
    const float y2 = yf * yf;
    const float r2 = fmaf(xf, xf, y2);
    if (!(yf > 0.0f) || !(r2 >= kT6R2))
      return fail(XS_EINVAL, "point %zu (x %g, y %g) outside the series region", i, x[i], y[i]);
    const int v = variant < 0 ? asym_variant(y2, r2, eps) : variant;
    K_out[i] = (double)((float)kInvSqrtPi * yf * asym_scaled_v(v, y2, r2));
    if (variant_out) variant_out[i] = v;
  }
  return XS_OK;
}

int xs_eval_far_host(const double* X, const double* H, const double* y, const double* t,
                     size_t n, double tol, double* K_out, int* kind_out) {
  if (n && (!X || !H || !y || !t || !K_out)) return fail(XS_EINVAL, "NULL argument");
  float eps;
  if (int rc = tol_budget(tol, &eps)) return rc;
  const float kappa = far_kappa(eps);
  for (size_t i = 0; i < n; ++i) {
    const float xf = (float)X[i], hf = (float)H[i], yf = (float)y[i], tf = (float)t[i];
    const float y2 = yf * yf;
    const float xn = fabsf(xf) - hf;   // the nearest point of the tile
    const float r2n = fmaf(xn, xn, y2);
    if (!(yf > 0.0f) || !(hf >= 0.0f) || !(fabsf(tf) <= 1.0f) || !far_ok(xf, hf, kappa) ||
        !(xn >= 0.0f) || !dshift_ok(r2n, eps))
      return fail(XS_EINVAL, "case %zu (X %g, H %g, y %g, t %g) is not a far line", i, X[i],
                  H[i], y[i], t[i]);
    const bool ds = !shifted_lorentz_ok(y2, r2n, eps);
    float b[kFarDeg + 1];
    if (ds) far_coeffs_ds((float)kInvSqrtPi * yf, xf, hf, y2, b);
    else far_coeffs((float)kInvSqrtPi * yf, xf, hf, y2 - 1.5f, b);
    K_out[i] = (double)far_eval(b, tf);
    if (kind_out) kind_out[i] = ds ? 1 : 0;
  }
  return XS_OK;
}

}  // extern "C"
