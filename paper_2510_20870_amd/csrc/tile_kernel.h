// Device code of the tile kernel (template over points per lane, precision and occupancy
// target) and the helpers it shares with the count kernel; the instantiations live in
// tile_p1.hip .. tile_p8.hip so that they compile in parallel.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "kernel_args.h"
#include "physics.h"
#include "voigt.h"

namespace xs {


// exponent of the strongest line's FP32 scale: leaves 2^80 of headroom for sums and keeps
// the expanded two-term coefficient 2 y^2 c1 finite for y up to 8e7
constexpr int kScaleTarget = 48;
constexpr int kNoScale = -(1 << 28);

// ------------------------------------------------------------------ tile kernel
// Record of one staged line in LDS. cls holds 2 bits per row p of the wave's tile:
// 0 = no point of the row is inside the cut, 1 = general path, 2 / 3 = every point of the
// row is in the FP32 series region (|z| >= 7), the line lying left / right of the row; xr[p]
// is then x at the row's nearest end (first / last point) and info[p] = bnd | var << 8:
// the points inside the cut are the lanes < bnd (class 2) or >= bnd (class 3), found
// exactly at staging time, and var is the series variant the row's nearest point needs.
// y2 is y^2, except for lines of a shifted-Lorentzian series mode, where it is
// y^2 - 3/2 (their only use of it is the shifted r^2).
// For a general row (class 1) of the FP32 path, info[p] = lo | hi << 7 | a << 14 | n << 21
// holds the lanes inside the cut, [lo, hi), and the lanes of the FP64 core region
// (r^2 < 49), [a, a + n), found exactly at staging time with the same FP64 difference and
// FP32 r^2 as the per-point evaluation. The core points of all lines are evaluated packed
// across lines, one point per lane.
// The line's mode (kept outside the record: lines are grouped by mode) selects its
// hot-loop path: kSkip (no row inside the cut), kRows (per-row classes), or a series mode
// when the line lies on one side of the whole tile with every row of class 2 (or 3) or 0:
// then all rows take the series with the variant of the tile's nearest point, masked by
// the rows' lane bounds unless every point is inside the cut.
enum {
  kSkip = 0,
  kRows = 1,
  kSeries = 2,   // + side * 2 kNVar + masked * kNVar + variant
  kModes = kSeries + 4 * kNVar
};
__host__ __device__ constexpr int series_mode(int side, int masked, int var) {
  return kSeries + side * 2 * kNVar + masked * kNVar + var;
}

template <bool F64, int P> struct Rec;
template <int P> struct alignas(16) Rec<false, P> {
  double nu0, ib;
  float y, y2, sc;
  float c1, c2, c3;   // c1 = sc y / sqrt(pi); two-term series = u (c1 + u (c2 + u c3))
  float ib32;
  int cls;
  float xr[P];
  unsigned int info[P];
};
template <int P> struct alignas(16) Rec<true, P> {
  double nu0, cut, ib, y, sc;
  int cls;
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}

// Sum over the wavefront as a wave-uniform value: an inclusive scan with DPP (shifts by
// 1, 2, 4, 8 inside each row of 16 lanes, then the broadcasts of lane 15 and lane 31 into
// the rows above), whose last lane holds the total.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                           0, __builtin_bit_cast(int, v), kCtrl, kRowMask,
                                           0xf, false));
}
__device__ __forceinline__ float wave_total(float v) {
  v = dpp_add<0x111, 0xf>(v);   // row_shr:1
  v = dpp_add<0x112, 0xf>(v);   // row_shr:2
  v = dpp_add<0x114, 0xf>(v);   // row_shr:4
  v = dpp_add<0x118, 0xf>(v);   // row_shr:8
  v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Far lines of a chunk are summed as one polynomial over the tile (far_coeffs) when at
// least this many of its lines qualify (fewer cost less on the per-line walk).
constexpr int kFarMinLines = 16;
// Consecutive chunks of far lines only add their coefficients per lane for at most this
// many chunks before the sum over the wavefront (plain FP32 sums of terms of one sign:
// the lines of such a run all lie on one side of the tile).
constexpr int kFarRun = 8;

// Workgroups are dispatched round-robin over the 8 XCDs. Logical workgroups are grouped in
// blocks of kXcdBlock consecutive ones (neighbouring tiles, which share most of their line
// windows, so they reuse one XCD's L2), and the blocks are dealt round-robin to the XCDs,
// so every XCD gets a share of cheap and expensive tiles.
constexpr int64_t kXcdBlock = 16;
__device__ __forceinline__ int64_t xcd_logical_wg(int64_t phys) {
  const int64_t xcd = phys & 7, slot = phys >> 3;
  return (slot / kXcdBlock) * (8 * kXcdBlock) + xcd * kXcdBlock + (slot % kXcdBlock);
}

// First index i in [0, n) with a[i] >= key (n if none); LE selects a[i] > key instead.
// 64-ary search: every lane probes one position per level.
template <bool LE>
__device__ int64_t wave_search(const double* __restrict__ a, int64_t n, double key, int lane) {
  int64_t lo = 0, hi = n;   // the answer lies in [lo, hi]
  while (hi - lo > kWave) {
    const int64_t span = hi - lo;
    const int64_t idx = lo + span * (lane + 1) / (kWave + 1);
    const double v = a[idx];
    const bool before = LE ? (v <= key) : (v < key);
    const uint64_t mask = __ballot(before);
    const int c = __popcll(mask);
    const int64_t nlo = (c > 0) ? lo + span * c / (kWave + 1) + 1 : lo;
    const int64_t nhi = (c < kWave) ? lo + span * (c + 1) / (kWave + 1) : hi;
    lo = nlo;
    hi = nhi;
  }
  const int64_t idx = lo + lane;
  bool before = false;
  if (idx < hi) {
    const double v = a[idx];
    before = LE ? (v <= key) : (v < key);
  }
  return lo + __popcll(__ballot(before));
}

// First index i in [0, n) with pred(a[i]), for a predicate that is false and then true
// along the array (n if none): the same 64-ary search with the predicate in place of the
// comparison with a key.
template <class F>
__device__ int64_t wave_search_pred(const double* __restrict__ a, int64_t n, F pred,
                                    int lane) {
  int64_t lo = 0, hi = n;   // the answer lies in [lo, hi]
  while (hi - lo > kWave) {
    const int64_t span = hi - lo;
    const int64_t idx = lo + span * (lane + 1) / (kWave + 1);
    const uint64_t mask = __ballot(!pred(a[idx]));
    const int c = __popcll(mask);
    const int64_t nlo = (c > 0) ? lo + span * c / (kWave + 1) + 1 : lo;
    const int64_t nhi = (c < kWave) ? lo + span * (c + 1) / (kWave + 1) : hi;
    lo = nlo;
    hi = nhi;
  }
  const int64_t idx = lo + lane;
  bool before = false;
  if (idx < hi) before = !pred(a[idx]);
  return lo + __popcll(__ballot(before));
}

struct ItemInfo {
  int64_t j0;        // first grid index of the tile
  int64_t tile;      // the tile
  double nu_last;    // the tile's last grid value
  int k;             // (P, T) index within the batch
  int s;             // split index
  int64_t b, e;      // line range of this item (global line indices)
};

// Lines [lo, hi) whose cut can reach the grid range [nu_first, nu_last] at (P, T) point k
// of the batch: two 64-ary wave searches with the range's widest possible cut.
__device__ __forceinline__ void line_window(const TileArgs& A, int k, double nu_first,
                                           double nu_last, int lane, int64_t* lo,
                                           int64_t* hi) {
  const int pt = A.pt0 + k;
  const PtConst pc = make_pt(A.sp, A.pts[2 * pt], A.pts[2 * pt + 1]);
  const double cb = cut_bound(A.sp, pc, A.cut, nu_last);
  // widen the keys by a few ulps of nu so that rounding of nu -+ cb never drops a line
  const double lk = nu_first - cb - fabs(nu_first) * 0x1p-48;
  const double hk = nu_last + cb + fabs(nu_last) * 0x1p-48;
  // search inside the record range only (the host sized it to cover every tile)
  const double* base = A.L.nu0 + A.rec_lo;
  *lo = A.rec_lo + wave_search<false>(base, A.rec_n, lk, lane);
  *hi = A.rec_lo + wave_search<true>(base, A.rec_n, hk, lane);
}

// Main-contributor selection works on groups of kSelGroup neighbouring tiles (one
// threshold per group and (P, T) point): bounds of line i's contribution over the group's
// grid span [g_first, g_last]. Upper: at the span's point nearest to the line (zero when
// that point is outside the cut). Lower: at the farthest point, zero unless every point of
// the span is inside the cut (K falls with |x|, so these points bound it). The offsets and
// the cut tests are FP64, the bounds of K FP32 with margins, the scale FP64.
__device__ __forceinline__ double contrib_upper(double nu0, const LineRec& lr,
                                                double g_first, double g_last) {
  const double d = nu0 < g_first ? g_first - nu0 : nu0 > g_last ? nu0 - g_last : 0.0;
  if (d > lr.cut) return 0.0;
  return lr.sc * (double)voigt_upper((float)(d * lr.ib), (float)lr.y);
}
__device__ __forceinline__ double contrib_lower(double nu0, const LineRec& lr,
                                                double g_first, double g_last) {
  const double d = fmax(fabs(g_first - nu0), fabs(g_last - nu0));
  if (d > lr.cut) return 0.0;
  return lr.sc * (double)voigt_lower((float)(d * lr.ib), (float)lr.y);
}
// The grid span of the selection group of tile t (tiles of 64 P points).
template <int P>
__device__ __forceinline__ void sel_span(const TileArgs& A, int64_t t, double* g_first,
                                         double* g_last) {
  constexpr int64_t kSpan = (int64_t)kWave * P * kSelGroup;
  const int64_t j0 = (t / kSelGroup) * kSpan;
  *g_first = A.grid[j0];
  *g_last = A.grid[min(j0 + kSpan, A.n_grid) - 1];
}

// Far lines (FP32 path): a wave's tile of 64 P points from j0, over its valid points
// [g0, nu_last]: the first and last of them, half-width and centre offsets in FP32, and
// whether the tile's last row holds points (otherwise no line is a far line of it).
struct FarTile {
  double ra0, rbl;
  float h, ca, cb;   // half-width, centre - first point, centre - last point
  float eps, kappa;  // the launch's error budget and far threshold
  bool ok;
};
template <int P>
__device__ __forceinline__ FarTile far_tile(const TileArgs& A, int64_t j0, double nu_last) {
  FarTile t;
  const double g0 = A.grid[j0];
  const double nc = 0.5 * (g0 + nu_last);
  t.ra0 = g0;
  t.rbl = nu_last;
  t.h = (float)(0.5 * (nu_last - g0));
  t.ca = (float)(nc - g0);
  t.cb = (float)(nc - nu_last);
  t.eps = A.l1_eps;
  t.kappa = A.far_kappa;
  t.ok = j0 + (int64_t)kWave * (P - 1) < A.n_grid;
  return t;
}
// Whether a line (centre nu0, record lr) is a far line of the tile: the tests of stage_line
// and of the far split of the tile kernel's chunk loop, on the tile's first or last point:
// the whole tile inside the cut, the doubly shifted Lorentzian valid at the nearest point,
// far_ok at the centre; with x at the centre and H (Doppler units), and whether the line
// needs the doubly shifted expansion (ds: the shifted Lorentzian fails at the nearest
// point).
struct FarLine {
  bool far, ds;
  float x, h;
};
// (every test is evaluated and combined with &, so that the code has no branches)
__device__ __forceinline__ FarLine far_line(const FarTile& ft, double nu0, const LineRec& lr) {
  const double da = ft.ra0 - nu0, db = ft.rbl - nu0;
  const bool left = da > 0.0;
  const bool in_cut = left ? db <= lr.cut : ((db < 0.0) & (da >= -lr.cut));
  const float y = (float)lr.y;
  const float y2 = y * y;
  const float ib32 = (float)lr.ib;
  const float xn = (float)((left ? da : db) * lr.ib);
  const float r2n = fmaf(xn, xn, y2);
  const float h = ft.h * ib32;
  const float x = fmaf(ib32, left ? ft.ca : ft.cb, xn);
  const bool far = ft.ok & in_cut & dshift_ok(r2n, ft.eps) & far_ok(x, h, ft.kappa);
  const bool ds = far & !shifted_lorentz_ok(y2, r2n, ft.eps);
  return FarLine{far, ds, far ? x : 1.0f, far ? h : 0.0f};
}

template <int P>
__device__ __forceinline__ bool decode_item(const TileArgs& A, int lane, ItemInfo& it) {
  const int64_t phys = blockIdx.x;
  const int64_t wg = xcd_logical_wg(phys);
  // the wave index is wave-uniform; say so, so that everything derived from it is scalar
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t item = wg * kWavesPerWG + wave;
  if (wg >= A.n_wg || item >= A.n_items) return false;
  it.s = (int)(item % A.split);
  const int64_t r = item / A.split;
  it.k = (int)(r % A.n_pt);
  // tiles are issued in the order the host chose (most expensive first)
  const int64_t tile = A.tile_order ? (int64_t)A.tile_order[r / A.n_pt] : r / A.n_pt;
  it.j0 = tile * (int64_t)(kWave * P);
  const int64_t jl = min(it.j0 + (int64_t)(kWave * P), A.n_grid) - 1;
  it.tile = tile;
  it.nu_last = A.grid[jl];
  int64_t lo, hi;
  line_window(A, it.k, A.grid[it.j0], it.nu_last, lane, &lo, &hi);
  const int64_t cnt = hi > lo ? hi - lo : 0;
  it.b = lo + cnt * it.s / A.split;
  it.e = lo + cnt * (it.s + 1) / A.split;
  return true;
}

// Grouped far field (tile_group = kGroup): the kGroup wavefronts of a workgroup take
// kGroup neighbouring tiles of one (P, T) point and split. The group's grid span [ga, gb]
// (centre c, half-width hv) sets its line window for the fixed cut, and the window is cut
// by nu0 into five consecutive ranges: lines whose cut covers only part of the span, on
// the left [lo, i1); far lines on the left whose cut covers the whole span [i1, i2); lines
// near the span [i2, i3); far lines on the right that cover the span [i3, i4); lines that
// cover only part of it on the right [i4, hi). "Far" is a distance R from the centre,
// chosen from a bound of the window's Doppler widths so that every line beyond it meets
// the conditions of the tile polynomial for the whole span: |X| >= kappa H + 1.25 in the
// line's Doppler units (kappa = 4.09 at the default error budget), and the doubly shifted
// Lorentzian within its bound at the span's nearest point (which holds for every y
// there). The two far ranges are summed as one polynomial over the span, their chunks
// dealt to the wavefronts in turn; the other three ranges go through each wavefront's
// per-tile path (restricted to the lines that can reach its tile). The ranges depend on
// nu0 alone, so each line is taken exactly once. A split divides the group window for
// the far lines and each tile's own window for the per-tile path (so that every
// wavefront's share of the per-tile work sits at the same place in its window, and the
// wavefronts of a workgroup stay balanced).
struct GroupGeo {
  int64_t j_first;          // first grid index of the span
  double c, ihv;            // centre and 1 / half-width (0 for a one-point span)
  float hv32;               // half-width
  int64_t i1, i2, i3, i4;   // range boundaries (global line indices)
  int64_t fb, fe;           // this item's part of the group window (its far lines)
};

template <int P>
__device__ __forceinline__ bool decode_group(const TileArgs& A, int lane, int wave,
                                             ItemInfo& it, GroupGeo& gg) {
  const int64_t wg = xcd_logical_wg(blockIdx.x);
  if (wg >= A.n_items) return false;   // one work item per workgroup
  it.s = (int)(wg % A.split);
  const int64_t r = wg / A.split;
  it.k = (int)(r % A.n_pt);
  const int64_t unit = A.tile_order ? (int64_t)A.tile_order[r / A.n_pt] : r / A.n_pt;
  constexpr int64_t kTilePts = (int64_t)kWave * P;
  gg.j_first = unit * kGroup * kTilePts;
  const int64_t j_last = min(gg.j_first + kGroup * kTilePts, A.n_grid) - 1;
  it.tile = unit * kGroup + wave;
  it.j0 = it.tile * kTilePts;   // past the grid's end for the last group's spare waves
  it.nu_last = A.grid[min(it.j0 + kTilePts, A.n_grid) - 1];
  const double ga = A.grid[gg.j_first], gb = A.grid[j_last];
  gg.c = 0.5 * (ga + gb);
  const double hv = 0.5 * (gb - ga);
  gg.ihv = hv > 0.0 ? 1.0 / hv : 0.0;
  gg.hv32 = (float)hv;
  const double cut = A.cut.cut;
  const double* base = A.L.nu0 + A.rec_lo;
  const int64_t lo = wave_search<false>(base, A.rec_n, ga - cut - fabs(ga) * 0x1p-48, lane);
  const int64_t hi = wave_search<true>(base, A.rec_n, gb + cut + fabs(gb) * 0x1p-48, lane);
  // bound over the window: b_D <= kd (gb + cut)
  const int pt = A.pt0 + it.k;
  const PtConst pc = make_pt(A.sp, A.pts[2 * pt], A.pts[2 * pt + 1]);
  const double kd = pc.dopp / kCLight;
  const double bmax = kd * (gb + cut) * (1.0 + 1e-12);
  // the doubly shifted Lorentzian holds where r^4 >= (3/2) / eps, for any y; x^2 at
  // least that bound is enough
  const double x2 = sqrt(1.5 / (double)A.l1_eps);
  const double R = fmax((double)A.far_kappa * hv + (double)kFarMargin * bmax,
                        hv + sqrt(x2) * bmax) *
                   (1.0 + 1e-6);
  const double cl = gg.c - R, cr = gg.c + R;
  const double* w = base + lo;
  const int64_t n = hi - lo;
  const int64_t i1 = lo + wave_search_pred(w, n, [&](double v) { return gb - v <= cut; }, lane);
  int64_t i2 = lo + wave_search_pred(w, n, [&](double v) { return v >= cl; }, lane);
  int64_t i3 = lo + wave_search_pred(w, n, [&](double v) { return v > cr; }, lane);
  int64_t i4 = lo + wave_search_pred(w, n, [&](double v) { return v - ga > cut; }, lane);
  i2 = max(i2, i1);
  i3 = max(i2, min(i3, i4));
  i4 = max(i3, i4);
  gg.i1 = A.rec_lo + i1;
  gg.i2 = A.rec_lo + i2;
  gg.i3 = A.rec_lo + i3;
  gg.i4 = A.rec_lo + i4;
  const int64_t cnt = hi > lo ? hi - lo : 0;
  gg.fb = A.rec_lo + lo + cnt * it.s / A.split;
  gg.fe = A.rec_lo + lo + cnt * (it.s + 1) / A.split;
  // this wave's part of its own tile's window (none for a spare wave past the grid)
  it.b = it.e = 0;
  if (it.j0 < A.n_grid) {
    int64_t lo_t, hi_t;
    line_window(A, it.k, A.grid[it.j0], it.nu_last, lane, &lo_t, &hi_t);
    const int64_t ct = hi_t > lo_t ? hi_t - lo_t : 0;
    it.b = lo_t + ct * it.s / A.split;
    it.e = lo_t + ct * (it.s + 1) / A.split;
  }
  return true;
}

// Row bounds of a wave's tile: row p holds points j0 + 64p + lane; ra/rb are its first and
// last valid grid values (wave-uniform).
template <int P>
struct Rows {
  double ra[P], rb[P];
  double lanes_per_nu[P];   // last / (rb - ra): linear estimate of a lane from nu
  bool valid[P];
  int last[P];          // lane of the last valid point of the row
};

// First j in [lo, hi) with pred(j), for pred false then true over [lo, hi); hi if none.
template <class F>
__device__ __forceinline__ int first_true(int lo, int hi, F pred) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (pred(mid)) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// The same answer, starting from a guess: two probes around est settle it when the guess
// is within one lane (grids that are close to uniform over a row), else a binary search
// over the side the probes leave.
template <class F>
__device__ __forceinline__ int first_true_near(int lo, int hi, int est, F pred) {
  if (lo >= hi) return lo;
  est = min(max(est, lo), hi - 1);
  if (pred(est)) {
    if (est == lo || !pred(est - 1)) return est;
    return first_true(lo, est - 1, pred);   // pred(est - 1) holds
  }
  if (est + 1 == hi || pred(est + 1)) return est + 1;
  return first_true(est + 2, hi, pred);     // pred(est + 1) fails
}

// Lane guess for the first point with nu >= v in a row (linear in nu, clamped to a small
// range so that the conversion is always defined).
template <int P>
__device__ __forceinline__ int lane_guess(const Rows<P>& rows, int p, double v) {
  const double g = (v - rows.ra[p]) * rows.lanes_per_nu[p];
  return (int)ceil(fmin(fmax(g, -1.0), (double)kWave));
}


// Stages line i: the record (except the FP32 scales, set once the chunk's scale is known)
// with the row classes; returns the FP64 profile scale in *sc64, the line's mode in
// *mode_out and its number of core points (FP32 path) in *npairs_out. The lane ranges of
// general rows are found only when `general` is set (their lines are staged again later).
// recs_k: the line records of the item's (P, T) point, indexed by global line index.
template <bool F64, int P>
__device__ __forceinline__ Rec<F64, P> stage_line(const TileArgs& A, const LineRec* recs_k,
                                                  const Rows<P>& rows,
                                                  const double* rowv, int64_t i,
                                                  double* sc64, int* mode_out,
                                                  int* npairs_out, bool general) {
  const double nu0 = A.L.nu0[i];
  const LineRec lr = recs_k[i];
  Rec<F64, P> r;
  r.nu0 = nu0;
  if constexpr (F64) r.cut = lr.cut;
  r.ib = lr.ib;
  *sc64 = lr.sc;
  const float y = (float)lr.y;
  const float y2 = y * y;
  const double cut = lr.cut;
  int npairs = 0;
  // Classify each row with the same FP64 difference and test the per-point path uses;
  // the difference is monotone in nu_j, so the row's two ends decide for every point, and
  // searches over the row's grid values (rowv, LDS) find the cut and core boundaries.
  int cls = 0;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    int c = 0;
    float xr = 0.0f;
    unsigned int info = 0;
    if (rows.valid[p]) {
      const double da = rows.ra[p] - nu0, db = rows.rb[p] - nu0;
      const bool none = (da > cut) || (db < -cut);
      if (!none) {
        c = 1;
        const double* rv = rowv + kWave * p;
        const int n = rows.last[p] + 1;
        if (!F64 && (da > 0.0 || db < 0.0)) {
          const bool left = da > 0.0;   // the line lies left of the row
          const float x = (float)((left ? da : db) * lr.ib);
          const float r2n = fmaf(x, x, y2);
          if (r2n >= kFarR2) {
            c = left ? 2 : 3;
            xr = x;
            int bnd;
            if (left) {
              // lanes before the first one with nu - nu0 > cut (lane 0 is inside: da <= cut)
              bnd = db <= cut ? kWave
                    : first_true_near(1, n, lane_guess(rows, p, nu0 + cut),
                                      [&](int j) { return rv[j] - nu0 > cut; });
            } else {
              // the first lane with nu - nu0 >= -cut (the last lane is inside: db >= -cut)
              bnd = da >= -cut ? 0
                    : first_true_near(0, n - 1, lane_guess(rows, p, nu0 - cut),
                                      [&](int j) { return rv[j] - nu0 >= -cut; });
            }
            info = (unsigned)bnd | ((unsigned)asym_variant(y2, r2n, A.l1_eps) << 8);
          }
        }
        if (!F64 && c == 1 && general) {
          // general row: the lanes inside the cut and the core segment among them, from
          // linear guesses checked with the exact predicates
          const int lo = da >= -cut ? 0
                         : first_true_near(0, n, lane_guess(rows, p, nu0 - cut),
                                           [&](int j) { return rv[j] - nu0 >= -cut; });
          const int hi = db <= cut ? n
                         : first_true_near(lo, n, lane_guess(rows, p, nu0 + cut),
                                           [&](int j) { return rv[j] - nu0 > cut; });
          const int js = first_true_near(lo, hi, lane_guess(rows, p, nu0),
                                         [&](int j) { return rv[j] - nu0 >= 0.0; });
          auto core = [&](int j) {
            const float x = (float)((rv[j] - nu0) * lr.ib);
            return fmaf(x, x, y2) < kT6R2;
          };
          // the core reaches |x| = sqrt(49 - y^2), i.e. nu0 -+ b_D times that
          const double xc =
              (double)(sqrtf(fmaxf(49.0f - y2, 0.0f)) * rcp32((float)lr.ib));
          const int a = first_true_near(lo, js, lane_guess(rows, p, nu0 - xc), core);
          const int b = first_true_near(js, hi, lane_guess(rows, p, nu0 + xc),
                                        [&](int j) { return !core(j); });
          npairs += b - a;
          info = (unsigned)lo | ((unsigned)hi << 7) | ((unsigned)a << 14) |
                 ((unsigned)(b - a) << 21);
        }
      }
    }
    cls |= c << (2 * p);
    if constexpr (!F64) {
      r.xr[p] = xr;
      r.info[p] = info;
    }
  }
  int mode = cls == 0 ? kSkip : kRows;
  bool shifted = false;
  if constexpr (!F64) {
    // series modes: the line on one side of the whole tile, every row of that side's
    // series class or out of the cut (the rows out of the cut get an empty lane range);
    // the variant is that of the tile's point nearest to the line
    constexpr unsigned kOnes = (unsigned)(0x55555555u & ((1u << (2 * P)) - 1u));
    const unsigned uc = (unsigned)cls;
    // per row: class in {0, 2} (left) or {0, 3} (right)
    const bool left_ok = cls != 0 && ((uc & kOnes) == 0u);
    const bool right_ok = cls != 0 && ((uc & (uc >> 1) & kOnes) == ((uc | (uc >> 1)) & kOnes));
    if (left_ok || right_ok) {
      const int side = left_ok ? 0 : 1;
      bool full = true;
      int var = 0;   // the nearest row needs the most terms
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const int cp = (cls >> (2 * p)) & 3;
        if (cp == 0) r.info[p] = side ? (unsigned)kWave : 0u;
        else var = max(var, (int)(r.info[p] >> 8));
        const int bnd = (int)(r.info[p] & 255u);
        full = full && cp != 0 && bnd == (side ? 0 : kWave);
      }
      mode = series_mode(side, full ? 0 : 1, var);
      shifted = var == 0;
    }
  }
  r.cls = cls;
  *mode_out = mode;
  *npairs_out = npairs;
  if constexpr (F64) {
    r.y = lr.y;
    r.sc = lr.sc;
  } else {
    r.y = y;
    r.y2 = shifted ? y2 - 1.5f : y2;
    r.ib32 = (float)lr.ib;
    r.sc = 0.0f;
    r.c1 = r.c2 = r.c3 = 0.0f;
  }
  return r;
}

__device__ __forceinline__ void kahan_add(float& s, float& c, float v) {
  const float yk = v - c;
  const float t = s + yk;
  c = (t - s) - yk;
  s = t;
}

// The two-term series of a line, scaled: u (c1 + u (c2 + u c3)), u = 1/r^2.
template <int P>
__device__ __forceinline__ float two_term(const Rec<false, P>& q, float r2) {
  const float u = rcp32(r2);
  return u * fmaf(u, fmaf(u, q.c3, q.c2), q.c1);
}

// Adds the scaled contributions of one line to all P rows in the series region with NT
// terms, NT = 1 being the shifted Lorentzian (x from the row's nearer end, off = the lane's
// offsets from that end); with MASKED only the lanes inside the cut add: lanes < bnd
// (SIDE 0) or >= bnd (SIDE 1).
template <int P, int NT, int SIDE, bool MASKED>
__device__ __forceinline__ void series_add(const Rec<false, P>& q, const float (&off)[P],
                                           int lane, float (&t)[P]) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const float x = fmaf(off[p], q.ib32, q.xr[p]);
    const float r2 = fmaf(x, x, q.y2);
    float tn;
    if constexpr (NT == 1) {
      tn = fmaf(q.c1, rcp32(r2), t[p]);   // r2 holds x^2 + y^2 - 3/2 here
    } else if constexpr (NT == 2) {
      const float u = rcp32(r2);
      tn = fmaf(u, fmaf(u, fmaf(u, q.c3, q.c2), q.c1), t[p]);
    } else {
      tn = fmaf(q.c1, asym_scaled<NT>(q.y2, r2), t[p]);
    }
    if constexpr (MASKED) {
      const int bnd = __builtin_amdgcn_readfirstlane((int)q.info[p]) & 255;
      const bool in = SIDE == 0 ? lane < bnd : lane >= bnd;
      t[p] = in ? tn : t[p];
    } else {
      t[p] = tn;
    }
  }
}

// Scaled series value of one row with variant code `var` (wave-uniform) in a line of the
// general mode (y2 unshifted).
template <int P>
__device__ __forceinline__ float series_row(int var, const Rec<false, P>& q, float r2) {
  return var == 1 ? two_term(q, r2) : q.c1 * asym_scaled_v(var, q.y2, r2);
}

// Lines per plain FP32 partial sum before it enters the Kahan-compensated sum: the
// partial of at most kChunk positive terms carries a relative error below kChunk u32.
constexpr int kChunk = 16;

// W > 0 asks the compiler for at least W waves per SIMD (capping VGPRs at 512/W).
// SEL: main-contributor selection (a variant of its own, so that the kernel without it
// keeps its register allocation).
// GRP: the grouped far field (tile_group = kGroup; FP32 path without selection only).
template <int P, bool F64, int W, bool SEL, bool GRP = false>
__global__ __launch_bounds__(kBlock, (W > 0 ? W : 1)) void xs_tile_kernel(TileArgs A) {
  static_assert(!GRP || (!F64 && !SEL && P <= 2), "grouped far field: FP32, P <= 2");
  __shared__ Rec<F64, P> recs[kWavesPerWG][kWave];
  __shared__ double rowvals[kWavesPerWG][kWave * P];
  __shared__ int incl[kWavesPerWG][kWave];           // packed core points, inclusive prefix
  __shared__ int dlist[kWavesPerWG][F64 ? 1 : 2 * kWave];   // lines put aside (FP32 path)
  // packed core contributions: a pass holds the core points of whole lines, at most
  // kCoreQ (one line brings at most 64 P)
  constexpr int kCoreQ = kWave * P;
  __shared__ float cval[kWavesPerWG][F64 ? 1 : kCoreQ];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x >> 6;
  ItemInfo it;
  [[maybe_unused]] GroupGeo gg;
  // the exponents of the group's partial sums (one per wavefront)
  [[maybe_unused]] __shared__ int grp_e[GRP ? kGroup : 1];
  // the wave index is wave-uniform; say so, so that the tile and everything derived from
  // it stay scalar
  [[maybe_unused]] const int wvu = __builtin_amdgcn_readfirstlane(wv);
  if constexpr (GRP) {
    if (!decode_group<P>(A, lane, wvu, it, gg)) return;   // the whole workgroup
  } else {
    if (!decode_item<P>(A, lane, it)) return;
  }
  // a spare wave of the last group has no tile (its reads below use a valid index)
  const bool tile_ok = it.j0 < A.n_grid;
  const int64_t j0r = tile_ok ? it.j0 : A.n_grid - 1;
  // main-contributor selection: the drop threshold of the tile's group (0: every line is
  // kept)
  double tau = 0.0, g_first = 0.0, g_last = 0.0;
  if constexpr (SEL) {
    tau = A.tau[(int64_t)it.k * A.tau_stride + it.tile / kSelGroup];
    sel_span<P>(A, it.tile, &g_first, &g_last);
  }

  Rows<P> rows;
  double nu[P];
  float da32[P], db32[P];   // offsets of this lane's points from the row ends
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t ja = it.j0 + kWave * p;
    rows.valid[p] = ja < A.n_grid;
    const int64_t jb = min(ja + kWave - 1, A.n_grid - 1);
    rows.ra[p] = rows.valid[p] ? A.grid[ja] : 0.0;
    rows.rb[p] = rows.valid[p] ? A.grid[jb] : 0.0;
    rows.last[p] = rows.valid[p] ? (int)(jb - ja) : 0;
    rows.lanes_per_nu[p] =
        rows.last[p] > 0 ? (double)rows.last[p] / (rows.rb[p] - rows.ra[p]) : 0.0;
    const int64_t j = ja + lane;
    nu[p] = (j < A.n_grid) ? A.grid[j] : __builtin_nan("");
    da32[p] = (float)(nu[p] - rows.ra[p]);
    db32[p] = (float)(nu[p] - rows.rb[p]);
    rowvals[wv][kWave * p + lane] = nu[p];
  }
  wave_sync();
  // FP32 path: the tile's centre and half-width (over its valid points) for the far-line
  // polynomial; a point's coordinate t in [-1, 1] is da32 * f_ih + f_t0 of its row
  [[maybe_unused]] const FarTile ft = far_tile<P>(A, j0r, it.nu_last);
  [[maybe_unused]] float f_ih = 0.0f, f_t0[P];
  if constexpr (!F64) {
    const double g0 = A.grid[j0r];
    const double nc = 0.5 * (g0 + it.nu_last), h = 0.5 * (it.nu_last - g0);
    const double ih = h > 0.0 ? 1.0 / h : 0.0;
    f_ih = (float)ih;
#pragma unroll
    for (int p = 0; p < P; ++p) f_t0[p] = (float)((rows.ra[p] - nc) * ih);
  }
  using acc_t = typename std::conditional<F64, double, float>::type;
  acc_t s[P], c[P];
#pragma unroll
  for (int p = 0; p < P; ++p) { s[p] = 0; c[p] = 0; }
  int e_ref = kNoScale;   // FP32 path: contributions are scaled by 2^(kScaleTarget - e_ref)

  // FP32 path: the power-of-two scale of a staged chunk (every lane's line): a stronger
  // line than any before lowers the scale, and the running sums are rescaled exactly
  auto set_scale = [&](Rec<F64, P>& r, double sc64) {
    if constexpr (!F64) {
      // (the wavefront maximum only when some line is stronger than all before)
      const int exl = sc64 > 0.0 ? ilogb(sc64) : kNoScale;
      if (__ballot(exl > e_ref) != 0ull) {
        const int ex = wave_max(exl);
        const int d = max(e_ref - ex, -1000);
#pragma unroll
        for (int p = 0; p < P; ++p) {
          s[p] = ldexpf(s[p], d);
          c[p] = ldexpf(c[p], d);
        }
        e_ref = ex;
      }
      const double scd = ldexp(sc64, kScaleTarget - e_ref);
      r.sc = (float)scd;
      r.c1 = (float)(scd * (double)r.y * (double)kInvSqrtPi);
      r.c2 = 1.5f * r.c1;
      r.c3 = -2.0f * r.y2 * r.c1;
    }
  };
  // FP32 path: far lines (one per lane; c1 = 0 on the other lanes) summed as one
  // polynomial over the tile. far_add adds a line's coefficients to the lane's acc: those
  // of the shifted Lorentzian (far_coeffs), or, when ds is set (wave-uniform: some line of
  // the chunk needs it), those of the doubly shifted one (far_coeffs_ds), which hold for
  // every far line; y2 is y^2. far_flush sums acc over the wavefront, evaluates the
  // polynomial at the lane's points and adds it to the compensated sums.
  auto far_zero = [&](float (&acc)[kFarDeg + 1]) {
#pragma unroll
    for (int kk = 0; kk <= kFarDeg; ++kk) acc[kk] = 0.0f;
  };
  auto far_add = [&](float (&acc)[kFarDeg + 1], float c1, float x, float h, float y2,
                     bool ds) {
    if constexpr (!F64) {
      if (ds) {
        const FarRecD f = fard_start(c1, x, h, y2);
        float bm4 = f.b0, bm3 = f.b1, bm2 = f.b2, bm1 = f.b3;
        acc[0] += bm4;
        acc[1] += bm3;
        acc[2] += bm2;
        acc[3] += bm1;
#pragma unroll
        for (int kk = 4; kk <= kFarDeg; ++kk) {
          const float bk = fard_next(f, bm1, bm2, bm3, bm4);
          acc[kk] += bk;
          bm4 = bm3;
          bm3 = bm2;
          bm2 = bm1;
          bm1 = bk;
        }
      } else {
        const FarRec f = far_start(c1, x, h, y2 - 1.5f);
        float bm2 = f.b0, bm1 = f.b1;
        acc[0] += bm2;
        acc[1] += bm1;
#pragma unroll
        for (int kk = 2; kk <= kFarDeg; ++kk) {
          const float bk = far_next(f, bm1, bm2);
          acc[kk] += bk;
          bm2 = bm1;
          bm1 = bk;
        }
      }
    }
  };
  auto far_flush = [&](const float (&acc)[kFarDeg + 1]) {
    if constexpr (!F64) {
      float B[kFarDeg + 1];
#pragma unroll
      for (int kk = 0; kk <= kFarDeg; ++kk) B[kk] = wave_total(acc[kk]);
#pragma unroll
      for (int p = 0; p < P; ++p)
        kahan_add(s[p], c[p], far_eval(B, fmaf(da32[p], f_ih, f_t0[p])));
    }
  };
  auto far_sum = [&](float c1, float x, float h, float y2, bool ds) {
    float acc[kFarDeg + 1];
    far_zero(acc);
    far_add(acc, c1, x, h, y2, ds);
    far_flush(acc);
  };
  // Whether line j is a far line of the tile (far_line); also its x at the centre, H, y,
  // FP64 scale and whether it needs the doubly shifted expansion.
  // the line records of the item's (P, T) point, indexed by global line index (one base
  // for every record load, which keeps the loop-invariant scalars of the line loops few)
  const LineRec* const recs_k = A.recs + ((int64_t)it.k * A.rec_n - A.rec_lo);
  // end of the line range being walked (the item's, or one of a group's ranges)
  int64_t e_cur = it.e;
  auto far_line_j = [&](int64_t j, float& fx, float& fh, float& y, double& sc,
                        bool& ds) -> bool {
    const double nu0 = A.L.nu0[j];
    const LineRec lr = recs_k[j];
    y = (float)lr.y;
    sc = lr.sc;
    const FarLine f = far_line(ft, nu0, lr);
    if (f.far) {
      fx = f.x;
      fh = f.h;
    }
    ds = f.ds;
    return f.far;
  };
  // FP32 path without selection: a run of chunks of far lines only, from base on (left at
  // the first chunk that holds another line); each adds its lines' coefficients per lane,
  // summed over the wavefront every kFarRun chunks. The scale update is set_scale's, with
  // the pending coefficients rescaled like the sums.
  auto far_run = [&](int64_t& b) {
    if constexpr (!F64 && !SEL) {
      if (!ft.ok) return;
      float acc[kFarDeg + 1];
      far_zero(acc);
      int nrun = 0;
      while (b < e_cur) {
        const int64_t j = b + lane;
        float fx0 = 1.0f, fh0 = 0.0f, y = 0.0f;
        double sc = 0.0;
        bool ds = false;
        const bool is_far = j >= e_cur || far_line_j(j, fx0, fh0, y, sc, ds);
        if (__ballot(!is_far) != 0ull) break;
        const int exl = sc > 0.0 ? ilogb(sc) : kNoScale;
        if (__ballot(exl > e_ref) != 0ull) {
          const int ex = wave_max(exl);
          const int d = max(e_ref - ex, -1000);
#pragma unroll
          for (int p = 0; p < P; ++p) {
            s[p] = ldexpf(s[p], d);
            c[p] = ldexpf(c[p], d);
          }
#pragma unroll
          for (int kk = 0; kk <= kFarDeg; ++kk) acc[kk] = ldexpf(acc[kk], d);
          e_ref = ex;
        }
        const double scd = ldexp(sc, kScaleTarget - e_ref);
        const float c1 = j < e_cur ? (float)(scd * (double)y * (double)kInvSqrtPi) : 0.0f;
        far_add(acc, c1, fx0, fh0, j < e_cur ? y * y : 0.0f, __ballot(ds) != 0ull);
        b += kWave;
        if (++nrun == kFarRun) {
          far_flush(acc);
          far_zero(acc);
          nrun = 0;
        }
      }
      if (nrun > 0) far_flush(acc);
    }
  };
  // Blocks of kChunk lines summed in plain FP32, each block then added to the
  // Kahan-compensated sums.
  auto run = [&](int g0, int g1, auto&& add) {
    for (int b0 = g0; b0 < g1; b0 += kChunk) {
      const int b1 = min(b0 + kChunk, g1);
      float t[P];
#pragma unroll
      for (int p = 0; p < P; ++p) t[p] = 0.0f;
#pragma unroll 2
      for (int kk = b0; kk < b1; ++kk) add(recs[wv][kk], t);
      if constexpr (!F64) {
#pragma unroll
        for (int p = 0; p < P; ++p) kahan_add(s[p], c[p], t[p]);
      }
    }
  };
  // FP32 general rows of the lines in LDS slots [g0, g1), in sub-batches of lines whose
  // core segments hold at most kCoreQ points: first every core point of the sub-batch is
  // evaluated, one point per lane (FP64 core), into cval; then the lines are walked in
  // order, each general row taking the series for its in-cut lanes outside the core and
  // the core values from cval (incl holds the inclusive prefix of core points).
  auto rows_group = [&](int g0, int g1) {
    if constexpr (!F64) {
      int k = g0;
      int base = 0;   // packed points of the lines before k
      while (k < g1) {
        const int ke =
            first_true(k + 1, g1, [&](int kk) { return incl[wv][kk] - base > kCoreQ; });
        const int npk = incl[wv][ke - 1] - base;
        // one evaluation path for the sub-batch (a loop of its own per path): the FP32
        // small-y core when every line has y < kTaylorY, else the FP64 core with the
        // largest term count its lines need
        const float ly = lane < ke - k ? recs[wv][k + lane].y : 0.0f;
        const int lt = lane < ke - k ? core_tier((double)ly) : 0;
        int tier = -1;
        if (__ballot(lane < ke - k && !(ly < kTaylorY)) != 0ull) {
          tier = 0;
          for (int cc = 1; cc < kCoreTiers; ++cc)
            if (__ballot(lt >= cc) != 0ull) tier = cc;
        }
        // KIND 0: the small-y core; 16, 20: Weideman's series with that many terms,
        // unrolled (the coefficients are constants); 1: the series with the tier's term
        // count known at run time (the rarer counts)
        auto packed = [&](auto kind) {
          constexpr int KIND = decltype(kind)::value;
          const double* wa = core_coef(max(tier, 0));
          const int wn = core_terms(max(tier, 0));
          const double wl = core_L(max(tier, 0));
          for (int r0 = 0; r0 < npk; r0 += kWave) {
            const int g = r0 + lane;
            if (g < npk) {
              const int kk =
                  first_true(k, ke, [&](int m) { return incl[wv][m] - base > g; });
              const int local = g - (kk > k ? incl[wv][kk - 1] - base : 0);
              const Rec<false, P>& q = recs[wv][kk];
              // the row holding point `local` of this line (rows in order)
              int row = 0, j = 0;
              int acc = 0;
              bool found = false;
#pragma unroll
              for (int p = 0; p < P; ++p) {
                const unsigned gi = q.info[p];
                const int n =
                    (((q.cls >> (2 * p)) & 3) == 1) ? (int)((gi >> 21) & 127u) : 0;
                if (!found && local < acc + n) {
                  row = p;
                  j = (int)((gi >> 14) & 127u) + (local - acc);
                  found = true;
                }
                acc += n;
              }
              const double d = rowvals[wv][kWave * row + j] - q.nu0;
              if constexpr (KIND == 0)
                cval[wv][g] = q.sc * voigt_core_small(d * q.ib, q.y);
              else if constexpr (KIND == 16)
                cval[wv][g] = q.sc * (float)voigt_core64_n<16>(kWeidA16, kWeidL16, d * q.ib,
                                                               (double)q.y);
              else if constexpr (KIND == 20)
                cval[wv][g] = q.sc * (float)voigt_core64_n<20>(kWeidA20, kWeidL20, d * q.ib,
                                                               (double)q.y);
              else
                cval[wv][g] = q.sc * (float)voigt_core64_rt(wa, wn, wl, d * q.ib, (double)q.y);
            }
          }
        };
        if (tier < 0) packed(std::integral_constant<int, 0>{});
        else if (tier == 0) packed(std::integral_constant<int, 16>{});
        else if (tier == 1) packed(std::integral_constant<int, 20>{});
        else packed(std::integral_constant<int, 1>{});
        wave_sync();
        int off = 0;   // packed points of the sub-batch's lines walked so far
        run(k, ke, [&](const Rec<false, P>& q, float (&t)[P]) {
          const int cls = __builtin_amdgcn_readfirstlane(q.cls);
          float v[P];
#pragma unroll
          for (int p = 0; p < P; ++p) {
            const int cp = (cls >> (2 * p)) & 3;
            v[p] = 0.0f;
            const unsigned info = (unsigned)__builtin_amdgcn_readfirstlane((int)q.info[p]);
            if (cp == 1) {
              const int lo = (int)(info & 127u), hi = (int)((info >> 7) & 127u);
              const int a = (int)((info >> 14) & 127u), n = (int)((info >> 21) & 127u);
              // x from the FP64 difference: x changes sign along a general row, so the
              // offset form would cancel
              // (the per-tile kernel reads the point's grid value from LDS: keeping it in
              // registers made it spill at 6 waves per SIMD; the grouped one keeps it)
              const double nup = GRP ? nu[p] : rowvals[wv][kWave * p + lane];
              const float x = (float)((nup - q.nu0) * q.ib);
              const float f = q.c1 * asym_scaled<6>(q.y2, fmaf(x, x, q.y2));
              const bool in_cut = lane >= lo && lane < hi;
              const bool in_core = lane >= a && lane < a + n;
              const float cv = cval[wv][min(max(off + lane - a, 0), kCoreQ - 1)];
              off += n;
              v[p] = in_cut ? (in_core ? cv : f) : 0.0f;
            } else if (cp >= 2) {
              // whole row in the series region; the lanes inside the cut are one side of
              // bnd
              const float x = fmaf(cp == 2 ? da32[p] : db32[p], q.ib32, q.xr[p]);
              const float f = series_row((int)(info >> 8), q, fmaf(x, x, q.y2));
              const int bnd = (int)(info & 255u);
              const bool in = cp == 2 ? (lane < bnd) : (lane >= bnd);
              v[p] = in ? f : 0.0f;
            }
          }
#pragma unroll
          for (int p = 0; p < P; ++p) t[p] += v[p];
        });
        wave_sync();   // cval is refilled by the next sub-batch
        base = incl[wv][ke - 1];
        k = ke;
      }
    }
  };
  // FP32 path: lines needing per-row classes (general rows) are put aside in dlist (line
  // offsets from it.b, in order) and staged again, with their lane ranges, 64 at a time,
  // so that the search code runs with full wavefronts instead of in almost every chunk.
  auto deferred_pass = [&](int nd) {
    if constexpr (!F64) {
      Rec<F64, P> r;
      double sc64 = 0.0;
      int mode = kSkip, npairs = 0;
      if (lane < nd) {
        r = stage_line<F64, P>(A, recs_k, rows, rowvals[wv], it.b + dlist[wv][lane], &sc64,
                               &mode, &npairs, true);
      }
      set_scale(r, sc64);
      int w = lane < nd ? npairs : 0;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int u = __shfl_up(w, o, kWave);
        if (lane >= o) w += u;
      }
      if (lane < nd) {
        recs[wv][lane] = r;
        incl[wv][lane] = w;
      }
      wave_sync();
      rows_group(0, nd);
      wave_sync();
    }
  };
  int ndef = 0;   // lines waiting in dlist

  // Main-contributor selection (SEL): the lines whose bound over the tile's group reaches
  // tau are gathered into a queue of line offsets from it.b (q0: the next 64, q1: the
  // overflow; compacted through incl, which is free between passes), so that only kept
  // lines are staged, 64 at a time. Without selection the chunks are consecutive lines.
  [[maybe_unused]] int q0 = 0, q1 = 0, nq = 0;
  auto walk = [&](int64_t first) {
  for (int64_t base = first; SEL || base < e_cur; base += SEL ? 0 : kWave) {
    if constexpr (!F64 && !SEL) {
      far_run(base);
      if (base >= e_cur) break;
    }
    int64_t i = base + lane;   // this lane's line in the chunk (e_cur or later: none)
    if constexpr (SEL) {
      const uint64_t lt = (1ull << lane) - 1ull;
      while (nq < kWave && base < e_cur) {
        const int64_t j = base + lane;
        bool keep = false;
        if (j < e_cur) {
          const LineRec lr = recs_k[j];
          keep = contrib_upper(A.L.nu0[j], lr, g_first, g_last) >= tau;
        }
        const uint64_t km = __ballot(keep);
        const int cnt = __popcll(km);
        if (keep) incl[wv][__popcll(km & lt)] = (int)(j - it.b);
        wave_sync();
        // queue position nq + r of the r-th kept line: lane (nq + r) mod 64 of q0 or q1
        const int src = (lane - nq) & (kWave - 1);
        const int q = src < cnt ? incl[wv][src] : 0;
        if (lane >= nq && lane - nq < cnt) q0 = q;
        if (lane < nq && lane + kWave - nq < cnt) q1 = q;
        wave_sync();
        nq += cnt;
        base += kWave;
      }
      if (nq == 0) break;
      i = lane < nq ? it.b + q0 : e_cur;
      q0 = q1;
      nq = max(nq - kWave, 0);
    }
    Rec<F64, P> r;
    double sc64 = 0.0;
    int mode = kSkip, npairs = 0;
    if constexpr (!F64 && SEL) {
      // a chunk of kept far lines only skips the staging and the grouping (without
      // selection far_run has taken such chunks)
      if (ft.ok) {
        float fx0 = 1.0f, fh0 = 0.0f;
        bool ds = false;
        const bool is_far = i >= e_cur || far_line_j(i, fx0, fh0, r.y, sc64, ds);
        if (__ballot(!is_far) == 0ull) {
          r.y2 = r.y * r.y;
          set_scale(r, sc64);
          far_sum(i < e_cur ? r.c1 : 0.0f, fx0, fh0, i < e_cur ? r.y2 : 0.0f,
                  __ballot(ds) != 0ull);
          continue;
        }
        sc64 = 0.0;
      }
    }
    if (i < e_cur) {
      r = stage_line<F64, P>(A, recs_k, rows, rowvals[wv], i, &sc64, &mode, &npairs, false);
    } else {
      r.cls = 0;
    }
    set_scale(r, sc64);
    // FP32 path: lines of the unmasked series modes far enough from the tile (far_ok at
    // the tile's centre, the doubly shifted Lorentzian valid at its nearest point) are
    // summed as one polynomial when the chunk holds enough of them; they then leave the
    // per-line walk
    [[maybe_unused]] float fc1 = 0.0f, fx = 1.0f, fhl = 0.0f, fy2 = 0.0f;
    [[maybe_unused]] bool far_chunk = false, far_ds = false;
    if constexpr (!F64) {
      bool far = false, ds = false;
      const int ms = mode - kSeries;   // series modes: side * 2 kNVar + masked * kNVar + var
      if (ms >= 0 && ms % (2 * kNVar) < kNVar) {
        const bool left = ms < 2 * kNVar;
        const float hl = ft.h * r.ib32;
        const float xn = left ? r.xr[0] : r.xr[P - 1];
        const float x = fmaf(r.ib32, left ? ft.ca : ft.cb, xn);
        const float y2 = r.y * r.y;
        const float r2n = fmaf(xn, xn, y2);
        if (dshift_ok(r2n, A.l1_eps) && far_ok(x, hl, A.far_kappa)) {
          far = true;
          ds = !shifted_lorentz_ok(y2, r2n, A.l1_eps);
          fc1 = r.c1;
          fx = x;
          fhl = hl;
          fy2 = y2;
        }
      }
      far_chunk = __popcll(__ballot(far)) >= kFarMinLines;
      far_ds = __ballot(ds) != 0ull;
      if (far_chunk && far) mode = kSkip;
    }
    // Group the chunk's lines by mode (stable inside each mode) so that the walk below
    // runs every mode's lines in a loop of its own with no per-line dispatch; lines with
    // no point inside the cut are dropped. The order is fixed by the data alone.
    int gstart[kModes + 1];
    {
      const uint64_t lt = (1ull << lane) - 1ull;
      int pos = -1, acc = 0;
      gstart[0] = 0;
#pragma unroll
      for (int m = 1; m < (F64 ? 2 : kModes); ++m) {
        const uint64_t mk = __ballot(mode == m);
        gstart[m] = acc;
        if (mk) {   // wave-uniform: most chunks hold only a few of the modes
          if (mode == m) pos = acc + __popcll(mk & lt);
          acc += __popcll(mk);
        }
      }
#pragma unroll
      for (int m = F64 ? 2 : kModes; m <= kModes; ++m) gstart[m] = acc;
      if constexpr (F64) {
        if (pos >= 0) recs[wv][pos] = r;
      } else {
        // general lines wait in dlist; the series groups start at slot 0
        const int nrows = gstart[kRows + 1];
        if (mode == kRows) dlist[wv][ndef + pos] = (int)(i - it.b);
        else if (pos >= 0) recs[wv][pos - nrows] = r;
#pragma unroll
        for (int m = kRows + 1; m <= kModes; ++m) gstart[m] -= nrows;
        ndef += nrows;
      }
    }
    wave_sync();
    if constexpr (!F64) {
      if (far_chunk) far_sum(fc1, fx, fhl, fy2, far_ds);
    }
    if constexpr (F64) {
      for (int kk = gstart[kRows]; kk < gstart[kRows + 1]; ++kk) {
        const Rec<F64, P>& q = recs[wv][kk];
        const int cls = __builtin_amdgcn_readfirstlane(q.cls);
#pragma unroll
        for (int p = 0; p < P; ++p) {
          if (((cls >> (2 * p)) & 3) == 0) continue;
          const double d = rowvals[wv][kWave * p + lane] - q.nu0;
          if (fabs(d) <= q.cut) s[p] += q.sc * voigt_k64(d * q.ib, q.y);
        }
      }
    } else {
      // series modes: the line lies left (right) of the tile; all rows take the series
      // of the mode's variant, masked by the rows' lane bounds unless every point is
      // inside the cut
#define XS_SERIES_GROUP(SIDE, MASKED, VAR, NT)                                        \
  run(gstart[series_mode(SIDE, MASKED, VAR)], gstart[series_mode(SIDE, MASKED, VAR) + 1], \
      [&](const Rec<false, P>& q, float (&t)[P]) {                                    \
        series_add<P, NT, SIDE, MASKED>(q, SIDE ? db32 : da32, lane, t);              \
      })
      XS_SERIES_GROUP(0, 0, 0, 1);
      XS_SERIES_GROUP(0, 0, 1, 2);
      XS_SERIES_GROUP(0, 0, 2, 3);
      XS_SERIES_GROUP(0, 0, 3, 4);
      XS_SERIES_GROUP(0, 0, 4, 6);
      XS_SERIES_GROUP(0, 1, 0, 1);
      XS_SERIES_GROUP(0, 1, 1, 2);
      XS_SERIES_GROUP(0, 1, 2, 3);
      XS_SERIES_GROUP(0, 1, 3, 4);
      XS_SERIES_GROUP(0, 1, 4, 6);
      XS_SERIES_GROUP(1, 0, 0, 1);
      XS_SERIES_GROUP(1, 0, 1, 2);
      XS_SERIES_GROUP(1, 0, 2, 3);
      XS_SERIES_GROUP(1, 0, 3, 4);
      XS_SERIES_GROUP(1, 0, 4, 6);
      XS_SERIES_GROUP(1, 1, 0, 1);
      XS_SERIES_GROUP(1, 1, 1, 2);
      XS_SERIES_GROUP(1, 1, 2, 3);
      XS_SERIES_GROUP(1, 1, 3, 4);
      XS_SERIES_GROUP(1, 1, 4, 6);
#undef XS_SERIES_GROUP
    }
    wave_sync();
    if (!F64 && ndef >= kWave) {
      deferred_pass(kWave);
      // the lines still waiting move to the front
      const int left = ndef - kWave;
      const int keep = lane < left ? dlist[wv][kWave + lane] : 0;
      wave_sync();
      if (lane < left) dlist[wv][lane] = keep;
      wave_sync();
      ndef = left;
    }
  }
  };
  if constexpr (GRP) {
    // this wave's part of its tile's window without the group's far lines
    const int64_t r0[3] = {it.b, max(gg.i2, it.b), max(gg.i4, it.b)};
    const int64_t r1[3] = {min(gg.i1, it.e), min(gg.i3, it.e), it.e};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      e_cur = r1[q];
      if (r0[q] < e_cur) walk(r0[q]);
    }
  } else {
    walk(it.b);
  }
  if (!F64 && ndef > 0) deferred_pass(ndef);

  // grouped far field: the group's far lines summed as one polynomial over its span,
  // their 64-line chunks dealt to the wavefronts in turn; each wavefront evaluates its
  // partial polynomial at every point of the span (Kahan sums per point), and after a
  // workgroup barrier each adds the kGroup partials of its own points in wave order
  [[maybe_unused]] double gv[P];
  if constexpr (GRP) {
    constexpr int kRows = kGroup * P;
    const int64_t L1 = max(gg.i1, gg.fb), L2 = min(gg.i2, gg.fe);
    const int64_t R1 = max(gg.i3, gg.fb), R2 = min(gg.i4, gg.fe);
    const int64_t ncl = L2 > L1 ? (L2 - L1 + kWave - 1) / kWave : 0;
    const int64_t ncr = R2 > R1 ? (R2 - R1 + kWave - 1) / kWave : 0;
    float gt[kRows], gs[kRows], gc[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const int64_t j = gg.j_first + kWave * r + lane;
      gt[r] = j < A.n_grid ? (float)((A.grid[j] - gg.c) * gg.ihv) : 0.0f;
      gs[r] = 0.0f;
      gc[r] = 0.0f;
    }
    int e_g = kNoScale;
    float acc[kFarDeg + 1];
    far_zero(acc);
    int nrun = 0;
    auto gflush = [&]() {
      float B[kFarDeg + 1];
#pragma unroll
      for (int kk = 0; kk <= kFarDeg; ++kk) B[kk] = wave_total(acc[kk]);
#pragma unroll
      for (int r = 0; r < kRows; ++r) kahan_add(gs[r], gc[r], far_eval(B, gt[r]));
    };
    for (int64_t q = wvu; q < ncl + ncr; q += kGroup) {
      const bool left = q < ncl;
      const int64_t j = (left ? L1 + q * kWave : R1 + (q - ncl) * kWave) + lane;
      const bool ok = j < (left ? L2 : R2);
      double sc = 0.0;
      float X = 1.0f, h = 0.0f, y = 0.0f;
      if (ok) {
        const double nu0 = A.L.nu0[j];
        const LineRec lr = recs_k[j];
        X = (float)((gg.c - nu0) * lr.ib);
        h = gg.hv32 * (float)lr.ib;
        y = (float)lr.y;
        sc = lr.sc;
      }
      const int exl = sc > 0.0 ? ilogb(sc) : kNoScale;
      if (__ballot(exl > e_g) != 0ull) {
        const int ex = wave_max(exl);
        const int d = max(e_g - ex, -1000);
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          gs[r] = ldexpf(gs[r], d);
          gc[r] = ldexpf(gc[r], d);
        }
#pragma unroll
        for (int kk = 0; kk <= kFarDeg; ++kk) acc[kk] = ldexpf(acc[kk], d);
        e_g = ex;
      }
      const float c1 =
          ok ? (float)(ldexp(sc, kScaleTarget - e_g) * (double)y * (double)kInvSqrtPi) : 0.0f;
      // the doubly shifted expansion when a line's nearest point of the span is outside the
      // shifted Lorentzian's region
      const float xn = fabsf(X) - h;
      const bool ds = ok && !shifted_lorentz_ok(y * y, fmaf(xn, xn, y * y), A.l1_eps);
      far_add(acc, c1, X, h, ok ? y * y : 0.0f, __ballot(ds) != 0ull);
      if (++nrun == kFarRun) {
        gflush();
        far_zero(acc);
        nrun = 0;
      }
    }
    if (nrun > 0) gflush();
    // exchange through this wave's record slots (no longer used)
    static_assert(sizeof(recs[0]) >= (size_t)kRows * kWave * sizeof(double),
                  "record slots hold a wave's partial sums of the span");
    typedef double __attribute__((may_alias)) alias_double;
    alias_double* xb = reinterpret_cast<alias_double*>(&recs[wv][0]);
#pragma unroll
    for (int r = 0; r < kRows; ++r) xb[r * kWave + lane] = (double)gs[r] - (double)gc[r];
    if (lane == 0) grp_e[wvu] = e_g;
    __syncthreads();
#pragma unroll
    for (int p = 0; p < P; ++p) {
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < kGroup; ++w) {
        const alias_double* xw = reinterpret_cast<const alias_double*>(&recs[w][0]);
        v += ldexp(xw[(wvu * P + p) * kWave + lane], grp_e[w] - kScaleTarget);
      }
      gv[p] = v;
    }
  }

  const int64_t row = (A.split == 1) ? (int64_t)(A.pt0 + it.k)
                                     : ((int64_t)it.k * A.split + it.s);
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t j = it.j0 + kWave * p + lane;
    if (j < A.n_grid) {
      double v;
      if constexpr (F64) v = s[p];
      else v = ldexp((double)s[p] - (double)c[p], e_ref - kScaleTarget);
      if constexpr (GRP) v += gv[p];
      if (A.out_f32) ((float*)A.out)[row * A.n_grid + j] = (float)v;
      else A.out[row * A.n_grid + j] = v;
    }
  }
}

template <int P, bool F64, bool SEL, bool GRP = false>
static hipError_t launch_tile_ws(const TileArgs& A, int W, hipStream_t st, dim3 grid) {
  const dim3 block(kBlock);
  switch (W) {
    case 0:
      hipLaunchKernelGGL((xs_tile_kernel<P, F64, 0, SEL, GRP>), grid, block, 0, st, A);
      break;
    case 3:
      hipLaunchKernelGGL((xs_tile_kernel<P, F64, 3, SEL, GRP>), grid, block, 0, st, A);
      break;
    case 4:
      hipLaunchKernelGGL((xs_tile_kernel<P, F64, 4, SEL, GRP>), grid, block, 0, st, A);
      break;
    case 5:
      hipLaunchKernelGGL((xs_tile_kernel<P, F64, 5, SEL, GRP>), grid, block, 0, st, A);
      break;
    case 6:
      hipLaunchKernelGGL((xs_tile_kernel<P, F64, 6, SEL, GRP>), grid, block, 0, st, A);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The tile kernel for occupancy target W, with main-contributor selection when A.tau is
// set.
template <int P, bool F64>
static hipError_t launch_tile_w(const TileArgs& A, int W, hipStream_t st, dim3 grid) {
  if (A.group > 1) {
    // grouped far field: FP32 path without selection, 1 or 2 points per lane
    if constexpr (!F64 && P <= 2) {
      if (!A.tau) return launch_tile_ws<P, false, false, true>(A, W, st, grid);
    }
    return hipErrorInvalidValue;
  }
  return A.tau ? launch_tile_ws<P, F64, true>(A, W, st, grid)
               : launch_tile_ws<P, F64, false>(A, W, st, grid);
}

}  // namespace xs
