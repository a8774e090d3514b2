// gfx950 kernels of the cross-section sum: the Voigt profiles of all lines are summed into
// a cross-section for each temperature-pressure point (paper, "Functionality of pyROX",
// bullets "Compute line-strengths and -widths", "Compute line profiles", "Combine and
// save").
//
// Two kernels carry the path:
//
// 1. xs_params_kernel (HBM-bound): for every line in the range a grid can reach and every
//    (P, T) point of a batch, the FP64 line parameters (cutoff, 1/b_D, S/(b_D sqrt(pi)),
//    y = gamma_L/b_D) as one 32-byte record. Each line is derived once per (P, T) instead
//    of once per tile that visits it, and the transcendental FP64 code stays out of the
//    register budget of the tile kernel.
//
// 2. xs_tile_kernel (VALU-bound; tile_kernel.h, instantiated in tile_p*.hip). One work
//    item = (grid tile, (P, T) point, line split). A tile is 64 * P consecutive grid
//    points owned by ONE wavefront: lane l holds points j0 + 64 p + l for p < P, so each
//    of the P rows is 64 consecutive points. Waves are independent: no workgroup barrier
//    and no atomics on results. Per item the wave
//      a. bounds the cutoff of every line that can reach the tile (cut_bound),
//      b. finds the line window [lo, hi) by a 64-ary search on the sorted centres (one
//         load per lane per level, five levels for 1e9 lines),
//      c. walks the window in chunks of 64 lines: each lane loads one line's centre and
//         record (coalesced), classifies the line against each row and writes a record to
//         the wave's LDS slice grouped by mode; after a wave-level fence every lane reads
//         the records back as LDS broadcasts and evaluates its points against each line,
//      d. writes its sums: the final value, or a partial for the fixed-order reduction.
//
// Arithmetic of one (line, point) pair: lines on one side of a row (the large majority)
// take x = (nu_j - nu_end) / b_D + x_end from the row's nearer end in FP32 (x does not
// change sign along the row, so there is no cancellation), the cheapest far-region form
// the row's nearest point allows (a shifted Lorentzian, or the asymptotic series with 2 to
// 6 terms) and the cut as a lane bound found at staging time with the FP64 test; rows a
// line reaches inside |z| = 7 take x from the FP64 difference, the six-term series for
// their points outside |z| = 7 and the FP64 Weideman core inside. Lines far from the
// tile on the FP32 path (the whole tile inside the cut, shifted Lorentzian, |x| at the
// tile's centre at least five half-widths away) are not evaluated per point: their Taylor
// coefficients in the tile coordinate are summed over the wavefront and the polynomial is
// evaluated once per point (voigt.h, far_coeffs). Contributions are summed in FP32 over
// blocks of 16 lines, each block added to a Kahan-compensated FP32 sum (a plain FP64 sum
// on the FP64 path). FP32 contributions carry a power-of-two scale chosen
// per wavefront: whenever a staged chunk holds a line stronger than any before, the scale
// is lowered so the strongest line's scale is about 2^48 and the running sums are
// rescaled exactly, so any absolute magnitude of sigma stays inside FP32 range; the scale
// is removed exactly when the FP64 result is stored.
//
// Around them: the fixed-order reduction of split partials, the evaluation count by tier
// (accounting), the main-contributor selection thresholds, the CIA regridding, fills and
// the point evaluation of K used by the tests.

#include <algorithm>

#include "tile_kernel.h"

namespace xs {

// ------------------------------------------------------------------ parameter kernel
__global__ __launch_bounds__(256) void xs_params_kernel(ParamArgs A) {
  const int k = blockIdx.y;
  const PtConst pc = make_pt(A.sp, A.pts[2 * (A.pt0 + k)], A.pts[2 * (A.pt0 + k) + 1]);
  LineRec* out = A.out + (int64_t)k * A.n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < A.n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = A.lo + t;
    const double nu0 = A.L.nu0[i];
    const LineParams lp = line_params(A.sp, pc, A.cut, nu0, A.L.A[i], A.L.E[i], A.L.gam[i],
                                      A.L.nT[i], A.L.g[i], A.L.J ? A.L.J[i] : (uint16_t)0);
    LineRec r;
    r.cut = lp.cut;
    r.ib = 1.0 / lp.bD;
    r.sc = lp.S * r.ib * (1.0 / kSqrtPiD);
    r.y = lp.gL * r.ib;
    out[t] = r;
  }
}

// Fixed-order reduction of split partials: out[k][j] = sum_s part[k][s][j], s ascending,
// stored as OUT (double, or float rounded once from the FP64 sum).
template <typename OUT>
__global__ __launch_bounds__(256) void xs_reduce_kernel(const double* __restrict__ part,
                                                        OUT* __restrict__ out,
                                                        int64_t n_grid, int n_pts, int split) {
  const int64_t total = (int64_t)n_pts * n_grid;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / n_grid, j = t - k * n_grid;
    const double* p = part + k * split * n_grid + j;
    double acc = 0.0;
    for (int s = 0; s < split; ++s) acc += p[(int64_t)s * n_grid];
    out[t] = (OUT)acc;
  }
}

// Count of (line, point) pairs inside the cutoff, per (P, T) point and evaluation tier;
// same traversal and the same FP64 cut test as the tile kernel. The tier is the one the
// point itself needs (its own FP32 r^2 and y): the far-region variants 0..kNVar-1, then
// the core (kNVar + core_eval_tier: the FP64 core's y-dependent term counts, the FP32
// small-y core). counts is [n_pt][kNEvalTiers].
template <int P>
__global__ __launch_bounds__(kBlock) void xs_count_kernel(TileArgs A) {
  __shared__ double cen[kWavesPerWG][kWave], cut[kWavesPerWG][kWave];
  __shared__ double ibs[kWavesPerWG][kWave], ys[kWavesPerWG][kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x >> 6;
  ItemInfo it;
  if (!decode_item<P>(A, lane, it)) return;
  double nu[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t j = it.j0 + kWave * p + lane;
    nu[p] = (j < A.n_grid) ? A.grid[j] : __builtin_nan("");
  }
  // with main-contributor selection, only the kept lines count
  const double tau = A.tau ? A.tau[(int64_t)it.k * A.tau_stride + it.tile / kSelGroup] : 0.0;
  double g_first = 0.0, g_last = 0.0;
  if (tau > 0.0) sel_span<P>(A, it.tile, &g_first, &g_last);
  unsigned long long cnt[kNEvalTiers];
#pragma unroll
  for (int t = 0; t < kNEvalTiers; ++t) cnt[t] = 0;
  for (int64_t base = it.b; base < it.e; base += kWave) {
    const int64_t i = base + lane;
    double c0 = 0.0, ct = -1.0, ib = 0.0, yv = 0.0;
    if (i < it.e) {
      const LineRec lr = A.recs[(int64_t)it.k * A.rec_n + (i - A.rec_lo)];
      c0 = A.L.nu0[i];
      ct = (tau > 0.0 && contrib_upper(c0, lr, g_first, g_last) < tau) ? -1.0 : lr.cut;
      ib = lr.ib;
      yv = lr.y;
    }
    cen[wv][lane] = c0;
    cut[wv][lane] = ct;
    ibs[wv][lane] = ib;
    ys[wv][lane] = yv;
    wave_sync();
    const int nk = (int)min((int64_t)kWave, it.e - base);
    for (int kk = 0; kk < nk; ++kk) {
      const double q0 = cen[wv][kk], qc = cut[wv][kk];
      const float y = (float)ys[wv][kk];
      const float y2 = y * y;
      const int core = kNVar + core_eval_tier(y);
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const double d = nu[p] - q0;
        if (fabs(d) <= qc) {
          const float x = (float)(d * ibs[wv][kk]);
          const float r2 = fmaf(x, x, y2);
          const int tier = r2 >= kT6R2 ? asym_variant(y2, r2, A.l1_eps) : core;
#pragma unroll
          for (int t = 0; t < kNEvalTiers; ++t) cnt[t] += (tier == t) ? 1ull : 0ull;
        }
      }
    }
    wave_sync();
  }
  // wave reductions, then one 64-bit integer atomic per tier and wave (exact, order-free)
#pragma unroll
  for (int t = 0; t < kNEvalTiers; ++t) {
    unsigned long long v = cnt[t];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0 && v) atomicAdd(A.counts + (int64_t)(A.pt0 + it.k) * kNEvalTiers + t, v);
  }
}

// Main-contributor selection (the paper names it as a way to speed up the line-profile
// computation, "Functionality of pyROX", without defining it). For one group of kSelGroup
// neighbouring tiles and one (P, T) point: a lower bound of sigma at every point of the
// group, L = sum of the lines' lower bounds (contrib_lower), and the largest power-of-two
// threshold tau such that the upper bounds (contrib_upper) of all lines below tau add up
// to at most eps L. Dropping those lines changes sigma by at most eps sigma at every point
// of the group. The bounds are binned by binary exponent into an exact integer histogram
// (fixed point, rounded up), so tau does not depend on the order of the additions.
// One workgroup per (group, point), its waves taking interleaved 64-line slices of the
// window: A.n_tiles counts groups here. L is the sum of the waves' partial sums in wave
// order, and the histogram is shared (integer additions), so tau depends on the data only.
template <int P>
__global__ __launch_bounds__(kBlock) void xs_select_kernel(TileArgs A) {
  __shared__ unsigned long long hist[kWave];
  __shared__ double part[kWavesPerWG];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t item = blockIdx.x;
  if (item >= A.n_tiles * A.n_pt) return;   // the whole workgroup
  const int k = (int)(item % A.n_pt);
  const int64_t group = item / A.n_pt;
  double t_first, t_last;
  sel_span<P>(A, group * kSelGroup, &t_first, &t_last);
  int64_t lo, hi;
  line_window(A, k, t_first, t_last, lane, &lo, &hi);
  const LineRec* rec = A.recs + (int64_t)k * A.rec_n - A.rec_lo;
  double acc = 0.0;
  for (int64_t i = lo + (int64_t)wv * kWave + lane; i < hi; i += kBlock)
    acc += contrib_lower(A.L.nu0[i], rec[i], t_first, t_last);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) part[wv] = acc;
  if (wv == 0) hist[lane] = 0ull;
  __syncthreads();
  double L = part[0];
#pragma unroll
  for (int w = 1; w < kWavesPerWG; ++w) L += part[w];
  double tau = 0.0;
  const double budget = A.select_eps * L;
  // (a budget so small that its fixed-point unit would overflow drops nothing; the test
  // has the same outcome in every wave)
  if (budget > 0x1p-960 && isfinite(budget)) {
    // bins: 0 for bounds below 2^elo, 1 + ilogb - elo for [2^elo, 2^eL), eL = ilogb(eps L)
    const int eL = ilogb(budget);
    const int elo = eL - 62;
    const double top = ldexp(1.0, eL), low = ldexp(1.0, elo);
    const double unit = ldexp(1.0, 40) / budget;   // histogram units per unit of sigma
    for (int64_t i = lo + (int64_t)wv * kWave + lane; i < hi; i += kBlock) {
      const double c = contrib_upper(A.L.nu0[i], rec[i], t_first, t_last);
      if (c < top) {
        const int bin = c < low ? 0 : ilogb(c) - elo + 1;
        atomicAdd(&hist[bin], (unsigned long long)(c * unit) + 1ull);
      }
    }
    __syncthreads();
    // the bins below b stay within the budget (2^40 units) for b = 0 .. b*: an exclusive
    // prefix sum over the bins, one bin per lane
    const unsigned long long h = hist[lane];
    unsigned long long incl = h;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const unsigned long long u = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += u;
    }
    const bool ok = incl - h <= (1ull << 40);
    const int bstar = __popcll(__ballot(ok)) - 1;
    tau = bstar == 0 ? 0.0 : ldexp(1.0, elo + bstar - 1);
  }
  if (threadIdx.x == 0) A.tau[(int64_t)k * A.tau_stride + group] = tau;
}

__global__ void xs_fill_u64_kernel(unsigned long long* p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0ull;
}

// Scratch of the allocation-free entry point: the point table, line records and split
// partials of one call live here instead of in allocated memory. Each device that loads
// the library holds its own copy until the process ends; host code reaches it only
// through the address noalloc_scratch_address() returns for the current device (the
// array's name is not a device address on the host).
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch_address(void** out) {
  return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

struct PtsBlock {
  int n;
  double v[2 * kPtsPerFill];
};

__global__ void xs_fill_pts_kernel(double* __restrict__ dst, PtsBlock b) {
  const int t = threadIdx.x;
  if (t < 2 * b.n) dst[t] = b.v[t];
}

__global__ void xs_fill_uniform_kernel(double* __restrict__ g, int64_t n, double a, double h) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) g[t] = __dadd_rn(a, __dmul_rn((double)t, h));
}

// Collision-induced absorption restructured onto the grid ("Combine and save": CIA
// coefficients on a wavelength- and temperature-dependent grid): one thread per (block,
// grid point); the bracketing nodes by binary search, linear interpolation between them,
// zero outside the block's range (the end nodes included).
__global__ void xs_cia_kernel(const double* __restrict__ grid, int64_t n_grid,
                              const int64_t* __restrict__ off, int n_blocks,
                              const double* __restrict__ nu, const double* __restrict__ alpha,
                              double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_grid * n_blocks) return;
  const int k = (int)(t / n_grid);
  const int64_t j = t - (int64_t)k * n_grid;
  const double v = grid[j];
  const int64_t a = off[k], b = off[k + 1];
  double r = 0.0;
  if (b > a && v >= nu[a] && v <= nu[b - 1]) {
    // last node <= v
    int64_t lo = a, hi = b - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (nu[mid] <= v) lo = mid;
      else hi = mid - 1;
    }
    if (lo == b - 1) {
      r = alpha[lo];
    } else {
      const double f = (v - nu[lo]) / (nu[lo + 1] - nu[lo]);
      r = alpha[lo] + f * (alpha[lo + 1] - alpha[lo]);
    }
  }
  out[t] = r;
}

__global__ void xs_eval_voigt_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                     int64_t n, int f64, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[t] = f64 ? voigt_k64(x[t], y[t]) : (double)voigt_k32(x[t], (float)y[t]);
}

// --------------------------------------------------------------------------- launchers
hipError_t launch_params(const ParamArgs& A, hipStream_t st) {
  if (A.n <= 0 || A.n_pt <= 0) return hipSuccess;
  int64_t blocks = (A.n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(xs_params_kernel, dim3((unsigned)blocks, (unsigned)A.n_pt), dim3(256), 0,
                     st, A);
  return hipGetLastError();
}

hipError_t launch_tile(const TileArgs& A, int P, bool f64, int W, hipStream_t st,
                       int64_t phys_wg) {
  const dim3 grid((unsigned)phys_wg);
  switch (P) {
    case 1: return launch_tile_p1(A, f64, W, st, grid);
    case 2: return launch_tile_p2(A, f64, W, st, grid);
    case 4: return launch_tile_p4(A, f64, W, st, grid);
    case 8: return launch_tile_p8(A, f64, W, st, grid);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_count(const TileArgs& A, int P, hipStream_t st, int64_t phys_wg) {
  const dim3 grid((unsigned)phys_wg), block(kBlock);
  switch (P) {
    case 1: hipLaunchKernelGGL((xs_count_kernel<1>), grid, block, 0, st, A); break;
    case 2: hipLaunchKernelGGL((xs_count_kernel<2>), grid, block, 0, st, A); break;
    case 4: hipLaunchKernelGGL((xs_count_kernel<4>), grid, block, 0, st, A); break;
    case 8: hipLaunchKernelGGL((xs_count_kernel<8>), grid, block, 0, st, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_select(const TileArgs& A, int P, hipStream_t st) {
  const int64_t items = A.n_tiles * A.n_pt;
  if (items <= 0) return hipSuccess;
  const dim3 grid((unsigned)items), block(kBlock);
  switch (P) {
    case 1: hipLaunchKernelGGL((xs_select_kernel<1>), grid, block, 0, st, A); break;
    case 2: hipLaunchKernelGGL((xs_select_kernel<2>), grid, block, 0, st, A); break;
    case 4: hipLaunchKernelGGL((xs_select_kernel<4>), grid, block, 0, st, A); break;
    case 8: hipLaunchKernelGGL((xs_select_kernel<8>), grid, block, 0, st, A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const double* part, void* out, int out_f32, int64_t n_grid, int n_pts,
                         int split, hipStream_t st) {
  const int64_t total = (int64_t)n_pts * n_grid;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  if (out_f32)
    hipLaunchKernelGGL(xs_reduce_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, part,
                       (float*)out, n_grid, n_pts, split);
  else
    hipLaunchKernelGGL(xs_reduce_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       part, (double*)out, n_grid, n_pts, split);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(xs_fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     p, n);
  return hipGetLastError();
}

hipError_t launch_fill_pts(double* dst, const double* pairs, int64_t n, hipStream_t st) {
  for (int64_t k0 = 0; k0 < n; k0 += kPtsPerFill) {
    PtsBlock b;
    b.n = (int)std::min<int64_t>(kPtsPerFill, n - k0);
    for (int i = 0; i < 2 * b.n; ++i) b.v[i] = pairs[2 * k0 + i];
    hipLaunchKernelGGL(xs_fill_pts_kernel, dim3(1), dim3(2 * kPtsPerFill), 0, st, dst + 2 * k0,
                       b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fill_uniform(double* g, int64_t n, double a, double h, hipStream_t st) {
  const int64_t blocks = (n + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(xs_fill_uniform_kernel, dim3((unsigned)blocks), dim3(256), 0, st, g, n, a,
                     h);
  return hipGetLastError();
}

hipError_t launch_cia(const double* grid, int64_t n_grid, const int64_t* off, int n_blocks,
                      const double* nu, const double* alpha, double* out, hipStream_t st) {
  const int64_t total = n_grid * n_blocks;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(xs_cia_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     grid, n_grid, off, n_blocks, nu, alpha, out);
  return hipGetLastError();
}

hipError_t launch_eval_voigt(const double* x, const double* y, int64_t n, int f64,
                             double* out, hipStream_t st) {
  const int64_t blocks = (n + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(xs_eval_voigt_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, y, n,
                     f64, out);
  return hipGetLastError();
}

}  // namespace xs
