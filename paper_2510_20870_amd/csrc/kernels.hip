// gfx950 kernels of the cross-section sum (paper, "Functionality of pyROX": the Voigt
// profiles of all lines "are summed into ... cross-sections for each temperature-pressure
// point").
//
// Work decomposition. One work item = (grid tile, (P, T) point, line split). A tile is
// 64 * P consecutive grid points owned by ONE wavefront: lane l holds points
// j0 + 64 p + l for p < P, so each of the P rows is 64 consecutive points and the
// cutoff/core branches diverge only inside the one or two rows a line's core touches.
// Waves are independent: no workgroup barrier, no atomics on results.
//
// Per item the wave
//   1. bounds the cutoff of every line that can reach the tile (cut_bound),
//   2. finds the line window [lo, hi) by a 64-ary search on the sorted centres (one load
//      per lane per level, five levels for 1e9 lines),
//   3. walks the window in chunks of 64 lines: each lane loads one line (coalesced
//      structure-of-arrays loads), derives its FP64 parameters and writes a 32-byte record
//      to the wave's LDS slice; after a wave-level fence every lane reads the records back
//      as LDS broadcasts and evaluates all its points against each line,
//   4. writes its sums: the final value, or a partial for the fixed-order reduction.
//
// Arithmetic of one (line, point) pair: d = nu_j - nu0 (FP64), the cut test |d| <= cut
// (FP64), x = d / b_D (FP64, rounded once to FP32), K(x, y) in FP32 outside the core and
// FP64 inside it, then a Kahan-compensated FP32 add (or a plain FP64 add for the FP64
// path). FP32 contributions carry a power-of-two scale chosen per wavefront: whenever a
// staged chunk holds a line stronger than any before, the scale is lowered so the
// strongest contribution is about 2^97 and the running sums are rescaled exactly (a
// power-of-two multiply), so any absolute magnitude of sigma stays inside FP32 range; the
// scale is removed exactly when the FP64 result is stored.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "kernel_args.h"
#include "physics.h"
#include "voigt.h"

namespace xs {

constexpr int kScaleTarget = 96;   // exponent of the strongest FP32 contribution scale
constexpr int kNoScale = -(1 << 28);

// Record of one staged line in LDS.
template <bool F64> struct Rec;
template <> struct alignas(16) Rec<false> {
  double nu0, cut, ib;
  float y, sc;
};
template <> struct alignas(16) Rec<true> {
  double nu0, cut, ib, y, sc, pad;
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroups are dispatched round-robin over the 8 XCDs; map them so that each XCD (and
// its L2) works on a contiguous range of tiles, which share most of their line windows.
__device__ __forceinline__ int64_t xcd_logical_wg(int64_t phys, int64_t per_xcd) {
  return (phys & 7) * per_xcd + (phys >> 3);
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

struct ItemInfo {
  int64_t j0;        // first grid index of the tile
  int pt;            // (P, T) index
  int s;             // split index
  int64_t b, e;      // line range of this item
  PtConst pc;
};

template <int P>
__device__ __forceinline__ bool decode_item(const TileArgs& A, int lane, ItemInfo& it) {
  const int64_t phys = blockIdx.x;
  const int64_t wg = xcd_logical_wg(phys, A.per_xcd);
  const int64_t item = wg * kWavesPerWG + (threadIdx.x >> 6);
  if (wg >= A.n_wg || item >= A.n_items) return false;
  it.s = (int)(item % A.split);
  const int64_t r = item / A.split;
  it.pt = (int)(r % A.n_pts);
  const int64_t tile = r / A.n_pts;
  it.j0 = tile * (int64_t)(kWave * P);
  const int64_t jl = min(it.j0 + (int64_t)(kWave * P), A.n_grid) - 1;
  const double P_bar = A.pts[2 * it.pt], T_K = A.pts[2 * it.pt + 1];
  it.pc = make_pt(A.sp, P_bar, T_K);
  const double nu_first = A.grid[it.j0];
  const double nu_last = A.grid[jl];
  const double cb = cut_bound(A.sp, it.pc, A.cut, nu_last);
  // widen the keys by a few ulps of nu so that rounding of nu -+ cb never drops a line
  const double lk = nu_first - cb - fabs(nu_first) * 0x1p-48;
  const double hk = nu_last + cb + fabs(nu_last) * 0x1p-48;
  const int64_t lo = wave_search<false>(A.L.nu0, A.L.n, lk, lane);
  const int64_t hi = wave_search<true>(A.L.nu0, A.L.n, hk, lane);
  const int64_t cnt = hi > lo ? hi - lo : 0;
  it.b = lo + cnt * it.s / A.split;
  it.e = lo + cnt * (it.s + 1) / A.split;
  return true;
}

// Stages line i: fills the record except the FP32 scale and returns the FP64 profile
// scale S / (b_D sqrt(pi)) in *sc64.
template <bool F64>
__device__ __forceinline__ Rec<F64> stage_line(const TileArgs& A, const PtConst& pc, int64_t i,
                                               double* sc64) {
  const double nu0 = A.L.nu0[i];
  const LineParams lp = line_params(A.sp, pc, A.cut, nu0, A.L.A[i], A.L.E[i], A.L.gam[i],
                                    A.L.nT[i], A.L.g[i]);
  Rec<F64> r;
  r.nu0 = nu0;
  r.cut = lp.cut;
  r.ib = 1.0 / lp.bD;
  *sc64 = lp.S / (lp.bD * kSqrtPiD);
  if constexpr (F64) {
    r.y = lp.gL / lp.bD;
    r.sc = *sc64;
    r.pad = 0.0;
  } else {
    r.y = (float)(lp.gL / lp.bD);
    r.sc = 0.0f;
  }
  return r;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  return v;
}

template <int P, bool F64>
__global__ __launch_bounds__(kBlock) void xs_tile_kernel(TileArgs A) {
  __shared__ Rec<F64> recs[kWavesPerWG][kWave];
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
  using acc_t = typename std::conditional<F64, double, float>::type;
  acc_t s[P], c[P];
#pragma unroll
  for (int p = 0; p < P; ++p) { s[p] = 0; c[p] = 0; }
  int e_ref = kNoScale;   // FP32 path: contributions are scaled by 2^(kScaleTarget - e_ref)

  for (int64_t base = it.b; base < it.e; base += kWave) {
    const int64_t i = base + lane;
    Rec<F64> r;
    double sc64 = 0.0;
    if (i < it.e) {
      r = stage_line<F64>(A, it.pc, i, &sc64);
    } else {
      r.nu0 = 0.0; r.cut = -1.0; r.ib = 0.0; r.y = 0; r.sc = 0;
    }
    if constexpr (!F64) {
      const int ex = wave_max(sc64 > 0.0 ? ilogb(sc64) : kNoScale);
      if (ex > e_ref) {
        // a stronger line: lower the scale and rescale the sums exactly
        const int d = max(e_ref - ex, -1000);
#pragma unroll
        for (int p = 0; p < P; ++p) {
          s[p] = ldexpf(s[p], d);
          c[p] = ldexpf(c[p], d);
        }
        e_ref = ex;
      }
      r.sc = (float)ldexp(sc64, kScaleTarget - e_ref);
    }
    recs[wv][lane] = r;
    wave_sync();
    const int nk = (int)min((int64_t)kWave, it.e - base);
    for (int k = 0; k < nk; ++k) {
      const Rec<F64> q = recs[wv][k];
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const double d = nu[p] - q.nu0;
        if (fabs(d) <= q.cut) {
          const double xd = d * q.ib;
          if constexpr (F64) {
            s[p] += q.sc * voigt_k64(xd, q.y, A.wc);
          } else {
            const float v = q.sc * voigt_k32(xd, q.y, A.wc);
            const float yk = v - c[p];
            const float t = s[p] + yk;
            c[p] = (t - s[p]) - yk;
            s[p] = t;
          }
        }
      }
    }
    wave_sync();
  }

  double* out = A.out;
  const int64_t row = (A.split == 1) ? (int64_t)it.pt : ((int64_t)it.pt * A.split + it.s);
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t j = it.j0 + kWave * p + lane;
    if (j < A.n_grid) {
      double v;
      if constexpr (F64) v = s[p];
      else v = ldexp((double)s[p] - (double)c[p], e_ref - kScaleTarget);
      out[row * A.n_grid + j] = v;
    }
  }
}

// Fixed-order reduction of split partials: out[k][j] = sum_s part[k][s][j], s ascending.
__global__ __launch_bounds__(256) void xs_reduce_kernel(const double* __restrict__ part,
                                                        double* __restrict__ out,
                                                        int64_t n_grid, int n_pts, int split) {
  const int64_t total = (int64_t)n_pts * n_grid;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / n_grid, j = t - k * n_grid;
    const double* p = part + k * split * n_grid + j;
    double acc = 0.0;
    for (int s = 0; s < split; ++s) acc += p[(int64_t)s * n_grid];
    out[t] = acc;
  }
}

// Count of (line, point) pairs inside the cutoff, per (P, T) point; same traversal and
// the same FP64 test as the tile kernel.
template <int P>
__global__ __launch_bounds__(kBlock) void xs_count_kernel(TileArgs A) {
  __shared__ double cen[kWavesPerWG][kWave], cut[kWavesPerWG][kWave];
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
  unsigned long long cnt = 0;
  for (int64_t base = it.b; base < it.e; base += kWave) {
    const int64_t i = base + lane;
    double c0 = 0.0, ct = -1.0;
    if (i < it.e) {
      c0 = A.L.nu0[i];
      ct = line_params(A.sp, it.pc, A.cut, c0, A.L.A[i], A.L.E[i], A.L.gam[i], A.L.nT[i],
                       A.L.g[i]).cut;
    }
    cen[wv][lane] = c0;
    cut[wv][lane] = ct;
    wave_sync();
    const int nk = (int)min((int64_t)kWave, it.e - base);
    for (int k = 0; k < nk; ++k) {
      const double q0 = cen[wv][k], qc = cut[wv][k];
#pragma unroll
      for (int p = 0; p < P; ++p) cnt += (fabs(nu[p] - q0) <= qc) ? 1ull : 0ull;
    }
    wave_sync();
  }
  // wave reduction, then one 64-bit integer atomic per wave (exact, order-free)
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
  if (lane == 0) atomicAdd(A.counts + it.pt, cnt);
}

__global__ void xs_eval_voigt_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                     int64_t n, int f64, const double* __restrict__ wc,
                                     double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[t] = f64 ? voigt_k64(x[t], y[t], wc) : (double)voigt_k32(x[t], (float)y[t], wc);
}

}  // namespace xs

// --------------------------------------------------------------------------- launchers
namespace xs {

hipError_t launch_tile(const TileArgs& A, int P, bool f64, hipStream_t st, int64_t phys_wg) {
  const dim3 grid((unsigned)phys_wg), block(kBlock);
#define XS_TILE_CASE(PP)                                                             \
  case PP:                                                                           \
    if (f64) hipLaunchKernelGGL((xs_tile_kernel<PP, true>), grid, block, 0, st, A);  \
    else hipLaunchKernelGGL((xs_tile_kernel<PP, false>), grid, block, 0, st, A);     \
    break;
  switch (P) {
    XS_TILE_CASE(1)
    XS_TILE_CASE(2)
    XS_TILE_CASE(4)
    XS_TILE_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef XS_TILE_CASE
  return hipGetLastError();
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

hipError_t launch_reduce(const double* part, double* out, int64_t n_grid, int n_pts, int split,
                         hipStream_t st) {
  const int64_t total = (int64_t)n_pts * n_grid;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(xs_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, part, out,
                     n_grid, n_pts, split);
  return hipGetLastError();
}

hipError_t launch_eval_voigt(const double* x, const double* y, int64_t n, int f64,
                             const double* wc, double* out, hipStream_t st) {
  const int64_t blocks = (n + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(xs_eval_voigt_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, y, n,
                     f64, wc, out);
  return hipGetLastError();
}

}  // namespace xs
