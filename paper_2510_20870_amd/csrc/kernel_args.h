// Argument blocks shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.h"

namespace xs {

constexpr int kWave = 64;
constexpr int kWavesPerWG = 4;
constexpr int kBlock = kWave * kWavesPerWG;
constexpr int kMaxSplit = 256;
constexpr int kSelGroup = 4;   // tiles per main-contributor selection group
// Tiles of a workgroup that share one far-field expansion (one tile per wavefront).
constexpr int kGroup = kWavesPerWG;
// Device scratch of the allocation-free entry point (one array per device, kernels.hip).
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;
constexpr int kPtsPerFill = 64;   // P-T pairs per fill launch (passed as kernel arguments)

struct LinesDev {
  const double* nu0;
  const float* A;
  const float* E;
  const float* gam;
  const float* nT;
  const uint16_t* g;
  const uint16_t* J;   // lower-state J (nullptr: 0 for every line)
  int64_t n;
};

// Per (line, P-T point) parameters written by the parameter kernel: the cutoff half-width,
// 1/b_D, the profile scale S/(b_D sqrt(pi)) and y = gamma_L/b_D (all FP64, 32 bytes).
struct LineRec {
  double cut, ib, sc, y;
};

struct ParamArgs {
  LinesDev L;
  SpeciesDev sp;
  CutDev cut;
  const double* pts;      // [n_pts][2] = (P bar, T K), whole table
  int pt0, n_pt;          // this batch: points pt0 .. pt0 + n_pt - 1
  int64_t lo, n;          // line range [lo, lo + n)
  LineRec* out;           // [n_pt][n]
};

struct TileArgs {
  LinesDev L;
  SpeciesDev sp;
  CutDev cut;
  const double* grid;
  int64_t n_grid;
  const double* pts;      // [n_pts][2], whole table
  int pt0, n_pt;          // this batch
  int split;
  int group;              // 1: a work item is one tile (one wavefront); kGroup: a work
                          // item is kGroup neighbouring tiles (one workgroup)
  int64_t n_tiles;        // units issued: tiles, or groups of kGroup tiles
  int64_t n_items;        // n_tiles * n_pt * split
  int64_t n_wg;           // logical workgroups (ceil(n_items / 4), or n_items grouped)
  const int* tile_order;  // issue order of the units (nullptr: ascending)
  const LineRec* recs;    // [n_pt][rec_n] records of lines [rec_lo, rec_lo + rec_n)
  int64_t rec_lo, rec_n;
  double* out;            // split == 1: sigma rows [n_pts][n_grid] (row pt0 + k);
                          // else partials [n_pt][split][n_grid] of this batch
  int out_f32;            // split == 1 only: out holds float rows instead of double
  unsigned long long* counts;  // count kernel only: [n_pts][kNEvalTiers]
  // main-contributor selection (nullptr: off): per (P, T) point of the batch and group of
  // kSelGroup neighbouring tiles (tile / kSelGroup), the contribution bound below which a
  // line is dropped, [n_pt][tau_stride]
  double* tau;
  int64_t tau_stride;     // groups of the whole grid
  double select_eps;      // select kernel: the allowed relative error
  // error budget of the shifted forms (shifted_lorentz_ok, dshift_ok) and the far-line
  // threshold kappa (far_ok) for that budget
  float l1_eps, far_kappa;
};

// Launchers (kernels.hip). phys_wg = number of workgroups launched: n_wg rounded up to a
// multiple of 8 * 16 (whole XCD blocks).
inline int64_t phys_workgroups(int64_t n_wg) { return (n_wg + 127) / 128 * 128; }
hipError_t launch_params(const ParamArgs& A, hipStream_t st);
hipError_t launch_tile(const TileArgs& A, int P, bool f64, int W, hipStream_t st,
                       int64_t phys_wg);
hipError_t launch_count(const TileArgs& A, int P, hipStream_t st, int64_t phys_wg);
// one wavefront per (group of 4 tiles, P-T point), A.n_tiles groups: writes A.tau
hipError_t launch_select(const TileArgs& A, int P, hipStream_t st);
// per points-per-lane instantiations of the tile kernel (tile_p*.hip)
hipError_t launch_tile_p1(const TileArgs& A, bool f64, int W, hipStream_t st, dim3 grid);
hipError_t launch_tile_p2(const TileArgs& A, bool f64, int W, hipStream_t st, dim3 grid);
hipError_t launch_tile_p4(const TileArgs& A, bool f64, int W, hipStream_t st, dim3 grid);
hipError_t launch_tile_p8(const TileArgs& A, bool f64, int W, hipStream_t st, dim3 grid);
// out: float rows when out_f32, else double rows
hipError_t launch_reduce(const double* part, void* out, int out_f32, int64_t n_grid, int n_pts,
                         int split, hipStream_t st);
// collision-induced absorption: block k (nodes [off[k], off[k+1]) of nu, alpha) linearly
// interpolated onto the grid, zero outside the block, out[k][j]
hipError_t launch_cia(const double* grid, int64_t n_grid, const int64_t* off, int n_blocks,
                      const double* nu, const double* alpha, double* out, hipStream_t st);
hipError_t launch_eval_voigt(const double* x, const double* y, int64_t n, int f64,
                             double* out, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t st);
// dst[0 .. 2 n) = pairs[0 .. 2 n), the values passed as kernel arguments (no copy from
// host memory), kPtsPerFill pairs per launch
hipError_t launch_fill_pts(double* dst, const double* pairs, int64_t n, hipStream_t st);
// Device address of the allocation-free scratch array on the current device (called once
// per device, with that device current).
hipError_t noalloc_scratch_address(void** out);
// g[j] = a + j * h (FP64, one rounding per operation, no contraction)
hipError_t launch_fill_uniform(double* g, int64_t n, double a, double h, hipStream_t st);

}  // namespace xs
