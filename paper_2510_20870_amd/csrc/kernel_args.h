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

struct LinesDev {
  const double* nu0;
  const float* A;
  const float* E;
  const float* gam;
  const float* nT;
  const uint16_t* g;
  int64_t n;
};

struct TileArgs {
  LinesDev L;
  SpeciesDev sp;
  CutDev cut;
  const double* grid;
  int64_t n_grid;
  const double* pts;      // [n_pts][2] = (P bar, T K)
  int n_pts;
  int split;
  int64_t n_tiles;
  int64_t n_items;        // n_tiles * n_pts * split
  int64_t n_wg;           // logical workgroups (ceil(n_items / 4))
  int64_t per_xcd;        // ceil(n_wg / 8)
  double* out;            // [n_pts][n_grid], or partials [n_pts][split][n_grid]
  unsigned long long* counts;  // count kernel only: [n_pts]
  const double* wc;       // Weideman coefficients a_1..a_40
};

// Launchers (kernels.hip). phys_wg = number of workgroups launched (a multiple of 8).
hipError_t launch_tile(const TileArgs& A, int P, bool f64, hipStream_t st, int64_t phys_wg);
hipError_t launch_count(const TileArgs& A, int P, hipStream_t st, int64_t phys_wg);
hipError_t launch_reduce(const double* part, double* out, int64_t n_grid, int n_pts, int split,
                         hipStream_t st);
hipError_t launch_eval_voigt(const double* x, const double* y, int64_t n, int f64,
                             const double* wc, double* out, hipStream_t st);

}  // namespace xs
