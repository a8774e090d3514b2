// Output regridding: cross-sections computed on one resident grid resampled onto another,
// for results on a user grid of fixed resolving power (section "Similar tools": any user
// wavelength or wavenumber grid, which fixes the spectral resolution; closing paragraph of
// "Functionality of pyROX": results converted for other codes' grids).
//
// Each source row is read as the piecewise-linear function through its grid nodes, zero
// outside the source range. Two forms:
//   linear  : that function at each destination point;
//   bin mean: its mean over each destination point's bin. Bin k spans from the midpoint
//             with the previous destination point to the midpoint with the next one (the
//             first and last bins mirrored to the same half-widths), clipped to the source
//             range; a bin wholly outside the source range gives 0. The integral over a bin
//             is summed over the source intervals it covers (trapezoids, partial ones at
//             its ends), so bin means times bin widths add up to the integral of the
//             function over the bins' union.
// One thread per (row, destination point): HBM-bound, tiny beside the line work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/xsec.h"
#include "kernel_args.h"
#include "runtime_internal.h"

namespace xs {

// First i in [0, n) with x[i] > v (n if none).
__device__ __forceinline__ int64_t upper_index(const double* __restrict__ x, int64_t n,
                                               double v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (x[mid] > v) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// The linear interpolant of (x, y) at v inside [x[0], x[n-1]], given i = upper_index(v).
__device__ __forceinline__ double interp_at(const double* __restrict__ x,
                                            const double* __restrict__ y, int64_t n,
                                            int64_t i, double v) {
  if (i >= n) return y[n - 1];   // v == x[n - 1]
  if (i == 0) return y[0];
  const double t = (v - x[i - 1]) / (x[i] - x[i - 1]);
  return y[i - 1] + t * (y[i] - y[i - 1]);
}

__global__ void xs_regrid_kernel(const double* __restrict__ src_x, int64_t n_src,
                                 const double* __restrict__ src, const double* __restrict__ dst_x,
                                 int64_t n_dst, int64_t n_rows, int bin_mean,
                                 double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_rows * n_dst) return;
  const int64_t r = t / n_dst, k = t - r * n_dst;
  const double* y = src + r * n_src;
  const double lo = src_x[0], hi = src_x[n_src - 1];
  if (!bin_mean) {
    const double v = dst_x[k];
    out[t] = (v < lo || v > hi) ? 0.0 : interp_at(src_x, y, n_src, upper_index(src_x, n_src, v),
                                                  v);
    return;
  }
  // bin edges: midpoints between neighbours, the end bins mirrored
  double a, b;
  if (n_dst == 1) {
    a = lo;
    b = hi;
  } else {
    a = k > 0 ? 0.5 * (dst_x[k - 1] + dst_x[k]) : dst_x[0] - 0.5 * (dst_x[1] - dst_x[0]);
    b = k + 1 < n_dst ? 0.5 * (dst_x[k] + dst_x[k + 1])
                      : dst_x[k] + 0.5 * (dst_x[k] - dst_x[k - 1]);
  }
  a = fmax(a, lo);
  b = fmin(b, hi);
  if (!(b > a)) {
    out[t] = 0.0;
    return;
  }
  // nodes strictly inside (a, b): [i0, i1)
  const int64_t i0 = upper_index(src_x, n_src, a);
  int64_t i1 = i0;
  while (i1 < n_src && src_x[i1] < b) ++i1;
  const double ya = interp_at(src_x, y, n_src, i0, a);
  const double yb = interp_at(src_x, y, n_src, upper_index(src_x, n_src, b), b);
  double s = 0.0;
  if (i1 == i0) {
    s = 0.5 * (ya + yb) * (b - a);
  } else {
    s = 0.5 * (ya + y[i0]) * (src_x[i0] - a);
    for (int64_t i = i0; i + 1 < i1; ++i) s += 0.5 * (y[i] + y[i + 1]) * (src_x[i + 1] - src_x[i]);
    s += 0.5 * (y[i1 - 1] + yb) * (b - src_x[i1 - 1]);
  }
  out[t] = s / (b - a);
}

}  // namespace xs

using namespace xs;

extern "C" int xs_regrid(xs_ctx* c, xs_grid_t src_h, xs_grid_t dst_h, const double* sigma_src,
                         size_t n_rows, int mode, double* out, int on_device, void* stream) {
  if (!c || !sigma_src || !out) return fail(XS_EINVAL, "NULL argument");
  if (mode != XS_REGRID_LINEAR && mode != XS_REGRID_BIN_MEAN)
    return fail(XS_EINVAL, "unknown regrid mode %d", mode);
  if (n_rows == 0 || n_rows > ((size_t)1 << 20))
    return fail(XS_EINVAL, "n_rows must be in [1, 2^20] (got %zu)", n_rows);
  GridRes* S;
  GridRes* D;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    S = c->find_grid(src_h);
    D = c->find_grid(dst_h);
  }
  if (!S || !D) return fail(XS_ENOTFOUND, "unknown source or destination grid");
  if (S->n < 2) return fail(XS_EINVAL, "the source grid needs at least 2 points");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const size_t in_bytes = n_rows * S->n * sizeof(double);
  const size_t out_bytes = n_rows * D->n * sizeof(double);
  void* buf = nullptr;
  const double* src_dev = sigma_src;
  double* out_dev = out;
  if (!on_device) {
    const size_t in_al = (in_bytes + 255) & ~(size_t)255;
    int rc = c->dev_alloc(&buf, in_al + out_bytes, "regrid staging");
    if (rc) return rc;
    e = hipMemcpyAsync(buf, sigma_src, in_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
      c->dev_free(buf, in_al + out_bytes);
      return hip_fail(e, "regrid upload");
    }
    src_dev = (const double*)buf;
    out_dev = (double*)((char*)buf + in_al);
  }
  const int64_t total = (int64_t)(n_rows * D->n);
  hipLaunchKernelGGL(xs_regrid_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     S->d, (int64_t)S->n, src_dev, D->d, (int64_t)D->n, (int64_t)n_rows,
                     mode == XS_REGRID_BIN_MEAN, out_dev);
  e = hipGetLastError();
  if (e == hipSuccess && !on_device) {
    e = hipMemcpyAsync(out, out_dev, out_bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (buf) c->dev_free(buf, ((in_bytes + 255) & ~(size_t)255) + out_bytes);
  if (e != hipSuccess) return hip_fail(e, "regrid");
  return XS_OK;
}
