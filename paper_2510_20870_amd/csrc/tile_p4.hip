// Instantiations of the tile kernel for 4 grid points per lane (all precisions and
// occupancy targets).
#include "tile_kernel.h"

namespace xs {

hipError_t launch_tile_p4(const TileArgs& A, bool f64, int W, hipStream_t st, dim3 grid) {
  return f64 ? launch_tile_w<4, true>(A, W, st, grid) : launch_tile_w<4, false>(A, W, st, grid);
}

}  // namespace xs
