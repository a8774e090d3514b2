// Instantiations of the tile kernel for 1 grid point per lane (all precisions and
// occupancy targets).
#include "tile_kernel.h"

namespace xs {

hipError_t launch_tile_p1(const TileArgs& A, bool f64, int W, hipStream_t st, dim3 grid) {
  return f64 ? launch_tile_w<1, true>(A, W, st, grid) : launch_tile_w<1, false>(A, W, st, grid);
}

}  // namespace xs
