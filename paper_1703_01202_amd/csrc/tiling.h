// Tile scheduling shared by the stencil and network kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace pfc {

// Tile of this block in a 1-D launch over ntx x nty tiles.  Blocks are dispatched round-robin
// over the 8 XCDs, each with its own L2; XCD k = b mod 8 is given a contiguous range of tiles
// in row-major order, so vertically adjacent tiles (which share halo rows) run on the same
// XCD and their halo reads hit its L2.  A bijection for any tile count.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb / 8, r = nb % 8, k = b % 8;
    return k * q + (k < r ? k : r) + b / 8;
}

// Tiles of a persistent block: block b (after the XCD remap) owns the contiguous range
// [first, last) of the row-major tile order.
struct TileRange {
    int first, last;
};
__device__ __forceinline__ TileRange tile_range(int ntiles) {
    const int L = xcd_tile(blockIdx.x, gridDim.x);
    const int per = ntiles / gridDim.x, extra = ntiles % gridDim.x;
    const int first = L * per + (L < extra ? L : extra);
    return {first, first + per + (L < extra ? 1 : 0)};
}

}  // namespace pfc
