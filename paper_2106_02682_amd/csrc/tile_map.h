// Workgroup -> output-tile maps of the symmetric-product kernels (sign_batched.hip, polar.hip),
// shared by the kernels, their launchers and the host-side check exported by the library.
#pragma once

#include <hip/hip_runtime.h>

namespace vemb {

// Upper-triangle tile (ti <= tj) number idx of a tiles x tiles grid, row by row; false past the end.
__host__ __device__ inline bool upper_tile(int idx, int tiles, int* ti, int* tj) {
  if (idx < 0 || tiles <= 0 || idx >= tiles * (tiles + 1) / 2) return false;
  int r = 0, rem = idx;
  while (rem >= tiles - r) {
    rem -= tiles - r;
    ++r;
  }
  *ti = r;
  *tj = r + rem;
  return true;
}

// Workgroups of a single-matrix product: one per upper-triangle tile.
__host__ __device__ inline int upper_tile_count(int tiles) { return tiles * (tiles + 1) / 2; }

// Batched product over `count` blocks: grid (upper_tile_count(tiles), count); workgroup (bx, by) computes
// upper-triangle tile bx of block by.  (Giving all tiles of a block to one XCD, so that its operand
// slices come through one L2, measured 14 % slower on the 256 x 256 products and is not used.)
__host__ __device__ inline bool batched_tile_of(int bx, int by, int count, int tiles, int* block, int* ti, int* tj) {
  if (by < 0 || by >= count) return false;
  *block = by;
  return upper_tile(bx, tiles, ti, tj);
}

}  // namespace vemb
