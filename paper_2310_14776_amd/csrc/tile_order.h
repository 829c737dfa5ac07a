// Work order of the tall-skinny contractions on gfx950: which workgroup
// takes which (K chunk, tile, matrix) or (column block, row group), so that
// the workgroups resident on one XCD at the same time read the same rows
// and the XCD's L2 serves the repeats.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gfd {

// Workgroups are dealt to the 8 XCDs round-robin by id and each XCD starts
// its share in id order; the grid is a multiple of 8 and XCD x takes the
// contiguous work items [x per, (x + 1) per), so the workgroups resident on
// one XCD at a time are neighbours in the work order (and share its L2).
__device__ inline int64_t xcd_item() {
  const int64_t per = static_cast<int64_t>(gridDim.x) >> 3;
  return static_cast<int64_t>(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// Tile (tm, tn), tm <= tn, and matrix of item r of one K chunk. Tiles go in
// super-blocks of sb x sb tiles (row-major over the upper triangle of
// super-blocks); inside one, matrix-major, then row-major: sb^2 consecutive
// items read sb tile rows of A and sb of one B, so a round of resident
// workgroups reads each row from HBM about once for sb tiles.
__device__ inline void tile_of(int r, int tiles_n, int nmat, int sb, int &mat, int &tm, int &tn) {
  const int P = (tiles_n + sb - 1) / sb;
  for (int p = 0; p < P; ++p) {
    const int rows = min(sb, tiles_n - p * sb);
    for (int q = p; q < P; ++q) {
      const int cols = min(sb, tiles_n - q * sb);
      const int cnt = p == q ? rows * (rows + 1) / 2 : rows * cols;
      if (r >= cnt * nmat) {
        r -= cnt * nmat;
        continue;
      }
      mat = r / cnt;
      int t = r - mat * cnt;
      if (p == q) {
        int i = 0;
        while (t >= rows - i) {
          t -= rows - i;
          ++i;
        }
        tm = p * sb + i;
        tn = tm + t;
      } else {
        tm = p * sb + t / cols;
        tn = q * sb + t % cols;
      }
      return;
    }
  }
  mat = tm = tn = 0;
}

// Super-block side for slots resident workgroups on the whole chip: about
// the number one XCD holds at a time.
inline int super_block(int64_t slots, int tiles_n) {
  int sb = 1;
  while (static_cast<int64_t>(sb + 1) * (sb + 1) * 8 <= slots) ++sb;
  return sb < tiles_n ? sb : (tiles_n > 0 ? tiles_n : 1);
}

}  // namespace gfd
