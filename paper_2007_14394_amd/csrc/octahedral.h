// Octahedral map border rule shared by the kernels that write padded tiles.
#pragma once

#include <hip/hip_runtime.h>

namespace sdfddgi {

// Write interior texel (i, j) of an n x n map with `comps` channels into its padded
// tile, together with every border texel that copies it: crossing an edge of the
// octahedral square lands on the same edge reflected about its midpoint, and the
// four corners take the diagonally opposite interior corner.
__device__ __forceinline__ void store_with_border(float *__restrict__ tile, int n, int comps,
                                                  int i, int j, int c, float v) {
    const int side = n + 2;
    tile[((j + 1) * side + (i + 1)) * comps + c] = v;
    if (j == 0) tile[(0 * side + (n - i)) * comps + c] = v;
    if (j == n - 1) tile[((n + 1) * side + (n - i)) * comps + c] = v;
    if (i == 0) tile[((n - j) * side + 0) * comps + c] = v;
    if (i == n - 1) tile[((n - j) * side + (n + 1)) * comps + c] = v;
    if (i == n - 1 && j == n - 1) tile[0 * comps + c] = v;
    if (i == 0 && j == n - 1) tile[(n + 1) * comps + c] = v;
    if (i == n - 1 && j == 0) tile[((n + 1) * side) * comps + c] = v;
    if (i == 0 && j == 0) tile[((n + 1) * side + (n + 1)) * comps + c] = v;
}

}  // namespace sdfddgi
