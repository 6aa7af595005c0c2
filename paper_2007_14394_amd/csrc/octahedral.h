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

// The interior texel (i, j) whose value padded position (x, y) of an n x n tile
// holds (0 <= x, y <= n+1): itself inside, else the texel store_with_border copies
// there.
__host__ __device__ __forceinline__ void padded_source(int n, int x, int y, int &i, int &j) {
    const bool in_x = x >= 1 && x <= n, in_y = y >= 1 && y <= n;
    if (in_x && in_y) { i = x - 1; j = y - 1; return; }
    if (in_x) { i = n - x; j = y == 0 ? 0 : n - 1; return; }           // top / bottom rows
    if (in_y) { j = n - y; i = x == 0 ? 0 : n - 1; return; }           // left / right columns
    i = x == 0 ? n - 1 : 0;                                             // corners
    j = y == 0 ? n - 1 : 0;
}

}  // namespace sdfddgi
