// common.hpp -- device-side constants, tiling and index helpers shared by the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace adjns {

// Work-group tile of output cells for the stencil kernels: 16 x 4 x 4 = 256 threads (four
// 64-wide wavefronts).  x is the unit-stride direction, so each wavefront reads 16-element
// contiguous rows (128 B in FP64, 64 B in FP32) of every plane it touches.
constexpr int TX = 16, TY = 4, TZ = 4, NT = TX * TY * TZ;

// Block size of the 1-D element-wise and reduction kernels.
constexpr int RB = 256;
// Upper bound on the number of per-block FP64 partial sums a reduction writes to the workspace.
constexpr int MAX_PARTIALS = 4096;

template <typename T>
struct Consts {
  int nx, ny, nz, wall;  // wall: 1 = slip walls at x = 0 and x = L_x (mirror ghosts)
  long long N;           // cells
  T dx[3], idx[3];       // cell size and its inverse
  T gamma, mu, alpha, dt;
};

__device__ __forceinline__ int wrap_index(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// x index of a cell or ghost: periodic wrap, or the mirror image across a slip wall.  Ghosts
// further than one cell beyond a wall are only ever read by ragged-tile padding and are clamped.
__device__ __forceinline__ int map_x(int i, int nx, int wall, int& mirror) {
  mirror = 0;
  if (!wall) return wrap_index(i, nx);
  if (i < 0) {
    mirror = 1;
    i = -1 - i;
  } else if (i >= nx) {
    mirror = 1;
    i = 2 * nx - 1 - i;
  }
  return i < 0 ? 0 : (i >= nx ? nx - 1 : i);
}

// Linear cell index of tile-box position (bx, by, bz) for a box whose origin (halo included) is
// at global (x0 - hx, y0 - 1, z0 - 1).
__device__ __forceinline__ long long box_cell(const int nx, const int ny, const int nz, const int wall,
                                              int gx, int gy, int gz, int& mirror, int& real) {
  real = (gx >= 0 && gx < nx) || !wall;
  gx = map_x(gx, nx, wall, mirror);
  gy = wrap_index(gy, ny);
  gz = wrap_index(gz, nz);
  return ((long long)gz * ny + gy) * nx + gx;
}

}  // namespace adjns
