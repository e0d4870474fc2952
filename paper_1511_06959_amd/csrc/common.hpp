// common.hpp -- device-side constants, tiling and index helpers shared by the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace adjns {

// Reference tiling of 16 x 4 x 4 cells: an upper bound on the number of tiles of any kernel that
// writes one partial sum per tile (the workspace's partial-sum region is sized with it).  The
// stencil kernels take their own tile shape (TILE_* below).
constexpr int TX = 16, TY = 4, TZ = 4, NT = TX * TY * TZ;

// Block size of the 1-D element-wise and reduction kernels.
constexpr int RB = 256;
// Upper bound on the number of per-block FP64 partial sums a reduction writes to the workspace.
constexpr int MAX_PARTIALS = 4096;

// LDS box of a TX_ x TY_ x TZ_ tile plus its halo: HX cells in x, HY in y and z.
template <int TX_, int TY_, int TZ_, int HX, int HY>
struct TBox {
  static constexpr int BX = TX_ + 2 * HX, BY = TY_ + 2 * HY, BZ = TZ_ + 2 * HY;
  static constexpr int SY = BX, SZ = BX * BY, NB = BX * BY * BZ;
};

// Tile shapes the stencil kernels are compiled for (index = adj_set_tile's tile id).  A
// wavefront covers 64 consecutive threads, x fastest: rows of 32 let each half-wavefront read 32
// consecutive LDS words (conflict-free) and 128-byte global segments.
enum { TILE_16x4x4 = 0, TILE_32x4x2 = 1, TILE_32x4x4 = 2, TILE_32x8x2 = 3, TILE_32x8x4 = 4, TILE_16x8x8 = 5, NTILES = 6 };
int& tile_choice(int kernel_class, int fp64);

template <typename T>
struct Consts {
  int nx, ny, nz, wall;  // wall: 1 = slip walls at x = 0 and x = L_x (mirror ghosts)
  long long N;           // cells
  T dx[3], idx[3];       // cell size and its inverse
  T gamma, mu, alpha, dt;
  T wref[5];  // reference state: state arrays hold w - wref
  T nuw[5];   // weight of the artificial viscosity on each adjoint component
};

// FP64 primitives of one cell from its five stored values (deviations w - wref), in one fixed order
// of operations shared by every kernel that evaluates the mean-pressure objective or its gradient
// (the objective kernels and the stage kernels that fuse them), so that they round alike.
struct Q64 {
  double rho, u[3], e, p, ri;
};

template <typename T>
__device__ __forceinline__ Q64 q64_of(const Consts<T>& c, T w0, T w1, T w2, T w3, T w4, int mirror, double gamma) {
  Q64 q;
  q.rho = (double)w0 + (double)c.wref[0];
  double m1 = (double)w1 + (double)c.wref[1];
  if (mirror) m1 = -m1;
  const double m2 = (double)w2 + (double)c.wref[2], m3 = (double)w3 + (double)c.wref[3];
  const double Et = (double)w4 + (double)c.wref[4];
  q.ri = 1.0 / q.rho;
  q.u[0] = m1 * q.ri;
  q.u[1] = m2 * q.ri;
  q.u[2] = m3 * q.ri;
  q.e = Et * q.ri - 0.5 * (q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2]);
  q.p = (gamma - 1.0) * q.rho * q.e;
  return q;
}

// Mean pressure j = (1/N) sum p: weight * dj/dw at a cell is f (|u|^2/2, -u, 1) with
// f = weight (gamma - 1)/N (gamma as the kernels hold it, in the state precision).
__device__ __forceinline__ double meanp_factor(double weight, double gamma, long long N) {
  return weight * (gamma - 1.0) / (double)N;
}
template <typename T>
__device__ __forceinline__ void meanp_grad_terms(const Q64& q, double f, T t[5]) {
  const double usq = q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2];
  t[0] = (T)(f * 0.5 * usq);
  t[1] = (T)(-f * q.u[0]);
  t[2] = (T)(-f * q.u[1]);
  t[3] = (T)(-f * q.u[2]);
  t[4] = (T)f;
}

// Buffer loads: a 128-bit resource (base, byte size) in scalar registers plus a 32-bit per-lane
// byte offset and a scalar offset.  One offset per cell then serves every field of every array
// (the scalar offset selects the field), instead of a 64-bit address per load; a read outside
// the resource returns zero.  Arrays must span less than 4 GiB.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const T* p, long long n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), (short)0, (int)(unsigned)(n * (long long)sizeof(T)),
                                           0x00020000);
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// 1/x: the hardware reciprocal in FP32 (within 1 ulp, instead of the ten-instruction correctly
// rounded division), a division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Work-groups of a 1-D launch are dispatched to the eight XCDs round-robin (work-group b on XCD
// b mod 8), and each XCD has its own L2.  xcd_tile turns the dispatch index into a logical tile
// index such that every XCD walks one contiguous run of tiles: tiles that share halo lines (the
// x and y neighbours) then run on the same XCD, close in time, and the lines hit in its L2.
// It is a bijection of [0, nb).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

#ifndef ADJNS_TILE_SLAB
#define ADJNS_TILE_SLAB 4
#endif

// Origin of logical tile t of a TX x TY x TZ tiling of an nx x ny x nz grid.  The tiles are taken
// in slabs of ADJNS_TILE_SLAB tile rows in y: x fastest, then y inside the slab, then z, then the
// next slab.  A tile's x, y and z neighbours then run at most ntx * ADJNS_TILE_SLAB tiles before
// or after it (not a whole x-y layer of tiles), on the same XCD, so the halo planes that they
// share are still in its L2 when the second of them stages its box.  A bijection of [0, ntiles).
template <int TX_, int TY_, int TZ_>
__device__ __forceinline__ void tile_origin(int t, int nx, int ny, int nz, int& x0, int& y0, int& z0) {
  constexpr int SB = ADJNS_TILE_SLAB;
  const int ntx = (nx + TX_ - 1) / TX_, nty = (ny + TY_ - 1) / TY_, ntz = (nz + TZ_ - 1) / TZ_;
  const int slab = ntx * SB * ntz;  // tiles of a full slab; the last slab may hold fewer rows
  const int yb = t / slab;
  const int r = t - yb * slab;
  const int by = min(SB, nty - yb * SB);
  const int r2 = r / ntx;
  x0 = (r - r2 * ntx) * TX_;
  y0 = (yb * SB + r2 % by) * TY_;
  z0 = (r2 / by) * TZ_;
}

// One box of an ensemble (batched launches).  Ensemble arrays are packed box after box: the
// fields of a box start at element 5 * off (state arrays of the boxes) or 5 * aoff (adjoint
// arrays of the members), scalar fields at off; inside a box the layout is the single-box one.
// A member is one adjoint sweep over the trajectory of its box (several members of one box form
// a lambda sweep); for a box entry aoff = off and lam = 0.
template <typename T>
struct BoxDesc {
  Consts<T> c;
  long long off, aoff;
  T lam;  // artificial viscosity coefficient: nu = lam * sigma_1
};

// Index of the box that owns work-group `blk` of a batched launch, given the non-decreasing work
// offsets start[0..n] (start[b] = first work-group of box b).  Every wavefront computes it with
// one vector load and a ballot per 64 boxes; the result is wavefront-uniform.
__device__ __forceinline__ int find_box(const int* __restrict__ start, int n, int blk) {
  int b = 0;
  for (int base = 0; base < n; base += 64) {
    const int i = base + (int)__lane_id();
    const bool before = i < n && start[i + 1] <= blk;
    b += __popcll(__ballot(before));
  }
  return __builtin_amdgcn_readfirstlane(b);
}

// Periodic index.  Halo indices are at most a tile away from [0, n): one conditional shift covers
// them unless the grid is smaller than the tile, which takes the remainder.
__device__ __forceinline__ int wrap_index(int i, int n) {
  int r = i < 0 ? i + n : (i >= n ? i - n : i);
  if (r < 0 || r >= n) {
    r = i % n;
    r = r < 0 ? r + n : r;
  }
  return r;
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

// 32-bit form of box_cell for grids of fewer than 2^31 cells, with the x boundary known at compile
// time (WALL = 1: slip walls, 0: periodic).
template <int WALL>
__device__ __forceinline__ int box_cell32(const int nx, const int ny, const int nz, int gx, int gy, int gz,
                                          int& mirror, int& real) {
  if (WALL) {
    real = gx >= 0 && gx < nx;
    gx = map_x(gx, nx, 1, mirror);
  } else {
    real = 1;
    mirror = 0;
    gx = wrap_index(gx, nx);
  }
  gy = wrap_index(gy, ny);
  gz = wrap_index(gz, nz);
  return (gz * ny + gy) * nx + gx;
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
