// roe.hip -- gfx950 kernels of the Roe upwind flux option (grid flux ADJ_FLUX_ROE).
//
// The paper's solver propagates waves with Roe's approximate Riemann solver [Numerical methods].
// With that option the convective face flux is Roe's flux of face states reconstructed linearly
// from central cell gradients (second order):
//   w_l = w_L + (w_R - w_{L-e_d})/4,  w_r = w_R - (w_{R+e_d} - w_L)/4,
//   F = (F_d(w_l) + F_d(w_r))/2 - (1/2) sum_k |lam_k|_s a_k r_k
// with the Roe averages (weights sqrt(rho)), the acoustic, entropy and shear waves, and every
// |lam| smoothed within delta = roe_delta c~ of zero ((lam^2 + delta^2)/(2 delta) there), so that
// the flux has a derivative everywhere.
//
// On such grids the stage kernels (stencil.hip) run without their split-form convective flux and
// evaluate the viscous terms, the source and the stage update; the kernels here add the Roe
// convective terms to their output:
//   roe_primal:  out += coef * (-sum_d (F_{d,i+1/2} - F_{d,i-1/2}) / dx_d)
//   roe_adjoint: out += J_F(W)^T kh,  kh = ca a + cg gnext
// (after the stage kernel that wrote `out` with the same W, coefficients and kh).  The reverse
// kernel is the exact transpose: per face, the hand-written reverse of F's evaluation turns
// G = (kh_R - kh_L)/dx_d into adjoint shares of the four cells of the face's stencil.
//
// Both kernels treat one direction at a time: the tile's cells plus a halo along that direction
// only (2 cells forward, 3 in reverse) are staged in LDS, every face of the direction that the
// tile needs is evaluated once into LDS (in reverse: the adjoints of its two face states), and
// each cell then gathers from its faces.  Slip walls:
// ghost cells hold mirrored states and kh = 0; faces between two ghosts do not exist; a wall
// cell adds the shares its ghost images receive, mapped back through the mirror (rho u_x odd).
#include "kernels.hpp"
#include "roe_flux.hpp"

namespace adjns {
namespace {
using namespace roeflux;

// Output tile of both kernels: rows of 16 cells (x), 4 x 4 rows, one cell per thread.
constexpr int RX = 16, RY = 4, RZ = 4, RNT = RX * RY * RZ;

// The tile plus H cells on both sides along direction D (x fastest).
template <int D, int H>
struct Ext {
  static constexpr int EX = RX + (D == 0 ? 2 * H : 0), EY = RY + (D == 1 ? 2 * H : 0), EZ = RZ + (D == 2 ? 2 * H : 0);
  static constexpr int N = EX * EY * EZ;
  static constexpr int S = D == 0 ? 1 : (D == 1 ? EX : EX * EY);  // stride along D
  __device__ static int at(int p, int x, int y, int z) {  // position p along D, tile cross coordinates
    return D == 0 ? (z * EY + y) * EX + p : (D == 1 ? (z * EY + p) * EX + x : (p * EY + y) * EX + x);
  }
};

// NF faces per line along D, lines over the tile's cross section (x fastest).
template <int D, int NF>
struct Faces {
  static constexpr int FX = D == 0 ? NF : RX, FY = D == 1 ? NF : RY, FZ = D == 2 ? NF : RZ;
  static constexpr int N = FX * FY * FZ;
  static constexpr int S = D == 0 ? 1 : (D == 1 ? FX : FX * FY);
  __device__ static int at(int p, int x, int y, int z) {
    return D == 0 ? (z * FY + y) * FX + p : (D == 1 ? (z * FY + p) * FX + x : (p * FY + y) * FX + x);
  }
  __device__ static void coords(int f, int& p, int& x, int& y, int& z) {
    const int fx = f % FX, fy = (f / FX) % FY, fz = f / (FX * FY);
    p = D == 0 ? fx : (D == 1 ? fy : fz);
    x = fx;
    y = fy;
    z = fz;
  }
};

template <int A, int B, int C>
struct Max3c {
  static constexpr int v = A > B ? (A > C ? A : C) : (B > C ? B : C);
};

// Stages the direction-D extended region of the tile at (x0, y0, z0) in LDS: planes 0-4 the cell
// values, and with KH planes 5-9 kh = ca a + cg gnext (zero in ghost cells).
template <typename T, int D, int H, bool KH>
__device__ __forceinline__ void stage(const Consts<T>& c, int x0, int y0, int z0, __amdgpu_buffer_rsrc_t rW,
                                      __amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rg, bool has_g, T ca, T cg,
                                      T* lds, int np) {
  using E = Ext<D, H>;
  constexpr int NIT = (E::N + RNT - 1) / RNT;
  constexpr int NV = KH ? 15 : 5;
  const unsigned fb = (unsigned)(c.N * (long long)sizeof(T));
  // every load of this thread is issued before any is used (one memory latency, not NIT); the
  // tail iteration re-reads the last cell of the region and does not store it
  T w[NIT][NV];
  int mir[NIT], real[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int e = min((int)threadIdx.x + it * RNT, E::N - 1);
    const int ex = e % E::EX, ey = (e / E::EX) % E::EY, ez = e / (E::EX * E::EY);
    const int gx = x0 + ex - (D == 0 ? H : 0), gy = y0 + ey - (D == 1 ? H : 0), gz = z0 + ez - (D == 2 ? H : 0);
    const unsigned off = (unsigned)(c.wall ? box_cell32<1>(c.nx, c.ny, c.nz, gx, gy, gz, mir[it], real[it])
                                           : box_cell32<0>(c.nx, c.ny, c.nz, gx, gy, gz, mir[it], real[it])) *
                         (unsigned)sizeof(T);
#pragma unroll
    for (int v = 0; v < 5; ++v) w[it][v] = buf_load(rW, off, v * fb, T());
    if (KH) {
#pragma unroll
      for (int v = 0; v < 5; ++v) w[it][KH ? 5 + v : 0] = buf_load(ra, off, v * fb, T());
      if (has_g) {
#pragma unroll
        for (int v = 0; v < 5; ++v) w[it][KH ? 10 + v : 0] = buf_load(rg, off, v * fb, T());
      }
    }
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int e = threadIdx.x + it * RNT;
    if (it + 1 < NIT || e < E::N) {
      const T mx = w[it][1] + c.wref[1];
      lds[e] = w[it][0] + c.wref[0];
      lds[np + e] = mir[it] ? -mx : mx;
      lds[2 * np + e] = w[it][2] + c.wref[2];
      lds[3 * np + e] = w[it][3] + c.wref[3];
      lds[4 * np + e] = w[it][4];
      if (KH) {
        // kh = ca a + cg gnext, zero in ghost cells
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          T kh = T(0);
          if (real[it]) {
            kh = ca * w[it][KH ? 5 + v : 0];
            if (has_g) kh += cg * w[it][KH ? 10 + v : 0];
          }
          lds[(5 + v) * np + e] = kh;
        }
      }
    }
  }
}

template <typename T, int D>
__device__ __forceinline__ void load4(const T* lds, int np, int e0, T w[4][5]) {
  constexpr int S = Ext<D, 2>::S;  // the stride along D is the same for every halo
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 5; ++v) w[j][v] = lds[v * np + e0 + j * S];
}

// ---------------------------------------------------------------------------------- forward
constexpr int NSP = Max3c<Ext<0, 2>::N, Ext<1, 2>::N, Ext<2, 2>::N>::v;
constexpr int NFP = Max3c<Faces<0, RX + 1>::N, Faces<1, RY + 1>::N, Faces<2, RZ + 1>::N>::v;

template <typename T, int D>
__device__ __forceinline__ void primal_dir(const Consts<T>& c, const RoeC<T>& k, int x0, int y0, int z0,
                                           __amdgpu_buffer_rsrc_t rW, T* sw, T* sf, int tx, int ty, int tz,
                                           T acc[5]) {
  constexpr int TD = D == 0 ? RX : (D == 1 ? RY : RZ);
  using F = Faces<D, TD + 1>;
  using E = Ext<D, 2>;
  stage<T, D, 2, false>(c, x0, y0, z0, rW, rW, rW, false, T(0), T(0), sw, NSP);
  __syncthreads();
  // face p lies between tile cells p - 1 and p; its stencil is extended positions p .. p + 3
  for (int f = threadIdx.x; f < F::N; f += RNT) {
    int p, x, y, z;
    F::coords(f, p, x, y, z);
    T w[4][5], o[1][5] = {};
    T ql = T(0.25), qr = T(0.25);
    bool live = true;
    if (D == 0 && k.open) {
      // the boundary faces carry the characteristic flux (boundary kernels); next to them the
      // reconstruction does not reach into the ghost cells
      const int gl = x0 + p - 1;
      live = gl >= 0 && gl <= c.nx - 2;
      ql = gl >= 1 ? T(0.25) : T(0);
      qr = gl + 2 <= c.nx - 1 ? T(0.25) : T(0);
    }
    if (live) {
      load4<T, D>(sw, NSP, E::at(p, x, y, z), w);
      roe_face<T, D, false>(w[0], w[1], w[2], w[3], k, ql, qr, nullptr, o);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) sf[v * NFP + f] = o[0][v];
  }
  __syncthreads();
  const int t = D == 0 ? tx : (D == 1 ? ty : tz);
  const int f = F::at(t, tx, ty, tz);
#pragma unroll
  for (int v = 0; v < 5; ++v) acc[v] -= (sf[v * NFP + f + F::S] - sf[v * NFP + f]) * c.idx[D];
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(RNT) void k_roe_primal(Consts<T> c, RoeC<T> k, const T* __restrict__ W, T coef,
                                                    T* __restrict__ out) {
  __shared__ T sw[5 * NSP];
  __shared__ T sf[5 * NFP];
  int x0, y0, z0;
  tile_origin<RX, RY, RZ>(xcd_tile(blockIdx.x, gridDim.x), c.nx, c.ny, c.nz, x0, y0, z0);
  const int tid = threadIdx.x, tx = tid % RX, ty = (tid / RX) % RY, tz = tid / (RX * RY);
  const auto rW = buf_rsrc(W, 5 * c.N);
  T acc[5] = {T(0), T(0), T(0), T(0), T(0)};
  primal_dir<T, 0>(c, k, x0, y0, z0, rW, sw, sf, tx, ty, tz, acc);
  primal_dir<T, 1>(c, k, x0, y0, z0, rW, sw, sf, tx, ty, tz, acc);
  primal_dir<T, 2>(c, k, x0, y0, z0, rW, sw, sf, tx, ty, tz, acc);
  const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
  if (gx >= c.nx || gy >= c.ny || gz >= c.nz) return;
  const long long gi = ((long long)gz * c.ny + gy) * c.nx + gx;
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v * c.N + gi] += coef * acc[v];
}

// ---------------------------------------------------------------------------------- reverse
constexpr int NSA = Max3c<Ext<0, 3>::N, Ext<1, 3>::N, Ext<2, 3>::N>::v;
constexpr int NFA = Max3c<Faces<0, RX + 3>::N, Faces<1, RY + 3>::N, Faces<2, RZ + 3>::N>::v;
constexpr int NLA = 10 * NSA > 10 * NFA ? 10 * NSA : 10 * NFA;

// Reconstruction weights (ql, qr) of the direction-D face with lower cell gl (global index along
// D): 1/4, or 0 where the reconstruction would reach beyond an open boundary.
template <typename T, int D>
__device__ __forceinline__ void face_q(const Consts<T>& c, const RoeC<T>& k, int gl, T& ql, T& qr) {
  ql = qr = T(0.25);
  if (D == 0 && k.open) {
    ql = gl >= 1 ? T(0.25) : T(0);
    qr = gl + 2 <= c.nx - 1 ? T(0.25) : T(0);
  }
}

// Adjoint shares gathered by the cell at tile position t along D (cross coordinates x, y, z)
// from the records (w_l^, w_r^) of the faces p = t .. t + 3 (lower cells t - 2 .. t + 1):
// -qr w_r^ (p = t), ql w_l^ + w_r^ (p = t + 1), w_l^ + qr w_r^ (p = t + 2), -ql w_l^ (p = t + 3).
template <typename T, int D>
__device__ __forceinline__ void gather(const Consts<T>& c, const RoeC<T>& k, const T* fr, int x0, int t, int x, int y,
                                       int z, T sgn1, T acc[5]) {
  constexpr int TD = D == 0 ? RX : (D == 1 ? RY : RZ);
  using F = Faces<D, TD + 3>;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int p = t + q;
    if (p < 0 || p >= TD + 3) continue;
    const int f = F::at(p, x, y, z);
    T ql, qr;
    face_q<T, D>(c, k, x0 + p - 2, ql, qr);
    const T cl = q == 3 ? -ql : (q == 2 ? T(1) : (q == 1 ? ql : T(0)));
    const T cr = q == 0 ? -qr : (q == 1 ? T(1) : (q == 2 ? qr : T(0)));
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T sh = T(0);
      if (q >= 1) sh += cl * fr[v * NFA + f];
      if (q <= 2) sh += cr * fr[(5 + v) * NFA + f];
      acc[v] += (v == 1 ? sgn1 : T(1)) * sh;
    }
  }
}

template <typename T, int D>
__device__ __forceinline__ void adjoint_dir(const Consts<T>& c, const RoeC<T>& k, int x0, int y0, int z0,
                                            __amdgpu_buffer_rsrc_t rW, __amdgpu_buffer_rsrc_t ra,
                                            __amdgpu_buffer_rsrc_t rg, bool has_g, T ca, T cg, T* lds, int tx,
                                            int ty, int tz, bool active, T acc[5]) {
  constexpr int TD = D == 0 ? RX : (D == 1 ? RY : RZ);
  using F = Faces<D, TD + 3>;
  using E = Ext<D, 3>;
  constexpr int NPT = (F::N + RNT - 1) / RNT;
  stage<T, D, 3, true>(c, x0, y0, z0, rW, ra, rg, has_g, ca, cg, lds, NSA);
  __syncthreads();
  // face p lies between tile cells p - 3 and p - 2 (lower cell p - 2); stencil: extended p .. p + 3
  T rec[NPT][2][5];
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int f = threadIdx.x + i * RNT;
    bool live = f < F::N;
    int p = 0, x = 0, y = 0, z = 0;
    if (live) F::coords(f, p, x, y, z);
    T ql, qr;
    face_q<T, D>(c, k, x0 + p - 2, ql, qr);
    if (live && D == 0 && c.wall) {
      const int gl = x0 + p - 2;
      // open boundaries: the boundary faces carry the characteristic flux (boundary kernels);
      // slip walls: a face needs a real cell on at least one side
      live = k.open ? (gl >= 0 && gl <= c.nx - 2) : (gl >= -1 && gl <= c.nx - 1);
    }
    if (live) {
      const int e0 = E::at(p, x, y, z);
      T w[4][5], G[5];
      load4<T, D>(lds, NSA, e0, w);
#pragma unroll
      for (int v = 0; v < 5; ++v) G[v] = (lds[(5 + v) * NSA + e0 + 2 * E::S] - lds[(5 + v) * NSA + e0 + E::S]) * c.idx[D];
      roe_face<T, D, true>(w[0], w[1], w[2], w[3], k, ql, qr, G, rec[i]);
    } else {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 5; ++v) rec[i][j][v] = T(0);
    }
  }
  __syncthreads();  // the face records replace the staged cells
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int f = threadIdx.x + i * RNT;
    if (f < F::N) {
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 5; ++v) lds[(j * 5 + v) * NFA + f] = rec[i][j][v];
    }
  }
  __syncthreads();
  if (active) {
    const int t = D == 0 ? tx : (D == 1 ? ty : tz);
    gather<T, D>(c, k, lds, x0, t, tx, ty, tz, T(1), acc);
    if (D == 0 && c.wall) {
      // shares of the ghost images of this cell (x <= 1: left wall, x >= nx - 2: right wall)
      const int gx = x0 + tx;
      if (gx <= 1) gather<T, D>(c, k, lds, x0, -1 - gx - x0, tx, ty, tz, T(-1), acc);
      if (gx >= c.nx - 2) gather<T, D>(c, k, lds, x0, 2 * c.nx - 1 - gx - x0, tx, ty, tz, T(-1), acc);
    }
  }
  __syncthreads();
}

// FP32: at most 128 registers, so that four work-groups (16 wavefronts) share a compute unit and
// a 64^3 grid (1024 work-groups) runs in one round; FP64 holds two (registers).
template <typename T>
__global__ __launch_bounds__(RNT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
void k_roe_adjoint(Consts<T> c, RoeC<T> k, const T* __restrict__ W,
                                                     const T* __restrict__ a, const T* __restrict__ gnext, T ca, T cg,
                                                     T* __restrict__ out) {
  __shared__ T lds[NLA];
  int x0, y0, z0;
  tile_origin<RX, RY, RZ>(xcd_tile(blockIdx.x, gridDim.x), c.nx, c.ny, c.nz, x0, y0, z0);
  const int tid = threadIdx.x, tx = tid % RX, ty = (tid / RX) % RY, tz = tid / (RX * RY);
  const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
  const bool active = gx < c.nx && gy < c.ny && gz < c.nz;
  const auto rW = buf_rsrc(W, 5 * c.N), ra = buf_rsrc(a, 5 * c.N);
  const bool has_g = gnext != nullptr;
  const auto rg = buf_rsrc(has_g ? gnext : a, 5 * c.N);
  T acc[5] = {T(0), T(0), T(0), T(0), T(0)};
  adjoint_dir<T, 0>(c, k, x0, y0, z0, rW, ra, rg, has_g, ca, cg, lds, tx, ty, tz, active, acc);
  adjoint_dir<T, 1>(c, k, x0, y0, z0, rW, ra, rg, has_g, ca, cg, lds, tx, ty, tz, active, acc);
  adjoint_dir<T, 2>(c, k, x0, y0, z0, rW, ra, rg, has_g, ca, cg, lds, tx, ty, tz, active, acc);
  if (!active) return;
  const long long gi = ((long long)gz * c.ny + gy) * c.nx + gx;
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v * c.N + gi] += acc[v];
}

template <typename T>
int roe_tiles(const Consts<T>& c) {
  return ((c.nx + RX - 1) / RX) * ((c.ny + RY - 1) / RY) * ((c.nz + RZ - 1) / RZ);
}

}  // namespace

template <typename T>
hipError_t launch_roe_primal(const Consts<T>& c, T roe_delta, int open, const T* W, T coef, T* out, hipStream_t st) {
  ProfScope ps(ADJ_PROF_ROE_PRIMAL, st, true);
  timed_launch(ps, k_roe_primal<T>, dim3(roe_tiles(c)), dim3(RNT), st, c, roe_consts(c, roe_delta, open), W, coef,
               out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_roe_adjoint(const Consts<T>& c, T roe_delta, int open, const T* W, const T* a, const T* gnext, T ca,
                              T cg, T* out, hipStream_t st) {
  ProfScope ps(ADJ_PROF_ROE_ADJOINT, st, true);
  timed_launch(ps, k_roe_adjoint<T>, dim3(roe_tiles(c)), dim3(RNT), st, c, roe_consts(c, roe_delta, open), W, a,
               gnext, ca, cg, out);
  return hipGetLastError();
}

#define ADJNS_ROE_INST(T)                                                                                          \
  template hipError_t launch_roe_primal<T>(const Consts<T>&, T, int, const T*, T, T*, hipStream_t);                \
  template hipError_t launch_roe_adjoint<T>(const Consts<T>&, T, int, const T*, const T*, const T*, T, T, T*,       \
                                            hipStream_t);
ADJNS_ROE_INST(float)
ADJNS_ROE_INST(double)
#undef ADJNS_ROE_INST

}  // namespace adjns
