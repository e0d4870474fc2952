// char.hip -- gfx950 kernels of the characteristic inflow/outflow boundaries in x
// (grid bc_x ADJ_BC_CHARACTERISTIC): the flux through the two boundary faces replaced by Roe's
// flux against far-field states, and its transpose.
#include "kernels.hpp"
#include "roe_flux.hpp"

namespace adjns {
namespace {
using namespace roeflux;

// The stage kernels treat the open boundaries as slip walls (mirror ghosts), so through each
// boundary face they evaluate the mirror-pair flux H_w = (0, p - p0 - s_xx, 0, 0, 0), or
// (0, -s_xx, 0, 0, 0) when they run without the split-form convective flux (Roe grids, whose Roe
// kernels skip the boundary faces): the mirror pair carries no mass, energy, tangential stress or
// heat, and s_xx = (4/3) mu g_n - (2/3) mu (d_y u_y + d_z u_z) with the normal gradient
// g_n = +-2 u_x/dx of the pair and the boundary cell's central tangential divergence.  The
// kernels here replace H_w by the characteristic flux F_c, Roe's flux between the far-field state
// and the boundary cell (x = 0) or the boundary cell and the far-field state (x = L_x), which
// takes the entering waves from the far field and the leaving ones from inside
// [Numerical methods; Boundary conditions of the adjoint]:
//   char_primal:  out += coef * (+-)(F_c - H_w)/dx at the boundary cells (+ at x = 0)
//   char_adjoint: out += (its Jacobian)^T kh, gathered per boundary cell (s_xx also reaches the
//                 y and z neighbours of a boundary cell through the tangential divergence)
// One thread per boundary cell of either side.
template <typename T>
struct Far {
  T w[2][5];  // held far-field states beyond x = 0 and beyond x = L_x
};

constexpr int CB = 256;

template <typename T>
struct BCell {
  int side;
  long long q, jm, jp, km, kp;  // the cell and its y and z neighbours (periodic)
};

template <typename T>
__device__ __forceinline__ bool bcell(const Consts<T>& c, int t, BCell<T>& b) {
  const int ncol = c.ny * c.nz;
  if (t >= 2 * ncol) return false;
  b.side = t >= ncol;
  const int r = t - b.side * ncol, j = r % c.ny, kz = r / c.ny, i = b.side ? c.nx - 1 : 0;
  const int jp = j + 1 < c.ny ? j + 1 : 0, jm = j > 0 ? j - 1 : c.ny - 1;
  const int kp = kz + 1 < c.nz ? kz + 1 : 0, km = kz > 0 ? kz - 1 : c.nz - 1;
  auto at = [&](int jj, int kk) { return ((long long)kk * c.ny + jj) * c.nx + i; };
  b.q = at(j, kz);
  b.jm = at(jm, kz);
  b.jp = at(jp, kz);
  b.km = at(j, km);
  b.kp = at(j, kp);
  return true;
}

template <typename T>
__device__ __forceinline__ void held(const Consts<T>& c, const T* __restrict__ W, long long q, T w[5]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) w[v] = W[v * c.N + q] + c.wref[v];
  w[4] = W[4 * c.N + q];
}

template <typename T>
__global__ __launch_bounds__(CB) void k_char_primal(Consts<T> c, RoeC<T> k, Far<T> far, const T* __restrict__ W,
                                                    T coef, T* __restrict__ out) {
  BCell<T> b;
  if (!bcell(c, (int)(blockIdx.x * CB + threadIdx.x), b)) return;
  T w[5], o[5];
  held(c, W, b.q, w);
#pragma unroll
  for (int v = 0; v < 5; ++v) o[v] = out[v * c.N + b.q];  // issued with the state loads
  auto uy = [&](long long q) { return (W[2 * c.N + q] + c.wref[2]) / (W[q] + c.wref[0]); };
  auto uz = [&](long long q) { return (W[3 * c.N + q] + c.wref[3]) / (W[q] + c.wref[0]); };
  const T div_t = (uy(b.jp) - uy(b.jm)) * (T(0.5) * c.idx[1]) + (uz(b.kp) - uz(b.km)) * (T(0.5) * c.idx[2]);
  const T gn = (b.side ? T(-2) : T(2)) * (w[1] / w[0]) * c.idx[0];
  const T sxx = (T(4) / T(3)) * c.mu * gn - (T(2) / T(3)) * c.mu * div_t;
  T F[5];
  if (b.side)
    roe_flux2<T, 0, false>(w, far.w[1], k, nullptr, F, nullptr, nullptr);
  else
    roe_flux2<T, 0, false>(far.w[0], w, k, nullptr, F, nullptr, nullptr);
  F[1] -= (k.split ? prim_of(w, k).pd : T(0)) - sxx;
  const T f = coef * (b.side ? -c.idx[0] : c.idx[0]);
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v * c.N + b.q] = o[v] + f * F[v];
}

template <typename T>
__global__ __launch_bounds__(CB) void k_char_adjoint(Consts<T> c, RoeC<T> k, Far<T> far, const T* __restrict__ W,
                                                     const T* __restrict__ a, const T* __restrict__ gnext, T ca, T cg,
                                                     T* __restrict__ out) {
  BCell<T> b;
  if (!bcell(c, (int)(blockIdx.x * CB + threadIdx.x), b)) return;
  auto kh = [&](int v, long long q) { return ca * a[v * c.N + q] + (gnext ? cg * gnext[v * c.N + q] : T(0)); };
  const T sg = b.side ? -c.idx[0] : c.idx[0];
  T w[5], G[5], o[5];
  held(c, W, b.q, w);
#pragma unroll
  for (int v = 0; v < 5; ++v) o[v] = out[v * c.N + b.q];  // issued with the state loads
#pragma unroll
  for (int v = 0; v < 5; ++v) G[v] = sg * kh(v, b.q);
  T wb[5] = {T(0), T(0), T(0), T(0), T(0)}, fb[5] = {T(0), T(0), T(0), T(0), T(0)};
  if (b.side)
    roe_flux2<T, 0, true>(w, far.w[1], k, G, nullptr, wb, fb);
  else
    roe_flux2<T, 0, true>(far.w[0], w, k, G, nullptr, fb, wb);
  // - G_1 (p - p0 - s_xx) of this cell and of its y / z neighbours (through their divergence)
  const T m23 = (T(2) / T(3)) * c.mu;
  T ub[3];
  ub[0] = G[1] * (T(4) / T(3)) * c.mu * (b.side ? T(-2) : T(2)) * c.idx[0];
  ub[1] = -m23 * (T(0.5) * c.idx[1]) * sg * (kh(1, b.jm) - kh(1, b.jp));
  ub[2] = -m23 * (T(0.5) * c.idx[2]) * sg * (kh(1, b.km) - kh(1, b.kp));
  prim_of_vjp(w, prim_of(w, k), k, ub, k.split ? -G[1] : T(0), T(0), T(0), wb);
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v * c.N + b.q] = o[v] + wb[v];
}

}  // namespace

template <typename T>
static Far<T> far_held(const Consts<T>& c, const double* w_far) {
  Far<T> f;
  for (int s = 0; s < 2; ++s)
    for (int v = 0; v < 5; ++v) f.w[s][v] = (T)(v == 4 ? w_far[5 * s + 4] - (double)c.wref[4] : w_far[5 * s + v]);
  return f;
}

template <typename T>
hipError_t launch_char_primal(const Consts<T>& c, T roe_delta, int split, const double* w_far, const T* W, T coef,
                              T* out, hipStream_t st) {
  ProfScope ps(ADJ_PROF_BOUNDARY, st, true);
  const int n = 2 * c.ny * c.nz;
  timed_launch(ps, k_char_primal<T>, dim3((n + CB - 1) / CB), dim3(CB), st, c, roe_consts(c, roe_delta, 1, split),
               far_held(c, w_far), W, coef, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_char_adjoint(const Consts<T>& c, T roe_delta, int split, const double* w_far, const T* W,
                               const T* a, const T* gnext, T ca, T cg, T* out, hipStream_t st) {
  ProfScope ps(ADJ_PROF_BOUNDARY, st, true);
  const int n = 2 * c.ny * c.nz;
  timed_launch(ps, k_char_adjoint<T>, dim3((n + CB - 1) / CB), dim3(CB), st, c, roe_consts(c, roe_delta, 1, split),
               far_held(c, w_far), W, a, gnext, ca, cg, out);
  return hipGetLastError();
}

#define ADJNS_CHAR_INST(T)                                                                                          \
  template hipError_t launch_char_primal<T>(const Consts<T>&, T, int, const double*, const T*, T, T*, hipStream_t); \
  template hipError_t launch_char_adjoint<T>(const Consts<T>&, T, int, const double*, const T*, const T*, const T*, \
                                             T, T, T*, hipStream_t);
ADJNS_CHAR_INST(float)
ADJNS_CHAR_INST(double)
#undef ADJNS_CHAR_INST

}  // namespace adjns
