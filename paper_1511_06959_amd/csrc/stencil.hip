// stencil.hip -- gfx950 kernels for one Runge-Kutta stage of the primal residual and one reverse
// stage of the discrete adjoint (transposed convective, viscous and artificial-viscosity operators).
//
// Both kernels stage a box of cells (the work-group's output tile, one of the TILE_* shapes, plus
// a halo of one cell, two in x beside slip walls) in LDS, derive the primitive variables once per
// box cell, and then evaluate each output cell's 19-point stencil from LDS.  SoA var-major global
// layout; every global access of a wavefront is to consecutive x addresses.  A CONV = 0
// instantiation leaves the split-form convective terms out, for grids whose convective flux the
// Roe kernels (roe.hip) add.
#include <type_traits>

#include "kernels.hpp"

namespace adjns {

// ------------------------------------------------------------------------------------------
// Primal residual  R = -sum_d (F~_{d,+} - F~_{d,-})/dx_d + s  with the face flux
//   F~ = r v_d (1, v, H) + P (0, e_d, v_d) - (0, sigma_d., u_f . sigma_d. + alpha d_d e)
// where r, v, H, P are the face means of rho, u, E/rho and p (split product form of Kennedy &
// Gruber, which conserves kinetic energy under convection; the paper's LES instead leans on the
// dissipation of its upwind flux) [Physics, Eq. navier; Unsteady adjoint, vector form with source].
// ------------------------------------------------------------------------------------------
namespace {

// LDS field order of the primal box (P_H: specific total energy E/rho).  The planes hold HALF of
// each field, so that a face mean is one addition (halving is exact: the sums round exactly as
// the halved sums of the full values would).
enum { P_RHO = 0, P_U1, P_U2, P_U3, P_E, P_P, P_H, P_NF };

// Convective flux through the direction-D face between box cells a (lower) and b.  The P_P planes
// hold p - p0 (p0 = (gamma-1) wref_E, the pressure of the reference state): the momentum flux
// carries that deviation, since a uniform pressure has no divergence, and keeps its low-order
// digits in FP32 at low Mach number; the energy flux takes the full mean pressure.
template <typename T, int NB, int D>
__device__ __forceinline__ void conv_face(const T (*sm)[NB], int a, int b, T p0, T F[5]) {
  const T r = sm[P_RHO][a] + sm[P_RHO][b];
  const T v[3] = {sm[P_U1][a] + sm[P_U1][b], sm[P_U2][a] + sm[P_U2][b], sm[P_U3][a] + sm[P_U3][b]};
  const T H = sm[P_H][a] + sm[P_H][b], Pd = sm[P_P][a] + sm[P_P][b];
  const T m = r * v[D];
  F[0] = m;
#pragma unroll
  for (int k = 0; k < 3; ++k) F[1 + k] = m * v[k] + (k == D ? Pd : T(0));
  F[4] = m * H + (Pd + p0) * v[D];
}

// Forward viscous stress row sigma_d. on the face between box cells A and A + e_d.
// Velocity fields are read from `U` (three LDS planes of NB values holding u/2).
template <typename T, int NB, int D>
__device__ __forceinline__ void face_stress(const T* __restrict__ U, const int st[3], int A, T mu,
                                            const T idx[3], T sig[3]) {
  constexpr int t1 = D == 0 ? 1 : 0, t2 = D == 2 ? 1 : 2;
  const int B = A + st[D];
  const T in = T(2) * idx[D];
  T gn[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gn[k] = (U[k * NB + B] - U[k * NB + A]) * in;
  // tangential gradients d_t u_D and d_t u_t at the face: mean of the two cells' central differences
  const T q1 = T(0.5) * idx[t1], q2 = T(0.5) * idx[t2];
  const int s1 = st[t1], s2 = st[t2];
  const T g1D = (U[D * NB + A + s1] - U[D * NB + A - s1] + U[D * NB + B + s1] - U[D * NB + B - s1]) * q1;
  const T g11 = (U[t1 * NB + A + s1] - U[t1 * NB + A - s1] + U[t1 * NB + B + s1] - U[t1 * NB + B - s1]) * q1;
  const T g2D = (U[D * NB + A + s2] - U[D * NB + A - s2] + U[D * NB + B + s2] - U[D * NB + B - s2]) * q2;
  const T g22 = (U[t2 * NB + A + s2] - U[t2 * NB + A - s2] + U[t2 * NB + B + s2] - U[t2 * NB + B - s2]) * q2;
  const T div = gn[D] + g11 + g22;
  sig[D] = mu * (T(2) * gn[D]) - (T(2) / T(3)) * mu * div;
  sig[t1] = mu * (gn[t1] + g1D);
  sig[t2] = mu * (gn[t2] + g2D);
}

template <typename T, int NB, int D>
__device__ __forceinline__ void visc_flux(const T (*sm)[NB], const int st[3], int A, const Consts<T>& c,
                                          T G[4]) {
  T sig[3];
  face_stress<T, NB, D>(&sm[P_U1][0], st, A, c.mu, c.idx, sig);
  const int B = A + st[D];
  T work = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) work += (sm[P_U1 + k][A] + sm[P_U1 + k][B]) * sig[k];
  G[0] = sig[0];
  G[1] = sig[1];
  G[2] = sig[2];
  G[3] = work + (T(2) * c.alpha) * (sm[P_E][B] - sm[P_E][A]) * c.idx[D];
}

// CONV = 0: the viscous terms only (grids whose convective flux another kernel adds).
template <typename T, int NB, int D, int CONV>
__device__ __forceinline__ void residual_dir(const T (*sm)[NB], const int st[3], int p, const Consts<T>& c,
                                             T R[5]) {
  if constexpr (CONV) {
    T Fp[5], Fm[5];
    const T p0 = (c.gamma - T(1)) * c.wref[4];
    conv_face<T, NB, D>(sm, p, p + st[D], p0, Fp);
    conv_face<T, NB, D>(sm, p - st[D], p, p0, Fm);
    const T h = c.idx[D];
#pragma unroll
    for (int v = 0; v < 5; ++v) R[v] -= (Fp[v] - Fm[v]) * h;
  }
  T Gp[4], Gm[4];
  visc_flux<T, NB, D>(sm, st, p, c, Gp);
  visc_flux<T, NB, D>(sm, st, p - st[D], c, Gm);
#pragma unroll
  for (int k = 0; k < 4; ++k) R[1 + k] += (Gp[k] - Gm[k]) * c.idx[D];
}

}  // namespace

// MODE: RES  out = R(W; s)
//       LIN  out = wn + cR * R(W; s)                           (RK4 stages 1-3)
//       LIN_DISS  LIN that also sums the viscous dissipation of W over the tile into jpart (stage 1:
//            W = w_n; a mode of its own, so that the other stage launches carry none of its work)
//       AFF  out = ca wn + cb W + cR * R(W; s)                 (SSP-RK3 stages)
//       FIN  out = (W2 + 2 W3 + W - wn)/3 + (dt/6) R(W; s)      (stage 4, W = W4;
//            equals wn + dt/6 (k1 + 2 k2 + 2 k3 + k4) since k1 = 2(W2-wn)/dt, k2 = 2(W3-wn)/dt,
//            k3 = (W4-wn)/dt)
// CONV = 0 leaves out the split-form convective flux (the Roe option adds its own).
// One work-group: the tile with origin (x0, y0, z0).
constexpr int STAGE_LIN_DISS = 4;

template <typename T, int MODE, int CONV, int TX, int TY, int TZ>
__device__ __forceinline__ void primal_tile_body(const Consts<T>& c, const int x0, const int y0, const int z0,
                                                 const T* __restrict__ W, const T* __restrict__ wn,
                                                 const T* __restrict__ s, const T* __restrict__ W2,
                                                 const T* __restrict__ W3, const T cR, T* __restrict__ out,
                                                 const T ca = T(0), const T cb = T(0), double* __restrict__ jpart = nullptr,
                                                 const int tile = 0) {
  constexpr int NT = TX * TY * TZ;
  using Bx = TBox<TX, TY, TZ, 1, 1>;
  constexpr int NB = Bx::NB;
  __shared__ T sm[P_NF][NB];
  const int tid = threadIdx.x;
  const long long N = c.N;
  const T gm1 = c.gamma - T(1);
  // all of this thread's box loads are issued before any is used: one memory latency, not NIT
  // (branch-free: the tail iteration re-reads the last box cell and does not store it)
  constexpr int NIT = (NB + NT - 1) / NT;
  T wv[NIT][5];
  int mir[NIT];
  const auto rW = buf_rsrc(W, 5 * N);
  const unsigned fb = (unsigned)(N * (long long)sizeof(T));  // bytes per field
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int b = min(tid + it * NT, NB - 1);
    const int bx = b % Bx::BX, by = (b / Bx::BX) % Bx::BY, bz = b / (Bx::BX * Bx::BY);
    int real;
    const int gx = x0 + bx - 1, gy = y0 + by - 1, gz = z0 + bz - 1;
    const unsigned off = (unsigned)(c.wall ? box_cell32<1>(c.nx, c.ny, c.nz, gx, gy, gz, mir[it], real)
                                           : box_cell32<0>(c.nx, c.ny, c.nz, gx, gy, gz, mir[it], real)) *
                         (unsigned)sizeof(T);
#pragma unroll
    for (int v = 0; v < 5; ++v) wv[it][v] = buf_load(rW, off, v * fb, T());
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int b = tid + it * NT;
    if (it + 1 < NIT || b < NB) {
      // stored deviations w - wref; Ed = rho E - wref_E stays a deviation
      const T r = wv[it][0] + c.wref[0], Ed = wv[it][4];
      const T mx = wv[it][1] + c.wref[1], m1 = mir[it] ? -mx : mx;
      const T ri = recip(r), hri = T(0.5) * ri;
      const T h1 = m1 * hri, h2 = (wv[it][2] + c.wref[2]) * hri, h3 = (wv[it][3] + c.wref[3]) * hri;  // u/2
      const T hk = r * (h1 * h1 + h2 * h2 + h3 * h3);                      // kinetic energy / 2
      // pressure deviation from the small stored deviation: p - p0 = (gamma-1)(Ed - K)
      const T hp = gm1 * (T(0.5) * Ed - hk);                               // (p - p0)/2
      sm[P_RHO][b] = T(0.5) * r;
      sm[P_U1][b] = h1;
      sm[P_U2][b] = h2;
      sm[P_U3][b] = h3;
      const T hH = (Ed + c.wref[4]) * hri;                                 // (E/rho)/2
      sm[P_E][b] = hH - (h1 * h1 + h2 * h2 + h3 * h3);                     // e/2
      sm[P_P][b] = hp;
      sm[P_H][b] = hH;

    }
  }
  const int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / (TX * TY);
  const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
  const bool active = gx < c.nx && gy < c.ny && gz < c.nz;
  const long long gi = ((long long)(active ? gz : 0) * c.ny + (active ? gy : 0)) * c.nx + (active ? gx : 0);
  // per-cell operands, fetched before the barrier so that their latency overlaps the staging
  T sv[5] = {T(0), T(0), T(0), T(0), T(0)}, base[5], wq[5];
  // the final stage fetches the cell's own W here too, except where the five more registers would
  // spill (FP64 work-groups of 1024 threads, capped at 128 registers)
  constexpr bool PREW = sizeof(T) == 4 || NT <= 512;
  if (active) {
    if (s) {
#pragma unroll
      for (int v = 0; v < 5; ++v) sv[v] = s[v * N + gi];
    }
    if (MODE == STAGE_LIN || MODE == STAGE_LIN_DISS) {
#pragma unroll
      for (int v = 0; v < 5; ++v) base[v] = wn[v * N + gi];
    } else if (MODE == STAGE_AFF) {
#pragma unroll
      for (int v = 0; v < 5; ++v) base[v] = ca * wn[v * N + gi] + cb * W[v * N + gi];
    } else if (MODE == STAGE_FIN) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const long long q = v * N + gi;
        base[v] = (W2[q] + T(2) * W3[q] - wn[q]);
        if (PREW) wq[v] = W[q];
      }
    }
  }
  __syncthreads();
  double pv = 0.0;  // the new state's pressure (final stage) or w_n's dissipation (stage 1) at the cell
  if (active) {
    const int st[3] = {1, Bx::SY, Bx::SZ};
    const int p = (tz + 1) * Bx::SZ + (ty + 1) * Bx::SY + (tx + 1);
    if (MODE == STAGE_LIN_DISS) {
      // the viscous dissipation sigma : grad u of the staged state at the cell (stage 1 of a step,
      // W = w_n): central velocity gradients from the LDS planes, which hold u/2, so that a
      // difference times 1/dx is the central derivative
      T G[3][3];
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int k = 0; k < 3; ++k) G[l][k] = (sm[P_U1 + k][p + st[l]] - sm[P_U1 + k][p - st[l]]) * c.idx[l];
      const T div = G[0][0] + G[1][1] + G[2][2];
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          T sg = c.mu * (G[l][k] + G[k][l]);
          if (l == k) sg -= (T(2) / T(3)) * c.mu * div;
          acc += sg * G[l][k];
        }
      pv = (double)acc;
    }
    T R[5] = {sv[0], sv[1], sv[2], sv[3], sv[4]};
    residual_dir<T, NB, 0, CONV>(sm, st, p, c, R);
    __builtin_amdgcn_sched_barrier(0);
    residual_dir<T, NB, 1, CONV>(sm, st, p, c, R);
    __builtin_amdgcn_sched_barrier(0);
    residual_dir<T, NB, 2, CONV>(sm, st, p, c, R);
    __builtin_amdgcn_sched_barrier(0);
    if (MODE == STAGE_RES) {
#pragma unroll
      for (int v = 0; v < 5; ++v) out[v * N + gi] = R[v];
    } else if (MODE == STAGE_LIN || MODE == STAGE_LIN_DISS || MODE == STAGE_AFF) {
#pragma unroll
      for (int v = 0; v < 5; ++v) out[v * N + gi] = base[v] + cR * R[v];
    } else {
      const T third = T(1) / T(3), h6 = c.dt / T(6);
      T o[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        o[v] = (base[v] + (PREW ? wq[v] : W[v * N + gi])) * third + h6 * R[v];
        out[v * N + gi] = o[v];
      }
      if (MODE == STAGE_FIN && jpart) pv = q64_of(c, o[0], o[1], o[2], o[3], o[4], 0, (double)c.gamma).p;
    }
  }
  if ((MODE == STAGE_FIN && jpart) || MODE == STAGE_LIN_DISS) {
    // the tile's sum of the new state's pressures (final stage: the mean-pressure objective of
    // the step's output) or of the input state's dissipation (stage 1), in a fixed order:
    // butterfly within each wavefront, then the wavefronts in order
    __shared__ double red[NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) pv += __shfl_xor(pv, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = pv;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < NT / 64; ++k) t += red[k];
      jpart[tile] = t;
    }
  }
}

template <typename T, int MODE, int CONV, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX * TY * TZ) void k_primal_stage(Consts<T> c, const T* __restrict__ W,
                                                               const T* __restrict__ wn, const T* __restrict__ s,
                                                               const T* __restrict__ W2, const T* __restrict__ W3,
                                                               T cR, T* __restrict__ out, T ca, T cb,
                                                               double* __restrict__ jpart) {
  int x0, y0, z0;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  tile_origin<TX, TY, TZ>(t, c.nx, c.ny, c.nz, x0, y0, z0);
  primal_tile_body<T, MODE, CONV, TX, TY, TZ>(c, x0, y0, z0, W, wn, s, W2, W3, cR, out, ca, cb, jpart, t);
}

// Ensemble form: work-group -> (box, tile) through the tile offsets `start`; every array is
// packed box after box.  cfac scales the box's own dt into the stage coefficient.
template <typename T, int MODE, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX * TY * TZ) void k_primal_stage_batch(const BoxDesc<T>* __restrict__ boxes,
                                                                     const int* __restrict__ start, int nbox,
                                                                     const T* __restrict__ W, const T* __restrict__ wn,
                                                                     const T* __restrict__ s, const T* __restrict__ W2,
                                                                     const T* __restrict__ W3, T cfac,
                                                                     T* __restrict__ out) {
  const int blk = xcd_tile(blockIdx.x, gridDim.x);
  const int b = find_box(start, nbox, blk);
  const Consts<T> c = boxes[b].c;
  const long long o = 5 * boxes[b].off;
  int x0, y0, z0;
  tile_origin<TX, TY, TZ>(blk - start[b], c.nx, c.ny, c.nz, x0, y0, z0);
  primal_tile_body<T, MODE, 1, TX, TY, TZ>(c, x0, y0, z0, W + o, wn + o, s ? s + o : nullptr,
                                        W2 ? W2 + o : nullptr, W3 ? W3 + o : nullptr, c.dt * cfac, out + o);
}

// ------------------------------------------------------------------------------------------
// Reverse stage:  g = J_R(W)^T kh + L_nu kh,  kh = ca * a + cg * gnext formed on load
// [Unsteady adjoint: A_ijk, A^v_ijk, D_ijkl and the adjoint equation; Implementation: discrete
// adjoint; Stabilizing adjoint equations: lambda sigma_1 delta_ki delta_jl term].
//
// Gather form for output cell j (all terms are the exact transpose of the primal residual):
//   convective  each face f of j (direction d, cells L|R) with face means r, v, H, P and
//               G = (kh_R - kh_L)/dx_d, phi = G_0 + v.G_m + H G_E, m = r v_d hands j half of
//                 r^ = v_d phi,  v^ = m G_m + (r phi + P G_E) e_d,  H^ = m G_E,  P^ = G_m,d + v_d G_E
//               (the adjoints of the face means; each mean is half of each cell's value);
//               H^ and P^ then move to (rho, u, e) through E/rho = e + |u|^2/2, p = (gamma-1) rho e
//   viscous     adjoint of the primitive fields (u^, e^) at j collected from
//               - its six faces f (direction d, cells L|R):  G^ = (kh_L - kh_R)/dx_d,
//                 sigma^_k = G^_mk + G^_E u_f,k,
//                 normal part  tau^_dk/dx_d = (mu sigma^_k + (mu/3) sigma^_d delta_kd)/dx_d
//                 (to R with +, to L with -), work part 0.5 G^_E sigma_dk (to both),
//                 heat part alpha G^_E / dx_d (to R with +, to L with -);
//               - the tangential-gradient chain:  u^_j += sum_l (C_l(j-e_l) - C_l(j+e_l))/(2 dx_l)
//                 with C_l(c) = 0.5 sum_{d != l} sum_{faces of c in d} (mu sigma^_l e_d - (2mu/3) sigma^_d e_l);
//               then (rho^, u^, e^) -> conservative adjoint through u = m/rho, e = E/rho - |u|^2/2.
//   L_nu        sum_d sum_{+-} nu_f (kh_nb - kh_j)/dx_d^2, nu_f = (nu_j + nu_nb)/2, no wall faces.
// Slip walls: ghost cells carry mirrored primitives and kh = 0 (they own no residual); a cell
// next to a wall adds what its ghost image receives, mapped back through the mirror (u_x odd).
// For the convective part that is the wall face's second half-share; the viscous part gathers
// at the ghost image.
//
// Every viscous face adjoint sigma^ is shared by six cells (the two it separates and four
// tangential neighbours), so the kernel evaluates those faces once per work-group, one direction
// at a time: a face-record buffer in LDS receives s~ = dx_d sigma^ and dK_E = kh_E,L - kh_E,R of
// all direction-d faces of the box, plus the work term 0.5 G^_E sigma_d. of the faces bounding
// the tile; the cells then gather from the records.  Three record phases reuse one buffer, which
// before them holds rho, E/rho and p of the box for the convective gather.
// ------------------------------------------------------------------------------------------
namespace {

enum { A_K0 = 0, A_K1, A_K2, A_K3, A_K4, A_U1, A_U2, A_U3, A_NU };

// Direction-D faces of the box, indexed by their lower cell (ax, ay, az) in box coordinates.
// Records cover every lower cell that a tile cell or a tangential neighbour needs, in a compact
// array (rows of NX lower cells); work terms (Q) cover the faces bounding tile cells.
template <int TX, int TY, int TZ, int HX, int D>
struct FaceSet {
  using B = TBox<TX, TY, TZ, HX, 1>;
  static constexpr int X0 = D == 0 ? HX - 1 : 0;
  static constexpr int NX = D == 0 ? TX + 1 : B::BX;
  static constexpr int NY = D == 1 ? TY + 1 : B::BY;
  static constexpr int NZ = D == 2 ? TZ + 1 : B::BZ;
  static constexpr int N = NX * NY * NZ;
  static constexpr int STEP = D == 0 ? 1 : (D == 1 ? B::SY : B::SZ);  // box-index step to the upper cell
  static constexpr int QX0 = D == 0 ? HX - 1 : HX;
  static constexpr int QY0 = D == 1 ? 0 : 1;
  static constexpr int QZ0 = D == 2 ? 0 : 1;
  static constexpr int NQX = D == 0 ? TX + 1 : TX;
  static constexpr int NQY = D == 1 ? TY + 1 : TY;
  static constexpr int NQZ = D == 2 ? TZ + 1 : TZ;
  static constexpr int NQ = NQX * NQY * NQZ;
  __device__ static int idx(int ax, int ay, int az) { return (ax - X0) + NX * (ay + NY * az); }
  // box index of the lower cell of record f: the records skip BX - NX box cells per row (D = 0)
  // or BX per z-layer (D = 1) and none for D = 2, so one constant division finds it
  __device__ static int box(int f) {
    if constexpr (D == 0) return f + (f / NX) * (B::BX - NX) + X0;
    else if constexpr (D == 1) return f + (f / (NX * NY)) * (B::SZ - NX * NY);
    else return f;
  }
  __device__ static int qidx(int ax, int ay, int az) { return (ax - QX0) + NQX * ((ay - QY0) + NQY * (az - QZ0)); }
  __device__ static bool has(int ax) { return ax >= X0 && ax < X0 + NX; }
  __device__ static bool hasq(int ax) { return ax >= QX0 && ax < QX0 + NQX; }
};

template <int A, int B, int C>
struct Max3 {
  static constexpr int v = A > B ? (A > C ? A : C) : (B > C ? B : C);
};

// Record phase of direction D (all threads).
template <typename T, int TX, int TY, int TZ, int HX, int D, int NB, int NF, int NQF>
__device__ __forceinline__ void face_records(const T (*sm)[NB], T (*fr)[NF], T (*fq)[NQF], const int st[3],
                                             const Consts<T>& c) {
  using F = FaceSet<TX, TY, TZ, HX, D>;
  using B = TBox<TX, TY, TZ, HX, 1>;
  constexpr int NT = TX * TY * TZ;
  for (int f = threadIdx.x; f < F::N; f += NT) {
    const int A = F::box(f), Bc = A + F::STEP;
    const T dK4 = sm[A_K4][A] - sm[A_K4][Bc];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      fr[k][f] = (sm[A_K1 + k][A] - sm[A_K1 + k][Bc]) + dK4 * (sm[A_U1 + k][A] + sm[A_U1 + k][Bc]);
    fr[3][f] = dK4;
  }
  const T qs = T(0.5) * c.idx[D];
  for (int q = threadIdx.x; q < F::NQ; q += NT) {
    const int ax = F::QX0 + q % F::NQX, ay = F::QY0 + (q / F::NQX) % F::NQY, az = F::QZ0 + q / (F::NQX * F::NQY);
    const int A = az * B::SZ + ay * B::SY + ax;
    T sig[3];
    face_stress<T, NB, D>(&sm[A_U1][0], st, A, c.mu, c.idx, sig);
    const T g = qs * (sm[A_K4][A] - sm[A_K4][A + st[D]]);
#pragma unroll
    for (int k = 0; k < 3; ++k) fq[k][q] = g * sig[k];
  }
}

// Gather of the direction-D records at box cell (qx, qy, qz).  VIRT: the cell is the ghost image
// of a wall cell (only faces with a real cell contribute; lower cells outside the record set
// are faces between two ghosts and count as zero).
template <typename T, int TX, int TY, int TZ, int HX, int D, int NF, int NQF, bool VIRT>
__device__ __forceinline__ void face_gather(const T (*fr)[NF], const T (*fq)[NQF], int qx, int qy, int qz,
                                            const Consts<T>& c, T uh[3], T& eh) {
  using F = FaceSet<TX, TY, TZ, HX, D>;
  const T in = c.idx[D];
  const T pm = c.mu * in * in, pe = c.alpha * in * in;
  // direct faces: lower cell q - e_D (sign +) and q (sign -)
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int ax = qx - (D == 0 && side == 0), ay = qy - (D == 1 && side == 0), az = qz - (D == 2 && side == 0);
    if (VIRT && D != 0) continue;
    if (VIRT && !F::has(ax)) continue;
    const int f = F::idx(ax, ay, az);
    const T sg = side == 0 ? T(1) : T(-1);
    const T sD = fr[D][f];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T P = fr[k][f];
      if (k == D) P += sD * (T(1) / T(3));
      uh[k] += sg * pm * P;
    }
    eh += sg * pe * fr[3][f];
    if (!VIRT || F::hasq(ax)) {
      const int qi = F::qidx(ax, ay, az);
#pragma unroll
      for (int k = 0; k < 3; ++k) uh[k] += fq[k][qi];
    }
  }
  // tangential chain: cells q -+ e_l (l != D), each with its two direction-D faces
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (l == D) continue;
    T tl = T(0), tD = T(0);
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int cx = qx + (l == 0 ? (sl ? 1 : -1) : 0), cy = qy + (l == 1 ? (sl ? 1 : -1) : 0),
                cz = qz + (l == 2 ? (sl ? 1 : -1) : 0);
      const T sgn = sl ? T(-1) : T(1);
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int ax = cx - (D == 0 && side == 0), ay = cy - (D == 1 && side == 0), az = cz - (D == 2 && side == 0);
        if (VIRT && D == 0 && !F::has(ax)) continue;
        const int f = F::idx(ax, ay, az);
        tl += sgn * fr[l][f];
        tD += sgn * fr[D][f];
      }
    }
    const T h = T(0.5) * c.idx[l] * in;
    uh[D] += (T(0.5) * c.mu * h) * tl;
    uh[l] -= ((c.mu / T(3)) * h) * tD;
  }
}

// Convective transpose at box cell p (own fields r0, u, H0, P0, all halved like the LDS planes):
// half of the adjoint of every
// face mean, accumulated as (rho^, u^, H^, P^).  The fields of the neighbours come from the LDS
// planes K (kh), U (u) and Q (rho, E/rho, p).  wallside: the direction-0 face on this side is a
// slip wall, whose ghost-image share (u^_x odd) folds into the cell as well.
template <typename T, int NB, int NBQ, int D>
__device__ __forceinline__ void adj_conv_dir(const T (*K)[NB], const T (*U)[NB], const T (*Q)[NBQ], int p, int sd,
                                             const Consts<T>& c, T r0, const T u[3], T H0, T P0, const T k0[5],
                                             bool wall_lo, bool wall_hi, T& rh, T uh[3], T& Hh, T& Ph) {
  // Both faces of direction D, accumulated with the unscaled kh differences dk = kh_nb - kh_j
  // (G = +-dk/dx_d) and the face sign applied by addition or subtraction; the common factor
  // 0.5/dx_d (the half-share of the face means) is applied once per direction.
  T ar = T(0), aH = T(0), aP = T(0), au[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int q = side ? p + sd : p - sd;
    T dk[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) dk[v] = K[v][q] - k0[v];
    const T r = r0 + Q[0][q];
    const T v[3] = {u[0] + U[0][q], u[1] + U[1][q], u[2] + U[2][q]};
    const T H = H0 + Q[1][q], P = P0 + Q[2][q];
    const T m = r * v[D];
    const T phi = dk[0] + v[0] * dk[1] + v[1] * dk[2] + v[2] * dk[3] + H * dk[4];
    T tr = v[D] * phi, tH = m * dk[4], tP = dk[1 + D] + v[D] * dk[4], tu[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) tu[k] = m * dk[1 + k] + (k == D ? r * phi + P * dk[4] : T(0));
    // at a slip wall the ghost image's half-share folds back through the mirror: u^_x cancels,
    // the rest doubles
    const bool wl = D == 0 && (side ? wall_hi : wall_lo);
    if (wl) {
      tr *= T(2);
      tH *= T(2);
      tP *= T(2);
      tu[0] = T(0);
      tu[1] *= T(2);
      tu[2] *= T(2);
    }
    if (side) {
      ar += tr;
      aH += tH;
      aP += tP;
#pragma unroll
      for (int k = 0; k < 3; ++k) au[k] += tu[k];
    } else {
      ar -= tr;
      aH -= tH;
      aP -= tP;
#pragma unroll
      for (int k = 0; k < 3; ++k) au[k] -= tu[k];
    }
  }
  const T s = T(0.5) * c.idx[D];
  rh += s * ar;
  Hh += s * aH;
  Ph += s * aP;
#pragma unroll
  for (int k = 0; k < 3; ++k) uh[k] += s * au[k];
}

// (u^, e^) -> conservative adjoint at a cell with velocity u, internal energy e, 1/rho = ri
// (the direct rho^ is added by the caller).
template <typename T>
__device__ __forceinline__ void prim_to_cons(const T u[3], T e, T ri, const T uh[3], T eh, T acc[5]) {
  const T usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T uu = u[0] * uh[0] + u[1] * uh[1] + u[2] * uh[2];
  acc[0] += -ri * uu + eh * ri * (T(0.5) * usq - e);
#pragma unroll
  for (int k = 0; k < 3; ++k) acc[1 + k] += ri * (uh[k] - eh * u[k]);
  acc[4] += eh * ri;
}

}  // namespace

// MODE: STAGE_VJP  out = g = J^T kh (+ L_nu kh)
//       STAGE_FIN  (RK4 stage 1) g1 = J(w_n)^T kh + ...; out = w^_n = a + g1 + gnext + g3 + g4;
//                  grad_s += dt a + dt g4 + dt/2 (g3 + gnext)   (= k^1 + k^2 + k^3 + k^4)
// CONV = 0 leaves out the transpose of the split-form convective flux (the Roe option adds its own).
// One work-group: the tile with origin (x0, y0, z0); the artificial viscosity is nscale * nu.
template <typename T, int MODE, int WALL, int LNU, int CONV, int TX, int TY, int TZ>
__device__ __forceinline__ void adjoint_tile_body(const Consts<T>& c, const int x0, const int y0, const int z0,
                                                  const T* __restrict__ W, const T* __restrict__ a,
                                                  const T* __restrict__ gnext, const T* __restrict__ nu,
                                                  const T nscale, const T ca, const T cg, const T* __restrict__ g3,
                                                  const T* __restrict__ g4, T* __restrict__ out,
                                                  T* __restrict__ grad_s, const double objw) {
  constexpr int NT = TX * TY * TZ;
  constexpr int HX = WALL ? 2 : 1;
  using Bx = TBox<TX, TY, TZ, HX, 1>;
  constexpr int NB = Bx::NB;
  using F0 = FaceSet<TX, TY, TZ, HX, 0>;
  using F1 = FaceSet<TX, TY, TZ, HX, 1>;
  using F2 = FaceSet<TX, TY, TZ, HX, 2>;
  constexpr int NF = Max3<F0::N, F1::N, F2::N>::v;
  constexpr int NQF = Max3<F0::NQ, F1::NQ, F2::NQ>::v;
  // one LDS region serves first as the (rho, E/rho, p) planes of the box, then as the face records
  constexpr int NUN = 4 * NF + 3 * NQF > 3 * NB ? 4 * NF + 3 * NQF : 3 * NB;
  __shared__ T sm[LNU ? A_NU + 1 : A_NU][NB];
  __shared__ T un[NUN];
  T (*fr)[NF] = reinterpret_cast<T (*)[NF]>(un);
  T (*fq)[NQF] = reinterpret_cast<T (*)[NQF]>(un + 4 * NF);
  T (*Q)[NB] = reinterpret_cast<T (*)[NB]>(un);
  const int tid = threadIdx.x;
  const long long N = c.N;
  const T gm1 = c.gamma - T(1);
  // all of this thread's box loads are issued before any is used: one memory latency, not NIT
  // (branch-free: the tail iteration re-reads the last box cell and does not store it; a missing
  // g_next is read as a with weight 0)
  constexpr int NIT = (NB + NT - 1) / NT;
  const T* __restrict__ gn = gnext ? gnext : a;
  const T cgn = gnext ? cg : T(0);
  T wv[NIT][5], av[NIT][5], gv[NIT][5], nv[NIT];
  int mir[NIT], rl[NIT];
  const auto rW = buf_rsrc(W, 5 * N), rA = buf_rsrc(a, 5 * N), rG = buf_rsrc(gn, 5 * N);
  const auto rN = buf_rsrc(LNU ? nu : W, N);
  const unsigned fb = (unsigned)(N * (long long)sizeof(T));  // bytes per field
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int b = min(tid + it * NT, NB - 1);
    const int bx = b % Bx::BX, by = (b / Bx::BX) % Bx::BY, bz = b / (Bx::BX * Bx::BY);
    const unsigned off =
        (unsigned)box_cell32<WALL>(c.nx, c.ny, c.nz, x0 + bx - HX, y0 + by - 1, z0 + bz - 1, mir[it], rl[it]) *
        (unsigned)sizeof(T);
#pragma unroll
    for (int v = 0; v < 5; ++v) wv[it][v] = buf_load(rW, off, v * fb, T());
#pragma unroll
    for (int v = 0; v < 5; ++v) av[it][v] = buf_load(rA, off, v * fb, T());
#pragma unroll
    for (int v = 0; v < 5; ++v) gv[it][v] = buf_load(rG, off, v * fb, T());
    nv[it] = LNU ? nscale * buf_load(rN, off, 0, T()) : T(0);
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int b = tid + it * NT;
    if (it + 1 < NIT || b < NB) {
      const T r = wv[it][0] + c.wref[0], ri = recip(r);  // stored deviations w - wref
      const T hri = T(0.5) * ri;
      const T mx = wv[it][1] + c.wref[1];
      const T h1 = (mir[it] ? -mx : mx) * hri, h2 = (wv[it][2] + c.wref[2]) * hri, h3 = (wv[it][3] + c.wref[3]) * hri;
      sm[A_U1][b] = h1;
      sm[A_U2][b] = h2;
      sm[A_U3][b] = h3;
      Q[0][b] = T(0.5) * r;
      Q[1][b] = (wv[it][4] + c.wref[4]) * hri;
      Q[2][b] = gm1 * (T(0.5) * wv[it][4] - r * (h1 * h1 + h2 * h2 + h3 * h3)) + T(0.5) * gm1 * c.wref[4];
#pragma unroll
      for (int v = 0; v < 5; ++v) sm[A_K0 + v][b] = rl[it] ? ca * av[it][v] + cgn * gv[it][v] : T(0);
      if (LNU) sm[LNU ? A_NU : 0][b] = rl[it] ? nv[it] : T(0);
    }
  }
  const int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / (TX * TY);
  const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
  const bool active = gx < c.nx && gy < c.ny && gz < c.nz;
  const bool virt = WALL && active && (gx == 0 || gx == c.nx - 1);
  const int qx = tx + HX, qy = ty + 1, qz = tz + 1;
  const int vx = gx == 0 ? qx - 1 : qx + 1;  // box x of the ghost image
  const int st[3] = {1, Bx::SY, Bx::SZ};
  const int p = qz * Bx::SZ + qy * Bx::SY + qx;
  const long long gi = ((long long)(active ? gz : 0) * c.ny + (active ? gy : 0)) * c.nx + (active ? gx : 0);
  T r0 = T(1), ri = T(0), e = T(0), uc[3] = {T(0), T(0), T(0)};
  // stage-1 operands at the cell itself, fetched now so that their latency hides behind the
  // face phases
  T fa[5], f2[5], f3[5], f4[5], gs[5];
  if (MODE != STAGE_VJP && active) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const long long q = v * N + gi;
      fa[v] = a[q];
      f2[v] = gnext[q];
      f3[v] = g3[q];
      f4[v] = g4[q];
      if (grad_s) gs[v] = grad_s[q];
    }
  }
  T uh[3] = {T(0), T(0), T(0)}, eh = T(0), rh = T(0);
  T uhv[3] = {T(0), T(0), T(0)}, ehv = T(0);
  __syncthreads();
  if (active) {
    // the cell's own fields, halved as in the LDS planes
    const T hr0 = Q[0][p], hu[3] = {sm[A_U1][p], sm[A_U2][p], sm[A_U3][p]};
    const T H0 = Q[1][p], P0 = Q[2][p];
    r0 = T(2) * hr0;
    ri = recip(r0);
#pragma unroll
    for (int k = 0; k < 3; ++k) uc[k] = T(2) * hu[k];
    e = T(2) * (H0 - (hu[0] * hu[0] + hu[1] * hu[1] + hu[2] * hu[2]));
    // convective transpose, in (rho, u, E/rho, p), then moved to (rho, u, e)
    T k0[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) k0[v] = sm[A_K0 + v][p];
    const bool wlo = WALL && gx == 0, whi = WALL && gx == c.nx - 1;
    if constexpr (CONV) {
      T Hh = T(0), Ph = T(0);
      adj_conv_dir<T, NB, NB, 0>(&sm[A_K0], &sm[A_U1], Q, p, st[0], c, hr0, hu, H0, P0, k0, wlo, whi, rh, uh, Hh, Ph);
      adj_conv_dir<T, NB, NB, 1>(&sm[A_K0], &sm[A_U1], Q, p, st[1], c, hr0, hu, H0, P0, k0, false, false, rh, uh, Hh,
                                 Ph);
      adj_conv_dir<T, NB, NB, 2>(&sm[A_K0], &sm[A_U1], Q, p, st[2], c, hr0, hu, H0, P0, k0, false, false, rh, uh, Hh,
                                 Ph);
      rh += gm1 * e * Ph;
      eh += Hh + gm1 * r0 * Ph;
#pragma unroll
      for (int k = 0; k < 3; ++k) uh[k] += Hh * uc[k];
    }
  }
  __syncthreads();
  face_records<T, TX, TY, TZ, HX, 0, NB, NF, NQF>(sm, fr, fq, st, c);
  __syncthreads();
  if (active) face_gather<T, TX, TY, TZ, HX, 0, NF, NQF, false>(fr, fq, qx, qy, qz, c, uh, eh);
  if (virt) face_gather<T, TX, TY, TZ, HX, 0, NF, NQF, true>(fr, fq, vx, qy, qz, c, uhv, ehv);
  __syncthreads();
  face_records<T, TX, TY, TZ, HX, 1, NB, NF, NQF>(sm, fr, fq, st, c);
  __syncthreads();
  if (active) face_gather<T, TX, TY, TZ, HX, 1, NF, NQF, false>(fr, fq, qx, qy, qz, c, uh, eh);
  if (virt) face_gather<T, TX, TY, TZ, HX, 1, NF, NQF, true>(fr, fq, vx, qy, qz, c, uhv, ehv);
  __syncthreads();
  face_records<T, TX, TY, TZ, HX, 2, NB, NF, NQF>(sm, fr, fq, st, c);
  __syncthreads();
  if (active) face_gather<T, TX, TY, TZ, HX, 2, NF, NQF, false>(fr, fq, qx, qy, qz, c, uh, eh);
  if (virt) face_gather<T, TX, TY, TZ, HX, 2, NF, NQF, true>(fr, fq, vx, qy, qz, c, uhv, ehv);
  if (!active) return;
  if (virt) {
    // what the ghost image gathered from the viscous faces folds back through the mirror: the
    // ghost carries the cell's rho and e and the velocity (-u_x, u_y, u_z)
    uh[0] -= uhv[0];
    uh[1] += uhv[1];
    uh[2] += uhv[2];
    eh += ehv;
  }
  T g[5] = {rh, T(0), T(0), T(0), T(0)};
  prim_to_cons(uc, e, ri, uh, eh, g);
  if (LNU) {
    // L_nu k^ with the face nu the mean of its cells, weighted per component (variable group)
    T lv[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int D = 0; D < 3; ++D) {
      const T i2 = c.idx[D] * c.idx[D];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        if (D == 0 && c.wall && ((side == 0 && gx == 0) || (side == 1 && gx == c.nx - 1))) continue;
        const int q = side ? p + st[D] : p - st[D];
        const T nf = T(0.5) * (sm[LNU ? A_NU : 0][p] + sm[LNU ? A_NU : 0][q]) * i2;
#pragma unroll
        for (int v = 0; v < 5; ++v) lv[v] = fma(nf, sm[A_K0 + v][q] - sm[A_K0 + v][p], lv[v]);
      }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) g[v] = fma(c.nuw[v], lv[v], g[v]);
  }
  if (MODE == STAGE_VJP) {
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v * N + gi] = g[v];
  } else {
    const T dt = c.dt, h2 = T(0.5) * c.dt;
    // the mean-pressure objective's c_n dj/dw(w_n) at the cell (W is w_n in this stage), added to
    // w^_n as the objective kernel would add it afterwards
    T inj[5] = {T(0), T(0), T(0), T(0), T(0)};
    if (objw != 0.0) {
      const Q64 qc = q64_of(c, W[gi], W[N + gi], W[2 * N + gi], W[3 * N + gi], W[4 * N + gi], 0, (double)c.gamma);
      meanp_grad_terms(qc, meanp_factor(objw, (double)c.gamma, N), inj);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const long long q = v * N + gi;
      T o = fa[v] + g[v] + f2[v] + f3[v] + f4[v];
      if (objw != 0.0) o += inj[v];
      out[q] = o;
      // explicit fused order: every instantiation (and the ensemble form) rounds identically
      if (grad_s) grad_s[q] = fma(dt, fa[v], fma(dt, f4[v], fma(h2, f3[v] + f2[v], gs[v])));
    }
  }
}

template <typename T, int MODE, int WALL, int LNU, int CONV, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX * TY * TZ) void k_adjoint_stage(Consts<T> c, const T* __restrict__ W,
                                                                const T* __restrict__ a, const T* __restrict__ gnext,
                                                                const T* __restrict__ nu, T ca, T cg,
                                                                const T* __restrict__ g3, const T* __restrict__ g4,
                                                                T* __restrict__ out, T* __restrict__ grad_s,
                                                                double objw) {
  int x0, y0, z0;
  tile_origin<TX, TY, TZ>(xcd_tile(blockIdx.x, gridDim.x), c.nx, c.ny, c.nz, x0, y0, z0);
  adjoint_tile_body<T, MODE, WALL, LNU, CONV, TX, TY, TZ>(c, x0, y0, z0, W, a, gnext, nu, T(1), ca, cg, g3, g4, out,
                                                          grad_s, objw);
}

// Ensemble form over the members: state arrays (W, the sigma_1 field) at the member's box,
// adjoint arrays at the member itself; nu = lam * sigma_1; ca = dt / da, cg = dt * mg with the
// member's own dt (the same operations the single-box launch performs on the host).
template <typename T, int MODE, int WALL, int LNU, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX * TY * TZ) void k_adjoint_stage_batch(
    const BoxDesc<T>* __restrict__ mems, const int* __restrict__ start, int nmem, const T* __restrict__ W,
    const T* __restrict__ a, const T* __restrict__ gnext, const T* __restrict__ sigma1, T da, T mg,
    const T* __restrict__ g3, const T* __restrict__ g4, T* __restrict__ out, T* __restrict__ grad_s,
    const double* __restrict__ cn) {
  const int blk = xcd_tile(blockIdx.x, gridDim.x);
  const int m = find_box(start, nmem, blk);
  const Consts<T> c = mems[m].c;
  const long long o = 5 * mems[m].off, ao = 5 * mems[m].aoff;
  int x0, y0, z0;
  tile_origin<TX, TY, TZ>(blk - start[m], c.nx, c.ny, c.nz, x0, y0, z0);
  adjoint_tile_body<T, MODE, WALL, LNU, 1, TX, TY, TZ>(
      c, x0, y0, z0, W + o, a + ao, gnext ? gnext + ao : nullptr, LNU ? sigma1 + mems[m].off : nullptr,
      mems[m].lam, c.dt / da, c.dt * mg, g3 ? g3 + ao : nullptr, g4 ? g4 + ao : nullptr, out + ao,
      grad_s ? grad_s + ao : nullptr, (MODE != STAGE_VJP && cn) ? cn[m] : 0.0);
}

// ------------------------------------------------------------------------------------------
// Host-side launchers: the tile shape of each kernel class and precision is a process-wide
// setting (adj_set_tile), dispatched here to the matching instantiation.
// ------------------------------------------------------------------------------------------
template <int X, int Y, int Z>
struct Shape {
  static constexpr int tx = X, ty = Y, tz = Z;
};

// Calls f(Shape<...>{}) for tile id `tile`.
template <class F>
static void with_tile(int tile, F&& f) {
  switch (tile) {
    case TILE_16x4x4: f(Shape<16, 4, 4>{}); break;
    case TILE_32x4x2: f(Shape<32, 4, 2>{}); break;
    case TILE_32x4x4: f(Shape<32, 4, 4>{}); break;
    case TILE_32x8x2: f(Shape<32, 8, 2>{}); break;
    case TILE_32x8x4: f(Shape<32, 8, 4>{}); break;
    default: f(Shape<16, 8, 8>{}); break;
  }
}

// Calls f(integral WALL, integral LNU) for the boundary / artificial-viscosity variant.
template <class F>
static void with_variant(int wall, int lnu, F&& f) {
  if (wall) {
    if (lnu)
      f(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{});
    else
      f(std::integral_constant<int, 1>{}, std::integral_constant<int, 0>{});
  } else {
    if (lnu)
      f(std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{});
    else
      f(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{});
  }
}

template <int TX, int TY, int TZ>
static dim3 tile_grid(int nx, int ny, int nz) {
  return dim3(((nx + TX - 1) / TX) * ((ny + TY - 1) / TY) * ((nz + TZ - 1) / TZ));
}

// LDS bytes of one work-group of the reverse-stage kernel (box fields + the region shared by the
// convective planes and the face records / work terms)
template <typename T, int WALL, int LNU, int TX, int TY, int TZ>
constexpr int adjoint_lds_bytes() {
  constexpr int HX = WALL ? 2 : 1;
  using B = TBox<TX, TY, TZ, HX, 1>;
  using F0 = FaceSet<TX, TY, TZ, HX, 0>;
  using F1 = FaceSet<TX, TY, TZ, HX, 1>;
  using F2 = FaceSet<TX, TY, TZ, HX, 2>;
  constexpr int rec = 4 * Max3<F0::N, F1::N, F2::N>::v + 3 * Max3<F0::NQ, F1::NQ, F2::NQ>::v;
  return (int)sizeof(T) * ((LNU ? A_NU + 1 : A_NU) * B::NB + (rec > 3 * B::NB ? rec : 3 * B::NB));
}

// A tile shape whose reverse-stage LDS footprint exceeds the 160 KB of a CU runs as 16x4x4.
template <typename T, int WALL, int LNU, class S>
constexpr bool adjoint_fits() {
  return adjoint_lds_bytes<T, WALL, LNU, S::tx, S::ty, S::tz>() <= 160 * 1024;
}

template <typename T, int CONV, int TX, int TY, int TZ>
static void primal_launch(ProfScope& ps, int mode, const Consts<T>& c, const T* W, const T* wn, const T* s,
                          const T* W2, const T* W3, T cR, T* out, hipStream_t st, T ca, T cb, double* jpart) {
  const dim3 grid = tile_grid<TX, TY, TZ>(c.nx, c.ny, c.nz), blk(TX * TY * TZ);
  double* nj = nullptr;
  if (mode == STAGE_RES)
    timed_launch(ps, k_primal_stage<T, STAGE_RES, CONV, TX, TY, TZ>, grid, blk, st, c, W, wn, s, W2, W3, cR, out, ca,
                 cb, nj);
  else if (mode == STAGE_LIN && jpart)
    timed_launch(ps, k_primal_stage<T, STAGE_LIN_DISS, CONV, TX, TY, TZ>, grid, blk, st, c, W, wn, s, W2, W3, cR, out,
                 ca, cb, jpart);
  else if (mode == STAGE_LIN)
    timed_launch(ps, k_primal_stage<T, STAGE_LIN, CONV, TX, TY, TZ>, grid, blk, st, c, W, wn, s, W2, W3, cR, out, ca,
                 cb, nj);
  else if (mode == STAGE_AFF)
    timed_launch(ps, k_primal_stage<T, STAGE_AFF, CONV, TX, TY, TZ>, grid, blk, st, c, W, wn, s, W2, W3, cR, out, ca,
                 cb, nj);
  else
    timed_launch(ps, k_primal_stage<T, STAGE_FIN, CONV, TX, TY, TZ>, grid, blk, st, c, W, wn, s, W2, W3, cR, out, ca,
                 cb, jpart);
}

// Work-groups (tiles) of a primal-stage launch in the current tile shape: the number of per-tile
// partial sums a final stage or a stage 1 (STAGE_LIN) with jpart writes.
template <typename T>
int primal_tiles(const Consts<T>& c) {
  int n = 0;
  with_tile(tile_choice(ADJ_PROF_PRIMAL_STAGE, sizeof(T) == 8), [&](auto S) {
    using Sh = decltype(S);
    n = (int)tile_grid<Sh::tx, Sh::ty, Sh::tz>(c.nx, c.ny, c.nz).x;
  });
  return n;
}
template int primal_tiles<float>(const Consts<float>&);
template int primal_tiles<double>(const Consts<double>&);

template <typename T>
hipError_t launch_primal_stage(int mode, const Consts<T>& c, const T* W, const T* wn, const T* s, const T* W2,
                               const T* W3, T cR, T* out, hipStream_t st, T ca, T cb, int conv, double* jpart) {
  ProfScope ps(ADJ_PROF_PRIMAL_STAGE, st, true);
  with_tile(tile_choice(ADJ_PROF_PRIMAL_STAGE, sizeof(T) == 8), [&](auto S) {
    using Sh = decltype(S);
    if (conv)
      primal_launch<T, 1, Sh::tx, Sh::ty, Sh::tz>(ps, mode, c, W, wn, s, W2, W3, cR, out, st, ca, cb, jpart);
    else
      primal_launch<T, 0, Sh::tx, Sh::ty, Sh::tz>(ps, mode, c, W, wn, s, W2, W3, cR, out, st, ca, cb, jpart);
  });
  return hipGetLastError();
}

template <typename T, int WALL, int LNU, int CONV, int TX, int TY, int TZ>
static void adjoint_launch_conv(ProfScope& ps, int mode, const Consts<T>& c, const T* W, const T* a, const T* gnext,
                                const T* nu, T ca, T cg, const T* g3, const T* g4, T* out, T* grad_s,
                                hipStream_t st, double objw) {
  const dim3 grid = tile_grid<TX, TY, TZ>(c.nx, c.ny, c.nz), blk(TX * TY * TZ);
  if (mode == STAGE_VJP)
    timed_launch(ps, k_adjoint_stage<T, STAGE_VJP, WALL, LNU, CONV, TX, TY, TZ>, grid, blk, st, c, W, a, gnext, nu, ca,
                 cg, g3, g4, out, grad_s, 0.0);
  else
    timed_launch(ps, k_adjoint_stage<T, STAGE_FIN, WALL, LNU, CONV, TX, TY, TZ>, grid, blk, st, c, W, a, gnext, nu, ca,
                 cg, g3, g4, out, grad_s, objw);
}

template <typename T, int WALL, int LNU, int TX, int TY, int TZ>
static void adjoint_launch(ProfScope& ps, int mode, int conv, const Consts<T>& c, const T* W, const T* a,
                           const T* gnext, const T* nu, T ca, T cg, const T* g3, const T* g4, T* out, T* grad_s,
                           hipStream_t st, double objw) {
  if (conv)
    adjoint_launch_conv<T, WALL, LNU, 1, TX, TY, TZ>(ps, mode, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st,
                                                     objw);
  else
    adjoint_launch_conv<T, WALL, LNU, 0, TX, TY, TZ>(ps, mode, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st,
                                                     objw);
}

template <typename T>
hipError_t launch_adjoint_stage(int mode, const Consts<T>& c, const T* W, const T* a, const T* gnext, const T* nu,
                                T ca, T cg, const T* g3, const T* g4, T* out, T* grad_s, hipStream_t st, int conv,
                                double objw) {
  ProfScope ps(ADJ_PROF_ADJOINT_STAGE, st, true);
  with_variant(c.wall, nu != nullptr, [&](auto WL, auto LN) {
    constexpr int WALL = decltype(WL)::value, LNU = decltype(LN)::value;
    with_tile(tile_choice(ADJ_PROF_ADJOINT_STAGE, sizeof(T) == 8), [&](auto S) {
      using Sh = decltype(S);
      if constexpr (adjoint_fits<T, WALL, LNU, Sh>())
        adjoint_launch<T, WALL, LNU, Sh::tx, Sh::ty, Sh::tz>(ps, mode, conv, c, W, a, gnext, nu, ca, cg, g3, g4, out,
                                                             grad_s, st, objw);
      else
        adjoint_launch<T, WALL, LNU, 16, 4, 4>(ps, mode, conv, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st,
                                               objw);
    });
  });
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Ensemble launchers: one launch covers the first nbox boxes (or members) of the packed arrays;
// the tile shape is fixed when the ensemble is set up, so that `start` matches it.
// ------------------------------------------------------------------------------------------
void tile_dims(int tile, int& tx, int& ty, int& tz) {
  with_tile(tile, [&](auto S) {
    using Sh = decltype(S);
    tx = Sh::tx;
    ty = Sh::ty;
    tz = Sh::tz;
  });
}

int adjoint_tile_used(int fp64, int wall, int lnu, int tile) {
  int used = tile;
  with_variant(wall, lnu, [&](auto WL, auto LN) {
    constexpr int WALL = decltype(WL)::value, LNU = decltype(LN)::value;
    with_tile(tile, [&](auto S) {
      using Sh = decltype(S);
      const bool fits = fp64 ? adjoint_fits<double, WALL, LNU, Sh>() : adjoint_fits<float, WALL, LNU, Sh>();
      used = fits ? tile : (int)TILE_16x4x4;
    });
  });
  return used;
}

template <typename T>
hipError_t launch_primal_stage_batch(int mode, int tile, const BoxDesc<T>* boxes, const int* start, int nbox,
                                     int nblocks, const T* W, const T* wn, const T* s, const T* W2, const T* W3,
                                     T cfac, T* out, hipStream_t st) {
  ProfScope ps(ADJ_PROF_PRIMAL_STAGE, st, true);
  with_tile(tile, [&](auto S) {
    using Sh = decltype(S);
    const dim3 grid(nblocks), blk(Sh::tx * Sh::ty * Sh::tz);
    if (mode == STAGE_RES)
      timed_launch(ps, k_primal_stage_batch<T, STAGE_RES, Sh::tx, Sh::ty, Sh::tz>, grid, blk, st, boxes, start, nbox, W, wn, s, W2, W3, cfac, out);
    else if (mode == STAGE_LIN)
      timed_launch(ps, k_primal_stage_batch<T, STAGE_LIN, Sh::tx, Sh::ty, Sh::tz>, grid, blk, st, boxes, start, nbox, W, wn, s, W2, W3, cfac, out);
    else
      timed_launch(ps, k_primal_stage_batch<T, STAGE_FIN, Sh::tx, Sh::ty, Sh::tz>, grid, blk, st, boxes, start, nbox, W, wn, s, W2, W3, cfac, out);
  });
  return hipGetLastError();
}

// `tile` is the shape after the LDS fit (adjoint_tile_used), so no fallback happens here
template <typename T>
hipError_t launch_adjoint_stage_batch(int mode, int tile, int wall, int lnu, const BoxDesc<T>* mems, const int* start,
                                      int nmem, int nblocks, const T* W, const T* a, const T* gnext, const T* sigma1,
                                      T da, T mg, const T* g3, const T* g4, T* out, T* grad_s, hipStream_t st,
                                      const double* cn) {
  ProfScope ps(ADJ_PROF_ADJOINT_STAGE, st, true);
  with_variant(wall, lnu, [&](auto WL, auto LN) {
    constexpr int WALL = decltype(WL)::value, LNU = decltype(LN)::value;
    with_tile(tile, [&](auto S) {
      using Sh = decltype(S);
      if constexpr (adjoint_fits<T, WALL, LNU, Sh>()) {
        const dim3 grid(nblocks), blk(Sh::tx * Sh::ty * Sh::tz);
        if (mode == STAGE_VJP)
          timed_launch(ps, k_adjoint_stage_batch<T, STAGE_VJP, WALL, LNU, Sh::tx, Sh::ty, Sh::tz>, grid, blk, st, mems,
                       start, nmem, W, a, gnext, sigma1, da, mg, g3, g4, out, grad_s, (const double*)nullptr);
        else
          timed_launch(ps, k_adjoint_stage_batch<T, STAGE_FIN, WALL, LNU, Sh::tx, Sh::ty, Sh::tz>, grid, blk, st, mems,
                       start, nmem, W, a, gnext, sigma1, da, mg, g3, g4, out, grad_s, cn);
      }
    });
  });
  return hipGetLastError();
}

#define ADJNS_BATCH_INST(T)                                                                                        \
  template hipError_t launch_primal_stage_batch<T>(int, int, const BoxDesc<T>*, const int*, int, int, const T*,   \
                                                   const T*, const T*, const T*, const T*, T, T*, hipStream_t);  \
  template hipError_t launch_adjoint_stage_batch<T>(int, int, int, int, const BoxDesc<T>*, const int*, int, int,  \
                                                    const T*, const T*, const T*, const T*, T, T, const T*,       \
                                                    const T*, T*, T*, hipStream_t, const double*);
ADJNS_BATCH_INST(float)
ADJNS_BATCH_INST(double)
#undef ADJNS_BATCH_INST

template hipError_t launch_primal_stage<float>(int, const Consts<float>&, const float*, const float*, const float*,
                                               const float*, const float*, float, float*, hipStream_t, float, float,
                                               int, double*);
template hipError_t launch_primal_stage<double>(int, const Consts<double>&, const double*, const double*, const double*,
                                                const double*, const double*, double, double*, hipStream_t, double,
                                                double, int, double*);
template hipError_t launch_adjoint_stage<float>(int, const Consts<float>&, const float*, const float*, const float*,
                                                const float*, float, float, const float*, const float*, float*,
                                                float*, hipStream_t, int, double);
template hipError_t launch_adjoint_stage<double>(int, const Consts<double>&, const double*, const double*,
                                                 const double*, const double*, double, double, const double*,
                                                 const double*, double*, double*, hipStream_t, int, double);

}  // namespace adjns
