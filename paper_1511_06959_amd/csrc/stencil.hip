// stencil.hip -- gfx950 kernels for one RK4 stage of the primal residual and one reverse stage of
// the discrete adjoint (transposed convective, viscous and artificial-viscosity operators).
//
// Both kernels stage a (16+2h) x 6 x 6 box of cells (the 16x4x4 output tile plus its halo) in
// LDS, derive the primitive variables once per box cell, and then evaluate each output cell's
// 19-point stencil from LDS.  SoA var-major global layout; every global access of a wavefront is
// to consecutive x addresses.
#include "kernels.hpp"

namespace adjns {

// ------------------------------------------------------------------------------------------
// Primal residual  R = -sum_d (F~_{d,+} - F~_{d,-})/dx_d + s  with
//   F~ = 0.5 (F(w_L) + F(w_R)) - (0, sigma_d., u_f . sigma_d. + alpha d_d e)
// [Physics, Eq. navier; Unsteady adjoint, vector form with source].
// ------------------------------------------------------------------------------------------
namespace {

// LDS field order of the primal box
enum { P_RHO = 0, P_U1, P_U2, P_U3, P_E, P_P, P_ET, P_NF };

template <typename T, int NB>
__device__ __forceinline__ void conv_flux(const T (*sm)[NB], int d, int q, T gm1, T F[5]) {
  const T r = sm[P_RHO][q], u1 = sm[P_U1][q], u2 = sm[P_U2][q], u3 = sm[P_U3][q];
  const T p = sm[P_P][q];
  const T ud = d == 0 ? u1 : (d == 1 ? u2 : u3);
  const T m = r * ud;
  F[0] = m;
  F[1] = m * u1 + (d == 0 ? p : T(0));
  F[2] = m * u2 + (d == 1 ? p : T(0));
  F[3] = m * u3 + (d == 2 ? p : T(0));
  F[4] = (sm[P_ET][q] + p) * ud;
  (void)gm1;
}

// Forward viscous stress row sigma_d. on the face between box cells A and A + e_d.
// Velocity fields are read from `U` (three LDS planes of NB values).
template <typename T, int NB, int D>
__device__ __forceinline__ void face_stress(const T* __restrict__ U, const int st[3], int A, T mu,
                                            const T idx[3], T sig[3]) {
  constexpr int t1 = D == 0 ? 1 : 0, t2 = D == 2 ? 1 : 2;
  const int B = A + st[D];
  const T in = idx[D];
  T gn[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) gn[k] = (U[k * NB + B] - U[k * NB + A]) * in;
  // tangential gradients d_t u_D and d_t u_t at the face: mean of the two cells' central differences
  const T q1 = T(0.25) * idx[t1], q2 = T(0.25) * idx[t2];
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
  for (int k = 0; k < 3; ++k) work += T(0.5) * (sm[P_U1 + k][A] + sm[P_U1 + k][B]) * sig[k];
  G[0] = sig[0];
  G[1] = sig[1];
  G[2] = sig[2];
  G[3] = work + c.alpha * (sm[P_E][B] - sm[P_E][A]) * c.idx[D];
}

template <typename T, int NB, int D>
__device__ __forceinline__ void residual_dir(const T (*sm)[NB], const int st[3], int p, const Consts<T>& c,
                                             T R[5]) {
  T Fp[5], Fm[5];
  conv_flux<T, NB>(sm, D, p + st[D], c.gamma - T(1), Fp);
  conv_flux<T, NB>(sm, D, p - st[D], c.gamma - T(1), Fm);
  const T h = T(0.5) * c.idx[D];
#pragma unroll
  for (int v = 0; v < 5; ++v) R[v] -= (Fp[v] - Fm[v]) * h;
  T Gp[4], Gm[4];
  visc_flux<T, NB, D>(sm, st, p, c, Gp);
  visc_flux<T, NB, D>(sm, st, p - st[D], c, Gm);
#pragma unroll
  for (int k = 0; k < 4; ++k) R[1 + k] += (Gp[k] - Gm[k]) * c.idx[D];
}

}  // namespace

// MODE: RES  out = R(W; s)
//       LIN  out = wn + cR * R(W; s)                           (RK4 stages 1-3)
//       FIN  out = (W2 + 2 W3 + W - wn)/3 + (dt/6) R(W; s)      (stage 4, W = W4;
//            equals wn + dt/6 (k1 + 2 k2 + 2 k3 + k4) since k1 = 2(W2-wn)/dt, k2 = 2(W3-wn)/dt,
//            k3 = (W4-wn)/dt)
template <typename T, int MODE, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX * TY * TZ) void k_primal_stage(Consts<T> c, const T* __restrict__ W,
                                                               const T* __restrict__ wn, const T* __restrict__ s,
                                                               const T* __restrict__ W2, const T* __restrict__ W3,
                                                               T cR, T* __restrict__ out) {
  constexpr int NT = TX * TY * TZ;
  using Bx = TBox<TX, TY, TZ, 1, 1>;
  constexpr int NB = Bx::NB;
  __shared__ T sm[P_NF][NB];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
  const long long N = c.N;
  const T gm1 = c.gamma - T(1);
  for (int b = tid; b < NB; b += NT) {
    const int bx = b % Bx::BX, by = (b / Bx::BX) % Bx::BY, bz = b / (Bx::BX * Bx::BY);
    int mirror, real;
    const long long gi = box_cell(c.nx, c.ny, c.nz, c.wall, x0 + bx - 1, y0 + by - 1, z0 + bz - 1, mirror, real);
    const T r = W[gi];
    T m1 = W[N + gi];
    const T m2 = W[2 * N + gi], m3 = W[3 * N + gi], Et = W[4 * N + gi];
    if (mirror) m1 = -m1;
    const T ri = T(1) / r;
    const T u1 = m1 * ri, u2 = m2 * ri, u3 = m3 * ri;
    const T e = Et * ri - T(0.5) * (u1 * u1 + u2 * u2 + u3 * u3);
    sm[P_RHO][b] = r;
    sm[P_U1][b] = u1;
    sm[P_U2][b] = u2;
    sm[P_U3][b] = u3;
    sm[P_E][b] = e;
    sm[P_P][b] = gm1 * r * e;
    sm[P_ET][b] = Et;
  }
  __syncthreads();
  const int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / (TX * TY);
  const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
  if (gx >= c.nx || gy >= c.ny || gz >= c.nz) return;
  const int st[3] = {1, Bx::SY, Bx::SZ};
  const int p = (tz + 1) * Bx::SZ + (ty + 1) * Bx::SY + (tx + 1);
  T R[5] = {T(0), T(0), T(0), T(0), T(0)};
  residual_dir<T, NB, 0>(sm, st, p, c, R);
  __builtin_amdgcn_sched_barrier(0);
  residual_dir<T, NB, 1>(sm, st, p, c, R);
  __builtin_amdgcn_sched_barrier(0);
  residual_dir<T, NB, 2>(sm, st, p, c, R);
  __builtin_amdgcn_sched_barrier(0);
  const long long gi = ((long long)gz * c.ny + gy) * c.nx + gx;
  if (s) {
#pragma unroll
    for (int v = 0; v < 5; ++v) R[v] += s[v * N + gi];
  }
  if (MODE == STAGE_RES) {
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v * N + gi] = R[v];
  } else if (MODE == STAGE_LIN) {
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v * N + gi] = wn[v * N + gi] + cR * R[v];
  } else {
    const T third = T(1) / T(3), h6 = c.dt / T(6);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const long long q = v * N + gi;
      out[q] = (W2[q] + T(2) * W3[q] + W[q] - wn[q]) * third + h6 * R[v];
    }
  }
}

// ------------------------------------------------------------------------------------------
// Reverse stage:  g = J_R(W)^T kh + L_nu kh,  kh = ca * a + cg * gnext formed on load
// [Unsteady adjoint: A_ijk, A^v_ijk, D_ijkl and the adjoint equation; Implementation: discrete
// adjoint; Stabilizing adjoint equations: lambda sigma_1 delta_ki delta_jl term].
//
// Gather form for output cell j (all terms are the exact transpose of the primal residual):
//   convective  sum_d A_d(W_j)^T (kh_{j+e_d} - kh_{j-e_d}) / (2 dx_d), A_d = dF_d/dw
//   viscous     adjoint of the primitive fields (u^, e^) at j collected from
//               - its six faces f (direction d, cells L|R):  G^ = (kh_L - kh_R)/dx_d,
//                 sigma^_k = G^_mk + G^_E u_f,k,
//                 normal part  tau^_dk/dx_d = (mu sigma^_k + (mu/3) sigma^_d delta_kd)/dx_d
//                 (to R with +, to L with -), work part 0.5 G^_E sigma_dk (to both),
//                 heat part alpha G^_E / dx_d (to R with +, to L with -);
//               - the tangential-gradient chain:  u^_j += sum_l (C_l(j-e_l) - C_l(j+e_l))/(2 dx_l)
//                 with C_l(c) = 0.5 sum_{d != l} sum_{faces of c in d} (mu sigma^_l e_d - (2mu/3) sigma^_d e_l);
//               then (u^, e^) -> conservative adjoint through u = m/rho, e = E/rho - |u|^2/2.
//   L_nu        sum_d sum_{+-} nu_f (kh_nb - kh_j)/dx_d^2, nu_f = (nu_j + nu_nb)/2, no wall faces.
// Slip walls: ghost cells carry mirrored primitives and kh = 0 (they own no residual); a cell
// next to a wall adds M^T times the gather evaluated at its ghost image (M flips x-momentum).
// ------------------------------------------------------------------------------------------
namespace {

enum { A_K0 = 0, A_K1, A_K2, A_K3, A_K4, A_U1, A_U2, A_U3, A_NU };

template <typename T, int NB>
__device__ __forceinline__ void face_adj(const T (*sm)[NB], int A, int B, T in, T sh[3], T& GhE) {
  GhE = (sm[A_K4][A] - sm[A_K4][B]) * in;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    sh[k] = (sm[A_K1 + k][A] - sm[A_K1 + k][B]) * in + GhE * (T(0.5) * (sm[A_U1 + k][A] + sm[A_U1 + k][B]));
}

// C_l at box cell q (tangential-gradient adjoint), all 3 components
template <typename T, int NB, int L>
__device__ __forceinline__ void chat(const T (*sm)[NB], const int st[3], int q, const Consts<T>& c, T C[3]) {
  C[0] = C[1] = C[2] = T(0);
#pragma unroll
  for (int D = 0; D < 3; ++D) {
    if (D == L) continue;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int A = side ? q : q - st[D];
      const int B = A + st[D];
      const T in = c.idx[D];
      const T GhE = (sm[A_K4][A] - sm[A_K4][B]) * in;
      const T shl = (sm[A_K1 + L][A] - sm[A_K1 + L][B]) * in + GhE * (T(0.5) * (sm[A_U1 + L][A] + sm[A_U1 + L][B]));
      const T shd = (sm[A_K1 + D][A] - sm[A_K1 + D][B]) * in + GhE * (T(0.5) * (sm[A_U1 + D][A] + sm[A_U1 + D][B]));
      C[D] += T(0.5) * c.mu * shl;
      C[L] -= (c.mu / T(3)) * shd;
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <typename T, int NB, int D>
__device__ __forceinline__ void adj_faces_dir(const T (*sm)[NB], const int st[3], int p, const Consts<T>& c,
                                              T uh[3], T& eh) {
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    // side 0: face (p - e_D | p), p is R;  side 1: face (p | p + e_D), p is L
    const int A = side ? p : p - st[D];
    const int B = A + st[D];
    const T in = c.idx[D];
    T sh[3], GhE;
    face_adj<T, NB>(sm, A, B, in, sh, GhE);
    T sig[3];
    face_stress<T, NB, D>(&sm[A_U1][0], st, A, c.mu, c.idx, sig);
    const T sgn = side ? T(-1) : T(1);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T P = c.mu * sh[k];
      if (k == D) P += (c.mu / T(3)) * sh[D];
      uh[k] += sgn * P * in + T(0.5) * GhE * sig[k];
    }
    eh += sgn * c.alpha * GhE * in;
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <typename T, int NB, int D>
__device__ __forceinline__ void adj_conv_dir(const T (*sm)[NB], const int st[3], int p, const Consts<T>& c,
                                             const T u[3], T H, T phi, T acc[5]) {
  const T h = T(0.5) * c.idx[D];
  T v[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) v[q] = (sm[A_K0 + q][p + st[D]] - sm[A_K0 + q][p - st[D]]) * h;
  const T gm1 = c.gamma - T(1);
  const T um = u[0] * v[1] + u[1] * v[2] + u[2] * v[3];
  const T ud = u[D];
  acc[0] += -ud * um + phi * v[1 + D] + ud * (phi - H) * v[4];
  const T common = v[0] + um + H * v[4];
  const T mdp = v[1 + D] + ud * v[4];
#pragma unroll
  for (int j = 0; j < 3; ++j) acc[1 + j] += (j == D ? common : T(0)) + ud * v[1 + j] - gm1 * u[j] * mdp;
  acc[4] += gm1 * v[1 + D] + c.gamma * ud * v[4];
}

// Full gather at box cell p.  gx: global x of the cell (for wall faces of L_nu); LNU: add L_nu.
// e and ri (internal energy and 1/rho of the cell) come from the calling thread: a wall ghost
// image has the same e and rho as its cell.
template <typename T, int NB, int SY, int SZ, int LNU>
__device__ __forceinline__ void adj_cell(const T (*sm)[NB], int p, const Consts<T>& c, int gx, T e, T ri, T acc[5]) {
  const int st[3] = {1, SY, SZ};
  const T u[3] = {sm[A_U1][p], sm[A_U2][p], sm[A_U3][p]};
  const T usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T H = c.gamma * e + T(0.5) * usq;
  const T phi = T(0.5) * (c.gamma - T(1)) * usq;
#pragma unroll
  for (int v = 0; v < 5; ++v) acc[v] = T(0);
  // The scheduling barriers keep each direction's LDS reads next to their use: hoisting them
  // across directions raises the live register count and halves the resident wavefronts.
  adj_conv_dir<T, NB, 0>(sm, st, p, c, u, H, phi, acc);
  __builtin_amdgcn_sched_barrier(0);
  adj_conv_dir<T, NB, 1>(sm, st, p, c, u, H, phi, acc);
  __builtin_amdgcn_sched_barrier(0);
  adj_conv_dir<T, NB, 2>(sm, st, p, c, u, H, phi, acc);
  __builtin_amdgcn_sched_barrier(0);
  T uh[3] = {T(0), T(0), T(0)}, eh = T(0);
  adj_faces_dir<T, NB, 0>(sm, st, p, c, uh, eh);
  __builtin_amdgcn_sched_barrier(0);
  adj_faces_dir<T, NB, 1>(sm, st, p, c, uh, eh);
  __builtin_amdgcn_sched_barrier(0);
  adj_faces_dir<T, NB, 2>(sm, st, p, c, uh, eh);
  __builtin_amdgcn_sched_barrier(0);
  {
    T Cm[3], Cp[3];
    chat<T, NB, 0>(sm, st, p - st[0], c, Cm);
    chat<T, NB, 0>(sm, st, p + st[0], c, Cp);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) uh[k] += (Cm[k] - Cp[k]) * (T(0.5) * c.idx[0]);
    chat<T, NB, 1>(sm, st, p - st[1], c, Cm);
    chat<T, NB, 1>(sm, st, p + st[1], c, Cp);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) uh[k] += (Cm[k] - Cp[k]) * (T(0.5) * c.idx[1]);
    chat<T, NB, 2>(sm, st, p - st[2], c, Cm);
    chat<T, NB, 2>(sm, st, p + st[2], c, Cp);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) uh[k] += (Cm[k] - Cp[k]) * (T(0.5) * c.idx[2]);
  }
  const T uu = u[0] * uh[0] + u[1] * uh[1] + u[2] * uh[2];
  acc[0] += -ri * uu + eh * ri * (T(0.5) * usq - e);
#pragma unroll
  for (int k = 0; k < 3; ++k) acc[1 + k] += ri * (uh[k] - eh * u[k]);
  acc[4] += eh * ri;
  if (LNU) {
#pragma unroll
    for (int D = 0; D < 3; ++D) {
      const T i2 = c.idx[D] * c.idx[D];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        if (D == 0 && c.wall && ((side == 0 && gx == 0) || (side == 1 && gx == c.nx - 1))) continue;
        const int q = side ? p + st[D] : p - st[D];
        const T nf = T(0.5) * (sm[LNU ? A_NU : 0][p] + sm[LNU ? A_NU : 0][q]) * i2;
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] += nf * (sm[A_K0 + v][q] - sm[A_K0 + v][p]);
      }
    }
  }
}

}  // namespace

// MODE: STAGE_VJP  out = g = J^T kh (+ L_nu kh)
//       STAGE_FIN  (RK4 stage 1) g1 = J(w_n)^T kh + ...; out = w^_n = a + g1 + gnext + g3 + g4;
//                  grad_s += dt a + dt g4 + dt/2 (g3 + gnext)   (= k^1 + k^2 + k^3 + k^4)
template <typename T, int MODE, int WALL, int LNU, int TX, int TY, int TZ>
__global__ __launch_bounds__(TX * TY * TZ) void k_adjoint_stage(Consts<T> c, const T* __restrict__ W,
                                                      const T* __restrict__ a, const T* __restrict__ gnext,
                                                      const T* __restrict__ nu, T ca, T cg,
                                                      const T* __restrict__ g3, const T* __restrict__ g4,
                                                      T* __restrict__ out, T* __restrict__ grad_s) {
  constexpr int NT = TX * TY * TZ;
  constexpr int HX = WALL ? 2 : 1;
  using Bx = TBox<TX, TY, TZ, HX, 1>;
  constexpr int NB = Bx::NB;
  __shared__ T sm[LNU ? A_NU + 1 : A_NU][NB];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
  const long long N = c.N;
  for (int b = tid; b < NB; b += NT) {
    const int bx = b % Bx::BX, by = (b / Bx::BX) % Bx::BY, bz = b / (Bx::BX * Bx::BY);
    int mirror, real;
    const long long gi = box_cell(c.nx, c.ny, c.nz, c.wall, x0 + bx - HX, y0 + by - 1, z0 + bz - 1, mirror, real);
    const T ri = T(1) / W[gi];
    T m1 = W[N + gi];
    if (mirror) m1 = -m1;
    sm[A_U1][b] = m1 * ri;
    sm[A_U2][b] = W[2 * N + gi] * ri;
    sm[A_U3][b] = W[3 * N + gi] * ri;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T k = ca * a[v * N + gi];
      if (gnext) k += cg * gnext[v * N + gi];
      sm[A_K0 + v][b] = real ? k : T(0);
    }
    if (LNU) sm[LNU ? A_NU : 0][b] = real ? nu[gi] : T(0);
  }
  __syncthreads();
  const int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / (TX * TY);
  const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
  if (gx >= c.nx || gy >= c.ny || gz >= c.nz) return;
  const int p = (tz + 1) * Bx::SZ + (ty + 1) * Bx::SY + (tx + HX);
  const long long gi = ((long long)gz * c.ny + gy) * c.nx + gx;
  const T ri = T(1) / W[gi];
  const T uc[3] = {W[N + gi] * ri, W[2 * N + gi] * ri, W[3 * N + gi] * ri};
  const T e = W[4 * N + gi] * ri - T(0.5) * (uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2]);
  T g[5];
  adj_cell<T, NB, Bx::SY, Bx::SZ, LNU>(sm, p, c, gx, e, ri, g);
  if (WALL) {
    // contributions through the mirror ghost of a wall-adjacent cell: g += M^T gather(ghost)
    if (gx == 0 || gx == c.nx - 1) {
      T gv[5];
      adj_cell<T, NB, Bx::SY, Bx::SZ, 0>(sm, gx == 0 ? p - 1 : p + 1, c, gx, e, ri, gv);
      g[0] += gv[0];
      g[1] -= gv[1];
      g[2] += gv[2];
      g[3] += gv[3];
      g[4] += gv[4];
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  if (MODE == STAGE_VJP) {
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v * N + gi] = g[v];
  } else {
    const T dt = c.dt, h2 = T(0.5) * c.dt;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const long long q = v * N + gi;
      const T av = a[q], g2v = gnext[q], g3v = g3[q], g4v = g4[q];
      out[q] = av + g[v] + g2v + g3v + g4v;
      if (grad_s) grad_s[q] += dt * av + dt * g4v + h2 * (g3v + g2v);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Host-side launchers: the tile shape of each kernel class and precision is a process-wide
// setting (adj_set_tile), dispatched here to the matching instantiation.
// ------------------------------------------------------------------------------------------
template <int TX, int TY, int TZ>
static dim3 tile_grid(int nx, int ny, int nz) {
  return dim3((nx + TX - 1) / TX, (ny + TY - 1) / TY, (nz + TZ - 1) / TZ);
}

template <typename T, int TX, int TY, int TZ>
static void primal_tile(int mode, const Consts<T>& c, const T* W, const T* wn, const T* s, const T* W2, const T* W3,
                        T cR, T* out, hipStream_t st) {
  const dim3 grid = tile_grid<TX, TY, TZ>(c.nx, c.ny, c.nz), blk(TX * TY * TZ);
  if (mode == STAGE_RES)
    hipLaunchKernelGGL((k_primal_stage<T, STAGE_RES, TX, TY, TZ>), grid, blk, 0, st, c, W, wn, s, W2, W3, cR, out);
  else if (mode == STAGE_LIN)
    hipLaunchKernelGGL((k_primal_stage<T, STAGE_LIN, TX, TY, TZ>), grid, blk, 0, st, c, W, wn, s, W2, W3, cR, out);
  else
    hipLaunchKernelGGL((k_primal_stage<T, STAGE_FIN, TX, TY, TZ>), grid, blk, 0, st, c, W, wn, s, W2, W3, cR, out);
}

template <typename T>
hipError_t launch_primal_stage(int mode, const Consts<T>& c, const T* W, const T* wn, const T* s, const T* W2,
                               const T* W3, T cR, T* out, hipStream_t st) {
  ProfScope ps(ADJ_PROF_PRIMAL_STAGE, st);
  switch (tile_choice(ADJ_PROF_PRIMAL_STAGE, sizeof(T) == 8)) {
    case TILE_16x4x4: primal_tile<T, 16, 4, 4>(mode, c, W, wn, s, W2, W3, cR, out, st); break;
    case TILE_32x4x2: primal_tile<T, 32, 4, 2>(mode, c, W, wn, s, W2, W3, cR, out, st); break;
    case TILE_32x4x4: primal_tile<T, 32, 4, 4>(mode, c, W, wn, s, W2, W3, cR, out, st); break;
    default: primal_tile<T, 32, 8, 2>(mode, c, W, wn, s, W2, W3, cR, out, st); break;
  }
  return hipGetLastError();
}

template <typename T, int WALL, int LNU, int TX, int TY, int TZ>
static void adjoint_tile(int mode, const Consts<T>& c, const T* W, const T* a, const T* gnext, const T* nu, T ca, T cg,
                         const T* g3, const T* g4, T* out, T* grad_s, hipStream_t st) {
  const dim3 grid = tile_grid<TX, TY, TZ>(c.nx, c.ny, c.nz), blk(TX * TY * TZ);
  if (mode == STAGE_VJP)
    hipLaunchKernelGGL((k_adjoint_stage<T, STAGE_VJP, WALL, LNU, TX, TY, TZ>), grid, blk, 0, st, c, W, a, gnext, nu, ca,
                       cg, g3, g4, out, grad_s);
  else
    hipLaunchKernelGGL((k_adjoint_stage<T, STAGE_FIN, WALL, LNU, TX, TY, TZ>), grid, blk, 0, st, c, W, a, gnext, nu, ca,
                       cg, g3, g4, out, grad_s);
}

template <typename T, int WALL, int LNU>
static void adjoint_variant(int mode, const Consts<T>& c, const T* W, const T* a, const T* gnext, const T* nu, T ca,
                            T cg, const T* g3, const T* g4, T* out, T* grad_s, hipStream_t st) {
  switch (tile_choice(ADJ_PROF_ADJOINT_STAGE, sizeof(T) == 8)) {
    case TILE_16x4x4: adjoint_tile<T, WALL, LNU, 16, 4, 4>(mode, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st); break;
    case TILE_32x4x2: adjoint_tile<T, WALL, LNU, 32, 4, 2>(mode, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st); break;
    case TILE_32x4x4: adjoint_tile<T, WALL, LNU, 32, 4, 4>(mode, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st); break;
    default: adjoint_tile<T, WALL, LNU, 32, 8, 2>(mode, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st); break;
  }
}

template <typename T>
hipError_t launch_adjoint_stage(int mode, const Consts<T>& c, const T* W, const T* a, const T* gnext, const T* nu,
                                T ca, T cg, const T* g3, const T* g4, T* out, T* grad_s, hipStream_t st) {
  ProfScope ps(ADJ_PROF_ADJOINT_STAGE, st);
  if (c.wall) {
    if (nu)
      adjoint_variant<T, 1, 1>(mode, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st);
    else
      adjoint_variant<T, 1, 0>(mode, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st);
  } else {
    if (nu)
      adjoint_variant<T, 0, 1>(mode, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st);
    else
      adjoint_variant<T, 0, 0>(mode, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st);
  }
  return hipGetLastError();
}

template hipError_t launch_primal_stage<float>(int, const Consts<float>&, const float*, const float*, const float*,
                                               const float*, const float*, float, float*, hipStream_t);
template hipError_t launch_primal_stage<double>(int, const Consts<double>&, const double*, const double*, const double*,
                                                const double*, const double*, double, double*, hipStream_t);
template hipError_t launch_adjoint_stage<float>(int, const Consts<float>&, const float*, const float*, const float*,
                                                const float*, float, float, const float*, const float*, float*,
                                                float*, hipStream_t);
template hipError_t launch_adjoint_stage<double>(int, const Consts<double>&, const double*, const double*,
                                                 const double*, const double*, double, double, const double*,
                                                 const double*, double*, double*, hipStream_t);

}  // namespace adjns
