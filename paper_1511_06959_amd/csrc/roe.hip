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
// tile needs is evaluated once into LDS, and each cell then gathers from its faces.  Slip walls:
// ghost cells hold mirrored states and kh = 0; faces between two ghosts do not exist; a wall
// cell adds the shares its ghost images receive, mapped back through the mirror (rho u_x odd).
#include "kernels.hpp"

namespace adjns {
namespace {

// Output tile of both kernels: rows of 16 cells (x), 4 x 4 rows, one cell per thread.
constexpr int RX = 16, RY = 4, RZ = 4, RNT = RX * RY * RZ;

// 1/sqrt(x): the hardware approximation in FP32 (about 1 ulp), exact operations in FP64.
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

template <typename T>
struct RoeC {
  T gm1, eref, p0, dfrac;  // gamma - 1, wref_E, (gamma - 1) wref_E, roe_delta
  int open;                // characteristic boundaries in x (the Roe kernels leave their faces alone)
  int split;               // boundary kernels: the stage kernels included the split-form flux
};

// Cell and face values are held as (rho, rho u (full values), rho E - wref_E).  Primitive form:
template <typename T>
struct Pr {
  T ir, u[3], pd, Ep;  // 1/rho, velocity, p - p0, rho E + p
};

template <typename T>
__device__ __forceinline__ Pr<T> prim_of(const T w[5], const RoeC<T>& k) {
  Pr<T> q;
  q.ir = recip(w[0]);
#pragma unroll
  for (int j = 0; j < 3; ++j) q.u[j] = w[1 + j] * q.ir;
  q.pd = k.gm1 * (w[4] - T(0.5) * (w[1] * q.u[0] + w[2] * q.u[1] + w[3] * q.u[2]));
  q.Ep = w[4] + k.eref + q.pd + k.p0;
  return q;
}

// Reverse of prim_of: the adjoints of u, p - p0, rho E + p and 1/rho, accumulated into wb.
template <typename T>
__device__ __forceinline__ void prim_of_vjp(const T w[5], const Pr<T>& q, const RoeC<T>& k, const T ub_in[3], T pdb,
                                            T Epb, T irb, T wb[5]) {
  T ub[3] = {ub_in[0], ub_in[1], ub_in[2]};
  wb[4] += Epb;  // Ep = w4 + wref_E + pd + p0
  pdb += Epb;
  wb[4] += k.gm1 * pdb;  // pd = (gamma - 1)(w4 - K),  K = m.u/2
  const T Kb = -k.gm1 * pdb;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    ub[j] += T(0.5) * Kb * w[1 + j];
    wb[1 + j] += T(0.5) * Kb * q.u[j] + ub[j] * q.ir;  // u = m / rho
    irb += ub[j] * w[1 + j];
  }
  wb[0] -= irb * q.ir * q.ir;
}

// |x| smoothed within del of zero (id = 1/del); dx, dd: its derivatives with respect to x and del.
template <typename T>
__device__ __forceinline__ T sabs(T x, T del, T id, T& dx, T& dd) {
  if (x >= del) {
    dx = T(1);
    dd = T(0);
    return x;
  }
  if (x <= -del) {
    dx = T(-1);
    dd = T(0);
    return -x;
  }
  dx = x * id;
  dd = T(0.5) * (T(1) - x * x * id * id);
  return T(0.5) * (x * x + del * del) * id;
}

// Roe's flux between the face states wl and wr in direction D (momentum flux with p - p0).
// REV = false: F = the flux.  REV = true: the adjoints of G . F with respect to wl and wr are
// added to wlb and wrb.
template <typename T, int D, bool REV>
__device__ __forceinline__ void roe_flux2(const T wl[5], const T wr[5], const RoeC<T>& k, const T G[5], T F[5],
                                          T wlb[5], T wrb[5]) {
  const Pr<T> L = prim_of(wl, k), R = prim_of(wr, k);
  const T Hl = L.Ep * L.ir, Hr = R.Ep * R.ir;
  const T isl = rsq(wl[0]), isr = rsq(wr[0]), sl = wl[0] * isl, sr = wr[0] * isr;
  const T is = recip(sl + sr), fl = sl * is, fr = sr * is;
  T ut[3], du[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    ut[j] = fl * L.u[j] + fr * R.u[j];
    du[j] = R.u[j] - L.u[j];
  }
  const T Ht = fl * Hl + fr * Hr;
  const T q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  const T c2 = k.gm1 * (Ht - T(0.5) * q2);
  const T ics = rsq(c2), cs = c2 * ics, ic2 = ics * ics;
  const T rt = sl * sr, un = ut[D], dun = du[D];
  const T drho = wr[0] - wl[0], dp = R.pd - L.pd;
  const T del = k.dfrac * cs, idel = recip(del);
  T d1x, d1d, d2x, d2d, d5x, d5d;
  const T l1 = sabs(un - cs, del, idel, d1x, d1d), l2 = sabs(un, del, idel, d2x, d2d),
          l5 = sabs(un + cs, del, idel, d5x, d5d);
  const T rcd = rt * cs * dun;
  const T t1 = dp - rcd, t5 = dp + rcd, hi = T(0.5) * ic2;
  const T s1 = l1 * t1 * hi, s5 = l5 * t5 * hi;  // |lam| a of the acoustic waves
  const T e2 = drho - dp * ic2, s2 = l2 * e2;    // |lam| a of the entropy wave
  const T S = s1 + s5 + s2, Ls = l2 * rt, dif = s5 - s1;
  const T udu = ut[0] * du[0] + ut[1] * du[1] + ut[2] * du[2];
  if constexpr (!REV) {
    // F = mean of the cell fluxes of the face states - (1/2) sum_k |lam_k| a_k r_k
    T Dv[5];
    Dv[0] = S;
#pragma unroll
    for (int j = 0; j < 3; ++j) Dv[1 + j] = j == D ? S * un + dif * cs : S * ut[j] + Ls * du[j];
    Dv[4] = (s1 + s5) * Ht + dif * un * cs + s2 * T(0.5) * q2 + Ls * (udu - un * dun);
    F[0] = T(0.5) * (wl[1 + D] + wr[1 + D]);
#pragma unroll
    for (int j = 0; j < 3; ++j) F[1 + j] = T(0.5) * (wl[1 + D] * L.u[j] + wr[1 + D] * R.u[j]);
    F[1 + D] += T(0.5) * (L.pd + R.pd);
    F[4] = T(0.5) * (L.Ep * L.u[D] + R.Ep * R.u[D]);
#pragma unroll
    for (int q = 0; q < 5; ++q) F[q] -= T(0.5) * Dv[q];
  } else {
    // ---- reverse of the dissipation term (weight -G/2)
    T gD[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) gD[q] = T(-0.5) * G[q];
    T Sb = gD[0], Lsb = T(0), unb = T(0), s1b = T(0), s5b = T(0), s2b = T(0), csb = T(0), Htb = T(0), q2b = T(0),
      udub = T(0), dunb = T(0);
    T utb[3] = {T(0), T(0), T(0)}, dub[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (j == D) {  // S un + (s5 - s1) cs
        Sb += gD[1 + j] * un;
        unb += gD[1 + j] * S;
        s5b += gD[1 + j] * cs;
        s1b -= gD[1 + j] * cs;
        csb += gD[1 + j] * dif;
      } else {  // S ut_j + Ls du_j
        Sb += gD[1 + j] * ut[j];
        utb[j] += gD[1 + j] * S;
        Lsb += gD[1 + j] * du[j];
        dub[j] += gD[1 + j] * Ls;
      }
    }
    {  // (s1 + s5) Ht + (s5 - s1) un cs + s2 q2/2 + Ls (udu - un dun)
      const T g4 = gD[4];
      s1b += g4 * (Ht - un * cs);
      s5b += g4 * (Ht + un * cs);
      Htb += g4 * (s1 + s5);
      unb += g4 * (dif * cs - Ls * dun);
      csb += g4 * dif * un;
      s2b += g4 * T(0.5) * q2;
      q2b += g4 * T(0.5) * s2;
      Lsb += g4 * (udu - un * dun);
      udub += g4 * Ls;
      dunb -= g4 * Ls * un;
    }
    s1b += Sb;
    s5b += Sb;
    s2b += Sb;
    T l2b = Lsb * rt, rtb = Lsb * l2;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      utb[j] += udub * du[j];
      dub[j] += udub * ut[j];
    }
    l2b += s2b * e2;
    const T e2b = s2b * l2;
    const T drhob = e2b;
    T dpb = -e2b * ic2, ic2b = -e2b * dp;
    const T l1b = s1b * t1 * hi, t1b = s1b * l1 * hi, l5b = s5b * t5 * hi, t5b = s5b * l5 * hi;
    ic2b += T(0.5) * (s1b * l1 * t1 + s5b * l5 * t5);
    dpb += t1b + t5b;
    const T rcdb = t5b - t1b;
    rtb += rcdb * cs * dun;
    csb += rcdb * rt * dun;
    dunb += rcdb * rt * cs;
    unb += l1b * d1x + l2b * d2x + l5b * d5x;
    csb += l5b * d5x - l1b * d1x + (l1b * d1d + l2b * d2d + l5b * d5d) * k.dfrac;
    utb[D] += unb;
    dub[D] += dunb;
    const T c2b = csb * T(0.5) * ics - ic2b * ic2 * ic2;
    Htb += c2b * k.gm1;
    q2b -= c2b * k.gm1 * T(0.5);
    T flb = Htb * Hl, frb = Htb * Hr;
    const T Hlb = Htb * fl, Hrb = Htb * fr;
    T ulb[3], urb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      utb[j] += T(2) * q2b * ut[j];
      flb += utb[j] * L.u[j];
      frb += utb[j] * R.u[j];
      ulb[j] = utb[j] * fl - dub[j];
      urb[j] = utb[j] * fr + dub[j];
    }
    const T slb = (flb - frb) * fr * is + rtb * sr;
    const T srb = (frb - flb) * fl * is + rtb * sl;
    wlb[0] += -drhob + slb * T(0.5) * isl;
    wrb[0] += drhob + srb * T(0.5) * isr;
    // ---- reverse of the mean of the cell fluxes (weight G)
    T pdlb = -dpb + T(0.5) * G[1 + D], pdrb = dpb + T(0.5) * G[1 + D];
    wlb[1 + D] += T(0.5) * G[0];
    wrb[1 + D] += T(0.5) * G[0];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      wlb[1 + D] += T(0.5) * G[1 + j] * L.u[j];
      wrb[1 + D] += T(0.5) * G[1 + j] * R.u[j];
      ulb[j] += T(0.5) * G[1 + j] * wl[1 + D];
      urb[j] += T(0.5) * G[1 + j] * wr[1 + D];
    }
    ulb[D] += T(0.5) * G[4] * L.Ep;
    urb[D] += T(0.5) * G[4] * R.Ep;
    const T Eplb = T(0.5) * G[4] * L.u[D] + Hlb * L.ir, Eprb = T(0.5) * G[4] * R.u[D] + Hrb * R.ir;
    prim_of_vjp(wl, L, k, ulb, pdlb, Eplb, Hlb * L.Ep, wlb);
    prim_of_vjp(wr, R, k, urb, pdrb, Eprb, Hrb * R.Ep, wrb);
  }
}

// Roe's flux through the direction-D face between cells b and c; a and e are the next cells
// outward, the face states w_l = b + ql (c - a), w_r = c - qr (e - b) with ql, qr = 1/4 (0 where
// the reconstruction would reach beyond an open boundary).  REV = false: out[0] = F.  REV = true:
// out[j] = d(G . F)/d(cell j) for the cells (a, b, c, e).
template <typename T, int D, bool REV>
__device__ __forceinline__ void roe_face(const T a[5], const T b[5], const T c[5], const T e[5], const RoeC<T>& k,
                                         T ql, T qr, const T G[5], T out[4][5]) {
  T wl[5], wr[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    wl[v] = b[v] + ql * (c[v] - a[v]);
    wr[v] = c[v] - qr * (e[v] - b[v]);
  }
  if constexpr (!REV) {
    roe_flux2<T, D, false>(wl, wr, k, G, out[0], nullptr, nullptr);
  } else {
    T wlb[5] = {T(0), T(0), T(0), T(0), T(0)}, wrb[5] = {T(0), T(0), T(0), T(0), T(0)};
    roe_flux2<T, D, true>(wl, wr, k, G, nullptr, wlb, wrb);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      out[0][q] = -ql * wlb[q];
      out[1][q] = wlb[q] + qr * wrb[q];
      out[2][q] = ql * wlb[q] + wrb[q];
      out[3][q] = -qr * wrb[q];
    }
  }
}

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
  const unsigned fb = (unsigned)(c.N * (long long)sizeof(T));
  for (int e = threadIdx.x; e < E::N; e += RNT) {
    const int ex = e % E::EX, ey = (e / E::EX) % E::EY, ez = e / (E::EX * E::EY);
    const int gx = x0 + ex - (D == 0 ? H : 0), gy = y0 + ey - (D == 1 ? H : 0), gz = z0 + ez - (D == 2 ? H : 0);
    int mir, real;
    const unsigned off = (unsigned)(c.wall ? box_cell32<1>(c.nx, c.ny, c.nz, gx, gy, gz, mir, real)
                                           : box_cell32<0>(c.nx, c.ny, c.nz, gx, gy, gz, mir, real)) *
                         (unsigned)sizeof(T);
    T w[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) w[v] = buf_load(rW, off, v * fb, T());
    const T mx = w[1] + c.wref[1];
    lds[e] = w[0] + c.wref[0];
    lds[np + e] = mir ? -mx : mx;
    lds[2 * np + e] = w[2] + c.wref[2];
    lds[3 * np + e] = w[3] + c.wref[3];
    lds[4 * np + e] = w[4];
    if (KH) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        T kh = T(0);
        if (real) {
          kh = ca * buf_load(ra, off, v * fb, T());
          if (has_g) kh += cg * buf_load(rg, off, v * fb, T());
        }
        lds[(5 + v) * np + e] = kh;
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
    T w[4][5], o[4][5] = {};
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
  tile_origin<RX, RY, RZ>(xcd_tile(blockIdx.x, gridDim.x), c.nx, c.ny, x0, y0, z0);
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
constexpr int NLA = 10 * NSA > 20 * NFA ? 10 * NSA : 20 * NFA;

// Shares that the direction-D faces hand to the cell at tile position t along D (cross
// coordinates x, y, z): face p (lower cell p - 2) gives share 3 - (p - t) for p = t .. t + 3.
template <typename T, int D>
__device__ __forceinline__ void gather(const T* fr, int t, int x, int y, int z, T sgn1, T acc[5]) {
  constexpr int TD = D == 0 ? RX : (D == 1 ? RY : RZ);
  using F = Faces<D, TD + 3>;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int p = t + q;
    if (p < 0 || p >= TD + 3) continue;
    const int f = F::at(p, x, y, z);
    const int j = 3 - q;
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[v] += (v == 1 ? sgn1 : T(1)) * fr[(j * 5 + v) * NFA + f];
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
  T rec[NPT][4][5];
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int f = threadIdx.x + i * RNT;
    bool live = f < F::N;
    int p = 0, x = 0, y = 0, z = 0;
    if (live) F::coords(f, p, x, y, z);
    T ql = T(0.25), qr = T(0.25);
    if (live && D == 0 && c.wall) {
      const int gl = x0 + p - 2;
      if (k.open) {  // as in the forward kernel
        live = gl >= 0 && gl <= c.nx - 2;
        ql = gl >= 1 ? T(0.25) : T(0);
        qr = gl + 2 <= c.nx - 1 ? T(0.25) : T(0);
      } else {  // slip walls: a face needs a real cell on at least one side
        live = gl >= -1 && gl <= c.nx - 1;
      }
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
      for (int j = 0; j < 4; ++j)
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
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 5; ++v) lds[(j * 5 + v) * NFA + f] = rec[i][j][v];
    }
  }
  __syncthreads();
  if (active) {
    const int t = D == 0 ? tx : (D == 1 ? ty : tz);
    gather<T, D>(lds, t, tx, ty, tz, T(1), acc);
    if (D == 0 && c.wall) {
      // shares of the ghost images of this cell (x <= 1: left wall, x >= nx - 2: right wall)
      const int gx = x0 + tx;
      if (gx <= 1) gather<T, D>(lds, -1 - gx - x0, tx, ty, tz, T(-1), acc);
      if (gx >= c.nx - 2) gather<T, D>(lds, 2 * c.nx - 1 - gx - x0, tx, ty, tz, T(-1), acc);
    }
  }
  __syncthreads();
}

// FP32: at most 128 registers, so that four work-groups (16 wavefronts) share a compute unit and
// a 64^3 grid (1024 work-groups) runs in one round; FP64 holds two (LDS and registers).
template <typename T>
__global__ __launch_bounds__(RNT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
void k_roe_adjoint(Consts<T> c, RoeC<T> k, const T* __restrict__ W,
                                                     const T* __restrict__ a, const T* __restrict__ gnext, T ca, T cg,
                                                     T* __restrict__ out) {
  __shared__ T lds[NLA];
  int x0, y0, z0;
  tile_origin<RX, RY, RZ>(xcd_tile(blockIdx.x, gridDim.x), c.nx, c.ny, x0, y0, z0);
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

// ------------------------------------------------------------------------ open boundaries in x
// Characteristic inflow/outflow boundaries (bc_x = ADJ_BC_CHARACTERISTIC).  The stage kernels
// treat them as slip walls (mirror ghosts), so through each boundary face they evaluate the
// mirror-pair flux H_w = (0, p - p0 - s_xx, 0, 0, 0), or (0, -s_xx, 0, 0, 0) when they run
// without the split-form convective flux (Roe grids, whose Roe kernels skip the boundary faces):
// the mirror pair carries no mass, energy, tangential stress or heat, and
// s_xx = (4/3) mu g_n - (2/3) mu (d_y u_y + d_z u_z) with the normal gradient g_n = +-2 u_x/dx of
// the pair and the boundary cell's central tangential divergence.  The kernels here replace H_w by the characteristic flux F_c, Roe's flux between the
// far-field state and the boundary cell (x = 0) or the boundary cell and the far-field state
// (x = L_x), which takes the entering waves from the far field and the leaving ones from inside:
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
  T w[5];
  held(c, W, b.q, w);
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
  for (int v = 0; v < 5; ++v) out[v * c.N + b.q] += f * F[v];
}

template <typename T>
__global__ __launch_bounds__(CB) void k_char_adjoint(Consts<T> c, RoeC<T> k, Far<T> far, const T* __restrict__ W,
                                                     const T* __restrict__ a, const T* __restrict__ gnext, T ca, T cg,
                                                     T* __restrict__ out) {
  BCell<T> b;
  if (!bcell(c, (int)(blockIdx.x * CB + threadIdx.x), b)) return;
  auto kh = [&](int v, long long q) { return ca * a[v * c.N + q] + (gnext ? cg * gnext[v * c.N + q] : T(0)); };
  const T sg = b.side ? -c.idx[0] : c.idx[0];
  T w[5], G[5];
  held(c, W, b.q, w);
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
  for (int v = 0; v < 5; ++v) out[v * c.N + b.q] += wb[v];
}

template <typename T>
RoeC<T> roe_consts(const Consts<T>& c, T roe_delta, int open, int split = 0) {
  RoeC<T> k;
  k.gm1 = c.gamma - T(1);
  k.eref = c.wref[4];
  k.p0 = k.gm1 * c.wref[4];
  k.dfrac = roe_delta;
  k.open = open;
  k.split = split;
  return k;
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

#define ADJNS_ROE_INST(T)                                                                                          \
  template hipError_t launch_roe_primal<T>(const Consts<T>&, T, int, const T*, T, T*, hipStream_t);                \
  template hipError_t launch_roe_adjoint<T>(const Consts<T>&, T, int, const T*, const T*, const T*, T, T, T*,       \
                                            hipStream_t);                                                          \
  template hipError_t launch_char_primal<T>(const Consts<T>&, T, int, const double*, const T*, T, T*, hipStream_t); \
  template hipError_t launch_char_adjoint<T>(const Consts<T>&, T, int, const double*, const T*, const T*, const T*, \
                                             T, T, T*, hipStream_t);
ADJNS_ROE_INST(float)
ADJNS_ROE_INST(double)
#undef ADJNS_ROE_INST

}  // namespace adjns
