// roe_flux.hpp -- Roe's approximate Riemann flux of two face states and its hand-written
// reverse, shared by the Roe-flux kernels (roe.hip) and the characteristic-boundary kernels
// (char.hip).
//
// Roe's solver [Numerical methods]: F = (F_d(w_l) + F_d(w_r))/2 - (1/2) sum_k |lam_k|_s a_k r_k
// with the Roe averages (weights sqrt(rho)), the acoustic, entropy and shear waves, and every
// |lam| smoothed within delta = roe_delta c~ of zero ((lam^2 + delta^2)/(2 delta) there), so that
// the flux has a derivative everywhere.  States are held as (rho, rho u (full values),
// rho E - wref_E); momentum fluxes carry p - p0, p0 = (gamma - 1) wref_E (a uniform pressure has
// no divergence).
#pragma once
#include "common.hpp"

namespace adjns {
namespace roeflux {

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
// out[0], out[1] = d(G . F)/d(w_l), d(G . F)/d(w_r); the cells (a, b, c, e) then receive
// (-ql out[0], out[0] + qr out[1], ql out[0] + out[1], -qr out[1]).
template <typename T, int D, bool REV>
__device__ __forceinline__ void roe_face(const T a[5], const T b[5], const T c[5], const T e[5], const RoeC<T>& k,
                                         T ql, T qr, const T G[5], T out[][5]) {
  T wl[5], wr[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    wl[v] = b[v] + ql * (c[v] - a[v]);
    wr[v] = c[v] - qr * (e[v] - b[v]);
  }
  if constexpr (!REV) {
    roe_flux2<T, D, false>(wl, wr, k, G, out[0], nullptr, nullptr);
  } else {
#pragma unroll
    for (int q = 0; q < 5; ++q) out[0][q] = out[1][q] = T(0);
    roe_flux2<T, D, true>(wl, wr, k, G, nullptr, out[0], out[1]);
  }
}

template <typename T>
__host__ RoeC<T> roe_consts(const Consts<T>& c, T roe_delta, int open, int split = 0) {
  RoeC<T> k;
  k.gm1 = c.gamma - T(1);
  k.eref = c.wref[4];
  k.p0 = k.gm1 * c.wref[4];
  k.dfrac = roe_delta;
  k.open = open;
  k.split = split;
  return k;
}

}  // namespace roeflux
}  // namespace adjns
