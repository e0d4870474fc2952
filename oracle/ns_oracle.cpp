// ns_oracle.cpp -- plain FP64 CPU oracle for the stabilised discrete unsteady adjoint of the
// compressible Navier-Stokes equations (Talnikar, Wang & Laskowski, GT2016-56689).
//
// TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library against the paper.
// Only the test suite, the smoke check and the benchmark's CPU-baseline leg load it; the
// product path never links, imports or calls it, and it shares no code, header, table or
// helper with the GPU kernels.
//
// Written for clarity, not speed: every residual is a loop over faces, every derivative comes
// from forward-mode dual numbers (automatic differentiation, the tool the paper used to obtain
// its discrete adjoint, section "Implementation"), and every reduction is a serial sum in a
// fixed order.  The only parallelism is OpenMP over independent faces/cells with per-thread
// accumulators that are summed in thread order afterwards.
//
// What is computed (paper section / equation in brackets):
//   * residual  R(w; s) = -div_h F(w) + div_h F^v(w) + s          [Physics, Eq. (navier); vector form; index form with s_i]
//       - convective face flux  (split central form of Kennedy & Gruber, JCP 227, 2008):
//         with face means  r = <rho>, v = <u>, H = <E/rho>, P = <p>  (<q> = (q_L + q_R)/2)
//           F~ = r v_d (1, v, H) + P (0, e_d, v_d)
//         The paper's solver relied on the numerical dissipation of its upwind flux and adds no
//         subgrid model (section "Large Eddy Simulation"); a plain average of the two cell
//         fluxes has neither, and on the under-resolved wake box (Re 5e4 on the wake width,
//         512x256x32 cells) it diverged within 1700 steps, so the convective terms use this
//         kinetic-energy-preserving product of means instead (still conservative, second order,
//         and identical to the cell-flux average to first order about a uniform state).
//       - viscous face flux     (0, sigma_d., u_f . sigma_d. + alpha d_d e) with face gradients:
//         normal (phi_R - phi_L)/dx_d, tangential = mean of the two cells' central differences
//       - sigma = mu (grad u + grad u^T) - (2 mu / 3) (div u) I,  p = (gamma-1) rho e,
//         e = E - |u|^2/2,  alpha = gamma mu / Pr  (heat flux alpha grad e = k grad T)
//       - or (option) Roe's approximate Riemann solver on linearly reconstructed face states
//         [Numerical methods], every |wave speed| smoothed near zero (Harten)
//   * classical RK4 in time with fixed dt (or the strong-stability-preserving RK3)
//   * discrete adjoint of the RK4 step [Implementation; terminal condition and backward solve]:
//       the transposed Jacobian of every face flux is assembled from dual-number local Jacobians
//   * artificial adjoint viscosity  d_l( lambda sigma_1 delta_ki delta_jl d_j w^_k )  [Stabilizing
//     adjoint equations, last equation], discretised as a symmetric face-based Laplacian; with
//     one lambda per variable group (rho, rho u, rho E), the separate adjoint viscosities the
//     Conclusion proposes
//   * growth matrix M = M1 - M2 and its largest singular value sigma_1 [Energy Analysis, M1/M2]
//   * adjoint energy E = int |v^|^2 dV with v^ = T^{-T} w^ [Symmetrization, Energy Analysis]
//   * objectives: volume-mean pressure, volume-mean viscous dissipation sigma:grad u, and the
//     density-weighted stagnation-pressure loss on a plane [Eqs. (1)-(3), pressure loss]
//
// Layout: SoA, var-major, w[v*N + (k*ny + j)*nx + i], v = (rho, rho u1, rho u2, rho u3, rho E).
// Boundaries: periodic in y and z; x either periodic, inviscid-mirror slip walls (ghost cell
// mirrors the first interior cell with the x-momentum sign flipped), or characteristic inflow /
// outflow boundaries: the same mirror ghosts in every stencil, and through the two boundary faces
// the inviscid upwind (Roe) flux between the boundary cell and a far-field state.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {
typedef struct orc_grid {
  int32_t n[3];
  int32_t bc_x;  // 0: periodic in x, 1: slip walls at x = 0 and x = L_x, 2: characteristic
                 //    inflow/outflow boundaries there (far-field states w_far)
  double L[3];
  double gamma, prandtl, mu, dt;
  int32_t scheme;  // time marching: 0 classical RK4, 1 strong-stability-preserving RK3
  int32_t flux;    // convective face flux: 0 split central form, 1 Roe upwind flux
  double roe_delta;  // flux 1: width of the smoothing of |wave speed|, as a fraction of the Roe sound speed
  double w_far[2][5];  // bc_x 2: far-field conservative states beyond x = 0 and beyond x = L_x
} orc_grid;

typedef struct orc_obj {
  int32_t kind;     // 0 none, 1 mean pressure, 2 viscous dissipation, 3 stagnation-pressure loss
  int32_t plane_i;  // kind 3: the x-face between cells plane_i-1 and plane_i
  double pt_ref;    // kind 3: reference (inlet / free-stream) stagnation pressure
} orc_obj;
}

namespace {

// ------------------------------------------------------------------------------------------
// Forward-mode dual numbers: value plus N directional derivatives.
// ------------------------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
};
template <int N> Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a) { Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
template <int N> Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> Dual<N> operator+(double a, const Dual<N>& b) { return b + a; }
template <int N> Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> Dual<N> operator-(double a, const Dual<N>& b) { return -(b - a); }
template <int N> Dual<N> operator*(const Dual<N>& a, double b) { Dual<N> r; r.v = a.v * b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r; }
template <int N> Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> Dual<N> operator/(const Dual<N>& a, double b) { Dual<N> r; r.v = a.v / b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / b; return r; }
template <int N> Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N> Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) { a = a - b; return a; }
template <int N> Dual<N> sqrt(const Dual<N>& a) {
  Dual<N> r; r.v = std::sqrt(a.v);
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / (2.0 * r.v);
  return r;
}
template <int N> Dual<N> pow(const Dual<N>& a, double e) {
  Dual<N> r; r.v = std::pow(a.v, e);
  const double dr = e * std::pow(a.v, e - 1.0);
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * dr;
  return r;
}
using std::sqrt;
using std::pow;

// Value of a plain or dual number, for branch decisions.
inline double val(double x) { return x; }
inline double val(const std::complex<double>& x) { return x.real(); }
template <int N> double val(const Dual<N>& x) { return x.v; }

// ------------------------------------------------------------------------------------------
// Grid helpers
// ------------------------------------------------------------------------------------------
struct G {
  long nx, ny, nz, N;
  double dx[3];
  int wall, bc, scheme, flux;
  double gamma, pr, mu, alpha, dt, roe_delta;
  double wfar[2][5];
  explicit G(const orc_grid* g) {
    nx = g->n[0]; ny = g->n[1]; nz = g->n[2]; N = nx * ny * nz;
    for (int d = 0; d < 3; ++d) dx[d] = g->L[d] / (double)g->n[d];
    wall = g->bc_x != 0;  // walls and open boundaries both keep mirror ghosts in every stencil
    bc = g->bc_x;
    for (int s = 0; s < 2; ++s)
      for (int v = 0; v < 5; ++v) wfar[s][v] = g->w_far[s][v];
    scheme = g->scheme;
    flux = g->flux;
    roe_delta = g->roe_delta;
    gamma = g->gamma; pr = g->prandtl; mu = g->mu; dt = g->dt;
    alpha = gamma * mu / pr;  // heat flux alpha grad e == (mu c_p / Pr) grad T, since e = c_v T
  }
  long n(int d) const { return d == 0 ? nx : (d == 1 ? ny : nz); }
  long idx(long i, long j, long k) const { return (k * ny + j) * nx + i; }
};

inline long wrap(long i, long n) { i %= n; return i < 0 ? i + n : i; }

// A stencil slot: which cell provides the value, and whether it is the x-wall mirror image.
struct Slot { long c; int mirror; bool real; };

Slot slot(const G& g, long i, long j, long k) {
  Slot s; s.mirror = 0; s.real = true;
  j = wrap(j, g.ny); k = wrap(k, g.nz);
  if (!g.wall) {
    i = wrap(i, g.nx);
  } else if (i < 0) {
    i = -1 - i; s.mirror = 1; s.real = false;
  } else if (i >= g.nx) {
    i = 2 * g.nx - 1 - i; s.mirror = 1; s.real = false;
  }
  s.c = g.idx(i, j, k);
  return s;
}
// Mirror ghost: rho, tangential momentum and total energy even; x-momentum odd.
inline double mirror_sign(int mirror, int v) { return (mirror && v == 1) ? -1.0 : 1.0; }

template <class T>
void load_slot(const G& g, const T* w, const Slot& s, T out[5]) {
  for (int v = 0; v < 5; ++v) out[v] = mirror_sign(s.mirror, v) * w[v * g.N + s.c];
}

template <class T>
struct Prim { T rho, u[3], e, p, E; };

// Primitive variables from w = (rho, rho u, rho E)   [Physics: p = (gamma-1) rho e, e = E - u.u/2]
template <class T>
Prim<T> prim(const G& g, const T w[5]) {
  Prim<T> q;
  q.rho = w[0];
  for (int k = 0; k < 3; ++k) q.u[k] = w[1 + k] / q.rho;
  q.E = w[4];
  q.e = q.E / q.rho - 0.5 * (q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2]);
  q.p = (g.gamma - 1.0) * q.rho * q.e;
  return q;
}

// Convective face flux in direction d between cells L and R   [vector form: F = (rho u,
// rho u u + p I, (rho E + p) u)], each product of cell fields replaced by the product of the
// face means of its factors (Kennedy & Gruber):  mass r v_d, momentum r v_d v + P e_d,
// energy r v_d H + P v_d, with H the mean of the specific total energy E/rho.
template <class T>
void conv_face_flux(int d, const Prim<T>& L, const Prim<T>& R, T F[5]) {
  T r = 0.5 * (L.rho + R.rho);
  T v[3];
  for (int k = 0; k < 3; ++k) v[k] = 0.5 * (L.u[k] + R.u[k]);
  T H = 0.5 * (L.E / L.rho + R.E / R.rho);
  T P = 0.5 * (L.p + R.p);
  T m = r * v[d];
  F[0] = m;
  for (int k = 0; k < 3; ++k) F[1 + k] = m * v[k];
  F[1 + d] = F[1 + d] + P;
  F[4] = m * H + P * v[d];
}

// |lam| smoothed inside |lam| < delta (Harten's entropy fix): (lam^2 + delta^2) / (2 delta) there.
// Value and slope match |lam| at |lam| = delta, so the flux is differentiable everywhere and its
// discrete adjoint exists (plain |lam| has no derivative where a wave speed is zero).
template <class T>
T smooth_abs(const T& lam, const T& delta) {
  if (val(lam) >= val(delta)) return lam;
  if (val(lam) <= -val(delta)) return -lam;
  return (lam * lam + delta * delta) / (2.0 * delta);
}

// Roe's approximate Riemann solver between face states wl and wr in direction d [Numerical
// methods: approximate Roe solver]:  F = (F_d(wl) + F_d(wr))/2 - (1/2) sum_k |lam_k| a_k r_k, with
// the Roe averages (weights sqrt(rho)) u~, H~ (H = (rho E + p)/rho), rho~ = sqrt(rho_l rho_r),
// c~^2 = (gamma-1)(H~ - |u~|^2/2), and the jumps d(.) = (.)_r - (.)_l of rho, u and p:
//   acoustic waves  lam = u~_d -+ c~,  a = (dp -+ rho~ c~ du_d) / (2 c~^2),  r = (1, u~ -+ c~ e_d, H~ -+ u~_d c~)
//   entropy wave    lam = u~_d,        a = drho - dp / c~^2,                r = (1, u~, |u~|^2/2)
//   shear waves     lam = u~_d,        a r = rho~ (0, du - du_d e_d, u~.du - u~_d du_d)
// Every |lam| is smoothed with delta = roe_delta c~ (smooth_abs).
template <class T>
void roe_face_flux(const G& g, int d, const T wl[5], const T wr[5], T F[5]) {
  const Prim<T> L = prim(g, wl), R = prim(g, wr);
  const T HL = (L.E + L.p) / L.rho, HR = (R.E + R.p) / R.rho;
  const T sl = sqrt(L.rho), sr = sqrt(R.rho);
  const T fl = sl / (sl + sr), fr = sr / (sl + sr);
  T u[3], du[3];
  for (int k = 0; k < 3; ++k) {
    u[k] = fl * L.u[k] + fr * R.u[k];
    du[k] = R.u[k] - L.u[k];
  }
  const T H = fl * HL + fr * HR;
  const T q2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const T c2 = (g.gamma - 1.0) * (H - 0.5 * q2);
  const T c = sqrt(c2);
  const T rt = sl * sr;
  const T un = u[d], dun = du[d];
  const T drho = R.rho - L.rho, dp = R.p - L.p;
  const T delta = g.roe_delta * c;
  const T l1 = smooth_abs(un - c, delta), l2 = smooth_abs(un, delta), l5 = smooth_abs(un + c, delta);
  const T s1 = l1 * (dp - rt * c * dun) / (2.0 * c2);  // |lam| a of the acoustic waves
  const T s5 = l5 * (dp + rt * c * dun) / (2.0 * c2);
  const T s2 = l2 * (drho - dp / c2);                    // |lam| a of the entropy wave
  const T udu = u[0] * du[0] + u[1] * du[1] + u[2] * du[2];
  T D[5];
  D[0] = s1 + s5 + s2;
  for (int k = 0; k < 3; ++k) {
    D[1 + k] = (s1 + s5 + s2) * u[k] + l2 * rt * du[k];
    if (k == d) D[1 + k] = D[1 + k] + (s5 - s1) * c - l2 * rt * dun;
  }
  D[4] = s1 * (H - un * c) + s5 * (H + un * c) + s2 * (0.5 * q2) + l2 * rt * (udu - un * dun);
  // cell fluxes F_d(w) = (rho u_d, rho u_d u + p e_d, (rho E + p) u_d)
  T FL[5], FR[5];
  FL[0] = wl[1 + d];
  FR[0] = wr[1 + d];
  for (int k = 0; k < 3; ++k) {
    FL[1 + k] = wl[1 + d] * L.u[k];
    FR[1 + k] = wr[1 + d] * R.u[k];
  }
  FL[1 + d] = FL[1 + d] + L.p;
  FR[1 + d] = FR[1 + d] + R.p;
  FL[4] = (L.E + L.p) * L.u[d];
  FR[4] = (R.E + R.p) * R.u[d];
  for (int v = 0; v < 5; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * D[v];
}

inline void tangents(int d, int& t1, int& t2) { t1 = (d == 0) ? 1 : 0; t2 = (d == 2) ? 1 : 2; }

// Stencil of the face between cell L=(i,j,k) and R=L+e_d: slots
//   0 L, 1 R, 2 L+e_t1, 3 L-e_t1, 4 L+e_t2, 5 L-e_t2, 6 R+e_t1, 7 R-e_t1, 8 R+e_t2, 9 R-e_t2,
//   and with the Roe flux 10 L-e_d, 11 R+e_d (the reconstruction stencil)
constexpr int NSLOT = 12;
inline int nslots(const G& g) { return g.flux == 1 ? 12 : 10; }
void face_slots(const G& g, int d, long i, long j, long k, Slot st[NSLOT]) {
  long L[3] = {i, j, k};
  long R[3] = {i, j, k};
  R[d] += 1;
  int t1, t2; tangents(d, t1, t2);
  auto sl = [&](const long* c, int t, int sgn) {
    long p[3] = {c[0], c[1], c[2]};
    if (t >= 0) p[t] += sgn;
    return slot(g, p[0], p[1], p[2]);
  };
  st[0] = sl(L, -1, 0); st[1] = sl(R, -1, 0);
  st[2] = sl(L, t1, +1); st[3] = sl(L, t1, -1); st[4] = sl(L, t2, +1); st[5] = sl(L, t2, -1);
  st[6] = sl(R, t1, +1); st[7] = sl(R, t1, -1); st[8] = sl(R, t2, +1); st[9] = sl(R, t2, -1);
  st[10] = sl(L, d, -1); st[11] = sl(R, d, +1);
}

// Total face flux H = F~ - F~^v on the face between slot 0 (L) and slot 1 (R) in direction d.
//   F~   = split-form convective face flux (conv_face_flux), or with the Roe flux roe_face_flux of
//          the face states reconstructed linearly with central cell gradients (second order):
//          w_l = w_L + (w_R - w_{L-e_d})/4,  w_r = w_R - (w_{R+e_d} - w_L)/4
//   F~^v = (0, sigma_d., u_f . sigma_d. + alpha d_d e), u_f = 0.5 (u_L + u_R)
//   face gradient d_l u_k: l == d -> (u_R - u_L)/dx_d ; l != d -> mean of the central
//   differences of cells L and R in direction l.
// Characteristic boundary face (side 0: x = 0, side 1: x = L_x): the inviscid upwind flux between
// the boundary cell and the far-field state (Roe's solver, first order), which takes the waves
// entering the box from the far field and those leaving it from the interior [Boundary
// conditions: characteristic inlet and outlet].
template <class T>
void char_face_flux(const G& g, int side, const T (*st)[5], T H[5]) {
  T far[5];
  for (int v = 0; v < 5; ++v) far[v] = T(g.wfar[side][v]);
  if (side == 0)
    roe_face_flux(g, 0, far, st[1], H);
  else
    roe_face_flux(g, 0, st[0], far, H);
}

// Whether a Roe reconstruction may use the cell of slot s (not a ghost beyond an open boundary).
inline bool recon_ok(const G& g, const Slot& s) { return g.bc != 2 || s.real; }

// Which characteristic boundary face (0 or 1) the direction-d face with lower cell i is, or -1.
inline int open_side(const G& g, int d, long i) {
  if (d != 0 || g.bc != 2) return -1;
  return i == -1 ? 0 : (i == g.nx - 1 ? 1 : -1);
}

// rl, rr: whether the Roe face states are reconstructed on the left / right; next to a
// characteristic boundary a reconstruction that would reach the ghost cell is dropped (the face
// state is the cell value there), since a mirror image is no estimate of the flow beyond an
// open boundary.
template <class T>
void face_flux(const G& g, int d, const T (*st)[5], T H[5], int side = -1, bool rl = true, bool rr = true) {
  if (side >= 0) {
    char_face_flux(g, side, st, H);
    return;
  }
  Prim<T> q[10];
  for (int s = 0; s < 10; ++s) q[s] = prim(g, st[s]);
  T Fc[5];
  if (g.flux == 1) {
    T wl[5], wr[5];
    for (int v = 0; v < 5; ++v) {
      wl[v] = rl ? st[0][v] + 0.25 * (st[1][v] - st[10][v]) : st[0][v];
      wr[v] = rr ? st[1][v] - 0.25 * (st[11][v] - st[0][v]) : st[1][v];
    }
    roe_face_flux(g, d, wl, wr, Fc);
  } else {
    conv_face_flux(d, q[0], q[1], Fc);
  }
  int t[2]; tangents(d, t[0], t[1]);
  T gu[3][3];  // gu[l][k] = d_l u_k at the face
  for (int k = 0; k < 3; ++k) {
    gu[d][k] = (q[1].u[k] - q[0].u[k]) / g.dx[d];
    for (int a = 0; a < 2; ++a) {
      int l = t[a];
      const Prim<T>& Lp = q[2 + 2 * a]; const Prim<T>& Lm = q[3 + 2 * a];
      const Prim<T>& Rp = q[6 + 2 * a]; const Prim<T>& Rm = q[7 + 2 * a];
      gu[l][k] = ((Lp.u[k] - Lm.u[k]) + (Rp.u[k] - Rm.u[k])) / (4.0 * g.dx[l]);
    }
  }
  T de = (q[1].e - q[0].e) / g.dx[d];
  T div = gu[0][0] + gu[1][1] + gu[2][2];
  T sig[3];
  for (int k = 0; k < 3; ++k) {
    sig[k] = g.mu * (gu[d][k] + gu[k][d]);
    if (k == d) sig[k] = sig[k] - (2.0 * g.mu / 3.0) * div;
  }
  T work = 0.0;
  for (int k = 0; k < 3; ++k) work = work + 0.5 * (q[0].u[k] + q[1].u[k]) * sig[k];
  H[0] = Fc[0];
  for (int k = 0; k < 3; ++k) H[1 + k] = Fc[1 + k] - sig[k];
  H[4] = Fc[4] - (work + g.alpha * de);
}

// Face ranges: in x with walls the faces run from the wall face (ghost -1 | 0) to (nx-1 | ghost nx).
void face_range(const G& g, int d, long& i0, long& i1) {
  if (d == 0 && g.wall) { i0 = -1; i1 = g.nx; } else { i0 = 0; i1 = g.n(d); }
}

int nthreads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
int thread_id() {
#ifdef _OPENMP
  return omp_get_thread_num();
#else
  return 0;
#endif
}

// Runs body(d, i, j, k, acc) over every face, in parallel over the outermost face index, with a
// private accumulator per thread; the accumulators are added into `out` in thread order.
template <class T, class Body>
void face_scatter(const G& g, long out_len, T* out, Body body) {
  int nt = nthreads();
  std::vector<std::vector<T>> acc(nt, std::vector<T>(out_len, T(0.0)));
  for (int d = 0; d < 3; ++d) {
    long i0, i1; face_range(g, d, i0, i1);
    // faces of direction d are indexed by the L cell (i,j,k); i in [i0, i1) along x
    long ilen = (d == 0) ? (i1 - i0) : g.nx;
    long jlen = (d == 1) ? g.ny : g.ny;
    long nfaces = ilen * jlen * g.nz;
#pragma omp parallel for schedule(static)
    for (long f = 0; f < nfaces; ++f) {
      long ii = f % ilen, rest = f / ilen;
      long j = rest % jlen, k = rest / jlen;
      long i = (d == 0) ? ii + i0 : ii;
      body(d, i, j, k, acc[thread_id()].data());
    }
  }
  for (int t = 0; t < nt; ++t)
    for (long x = 0; x < out_len; ++x) out[x] += acc[t][x];
}

// ------------------------------------------------------------------------------------------
// Residual R(w; s)
// ------------------------------------------------------------------------------------------
template <class T>
void residual(const G& g, const T* w, const T* s, T* R) {
  for (long x = 0; x < 5 * g.N; ++x) R[x] = T(0.0);
  face_scatter<T>(g, 5 * g.N, R, [&](int d, long i, long j, long k, T* acc) {
    Slot sl[NSLOT]; face_slots(g, d, i, j, k, sl);
    T st[NSLOT][5];
    for (int a = 0; a < nslots(g); ++a) load_slot(g, w, sl[a], st[a]);
    T H[5]; face_flux(g, d, st, H, open_side(g, d, i), recon_ok(g, sl[10]), recon_ok(g, sl[11]));
    for (int v = 0; v < 5; ++v) {
      if (sl[0].real) acc[v * g.N + sl[0].c] -= H[v] / g.dx[d];
      if (sl[1].real) acc[v * g.N + sl[1].c] += H[v] / g.dx[d];
    }
  });
  if (s)
    for (long x = 0; x < 5 * g.N; ++x) R[x] += s[x];
}

// out = J_R(W)^T kh : for every face, the local Jacobian dH/d(stencil) (5 x 5NS, NS slots) from
// dual numbers, contracted with the adjoint weights (kh_R - kh_L)/dx_d and scattered to the
// stencil cells.
template <int NS>
void vjp_slots(const G& g, const double* W, const double* kh, double* out) {
  constexpr int ND = 5 * NS;
  for (long x = 0; x < 5 * g.N; ++x) out[x] = 0.0;
  face_scatter<double>(g, 5 * g.N, out, [&](int d, long i, long j, long k, double* acc) {
    Slot sl[NSLOT]; face_slots(g, d, i, j, k, sl);
    Dual<ND> st[NSLOT][5];
    for (int a = 0; a < NS; ++a)
      for (int v = 0; v < 5; ++v) {
        double sg = mirror_sign(sl[a].mirror, v);
        st[a][v] = Dual<ND>(sg * W[v * g.N + sl[a].c]);
        st[a][v].d[a * 5 + v] = sg;
      }
    Dual<ND> H[5]; face_flux(g, d, st, H, open_side(g, d, i), recon_ok(g, sl[10]), recon_ok(g, sl[11]));
    double om[5];
    for (int o = 0; o < 5; ++o) {
      double r = sl[1].real ? kh[o * g.N + sl[1].c] : 0.0;
      double l = sl[0].real ? kh[o * g.N + sl[0].c] : 0.0;
      om[o] = (r - l) / g.dx[d];
    }
    for (int a = 0; a < NS; ++a)
      for (int v = 0; v < 5; ++v) {
        double sum = 0.0;
        for (int o = 0; o < 5; ++o) sum += om[o] * H[o].d[a * 5 + v];
        acc[v * g.N + sl[a].c] += sum;
      }
  });
}

void vjp(const G& g, const double* W, const double* kh, double* out) {
  if (nslots(g) == 12)
    vjp_slots<12>(g, W, kh, out);
  else
    vjp_slots<10>(g, W, kh, out);
}

// out = J_R(W) v  (tangent), by evaluating the residual on single-direction dual numbers.
void jvp(const G& g, const double* W, const double* v, double* out) {
  std::vector<Dual<1>> wd(5 * g.N), Rd(5 * g.N);
  for (long x = 0; x < 5 * g.N; ++x) { wd[x] = Dual<1>(W[x]); wd[x].d[0] = v[x]; }
  residual<Dual<1>>(g, wd.data(), nullptr, Rd.data());
  for (long x = 0; x < 5 * g.N; ++x) out[x] = Rd[x].d[0];
}

// ------------------------------------------------------------------------------------------
// Artificial adjoint viscosity  (L_nu q)_i = sum_d [nu_{i+1/2}(q_{i+1}-q_i) - nu_{i-1/2}(q_i-q_{i-1})]/dx_d^2
// with nu_f = (nu_L + nu_R)/2, applied to each of the 5 components (delta_ki delta_jl); component
// v uses the cell field nu[v].  Wall faces carry no artificial flux.  Accumulates into out.
// ------------------------------------------------------------------------------------------
void lnu_apply(const G& g, const double* const nu[5], const double* q, double* out) {
  face_scatter<double>(g, 5 * g.N, out, [&](int d, long i, long j, long k, double* acc) {
    Slot sl[NSLOT]; face_slots(g, d, i, j, k, sl);
    if (!sl[0].real || !sl[1].real) return;
    for (int v = 0; v < 5; ++v) {
      double nf = 0.5 * (nu[v][sl[0].c] + nu[v][sl[1].c]);
      double flux = nf * (q[v * g.N + sl[1].c] - q[v * g.N + sl[0].c]) / (g.dx[d] * g.dx[d]);
      acc[v * g.N + sl[0].c] += flux;
      acc[v * g.N + sl[1].c] -= flux;
    }
  });
}

// ------------------------------------------------------------------------------------------
// Growth matrix M = M1 - M2 and sigma_1   [Energy Analysis: M1, M2 as printed; sigma_1 = largest
// singular value of M].  a = sqrt((gamma-1)/gamma) c, b = c / sqrt(gamma).
// grads: grho[3], gu[3][3] with gu[k][j] = d_j u_k, gp[3], ga[3], gb[3].
// ------------------------------------------------------------------------------------------
void cell_growth_matrix(double gamma, double rho, double p, double a, double b, const double grho[3],
                        const double gu[3][3], const double gp[3], const double ga[3],
                        const double gb[3], double M[5][5]) {
  double div = gu[0][0] + gu[1][1] + gu[2][2];
  double M1[5][5] = {{0}}, M2[5][5] = {{0}};
  M1[0][0] = div;
  for (int j = 0; j < 3; ++j) {
    M1[0][1 + j] = gb[j]; M1[1 + j][0] = gb[j];
    M1[1 + j][1 + j] = div;
    M1[1 + j][4] = ga[j]; M1[4][1 + j] = ga[j];
  }
  M1[4][4] = div;
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) M1[r][c] *= 0.5;
  for (int j = 0; j < 3; ++j) M2[0][1 + j] = (b / rho) * grho[j];
  M2[0][4] = 0.5 * std::sqrt(gamma - 1.0) * div;
  for (int k = 0; k < 3; ++k) {
    for (int j = 0; j < 3; ++j) M2[1 + k][1 + j] = gu[k][j];
    M2[1 + k][4] = (a / (2.0 * p)) * gp[k];
  }
  for (int j = 0; j < 3; ++j) M2[4][1 + j] = (2.0 / (gamma - 1.0)) * ga[j];
  M2[4][4] = 0.5 * (gamma - 1.0) * div;
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) M[r][c] = M1[r][c] - M2[r][c];
}

// Largest eigenvalue of a symmetric 5x5 matrix by cyclic Jacobi rotations, iterated until the
// off-diagonal mass is below 1e-30 of the total (or 100 sweeps).
double sym_lambda_max(double A[5][5]) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int p = 0; p < 5; ++p)
      for (int q = 0; q < 5; ++q) {
        tot += A[p][q] * A[p][q];
        if (p != q) off += A[p][q] * A[p][q];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < 4; ++p)
      for (int q = p + 1; q < 5; ++q) {
        if (A[p][q] == 0.0) continue;
        double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < 5; ++r) {  // A <- A J
          double arp = A[r][p], arq = A[r][q];
          A[r][p] = c * arp - s * arq;
          A[r][q] = s * arp + c * arq;
        }
        for (int r = 0; r < 5; ++r) {  // A <- J^T A
          double apr = A[p][r], aqr = A[q][r];
          A[p][r] = c * apr - s * aqr;
          A[q][r] = s * apr + c * aqr;
        }
      }
  }
  double m = A[0][0];
  for (int i = 1; i < 5; ++i) m = std::max(m, A[i][i]);
  return m;
}

double sigma1_of(const double M[5][5]) {
  double A[5][5];
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) {
      double s = 0.0;
      for (int k = 0; k < 5; ++k) s += M[k][r] * M[k][c];
      A[r][c] = s;
    }
  return std::sqrt(std::max(sym_lambda_max(A), 0.0));
}

struct CellQ { double rho, u[3], p, a, b; };
CellQ cellq(const G& g, const double w[5]) {
  Prim<double> q = prim(g, w);
  CellQ c; c.rho = q.rho; for (int k = 0; k < 3; ++k) c.u[k] = q.u[k]; c.p = q.p;
  double cs = std::sqrt(g.gamma * q.p / q.rho);
  c.a = std::sqrt((g.gamma - 1.0) / g.gamma) * cs;
  c.b = cs / std::sqrt(g.gamma);
  return c;
}

// M at cell (i,j,k) with cell-centred central differences of rho, u, p, a, b.
void grid_growth_matrix(const G& g, const double* w, long i, long j, long k, double M[5][5]) {
  double wc[5]; load_slot(g, w, slot(g, i, j, k), wc);
  CellQ c = cellq(g, wc);
  double grho[3], gu[3][3], gp[3], ga[3], gb[3];
  for (int l = 0; l < 3; ++l) {
    long pp[3] = {i, j, k}, mm[3] = {i, j, k};
    pp[l] += 1; mm[l] -= 1;
    double wp[5], wm[5];
    load_slot(g, w, slot(g, pp[0], pp[1], pp[2]), wp);
    load_slot(g, w, slot(g, mm[0], mm[1], mm[2]), wm);
    CellQ P = cellq(g, wp), Mq = cellq(g, wm);
    double h = 2.0 * g.dx[l];
    grho[l] = (P.rho - Mq.rho) / h;
    for (int kk = 0; kk < 3; ++kk) gu[kk][l] = (P.u[kk] - Mq.u[kk]) / h;
    gp[l] = (P.p - Mq.p) / h;
    ga[l] = (P.a - Mq.a) / h;
    gb[l] = (P.b - Mq.b) / h;
  }
  cell_growth_matrix(g.gamma, c.rho, c.p, c.a, c.b, grho, gu, gp, ga, gb, M);
}

void sigma1_field(const G& g, const double* w, double* sig) {
#pragma omp parallel for schedule(static)
  for (long c = 0; c < g.N; ++c) {
    long i = c % g.nx, j = (c / g.nx) % g.ny, k = c / (g.nx * g.ny);
    double M[5][5];
    grid_growth_matrix(g, w, i, j, k, M);
    sig[c] = sigma1_of(M);
  }
}

// ------------------------------------------------------------------------------------------
// Objectives j(w) and dj/dw (dual numbers on each local contribution; serial fixed-order sums)
// ------------------------------------------------------------------------------------------
// Volume-mean viscous dissipation contribution of one cell from its 6 face neighbours
// (slots: 0 +x, 1 -x, 2 +y, 3 -y, 4 +z, 5 -z), Phi = sigma_ij d_j u_i with central gradients.
template <class T>
T dissipation_cell(const G& g, const T nb[6][5]) {
  T gu[3][3];  // gu[l][k] = d_l u_k
  for (int l = 0; l < 3; ++l) {
    Prim<T> P = prim(g, nb[2 * l]), Mq = prim(g, nb[2 * l + 1]);
    for (int k = 0; k < 3; ++k) gu[l][k] = (P.u[k] - Mq.u[k]) / (2.0 * g.dx[l]);
  }
  T div = gu[0][0] + gu[1][1] + gu[2][2];
  T phi = 0.0;
  for (int l = 0; l < 3; ++l)
    for (int k = 0; k < 3; ++k) {
      T sig = g.mu * (gu[l][k] + gu[k][l]);
      if (l == k) sig = sig - (2.0 * g.mu / 3.0) * div;
      phi = phi + sig * gu[l][k];
    }
  return phi;
}

// Stagnation pressure of the face state  p_t = p (1 + (gamma-1)/2 M^2)^(gamma/(gamma-1))   [Eq. (3)]
template <class T>
void plane_terms(const G& g, double pt_ref, const T wf[5], T& num, T& den) {
  Prim<T> q = prim(g, wf);
  T u2 = q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2];
  T c2 = g.gamma * q.p / q.rho;
  T pt = q.p * pow(1.0 + 0.5 * (g.gamma - 1.0) * u2 / c2, g.gamma / (g.gamma - 1.0));
  num = q.rho * (pt_ref - pt);
  den = q.rho;
}

int objective(const G& g, const orc_obj* ob, const double* w, double* jout, double* djdw) {
  const long N = g.N;
  if (djdw)
    for (long x = 0; x < 5 * N; ++x) djdw[x] = 0.0;
  if (ob->kind == 0) { *jout = 0.0; return 0; }
  if (ob->kind == 1) {  // j = (1/N) sum_c p_c
    std::vector<double> pc(N);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
      Dual<5> wd[5];
      for (int v = 0; v < 5; ++v) { wd[v] = Dual<5>(w[v * N + c]); wd[v].d[v] = 1.0; }
      Prim<Dual<5>> q = prim(g, wd);
      pc[c] = q.p.v;
      if (djdw)
        for (int v = 0; v < 5; ++v) djdw[v * N + c] = q.p.d[v] / (double)N;
    }
    double s = 0.0;
    for (long c = 0; c < N; ++c) s += pc[c];
    *jout = s / (double)N;
    return 0;
  }
  if (ob->kind == 2) {  // j = (1/N) sum_c Phi_c
    std::vector<double> phic(N);
    std::vector<double> contrib(djdw ? 30 * N : 0);
    std::vector<long> cells(djdw ? 6 * N : 0);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
      long i = c % g.nx, j = (c / g.nx) % g.ny, k = c / (g.nx * g.ny);
      Slot sl[6];
      for (int l = 0; l < 3; ++l) {
        long pp[3] = {i, j, k}, mm[3] = {i, j, k};
        pp[l] += 1; mm[l] -= 1;
        sl[2 * l] = slot(g, pp[0], pp[1], pp[2]);
        sl[2 * l + 1] = slot(g, mm[0], mm[1], mm[2]);
      }
      Dual<30> nb[6][5];
      for (int a = 0; a < 6; ++a)
        for (int v = 0; v < 5; ++v) {
          double sg = mirror_sign(sl[a].mirror, v);
          nb[a][v] = Dual<30>(sg * w[v * N + sl[a].c]);
          nb[a][v].d[a * 5 + v] = sg;
        }
      Dual<30> phi = dissipation_cell(g, nb);
      phic[c] = phi.v;
      if (djdw) {
        for (int a = 0; a < 30; ++a) contrib[30 * c + a] = phi.d[a] / (double)N;
        for (int a = 0; a < 6; ++a) cells[6 * c + a] = sl[a].c;
      }
    }
    double s = 0.0;
    for (long c = 0; c < N; ++c) s += phic[c];
    *jout = s / (double)N;
    if (djdw)
      for (long c = 0; c < N; ++c)
        for (int a = 0; a < 6; ++a)
          for (int v = 0; v < 5; ++v) djdw[v * N + cells[6 * c + a]] += contrib[30 * c + a * 5 + v];
    return 0;
  }
  if (ob->kind == 3) {  // j = sum rho_f (pt_ref - pt_f) / (pt_ref sum rho_f), face state = mean of L, R
    if (ob->plane_i < 1 || ob->plane_i >= g.nx) return -1;
    long il = ob->plane_i - 1, ir = ob->plane_i;
    double num = 0.0, den = 0.0;
    std::vector<double> dnum(djdw ? 10 * g.ny * g.nz : 0), dden(djdw ? 10 * g.ny * g.nz : 0);
    for (long k = 0; k < g.nz; ++k)
      for (long j = 0; j < g.ny; ++j) {
        long cl = g.idx(il, j, k), cr = g.idx(ir, j, k);
        Dual<10> wf[5];
        for (int v = 0; v < 5; ++v) {
          wf[v] = Dual<10>(0.5 * (w[v * N + cl] + w[v * N + cr]));
          wf[v].d[v] = 0.5; wf[v].d[5 + v] = 0.5;
        }
        Dual<10> nm, dn;
        plane_terms(g, ob->pt_ref, wf, nm, dn);
        num += nm.v; den += dn.v;
        if (djdw) {
          long f = k * g.ny + j;
          for (int a = 0; a < 10; ++a) { dnum[10 * f + a] = nm.d[a]; dden[10 * f + a] = dn.d[a]; }
        }
      }
    double jv = num / (den * ob->pt_ref);
    *jout = jv;
    if (djdw)
      for (long k = 0; k < g.nz; ++k)
        for (long j = 0; j < g.ny; ++j) {
          long f = k * g.ny + j;
          long cl = g.idx(il, j, k), cr = g.idx(ir, j, k);
          for (int v = 0; v < 5; ++v) {
            // quotient rule: d(num/(den pt))/dx = (dnum - (num/den) dden) / (den pt)
            double gl = (dnum[10 * f + v] - (num / den) * dden[10 * f + v]) / (den * ob->pt_ref);
            double gr = (dnum[10 * f + 5 + v] - (num / den) * dden[10 * f + 5 + v]) / (den * ob->pt_ref);
            djdw[v * N + cl] += gl;
            djdw[v * N + cr] += gr;
          }
        }
    return 0;
  }
  return -1;
}

// ------------------------------------------------------------------------------------------
// RK4 stages
// ------------------------------------------------------------------------------------------
template <class T>
void rk4_step(const G& g, const T* w, const T* s, T* wn) {
  const long M = 5 * g.N;
  std::vector<T> k1(M), k2(M), k3(M), k4(M), W(M);
  residual<T>(g, w, s, k1.data());
  for (long x = 0; x < M; ++x) W[x] = w[x] + (0.5 * g.dt) * k1[x];
  residual<T>(g, W.data(), s, k2.data());
  for (long x = 0; x < M; ++x) W[x] = w[x] + (0.5 * g.dt) * k2[x];
  residual<T>(g, W.data(), s, k3.data());
  for (long x = 0; x < M; ++x) W[x] = w[x] + g.dt * k3[x];
  residual<T>(g, W.data(), s, k4.data());
  for (long x = 0; x < M; ++x)
    wn[x] = w[x] + (g.dt / 6.0) * (k1[x] + 2.0 * k2[x] + 2.0 * k3[x] + k4[x]);
}

// Strong-stability-preserving third-order Runge-Kutta step in Shu-Osher form [Numerical methods]:
//   u1 = w + dt R(w);  u2 = 3/4 w + 1/4 (u1 + dt R(u1));  w_next = 1/3 w + 2/3 (u2 + dt R(u2)).
template <class T>
void ssprk3_step(const G& g, const T* w, const T* s, T* wn) {
  const long M = 5 * g.N;
  std::vector<T> k(M), u1(M), u2(M);
  residual<T>(g, w, s, k.data());
  for (long x = 0; x < M; ++x) u1[x] = w[x] + g.dt * k[x];
  residual<T>(g, u1.data(), s, k.data());
  for (long x = 0; x < M; ++x) u2[x] = 0.75 * w[x] + 0.25 * (u1[x] + g.dt * k[x]);
  residual<T>(g, u2.data(), s, k.data());
  for (long x = 0; x < M; ++x) wn[x] = (1.0 / 3.0) * w[x] + (2.0 / 3.0) * (u2[x] + g.dt * k[x]);
}

// One step of the grid's time scheme.
template <class T>
void time_step(const G& g, const T* w, const T* s, T* wn) {
  if (g.scheme == 1)
    ssprk3_step<T>(g, w, s, wn);
  else
    rk4_step<T>(g, w, s, wn);
}

// The SSP-RK3 stage states u0 = w, u1, u2 of one step.
void ssprk3_stage_states(const G& g, const double* w, const double* s, std::vector<double> U[3]) {
  const long M = 5 * g.N;
  std::vector<double> k(M);
  U[0].assign(w, w + M);
  residual<double>(g, w, s, k.data());
  U[1].resize(M);
  for (long x = 0; x < M; ++x) U[1][x] = w[x] + g.dt * k[x];
  residual<double>(g, U[1].data(), s, k.data());
  U[2].resize(M);
  for (long x = 0; x < M; ++x) U[2][x] = 0.75 * w[x] + 0.25 * (U[1][x] + g.dt * k[x]);
}

// The four RK4 stage states W1 = w, W2, W3, W4 of one step.
void rk4_stage_states(const G& g, const double* w, const double* s, std::vector<double> Ws[4]) {
  const long M = 5 * g.N;
  std::vector<double> k(M);
  Ws[0].assign(w, w + M);
  const double c[3] = {0.5 * g.dt, 0.5 * g.dt, g.dt};
  for (int m = 0; m < 3; ++m) {
    residual<double>(g, Ws[m].data(), s, k.data());
    Ws[m + 1].resize(M);
    for (long x = 0; x < M; ++x) Ws[m + 1][x] = w[x] + c[m] * k[x];
  }
}

}  // namespace

// ==========================================================================================
// C entry points (ctypes).  All arrays are host FP64 SoA; return 0 on success, -1 on bad input.
// ==========================================================================================
extern "C" {

int orc_num_threads(void) { return nthreads(); }

// OpenMP threads of the following calls (timing on one core or all of them)
int orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#endif
  return nthreads();
}

static int check(const orc_grid* g) {
  if (!g) return -1;
  for (int d = 0; d < 3; ++d)
    if (g->n[d] < 1 || !(g->L[d] > 0)) return -1;
  if (g->bc_x < 0 || g->bc_x > 2) return -1;
  if (g->bc_x != 0 && g->n[0] < 2) return -1;
  if (g->bc_x == 2 && !(g->w_far[0][0] > 0.0 && g->w_far[1][0] > 0.0)) return -1;
  if (g->scheme != 0 && g->scheme != 1) return -1;
  if (g->flux != 0 && g->flux != 1) return -1;
  if (g->flux == 1 && !(g->roe_delta > 0.0)) return -1;
  return 0;
}

// F = flux through the characteristic boundary face of `side` (0: x = 0, 1: x = L_x) next to the
// boundary cell state w
int orc_char_flux(const orc_grid* gr, int side, const double* w, double* F) {
  if (check(gr) || gr->bc_x != 2 || side < 0 || side > 1) return -1;
  G g(gr);
  double st[2][5];
  for (int v = 0; v < 5; ++v) st[0][v] = st[1][v] = w[v];
  char_face_flux<double>(g, side, st, F);
  return 0;
}

// F = Roe flux between the face states wl and wr in direction d (no reconstruction)
int orc_roe_flux(const orc_grid* gr, int d, const double* wl, const double* wr, double* F) {
  if (check(gr) || d < 0 || d > 2) return -1;
  G g(gr);
  roe_face_flux<double>(g, d, wl, wr, F);
  return 0;
}

// R = R(w; s)
int orc_residual(const orc_grid* gr, const double* w, const double* s, double* R) {
  if (check(gr)) return -1;
  G g(gr);
  residual<double>(g, w, s, R);
  return 0;
}

// out = J_R(W) v
int orc_jvp(const orc_grid* gr, const double* W, const double* v, double* out) {
  if (check(gr)) return -1;
  G g(gr);
  jvp(g, W, v, out);
  return 0;
}

// out = J_R(W)^T kh
int orc_vjp(const orc_grid* gr, const double* W, const double* kh, double* out) {
  if (check(gr)) return -1;
  G g(gr);
  vjp(g, W, kh, out);
  return 0;
}

// out += L_nu q
int orc_lnu_apply(const orc_grid* gr, const double* nu, const double* q, double* out) {
  if (check(gr)) return -1;
  G g(gr);
  const double* const nus[5] = {nu, nu, nu, nu, nu};
  lnu_apply(g, nus, q, out);
  return 0;
}

// w_next = one step (RK4 or SSP-RK3) of w with source s (s may be NULL)
int orc_primal_step(const orc_grid* gr, const double* w, const double* s, double* wn) {
  if (check(gr)) return -1;
  G g(gr);
  time_step<double>(g, w, s, wn);
  return 0;
}

// Complex-step primal: the state and source carry imaginary parts (re, im arrays).
int orc_primal_step_complex(const orc_grid* gr, const double* w_re, const double* w_im,
                            const double* s_re, const double* s_im, double* out_re, double* out_im) {
  if (check(gr)) return -1;
  G g(gr);
  const long M = 5 * g.N;
  std::vector<std::complex<double>> w(M), s(M), wn(M);
  for (long x = 0; x < M; ++x) {
    w[x] = {w_re[x], w_im ? w_im[x] : 0.0};
    s[x] = {s_re ? s_re[x] : 0.0, s_im ? s_im[x] : 0.0};
  }
  time_step<std::complex<double>>(g, w.data(), s.data(), wn.data());
  for (long x = 0; x < M; ++x) { out_re[x] = wn[x].real(); out_im[x] = wn[x].imag(); }
  return 0;
}

// Cell fields nu_g = lambda_g sigma_1(w) of the three variable groups (rho), (rho u), (rho E) and
// the field each component uses.
struct NuFields {
  std::vector<double> f[3];
  const double* comp[5];
  bool any = false;
  NuFields(const G& g, const double* w, const double lam[3]) {
    any = lam[0] != 0.0 || lam[1] != 0.0 || lam[2] != 0.0;
    if (!any) return;
    std::vector<double> sig(g.N);
    sigma1_field(g, w, sig.data());
    for (int k = 0; k < 3; ++k) {
      f[k].resize(g.N);
      for (long c = 0; c < g.N; ++c) f[k][c] = lam[k] * sig[c];
    }
    const int group[5] = {0, 1, 1, 1, 2};
    for (int v = 0; v < 5; ++v) comp[v] = f[group[v]].data();
  }
};

// out += L_nu q with the group fields nu_g = lambda_g sigma_1(w) (lambda: 3 values)
int orc_lnu_apply_groups(const orc_grid* gr, const double* w, const double* lambda, const double* q,
                         double* out) {
  if (check(gr)) return -1;
  G g(gr);
  const NuFields nu(g, w, lambda);
  if (nu.any) lnu_apply(g, nu.comp, q, out);
  return 0;
}

// Tangent-linear RK4 step: (w, dw) -> (w_next, dw_next) for perturbations dw of the state and ds
// of the source.  With lambda > 0 the tangent of every stage also carries L_nu dW with
// nu_g = lambda_g sigma_1(w) frozen over the step (the operator whose transpose the stabilised
// adjoint applies); lambda holds one value per variable group (rho, rho u, rho E).
int orc_tlm_step(const orc_grid* gr, const double* w, const double* s, const double* dw,
                 const double* ds, const double* lambda, double* wn, double* dwn) {
  if (check(gr)) return -1;
  G g(gr);
  const long M = 5 * g.N;
  const NuFields nu(g, w, lambda);
  // tangent of one stage: (J_R(W) + L_nu) dW + ds
  auto stage_tangent = [&](const std::vector<double>& W, const std::vector<double>& dW, std::vector<double>& dk) {
    dk.assign(M, 0.0);
    jvp(g, W.data(), dW.data(), dk.data());
    if (nu.any) lnu_apply(g, nu.comp, dW.data(), dk.data());
    if (ds)
      for (long x = 0; x < M; ++x) dk[x] += ds[x];
  };
  if (g.scheme == 1) {
    // SSP-RK3, the Shu-Osher stages differentiated one by one
    std::vector<double> U[3], du1(M), du2(M), dk;
    ssprk3_stage_states(g, w, s, U);
    stage_tangent(U[0], std::vector<double>(dw, dw + M), dk);
    for (long x = 0; x < M; ++x) du1[x] = dw[x] + g.dt * dk[x];
    stage_tangent(U[1], du1, dk);
    for (long x = 0; x < M; ++x) du2[x] = 0.75 * dw[x] + 0.25 * (du1[x] + g.dt * dk[x]);
    stage_tangent(U[2], du2, dk);
    for (long x = 0; x < M; ++x) dwn[x] = (1.0 / 3.0) * dw[x] + (2.0 / 3.0) * (du2[x] + g.dt * dk[x]);
    if (wn) ssprk3_step<double>(g, w, s, wn);
    return 0;
  }
  std::vector<double> Ws[4];
  rk4_stage_states(g, w, s, Ws);
  std::vector<double> dW(dw, dw + M), dk[4];
  const double c[3] = {0.5 * g.dt, 0.5 * g.dt, g.dt};
  for (int m = 0; m < 4; ++m) {
    dk[m].assign(M, 0.0);
    jvp(g, Ws[m].data(), dW.data(), dk[m].data());
    if (nu.any) lnu_apply(g, nu.comp, dW.data(), dk[m].data());
    if (ds)
      for (long x = 0; x < M; ++x) dk[m][x] += ds[x];
    if (m < 3)
      for (long x = 0; x < M; ++x) dW[x] = dw[x] + c[m] * dk[m][x];
  }
  for (long x = 0; x < M; ++x)
    dwn[x] = dw[x] + (g.dt / 6.0) * (dk[0][x] + 2.0 * dk[1][x] + 2.0 * dk[2][x] + dk[3][x]);
  if (wn) rk4_step<double>(g, w, s, wn);
  return 0;
}

// One reverse RK4 step of the discrete adjoint   [Implementation; adjoint terminal condition and
// backward integration; stabilised adjoint equation]:
//   recompute W1..W4 from w_n;  nu_g = lambda_g sigma_1(w_n) per variable group
//   k^4 = dt/6 a;           g4 = (J(W4)^T + L_nu) k^4
//   k^3 = dt/3 a + dt g4;   g3 = (J(W3)^T + L_nu) k^3
//   k^2 = dt/3 a + dt/2 g3; g2 = (J(W2)^T + L_nu) k^2
//   k^1 = dt/6 a + dt/2 g2; g1 = (J(W1)^T + L_nu) k^1
//   w^_n = a + g1 + g2 + g3 + g4 + c_n dj/dw(w_n);   grad_s += k^1 + k^2 + k^3 + k^4
// where a = w^_{n+1}.  grad_s may be NULL; obj may be NULL (no injection).
int orc_adjoint_step(const orc_grid* gr, const double* w, const double* s, const double* a,
                     const double* lambda, const orc_obj* ob, double c_n, double* wh, double* grad_s) {
  if (check(gr)) return -1;
  G g(gr);
  const long M = 5 * g.N;
  const NuFields nu(g, w, lambda);
  const double dt = g.dt;
  std::vector<double> dj(M, 0.0);
  if (ob && ob->kind != 0 && c_n != 0.0) {
    double jv;
    if (objective(g, ob, w, &jv, dj.data())) return -1;
  }
  if (g.scheme == 1) {
    // SSP-RK3 reversed stage by stage: each stage u_i = sum_k alpha_ik u_k + beta_i dt R(u_{i-1})
    // hands u^_i to its inputs: alpha_ik u^_i to u_k and beta_i dt (J_R(u_{i-1})^T + L_nu) u^_i
    // to u_{i-1}, and beta_i dt u^_i to s^
    std::vector<double> U[3], r(M), u0(M, 0.0), u1(M, 0.0), u2(M, 0.0), sh(M, 0.0);
    ssprk3_stage_states(g, w, s, U);
    auto stage_adjoint = [&](const std::vector<double>& W, const double* q, std::vector<double>& out) {
      vjp(g, W.data(), q, out.data());
      if (nu.any) lnu_apply(g, nu.comp, q, out.data());
    };
    // w_next = 1/3 u0 + 2/3 u2 + 2/3 dt R(u2)
    stage_adjoint(U[2], a, r);
    for (long x = 0; x < M; ++x) {
      u2[x] = (2.0 / 3.0) * a[x] + (2.0 / 3.0) * dt * r[x];
      u0[x] = (1.0 / 3.0) * a[x];
      sh[x] = (2.0 / 3.0) * dt * a[x];
    }
    // u2 = 3/4 u0 + 1/4 u1 + 1/4 dt R(u1)
    stage_adjoint(U[1], u2.data(), r);
    for (long x = 0; x < M; ++x) {
      u1[x] = 0.25 * u2[x] + 0.25 * dt * r[x];
      u0[x] += 0.75 * u2[x];
      sh[x] += 0.25 * dt * u2[x];
    }
    // u1 = u0 + dt R(u0)
    stage_adjoint(U[0], u1.data(), r);
    for (long x = 0; x < M; ++x) {
      u0[x] += u1[x] + dt * r[x];
      sh[x] += dt * u1[x];
    }
    for (long x = 0; x < M; ++x) wh[x] = u0[x] + c_n * dj[x];
    if (grad_s)
      for (long x = 0; x < M; ++x) grad_s[x] += sh[x];
    return 0;
  }
  std::vector<double> Ws[4];
  rk4_stage_states(g, w, s, Ws);
  const double ca[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};  // weight of a in k^m, m = 1..4
  const double cg[4] = {dt / 2.0, dt / 2.0, dt, 0.0};             // weight of g_{m+1} in k^m
  std::vector<double> gnext(M, 0.0), gm(M), kh(M), sum_g(M, 0.0), sum_k(M, 0.0);
  for (int m = 3; m >= 0; --m) {
    for (long x = 0; x < M; ++x) kh[x] = ca[m] * a[x] + cg[m] * gnext[x];
    vjp(g, Ws[m].data(), kh.data(), gm.data());
    if (nu.any) lnu_apply(g, nu.comp, kh.data(), gm.data());
    for (long x = 0; x < M; ++x) { sum_g[x] += gm[x]; sum_k[x] += kh[x]; }
    gnext = gm;
  }
  for (long x = 0; x < M; ++x) wh[x] = a[x] + sum_g[x] + c_n * dj[x];
  if (grad_s)
    for (long x = 0; x < M; ++x) grad_s[x] += sum_k[x];
  return 0;
}

// Objective value and (optionally) gradient dj/dw (overwritten).
int orc_objective(const orc_grid* gr, const orc_obj* ob, const double* w, double* j, double* djdw) {
  if (check(gr) || !ob) return -1;
  G g(gr);
  return objective(g, ob, w, j, djdw);
}

// sigma_1 per cell
int orc_sigma1(const orc_grid* gr, const double* w, double* sig) {
  if (check(gr)) return -1;
  G g(gr);
  sigma1_field(g, w, sig);
  return 0;
}

// Growth matrix at every cell, row-major 25 values per cell (for tests).
int orc_growth_matrix_field(const orc_grid* gr, const double* w, double* Mout) {
  if (check(gr)) return -1;
  G g(gr);
  for (long c = 0; c < g.N; ++c) {
    long i = c % g.nx, j = (c / g.nx) % g.ny, k = c / (g.nx * g.ny);
    double M[5][5];
    grid_growth_matrix(g, w, i, j, k, M);
    for (int r = 0; r < 5; ++r)
      for (int q = 0; q < 5; ++q) Mout[25 * c + 5 * r + q] = M[r][q];
  }
  return 0;
}

// Pointwise growth matrix from given gradients: grads = [grho(3), gu(9, gu[k][j] = d_j u_k),
// gp(3), ga(3), gb(3)]; a and b derive from (gamma, rho, p).
int orc_cell_growth_matrix(double gamma, double rho, double p, const double* grads, double* Mout) {
  double cs = std::sqrt(gamma * p / rho);
  double a = std::sqrt((gamma - 1.0) / gamma) * cs, b = cs / std::sqrt(gamma);
  double gu[3][3];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) gu[k][j] = grads[3 + 3 * k + j];
  double M[5][5];
  cell_growth_matrix(gamma, rho, p, a, b, grads, gu, grads + 12, grads + 15, grads + 18, M);
  for (int r = 0; r < 5; ++r)
    for (int q = 0; q < 5; ++q) Mout[5 * r + q] = M[r][q];
  return 0;
}

// Largest singular value of a single 5x5 matrix (row-major), for tests.
double orc_matrix_sigma1(const double* Min) {
  double M[5][5];
  for (int r = 0; r < 5; ++r)
    for (int q = 0; q < 5; ++q) M[r][q] = Min[5 * r + q];
  return sigma1_of(M);
}

// Symmetrised adjoint v^ = T^{-T} w^ per cell (closed form, out: 5N) and the adjoint energy
// E = (1/dV) sum_cells |v^|^2  [Symmetrization: w^ = T^T v^; Energy Analysis: E_v^].
//   q^ = V^{-T} w^: q^_rho = w^_1 + u.w^_m + |u|^2/2 w^_E, q^_u = rho w^_m + rho u w^_E,
//                   q^_p = w^_E/(gamma-1)
//   v^ = S^{-T} q^: v^_1 = (rho/b) q^_rho + rho b q^_p, v^_{2..4} = q^_u, v^_5 = rho a q^_p
int orc_energy_vhat(const orc_grid* gr, const double* w, const double* wh, double* vhat, double* E) {
  if (check(gr)) return -1;
  G g(gr);
  const long N = g.N;
  std::vector<double> e2(N);
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    double wc[5], h[5];
    for (int v = 0; v < 5; ++v) { wc[v] = w[v * N + c]; h[v] = wh[v * N + c]; }
    CellQ q = cellq(g, wc);
    double u2 = q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2];
    double qr = h[0] + q.u[0] * h[1] + q.u[1] * h[2] + q.u[2] * h[3] + 0.5 * u2 * h[4];
    double qu[3];
    for (int k = 0; k < 3; ++k) qu[k] = q.rho * h[1 + k] + q.rho * q.u[k] * h[4];
    double qp = h[4] / (g.gamma - 1.0);
    double vv[5] = {(q.rho / q.b) * qr + q.rho * q.b * qp, qu[0], qu[1], qu[2], q.rho * q.a * qp};
    double s = 0.0;
    for (int v = 0; v < 5; ++v) { s += vv[v] * vv[v]; if (vhat) vhat[v * N + c] = vv[v]; }
    e2[c] = s;
  }
  double tot = 0.0;
  for (long c = 0; c < N; ++c) tot += e2[c];
  if (E) *E = tot / (g.dx[0] * g.dx[1] * g.dx[2]);
  return 0;
}

// ------------------------------------------------------------------------------------------
// BF16 checkpoint codec, block-scaled with a plane predictor (the precision form of the method:
// primal snapshots kept in BF16 under per-variable scaling; the paper's own snapshots are full
// precision, "Implementation").  The grid is cut into 4 x 4 x 4 blocks of cells (ragged at the
// far ends); block b = (bz * nby + by) * nbx + bx.  Per block and variable, over its present
// cells with centred local coordinates c_d = l_d - (n'_d - 1)/2:
//   (a, g) = least-squares plane of the values: a = S_0 / n', g_d = S_d / sum c_d^2 (0 if n'_d = 1)
//            with S_0 = sum w, S_d = sum c_d w in FP64, each rounded to FP32;
//   P(a) = fma(g_z, c_z, fma(g_y, c_y, fma(g_x, c_x, a))) in FP32; r0 = w - P(a);
//   a' = a + (max r0 + min r0)/2, s = (max r0 - min r0)/2 (1 if the range is 0);
//   q = bf16_round_nearest_even((w - P(a')) / s),   decode w' = fma(s, q, P(a'));
//   or, with 16-bit fixed-point codes, q = i16 of (w - P(a')) / s (below), same decode form.
// header[(b * 5 + v) * 5 + {0..4}] = a', g_x, g_y, g_z, s.  Codes keep the state layout.
// The FP64 sums run in one fixed order (so that two implementations round alike): per (x, y)
// column the cells z = 0..3 accumulate by fma (c w is exact in FP64), then columns add pairwise
// along x ((x0 + x1) + (x2 + x3)) and the rows likewise along y.
// ------------------------------------------------------------------------------------------
static uint16_t f32_to_bf16_rne(float f) {
  uint32_t u; std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
static float bf16_to_f32(uint16_t h) { uint32_t u = (uint32_t)h << 16; float f; std::memcpy(&f, &u, 4); return f; }

// The fixed-point alternative of the same size: code = the int16 nearest to t * 32767 (ties to
// even, the product rounded to FP32), clamped to +-32767; its value is code * h with
// h = 1/32767 rounded to FP32 (the product rounded to FP32).
static uint16_t f32_to_i16(float t) {
  float k = std::nearbyint(t * 32767.0f);
  if (k > 32767.0f) k = 32767.0f;
  if (k < -32767.0f) k = -32767.0f;
  return (uint16_t)(int16_t)k;
}
static float i16_to_f32(uint16_t q) { return (float)(int16_t)q * (1.0f / 32767.0f); }

static void codec_blocks(const orc_grid* g, long& nbx, long& nby, long& nbz) {
  nbx = (g->n[0] + 3) / 4; nby = (g->n[1] + 3) / 4; nbz = (g->n[2] + 3) / 4;
}

long orc_ckpt_blocks(const orc_grid* g) {
  long a, b, c; codec_blocks(g, a, b, c);
  return a * b * c;
}

static double side_sq(long m) { double s = 0.0; for (long l = 0; l < m; ++l) s += (l - 0.5 * (m - 1)) * (l - 0.5 * (m - 1)); return s; }
static float centred(long l, long m) { return (float)l - 0.5f * (float)(m - 1); }
static float plane_at(const float* h, float cx, float cy, float cz) {
  return std::fma(h[3], cz, std::fma(h[2], cy, std::fma(h[1], cx, h[0])));
}

int orc_ckpt_encode(const orc_grid* g, const float* w, uint16_t* q, float* header, int i16) {
  const long nx = g->n[0], ny = g->n[1], nz = g->n[2], N = nx * ny * nz;
  long nbx, nby, nbz; codec_blocks(g, nbx, nby, nbz);
  for (long bz = 0; bz < nbz; ++bz)
    for (long by = 0; by < nby; ++by)
      for (long bx = 0; bx < nbx; ++bx) {
        const long b = (bz * nby + by) * nbx + bx;
        const long mx = std::min(4L, nx - 4 * bx), my = std::min(4L, ny - 4 * by), mz = std::min(4L, nz - 4 * bz);
        for (int v = 0; v < 5; ++v) {
          const float* wv = w + v * N;
          auto at = [&](long i, long j, long k) { return wv[((4 * bz + k) * ny + 4 * by + j) * nx + 4 * bx + i]; };
          // column sums (S_0, S_x, S_y, S_z) at (i, j), then the pairwise x and y order
          double col[4][4][4] = {};
          for (long j = 0; j < my; ++j)
            for (long i = 0; i < mx; ++i)
              for (long k = 0; k < mz; ++k) {
                const double x = at(i, j, k);
                const double c[4] = {1.0, centred(i, mx), centred(j, my), centred(k, mz)};
                for (int t = 0; t < 4; ++t) col[j][i][t] = std::fma(c[t], x, col[j][i][t]);
              }
          double S[4];
          for (int t = 0; t < 4; ++t) {
            double row[4];
            for (int j = 0; j < 4; ++j) row[j] = (col[j][0][t] + col[j][1][t]) + (col[j][2][t] + col[j][3][t]);
            S[t] = (row[0] + row[1]) + (row[2] + row[3]);
          }
          const double dx2 = (double)(my * mz) * side_sq(mx), dy2 = (double)(mx * mz) * side_sq(my),
                       dz2 = (double)(mx * my) * side_sq(mz);
          float h[5];
          h[0] = (float)(S[0] / (double)(mx * my * mz));
          h[1] = dx2 > 0.0 ? (float)(S[1] / dx2) : 0.0f;
          h[2] = dy2 > 0.0 ? (float)(S[2] / dy2) : 0.0f;
          h[3] = dz2 > 0.0 ? (float)(S[3] / dz2) : 0.0f;
          float rmn = INFINITY, rmx = -INFINITY;
          for (long k = 0; k < mz; ++k)
            for (long j = 0; j < my; ++j)
              for (long i = 0; i < mx; ++i) {
                const float r = at(i, j, k) - plane_at(h, centred(i, mx), centred(j, my), centred(k, mz));
                rmn = std::min(rmn, r); rmx = std::max(rmx, r);
              }
          h[0] = h[0] + 0.5f * (rmx + rmn);
          float s = 0.5f * (rmx - rmn);
          if (!(s > 0.0f)) s = 1.0f;
          h[4] = s;
          for (int t = 0; t < 5; ++t) header[(b * 5 + v) * 5 + t] = h[t];
          for (long k = 0; k < mz; ++k)
            for (long j = 0; j < my; ++j)
              for (long i = 0; i < mx; ++i) {
                const long c = v * N + ((4 * bz + k) * ny + 4 * by + j) * nx + 4 * bx + i;
                const float t = (w[c] - plane_at(h, centred(i, mx), centred(j, my), centred(k, mz))) / s;
                q[c] = i16 ? f32_to_i16(t) : f32_to_bf16_rne(t);
              }
        }
      }
  return 0;
}

int orc_ckpt_decode(const orc_grid* g, const uint16_t* q, const float* header, float* w, int i16) {
  const long nx = g->n[0], ny = g->n[1], nz = g->n[2], N = nx * ny * nz;
  long nbx, nby, nbz; codec_blocks(g, nbx, nby, nbz);
  for (int v = 0; v < 5; ++v)
    for (long k = 0; k < nz; ++k)
      for (long j = 0; j < ny; ++j)
        for (long i = 0; i < nx; ++i) {
          const long b = ((k / 4) * nby + j / 4) * nbx + i / 4, c = v * N + (k * ny + j) * nx + i;
          const long mx = std::min(4L, nx - 4 * (i / 4)), my = std::min(4L, ny - 4 * (j / 4)),
                     mz = std::min(4L, nz - 4 * (k / 4));
          const float* h = header + (b * 5 + v) * 5;
          w[c] = std::fma(h[4], i16 ? i16_to_f32(q[c]) : bf16_to_f32(q[c]),
                          plane_at(h, centred(i % 4, mx), centred(j % 4, my), centred(k % 4, mz)));
        }
  return 0;
}

}  // extern "C"
