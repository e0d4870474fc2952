// capi.hip -- the C ABI declared in include/adjns.h: host-side validation, workspace layout and
// the launch sequences of one primal step and one reverse step.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/adjns.h"
#include "kernels.hpp"

using namespace adjns;

namespace adjns {
ProfState& prof_state() {
  static ProfState st;
  return st;
}

// Tile shape per stencil kernel class (adjoint stage, primal stage) and precision (FP32, FP64).
int& tile_choice(int kernel_class, int fp64) {
  static int choice[2][2] = {{TILE_32x4x4, TILE_32x4x2}, {TILE_32x4x4, TILE_32x4x2}};
  return choice[kernel_class == ADJ_PROF_PRIMAL_STAGE ? 1 : 0][fp64 ? 1 : 0];
}
}  // namespace adjns

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(ADJ_EHIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr size_t ALIGN = 256;
inline size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

long long ncells(const adj_grid* g) { return (long long)g->n[0] * g->n[1] * g->n[2]; }
size_t elem(const adj_grid* g) { return g->precision == ADJ_F64 ? sizeof(double) : sizeof(float); }

// Workspace layout (each region 256-byte aligned): five state-sized stage buffers
// (W2, W3, W4 / g2, g4, g3), one decoded checkpoint, the nu field, reduction partials, scalars.
struct WsLayout {
  size_t W2, W3, W4, g4, g3, wdec, nu, partials, scratch, total;
};

WsLayout layout(const adj_grid* g) {
  const size_t S = up(5 * (size_t)ncells(g) * elem(g));
  WsLayout L;
  L.W2 = 0;
  L.W3 = L.W2 + S;
  L.W4 = L.W3 + S;
  L.g4 = L.W4 + S;
  L.g3 = L.g4 + S;
  L.wdec = L.g3 + S;
  L.nu = L.wdec + S;
  L.partials = L.nu + up((size_t)ncells(g) * elem(g));
  const size_t tiles = (size_t)((g->n[0] + TX - 1) / TX) * ((g->n[1] + TY - 1) / TY) * ((g->n[2] + TZ - 1) / TZ);
  const size_t npart = tiles > (size_t)MAX_PARTIALS * 10 ? tiles : (size_t)MAX_PARTIALS * 10;
  L.scratch = L.partials + up(npart * sizeof(double));
  L.total = L.scratch + up(64 * sizeof(double));
  return L;
}

int check_grid(const adj_grid* g, bool need_dt) {
  if (!g) return fail(ADJ_EINVAL, "grid is NULL");
  for (int d = 0; d < 3; ++d) {
    if (g->n[d] < 1) return fail(ADJ_EINVAL, "n[%d] = %d must be >= 1", d, g->n[d]);
    if (!(g->L[d] > 0.0) || !std::isfinite(g->L[d])) return fail(ADJ_EINVAL, "L[%d] must be positive", d);
  }
  if ((long long)((g->n[0] + 15) / 16) * ((g->n[1] + 3) / 4) * ((g->n[2] + 3) / 4) > 0x7fffffffLL)
    return fail(ADJ_ESHAPE, "grid too large for one tile launch");
  if (g->bc_x != ADJ_BC_PERIODIC && g->bc_x != ADJ_BC_SLIP_WALLS && g->bc_x != ADJ_BC_CHARACTERISTIC)
    return fail(ADJ_EINVAL, "bad bc_x %d", g->bc_x);
  if (g->bc_x != ADJ_BC_PERIODIC && g->n[0] < 2) return fail(ADJ_ESHAPE, "x boundaries need n[0] >= 2");
  if (!(g->gamma > 1.0) || !std::isfinite(g->gamma)) return fail(ADJ_EINVAL, "gamma must be > 1");
  if (!(g->prandtl > 0.0)) return fail(ADJ_EINVAL, "prandtl must be > 0");
  if (!(g->mu >= 0.0) || !std::isfinite(g->mu)) return fail(ADJ_EINVAL, "mu must be >= 0");
  if (need_dt && (!(g->dt > 0.0) || !std::isfinite(g->dt))) return fail(ADJ_EINVAL, "dt must be > 0");
  for (int v = 0; v < 5; ++v)
    if (!std::isfinite(g->w_ref[v])) return fail(ADJ_EINVAL, "w_ref[%d] must be finite", v);
  for (int k = 0; k < 3; ++k)
    if (!(g->nu_weight[k] >= 0.0) || !std::isfinite(g->nu_weight[k]))
      return fail(ADJ_EINVAL, "nu_weight[%d] must be finite and >= 0", k);
  if (g->precision != ADJ_F64 && g->precision != ADJ_F32) return fail(ADJ_EINVAL, "bad precision %d", g->precision);
  if (g->time_scheme != ADJ_RK4 && g->time_scheme != ADJ_SSPRK3)
    return fail(ADJ_EINVAL, "bad time_scheme %d", g->time_scheme);
  if (g->flux != ADJ_FLUX_SPLIT && g->flux != ADJ_FLUX_ROE) return fail(ADJ_EINVAL, "bad flux %d", g->flux);
  if ((g->flux == ADJ_FLUX_ROE || g->bc_x == ADJ_BC_CHARACTERISTIC) &&
      (!(g->roe_delta > 0.0) || !std::isfinite(g->roe_delta)))
    return fail(ADJ_EINVAL, "roe_delta must be finite and > 0");
  if (g->bc_x == ADJ_BC_CHARACTERISTIC) {
    for (int s = 0; s < 2; ++s) {
      const double* f = g->w_far[s];
      for (int v = 0; v < 5; ++v)
        if (!std::isfinite(f[v])) return fail(ADJ_EINVAL, "w_far[%d][%d] must be finite", s, v);
      const double p = (g->gamma - 1.0) * (f[4] - 0.5 * (f[1] * f[1] + f[2] * f[2] + f[3] * f[3]) / f[0]);
      if (!(f[0] > 0.0) || !(p > 0.0)) return fail(ADJ_EINVAL, "w_far[%d] needs rho > 0 and p > 0", s);
    }
  }
  if (5 * (double)ncells(g) * (g->precision == ADJ_F64 ? 8.0 : 4.0) >= 4294967296.0)
    return fail(ADJ_ESHAPE, "state arrays must span less than 4 GiB (%lld cells)", ncells(g));
  if (g->ckpt_format != ADJ_CKPT_NATIVE && g->ckpt_format != ADJ_CKPT_BF16 && g->ckpt_format != ADJ_CKPT_I16)
    return fail(ADJ_EINVAL, "bad ckpt_format %d", g->ckpt_format);
  if (g->ckpt_format != ADJ_CKPT_NATIVE && g->precision != ADJ_F32)
    return fail(ADJ_EINVAL, "checkpoint records need precision ADJ_F32");
  return ADJ_OK;
}

int check_ws(const adj_grid* g, const void* ws, size_t ws_bytes) {
  if (!ws) return fail(ADJ_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % ALIGN) return fail(ADJ_EWORKSPACE, "workspace must be 256-byte aligned");
  const size_t need = layout(g).total;
  if (ws_bytes < need) return fail(ADJ_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  return ADJ_OK;
}

int check_obj(const adj_grid* g, const adj_objective* o) {
  if (!o) return ADJ_OK;
  if (o->kind < ADJ_OBJ_NONE || o->kind > ADJ_OBJ_PT_LOSS_PLANE) return fail(ADJ_EINVAL, "bad objective kind %d", o->kind);
  if (o->kind == ADJ_OBJ_PT_LOSS_PLANE) {
    if (o->plane_i < 1 || o->plane_i > g->n[0] - 1)
      return fail(ADJ_ESHAPE, "plane_i = %d outside [1, n[0]-1]", o->plane_i);
    if (!(o->pt_ref > 0.0)) return fail(ADJ_EINVAL, "pt_ref must be > 0");
  }
  return ADJ_OK;
}

template <typename T>
Consts<T> consts(const adj_grid* g) {
  Consts<T> c;
  c.nx = g->n[0];
  c.ny = g->n[1];
  c.nz = g->n[2];
  c.wall = g->bc_x != ADJ_BC_PERIODIC;  // characteristic boundaries keep the mirror ghosts
  c.N = ncells(g);
  for (int d = 0; d < 3; ++d) {
    const double h = g->L[d] / g->n[d];
    c.dx[d] = (T)h;
    c.idx[d] = (T)(1.0 / h);
  }
  c.gamma = (T)g->gamma;
  c.mu = (T)g->mu;
  c.alpha = (T)(g->gamma * g->mu / g->prandtl);
  c.dt = (T)g->dt;
  for (int v = 0; v < 5; ++v) c.wref[v] = (T)g->w_ref[v];
  // per-component weight of the artificial viscosity: groups (rho), (rho u_1..3), (rho E)
  const bool unit = g->nu_weight[0] == 0.0 && g->nu_weight[1] == 0.0 && g->nu_weight[2] == 0.0;
  static constexpr int group[5] = {0, 1, 1, 1, 2};
  for (int v = 0; v < 5; ++v) c.nuw[v] = unit ? T(1) : (T)g->nu_weight[group[v]];
  return c;
}

inline char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

// A BF16 record: the block header (25 floats per 4x4x4 block: a plane and a scale per variable),
// 256-byte aligned, then 5N codes.
size_t ckpt_header_bytes(const adj_grid* g) {
  const size_t nb = (size_t)((g->n[0] + 3) / 4) * ((g->n[1] + 3) / 4) * ((g->n[2] + 3) / 4);
  return up(nb * 25 * sizeof(float));
}

// One primal stage (launch_primal_stage; on a Roe-flux grid without its split-form convective
// flux) and, on a Roe-flux grid, the Roe convective terms, on a grid with characteristic
// boundaries the correction of the boundary faces, each weighted like R in the stage (cR; dt/6 in
// stage 4; 1 for the plain residual).
template <typename T>
int primal_stage(const adj_grid* g, int mode, const Consts<T>& c, const T* W, const T* wn, const T* s, const T* W2,
                 const T* W3, T cR, T* out, hipStream_t st, const char* what, T ca = T(0), T cb = T(0),
                 double* jpart = nullptr) {
  hipError_t e;
  const int split = g->flux == ADJ_FLUX_SPLIT;
  if ((e = launch_primal_stage<T>(mode, c, W, wn, s, W2, W3, cR, out, st, ca, cb, split, jpart)))
    return hip_fail(e, what);
  const T coef = mode == STAGE_FIN ? c.dt / T(6) : (mode == STAGE_RES ? T(1) : cR);
  const int open = g->bc_x == ADJ_BC_CHARACTERISTIC;
  if (!split) {
    if ((e = launch_roe_primal<T>(c, (T)g->roe_delta, open, W, coef, out, st))) return hip_fail(e, what);
  }
  if (open) {
    if ((e = launch_char_primal<T>(c, (T)g->roe_delta, split, &g->w_far[0][0], W, coef, out, st)))
      return hip_fail(e, what);
  }
  return ADJ_OK;
}

// One reverse stage (launch_adjoint_stage, as the primal stage) and the transposes of the Roe
// terms and boundary corrections applied to the same kh = ca a + cg gnext, added into `out` (g, or
// w^_n in stage 1).
template <typename T>
int adjoint_stage(const adj_grid* g, int mode, const Consts<T>& c, const T* W, const T* a, const T* gnext,
                  const T* nu, T ca, T cg, const T* g3, const T* g4, T* out, T* grad_s, hipStream_t st,
                  const char* what, double objw = 0.0) {
  hipError_t e;
  const int split = g->flux == ADJ_FLUX_SPLIT;
  if ((e = launch_adjoint_stage<T>(mode, c, W, a, gnext, nu, ca, cg, g3, g4, out, grad_s, st, split, objw)))
    return hip_fail(e, what);
  const int open = g->bc_x == ADJ_BC_CHARACTERISTIC;
  if (!split) {
    if ((e = launch_roe_adjoint<T>(c, (T)g->roe_delta, open, W, a, gnext, ca, cg, out, st))) return hip_fail(e, what);
  }
  if (open) {
    if ((e = launch_char_adjoint<T>(c, (T)g->roe_delta, split, &g->w_far[0][0], W, a, gnext, ca, cg, out, st)))
      return hip_fail(e, what);
  }
  return ADJ_OK;
}

// jpart: per-tile pressure sums of the new state from the final RK4 stage (see fuse_meanp), or NULL;
// jin: per-tile dissipation sums of w_n from stage 1 (see fuse_dissipation_in), folded into
// *J_in with factor jin_scale right after that stage, or NULL
template <typename T>
int primal_step(const adj_grid* g, const T* wn, const T* s, T* out, void* ckpt, T* stages, void* ws, hipStream_t st,
                double* jpart = nullptr, double* jin = nullptr, double* J_in = nullptr, double jin_scale = 0.0) {
  const Consts<T> c = consts<T>(g);
  const WsLayout L = layout(g);
  const long long S5 = 5 * c.N;
  T* W2 = stages ? stages : (T*)at(ws, L.W2);
  T* W3 = stages ? stages + S5 : (T*)at(ws, L.W3);
  T* W4 = stages ? stages + 2 * S5 : (T*)at(ws, L.W4);
  const T h = c.dt * T(0.5);
  hipError_t e;
  int r;
  if (g->time_scheme == ADJ_SSPRK3) {
    // u1 = w + dt R(w) (in W2), u2 = 3/4 w + 1/4 u1 + dt/4 R(u1) (in W3), w_next = 1/3 w + 2/3 u2 +
    // 2 dt/3 R(u2); the affine weights sum to one, so stored deviations w - w_ref combine alike
    if ((r = primal_stage<T>(g, STAGE_LIN, c, wn, wn, s, nullptr, nullptr, c.dt, W2, st, "primal stage 1", T(0), T(0),
                             jin)))
      return r;
    if (jin && (e = launch_fold(jin, primal_tiles<T>(c), J_in, jin_scale, 1.0, st)))
      return hip_fail(e, "dissipation of the step's state");
    if ((r = primal_stage<T>(g, STAGE_AFF, c, W2, wn, s, nullptr, nullptr, c.dt * T(0.25), W3, st, "primal stage 2",
                             T(0.75), T(0.25))))
      return r;
    if ((r = primal_stage<T>(g, STAGE_AFF, c, W3, wn, s, nullptr, nullptr, c.dt * T(2.0 / 3.0), out, st,
                             "primal stage 3", T(1.0 / 3.0), T(2.0 / 3.0))))
      return r;
  } else {
    if ((r = primal_stage<T>(g, STAGE_LIN, c, wn, wn, s, nullptr, nullptr, h, W2, st, "primal stage 1", T(0), T(0),
                             jin)))
      return r;
    if (jin && (e = launch_fold(jin, primal_tiles<T>(c), J_in, jin_scale, 1.0, st)))
      return hip_fail(e, "dissipation of the step's state");
    if ((r = primal_stage<T>(g, STAGE_LIN, c, W2, wn, s, nullptr, nullptr, h, W3, st, "primal stage 2"))) return r;
    if ((r = primal_stage<T>(g, STAGE_LIN, c, W3, wn, s, nullptr, nullptr, c.dt, W4, st, "primal stage 3"))) return r;
    if ((r = primal_stage<T>(g, STAGE_FIN, c, W4, wn, s, W2, W3, T(0), out, st, "primal stage 4", T(0), T(0), jpart)))
      return r;
  }
  if (ckpt) {
    if constexpr (sizeof(T) == sizeof(float)) {
      float* hdr = (float*)ckpt;
      uint16_t* codes = (uint16_t*)at(ckpt, ckpt_header_bytes(g));
      if ((e = launch_ckpt_encode(c, (const float*)out, hdr, codes, g->ckpt_format == ADJ_CKPT_I16, st)))
        return hip_fail(e, "checkpoint encode");
    }
  }
  return ADJ_OK;
}

// SSP-RK3 reverse step: with a = w^_{n+1}, the stage transposes
//   g3 = (J(u2)^T + L_nu) k3, k3 = 2dt/3 a;   g2 = (J(u1)^T + L_nu) k2, k2 = dt/6 a + dt/4 g3;
//   g1 = (J(w_n)^T + L_nu) k1, k1 = dt/6 a + dt (g2 + g3/4);
//   w^_n = a + g1 + g2 + g3 (+ c_n dj/dw),  grad_s += k1 + k2 + k3 = dt a + dt (g2 + g3/4) + dt/4 g3
// (the Shu-Osher stages reversed one by one and summed; wn is the decoded state).
template <typename T>
int adjoint_step_rk3(const adj_grid* g, const Consts<T>& c, const WsLayout& L, const T* wn, const T* stages,
                     const T* s, const T* a, double lambda, const adj_objective* o, double c_n, T* wh, T* grad_s,
                     void* ws, hipStream_t st) {
  const long long S5 = 5 * c.N;
  const T dt = c.dt;
  hipError_t e;
  int r;
  const T *u1 = (T*)at(ws, L.W2), *u2 = (T*)at(ws, L.W3);
  if (stages) {
    u1 = stages;
    u2 = stages + S5;
  } else {
    if ((r = primal_stage<T>(g, STAGE_LIN, c, wn, wn, s, nullptr, nullptr, dt, (T*)at(ws, L.W2), st, "recompute u1")))
      return r;
    if ((r = primal_stage<T>(g, STAGE_AFF, c, (T*)at(ws, L.W2), wn, s, nullptr, nullptr, dt * T(0.25),
                             (T*)at(ws, L.W3), st, "recompute u2", T(0.75), T(0.25))))
      return r;
  }
  T* nu = (T*)at(ws, L.nu);
  const T* nup = nullptr;
  if (lambda > 0.0) {
    if ((e = launch_sigma1<T>(c, wn, (T)lambda, nu, st))) return hip_fail(e, "sigma_1");
    nup = nu;
  }
  T* g3 = (T*)at(ws, L.g3);
  T* g2 = (T*)at(ws, L.g4);
  T* g1 = (T*)at(ws, L.W4);
  if ((r = adjoint_stage<T>(g, STAGE_VJP, c, u2, a, nullptr, nup, dt * T(2.0 / 3.0), T(0), nullptr, nullptr, g3,
                            nullptr, st, "adjoint stage 3")))
    return r;
  if ((r = adjoint_stage<T>(g, STAGE_VJP, c, u1, a, g3, nup, dt / T(6), dt * T(0.25), nullptr, nullptr, g2, nullptr,
                            st, "adjoint stage 2")))
    return r;
  if ((e = launch_rk3_mid<T>(g2, g3, S5, st))) return hip_fail(e, "adjoint stage combination");
  if ((r = adjoint_stage<T>(g, STAGE_VJP, c, wn, a, g2, nup, dt / T(6), dt, nullptr, nullptr, g1, nullptr, st,
                            "adjoint stage 1")))
    return r;
  if ((e = launch_rk3_combine<T>(a, g1, g2, g3, dt, wh, grad_s, S5, st))) return hip_fail(e, "adjoint combination");
  if (o && o->kind != ADJ_OBJ_NONE && c_n != 0.0) {
    if ((e = launch_objective<T>(c, o->kind, o->plane_i, o->pt_ref, wn, c_n, nullptr, wh,
                                 (double*)at(ws, L.partials), (double*)at(ws, L.scratch), st)))
      return hip_fail(e, "objective gradient");
  }
  return ADJ_OK;
}

template <typename T>
int adjoint_step(const adj_grid* g, const void* wn_in, const T* stages, const T* s, const T* a, double lambda,
                 const adj_objective* o, double c_n, T* wh, T* grad_s, void* ws, hipStream_t st) {
  const Consts<T> c = consts<T>(g);
  const WsLayout L = layout(g);
  const long long S5 = 5 * c.N;
  T* W2 = (T*)at(ws, L.W2);
  T* W3 = (T*)at(ws, L.W3);
  T* W4 = (T*)at(ws, L.W4);
  T* g4 = (T*)at(ws, L.g4);
  T* g3 = (T*)at(ws, L.g3);
  T* g2 = W4;  // W4 is dead once the stage-4 gather has run (or unused when stages are given)
  T* nu = (T*)at(ws, L.nu);
  hipError_t e;
  const T* wn = (const T*)wn_in;
  if (g->ckpt_format != ADJ_CKPT_NATIVE) {
    if constexpr (sizeof(T) == sizeof(float)) {
      float* dec = (float*)at(ws, L.wdec);
      if ((e = launch_ckpt_decode(c, (const float*)wn_in,
                                  (const uint16_t*)((const char*)wn_in + ckpt_header_bytes(g)), dec,
                                  g->ckpt_format == ADJ_CKPT_I16, st)))
        return hip_fail(e, "checkpoint decode");
      wn = (const T*)dec;
    }
  }
  if (g->time_scheme == ADJ_SSPRK3) return adjoint_step_rk3<T>(g, c, L, wn, stages, s, a, lambda, o, c_n, wh, grad_s,
                                                              ws, st);
  const T *sW2 = W2, *sW3 = W3, *sW4 = W4;
  if (stages) {
    // stage states stored by the forward sweep (adj_primal_step_stages)
    sW2 = stages;
    sW3 = stages + S5;
    sW4 = stages + 2 * S5;
  } else {
    // forward recompute of the stage states
    const T h = c.dt * T(0.5);
    int r;
    if ((r = primal_stage<T>(g, STAGE_LIN, c, wn, wn, s, nullptr, nullptr, h, W2, st, "recompute W2"))) return r;
    if ((r = primal_stage<T>(g, STAGE_LIN, c, W2, wn, s, nullptr, nullptr, h, W3, st, "recompute W3"))) return r;
    if ((r = primal_stage<T>(g, STAGE_LIN, c, W3, wn, s, nullptr, nullptr, c.dt, W4, st, "recompute W4"))) return r;
  }
  const T* nup = nullptr;
  if (lambda > 0.0) {
    if ((e = launch_sigma1<T>(c, wn, (T)lambda, nu, st))) return hip_fail(e, "sigma_1");
    nup = nu;
  }
  const T dt = c.dt;
  int r;
  if ((r = adjoint_stage<T>(g, STAGE_VJP, c, sW4, a, nullptr, nup, dt / T(6), T(0), nullptr, nullptr, g4, nullptr, st,
                            "adjoint stage 4")))
    return r;
  if ((r = adjoint_stage<T>(g, STAGE_VJP, c, sW3, a, g4, nup, dt / T(3), dt, nullptr, nullptr, g3, nullptr, st,
                            "adjoint stage 3")))
    return r;
  if ((r = adjoint_stage<T>(g, STAGE_VJP, c, sW2, a, g3, nup, dt / T(3), dt * T(0.5), nullptr, nullptr, g2, nullptr, st,
                            "adjoint stage 2")))
    return r;
  // the mean-pressure objective's injection rides in the stage-1 kernel when nothing is added to
  // w^_n after it (no Roe or boundary corrections)
  const bool fuse = o && o->kind == ADJ_OBJ_MEAN_PRESSURE && c_n != 0.0 && g->flux == ADJ_FLUX_SPLIT &&
                    g->bc_x != ADJ_BC_CHARACTERISTIC;
  if ((r = adjoint_stage<T>(g, STAGE_FIN, c, wn, a, g2, nup, dt / T(6), dt * T(0.5), g3, g4, wh, grad_s, st,
                            "adjoint stage 1", fuse ? c_n : 0.0)))
    return r;
  if (!fuse && o && o->kind != ADJ_OBJ_NONE && c_n != 0.0) {
    if ((e = launch_objective<T>(c, o->kind, o->plane_i, o->pt_ref, wn, c_n, nullptr, wh,
                                 (double*)at(ws, L.partials), (double*)at(ws, L.scratch), st)))
      return hip_fail(e, "objective gradient");
  }
  return ADJ_OK;
}

}  // namespace

extern "C" {

size_t adj_workspace_bytes(const adj_grid* grid) {
  if (check_grid(grid, false)) return 0;
  return layout(grid).total;
}

size_t adj_ckpt_bytes(const adj_grid* grid) {
  if (check_grid(grid, false)) return 0;
  return ckpt_header_bytes(grid) + 5 * (size_t)ncells(grid) * sizeof(uint16_t);
}

static int primal_entry(const adj_grid* grid, const void* w_n, const void* s, void* w_np1, void* ckpt_out,
                        void* stages, void* ws, size_t ws_bytes, void* stream) {
  int r;
  if ((r = check_grid(grid, true))) return r;
  if ((r = check_ws(grid, ws, ws_bytes))) return r;
  if (!w_n || !w_np1) return fail(ADJ_EINVAL, "w_n and w_np1 must be non-NULL");
  if (w_n == w_np1) return fail(ADJ_EINVAL, "w_np1 must not alias w_n");
  if (ckpt_out && grid->precision != ADJ_F32) return fail(ADJ_EINVAL, "BF16 checkpoints need precision ADJ_F32");
  hipStream_t st = (hipStream_t)stream;
  if (grid->precision == ADJ_F64)
    return primal_step<double>(grid, (const double*)w_n, (const double*)s, (double*)w_np1, nullptr, (double*)stages,
                               ws, st);
  return primal_step<float>(grid, (const float*)w_n, (const float*)s, (float*)w_np1, ckpt_out, (float*)stages, ws, st);
}

int adj_primal_step(const adj_grid* grid, const void* w_n, const void* s, void* w_np1, void* ckpt_out, void* ws,
                    size_t ws_bytes, void* stream) {
  return primal_entry(grid, w_n, s, w_np1, ckpt_out, nullptr, ws, ws_bytes, stream);
}

extern "C++" {
// The mean-pressure objective of the new state rides in the final RK4 stage when that stage's output
// is the new state (no Roe or boundary correction follows it).
static bool fuse_meanp(const adj_grid* g, const adj_objective* o) {
  return o->kind == ADJ_OBJ_MEAN_PRESSURE && g->time_scheme == ADJ_RK4 && g->flux == ADJ_FLUX_SPLIT &&
         g->bc_x != ADJ_BC_CHARACTERISTIC;
}

// The dissipation of the step's own state w_n rides in stage 1, which stages w_n with one halo
// cell: periodic or slip-wall x boundaries (whose ghost cells the objective kernel mirrors alike).
static bool fuse_dissipation_in(const adj_grid* g, const adj_objective* o) {
  return o->kind == ADJ_OBJ_KE_DISSIPATION && g->bc_x != ADJ_BC_CHARACTERISTIC;
}

template <typename T>
static int primal_obj(const adj_grid* grid, const T* w_n, const T* s, T* w_np1, void* ckpt, T* stages,
                      const adj_objective* obj, double weight_in, double weight, double* J_accum, void* ws,
                      hipStream_t st) {
  const Consts<T> c = consts<T>(grid);
  const WsLayout L = layout(grid);
  double* part = (double*)at(ws, L.partials);
  double* scr = (double*)at(ws, L.scratch);
  const bool fuse_in = weight_in != 0.0 && fuse_dissipation_in(grid, obj);
  const bool fuse_out = weight != 0.0 && fuse_meanp(grid, obj);
  hipError_t e;
  int r;
  if (weight_in != 0.0 && !fuse_in &&
      (e = launch_objective<T>(c, obj->kind, obj->plane_i, obj->pt_ref, w_n, weight_in, J_accum, nullptr, part, scr,
                               st)))
    return hip_fail(e, "objective of the step's state");
  // the stage-1 partials are folded before the final stage writes its own into the same region
  if ((r = primal_step<T>(grid, w_n, s, w_np1, ckpt, stages, ws, st, fuse_out ? part : nullptr,
                          fuse_in ? part : nullptr, J_accum, weight_in / (double)c.N)))
    return r;
  if (weight == 0.0) return ADJ_OK;
  if (fuse_out)
    e = launch_fold(part, primal_tiles<T>(c), J_accum, weight / (double)c.N, 1.0, st);
  else
    e = launch_objective<T>(c, obj->kind, obj->plane_i, obj->pt_ref, w_np1, weight, J_accum, nullptr, part, scr, st);
  return e ? hip_fail(e, "objective of the new state") : ADJ_OK;
}
}  // extern "C++"

int adj_primal_step_obj(const adj_grid* grid, const void* w_n, const void* s, void* w_np1, void* ckpt_out,
                        void* stages_out, const adj_objective* obj, double weight_in, double weight, double* J_accum,
                        void* ws, size_t ws_bytes, void* stream) {
  int r;
  if ((r = check_grid(grid, true))) return r;
  if ((r = check_ws(grid, ws, ws_bytes))) return r;
  if ((r = check_obj(grid, obj))) return r;
  if (!std::isfinite(weight) || !std::isfinite(weight_in)) return fail(ADJ_EINVAL, "weights must be finite");
  const bool active = obj && obj->kind != ADJ_OBJ_NONE && (weight != 0.0 || weight_in != 0.0);
  if (active && !J_accum) return fail(ADJ_EINVAL, "J_accum must be non-NULL");
  if (!w_n || !w_np1) return fail(ADJ_EINVAL, "w_n and w_np1 must be non-NULL");
  if (w_n == w_np1) return fail(ADJ_EINVAL, "w_np1 must not alias w_n");
  if (ckpt_out && grid->precision != ADJ_F32) return fail(ADJ_EINVAL, "BF16 checkpoints need precision ADJ_F32");
  if (stages_out && grid->ckpt_format != ADJ_CKPT_NATIVE) return fail(ADJ_EINVAL, "stage states are stored natively");
  if (!active) return primal_entry(grid, w_n, s, w_np1, ckpt_out, stages_out, ws, ws_bytes, stream);
  hipStream_t st = (hipStream_t)stream;
  if (grid->precision == ADJ_F64)
    return primal_obj<double>(grid, (const double*)w_n, (const double*)s, (double*)w_np1, nullptr, (double*)stages_out,
                              obj, weight_in, weight, J_accum, ws, st);
  return primal_obj<float>(grid, (const float*)w_n, (const float*)s, (float*)w_np1, ckpt_out, (float*)stages_out, obj,
                           weight_in, weight, J_accum, ws, st);
}

int adj_primal_step_stages(const adj_grid* grid, const void* w_n, const void* s, void* w_np1, void* stages_out,
                           void* ws, size_t ws_bytes, void* stream) {
  if (!stages_out) return fail(ADJ_EINVAL, "stages_out must be non-NULL");
  if (grid && grid->ckpt_format != ADJ_CKPT_NATIVE) return fail(ADJ_EINVAL, "stage states are stored natively");
  return primal_entry(grid, w_n, s, w_np1, nullptr, stages_out, ws, ws_bytes, stream);
}

static int adjoint_entry(const adj_grid* grid, const void* w_n, const void* stages, const void* s, const void* wh_np1,
                         double lambda, const adj_objective* obj, double c_n, void* wh_n, void* grad_s, void* ws,
                         size_t ws_bytes, void* stream) {
  int r;
  if ((r = check_grid(grid, true))) return r;
  if ((r = check_ws(grid, ws, ws_bytes))) return r;
  if ((r = check_obj(grid, obj))) return r;
  if (!w_n || !wh_np1 || !wh_n) return fail(ADJ_EINVAL, "w_n, wh_np1 and wh_n must be non-NULL");
  if (wh_n == wh_np1) return fail(ADJ_EINVAL, "wh_n must not alias wh_np1");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(ADJ_EINVAL, "lambda must be finite and >= 0");
  if (!std::isfinite(c_n)) return fail(ADJ_EINVAL, "c_n must be finite");
  hipStream_t st = (hipStream_t)stream;
  if (grid->precision == ADJ_F64)
    return adjoint_step<double>(grid, w_n, (const double*)stages, (const double*)s, (const double*)wh_np1, lambda, obj,
                                c_n, (double*)wh_n, (double*)grad_s, ws, st);
  return adjoint_step<float>(grid, w_n, (const float*)stages, (const float*)s, (const float*)wh_np1, lambda, obj, c_n,
                             (float*)wh_n, (float*)grad_s, ws, st);
}

int adj_adjoint_step(const adj_grid* grid, const void* w_n, const void* s, const void* wh_np1, double lambda,
                     const adj_objective* obj, double c_n, void* wh_n, void* grad_s, void* ws, size_t ws_bytes,
                     void* stream) {
  return adjoint_entry(grid, w_n, nullptr, s, wh_np1, lambda, obj, c_n, wh_n, grad_s, ws, ws_bytes, stream);
}

int adj_adjoint_step_stages(const adj_grid* grid, const void* w_n, const void* stages, const void* s,
                            const void* wh_np1, double lambda, const adj_objective* obj, double c_n, void* wh_n,
                            void* grad_s, void* ws, size_t ws_bytes, void* stream) {
  if (!stages) return fail(ADJ_EINVAL, "stages must be non-NULL");
  if (grid && grid->ckpt_format != ADJ_CKPT_NATIVE) return fail(ADJ_EINVAL, "stage states are stored natively");
  return adjoint_entry(grid, w_n, stages, s, wh_np1, lambda, obj, c_n, wh_n, grad_s, ws, ws_bytes, stream);
}

int adj_growth_sigma1(const adj_grid* grid, const void* w, double scale, void* out, void* stream) {
  int r;
  if ((r = check_grid(grid, false))) return r;
  if (!w || !out) return fail(ADJ_EINVAL, "w and out must be non-NULL");
  if (!std::isfinite(scale)) return fail(ADJ_EINVAL, "scale must be finite");
  hipError_t e;
  hipStream_t st = (hipStream_t)stream;
  if (grid->precision == ADJ_F64)
    e = launch_sigma1<double>(consts<double>(grid), (const double*)w, scale, (double*)out, st);
  else
    e = launch_sigma1<float>(consts<float>(grid), (const float*)w, (float)scale, (float*)out, st);
  return e ? hip_fail(e, "sigma_1") : ADJ_OK;
}

int adj_stability(const adj_grid* grid, const void* w, double lambda, double* out, void* ws, size_t ws_bytes,
                  void* stream) {
  int r;
  if ((r = check_grid(grid, true))) return r;
  if ((r = check_ws(grid, ws, ws_bytes))) return r;
  if (!w || !out) return fail(ADJ_EINVAL, "w and out must be non-NULL");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(ADJ_EINVAL, "lambda must be finite and >= 0");
  const WsLayout L = layout(grid);
  hipStream_t st = (hipStream_t)stream;
  double s4 = 0.0;
  for (int d = 0; d < 3; ++d) s4 += 4.0 * (grid->n[d] / grid->L[d]) * (grid->n[d] / grid->L[d]);
  const bool unit = grid->nu_weight[0] == 0.0 && grid->nu_weight[1] == 0.0 && grid->nu_weight[2] == 0.0;
  const double wmax = unit ? 1.0 : std::max(grid->nu_weight[0], std::max(grid->nu_weight[1], grid->nu_weight[2]));
  const double s_art = grid->dt * lambda * wmax * s4;
  hipError_t e;
  if (grid->precision == ADJ_F64) {
    const Consts<double> c = consts<double>(grid);
    double* sig = (double*)at(ws, L.nu);
    if (lambda > 0.0 && (e = launch_sigma1<double>(c, (const double*)w, 1.0, sig, st))) return hip_fail(e, "sigma_1");
    e = launch_stability<double>(c, (const double*)w, lambda > 0.0 ? sig : nullptr, grid->dt, grid->dt, s_art,
                                 (double*)at(ws, L.partials), out, st);
  } else {
    const Consts<float> c = consts<float>(grid);
    float* sig = (float*)at(ws, L.nu);
    if (lambda > 0.0 && (e = launch_sigma1<float>(c, (const float*)w, 1.0f, sig, st))) return hip_fail(e, "sigma_1");
    e = launch_stability<float>(c, (const float*)w, lambda > 0.0 ? sig : nullptr, grid->dt, grid->dt, s_art,
                                (double*)at(ws, L.partials), out, st);
  }
  return e ? hip_fail(e, "stability") : ADJ_OK;
}

int adj_check_stable(const adj_grid* grid, const void* w, double lambda, double* out_host, void* ws,
                     size_t ws_bytes, void* stream) {
  int r;
  if ((r = check_grid(grid, true))) return r;
  if ((r = check_ws(grid, ws, ws_bytes))) return r;
  double* dev = (double*)at(ws, layout(grid).scratch);
  if ((r = adj_stability(grid, w, lambda, dev, ws, ws_bytes, stream))) return r;
  double h[3];
  hipError_t e;
  if ((e = hipMemcpyAsync(h, dev, sizeof h, hipMemcpyDeviceToHost, (hipStream_t)stream)) ||
      (e = hipStreamSynchronize((hipStream_t)stream)))
    return hip_fail(e, "stability read-back");
  if (out_host) std::memcpy(out_host, h, sizeof h);
  const bool rk3 = grid->time_scheme == ADJ_SSPRK3;
  const double im = rk3 ? ADJ_SSPRK3_IMAG_BOUND : ADJ_RK4_IMAG_BOUND, re = rk3 ? ADJ_SSPRK3_REAL_BOUND : ADJ_RK4_REAL_BOUND;
  const double bound[3] = {im, re, re};
  const char* what[3] = {"convective", "viscous", "artificial-viscosity"};
  for (int k = 0; k < 3; ++k)
    if (!(h[k] <= bound[k]))
      return fail(ADJ_EUNSTABLE, "%s stability number %.4g exceeds the %s bound %.4g", what[k], h[k],
                  rk3 ? "SSP-RK3" : "RK4", bound[k]);
  return ADJ_OK;
}

int adj_check_status(void* stream) {
  hipError_t e;
  if ((e = hipStreamSynchronize((hipStream_t)stream))) return hip_fail(e, "status: stream");
  unsigned int flag = 0;
  if ((e = read_clear_nonfinite(&flag))) return hip_fail(e, "status: flag");
  if (flag) return fail(ADJ_ENONFINITE, "a reduction met NaN or Inf since the last status check");
  return ADJ_OK;
}

int adj_objective_and_grad(const adj_grid* grid, const adj_objective* obj, const void* w, double weight,
                           double* J_accum, void* djdw, void* ws, size_t ws_bytes, void* stream) {
  int r;
  if ((r = check_grid(grid, false))) return r;
  if (!obj) return fail(ADJ_EINVAL, "objective is NULL");
  if ((r = check_obj(grid, obj))) return r;
  if ((r = check_ws(grid, ws, ws_bytes))) return r;
  if (!w) return fail(ADJ_EINVAL, "w must be non-NULL");
  if (!std::isfinite(weight)) return fail(ADJ_EINVAL, "weight must be finite");
  if (obj->kind == ADJ_OBJ_NONE) return ADJ_OK;
  const WsLayout L = layout(grid);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (grid->precision == ADJ_F64)
    e = launch_objective<double>(consts<double>(grid), obj->kind, obj->plane_i, obj->pt_ref, (const double*)w, weight,
                                 J_accum, (double*)djdw, (double*)at(ws, L.partials), (double*)at(ws, L.scratch), st);
  else
    e = launch_objective<float>(consts<float>(grid), obj->kind, obj->plane_i, obj->pt_ref, (const float*)w, weight,
                                J_accum, (float*)djdw, (double*)at(ws, L.partials), (double*)at(ws, L.scratch), st);
  return e ? hip_fail(e, "objective") : ADJ_OK;
}

int adj_energy_vhat(const adj_grid* grid, const void* w, const void* wh, double* E, void* ws, size_t ws_bytes,
                    void* stream) {
  int r;
  if ((r = check_grid(grid, false))) return r;
  if ((r = check_ws(grid, ws, ws_bytes))) return r;
  if (!w || !wh || !E) return fail(ADJ_EINVAL, "w, wh and E must be non-NULL");
  const WsLayout L = layout(grid);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (grid->precision == ADJ_F64)
    e = launch_energy_vhat<double>(consts<double>(grid), (const double*)w, (const double*)wh, (double*)at(ws, L.partials), E, st);
  else
    e = launch_energy_vhat<float>(consts<float>(grid), (const float*)w, (const float*)wh, (double*)at(ws, L.partials), E, st);
  return e ? hip_fail(e, "energy") : ADJ_OK;
}

int adj_dot(const adj_grid* grid, const void* a, const void* b, double* out, void* ws, size_t ws_bytes, void* stream) {
  int r;
  if ((r = check_grid(grid, false))) return r;
  if ((r = check_ws(grid, ws, ws_bytes))) return r;
  if (!a || !b || !out) return fail(ADJ_EINVAL, "a, b and out must be non-NULL");
  const WsLayout L = layout(grid);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (grid->precision == ADJ_F64)
    e = launch_dot<double>(consts<double>(grid), (const double*)a, (const double*)b, (double*)at(ws, L.partials), out, 1.0, 0.0, st);
  else
    e = launch_dot<float>(consts<float>(grid), (const float*)a, (const float*)b, (double*)at(ws, L.partials), out, 1.0, 0.0, st);
  return e ? hip_fail(e, "dot") : ADJ_OK;
}

int adj_ckpt_encode(const adj_grid* grid, const float* w, void* ckpt, void* ws, size_t ws_bytes, void* stream) {
  int r;
  if ((r = check_grid(grid, false))) return r;
  if (grid->precision != ADJ_F32) return fail(ADJ_EINVAL, "checkpoint records need precision ADJ_F32");
  if ((r = check_ws(grid, ws, ws_bytes))) return r;
  if (!w || !ckpt) return fail(ADJ_EINVAL, "w and ckpt must be non-NULL");
  if ((uintptr_t)ckpt % 64) return fail(ADJ_EINVAL, "ckpt must be 64-byte aligned");
  hipError_t e = launch_ckpt_encode(consts<float>(grid), w, (float*)ckpt, (uint16_t*)at(ckpt, ckpt_header_bytes(grid)),
                                    grid->ckpt_format == ADJ_CKPT_I16, (hipStream_t)stream);
  return e ? hip_fail(e, "encode") : ADJ_OK;
}

int adj_ckpt_decode(const adj_grid* grid, const void* ckpt, float* w, void* stream) {
  int r;
  if ((r = check_grid(grid, false))) return r;
  if (grid->precision != ADJ_F32) return fail(ADJ_EINVAL, "checkpoint records need precision ADJ_F32");
  if (!w || !ckpt) return fail(ADJ_EINVAL, "w and ckpt must be non-NULL");
  if ((uintptr_t)ckpt % 64) return fail(ADJ_EINVAL, "ckpt must be 64-byte aligned");
  hipError_t e = launch_ckpt_decode(consts<float>(grid), (const float*)ckpt,
                                    (const uint16_t*)((const char*)ckpt + ckpt_header_bytes(grid)), w,
                                    grid->ckpt_format == ADJ_CKPT_I16, (hipStream_t)stream);
  return e ? hip_fail(e, "decode") : ADJ_OK;
}

int adj_residual(const adj_grid* grid, const void* w, const void* s, void* R, void* stream) {
  int r;
  if ((r = check_grid(grid, false))) return r;
  if (!w || !R) return fail(ADJ_EINVAL, "w and R must be non-NULL");
  if (w == R) return fail(ADJ_EINVAL, "R must not alias w");
  hipStream_t st = (hipStream_t)stream;
  if (grid->precision == ADJ_F64)
    return primal_stage<double>(grid, STAGE_RES, consts<double>(grid), (const double*)w, nullptr, (const double*)s,
                                nullptr, nullptr, 0.0, (double*)R, st, "residual");
  return primal_stage<float>(grid, STAGE_RES, consts<float>(grid), (const float*)w, nullptr, (const float*)s, nullptr,
                             nullptr, 0.0f, (float*)R, st, "residual");
}

int adj_vjp(const adj_grid* grid, const void* W, const void* kh, const void* nu, void* out, void* stream) {
  int r;
  if ((r = check_grid(grid, false))) return r;
  if (!W || !kh || !out) return fail(ADJ_EINVAL, "W, kh and out must be non-NULL");
  if (out == kh || out == W) return fail(ADJ_EINVAL, "out must not alias its inputs");
  hipStream_t st = (hipStream_t)stream;
  if (grid->precision == ADJ_F64)
    return adjoint_stage<double>(grid, STAGE_VJP, consts<double>(grid), (const double*)W, (const double*)kh, nullptr,
                                 (const double*)nu, 1.0, 0.0, nullptr, nullptr, (double*)out, nullptr, st, "vjp");
  return adjoint_stage<float>(grid, STAGE_VJP, consts<float>(grid), (const float*)W, (const float*)kh, nullptr,
                              (const float*)nu, 1.0f, 0.0f, nullptr, nullptr, (float*)out, nullptr, st, "vjp");
}

int adj_profile_enable(int on) {
  ProfState& P = prof_state();
  if (on)
    for (int k = 0; k < ADJ_PROF_NCLASS; ++k) P.used[k] = 0;
  P.on = on != 0;
  return ADJ_OK;
}

int adj_profile_read(int kernel_class, double* total_ms, long long* launches) {
  if (kernel_class < 0 || kernel_class >= ADJ_PROF_NCLASS) return fail(ADJ_EINVAL, "bad kernel class %d", kernel_class);
  if (!total_ms || !launches) return fail(ADJ_EINVAL, "total_ms and launches must be non-NULL");
  ProfState& P = prof_state();
  double tot = 0.0;
  for (size_t i = 0; i < P.used[kernel_class]; ++i) {
    auto& pr = P.ev[kernel_class][i];
    hipError_t e = hipEventSynchronize(pr.second);
    if (e != hipSuccess) return hip_fail(e, "profile read");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess) return hip_fail(e, "profile read");
    tot += ms;
  }
  *total_ms = tot;
  *launches = (long long)P.used[kernel_class];
  return ADJ_OK;
}

int adj_set_tile(int kernel_class, int precision, int tile) {
  if (kernel_class != ADJ_PROF_ADJOINT_STAGE && kernel_class != ADJ_PROF_PRIMAL_STAGE)
    return fail(ADJ_EINVAL, "tile shapes exist for the adjoint- and primal-stage kernels only");
  if (precision != ADJ_F64 && precision != ADJ_F32) return fail(ADJ_EINVAL, "bad precision %d", precision);
  if (tile < 0 || tile >= NTILES) return fail(ADJ_EINVAL, "bad tile id %d", tile);
  tile_choice(kernel_class, precision == ADJ_F64) = tile;
  return ADJ_OK;
}

int adj_get_tile(int kernel_class, int precision) {
  if (kernel_class != ADJ_PROF_ADJOINT_STAGE && kernel_class != ADJ_PROF_PRIMAL_STAGE) return fail(ADJ_EINVAL, "bad class");
  if (precision != ADJ_F64 && precision != ADJ_F32) return fail(ADJ_EINVAL, "bad precision %d", precision);
  return tile_choice(kernel_class, precision == ADJ_F64);
}

int adj_tile_launched(int kernel_class, int precision, int bc_x, int lnu, int tile) {
  if (kernel_class != ADJ_PROF_ADJOINT_STAGE && kernel_class != ADJ_PROF_PRIMAL_STAGE) return fail(ADJ_EINVAL, "bad class");
  if (precision != ADJ_F64 && precision != ADJ_F32) return fail(ADJ_EINVAL, "bad precision %d", precision);
  if (bc_x != ADJ_BC_PERIODIC && bc_x != ADJ_BC_SLIP_WALLS && bc_x != ADJ_BC_CHARACTERISTIC)
    return fail(ADJ_EINVAL, "bad bc_x %d", bc_x);
  if (tile < 0 || tile >= NTILES) return fail(ADJ_EINVAL, "bad tile id %d", tile);
  if (kernel_class == ADJ_PROF_PRIMAL_STAGE) return tile;  // every primal tile fits
  return adjoint_tile_used(precision == ADJ_F64, bc_x != ADJ_BC_PERIODIC, lnu != 0, tile);
}

// ------------------------------------------------------------------------------------------
// Ensembles
// ------------------------------------------------------------------------------------------
}  // extern "C"

// Host side of an ensemble; the device table it points into belongs to the caller.
struct adj_batch {
  int nbox = 0, nmem = 0, fp64 = 0, wall = 0, lnu = 0, obj = ADJ_OBJ_NONE;
  int tile_p = 0, tile_a = 0;
  std::vector<long long> boff, moff;    // cell offsets of boxes / members (n + 1 entries)
  std::vector<int> sp, sa, slb, slm;    // work-group offsets: primal tiles, adjoint tiles, RB cells
  std::vector<int> mem_box;
  const void *dbox = nullptr, *dmem = nullptr;
  const int *dsp = nullptr, *dsa = nullptr, *dslb = nullptr, *dslm = nullptr;
};

namespace {

struct BatchTable {
  size_t box, mem, sp, sa, slb, slm, total;
};

BatchTable batch_table(int nbox, int nmem, int fp64) {
  const size_t d = fp64 ? sizeof(BoxDesc<double>) : sizeof(BoxDesc<float>);
  BatchTable t;
  t.box = 0;
  t.mem = t.box + up(nbox * d);
  t.sp = t.mem + up(nmem * d);
  t.sa = t.sp + up((nbox + 1) * sizeof(int));
  t.slb = t.sa + up((nmem + 1) * sizeof(int));
  t.slm = t.slb + up((nbox + 1) * sizeof(int));
  t.total = t.slm + up((nmem + 1) * sizeof(int));
  return t;
}

struct BatchWs {
  size_t W2, W3, W4, sig, g4, g3, g2, partials, total;
};

BatchWs batch_ws(const adj_batch* b) {
  const size_t e = b->fp64 ? sizeof(double) : sizeof(float);
  const size_t P = (size_t)b->boff[b->nbox], Q = (size_t)b->moff[b->nmem];
  BatchWs L;
  L.W2 = 0;
  L.W3 = L.W2 + up(5 * P * e);
  L.W4 = L.W3 + up(5 * P * e);
  L.sig = L.W4 + up(5 * P * e);
  L.g4 = L.sig + up(P * e);
  L.g3 = L.g4 + up(5 * Q * e);
  L.g2 = L.g3 + up(5 * Q * e);
  L.partials = L.g2 + up(5 * Q * e);
  L.total = L.partials + up((size_t)b->slm[b->nmem] * sizeof(double));
  return L;
}

template <typename T>
BoxDesc<T> box_desc(const adj_grid* g, long long off, long long aoff, double lam) {
  BoxDesc<T> d;
  std::memset(&d, 0, sizeof d);
  d.c = consts<T>(g);
  d.off = off;
  d.aoff = aoff;
  d.lam = (T)lam;
  return d;
}

int check_batch_ws(const adj_batch* b, const void* ws, size_t ws_bytes) {
  if (!ws) return fail(ADJ_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % ALIGN) return fail(ADJ_EWORKSPACE, "workspace must be 256-byte aligned");
  const size_t need = batch_ws(b).total;
  if (ws_bytes < need) return fail(ADJ_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  return ADJ_OK;
}

template <typename T>
int batch_primal(const adj_batch* b, int nb, const T* wn, const T* s, T* out, void* ws, hipStream_t st) {
  const BatchWs L = batch_ws(b);
  T* W2 = (T*)at(ws, L.W2);
  T* W3 = (T*)at(ws, L.W3);
  T* W4 = (T*)at(ws, L.W4);
  const auto* bx = (const BoxDesc<T>*)b->dbox;
  const int nblk = b->sp[nb];
  hipError_t e;
  if ((e = launch_primal_stage_batch<T>(STAGE_LIN, b->tile_p, bx, b->dsp, nb, nblk, wn, wn, s, nullptr, nullptr,
                                        T(0.5), W2, st)))
    return hip_fail(e, "ensemble primal stage 1");
  if ((e = launch_primal_stage_batch<T>(STAGE_LIN, b->tile_p, bx, b->dsp, nb, nblk, W2, wn, s, nullptr, nullptr,
                                        T(0.5), W3, st)))
    return hip_fail(e, "ensemble primal stage 2");
  if ((e = launch_primal_stage_batch<T>(STAGE_LIN, b->tile_p, bx, b->dsp, nb, nblk, W3, wn, s, nullptr, nullptr,
                                        T(1), W4, st)))
    return hip_fail(e, "ensemble primal stage 3");
  if ((e = launch_primal_stage_batch<T>(STAGE_FIN, b->tile_p, bx, b->dsp, nb, nblk, W4, wn, s, W2, W3, T(0), out, st)))
    return hip_fail(e, "ensemble primal stage 4");
  return ADJ_OK;
}

template <typename T>
int batch_adjoint(const adj_batch* b, int nm, const T* wn, const T* s, const T* a, const double* c_n, T* wh,
                  T* grad_s, void* ws, hipStream_t st) {
  const BatchWs L = batch_ws(b);
  T* W2 = (T*)at(ws, L.W2);
  T* W3 = (T*)at(ws, L.W3);
  T* W4 = (T*)at(ws, L.W4);
  T* sig = (T*)at(ws, L.sig);
  T* g4 = (T*)at(ws, L.g4);
  T* g3 = (T*)at(ws, L.g3);
  T* g2 = (T*)at(ws, L.g2);
  const auto* bx = (const BoxDesc<T>*)b->dbox;
  const auto* mm = (const BoxDesc<T>*)b->dmem;
  const int nb = b->mem_box[nm - 1] + 1;  // boxes whose trajectory an active member reads
  const int pblk = b->sp[nb];
  hipError_t e;
  if ((e = launch_primal_stage_batch<T>(STAGE_LIN, b->tile_p, bx, b->dsp, nb, pblk, wn, wn, s, nullptr, nullptr,
                                        T(0.5), W2, st)))
    return hip_fail(e, "ensemble recompute W2");
  if ((e = launch_primal_stage_batch<T>(STAGE_LIN, b->tile_p, bx, b->dsp, nb, pblk, W2, wn, s, nullptr, nullptr,
                                        T(0.5), W3, st)))
    return hip_fail(e, "ensemble recompute W3");
  if ((e = launch_primal_stage_batch<T>(STAGE_LIN, b->tile_p, bx, b->dsp, nb, pblk, W3, wn, s, nullptr, nullptr,
                                        T(1), W4, st)))
    return hip_fail(e, "ensemble recompute W4");
  if (b->lnu && (e = launch_sigma1_batch<T>(bx, b->dslb, nb, b->slb[nb], wn, sig, st)))
    return hip_fail(e, "ensemble sigma_1");
  const int ablk = b->sa[nm];
  const int tl = b->tile_a, wl = b->wall, ln = b->lnu;
  if ((e = launch_adjoint_stage_batch<T>(STAGE_VJP, tl, wl, ln, mm, b->dsa, nm, ablk, W4, a, nullptr, sig, T(6), T(0),
                                         nullptr, nullptr, g4, nullptr, st)))
    return hip_fail(e, "ensemble adjoint stage 4");
  if ((e = launch_adjoint_stage_batch<T>(STAGE_VJP, tl, wl, ln, mm, b->dsa, nm, ablk, W3, a, g4, sig, T(3), T(1),
                                         nullptr, nullptr, g3, nullptr, st)))
    return hip_fail(e, "ensemble adjoint stage 3");
  if ((e = launch_adjoint_stage_batch<T>(STAGE_VJP, tl, wl, ln, mm, b->dsa, nm, ablk, W2, a, g3, sig, T(3), T(0.5),
                                         nullptr, nullptr, g2, nullptr, st)))
    return hip_fail(e, "ensemble adjoint stage 2");
  // the mean-pressure objective's c_n dj/dw(w_n) of every member is added inside the stage-1 kernel
  const double* cn = b->obj == ADJ_OBJ_MEAN_PRESSURE ? c_n : nullptr;
  if ((e = launch_adjoint_stage_batch<T>(STAGE_FIN, tl, wl, ln, mm, b->dsa, nm, ablk, wn, a, g2, sig, T(6), T(0.5), g3,
                                         g4, wh, grad_s, st, cn)))
    return hip_fail(e, "ensemble adjoint stage 1");
  return ADJ_OK;
}

int check_batch(const adj_batch* b) {
  if (!b) return fail(ADJ_EINVAL, "ensemble handle is NULL");
  return ADJ_OK;
}

}  // namespace

extern "C" {

size_t adj_batch_table_bytes(int nbox, int nmem, int precision) {
  if (nbox < 1 || nmem < 1 || (precision != ADJ_F64 && precision != ADJ_F32)) return 0;
  return batch_table(nbox, nmem, precision == ADJ_F64).total;
}

int adj_batch_create(adj_batch** out, int nbox, const adj_grid* grids, const adj_objective* obj, int nmem,
                     const int* member_box, const double* member_lambda, void* table, size_t table_bytes) {
  if (!out) return fail(ADJ_EINVAL, "out is NULL");
  *out = nullptr;
  if (nbox < 1 || nmem < 1) return fail(ADJ_EINVAL, "an ensemble needs at least one box and one member");
  if (!grids || !member_box || !member_lambda) return fail(ADJ_EINVAL, "grids, member_box and member_lambda must be non-NULL");
  int r;
  for (int i = 0; i < nbox; ++i) {
    if ((r = check_grid(&grids[i], true))) return fail(r, "box %d: %s", i, g_err.c_str());
    if (grids[i].precision != grids[0].precision) return fail(ADJ_EINVAL, "box %d: every box needs one precision", i);
    if (grids[i].bc_x != grids[0].bc_x) return fail(ADJ_EINVAL, "box %d: every box needs one x boundary", i);
    if (grids[i].ckpt_format != ADJ_CKPT_NATIVE) return fail(ADJ_EINVAL, "box %d: ensembles keep native states", i);
    if (grids[i].time_scheme != ADJ_RK4) return fail(ADJ_EINVAL, "box %d: ensembles march with RK4", i);
    if (grids[i].flux != ADJ_FLUX_SPLIT) return fail(ADJ_EINVAL, "box %d: ensembles take the split-form flux", i);
    if (grids[i].bc_x == ADJ_BC_CHARACTERISTIC)
      return fail(ADJ_EINVAL, "box %d: ensembles take periodic or walled boxes", i);
  }
  const int kind = obj ? obj->kind : ADJ_OBJ_NONE;
  if (kind != ADJ_OBJ_NONE && kind != ADJ_OBJ_MEAN_PRESSURE)
    return fail(ADJ_EINVAL, "ensembles support the mean-pressure objective (kind %d given)", kind);
  for (int m = 0; m < nmem; ++m) {
    if (member_box[m] < 0 || member_box[m] >= nbox) return fail(ADJ_EINVAL, "member %d: box %d out of range", m, member_box[m]);
    if (m && member_box[m] < member_box[m - 1]) return fail(ADJ_EINVAL, "member boxes must be non-decreasing");
    if (!(member_lambda[m] >= 0.0) || !std::isfinite(member_lambda[m]))
      return fail(ADJ_EINVAL, "member %d: lambda must be finite and >= 0", m);
  }
  const int fp64 = grids[0].precision == ADJ_F64;
  const BatchTable tb = batch_table(nbox, nmem, fp64);
  if (!table || (uintptr_t)table % ALIGN) return fail(ADJ_EWORKSPACE, "table must be non-NULL and 256-byte aligned");
  if (table_bytes < tb.total) return fail(ADJ_EWORKSPACE, "table has %zu bytes, needs %zu", table_bytes, tb.total);

  adj_batch* b = new adj_batch;
  b->nbox = nbox;
  b->nmem = nmem;
  b->fp64 = fp64;
  b->wall = grids[0].bc_x == ADJ_BC_SLIP_WALLS;
  b->obj = kind;
  for (int m = 0; m < nmem; ++m) b->lnu |= member_lambda[m] > 0.0;
  b->tile_p = tile_choice(ADJ_PROF_PRIMAL_STAGE, fp64);
  b->tile_a = adjoint_tile_used(fp64, b->wall, b->lnu, tile_choice(ADJ_PROF_ADJOINT_STAGE, fp64));
  int ptx, pty, ptz, atx, aty, atz;
  tile_dims(b->tile_p, ptx, pty, ptz);
  tile_dims(b->tile_a, atx, aty, atz);
  auto tiles = [](const adj_grid& g, int tx, int ty, int tz) {
    return (long long)((g.n[0] + tx - 1) / tx) * ((g.n[1] + ty - 1) / ty) * ((g.n[2] + tz - 1) / tz);
  };
  b->boff.assign(nbox + 1, 0);
  b->sp.assign(nbox + 1, 0);
  b->slb.assign(nbox + 1, 0);
  long long sp = 0, slb = 0;
  for (int i = 0; i < nbox; ++i) {
    const long long N = ncells(&grids[i]);
    b->boff[i + 1] = b->boff[i] + N;
    sp += tiles(grids[i], ptx, pty, ptz);
    slb += (N + RB - 1) / RB;
    b->sp[i + 1] = (int)sp;
    b->slb[i + 1] = (int)slb;
  }
  b->moff.assign(nmem + 1, 0);
  b->sa.assign(nmem + 1, 0);
  b->slm.assign(nmem + 1, 0);
  b->mem_box.assign(member_box, member_box + nmem);
  long long sa = 0, slm = 0;
  for (int m = 0; m < nmem; ++m) {
    const adj_grid& g = grids[member_box[m]];
    const long long N = ncells(&g);
    b->moff[m + 1] = b->moff[m] + N;
    sa += tiles(g, atx, aty, atz);
    slm += (N + RB - 1) / RB;
    b->sa[m + 1] = (int)sa;
    b->slm[m + 1] = (int)slm;
  }
  if (sp > INT32_MAX / 2 || sa > INT32_MAX / 2 || slb > INT32_MAX / 2 || slm > INT32_MAX / 2) {
    delete b;
    return fail(ADJ_ESHAPE, "ensemble too large for one launch");
  }
  // descriptors, written to the caller's device table with blocking copies
  std::vector<char> hb(tb.total, 0);
  for (int i = 0; i < nbox; ++i) {
    if (fp64) {
      const BoxDesc<double> d = box_desc<double>(&grids[i], b->boff[i], b->boff[i], 0.0);
      std::memcpy(hb.data() + tb.box + i * sizeof d, &d, sizeof d);
    } else {
      const BoxDesc<float> d = box_desc<float>(&grids[i], b->boff[i], b->boff[i], 0.0);
      std::memcpy(hb.data() + tb.box + i * sizeof d, &d, sizeof d);
    }
  }
  for (int m = 0; m < nmem; ++m) {
    const int i = member_box[m];
    if (fp64) {
      const BoxDesc<double> d = box_desc<double>(&grids[i], b->boff[i], b->moff[m], member_lambda[m]);
      std::memcpy(hb.data() + tb.mem + m * sizeof d, &d, sizeof d);
    } else {
      const BoxDesc<float> d = box_desc<float>(&grids[i], b->boff[i], b->moff[m], member_lambda[m]);
      std::memcpy(hb.data() + tb.mem + m * sizeof d, &d, sizeof d);
    }
  }
  std::memcpy(hb.data() + tb.sp, b->sp.data(), (nbox + 1) * sizeof(int));
  std::memcpy(hb.data() + tb.sa, b->sa.data(), (nmem + 1) * sizeof(int));
  std::memcpy(hb.data() + tb.slb, b->slb.data(), (nbox + 1) * sizeof(int));
  std::memcpy(hb.data() + tb.slm, b->slm.data(), (nmem + 1) * sizeof(int));
  hipError_t e = hipMemcpy(table, hb.data(), tb.total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "ensemble table upload");
  }
  char* t = (char*)table;
  b->dbox = t + tb.box;
  b->dmem = t + tb.mem;
  b->dsp = (const int*)(t + tb.sp);
  b->dsa = (const int*)(t + tb.sa);
  b->dslb = (const int*)(t + tb.slb);
  b->dslm = (const int*)(t + tb.slm);
  *out = b;
  return ADJ_OK;
}

void adj_batch_destroy(adj_batch* batch) { delete batch; }

long long adj_batch_offset(const adj_batch* batch, int which, int index) {
  if (!batch) return -1;
  if (which == 0) return (index < 0 || index > batch->nbox) ? -1 : batch->boff[index];
  if (which == 1) return (index < 0 || index > batch->nmem) ? -1 : batch->moff[index];
  return -1;
}

size_t adj_batch_workspace_bytes(const adj_batch* batch) { return batch ? batch_ws(batch).total : 0; }

int adj_batch_primal_step(const adj_batch* batch, int nbox, const void* w_n, const void* s, void* w_np1, void* ws,
                          size_t ws_bytes, void* stream) {
  int r;
  if ((r = check_batch(batch))) return r;
  if (nbox < 1 || nbox > batch->nbox) return fail(ADJ_EINVAL, "nbox = %d outside [1, %d]", nbox, batch->nbox);
  if ((r = check_batch_ws(batch, ws, ws_bytes))) return r;
  if (!w_n || !w_np1) return fail(ADJ_EINVAL, "w_n and w_np1 must be non-NULL");
  if (w_n == w_np1) return fail(ADJ_EINVAL, "w_np1 must not alias w_n");
  hipStream_t st = (hipStream_t)stream;
  if (batch->fp64)
    return batch_primal<double>(batch, nbox, (const double*)w_n, (const double*)s, (double*)w_np1, ws, st);
  return batch_primal<float>(batch, nbox, (const float*)w_n, (const float*)s, (float*)w_np1, ws, st);
}

int adj_batch_adjoint_step(const adj_batch* batch, int nmem, const void* w_n, const void* s, const void* wh_np1,
                           const double* c_n, void* wh_n, void* grad_s, void* ws, size_t ws_bytes, void* stream) {
  int r;
  if ((r = check_batch(batch))) return r;
  if (nmem < 1 || nmem > batch->nmem) return fail(ADJ_EINVAL, "nmem = %d outside [1, %d]", nmem, batch->nmem);
  if ((r = check_batch_ws(batch, ws, ws_bytes))) return r;
  if (!w_n || !wh_np1 || !wh_n) return fail(ADJ_EINVAL, "w_n, wh_np1 and wh_n must be non-NULL");
  if (wh_n == wh_np1) return fail(ADJ_EINVAL, "wh_n must not alias wh_np1");
  hipStream_t st = (hipStream_t)stream;
  if (batch->fp64)
    return batch_adjoint<double>(batch, nmem, (const double*)w_n, (const double*)s, (const double*)wh_np1, c_n,
                                 (double*)wh_n, (double*)grad_s, ws, st);
  return batch_adjoint<float>(batch, nmem, (const float*)w_n, (const float*)s, (const float*)wh_np1, c_n,
                              (float*)wh_n, (float*)grad_s, ws, st);
}

int adj_batch_objective_and_grad(const adj_batch* batch, int first, int count, const void* w, const double* weights,
                                 double* J_accum, void* djdw, void* ws, size_t ws_bytes, void* stream) {
  int r;
  if ((r = check_batch(batch))) return r;
  if (first < 0 || count < 1 || first + count > batch->nmem)
    return fail(ADJ_EINVAL, "members [%d, %d) outside [0, %d)", first, first + count, batch->nmem);
  if ((r = check_batch_ws(batch, ws, ws_bytes))) return r;
  if (!w || !weights) return fail(ADJ_EINVAL, "w and weights must be non-NULL");
  if (batch->obj == ADJ_OBJ_NONE) return ADJ_OK;
  const BatchWs L = batch_ws(batch);
  hipError_t e;
  hipStream_t st = (hipStream_t)stream;
  if (batch->fp64)
    e = launch_meanp_batch<double>((const BoxDesc<double>*)batch->dmem, batch->dslm, batch->slm.data(), first, count,
                                   (const double*)w, weights, J_accum, (double*)djdw, (double*)at(ws, L.partials), st);
  else
    e = launch_meanp_batch<float>((const BoxDesc<float>*)batch->dmem, batch->dslm, batch->slm.data(), first, count,
                                  (const float*)w, weights, J_accum, (float*)djdw, (double*)at(ws, L.partials), st);
  return e ? hip_fail(e, "ensemble objective") : ADJ_OK;
}

int adj_batch_energy_vhat(const adj_batch* batch, int nmem, const void* w, const void* wh, double* E, void* ws,
                          size_t ws_bytes, void* stream) {
  int r;
  if ((r = check_batch(batch))) return r;
  if (nmem < 1 || nmem > batch->nmem) return fail(ADJ_EINVAL, "nmem = %d outside [1, %d]", nmem, batch->nmem);
  if ((r = check_batch_ws(batch, ws, ws_bytes))) return r;
  if (!w || !wh || !E) return fail(ADJ_EINVAL, "w, wh and E must be non-NULL");
  const BatchWs L = batch_ws(batch);
  hipError_t e;
  hipStream_t st = (hipStream_t)stream;
  if (batch->fp64)
    e = launch_energy_batch<double>((const BoxDesc<double>*)batch->dmem, batch->dslm, batch->slm.data(), nmem,
                                    (const double*)w, (const double*)wh, (double*)at(ws, L.partials), E, st);
  else
    e = launch_energy_batch<float>((const BoxDesc<float>*)batch->dmem, batch->dslm, batch->slm.data(), nmem,
                                   (const float*)w, (const float*)wh, (double*)at(ws, L.partials), E, st);
  return e ? hip_fail(e, "ensemble energy") : ADJ_OK;
}

// ---------------------------------------------------------------------------------------------
// Reverse step without a caller workspace: the scratch lives in a file-scope device array (one
// copy per GPU, allocated when the code object loads and held until the process ends).  Host code
// never uses the array's name as an address: hipGetSymbolAddress gives each device's own address
// once, with that device current, and that pointer is what the kernels receive as their workspace.
// ---------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[ADJ_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 256;
std::mutex g_scratch_mtx;
void* g_scratch_ptr[MAX_DEVICES] = {};

// This device's address of `scratch` (looked up on the device's first call).
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e;
  if ((e = hipGetDevice(&dev))) return hip_fail(e, "no-alloc scratch: current device");
  if (dev < 0 || dev >= MAX_DEVICES) return fail(ADJ_EHIP, "no-alloc scratch: device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mtx);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)))) return hip_fail(e, "no-alloc scratch: symbol address");
    if (!p || (uintptr_t)p % ALIGN) return fail(ADJ_EHIP, "no-alloc scratch: bad symbol address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ADJ_OK;
}
}  // namespace

int adj_adjoint_step_noalloc(const adj_grid* grid, const void* w_n, const void* s, const void* wh_np1,
                             double lambda, const adj_objective* obj, double c_n, void* wh_n, void* grad_s,
                             void* stream) {
  int r;
  if ((r = check_grid(grid, true))) return r;
  const size_t need = layout(grid).total;
  if (need > (size_t)ADJ_NOALLOC_SCRATCH_BYTES)
    return fail(ADJ_EWORKSPACE,
                "adj_adjoint_step_noalloc: this grid needs %zu bytes of scratch, more than the %zu bytes of the "
                "static scratch array; use adj_adjoint_step with a workspace",
                need, (size_t)ADJ_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  if ((r = scratch_address(&ws))) return r;
  // every scratch region of the reverse step is written before it is read, so nothing needs
  // clearing between calls
  return adjoint_entry(grid, w_n, nullptr, s, wh_np1, lambda, obj, c_n, wh_n, grad_s, ws,
                       (size_t)ADJ_NOALLOC_SCRATCH_BYTES, stream);
}

const char* adj_last_error(void) { return g_err.c_str(); }

const char* adj_version(void) { return "adjns 0.1 gfx950"; }

}  // extern "C"
