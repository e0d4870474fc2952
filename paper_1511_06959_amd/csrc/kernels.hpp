// kernels.hpp -- launchers of the gfx950 kernels (host-side declarations).
#pragma once
#include "common.hpp"
#include "prof.hpp"

namespace adjns {

enum { STAGE_RES = 0, STAGE_LIN = 1, STAGE_FIN = 2, STAGE_AFF = 3 };  // primal stage modes
enum { STAGE_VJP = 0 };                                  // adjoint stage modes (STAGE_FIN shared)

// STAGE_AFF: out = ca * wn + cb * W + cR * R(W; s)  (the SSP-RK3 stages)
// conv = 0: R without the split-form convective flux (the Roe option adds its own afterwards)
// jpart (STAGE_FIN or STAGE_LIN, may be NULL): receives one FP64 partial per tile (primal_tiles of
// them): for STAGE_FIN the sum of the pressures of the stage output over the tile's cells (the
// mean-pressure objective of the step's new state), for STAGE_LIN the sum of the viscous dissipation
// of the staged state W (in stage 1, W = w_n: the dissipation objective of the step's own state)
template <typename T>
hipError_t launch_primal_stage(int mode, const Consts<T>& c, const T* W, const T* wn, const T* s, const T* W2,
                               const T* W3, T cR, T* out, hipStream_t st, T ca = T(0), T cb = T(0), int conv = 1,
                               double* jpart = nullptr);
template <typename T>
int primal_tiles(const Consts<T>& c);
// dst = beta dst + alpha (sum of the n partials), in a fixed order (one work-group)
hipError_t launch_fold(const double* partials, int n, double* dst, double alpha, double beta, hipStream_t st);

// SSP-RK3 reverse step, after the three stage transposes g3 (at u2), g2 (at u1), g1 (at w_n):
// rk3_mid:     h = g2 + g3/4                               (in place of g2; k^1 = dt/6 a + dt h)
// rk3_combine: w^_n = a + g1 + h + 3/4 g3,  grad_s += dt a + dt h + dt/4 g3 (grad_s may be NULL)
template <typename T>
hipError_t launch_rk3_mid(T* g2, const T* g3, long long n, hipStream_t st);
template <typename T>
hipError_t launch_rk3_combine(const T* a, const T* g1, const T* h, const T* g3, T dt, T* wh, T* grad_s, long long n,
                              hipStream_t st);

// conv = 0: without the transpose of the split-form convective flux
// objw (STAGE_FIN only): weight c_n of the mean-pressure objective, whose c_n dj/dw(w_n) is added to
// w^_n at each cell (0: none)
template <typename T>
hipError_t launch_adjoint_stage(int mode, const Consts<T>& c, const T* W, const T* a, const T* gnext, const T* nu,
                                T ca, T cg, const T* g3, const T* g4, T* out, T* grad_s, hipStream_t st, int conv = 1,
                                double objw = 0.0);

// Roe flux option: the Roe convective flux F of every face (roe.hip), added after the stage
// kernel (launched with conv = 0) that wrote `out` from the same W:
//   roe_primal:  out += coef * (-sum_d (F_{d,+} - F_{d,-}) / dx_d)
//   roe_adjoint: out += J_F(W)^T kh,  kh = ca a + cg gnext (gnext may be NULL)
// (open: characteristic boundaries in x, whose faces these kernels leave alone)
template <typename T>
hipError_t launch_roe_primal(const Consts<T>& c, T roe_delta, int open, const T* W, T coef, T* out, hipStream_t st);
template <typename T>
hipError_t launch_roe_adjoint(const Consts<T>& c, T roe_delta, int open, const T* W, const T* a, const T* gnext, T ca,
                              T cg, T* out, hipStream_t st);
// Characteristic boundaries in x: the flux the stage kernels evaluated through the two boundary
// faces (a slip-wall mirror pair; split: whether they included the split-form convective flux)
// replaced by Roe's flux against the far-field states w_far (2 x 5 conservative values), after
// the stage kernel (and Roe kernel) that wrote `out`:
//   char_primal:  out += coef * (boundary-face flux difference) / dx at the boundary cells
//   char_adjoint: out += its transpose applied to kh = ca a + cg gnext
template <typename T>
hipError_t launch_char_primal(const Consts<T>& c, T roe_delta, int split, const double* w_far, const T* W, T coef,
                              T* out, hipStream_t st);
template <typename T>
hipError_t launch_char_adjoint(const Consts<T>& c, T roe_delta, int split, const double* w_far, const T* W,
                               const T* a, const T* gnext, T ca, T cg, T* out, hipStream_t st);

// out[c] = scale * sigma_1(w) at every cell
template <typename T>
hipError_t launch_sigma1(const Consts<T>& c, const T* w, T scale, T* out, hipStream_t st);

// Reductions write FP64 per-block partials to `partials` and a single-block pass folds them in a
// fixed order:  *dst = beta * (*dst) + alpha * sum   (beta 0 overwrites, 1 accumulates).
template <typename T>
hipError_t launch_dot(const Consts<T>& c, const T* a, const T* b, double* partials, double* dst, double alpha,
                      double beta, hipStream_t st);
template <typename T>
hipError_t launch_energy_vhat(const Consts<T>& c, const T* w, const T* wh, double* partials, double* dst,
                              hipStream_t st);
// dst[0..2] = (s_conv, s_visc, s_art) x the maxima over cells of the convective rate
// sum_d (|u_d| + c)/dx_d, the viscous rate max(4/3, gamma/Pr)(mu/rho) sum_d 4/dx_d^2 and sigma1
// (sigma1 may be NULL: 0); partials holds 3 MAX_PARTIALS values
template <typename T>
hipError_t launch_stability(const Consts<T>& c, const T* w, const T* sigma1, double s_conv, double s_visc,
                            double s_art, double* partials, double* dst, hipStream_t st);
// copies the device's non-finite indication of the reductions to *flag and clears it (synchronous)
hipError_t read_clear_nonfinite(unsigned int* flag);

// objective kinds follow adjns.h; scratch holds 4 doubles of intermediate plane sums
template <typename T>
hipError_t launch_objective(const Consts<T>& c, int kind, int plane_i, double pt_ref, const T* w, double weight,
                            double* J_accum, T* djdw, double* partials, double* scratch, hipStream_t st);

// Ensemble launchers (packed arrays, work-group offsets `start` on the device; see BoxDesc).
// The stencil launches cover boxes / members [0, n) in nblocks work-groups of the given tile.
void tile_dims(int tile, int& tx, int& ty, int& tz);
int adjoint_tile_used(int fp64, int wall, int lnu, int tile);  // tile after the LDS fit
template <typename T>
hipError_t launch_primal_stage_batch(int mode, int tile, const BoxDesc<T>* boxes, const int* start, int nbox,
                                     int nblocks, const T* W, const T* wn, const T* s, const T* W2, const T* W3,
                                     T cfac, T* out, hipStream_t st);
// cn (STAGE_FIN, may be NULL): per-member weights of the mean-pressure objective (see objw)
template <typename T>
hipError_t launch_adjoint_stage_batch(int mode, int tile, int wall, int lnu, const BoxDesc<T>* mems, const int* start,
                                      int nmem, int nblocks, const T* W, const T* a, const T* gnext, const T* sigma1,
                                      T da, T mg, const T* g3, const T* g4, T* out, T* grad_s, hipStream_t st,
                                      const double* cn = nullptr);
template <typename T>
hipError_t launch_sigma1_batch(const BoxDesc<T>* boxes, const int* start, int nbox, int nblocks, const T* w, T* out,
                               hipStream_t st);
// members [first, first + count); start_host mirrors start on the host
template <typename T>
hipError_t launch_meanp_batch(const BoxDesc<T>* mems, const int* start, const int* start_host, int first, int count,
                              const T* w, const double* wgt, double* J_accum, T* djdw, double* partials,
                              hipStream_t st);
template <typename T>
hipError_t launch_energy_batch(const BoxDesc<T>* mems, const int* start, const int* start_host, int count, const T* w,
                               const T* wh, double* partials, double* E, hipStream_t st);

// block-scaled checkpoint codec (BF16 codes, or 16-bit fixed-point codes when i16); header = 25
// floats (plane a, g_x, g_y, g_z and scale s) x 5 per 4x4x4 block
hipError_t launch_ckpt_encode(const Consts<float>& c, const float* w, float* header, uint16_t* codes, bool i16,
                              hipStream_t st);
hipError_t launch_ckpt_decode(const Consts<float>& c, const float* header, const uint16_t* codes, float* w, bool i16,
                              hipStream_t st);

}  // namespace adjns
