/* adjns.h -- C ABI of the MI355X (gfx950) library for the stabilised discrete unsteady adjoint
 * of the compressible Navier-Stokes equations (Talnikar, Wang & Laskowski, GT2016-56689).
 *
 * The method: the primal state w = (rho, rho u1, rho u2, rho u3, rho E) obeys the compressible
 * Navier-Stokes equations with an ideal gas and a source term s (section "Physics", Eq. navier;
 * "Unsteady adjoint", vector and index forms).  A time-averaged objective J = sum_n c_n j(w_n)
 * is differentiated with the discrete adjoint, integrated backwards in time from a zero terminal
 * value ("Unsteady adjoint", terminal condition; "Implementation": discrete adjoint), optionally
 * stabilised by the artificial adjoint viscosity d_l(lambda sigma_1 d_l w^) where sigma_1 is the
 * largest singular value of the adjoint-energy growth matrix M = M1 - M2 ("Stabilizing adjoint
 * equations": Energy Analysis, last equation).
 *
 * Discretisation (identical in every entry point; the defaults below, the options of adj_grid
 * flux, time_scheme and bc_x replace the flux, the time marching or the x boundaries):
 *   - uniform Cartesian cells, n[d] cells over length L[d], dx_d = L[d]/n[d]; periodic in y, z;
 *     x periodic, slip walls (mirror ghost cell, x-momentum odd) or characteristic inlet/outlet;
 *   - residual R(w; s) = -sum_d (F~_{d,+} - F~_{d,-})/dx_d + s, with the convective face flux
 *     r v_d (1, v, H) + P (0, e_d, v_d) built from the face means r, v, H, P of rho, u, E/rho
 *     and p (the kinetic-energy-preserving split form of Kennedy & Gruber, JCP 227, 2008: the
 *     paper's own LES leans on the dissipation of its upwind flux, and a plain average of the two
 *     cell fluxes diverges on under-resolved flows), minus the viscous face flux
 *     (0, sigma_d., u_f . sigma_d. + alpha d_d e): normal face
 *     gradients (phi_R - phi_L)/dx_d, tangential ones the mean of the two cells' central
 *     differences; sigma = mu (grad u + grad u^T) - (2/3) mu (div u) I; alpha = gamma mu / Pr;
 *   - classical RK4 with fixed dt (or the paper's SSP-RK3);
 *   - options: the paper's Roe upwind flux on reconstructed face states (adj_grid.flux) and its
 *     characteristic inlet and outlet (adj_grid.bc_x, w_far).
 *
 * Size limit: a state array (5 N values) must span less than 4 GiB (N < 2^28 / 1.25 cells in FP32,
 * half that in FP64); larger grids are rejected with ADJ_ESHAPE.
 *
 * Memory: every state-sized array is a DEVICE pointer owned by the caller, structure-of-arrays,
 * var-major: a[v*N + (k*ny + j)*nx + i], v = 0..4, N = nx*ny*nz, element type double when
 * grid->precision == ADJ_F64 and float when ADJ_F32.  Scalars marked "device double" are FP64 in
 * device memory in both precisions.  The library never allocates, frees or synchronises: every
 * call enqueues kernels on `stream` (a hipStream_t; NULL = the default stream) and returns.
 * Scratch memory is the caller's `ws` of at least adj_workspace_bytes(grid) bytes, 256-byte
 * aligned; calls that share a `ws` must be ordered on one stream (adj_adjoint_step_noalloc takes
 * its scratch from a static device array instead).
 *
 * Errors: every entry point validates its arguments on the host before launching anything and
 * returns a negative adj_status without touching device memory when they are invalid;
 * adj_last_error() then describes the problem (thread-local).  Launch failures return ADJ_EHIP.
 */
#ifndef ADJNS_H
#define ADJNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum adj_status {
  ADJ_OK = 0,
  ADJ_EINVAL = -1,     /* null pointer, bad enum, non-positive size or parameter */
  ADJ_ESHAPE = -2,     /* grid too small for the requested boundary treatment or objective */
  ADJ_EUNSTABLE = -3,  /* requested dt / lambda outside the explicit stability bound */
  ADJ_ENONFINITE = -4, /* a reduction met a NaN or Inf */
  ADJ_EHIP = -5,       /* a HIP runtime call or kernel launch failed */
  ADJ_EWORKSPACE = -6  /* workspace missing, too small or misaligned */
} adj_status;

enum { ADJ_BC_PERIODIC = 0, ADJ_BC_SLIP_WALLS = 1, ADJ_BC_CHARACTERISTIC = 2 };
enum { ADJ_F64 = 0, ADJ_F32 = 1 };
enum { ADJ_CKPT_NATIVE = 0, ADJ_CKPT_BF16 = 1, ADJ_CKPT_I16 = 2 };
enum { ADJ_RK4 = 0, ADJ_SSPRK3 = 1 };
enum { ADJ_FLUX_SPLIT = 0, ADJ_FLUX_ROE = 1 };
enum {
  ADJ_OBJ_NONE = 0,
  ADJ_OBJ_MEAN_PRESSURE = 1,  /* j = (1/N) sum_cells p                                         */
  ADJ_OBJ_KE_DISSIPATION = 2, /* j = (1/N) sum_cells sigma_ij d_j u_i, central cell gradients     */
  ADJ_OBJ_PT_LOSS_PLANE = 3   /* j = sum_f rho_f (pt_ref - p_t,f) / (pt_ref sum_f rho_f) on the
                                 x-face between cells plane_i-1 and plane_i, face state the mean of
                                 its two cells, p_t = p (1 + (gamma-1)/2 M^2)^(gamma/(gamma-1))
                                 (Eqs. (1)-(3), pressure loss)                                    */
};

/* Grid, gas and scheme.  dt is fixed over a window. */
typedef struct adj_grid {
  int32_t n[3];        /* cells in x, y, z (each >= 1; >= 2 in x with slip walls)           */
  int32_t bc_x;        /* ADJ_BC_PERIODIC, ADJ_BC_SLIP_WALLS, or ADJ_BC_CHARACTERISTIC: open
                          inflow/outflow boundaries at x = 0 and x = L_x (see w_far)           */
  double L[3];         /* box lengths                                                        */
  double gamma;        /* ratio of specific heats                                            */
  double prandtl;      /* Prandtl number; heat conduction coefficient alpha = gamma mu / Pr  */
  double mu;           /* constant dynamic viscosity                                         */
  double dt;           /* time step                                                          */
  int32_t precision;   /* ADJ_F64 or ADJ_F32: element type of states and stencil arithmetic  */
  int32_t ckpt_format; /* ADJ_CKPT_NATIVE, ADJ_CKPT_BF16 or ADJ_CKPT_I16 (the two records:
                          ADJ_F32 only): form of w_n handed to adj_adjoint_step and of ckpt_out
                          written by adj_primal_step (see adj_ckpt_encode)                     */
  double w_ref[5];     /* reference state: every state array holds w - w_ref (all zero = the
                          plain state).  A constant near the mean state keeps FP32 states
                          accurate at low Mach number, where rho E is dominated by the internal
                          energy and rho by its mean: the stored deviations are O(the flow's
                          fluctuations) and lose no digits to the offset, and pressures are
                          formed from them.  The scheme is unchanged; adjoint fields are
                          gradients with respect to the stored variables, the same as those
                          with respect to w.                                                   */
  double nu_weight[3]; /* artificial-viscosity weights of the variable groups (rho, rho u,
                          rho E): the adjoint components of group g are diffused with
                          nu_g = lambda nu_weight[g] sigma_1 (each >= 0; all three 0 means
                          1, 1, 1, the single viscosity of the paper)  [Conclusion: separate
                          adjoint viscosities for rho, rho U, rho E]                           */
  int32_t time_scheme; /* ADJ_RK4 (classical four-stage, the default) or ADJ_SSPRK3, the
                          paper's strong-stability-preserving third-order Runge-Kutta in
                          Shu-Osher form: u1 = w + dt R(w), u2 = 3/4 w + 1/4 (u1 + dt R(u1)),
                          w_next = 1/3 w + 2/3 (u2 + dt R(u2))  [Numerical methods].  Every
                          single-box call follows it, with the exact discrete adjoint of the
                          chosen scheme; ensembles (adj_batch_*) take ADJ_RK4 grids only.       */
  int32_t flux;        /* convective face flux: ADJ_FLUX_SPLIT (the default) takes the face means
                          of rho, u, E/rho and p in the split product form of Kennedy & Gruber,
                          F = r v_d (1, v, H) + P (0, e_d, v_d); ADJ_FLUX_ROE is Roe's
                          approximate Riemann solver, the paper's flux [Numerical methods], on
                          face states reconstructed linearly with central cell gradients,
                          w_l = w_L + (w_R - w_{L-e_d})/4, w_r = w_R - (w_{R+e_d} - w_L)/4:
                          F = (F_d(w_l) + F_d(w_r))/2 - (1/2) sum_k |lam_k| a_k r_k over the
                          acoustic, entropy and shear waves of the Roe average (weights
                          sqrt(rho)).  Ensembles take ADJ_FLUX_SPLIT grids only.                */
  double roe_delta;    /* ADJ_FLUX_ROE: every |lam| is smoothed within delta = roe_delta c~ of
                          zero (Harten: (lam^2 + delta^2)/(2 delta) there), so that the flux is
                          differentiable and its discrete adjoint exists; finite and > 0.  The
                          characteristic boundaries use it too.                                */
  double w_far[2][5];  /* ADJ_BC_CHARACTERISTIC: the far-field conservative states beyond x = 0
                          and beyond x = L_x (rho > 0, p > 0).  Through each boundary face the
                          flux is Roe's inviscid flux between the far-field state and the
                          boundary cell (first order): the characteristics that enter the box
                          carry far-field data and those that leave it interior data, the
                          non-reflecting inlet and outlet of the paper's solver [Numerical
                          methods; Boundary conditions of the adjoint: characteristic
                          boundaries].  Every other stencil sees mirror ghosts beyond x = 0
                          and x = L_x, as with slip walls, except that a Roe reconstruction does
                          not reach into them.  Ensembles take no characteristic grids.        */
} adj_grid;

typedef struct adj_objective {
  int32_t kind;    /* ADJ_OBJ_*                                       */
  int32_t plane_i; /* PT_LOSS_PLANE: 1 <= plane_i <= n[0]-1           */
  double pt_ref;   /* PT_LOSS_PLANE: reference stagnation pressure > 0 */
} adj_objective;

/* Bytes of scratch the caller must pass as `ws` to any call on this grid. */
size_t adj_workspace_bytes(const adj_grid* grid);

/* Bytes of one checkpoint record: the block header (25 FP32 values per 4x4x4 block of cells,
 * padded to a multiple of 256 bytes) followed by 5N 16-bit codes in the state layout (see
 * adj_ckpt_encode; the same size for BF16 and fixed-point codes). */
size_t adj_ckpt_bytes(const adj_grid* grid);

/* One time step of the primal (classical RK4, or SSP-RK3 when grid->time_scheme says so)
 * [Physics; Numerical methods (time marching)].
 *   w_n   in : state at step n                     (state-sized)
 *   s     in : source field, or NULL for s = 0      (state-sized)
 *   w_np1 out: state at step n+1 (must not alias w_n)
 *   ckpt_out : NULL, or an adj_ckpt_bytes() record receiving the encoding of w_np1 (BF16
 *              codes, fixed-point codes when ckpt_format is ADJ_CKPT_I16; precision ADJ_F32
 *              only)  [Implementation: checkpointing] */
int adj_primal_step(const adj_grid* grid, const void* w_n, const void* s, void* w_np1, void* ckpt_out,
                    void* ws, size_t ws_bytes, void* stream);

/* adj_primal_step (or adj_primal_step_stages when stages_out is non-NULL) that also accumulates the
 * objective of its input and of its new state: J_accum (device double) += weight_in * j(w_n) +
 * weight * j(w_np1)  [Eqs. (1)-(3); the time-averaged objective is the sum of such terms over the
 * steps of a window].  Where a stage kernel already stages the state, the objective rides in it
 * (per-tile partials in the workspace, then a fixed-order fold): the mean pressure of w_np1 in the
 * final stage (RK4, split flux, no characteristic boundaries), the dissipation of w_n in stage 1
 * (periodic or slip-wall x boundaries); otherwise the objective kernel runs before or after the
 * step.  obj NULL, kind NONE or both weights 0: plain step. */
int adj_primal_step_obj(const adj_grid* grid, const void* w_n, const void* s, void* w_np1, void* ckpt_out,
                        void* stages_out, const adj_objective* obj, double weight_in, double weight, double* J_accum,
                        void* ws, size_t ws_bytes, void* stream);

/* One reverse step of the discrete adjoint with artificial viscosity (below for RK4; an
 * ADJ_SSPRK3 grid reverses its three Shu-Osher stages the same way, see time_scheme)  [Unsteady adjoint:
 * terminal condition and backward integration; Implementation; Stabilizing adjoint equations]:
 *   recompute the stage states W1 = w_n, W2, W3, W4; nu = lambda sigma_1(w_n) held over the step;
 *   k^4 = dt/6 a, g4 = (J_R(W4)^T + L_nu) k^4; k^3 = dt/3 a + dt g4, g3 = ...;
 *   k^2 = dt/3 a + dt/2 g3, g2 = ...; k^1 = dt/6 a + dt/2 g2, g1 = ...;
 *   w^_n = a + g1 + g2 + g3 + g4 + c_n dj/dw(w_n);  grad_s += k^1 + k^2 + k^3 + k^4,
 * where a = w^_{n+1} and (L_nu q)_i = sum_d [nu_{i+1/2}(q_{i+1}-q_i) - nu_{i-1/2}(q_i-q_{i-1})]/dx_d^2
 * with face nu the mean of its cells (no artificial flux through slip walls), applied to each
 * component with the nu of its variable group (grid->nu_weight).
 *   w_n     in : primal state at step n (state-sized), or a record when ckpt_format says so
 *   s       in : source field or NULL
 *   wh_np1  in : adjoint at step n+1 (state-sized)
 *   lambda  in : artificial-viscosity scale, units length^2 (>= 0; 0 = plain adjoint)
 *   obj, c_n   : objective injected with weight c_n (obj NULL or kind NONE or c_n == 0: none)
 *   wh_n   out : adjoint at step n (must not alias wh_np1)
 *   grad_s inout: accumulated dJ/ds (+=), or NULL */
int adj_adjoint_step(const adj_grid* grid, const void* w_n, const void* s, const void* wh_np1,
                     double lambda, const adj_objective* obj, double c_n, void* wh_n, void* grad_s,
                     void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory, not even a workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): adj_adjoint_step with its
 * scratch taken from a static device array of ADJ_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on every GPU it runs on until the process ends (64 MiB: grids up to 64^3 cells in FP64
 * or FP32; adj_workspace_bytes(grid) must not exceed it).  Same arguments and results as
 * adj_adjoint_step without ws / ws_bytes; it allocates nothing (the device's address of the array
 * is looked up once, on that device's first call).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other host threads) race and give
 * undefined results; order them on one stream.  Returns ADJ_EWORKSPACE when the grid needs more
 * scratch than the array holds, the other codes as adj_adjoint_step. */
#define ADJ_NOALLOC_SCRATCH_BYTES (64u << 20)
int adj_adjoint_step_noalloc(const adj_grid* grid, const void* w_n, const void* s, const void* wh_np1, double lambda,
                             const adj_objective* obj, double c_n, void* wh_n, void* grad_s, void* stream);

/* Store-stages schedule (for windows whose stage states fit in memory): adj_primal_step_stages
 * is adj_primal_step that also writes the stage states of the step into stages_out (3
 * consecutive state-sized arrays: W2, W3, W4 for RK4; u1, u2 and an unused third for SSP-RK3);
 * adj_adjoint_step_stages is adj_adjoint_step that reads them from `stages` instead of
 * recomputing them from w_n.  Native states only. */
int adj_primal_step_stages(const adj_grid* grid, const void* w_n, const void* s, void* w_np1, void* stages_out,
                           void* ws, size_t ws_bytes, void* stream);
int adj_adjoint_step_stages(const adj_grid* grid, const void* w_n, const void* stages, const void* s,
                            const void* wh_np1, double lambda, const adj_objective* obj, double c_n, void* wh_n,
                            void* grad_s, void* ws, size_t ws_bytes, void* stream);

/* out[c] = scale * sigma_1(c): largest singular value of M = M1 - M2 at every cell, from central
 * differences of rho, u, p, a = sqrt((gamma-1)/gamma) c, b = c/sqrt(gamma)  [Energy Analysis].
 *   w in: state; out: N elements of the grid's precision. */
int adj_growth_sigma1(const adj_grid* grid, const void* w, double scale, void* out, void* stream);

/* Objective j(w) and its gradient  [Eqs. (1)-(3); time-averaged objective]:
 *   J_accum (device double, may be NULL): J_accum += weight * j(w)
 *   djdw    (state-sized, may be NULL)   : djdw += weight * dj/dw(w) */
int adj_objective_and_grad(const adj_grid* grid, const adj_objective* obj, const void* w, double weight,
                           double* J_accum, void* djdw, void* ws, size_t ws_bytes, void* stream);

/* Adjoint energy E = (1/dV) sum_cells |T^{-T} w^|^2 in symmetrised variables  [Symmetrization:
 * w^ = T^T v^; Energy Analysis: E_v^]; E is a device double (overwritten), FP64 accumulation. */
int adj_energy_vhat(const adj_grid* grid, const void* w, const void* wh, double* E, void* ws,
                    size_t ws_bytes, void* stream);

/* out (device double) = sum over all 5N entries of a*b, FP64 accumulation in a fixed order. */
int adj_dot(const adj_grid* grid, const void* a, const void* b, double* out, void* ws, size_t ws_bytes,
            void* stream);

/* Checkpoint codec (ADJ_F32 states), block-scaled with a plane predictor: the grid is cut
 * into 4x4x4 blocks of cells (ragged at the far ends), block b = (bz*nby + by)*nbx + bx,
 * nbd = ceil(n[d]/4).  Per block and variable v, over the block's present cells with centred
 * local coordinates c_d = l_d - (n'_d - 1)/2 (n'_d present cells along d):
 *   a = S_0/n', g_d = S_d / sum c_d^2 (0 when n'_d = 1): the least-squares plane, from the FP64
 *     sums S_0 = sum w and S_d = sum c_d w (each column z = 0..3 accumulated by fma, the columns
 *     added pairwise along x, then the rows pairwise along y), rounded to FP32;
 *   P(a) = fma(g_z, c_z, fma(g_y, c_y, fma(g_x, c_x, a))); r0 = w - P(a);
 *   a' = a + (max r0 + min r0)/2, s = (max r0 - min r0)/2 (1 when the range is empty);
 *   t = (w - P(a'))/s in FP32 with IEEE division (|t| <= 1 up to rounding);
 *   BF16 codes (ckpt_format ADJ_CKPT_BF16, and NATIVE grids calling the codec directly):
 *     code = bf16_round_nearest_even(t), decode w' = fma(s, code, P(a'));
 *   fixed-point codes (ADJ_CKPT_I16): code = the int16 nearest (ties to even) to the FP32
 *     product t * 32767, clamped to +-32767; decode w' = fma(s, code * h, P(a')) with
 *     h = 1/32767 rounded to FP32 and the product rounded to FP32.  The BF16 code keeps 2^-9
 *     of each value's own magnitude; the fixed-point code keeps s/65534 whatever the value
 *     (128 times finer at the ends of the range), which matters for fields whose blocks are
 *     perturbations at the grid scale.
 * Record (adj_ckpt_bytes): header of 25 floats per block, header[(b*5 + v)*5 + {0..4}] =
 * a', g_x, g_y, g_z, s, padded to a multiple of 256 bytes, then the 5N codes in the state
 * layout.  Records must be 64-byte aligned  [Implementation: checkpointing; the precision form
 * keeps the primal snapshots in BF16 under per-variable scaling; the fixed-point codes are an
 * alternative of the same size]. */
int adj_ckpt_encode(const adj_grid* grid, const float* w, void* ckpt, void* ws, size_t ws_bytes, void* stream);
int adj_ckpt_decode(const adj_grid* grid, const void* ckpt, float* w, void* stream);

/* Operator-level entry points (used to check single stages):
 *   adj_residual: R = R(w; s)
 *   adj_vjp     : out = J_R(W)^T kh + (nu ? L_nu kh : 0), nu an N-element field or NULL */
int adj_residual(const adj_grid* grid, const void* w, const void* s, void* R, void* stream);
int adj_vjp(const adj_grid* grid, const void* W, const void* kh, const void* nu, void* out, void* stream);

/* Instrumentation.  While enabled, every kernel the library launches is bracketed by a pair of
 * HIP events recorded on the same stream, grouped by class; adj_profile_read waits for the
 * recorded events and returns the summed kernel time (milliseconds) and the launch count of one
 * class.  adj_profile_enable(1) clears earlier records and starts recording, adj_profile_enable(0)
 * stops recording and keeps the records; not thread-safe (one host thread). */
enum {
  ADJ_PROF_ADJOINT_STAGE = 0, /* reverse-stage gather kernels                   */
  ADJ_PROF_PRIMAL_STAGE = 1,  /* primal stage kernels (also recomputation)      */
  ADJ_PROF_SIGMA1 = 2,        /* growth-matrix singular value                   */
  ADJ_PROF_OBJECTIVE = 3,     /* objective values and gradients                 */
  ADJ_PROF_CODEC = 4,         /* checkpoint encode / decode                     */
  ADJ_PROF_REDUCE = 5,        /* energy and inner products                      */
  ADJ_PROF_ROE_PRIMAL = 6,    /* Roe convective terms of primal stages          */
  ADJ_PROF_ROE_ADJOINT = 7,   /* its transpose in reverse stages                */
  ADJ_PROF_BOUNDARY = 8,      /* characteristic boundary fluxes and transposes  */
  ADJ_PROF_NCLASS = 9
};
int adj_profile_enable(int on);
int adj_profile_read(int kernel_class, double* total_ms, long long* launches);

/* Launch configuration of the two stencil kernel classes (ADJ_PROF_ADJOINT_STAGE and
 * ADJ_PROF_PRIMAL_STAGE), per precision: the output tile each work-group covers.  Process-wide;
 * set it before enqueuing work that should use it (the autotuner does).  adj_get_tile returns
 * the tile id or a negative status. */
enum {
  ADJ_TILE_16x4x4 = 0,
  ADJ_TILE_32x4x2 = 1,
  ADJ_TILE_32x4x4 = 2,
  ADJ_TILE_32x8x2 = 3,
  ADJ_TILE_32x8x4 = 4,
  ADJ_TILE_16x8x8 = 5,
  ADJ_NTILES = 6
};
int adj_set_tile(int kernel_class, int precision, int tile);
int adj_get_tile(int kernel_class, int precision);
/* The tile a launch of `kernel_class` actually uses when `tile` is selected, for the boundary
 * (bc_x, ADJ_BC_*) and lambda variant (lnu: 1 when a lambda term is applied): a reverse-stage
 * tile whose shared-memory footprint exceeds a work-group's 160 KiB (the largest FP64 tiles)
 * runs as ADJ_TILE_16x4x4 instead.  Returns the tile id or a negative status. */
int adj_tile_launched(int kernel_class, int precision, int bc_x, int lnu, int tile);

/* Explicit stability of a step from state w, three numbers written to out (device FP64[3]):
 *   out[0] = dt max_cells sum_d (|u_d| + c)/dx_d                       convective
 *   out[1] = dt max_cells max(4 mu/3, alpha)/rho sum_d 4/dx_d^2         viscous and heat conduction
 *   out[2] = dt lambda max_g w_g max_cells sigma_1 sum_d 4/dx_d^2       artificial viscosity
 * (w_g: grid->nu_weight).  The central scheme's convective eigenvalues lie on the imaginary axis
 * and its diffusive ones on the negative real axis; classical RK4 is stable there for |z| up to
 * ADJ_RK4_IMAG_BOUND and ADJ_RK4_REAL_BOUND, SSP-RK3 (amplification 1 + z + z^2/2 + z^3/6) up to
 * ADJ_SSPRK3_IMAG_BOUND (sqrt 3) and ADJ_SSPRK3_REAL_BOUND.  Each number bounds its part of the
 * spectrum alone (a necessary condition; the Roe flux's dissipation moves its convective
 * eigenvalues into the left half-plane)  [Numerical methods: explicit Runge-Kutta time marching].
 * Uses the workspace; asynchronous. */
#define ADJ_RK4_IMAG_BOUND 2.8284
#define ADJ_RK4_REAL_BOUND 2.7853
#define ADJ_SSPRK3_IMAG_BOUND 1.7320
#define ADJ_SSPRK3_REAL_BOUND 2.5127
int adj_stability(const adj_grid* grid, const void* w, double lambda, double* out, void* ws, size_t ws_bytes,
                  void* stream);
/* adj_stability, then waits for the stream: ADJ_EUNSTABLE when a number exceeds the bound of the
 * grid's time scheme, ADJ_OK otherwise; out_host (NULL or host FP64[3]) receives the numbers. */
int adj_check_stable(const adj_grid* grid, const void* w, double lambda, double* out_host, void* ws,
                     size_t ws_bytes, void* stream);
/* Waits for the stream, then ADJ_ENONFINITE when a reduction on the current device (J, E_v^, inner
 * products, plane sums) produced NaN or Inf since the previous call, ADJ_OK otherwise; clears the
 * indication. */
int adj_check_status(void* stream);

/* ---------------------------------------------------------------------------------------------
 * Ensembles: many independent boxes (each its own adj_grid: size, dt, viscosity) and many adjoint
 * sweeps ("members") in one launch per RK stage, the batched form of the calls above.  A member
 * is one reverse sweep over the trajectory of its box with its own lambda, so several members of
 * one box form a lambda sweep that recomputes the box's stage states once.
 *
 * Packed layout: ensemble arrays hold box after box (member after member), each in the
 * single-box layout above.  State arrays (w, s) are packed over boxes: box b occupies elements
 * [5 o_b, 5 o_{b+1}) with o_b = adj_batch_offset(batch, 0, b); adjoint arrays (w^, grad_s, dJ/dw)
 * are packed over members with offsets adj_batch_offset(batch, 1, m).  A call that names
 * `nbox` / `nmem` covers boxes [0, nbox) / members [0, nmem) only (ordering boxes by decreasing
 * window length makes the live part of a window of uneven lengths such a prefix), so arrays need
 * only hold that prefix.  Per-member FP64 scalars (weights, J, E) are device arrays indexed by
 * member.  Every box shares precision and x boundary; states are stored natively.  The tile
 * shapes in force when the ensemble is created (adj_set_tile) are the ones its launches use.
 *
 *   adj_batch_table_bytes : device bytes of the ensemble's descriptor table
 *   adj_batch_create      : validates, writes the table into the caller's device memory `table`
 *                           (256-byte aligned, blocking copy: call outside graph capture) and
 *                           returns a host handle; member_box non-decreasing; obj NULL, NONE or
 *                           MEAN_PRESSURE.  The table must outlive the handle.
 *   adj_batch_destroy     : frees the host handle
 *   adj_batch_offset      : which = 0 boxes, 1 members; index in [0, count] (count = the total)
 *   adj_batch_workspace_bytes : scratch for every ensemble call (stage states of all boxes, stage
 *                           adjoints of all members, sigma_1, partial sums)
 *   adj_batch_primal_step : one RK4 step of boxes [0, nbox)                (adj_primal_step)
 *   adj_batch_adjoint_step: one reverse RK4 step of members [0, nmem), recomputing the stage
 *                           states of their boxes; nu = lambda_m sigma_1(w_n); then
 *                           w^_n += c_n[m] dj/dw(w_n) when c_n (device double, per member) is
 *                           non-NULL; grad_s (member-packed) += the source gradient if non-NULL
 *                           (adj_adjoint_step, member by member)
 *   adj_batch_objective_and_grad : members [first, first + count): J_accum[m] += weights[m] j(w of
 *                           the member's box), dJ/dw (member-packed) += weights[m] dj/dw; either
 *                           output may be NULL                             (adj_objective_and_grad)
 *   adj_batch_energy_vhat : E[m] = adjoint energy of member m's w^ at its box's state w, members
 *                           [0, nmem)                                      (adj_energy_vhat)
 * Each member's fields equal those of the single-box calls bit for bit; FP64 scalars agree to
 * rounding (the partial sums run in another order). */
typedef struct adj_batch adj_batch;
size_t adj_batch_table_bytes(int nbox, int nmem, int precision);
int adj_batch_create(adj_batch** out, int nbox, const adj_grid* grids, const adj_objective* obj, int nmem,
                     const int* member_box, const double* member_lambda, void* table, size_t table_bytes);
void adj_batch_destroy(adj_batch* batch);
long long adj_batch_offset(const adj_batch* batch, int which, int index);
size_t adj_batch_workspace_bytes(const adj_batch* batch);
int adj_batch_primal_step(const adj_batch* batch, int nbox, const void* w_n, const void* s, void* w_np1, void* ws,
                          size_t ws_bytes, void* stream);
int adj_batch_adjoint_step(const adj_batch* batch, int nmem, const void* w_n, const void* s, const void* wh_np1,
                           const double* c_n, void* wh_n, void* grad_s, void* ws, size_t ws_bytes, void* stream);
int adj_batch_objective_and_grad(const adj_batch* batch, int first, int count, const void* w, const double* weights,
                                 double* J_accum, void* djdw, void* ws, size_t ws_bytes, void* stream);
int adj_batch_energy_vhat(const adj_batch* batch, int nmem, const void* w, const void* wh, double* E, void* ws,
                          size_t ws_bytes, void* stream);

const char* adj_last_error(void);
const char* adj_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ADJNS_H */
