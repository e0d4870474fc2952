// aux.hip -- gfx950 kernels for the growth-matrix singular value sigma_1, the objectives and their
// gradients, the FP64 reductions (adjoint energy, inner products) and the BF16 checkpoint codec.
#include "kernels.hpp"

namespace adjns {

namespace {

// ------------------------------------------------------------------------------------------
// Deterministic FP64 reductions: fixed grid, grid-stride per-thread sums, LDS tree per block,
// then one block folds the per-block partials in index order.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
#pragma unroll
  for (int o = RB / 2; o > 0; o >>= 1) {
    __syncthreads();
    if (t < o) sh[t] += sh[t + o];
  }
  __syncthreads();
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Sum over a work-group of NTH threads (a multiple of 64, at most 64 wavefronts), valid in thread
// 0 only: a butterfly within each 64-lane wavefront, then the wavefront sums, in wavefront order,
// by the same butterfly in wavefront 0.  A fixed order: the result does not depend on timing.  sh
// holds NTH / 64 values.
template <int NTH>
__device__ __forceinline__ double block_sum_n(double v, double* sh) {
  static_assert(NTH % 64 == 0 && NTH <= 64 * 64, "block_sum_n: whole wavefronts, at most 64");
  constexpr int NW = NTH / 64;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (wv == 0) {
    r = lane < NW ? sh[lane] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
  }
  return r;
}

inline int reduce_blocks(long long n) {
  long long b = (n + RB - 1) / RB;
  if (b > MAX_PARTIALS) b = MAX_PARTIALS;
  return (int)(b < 1 ? 1 : b);
}

// Set (never cleared by a kernel) when a reduction's result is NaN or Inf; per device, zero when
// the library is loaded; read and cleared by read_clear_nonfinite (adj_check_status).
__device__ unsigned int g_nonfinite = 0;

__device__ __forceinline__ void note_nonfinite(double x) {
  if (!isfinite(x)) __hip_atomic_fetch_or(&g_nonfinite, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// partials has `nsets` consecutive arrays of `nblk` values; dst[s] = beta dst[s] + alpha[s] sum_s
// Each thread adds the values i = t, t + RB, t + 2 RB, ... in that order; it issues their loads
// FOLD_BATCH at a time, so that the memory latency is paid once per batch (a fold over the
// per-tile partials of a large grid holds 10^5 values), and the order of the additions, so the
// result, is the same as one load at a time.
constexpr int FOLD_BATCH = 16;

__global__ __launch_bounds__(RB) void k_fold(const double* __restrict__ partials, int nblk, int nsets,
                                             double* __restrict__ dst, double alpha, double beta) {
  __shared__ double sh[RB];
  for (int s = 0; s < nsets; ++s) {
    const double* __restrict__ p = partials + (long long)s * nblk;
    double v = 0.0;
    int i = threadIdx.x;
    for (; i + (FOLD_BATCH - 1) * RB < nblk; i += FOLD_BATCH * RB) {
      double q[FOLD_BATCH];
#pragma unroll
      for (int k = 0; k < FOLD_BATCH; ++k) q[k] = p[i + k * RB];
#pragma unroll
      for (int k = 0; k < FOLD_BATCH; ++k) v += q[k];
    }
    for (; i < nblk; i += RB) v += p[i];
    const double tot = block_sum(v, sh);
    if (threadIdx.x == 0) {
      dst[s] = beta * dst[s] + alpha * tot;
      note_nonfinite(dst[s]);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(RB) void k_dot_partial(const T* __restrict__ a, const T* __restrict__ b, long long n,
                                                    double* __restrict__ partials) {
  __shared__ double sh[RB];
  double v = 0.0;
  for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < n; i += (long long)gridDim.x * RB)
    v += (double)a[i] * (double)b[i];
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Primitive quantities of a cell (or its wall mirror image), in FP64.
template <typename T>
__device__ __forceinline__ Q64 load_q64(const Consts<T>& c, const T* __restrict__ w, long long gi, int mirror,
                                        double gamma) {
  const long long N = c.N;
  return q64_of(c, w[gi], w[N + gi], w[2 * N + gi], w[3 * N + gi], w[4 * N + gi], mirror, gamma);
}

// ------------------------------------------------------------------------------------------
// Adjoint energy: v^ = T^{-T} w^ per cell (closed form from S and V)
//   q^_rho = w^_1 + u.w^_m + |u|^2/2 w^_E, q^_u = rho (w^_m + u w^_E), q^_p = w^_E/(gamma-1)
//   v^_1 = (rho/b) q^_rho + rho b q^_p, v^_{2..4} = q^_u, v^_5 = rho a q^_p
// [Symmetrization: S, V, T = S V, w^ = T^T v^; Energy Analysis: E_v^]
// ------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double vhat_sq(const Consts<T>& c, const T* __restrict__ w, const T* __restrict__ wh,
                                          const long long i, const double g, const double sa, const double sb) {
  const long long N = c.N;
  const Q64 q = load_q64(c, w, i, 0, g);
  const double cs = sqrt(g * q.p * q.ri);
  const double a = sa * cs, b = sb * cs;
  double h[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) h[k] = (double)wh[k * N + i];
  const double usq = q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2];
  const double qr = h[0] + q.u[0] * h[1] + q.u[1] * h[2] + q.u[2] * h[3] + 0.5 * usq * h[4];
  const double qp = h[4] / (g - 1.0);
  const double v1 = (q.rho / b) * qr + q.rho * b * qp;
  const double v5 = q.rho * a * qp;
  double s = v1 * v1 + v5 * v5;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double qu = q.rho * (h[1 + k] + q.u[k] * h[4]);
    s += qu * qu;
  }
  return s;
}

template <typename T>
__global__ __launch_bounds__(RB) void k_energy_partial(Consts<T> c, const T* __restrict__ w,
                                                       const T* __restrict__ wh, double* __restrict__ partials) {
  __shared__ double sh[RB];
  const double g = (double)c.gamma;
  const double sa = sqrt((g - 1.0) / g), sb = 1.0 / sqrt(g);
  const long long N = c.N;
  double v = 0.0;
  for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < N; i += (long long)gridDim.x * RB)
    v += vhat_sq(c, w, wh, i, g, sa, sb);
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// ------------------------------------------------------------------------------------------
// sigma_1: M = M1 - M2 from central differences [Energy Analysis, printed M1 and M2], then
// sigma_1 = sqrt(lambda_max(M^T M)).
// ------------------------------------------------------------------------------------------
template <typename T>
struct QS {
  T rho, u[3], p, a, b;
};

template <typename T>
__device__ __forceinline__ QS<T> load_qs(const Consts<T>& c, const T* __restrict__ w, int gx, int gy, int gz) {
  int mirror, real;
  const long long gi = box_cell(c.nx, c.ny, c.nz, c.wall, gx, gy, gz, mirror, real);
  const long long N = c.N;
  QS<T> q;
  // stored deviations w - wref
  q.rho = w[gi] + c.wref[0];
  T m1 = w[N + gi] + c.wref[1];
  if (mirror) m1 = -m1;
  const T ri = recip(q.rho);
  q.u[0] = m1 * ri;
  q.u[1] = (w[2 * N + gi] + c.wref[2]) * ri;
  q.u[2] = (w[3 * N + gi] + c.wref[3]) * ri;
  const T g = c.gamma;
  // p = (gamma-1)((Ed - K) + wref_E), Ed = rho E - wref_E the stored deviation
  q.p = (g - T(1)) * ((w[4 * N + gi] - T(0.5) * q.rho * (q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2])) +
                      c.wref[4]);
  const T cs = sqrt(g * q.p * ri);
  q.a = sqrt((g - T(1)) / g) * cs;  // the constant factors are common to every call of a thread
  q.b = cs * recip(sqrt(g));
  return q;
}

// Largest eigenvalue of a symmetric positive semidefinite 5x5 matrix A (destroyed): Householder
// reduction to tridiagonal form T (Golub & Van Loan, section 8.3.1), then bisection on
// [max_i T_ii, Gershgorin bound] with the leading principal minors of x I - T, which are all
// positive exactly when x exceeds every eigenvalue.  The iteration count is fixed (the bracket
// starts no wider than 2 lambda_max), so every lane of a wavefront runs the same instructions.
template <typename T>
struct Bisect;
template <>
struct Bisect<double> {
  static constexpr int iters = 54;
};
template <>
struct Bisect<float> {
  static constexpr int iters = 25;
};

template <typename T>
__device__ __forceinline__ T sym5_lambda_max(T (&A)[5][5]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T ss = T(0);
#pragma unroll
    for (int i = k + 1; i < 5; ++i) ss += A[i][k] * A[i][k];
    const T x0 = A[k + 1][k];
    const T nrm = sqrt(ss);
    const T alpha = x0 >= T(0) ? -nrm : nrm;
    const T h = ss - x0 * alpha;  // |v|^2 / 2
    const T hi = h > T(0) ? recip(h) : T(0);
    T v[5], p[5];
#pragma unroll
    for (int i = k + 1; i < 5; ++i) v[i] = i == k + 1 ? x0 - alpha : A[i][k];
#pragma unroll
    for (int r = k + 1; r < 5; ++r) {
      T acc = T(0);
#pragma unroll
      for (int c = k + 1; c < 5; ++c) acc += A[r][c] * v[c];
      p[r] = acc * hi;
    }
    T K = T(0);
#pragma unroll
    for (int i = k + 1; i < 5; ++i) K += v[i] * p[i];
    K *= T(0.5) * hi;
#pragma unroll
    for (int i = k + 1; i < 5; ++i) p[i] -= K * v[i];  // p := q
#pragma unroll
    for (int r = k + 1; r < 5; ++r)
#pragma unroll
      for (int c = k + 1; c < 5; ++c) A[r][c] -= v[r] * p[c] + p[r] * v[c];
    // a vanishing column (h = 0) needs no reflection and keeps its sub-diagonal entry
    A[k + 1][k] = h > T(0) ? alpha : x0;
  }
  T d[5], e[4];
#pragma unroll
  for (int i = 0; i < 5; ++i) d[i] = A[i][i];
#pragma unroll
  for (int i = 0; i < 4; ++i) e[i] = A[i + 1][i];
  T sc = T(0);
#pragma unroll
  for (int i = 0; i < 5; ++i) sc = fmax(sc, fabs(d[i]));
#pragma unroll
  for (int i = 0; i < 4; ++i) sc = fmax(sc, fabs(e[i]));
  const T inv = sc > T(0) ? recip(sc) : T(0);
  T e2[4], lo = T(0), hi = T(0);
#pragma unroll
  for (int i = 0; i < 5; ++i) d[i] *= inv;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    e[i] = fabs(e[i] * inv);
    e2[i] = e[i] * e[i];
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    lo = fmax(lo, d[i]);
    hi = fmax(hi, d[i] + (i > 0 ? e[i - 1] : T(0)) + (i < 4 ? e[i] : T(0)));
  }
  for (int it = 0; it < Bisect<T>::iters; ++it) {
    const T x = T(0.5) * (lo + hi);
    const T m1 = x - d[0];
    const T m2 = (x - d[1]) * m1 - e2[0];
    const T m3 = (x - d[2]) * m2 - e2[1] * m1;
    const T m4 = (x - d[3]) * m3 - e2[2] * m2;
    const T m5 = (x - d[4]) * m4 - e2[3] * m3;
    const bool above = m1 > T(0) && m2 > T(0) && m3 > T(0) && m4 > T(0) && m5 > T(0);
    hi = above ? x : hi;
    lo = above ? lo : x;
  }
  return T(0.5) * (lo + hi) * sc;
}

// sigma_1 of cell i (0 <= i < N)
template <typename T>
__device__ __forceinline__ T sigma1_cell(const Consts<T>& c, const T* __restrict__ w, const long long i) {
  // 32-bit decomposition: the C ABI keeps every state array below 4 GiB (N < 2^28)
  const unsigned ui = (unsigned)i, t = ui / (unsigned)c.nx;
  const int gx = (int)(ui - t * (unsigned)c.nx), gy = (int)(t % (unsigned)c.ny), gz = (int)(t / (unsigned)c.ny);
  const QS<T> q0 = load_qs(c, w, gx, gy, gz);
  T grho[3], gu[3][3], gp[3], ga[3], gb[3];  // gu[k][j] = d_j u_k
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const QS<T> P = load_qs(c, w, gx + (l == 0), gy + (l == 1), gz + (l == 2));
    const QS<T> M = load_qs(c, w, gx - (l == 0), gy - (l == 1), gz - (l == 2));
    const T h = T(0.5) * c.idx[l];
    grho[l] = (P.rho - M.rho) * h;
#pragma unroll
    for (int k = 0; k < 3; ++k) gu[k][l] = (P.u[k] - M.u[k]) * h;
    gp[l] = (P.p - M.p) * h;
    ga[l] = (P.a - M.a) * h;
    gb[l] = (P.b - M.b) * h;
  }
  const T g = c.gamma;
  const T div = gu[0][0] + gu[1][1] + gu[2][2];
  T Mx[5][5];
  // M1 (halved as printed) minus M2
  Mx[0][0] = T(0.5) * div;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    Mx[0][1 + j] = T(0.5) * gb[j] - (q0.b * recip(q0.rho)) * grho[j];
    Mx[1 + j][0] = T(0.5) * gb[j];
#pragma unroll
    for (int k = 0; k < 3; ++k) Mx[1 + k][1 + j] = (j == k ? T(0.5) * div : T(0)) - gu[k][j];
    Mx[1 + j][4] = T(0.5) * ga[j] - (q0.a * recip(T(2) * q0.p)) * gp[j];
    Mx[4][1 + j] = T(0.5) * ga[j] - (T(2) * recip(g - T(1))) * ga[j];
    Mx[4][0] = T(0);
  }
  Mx[0][4] = -T(0.5) * sqrt(g - T(1)) * div;
  Mx[4][4] = T(0.5) * div - T(0.5) * (g - T(1)) * div;
  T A[5][5];
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int s = r; s < 5; ++s) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < 5; ++k) acc += Mx[k][r] * Mx[k][s];
      A[r][s] = acc;
      A[s][r] = acc;
    }
  const T lm = sym5_lambda_max(A);
  return sqrt(fmax(lm, T(0)));
}

template <typename T>
__global__ __launch_bounds__(RB) void k_sigma1(Consts<T> c, const T* __restrict__ w, T scale, T* __restrict__ out) {
  const long long i = (long long)xcd_tile(blockIdx.x, gridDim.x) * RB + threadIdx.x;
  if (i >= c.N) return;
  out[i] = scale * sigma1_cell(c, w, i);
}

// Ensemble form: RB cells of one box per work-group (offsets `start`), unscaled sigma_1.
template <typename T>
__global__ __launch_bounds__(RB) void k_sigma1_batch(const BoxDesc<T>* __restrict__ boxes,
                                                     const int* __restrict__ start, int nbox, const T* __restrict__ w,
                                                     T* __restrict__ out) {
  const int blk = xcd_tile(blockIdx.x, gridDim.x);
  const int b = find_box(start, nbox, blk);
  const Consts<T> c = boxes[b].c;
  const long long i = (long long)(blk - start[b]) * RB + threadIdx.x;
  if (i >= c.N) return;
  out[boxes[b].off + i] = sigma1_cell(c, w + 5 * boxes[b].off, i);
}

// ------------------------------------------------------------------------------------------
// Objectives (FP64 accumulation) and their gradients (added in the state precision)
// ------------------------------------------------------------------------------------------
// mean pressure: j = (1/N) sum p;  dp/dw = (gamma-1) (|u|^2/2, -u, 1)
template <typename T>
__global__ __launch_bounds__(RB) void k_meanp(Consts<T> c, const T* __restrict__ w, double wgt,
                                              double* __restrict__ partials, T* __restrict__ djdw) {
  __shared__ double sh[RB];
  const double g = (double)c.gamma;
  const long long N = c.N;
  double v = 0.0;
  for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < N; i += (long long)gridDim.x * RB) {
    const Q64 q = load_q64(c, w, i, 0, g);
    v += q.p;
    if (djdw) {
      T t[5];
      meanp_grad_terms(q, meanp_factor(wgt, g, N), t);
#pragma unroll
      for (int k = 0; k < 5; ++k) djdw[k * N + i] += t[k];
    }
  }
  if (partials) {
    const double tot = block_sum(v, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
  }
}

// Ensemble forms over members [first, first + count): RB cells of one member per work-group
// (offsets `start`, block blk = blockIdx.x + start[first]); one FP64 partial per work-group, folded
// per member by k_fold_members.  The per-cell gradient is the single-box formula with the
// member's own weight and size.
template <typename T>
__global__ __launch_bounds__(RB) void k_meanp_batch(const BoxDesc<T>* __restrict__ mems,
                                                    const int* __restrict__ start, int first, int count,
                                                    const T* __restrict__ w, const double* __restrict__ wgt,
                                                    double* __restrict__ partials, T* __restrict__ djdw) {
  __shared__ double sh[RB];
  const int blk = blockIdx.x + start[first];
  const int m = find_box(start, first + count, blk);
  const Consts<T> c = mems[m].c;
  const double g = (double)c.gamma;
  const long long N = c.N;
  const long long i = (long long)(blk - start[m]) * RB + threadIdx.x;
  double v = 0.0;
  if (i < N) {
    const Q64 q = load_q64(c, w + 5 * mems[m].off, i, 0, g);
    v = q.p;
    if (djdw) {
      T* d = djdw + 5 * mems[m].aoff;
      T t[5];
      meanp_grad_terms(q, meanp_factor(wgt[m], g, N), t);
#pragma unroll
      for (int k = 0; k < 5; ++k) d[k * N + i] += t[k];
    }
  }
  if (partials) {
    const double tot = block_sum(v, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
  }
}

template <typename T>
__global__ __launch_bounds__(RB) void k_energy_batch(const BoxDesc<T>* __restrict__ mems,
                                                     const int* __restrict__ start, int count,
                                                     const T* __restrict__ w, const T* __restrict__ wh,
                                                     double* __restrict__ partials) {
  __shared__ double sh[RB];
  const int m = find_box(start, count, blockIdx.x);
  const Consts<T> c = mems[m].c;
  const double g = (double)c.gamma;
  const double sa = sqrt((g - 1.0) / g), sb = 1.0 / sqrt(g);
  const long long N = c.N;
  const long long i = (long long)(blockIdx.x - start[m]) * RB + threadIdx.x;
  double v = 0.0;
  if (i < N) v = vhat_sq(c, w + 5 * mems[m].off, wh + 5 * mems[m].aoff, i, g, sa, sb);
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// One work-group per member m = first + blockIdx.x: its partials in block order, then
// dst[m] = dst[m] + (wgt[m] / N) sum   (objective)   or   dst[m] = sum / dV   (energy, wgt NULL).
template <typename T>
__global__ __launch_bounds__(RB) void k_fold_members(const double* __restrict__ partials, const int* __restrict__ start,
                                                     int first, const BoxDesc<T>* __restrict__ mems,
                                                     const double* __restrict__ wgt, double* __restrict__ dst) {
  __shared__ double sh[RB];
  const int m = first + blockIdx.x;
  const int b0 = start[m] - start[first], b1 = start[m + 1] - start[first];
  double v = 0.0;
  for (int i = b0 + threadIdx.x; i < b1; i += RB) v += partials[i];
  const double tot = block_sum(v, sh);
  if (threadIdx.x == 0) {
    const Consts<T>& c = mems[m].c;
    if (wgt)
      dst[m] = dst[m] + (wgt[m] / (double)c.N) * tot;
    else
      dst[m] = (1.0 / ((double)c.dx[0] * (double)c.dx[1] * (double)c.dx[2])) * tot;
    note_nonfinite(dst[m]);
  }
}

// Viscous dissipation j = (1/N) sum_cells sigma_lk d_l u_k with cell-centred central gradients.
// Both kernels stage the tile's velocities in LDS (halo 1 for the value, halo 2 for the gradient).
template <typename T, int NB>
__device__ __forceinline__ void tile_grad(const T (*su)[NB], int p, const int st[3], const T idx[3], T G[3][3]) {
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int k = 0; k < 3; ++k) G[l][k] = (su[k][p + st[l]] - su[k][p - st[l]]) * (T(0.5) * idx[l]);
}

// Loads velocities of the box whose origin is (x0 - hx, y0 - hy, z0 - hy) into su.
template <typename T, int KX, int KY, int KZ, int HX, int HY>
__device__ __forceinline__ void load_box_u(const Consts<T>& c, const T* __restrict__ w, int x0, int y0, int z0,
                                           T (*su)[TBox<KX, KY, KZ, HX, HY>::NB]) {
  using B = TBox<KX, KY, KZ, HX, HY>;
  constexpr int NTH = KX * KY * KZ;
  constexpr int NIT = (B::NB + NTH - 1) / NTH;
  const long long N = c.N;
  // every load of this thread is issued before any is used (one memory latency, not NIT); the
  // tail iteration re-reads the last box cell and does not store it
  T wv[NIT][4];
  int mir[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int b = min((int)threadIdx.x + it * NTH, B::NB - 1);
    const int bx = b % B::BX, by = (b / B::BX) % B::BY, bz = b / (B::BX * B::BY);
    int real;
    const long long gi =
        box_cell(c.nx, c.ny, c.nz, c.wall, x0 + bx - HX, y0 + by - HY, z0 + bz - HY, mir[it], real);
#pragma unroll
    for (int v = 0; v < 4; ++v) wv[it][v] = w[v * N + gi];
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int b = threadIdx.x + it * NTH;
    if (it + 1 < NIT || b < B::NB) {
      // stored deviations w - wref
      const T ri = recip(wv[it][0] + c.wref[0]);
      const T m1 = wv[it][1] + c.wref[1];
      su[0][b] = (mir[it] ? -m1 : m1) * ri;
      su[1][b] = (wv[it][2] + c.wref[2]) * ri;
      su[2][b] = (wv[it][3] + c.wref[3]) * ri;
    }
  }
}

// One work-group of KX x KY x KZ threads per tile of as many cells.
template <typename T, int KX, int KY, int KZ>
__global__ __launch_bounds__(KX * KY * KZ) void k_ked_tile(Consts<T> c, const T* __restrict__ w,
                                                           double* __restrict__ partials) {
  constexpr int NTH = KX * KY * KZ;
  using B = TBox<KX, KY, KZ, 1, 1>;
  __shared__ T su[3][B::NB];
  __shared__ double sh[NTH / 64];
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  int x0, y0, z0;
  tile_origin<KX, KY, KZ>(t, c.nx, c.ny, c.nz, x0, y0, z0);
  load_box_u<T, KX, KY, KZ, 1, 1>(c, w, x0, y0, z0, su);
  __syncthreads();
  const int tid = threadIdx.x;
  const int tx = tid % KX, ty = (tid / KX) % KY, tz = tid / (KX * KY);
  double phi = 0.0;
  if (x0 + tx < c.nx && y0 + ty < c.ny && z0 + tz < c.nz) {
    const int st[3] = {1, B::SY, B::SZ};
    const int p = (tz + 1) * B::SZ + (ty + 1) * B::SY + (tx + 1);
    T G[3][3];
    tile_grad<T, B::NB>(su, p, st, c.idx, G);
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
    phi = (double)acc;
  }
  const double tot = block_sum_n<NTH>(phi, sh);
  if (tid == 0) partials[t] = tot;
}

// Gradient: u^_k(j) = (wgt/N) sum_l (sigma_lk(j - e_l) - sigma_lk(j + e_l)) / dx_l (since
// d Phi / d G_lk = 2 sigma_lk); a ghost cell beyond a slip wall owns no dissipation term (sigma = 0),
// so the gather at the ghost image of a wall cell reduces to -+ sigma_xk(cell)/dx and is folded
// back through the mirror.  Then to conservative variables via u = m / rho.
template <typename T, int KX, int KY, int KZ>
__global__ __launch_bounds__(KX * KY * KZ) void k_ked_grad_tile(Consts<T> c, const T* __restrict__ w, double wgt,
                                                                T* __restrict__ djdw) {
  constexpr int NTH = KX * KY * KZ;
  using O = TBox<KX, KY, KZ, 2, 2>;
  using I = TBox<KX, KY, KZ, 1, 1>;
  __shared__ T su[3][O::NB];
  __shared__ T ss[6][I::NB];  // sigma xx, yy, zz, xy, xz, yz on the inner box
  int x0, y0, z0;
  tile_origin<KX, KY, KZ>(xcd_tile(blockIdx.x, gridDim.x), c.nx, c.ny, c.nz, x0, y0, z0);
  const int tid = threadIdx.x;
  const int tx = tid % KX, ty = (tid / KX) % KY, tz = tid / (KX * KY);
  const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
  const bool active = gx < c.nx && gy < c.ny && gz < c.nz;
  const long long N = c.N;
  const long long gi = active ? ((long long)gz * c.ny + gy) * c.nx + gx : 0;
  // the cell's own state and the output it accumulates into, fetched now so that their latency
  // hides behind the staging and the stress phase
  T wc[4], dj[4];
  if (active) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      wc[v] = w[v * N + gi];
      dj[v] = djdw[v * N + gi];
    }
  }
  load_box_u<T, KX, KY, KZ, 2, 2>(c, w, x0, y0, z0, su);
  __syncthreads();
  const int sto[3] = {1, O::SY, O::SZ};
  for (int b = threadIdx.x; b < I::NB; b += NTH) {
    const int bx = b % I::BX, by = (b / I::BX) % I::BY, bz = b / (I::BX * I::BY);
    const int gx = x0 + bx - 1;
    const bool real = !c.wall || (gx >= 0 && gx < c.nx);
    const int po = (bz + 1) * O::SZ + (by + 1) * O::SY + (bx + 1);
    T G[3][3];
    tile_grad<T, O::NB>(su, po, sto, c.idx, G);
    const T div = G[0][0] + G[1][1] + G[2][2];
    const T z = real ? T(1) : T(0);
    const T m = c.mu * z;
    ss[0][b] = m * (T(2) * G[0][0]) - (T(2) / T(3)) * m * div;
    ss[1][b] = m * (T(2) * G[1][1]) - (T(2) / T(3)) * m * div;
    ss[2][b] = m * (T(2) * G[2][2]) - (T(2) / T(3)) * m * div;
    ss[3][b] = m * (G[0][1] + G[1][0]);
    ss[4][b] = m * (G[0][2] + G[2][0]);
    ss[5][b] = m * (G[1][2] + G[2][1]);
  }
  __syncthreads();
  if (!active) return;
  const int sti[3] = {1, I::SY, I::SZ};
  const int p = (tz + 1) * I::SZ + (ty + 1) * I::SY + (tx + 1);
  // sym[l][k]: index of sigma_lk in ss
  constexpr int sym[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  T uh[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < 3; ++l) acc += (ss[sym[l][k]][p - sti[l]] - ss[sym[l][k]][p + sti[l]]) * c.idx[l];
    uh[k] = acc;
  }
  const T ri = recip(wc[0] + c.wref[0]);  // stored deviations w - wref
  const T u[3] = {(wc[1] + c.wref[1]) * ri, (wc[2] + c.wref[2]) * ri, (wc[3] + c.wref[3]) * ri};
  const T f = (T)(wgt / (double)N);
  T o0 = -f * ri * (u[0] * uh[0] + u[1] * uh[1] + u[2] * uh[2]);
  T o[3] = {f * ri * uh[0], f * ri * uh[1], f * ri * uh[2]};
  if (c.wall && (gx == 0 || gx == c.nx - 1)) {
    // ghost image: u^_k(ghost) = -+ sigma_xk(cell)/dx; ghost velocity (-u_x, u_y, u_z)
    const T sgn = gx == 0 ? T(-1) : T(1);
    T vh[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) vh[k] = sgn * ss[sym[0][k]][p] * c.idx[0];
    o0 += -f * ri * (-u[0] * vh[0] + u[1] * vh[1] + u[2] * vh[2]);
    o[0] -= f * ri * vh[0];
    o[1] += f * ri * vh[1];
    o[2] += f * ri * vh[2];
  }
  djdw[gi] = dj[0] + o0;
  djdw[N + gi] = dj[1] + o[0];
  djdw[2 * N + gi] = dj[2] + o[1];
  djdw[3 * N + gi] = dj[3] + o[2];
}

// Stagnation-pressure loss on an x-face plane [Eqs. (1)-(3)]: per face (j,k) the face state
// w_f = (w_L + w_R)/2; num_f = rho (pt_ref - p_t), den_f = rho, p_t = p X^kappa,
// X = 1 + (gamma-1) rho |u|^2 / (2 gamma p), kappa = gamma/(gamma-1).
struct PlaneTerms {
  double num, den;
  double dnum[5];  // d num / d w_f
};

__device__ __forceinline__ PlaneTerms plane_terms(double g, double pt_ref, const double wf[5]) {
  PlaneTerms t;
  const double r = wf[0], ri = 1.0 / r;
  const double m[3] = {wf[1], wf[2], wf[3]};
  const double E = wf[4];
  const double msq = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
  const double K = 0.5 * msq * ri;  // kinetic energy density
  const double p = (g - 1.0) * (E - K);
  const double X = 1.0 + K / (g * (E - K));
  const double kap = g / (g - 1.0);
  const double Xk = pow(X, kap);
  const double pt = p * Xk;
  t.num = r * (pt_ref - pt);
  t.den = r;
  // derivatives of K, p and X with respect to (rho, m, E)
  const double u[3] = {m[0] * ri, m[1] * ri, m[2] * ri};
  const double dK[5] = {-K * ri, u[0], u[1], u[2], 0.0};
  const double dXdK = E / (g * (E - K) * (E - K));
  const double dXdE = -K / (g * (E - K) * (E - K));
  const double dXk = kap * pow(X, kap - 1.0);
  for (int v = 0; v < 5; ++v) {
    const double dp = (g - 1.0) * ((v == 4 ? 1.0 : 0.0) - dK[v]);
    const double dX = dXdK * dK[v] + (v == 4 ? dXdE : 0.0);
    const double dpt = dp * Xk + p * dXk * dX;
    t.dnum[v] = (v == 0 ? (pt_ref - pt) : 0.0) - r * dpt;
  }
  return t;
}

template <typename T>
__device__ __forceinline__ void plane_face(const Consts<T>& c, const T* __restrict__ w, int plane_i, long long f,
                                           long long& il, long long& ir, double wf[5]) {
  const int j = (int)(f % c.ny), k = (int)(f / c.ny);
  il = ((long long)k * c.ny + j) * c.nx + (plane_i - 1);
  ir = il + 1;
  const long long N = c.N;
#pragma unroll
  // stored deviations w - wref, restored in FP64
  for (int v = 0; v < 5; ++v) wf[v] = 0.5 * ((double)w[v * N + il] + (double)w[v * N + ir]) + (double)c.wref[v];
}

template <typename T>
__global__ __launch_bounds__(RB) void k_ptloss_partial(Consts<T> c, const T* __restrict__ w, int plane_i,
                                                       double pt_ref, double* __restrict__ partials) {
  __shared__ double sh[RB];
  const long long nf = (long long)c.ny * c.nz;
  double vn = 0.0, vd = 0.0;
  for (long long f = (long long)blockIdx.x * RB + threadIdx.x; f < nf; f += (long long)gridDim.x * RB) {
    long long il, ir;
    double wf[5];
    plane_face(c, w, plane_i, f, il, ir, wf);
    const PlaneTerms t = plane_terms((double)c.gamma, pt_ref, wf);
    vn += t.num;
    vd += t.den;
  }
  const double tn = block_sum(vn, sh);
  const double td = block_sum(vd, sh);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = tn;
    partials[gridDim.x + blockIdx.x] = td;
  }
}

// scratch[0] = num, scratch[1] = den (already folded); J_accum += wgt num/(den pt_ref)
__global__ void k_ptloss_value(const double* __restrict__ scratch, double pt_ref, double wgt, double* J_accum) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *J_accum += wgt * scratch[0] / (scratch[1] * pt_ref);
    note_nonfinite(*J_accum);
  }
}

// dj/dw_L = dj/dw_R = 0.5 (dnum_f - (num/den) dden_f) / (den pt_ref)
template <typename T>
__global__ __launch_bounds__(RB) void k_ptloss_grad(Consts<T> c, const T* __restrict__ w, int plane_i,
                                                    double pt_ref, const double* __restrict__ scratch, double wgt,
                                                    T* __restrict__ djdw) {
  const long long f = (long long)blockIdx.x * RB + threadIdx.x;
  if (f >= (long long)c.ny * c.nz) return;
  long long il, ir;
  double wf[5];
  plane_face(c, w, plane_i, f, il, ir, wf);
  const PlaneTerms t = plane_terms((double)c.gamma, pt_ref, wf);
  const double num = scratch[0], den = scratch[1];
  const double sc = wgt * 0.5 / (den * pt_ref);
  const long long N = c.N;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double gv = sc * (t.dnum[v] - (v == 0 ? num / den : 0.0));
    djdw[v * N + il] += (T)gv;
    djdw[v * N + ir] += (T)gv;
  }
}

// ------------------------------------------------------------------------------------------
// BF16 codec (and its 16-bit fixed-point variant)
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Fixed-point code of t = r / s in [-1, 1]: the nearest integer (ties to even) of t * 32767,
// clamped to +-32767, as the bits of an int16; its value is code * (1/32767 rounded to FP32).
constexpr float I16_SCALE = 32767.0f;
constexpr float I16_STEP = 1.0f / 32767.0f;
__device__ __forceinline__ uint16_t i16_code(float t) {
  const float k = fminf(fmaxf(rintf(t * I16_SCALE), -I16_SCALE), I16_SCALE);
  return (uint16_t)(int16_t)(int)k;
}
__device__ __forceinline__ float i16_value(uint16_t q) { return (float)(int16_t)q * I16_STEP; }

// Block-scaled BF16 codec with a plane predictor: 4 x 4 x 4 cell blocks (ragged at the far ends).
// Per block and variable, with the present cells' local coordinates centred on the block
// (c_d = l_d - (n'_d - 1)/2, n'_d present cells along d):
//   a, g_x, g_y, g_z = the least-squares plane a + g . c of the block's values: FP64 sums
//     S_0 = sum w, S_d = sum c_d w in a fixed order, a = S_0 / n', g_d = S_d / sum c_d^2 (0 when
//     n'_d = 1), each rounded to FP32;
//   r0 = w - P(a), P(a) = fma(g_z, c_z, fma(g_y, c_y, fma(g_x, c_x, a)));
//   a' = a + (max r0 + min r0)/2, s = (max r0 - min r0)/2 (1 for an empty range);
//   code = RNE_bf16((w - P(a')) / s) with IEEE division;  decode w' = fma(s, code, P(a')).
//   The fixed-point variant (I16) codes the same quotient as i16_code and decodes
//   fma(s, i16_value(code), P(a')): an error of at most s / 65534 whatever the value, where BF16
//   keeps 2^-9 of each value (better near zero, 128 times worse at the edges of the range).
// header[(b * 5 + v) * 5 + {0, 1, 2, 3, 4}] = a', g_x, g_y, g_z, s with blocks numbered x fastest;
// codes keep the state layout.  The fixed summation order: each cell (lane) sums its z column,
// c(z) w_z accumulated z = 0..3 by fma (the products are exact in FP64); the columns then add
// pairwise in x (0+1, 2+3, then the pairs) and the rows pairwise in y the same way.
// One wavefront per strip of four blocks along x (16 x 4 x 4 cells): lane = (x, y) of the strip,
// each lane holds the four cells of its z column, and the four wavefronts of a work-group take
// consecutive strips, so that a row of 64 cells is read and written whole.  A block's lanes
// differ in lane bits 0, 1 (x) and 4, 5 (y), and the butterflies over those bits (1, 2, 16, 32)
// are the pairwise order above.
struct CodecStrip {
  long long i[4];  // cell index per z (valid when act[z])
  int b;           // block of the lane
  float cx, cy, cz[4];  // centred local coordinates of the lane's cells
  int np;               // present cells of the block
  double dx2, dy2, dz2; // sums of c_d^2 over the block's present cells
  bool act[4], live, any;
};

// sum over l = 0..m-1 of (l - (m-1)/2)^2 for a block side of m present cells
__device__ __forceinline__ double side_sq(int m) { return m == 4 ? 5.0 : (m == 3 ? 2.0 : (m == 2 ? 0.5 : 0.0)); }

__device__ __forceinline__ CodecStrip codec_strip(const Consts<float>& c) {
  const int lane = threadIdx.x & 63;
  const int nbx = (c.nx + 3) >> 2, nby = (c.ny + 3) >> 2, nbz = (c.nz + 3) >> 2, nsx = (nbx + 3) >> 2;
  const int sidx = blockIdx.x * (RB / 64) + (threadIdx.x >> 6);
  CodecStrip q;
  q.any = sidx < nsx * nby * nbz;  // the wavefront has a strip
  const int sx = sidx % nsx, by = (sidx / nsx) % nby, bz = sidx / (nsx * nby);
  const int bx = 4 * sx + ((lane >> 2) & 3);
  q.live = q.any && bx < nbx;
  q.b = (bz * nby + by) * nbx + bx;
  const int lx = lane & 3, ly = lane >> 4;
  const int x = 4 * bx + lx, y = 4 * by + ly;
  const int mx = min(4, c.nx - 4 * bx), my = min(4, c.ny - 4 * by), mz = min(4, c.nz - 4 * bz);
  q.cx = (float)lx - 0.5f * (float)(mx - 1);
  q.cy = (float)ly - 0.5f * (float)(my - 1);
  q.np = mx * my * mz;
  q.dx2 = (double)(my * mz) * side_sq(mx);
  q.dy2 = (double)(mx * mz) * side_sq(my);
  q.dz2 = (double)(mx * my) * side_sq(mz);
#pragma unroll
  for (int z = 0; z < 4; ++z) {
    const int gz = 4 * bz + z;
    q.cz[z] = (float)z - 0.5f * (float)(mz - 1);
    q.act[z] = q.live && x < c.nx && y < c.ny && gz < c.nz;
    q.i[z] = q.act[z] ? ((long long)gz * c.ny + y) * c.nx + x : 0;
  }
  return q;
}

// plane predictor at a cell: fma(g_z, c_z, fma(g_y, c_y, fma(g_x, c_x, a)))
__device__ __forceinline__ float plane(float a, float gx, float gy, float gz, float cx, float cy, float cz) {
  return fmaf(gz, cz, fmaf(gy, cy, fmaf(gx, cx, a)));
}

__device__ __forceinline__ double block_sum(double v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

template <bool I16>
__global__ __launch_bounds__(RB) void k_encode(Consts<float> c, const float* __restrict__ w, float* __restrict__ header,
                                               uint16_t* __restrict__ codes) {
  const CodecStrip q = codec_strip(c);
  if (!q.any) return;  // whole wavefronts only: every lane of a strip takes part in the shuffles
  const long long N = c.N;
  float x[5][4];
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int z = 0; z < 4; ++z) x[v][z] = q.act[z] ? w[v * N + q.i[z]] : 0.0f;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int z = 0; z < 4; ++z)
      if (q.act[z]) {
        const double xv = (double)x[v][z];
        s0 = fma(1.0, xv, s0);
        sx = fma((double)q.cx, xv, sx);
        sy = fma((double)q.cy, xv, sy);
        sz = fma((double)q.cz[z], xv, sz);
      }
    s0 = block_sum(s0);
    sx = block_sum(sx);
    sy = block_sum(sy);
    sz = block_sum(sz);
    const float a = (float)(s0 / (double)(q.np > 0 ? q.np : 1));
    const float gx = q.dx2 > 0.0 ? (float)(sx / q.dx2) : 0.0f;
    const float gy = q.dy2 > 0.0 ? (float)(sy / q.dy2) : 0.0f;
    const float gz = q.dz2 > 0.0 ? (float)(sz / q.dz2) : 0.0f;
    float mn = INFINITY, mx = -INFINITY;
#pragma unroll
    for (int z = 0; z < 4; ++z)
      if (q.act[z]) {
        const float r = x[v][z] - plane(a, gx, gy, gz, q.cx, q.cy, q.cz[z]);
        mn = fminf(mn, r);
        mx = fmaxf(mx, r);
      }
#pragma unroll
    for (int o = 1; o <= 32; o <<= 1) {
      if (o == 4 || o == 8) continue;  // lane bits 2, 3 select the block
      mn = fminf(mn, __shfl_xor(mn, o));
      mx = fmaxf(mx, __shfl_xor(mx, o));
    }
    const float a2 = a + 0.5f * (mx + mn);
    float s = 0.5f * (mx - mn);
    if (!(s > 0.0f)) s = 1.0f;
    if (q.live && (threadIdx.x & 0x33) == 0) {
      float* h = header + (q.b * 5 + v) * 5;
      h[0] = a2;
      h[1] = gx;
      h[2] = gy;
      h[3] = gz;
      h[4] = s;
    }
#pragma unroll
    for (int z = 0; z < 4; ++z)
      if (q.act[z]) {
        const float t = __fdiv_rn(x[v][z] - plane(a2, gx, gy, gz, q.cx, q.cy, q.cz[z]), s);
        codes[v * N + q.i[z]] = I16 ? i16_code(t) : bf16_rne(t);
      }
  }
}

template <bool I16>
__global__ __launch_bounds__(RB) void k_decode(Consts<float> c, const float* __restrict__ header,
                                               const uint16_t* __restrict__ codes, float* __restrict__ w) {
  const CodecStrip q = codec_strip(c);
  if (!q.live) return;
  const long long N = c.N;
  uint16_t k[5][4];
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int z = 0; z < 4; ++z) k[v][z] = q.act[z] ? codes[v * N + q.i[z]] : (uint16_t)0;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const float* h = header + (q.b * 5 + v) * 5;
    const float a = h[0], gx = h[1], gy = h[2], gz = h[3], s = h[4];
#pragma unroll
    for (int z = 0; z < 4; ++z)
      if (q.act[z])
        w[v * N + q.i[z]] = fmaf(s, I16 ? i16_value(k[v][z]) : __uint_as_float((uint32_t)k[v][z] << 16),
                                 plane(a, gx, gy, gz, q.cx, q.cy, q.cz[z]));
  }
}

inline int codec_groups(const Consts<float>& c) {
  const long long nbx = (c.nx + 3) >> 2;
  const long long ns = ((nbx + 3) >> 2) * ((c.ny + 3) >> 2) * ((c.nz + 3) >> 2);
  return (int)((ns + RB / 64 - 1) / (RB / 64));
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------
template <typename T>
hipError_t launch_sigma1(const Consts<T>& c, const T* w, T scale, T* out, hipStream_t st) {
  ProfScope ps(ADJ_PROF_SIGMA1, st, true);
  const int nb = (int)((c.N + RB - 1) / RB);
  timed_launch(ps, k_sigma1<T>, dim3(nb), dim3(RB), st, c, w, scale, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dot(const Consts<T>& c, const T* a, const T* b, double* partials, double* dst, double alpha,
                      double beta, hipStream_t st) {
  ProfScope ps(ADJ_PROF_REDUCE, st);
  const long long n = 5 * c.N;
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL((k_dot_partial<T>), dim3(nb), dim3(RB), 0, st, a, b, n, partials);
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(RB), 0, st, partials, nb, 1, dst, alpha, beta);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_energy_vhat(const Consts<T>& c, const T* w, const T* wh, double* partials, double* dst,
                              hipStream_t st) {
  ProfScope ps(ADJ_PROF_REDUCE, st);
  const int nb = reduce_blocks(c.N);
  hipLaunchKernelGGL((k_energy_partial<T>), dim3(nb), dim3(RB), 0, st, c, w, wh, partials);
  const double inv_dv = 1.0 / ((double)c.dx[0] * (double)c.dx[1] * (double)c.dx[2]);
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(RB), 0, st, partials, nb, 1, dst, inv_dv, 0.0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_objective(const Consts<T>& c, int kind, int plane_i, double pt_ref, const T* w, double weight,
                            double* J_accum, T* djdw, double* partials, double* scratch, hipStream_t st) {
  ProfScope ps(ADJ_PROF_OBJECTIVE, st);
  if (kind == 1) {
    const int nb = reduce_blocks(c.N);
    hipLaunchKernelGGL((k_meanp<T>), dim3(nb), dim3(RB), 0, st, c, w, weight, J_accum ? partials : nullptr, djdw);
    if (J_accum)
      hipLaunchKernelGGL(k_fold, dim3(1), dim3(RB), 0, st, partials, nb, 1, J_accum, weight / (double)c.N, 1.0);
  } else if (kind == 2) {
    // tiles of 32x4x4 cells: the halo-2 box of the gradient kernel holds 4.5 cells per output cell
    // (5 for 16x4x4); the larger 32x8x4 box (3.4) leaves one work-group of 1024 threads per compute
    // unit, and its FP32 launches take 19 % longer at 384^3 and 14 % at 128^3 (the same at 64^3)
    constexpr int KX = 32, KY = 4, KZ = 4;
    const dim3 grid(((c.nx + KX - 1) / KX) * ((c.ny + KY - 1) / KY) * ((c.nz + KZ - 1) / KZ));
    if (J_accum) {
      const int nb = (int)grid.x;
      // one partial per tile: the workspace partial region holds max(10 * MAX_PARTIALS, tiles of
      // 16x4x4 cells) values
      hipLaunchKernelGGL((k_ked_tile<T, KX, KY, KZ>), grid, dim3(KX * KY * KZ), 0, st, c, w, partials);
      hipLaunchKernelGGL(k_fold, dim3(1), dim3(RB), 0, st, partials, nb, 1, J_accum, weight / (double)c.N, 1.0);
    }
    if (djdw)
      hipLaunchKernelGGL((k_ked_grad_tile<T, KX, KY, KZ>), grid, dim3(KX * KY * KZ), 0, st, c, w, weight, djdw);
  } else if (kind == 3) {
    const long long nf = (long long)c.ny * c.nz;
    const int nb = reduce_blocks(nf);
    hipLaunchKernelGGL((k_ptloss_partial<T>), dim3(nb), dim3(RB), 0, st, c, w, plane_i, pt_ref, partials);
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(RB), 0, st, partials, nb, 2, scratch, 1.0, 0.0);
    if (J_accum) hipLaunchKernelGGL(k_ptloss_value, dim3(1), dim3(64), 0, st, scratch, pt_ref, weight, J_accum);
    if (djdw) {
      const int ng = (int)((nf + RB - 1) / RB);
      hipLaunchKernelGGL((k_ptloss_grad<T>), dim3(ng), dim3(RB), 0, st, c, w, plane_i, pt_ref, scratch, weight, djdw);
    }
  }
  return hipGetLastError();
}

hipError_t launch_fold(const double* partials, int n, double* dst, double alpha, double beta, hipStream_t st) {
  ProfScope ps(ADJ_PROF_OBJECTIVE, st);
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(RB), 0, st, partials, n, 1, dst, alpha, beta);
  return hipGetLastError();
}

hipError_t launch_ckpt_encode(const Consts<float>& c, const float* w, float* header, uint16_t* codes, bool i16,
                              hipStream_t st) {
  ProfScope ps(ADJ_PROF_CODEC, st, true);
  if (i16)
    timed_launch(ps, k_encode<true>, dim3(codec_groups(c)), dim3(RB), st, c, w, header, codes);
  else
    timed_launch(ps, k_encode<false>, dim3(codec_groups(c)), dim3(RB), st, c, w, header, codes);
  return hipGetLastError();
}

hipError_t launch_ckpt_decode(const Consts<float>& c, const float* header, const uint16_t* codes, float* w, bool i16,
                              hipStream_t st) {
  ProfScope ps(ADJ_PROF_CODEC, st, true);
  if (i16)
    timed_launch(ps, k_decode<true>, dim3(codec_groups(c)), dim3(RB), st, c, header, codes, w);
  else
    timed_launch(ps, k_decode<false>, dim3(codec_groups(c)), dim3(RB), st, c, header, codes, w);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sigma1_batch(const BoxDesc<T>* boxes, const int* start, int nbox, int nblocks, const T* w, T* out,
                               hipStream_t st) {
  ProfScope ps(ADJ_PROF_SIGMA1, st, true);
  timed_launch(ps, k_sigma1_batch<T>, dim3(nblocks), dim3(RB), st, boxes, start, nbox, w, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_meanp_batch(const BoxDesc<T>* mems, const int* start, const int* start_host, int first, int count,
                              const T* w, const double* wgt, double* J_accum, T* djdw, double* partials,
                              hipStream_t st) {
  ProfScope ps(ADJ_PROF_OBJECTIVE, st);
  const int nb = start_host[first + count] - start_host[first];
  hipLaunchKernelGGL((k_meanp_batch<T>), dim3(nb), dim3(RB), 0, st, mems, start, first, count, w, wgt,
                     J_accum ? partials : nullptr, djdw);
  if (J_accum)
    hipLaunchKernelGGL((k_fold_members<T>), dim3(count), dim3(RB), 0, st, partials, start, first, mems, wgt, J_accum);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_energy_batch(const BoxDesc<T>* mems, const int* start, const int* start_host, int count, const T* w,
                               const T* wh, double* partials, double* E, hipStream_t st) {
  ProfScope ps(ADJ_PROF_REDUCE, st);
  const int nb = start_host[count];
  hipLaunchKernelGGL((k_energy_batch<T>), dim3(nb), dim3(RB), 0, st, mems, start, count, w, wh, partials);
  hipLaunchKernelGGL((k_fold_members<T>), dim3(count), dim3(RB), 0, st, partials, start, 0, mems, nullptr, E);
  return hipGetLastError();
}

// Per-block maxima of the explicit-stability rates of a state: convective
// sum_d (|u_d| + c)/dx_d and viscous max(4/3, gamma/Pr) (mu/rho) sum_d 4/dx_d^2; set 2 of the
// partials takes the maximum of x (the sigma_1 field) when given.
template <typename T>
__global__ __launch_bounds__(RB) void k_stab_partial(Consts<T> c, const T* __restrict__ w, const T* __restrict__ x,
                                                     double* __restrict__ partials) {
  __shared__ double sh[3][RB];
  const long long N = c.N;
  double cv = 0.0, vv = 0.0, xv = 0.0;
  for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < N; i += (long long)gridDim.x * RB) {
    const double r = (double)w[i] + (double)c.wref[0];
    const double u[3] = {((double)w[N + i] + (double)c.wref[1]) / r, ((double)w[2 * N + i] + (double)c.wref[2]) / r,
                         ((double)w[3 * N + i] + (double)c.wref[3]) / r};
    const double g = (double)c.gamma;
    const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double p = (g - 1.0) * (((double)w[4 * N + i] + (double)c.wref[4]) - 0.5 * r * usq);
    const double snd = sqrt(fmax(g * p / r, 0.0));
    double s4 = 0.0, ci = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double h = (double)c.idx[d];
      ci += (fabs(u[d]) + snd) * h;
      s4 += 4.0 * h * h;
    }
    cv = fmax(cv, ci);
    // largest diffusivity: (4/3) mu / rho (normal stress) or alpha / rho = gamma mu / (Pr rho) (heat)
    vv = fmax(vv, fmax(4.0 / 3.0 * (double)c.mu, (double)c.alpha) / r * s4);
    if (x) xv = fmax(xv, (double)x[i]);
  }
  sh[0][threadIdx.x] = cv;
  sh[1][threadIdx.x] = vv;
  sh[2][threadIdx.x] = xv;
  for (int o = RB / 2; o > 0; o >>= 1) {
    __syncthreads();
    if (threadIdx.x < o)
      for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] = fmax(sh[k][threadIdx.x], sh[k][threadIdx.x + o]);
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) partials[k * gridDim.x + blockIdx.x] = sh[k][0];
}

// dst[k] = scale[k] * max over the nblk partials of set k, k = 0, 1, 2
__global__ __launch_bounds__(RB) void k_fold_max(const double* __restrict__ partials, int nblk, double s0, double s1,
                                                 double s2, double* __restrict__ dst) {
  __shared__ double sh[RB];
  const double sc[3] = {s0, s1, s2};
  for (int k = 0; k < 3; ++k) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += RB) v = fmax(v, partials[k * nblk + i]);
    sh[threadIdx.x] = v;
    for (int o = RB / 2; o > 0; o >>= 1) {
      __syncthreads();
      if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    }
    __syncthreads();
    if (threadIdx.x == 0) dst[k] = sc[k] * sh[0];
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_stability(const Consts<T>& c, const T* w, const T* sigma1, double s_conv, double s_visc,
                            double s_art, double* partials, double* dst, hipStream_t st) {
  const int nb = reduce_blocks(c.N);
  hipLaunchKernelGGL((k_stab_partial<T>), dim3(nb), dim3(RB), 0, st, c, w, sigma1, partials);
  hipLaunchKernelGGL(k_fold_max, dim3(1), dim3(RB), 0, st, partials, nb, s_conv, s_visc, s_art, dst);
  return hipGetLastError();
}

hipError_t read_clear_nonfinite(unsigned int* flag) {
  hipError_t e;
  if ((e = hipMemcpyFromSymbol(flag, HIP_SYMBOL(g_nonfinite), sizeof(unsigned int), 0, hipMemcpyDeviceToHost)))
    return e;
  const unsigned int zero = 0;
  return hipMemcpyToSymbol(HIP_SYMBOL(g_nonfinite), &zero, sizeof(unsigned int), 0, hipMemcpyHostToDevice);
}

template <typename T>
__global__ __launch_bounds__(RB) void k_rk3_mid(T* __restrict__ g2, const T* __restrict__ g3, long long n) {
  const long long i = (long long)blockIdx.x * RB + threadIdx.x;
  if (i < n) g2[i] = g2[i] + T(0.25) * g3[i];
}

template <typename T>
__global__ __launch_bounds__(RB) void k_rk3_combine(const T* __restrict__ a, const T* __restrict__ g1,
                                                    const T* __restrict__ h, const T* __restrict__ g3, T dt,
                                                    T* __restrict__ wh, T* __restrict__ grad_s, long long n) {
  const long long i = (long long)blockIdx.x * RB + threadIdx.x;
  if (i >= n) return;
  const T av = a[i], hv = h[i], g3v = g3[i];
  wh[i] = av + g1[i] + hv + T(0.75) * g3v;
  if (grad_s) grad_s[i] = fma(dt, av, fma(dt, hv, fma(T(0.25) * dt, g3v, grad_s[i])));
}

template <typename T>
hipError_t launch_rk3_mid(T* g2, const T* g3, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_rk3_mid<T>), dim3((unsigned)((n + RB - 1) / RB)), dim3(RB), 0, st, g2, g3, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rk3_combine(const T* a, const T* g1, const T* h, const T* g3, T dt, T* wh, T* grad_s, long long n,
                              hipStream_t st) {
  hipLaunchKernelGGL((k_rk3_combine<T>), dim3((unsigned)((n + RB - 1) / RB)), dim3(RB), 0, st, a, g1, h, g3, dt, wh,
                     grad_s, n);
  return hipGetLastError();
}

#define ADJNS_INST(T)                                                                                          \
  template hipError_t launch_rk3_mid<T>(T*, const T*, long long, hipStream_t);                                  \
  template hipError_t launch_rk3_combine<T>(const T*, const T*, const T*, const T*, T, T*, T*, long long,       \
                                            hipStream_t);                                                      \
  template hipError_t launch_stability<T>(const Consts<T>&, const T*, const T*, double, double, double, double*, \
                                          double*, hipStream_t);                                               \
  template hipError_t launch_sigma1<T>(const Consts<T>&, const T*, T, T*, hipStream_t);                        \
  template hipError_t launch_dot<T>(const Consts<T>&, const T*, const T*, double*, double*, double, double,    \
                                    hipStream_t);                                                              \
  template hipError_t launch_energy_vhat<T>(const Consts<T>&, const T*, const T*, double*, double*, hipStream_t); \
  template hipError_t launch_objective<T>(const Consts<T>&, int, int, double, const T*, double, double*, T*,   \
                                          double*, double*, hipStream_t);                                      \
  template hipError_t launch_sigma1_batch<T>(const BoxDesc<T>*, const int*, int, int, const T*, T*, hipStream_t); \
  template hipError_t launch_meanp_batch<T>(const BoxDesc<T>*, const int*, const int*, int, int, const T*,     \
                                            const double*, double*, T*, double*, hipStream_t);                 \
  template hipError_t launch_energy_batch<T>(const BoxDesc<T>*, const int*, const int*, int, const T*, const T*, \
                                             double*, double*, hipStream_t);
ADJNS_INST(float)
ADJNS_INST(double)
#undef ADJNS_INST

}  // namespace adjns
