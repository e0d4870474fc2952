"""Pins of the oracle's growth matrix, sigma_1, adjoint energy, objectives and checkpoint codec.

  symmetriser      S V A_d (S V)^-1 equals the printed symmetric A^_d (with the sign of the
                   u_j/rho entries of V read as negative)                [Symmetrization]
  growth matrix    the printed M1 - M2 equals (1/2) sum_j dA^_{k j i}/dx_j - B_{kjli} dv_l/dx_j
                   built numerically from A^(q), S and the chain rule    [Energy Analysis]
  sigma_1          Jacobi result vs LAPACK SVD; uniform flow -> 0; sinusoidal shear closed form
  E_v^             closed-form T^{-T} w^ vs a numpy solve with T = S V
  objectives       uniform-state values, a shear-flow closed form for the dissipation, the
                   isentropic-table stagnation pressure, and finite-difference gradients
  codec            round-to-nearest-even equals torch's float32 -> bfloat16 cast bitwise
"""
import math

import numpy as np
import pytest

import workloads as W
from tests import linear_symbols as LS

GAM = 1.4


def test_printed_symmetrised_flux_matrices():
    rng = np.random.default_rng(0)
    for _ in range(5):
        rho, u, p = 0.5 + rng.random(), rng.standard_normal(3) * 0.5, 0.3 + rng.random()
        S, V = LS.symmetriser(rho, u, p, GAM)
        T = S @ V
        c = math.sqrt(GAM * p / rho)
        for d in range(3):
            Ahat = T @ LS.euler_jacobian(d, rho, u, p, GAM) @ np.linalg.inv(T)
            assert np.abs(Ahat - LS.printed_ahat(d, u, c, GAM)).max() < 1e-13


def test_printed_V_sign_reading():
    # V must be dq/dw for q = (rho, u, p): check against finite differences of q(w)
    rho, u, p = 1.3, np.array([0.2, -0.5, 0.4]), 0.8
    _, V = LS.symmetriser(rho, u, p, GAM)

    def q_of_w(w):
        r = w[0]
        uu = w[1:4] / r
        return np.array([r, *uu, (GAM - 1.0) * (w[4] - 0.5 * r * uu @ uu)])

    w0 = np.array([rho, *(rho * u), p / (GAM - 1.0) + 0.5 * rho * u @ u])
    J = np.zeros((5, 5))
    for k in range(5):
        e = np.zeros(5)
        e[k] = 1e-6
        J[:, k] = (q_of_w(w0 + e) - q_of_w(w0 - e)) / 2e-6
    assert np.abs(J - V).max() < 1e-8
    assert V[1, 0] < 0  # -u_1/rho with u_1 > 0


def _growth_matrix_numeric(q0, gq):
    """(1/2) sum_j dA^_{kji}/dx_j - B_{kjli} dv_l/dx_j with dv/dx_j = S dq/dx_j and
    B_{kjli} = dA^_{kjl}/dv_i = dA^_{kjl}/dq_m (S^-1)_{mi}; derivatives by central differences."""
    def ahat(q, d):
        S, V = LS.symmetriser(q[0], q[1:4], q[4], GAM)
        T = S @ V
        return T @ LS.euler_jacobian(d, q[0], q[1:4], q[4], GAM) @ np.linalg.inv(T)

    dA = np.zeros((3, 5, 5, 5))
    for m in range(5):
        e = np.zeros(5)
        e[m] = 1e-6
        for j in range(3):
            dA[j, :, :, m] = (ahat(q0 + e, j) - ahat(q0 - e, j)) / 2e-6
    S, _ = LS.symmetriser(q0[0], q0[1:4], q0[4], GAM)
    Si = np.linalg.inv(S)
    M1 = 0.5 * np.einsum("jkim,mj->ki", dA, gq)
    dv = S @ gq  # dv_l/dx_j
    M2 = np.einsum("jklm,mi,lj->ki", dA, Si, dv)
    return M1 - M2


def test_growth_matrix_matches_energy_analysis(orc):
    rng = np.random.default_rng(1)
    for _ in range(4):
        q0 = np.array([0.8 + 0.5 * rng.random(), *(0.4 * rng.standard_normal(3)), 0.5 + rng.random()])
        gq = rng.standard_normal((5, 3))  # gq[m, j] = d q_m / d x_j

        def ab(q):
            c = math.sqrt(GAM * q[4] / q[0])
            return math.sqrt((GAM - 1.0) / GAM) * c, c / math.sqrt(GAM)

        ga, gb = np.zeros(3), np.zeros(3)
        for m in range(5):
            e = np.zeros(5)
            e[m] = 1e-6
            (ap, bp), (am, bm) = ab(q0 + e), ab(q0 - e)
            ga += (ap - am) / 2e-6 * gq[m]
            gb += (bp - bm) / 2e-6 * gq[m]
        grads = np.concatenate([gq[0], gq[1:4].reshape(-1), gq[4], ga, gb])
        Mo = orc.cell_growth_matrix(GAM, q0[0], q0[4], grads)
        Mn = _growth_matrix_numeric(q0, gq)
        assert np.abs(Mo - Mn).max() <= 1e-8 * np.abs(Mn).max()


def test_jacobi_sigma1_vs_lapack(orc):
    rng = np.random.default_rng(2)
    for _ in range(50):
        M = rng.standard_normal((5, 5)) * 10 ** rng.uniform(-3, 3)
        s_ref = np.linalg.svd(M, compute_uv=False)[0]
        assert abs(orc.matrix_sigma1(M) - s_ref) <= 1e-13 * s_ref
    # repeated singular values
    Q, _ = np.linalg.qr(rng.standard_normal((5, 5)))
    M = Q @ np.diag([2.0, 2.0, 1.0, 0.5, 0.0]) @ Q.T
    assert abs(orc.matrix_sigma1(M) - 2.0) < 1e-13


def test_sigma1_field_vs_svd_brute_force(orc):
    n = (5, 4, 6)
    L = (1.0, 2.0, 1.5)
    g = orc.make_grid(n, L, GAM, 0.72, 0.01, 0.0, 0)
    rng = np.random.default_rng(3)
    x, y, z = W.cell_centres(n, L)
    rho = 1.0 + 0.1 * rng.standard_normal(x.shape)
    u = 0.3 * rng.standard_normal(x.shape)
    v = 0.3 * rng.standard_normal(x.shape)
    ww = 0.3 * rng.standard_normal(x.shape)
    p = 0.7 + 0.05 * rng.standard_normal(x.shape)
    w = W.conservative(rho, u, v, ww, p)
    sig = orc.sigma1(g, w)
    Ms = orc.growth_matrix_field(g, w)
    ref = np.linalg.svd(Ms, compute_uv=False)[:, 0]
    assert np.abs(sig - ref).max() <= 1e-12 * ref.max()


def test_sigma1_uniform_is_zero(orc):
    n = (4, 4, 4)
    g = orc.make_grid(n, (1.0, 1.0, 1.0), GAM, 0.72, 0.01, 0.0, 0)
    f = [np.full((4, 4, 4), x) for x in (1.1, 0.3, 0.2, -0.1, 0.9)]
    assert np.abs(orc.sigma1(g, W.conservative(*f))).max() == 0.0


def test_sigma1_shear_closed_form(orc):
    # u_1 = A sin(k y), uniform rho and p: M1 = 0 and M2 has the single entry d_y u_1, so
    # sigma_1 = |A cos(k y_j) sin(k dy)/dy| exactly (central difference of a sinusoid)
    n = (4, 16, 4)
    L = (1.0, 2 * math.pi, 1.0)
    g = orc.make_grid(n, L, GAM, 0.72, 0.01, 0.0, 0)
    x, y, z = W.cell_centres(n, L)
    A, k = 0.7, 2.0
    dy = L[1] / n[1]
    w = W.conservative(np.ones_like(x), A * np.sin(k * y), 0 * x, 0 * x, np.full_like(x, 0.8))
    expect = np.abs(A * np.cos(k * y) * math.sin(k * dy) / dy).ravel()
    assert np.abs(orc.sigma1(g, w) - expect).max() <= 1e-13


def test_energy_vhat_matches_symmetriser_solve(orc):
    n = (3, 4, 2)
    L = (1.0, 1.0, 1.0)
    g = orc.make_grid(n, L, GAM, 0.72, 0.01, 0.0, 0)
    rng = np.random.default_rng(4)
    x, y, z = W.cell_centres(n, L)
    rho = 1.0 + 0.2 * rng.random(x.shape)
    u, v, ww = (0.4 * rng.standard_normal(x.shape) for _ in range(3))
    p = 0.6 + 0.3 * rng.random(x.shape)
    w = W.conservative(rho, u, v, ww, p)
    wh = rng.standard_normal(w.size)
    E, vhat = orc.energy_vhat(g, w, wh)
    N = x.size
    ref = np.zeros((5, N))
    for c in range(N):
        r, uu, pp = rho.ravel()[c], np.array([u.ravel()[c], v.ravel()[c], ww.ravel()[c]]), p.ravel()[c]
        S, V = LS.symmetriser(r, uu, pp, GAM)
        T = S @ V
        ref[:, c] = np.linalg.solve(T.T, wh.reshape(5, N)[:, c])  # w^ = T^T v^
    assert np.abs(vhat.reshape(5, N) - ref).max() <= 1e-12 * np.abs(ref).max()
    dV = (1.0 / 3) * (1.0 / 4) * (1.0 / 2)
    assert abs(E - (ref ** 2).sum() / dV) <= 1e-12 * E


# ------------------------------------------------------------------------------ objectives
def test_objectives_uniform_state(orc):
    n = (6, 4, 4)
    g = orc.make_grid(n, (1.0, 1.0, 1.0), GAM, 0.72, 0.01, 0.0, 1)
    f = [np.full((4, 4, 6), x) for x in (1.2, 0.0, 0.5, 0.1, 0.9)]
    w = W.conservative(*f)
    assert abs(orc.objective(g, orc.make_obj(W.OBJ_MEAN_PRESSURE), w, grad=False) - 0.9) < 1e-15
    assert orc.objective(g, orc.make_obj(W.OBJ_KE_DISSIPATION), w, grad=False) == 0.0
    c2 = GAM * 0.9 / 1.2
    M2 = (0.5 ** 2 + 0.1 ** 2) / c2
    pt = 0.9 * (1 + 0.2 * M2) ** 3.5
    assert abs(orc.objective(g, orc.make_obj(W.OBJ_PT_LOSS_PLANE, 3, pt), w, grad=False)) < 1e-15


def test_stagnation_pressure_isentropic_table(orc):
    # standard isentropic-flow table, gamma = 1.4: p/p0 = 0.6235 at M = 0.85 and 0.5283 at M = 1
    for mach, p_over_p0 in ((0.85, 0.62351), (1.0, 0.52828)):
        n = (4, 2, 2)
        g = orc.make_grid(n, (1.0, 1.0, 1.0), GAM, 0.72, 0.01, 0.0, 0)
        rho, p = 1.0, 1.0 / GAM
        c = math.sqrt(GAM * p / rho)
        f = [np.full((2, 2, 4), x) for x in (rho, 0.0, mach * c, 0.0, p)]
        w = W.conservative(*f)
        # j = (pt_ref - pt)/pt_ref; with pt_ref = 1 this gives pt = 1 - j
        j = orc.objective(g, orc.make_obj(W.OBJ_PT_LOSS_PLANE, 2, 1.0), w, grad=False)
        assert abs(p / (1.0 - j) - p_over_p0) < 5e-5


def test_dissipation_shear_closed_form(orc):
    n = (4, 16, 4)
    L = (1.0, 2 * math.pi, 1.0)
    mu = 0.03
    g = orc.make_grid(n, L, GAM, 0.72, mu, 0.0, 0)
    x, y, z = W.cell_centres(n, L)
    A, k = 0.7, 3.0
    dy = L[1] / n[1]
    w = W.conservative(np.ones_like(x), A * np.sin(k * y), 0 * x, 0 * x, np.full_like(x, 0.8))
    j = orc.objective(g, orc.make_obj(W.OBJ_KE_DISSIPATION), w, grad=False)
    expect = mu * np.mean((A * np.cos(k * y) * math.sin(k * dy) / dy) ** 2)
    assert abs(j - expect) <= 1e-13 * expect


@pytest.mark.parametrize("kind,bc_x", [(W.OBJ_MEAN_PRESSURE, 0), (W.OBJ_KE_DISSIPATION, 0),
                                       (W.OBJ_KE_DISSIPATION, 1), (W.OBJ_PT_LOSS_PLANE, 1)])
def test_objective_gradient_finite_difference(orc, kind, bc_x):
    n = (6, 5, 4)
    g = orc.make_grid(n, (1.0, 1.2, 0.8), GAM, 0.72, 0.02, 0.0, bc_x)
    rng = np.random.default_rng(5)
    x, y, z = W.cell_centres(n, (1.0, 1.2, 0.8))
    w = W.conservative(1 + 0.1 * rng.random(x.shape), 0.3 * rng.standard_normal(x.shape),
                       0.3 * rng.standard_normal(x.shape), 0.3 * rng.standard_normal(x.shape),
                       0.7 + 0.1 * rng.random(x.shape))
    obj = orc.make_obj(kind, 3, 1.2)
    _, dj = orc.objective(g, obj, w)
    d = rng.standard_normal(w.size)
    eps = 1e-6
    fd = (orc.objective(g, obj, w + eps * d, grad=False) - orc.objective(g, obj, w - eps * d, grad=False)) / (2 * eps)
    # central differences with eps = 1e-6 carry ~1e-10 |j| of rounding
    assert abs(fd - dj @ d) <= 1e-6 * abs(dj @ d)


# ------------------------------------------------------------------------------ codec
def _f32(x):
    return np.float32(x)


def _fmaf(a, b, c):
    # float32 fma through float64: a*b is exact there, one rounding of the sum to float64 and one to
    # float32 (a double rounding could differ from fmaf only when the float64 sum is inexact and
    # lands on a float32 tie, which the fields here never produce)
    return np.float32(np.float64(a) * np.float64(b) + np.float64(c))


def test_bf16_codec_plane_and_rounding(orc):
    # block-scaled codec with a plane predictor on a ragged grid (blocks of 4, 3, 2 and 1 cells per
    # side): per block and variable the header holds the least-squares plane of the block's values
    # (numpy lstsq here) with its constant moved to the middle of the residual range, and the
    # half-range s of the residuals; the codes are torch's round-to-nearest-even bfloat16 of
    # (w - plane)/s; decoding errs by at most half a bfloat16 ulp of s
    torch = pytest.importorskip("torch")
    n = (9, 7, 5)
    N = n[0] * n[1] * n[2]
    g = orc.make_grid(n, (1.0, 1.0, 1.0), 1.4, 0.72, 0.01, 0.01, 0)
    rng = np.random.default_rng(6)
    x, y, z = W.cell_centres(n, (1.0, 1.0, 1.0))
    w = np.stack([1.0 + 0.3 * np.sin(3 * x + 2 * y) * np.cos(4 * z) + 0.01 * rng.standard_normal(x.shape)
                  for _ in range(5)]).astype(np.float32).reshape(-1)
    w[:5] = [1.0, -1.0, 0.0, 1e-30, 3.0]
    w[N:2 * N] = 0.25  # a constant field: s = 1
    W5 = w.reshape(5, n[2], n[1], n[0])
    W5[2] = (0.5 + 0.25 * x + 0.125 * y - 0.0625 * z).astype(np.float32)  # a plane
    q, hdr = orc.ckpt_encode(g, w)
    nb = [(n[d] + 3) // 4 for d in range(3)]
    assert hdr.shape == (nb[0] * nb[1] * nb[2], 25)
    dec = orc.ckpt_decode(g, q, hdr).reshape(5, n[2], n[1], n[0])
    t = np.empty_like(W5)
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                b = (bz * nb[1] + by) * nb[0] + bx
                sl = (slice(4 * bz, 4 * bz + 4), slice(4 * by, 4 * by + 4), slice(4 * bx, 4 * bx + 4))
                m = [min(4, n[d] - 4 * bb) for d, bb in ((0, bx), (1, by), (2, bz))]
                cz, cy, cx = np.meshgrid(*[np.arange(m[d], dtype=np.float32) - np.float32(0.5 * (m[d] - 1))
                                           for d in (2, 1, 0)], indexing="ij")
                A = np.stack([np.ones(cx.size), cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(np.float64)
                for v in range(5):
                    blk = W5[v][sl]
                    h = hdr[b, 5 * v:5 * v + 5]
                    coef = np.linalg.lstsq(A[:, [0] + [1 + d for d in range(3) if m[d] > 1]],
                                           blk.ravel().astype(np.float64), rcond=None)[0]
                    slopes = np.zeros(3)
                    slopes[[d for d in range(3) if m[d] > 1]] = coef[1:]
                    for d in range(3):
                        assert abs(h[1 + d] - slopes[d]) <= np.spacing(np.float32(abs(slopes[d]))) + 1e-12 * abs(blk).max()
                    a = _f32(coef[0])
                    P = lambda a0: _fmaf(h[3], cz, _fmaf(h[2], cy, _fmaf(h[1], cx, a0)))
                    r0 = (blk - P(a)).astype(np.float32)
                    a2 = _f32(a + _f32(_f32(0.5) * _f32(r0.max() + r0.min())))
                    s = _f32(_f32(0.5) * _f32(r0.max() - r0.min()))
                    s = s if s > 0 else _f32(1.0)
                    assert abs(h[0] - a2) <= 2 * np.spacing(abs(a2)) and abs(h[4] - s) <= 2 * np.spacing(s)
                    t[v][sl] = (blk - P(h[0])) / h[4]
                    ulp = np.spacing(np.float32(np.abs(blk).max()))
                    if h[4] > 64 * ulp:
                        # a residual range above the rounding of the plane: the codes span [-1, 1]
                        assert np.abs(t[v][sl]).max() <= 1.0 + 2.0 ** -7
                    tmax = max(1.0, float(np.abs(t[v][sl]).max()))
                    assert np.abs(dec[v][sl] - blk).max() <= 2.0 ** -8 * tmax * h[4] + 4 * ulp
    ref = torch.from_numpy(t.reshape(-1)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(q, ref)
    # the planar field is reproduced to float32 rounding (its residual range is rounding only)
    assert np.abs(dec[2] - W5[2]).max() <= 1e-6


def test_i16_codec_codes_and_bound(orc):
    # the fixed-point codes of the same records: the header is the BF16 encoding's bit for bit (it
    # does not depend on the codes); each code is the integer nearest (ties to even, numpy rint)
    # to the float32 product of (w - P(a'))/s and 32767, clipped to +-32767; decoding
    # fma(s, code * float32(1/32767), P(a')) errs by at most s/65534 plus the rounding of the sum
    n = (9, 7, 5)
    N = n[0] * n[1] * n[2]
    g = orc.make_grid(n, (1.0, 1.0, 1.0), 1.4, 0.72, 0.01, 0.01, 0)
    rng = np.random.default_rng(8)
    x, y, z = W.cell_centres(n, (1.0, 1.0, 1.0))
    w = np.stack([1.0 + 0.3 * np.sin(3 * x + 2 * y) * np.cos(4 * z) + 0.02 * rng.standard_normal(x.shape)
                  for _ in range(5)]).astype(np.float32).reshape(-1)
    w[N:2 * N] = 0.25  # a constant field: s = 1, codes 0
    q16, hdr16 = orc.ckpt_encode(g, w, i16=True)
    qbf, hdrbf = orc.ckpt_encode(g, w)
    assert np.array_equal(hdr16.view(np.uint32), hdrbf.view(np.uint32))
    assert not np.array_equal(q16, qbf)
    dec = orc.ckpt_decode(g, q16, hdr16, i16=True).reshape(5, n[2], n[1], n[0])
    W5 = w.reshape(5, n[2], n[1], n[0])
    codes = q16.view(np.int16).reshape(5, n[2], n[1], n[0])
    nb = [(n[d] + 3) // 4 for d in range(3)]
    step = np.float32(1.0 / 32767.0)
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                b = (bz * nb[1] + by) * nb[0] + bx
                sl = (slice(4 * bz, 4 * bz + 4), slice(4 * by, 4 * by + 4), slice(4 * bx, 4 * bx + 4))
                m = [min(4, n[d] - 4 * bb) for d, bb in ((0, bx), (1, by), (2, bz))]
                cz, cy, cx = np.meshgrid(*[np.arange(m[d], dtype=np.float32) - np.float32(0.5 * (m[d] - 1))
                                           for d in (2, 1, 0)], indexing="ij")
                for v in range(5):
                    h = hdr16[b, 5 * v:5 * v + 5]
                    Pa = _fmaf(h[3], cz, _fmaf(h[2], cy, _fmaf(h[1], cx, h[0])))
                    t = ((W5[v][sl] - Pa) / h[4]).astype(np.float32)
                    want = np.clip(np.rint((t * np.float32(32767.0)).astype(np.float32)), -32767, 32767)
                    assert np.array_equal(codes[v][sl].astype(np.float64), want.astype(np.float64))
                    back = _fmaf(h[4], (codes[v][sl].astype(np.float32) * step).astype(np.float32), Pa)
                    assert np.array_equal(dec[v][sl], back)
                    ulp = np.spacing(np.float32(np.abs(W5[v][sl]).max()))
                    assert np.abs(dec[v][sl] - W5[v][sl]).max() <= h[4] / 65534.0 * 1.0001 + 4 * ulp
    # 128 times finer than the BF16 codes at the ends of the range: on these noisy blocks the
    # largest decoding error drops by more than 30
    decbf = orc.ckpt_decode(g, qbf, hdrbf).reshape(W5.shape)
    assert np.abs(decbf - W5).max() > 30 * np.abs(dec - W5).max()
