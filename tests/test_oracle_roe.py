"""Pins of the oracle's Roe flux option against what Roe's approximate Riemann solver and the
mathematics fix (CPU only).

  upwinding            all wave speeds beyond the smoothing band of one sign: the flux is the
                       cell flux of the upwind state, for arbitrary jumps (Roe's property
                       A~ (w_r - w_l) = F(w_r) - F(w_l) of the averaged matrix)
  linear waves         a contact and shear jump at uniform p and u_d: the upwind cell flux in
                       subsonic flow (the acoustic waves carry nothing), and inside the band the
                       mass flux takes the smoothed speed (u^2 + delta^2)/(2 delta)
  mirror states        the flux between a state and its mirror image (a slip wall): no mass,
                       energy or tangential momentum, normal momentum rho u^2 + p + rho c~ u with
                       c~^2 = c^2 + (gamma - 1) u^2/2
  reflection           F(w_l, w_r) and F(M w_r, M w_l) (M: normal momentum reversed) agree up to
                       the parity of each component
  Fourier symbol       jvp and vjp at a uniform state against the closed-form symbol built from
                       numpy's eigen-decomposition of the textbook Euler Jacobian
  second order         the inviscid residual of a smooth periodic wave converges to -dF/dx like dx^2
  invariants, AD       free stream, conservation, wall fluxes, complex step, window duality,
                       Taylor test of the source gradient
"""
import math

import numpy as np
import pytest

import workloads as W
from tests import linear_symbols as LS

GAM = 1.4


def _cons(rho, u, p, gamma=GAM):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (gamma - 1.0) + 0.5 * rho * (u @ u)])


def _cell_flux(w, d, gamma=GAM):
    rho = w[0]
    u = w[1:4] / rho
    p = (gamma - 1.0) * (w[4] - 0.5 * rho * (u @ u))
    f = np.array([rho * u[d], *(rho * u[d] * u), (w[4] + p) * u[d]])
    f[1 + d] += p
    return f


def _roe_grid(orc, n=(4, 4, 4), L=(1.0, 1.0, 1.0), mu=0.0, dt=0.01, bc_x=0, scheme=0, roe_delta=0.1):
    return orc.make_grid(n, L, GAM, 0.72, mu, dt, bc_x, scheme, orc.FLUX_ROE, roe_delta)


def _close(a, b, tol=1e-13):
    return np.abs(np.asarray(a) - np.asarray(b)).max() <= tol * max(1.0, np.abs(b).max())


# ------------------------------------------------------------------------------ the face flux
@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("sign", [1, -1])
def test_supersonic_flux_is_upwind_cell_flux(orc, d, sign):
    g = _roe_grid(orc)
    rng = np.random.default_rng(10 + d)
    for _ in range(5):
        ul = 0.2 * rng.standard_normal(3)
        ur = 0.2 * rng.standard_normal(3)
        ul[d] = ur[d] = 0.0
        ul[d] += sign * (2.5 + 0.2 * rng.random())
        ur[d] += sign * (2.5 + 0.2 * rng.random())
        wl = _cons(1.0 + 0.3 * rng.random(), ul, 0.8 + 0.3 * rng.random())
        wr = _cons(1.0 + 0.3 * rng.random(), ur, 0.8 + 0.3 * rng.random())
        F = orc.roe_flux(g, d, wl, wr)
        assert _close(F, _cell_flux(wl if sign > 0 else wr, d))


def test_equal_states_give_the_cell_flux(orc):
    g = _roe_grid(orc)
    w = _cons(1.3, [0.2, -0.1, 0.05], 0.9)
    for d in range(3):
        assert _close(orc.roe_flux(g, d, w, w), _cell_flux(w, d))


@pytest.mark.parametrize("d", [0, 1, 2])
def test_contact_and_shear_waves_upwinded(orc, d):
    g = _roe_grid(orc)
    un = 0.3  # subsonic (c ~ 1), beyond the smoothing band (0.1 c~)
    ul, ur = np.array([0.1, -0.2, 0.15]), np.array([-0.05, 0.3, 0.2])
    ul[d] = ur[d] = un
    wl, wr = _cons(1.1, ul, 1.0), _cons(0.8, ur, 1.0)
    assert _close(orc.roe_flux(g, d, wl, wr), _cell_flux(wl, d))
    ul[d] = ur[d] = -un
    wl, wr = _cons(1.1, ul, 1.0), _cons(0.8, ur, 1.0)
    assert _close(orc.roe_flux(g, d, wl, wr), _cell_flux(wr, d))


def test_smoothed_speed_inside_band(orc):
    delta_frac = 0.2
    g = _roe_grid(orc, roe_delta=delta_frac)
    rl, rr, p, un = 1.1, 0.8, 1.0, 0.03
    wl, wr = _cons(rl, [un, 0, 0], p), _cons(rr, [un, 0, 0], p)
    F = orc.roe_flux(g, 0, wl, wr)
    # Roe sound speed: c~^2 = (gamma-1)(H~ - u^2/2), H~ the sqrt(rho)-weighted mean of H
    H = lambda r: (p / (GAM - 1.0) + 0.5 * r * un * un + p) / r
    Ht = (math.sqrt(rl) * H(rl) + math.sqrt(rr) * H(rr)) / (math.sqrt(rl) + math.sqrt(rr))
    delta = delta_frac * math.sqrt((GAM - 1.0) * (Ht - 0.5 * un * un))
    sabs = (un * un + delta * delta) / (2.0 * delta)
    assert abs(F[0] - (0.5 * (rl + rr) * un - 0.5 * sabs * (rr - rl))) <= 1e-14


@pytest.mark.parametrize("ux", [0.3, -0.25, 0.0])
def test_mirror_state_flux(orc, ux):
    g = _roe_grid(orc)
    rho, u, p = 1.2, np.array([ux, 0.4, -0.3]), 0.85
    wl = _cons(rho, u, p)
    wr = wl.copy()
    wr[1] = -wr[1]
    F = orc.roe_flux(g, 0, wl, wr)
    c2 = GAM * p / rho
    ct = math.sqrt(c2 + 0.5 * (GAM - 1.0) * ux * ux)
    assert abs(F[0]) <= 1e-14 and abs(F[2]) <= 1e-14 and abs(F[3]) <= 1e-14 and abs(F[4]) <= 1e-14
    assert abs(F[1] - (rho * ux * ux + p + rho * ct * ux)) <= 1e-14


def test_reflection_parity(orc):
    g = _roe_grid(orc)
    rng = np.random.default_rng(3)
    par = np.array([-1.0, 1.0, -1.0, -1.0, -1.0])  # mass, normal momentum, tangential, energy
    for d in range(3):
        for _ in range(4):
            wl = _cons(1 + 0.2 * rng.random(), 0.4 * rng.standard_normal(3), 1 + 0.2 * rng.random())
            wr = _cons(1 + 0.2 * rng.random(), 0.4 * rng.standard_normal(3), 1 + 0.2 * rng.random())
            M = np.ones(5)
            M[1 + d] = -1.0
            F = orc.roe_flux(g, d, wl, wr)
            Fm = orc.roe_flux(g, d, M * wr, M * wl)
            p = par.copy()
            p[1:4] = -1.0
            p[1 + d] = 1.0
            assert _close(Fm, p * F)


# ------------------------------------------------------------------------------ the residual
@pytest.mark.parametrize("kvec", [(1, 0, 0), (0, 2, 0), (1, 1, 1), (3, -2, 1)])
@pytest.mark.parametrize("ux", [0.3, 0.04])
def test_fourier_symbol_jvp_and_vjp(orc, kvec, ux):
    n = (8, 8, 8)
    L = (2 * math.pi, 3.0, 4.0)
    mu, pr, dfrac = 0.05, 0.72, 0.1
    g = orc.make_grid(n, L, GAM, pr, mu, 0.0, 0, 0, orc.FLUX_ROE, dfrac)
    dx = [L[d] / n[d] for d in range(3)]
    rho, u, p = 1.2, np.array([ux, -0.4, 0.25]), 0.9  # ux = 0.04: entropy and shear speeds in the band
    W0 = W.conservative(*[np.full((n[2], n[1], n[0]), x) for x in (rho, u[0], u[1], u[2], p)])
    k = [2 * math.pi * kvec[d] / L[d] for d in range(3)]
    rng = np.random.default_rng(sum(kvec) + 11)
    what = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    v = LS.fourier_mode(n, dx, k, what)
    Lk = LS.semi_discrete_symbol(k, dx, rho, u, p, GAM, mu, pr, roe_delta=dfrac)
    expect = LS.fourier_mode(n, dx, k, Lk @ what)
    assert np.abs(orc.jvp(g, W0, v) - expect).max() <= 1e-11 * np.abs(expect).max()
    expectT = LS.fourier_mode(n, dx, k, Lk.conj().T @ what)
    assert np.abs(orc.vjp(g, W0, v) - expectT).max() <= 1e-11 * np.abs(expectT).max()


@pytest.mark.parametrize("d", [0, 1, 2])
def test_second_order_convergence(orc, d):
    """Inviscid residual of a smooth periodic wave along direction d against -dF_d/dx_d at the
    cell centres (exact derivative by complex step of the cell flux)."""

    def state(x):
        rho = 1.0 + 0.2 * np.sin(x)
        u = np.zeros((3,) + np.shape(x), dtype=np.result_type(x, float))
        u[d] = 0.5 + 0.1 * np.cos(x)
        u[(d + 1) % 3] = 0.2 * np.sin(2 * x)
        p = 1.0 + 0.1 * np.sin(2 * x + 1.0)
        E = p / (GAM - 1.0) + 0.5 * rho * (u * u).sum(0)
        return np.array([rho, *(rho * u), E])

    errs = []
    for N in (16, 32, 64):
        n = [1, 1, 1]
        n[d] = N
        L = [1.0, 1.0, 1.0]
        L[d] = 2 * math.pi
        g = _roe_grid(orc, n=tuple(n), L=tuple(L))
        x = (np.arange(N) + 0.5) * (2 * math.pi / N)
        w = state(x)
        R = orc.residual(g, w.ravel()).reshape(5, N)
        h = 1e-30
        wc = state(x + 1j * h)
        exact = -np.array([_cell_flux(wc[:, i], d).imag / h for i in range(N)]).T
        errs.append(np.abs(R - exact).max())
    assert errs[0] / errs[1] > 3.6 and errs[1] / errs[2] > 3.8, errs


@pytest.mark.parametrize("bc_x", [0, 1])
def test_freestream_preserved(orc, bc_x):
    n = (6, 5, 4)
    g = _roe_grid(orc, n=n, L=(1.0, 2.0, 3.0), mu=0.02, bc_x=bc_x)
    u = (0.0 if bc_x else 0.37, -0.21, 0.13)
    w = W.conservative(*[np.full((n[2], n[1], n[0]), x) for x in (1.13, u[0], u[1], u[2], 0.83)])
    assert np.abs(orc.residual(g, w)).max() <= 1e-13


def _smooth_state(n, seed):
    rng = np.random.default_rng(seed)
    x, y, z = W.cell_centres(n, (2 * math.pi,) * 3)
    rho = 1.0 + 0.1 * np.sin(x + 2 * y) * np.cos(z) + 0.01 * rng.standard_normal(x.shape)
    u = 0.3 * np.sin(x) * np.cos(y) + 0.02 * rng.standard_normal(x.shape)
    v = -0.2 * np.cos(x) * np.sin(z) + 0.02 * rng.standard_normal(x.shape)
    w = 0.1 * np.sin(y + z) + 0.02 * rng.standard_normal(x.shape)
    p = 1.0 / 1.4 * (1.0 + 0.1 * np.cos(2 * x - y)) + 0.01 * rng.standard_normal(x.shape)
    return W.conservative(rho, u, v, w, p)


def test_conservation(orc):
    n = (7, 6, 5)
    L = (2 * math.pi,) * 3
    w = _smooth_state(n, 1)
    s = np.random.default_rng(2).standard_normal(w.size)
    g = _roe_grid(orc, n=n, L=L, mu=0.02)
    R = orc.residual(g, w, s).reshape(5, -1)
    scale = np.abs(orc.residual(g, w).reshape(5, -1)).sum(axis=1)
    assert np.all(np.abs(R.sum(axis=1) - s.reshape(5, -1).sum(axis=1)) <= 1e-13 * scale)
    # slip walls: no mass, energy or tangential momentum crosses them
    gw = _roe_grid(orc, n=n, L=L, mu=0.02, bc_x=1)
    Rw = orc.residual(gw, w).reshape(5, -1)
    sw = np.abs(Rw).sum(axis=1)
    for v in (0, 2, 3, 4):
        assert abs(Rw[v].sum()) <= 1e-13 * sw[v]


def test_differs_from_split_form_by_dissipation(orc):
    """The Roe residual removes energy that the split form conserves: at uniform pressure and with
    mu = 0, the split form leaves sum rho |u|^2/2 unchanged to first order, the Roe flux lowers it."""
    n = (8, 8, 8)
    L = (2 * math.pi,) * 3
    x, y, z = W.cell_centres(n, L)
    rho = 1.0 + 0.1 * np.sin(x) * np.cos(y)
    w = W.conservative(rho, 0.3 * np.sin(x) * np.cos(y), -0.3 * np.cos(x) * np.sin(y), 0 * x, 0 * x + 1.0)
    rates = []
    for flux in (orc.FLUX_SPLIT, orc.FLUX_ROE):
        g = orc.make_grid(n, L, GAM, 0.72, 0.0, 0.0, 0, 0, flux, 0.1)
        R = orc.residual(g, w).reshape(5, -1)
        wf = w.reshape(5, -1)
        u = wf[1:4] / wf[0]
        # d/dt sum rho |u|^2 / 2 = sum (u . dm/dt - |u|^2/2 drho/dt)
        rates.append(float((u * R[1:4]).sum() - (0.5 * (u * u).sum(0) * R[0]).sum()))
    assert abs(rates[0]) <= 1e-12 * 8**3
    assert rates[1] < -1e-4


# ------------------------------------------------------------------------------ AD machinery
@pytest.mark.parametrize("scheme", [0, 1], ids=["rk4", "ssprk3"])
@pytest.mark.parametrize("bc_x", [0, 1])
def test_tangent_matches_complex_step(orc, bc_x, scheme):
    n = (6, 5, 4)
    g = _roe_grid(orc, n=n, L=(2 * math.pi,) * 3, mu=0.02, dt=0.02, bc_x=bc_x, scheme=scheme)
    w = _smooth_state(n, 4)
    rng = np.random.default_rng(5)
    s = 1e-2 * rng.standard_normal(w.size)
    dw = rng.standard_normal(w.size)
    ds = rng.standard_normal(w.size)
    wn, dwn = orc.tlm_step(g, w, s, dw, ds)
    h = 1e-30
    cs = orc.primal_step_complex(g, w + 1j * h * dw, s + 1j * h * ds)
    assert np.abs(cs.real - wn).max() <= 1e-15 * np.abs(wn).max()
    assert np.abs(cs.imag / h - dwn).max() <= 1e-13 * np.abs(dwn).max()


@pytest.mark.parametrize("scheme", [0, 1], ids=["rk4", "ssprk3"])
@pytest.mark.parametrize("bc_x,lam", [(0, 0.0), (1, 0.01), (0, (0.004, 0.01, 0.025))])
def test_window_duality(orc, bc_x, lam, scheme):
    n = (6, 6, 4)
    g = _roe_grid(orc, n=n, L=(2 * math.pi,) * 3, mu=0.02, dt=0.02, bc_x=bc_x, scheme=scheme)
    w0 = _smooth_state(n, 6)
    rng = np.random.default_rng(9)
    s = 1e-3 * np.random.default_rng(8).standard_normal(w0.size)
    dw0, ds = rng.standard_normal(w0.size), rng.standard_normal(w0.size)
    traj, dws = [w0], [dw0]
    for _ in range(4):
        wn, dwn = orc.tlm_step(g, traj[-1], s, dws[-1], ds, lam)
        traj.append(wn)
        dws.append(dwn)
    aN = rng.standard_normal(w0.size)
    gs = np.zeros(w0.size)
    a = aN
    for k in range(3, -1, -1):
        a = orc.adjoint_step(g, traj[k], s, a, lam, None, 0.0, gs)
    lhs, rhs = aN @ dws[-1], a @ dw0 + gs @ ds
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_taylor_gradient_wrt_source(orc):
    wl = W.tgv_small(n=6, nsteps=4)
    p = wl.params()
    p["mu"] = 0.05
    p["flux"] = orc.FLUX_ROE
    g = orc.grid_from(p)
    obj = orc.make_obj(W.OBJ_KE_DISSIPATION)
    weights = W.window_weights(wl.nsteps, 1, wl.nsteps)
    rng = np.random.default_rng(15)
    s0 = 1e-2 * rng.standard_normal(wl.w0.size)
    d = rng.standard_normal(wl.w0.size)

    def J(s):
        return orc.objective_window(g, obj, orc.primal_window(g, wl.w0, s, wl.nsteps), weights)

    traj = orc.primal_window(g, wl.w0, s0, wl.nsteps)
    _, gs = orc.adjoint_window(g, obj, traj, s0, weights)
    gd = gs @ d
    eps = 1e-4
    fd = (J(s0 + eps * d) - J(s0 - eps * d)) / (2 * eps)
    assert abs(fd - gd) <= 1e-7 * abs(gd)
