"""Pins of the oracle's characteristic inflow/outflow boundaries (bc_x = 2; CPU only).

  free stream        a uniform state equal to the far field is steady (any flux option)
  characteristics    the boundary flux linearised at the far-field state is A+ (outlet) and A-
                     (inlet) of the textbook Euler Jacobian's eigen-decomposition (numpy): the
                     waves entering the box carry only far-field data, the leaving ones only
                     interior data
  supersonic         a supersonic inlet takes the far-field flux, a supersonic outlet the
                     interior cell's flux, whatever the other side holds
  conservation       the box's total rates are the boundary fluxes (the interior faces cancel)
  non-reflection     an acoustic pulse leaves through the outlet and the box's acoustic energy
                     drops to a small fraction, while slip walls keep it
  AD                 complex step, window duality and a Taylor test on inflow/outflow boxes
"""
import math

import numpy as np
import pytest

import workloads as W
from tests import linear_symbols as LS

GAM = 1.4


def _cons(rho, u, p):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (GAM - 1.0) + 0.5 * rho * (u @ u)])


def _cell_flux(w, d=0):
    rho = w[0]
    u = w[1:4] / rho
    p = (GAM - 1.0) * (w[4] - 0.5 * rho * (u @ u))
    f = np.array([rho * u[d], *(rho * u[d] * u), (w[4] + p) * u[d]])
    f[1 + d] += p
    return f


FAR = _cons(1.0, [0.3, 0.05, -0.02], 1.0 / GAM)  # Mach ~0.3 inflow from x = 0


def _grid(orc, n, L=(1.0, 1.0, 1.0), mu=0.0, dt=0.01, flux=0, scheme=0, far=(FAR, FAR), delta=0.1):
    return orc.make_grid(n, L, GAM, 0.72, mu, dt, orc.BC_CHARACTERISTIC, scheme, flux, delta,
                         np.concatenate(far))


def _uniform(n, w):
    return np.repeat(np.asarray(w, dtype=float), n[0] * n[1] * n[2])


@pytest.mark.parametrize("flux", [0, 1], ids=["split", "roe"])
def test_free_stream_is_steady(orc, flux):
    n = (7, 4, 3)
    g = _grid(orc, n, mu=0.02, flux=flux)
    R = orc.residual(g, _uniform(n, FAR))
    assert np.abs(R).max() <= 1e-13


@pytest.mark.parametrize("side", [0, 1], ids=["inlet", "outlet"])
@pytest.mark.parametrize("ux", [0.3, 0.04], ids=["subsonic", "slow"])
def test_boundary_flux_is_characteristic(orc, side, ux):
    far = _cons(1.1, [ux, 0.1, -0.05], 0.8)
    g = _grid(orc, (4, 2, 2), far=(far, far))
    h = 1e-6
    J = np.zeros((5, 5))
    for k in range(5):
        e = np.zeros(5)
        e[k] = h * max(1.0, abs(far[k]))
        J[:, k] = (orc.char_flux(g, side, far + e) - orc.char_flux(g, side, far - e)) / (2 * e[k])
    rho, u = far[0], far[1:4] / far[0]
    p = (GAM - 1.0) * (far[4] - 0.5 * rho * (u @ u))
    A = LS.euler_jacobian(0, rho, u, p, GAM)
    absA = LS.abs_matrix(A, 0.1 * math.sqrt(GAM * p / rho))
    expect = 0.5 * (A - absA) if side == 0 else 0.5 * (A + absA)
    assert np.abs(J - expect).max() <= 1e-7 * np.abs(A).max()
    if ux > 0.2:  # every speed outside the smoothing band: incoming characteristics carry nothing
        lam, R = np.linalg.eig(A)
        Linv = np.linalg.inv(R)
        incoming = np.real(lam) > 0 if side == 0 else np.real(lam) < 0
        proj = Linv @ J
        assert np.abs(proj[incoming]).max() <= 1e-7 * np.abs(A).max()


def test_supersonic_inlet_and_outlet(orc):
    far = _cons(1.0, [2.5, 0.1, 0.0], 1.0 / GAM)  # Mach ~2.5
    g = _grid(orc, (4, 2, 2), far=(far, far))
    inner = _cons(1.3, [2.4, -0.2, 0.1], 0.9)
    assert np.abs(orc.char_flux(g, 0, inner) - _cell_flux(far)).max() <= 1e-13 * np.abs(_cell_flux(far)).max()
    assert np.abs(orc.char_flux(g, 1, inner) - _cell_flux(inner)).max() <= 1e-13 * np.abs(_cell_flux(inner)).max()


def _smooth(n, seed, L=(2.0, 1.0, 1.0)):
    rng = np.random.default_rng(seed)
    x, y, z = W.cell_centres(n, L)
    rho = 1.0 + 0.1 * np.sin(2 * math.pi * y) * np.cos(x) + 0.01 * rng.standard_normal(x.shape)
    u = 0.3 + 0.05 * np.cos(2 * math.pi * y) + 0.01 * rng.standard_normal(x.shape)
    v = 0.05 * np.sin(x) + 0.01 * rng.standard_normal(x.shape)
    w = 0.02 * np.sin(2 * math.pi * z) + 0.01 * rng.standard_normal(x.shape)
    p = 1.0 / GAM * (1.0 + 0.05 * np.cos(x + 2 * math.pi * y)) + 0.005 * rng.standard_normal(x.shape)
    return W.conservative(rho, u, v, w, p)


@pytest.mark.parametrize("flux", [0, 1], ids=["split", "roe"])
def test_conservation_through_the_boundaries(orc, flux):
    n, L = (8, 5, 4), (2.0, 1.0, 1.0)
    far0, far1 = _cons(1.0, [0.3, 0.0, 0.0], 1 / GAM), _cons(0.95, [0.32, 0.01, 0.0], 0.98 / GAM)
    g = _grid(orc, n, L=L, mu=0.01, flux=flux, far=(far0, far1))
    w = _smooth(n, 3, L)
    R = orc.residual(g, w).reshape(5, n[2], n[1], n[0])
    w5 = w.reshape(5, n[2], n[1], n[0])
    dx = L[0] / n[0]
    bnd = np.zeros(5)
    for k in range(n[2]):
        for j in range(n[1]):
            bnd += orc.char_flux(g, 0, w5[:, k, j, 0]) - orc.char_flux(g, 1, w5[:, k, j, -1])
    tot = R.sum(axis=(1, 2, 3)) * dx
    assert np.abs(tot - bnd).max() <= 1e-12 * np.abs(R).sum() * dx


def test_acoustic_pulse_leaves_the_box(orc):
    """A right-running acoustic pulse in a quiescent 1-D box: with characteristic boundaries it
    leaves through x = L (the remaining acoustic energy falls below 2 % of the initial), between
    slip walls it stays (above 80 %)."""
    n, L = (80, 1, 1), (1.0, 1.0, 1.0)
    rho0, p0 = 1.0, 1.0 / GAM
    c0 = math.sqrt(GAM * p0 / rho0)
    x = (np.arange(n[0]) + 0.5) / n[0]
    a = 1e-3 * np.exp(-((x - 0.5) / 0.06) ** 2)
    rho, u, p = rho0 + a / c0 ** 2 * p0 * GAM, a / (rho0 * c0) * p0 * GAM, p0 + a * p0 * GAM
    w0 = W.conservative(rho.reshape(1, 1, -1), u.reshape(1, 1, -1), 0 * u.reshape(1, 1, -1),
                        0 * u.reshape(1, 1, -1), p.reshape(1, 1, -1))
    far = _cons(rho0, [0.0, 0.0, 0.0], p0)
    dt = 0.4 / n[0] / c0
    steps = int(0.9 / c0 / dt)

    def energy(w):
        w5 = w.reshape(5, -1)
        pp = (GAM - 1.0) * (w5[4] - 0.5 * (w5[1] ** 2) / w5[0])
        return float(((pp - p0) ** 2).sum() + (w5[1] ** 2).sum() * GAM * p0)

    e0 = energy(w0)
    for bc, bound in ((2, lambda r: r < 0.02), (1, lambda r: r > 0.8)):
        g = orc.make_grid(n, L, GAM, 0.72, 0.0, dt, bc, 0, 0, 0.1, np.concatenate([far, far]))
        w = w0.copy()
        for _ in range(steps):
            w = orc.primal_step(g, w)
        assert bound(energy(w) / e0), (bc, energy(w) / e0)


@pytest.mark.parametrize("flux,scheme", [(0, 0), (1, 1)], ids=["split-rk4", "roe-ssprk3"])
def test_tangent_matches_complex_step(orc, flux, scheme):
    n, L = (6, 5, 4), (2.0, 1.0, 1.0)
    g = _grid(orc, n, L=L, mu=0.02, dt=0.01, flux=flux, scheme=scheme)
    w = _smooth(n, 4, L)
    rng = np.random.default_rng(5)
    s = 1e-2 * rng.standard_normal(w.size)
    dw, ds = rng.standard_normal(w.size), rng.standard_normal(w.size)
    wn, dwn = orc.tlm_step(g, w, s, dw, ds)
    h = 1e-30
    cs = orc.primal_step_complex(g, w + 1j * h * dw, s + 1j * h * ds)
    assert np.abs(cs.real - wn).max() <= 1e-15 * np.abs(wn).max()
    assert np.abs(cs.imag / h - dwn).max() <= 1e-13 * np.abs(dwn).max()


@pytest.mark.parametrize("flux,scheme,lam", [(0, 0, 0.0), (1, 0, 0.004), (0, 1, (0.002, 0.004, 0.01))],
                         ids=["split-rk4", "roe-rk4-lam", "split-ssprk3-groups"])
def test_window_duality(orc, flux, scheme, lam):
    n, L = (6, 6, 4), (2.0, 1.0, 1.0)
    g = _grid(orc, n, L=L, mu=0.02, dt=0.01, flux=flux, scheme=scheme)
    w0 = _smooth(n, 6, L)
    rng = np.random.default_rng(9)
    s = 1e-3 * rng.standard_normal(w0.size)
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


def test_taylor_plane_loss(orc):
    n, L = (10, 6, 4), (2.0, 1.0, 1.0)
    g = _grid(orc, n, L=L, mu=0.02, dt=0.01)
    w0 = _smooth(n, 7, L)
    far = FAR
    rho, u = far[0], far[1:4] / far[0]
    p = (GAM - 1.0) * (far[4] - 0.5 * rho * (u @ u))
    pt = p * (1 + 0.5 * (GAM - 1.0) * (u @ u) * rho / (GAM * p)) ** (GAM / (GAM - 1.0))
    obj = orc.make_obj(W.OBJ_PT_LOSS_PLANE, 7, pt)
    nsteps = 4
    weights = W.window_weights(nsteps, 1, nsteps)
    rng = np.random.default_rng(15)
    s0 = 1e-2 * rng.standard_normal(w0.size)
    d = rng.standard_normal(w0.size)

    def J(s):
        return orc.objective_window(g, obj, orc.primal_window(g, w0, s, nsteps), weights)

    traj = orc.primal_window(g, w0, s0, nsteps)
    _, gs = orc.adjoint_window(g, obj, traj, s0, weights)
    eps = 1e-4
    fd = (J(s0 + eps * d) - J(s0 - eps * d)) / (2 * eps)
    assert abs(fd - gs @ d) <= 1e-7 * abs(gs @ d)
