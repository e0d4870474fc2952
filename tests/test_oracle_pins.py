"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test is chosen so that a plausible slip in the oracle (a dropped term, a wrong sign,
index or stencil coefficient, a transposed operand, a wrong RK4 weight) fails at least one:

  freestream / conservation      invariants of the conservative central finite-volume residual
  split-form identity            the face flux of means equals Kennedy & Gruber's split
                                 derivative (1/4)[d(ruf) + r d(uf) + u d(rf) + f d(ru) + ru df
                                 + rf du + uf dr] with plain central differences d
  kinetic energy                 at uniform pressure the inviscid terms leave sum rho|u|^2/2 fixed
  Fourier symbol (J and J^T)     closed-form linearised operator at a uniform state
  RK4 polynomial                 one tangent step equals G(dt L) = 1 + Z + Z^2/2 + Z^3/6 + Z^4/24
                                 (SSP-RK3: 1 + Z + Z^2/2 + Z^3/6)
  complex step                   dual-number tangent vs complex-step derivative of the primal
  duality                        <w^_N, dw_N> = <w^_0, dw_0> + <g_s, ds> over whole windows,
                                 also with one artificial viscosity per variable group
  variable groups                nu_g acts on exactly the components of its group (rho; rho u;
                                 rho E) and equals the single-viscosity operator there
  Taylor / finite differences    gradient of the time-averaged objective vs J(s + eps d)
  constant adjoint               J_R^T const = 0 (dual of conservation), L_nu const = 0
"""
import math

import numpy as np
import pytest

import workloads as W
from tests import linear_symbols as LS


def _grid(orc, n, L=(2 * math.pi,) * 3, mu=0.02, dt=0.01, bc_x=0, gamma=1.4, prandtl=0.72, scheme=0):
    return orc.make_grid(n, L, gamma, prandtl, mu, dt, bc_x, scheme)


SCHEMES = [0, 1]
SCHEME_IDS = ["rk4", "ssprk3"]


def _uniform(n, rho, u, p):
    shp = (n[2], n[1], n[0])
    f = [np.full(shp, x) for x in (rho, u[0], u[1], u[2], p)]
    return W.conservative(*f)


def _smooth_state(n, seed=0, amp=0.1):
    rng = np.random.default_rng(seed)
    L = (2 * math.pi,) * 3
    x, y, z = W.cell_centres(n, L)
    rho = 1.0 + amp * np.sin(x + 2 * y) * np.cos(z) + 0.01 * rng.standard_normal(x.shape)
    u = 0.3 * np.sin(x) * np.cos(y) + 0.02 * rng.standard_normal(x.shape)
    v = -0.2 * np.cos(x) * np.sin(z) + 0.02 * rng.standard_normal(x.shape)
    w = 0.1 * np.sin(y + z) + 0.02 * rng.standard_normal(x.shape)
    p = 1.0 / 1.4 * (1.0 + amp * np.cos(2 * x - y)) + 0.01 * rng.standard_normal(x.shape)
    return W.conservative(rho, u, v, w, p)


# ------------------------------------------------------------------------------ invariants
@pytest.mark.parametrize("bc_x", [0, 1])
def test_freestream_preserved_exactly(orc, bc_x):
    n = (6, 5, 4)
    g = _grid(orc, n, L=(1.0, 2.0, 3.0), bc_x=bc_x)
    u = (0.0 if bc_x else 0.37, -0.21, 0.13)  # a slip wall admits no normal velocity
    w = _uniform(n, 1.13, u, 0.83)
    R = orc.residual(g, w)
    # every face flux is identical, so R vanishes up to the rounding of the summation order
    # of face contributions (each O(|F|/dx) ~ 5 here)
    assert np.abs(R).max() <= 1e-14


@pytest.mark.parametrize("scheme", SCHEMES, ids=SCHEME_IDS)
def test_conservation_periodic(orc, scheme):
    n = (7, 6, 5)
    g = _grid(orc, n, scheme=scheme)
    w = _smooth_state(n, 1)
    s = np.random.default_rng(2).standard_normal(w.size)
    R = orc.residual(g, w, s).reshape(5, -1)
    total = R.sum(axis=1) - s.reshape(5, -1).sum(axis=1)
    scale = np.abs(orc.residual(g, w).reshape(5, -1)).sum(axis=1)
    assert np.all(np.abs(total) <= 1e-13 * scale)
    # conserved over RK4 steps (no source)
    g.dt = 0.01
    w1 = orc.primal_step(g, w)
    w2 = orc.primal_step(g, w1)
    m0, m2 = w.reshape(5, -1).sum(1), w2.reshape(5, -1).sum(1)
    assert np.all(np.abs(m2 - m0) <= 1e-12 * np.abs(w.reshape(5, -1)).sum(1))


def test_wall_conserves_mass_and_energy(orc):
    # slip walls: no mass or energy crosses the wall faces (the mirror flux carries only pressure)
    n = (6, 5, 4)
    g = _grid(orc, n, bc_x=1)
    w = _smooth_state(n, 3)
    R = orc.residual(g, w).reshape(5, -1)
    scale = np.abs(R).sum(axis=1)
    assert abs(R[0].sum()) <= 1e-13 * scale[0]
    assert abs(R[4].sum()) <= 1e-13 * scale[4]
    assert abs(R[2].sum()) <= 1e-13 * scale[2]  # tangential momentum


def _central(q, d, dx):
    # plain second-order central difference along grid axis d (x = last numpy axis), periodic
    ax = 2 - d
    return (np.roll(q, -1, axis=ax) - np.roll(q, 1, axis=ax)) / (2.0 * dx)


def test_split_form_identity(orc):
    # Inviscid residual on a rough periodic state against the split derivative forms written with
    # central differences only: cubic split for rho u_d phi (phi = 1, u_k, E/rho), quadratic split
    # (1/2)[d(pu) + p du + u dp] for the pressure work and d p for the momentum pressure term.
    n = (6, 5, 7)
    L = (1.3, 2.0, 0.9)
    gam = 1.4
    g = _grid(orc, n, L=L, mu=0.0, gamma=gam)
    rng = np.random.default_rng(11)
    shp = (n[2], n[1], n[0])
    rho = 1.0 + 0.3 * rng.random(shp)
    u = [0.4 * rng.standard_normal(shp) for _ in range(3)]
    p = 0.7 + 0.2 * rng.random(shp)
    w = W.conservative(rho, u[0], u[1], u[2], p, gamma=gam)
    Es = w.reshape(5, *shp)[4] / rho
    dx = [L[d] / n[d] for d in range(3)]

    def cubic(a, b, c, d):
        D = lambda q: _central(q, d, dx[d])
        return 0.25 * (D(a * b * c) + a * D(b * c) + b * D(a * c) + c * D(a * b)
                       + a * b * D(c) + a * c * D(b) + b * c * D(a))

    one = np.ones(shp)
    expect = np.zeros((5,) + shp)
    for d in range(3):
        expect[0] -= cubic(rho, u[d], one, d)
        for k in range(3):
            expect[1 + k] -= cubic(rho, u[d], u[k], d)
        expect[1 + d] -= _central(p, d, dx[d])
        expect[4] -= cubic(rho, u[d], Es, d)
        expect[4] -= 0.5 * (_central(p * u[d], d, dx[d]) + p * _central(u[d], d, dx[d])
                            + u[d] * _central(p, d, dx[d]))
    R = orc.residual(g, w).reshape(5, *shp)
    assert np.abs(R - expect).max() <= 1e-13 * np.abs(expect).max()


@pytest.mark.parametrize("seed", [0, 1])
def test_kinetic_energy_preserved_by_convection(orc, seed):
    # d/dt sum rho|u|^2/2 = sum (u . R_m - |u|^2/2 R_rho): zero when only convection acts and the
    # pressure is uniform (the momentum flux is the mass flux times the face-mean velocity)
    n = (6, 7, 5)
    g = _grid(orc, n, L=(1.0, 1.4, 0.8), mu=0.0)
    rng = np.random.default_rng(40 + seed)
    shp = (n[2], n[1], n[0])
    rho = 1.0 + 0.5 * rng.random(shp)
    u = [rng.standard_normal(shp) for _ in range(3)]
    w = W.conservative(rho, u[0], u[1], u[2], np.full(shp, 0.8))
    R = orc.residual(g, w).reshape(5, *shp)
    terms = sum(u[k] * R[1 + k] for k in range(3)) - 0.5 * sum(uk * uk for uk in u) * R[0]
    assert abs(terms.sum()) <= 1e-13 * np.abs(terms).sum()


# ------------------------------------------------------------------------------ Fourier symbols
@pytest.mark.parametrize("kvec", [(1, 0, 0), (0, 2, 0), (1, 1, 1), (2, -1, 3), (3, 2, -2)])
def test_fourier_symbol_jvp_and_vjp(orc, kvec):
    n = (8, 8, 8)
    L = (2 * math.pi, 3.0, 4.0)
    mu, pr, gam = 0.05, 0.72, 1.4
    g = _grid(orc, n, L=L, mu=mu, prandtl=pr, gamma=gam)
    dx = [L[d] / n[d] for d in range(3)]
    rho, u, p = 1.2, np.array([0.3, -0.4, 0.25]), 0.9
    W0 = _uniform(n, rho, u, p)
    k = [2 * math.pi * kvec[d] / L[d] for d in range(3)]
    rng = np.random.default_rng(sum(kvec) + 7)
    what = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    v = LS.fourier_mode(n, dx, k, what)
    Lk = LS.semi_discrete_symbol(k, dx, rho, u, p, gam, mu, pr)
    Jv = orc.jvp(g, W0, v)
    expect = LS.fourier_mode(n, dx, k, Lk @ what)
    assert np.abs(Jv - expect).max() <= 1e-12 * np.abs(expect).max()
    JTv = orc.vjp(g, W0, v)
    expectT = LS.fourier_mode(n, dx, k, Lk.conj().T @ what)
    assert np.abs(JTv - expectT).max() <= 1e-12 * np.abs(expectT).max()


def test_rk4_amplification_polynomial(orc):
    n = (8, 6, 4)
    L = (2.0, 1.5, 1.0)
    mu, pr, gam = 0.01, 0.72, 1.4
    dt = 0.01
    g = _grid(orc, n, L=L, mu=mu, prandtl=pr, gamma=gam, dt=dt)
    dx = [L[d] / n[d] for d in range(3)]
    rho, u, p = 0.9, np.array([0.5, 0.1, -0.2]), 1.1
    W0 = _uniform(n, rho, u, p)
    k = [2 * math.pi * 1 / L[0], 2 * math.pi * 2 / L[1], 2 * math.pi * 1 / L[2]]
    what = np.array([1.0 + 0.5j, -0.3j, 0.2, 0.7 - 0.1j, 0.4j])
    v = LS.fourier_mode(n, dx, k, what)
    _, dwn = orc.tlm_step(g, W0, None, v)
    Gk = LS.rk4_polynomial(dt * LS.semi_discrete_symbol(k, dx, rho, u, p, gam, mu, pr))
    expect = LS.fourier_mode(n, dx, k, Gk @ what)
    assert np.abs(dwn - expect).max() <= 1e-13 * np.abs(expect).max()


def test_ssprk3_amplification_polynomial(orc):
    # a three-stage third-order method is exact to third order on a linear system:
    # G(Z) = I + Z + Z^2/2 + Z^3/6 (no Z^4 term, which RK4 has)
    n = (8, 6, 4)
    L = (2.0, 1.5, 1.0)
    mu, pr, gam = 0.01, 0.72, 1.4
    dt = 0.01
    g = _grid(orc, n, L=L, mu=mu, prandtl=pr, gamma=gam, dt=dt, scheme=1)
    dx = [L[d] / n[d] for d in range(3)]
    rho, u, p = 0.9, np.array([0.5, 0.1, -0.2]), 1.1
    W0 = _uniform(n, rho, u, p)
    k = [2 * math.pi * 1 / L[0], 2 * math.pi * 2 / L[1], 2 * math.pi * 1 / L[2]]
    what = np.array([1.0 + 0.5j, -0.3j, 0.2, 0.7 - 0.1j, 0.4j])
    v = LS.fourier_mode(n, dx, k, what)
    _, dwn = orc.tlm_step(g, W0, None, v)
    Z = dt * LS.semi_discrete_symbol(k, dx, rho, u, p, gam, mu, pr)
    Gk = np.eye(5) + Z + Z @ Z / 2.0 + Z @ Z @ Z / 6.0
    expect = LS.fourier_mode(n, dx, k, Gk @ what)
    assert np.abs(dwn - expect).max() <= 1e-13 * np.abs(expect).max()
    # and it differs from the RK4 step by the Z^4/24 term (far above rounding)
    _, dw4 = orc.tlm_step(_grid(orc, n, L=L, mu=mu, prandtl=pr, gamma=gam, dt=dt), W0, None, v)
    assert np.abs(dw4 - dwn).max() > 1e3 * 1e-13 * np.abs(expect).max()


# ------------------------------------------------------------------------------ AD machinery
@pytest.mark.parametrize("scheme", SCHEMES, ids=SCHEME_IDS)
@pytest.mark.parametrize("bc_x", [0, 1])
def test_tangent_matches_complex_step(orc, bc_x, scheme):
    n = (6, 5, 4)
    g = _grid(orc, n, bc_x=bc_x, dt=0.02, scheme=scheme)
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


def _duality_window(orc, g, w0, s, lam, nsteps, seed):
    rng = np.random.default_rng(seed)
    dw0 = rng.standard_normal(w0.size)
    ds = rng.standard_normal(w0.size)
    traj = [w0]
    dws = [dw0]
    for _ in range(nsteps):
        wn, dwn = orc.tlm_step(g, traj[-1], s, dws[-1], ds, lam)
        traj.append(wn)
        dws.append(dwn)
    aN = rng.standard_normal(w0.size)
    gs = np.zeros(w0.size)
    a = aN
    for n in range(nsteps - 1, -1, -1):
        a = orc.adjoint_step(g, traj[n], s, a, lam, None, 0.0, gs)
    lhs = aN @ dws[-1]
    rhs = a @ dw0 + gs @ ds
    return lhs, rhs


@pytest.mark.parametrize("scheme", SCHEMES, ids=SCHEME_IDS)
@pytest.mark.parametrize("bc_x,lam", [(0, 0.0), (0, 0.01), (1, 0.0), (1, 0.01), (0, (0.004, 0.01, 0.025)),
                                      (1, (0.02, 0.0, 0.006))])
def test_window_duality(orc, bc_x, lam, scheme):
    n = (6, 6, 4)
    g = _grid(orc, n, bc_x=bc_x, dt=0.02, mu=0.02, scheme=scheme)
    w0 = _smooth_state(n, 6)
    s = 1e-3 * np.random.default_rng(8).standard_normal(w0.size)
    lhs, rhs = _duality_window(orc, g, w0, s, lam, 4, 9)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_stagewise_dot_product(orc):
    n = (5, 6, 7)
    g = _grid(orc, n, bc_x=1)
    W0 = _smooth_state(n, 10)
    rng = np.random.default_rng(11)
    x, y = rng.standard_normal(W0.size), rng.standard_normal(W0.size)
    assert abs(y @ orc.jvp(g, W0, x) - x @ orc.vjp(g, W0, y)) <= 1e-12 * abs(y @ orc.jvp(g, W0, x))


def test_constant_adjoint_preserved(orc):
    n = (6, 5, 4)
    g = _grid(orc, n)
    W0 = _smooth_state(n, 12)
    c = np.repeat(np.array([0.3, -1.2, 0.7, 2.0, -0.4]), W0.size // 5)
    out = orc.vjp(g, W0, c)
    assert np.abs(out).max() <= 1e-12 * np.abs(orc.vjp(g, W0, np.random.default_rng(0).standard_normal(W0.size))).max()
    nu = np.abs(np.random.default_rng(13).standard_normal(W0.size // 5))
    assert np.abs(orc.lnu_apply(g, nu, c)).max() <= 1e-15


def test_artificial_viscosity_symmetric_negative(orc):
    n = (5, 4, 6)
    g = _grid(orc, n, bc_x=1)
    rng = np.random.default_rng(14)
    nu = np.abs(rng.standard_normal(n[0] * n[1] * n[2]))
    x, y = rng.standard_normal(5 * nu.size), rng.standard_normal(5 * nu.size)
    a, b = x @ orc.lnu_apply(g, nu, y), y @ orc.lnu_apply(g, nu, x)
    assert abs(a - b) <= 1e-13 * abs(a)
    assert x @ orc.lnu_apply(g, nu, x) < 0.0


def test_artificial_viscosity_closed_form(orc):
    # constant nu on a periodic grid: L_nu of a Fourier mode is nu * sum_d (-4 sin^2(k dx/2)/dx^2)
    n = (8, 6, 4)
    L = (2.0, 3.0, 1.0)
    g = _grid(orc, n, L=L)
    dx = [L[d] / n[d] for d in range(3)]
    k = [2 * math.pi * 3 / L[0], 2 * math.pi * 1 / L[1], 2 * math.pi * 1 / L[2]]
    what = np.array([1.0, 0.5j, -0.2, 0.3 + 0.3j, 0.1])
    v = LS.fourier_mode(n, dx, k, what)
    nu0 = 0.37
    out = orc.lnu_apply(g, np.full(n[0] * n[1] * n[2], nu0), v)
    sym = nu0 * sum(-4.0 * math.sin(0.5 * k[d] * dx[d]) ** 2 / dx[d] ** 2 for d in range(3))
    assert np.abs(out - sym * v).max() <= 1e-12 * np.abs(sym * v).max()


# ------------------------------------------------------------------------------ Taylor tests
@pytest.mark.parametrize("scheme", SCHEMES, ids=SCHEME_IDS)
@pytest.mark.parametrize("kind", [W.OBJ_MEAN_PRESSURE, W.OBJ_KE_DISSIPATION])
def test_taylor_gradient_wrt_source(orc, kind, scheme):
    wl = W.tgv_small(n=6, nsteps=4)
    p = wl.params()
    p["mu"] = 0.05
    p["scheme"] = scheme
    g = orc.grid_from(p)
    obj = orc.make_obj(kind)
    weights = W.window_weights(wl.nsteps, 1, wl.nsteps)
    rng = np.random.default_rng(15)
    s0 = 1e-2 * rng.standard_normal(wl.w0.size)
    d = rng.standard_normal(wl.w0.size)

    def J(s):
        return orc.objective_window(g, obj, orc.primal_window(g, wl.w0, s, wl.nsteps), weights)

    traj = orc.primal_window(g, wl.w0, s0, wl.nsteps)
    wh0, gs = orc.adjoint_window(g, obj, traj, s0, weights)
    gd = gs @ d
    J0 = J(s0)
    # first-order remainder shrinks like eps^2
    r = []
    for eps in (1e-2, 1e-3):
        r.append(abs(J(s0 + eps * d) - J0 - eps * gd))
    assert r[1] < r[0] / 50.0
    eps = 1e-4
    fd = (J(s0 + eps * d) - J(s0 - eps * d)) / (2 * eps)
    assert abs(fd - gd) <= 1e-7 * abs(gd)
    # gradient with respect to the initial state
    dw = rng.standard_normal(wl.w0.size) * np.repeat(np.array([0.01, 0.01, 0.01, 0.01, 0.1]), wl.w0.size // 5)

    def Jw(w0):
        return orc.objective_window(g, obj, orc.primal_window(g, w0, s0, wl.nsteps), weights)

    fdw = (Jw(wl.w0 + eps * dw) - Jw(wl.w0 - eps * dw)) / (2 * eps)
    assert abs(fdw - wh0 @ dw) <= 1e-7 * abs(wh0 @ dw)


def test_taylor_plane_loss_with_walls(orc):
    wl = W.wake(n=(10, 6, 4), nsteps=3)
    g = orc.grid_from(wl.params())
    obj = orc.make_obj(W.OBJ_PT_LOSS_PLANE, wl.plane_i, wl.pt_ref)
    rng = np.random.default_rng(16)
    d = rng.standard_normal(wl.w0.size)
    s0 = np.zeros(wl.w0.size)

    def J(s):
        return orc.objective_window(g, obj, orc.primal_window(g, wl.w0, s, wl.nsteps), wl.weights)

    traj = orc.primal_window(g, wl.w0, s0, wl.nsteps)
    _, gs = orc.adjoint_window(g, obj, traj, s0, wl.weights)
    eps = 1e-4
    fd = (J(s0 + eps * d) - J(s0 - eps * d)) / (2 * eps)
    assert abs(fd - gs @ d) <= 1e-7 * abs(gs @ d)


@pytest.mark.parametrize("bc_x", [0, 1])
def test_group_viscosity_acts_on_its_components(orc, bc_x):
    n = (6, 5, 4)
    g = _grid(orc, n, bc_x=bc_x)
    w = _smooth_state(n, 15)
    q = np.random.default_rng(16).standard_normal(w.size)
    lam = 0.03
    one = orc.lnu_apply(g, lam * orc.sigma1(g, w), q).reshape(5, -1)  # one nu on every component
    assert np.abs(one).max() > 0.0
    total = np.zeros_like(one)
    for grp, comps in ((0, [0]), (1, [1, 2, 3]), (2, [4])):
        lv = [0.0, 0.0, 0.0]
        lv[grp] = lam
        out = orc.lnu_apply_groups(g, w, lv, q).reshape(5, -1)
        for v in range(5):
            if v in comps:
                assert np.allclose(out[v], one[v], rtol=1e-14, atol=0.0), (grp, v)
            else:
                assert not out[v].any(), (grp, v)
        total += out
    assert np.allclose(total, orc.lnu_apply_groups(g, w, lam, q).reshape(5, -1), rtol=1e-14, atol=0.0)
