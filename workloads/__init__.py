"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the method itself: it only builds initial conditions,
source fields, time-step sizes and window weights with numpy (FP64), so that the GPU library
and the FP64 oracle receive bit-identical inputs.  It imports neither of them.

The paper's own workload (a wall-resolved LES of the VKI turbine vane on an unstructured mesh,
section "Numerical methods") is not available; these fields stand in for it with the shapes,
sizes and statistics listed below:

  tgv_small    16^3 Taylor-Green vortex, Mach 0.3, Re 100, velocity noise 1e-3 (seed 0),
               50 steps, objective = mean pressure averaged over steps 26..50, lambda = 0
  tgv_64       64^3 Taylor-Green vortex, Mach 0.1, Re 1600, 1000 steps, objective = mean viscous
               dissipation averaged over steps 1..N, body force iid N(0, 1e-4^2) with the mean of
               each component removed (seed 1)
  wake         512x256x32 temporally developing wake between slip walls in x (cross-stream),
               periodic y (streamwise) and z; Gaussian deficit, free stream Mach 0.85, centre
               Mach 0.5, Re 5e4 on the wake width; solenoidal flat-spectrum noise of 2 % (seed 2);
               objective = density-weighted stagnation-pressure loss on the face x = 0.75 L_x
  turbulence   periodic decaying turbulence, E(k) ~ k^4 exp(-2 k^2/k0^2), k0 = 4, random phases,
               solenoidal, scaled so that sqrt(<|u|^2>) = 1 and Mach_rms = sqrt(<|u|^2>)/c0
  ensemble     64 turbulence boxes with sizes from {32,48,64,96}^3 (seed 3), windows 50..400
               (seed 5), lambda factors from {0, 0.03, 0.1, 0.3, 1} (seed 6)
  turb_384     384^3 turbulence, Mach_rms 0.4, nu = 2.887e-3, 5000 steps, mean pressure, lambda 0.1

Layout of every state: FP64 array of shape (5 * N,), var-major, cell index (k*ny + j)*nx + i.
"""
from dataclasses import dataclass, field
import math

import numpy as np

GAMMA = 1.4
PRANDTL = 0.72

OBJ_NONE, OBJ_MEAN_PRESSURE, OBJ_KE_DISSIPATION, OBJ_PT_LOSS_PLANE = 0, 1, 2, 3


@dataclass
class Workload:
    name: str
    n: tuple
    L: tuple
    mu: float
    dt: float
    w0: np.ndarray
    s: np.ndarray
    nsteps: int
    obj_kind: int
    weights: np.ndarray          # c_n, n = 0..nsteps
    lam: float = 0.0             # artificial-viscosity scale in length^2 (nu = lam * sigma_1)
    lam_factor: float = 0.0      # lam / dx_min^2
    bc_x: int = 0
    plane_i: int = 0
    pt_ref: float = 0.0
    gamma: float = GAMMA
    prandtl: float = PRANDTL
    extra: dict = field(default_factory=dict)

    @property
    def ncells(self):
        return int(self.n[0] * self.n[1] * self.n[2])

    def params(self):
        p = dict(n=self.n, L=self.L, gamma=self.gamma, prandtl=self.prandtl, mu=self.mu, dt=self.dt,
                 bc_x=self.bc_x)
        if "w_far" in self.extra:
            p["w_far"] = np.concatenate([np.asarray(f, dtype=np.float64) for f in self.extra["w_far"]])
        return p


def cell_centres(n, L):
    xs = [(np.arange(n[d]) + 0.5) * (L[d] / n[d]) for d in range(3)]
    z, y, x = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return x, y, z


def conservative(rho, u, v, w, p, gamma=GAMMA):
    """(rho, rho u, rho E) from primitive fields, E = p/((gamma-1) rho) + |u|^2/2."""
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E]).reshape(5, -1).astype(np.float64).copy().ravel()


def cfl_dt(rho, u, v, w, p, dx, cfl=0.5, gamma=GAMMA):
    """dt = cfl / max_cells sum_d (|u_d| + c) / dx_d, evaluated on the initial state and frozen."""
    c = np.sqrt(gamma * p / rho)
    rate = (np.abs(u) + c) / dx[0] + (np.abs(v) + c) / dx[1] + (np.abs(w) + c) / dx[2]
    return float(cfl / rate.max())


def tgv_fields(n, L, mach, rng=None, noise=0.0, gamma=GAMMA):
    """Taylor-Green vortex, U0 = 1, rho0 = 1, c0 = 1/mach, isothermal density rho = p/p0."""
    x, y, z = cell_centres(n, L)
    c0 = 1.0 / mach
    p0 = c0 * c0 / gamma
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    if noise > 0.0:
        u = u + noise * rng.standard_normal(u.shape)
        v = v + noise * rng.standard_normal(u.shape)
        w = w + noise * rng.standard_normal(u.shape)
    p = p0 + (1.0 / 16.0) * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    rho = p / p0
    return rho, u, v, w, p


def window_weights(nsteps, first, last):
    """Rectangle rule of the time average: c_n = 1/K for n in [first, last], K = last-first+1."""
    c = np.zeros(nsteps + 1)
    c[first:last + 1] = 1.0 / (last - first + 1)
    return c


def tgv_small(n=16, nsteps=50, seed=0):
    L = (2 * math.pi,) * 3
    nn = (n, n, n)
    rng = np.random.default_rng(seed)
    rho, u, v, w, p = tgv_fields(nn, L, 0.3, rng, noise=1e-3)
    dx = [L[d] / nn[d] for d in range(3)]
    dt = cfl_dt(rho, u, v, w, p, dx)
    w0 = conservative(rho, u, v, w, p)
    first = nsteps // 2 + 1
    return Workload("tgv_small", nn, L, 1.0 / 100.0, dt, w0, np.zeros_like(w0), nsteps,
                    OBJ_MEAN_PRESSURE, window_weights(nsteps, first, nsteps))


def body_force(N, sigma, rng):
    s = sigma * rng.standard_normal((5, N))
    s -= s.mean(axis=1, keepdims=True)
    return s.ravel().copy()


def tgv_64(n=64, nsteps=1000, seed=1):
    L = (2 * math.pi,) * 3
    nn = (n, n, n)
    rng = np.random.default_rng(seed)
    rho, u, v, w, p = tgv_fields(nn, L, 0.1)
    dx = [L[d] / nn[d] for d in range(3)]
    dt = cfl_dt(rho, u, v, w, p, dx)
    w0 = conservative(rho, u, v, w, p)
    s = body_force(n ** 3, 1e-4, rng)
    return Workload("tgv_64", nn, L, 1.0 / 1600.0, dt, w0, s, nsteps, OBJ_KE_DISSIPATION,
                    window_weights(nsteps, 1, nsteps))


def solenoidal_field(n, L, rng, spectrum):
    """Random-phase periodic velocity field with energy spectrum E(k) (shell-normalised),
    projected onto divergence-free modes; returns (u, v, w) with zero mean."""
    k1 = [np.fft.fftfreq(n[d], d=L[d] / n[d]) * 2 * math.pi for d in range(3)]
    kz, ky, kx = np.meshgrid(k1[2], k1[1], k1[0], indexing="ij")
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    shape = kk.shape
    amp = np.zeros(shape)
    nz = kk > 0
    amp[nz] = np.sqrt(spectrum(kk[nz]) / (4 * math.pi * kk[nz] ** 2))
    comps = []
    for _ in range(3):
        ph = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        comps.append(amp * ph)
    # projection P = I - k k^T / |k|^2
    with np.errstate(invalid="ignore", divide="ignore"):
        kdot = (kx * comps[0] + ky * comps[1] + kz * comps[2]) / np.where(nz, kk * kk, 1.0)
    comps = [comps[0] - kx * kdot, comps[1] - ky * kdot, comps[2] - kz * kdot]
    out = [np.real(np.fft.ifftn(c)) for c in comps]
    out = [o - o.mean() for o in out]
    return out


def turbulence(n, L=(2 * math.pi,) * 3, mach_rms=0.3, nu=0.0175, k0=4.0, seed=4, nsteps=100,
               lam_factor=0.0, obj_kind=OBJ_MEAN_PRESSURE, cfl=0.5):
    nn = tuple(n) if hasattr(n, "__len__") else (n, n, n)
    rng = np.random.default_rng(seed)
    u, v, w = solenoidal_field(nn, L, rng, lambda k: k ** 4 * np.exp(-2.0 * k * k / (k0 * k0)))
    scale = 1.0 / math.sqrt(float(np.mean(u * u + v * v + w * w)))
    u, v, w = u * scale, v * scale, w * scale
    c0 = 1.0 / mach_rms
    rho = np.ones_like(u)
    p = np.full_like(u, c0 * c0 / GAMMA)
    dx = [L[d] / nn[d] for d in range(3)]
    dt = cfl_dt(rho, u, v, w, p, dx, cfl)
    w0 = conservative(rho, u, v, w, p)
    dmin = min(dx)
    return Workload(f"turbulence_{nn[0]}x{nn[1]}x{nn[2]}", nn, L, nu, dt, w0, np.zeros_like(w0), nsteps,
                    obj_kind, window_weights(nsteps, 1, nsteps), lam=lam_factor * dmin * dmin,
                    lam_factor=lam_factor)


def turb_384(n=384, nsteps=5000, lam_factor=0.1):
    return turbulence(n, mach_rms=0.4, nu=2.887e-3, seed=4, nsteps=nsteps, lam_factor=lam_factor)


def wake(n=(512, 256, 32), nsteps=4000, lam_factor=0.0, seed=2, delta=1.0):
    """Temporally developing wake; x cross-stream between slip walls, y streamwise, z span."""
    nn = tuple(n)
    dx0 = delta / 16.0
    L = tuple(nn[d] * dx0 for d in range(3))
    rng = np.random.default_rng(seed)
    cinf = 1.0
    Uinf, Uc = 0.85 * cinf, 0.5 * cinf
    x, y, z = cell_centres(nn, L)
    uy = Uinf - (Uinf - Uc) * np.exp(-(((x - 0.5 * L[0]) / delta) ** 2))
    kmax = math.pi / dx0
    pu, pv, pw = solenoidal_field(nn, L, rng, lambda k: np.where(k <= 0.5 * kmax, 1.0, 0.0))
    rms = math.sqrt(float(np.mean(pu * pu + pv * pv + pw * pw)) / 3.0)
    sc = 0.02 * Uinf / rms
    u, v, w = pu * sc, uy + pv * sc, pw * sc
    rho = np.ones_like(u)
    p = np.full_like(u, cinf * cinf / GAMMA)
    mu = 1.0 * Uinf * delta / 5e4
    dx = [L[d] / nn[d] for d in range(3)]
    dt = cfl_dt(rho, u, v, w, p, dx)
    w0 = conservative(rho, u, v, w, p)
    pinf = cinf * cinf / GAMMA
    minf = Uinf / cinf
    pt_ref = pinf * (1.0 + 0.5 * (GAMMA - 1.0) * minf * minf) ** (GAMMA / (GAMMA - 1.0))
    return Workload(f"wake_{nn[0]}x{nn[1]}x{nn[2]}", nn, L, mu, dt, w0, np.zeros_like(w0), nsteps,
                    OBJ_PT_LOSS_PLANE, window_weights(nsteps, 1, nsteps), lam=lam_factor * dx0 * dx0,
                    lam_factor=lam_factor, bc_x=1, plane_i=int(round(0.75 * nn[0])), pt_ref=pt_ref)


def spatial_wake(n=(512, 256, 32), nsteps=4000, lam_factor=0.0, seed=7, delta=1.0, mach=0.85, drag=0.05):
    """Spatially developing wake: x streamwise between a characteristic inlet (uniform free stream
    at Mach `mach`) and a characteristic outlet (the same far-field state), y cross-stream and z
    span periodic.  A streamwise body-force sink (peak `drag` U^2/delta, Gaussian of width delta
    across the stream and 2 cells along it, at x = 0.1 L_x) holds a wake deficit; the initial field
    carries that deficit downstream of the strip plus a 2 % solenoidal perturbation.  Objective: the density-
    weighted stagnation-pressure loss on the cross-stream plane at x = 0.75 L_x; the gradient is
    with respect to the body force (the source field)."""
    nn = tuple(n)
    dx0 = delta / 16.0
    L = tuple(nn[d] * dx0 for d in range(3))
    rng = np.random.default_rng(seed)
    cinf = 1.0
    Uinf, Uc = mach * cinf, 0.6 * mach * cinf
    x, y, z = cell_centres(nn, L)
    prof = np.exp(-(((y - 0.5 * L[1]) / delta) ** 2))
    ramp = 0.5 * (1.0 + np.tanh((x - 0.1 * L[0]) / (4.0 * dx0)))  # the deficit starts at the strip
    ux = Uinf - (Uinf - Uc) * prof * ramp
    kmax = math.pi / dx0
    pu, pv, pw = solenoidal_field(nn, L, rng, lambda k: np.where(k <= 0.5 * kmax, 1.0, 0.0))
    rms = math.sqrt(float(np.mean(pu * pu + pv * pv + pw * pw)) / 3.0)
    sc = 0.02 * Uinf / rms
    u, v, w = ux + pu * sc, pv * sc, pw * sc
    rho = np.ones_like(u)
    pinf = cinf * cinf / GAMMA
    p = np.full_like(u, pinf)
    mu = 1.0 * Uinf * delta / 5e4
    dx = [L[d] / nn[d] for d in range(3)]
    dt = cfl_dt(rho, u, v, w, p, dx)
    w0 = conservative(rho, u, v, w, p)
    # drag strip: momentum sink f_x and the work it does on the free stream, U_inf f_x
    fx = -drag * Uinf * Uinf / delta * prof * np.exp(-(((x - 0.1 * L[0]) / (2.0 * dx0)) ** 2))
    s = np.zeros_like(w0).reshape(5, -1)
    s[1] = fx.ravel()
    s[4] = Uinf * fx.ravel()
    far = conservative(np.ones(1), np.full(1, Uinf), np.zeros(1), np.zeros(1), np.full(1, pinf))
    minf = Uinf / cinf
    pt_ref = pinf * (1.0 + 0.5 * (GAMMA - 1.0) * minf * minf) ** (GAMMA / (GAMMA - 1.0))
    return Workload(f"spatial_wake_{nn[0]}x{nn[1]}x{nn[2]}", nn, L, mu, dt, w0, s.reshape(-1), nsteps,
                    OBJ_PT_LOSS_PLANE, window_weights(nsteps, 1, nsteps), lam=lam_factor * dx0 * dx0,
                    lam_factor=lam_factor, bc_x=2, plane_i=int(round(0.75 * nn[0])), pt_ref=pt_ref,
                    extra={"w_far": (tuple(far), tuple(far))})


def ensemble_draws(nboxes=64, seed_sizes=3, seed_windows=5, seed_lams=6):
    sizes = np.random.default_rng(seed_sizes).choice([32, 48, 64, 96], size=nboxes)
    windows = np.random.default_rng(seed_windows).integers(50, 401, size=nboxes)
    lams = np.random.default_rng(seed_lams).choice([0.0, 0.03, 0.1, 0.3, 1.0], size=nboxes)
    return [int(s) for s in sizes], [int(w) for w in windows], [float(l) for l in lams]


def random_state_perturbation(N, seed, scale=1.0):
    return scale * np.random.default_rng(seed).standard_normal(5 * N)
