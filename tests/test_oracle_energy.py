"""Adjoint-energy behaviour of the stabilised adjoint (CPU oracle, statistical pin).

Following the paper's stabilisation results: added adjoint viscosity lambda sigma_1 damps the
adjoint energy E_v^ of a backward sweep; for lambda large enough (inside the explicit RK4
diffusion bound) the energy does not grow over the window and ends far below the
lambda = 0 sweep started from the same terminal adjoint.  Resolved decaying turbulence, 16^3."""
import numpy as np

import workloads as W


def _sweep_energy(orc, g, traj, aN, lam):
    a = aN.copy()
    E = [orc.energy_vhat(g, traj[-1], a)[0]]
    for n in range(len(traj) - 2, -1, -1):
        a = orc.adjoint_step(g, traj[n], None, a, lam, None, 0.0, None)
        E.append(orc.energy_vhat(g, traj[n], a)[0])
    return np.array(E)


def test_large_lambda_stops_energy_growth(orc):
    wl = W.turbulence(16, mach_rms=0.3, nu=0.02, seed=4, nsteps=30)
    g = orc.grid_from(wl.params())
    traj = orc.primal_window(g, wl.w0, None, wl.nsteps)
    dx = wl.L[0] / 16
    sig_max = orc.sigma1(g, wl.w0).max()
    lam_big = 3.0 * dx * dx
    assert lam_big * sig_max * wl.dt / (dx * dx) < 0.232  # inside the RK4 diffusion bound
    aN = np.random.default_rng(0).standard_normal(wl.w0.size)
    E0 = _sweep_energy(orc, g, traj, aN, 0.0)
    Eb = _sweep_energy(orc, g, traj, aN, lam_big)
    assert np.all(np.isfinite(E0)) and np.all(np.isfinite(Eb))
    # no growth: every later value below the terminal one, late-window log-slope not positive
    assert Eb[1:].max() <= Eb[0]
    k = np.arange(len(Eb))
    assert np.polyfit(k[10:], np.log(Eb[10:]), 1)[0] <= 0.0
    # strongly damped compared with the plain adjoint from the same terminal field
    assert Eb[-1] < 0.05 * E0[-1]
