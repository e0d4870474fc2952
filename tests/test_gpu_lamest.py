"""Choice of lambda from the adjoint-energy growth (paper_1511_06959_amd.lamest) against the same
steps taken on the FP64 oracle: the stored window, one homogeneous reverse sweep per candidate
from the same white-noise terminal adjoint, E_v^ after every reverse step, the least-squares
growth rate of log E_v^, and the smallest candidate whose rate is at or below the target.

Decaying turbulence on 12^3 (Mach_rms 0.3, nu 0.002): the plain adjoint (lambda 0) grows slowly
over the window and every candidate from 0.03 dx^2 on damps it.  The target rate is set half way
between two neighbouring oracle rates, so the decision is not a near tie."""
import numpy as np
import pytest

import paper_1511_06959_amd as adj
import workloads as W
from paper_1511_06959_amd import lamest

pytestmark = pytest.mark.gpu

FACTORS = [0.0, 0.03, 0.1, 0.3]
T = 24
SKIP = 0.25


def _oracle_energies(orc, og, traj, aT, lam):
    a = aT.copy()
    E = [orc.energy_vhat(og, traj[-1], a)[0]]
    for n in range(len(traj) - 2, -1, -1):
        a = orc.adjoint_step(og, traj[n], None, a, lam, None, 0.0, None)
        E.append(orc.energy_vhat(og, traj[n], a)[0])
    return np.array(E[::-1])  # E[n], n = 0..T


def _oracle_rate(E, dt):
    # least squares of log E against reverse time over n = 0 .. T - ceil(SKIP T)
    n0 = T - int(np.ceil(SKIP * T))
    tau = [(T - n) * dt for n in range(n0 + 1)]
    y = [np.log(E[n]) for n in range(n0 + 1)]
    return np.polyfit(tau, y, 1)[0]


@pytest.fixture(scope="module")
def case(orc):
    wl = W.turbulence(12, mach_rms=0.3, nu=0.002, seed=4, nsteps=T)
    og = orc.grid_from(wl.params())
    traj = orc.primal_window(og, wl.w0, None, T)
    aT = np.random.default_rng(5).standard_normal(wl.w0.size)
    dx2 = (wl.L[0] / 12) ** 2
    E = {f: _oracle_energies(orc, og, traj, aT, f * dx2) for f in FACTORS}
    rates = {f: _oracle_rate(E[f], wl.dt) for f in FACTORS}
    return wl, aT, E, rates


@pytest.mark.parametrize("pick", [0, 1, 2])
def test_estimate_matches_oracle(case, pick):
    wl, aT, E, rates = case
    assert rates[0.0] > 0.0 > rates[0.03] > rates[0.1] > rates[0.3]
    target = 0.5 * (rates[FACTORS[pick]] + rates[FACTORS[pick + 1]])
    expect = next(f for f in FACTORS if rates[f] <= target)
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F64)
    est = lamest.estimate_lambda(g, wl.w0, None, T, FACTORS, target_rate=target, skip=SKIP, aT=aT)
    assert est.factors == FACTORS and all(est.stable)
    for f in FACTORS:
        assert np.allclose(est.energies[f], E[f], rtol=1e-10, atol=0.0), f
        assert abs(est.rates[FACTORS.index(f)] - rates[f]) <= 1e-9 * max(abs(r) for r in rates.values())
    assert est.factor == expect
    assert est.lam == expect * (wl.L[0] / 12) ** 2


def test_refinement_narrows_the_bracket(case):
    wl, aT, E, rates = case
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F64)
    coarse = lamest.estimate_lambda(g, wl.w0, None, T, FACTORS, target_rate=0.0, skip=SKIP, aT=aT)
    fine = lamest.estimate_lambda(g, wl.w0, None, T, FACTORS, target_rate=0.0, skip=SKIP, aT=aT, refine=2,
                                  refine_points=3)
    assert coarse.factor == 0.03
    assert len(fine.factors) == len(FACTORS) + 6
    assert 0.0 < fine.factor <= coarse.factor
    k = fine.factors.index(fine.factor)
    assert fine.rates[k] <= 0.0 and fine.rates[k - 1] > 0.0
