"""Host logic of the lambda estimate (CPU): the growth-rate fit against closed forms and a
library least-squares fit, the choice rule, and the RK4 diffusion bound."""
import math

import numpy as np

import paper_1511_06959_amd as adj
from paper_1511_06959_amd.lamest import choose, growth_rate, lambda_bound


def test_growth_rate_of_an_exponential():
    dt, T, r = 0.013, 40, -1.7
    n = np.arange(T + 1)
    E = 3.2 * np.exp(r * (T - n) * dt)  # E[n] after T - n reverse steps
    assert abs(growth_rate(E, dt, 0.25) - r) <= 1e-12 * abs(r)
    # the fit leaves out the first ceil(0.25 T) = 10 reverse steps (n = 31..40) and no others
    E2 = E.copy()
    E2[31:] *= 50.0
    assert abs(growth_rate(E2, dt, 0.25) - r) <= 1e-12 * abs(r)
    E2[30] *= 50.0
    assert abs(growth_rate(E2, dt, 0.25) - r) > 1e-3


def test_growth_rate_is_the_least_squares_slope():
    rng = np.random.default_rng(3)
    dt, T = 0.02, 33
    E = np.exp(rng.standard_normal(T + 1))
    n0 = T - math.ceil(0.3 * T)
    tau = (T - np.arange(n0 + 1)) * dt
    ref = np.polyfit(tau, np.log(E[:n0 + 1]), 1)[0]
    assert abs(growth_rate(E, dt, 0.3) - ref) <= 1e-12 * abs(ref)


def test_choice_rule():
    f = [0.0, 0.1, 0.3, 1.0]
    r = [0.5, 0.1, -0.2, -1.0]
    st = [True, True, True, False]
    assert choose(f, r, st, 0.0) == 2
    assert choose(f, r, st, 0.2) == 1
    assert choose(f, r, st, 1.0) == 0
    assert choose(f, r, st, -0.5) is None  # only the unstable candidate damps that much


def test_lambda_bound_is_the_rk4_diffusion_limit():
    n, L = 16, 2 * math.pi
    g = adj.Grid.make((n, n, n), (L, L, L), 0.01, 0.01, nu_weight=(0.5, 2.0, 1.0))
    dx = L / n
    sig = 2.0
    lam = lambda_bound(g, sig)
    # nu_max = lam * max weight * sigma; explicit RK4 needs nu_max dt sum_d 4/dx^2 <= 2.785,
    # i.e. nu_max dt / dx^2 <= 0.232 on a cube
    assert abs(lam * 2.0 * sig * g.dt / dx ** 2 - 2.785 / 12.0) <= 1e-12


def test_ensemble_plan_groups():
    from paper_1511_06959_amd.ensemble import plan, trajectory_bytes
    grids = [adj.Grid.make((n, n, n), (1.0, 1.0, 1.0), 0.01, 0.01, precision=adj.F32) for n in (16, 8, 8, 4)]
    windows = [10, 10, 5, 2]
    member_box = [0, 0, 1, 2, 3, 3]
    per = [trajectory_bytes([g], [t]) for g, t in zip(grids, windows)]
    assert per[0] == 5 * 16 ** 3 * 11 * 4
    assert plan(grids, windows, member_box, sum(per)) == [(0, 4, 0, 6)]
    groups = plan(grids, windows, member_box, per[0])
    assert groups[0] == (0, 1, 0, 2)
    assert [g[:2] for g in groups] == [(0, 1), (1, 4)]  # the three smaller boxes fit together
    assert [g[:2] for g in plan(grids, windows, member_box, per[1] + per[2])] == [(0, 1), (1, 3), (3, 4)]
    # every box and member exactly once, in order
    assert groups[-1][1] == 4 and groups[-1][3] == 6
    assert all(a[1] == b[0] and a[3] == b[2] for a, b in zip(groups, groups[1:]))
    # a box larger than the budget alone
    assert plan(grids, windows, member_box, 1)[0] == (0, 1, 0, 2)
