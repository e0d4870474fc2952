"""Stability numbers (adj_stability / adj_check_stable) against their closed forms computed from
the state on the host, and the non-finite indication of the reductions (adj_check_status)."""
import math

import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
import workloads as W
from tests.gpu_helpers import dev, host, smooth_state

pytestmark = pytest.mark.gpu


def _case(orc, precision=adj.F64, weights=(0.5, 2.0, 1.0), bc_x=0, dt=0.004, scheme=adj.RK4):
    shape, L = (19, 6, 9), (2.0, 1.3, 1.7)
    g = adj.Grid.make(shape, L, 0.02, dt, bc_x=bc_x, precision=precision, nu_weight=weights, time_scheme=scheme)
    og = orc.make_grid(shape, L, 1.4, 0.72, 0.02, dt, bc_x)
    return g, og, smooth_state(shape, L, seed=40)


def _expected(g, w, sig_max, lam, wmax):
    N = g.ncells
    r = w[:N]
    u = [w[(1 + d) * N:(2 + d) * N] / r for d in range(3)]
    p = (g.gamma - 1.0) * (w[4 * N:] - 0.5 * r * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2))
    c = np.sqrt(g.gamma * p / r)
    idx = [g.n[d] / g.L[d] for d in range(3)]
    s4 = sum(4.0 * h * h for h in idx)
    conv = g.dt * np.max(sum((np.abs(u[d]) + c) * idx[d] for d in range(3)))
    alpha = g.gamma * g.mu / g.prandtl
    visc = g.dt * np.max(max(4.0 / 3.0 * g.mu, alpha) / r) * s4
    art = g.dt * lam * wmax * sig_max * s4
    return np.array([conv, visc, art])


@pytest.mark.parametrize("precision", [adj.F64, adj.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("bc_x", [0, 1], ids=["periodic", "walls"])
def test_stability_numbers(orc, precision, bc_x):
    g, og, w = _case(orc, precision, bc_x=bc_x)
    if precision == adj.F32:
        w = w.astype(np.float32).astype(np.float64)
    lam = 3e-3
    out = torch.zeros(3, dtype=torch.float64, device="cuda")
    ws = adj.workspace(g)
    adj.stability(g, dev(w, g.dtype), out, ws, lam=lam)
    sig = orc.sigma1(og, w).max()
    exp = _expected(g, w, sig, lam, 2.0)
    got = host(out)
    # FP32 grids carry gamma, mu and 1/dx in FP32 and sigma_1 is computed in FP32
    tol = 1e-12 if precision == adj.F64 else 2e-6
    assert np.allclose(got, exp, rtol=tol, atol=0.0)
    # no lambda: the artificial number is 0
    adj.stability(g, dev(w, g.dtype), out, ws)
    assert host(out)[2] == 0.0


@pytest.mark.parametrize("scheme", [adj.RK4, adj.SSPRK3], ids=["rk4", "ssprk3"])
def test_check_stable_bounds(orc, scheme):
    g, og, w = _case(orc, scheme=scheme)
    im, re = adj.stability_bounds(g)
    ws = adj.workspace(g)
    nums = adj.check_stable(g, dev(w), ws, lam=1e-3)
    assert max(nums[0] / im, nums[1] / re, nums[2] / re) < 1.0
    big_dt, *_ = _case(orc, dt=g.dt * 1.05 * im / nums[0], scheme=scheme)
    with pytest.raises(adj.AdjError) as e:
        adj.check_stable(big_dt, dev(w), ws)
    assert e.value.code == -3 and "convective" in str(e.value)
    if scheme == adj.SSPRK3:  # between the SSP-RK3 and the RK4 bound: RK4 would pass it
        mid_dt, *_ = _case(orc, dt=g.dt * 0.5 * (im + adj.RK4_IMAG_BOUND) / nums[0], scheme=scheme)
        with pytest.raises(adj.AdjError):
            adj.check_stable(mid_dt, dev(w), ws)
    lam_big = 1e-3 * 1.05 * re / nums[2]
    with pytest.raises(adj.AdjError) as e:
        adj.check_stable(g, dev(w), ws, lam=lam_big)
    assert e.value.code == -3 and "artificial" in str(e.value)


def test_nonfinite_reduction_is_reported_once(orc):
    g, og, w = _case(orc)
    ws = adj.workspace(g)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    wh = np.random.default_rng(41).standard_normal(w.size)
    adj.check_status()  # clears whatever earlier tests left
    adj.energy_vhat(g, dev(w), dev(wh), E, ws)
    adj.check_status()
    wh[123] = math.nan
    adj.energy_vhat(g, dev(w), dev(wh), E, ws)
    with pytest.raises(adj.AdjError) as e:
        adj.check_status()
    assert e.value.code == -4
    adj.check_status()  # cleared by the previous call
