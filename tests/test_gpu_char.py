"""Characteristic inflow/outflow boundaries in x (adj_grid.bc_x = BC_CHARACTERISTIC) against the
FP64 oracle: the residual and its transpose, single primal and reverse steps (split-form and Roe
fluxes, RK4 and SSP-RK3, every objective, lambda 0 and > 0), tiny grids, FP32 with stored
deviations, and a whole 16^3 window with a source field.  The far-field states differ at the two
ends and from the interior, so the boundary faces carry real jumps."""
import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
import workloads as W
from paper_1511_06959_amd import sweep
from tests.gpu_helpers import dev, host, relerr, smooth_state

pytestmark = pytest.mark.gpu

SHAPE, L, MU, DT, DELTA = (37, 9, 6), (2.0, 1.3, 1.7), 0.02, 0.004, 0.1


def _cons(rho, u, p, gamma=1.4):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (gamma - 1.0) + 0.5 * rho * (u @ u)])


FAR = (_cons(1.02, [0.3, 0.02, -0.01], 0.72), _cons(0.98, [0.28, -0.01, 0.0], 0.70))


def _grids(orc, shape=SHAPE, precision=adj.F64, scheme=adj.RK4, flux=adj.FLUX_SPLIT, w_ref=None):
    g = adj.Grid.make(shape, L, MU, DT, bc_x=adj.BC_CHARACTERISTIC, precision=precision, w_ref=w_ref,
                      time_scheme=scheme, flux=flux, roe_delta=DELTA, w_far=FAR)
    og = orc.make_grid(shape, L, 1.4, 0.72, MU, DT, orc.BC_CHARACTERISTIC, scheme, flux, DELTA, np.concatenate(FAR))
    return g, og


def _state(shape, seed):
    return smooth_state(shape, L, seed=seed)


@pytest.mark.parametrize("flux", [adj.FLUX_SPLIT, adj.FLUX_ROE], ids=["split", "roe"])
def test_residual_and_transpose(orc, flux):
    g, og = _grids(orc, flux=flux)
    w = _state(SHAPE, 90)
    rng = np.random.default_rng(91)
    s = rng.standard_normal(w.size)
    R = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.residual(g, dev(w), dev(s), R)
    ref = orc.residual(og, w, s)
    assert relerr(host(R) - s, ref - s) <= 1e-12
    # the boundary faces differ from slip walls
    owall = orc.make_grid(SHAPE, L, 1.4, 0.72, MU, DT, 1, 0, flux, DELTA)
    assert relerr(orc.residual(owall, w, s) - s, ref - s) > 1e-4
    kh = rng.standard_normal(w.size)
    out = torch.empty_like(R)
    adj.vjp(g, dev(w), dev(kh), out)
    assert relerr(host(out), orc.vjp(og, w, kh)) <= 1e-12


@pytest.mark.parametrize("scheme", [adj.RK4, adj.SSPRK3], ids=["rk4", "ssprk3"])
@pytest.mark.parametrize("flux", [adj.FLUX_SPLIT, adj.FLUX_ROE], ids=["split", "roe"])
def test_primal_step(orc, flux, scheme):
    g, og = _grids(orc, flux=flux, scheme=scheme)
    w = _state(SHAPE, 92)
    s = 1e-2 * np.random.default_rng(93).standard_normal(w.size)
    out = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.primal_step(g, dev(w), dev(s), out, adj.workspace(g))
    ref = orc.primal_step(og, w, s)
    assert relerr(host(out) - w, ref - w) <= 1e-12


OBJS = [(W.OBJ_PT_LOSS_PLANE, 0.0), (W.OBJ_KE_DISSIPATION, 3e-3), (W.OBJ_MEAN_PRESSURE, 3e-3)]


@pytest.mark.parametrize("scheme", [adj.RK4, adj.SSPRK3], ids=["rk4", "ssprk3"])
@pytest.mark.parametrize("flux", [adj.FLUX_SPLIT, adj.FLUX_ROE], ids=["split", "roe"])
@pytest.mark.parametrize("kind,lam", OBJS, ids=["ptloss", "ked-lam", "meanp-lam"])
def test_adjoint_step(orc, kind, lam, flux, scheme):
    g, og = _grids(orc, flux=flux, scheme=scheme)
    w = _state(SHAPE, 94)
    rng = np.random.default_rng(95)
    s = 1e-2 * rng.standard_normal(w.size)
    a = rng.standard_normal(w.size)
    gs0 = rng.standard_normal(w.size)
    obj, oobj = adj.Objective.make(kind, 25, 1.1), orc.make_obj(kind, 25, 1.1)
    ws = adj.workspace(g)
    wh = torch.empty(w.size, dtype=torch.float64, device="cuda")
    gs = dev(gs0)
    adj.adjoint_step(g, dev(w), dev(s), dev(a), wh, ws, lam=lam, obj=obj, c_n=0.37, grad_s=gs)
    gref = gs0.copy()
    ref = orc.adjoint_step(og, w, s, a, lam, oobj, 0.37, gref)
    assert relerr(host(wh) - a, ref - a) <= 1e-12
    assert relerr(host(gs) - gs0, gref - gs0) <= 1e-12


@pytest.mark.parametrize("shape", [(2, 3, 1), (3, 1, 2), (5, 2, 3)], ids=["2x3x1", "3x1x2", "5x2x3"])
@pytest.mark.parametrize("flux", [adj.FLUX_SPLIT, adj.FLUX_ROE], ids=["split", "roe"])
def test_tiny_grids(orc, shape, flux):
    g, og = _grids(orc, shape=shape, flux=flux)
    w = _state(shape, 96)
    a = np.random.default_rng(97).standard_normal(w.size)
    R = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.residual(g, dev(w), None, R)
    ref = orc.residual(og, w)
    assert np.abs(host(R) - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    wh = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.adjoint_step(g, dev(w), None, dev(a), wh, adj.workspace(g), lam=2e-3)
    refa = orc.adjoint_step(og, w, None, a, 2e-3, None, 0.0, None)
    assert np.abs(host(wh) - refa).max() <= 1e-12 * np.abs(refa - a).max() + 1e-14 * np.abs(a).max()


@pytest.mark.parametrize("flux", [adj.FLUX_SPLIT, adj.FLUX_ROE], ids=["split", "roe"])
def test_fp32_stored_deviations(orc, flux):
    w = _state(SHAPE, 98)
    ref = adj.reference_state(w)
    g, og = _grids(orc, precision=adj.F32, flux=flux, w_ref=ref)
    stored = g.to_stored(w).astype(np.float32)
    w = g.from_stored(stored.astype(np.float64))
    a = np.random.default_rng(99).standard_normal(w.size).astype(np.float32).astype(np.float64)
    ws = adj.workspace(g)
    out = torch.empty(w.size, dtype=torch.float32, device="cuda")
    adj.primal_step(g, dev(stored, torch.float32), None, out, ws)
    assert relerr(g.from_stored(host(out)) - w, orc.primal_step(og, w) - w) <= 1e-5
    gs = torch.zeros(w.size, dtype=torch.float32, device="cuda")
    adj.adjoint_step(g, dev(stored, torch.float32), None, dev(a, torch.float32), out, ws, lam=3e-3, grad_s=gs)
    gref = np.zeros(w.size)
    refa = orc.adjoint_step(og, w, None, a, 3e-3, None, 0.0, gref)
    assert relerr(host(out) - a, refa - a) <= 1e-5
    assert relerr(host(gs), gref) <= 1e-5


@pytest.mark.parametrize("flux", [adj.FLUX_SPLIT, adj.FLUX_ROE], ids=["split", "roe"])
def test_window_16cubed(orc, flux):
    shape, nsteps = (16, 16, 16), 30
    g, og = _grids(orc, shape=shape, flux=flux)
    w0 = _state(shape, 100)
    s = 1e-2 * np.random.default_rng(101).standard_normal(w0.size)
    weights = W.window_weights(nsteps, 1, nsteps)
    obj = adj.Objective.make(W.OBJ_PT_LOSS_PLANE, 12, 1.1)
    oobj = orc.make_obj(W.OBJ_PT_LOSS_PLANE, 12, 1.1)
    ws = adj.workspace(g)
    traj, _, J = sweep.forward(g, dev(w0), dev(s), nsteps, obj, weights, ws)
    wh0, gs, _ = sweep.backward(g, traj, dev(s), obj, weights, 0.0, ws)
    otraj = orc.primal_window(og, w0, s, nsteps)
    Jr = orc.objective_window(og, oobj, otraj, weights)
    whr, gsr = orc.adjoint_window(og, oobj, otraj, s, weights)
    assert abs(host(J)[0] - Jr) <= 1e-10 * abs(Jr)
    assert np.linalg.norm(host(wh0) - whr) <= 1e-10 * np.linalg.norm(whr)
    assert np.linalg.norm(host(gs) - gsr) <= 1e-10 * np.linalg.norm(gsr)
