"""The paper's time marching, strong-stability-preserving RK3 (adj_grid.time_scheme = SSPRK3),
against the FP64 oracle's Shu-Osher stages: single primal and reverse steps (every objective,
lambda 0 and > 0, periodic and walls), FP32 operators, the stored-stage schedule, and a whole
16^3 window to the FP64 target."""
import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
import workloads as W
from paper_1511_06959_amd import sweep
from tests.gpu_helpers import dev, host, relerr, smooth_state

pytestmark = pytest.mark.gpu

SHAPE, L = (19, 6, 9), (2.0, 1.3, 1.7)


def _case(orc, bc_x, precision=adj.F64, seed=50):
    g = adj.Grid.make(SHAPE, L, 0.02, 0.004, bc_x=bc_x, precision=precision, time_scheme=adj.SSPRK3)
    og = orc.make_grid(SHAPE, L, 1.4, 0.72, 0.02, 0.004, bc_x, scheme=1)
    return g, og, smooth_state(SHAPE, L, seed=seed)


@pytest.mark.parametrize("bc_x", [0, 1], ids=["periodic", "walls"])
def test_primal_step(orc, bc_x):
    g, og, w = _case(orc, bc_x)
    s = 1e-2 * np.random.default_rng(51).standard_normal(w.size)
    out = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.primal_step(g, dev(w), dev(s), out, adj.workspace(g))
    ref = orc.primal_step(og, w, s)
    assert relerr(host(out) - w, ref - w) <= 1e-12
    # not the RK4 step
    g4 = orc.make_grid(SHAPE, L, 1.4, 0.72, 0.02, 0.004, bc_x)
    assert relerr(orc.primal_step(g4, w, s) - w, ref - w) > 1e-6


OBJS = [(W.OBJ_NONE, 0), (W.OBJ_MEAN_PRESSURE, 0), (W.OBJ_KE_DISSIPATION, 1), (W.OBJ_PT_LOSS_PLANE, 1)]


@pytest.mark.parametrize("kind,bc_x", OBJS, ids=["none", "meanp", "ked-walls", "ptloss-walls"])
@pytest.mark.parametrize("lam", [0.0, 3e-3], ids=["lam0", "lam"])
def test_adjoint_step(orc, kind, bc_x, lam):
    g, og, w = _case(orc, bc_x, seed=52)
    rng = np.random.default_rng(53)
    s = 1e-2 * rng.standard_normal(w.size)
    a = rng.standard_normal(w.size)
    gs0 = rng.standard_normal(w.size)
    obj, oobj = adj.Objective.make(kind, 7, 1.1), orc.make_obj(kind, 7, 1.1)
    ws = adj.workspace(g)
    wh = torch.empty(w.size, dtype=torch.float64, device="cuda")
    gs = dev(gs0)
    adj.adjoint_step(g, dev(w), dev(s), dev(a), wh, ws, lam=lam, obj=obj, c_n=0.37, grad_s=gs)
    gref = gs0.copy()
    ref = orc.adjoint_step(og, w, s, a, lam, oobj, 0.37, gref)
    assert relerr(host(wh) - a, ref - a) <= 1e-12
    assert relerr(host(gs) - gs0, gref - gs0) <= 1e-12
    # the stored-stage schedule reads the same stage states
    st = torch.empty(3 * w.size, dtype=torch.float64, device="cuda")
    w1 = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.primal_step_stages(g, dev(w), dev(s), w1, st, ws)
    wh2 = torch.empty_like(wh)
    gs2 = dev(gs0)
    adj.adjoint_step_stages(g, dev(w), st, dev(s), dev(a), wh2, ws, lam=lam, obj=obj, c_n=0.37, grad_s=gs2)
    assert torch.equal(wh2, wh) and torch.equal(gs2, gs)
    assert relerr(host(w1) - w, orc.primal_step(og, w, s) - w) <= 1e-12


def test_fp32_step(orc):
    g, og, w = _case(orc, 0, precision=adj.F32, seed=54)
    rng = np.random.default_rng(55)
    w = w.astype(np.float32).astype(np.float64)
    a = rng.standard_normal(w.size).astype(np.float32).astype(np.float64)
    ws = adj.workspace(g)
    wh = torch.empty(w.size, dtype=torch.float32, device="cuda")
    gs = torch.zeros(w.size, dtype=torch.float32, device="cuda")
    adj.adjoint_step(g, dev(w, torch.float32), None, dev(a, torch.float32), wh, ws, lam=3e-3, grad_s=gs)
    gref = np.zeros(w.size)
    ref = orc.adjoint_step(og, w, None, a, 3e-3, None, 0.0, gref)
    assert relerr(host(wh) - a, ref - a) <= 1e-5
    assert relerr(host(gs), gref) <= 1e-5


def test_window_16cubed(orc):
    wl = W.tgv_small(n=16, nsteps=50)
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F64, time_scheme=adj.SSPRK3)
    p = wl.params()
    p["scheme"] = 1
    og = orc.grid_from(p)
    obj = adj.Objective.make(wl.obj_kind)
    ws = adj.workspace(g)
    w0 = dev(wl.w0)
    traj, _, J = sweep.forward(g, w0, None, wl.nsteps, obj, wl.weights, ws)
    wh0, gs, _ = sweep.backward(g, traj, None, obj, wl.weights, 0.0, ws)
    otraj = orc.primal_window(og, wl.w0, None, wl.nsteps)
    Jr = orc.objective_window(og, orc.make_obj(wl.obj_kind), otraj, wl.weights)
    whr, gsr = orc.adjoint_window(og, orc.make_obj(wl.obj_kind), otraj, None, wl.weights)
    assert abs(host(J)[0] - Jr) <= 1e-10 * abs(Jr)
    assert np.linalg.norm(host(wh0) - whr) <= 1e-10 * np.linalg.norm(whr)
    assert np.linalg.norm(host(gs) - gsr) <= 1e-10 * np.linalg.norm(gsr)
