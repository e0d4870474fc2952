"""torch.autograd forms on the GPU: gradcheck of the step and objective Functions (FP64,
finite differences of the GPU forward against the GPU adjoint), the checkpointed window equal
bitwise to the store-all sweep with the binomial recompute count, the window gradient against
the FP64 oracle, and finite differences along seeded directions."""
import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
from paper_1511_06959_amd import revolve, sweep
from paper_1511_06959_amd.sweep import SegmentSweep
from paper_1511_06959_amd.autograd import CheckpointedWindow, ObjectiveValue, PrimalStep, WindowSpec
import workloads as W
from tests.gpu_helpers import dev, host, smooth_state

pytestmark = pytest.mark.gpu


def _tiny(precision=adj.F64, n=(5, 4, 3), bc_x=0):
    L = (1.0, 0.8, 0.6)
    g = adj.Grid.make(n, L, 0.02, 2e-3, bc_x=bc_x, precision=precision)
    w = smooth_state(n, L, seed=21)
    return g, w


@pytest.mark.parametrize("bc_x", [0, 1])
def test_gradcheck_primal_step(bc_x):
    g, w = _tiny(bc_x=bc_x)
    spec = WindowSpec(g)
    wt = dev(w).requires_grad_(True)
    st = dev(1e-2 * np.random.default_rng(22).standard_normal(w.size)).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: PrimalStep.apply(a, b, spec), (wt, st), eps=1e-6, atol=1e-8,
                                    rtol=1e-6)


@pytest.mark.parametrize("kind", [W.OBJ_MEAN_PRESSURE, W.OBJ_KE_DISSIPATION, W.OBJ_PT_LOSS_PLANE])
def test_gradcheck_objective(kind):
    g, w = _tiny(n=(6, 4, 3), bc_x=1)
    spec = WindowSpec(g, obj=adj.Objective.make(kind, 3, 1.1))
    wt = dev(w).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a: ObjectiveValue.apply(a, spec), (wt,), eps=1e-6, atol=1e-9, rtol=1e-6)


def test_step_chain_matches_reverse_step():
    # three PrimalStep applications under autograd give the same gradient as adjoint_step
    g, w = _tiny(n=(9, 6, 5))
    spec = WindowSpec(g, obj=adj.Objective.make(W.OBJ_MEAN_PRESSURE))
    wt = dev(w).requires_grad_(True)
    x = wt
    for _ in range(3):
        x = PrimalStep.apply(x, None, spec)
    J = ObjectiveValue.apply(x, spec)
    J.backward()
    ws = adj.workspace(g)
    states = [dev(w)]
    for _ in range(3):
        nxt = torch.empty_like(states[-1])
        adj.primal_step(g, states[-1], None, nxt, ws)
        states.append(nxt)
    a = torch.zeros_like(states[0])
    adj.objective_and_grad(g, spec.obj, states[3], ws, weight=1.0, djdw=a)
    for n in (2, 1, 0):
        b = torch.empty_like(a)
        adj.adjoint_step(g, states[n], None, a, b, ws)
        a = b
    assert np.array_equal(host(wt.grad), host(a))


@pytest.mark.parametrize("slots", [2, 3, 5, 13])
def test_checkpointed_window_equals_store_all(slots):
    wl = W.tgv_small(n=16, nsteps=12)
    wl.weights = W.window_weights(12, 3, 12)
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F64)
    obj = adj.Objective.make(W.OBJ_KE_DISSIPATION)
    s = dev(1e-3 * np.random.default_rng(23).standard_normal(wl.w0.size))
    w0 = dev(wl.w0)
    ws = adj.workspace(g)
    traj, _, Jr = sweep.forward(g, w0, s, wl.nsteps, obj, wl.weights, ws)
    whr, gsr, _ = sweep.backward(g, traj, s, obj, wl.weights, 2e-3, ws)
    spec = WindowSpec(g, wl.nsteps, obj, list(wl.weights), lam=2e-3, slots=slots)
    w0t = w0.clone().requires_grad_(True)
    st = s.clone().requires_grad_(True)
    J = CheckpointedWindow.apply(w0t, st, spec)
    J.backward()
    assert float(J.detach()) == host(Jr)[0]
    assert np.array_equal(host(w0t.grad), host(whr))
    assert np.array_equal(host(st.grad), host(gsr))
    total = spec.last["forward_steps"] + spec.last["recompute_steps"]
    assert total == revolve.min_advances(wl.nsteps, slots) + 1  # +1: the step to the final state


def test_checkpointed_window_vs_oracle(orc):
    wl = W.tgv_small(n=16, nsteps=10)
    wl.weights = W.window_weights(10, 4, 10)
    og = orc.grid_from(wl.params())
    oobj = orc.make_obj(W.OBJ_MEAN_PRESSURE)
    traj = orc.primal_window(og, wl.w0, wl.s, wl.nsteps)
    J = orc.objective_window(og, oobj, traj, wl.weights)
    wh0, gs = orc.adjoint_window(og, oobj, traj, wl.s, wl.weights)
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F64)
    spec = WindowSpec(g, wl.nsteps, adj.Objective.make(W.OBJ_MEAN_PRESSURE), list(wl.weights), slots=3)
    w0t = dev(wl.w0).requires_grad_(True)
    st = dev(wl.s).requires_grad_(True)
    Jg = CheckpointedWindow.apply(w0t, st, spec)
    Jg.backward()
    assert abs(float(Jg) - J) <= 1e-12 * abs(J)
    assert np.linalg.norm(host(w0t.grad) - wh0) <= 1e-10 * np.linalg.norm(wh0)
    assert np.linalg.norm(host(st.grad) - gs) <= 1e-10 * np.linalg.norm(gs)


def test_window_gradient_finite_differences_turbulence():
    # decaying turbulence, mean pressure, lambda = 0: central differences along 4 seeded
    # directions of the body force agree with <dJ/ds, d> (FP64, binomial checkpointing)
    wl = W.turbulence(24, mach_rms=0.4, nu=0.01, seed=4, nsteps=20)
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, 0, adj.F64)
    spec = WindowSpec(g, wl.nsteps, adj.Objective.make(W.OBJ_MEAN_PRESSURE), list(wl.weights), slots=4)
    w0 = dev(wl.w0)
    s0 = torch.zeros_like(w0)
    st = s0.clone().requires_grad_(True)
    J = CheckpointedWindow.apply(w0, st, spec)
    J.backward()
    grad = host(st.grad)
    # J carries ~1e-15 of rounding: eps = 1e-5 would leave ~3e-6 of noise in the quotient
    eps = 1e-4
    for seed in range(10, 14):
        d = np.random.default_rng(seed).standard_normal(w0.numel())
        with torch.no_grad():
            Jp = float(CheckpointedWindow.apply(w0, s0 + eps * dev(d), spec))
            Jm = float(CheckpointedWindow.apply(w0, s0 - eps * dev(d), spec))
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - grad @ d) <= 1e-6 * abs(grad @ d) + 1e-12


@pytest.mark.parametrize("seg", [1, 3, 5, 12])
def test_segment_sweep_equals_store_all(seg):
    # two-level checkpointing with native snapshots: every re-advanced state and stage state equals
    # the forward sweep's, so J, dJ/dw_0 and dJ/ds equal the store-all sweep's bit for bit
    wl = W.tgv_small(n=16, nsteps=12)
    wl.weights = W.window_weights(12, 3, 12)
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F64)
    obj = adj.Objective.make(W.OBJ_KE_DISSIPATION)
    s = dev(1e-3 * np.random.default_rng(24).standard_normal(wl.w0.size))
    w0 = dev(wl.w0)
    ws = adj.workspace(g)
    traj, _, Jr = sweep.forward(g, w0, s, wl.nsteps, obj, wl.weights, ws)
    whr, gsr, _ = sweep.backward(g, traj, s, obj, wl.weights, 2e-3, ws)
    sw = SegmentSweep(g, wl.nsteps, seg, s, obj, wl.weights, 2e-3, ws)
    J = sw.forward(w0)
    wh, gs = sw.backward()
    assert host(J)[0] == host(Jr)[0]
    assert np.array_equal(host(wh), host(whr))
    assert np.array_equal(host(gs), host(gsr))
    assert sw.advanced == 2 * wl.nsteps and sw.nsnap == -(-wl.nsteps // seg)


def test_checkpointed_window_plans_from_free_hbm():
    # with no slots or segment given, the window takes the plan that the free HBM allows (here the
    # two-level plan of least memory) and records it
    wl = W.tgv_small(n=16, nsteps=12)
    wl.weights = W.window_weights(12, 3, 12)
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F64)
    obj = adj.Objective.make(W.OBJ_MEAN_PRESSURE)
    w0 = dev(wl.w0)
    ws = adj.workspace(g)
    traj, _, Jr = sweep.forward(g, w0, None, wl.nsteps, obj, wl.weights, ws)
    whr, _, _ = sweep.backward(g, traj, None, obj, wl.weights, 0.0, ws)
    spec = WindowSpec(g, wl.nsteps, obj, list(wl.weights))
    w0t = w0.clone().requires_grad_(True)
    J = CheckpointedWindow.apply(w0t, None, spec)
    J.backward()
    assert spec.last["schedule"] == "segments" and spec.last["segment"] == sweep.segment_length(g, wl.nsteps)
    assert spec.last["forward_steps"] == wl.nsteps and spec.last["recompute_steps"] == wl.nsteps
    assert float(J.detach()) == host(Jr)[0]
    assert np.array_equal(host(w0t.grad), host(whr))
    binom = WindowSpec(g, wl.nsteps, obj, list(wl.weights), schedule="binomial", reserve_bytes=0)
    assert binom.plan(w0.device)[0] == "binomial"
