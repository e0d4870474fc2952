"""Batched ensembles (adj_batch_*): every member of one batched sweep equals the same box run
alone through the single-box calls, bit for bit in the fields (the per-cell arithmetic is the
same kernel body) and to rounding in the FP64 scalars (partial sums in another order)."""
import math

import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
from paper_1511_06959_amd import sweep
from paper_1511_06959_amd.ensemble import CapturedEnsemble, EnsembleWindow, PlannedEnsemble, trajectory_bytes
import workloads as W
from tests.gpu_helpers import host, smooth_state

pytestmark = pytest.mark.gpu


def _periodic_boxes():
    # uneven cubes (ragged against every tile shape), windows non-increasing, a lambda sweep on box 0
    sizes, windows = [12, 8, 16, 10], [6, 5, 5, 2]
    wls = [W.turbulence(n, mach_rms=0.3, nu=0.02, seed=50 + i, nsteps=windows[i]) for i, n in enumerate(sizes)]
    member_box = [0, 0, 1, 2, 2, 3]
    member_lam = [0.0, 0.5, 0.0, 0.3, 1.0, 0.0]
    return wls, windows, member_box, member_lam


def _wall_boxes():
    # slip walls in x; a lambda sweep on both boxes
    out = []
    for i, (n, T) in enumerate([((12, 8, 6), 4), ((10, 6, 4), 3)]):
        L = (2.0, 1.5, 1.0)
        wl = W.Workload(f"walls_{i}", n, L, 0.01, 0.0, smooth_state(n, L, seed=60 + i), None, T,
                        W.OBJ_MEAN_PRESSURE, W.window_weights(T, 1, T), bc_x=1)
        dx = [L[d] / n[d] for d in range(3)]
        wl.dt = 0.3 * min(dx) / 2.0
        out.append(wl)
    return out, [4, 3], [0, 0, 1, 1], [0.0, 0.4, 0.2, 0.0]


def _grid(wl, precision):
    return adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, precision)


def _sources(wls, seed):
    rng = np.random.default_rng(seed)
    return [None if i % 2 else 1e-3 * rng.standard_normal(wl.w0.size) for i, wl in enumerate(wls)]


def _single(wl, T, lam, s, precision):
    g = _grid(wl, precision)
    dt = g.dtype
    obj = adj.Objective.make(adj.OBJ_MEAN_PRESSURE)
    ws = adj.workspace(g)
    weights = W.window_weights(T, 1, T)
    w0 = torch.from_numpy(wl.w0).to("cuda", dt)
    sd = None if s is None else torch.from_numpy(s).to("cuda", dt)
    traj, _, J = sweep.forward(g, w0, sd, T, obj, weights, ws)
    wh0, gs, E = sweep.backward(g, traj, sd, obj, weights, lam, ws, energy=True)
    return host(J)[0], host(wh0), host(gs), host(E)


@pytest.mark.parametrize("precision", [adj.F64, adj.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("case", ["periodic", "walls"])
def test_members_equal_single_box_runs(case, precision):
    wls, windows, member_box, factors = _periodic_boxes() if case == "periodic" else _wall_boxes()
    grids = [_grid(wl, precision) for wl in wls]
    lams = []
    for m, b in enumerate(member_box):
        dx = min(wls[b].L[d] / wls[b].n[d] for d in range(3))
        lams.append(factors[m] * dx * dx)
    s = _sources(wls, 70)
    win = EnsembleWindow(grids, windows, [wl.w0 for wl in wls], s, member_box, lams, energy=True)
    win.forward()
    wh0, gs = win.backward()
    J, wh0, gs, E = host(win.J), host(wh0), host(gs), host(win.E)
    for m, b in enumerate(member_box):
        T = windows[b]
        Js, whs, gss, Es = _single(wls[b], T, lams[m], s[b], precision)
        lo, hi = 5 * win.ens.offset(1, m), 5 * win.ens.offset(1, m + 1)
        assert np.array_equal(wh0[lo:hi], whs), f"member {m}: w^_0"
        assert np.array_equal(gs[lo:hi], gss), f"member {m}: grad_s"
        assert abs(J[m] - Js) <= 1e-14 * abs(Js), f"member {m}: J {J[m]} vs {Js}"
        assert np.allclose(E[:T + 1, m], Es, rtol=1e-13, atol=0.0), f"member {m}: adjoint energy"


def test_captured_ensemble_replays_match_eager():
    wls, windows, member_box, factors = _periodic_boxes()
    grids = [_grid(wl, adj.F32) for wl in wls]
    lams = [f * (2 * math.pi / wls[b].n[0]) ** 2 for f, b in zip(factors, member_box)]
    win = EnsembleWindow(grids, windows, [wl.w0 for wl in wls], _sources(wls, 71), member_box, lams)
    win.forward()
    wh, gs = win.backward()
    Je, whe, gse = host(win.J), host(wh), host(gs)
    cap = CapturedEnsemble(win)
    tmp = torch.empty_like(win.a)
    for _ in range(3):
        J, wh, gs = cap.run()
        assert np.array_equal(host(J), Je)
        assert np.array_equal(host(wh), whe)
        assert np.array_equal(host(gs), gse)
        tmp.copy_(win.b)  # unrelated eager work between replays
        torch.cuda.synchronize()


def test_ensemble_rejects_bad_orderings():
    wls, windows, member_box, factors = _periodic_boxes()
    grids = [_grid(wl, adj.F64) for wl in wls]
    with pytest.raises(ValueError):
        EnsembleWindow(grids, windows[::-1], [wl.w0 for wl in wls])
    with pytest.raises(adj.AdjError):
        adj.Ensemble(grids, [1, 0], [0.0, 0.0])
    mixed = grids[:1] + [_grid(wls[1], adj.F32)]
    with pytest.raises(adj.AdjError):
        adj.Ensemble(mixed, [0, 1], [0.0, 0.0])


def test_planned_groups_equal_single_ensemble():
    wls, windows, member_box, factors = _periodic_boxes()
    grids = [_grid(wl, adj.F64) for wl in wls]
    lams = [f * (2 * math.pi / wls[b].n[0]) ** 2 for f, b in zip(factors, member_box)]
    s = _sources(wls, 72)
    win = EnsembleWindow(grids, windows, [wl.w0 for wl in wls], s, member_box, lams)
    win.forward()
    wh, gs = win.backward()
    J, wh, gs = host(win.J), host(wh), host(gs)
    # a budget that holds the first box's trajectory but not the first two
    budget = trajectory_bytes(grids[:1], windows[:1]) + 1
    pe = PlannedEnsemble(grids, windows, [wl.w0 for wl in wls], s, member_box, lams, budget_bytes=budget)
    assert len(pe.groups) >= 3 and pe.groups[0][:2] == (0, 1)
    pe.run()
    for m in range(len(member_box)):
        Jm, whm, gsm = pe.results(m)
        lo, hi = 5 * win.ens.offset(1, m), 5 * win.ens.offset(1, m + 1)
        assert Jm == J[m], f"member {m}: J"
        assert np.array_equal(whm.double().numpy(), wh[lo:hi]), f"member {m}: w^_0"
        assert np.array_equal(gsm.double().numpy(), gs[lo:hi]), f"member {m}: grad_s"


def _wake_like(n=(24, 12, 8), T=10, seed=80):
    # a small box between slip walls with a shear layer, the stagnation-pressure loss on an x-face
    L = (2.0, 1.0, 0.7)
    w = smooth_state(n, L, seed=seed, wall=True)
    dx = [L[d] / n[d] for d in range(3)]
    wl = W.Workload("wake_like", n, L, 2e-3, 0.25 * min(dx) / 2.0, w, None, T, W.OBJ_PT_LOSS_PLANE,
                    W.window_weights(T, 1, T), bc_x=1, plane_i=3 * n[0] // 4, pt_ref=1.05)
    return wl


@pytest.mark.parametrize("ckpt", [adj.CKPT_BF16, adj.CKPT_NATIVE], ids=["bf16", "native"])
def test_lambda_sweep_members_equal_single_sweeps(ckpt):
    # several lambdas swept backward together over one stored trajectory (BF16 records decoded once
    # per step): every member equals the single-box reverse sweep with its lambda bit for bit
    from paper_1511_06959_amd.ensemble import LambdaSweep
    wl = _wake_like()
    ref = adj.reference_state(wl.w0)
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F32, ckpt, ref)
    obj = adj.Objective.make(wl.obj_kind, wl.plane_i, wl.pt_ref)
    dx = min(wl.L[d] / wl.n[d] for d in range(3))
    lams = [0.0, 0.1 * dx * dx, 1.0 * dx * dx]
    s = torch.from_numpy(1e-3 * np.random.default_rng(81).standard_normal(wl.w0.size)).to("cuda", torch.float32)
    ws = adj.workspace(g)
    traj, _, _ = sweep.forward(g, torch.from_numpy(g.to_stored(wl.w0)).to("cuda", torch.float32), s, wl.nsteps, obj,
                               wl.weights, ws)
    ls = LambdaSweep(g, traj, lams, obj, wl.weights, s=s, energy=True)
    wh, gs = ls.backward()
    wh, gs, E = host(wh), host(gs), host(ls.E)
    for m, lam in enumerate(lams):
        whs, gss, Es = sweep.backward(g, traj, s, obj, wl.weights, lam, ws, energy=True)
        lo, hi = 5 * ls.ens.offset(1, m), 5 * ls.ens.offset(1, m + 1)
        assert np.array_equal(wh[lo:hi], host(whs)), f"member {m}: w^_0"
        assert np.array_equal(gs[lo:hi], host(gss)), f"member {m}: grad_s"
        assert np.allclose(E[:, m], host(Es), rtol=1e-13, atol=0.0), f"member {m}: adjoint energy"


def test_lambda_sweep_vs_oracle(orc):
    # FP64 native trajectory, three lambdas at once, against the oracle's window for each lambda
    from paper_1511_06959_amd.ensemble import LambdaSweep
    wl = _wake_like(n=(20, 10, 6), T=8, seed=82)
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, adj.F64)
    obj = adj.Objective.make(wl.obj_kind, wl.plane_i, wl.pt_ref)
    dx = min(wl.L[d] / wl.n[d] for d in range(3))
    lams = [0.0, 0.3 * dx * dx, 1.0 * dx * dx]
    ws = adj.workspace(g)
    traj, _, _ = sweep.forward(g, torch.from_numpy(wl.w0).to("cuda"), None, wl.nsteps, obj, wl.weights, ws)
    ls = LambdaSweep(g, traj, lams, obj, wl.weights)
    wh, gs = ls.backward()
    wh, gs = host(wh), host(gs)
    og = orc.grid_from(wl.params())
    oobj = orc.make_obj(wl.obj_kind, wl.plane_i, wl.pt_ref)
    otraj = orc.primal_window(og, wl.w0, None, wl.nsteps)
    for m, lam in enumerate(lams):
        who, gso = orc.adjoint_window(og, oobj, otraj, None, wl.weights, lam)
        lo, hi = 5 * ls.ens.offset(1, m), 5 * ls.ens.offset(1, m + 1)
        assert np.linalg.norm(wh[lo:hi] - who) <= 1e-10 * np.linalg.norm(who), f"member {m}: w^_0"
        assert np.linalg.norm(gs[lo:hi] - gso) <= 1e-10 * np.linalg.norm(gso), f"member {m}: grad_s"
