"""The scheme options (Roe flux, characteristic inlet/outlet, SSP-RK3) through the window machinery:
captured HIP-graph windows replay the eager window bit for bit, stored stage states equal their
recomputation, the binomially checkpointed window equals the store-all sweep, host-memory
trajectories equal the HBM sweeps, BF16 records on these grids, and gradcheck of the autograd step
(FP64 finite differences of the GPU forward against the GPU adjoint).  Each option's parity with
the oracle is tested in test_gpu_roe.py and test_gpu_char.py."""
import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
import workloads as W
from paper_1511_06959_amd import offload, sweep
from paper_1511_06959_amd.autograd import CheckpointedWindow, PrimalStep, WindowSpec
from tests.gpu_helpers import dev, host, smooth_state

pytestmark = pytest.mark.gpu

SHAPE, L = (16, 8, 8), (2.0, 1.0, 1.0)
NSTEPS = 8


def _cons(rho, u, p, gamma=1.4):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (gamma - 1.0) + 0.5 * rho * (u @ u)])


FAR = (_cons(1.02, [0.3, 0.02, -0.01], 0.72), _cons(0.98, [0.28, -0.01, 0.0], 0.70))
OPTIONS = {
    "roe-char-rk4": dict(flux=adj.FLUX_ROE, bc_x=adj.BC_CHARACTERISTIC, time_scheme=adj.RK4),
    "split-char-ssprk3": dict(flux=adj.FLUX_SPLIT, bc_x=adj.BC_CHARACTERISTIC, time_scheme=adj.SSPRK3),
    "roe-periodic-ssprk3": dict(flux=adj.FLUX_ROE, bc_x=adj.BC_PERIODIC, time_scheme=adj.SSPRK3),
}


def _grid(opt, precision=adj.F64, ckpt=adj.CKPT_NATIVE, w_ref=None, shape=SHAPE):
    o = OPTIONS[opt]
    return adj.Grid.make(shape, L, 0.02, 4e-3, bc_x=o["bc_x"], precision=precision, ckpt_format=ckpt, w_ref=w_ref,
                         time_scheme=o["time_scheme"], flux=o["flux"], roe_delta=0.1, w_far=FAR)


def _inputs(g, seed, dt=torch.float64):
    w = smooth_state(tuple(g.n), L, seed=seed)
    s = 1e-3 * np.random.default_rng(seed + 1).standard_normal(w.size)
    return dev(g.to_stored(w), dt), dev(s, dt)


OBJ = adj.Objective.make(W.OBJ_PT_LOSS_PLANE, 11, 1.1)
WEIGHTS = W.window_weights(NSTEPS, 1, NSTEPS)


@pytest.mark.parametrize("opt", sorted(OPTIONS))
def test_captured_window_and_stored_stages(opt):
    g = _grid(opt)
    w0, s = _inputs(g, 110)
    ws = adj.workspace(g)
    res = []
    for stages in (False, True):
        traj = sweep.Trajectory(g, NSTEPS, stages=stages)
        _, _, J = sweep.forward(g, w0, s, NSTEPS, OBJ, WEIGHTS, ws, traj=traj)
        wh, gs, _ = sweep.backward(g, traj, s, OBJ, WEIGHTS, 2e-3, ws)
        res.append((host(J), host(wh), host(gs)))
    for x, y in zip(*res):
        assert np.array_equal(x, y)
    cw = sweep.CapturedWindow(g, w0, s, NSTEPS, OBJ, WEIGHTS, lam=2e-3)
    for _ in range(2):
        J, wh, gs = cw.run()
        for x, y in zip((host(J), host(wh), host(gs)), res[0]):
            assert np.array_equal(x, y)
        tmp = torch.empty_like(w0)
        adj.primal_step(g, w0, s, tmp, ws)  # unrelated eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("opt", sorted(OPTIONS))
def test_checkpointed_window_equals_store_all(opt):
    g = _grid(opt)
    w0, s = _inputs(g, 112)
    ws = adj.workspace(g)
    traj, _, Jr = sweep.forward(g, w0, s, NSTEPS, OBJ, WEIGHTS, ws)
    whr, gsr, _ = sweep.backward(g, traj, s, OBJ, WEIGHTS, 2e-3, ws)
    spec = WindowSpec(g, NSTEPS, OBJ, list(WEIGHTS), lam=2e-3, slots=3)
    w0t, st = w0.clone().requires_grad_(True), s.clone().requires_grad_(True)
    J = CheckpointedWindow.apply(w0t, st, spec)
    J.backward()
    assert float(J.detach()) == host(Jr)[0]
    assert np.array_equal(host(w0t.grad), host(whr))
    assert np.array_equal(host(st.grad), host(gsr))


@pytest.mark.parametrize("opt", sorted(OPTIONS))
@pytest.mark.parametrize("bf16", [False, True], ids=["f64", "f32-bf16"])
def test_host_trajectory_matches_hbm(opt, bf16):
    if bf16:
        w = smooth_state(SHAPE, L, seed=114)
        g = _grid(opt, adj.F32, adj.CKPT_BF16, w_ref=adj.reference_state(w))
        w0, s = _inputs(g, 114, torch.float32)
    else:
        g = _grid(opt)
        w0, s = _inputs(g, 114)
    ws = adj.workspace(g)
    traj, _, J1 = sweep.forward(g, w0, s, NSTEPS, OBJ, WEIGHTS, ws)
    wh1, gs1, _ = sweep.backward(g, traj, s, OBJ, WEIGHTS, 2e-3, ws)
    ht = offload.HostTrajectory(g, NSTEPS, slots=2, device_tail=1)
    ht, _, J2 = offload.forward(g, w0, s, NSTEPS, OBJ, WEIGHTS, ws, traj=ht)
    wh2, gs2 = offload.backward(g, ht, s, OBJ, WEIGHTS, 2e-3, ws)
    torch.cuda.synchronize()
    assert np.array_equal(host(J2), host(J1))
    assert np.array_equal(host(wh2), host(wh1))
    assert np.array_equal(host(gs2), host(gs1))


@pytest.mark.parametrize("opt", sorted(OPTIONS))
def test_gradcheck_primal_step(opt):
    g = _grid(opt, shape=(6, 4, 3))
    w = smooth_state((6, 4, 3), L, seed=116)
    spec = WindowSpec(g)
    wt = dev(w).requires_grad_(True)
    st = dev(1e-2 * np.random.default_rng(117).standard_normal(w.size)).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: PrimalStep.apply(a, b, spec), (wt, st), eps=1e-6, atol=1e-8,
                                    rtol=1e-6)
