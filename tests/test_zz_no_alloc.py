"""adj_adjoint_step_noalloc (the reverse step whose scratch is the library's static per-GPU array)
against adj_adjoint_step with a caller workspace: identical outputs on two calls in a row, the
second on a smaller grid, and a grid beyond the array's size rejected before any launch."""
import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
import workloads as W
from tests.gpu_helpers import dev, host, smooth_state

pytestmark = pytest.mark.gpu


def _case(n, bc_x, precision, lam, obj_kind, seed):
    L = (2.0, 1.5, 1.0)
    w = smooth_state(n, L, seed=seed, wall=bc_x == adj.BC_SLIP_WALLS)
    g = adj.Grid.make(n, L, 1e-3, 2e-4, bc_x=bc_x, precision=precision)
    rng = np.random.default_rng(seed + 100)
    a = rng.standard_normal(w.size)
    s = 1e-3 * rng.standard_normal(w.size)
    gs0 = 1e-2 * rng.standard_normal(w.size)
    obj = adj.Objective.make(obj_kind, plane_i=n[0] // 2, pt_ref=1.3)
    return g, w, a, s, gs0, obj, lam


def _both(case):
    g, w, a, s, gs0, obj, lam = case
    dt = g.dtype
    wn, sd, ad = dev(w, dt), dev(s, dt), dev(a, dt)
    wh_ref = torch.empty_like(wn)
    gs_ref = dev(gs0, dt)
    ws = adj.workspace(g)
    adj.adjoint_step(g, wn, sd, ad, wh_ref, ws, lam=lam, obj=obj, c_n=0.25, grad_s=gs_ref)
    wh = torch.full_like(wn, float("nan"))
    gs = dev(gs0, dt)
    adj.adjoint_step_noalloc(g, wn, sd, ad, wh, lam=lam, obj=obj, c_n=0.25, grad_s=gs)
    return host(wh), host(wh_ref), host(gs), host(gs_ref)


def test_noalloc_matches_workspace_step_twice():
    print("no-alloc: 40x20x12 FP64 periodic, lambda > 0, then 18x8x6 FP32 slip walls", flush=True)
    big = _case((40, 20, 12), adj.BC_PERIODIC, adj.F64, 2e-4, W.OBJ_KE_DISSIPATION, 1)
    small = _case((18, 8, 6), adj.BC_SLIP_WALLS, adj.F32, 1e-4, W.OBJ_PT_LOSS_PLANE, 2)
    for case in (big, small):
        wh, wh_ref, gs, gs_ref = _both(case)
        assert np.all(np.isfinite(wh))
        np.testing.assert_array_equal(wh, wh_ref)
        np.testing.assert_array_equal(gs, gs_ref)


def test_noalloc_rejects_grid_beyond_the_array():
    g = adj.Grid.make((96, 96, 96), (1.0, 1.0, 1.0), 1e-3, 1e-4, precision=adj.F64)
    assert adj.workspace_bytes(g) > adj.NOALLOC_SCRATCH_BYTES
    x = torch.zeros(5 * g.ncells, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(adj.AdjError) as e:
        adj.adjoint_step_noalloc(g, x, None, x, y)
    assert e.value.code == -6 and "static scratch" in str(e.value)
