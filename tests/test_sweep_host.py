"""Host logic of the window drivers (paper_1511_06959_amd.sweep), no GPU: the per-step objective
weights add every state's weight exactly once, and the checkpointing plan picks the two-level
plan of least memory when it fits the budget, binomial slots otherwise."""
import numpy as np
import pytest

import paper_1511_06959_amd as adj
from paper_1511_06959_amd import sweep


@pytest.mark.parametrize("kind", [adj.OBJ_MEAN_PRESSURE, adj.OBJ_KE_DISSIPATION, adj.OBJ_PT_LOSS_PLANE])
@pytest.mark.parametrize("nsteps", [1, 2, 7])
def test_step_weights_cover_every_state_once(kind, nsteps):
    rng = np.random.default_rng(nsteps + 10 * kind)
    weights = rng.standard_normal(nsteps + 1)
    obj = adj.Objective.make(kind)
    coef = np.zeros(nsteps + 1)
    for n in range(nsteps):
        win, w = sweep.step_weights(obj, weights, n, nsteps)
        coef[n] += win      # weight of j(w_n), the step's input
        coef[n + 1] += w    # weight of j(w_{n+1}), the step's output
    assert np.array_equal(coef, weights)
    if kind == adj.OBJ_KE_DISSIPATION:
        # the dissipation rides in each step's first stage: the input carries its weight
        assert all(sweep.step_weights(obj, weights, n, nsteps)[1] == 0.0 for n in range(nsteps - 1))
    else:
        assert all(sweep.step_weights(obj, weights, n, nsteps)[0] == 0.0 for n in range(1, nsteps))
    assert sweep.step_weights(None, weights, 0, nsteps) == (0.0, 0.0)
    assert sweep.step_weights(adj.Objective.make(adj.OBJ_NONE), weights, 0, nsteps) == (0.0, 0.0)
    assert sweep.step_weights(obj, None, 0, nsteps) == (0.0, 0.0)


@pytest.mark.parametrize("precision,ckpt", [(adj.F32, adj.CKPT_BF16), (adj.F32, adj.CKPT_NATIVE),
                                            (adj.F64, adj.CKPT_NATIVE)])
def test_plan_window(precision, ckpt):
    g = adj.Grid.make((64, 48, 40), (1.0, 1.0, 1.0), 1e-3, 1e-3, precision=precision, ckpt_format=ckpt)
    T = 500
    L = sweep.segment_length(g, T)
    mem = sweep.segment_bytes(g, T, L)
    assert all(mem <= sweep.segment_bytes(g, T, k) for k in range(1, T + 1))
    # a snapshot is a record of the grid's format: 2 bytes per value plus the per-block headers
    state = 5 * g.ncells * (8 if precision == adj.F64 else 4)
    assert sweep.snapshot_bytes(g) == (adj.ckpt_bytes(g) if ckpt != adj.CKPT_NATIVE else state)
    if ckpt != adj.CKPT_NATIVE:
        assert 10 * g.ncells < sweep.snapshot_bytes(g) < state
    assert sweep.plan_window(g, T, mem) == ("segments", L)
    sched, slots = sweep.plan_window(g, T, mem - 1)
    assert sched == "binomial" and slots == max(2, min(T, (mem - 1) // sweep.snapshot_bytes(g)))
    assert sweep.plan_window(g, T, 0) == ("binomial", 2)
