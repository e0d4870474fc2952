"""One artificial adjoint viscosity per variable group (adj_grid.nu_weight): the adjoint
components of rho, rho u and rho E are diffused with nu_g = lambda nu_weight[g] sigma_1.

Parity against the oracle's per-group operator (lambda_g = lambda nu_weight[g]) for single
steps in both precisions, periodic and with slip walls; the stored-stage form, an ensemble
member and all-zero weights (read as 1, 1, 1) against the single-box FP64 call."""
import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
import workloads as W
from tests.gpu_helpers import dev, host, relerr, smooth_state

pytestmark = pytest.mark.gpu

WEIGHTS = (0.3, 1.0, 2.5)
LAM = 3e-3


def _case(orc, bc_x, precision=adj.F64, weights=WEIGHTS, shape=(19, 6, 9), seed=20):
    L = (2.0, 1.3, 1.7)
    g = adj.Grid.make(shape, L, 0.02, 0.004, bc_x=bc_x, precision=precision, nu_weight=weights)
    og = orc.make_grid(shape, L, 1.4, 0.72, 0.02, 0.004, bc_x)
    w = smooth_state(shape, L, seed=seed)
    rng = np.random.default_rng(seed + 1)
    return g, og, w, 1e-2 * rng.standard_normal(w.size), rng.standard_normal(w.size), rng.standard_normal(w.size)


def _gpu_step(g, w, s, a, gs0, stages=False):
    dt = g.dtype
    ws = adj.workspace(g)
    wh = torch.empty(w.size, dtype=dt, device="cuda")
    gs = dev(gs0, dt)
    obj = adj.Objective.make(W.OBJ_MEAN_PRESSURE)
    if stages:
        st = torch.empty(3 * w.size, dtype=dt, device="cuda")
        w1 = torch.empty(w.size, dtype=dt, device="cuda")
        adj.primal_step_stages(g, dev(w, dt), dev(s, dt), w1, st, ws)
        adj.adjoint_step_stages(g, dev(w, dt), st, dev(s, dt), dev(a, dt), wh, ws, lam=LAM, obj=obj, c_n=0.37,
                                grad_s=gs)
    else:
        adj.adjoint_step(g, dev(w, dt), dev(s, dt), dev(a, dt), wh, ws, lam=LAM, obj=obj, c_n=0.37, grad_s=gs)
    return host(wh), host(gs)


@pytest.mark.parametrize("bc_x", [0, 1], ids=["periodic", "walls"])
@pytest.mark.parametrize("precision", [adj.F64, adj.F32], ids=["f64", "f32"])
def test_group_viscosity_step_parity(orc, bc_x, precision):
    g, og, w, s, a, gs0 = _case(orc, bc_x, precision)
    if precision == adj.F32:
        # the oracle sees the FP32 inputs; grad_s starts at 0 so that its FP32 sum is the increment
        w, s, a = (x.astype(np.float32).astype(np.float64) for x in (w, s, a))
        gs0 = np.zeros_like(gs0)
    wh, gs = _gpu_step(g, w, s, a, gs0)
    gref = gs0.copy()
    lam_g = [LAM * x for x in WEIGHTS]
    ref = orc.adjoint_step(og, w, s, a, lam_g, orc.make_obj(W.OBJ_MEAN_PRESSURE), 0.37, gref)
    tol = 1e-12 if precision == adj.F64 else 1e-5
    assert relerr(wh - a, ref - a) <= tol
    assert relerr(gs - gs0, gref - gs0) <= tol
    # the weights matter: the single-viscosity step differs by far more than the tolerance
    one = orc.adjoint_step(og, w, s, a, LAM, orc.make_obj(W.OBJ_MEAN_PRESSURE), 0.37, gs0.copy())
    assert relerr(one - a, ref - a) > 100 * tol


@pytest.mark.parametrize("bc_x", [0, 1], ids=["periodic", "walls"])
def test_group_viscosity_operator_parity(orc, bc_x):
    # adj_vjp with a given nu field applies the grid's weights as well
    g, og, w, _, kh, _ = _case(orc, bc_x, seed=24)
    nu = LAM * orc.sigma1(og, w)
    out = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.vjp(g, dev(w), dev(kh), out, dev(nu))
    ref = orc.vjp(og, w, kh) + orc.lnu_apply_groups(og, w, [LAM * x for x in WEIGHTS], kh)
    assert relerr(host(out), ref) <= 1e-13


def test_stored_stages_and_zero_weights_match(orc):
    g, og, w, s, a, gs0 = _case(orc, 0, seed=26)
    wh, gs = _gpu_step(g, w, s, a, gs0)
    wh2, gs2 = _gpu_step(g, w, s, a, gs0, stages=True)
    assert relerr(wh2 - a, wh - a) <= 1e-13 and relerr(gs2 - gs0, gs - gs0) <= 1e-13
    g1, *_ = _case(orc, 0, weights=(1.0, 1.0, 1.0), seed=26)
    g0, *_ = _case(orc, 0, weights=(0.0, 0.0, 0.0), seed=26)
    wh1, gs1 = _gpu_step(g1, w, s, a, gs0)
    wh0, gs0b = _gpu_step(g0, w, s, a, gs0)
    assert np.array_equal(wh0, wh1) and np.array_equal(gs0b, gs1)


def test_ensemble_member_with_group_weights(orc):
    g, og, w, s, a, gs0 = _case(orc, 1, seed=28, shape=(12, 8, 6))
    lams = [0.0, LAM, 2 * LAM]
    ens = adj.Ensemble([g], [0, 0, 0], lams)
    ws = ens.workspace()
    P, Q = ens.offset(0, 1), ens.offset(1, 3)
    wd, sd = dev(w), dev(s)
    ad = torch.cat([dev(a)] * 3)
    out = torch.empty(5 * Q, dtype=torch.float64, device="cuda")
    gsd = torch.cat([dev(gs0)] * 3)
    assert P == w.size // 5
    ens.adjoint_step(3, wd, sd, ad, out, ws, c_n=None, grad_s=gsd)
    outh, gsh = host(out), host(gsd)
    for m, lam in enumerate(lams):
        ws1 = adj.workspace(g)
        wh = torch.empty(w.size, dtype=torch.float64, device="cuda")
        gs1 = dev(gs0)
        adj.adjoint_step(g, wd, sd, dev(a), wh, ws1, lam=lam, grad_s=gs1)
        lo, hi = 5 * ens.offset(1, m), 5 * ens.offset(1, m + 1)
        assert np.array_equal(outh[lo:hi], host(wh)), f"member {m}"
        assert np.array_equal(gsh[lo:hi], host(gs1)), f"member {m}"
