"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle, element by element.

Tolerances (FP64 path): a single operator or step on identical inputs agrees to 1e-13 of the
largest oracle value (the only differences are summation order); a whole 50-step window agrees
to 1e-10 (the target of the FP64 path).  FP32 operators agree to 1e-5 of the largest value.
Grids are ragged with respect to the 16x4x4 tile so that every tile shape, halo wrap and wall
mirror is exercised.
"""
import math

import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
import workloads as W
from tests.gpu_helpers import dev, grids, host, relerr, relerr_vars, smooth_state

pytestmark = pytest.mark.gpu

SHAPES = [((19, 6, 9), 0), ((19, 6, 9), 1), ((4, 4, 4), 0), ((33, 5, 1), 0), ((7, 1, 3), 1)]
IDS = ["19x6x9-periodic", "19x6x9-walls", "4x4x4", "33x5x1", "7x1x3-walls"]


def _setup(orc, shape, bc_x, precision=adj.F64, seed=0):
    L = (2.0, 1.3, 1.7)
    g, og = grids(orc, shape, L, mu=0.02, dt=0.004, bc_x=bc_x, precision=precision)
    w = smooth_state(shape, L, seed=seed)
    return g, og, w


@pytest.mark.parametrize("shape,bc_x", SHAPES, ids=IDS)
def test_residual_parity_f64(orc, shape, bc_x):
    g, og, w = _setup(orc, shape, bc_x)
    s = 1e-2 * np.random.default_rng(1).standard_normal(w.size)
    R = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.residual(g, dev(w), dev(s), R)
    ref = orc.residual(og, w, s)
    assert relerr(host(R), ref) <= 1e-13
    # each field against its own scale too (fields far smaller than the largest are held to theirs)
    assert relerr_vars(host(R), ref) <= 1e-11


@pytest.mark.parametrize("shape,bc_x", SHAPES, ids=IDS)
@pytest.mark.parametrize("with_nu", [False, True], ids=["plain", "lnu"])
def test_vjp_parity_f64(orc, shape, bc_x, with_nu):
    g, og, w = _setup(orc, shape, bc_x)
    rng = np.random.default_rng(2)
    kh = rng.standard_normal(w.size)
    nu = np.abs(rng.standard_normal(w.size // 5)) * 1e-2 if with_nu else None
    out = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.vjp(g, dev(w), dev(kh), out, dev(nu) if with_nu else None)
    ref = orc.vjp(og, w, kh)
    if with_nu:
        ref = ref + orc.lnu_apply(og, nu, kh)
    assert relerr(host(out), ref) <= 1e-13
    assert relerr_vars(host(out), ref) <= 1e-11


@pytest.mark.parametrize("shape,bc_x", SHAPES, ids=IDS)
def test_primal_step_parity_f64(orc, shape, bc_x):
    g, og, w = _setup(orc, shape, bc_x)
    s = 1e-2 * np.random.default_rng(3).standard_normal(w.size)
    ws = adj.workspace(g)
    out = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.primal_step(g, dev(w), dev(s), out, ws)
    ref = orc.primal_step(og, w, s)
    # compare the increment, which is what the step computes on top of w
    assert relerr(host(out) - w, ref - w) <= 1e-12
    assert relerr_vars(host(out) - w, ref - w) <= 1e-10


OBJS = [(W.OBJ_NONE, 0), (W.OBJ_MEAN_PRESSURE, 0), (W.OBJ_KE_DISSIPATION, 0), (W.OBJ_PT_LOSS_PLANE, 0),
        (W.OBJ_KE_DISSIPATION, 1), (W.OBJ_PT_LOSS_PLANE, 1)]


@pytest.mark.parametrize("kind,bc_x", OBJS, ids=["none", "meanp", "ked", "ptloss", "ked-walls", "ptloss-walls"])
@pytest.mark.parametrize("lam", [0.0, 3e-3], ids=["lam0", "lam"])
def test_adjoint_step_parity_f64(orc, kind, bc_x, lam):
    shape = (19, 6, 9)
    g, og, w = _setup(orc, shape, bc_x, seed=4)
    rng = np.random.default_rng(5)
    s = 1e-2 * rng.standard_normal(w.size)
    a = rng.standard_normal(w.size)
    gs0 = rng.standard_normal(w.size)
    obj = adj.Objective.make(kind, 7, 1.1)
    oobj = orc.make_obj(kind, 7, 1.1)
    ws = adj.workspace(g)
    wh = torch.empty(w.size, dtype=torch.float64, device="cuda")
    gs = dev(gs0)
    adj.adjoint_step(g, dev(w), dev(s), dev(a), wh, ws, lam=lam, obj=obj, c_n=0.37, grad_s=gs)
    gref = gs0.copy()
    ref = orc.adjoint_step(og, w, s, a, lam, oobj, 0.37, gref)
    assert relerr(host(wh) - a, ref - a) <= 1e-12
    assert relerr(host(gs) - gs0, gref - gs0) <= 1e-12
    assert relerr_vars(host(wh) - a, ref - a) <= 1e-10
    assert relerr_vars(host(gs) - gs0, gref - gs0) <= 1e-10


@pytest.mark.parametrize("shape,bc_x", SHAPES, ids=IDS)
def test_sigma1_parity_f64(orc, shape, bc_x):
    g, og, w = _setup(orc, shape, bc_x, seed=6)
    out = torch.empty(w.size // 5, dtype=torch.float64, device="cuda")
    adj.growth_sigma1(g, dev(w), out, scale=2.0)
    assert relerr(host(out), 2.0 * orc.sigma1(og, w)) <= 1e-12


@pytest.mark.parametrize("kind,bc_x", OBJS[1:], ids=["meanp", "ked", "ptloss", "ked-walls", "ptloss-walls"])
def test_objective_parity_f64(orc, kind, bc_x):
    g, og, w = _setup(orc, (19, 6, 9), bc_x, seed=7)
    obj = adj.Objective.make(kind, 5, 1.2)
    ws = adj.workspace(g)
    J = torch.full((1,), 0.25, dtype=torch.float64, device="cuda")
    jr, djr = orc.objective(og, orc.make_obj(kind, 5, 1.2), w)
    # the gradient is accumulated (+=) onto an existing field of the gradient's own magnitude
    base = np.random.default_rng(8).standard_normal(w.size) * np.abs(djr).max()
    dj = dev(base)
    adj.objective_and_grad(g, obj, dev(w), ws, weight=0.5, J_accum=J, djdw=dj)
    assert abs(host(J)[0] - (0.25 + 0.5 * jr)) <= 1e-13 * abs(0.25 + 0.5 * jr)
    assert relerr(host(dj) - base, 0.5 * djr) <= 1e-12


def test_energy_and_dot_parity(orc):
    g, og, w = _setup(orc, (19, 6, 9), 0, seed=9)
    rng = np.random.default_rng(10)
    wh = rng.standard_normal(w.size)
    ws = adj.workspace(g)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    adj.energy_vhat(g, dev(w), dev(wh), E, ws)
    Er, _ = orc.energy_vhat(og, w, wh)
    assert abs(host(E)[0] - Er) <= 1e-13 * Er
    b = rng.standard_normal(w.size)
    d = torch.zeros(1, dtype=torch.float64, device="cuda")
    adj.dot(g, dev(wh), dev(b), d, ws)
    assert abs(host(d)[0] - float(wh @ b)) <= 1e-12 * np.abs(wh * b).sum()


# (19, 6, 9): two strips of four blocks along x, the second with one block; (37, 13, 10): three
# strips, the last with two blocks, ragged blocks in every direction; (64, 8, 4): whole strips
@pytest.mark.parametrize("fmt", [adj.CKPT_BF16, adj.CKPT_I16], ids=["bf16", "i16"])
@pytest.mark.parametrize("shape", [(19, 6, 9), (37, 13, 10), (64, 8, 4)], ids=["19x6x9", "37x13x10", "64x8x4"])
def test_codec_bitwise(orc, shape, fmt):
    g = adj.Grid.make(shape, (1, 1, 1), 0.01, 0.01, precision=adj.F32, ckpt_format=fmt)
    i16 = fmt == adj.CKPT_I16
    w = smooth_state(shape, seed=11).astype(np.float32)
    ws = adj.workspace(g)
    rec = torch.zeros(adj.ckpt_bytes(g), dtype=torch.uint8, device="cuda")
    adj.ckpt_encode(g, dev(w, torch.float32), rec, ws)
    torch.cuda.synchronize()
    raw = rec.cpu().numpy()
    og = orc.make_grid(shape, (1, 1, 1), 1.4, 0.72, 0.01, 0.01, 0)
    q, hdr_ref = orc.ckpt_encode(og, w, i16=i16)
    hb = raw.size - 2 * w.size  # header bytes (block headers, padded)
    hdr = raw[:hdr_ref.size * 4].view(np.float32).reshape(hdr_ref.shape)
    codes = raw[hb:].view(np.uint16)
    assert hb % 256 == 0 and hb >= hdr_ref.size * 4
    assert np.array_equal(hdr, hdr_ref)
    assert np.array_equal(codes, q)
    out = torch.empty(w.size, dtype=torch.float32, device="cuda")
    adj.ckpt_decode(g, rec, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), orc.ckpt_decode(og, q, hdr_ref, i16=i16))


def test_adjoint_step_deterministic():
    shape = (19, 6, 9)
    g = adj.Grid.make(shape, (2.0, 1.3, 1.7), 0.02, 0.004)
    w = dev(smooth_state(shape, seed=12))
    a = dev(np.random.default_rng(13).standard_normal(w.numel()))
    ws = adj.workspace(g)
    outs = []
    for _ in range(2):
        wh = torch.empty_like(w)
        gs = torch.zeros_like(w)
        adj.adjoint_step(g, w, None, a, wh, ws, lam=2e-3, obj=adj.Objective.make(W.OBJ_KE_DISSIPATION), c_n=0.3,
                         grad_s=gs)
        E = torch.zeros(1, dtype=torch.float64, device="cuda")
        adj.energy_vhat(g, w, wh, E, ws)
        outs.append((host(wh), host(gs), host(E)))
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("bc_x", [0, 1], ids=["periodic", "walls"])
def test_sigma1_parity_f32(orc, bc_x):
    g, og, w = _setup(orc, (19, 6, 9), bc_x, precision=adj.F32, seed=18)
    w32 = w.astype(np.float32).astype(np.float64)
    out = torch.empty(w.size // 5, dtype=torch.float32, device="cuda")
    adj.growth_sigma1(g, dev(w32, torch.float32), out)
    assert relerr(host(out), orc.sigma1(og, w32)) <= 2e-5


def test_sigma1_repeated_singular_values(orc):
    # uniform state plus a pure shear in one velocity component: M has a single non-zero entry, so
    # M^T M has a four-fold zero eigenvalue below lambda_max (the bracket must not stall)
    n = (8, 8, 8)
    g, og, _ = _setup(orc, n, 0, seed=19)
    x, y, z = W.cell_centres(n, (2.0, 1.3, 1.7))
    rho = np.ones_like(x)
    w = W.conservative(rho, 0.3 * np.sin(2 * math.pi * y / 1.3), np.zeros_like(x), np.zeros_like(x),
                       np.full_like(x, 0.8))
    out = torch.empty(w.size // 5, dtype=torch.float64, device="cuda")
    adj.growth_sigma1(g, dev(w), out)
    assert relerr(host(out), orc.sigma1(og, w)) <= 1e-13


def test_fp32_operators(orc):
    shape = (19, 6, 9)
    g, og, w = _setup(orc, shape, 0, precision=adj.F32, seed=14)
    w32 = w.astype(np.float32).astype(np.float64)
    kh = np.random.default_rng(15).standard_normal(w.size).astype(np.float32).astype(np.float64)
    R = torch.empty(w.size, dtype=torch.float32, device="cuda")
    adj.residual(g, dev(w32, torch.float32), None, R)
    assert relerr(host(R), orc.residual(og, w32)) <= 1e-5
    out = torch.empty(w.size, dtype=torch.float32, device="cuda")
    adj.vjp(g, dev(w32, torch.float32), dev(kh, torch.float32), out)
    assert relerr(host(out), orc.vjp(og, w32, kh)) <= 1e-5


@pytest.fixture
def restore_tiles():
    saved = {(k, p): adj.get_tile(k, p) for k in (adj.PROF_ADJOINT_STAGE, adj.PROF_PRIMAL_STAGE)
             for p in (adj.F32, adj.F64)}
    yield
    for (k, p), t in saved.items():
        adj.set_tile(k, p, t)


@pytest.mark.parametrize("tile", sorted(adj.TILES), ids=[f"{a}x{b}x{c}" for a, b, c in adj.TILES.values()])
@pytest.mark.parametrize("bc_x", [0, 1], ids=["periodic", "walls"])
def test_every_tile_shape_f64(orc, restore_tiles, tile, bc_x):
    shape = (37, 7, 5)
    for k in (adj.PROF_ADJOINT_STAGE, adj.PROF_PRIMAL_STAGE):
        adj.set_tile(k, adj.F64, tile)
    g, og, w = _setup(orc, shape, bc_x, seed=16)
    rng = np.random.default_rng(17)
    s = 1e-2 * rng.standard_normal(w.size)
    R = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.residual(g, dev(w), dev(s), R)
    assert relerr(host(R), orc.residual(og, w, s)) <= 1e-13
    a = rng.standard_normal(w.size)
    ws = adj.workspace(g)
    wh = torch.empty(w.size, dtype=torch.float64, device="cuda")
    gs = torch.zeros(w.size, dtype=torch.float64, device="cuda")
    obj = adj.Objective.make(W.OBJ_KE_DISSIPATION)
    adj.adjoint_step(g, dev(w), dev(s), dev(a), wh, ws, lam=2e-3, obj=obj, c_n=0.2, grad_s=gs)
    gref = np.zeros(w.size)
    ref = orc.adjoint_step(og, w, s, a, 2e-3, orc.make_obj(W.OBJ_KE_DISSIPATION), 0.2, gref)
    assert relerr(host(wh) - a, ref - a) <= 1e-12
    assert relerr(host(gs), gref) <= 1e-12


# ------------------------------------------------------------------------------ reference state
@pytest.mark.parametrize("bc_x", [0, 1], ids=["periodic", "walls"])
def test_reference_state_offset_f64(orc, bc_x):
    # states stored as w - w_ref: every operator acts on the full state (the oracle's), so the
    # rates, the adjoint fields and the scalars are unchanged and the stored outputs are offset
    shape = (19, 6, 9)
    g0, og, w = _setup(orc, shape, bc_x, seed=21)
    w_ref = (1.02, 0.0 if bc_x else 0.13, -0.07, 0.05, 2.31)
    g = adj.Grid.make(shape, (2.0, 1.3, 1.7), 0.02, 0.004, bc_x=bc_x, w_ref=w_ref)
    ws = adj.workspace(g)
    wd = dev(g.to_stored(w))
    rng = np.random.default_rng(22)
    s = 1e-2 * rng.standard_normal(w.size)
    a = rng.standard_normal(w.size)
    R = torch.empty(w.size, dtype=torch.float64, device="cuda")
    adj.residual(g, wd, dev(s), R)
    assert relerr(host(R), orc.residual(og, w, s)) <= 1e-12
    out = torch.empty_like(R)
    adj.vjp(g, wd, dev(a), out)
    assert relerr(host(out), orc.vjp(og, w, a)) <= 1e-12
    adj.primal_step(g, wd, dev(s), out, ws)
    ref = orc.primal_step(og, w, s)
    assert relerr(g.from_stored(host(out)) - w, ref - w) <= 1e-12
    obj = adj.Objective.make(W.OBJ_PT_LOSS_PLANE if bc_x else W.OBJ_MEAN_PRESSURE, 7, 1.1)
    oobj = orc.make_obj(W.OBJ_PT_LOSS_PLANE if bc_x else W.OBJ_MEAN_PRESSURE, 7, 1.1)
    gs = torch.zeros_like(R)
    adj.adjoint_step(g, wd, dev(s), dev(a), out, ws, lam=3e-3, obj=obj, c_n=0.37, grad_s=gs)
    gref = np.zeros_like(w)
    ref = orc.adjoint_step(og, w, s, a, 3e-3, oobj, 0.37, gref)
    assert relerr(host(out) - a, ref - a) <= 1e-12
    assert relerr(host(gs), gref) <= 1e-12
    sig = torch.empty(w.size // 5, dtype=torch.float64, device="cuda")
    adj.growth_sigma1(g, wd, sig)
    assert relerr(host(sig), orc.sigma1(og, w)) <= 1e-12
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    adj.objective_and_grad(g, obj, wd, ws, weight=1.0, J_accum=J)
    jr, _ = orc.objective(og, oobj, w)
    assert abs(host(J)[0] - jr) <= 1e-13 * abs(jr)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    adj.energy_vhat(g, wd, dev(a), E, ws)
    Er, _ = orc.energy_vhat(og, w, a)
    assert abs(host(E)[0] - Er) <= 1e-12 * abs(Er)


@pytest.mark.parametrize("precision", [adj.F64, adj.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("kind,bc_x,scheme,flux", [
    (W.OBJ_MEAN_PRESSURE, 0, adj.RK4, adj.FLUX_SPLIT), (W.OBJ_MEAN_PRESSURE, 1, adj.RK4, adj.FLUX_SPLIT),
    (W.OBJ_MEAN_PRESSURE, 0, adj.SSPRK3, adj.FLUX_SPLIT), (W.OBJ_MEAN_PRESSURE, 1, adj.RK4, adj.FLUX_ROE),
    (W.OBJ_KE_DISSIPATION, 0, adj.RK4, adj.FLUX_SPLIT), (W.OBJ_PT_LOSS_PLANE, 1, adj.RK4, adj.FLUX_SPLIT)],
    ids=["meanp", "meanp-walls", "meanp-ssprk3", "meanp-roe", "ked", "ptloss-walls"])
def test_primal_step_with_objective(orc, precision, kind, bc_x, scheme, flux):
    # the step that also accumulates the objective of its new state (fused into the final stage for
    # the mean pressure on RK4 split-flux grids) writes the same state as the plain step, bit for
    # bit, and the same J as the objective call to rounding of the sum, which the oracle confirms
    shape = (37, 9, 6)
    L = (2.0, 1.3, 1.7)
    w = smooth_state(shape, L, seed=12)
    ref = tuple(w.reshape(5, -1).mean(axis=1)) if precision == adj.F32 else None
    g = adj.Grid.make(shape, L, 0.02, 0.004, bc_x=bc_x, precision=precision, w_ref=ref, time_scheme=scheme, flux=flux)
    og = orc.make_grid(shape, L, 1.4, 0.72, 0.02, 0.004, bc_x, scheme, flux)
    dt = g.dtype
    s = 1e-2 * np.random.default_rng(13).standard_normal(w.size)
    obj = adj.Objective.make(kind, 20, 1.1)
    ws = adj.workspace(g)
    wd, sd = dev(g.to_stored(w), dt), dev(s, dt)
    plain = torch.empty_like(wd)
    adj.primal_step(g, wd, sd, plain, ws)
    J1 = torch.full((1,), 0.5, dtype=torch.float64, device="cuda")
    adj.objective_and_grad(g, obj, plain, ws, weight=0.3, J_accum=J1)
    out = torch.empty_like(wd)
    J2 = torch.full((1,), 0.5, dtype=torch.float64, device="cuda")
    adj.primal_step_obj(g, wd, sd, out, ws, obj, 0.3, J2)
    assert np.array_equal(host(out), host(plain))
    assert abs(host(J2)[0] - host(J1)[0]) <= 1e-14 * abs(host(J1)[0])
    jr = orc.objective(og, orc.make_obj(kind, 20, 1.1), orc.primal_step(og, w, s), grad=False)
    tol = 1e-12 if precision == adj.F64 else 1e-6
    assert abs(host(J2)[0] - (0.5 + 0.3 * jr)) <= tol * abs(0.5 + 0.3 * jr)
    if precision == adj.F32 and scheme == adj.RK4:
        gb = adj.Grid.make(shape, L, 0.02, 0.004, bc_x=bc_x, precision=precision, ckpt_format=adj.CKPT_BF16, w_ref=ref,
                           flux=flux)
        r1 = torch.zeros(adj.ckpt_bytes(gb), dtype=torch.uint8, device="cuda")
        r2 = torch.zeros_like(r1)
        adj.primal_step(gb, wd, sd, plain, ws, ckpt_out=r1)
        adj.primal_step_obj(gb, wd, sd, out, ws, obj, 0.3, J2, ckpt_out=r2)
        assert torch.equal(r1, r2) and torch.equal(out, plain)
    if scheme == adj.RK4:
        st1 = torch.empty(3 * w.size, dtype=dt, device="cuda")
        st2 = torch.empty_like(st1)
        adj.primal_step_stages(g, wd, sd, plain, st1, ws)
        adj.primal_step_obj(g, wd, sd, out, ws, obj, 0.3, J2, stages_out=st2)
        assert torch.equal(st1, st2) and torch.equal(out, plain)
    # the objective of the step's input as well (the dissipation rides in stage 1, the others run
    # the objective kernel before the step): J += 0.7 j(w_n) + 0.3 j(w_np1)
    J3 = torch.full((1,), 0.5, dtype=torch.float64, device="cuda")
    adj.primal_step_obj(g, wd, sd, out, ws, obj, 0.3, J3, weight_in=0.7)
    assert np.array_equal(host(out), host(plain))
    J4 = torch.zeros(1, dtype=torch.float64, device="cuda")
    adj.objective_and_grad(g, obj, wd, ws, weight=1.0, J_accum=J4)
    want = host(J1)[0] + 0.7 * host(J4)[0]
    # the fused dissipation sums its cells in other tiles (and a cell's terms may contract
    # differently), so it agrees with the objective kernel to the rounding of its precision
    tol_in = 1e-14 if (kind != W.OBJ_KE_DISSIPATION or precision == adj.F64) else 1e-6
    assert abs(host(J3)[0] - want) <= tol_in * abs(want)
    jin = orc.objective(og, orc.make_obj(kind, 20, 1.1), g.from_stored(g.to_stored(w)), grad=False)
    assert abs(host(J3)[0] - (0.5 + 0.3 * jr + 0.7 * jin)) <= tol * abs(0.5 + 0.3 * jr + 0.7 * jin)
    # the input's objective alone, with the new state's weight zero
    J5 = torch.zeros(1, dtype=torch.float64, device="cuda")
    adj.primal_step_obj(g, wd, sd, out, ws, obj, 0.0, J5, weight_in=0.7)
    assert np.array_equal(host(out), host(plain))
    assert abs(host(J5)[0] - 0.7 * host(J4)[0]) <= tol_in * abs(0.7 * host(J4)[0])
