"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every symbol that
include/adjns.h declares, sizes its workspace and checkpoint records, and rejects bad arguments
with the documented status codes before launching anything."""
import ctypes
import os
import re

import pytest

import paper_1511_06959_amd as adj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "adjns.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(adj_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = adj.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(adj.EXPORTS) == set(names)


def test_version():
    assert "gfx950" in adj.version()


def _grid(**kw):
    p = dict(n=(16, 8, 4), L=(1.0, 1.0, 1.0), mu=0.01, dt=1e-3)
    p.update(kw)
    return adj.Grid.make(p.pop("n"), p.pop("L"), p.pop("mu"), p.pop("dt"), **p)


def test_workspace_and_record_sizes():
    g = _grid()
    N = 16 * 8 * 4
    ws = adj.workspace_bytes(g)
    assert ws >= 6 * 5 * N * 8 + N * 8
    g32 = _grid(precision=adj.F32)
    assert adj.workspace_bytes(g32) < ws
    # block header: 25 floats per 4x4x4 block (4 x 2 x 1 blocks: 800 bytes), padded to 256 bytes
    assert adj.ckpt_bytes(g32) == 1024 + 10 * N


@pytest.mark.parametrize("bad,code", [
    (dict(n=(0, 8, 4)), -1), (dict(L=(0.0, 1.0, 1.0)), -1), (dict(gamma=1.0), -1), (dict(prandtl=0.0), -1),
    (dict(mu=-1.0), -1), (dict(precision=7), -1), (dict(ckpt_format=adj.CKPT_BF16), -1),
    (dict(ckpt_format=adj.CKPT_I16), -1), (dict(ckpt_format=3), -1),
    (dict(n=(1, 8, 4), bc_x=adj.BC_SLIP_WALLS), -2), (dict(bc_x=5), -1), (dict(dt=0.0), -1),
    (dict(nu_weight=(1.0, -0.5, 1.0)), -1), (dict(nu_weight=(1.0, 1.0, float("nan"))), -1), (dict(time_scheme=2), -1),
    (dict(flux=2), -1), (dict(flux=adj.FLUX_ROE, roe_delta=0.0), -1),
    (dict(flux=adj.FLUX_ROE, roe_delta=float("inf")), -1),
    (dict(bc_x=adj.BC_CHARACTERISTIC), -1),  # no far-field states
    (dict(bc_x=adj.BC_CHARACTERISTIC, w_far=((1.0, 0.3, 0, 0, 1.8), (1.0, 0.3, 0, 0, 0.01))), -1),  # p < 0
    (dict(bc_x=adj.BC_CHARACTERISTIC, w_far=((1.0, 0.3, 0, 0, 1.8), (1.0, 0.3, 0, 0, 1.8)), roe_delta=0.0), -1),
    (dict(bc_x=adj.BC_CHARACTERISTIC, n=(1, 8, 4), w_far=((1.0, 0.3, 0, 0, 1.8), (1.0, 0.3, 0, 0, 1.8))), -2),
    (dict(bc_x=3), -1),
])
def test_bad_grid_rejected(bad, code):
    g = _grid(**bad)
    L = adj.lib()
    buf = ctypes.create_string_buffer(1 << 20)
    p = ctypes.c_void_p(ctypes.addressof(buf))
    rc = L.adj_primal_step(ctypes.byref(g), p, None, p, None, p, 1 << 20, None)
    assert rc == code, L.adj_last_error()
    assert L.adj_last_error()


def test_null_and_workspace_errors():
    L = adj.lib()
    g = _grid()
    assert L.adj_primal_step(None, None, None, None, None, None, 0, None) == -1
    fake = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    assert L.adj_primal_step(ctypes.byref(g), fake, None, ctypes.c_void_p(8192), None, None, 0, None) == -6
    assert L.adj_primal_step(ctypes.byref(g), fake, None, ctypes.c_void_p(8192), None, ctypes.c_void_p(4097),
                             1 << 30, None) == -6
    assert L.adj_primal_step(ctypes.byref(g), fake, None, ctypes.c_void_p(8192), None, fake, 16, None) == -6
    assert L.adj_primal_step(ctypes.byref(g), fake, None, fake, None, ctypes.c_void_p(1 << 20), 1 << 30, None) == -1


def test_adjoint_argument_errors():
    L = adj.lib()
    g = _grid()
    fake = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    big = 1 << 34
    o = adj.Objective.make(adj.OBJ_PT_LOSS_PLANE, 0, 1.0)
    rc = L.adj_adjoint_step(ctypes.byref(g), fake, None, fake, 0.0, ctypes.byref(o), 1.0, ctypes.c_void_p(8192),
                            None, ws, big, None)
    assert rc == -2 and "plane_i" in L.adj_last_error().decode()
    rc = L.adj_adjoint_step(ctypes.byref(g), fake, None, fake, -1.0, None, 1.0, ctypes.c_void_p(8192), None, ws,
                            big, None)
    assert rc == -1 and "lambda" in L.adj_last_error().decode()
    rc = L.adj_adjoint_step(ctypes.byref(g), fake, None, fake, 0.0, None, 1.0, fake, None, ws, big, None)
    assert rc == -1 and "alias" in L.adj_last_error().decode()


def test_binding_refuses_host_tensors():
    torch = pytest.importorskip("torch")
    g = _grid()
    w = torch.zeros(5 * g.ncells, dtype=torch.float64)
    with pytest.raises(ValueError):
        adj.residual(g, w, None, w.clone())


def _create(grids, member_box, member_lam, obj=None, table_bytes=None):
    L = adj.lib()
    nb, nm = len(grids), len(member_box)
    tb = L.adj_batch_table_bytes(nb, nm, grids[0].precision) if table_bytes is None else table_bytes
    buf = ctypes.create_string_buffer(max(tb, 1) + 256)
    addr = (ctypes.addressof(buf) + 255) // 256 * 256
    h = ctypes.c_void_p()
    rc = L.adj_batch_create(ctypes.byref(h), nb, (adj.Grid * nb)(*grids),
                            ctypes.byref(obj) if obj is not None else None, nm, (ctypes.c_int * nm)(*member_box),
                            (ctypes.c_double * nm)(*member_lam), ctypes.c_void_p(addr), ctypes.c_size_t(tb))
    return rc


def test_ensemble_table_size_grows_with_members():
    L = adj.lib()
    assert L.adj_batch_table_bytes(0, 1, adj.F64) == 0
    assert L.adj_batch_table_bytes(2, 3, 9) == 0
    assert L.adj_batch_table_bytes(4, 8, adj.F64) > L.adj_batch_table_bytes(4, 4, adj.F64)
    assert L.adj_batch_table_bytes(4, 16, adj.F64) > L.adj_batch_table_bytes(4, 16, adj.F32)


@pytest.mark.parametrize("case,code", [
    ("members_decreasing", -1), ("member_box_range", -1), ("negative_lambda", -1), ("mixed_precision", -1),
    ("mixed_boundary", -1), ("bf16_states", -1), ("objective_kind", -1), ("small_table", -6), ("bad_grid", -1),
    ("ssprk3", -1), ("roe", -1), ("characteristic", -1),
])
def test_ensemble_create_rejects(case, code):
    g = [_grid(), _grid(n=(8, 8, 8))]
    mb, ml, obj, tb = [0, 1], [0.0, 0.1], None, None
    if case == "members_decreasing":
        mb = [1, 0]
    elif case == "member_box_range":
        mb = [0, 2]
    elif case == "negative_lambda":
        ml = [0.0, -1.0]
    elif case == "mixed_precision":
        g[1] = _grid(n=(8, 8, 8), precision=adj.F32)
    elif case == "mixed_boundary":
        g[1] = _grid(n=(8, 8, 8), bc_x=adj.BC_SLIP_WALLS)
    elif case == "bf16_states":
        g = [_grid(precision=adj.F32, ckpt_format=adj.CKPT_BF16), _grid(n=(8, 8, 8), precision=adj.F32)]
    elif case == "objective_kind":
        obj = adj.Objective.make(adj.OBJ_KE_DISSIPATION)
    elif case == "small_table":
        tb = 64
    elif case == "bad_grid":
        g[1] = _grid(n=(8, 0, 8))
    elif case == "ssprk3":
        g[1] = _grid(n=(8, 8, 8), time_scheme=adj.SSPRK3)
    elif case == "roe":
        g[1] = _grid(n=(8, 8, 8), flux=adj.FLUX_ROE)
    elif case == "characteristic":
        far = ((1.0, 0.3, 0, 0, 1.8), (1.0, 0.3, 0, 0, 1.8))
        g = [_grid(bc_x=adj.BC_CHARACTERISTIC, w_far=far), _grid(n=(8, 8, 8), bc_x=adj.BC_CHARACTERISTIC, w_far=far)]
    assert _create(g, mb, ml, obj, tb) == code
    assert adj.lib().adj_last_error()


def test_ensemble_calls_reject_null_handle():
    L = adj.lib()
    buf = ctypes.create_string_buffer(1024)
    p = ctypes.c_void_p(ctypes.addressof(buf))
    assert L.adj_batch_primal_step(None, 1, p, None, p, p, 1024, None) == -1
    assert L.adj_batch_adjoint_step(None, 1, p, None, p, None, p, None, p, 1024, None) == -1
    assert L.adj_batch_offset(None, 0, 0) == -1
    assert L.adj_batch_workspace_bytes(None) == 0


def test_tile_launched():
    # reverse-stage LDS per work-group: 8 B x (8 box planes + max(4 record planes + 3 work-term
    # planes, 3 staging planes)); the FP64 32x8x4 box (34 x 10 x 6 cells) needs 226560 B > 160 KiB
    A, P = adj.PROF_ADJOINT_STAGE, adj.PROF_PRIMAL_STAGE
    for t in adj.TILES:
        assert adj.tile_launched(A, adj.F32, adj.BC_PERIODIC, False, t) == t
        assert adj.tile_launched(P, adj.F64, adj.BC_SLIP_WALLS, True, t) == t
    assert adj.tile_launched(A, adj.F64, adj.BC_PERIODIC, False, adj.TILE_32x8x4) == adj.TILE_16x4x4
    assert adj.tile_launched(A, adj.F64, adj.BC_PERIODIC, False, adj.TILE_32x4x4) == adj.TILE_32x4x4
    assert adj.tile_launched(A, adj.F64, adj.BC_SLIP_WALLS, True, adj.TILE_16x4x4) == adj.TILE_16x4x4
    with pytest.raises(adj.AdjError):
        adj.tile_launched(A, adj.F64, 3, False, 0)
    with pytest.raises(adj.AdjError):
        adj.tile_launched(A, adj.F64, adj.BC_PERIODIC, False, len(adj.TILES))


def test_stability_argument_errors():
    L = adj.lib()
    g = _grid()
    fake = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    wsp = ctypes.c_void_p(1 << 20)
    nb = ctypes.c_size_t(1 << 30)
    assert L.adj_stability(ctypes.byref(g), None, ctypes.c_double(0.0), fake, wsp, nb, None) == -1
    assert L.adj_stability(ctypes.byref(g), fake, ctypes.c_double(-1.0), fake, wsp, nb, None) == -1
    assert L.adj_stability(ctypes.byref(g), fake, ctypes.c_double(0.0), fake, None, nb, None) == -6
    bad = _grid(dt=0.0)
    assert L.adj_check_stable(ctypes.byref(bad), fake, ctypes.c_double(0.0), None, wsp, nb, None) == -1


def test_noalloc_step_validates_before_touching_the_device():
    """The no-allocation reverse step rejects bad grids and grids whose scratch exceeds its static
    array on the host, before it looks up the array or launches anything."""
    L = adj.lib()
    fake = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    big = _grid(n=(96, 96, 96))
    assert adj.workspace_bytes(big) > adj.NOALLOC_SCRATCH_BYTES
    rc = L.adj_adjoint_step_noalloc(ctypes.byref(big), fake, None, fake, 0.0, None, 0.0, ctypes.c_void_p(8192), None,
                                    None)
    assert rc == -6 and b"static scratch" in L.adj_last_error()
    bad = _grid(dt=0.0)
    rc = L.adj_adjoint_step_noalloc(ctypes.byref(bad), fake, None, fake, 0.0, None, 0.0, ctypes.c_void_p(8192), None,
                                    None)
    assert rc == -1
    # 64^3 FP64, the largest cube the array is sized for, fits
    assert adj.workspace_bytes(_grid(n=(64, 64, 64))) <= adj.NOALLOC_SCRATCH_BYTES
