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
    assert adj.ckpt_bytes(g32) == 64 + 10 * N


@pytest.mark.parametrize("bad,code", [
    (dict(n=(0, 8, 4)), -1), (dict(L=(0.0, 1.0, 1.0)), -1), (dict(gamma=1.0), -1), (dict(prandtl=0.0), -1),
    (dict(mu=-1.0), -1), (dict(precision=7), -1), (dict(ckpt_format=adj.CKPT_BF16), -1),
    (dict(n=(1, 8, 4), bc_x=adj.BC_SLIP_WALLS), -2), (dict(bc_x=5), -1), (dict(dt=0.0), -1),
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
