"""Window trajectories in pinned host memory or in a file (paper_1511_06959_amd.offload): the
same sweeps as with the trajectory in HBM, so J, dJ/dw_0 and dJ/ds agree bit for bit, and every
stored state (or BF16 record) equals the one the HBM sweep stores."""
import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
import workloads as W
from paper_1511_06959_amd import offload, sweep
from tests.gpu_helpers import host

pytestmark = pytest.mark.gpu

CASES = [(adj.F64, adj.CKPT_NATIVE, 2, 0, False), (adj.F32, adj.CKPT_NATIVE, 3, 0, False),
         (adj.F32, adj.CKPT_BF16, 2, 0, False), (adj.F64, adj.CKPT_NATIVE, 2, 4, False),
         (adj.F32, adj.CKPT_BF16, 3, 1, False), (adj.F32, adj.CKPT_BF16, 2, 10, False),
         (adj.F64, adj.CKPT_NATIVE, 2, 0, True), (adj.F32, adj.CKPT_BF16, 3, 3, True)]
IDS = ["f64", "f32-3slots", "f32-bf16", "f64-tail4", "f32-bf16-3slots-tail1", "f32-bf16-all-in-hbm",
       "f64-file", "f32-bf16-file-3slots-tail3"]


@pytest.mark.parametrize("precision,ckpt,slots,tail,to_file", CASES, ids=IDS)
@pytest.mark.parametrize("lam_factor", [0.0, 0.3], ids=["lam0", "lam"])
def test_host_trajectory_matches_hbm(tmp_path, precision, ckpt, slots, tail, to_file, lam_factor):
    T = 9
    wl = W.turbulence((12, 10, 8), mach_rms=0.3, nu=0.02, seed=31, nsteps=T)
    ref = adj.reference_state(wl.w0) if precision == adj.F32 else None
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, precision, ckpt, ref)
    dt = g.dtype
    w0 = torch.from_numpy(g.to_stored(wl.w0)).to("cuda", dt)
    s = torch.from_numpy(1e-3 * np.random.default_rng(32).standard_normal(wl.w0.size)).to("cuda", dt)
    obj = adj.Objective.make(W.OBJ_MEAN_PRESSURE)
    weights = W.window_weights(T, 1, T)
    lam = lam_factor * (wl.L[0] / wl.n[0]) ** 2
    ws = adj.workspace(g)
    traj, _, J1 = sweep.forward(g, w0, s, T, obj, weights, ws)
    wh1, gs1, _ = sweep.backward(g, traj, s, obj, weights, lam, ws)
    J1, wh1, gs1 = host(J1), host(wh1), host(gs1)
    ht = offload.HostTrajectory(g, T, slots=slots, device_tail=tail,
                                path=str(tmp_path / "traj.bin") if to_file else None)
    assert ht.nhost == T + 1 - tail
    if not to_file:
        assert ht.host.is_pinned()
    ht, _, J2 = offload.forward(g, w0, s, T, obj, weights, ws, traj=ht)
    wh2, gs2 = offload.backward(g, ht, s, obj, weights, lam, ws)
    # a second reverse sweep over the same trajectory (the ring now holds other states)
    wh3, gs3 = offload.backward(g, ht, s, obj, weights, lam, ws)
    torch.cuda.synchronize()
    # a BF16 record: the plane and scale of every variable of every 4x4x4 block (100 bytes each,
    # the header padded to 256 bytes; the padding is never written), then the codes
    N = g.ncells
    nbl = -(-wl.n[0] // 4) * -(-wl.n[1] // 4) * -(-wl.n[2] // 4)
    used = [slice(0, 100 * nbl), slice(adj.ckpt_bytes(g) - 10 * N, None)] if ckpt == adj.CKPT_BF16 else [slice(None)]
    for n in range(T + 1):
        stored = ht.stored(n)
        for u in used:
            assert torch.equal(stored[u], traj.slot(n).cpu()[u]), f"state {n}"
    assert np.array_equal(host(J2), J1)
    for wh, gs in ((wh2, gs2), (wh3, gs3)):
        assert np.array_equal(host(wh), wh1)
        assert np.array_equal(host(gs), gs1)
    ht.close()
