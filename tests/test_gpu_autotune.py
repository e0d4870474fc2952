"""The tile autotuner (paper_1511_06959_amd.autotune) on small grids of every scheme option: it
times every tile that launches as itself, installs the fastest (the incumbent on near-ties),
reports the primal class per stage of a whole RK step, caches the choice, and leaves the results
of a step unchanged to rounding (the tile only changes how cells are grouped into work-groups)."""
import json

import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
import workloads as W
from paper_1511_06959_amd import autotune
from tests.gpu_helpers import host

pytestmark = pytest.mark.gpu

CASES = [("rk4-periodic-f32", adj.F32, adj.RK4, adj.FLUX_SPLIT, adj.BC_PERIODIC),
         ("ssprk3-wall-f64", adj.F64, adj.SSPRK3, adj.FLUX_SPLIT, adj.BC_SLIP_WALLS),
         ("roe-periodic-f32", adj.F32, adj.RK4, adj.FLUX_ROE, adj.BC_PERIODIC)]


@pytest.mark.parametrize("name,precision,scheme,flux,bc", CASES, ids=[c[0] for c in CASES])
def test_tune_installs_and_caches(tmp_path, monkeypatch, name, precision, scheme, flux, bc):
    wl = W.turbulence((20, 12, 10), mach_rms=0.3, nu=0.02, seed=5, nsteps=1)
    ref = adj.reference_state(wl.w0) if precision == adj.F32 else None
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, bc, precision, adj.CKPT_NATIVE, ref,
                      time_scheme=scheme, flux=flux)
    w = torch.from_numpy(g.to_stored(wl.w0)).to("cuda", g.dtype)
    ws = adj.workspace(g)
    before = {}
    for kc in (adj.PROF_ADJOINT_STAGE, adj.PROF_PRIMAL_STAGE):
        before[kc] = adj.get_tile(kc, precision)
    out0 = torch.empty_like(w)
    adj.primal_step(g, w, None, out0, ws)
    ref_step = host(out0)
    cache = tmp_path / "tiles.json"
    monkeypatch.setattr(autotune, "CACHE", str(cache))
    try:
        res = autotune.tune(g, reps=4, rounds=1)
        for kc in (adj.PROF_ADJOINT_STAGE, adj.PROF_PRIMAL_STAGE):
            best, times = res[kc]
            assert adj.get_tile(kc, precision) == best
            lnu = False
            cands = [t for t in adj.TILES if adj.tile_launched(kc, precision, bc, lnu, t) == t]
            assert sorted(times) == sorted(cands) and best in times
            assert all(ms > 0.0 for ms in times.values())
            assert times[best] <= min(times.values()) * 1.03 + 1e-12
        db = json.loads(cache.read_text())
        assert len(db) == 2
        # a cached configuration is installed without timing again
        for kc in (adj.PROF_ADJOINT_STAGE, adj.PROF_PRIMAL_STAGE):
            adj.set_tile(kc, precision, before[kc])
        res2 = autotune.tune(g)
        for kc in (adj.PROF_ADJOINT_STAGE, adj.PROF_PRIMAL_STAGE):
            assert res2[kc][0] == res[kc][0] and adj.get_tile(kc, precision) == res[kc][0]
        # every primal tile gives the same state to rounding: the per-cell arithmetic is the same
        # expression in every instantiation, which the compiler may contract and order differently
        out1 = torch.empty_like(w)
        tol = 1e-13 if precision == adj.F64 else 1e-6
        scale = np.abs(ref_step).max()
        for t in res[adj.PROF_PRIMAL_STAGE][1]:
            adj.set_tile(adj.PROF_PRIMAL_STAGE, precision, t)
            adj.primal_step(g, w, None, out1, ws)
            assert np.abs(host(out1) - ref_step).max() <= tol * scale, adj.TILES[t]
    finally:
        for kc in (adj.PROF_ADJOINT_STAGE, adj.PROF_PRIMAL_STAGE):
            adj.set_tile(kc, precision, before[kc])
