"""Whole windows at the full benchmark sizes against the oracle's windows on blocks.

The GPU runs a K-step window (forward sweep, then the reverse sweep with the mean-pressure
objective c_n = 1/K on n = 1..K, lambda = 0.1 dx^2 sigma_1 and a body force: the workload's own
plus seeded noise) on the whole grid (384^3 turbulence, the 512x256x32 wake between slip walls, the
spatially developing wake with its characteristic inlet and outlet; split or Roe flux),
with the benchmark's checkpointing: the two-level segment sweep, with BF16 snapshots (the
benchmark's FP32 path) or native ones, as each case names.  Each 4x4x4 sample of dJ/dw_0 and dJ/ds is compared
with the oracle's own window (forward from the same initial field, then reverse) on a 36^3 block
around it.  The oracle treats the block as periodic (or, for the wake, as walled in x where the
real wall is), and an output of a K-step window depends only on cells within a bounded distance,
so samples 16 cells inside every artificial block face are exact for K = 3 (checked on the CPU by
tests/test_oracle_cone.py); the Roe flux's reconstruction reaches two cells per stage, and its
blocks are 44 cells (20-cell margins: exact to rounding, 16 leaves 8e-14 on a 48^3 check).  The mean pressure's gradient is local; on a block of M cells the
oracle's j averages over M cells, so its weights are scaled by M / N.

Bars: FP64 1e-10 per field.  FP32 stencils with BF16 snapshots: 1e-4 per field on the decaying
turbulence.  On the wake the initial field carries broadband perturbations up to the grid scale,
which no block plane predicts, so the BF16 snapshot keeps each perturbation value to its 8-bit
significand (2^-9 of itself): the adjoints of the small cross-stream and spanwise momenta
(an order of magnitude below the other fields) move by up to ~1e-3 of their own scale, while the
gradient as a whole stays within 1e-4.  The wake's FP32 path with native FP32 snapshots holds
1e-4 per field, so the excess is the BF16 storage, not the FP32 arithmetic; records of the same
size with 16-bit fixed-point codes (s/65534 whatever the value) hold 1e-4 per field as well.
"""
import numpy as np
import pytest
import torch

import paper_1511_06959_amd as adj
import workloads as W
from paper_1511_06959_amd import autotune
from paper_1511_06959_amd.sweep import SegmentSweep
from tests.gpu_helpers import host, relerr, relerr_vars

pytestmark = pytest.mark.gpu

K = 3
SAMPLE = 4


def _axis(n, s0, walled, block):
    """Block indices along one axis (see tests/test_gpu_fullsize.py): the whole axis if short, a
    block from the real boundary for samples near a wall or an open boundary, else a wrapped block
    centred on the sample."""
    off = (block - SAMPLE) // 2
    if n <= block:
        return np.arange(n), walled
    if walled and s0 < off:
        return np.arange(block), True
    if walled and s0 + SAMPLE > n - off:
        return np.arange(n - block, n), True
    return (s0 - off + np.arange(block)) % n, False


def _window_parity(orc, wl, precision, ckpt, starts, seed, flux=0, block=36):
    """Largest relative errors of the sampled dJ/dw_0 and dJ/ds: (per field, whole sample)."""
    f32 = precision == adj.F32
    ref = adj.reference_state(wl.w0) if f32 else None
    far = wl.params().get("w_far")
    g = adj.Grid.make(wl.n, wl.L, wl.mu, wl.dt, wl.gamma, wl.prandtl, wl.bc_x, precision, ckpt, ref,
                      w_far=wl.extra.get("w_far"), flux=flux, roe_delta=0.1)
    autotune.tune(g)
    lam = 0.1 * min(wl.L[d] / wl.n[d] for d in range(3)) ** 2
    nx, ny, nz = wl.n
    N = g.ncells
    npdt = np.float32 if f32 else np.float64
    stored = g.to_stored(wl.w0).astype(npdt)
    s = (wl.s + 1e-3 * np.random.default_rng(seed).standard_normal(5 * N)).astype(npdt)
    weights = W.window_weights(K, 1, K)
    obj = adj.Objective.make(W.OBJ_MEAN_PRESSURE)
    print(f"[window parity] {wl.name} {'f32' if f32 else 'f64'} {('native', 'bf16', 'i16')[ckpt]} "
          f"snapshots{' roe' if flux else ''} K={K}", flush=True)
    sw = SegmentSweep(g, K, K, torch.from_numpy(s).to("cuda"), obj, weights, lam, adj.workspace(g))
    sw.forward(torch.from_numpy(stored).to("cuda"))
    wh0, gs = sw.backward()
    wh5, gs5 = host(wh0).reshape(5, nz, ny, nx), host(gs).reshape(5, nz, ny, nx)
    w5 = g.from_stored(stored.astype(np.float64)).reshape(5, nz, ny, nx)
    s5 = s.astype(np.float64).reshape(5, nz, ny, nx)
    oobj = orc.make_obj(W.OBJ_MEAN_PRESSURE)
    worst = np.zeros(2)
    for start in starts:
        (ix, wall), (iy, _), (iz, _) = (_axis(wl.n[d], start[d], d == 0 and wl.bc_x != 0, block) for d in range(3))
        blk = np.ix_(np.arange(5), iz, iy, ix)
        bn = (len(ix), len(iy), len(iz))
        og = orc.make_grid(bn, tuple(bn[d] * wl.L[d] / wl.n[d] for d in range(3)), wl.gamma, wl.prandtl, wl.mu,
                           wl.dt, wl.bc_x if wall else 0, flux=flux, roe_delta=0.1, w_far=far)
        wb, sb = w5[blk].ravel(), s5[blk].ravel()
        traj = orc.primal_window(og, wb, sb, K)
        rw, rs = orc.adjoint_window(og, oobj, traj, sb, weights * (bn[0] * bn[1] * bn[2] / N), lam)
        rw, rs = rw.reshape(5, *bn[::-1]), rs.reshape(5, *bn[::-1])
        pos = [int(np.nonzero(ii == s0)[0][0]) for ii, s0 in zip((ix, iy, iz), start)]
        sl = (slice(None), slice(pos[2], pos[2] + SAMPLE), slice(pos[1], pos[1] + SAMPLE),
              slice(pos[0], pos[0] + SAMPLE))
        cells = np.ix_(np.arange(5), iz[sl[1]], iy[sl[2]], ix[sl[3]])
        e = np.array([max(relerr_vars(wh5[cells], rw[sl]), relerr_vars(gs5[cells], rs[sl])),
                      max(relerr(wh5[cells], rw[sl]), relerr(gs5[cells], rs[sl]))])
        print(f"[window parity]   sample {start}: per field {e[0]:.2e}, whole sample {e[1]:.2e}", flush=True)
        worst = np.maximum(worst, e)
    return worst


@pytest.fixture(scope="module")
def turb384():
    return W.turb_384(nsteps=K)


@pytest.fixture(scope="module")
def wake():
    return W.wake(nsteps=K)


@pytest.mark.parametrize("precision,ckpt,tol", [(adj.F64, adj.CKPT_NATIVE, 1e-10), (adj.F32, adj.CKPT_BF16, 1e-4)],
                         ids=["f64", "f32-bf16"])
def test_turb384_window_sampled(orc, turb384, precision, ckpt, tol):
    n = turb384.n[0]
    starts = [(0, 0, 0), (100, 200, 300), (n - 2, 17, n - 3)]
    per_field, whole = _window_parity(orc, turb384, precision, ckpt, starts, 70)
    assert per_field <= tol and whole <= tol


@pytest.mark.parametrize("precision,ckpt,tol_field,tol_whole",
                         [(adj.F64, adj.CKPT_NATIVE, 1e-10, 1e-10), (adj.F32, adj.CKPT_NATIVE, 1e-4, 1e-4),
                          (adj.F32, adj.CKPT_BF16, 2e-3, 1e-4), (adj.F32, adj.CKPT_I16, 1e-4, 1e-4)],
                         ids=["f64", "f32", "f32-bf16", "f32-i16"])
def test_wake_window_sampled(orc, wake, precision, ckpt, tol_field, tol_whole):
    nx = wake.n[0]
    starts = [(0, 10, 0), (nx - SAMPLE, 250, 8), (254, 100, 20)]
    per_field, whole = _window_parity(orc, wake, precision, ckpt, starts, 71)
    assert per_field <= tol_field and whole <= tol_whole


@pytest.fixture(scope="module")
def spatial_wake():
    return W.spatial_wake(nsteps=K)


@pytest.mark.parametrize("precision,ckpt,tol_field,tol_whole",
                         [(adj.F64, adj.CKPT_NATIVE, 1e-10, 1e-10), (adj.F32, adj.CKPT_BF16, 2e-3, 1e-4)],
                         ids=["f64", "f32-bf16"])
@pytest.mark.parametrize("flux", [0, adj.FLUX_ROE], ids=["split", "roe"])
def test_spatial_wake_window_sampled(orc, spatial_wake, flux, precision, ckpt, tol_field, tol_whole):
    """Characteristic inlet and outlet with the drag strip's body force: samples at the inlet, in
    the strip, on the loss plane and at the outlet; blocks at an open end keep it and its far field.
    With the Roe flux the blocks grow to 44 cells (its reconstruction reaches two cells per stage)."""
    nx = spatial_wake.n[0]
    starts = [(0, 126, 5), (49, 130, 14), (382, 120, 30), (nx - SAMPLE, 3, 0)]
    per_field, whole = _window_parity(orc, spatial_wake, precision, ckpt, starts, 72, flux=flux,
                                      block=44 if flux else 36)
    assert per_field <= tol_field and whole <= tol_whole


@pytest.mark.parametrize("precision,ckpt,tol", [(adj.F64, adj.CKPT_NATIVE, 1e-10), (adj.F32, adj.CKPT_BF16, 1e-4)],
                         ids=["f64", "f32-bf16"])
def test_turb384_roe_window_sampled(orc, turb384, precision, ckpt, tol):
    n = turb384.n[0]
    starts = [(0, 0, 0), (200, 100, 300)]
    per_field, whole = _window_parity(orc, turb384, precision, ckpt, starts, 73, flux=adj.FLUX_ROE, block=44)
    assert per_field <= tol and whole <= tol
