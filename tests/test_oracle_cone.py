"""Locality of a window (a CPU pin of the block sampling used at the full benchmark sizes).

The forward sweep and the reverse sweep of a K-step window move information a bounded number of
cells per RK stage, so the oracle's window on a block cut from the grid, treated as periodic (or as
walled in x where the real slip wall is), gives dJ/dw_0 and dJ/ds of the whole grid's window in
cells far enough from the artificial block faces.  For K = 3 a margin of 16 cells reproduces the
whole-grid values to rounding, which is what the sampled full-size window tests rely on; a margin
of 2 does not (the check has teeth).  The mean-pressure weights are scaled by the block's share of
the cells (its j averages over the block).
"""
import numpy as np

import workloads as W

K = 3


def _cut(f, n, lo, size):
    f = np.asarray(f).reshape(5, n[2], n[1], n[0])
    ix, iy, iz = [(lo[d] + np.arange(size[d])) % n[d] for d in range(3)]
    return f[np.ix_(np.arange(5), iz, iy, ix)].reshape(-1)


def _window(orc, g, w0, s, weights, lam):
    traj = orc.primal_window(g, w0, s, K)
    return orc.adjoint_window(g, orc.make_obj(W.OBJ_MEAN_PRESSURE), traj, s, weights, lam)


def _block_errors(orc, wl, lo, size, sample_at, margin_ok, bc_block):
    n = wl.n
    N = wl.ncells
    lam = 0.1 * min(wl.L[d] / n[d] for d in range(3)) ** 2
    s = 1e-3 * np.random.default_rng(9).standard_normal(5 * N)
    weights = W.window_weights(K, 1, K)
    g = orc.grid_from(wl.params())
    a_full, gs_full = _window(orc, g, wl.w0, s, weights, lam)
    p = wl.params()
    p["n"] = tuple(size)
    p["L"] = tuple(wl.L[d] / n[d] * size[d] for d in range(3))
    p["bc_x"] = bc_block
    gb = orc.grid_from(p)
    M = size[0] * size[1] * size[2]
    a_b, gs_b = _window(orc, gb, _cut(wl.w0, n, lo, size), _cut(s, n, lo, size), weights * (M / N), lam)
    out = []
    for full, blk in ((a_full, a_b), (gs_full, gs_b)):
        ref = _cut(full, n, tuple(lo[d] + sample_at[d] for d in range(3)), (4, 4, 4)).reshape(5, -1)
        got = blk.reshape(5, size[2], size[1], size[0])[:, sample_at[2]:sample_at[2] + 4,
                                                         sample_at[1]:sample_at[1] + 4,
                                                         sample_at[0]:sample_at[0] + 4].reshape(5, -1)
        out.append(np.abs(got - ref).max() / np.abs(ref).max())
    return out


def test_periodic_block_margin(orc):
    wl = W.turbulence(40, mach_rms=0.4, nu=2.887e-3, seed=4, nsteps=K)
    # a 36^3 block wrapping the periodic boundary, the sample 16 cells inside every face
    ew, es = _block_errors(orc, wl, (30, 21, 38), (36, 36, 36), (16, 16, 16), True, 0)
    assert ew <= 1e-13 and es <= 1e-13
    # with a 2-cell margin the artificial faces reach the sample
    ew, es = _block_errors(orc, wl, (44, 35, 52), (8, 8, 8), (2, 2, 2), False, 0)
    assert ew > 1e-6 and es > 1e-6


def test_walled_block_margin(orc):
    wl = W.wake(n=(48, 40, 8), nsteps=K)
    # the block starts at the slip wall x = 0 and ends 36 cells in (an artificial wall), wraps in y
    # and holds the whole span; the sample touches the real wall
    ew, es = _block_errors(orc, wl, (0, 30, 0), (36, 36, 8), (0, 16, 0), True, 1)
    assert ew <= 1e-13 and es <= 1e-13
