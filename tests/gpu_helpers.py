"""Shared helpers of the GPU parity tests (seeded states, device transfer, error metrics)."""
import math

import numpy as np
import torch

import paper_1511_06959_amd as adj
import workloads as W


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy().copy()


def smooth_state(n, L=(2 * math.pi,) * 3, seed=0, amp=0.1, wall=False):
    rng = np.random.default_rng(seed)
    x, y, z = W.cell_centres(n, L)
    k = [2 * math.pi / L[d] for d in range(3)]
    rho = 1.0 + amp * np.sin(k[0] * x + 2 * k[1] * y) * np.cos(k[2] * z) + 0.01 * rng.standard_normal(x.shape)
    u = 0.3 * np.sin(k[0] * x) * np.cos(k[1] * y) + 0.03 * rng.standard_normal(x.shape)
    v = -0.2 * np.cos(k[0] * x) * np.sin(k[2] * z) + 0.03 * rng.standard_normal(x.shape)
    w = 0.1 * np.sin(k[1] * y + k[2] * z) + 0.03 * rng.standard_normal(x.shape)
    p = 1.0 / 1.4 * (1.0 + amp * np.cos(2 * k[0] * x - k[1] * y)) + 0.01 * rng.standard_normal(x.shape)
    return W.conservative(rho, u, v, w, p)


def grids(orc, n, L, mu, dt, bc_x=0, precision=adj.F64, ckpt=adj.CKPT_NATIVE, gamma=1.4, prandtl=0.72):
    g = adj.Grid.make(n, L, mu, dt, gamma, prandtl, bc_x, precision, ckpt)
    og = orc.make_grid(n, L, gamma, prandtl, mu, dt, bc_x)
    return g, og


def relerr(a, b):
    """max |a - b| / max |b| (b the oracle)."""
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def relerr_vars(a, b, floor=1e-6):
    """Largest per-variable error: max over the five fields v of max |a_v - b_v| / max |b_v|
    (b the oracle), each field's scale floored at `floor` times the largest field's, so that a
    field that is orders of magnitude smaller than the others is held to its own scale."""
    a = np.asarray(a, dtype=np.float64).reshape(5, -1)
    b = np.asarray(b, dtype=np.float64).reshape(5, -1)
    top = np.abs(b).max()
    if top == 0:
        return float(np.abs(a).max())
    return float(max(np.abs(a[v] - b[v]).max() / max(np.abs(b[v]).max(), floor * top) for v in range(5)))
