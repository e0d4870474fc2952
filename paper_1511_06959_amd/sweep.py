"""Window schedules around the C ABI: forward sweep storing the trajectory in HBM, reverse sweep.

The paper stores periodic primal snapshots and recomputes in between ("Implementation",
checkpointing); with 288 GB of HBM the whole trajectory of a window usually fits, so the
default schedule here keeps every state (natively or as BF16 records) on the device and the
reverse sweep recomputes only the three inner RK4 stage states of each step, inside
``adjoint_step``.  Binomial checkpointing for windows that do not fit lives in ``revolve.py``.

Only scheduling happens here; all arithmetic runs in the library's kernels.
"""
import torch

from . import (CKPT_BF16, OBJ_NONE, Grid, Objective, adjoint_step, ckpt_bytes, energy_vhat, objective_and_grad,
               primal_step, workspace)


class Trajectory:
    """States w_0..w_N of one window, kept in HBM as full-precision states or BF16 records."""

    def __init__(self, g, nsteps, device="cuda"):
        self.g = g
        self.nsteps = nsteps
        N5 = 5 * g.ncells
        if g.ckpt_format == CKPT_BF16:
            self.rec_bytes = ckpt_bytes(g)
            self.store = torch.empty((nsteps + 1, self.rec_bytes), dtype=torch.uint8, device=device)
        else:
            self.store = torch.empty((nsteps + 1, N5), dtype=g.dtype, device=device)

    def slot(self, n):
        return self.store[n]


def forward(g, w0, s, nsteps, obj=None, weights=None, ws=None, traj=None, J=None):
    """Primal sweep w_0 -> w_N storing every state; J (device FP64 scalar) += sum_n c_n j(w_n).

    With BF16 storage the sweep itself still advances in FP32; only the stored copies are
    encoded (the adjoint then runs on the decoded states).  Returns (trajectory, w_N, J)."""
    ws = workspace(g) if ws is None else ws
    traj = Trajectory(g, nsteps, w0.device) if traj is None else traj
    J = torch.zeros(1, dtype=torch.float64, device=w0.device) if J is None else J
    bf16 = g.ckpt_format == CKPT_BF16
    cur = w0.clone()
    nxt = torch.empty_like(w0)
    if bf16:
        from . import ckpt_encode
        ckpt_encode(g, cur, traj.slot(0), ws)
    else:
        traj.slot(0).copy_(cur)
    use_obj = obj is not None and obj.kind != OBJ_NONE and weights is not None
    if use_obj and weights[0] != 0.0:
        objective_and_grad(g, obj, cur, ws, weight=float(weights[0]), J_accum=J)
    for n in range(nsteps):
        if bf16:
            primal_step(g, cur, s, nxt, ws, ckpt_out=traj.slot(n + 1))
        else:
            primal_step(g, cur, s, traj.slot(n + 1), ws)
            nxt = traj.slot(n + 1)
        if use_obj and weights[n + 1] != 0.0:
            objective_and_grad(g, obj, nxt, ws, weight=float(weights[n + 1]), J_accum=J)
        if bf16:
            cur, nxt = nxt, cur
        else:
            cur = nxt
    return traj, cur, J


def backward(g, traj, s, obj=None, weights=None, lam=0.0, ws=None, grad_s=None, terminal=None, energy=False):
    """Reverse sweep over a stored trajectory.  Returns (w^_0, grad_s, E) where E is a device
    FP64 tensor of the adjoint energy after each reverse step (index n = step n) or None."""
    ws = workspace(g) if ws is None else ws
    N = traj.nsteps
    dev = traj.store.device
    N5 = 5 * g.ncells
    a = torch.zeros(N5, dtype=g.dtype, device=dev)
    b = torch.empty_like(a)
    grad_s = torch.zeros(N5, dtype=g.dtype, device=dev) if grad_s is None else grad_s
    use_obj = obj is not None and obj.kind != OBJ_NONE and weights is not None
    bf16 = g.ckpt_format == CKPT_BF16
    dec = None
    if bf16 or energy:
        dec = torch.empty(N5, dtype=g.dtype, device=dev)

    def state(n):
        if not bf16:
            return traj.slot(n)
        from . import ckpt_decode
        ckpt_decode(g, traj.slot(n), dec)
        return dec

    if terminal is not None:
        a.copy_(terminal)
    if use_obj and weights[N] != 0.0:
        objective_and_grad(g, obj, state(N), ws, weight=float(weights[N]), djdw=a)
    E = torch.zeros(N + 1, dtype=torch.float64, device=dev) if energy else None
    if energy:
        energy_vhat(g, state(N), a, E[N:N + 1], ws)
    for n in range(N - 1, -1, -1):
        c_n = float(weights[n]) if use_obj else 0.0
        adjoint_step(g, traj.slot(n), s, a, b, ws, lam=lam, obj=obj if use_obj else None, c_n=c_n, grad_s=grad_s)
        a, b = b, a
        if energy:
            energy_vhat(g, state(n), a, E[n:n + 1], ws)
    return a, grad_s, E
