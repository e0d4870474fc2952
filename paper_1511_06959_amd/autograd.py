"""torch.autograd forms of the primal step, the objective and a whole checkpointed window.

The backward of each Function is the library's discrete adjoint ("Implementation": the
adjoint is the exact transpose of the discrete scheme, obtained in the paper by automatic
differentiation).  PyTorch only supplies memory, streams and the tape; every derivative is
computed by the HIP kernels behind the C ABI.

  PrimalStep.apply(w, s, spec)          -> w_next        backward: adj_adjoint_step
  ObjectiveValue.apply(w, spec)         -> j(w) (FP64)   backward: adj_objective_and_grad
  CheckpointedWindow.apply(w0, s, spec) -> J = sum_n c_n j(w_n)   backward: revolve schedule

``spec`` (a WindowSpec) carries the grid, objective, weights, lambda and slot budget.  With
lambda > 0 the backward is the paper's stabilised adjoint, deliberately not the exact gradient.
"""
from dataclasses import dataclass, field
from typing import Optional

import torch

from . import Grid, Objective, adjoint_step, objective_and_grad, primal_step, workspace
from .sweep import RevolveSweep


@dataclass(eq=False)
class WindowSpec:
    g: Grid
    nsteps: int = 1
    obj: Optional[Objective] = None
    weights: Optional[list] = None
    lam: float = 0.0
    slots: int = 2
    ws: Optional[torch.Tensor] = None
    last: dict = field(default_factory=dict)  # diagnostics of the last backward (advances etc.)

    def workspace(self):
        if self.ws is None:
            self.ws = workspace(self.g)
        return self.ws


def _zero_if_none(t, like):
    return torch.zeros_like(like) if t is None else t


class PrimalStep(torch.autograd.Function):
    """One RK4 step; the source s may be None."""

    @staticmethod
    def forward(ctx, w, s, spec):
        out = torch.empty_like(w)
        primal_step(spec.g, w.contiguous(), None if s is None else s.contiguous(), out, spec.workspace())
        ctx.spec = spec
        ctx.has_s = s is not None
        ctx.save_for_backward(w, s if s is not None else w.new_empty(0))
        return out

    @staticmethod
    def backward(ctx, gout):
        w, s = ctx.saved_tensors
        spec = ctx.spec
        wh = torch.empty_like(w)
        gs = torch.zeros_like(w)
        adjoint_step(spec.g, w, s if ctx.has_s else None, gout.contiguous(), wh, spec.workspace(), lam=spec.lam,
                     grad_s=gs)
        return wh, (gs if ctx.has_s else None), None


class ObjectiveValue(torch.autograd.Function):
    """j(w) as a 0-dim FP64 tensor."""

    @staticmethod
    def forward(ctx, w, spec):
        J = torch.zeros(1, dtype=torch.float64, device=w.device)
        objective_and_grad(spec.g, spec.obj, w.contiguous(), spec.workspace(), weight=1.0, J_accum=J)
        ctx.spec = spec
        ctx.save_for_backward(w)
        return J[0]

    @staticmethod
    def backward(ctx, gJ):
        (w,) = ctx.saved_tensors
        spec = ctx.spec
        dj = torch.zeros_like(w)
        objective_and_grad(spec.g, spec.obj, w, spec.workspace(), weight=float(gJ), djdw=dj)
        return dj, None


class CheckpointedWindow(torch.autograd.Function):
    """J = sum_n c_n j(w_n) over nsteps RK4 steps from w0, with binomial checkpointing in
    spec.slots snapshot slots (BF16 records when spec.g.ckpt_format says so)."""

    @staticmethod
    def forward(ctx, w0, s, spec):
        sweep = RevolveSweep(spec.g, spec.nsteps, spec.slots, None if s is None else s.contiguous(), spec.obj,
                             spec.weights, spec.lam, spec.workspace(), w0.device)
        J = sweep.forward(w0.contiguous())
        ctx.sweep = sweep
        ctx.spec = spec
        ctx.has_s = s is not None
        spec.last = {"forward_steps": sweep.advanced}
        return J[0]

    @staticmethod
    def backward(ctx, gJ):
        sweep, spec = ctx.sweep, ctx.spec
        before = sweep.advanced
        wh0, gs = sweep.backward(scale=float(gJ))
        spec.last["recompute_steps"] = sweep.advanced - before
        ctx.sweep = None
        return wh0, (gs if ctx.has_s else None), None


def window_objective(w0, s, spec):
    """Differentiable J(w0, s) of a window (see CheckpointedWindow)."""
    return CheckpointedWindow.apply(w0, s, spec)
