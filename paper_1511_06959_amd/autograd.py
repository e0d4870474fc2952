"""torch.autograd forms of the primal step, the objective and a whole checkpointed window.

The backward of each Function is the library's discrete adjoint ("Implementation": the
adjoint is the exact transpose of the discrete scheme, obtained in the paper by automatic
differentiation).  PyTorch only supplies memory, streams and the tape; every derivative is
computed by the HIP kernels behind the C ABI.

  PrimalStep.apply(w, s, spec)          -> w_next        backward: adj_adjoint_step
  ObjectiveValue.apply(w, spec)         -> j(w) (FP64)   backward: adj_objective_and_grad
  CheckpointedWindow.apply(w0, s, spec) -> J = sum_n c_n j(w_n)   backward: revolve schedule

``spec`` (a WindowSpec) carries the grid, objective, weights, lambda and the checkpointing plan:
``schedule = "binomial"`` (revolve with ``slots`` snapshot slots), ``"segments"`` (snapshots every
``segment`` steps, each segment re-advanced with its stage states kept, sweep.SegmentSweep) or
``"auto"`` (the default: the plan that sweep.plan_window picks for the free HBM less
``reserve_bytes``; slots or segment given explicitly take precedence).  With lambda > 0 the
backward is the paper's stabilised adjoint, deliberately not the exact gradient.
"""
from dataclasses import dataclass, field
from typing import Optional

import torch

from . import Grid, Objective, adjoint_step, objective_and_grad, primal_step, workspace
from .sweep import RevolveSweep, SegmentSweep, binomial_slots, plan_window, segment_length


@dataclass(eq=False)
class WindowSpec:
    g: Grid
    nsteps: int = 1
    obj: Optional[Objective] = None
    weights: Optional[list] = None
    lam: float = 0.0
    slots: Optional[int] = None
    ws: Optional[torch.Tensor] = None
    last: dict = field(default_factory=dict)  # diagnostics of the last backward (plan, advances)
    schedule: str = "auto"
    segment: Optional[int] = None
    reserve_bytes: int = 2 << 30  # HBM left free beside the checkpoints and working states (auto plans)
    energy_every: int = 0  # segment plans: keep the adjoint energy every so many reverse steps
    progress: Optional[object] = None  # called with the step index after every reverse step

    def workspace(self):
        if self.ws is None:
            self.ws = workspace(self.g)
        return self.ws

    def plan(self, device):
        """(schedule, size): ("binomial", slots) or ("segments", segment length)."""
        if self.slots is not None and self.schedule in ("auto", "binomial"):
            return "binomial", int(self.slots)
        if self.segment is not None and self.schedule in ("auto", "segments"):
            return "segments", int(self.segment)
        self.workspace()  # allocated before the free memory is read
        torch.cuda.empty_cache()  # blocks the caching allocator holds free count as free
        free, _ = torch.cuda.mem_get_info(device)
        # besides the checkpoints: the sweep's working states and adjoints (a, b, grad_s, current,
        # next and final state) and the caller's w0, s and gradients
        state = 5 * self.g.ncells * (8 if self.g.precision == 0 else 4)
        budget = max(0, free - self.reserve_bytes - 8 * state)
        if self.schedule == "binomial":
            return "binomial", binomial_slots(self.g, self.nsteps, budget)
        if self.schedule == "segments":
            return "segments", segment_length(self.g, self.nsteps)
        return plan_window(self.g, self.nsteps, budget)


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
    """J = sum_n c_n j(w_n) over nsteps RK4 steps from w0 with the checkpointing plan of spec
    (snapshots as BF16 records when spec.g.ckpt_format says so)."""

    @staticmethod
    def forward(ctx, w0, s, spec):
        kind, size = spec.plan(w0.device)
        cls = RevolveSweep if kind == "binomial" else SegmentSweep
        sweep = cls(spec.g, spec.nsteps, size, None if s is None else s.contiguous(), spec.obj, spec.weights,
                    spec.lam, spec.workspace(), w0.device)
        J = sweep.forward(w0.contiguous())
        ctx.sweep = sweep
        ctx.spec = spec
        ctx.has_s = s is not None
        spec.last = {"schedule": kind, "slots" if kind == "binomial" else "segment": size,
                     "forward_steps": sweep.advanced}
        return J[0]

    @staticmethod
    def backward(ctx, gJ):
        sweep, spec = ctx.sweep, ctx.spec
        before = sweep.advanced
        if isinstance(sweep, SegmentSweep):
            wh0, gs = sweep.backward(scale=float(gJ), energy_every=spec.energy_every, progress=spec.progress)
            spec.last["energy"] = [(n, float(E.cpu()[0])) for n, E in sweep.energy]
        else:
            wh0, gs = sweep.backward(scale=float(gJ), progress=spec.progress)
        spec.last["recompute_steps"] = sweep.advanced - before
        ctx.sweep = None
        return wh0, (gs if ctx.has_s else None), None


def window_objective(w0, s, spec):
    """Differentiable J(w0, s) of a window (see CheckpointedWindow)."""
    return CheckpointedWindow.apply(w0, s, spec)
