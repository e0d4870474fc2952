"""Ensembles of uneven adjoint windows and lambda sweeps, batched through the adj_batch_* calls.

Each box runs its own window of T_b RK4 steps from w_0 with the time-averaged objective
J_b = (1/T_b) sum_{n=1..T_b} j(w_n) (the rectangle rule of the averaged objectives of the paper,
Eqs. (1)-(3)); each member is one reverse sweep over its box's trajectory with its own lambda
("Stabilizing adjoint equations").  Boxes are ordered by non-increasing window length, so at
step t the boxes still running form a prefix of the packed arrays and one launch per RK stage
covers all of them; the whole ensemble window is then captured as two HIP graphs.

The trajectory of the ensemble is stored whole: slot t keeps w_t of the boxes with T_b >= t
(natively, in the state precision), so it holds sum_b 5 N_b (T_b + 1) values.  The reverse sweep
recomputes the inner RK4 stage states of each step inside the batched adjoint step.

When the stored trajectory of a whole ensemble exceeds the memory at hand, PlannedEnsemble runs
it in consecutive groups of boxes, each within a byte budget.

Only scheduling happens here; all arithmetic runs in the library's kernels.
"""
import bisect

import torch

from . import F64, OBJ_MEAN_PRESSURE, Ensemble, Objective


class EnsembleWindow:
    """Forward and reverse sweep of an ensemble.

    grids:      one Grid per box (same precision and x boundary), ordered by non-increasing window
    windows:    T_b per box (>= 1)
    w0, s:      lists of per-box initial states / sources (s may be None, or a list with Nones
                replaced by zeros)
    member_box: box of each member (non-decreasing); member_lam: lambda (L^2) of each member
    energy:     also record the adjoint energy of every member after every reverse step
    """

    def __init__(self, grids, windows, w0, s=None, member_box=None, member_lam=None, obj_kind=OBJ_MEAN_PRESSURE,
                 energy=False, device="cuda"):
        nb = len(grids)
        self.windows = [int(t) for t in windows]
        if len(self.windows) != nb or any(t < 1 for t in self.windows):
            raise ValueError("one window length >= 1 per box")
        if any(self.windows[i] < self.windows[i + 1] for i in range(nb - 1)):
            raise ValueError("boxes must be ordered by non-increasing window length")
        member_box = list(range(nb)) if member_box is None else [int(b) for b in member_box]
        member_lam = [0.0] * len(member_box) if member_lam is None else [float(x) for x in member_lam]
        self.obj = Objective.make(obj_kind)
        self.ens = Ensemble(grids, member_box, member_lam, self.obj, device)
        self.nbox, self.nmem = nb, len(member_box)
        self.member_box = member_box
        self.dtype = torch.float64 if grids[0].precision == F64 else torch.float32
        dt = self.dtype
        ens = self.ens
        self.Tmax = self.windows[0]
        # boxes with T_b >= t, as a count (windows are non-increasing): nbox_ge(t)
        neg = [-t for t in self.windows]
        self._nbox_ge = [bisect.bisect_right(neg, -t) for t in range(self.Tmax + 2)]
        self._nmem_of_nbox = [bisect.bisect_left(member_box, b) for b in range(nb + 1)]
        P = ens.offset(0, nb)
        Q = ens.offset(1, self.nmem)
        self.slots = [torch.empty(5 * ens.offset(0, self._nbox_ge[t]), dtype=dt, device=device)
                      for t in range(self.Tmax + 1)]
        self.w0 = torch.empty(5 * P, dtype=dt, device=device)
        for b in range(nb):
            ens.box_slice(self.w0, b).copy_(torch.as_tensor(w0[b]).to(device=device, dtype=dt).reshape(-1))
        self.s = None
        if s is not None:
            self.s = torch.zeros(5 * P, dtype=dt, device=device)
            for b in range(nb):
                if s[b] is not None:
                    ens.box_slice(self.s, b).copy_(torch.as_tensor(s[b]).to(device=device, dtype=dt).reshape(-1))
        self.wmem = torch.tensor([1.0 / self.windows[b] for b in member_box], dtype=torch.float64, device=device)
        self.J = torch.zeros(self.nmem, dtype=torch.float64, device=device)
        self.a = torch.zeros(5 * Q, dtype=dt, device=device)
        self.b = torch.zeros(5 * Q, dtype=dt, device=device)
        self.grad_s = torch.zeros(5 * Q, dtype=dt, device=device)
        self.wh0 = self.a
        self.E = torch.zeros((self.Tmax + 1, self.nmem), dtype=torch.float64, device=device) if energy else None
        self.ws = ens.workspace(device)

    def cell_steps(self):
        """Primal cell-steps of one window: sum_b N_b T_b."""
        return sum((self.ens.offset(0, b + 1) - self.ens.offset(0, b)) * self.windows[b] for b in range(self.nbox))

    def adjoint_cell_steps(self):
        return sum((self.ens.offset(1, m + 1) - self.ens.offset(1, m)) * self.windows[self.member_box[m]]
                   for m in range(self.nmem))

    def _nmem_running(self, t):
        """Members whose box runs step t (T_b > t)."""
        return self._nmem_of_nbox[self._nbox_ge[t + 1]]

    def forward(self):
        ens, ws = self.ens, self.ws
        self.J.zero_()
        self.slots[0].copy_(self.w0)
        for t in range(self.Tmax):
            nb = self._nbox_ge[t + 1]
            ens.primal_step(nb, self.slots[t], self.s, self.slots[t + 1], ws)
            nm = self._nmem_of_nbox[nb]
            if nm:
                ens.objective_and_grad(0, nm, self.slots[t + 1], self.wmem, ws, J_accum=self.J)
        return self.J

    def backward(self):
        ens, ws = self.ens, self.ws
        a, b = self.a, self.b
        self.grad_s.zero_()
        for n in range(self.Tmax - 1, -1, -1):
            nm = self._nmem_running(n)
            m0 = self._nmem_running(n + 1) if n + 1 < self.Tmax else 0
            if nm > m0:
                # members whose window ends at w_{n+1}: terminal adjoint c_T dj/dw(w_T)
                lo, hi = 5 * ens.offset(1, m0), 5 * ens.offset(1, nm)
                a[lo:hi].zero_()
                ens.objective_and_grad(m0, nm - m0, self.slots[n + 1], self.wmem, ws, djdw=a)
                if self.E is not None:
                    ens.energy_vhat(nm, self.slots[n + 1], a, self.E[n + 1], ws)
            if nm:
                ens.adjoint_step(nm, self.slots[n], self.s, a, b, ws, c_n=self.wmem if n >= 1 else None,
                                 grad_s=self.grad_s)
                a, b = b, a
                if self.E is not None:
                    ens.energy_vhat(nm, self.slots[n], a, self.E[n], ws)
        self.wh0 = a
        return a, self.grad_s

    def member(self, t, m):
        """Member m's part of a member-packed tensor."""
        return self.ens.member_slice(t, m)


class CapturedEnsemble:
    """An EnsembleWindow captured once as two HIP graphs (forward sweep, reverse sweep)."""

    def __init__(self, window):
        self.win = window
        self._fwd = torch.cuda.CUDAGraph()
        self._bwd = torch.cuda.CUDAGraph()
        window.forward()
        window.backward()
        torch.cuda.synchronize()
        with torch.cuda.graph(self._fwd):
            window.forward()
        with torch.cuda.graph(self._bwd):
            window.backward()
        torch.cuda.synchronize()

    def run_forward(self):
        self._fwd.replay()

    def run_backward(self):
        self._bwd.replay()

    def run(self):
        """Replay both sweeps; returns (J per member, packed w^_0, packed grad_s)."""
        self._fwd.replay()
        self._bwd.replay()
        return self.win.J, self.win.wh0, self.win.grad_s


def trajectory_bytes(grids, windows):
    """HBM held by an EnsembleWindow's stored trajectory: 5 N_b (T_b + 1) state values per box."""
    return sum(5 * g.ncells * (int(t) + 1) * (8 if g.precision == F64 else 4) for g, t in zip(grids, windows))


def plan(grids, windows, member_box, budget_bytes):
    """Split an ensemble (boxes ordered by non-increasing window) into consecutive groups of boxes
    whose stored trajectories each fit in `budget_bytes`; a box that alone exceeds the budget
    forms a group of its own.  Returns [(first_box, end_box, first_member, end_member)]."""
    groups, start, used = [], 0, 0
    for b in range(len(grids)):
        need = trajectory_bytes([grids[b]], [windows[b]])
        if b > start and used + need > budget_bytes:
            groups.append((start, b))
            start, used = b, 0
        used += need
    groups.append((start, len(grids)))
    out = []
    for b0, b1 in groups:
        m0 = bisect.bisect_left(member_box, b0)
        m1 = bisect.bisect_left(member_box, b1)
        out.append((b0, b1, m0, m1))
    return out


class PlannedEnsemble:
    """An ensemble run group by group when its whole trajectory exceeds a memory budget (the
    worst-case draws of the batched configuration need more than one GPU's HBM): each group of
    consecutive boxes is one EnsembleWindow, built, swept forward and backward, and released
    before the next.  Every member's results equal those of the single ensemble bit for bit (the
    kernels see the same boxes and members, only fewer of them per launch).

    results(m) -> (J_m, w^_0 of member m, dJ/ds of member m) as host copies after run()."""

    def __init__(self, grids, windows, w0, s=None, member_box=None, member_lam=None, obj_kind=OBJ_MEAN_PRESSURE,
                 budget_bytes=None, device="cuda"):
        self.grids, self.windows, self.w0, self.s = list(grids), [int(t) for t in windows], list(w0), s
        nb = len(self.grids)
        self.member_box = list(range(nb)) if member_box is None else [int(b) for b in member_box]
        self.member_lam = [0.0] * len(self.member_box) if member_lam is None else [float(x) for x in member_lam]
        self.obj_kind, self.device = obj_kind, device
        if budget_bytes is None:
            torch.cuda.empty_cache()
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.5 * free)
        self.groups = plan(self.grids, self.windows, self.member_box, budget_bytes)
        self._res = {}

    def run(self):
        for b0, b1, m0, m1 in self.groups:
            win = EnsembleWindow(self.grids[b0:b1], self.windows[b0:b1], self.w0[b0:b1],
                                 None if self.s is None else self.s[b0:b1],
                                 [b - b0 for b in self.member_box[m0:m1]], self.member_lam[m0:m1],
                                 obj_kind=self.obj_kind, device=self.device)
            win.forward()
            wh0, gs = win.backward()
            J = win.J.cpu()
            for k in range(m1 - m0):
                self._res[m0 + k] = (float(J[k]), win.member(wh0, k).cpu().clone(), win.member(gs, k).cpu().clone())
            del win
            torch.cuda.empty_cache()
        return self

    def results(self, m):
        return self._res[m]


class LambdaSweep:
    """Reverse sweeps of one stored window for several artificial-viscosity scales at once (the
    lambda study of the paper, "Stabilizing adjoint equations" and Results, Table 2): one batched
    ensemble of one box and one member per lambda.  Each reverse step reads the stored state once
    (a BF16 record is decoded once), recomputes the box's stage states once inside the batched
    adjoint step, and transposes the stages of every member; the objective gradient is then added
    to each member (any objective kind) and, optionally, each member's adjoint energy recorded.

    g:       the grid of the trajectory (BF16 records or native states, RK4, split flux)
    traj:    a sweep.Trajectory of the window (states 0..T)
    lams:    lambda of each member (length^2 units: nu = lambda sigma_1)
    Every member's w^_0 and dJ/ds equal those of a single-box reverse sweep with its lambda over
    the same trajectory bit for bit (same kernels, same order of operations).
    """

    def __init__(self, g, traj, lams, obj=None, weights=None, s=None, energy=False, device="cuda"):
        from . import CKPT_NATIVE, Grid
        self.g, self.traj = g, traj
        self.records = g.ckpt_format != CKPT_NATIVE
        self.gn = Grid.make(tuple(g.n), tuple(g.L), g.mu, g.dt, g.gamma, g.prandtl, g.bc_x, g.precision, 0,
                            tuple(g.w_ref), tuple(g.nu_weight), g.time_scheme, g.flux, g.roe_delta)
        self.lams = [float(x) for x in lams]
        self.M = len(self.lams)
        self.obj, self.weights, self.s = obj, weights, s
        self.ens = Ensemble([self.gn], [0] * self.M, self.lams, None, device)
        N5 = 5 * g.ncells
        self.ws = self.ens.workspace(device)
        from . import workspace
        self.ws1 = workspace(self.gn, device)
        self.dec = torch.empty(N5, dtype=self.gn.dtype, device=device)
        self.a = torch.zeros(self.M * N5, dtype=self.gn.dtype, device=device)
        self.b = torch.zeros_like(self.a)
        self.grad_s = torch.zeros_like(self.a)
        T = traj.nsteps
        self.E = torch.zeros((T + 1, self.M), dtype=torch.float64, device=device) if energy else None
        self.use_obj = obj is not None and obj.kind != 0 and weights is not None

    def _state(self, n):
        if not self.records:
            return self.traj.slot(n)
        from . import ckpt_decode
        ckpt_decode(self.g, self.traj.slot(n), self.dec)
        return self.dec

    def _inject(self, w, c, dst):
        from . import objective_and_grad
        for m in range(self.M):
            objective_and_grad(self.gn, self.obj, w, self.ws1, weight=c, djdw=self.ens.member_slice(dst, m))

    def backward(self, progress=None):
        """Returns (w^_0, grad_s) member-packed (member m: ens.member_slice(t, m)); self.E holds the
        adjoint energies (index [n, m]) when energy=True.  progress(n) is called every step."""
        T = self.traj.nsteps
        a, b = self.a, self.b
        a.zero_()
        self.grad_s.zero_()
        w = self._state(T)
        if self.use_obj and self.weights[T] != 0.0:
            self._inject(w, float(self.weights[T]), a)
        if self.E is not None:
            self.ens.energy_vhat(self.M, w, a, self.E[T], self.ws)
        for n in range(T - 1, -1, -1):
            w = self._state(n)
            self.ens.adjoint_step(self.M, w, self.s, a, b, self.ws, grad_s=self.grad_s)
            if self.use_obj and self.weights[n] != 0.0:
                self._inject(w, float(self.weights[n]), b)
            a, b = b, a
            if self.E is not None:
                self.ens.energy_vhat(self.M, w, a, self.E[n], self.ws)
            if progress is not None:
                progress(n)
        self.wh0 = a
        return a, self.grad_s

    def member(self, t, m):
        return self.ens.member_slice(t, m)
