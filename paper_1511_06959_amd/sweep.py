"""Window schedules around the C ABI: forward sweep storing the trajectory in HBM, reverse sweep.

The paper stores periodic primal snapshots and recomputes in between ("Implementation",
checkpointing).  With 288 GB of HBM the whole trajectory of a moderate window fits, so the plain
schedule keeps every state (natively or as 16-bit records) on the device and the reverse sweep
recomputes only the three inner RK4 stage states of each step, inside ``adjoint_step``
(``Trajectory``, ``forward``, ``backward``).  Longer windows keep snapshots: ``SegmentSweep``
every seg steps, re-advancing one segment at a time with its stage states kept, and
``RevolveSweep`` in a fixed number of slots with the binomial schedule of ``revolve.py``;
``plan_window`` picks between them for a byte budget.

Only scheduling happens here; all arithmetic runs in the library's kernels.
"""
import torch

from . import (CKPT_NATIVE, OBJ_KE_DISSIPATION, OBJ_NONE, Grid, Objective, adjoint_step, adjoint_step_stages, ckpt_bytes, energy_vhat,
               objective_and_grad, primal_step, primal_step_obj, primal_step_stages, workspace)


def step_weights(obj, weights, n, nsteps):
    """(weight_in, weight) of step n (w_n -> w_{n+1}) such that the steps of an nsteps window
    together add J = sum_m c_m j(w_m): the dissipation, which the library evaluates inside a
    step's first stage for the step's own state, is taken as each step's input (and the last
    state as the last step's output); every other objective as each step's output (and w_0 as the
    first step's input).  (0, 0) without an objective."""
    if obj is None or obj.kind == OBJ_NONE or weights is None:
        return 0.0, 0.0
    if obj.kind == OBJ_KE_DISSIPATION:
        return float(weights[n]), (float(weights[nsteps]) if n == nsteps - 1 else 0.0)
    return (float(weights[0]) if n == 0 else 0.0), float(weights[n + 1])


def step_obj(g, w, s, out, ws, obj, weight_in, weight, J, ckpt_out=None, stages_out=None):
    """One primal step w -> out that adds weight_in * j(w) + weight * j(out) to J when an objective
    and a non-zero weight are given (the library fuses what it can into the step's stages), else a
    plain step."""
    if obj is not None and obj.kind != OBJ_NONE and (weight != 0.0 or weight_in != 0.0) and J is not None:
        primal_step_obj(g, w, s, out, ws, obj, weight, J, ckpt_out=ckpt_out, stages_out=stages_out,
                        weight_in=weight_in)
    elif stages_out is not None:
        primal_step_stages(g, w, s, out, stages_out, ws)
    else:
        primal_step(g, w, s, out, ws, ckpt_out=ckpt_out)


class Trajectory:
    """States w_0..w_N of one window, kept in HBM as full-precision states or 16-bit records;
    with ``stages=True`` also the RK4 stage states W2, W3, W4 of every step (native states),
    so that the reverse sweep needs no recomputation (4x the memory of the states)."""

    def __init__(self, g, nsteps, device="cuda", stages=False):
        self.g = g
        self.nsteps = nsteps
        N5 = 5 * g.ncells
        if g.ckpt_format != CKPT_NATIVE:
            if stages:
                raise ValueError("stage states are stored natively, not as 16-bit records")
            self.rec_bytes = ckpt_bytes(g)
            self.store = torch.empty((nsteps + 1, self.rec_bytes), dtype=torch.uint8, device=device)
        else:
            self.store = torch.empty((nsteps + 1, N5), dtype=g.dtype, device=device)
        self.stages = torch.empty((nsteps, 3 * N5), dtype=g.dtype, device=device) if stages else None

    def slot(self, n):
        return self.store[n]

    def stage_slot(self, n):
        return self.stages[n]


def forward(g, w0, s, nsteps, obj=None, weights=None, ws=None, traj=None, J=None):
    """Primal sweep w_0 -> w_N storing every state; J (device FP64 scalar) += sum_n c_n j(w_n).

    With BF16 storage the sweep itself still advances in FP32; only the stored copies are
    encoded (the adjoint then runs on the decoded states).  Returns (trajectory, w_N, J)."""
    ws = workspace(g) if ws is None else ws
    traj = Trajectory(g, nsteps, w0.device) if traj is None else traj
    J = torch.zeros(1, dtype=torch.float64, device=w0.device) if J is None else J
    records = g.ckpt_format != CKPT_NATIVE
    cur = w0.clone()
    nxt = torch.empty_like(w0)
    if records:
        from . import ckpt_encode
        ckpt_encode(g, cur, traj.slot(0), ws)
    else:
        traj.slot(0).copy_(cur)
    use_obj = obj is not None and obj.kind != OBJ_NONE and weights is not None
    if use_obj and nsteps == 0 and weights[0] != 0.0:
        objective_and_grad(g, obj, cur, ws, weight=float(weights[0]), J_accum=J)
    for n in range(nsteps):
        win, wgt = step_weights(obj if use_obj else None, weights, n, nsteps)
        if records:
            step_obj(g, cur, s, nxt, ws, obj, win, wgt, J, ckpt_out=traj.slot(n + 1))
        else:
            step_obj(g, cur, s, traj.slot(n + 1), ws, obj, win, wgt, J,
                     stages_out=traj.stage_slot(n) if traj.stages is not None else None)
            nxt = traj.slot(n + 1)
        if records:
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
    records = g.ckpt_format != CKPT_NATIVE
    dec = None
    if records or energy:
        dec = torch.empty(N5, dtype=g.dtype, device=dev)

    def state(n):
        if not records:
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
        if traj.stages is not None:
            adjoint_step_stages(g, traj.slot(n), traj.stage_slot(n), s, a, b, ws, lam=lam,
                                obj=obj if use_obj else None, c_n=c_n, grad_s=grad_s)
        else:
            adjoint_step(g, traj.slot(n), s, a, b, ws, lam=lam, obj=obj if use_obj else None, c_n=c_n, grad_s=grad_s)
        a, b = b, a
        if energy:
            energy_vhat(g, state(n), a, E[n:n + 1], ws)
    return a, grad_s, E


class CapturedWindow:
    """A whole window captured once as two HIP graphs (forward sweep, reverse sweep) and replayed.

    Every buffer the sweeps touch is allocated up front, so a replay launches the recorded
    kernels only (no host work per step).  Buffers are reused across replays: ``run`` returns
    views that the next replay overwrites.  Profiling must be off while capturing.
    """

    def __init__(self, g, w0, s, nsteps, obj=None, weights=None, lam=0.0, ws=None, stages=False):
        dev = w0.device
        self.g, self.nsteps, self.obj, self.weights, self.lam = g, nsteps, obj, weights, lam
        self.ws = workspace(g) if ws is None else ws
        self.w0 = w0.clone()
        self.s = None if s is None else s.clone()
        self.traj = Trajectory(g, nsteps, dev, stages=stages)
        self.J = torch.zeros(1, dtype=torch.float64, device=dev)
        self.grad_s = torch.zeros(5 * g.ncells, dtype=g.dtype, device=dev)
        self.wh0 = torch.zeros(5 * g.ncells, dtype=g.dtype, device=dev)
        self._fwd = torch.cuda.CUDAGraph()
        self._bwd = torch.cuda.CUDAGraph()
        # one eager pass settles torch's allocator state for the buffers used inside the sweeps
        self._forward()
        self._backward()
        torch.cuda.synchronize()
        with torch.cuda.graph(self._fwd):
            self._forward()
        with torch.cuda.graph(self._bwd):
            self._backward()
        torch.cuda.synchronize()

    def _forward(self):
        self.J.zero_()
        forward(self.g, self.w0, self.s, self.nsteps, self.obj, self.weights, self.ws, traj=self.traj, J=self.J)

    def _backward(self):
        self.grad_s.zero_()
        wh0, _, _ = backward(self.g, self.traj, self.s, self.obj, self.weights, self.lam, self.ws, grad_s=self.grad_s)
        self.wh0.copy_(wh0)

    def run_forward(self):
        self._fwd.replay()

    def run_backward(self):
        self._bwd.replay()

    def run(self):
        """Replay both sweeps; returns (J, dJ/dw_0, dJ/ds) device tensors owned by this object."""
        self._fwd.replay()
        self._bwd.replay()
        return self.J, self.wh0, self.grad_s


class RevolveSweep:
    """Forward and reverse sweep with a fixed number of snapshot slots (binomial checkpointing).

    ``forward(w0)`` runs the primal once over the window, accumulating J on every state and
    storing the snapshots the reverse schedule starts from; ``backward(scale)`` replays the rest
    of the schedule: recomputation from snapshots and reverse steps, with objective weights
    multiplied by ``scale``.  With ``g.ckpt_format != CKPT_NATIVE`` the slots hold 16-bit records
    (BF16 or fixed-point codes); the working state is always full precision.  Slots = nsteps + 1
    reproduces the store-all sweep.
    """

    def __init__(self, g, nsteps, slots, s=None, obj=None, weights=None, lam=0.0, ws=None, device="cuda"):
        from . import revolve
        self.g = g
        self.records = g.ckpt_format != CKPT_NATIVE
        self.gn = Grid.make(tuple(g.n), tuple(g.L), g.mu, g.dt, g.gamma, g.prandtl, g.bc_x, g.precision, 0,
                            tuple(g.w_ref), tuple(g.nu_weight), g.time_scheme, g.flux, g.roe_delta,
                            (tuple(g.w_far[0:5]), tuple(g.w_far[5:10])))
        self.nsteps, self.slots = nsteps, int(slots)
        self.s, self.obj, self.weights, self.lam = s, obj, weights, lam
        self.ws = workspace(g, device) if ws is None else ws
        self.acts = revolve.schedule(nsteps, self.slots)
        self.first_rev = next(i for i, a in enumerate(self.acts) if a[0] == "reverse")
        N5 = 5 * g.ncells
        if self.records:
            self.pool = torch.empty((self.slots, ckpt_bytes(g)), dtype=torch.uint8, device=device)
        else:
            self.pool = torch.empty((self.slots, N5), dtype=g.dtype, device=device)
        self.free = list(range(self.slots))
        self.where = {}
        self.cur = torch.empty(N5, dtype=g.dtype, device=device)
        self.tmp = torch.empty(N5, dtype=g.dtype, device=device)
        self.wN = torch.empty(N5, dtype=g.dtype, device=device)
        self.cur_step = None
        self.advanced = 0
        self.use_obj = obj is not None and obj.kind != OBJ_NONE and weights is not None

    # -- slot handling ----------------------------------------------------------------------
    def _store(self, n, state):
        k = self.free.pop()
        self.where[n] = k
        if self.records:
            from . import ckpt_encode
            ckpt_encode(self.g, state, self.pool[k], self.ws)
        else:
            self.pool[k].copy_(state)

    def _load(self, n):
        """Working state := stored state n."""
        k = self.where[n]
        if self.records:
            from . import ckpt_decode
            ckpt_decode(self.g, self.pool[k], self.cur)
        else:
            self.cur.copy_(self.pool[k])
        self.cur_step = n

    def _advance(self, i, j, J=None):
        if self.cur_step != i:
            self._load(i)
        for n in range(i, j):
            win, wgt = step_weights(self.obj if (J is not None and self.use_obj) else None, self.weights, n,
                                    self.nsteps)
            step_obj(self.gn, self.cur, self.s, self.tmp, self.ws, self.obj, win, wgt, J)
            self.cur, self.tmp = self.tmp, self.cur
            self.advanced += 1
        self.cur_step = j

    # -- sweeps ------------------------------------------------------------------------------
    def forward(self, w0, J=None):
        dev = w0.device
        J = torch.zeros(1, dtype=torch.float64, device=dev) if J is None else J
        self.free = list(range(self.slots))
        self.where = {}
        self.cur.copy_(w0)
        self.cur_step = 0
        self.advanced = 0
        self._store(0, self.cur)
        for act in self.acts[:self.first_rev]:
            if act[0] == "advance":
                self._advance(act[1], act[2], J)
            elif act[0] == "store":
                self._store(act[1], self.cur)
            else:
                raise AssertionError(act)
        # the working state is w_{N-1}; the final state w_N feeds J and the terminal adjoint
        if self.cur_step != self.nsteps - 1:
            self._advance(self.cur_step, self.nsteps - 1, J)
        win, wgt = step_weights(self.obj if self.use_obj else None, self.weights, self.nsteps - 1, self.nsteps)
        step_obj(self.gn, self.cur, self.s, self.wN, self.ws, self.obj, win, wgt, J)
        self.advanced += 1
        return J

    def backward(self, scale=1.0, grad_s=None, progress=None):
        """Replays the reverse part of the schedule.  progress(n) is called after every reverse
        step.  Returns (w^_0, grad_s)."""
        g, dev = self.g, self.cur.device
        N5 = 5 * g.ncells
        a = torch.zeros(N5, dtype=g.dtype, device=dev)
        b = torch.empty_like(a)
        grad_s = torch.zeros(N5, dtype=g.dtype, device=dev) if grad_s is None else grad_s
        if self.use_obj and self.weights[self.nsteps] != 0.0:
            objective_and_grad(self.gn, self.obj, self.wN, self.ws, weight=scale * float(self.weights[self.nsteps]),
                               djdw=a)
        for act in self.acts[self.first_rev:]:
            kind = act[0]
            if kind == "advance":
                self._advance(act[1], act[2])
            elif kind == "store":
                self._store(act[1], self.cur)
            elif kind == "free":
                self.free.append(self.where.pop(act[1]))
            else:
                n = act[1]
                c_n = scale * float(self.weights[n]) if self.use_obj else 0.0
                o = self.obj if self.use_obj else None
                if self.cur_step == n:
                    adjoint_step(self.gn, self.cur, self.s, a, b, self.ws, lam=self.lam, obj=o, c_n=c_n, grad_s=grad_s)
                else:
                    gg = self.g if self.records else self.gn
                    adjoint_step(gg, self.pool[self.where[n]], self.s, a, b, self.ws, lam=self.lam, obj=o, c_n=c_n,
                                 grad_s=grad_s)
                a, b = b, a
                if progress is not None:
                    progress(n)
        return a, grad_s


class SegmentSweep:
    """Two-level checkpointing: the forward sweep keeps a snapshot (a 16-bit record when
    ``g.ckpt_format != CKPT_NATIVE``, else a native state) every ``seg`` steps; the reverse sweep
    re-advances one segment at a time from its snapshot, keeping every state of the segment and the
    stage states of each of its steps in HBM (``primal_step_stages``), and then reverses the
    segment with ``adjoint_step_stages``, so that no reverse step recomputes a stage state.

    Per time step this costs one primal step in the forward sweep and one in the re-advance, against
    the binomial schedule's (1 + recomputation) primal steps plus three stage evaluations inside
    every reverse step; it needs ``nsnap`` snapshots plus one segment of states and stage states
    (see ``segment_bytes``).  The paper keeps periodic snapshots and recomputes between them
    ("Implementation", checkpointing); the working state is always full precision.
    """

    def __init__(self, g, nsteps, seg, s=None, obj=None, weights=None, lam=0.0, ws=None, device="cuda"):
        self.g = g
        self.records = g.ckpt_format != CKPT_NATIVE
        self.gn = Grid.make(tuple(g.n), tuple(g.L), g.mu, g.dt, g.gamma, g.prandtl, g.bc_x, g.precision, 0,
                            tuple(g.w_ref), tuple(g.nu_weight), g.time_scheme, g.flux, g.roe_delta,
                            (tuple(g.w_far[0:5]), tuple(g.w_far[5:10])))
        self.nsteps, self.seg = int(nsteps), max(1, min(int(seg), int(nsteps)))
        self.nsnap = -(-self.nsteps // self.seg)
        self.s, self.obj, self.weights, self.lam = s, obj, weights, lam
        self.ws = workspace(g, device) if ws is None else ws
        N5 = 5 * g.ncells
        if self.records:
            self.snaps = torch.empty((self.nsnap, ckpt_bytes(g)), dtype=torch.uint8, device=device)
        else:
            self.snaps = torch.empty((self.nsnap, N5), dtype=g.dtype, device=device)
        self.states = torch.empty((self.seg + 1, N5), dtype=g.dtype, device=device)
        self.stages = torch.empty((self.seg, 3 * N5), dtype=g.dtype, device=device)
        self.wN = torch.empty(N5, dtype=g.dtype, device=device)
        self.advanced = 0
        self.use_obj = obj is not None and obj.kind != OBJ_NONE and weights is not None

    def _store(self, k, state):
        if self.records:
            from . import ckpt_encode
            ckpt_encode(self.g, state, self.snaps[k], self.ws)
        else:
            self.snaps[k].copy_(state)

    def _load(self, k, dst):
        if self.records:
            from . import ckpt_decode
            ckpt_decode(self.g, self.snaps[k], dst)
        else:
            dst.copy_(self.snaps[k])

    def forward(self, w0, J=None):
        """Primal sweep keeping the snapshots; J (device FP64) += sum_n c_n j(w_n).  Returns J."""
        dev = w0.device
        J = torch.zeros(1, dtype=torch.float64, device=dev) if J is None else J
        cur, nxt = self.states[0], self.states[1]
        cur.copy_(w0)
        self.advanced = 0
        self._store(0, cur)
        for n in range(self.nsteps):
            out = self.wN if n + 1 == self.nsteps else nxt
            win, wgt = step_weights(self.obj if self.use_obj else None, self.weights, n, self.nsteps)
            step_obj(self.gn, cur, self.s, out, self.ws, self.obj, win, wgt, J)
            self.advanced += 1
            if (n + 1) % self.seg == 0 and n + 1 < self.nsteps:
                self._store((n + 1) // self.seg, out)
            cur, nxt = out, cur
        return J

    def backward(self, scale=1.0, grad_s=None, energy_every=0, progress=None):
        """Reverse sweep, segment by segment.  Returns (w^_0, grad_s).  energy_every > 0: the
        adjoint energy after every energy_every-th reverse step (and the terminal one) is kept in
        self.energy, a list of (step, device FP64 scalar).  progress(n) is called after every
        reverse step."""
        g, dev = self.g, self.states.device
        self.energy = []
        N5 = 5 * g.ncells
        a = torch.zeros(N5, dtype=g.dtype, device=dev)
        b = torch.empty_like(a)
        grad_s = torch.zeros(N5, dtype=g.dtype, device=dev) if grad_s is None else grad_s
        if self.use_obj and self.weights[self.nsteps] != 0.0:
            objective_and_grad(self.gn, self.obj, self.wN, self.ws, weight=scale * float(self.weights[self.nsteps]),
                               djdw=a)
        o = self.obj if self.use_obj else None
        if energy_every > 0:
            E = torch.zeros(1, dtype=torch.float64, device=dev)
            energy_vhat(self.gn, self.wN, a, E, self.ws)
            self.energy.append((self.nsteps, E))
        for k in range(self.nsnap - 1, -1, -1):
            first, last = k * self.seg, min(self.nsteps, (k + 1) * self.seg)
            L = last - first
            self._load(k, self.states[0])
            for i in range(L):
                # the state after the segment's last step is the next segment's start, already reversed
                primal_step_stages(self.gn, self.states[i], self.s, self.states[i + 1], self.stages[i], self.ws)
                self.advanced += 1
            for n in range(last - 1, first - 1, -1):
                c_n = scale * float(self.weights[n]) if self.use_obj else 0.0
                adjoint_step_stages(self.gn, self.states[n - first], self.stages[n - first], self.s, a, b, self.ws,
                                    lam=self.lam, obj=o, c_n=c_n, grad_s=grad_s)
                a, b = b, a
                if energy_every > 0 and (n % energy_every == 0):
                    E = torch.zeros(1, dtype=torch.float64, device=dev)
                    energy_vhat(self.gn, self.states[n - first], a, E, self.ws)
                    self.energy.append((n, E))
                if progress is not None:
                    progress(n)
        return a, grad_s


def segment_bytes(g, nsteps, seg):
    """HBM of a SegmentSweep: the snapshots plus one segment of states and stage states."""
    N5 = 5 * g.ncells
    esz = 8 if g.precision == 0 else 4
    return -(-nsteps // seg) * snapshot_bytes(g) + (seg + 1) * N5 * esz + seg * 3 * N5 * esz


def snapshot_bytes(g):
    """Bytes of one snapshot: a BF16 record or a native state."""
    return ckpt_bytes(g) if g.ckpt_format != CKPT_NATIVE else 5 * g.ncells * (8 if g.precision == 0 else 4)


def segment_length(g, nsteps):
    """Segment length of least HBM for a SegmentSweep of nsteps steps."""
    return min(range(1, nsteps + 1), key=lambda L: segment_bytes(g, nsteps, L))


def binomial_slots(g, nsteps, budget_bytes):
    """Snapshot slots of a RevolveSweep that fit budget_bytes (revolve.slots_for_budget)."""
    from . import revolve
    return revolve.slots_for_budget(snapshot_bytes(g), budget_bytes, nsteps)


def plan_window(g, nsteps, budget_bytes):
    """Checkpointing plan of an nsteps window within budget_bytes of HBM: ("segments", seg) with
    the segment length of least memory when that two-level plan fits, else ("binomial", slots)
    with the snapshot slots that fit."""
    best = segment_length(g, nsteps)
    if segment_bytes(g, nsteps, best) <= budget_bytes:
        return "segments", best
    return "binomial", binomial_slots(g, nsteps, budget_bytes)
