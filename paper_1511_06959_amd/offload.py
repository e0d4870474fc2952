"""Window trajectories kept in pinned host memory, streamed over PCIe while the kernels run.

The paper writes its primal snapshots to disk and reads them back during the adjoint sweep
("Implementation").  Here the states of a window (native states or BF16 records) go to pinned
host memory instead of HBM when the window does not fit on the GPU: after each primal step the
new state is copied device-to-host on a copy stream while the next step computes, and the
reverse sweep prefetches w_{n-1} host-to-device while step n runs.  A small ring of device
slots holds the states in flight; events order every reuse of a slot after the copy or the
kernel that last touched it.  The last states of the window may stay in HBM (`device_tail`):
the reverse sweep consumes them first, while the first host states are already on their way.

The kernels and their inputs are those of the HBM sweeps (sweep.forward / sweep.backward), so
the results are identical bit for bit; only where the states wait between the sweeps differs.
Only scheduling and copies happen here.
"""
import torch

from . import (CKPT_BF16, OBJ_NONE, adjoint_step, ckpt_bytes, ckpt_decode, ckpt_encode, objective_and_grad,
               primal_step, workspace)


class HostTrajectory:
    """States w_0..w_N of one window: the last `device_tail` of them in HBM, the others in pinned
    host memory (full-precision states, or BF16 records when g.ckpt_format says so).  A ring of
    `slots` device buffers holds the host states in flight; a copy stream of its own (default
    priority) moves them.  The reverse sweep starts with the states kept in HBM and in the ring,
    so its first host fetches overlap computation."""

    def __init__(self, g, nsteps, device="cuda", slots=2, device_tail=0):
        if slots < 2:
            raise ValueError("at least two device slots")
        self.g, self.nsteps = g, nsteps
        self.bf16 = g.ckpt_format == CKPT_BF16
        if self.bf16:
            self.rec_len, dt = ckpt_bytes(g), torch.uint8
        else:
            self.rec_len, dt = 5 * g.ncells, g.dtype
        self.tail = max(0, min(int(device_tail), nsteps + 1))
        self.nhost = nsteps + 1 - self.tail  # states 0 .. nhost-1 live in host memory
        self.host = torch.empty((max(self.nhost, 1), self.rec_len), dtype=dt, pin_memory=True)
        self.dev_tail = [torch.empty(self.rec_len, dtype=dt, device=device) for _ in range(self.tail)]
        self.ring = [torch.empty(self.rec_len, dtype=dt, device=device) for _ in range(slots)]
        self.in_ring = [None] * slots  # host state that each ring slot holds, as the forward sweep left it
        self.copy = torch.cuda.Stream(device=device)
        self.device = device

    @property
    def nbytes(self):
        return self.nhost * self.rec_len * self.host.element_size()

    def buffer(self, n):
        """Device buffer of state n during the forward sweep."""
        return self.dev_tail[n - self.nhost] if n >= self.nhost else self.ring[n % len(self.ring)]


def forward(g, w0, s, nsteps, obj=None, weights=None, ws=None, traj=None, J=None):
    """Primal sweep w_0 -> w_N storing every state (host memory or the HBM tail); J (device
    FP64) += sum_n c_n j(w_n).  Same kernels and order as sweep.forward.  Returns (trajectory,
    w_N, J); the host copies are complete when the caller's stream reaches the end of the sweep."""
    dev = w0.device
    ws = workspace(g) if ws is None else ws
    traj = HostTrajectory(g, nsteps, dev) if traj is None else traj
    J = torch.zeros(1, dtype=torch.float64, device=dev) if J is None else J
    main = torch.cuda.current_stream(dev)
    K = len(traj.ring)
    done = [None] * K  # copy-out of each ring slot finished
    traj.in_ring = [None] * K

    def take(n):
        if n < traj.nhost and done[n % K] is not None:
            main.wait_event(done[n % K])

    def send(n):
        if n >= traj.nhost:
            return
        k = n % K
        ev = main.record_event()
        traj.copy.wait_event(ev)
        with torch.cuda.stream(traj.copy):
            traj.host[n].copy_(traj.ring[k], non_blocking=True)
        done[k] = traj.copy.record_event()
        traj.in_ring[k] = n

    use_obj = obj is not None and obj.kind != OBJ_NONE and weights is not None
    cur = w0.clone()
    nxt = torch.empty_like(w0)
    take(0)
    if traj.bf16:
        ckpt_encode(g, cur, traj.buffer(0), ws)
    else:
        traj.buffer(0).copy_(cur)
    send(0)
    if use_obj and weights[0] != 0.0:
        objective_and_grad(g, obj, cur, ws, weight=float(weights[0]), J_accum=J)
    for n in range(nsteps):
        take(n + 1)
        if traj.bf16:
            primal_step(g, cur, s, nxt, ws, ckpt_out=traj.buffer(n + 1))
        else:
            # the step reads w_n from its buffer and writes w_{n+1} into the next one
            primal_step(g, cur, s, traj.buffer(n + 1), ws)
            nxt = traj.buffer(n + 1)
        if use_obj and weights[n + 1] != 0.0:
            objective_and_grad(g, obj, nxt, ws, weight=float(weights[n + 1]), J_accum=J)
        send(n + 1)
        if traj.bf16:
            cur, nxt = nxt, cur
        else:
            cur = nxt
    wN = cur.clone()
    for ev in done:
        if ev is not None:
            main.wait_event(ev)
    return traj, wN, J


def backward(g, traj, s, obj=None, weights=None, lam=0.0, ws=None, grad_s=None):
    """Reverse sweep over a host trajectory, the next host state fetched while a step runs.
    Same kernels and order as sweep.backward.  Returns (w^_0, grad_s)."""
    dev = traj.ring[0].device
    ws = workspace(g) if ws is None else ws
    N = traj.nsteps
    N5 = 5 * g.ncells
    main = torch.cuda.current_stream(dev)
    K = len(traj.ring)
    a = torch.zeros(N5, dtype=g.dtype, device=dev)
    b = torch.empty_like(a)
    grad_s = torch.zeros(N5, dtype=g.dtype, device=dev) if grad_s is None else grad_s
    use_obj = obj is not None and obj.kind != OBJ_NONE and weights is not None
    dec = torch.empty(N5, dtype=g.dtype, device=dev) if traj.bf16 else None
    free = [None] * K   # last kernel reading each ring slot finished
    ready = {}          # host state n has arrived in its ring slot (None: it was there already)
    held = list(traj.in_ring)

    def fetch(n):
        if n < 0 or n >= traj.nhost:
            return
        k = n % K
        if held[k] == n:  # left in the ring by the forward sweep
            ready[n] = None
            return
        held[k] = n
        traj.copy.wait_stream(main) if free[k] is None else traj.copy.wait_event(free[k])
        with torch.cuda.stream(traj.copy):
            traj.ring[k].copy_(traj.host[n], non_blocking=True)
        ready[n] = traj.copy.record_event()

    def state(n):
        if n >= traj.nhost:
            return traj.dev_tail[n - traj.nhost]
        ev = ready.pop(n)
        if ev is not None:
            main.wait_event(ev)
        return traj.ring[n % K]

    def release(n):
        if n < traj.nhost:
            free[n % K] = main.record_event()

    def full(rec):
        if not traj.bf16:
            return rec
        ckpt_decode(g, rec, dec)
        return dec

    # the first host states are on their way while the HBM tail is processed
    top = traj.nhost - 1
    fetch(top)
    if top == N:
        fetch(N - 1)
    wN = state(N)
    if use_obj and weights[N] != 0.0:
        objective_and_grad(g, obj, full(wN), ws, weight=float(weights[N]), djdw=a)
    release(N)
    for n in range(N - 1, -1, -1):
        w = state(n)
        if n <= top:
            fetch(n - 1)
        c_n = float(weights[n]) if use_obj else 0.0
        adjoint_step(g, w, s, a, b, ws, lam=lam, obj=obj if use_obj else None, c_n=c_n, grad_s=grad_s)
        release(n)
        a, b = b, a
    traj.in_ring = held  # what the ring holds now, for a later sweep over the same trajectory
    return a, grad_s
