"""Window trajectories kept in pinned host memory or in a file, streamed while the kernels run.

The paper writes its primal snapshots to disk and reads them back during the adjoint sweep
("Implementation").  Here the states of a window (native states or BF16 records) that do not fit
in HBM go to pinned host memory, or through pinned staging buffers to a file (an NVMe scratch
file, say): after each primal step the new state is copied device-to-host on a copy stream while
the next step computes, and the reverse sweep fetches w_{n-1} while step n runs.  A small ring of
device slots holds the states in flight; events order every reuse of a slot after the copy or the
kernel that last touched it, and file reads and writes run on worker threads (a record in
page-aligned slices, moved in parallel).  The last states of
the window may stay in HBM (`device_tail`): the reverse sweep consumes them first, while the first
stored states are already on their way.

The kernels and their inputs are those of the HBM sweeps (sweep.forward / sweep.backward), so
the results are identical bit for bit; only where the states wait between the sweeps differs.
Only scheduling and copies happen here.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import torch

from . import (CKPT_NATIVE, OBJ_NONE, adjoint_step, ckpt_bytes, ckpt_decode, ckpt_encode, objective_and_grad,
               workspace)
from .sweep import step_obj, step_weights


class _PinnedStore:
    """Stored states in one pinned host tensor."""

    def __init__(self, n, rec_len, dtype):
        self.host = torch.empty((max(n, 1), rec_len), dtype=dtype, pin_memory=True)

    def put(self, n, src, copy):
        with torch.cuda.stream(copy):
            self.host[n].copy_(src, non_blocking=True)
        return copy.record_event()

    def prefetch(self, n):
        pass

    def get(self, n, dst, copy):
        with torch.cuda.stream(copy):
            dst.copy_(self.host[n], non_blocking=True)
        return copy.record_event()

    def finish(self):
        pass

    def read(self, n):
        return self.host[n]


class _FileStore:
    """Stored states in a file, moved through `nstage` staging buffers (pinned unless pin=False).
    One scheduling thread orders the transfers (a file write after its device-to-host copy has
    landed, a file read ahead of its host-to-device copy); `io_threads` threads move the slices
    of one record with positioned writes and reads, which release the interpreter lock, so a
    record's slices go to and from the page cache (or the drive) in parallel.  Page-aligned
    slices; the file is sized once, so no write extends it."""

    def __init__(self, n, rec_len, dtype, path, nstage=3, io_threads=4, pin=True):
        self.path = path
        self.rec_len, self.dtype = rec_len, dtype
        self.rec_bytes = rec_len * torch.empty(0, dtype=dtype).element_size()
        self.fd = os.open(path, os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o600)
        os.ftruncate(self.fd, max(n, 1) * self.rec_bytes)
        self.stage = [torch.empty(rec_len, dtype=dtype, pin_memory=pin) for _ in range(nstage)]
        self.busy = [None] * nstage     # pending scheduled job on each staging buffer
        self.h2d = [None] * nstage      # host-to-device copy out of each staging buffer
        self.reads = {}
        self.pool = ThreadPoolExecutor(max_workers=1)
        self.io = ThreadPoolExecutor(max_workers=io_threads)
        step = -(-self.rec_bytes // io_threads)
        step = -(-step // 4096) * 4096
        self.slices = [(o, min(step, self.rec_bytes - o)) for o in range(0, self.rec_bytes, step)]

    def _slot(self, n):
        return n % len(self.stage)

    @staticmethod
    def _bytes(t):
        return memoryview(t.numpy()).cast("B")

    def _pwrite(self, view, off):
        while len(view):
            k = os.pwrite(self.fd, view, off)
            view, off = view[k:], off + k

    def _pread(self, view, off):
        while len(view):
            k = os.preadv(self.fd, [view], off)
            if k == 0:
                raise OSError(f"{self.path}: end of file inside a stored record")
            view, off = view[k:], off + k

    def _move(self, fn, t, n):
        """fn (_pwrite or _pread) over every slice of record n and host tensor t, in parallel."""
        view, base = self._bytes(t), n * self.rec_bytes
        for f in [self.io.submit(fn, view[o:o + ln], base + o) for o, ln in self.slices]:
            f.result()

    def _write(self, n, j, ev):
        ev.synchronize()
        self._move(self._pwrite, self.stage[j], n)

    def _read(self, n, j, prior):
        if prior is not None:
            prior.synchronize()
        self._move(self._pread, self.stage[j], n)

    def _claim(self, j):
        if self.busy[j] is not None:
            self.busy[j].result()
            self.busy[j] = None

    def put(self, n, src, copy):
        j = self._slot(n)
        self._claim(j)
        with torch.cuda.stream(copy):
            self.stage[j].copy_(src, non_blocking=True)
        ev = copy.record_event()
        self.busy[j] = self.pool.submit(self._write, n, j, ev)
        return ev

    def prefetch(self, n):
        if n < 0 or n in self.reads:
            return
        j = self._slot(n)
        self._claim(j)
        self.reads[n] = self.busy[j] = self.pool.submit(self._read, n, j, self.h2d[j])

    def get(self, n, dst, copy):
        j = self._slot(n)
        self.prefetch(n)
        self.reads.pop(n).result()
        self.busy[j] = None
        with torch.cuda.stream(copy):
            dst.copy_(self.stage[j], non_blocking=True)
        self.h2d[j] = copy.record_event()
        return self.h2d[j]

    def finish(self):
        for j in range(len(self.stage)):
            self._claim(j)

    def read(self, n):
        out = torch.empty(self.rec_len, dtype=self.dtype)
        self._move(self._pread, out, n)
        return out

    def close(self):
        for j in range(len(self.stage)):
            self._claim(j)
        self.pool.shutdown()
        self.io.shutdown()
        os.close(self.fd)
        if os.path.exists(self.path):
            os.remove(self.path)


class HostTrajectory:
    """States w_0..w_N of one window: the last `device_tail` of them in HBM, the others in pinned
    host memory, or in the file `path` when given (full-precision states, or BF16 records when
    g.ckpt_format says so).  A ring of `slots` device buffers holds the stored states in flight; a
    copy stream of its own (default priority) moves them.  The reverse sweep starts with the states
    kept in HBM and in the ring, so its first fetches overlap computation."""

    def __init__(self, g, nsteps, device="cuda", slots=2, device_tail=0, path=None):
        if slots < 2:
            raise ValueError("at least two device slots")
        self.g, self.nsteps = g, nsteps
        self.records = g.ckpt_format != CKPT_NATIVE
        if self.records:
            self.rec_len, dt = ckpt_bytes(g), torch.uint8
        else:
            self.rec_len, dt = 5 * g.ncells, g.dtype
        self.elem = torch.empty(0, dtype=dt).element_size()
        self.tail = max(0, min(int(device_tail), nsteps + 1))
        self.nhost = nsteps + 1 - self.tail  # states 0 .. nhost-1 live in host memory or the file
        if path:
            self.store = _FileStore(self.nhost, self.rec_len, dt, path)
        else:
            self.store = _PinnedStore(self.nhost, self.rec_len, dt)
        self.dev_tail = [torch.empty(self.rec_len, dtype=dt, device=device) for _ in range(self.tail)]
        self.ring = [torch.empty(self.rec_len, dtype=dt, device=device) for _ in range(slots)]
        self.in_ring = [None] * slots  # stored state that each ring slot holds, as the last sweep left it
        self.copy = torch.cuda.Stream(device=device)
        self.device = device

    @property
    def nbytes(self):
        return self.nhost * self.rec_len * self.elem

    @property
    def host(self):
        """The pinned host tensor of the stored states (pinned-memory trajectories)."""
        return self.store.host

    def stored(self, n):
        """State or record n as stored (a host tensor; complete once the forward sweep's stream
        has finished)."""
        return self.store.read(n) if n < self.nhost else self.dev_tail[n - self.nhost].cpu()

    def buffer(self, n):
        """Device buffer of state n during the forward sweep."""
        return self.dev_tail[n - self.nhost] if n >= self.nhost else self.ring[n % len(self.ring)]

    def close(self):
        if isinstance(self.store, _FileStore):
            self.store.close()


def forward(g, w0, s, nsteps, obj=None, weights=None, ws=None, traj=None, J=None):
    """Primal sweep w_0 -> w_N storing every state (host memory, file or the HBM tail); J (device
    FP64) += sum_n c_n j(w_n).  Same kernels and order as sweep.forward.  Returns (trajectory,
    w_N, J); the stored copies are complete when the caller's stream reaches the end of the sweep
    (and, for a file, when this call returns)."""
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
        traj.copy.wait_event(main.record_event())
        done[k] = traj.store.put(n, traj.ring[k], traj.copy)
        traj.in_ring[k] = n

    use_obj = obj is not None and obj.kind != OBJ_NONE and weights is not None
    cur = w0.clone()
    nxt = torch.empty_like(w0)
    take(0)
    if traj.records:
        ckpt_encode(g, cur, traj.buffer(0), ws)
    else:
        traj.buffer(0).copy_(cur)
    send(0)
    if use_obj and nsteps == 0 and weights[0] != 0.0:
        objective_and_grad(g, obj, cur, ws, weight=float(weights[0]), J_accum=J)
    for n in range(nsteps):
        take(n + 1)
        win, wgt = step_weights(obj if use_obj else None, weights, n, nsteps)
        if traj.records:
            step_obj(g, cur, s, nxt, ws, obj, win, wgt, J, ckpt_out=traj.buffer(n + 1))
        else:
            # the step reads w_n from its buffer and writes w_{n+1} into the next one
            step_obj(g, cur, s, traj.buffer(n + 1), ws, obj, win, wgt, J)
            nxt = traj.buffer(n + 1)
        send(n + 1)
        if traj.records:
            cur, nxt = nxt, cur
        else:
            cur = nxt
    wN = cur.clone()
    for ev in done:
        if ev is not None:
            main.wait_event(ev)
    traj.store.finish()
    return traj, wN, J


def backward(g, traj, s, obj=None, weights=None, lam=0.0, ws=None, grad_s=None):
    """Reverse sweep over a stored trajectory, the next stored state fetched while a step runs.
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
    dec = torch.empty(N5, dtype=g.dtype, device=dev) if traj.records else None
    free = [None] * K   # last kernel reading each ring slot finished
    ready = {}          # stored state n has arrived in its ring slot (None: it was there already)
    held = list(traj.in_ring)

    def fetch(n):
        if n < 0 or n >= traj.nhost:
            return
        k = n % K
        if held[k] == n:  # left in the ring by the last sweep
            ready[n] = None
            return
        held[k] = n
        traj.copy.wait_stream(main) if free[k] is None else traj.copy.wait_event(free[k])
        ready[n] = traj.store.get(n, traj.ring[k], traj.copy)

    def prefetch(n):
        if 0 <= n < traj.nhost and held[n % K] != n:
            traj.store.prefetch(n)

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
        if not traj.records:
            return rec
        ckpt_decode(g, rec, dec)
        return dec

    # the first stored states are on their way while the HBM tail is processed
    top = traj.nhost - 1
    for n in (top, top - 1, top - 2):
        prefetch(n)
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
            prefetch(n - 2)
        c_n = float(weights[n]) if use_obj else 0.0
        adjoint_step(g, w, s, a, b, ws, lam=lam, obj=obj if use_obj else None, c_n=c_n, grad_s=grad_s)
        release(n)
        a, b = b, a
    traj.in_ring = held  # what the ring holds now, for a later sweep over the same trajectory
    return a, grad_s
