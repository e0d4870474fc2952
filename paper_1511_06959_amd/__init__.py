"""MI355X (gfx950) stabilised discrete unsteady adjoint of compressible Navier-Stokes.

Thin ctypes binding over ``libadjns.so`` (the C ABI of ``include/adjns.h``).  Every function
here only marshals arguments: tensors are passed as device pointers, the stream is torch's
current HIP stream, and all arithmetic runs in the library's kernels.  There is no fallback:
if the library is missing or cannot be loaded, every call raises.

Functions keep the names of the C entry points without the ``adj_`` prefix:
``primal_step``, ``adjoint_step``, ``growth_sigma1``, ``objective_and_grad``, ``energy_vhat``,
``dot``, ``ckpt_encode``, ``ckpt_decode``, ``residual``, ``vjp``, ``workspace_bytes``,
``ckpt_bytes``.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadjns.so")

F64, F32 = 0, 1
CKPT_NATIVE, CKPT_BF16, CKPT_I16 = 0, 1, 2  # CKPT_BF16 and CKPT_I16 keep 16-bit records
BC_PERIODIC, BC_SLIP_WALLS, BC_CHARACTERISTIC = 0, 1, 2
RK4, SSPRK3 = 0, 1
FLUX_SPLIT, FLUX_ROE = 0, 1
OBJ_NONE, OBJ_MEAN_PRESSURE, OBJ_KE_DISSIPATION, OBJ_PT_LOSS_PLANE = 0, 1, 2, 3
(PROF_ADJOINT_STAGE, PROF_PRIMAL_STAGE, PROF_SIGMA1, PROF_OBJECTIVE, PROF_CODEC, PROF_REDUCE, PROF_ROE_PRIMAL,
 PROF_ROE_ADJOINT, PROF_BOUNDARY) = range(9)
TILES = {0: (16, 4, 4), 1: (32, 4, 2), 2: (32, 4, 4), 3: (32, 8, 2), 4: (32, 8, 4), 5: (16, 8, 8)}
TILE_16x4x4, TILE_32x4x2, TILE_32x4x4, TILE_32x8x2, TILE_32x8x4, TILE_16x8x8 = range(6)

STATUS = {0: "ADJ_OK", -1: "ADJ_EINVAL", -2: "ADJ_ESHAPE", -3: "ADJ_EUNSTABLE", -4: "ADJ_ENONFINITE",
          -5: "ADJ_EHIP", -6: "ADJ_EWORKSPACE"}


class AdjError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    """Mirror of ``adj_grid``."""
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("bc_x", ctypes.c_int32),
        ("L", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("ckpt_format", ctypes.c_int32),
        ("w_ref", ctypes.c_double * 5),
        ("nu_weight", ctypes.c_double * 3),
        ("time_scheme", ctypes.c_int32),
        ("flux", ctypes.c_int32),
        ("roe_delta", ctypes.c_double),
        ("w_far", ctypes.c_double * 10),
    ]

    @classmethod
    def make(cls, n, L, mu, dt, gamma=1.4, prandtl=0.72, bc_x=0, precision=F64, ckpt_format=CKPT_NATIVE,
             w_ref=None, nu_weight=None, time_scheme=0, flux=FLUX_SPLIT, roe_delta=0.1, w_far=None):
        """w_ref: five reference values; state arrays then hold w - w_ref (see to_stored).
        nu_weight: artificial-viscosity weights of the groups (rho, rho u, rho E), the adjoint
        components of group g diffused with nu_g = lambda nu_weight[g] sigma_1 (None: 1, 1, 1).
        time_scheme: RK4 (classical) or SSPRK3 (strong-stability-preserving third order).
        flux: FLUX_SPLIT (split central form) or FLUX_ROE (Roe's flux on linearly reconstructed
        face states, wave speeds smoothed within roe_delta times the Roe sound speed).
        w_far: with bc_x = BC_CHARACTERISTIC, the far-field conservative states beyond x = 0 and
        beyond x = L_x (two sequences of five values)."""
        g = cls()
        for d in range(3):
            g.n[d] = int(n[d])
            g.L[d] = float(L[d])
        g.bc_x = int(bc_x)
        g.gamma, g.prandtl, g.mu, g.dt = float(gamma), float(prandtl), float(mu), float(dt)
        g.precision, g.ckpt_format = int(precision), int(ckpt_format)
        for v in range(5):
            g.w_ref[v] = 0.0 if w_ref is None else float(w_ref[v])
        for k in range(3):
            g.nu_weight[k] = 1.0 if nu_weight is None else float(nu_weight[k])
        g.time_scheme = int(time_scheme)
        g.flux = int(flux)
        g.roe_delta = float(roe_delta)
        if w_far is not None:
            far = [float(x) for pair in w_far for x in pair]
            for i in range(10):
                g.w_far[i] = far[i]
        return g

    def to_stored(self, w):
        """A full state (numpy or torch, (rho, rho u, rho E)) as the library stores it for this
        grid: w - w_ref field by field, in the input's precision (form it in FP64, then cast)."""
        w = w.clone() if hasattr(w, "clone") else w.copy()
        for v in range(5):
            w.reshape(5, -1)[v] -= self.w_ref[v]
        return w

    def from_stored(self, w):
        w = w.clone() if hasattr(w, "clone") else w.copy()
        for v in range(5):
            w.reshape(5, -1)[v] += self.w_ref[v]
        return w

    @property
    def ncells(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def dtype(self):
        return torch.float64 if self.precision == F64 else torch.float32


def reference_state(w):
    """Field means of a full state: a w_ref for Grid.make that keeps the stored deviations small."""
    import numpy as np
    a = np.asarray(w.detach().cpu() if hasattr(w, "detach") else w, dtype=np.float64).reshape(5, -1)
    return tuple(float(x) for x in a.mean(axis=1))


class Objective(ctypes.Structure):
    """Mirror of ``adj_objective``."""
    _fields_ = [("kind", ctypes.c_int32), ("plane_i", ctypes.c_int32), ("pt_ref", ctypes.c_double)]

    @classmethod
    def make(cls, kind, plane_i=0, pt_ref=0.0):
        o = cls()
        o.kind, o.plane_i, o.pt_ref = int(kind), int(plane_i), float(pt_ref)
        return o


_lib = None
EXPORTS = ("adj_workspace_bytes", "adj_ckpt_bytes", "adj_primal_step", "adj_primal_step_obj", "adj_adjoint_step",
           "adj_adjoint_step_noalloc",
           "adj_primal_step_stages",
           "adj_adjoint_step_stages", "adj_growth_sigma1",
           "adj_objective_and_grad", "adj_energy_vhat", "adj_dot", "adj_ckpt_encode", "adj_ckpt_decode",
           "adj_residual", "adj_vjp", "adj_profile_enable", "adj_profile_read", "adj_set_tile", "adj_get_tile",
           "adj_tile_launched", "adj_stability", "adj_check_stable", "adj_check_status", "adj_batch_table_bytes", "adj_batch_create", "adj_batch_destroy", "adj_batch_offset",
           "adj_batch_workspace_bytes", "adj_batch_primal_step", "adj_batch_adjoint_step",
           "adj_batch_objective_and_grad", "adj_batch_energy_vhat",
           "adj_last_error", "adj_version")


def lib():
    """Load libadjns.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1511_06959_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, gp, op = ctypes.c_void_p, ctypes.POINTER(Grid), ctypes.POINTER(Objective)
    sz, dbl = ctypes.c_size_t, ctypes.c_double
    sig = {
        "adj_workspace_bytes": ([gp], sz),
        "adj_ckpt_bytes": ([gp], sz),
        "adj_primal_step": ([gp, vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_primal_step_obj": ([gp, vp, vp, vp, vp, vp, op, dbl, dbl, vp, vp, sz, vp], ctypes.c_int),
        "adj_adjoint_step": ([gp, vp, vp, vp, dbl, op, dbl, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_adjoint_step_noalloc": ([gp, vp, vp, vp, dbl, op, dbl, vp, vp, vp], ctypes.c_int),
        "adj_primal_step_stages": ([gp, vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_adjoint_step_stages": ([gp, vp, vp, vp, vp, dbl, op, dbl, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_growth_sigma1": ([gp, vp, dbl, vp, vp], ctypes.c_int),
        "adj_objective_and_grad": ([gp, op, vp, dbl, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_energy_vhat": ([gp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_dot": ([gp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_ckpt_encode": ([gp, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_ckpt_decode": ([gp, vp, vp, vp], ctypes.c_int),
        "adj_residual": ([gp, vp, vp, vp, vp], ctypes.c_int),
        "adj_vjp": ([gp, vp, vp, vp, vp, vp], ctypes.c_int),
        "adj_profile_enable": ([ctypes.c_int], ctypes.c_int),
        "adj_profile_read": ([ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)],
                             ctypes.c_int),
        "adj_set_tile": ([ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "adj_get_tile": ([ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "adj_tile_launched": ([ctypes.c_int] * 5, ctypes.c_int),
        "adj_stability": ([gp, vp, dbl, vp, vp, sz, vp], ctypes.c_int),
        "adj_check_stable": ([gp, vp, dbl, ctypes.POINTER(dbl), vp, sz, vp], ctypes.c_int),
        "adj_check_status": ([vp], ctypes.c_int),
        "adj_batch_table_bytes": ([ctypes.c_int, ctypes.c_int, ctypes.c_int], sz),
        "adj_batch_create": ([ctypes.POINTER(vp), ctypes.c_int, gp, op, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(dbl), vp, sz], ctypes.c_int),
        "adj_batch_destroy": ([vp], None),
        "adj_batch_offset": ([vp, ctypes.c_int, ctypes.c_int], ctypes.c_longlong),
        "adj_batch_workspace_bytes": ([vp], sz),
        "adj_batch_primal_step": ([vp, ctypes.c_int, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_batch_adjoint_step": ([vp, ctypes.c_int, vp, vp, vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_batch_objective_and_grad": ([vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_batch_energy_vhat": ([vp, ctypes.c_int, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "adj_last_error": ([], ctypes.c_char_p),
        "adj_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise AdjError(rc, lib().adj_last_error().decode())


def _ptr(t, dtype=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _state(g, t):
    p = _ptr(t, g.dtype)
    if t is not None and t.numel() != 5 * g.ncells:
        raise ValueError(f"state tensors hold 5*N = {5 * g.ncells} values, got {t.numel()}")
    return p


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def version():
    return lib().adj_version().decode()


def workspace_bytes(g):
    n = lib().adj_workspace_bytes(ctypes.byref(g))
    if n == 0:
        raise AdjError(-1, lib().adj_last_error().decode())
    return n


def ckpt_bytes(g):
    return lib().adj_ckpt_bytes(ctypes.byref(g))


def workspace(g, device="cuda"):
    """A workspace tensor (uint8) of adj_workspace_bytes(g) bytes."""
    return torch.empty(workspace_bytes(g), dtype=torch.uint8, device=device)


def _ws(ws):
    return _ptr(ws, torch.uint8), ctypes.c_size_t(ws.numel())


def primal_step(g, w_n, s, w_np1, ws, ckpt_out=None):
    wp, wb = _ws(ws)
    _check(lib().adj_primal_step(ctypes.byref(g), _state(g, w_n), _state(g, s), _state(g, w_np1),
                                 _ptr(ckpt_out, torch.uint8), wp, wb, _stream()))


def primal_step_obj(g, w_n, s, w_np1, ws, obj, weight, J_accum, ckpt_out=None, stages_out=None, weight_in=0.0):
    """primal_step (primal_step_stages with stages_out) that also adds weight_in * j(w_n) +
    weight * j(w_np1) to J_accum."""
    wp, wb = _ws(ws)
    _check(lib().adj_primal_step_obj(ctypes.byref(g), _state(g, w_n), _state(g, s), _state(g, w_np1),
                                     _ptr(ckpt_out, torch.uint8), None if stages_out is None else _stages(g, stages_out),
                                     ctypes.byref(obj) if obj is not None else None, float(weight_in), float(weight),
                                     _ptr(J_accum, torch.float64), wp, wb, _stream()))


def adjoint_step(g, w_n, s, wh_np1, wh_n, ws, lam=0.0, obj=None, c_n=0.0, grad_s=None):
    """w_n is a state tensor, or a uint8 record (BF16 or fixed-point codes) when g.ckpt_format != CKPT_NATIVE."""
    wp, wb = _ws(ws)
    wn_p = _ptr(w_n, torch.uint8) if g.ckpt_format != CKPT_NATIVE else _state(g, w_n)
    _check(lib().adj_adjoint_step(ctypes.byref(g), wn_p, _state(g, s), _state(g, wh_np1), float(lam),
                                  ctypes.byref(obj) if obj is not None else None, float(c_n), _state(g, wh_n),
                                  _state(g, grad_s), wp, wb, _stream()))


NOALLOC_SCRATCH_BYTES = 64 << 20  # ADJ_NOALLOC_SCRATCH_BYTES


def adjoint_step_noalloc(g, w_n, s, wh_np1, wh_n, lam=0.0, obj=None, c_n=0.0, grad_s=None):
    """adjoint_step without a workspace: the library's static per-GPU scratch array serves instead
    (grids whose workspace_bytes(g) <= NOALLOC_SCRATCH_BYTES; calls overlapping on one GPU race)."""
    wn_p = _ptr(w_n, torch.uint8) if g.ckpt_format != CKPT_NATIVE else _state(g, w_n)
    _check(lib().adj_adjoint_step_noalloc(ctypes.byref(g), wn_p, _state(g, s), _state(g, wh_np1), float(lam),
                                          ctypes.byref(obj) if obj is not None else None, float(c_n),
                                          _state(g, wh_n), _state(g, grad_s), _stream()))


def _stages(g, t):
    p = _ptr(t, g.dtype)
    if t.numel() != 15 * g.ncells:
        raise ValueError("stage tensors hold 3 states (15*N values)")
    return p


def primal_step_stages(g, w_n, s, w_np1, stages_out, ws):
    """primal_step that also stores the stage states W2, W3, W4 in stages_out (15*N values)."""
    wp, wb = _ws(ws)
    _check(lib().adj_primal_step_stages(ctypes.byref(g), _state(g, w_n), _state(g, s), _state(g, w_np1),
                                        _stages(g, stages_out), wp, wb, _stream()))


def adjoint_step_stages(g, w_n, stages, s, wh_np1, wh_n, ws, lam=0.0, obj=None, c_n=0.0, grad_s=None):
    """adjoint_step reading the stored stage states instead of recomputing them."""
    wp, wb = _ws(ws)
    _check(lib().adj_adjoint_step_stages(ctypes.byref(g), _state(g, w_n), _stages(g, stages), _state(g, s),
                                         _state(g, wh_np1), float(lam), ctypes.byref(obj) if obj is not None else None,
                                         float(c_n), _state(g, wh_n), _state(g, grad_s), wp, wb, _stream()))


def growth_sigma1(g, w, out, scale=1.0):
    if out.numel() != g.ncells:
        raise ValueError("sigma_1 output holds N values")
    _check(lib().adj_growth_sigma1(ctypes.byref(g), _state(g, w), float(scale), _ptr(out, g.dtype), _stream()))


def objective_and_grad(g, obj, w, ws, weight=1.0, J_accum=None, djdw=None):
    wp, wb = _ws(ws)
    _check(lib().adj_objective_and_grad(ctypes.byref(g), ctypes.byref(obj), _state(g, w), float(weight),
                                        _ptr(J_accum, torch.float64), _state(g, djdw), wp, wb, _stream()))


def energy_vhat(g, w, wh, E, ws):
    wp, wb = _ws(ws)
    _check(lib().adj_energy_vhat(ctypes.byref(g), _state(g, w), _state(g, wh), _ptr(E, torch.float64), wp, wb,
                                 _stream()))


RK4_IMAG_BOUND, RK4_REAL_BOUND = 2.8284, 2.7853
SSPRK3_IMAG_BOUND, SSPRK3_REAL_BOUND = 1.7320, 2.5127


def stability_bounds(g):
    """(imaginary-axis, real-axis) stability bounds of the grid's time scheme."""
    return (SSPRK3_IMAG_BOUND, SSPRK3_REAL_BOUND) if g.time_scheme == SSPRK3 else (RK4_IMAG_BOUND, RK4_REAL_BOUND)


def stability(g, w, out, ws, lam=0.0):
    """Explicit-stability numbers (convective, viscous, artificial viscosity) of a step from w
    into out (device FP64[3]); bounds (imaginary, real, real) of stability_bounds(g)."""
    wp, wb = _ws(ws)
    _check(lib().adj_stability(ctypes.byref(g), _state(g, w), float(lam), _ptr(out, torch.float64), wp, wb,
                               _stream()))


def check_stable(g, w, ws, lam=0.0):
    """Waits for the stream; raises AdjError (ADJ_EUNSTABLE) when a number exceeds its bound,
    else returns the three numbers."""
    h = (ctypes.c_double * 3)()
    wp, wb = _ws(ws)
    _check(lib().adj_check_stable(ctypes.byref(g), _state(g, w), float(lam), h, wp, wb, _stream()))
    return tuple(h)


def check_status():
    """Waits for the stream; raises AdjError (ADJ_ENONFINITE) when a reduction produced NaN or Inf
    since the previous check (the indication is cleared)."""
    _check(lib().adj_check_status(_stream()))


def dot(g, a, b, out, ws):
    wp, wb = _ws(ws)
    _check(lib().adj_dot(ctypes.byref(g), _state(g, a), _state(g, b), _ptr(out, torch.float64), wp, wb, _stream()))


def ckpt_encode(g, w, ckpt, ws):
    wp, wb = _ws(ws)
    _check(lib().adj_ckpt_encode(ctypes.byref(g), _state(g, w), _ptr(ckpt, torch.uint8), wp, wb, _stream()))


def ckpt_decode(g, ckpt, w):
    _check(lib().adj_ckpt_decode(ctypes.byref(g), _ptr(ckpt, torch.uint8), _state(g, w), _stream()))


def residual(g, w, s, R):
    _check(lib().adj_residual(ctypes.byref(g), _state(g, w), _state(g, s), _state(g, R), _stream()))


def vjp(g, W, kh, out, nu=None):
    _check(lib().adj_vjp(ctypes.byref(g), _state(g, W), _state(g, kh), _ptr(nu, g.dtype), _state(g, out),
                         _stream()))


def profile_enable(on=True):
    """Start (clearing earlier records) or stop event timing of every library kernel launch."""
    _check(lib().adj_profile_enable(1 if on else 0))


def profile_read(kernel_class):
    """(total milliseconds, launches) of one kernel class since profile_enable(True)."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_longlong(0)
    _check(lib().adj_profile_read(int(kernel_class), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def set_tile(kernel_class, precision, tile):
    """Tile shape id (see TILES) of the adjoint- or primal-stage kernels for one precision."""
    _check(lib().adj_set_tile(int(kernel_class), int(precision), int(tile)))


def get_tile(kernel_class, precision):
    t = lib().adj_get_tile(int(kernel_class), int(precision))
    if t < 0:
        _check(t)
    return t


def tile_launched(kernel_class, precision, bc_x, lnu, tile):
    """The tile a launch really uses when `tile` is selected (reverse-stage tiles too large for a
    work-group's shared memory run as 16x4x4)."""
    t = lib().adj_tile_launched(int(kernel_class), int(precision), int(bc_x), int(bool(lnu)), int(tile))
    if t < 0:
        _check(t)
    return t


class Ensemble:
    """Many boxes and adjoint members in one launch per stage (adj_batch_*).

    grids: one Grid per box (same precision and x boundary); member_box: the box of each member
    (non-decreasing); member_lam: lambda (L^2 units) of each member.  State arrays are packed
    over boxes and adjoint arrays over members (see offset()); a call covering boxes [0, nbox)
    or members [0, nmem) reads and writes only that prefix.
    """

    def __init__(self, grids, member_box, member_lam, obj=None, device="cuda"):
        self.grids = list(grids)
        self.member_box = [int(b) for b in member_box]
        self.member_lam = [float(x) for x in member_lam]
        nb, nm = len(self.grids), len(self.member_box)
        if nm != len(self.member_lam):
            raise ValueError("member_box and member_lam differ in length")
        self.precision = self.grids[0].precision if nb else F64
        self.dtype = torch.float64 if self.precision == F64 else torch.float32
        L = lib()
        tb = L.adj_batch_table_bytes(nb, nm, self.precision)
        if tb == 0:
            raise AdjError(-1, "an ensemble needs at least one box and one member")
        self.table = torch.empty(tb, dtype=torch.uint8, device=device)
        garr = (Grid * nb)(*self.grids)
        marr = (ctypes.c_int * nm)(*self.member_box)
        larr = (ctypes.c_double * nm)(*self.member_lam)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        _check(L.adj_batch_create(ctypes.byref(h), nb, garr, ctypes.byref(obj) if obj is not None else None, nm,
                                  marr, larr, _ptr(self.table, torch.uint8), ctypes.c_size_t(tb)))
        self._h = h
        self.nbox, self.nmem = nb, nm

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.adj_batch_destroy(h)
            self._h = None

    def offset(self, which, index):
        """Cell offset of box (which = 0) or member (which = 1) `index`; index = count gives the total."""
        o = lib().adj_batch_offset(self._h, int(which), int(index))
        if o < 0:
            raise AdjError(-1, f"offset({which}, {index}) out of range")
        return o

    def box_slice(self, t, b):
        """View of box b's five fields in a box-packed tensor."""
        return t[5 * self.offset(0, b):5 * self.offset(0, b + 1)]

    def member_slice(self, t, m):
        return t[5 * self.offset(1, m):5 * self.offset(1, m + 1)]

    def workspace(self, device="cuda"):
        return torch.empty(lib().adj_batch_workspace_bytes(self._h), dtype=torch.uint8, device=device)

    def _packed(self, t, which, count):
        if t is None:
            return None
        p = _ptr(t, self.dtype)
        if t.numel() < 5 * self.offset(which, count):
            raise ValueError(f"packed tensor holds {t.numel()} values, needs {5 * self.offset(which, count)}")
        return p

    def primal_step(self, nbox, w_n, s, w_np1, ws):
        wp, wb = _ws(ws)
        _check(lib().adj_batch_primal_step(self._h, int(nbox), self._packed(w_n, 0, nbox), self._packed(s, 0, nbox),
                                           self._packed(w_np1, 0, nbox), wp, wb, _stream()))

    def adjoint_step(self, nmem, w_n, s, wh_np1, wh_n, ws, c_n=None, grad_s=None):
        nb = self.member_box[nmem - 1] + 1 if 0 < nmem <= self.nmem else 1
        wp, wb = _ws(ws)
        _check(lib().adj_batch_adjoint_step(self._h, int(nmem), self._packed(w_n, 0, nb), self._packed(s, 0, nb),
                                            self._packed(wh_np1, 1, nmem), _ptr(c_n, torch.float64),
                                            self._packed(wh_n, 1, nmem), self._packed(grad_s, 1, nmem), wp, wb,
                                            _stream()))

    def objective_and_grad(self, first, count, w, weights, ws, J_accum=None, djdw=None):
        nb = self.member_box[first + count - 1] + 1 if 0 < count and first + count <= self.nmem else 1
        wp, wb = _ws(ws)
        _check(lib().adj_batch_objective_and_grad(self._h, int(first), int(count), self._packed(w, 0, nb),
                                                  _ptr(weights, torch.float64), _ptr(J_accum, torch.float64),
                                                  self._packed(djdw, 1, first + count), wp, wb, _stream()))

    def energy_vhat(self, nmem, w, wh, E, ws):
        nb = self.member_box[nmem - 1] + 1 if 0 < nmem <= self.nmem else 1
        wp, wb = _ws(ws)
        _check(lib().adj_batch_energy_vhat(self._h, int(nmem), self._packed(w, 0, nb), self._packed(wh, 1, nmem),
                                           _ptr(E, torch.float64), wp, wb, _stream()))
