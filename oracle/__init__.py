"""FP64 CPU oracle for the stabilised discrete unsteady adjoint (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  The product package never imports it and shares no code with it.

Thin ctypes wrapper around ``libnsoracle.so`` (built from ``ns_oracle.cpp`` by ``build()``).
Every function takes and returns numpy FP64 arrays in the SoA layout ``w[v, k, j, i]``
flattened var-major, v = (rho, rho u1, rho u2, rho u3, rho E).  The paper passages each
function follows are cited in ``ns_oracle.cpp``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ADJNS_ORACLE_SO selects another build of the same source (the sanitizer build of the tests)
_SO = os.environ.get("ADJNS_ORACLE_SO") or os.path.join(_HERE, "libnsoracle.so")
_SRC = os.path.join(_HERE, "ns_oracle.cpp")
SANITIZED_SO = os.path.join(_HERE, "libnsoracle_san.so")


class OrcGrid(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("bc_x", ctypes.c_int32),
        ("L", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("scheme", ctypes.c_int32),
        ("flux", ctypes.c_int32),
        ("roe_delta", ctypes.c_double),
        ("w_far", ctypes.c_double * 10),
    ]


class OrcObj(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("plane_i", ctypes.c_int32), ("pt_ref", ctypes.c_double)]


OBJ_NONE, OBJ_MEAN_PRESSURE, OBJ_KE_DISSIPATION, OBJ_PT_LOSS_PLANE = 0, 1, 2, 3


def build(force=True):
    """Compile the oracle with g++ (OpenMP).  Returns the path of the shared library."""
    if force or not os.path.exists(_SO):
        cmd = ["g++", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c++17",
               "-o", _SO + ".tmp", _SRC]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def build_sanitized():
    """The oracle built for checking the oracle itself: AddressSanitizer and UndefinedBehaviorSanitizer
    (every report fatal), no optimisation that hides frames, one OpenMP thread per call as usual.
    Load it in a process started with the ASan runtime preloaded (see tests/test_oracle_sanitized.py)."""
    cmd = ["g++", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fopenmp", "-fPIC", "-shared", "-std=c++17",
           "-o", SANITIZED_SO + ".tmp", _SRC]
    subprocess.check_call(cmd)
    os.replace(SANITIZED_SO + ".tmp", SANITIZED_SO)
    return SANITIZED_SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        gp = P(OrcGrid)
        op = P(OrcObj)
        sig = {
            "orc_residual": [gp, dp, dp, dp],
            "orc_jvp": [gp, dp, dp, dp],
            "orc_roe_flux": [gp, ctypes.c_int, dp, dp, dp],
            "orc_char_flux": [gp, ctypes.c_int, dp, dp],
            "orc_vjp": [gp, dp, dp, dp],
            "orc_lnu_apply": [gp, dp, dp, dp],
            "orc_primal_step": [gp, dp, dp, dp],
            "orc_primal_step_complex": [gp, dp, dp, dp, dp, dp, dp],
            "orc_tlm_step": [gp, dp, dp, dp, dp, dp, dp, dp],
            "orc_lnu_apply_groups": [gp, dp, dp, dp, dp],
            "orc_adjoint_step": [gp, dp, dp, dp, dp, op, ctypes.c_double, dp, dp],
            "orc_objective": [gp, op, dp, dp, dp],
            "orc_sigma1": [gp, dp, dp],
            "orc_growth_matrix_field": [gp, dp, dp],
            "orc_cell_growth_matrix": [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp],
            "orc_energy_vhat": [gp, dp, dp, dp, dp],
            "orc_ckpt_blocks": [ctypes.POINTER(OrcGrid)],
            "orc_ckpt_encode": [ctypes.POINTER(OrcGrid), P(ctypes.c_float), P(ctypes.c_uint16), P(ctypes.c_float),
                                ctypes.c_int],
            "orc_ckpt_decode": [ctypes.POINTER(OrcGrid), P(ctypes.c_uint16), P(ctypes.c_float), P(ctypes.c_float),
                                ctypes.c_int],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.orc_matrix_sigma1.argtypes = [dp]
        L.orc_matrix_sigma1.restype = ctypes.c_double
        L.orc_ckpt_blocks.restype = ctypes.c_long
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_set_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    """OpenMP threads of the following oracle calls; returns the count in force."""
    return lib().orc_set_num_threads(int(n))


# ---------------------------------------------------------------------------------------------
SCHEME_RK4, SCHEME_SSPRK3 = 0, 1
BC_PERIODIC, BC_SLIP_WALLS, BC_CHARACTERISTIC = 0, 1, 2
FLUX_SPLIT, FLUX_ROE = 0, 1


def make_grid(n, L, gamma=1.4, prandtl=0.72, mu=0.01, dt=0.0, bc_x=0, scheme=SCHEME_RK4, flux=FLUX_SPLIT,
              roe_delta=0.1, w_far=None):
    """scheme: time marching, SCHEME_RK4 (classical RK4) or SCHEME_SSPRK3 (Shu-Osher SSP-RK3).
    flux: convective face flux, FLUX_SPLIT (split central form) or FLUX_ROE (Roe's approximate
    Riemann solver on linearly reconstructed face states, wave speeds |lam| smoothed within
    roe_delta times the Roe sound speed).
    bc_x 2 (characteristic inflow/outflow in x): w_far = two far-field conservative states (beyond
    x = 0, beyond x = L_x)."""
    g = OrcGrid()
    for d in range(3):
        g.n[d] = int(n[d])
        g.L[d] = float(L[d])
    g.bc_x = int(bc_x)
    g.gamma, g.prandtl, g.mu, g.dt = float(gamma), float(prandtl), float(mu), float(dt)
    g.scheme = int(scheme)
    g.flux = int(flux)
    g.roe_delta = float(roe_delta)
    if w_far is not None:
        far = np.asarray(w_far, dtype=np.float64).reshape(10)
        for i in range(10):
            g.w_far[i] = float(far[i])
    return g


def grid_from(p):
    """Oracle grid from a plain parameter mapping (keys n, L, gamma, prandtl, mu, dt, bc_x[, scheme,
    flux, roe_delta])."""
    return make_grid(p["n"], p["L"], p.get("gamma", 1.4), p.get("prandtl", 0.72), p["mu"],
                     p.get("dt", 0.0), p.get("bc_x", 0), p.get("scheme", SCHEME_RK4), p.get("flux", FLUX_SPLIT),
                     p.get("roe_delta", 0.1), p.get("w_far"))


def make_obj(kind=0, plane_i=0, pt_ref=0.0):
    o = OrcObj()
    o.kind, o.plane_i, o.pt_ref = int(kind), int(plane_i), float(pt_ref)
    return o


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _null():
    return ctypes.POINTER(ctypes.c_double)()


def _ncells(g):
    return g.n[0] * g.n[1] * g.n[2]


def _chk(rc, name):
    if rc != 0:
        raise ValueError(f"oracle {name} rejected its input (rc={rc})")


def residual(g, w, s=None):
    N = _ncells(g)
    w, wp = _d(w)
    sp = _null()
    if s is not None:
        s, sp = _d(s)
    out = np.zeros(5 * N)
    _chk(lib().orc_residual(ctypes.byref(g), wp, sp, _d(out)[1]), "residual")
    return out


def roe_flux(g, d, wl, wr):
    """Roe flux between two face states (5 conservative values each) in direction d."""
    wl, pl = _d(wl)
    wr, pr = _d(wr)
    F, pF = _d(np.zeros(5))
    _chk(lib().orc_roe_flux(ctypes.byref(g), int(d), pl, pr, pF), "roe_flux")
    return F


def char_flux(g, side, w):
    """Flux through the characteristic boundary face of side 0 (x = 0) or 1 (x = L_x) next to the
    boundary cell state w."""
    w, pw = _d(w)
    F, pF = _d(np.zeros(5))
    _chk(lib().orc_char_flux(ctypes.byref(g), int(side), pw, pF), "char_flux")
    return F


def jvp(g, W, v):
    W, Wp = _d(W)
    v, vp = _d(v)
    out = np.zeros(5 * _ncells(g))
    _chk(lib().orc_jvp(ctypes.byref(g), Wp, vp, _d(out)[1]), "jvp")
    return out


def vjp(g, W, kh):
    W, Wp = _d(W)
    kh, kp = _d(kh)
    out = np.zeros(5 * _ncells(g))
    _chk(lib().orc_vjp(ctypes.byref(g), Wp, kp, _d(out)[1]), "vjp")
    return out


def lnu_apply(g, nu, q):
    nu, nup = _d(nu)
    q, qp = _d(q)
    out = np.zeros(5 * _ncells(g))
    _chk(lib().orc_lnu_apply(ctypes.byref(g), nup, qp, _d(out)[1]), "lnu_apply")
    return out


def primal_step(g, w, s=None):
    w, wp = _d(w)
    sp = _null()
    if s is not None:
        s, sp = _d(s)
    out = np.zeros_like(w)
    _chk(lib().orc_primal_step(ctypes.byref(g), wp, sp, _d(out)[1]), "primal_step")
    return out


def primal_step_complex(g, w, s=None):
    """RK4 step on complex state/source (complex-step differentiation)."""
    w = np.asarray(w, dtype=np.complex128)
    wr, wrp = _d(w.real.copy())
    wi, wip = _d(w.imag.copy())
    if s is None:
        s = np.zeros_like(w)
    s = np.asarray(s, dtype=np.complex128)
    sr, srp = _d(s.real.copy())
    si, sip = _d(s.imag.copy())
    outr = np.zeros(w.size)
    outi = np.zeros(w.size)
    _chk(lib().orc_primal_step_complex(ctypes.byref(g), wrp, wip, srp, sip, _d(outr)[1], _d(outi)[1]),
         "primal_step_complex")
    return outr + 1j * outi


def _lam3(lam):
    """lambda per variable group (rho, rho u, rho E): a scalar applies to all three."""
    v = np.broadcast_to(np.asarray(lam, dtype=np.float64), (3,)).copy()
    return v, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lnu_apply_groups(g, w, lam, q):
    """L_nu q with nu_g = lam_g sigma_1(w) on the components of group g (rho, rho u, rho E)."""
    w, wp = _d(w)
    q, qp = _d(q)
    lam, lp = _lam3(lam)
    out = np.zeros(5 * _ncells(g))
    _chk(lib().orc_lnu_apply_groups(ctypes.byref(g), wp, lp, qp, _d(out)[1]), "lnu_apply_groups")
    return out


def tlm_step(g, w, s, dw, ds=None, lam=0.0):
    w, wp = _d(w)
    sp = _null()
    if s is not None:
        s, sp = _d(s)
    dw, dwp = _d(dw)
    dsp = _null()
    if ds is not None:
        ds, dsp = _d(ds)
    wn = np.zeros_like(w)
    dwn = np.zeros_like(w)
    lam, lp = _lam3(lam)
    _chk(lib().orc_tlm_step(ctypes.byref(g), wp, sp, dwp, dsp, lp, _d(wn)[1], _d(dwn)[1]),
         "tlm_step")
    return wn, dwn


def adjoint_step(g, w, s, a, lam=0.0, obj=None, c_n=0.0, grad_s=None):
    """Returns w^_n; accumulates into grad_s (FP64 array, modified in place) when given.
    lam: one lambda for all components, or three (rho, rho u, rho E groups)."""
    w, wp = _d(w)
    sp = _null()
    if s is not None:
        s, sp = _d(s)
    a, ap = _d(a)
    wh = np.zeros_like(w)
    gsp = _null()
    if grad_s is not None:
        assert grad_s.dtype == np.float64 and grad_s.flags.c_contiguous
        gsp = grad_s.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    op = ctypes.byref(obj) if obj is not None else ctypes.POINTER(OrcObj)()
    lam, lp = _lam3(lam)
    _chk(lib().orc_adjoint_step(ctypes.byref(g), wp, sp, ap, lp, op, float(c_n), _d(wh)[1], gsp),
         "adjoint_step")
    return wh


def objective(g, obj, w, grad=True):
    w, wp = _d(w)
    j = ctypes.c_double(0.0)
    dj = np.zeros_like(w) if grad else None
    djp = _d(dj)[1] if grad else _null()
    _chk(lib().orc_objective(ctypes.byref(g), ctypes.byref(obj), wp, ctypes.byref(j), djp), "objective")
    return (j.value, dj) if grad else j.value


def sigma1(g, w):
    w, wp = _d(w)
    out = np.zeros(_ncells(g))
    _chk(lib().orc_sigma1(ctypes.byref(g), wp, _d(out)[1]), "sigma1")
    return out


def growth_matrix_field(g, w):
    w, wp = _d(w)
    out = np.zeros(25 * _ncells(g))
    _chk(lib().orc_growth_matrix_field(ctypes.byref(g), wp, _d(out)[1]), "growth_matrix_field")
    return out.reshape(-1, 5, 5)


def cell_growth_matrix(gamma, rho, p, grads):
    grads, gp = _d(grads)
    assert grads.size == 21
    out = np.zeros(25)
    _chk(lib().orc_cell_growth_matrix(float(gamma), float(rho), float(p), gp, _d(out)[1]),
         "cell_growth_matrix")
    return out.reshape(5, 5)


def matrix_sigma1(M):
    M, Mp = _d(np.asarray(M, dtype=np.float64).reshape(25))
    return lib().orc_matrix_sigma1(Mp)


def energy_vhat(g, w, wh):
    w, wp = _d(w)
    wh, whp = _d(wh)
    vhat = np.zeros_like(w)
    E = ctypes.c_double(0.0)
    _chk(lib().orc_energy_vhat(ctypes.byref(g), wp, whp, _d(vhat)[1], ctypes.byref(E)), "energy_vhat")
    return E.value, vhat


def ckpt_encode(g, w32, i16=False):
    """Block-scaled encoding of an FP32 state with a plane predictor per block and variable:
    (codes, header[blocks, 25]) with header[b, 5 v + (0..4)] = a', g_x, g_y, g_z, s; BF16 codes,
    or 16-bit fixed-point codes when i16."""
    w32 = np.ascontiguousarray(w32, dtype=np.float32)
    nb = lib().orc_ckpt_blocks(ctypes.byref(g))
    q = np.zeros(w32.size, dtype=np.uint16)
    hdr = np.zeros((nb, 25), dtype=np.float32)
    lib().orc_ckpt_encode(ctypes.byref(g), w32.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                          q.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                          hdr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(bool(i16)))
    return q, hdr


def ckpt_decode(g, q, hdr, i16=False):
    q = np.ascontiguousarray(q, dtype=np.uint16)
    hdr = np.ascontiguousarray(hdr, dtype=np.float32)
    out = np.zeros(q.size, dtype=np.float32)
    lib().orc_ckpt_decode(ctypes.byref(g), q.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)),
                          hdr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(bool(i16)))
    return out


# ---------------------------------------------------------------------------------------------
# Window drivers (plain Python loops over the step functions above)
# ---------------------------------------------------------------------------------------------
def primal_window(g, w0, s, nsteps):
    """States w_0 .. w_N (list of arrays)."""
    traj = [np.array(w0, dtype=np.float64)]
    for _ in range(nsteps):
        traj.append(primal_step(g, traj[-1], s))
    return traj


def objective_window(g, obj, traj, weights):
    """J = sum_n c_n j(w_n)  (rectangle rule of the time average)."""
    J = 0.0
    for n, c in enumerate(weights):
        if c != 0.0:
            J += c * objective(g, obj, traj[n], grad=False)
    return J


def adjoint_window(g, obj, traj, s, weights, lam=0.0, energy=False):
    """Reverse sweep over a stored trajectory.  Returns (w^_0, grad_s[, E history])."""
    N = len(traj) - 1
    M = traj[0].size
    grad_s = np.zeros(M)
    a = np.zeros(M)
    if weights[N] != 0.0:
        _, dj = objective(g, obj, traj[N])
        a = weights[N] * dj
    Ehist = []
    if energy:
        Ehist.append(energy_vhat(g, traj[N], a)[0])
    for n in range(N - 1, -1, -1):
        a = adjoint_step(g, traj[n], s, a, lam, obj, weights[n], grad_s)
        if energy:
            Ehist.append(energy_vhat(g, traj[n], a)[0])
    if energy:
        return a, grad_s, Ehist[::-1]
    return a, grad_s
