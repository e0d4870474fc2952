"""Closed-form linear operators used to pin the oracle (test helper; imports nothing of the method).

Everything here is derived from the continuous equations of the paper (section "Physics",
Eq. (navier); "Unsteady adjoint", vector form) and from the stencils' Fourier symbols, not from
the oracle's code:

* Euler flux Jacobian A_d = dF_d/dw written in the textbook (u, H, phi) form.
* Symbol of the semi-discrete operator at a uniform base state, acting on a Fourier mode
  w' = w^ exp(i k.x):
    convective  -i sum_d A_d sin(k_d dx_d)/dx_d             (any consistent central face flux built
                from face means, the split product form included, linearises to this)
    viscous     momentum_k = mu sum_d D_dd u'_k + mu sum_d D_dk u'_d - (2 mu/3) sum_l D_kl u'_l
                energy     = u0 . momentum + alpha sum_d D_dd e'
    with D_dd = -4 sin^2(k_d dx_d / 2)/dx_d^2 (normal face gradient) and
    D_dt = -sin(k_d dx_d) sin(k_t dx_t)/(dx_d dx_t) (face-averaged central tangential gradient).
    Roe upwind flux on linearly reconstructed face states, at theta = k_d dx_d:
      face states  w_l = a_l w', w_r = a_r w' with a_l = 1 + i sin(theta)/2,
                   a_r = e^{i theta} (1 - i sin(theta)/2)   (w_l = w_i + (w_{i+1}-w_{i-1})/4, ...)
      face flux    A_d (a_l + a_r)/2 - |A_d| (a_r - a_l)/2, |A_d| = R diag(|lam|_s) R^-1 from the
                   eigen-decomposition of A_d (the Roe matrix of two equal states is A_d), |lam|_s
                   = |lam| outside |lam| < delta, (lam^2 + delta^2)/(2 delta) inside
      residual     -(1 - e^{-i theta}) face flux / dx_d
* Symmetriser S (printed), V = dq/dw (printed, with the sign of the u_j/rho entries corrected),
  T = S V, and the printed symmetrised flux matrices A^_d.
"""
import numpy as np


def euler_jacobian(d, rho, u, p, gamma):
    u = np.asarray(u, dtype=float)
    E = p / (gamma - 1.0) + 0.5 * rho * (u @ u)
    H = (E + p) / rho
    phi = 0.5 * (gamma - 1.0) * (u @ u)
    A = np.zeros((5, 5))
    A[0, 1 + d] = 1.0
    for k in range(3):
        A[1 + k, 0] = -u[k] * u[d] + (phi if k == d else 0.0)
        for j in range(3):
            A[1 + k, 1 + j] = ((u[k] if j == d else 0.0) + (u[d] if k == j else 0.0)
                               - ((gamma - 1.0) * u[j] if k == d else 0.0))
        A[1 + k, 4] = (gamma - 1.0) if k == d else 0.0
    A[4, 0] = u[d] * (phi - H)
    for j in range(3):
        A[4, 1 + j] = (H if j == d else 0.0) - (gamma - 1.0) * u[j] * u[d]
    A[4, 4] = gamma * u[d]
    return A


def prim_linearisation(rho, u, p, gamma):
    """Rows: (u1', u2', u3', e') as linear functions of w' = (rho', m', E')."""
    u = np.asarray(u, dtype=float)
    E = p / (gamma - 1.0) + 0.5 * rho * (u @ u)
    P = np.zeros((4, 5))
    for k in range(3):
        P[k, 0] = -u[k] / rho
        P[k, 1 + k] = 1.0 / rho
    P[3, 0] = (-E / rho + u @ u) / rho
    P[3, 1:4] = -u / rho
    P[3, 4] = 1.0 / rho
    return P


def smoothed_abs(lam, delta):
    lam = np.asarray(lam)
    return np.where(np.abs(lam) >= delta, np.abs(lam), (lam * lam + delta * delta) / (2.0 * delta))


def abs_matrix(A, delta):
    """R diag(|lam|_s) R^-1 of a matrix with real eigenvalues (numpy's eigen-decomposition)."""
    lam, R = np.linalg.eig(A)
    return np.real(R @ np.diag(smoothed_abs(np.real(lam), delta)) @ np.linalg.inv(R))


def semi_discrete_symbol(k, dx, rho, u, p, gamma, mu, prandtl, roe_delta=None):
    """5x5 complex symbol L(k) of the linearised residual at a uniform state (convective part of
    the central flux, or of the Roe flux when roe_delta is given)."""
    u = np.asarray(u, dtype=float)
    alpha = gamma * mu / prandtl
    Lk = np.zeros((5, 5), dtype=complex)
    for d in range(3):
        A = euler_jacobian(d, rho, u, p, gamma)
        th = k[d] * dx[d]
        if roe_delta is None:
            Lk += -1j * A * np.sin(th) / dx[d]
        else:
            al = 1.0 + 0.5j * np.sin(th)
            ar = np.exp(1j * th) * (1.0 - 0.5j * np.sin(th))
            absA = abs_matrix(A, roe_delta * np.sqrt(gamma * p / rho))
            Lk += -(1.0 - np.exp(-1j * th)) / dx[d] * (0.5 * (al + ar) * A - 0.5 * (ar - al) * absA)
    D = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            if a == b:
                D[a, a] = -4.0 * np.sin(0.5 * k[a] * dx[a]) ** 2 / dx[a] ** 2
            else:
                D[a, b] = -np.sin(k[a] * dx[a]) * np.sin(k[b] * dx[b]) / (dx[a] * dx[b])
    lap = np.trace(D)
    # viscous operator on (u', e') -> momentum and energy rows
    Vv = np.zeros((4, 4))
    for kk in range(3):
        Vv[kk, kk] += mu * lap
        for dd in range(3):
            Vv[kk, dd] += mu * D[dd, kk]
        for ll in range(3):
            Vv[kk, ll] -= (2.0 * mu / 3.0) * D[kk, ll]
    Vv[3, :3] = u @ Vv[:3, :3]
    Vv[3, 3] = alpha * lap
    P = prim_linearisation(rho, u, p, gamma)
    visc = np.zeros((5, 5))
    visc[1:5, :] = Vv @ P
    return Lk + visc


def rk4_polynomial(Z):
    I = np.eye(Z.shape[0], dtype=Z.dtype)
    Z2 = Z @ Z
    Z3 = Z2 @ Z
    return I + Z + Z2 / 2.0 + Z3 / 6.0 + Z3 @ Z / 24.0


def fourier_mode(n, dx, k, what):
    """Real field Re(what e^{i k.x}) on cell centres, SoA var-major flattened."""
    xs = [(np.arange(n[d]) + 0.5) * dx[d] for d in range(3)]
    z, y, x = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    ph = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    return np.stack([np.real(what[v] * ph) for v in range(5)]).ravel()


def symmetriser(rho, u, p, gamma):
    """S (printed, primitive -> symmetrised) and V = dq/dw with q = (rho, u, p)."""
    u = np.asarray(u, dtype=float)
    c = np.sqrt(gamma * p / rho)
    S = np.zeros((5, 5))
    S[0, 0] = c / (np.sqrt(gamma) * rho)
    S[1, 1] = S[2, 2] = S[3, 3] = 1.0
    S[4, 0] = -c / (rho * np.sqrt(gamma * (gamma - 1.0)))
    S[4, 4] = np.sqrt(gamma / (gamma - 1.0)) / (rho * c)
    V = np.zeros((5, 5))
    V[0, 0] = 1.0
    for j in range(3):
        V[1 + j, 0] = -u[j] / rho
        V[1 + j, 1 + j] = 1.0 / rho
    V[4, 0] = 0.5 * (gamma - 1.0) * (u @ u)
    V[4, 1:4] = -(gamma - 1.0) * u
    V[4, 4] = gamma - 1.0
    return S, V


def printed_ahat(d, u, c, gamma):
    """The symmetric matrices A^_{:d:} as printed (b = c/sqrt(gamma), a = sqrt((gamma-1)/gamma) c)."""
    b = c / np.sqrt(gamma)
    a = np.sqrt((gamma - 1.0) / gamma) * c
    A = u[d] * np.eye(5)
    A[0, 1 + d] = A[1 + d, 0] = b
    A[1 + d, 4] = A[4, 1 + d] = a
    return A
