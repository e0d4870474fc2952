"""The explicit-stability bounds of the C ABI (ADJ_RK4_* and ADJ_SSPRK3_*, mirrored in the binding)
against the amplification polynomials of the two time schemes, solved with numpy: the largest y
with |G(iy)| <= 1 and the negative real x closest to 0 with |G(x)| = 1 (CPU only)."""
import numpy as np
import pytest

import paper_1511_06959_amd as adj

POLYS = {
    "rk4": [1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0],
    "ssprk3": [1.0, 1.0, 1.0 / 2.0, 1.0 / 6.0],
}
BOUNDS = {"rk4": (adj.RK4_IMAG_BOUND, adj.RK4_REAL_BOUND), "ssprk3": (adj.SSPRK3_IMAG_BOUND, adj.SSPRK3_REAL_BOUND)}


def _imag_limit(c):
    # |G(iy)|^2 - 1 as a polynomial in y, largest positive root
    G = np.polynomial.Polynomial(c)
    re = np.polynomial.Polynomial([c[k] * (1j ** k).real for k in range(len(c))])
    im = np.polynomial.Polynomial([c[k] * (1j ** k).imag for k in range(len(c))])
    roots = (re * re + im * im - 1.0).roots()
    pos = [r.real for r in roots if abs(r.imag) < 1e-9 and r.real > 1e-6]
    return max(pos)


def _real_limit(c):
    # G(x)^2 - 1: RK4 returns to G = +1, SSP-RK3 falls through G = -1
    G = np.polynomial.Polynomial(c)
    roots = (G * G - 1.0).roots()
    return -max(r.real for r in roots if abs(r.imag) < 1e-9 and r.real < -1e-6)


@pytest.mark.parametrize("scheme", sorted(POLYS))
def test_bounds_match_amplification_polynomial(scheme):
    im, re = BOUNDS[scheme]
    assert abs(im - _imag_limit(POLYS[scheme])) <= 1e-4
    assert abs(re - _real_limit(POLYS[scheme])) <= 1e-4


def test_binding_picks_the_scheme():
    g = adj.Grid.make((4, 4, 4), (1.0, 1.0, 1.0), 0.01, 1e-3, time_scheme=adj.SSPRK3)
    assert adj.stability_bounds(g) == BOUNDS["ssprk3"]
    g.time_scheme = adj.RK4
    assert adj.stability_bounds(g) == BOUNDS["rk4"]
