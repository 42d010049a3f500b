"""Pins of the oracle's softening kernel against the M4 cubic spline itself.

Eq. (softdirectsum) needs a softening kernel phi -> 1/r outside its support;
the oracle uses the M4 cubic spline with support 2h.  The pins below start
from the kernel's density shape w(q) (written here independently of the
oracle) and integrate it numerically, so a wrong coefficient, sign or branch
in the oracle's closed forms fails.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


def w_m4(q):
    """M4 cubic spline shape; W(r, h) = w(r/h) / (pi h^3)."""
    if q < 1.0:
        return 1.0 - 1.5 * q * q + 0.75 * q ** 3
    if q < 2.0:
        return 0.25 * (2.0 - q) ** 3
    return 0.0


def enclosed(q):
    """Mass fraction inside radius q h: 4 pi int_0^q W r^2 dr with h = 1."""
    f = lambda s: w_m4(s) * s * s
    q = min(q, 2.0)
    if q <= 1.0:
        return 4.0 * quad(f, 0.0, q, epsabs=1e-15, epsrel=1e-14)[0]
    return 4.0 * (quad(f, 0.0, 1.0, epsabs=1e-15, epsrel=1e-14)[0]
                  + quad(f, 1.0, q, epsabs=1e-15, epsrel=1e-14)[0])


def test_normalisation():
    assert enclosed(2.0) == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("q", [0.05, 0.3, 0.7, 0.999, 1.0, 1.2, 1.5, 1.9, 2.0, 2.5, 10.0])
def test_force_is_enclosed_mass_over_q2(orc, q):
    assert orc.f_hat(q) == pytest.approx(enclosed(q) / (q * q), rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("q", [0.0, 0.1, 0.5, 0.999, 1.0, 1.3, 1.999, 2.0])
def test_potential_is_integral_of_force(orc, q):
    # psi_hat(q) = int_q^inf f_hat = int_q^2 f_hat + 1/2
    f = lambda s: enclosed(s) / (s * s) if s > 0 else 0.0
    if q < 1.0:
        tail = quad(f, q, 1.0, epsabs=1e-14)[0] + quad(f, 1.0, 2.0, epsabs=1e-14)[0]
    else:
        tail = quad(f, q, 2.0, epsabs=1e-14)[0] if q < 2.0 else 0.0
    assert orc.psi_hat(q) == pytest.approx(tail + 0.5, rel=1e-11)


def test_closed_values(orc):
    assert orc.psi_hat(0.0) == pytest.approx(7.0 / 5.0, rel=1e-15)
    assert orc.psi_hat(1.0) == pytest.approx(14.0 / 15.0, rel=1e-14)
    assert orc.psi_hat(2.0) == pytest.approx(0.5, rel=1e-14)
    assert orc.f_hat(1.0) == pytest.approx(19.0 / 30.0, rel=1e-14)
    assert orc.f_hat(2.0) == pytest.approx(0.25, rel=1e-14)


@pytest.mark.parametrize("q0", [1.0, 2.0])
def test_continuity(orc, q0):
    e = 1e-9
    assert orc.psi_hat(q0 - e) == pytest.approx(orc.psi_hat(q0 + e), abs=1e-8)
    assert orc.f_hat(q0 - e) == pytest.approx(orc.f_hat(q0 + e), abs=1e-8)


@pytest.mark.parametrize("q", [0.2, 0.8, 1.1, 1.6, 2.4])
def test_force_is_minus_potential_derivative(orc, q):
    e = 1e-5
    fd = -(orc.psi_hat(q + e) - orc.psi_hat(q - e)) / (2 * e)
    assert orc.f_hat(q) == pytest.approx(fd, rel=1e-8)


@pytest.mark.parametrize("r,h", [(0.3, 1.0), (1.5, 1.0), (2.5, 1.0), (0.01, 0.02), (5.0, 0.1)])
def test_g_and_psi_scaling(orc, r, h):
    q = r / h
    assert orc.g(r, h) * r * h * h == pytest.approx(orc.f_hat(q), rel=1e-13)
    assert orc.psi(r, h) * h == pytest.approx(orc.psi_hat(q), rel=1e-14)
    if q >= 2.0:
        assert orc.g(r, h) == pytest.approx(1.0 / r ** 3, rel=1e-14)
        assert orc.psi(r, h) == pytest.approx(1.0 / r, rel=1e-14)


def test_g_finite_at_zero(orc):
    assert orc.g(0.0, 0.5) == pytest.approx((4.0 / 3.0) / 0.125, rel=1e-15)
    assert math.isfinite(orc.g(0.0, 1e-3))


def test_direct_pair_is_antisymmetric_and_softened(orc):
    # two particles with unequal h inside each other's kernel
    x = np.array([[0.0, 0.0, 0.0], [0.3, 0.1, -0.2]])
    m = np.array([0.7, 1.3])
    h = np.array([0.2, 0.5])
    acc, pot = orc.direct(x, m, h, G=1.0, include_self=False)
    F = m[:, None] * acc
    assert np.abs(F.sum(0)).max() < 1e-15 * np.abs(F).max()
    r = np.linalg.norm(x[1] - x[0])
    gs = 0.5 * (orc.f_hat(r / h[0]) / (h[0] ** 2 * r) + orc.f_hat(r / h[1]) / (h[1] ** 2 * r))
    assert acc[0] == pytest.approx(m[1] * gs * (x[1] - x[0]), rel=1e-14)
    assert pot[0] == pytest.approx(-m[1] * 0.5 * (orc.psi_hat(r / h[0]) / h[0]
                                                  + orc.psi_hat(r / h[1]) / h[1]), rel=1e-14)
