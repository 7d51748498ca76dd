"""Pins of the oracle's absorbing potentials (Sec. IV, Eqs. CAP_via_q, qSECS,
TFAP, yTFAP) against facts that follow from the printed formulas without
retyping them: the series of y(s) at s = 0 and its pole at s = 1, the CAP's
link to the SECS contour module, its end value and initial slope, and the
absorption they cause in the oracle's propagation (the norm can only fall
where Im U <= 0)."""
import numpy as np
import pytest

from oracle import absorbers as ab
from oracle import contour
from oracle import tdse as ot

C = ab.C_TFAP


def test_tfap_y_vanishes_and_is_odd():
    s = np.linspace(-0.9, 0.9, 37)
    assert ab.tfap_y(0.0) == 0.0
    assert np.allclose(ab.tfap_y(-s), -ab.tfap_y(s), rtol=0, atol=1e-12)


def test_tfap_y_series_at_zero():
    """4/(1-s)^2 - 4/(1+s)^2 = 16 s + 32 s^3 + 48 s^5 + ..., so with a = c^3 - 16
    and b = c^3 - 17: y = c s + (49 - c^3)/c^2 s^3 + O(s^5).  A wrong sign or
    offset in any printed term changes one of the two coefficients."""
    h = 1e-5
    slope = (ab.tfap_y(h) - ab.tfap_y(-h)) / (2 * h)
    assert abs(slope - C) < 1e-8
    s = 2e-3
    cubic = (ab.tfap_y(s) - C * s) / s ** 3
    assert abs(cubic - (49.0 - C ** 3) / C ** 2) < 1e-3 * abs((49.0 - C ** 3) / C ** 2)


def test_tfap_y_pole_at_the_box_edge():
    """(1 - s)^2 y(s) -> 4/c^2 as s -> 1 (only the 4/(1 - s)^2 term diverges)."""
    for eps in (1e-4, 1e-6):
        s = 1.0 - eps
        assert abs((1.0 - s) ** 2 * ab.tfap_y(s) - 4.0 / C ** 2) < 10 * eps


def test_tfap_potential_on_a_grid():
    n, L, R0 = 1024, 102.4, 40.0
    ax = ot.Axis(n, L, kind=contour.OFF, R0=R0, theta=0.5)
    U = ab.tfap_potential(ax.x, R0, L / 2, kmin=0.25)
    assert np.all(np.isfinite(U))
    assert np.all(U.real == 0.0) and np.all(U.imag <= 0.0)
    assert np.all(U[np.abs(ax.x) <= R0] == 0.0)
    assert np.allclose(U, U[::-1], rtol=1e-12, atol=0)   # even in x (nodes symmetric to rounding)
    # k_min scales it by k_min^2
    assert np.allclose(ab.tfap_potential(ax.x, R0, L / 2, kmin=0.5), 4 * U, rtol=1e-15, atol=0)


def test_cap_is_e_cap_times_one_minus_secs_q_squared():
    """Eq. CAP_via_q read through the contour module's own SECS q (end angle pi/4)."""
    n, L, R0 = 256, 51.2, 15.0
    ax = ot.Axis(n, L, kind=contour.OFF, R0=R0, theta=0.5)
    q = contour.q_of_x(ax.x, contour.SECS, R0, L / 2, np.pi / 4, ax.h)
    U = ab.cap_potential(ax.x, R0, L / 2, E_cap=2.0)
    assert np.max(np.abs(U - 2.0 * (1.0 - q * q))) < 1e-14


def test_cap_end_value_slope_and_sign():
    R0, rmax, E = 10.0, 15.0, 2.0
    # at r_max, q^2 = exp(i pi/2) = i
    assert abs(ab.cap_potential(np.array([rmax]), R0, rmax, E)[0] - E * (1 - 1j)) < 1e-15
    # near r_s it is the linear CAP -i E pi s/2
    d = 1e-6
    u = ab.cap_potential(np.array([R0 + d]), R0, rmax, E)[0]
    slope = E * np.pi / 2 / (rmax - R0)
    assert abs(u.imag / d + slope) < 1e-8 * slope and 0 <= u.real < (slope * d) ** 2
    x = np.linspace(-rmax, rmax, 201)
    U = ab.cap_potential(x, R0, rmax, E)
    assert np.all(U.imag <= 0.0)
    assert np.allclose(np.abs(1.0 - U / E), 1.0, rtol=0, atol=1e-15)   # |q^2| = 1
    assert np.all(U[np.abs(x) <= R0] == 0.0)


def test_absorber_grid_sums_the_axes():
    ax = ot.Axis(32, 6.4, kind=contour.OFF, R0=2.0, theta=0.5)
    ay = ot.Axis(24, 4.8, kind=contour.OFF, R0=1.5, theta=0.5)
    U = ab.absorber_grid("tfap", [ax.x, ay.x], [2.0, 1.5], [3.2, 2.4], 0.3)
    assert U.shape == (24, 32)
    ux = ab.tfap_potential(ax.x, 2.0, 3.2, 0.3)
    uy = ab.tfap_potential(ay.x, 1.5, 2.4, 0.3)
    assert np.array_equal(U[5], ux + uy[5]) and np.array_equal(U[:, 7], ux[7] + uy)


@pytest.mark.parametrize("kind,param", [("cap", 2.0), ("tfap", 0.25)])
def test_absorbers_absorb_an_outgoing_packet(kind, param):
    """d||psi||^2/dt = 2 <psi|Im U|psi> <= 0: the oracle's norm never rises, and
    a packet sent into the absorbing region loses most of it."""
    n, L, R0 = 256, 51.2, 15.0
    ax = ot.Axis(n, L, kind=contour.OFF, R0=R0, theta=0.5)
    U = ab.absorber_grid(kind, [ax.x], [R0], [L / 2], param)
    pr = ot.Problem1D(ax, Zc=0.0, V0=U)
    psi = np.exp(-(ax.x - 5.0) ** 2 / 2 + 2j * ax.x)
    psi /= np.linalg.norm(psi)
    norms = [1.0]
    for _ in range(40):
        psi = pr.propagate(psi, 0.02, np.zeros(50))
        norms.append(np.linalg.norm(psi) ** 2)
    assert np.all(np.diff(norms) <= 1e-14)
    assert norms[-1] < 0.05
