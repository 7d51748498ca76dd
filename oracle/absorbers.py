"""Complex absorbing potentials of Sec. IV (test infrastructure only).

Sec. IV compares ECS with two absorbing potentials added to U on an unscaled
grid (contour off, q = 1).  On one axis, with the absorbing region
r_s < |x| < r_max, Dx_CS = r_max - r_s and s = (|x| - r_s)/Dx_CS:

* CAP (Eq. CAP_via_q): U_a = E_CAP [1 - q(x)^2], q the smooth contour of
  Eq. qSECS, whose end angle the paper fixes at pi/4, so that
  U_a = E_CAP [1 - exp(i pi s / 2)].  The paper uses E_CAP = 2.
* TFAP (Eqs. TFAP, yTFAP): U_a = -i (k_min^2 / 2) y(s),
  y(s) = [a s - b s^3 + 4/(1 - s)^2 - 4/(1 + s)^2] / c^2,
  a = c^3 - 16, b = c^3 - 17, c = 2.622057 (the printed value).
  The paper uses k_min = 0.25.

Both vanish for |x| <= r_s.  Readings:
* r_max is the box edge L/2 (as for the contours); the cell-centred nodes
  stop half a cell short of it, so y(s) is finite at every node.
* On a grid of several dimensions the axis terms are summed, as the contour
  factors of ECS are per axis.
"""
import numpy as np

C_TFAP = 2.622057   # c of Eq. yTFAP, as printed


def _s(x, R0, rmax):
    """s = (|x| - r_s)/Dx_CS beyond r_s, and the mask of those nodes."""
    ax = np.abs(np.asarray(x, dtype=float))
    out = ax > R0
    return (ax - R0) / (rmax - R0), out


def cap_potential(x, R0, rmax, E_cap=2.0):
    """U_a = E_CAP [1 - q_SECS(x)^2] (Eq. CAP_via_q with Eq. qSECS, end angle pi/4)."""
    s, out = _s(x, R0, rmax)
    U = np.zeros(s.shape, dtype=complex)
    q = np.exp(1j * (np.pi / 4) * s[out])
    U[out] = E_cap * (1.0 - q * q)
    return U


def tfap_y(s, c=C_TFAP):
    """y(s) of Eq. yTFAP, term by term as printed."""
    s = np.asarray(s, dtype=float)
    a = c ** 3 - 16.0
    b = c ** 3 - 17.0
    return (a * s - b * s ** 3 + 4.0 / (1.0 - s) ** 2 - 4.0 / (1.0 + s) ** 2) / c ** 2


def tfap_potential(x, R0, rmax, kmin=0.25):
    """U_a = -i (k_min^2 / 2) y(s) for |x| > r_s (Eq. TFAP)."""
    s, out = _s(x, R0, rmax)
    U = np.zeros(s.shape, dtype=complex)
    U[out] = -0.5j * kmin * kmin * tfap_y(s[out])
    return U


def absorber_grid(kind, axes_x, R0s, rmaxs, param):
    """The sum over axes of the 1D absorber on a [.., ny, nx] grid (axis 0 = x,
    the fastest).  ``kind`` is "cap" (param = E_CAP) or "tfap" (param = k_min)."""
    f = {"cap": cap_potential, "tfap": tfap_potential}[kind]
    nd = len(axes_x)
    U = 0.0
    for a, (x, R0, rmax) in enumerate(zip(axes_x, R0s, rmaxs)):
        shape = [1] * nd
        shape[nd - 1 - a] = len(x)
        U = U + f(x, R0, rmax, param).reshape(shape)
    return np.asarray(U, dtype=complex)
