"""ECS contours q(x) and z(x) = int_0^x q(x') dx' (test infrastructure only).

Sec. II, Eq. ECSintdef defines the complex coordinate z(x) = int_0^x q.
Sec. IV gives the contours compared in the paper:

* sharp:  q = 1 for |x| < r_s, q = exp(i theta_s) beyond;
* SECS (Eq. qSECS): q = exp[i phi (|x| - r_s)/Dx_CS] for |x| > r_s with
  Dx_CS = r_max - r_s.  The paper fixes the end angle phi = pi/4; here the end
  angle is a parameter ``theta`` (pi/4 reproduces the paper);
* off:    q = 1, z = x (plain SO-FFT);
* TFECS (Eq. qTFECS): q = sqrt(1 + i y(s)) for |x| > r_s, s = (|x| - r_s)/Dx_CS,
  y(s) = alpha [(1 - s)^-2 - (1 + s)^-2 - 4 s]; the parameter ``theta`` carries
  alpha (the paper uses 0.5).  q is infinite at the box edge (s = 1), so only
  1/q (= 0) is used there; z(x) has no closed form and is integrated
  numerically (adaptive quadrature), finite at every node because the nodes
  stop half a cell short of the edge.

Readings:
* r_max is the box edge b = L/2, so q reaches its end angle at the box edge.
* Sharp contour at a tie |x| = r_s: the point is unscaled unless
  |x| - r_s > 1e-9 h (h the grid step).  SECS is continuous there.
"""
import numpy as np
from scipy.integrate import quad

SECS = "secs"
SHARP = "sharp"
OFF = "off"
TFECS = "tfecs"


def tfecs_y(s, alpha):
    """y(s) = alpha [(1 - s)^-2 - (1 + s)^-2 - 4 s] of Eq. qTFECS, as printed.
    Near s = 0 the three terms cancel to O(s^3); q = sqrt(1 + i y) then carries
    an absolute rounding error of a few 1e-16, far below every tolerance."""
    s = np.asarray(s, dtype=float)
    return alpha * ((1.0 - s) ** -2 - (1.0 + s) ** -2 - 4.0 * s)


def _tfecs_q_scalar(u, R0, D, alpha):
    s = (u - R0) / D
    return np.sqrt(1.0 + 1j * tfecs_y(s, alpha))


def q_of_x(x, kind, R0, rmax, theta, h):
    """q(x) for the contour ``kind`` (Sec. IV)."""
    x = np.asarray(x, dtype=float)
    ax = np.abs(x)
    q = np.ones(x.shape, dtype=complex)
    if kind == OFF:
        return q
    if kind == SECS:
        D = rmax - R0
        out = ax > R0
        q[out] = np.exp(1j * theta * (ax[out] - R0) / D)
        return q
    if kind == SHARP:
        out = (ax - R0) > 1e-9 * h
        q[out] = np.exp(1j * theta)
        return q
    if kind == TFECS:
        D = rmax - R0
        s = (ax - R0) / D
        inner = (ax > R0) & (s < 1.0)
        q[inner] = np.sqrt(1.0 + 1j * tfecs_y(s[inner], theta))
        q[s >= 1.0] = complex(np.inf, 0.0)
        return q
    raise ValueError(kind)


def z_of_x(x, kind, R0, rmax, theta, h):
    """z(x) = int_0^x q (Sec. II, Eq. ECSintdef), in closed form per contour."""
    x = np.asarray(x, dtype=float)
    ax = np.abs(x)
    z = x.astype(complex)
    if kind == OFF:
        return z
    if kind == SECS:
        D = rmax - R0
        out = ax > R0
        s = (ax[out] - R0) / D
        # int_{R0}^{|x|} exp(i theta (u - R0)/D) du = D/(i theta) (exp(i theta s) - 1)
        z[out] = np.sign(x[out]) * (R0 + D / (1j * theta) * (np.exp(1j * theta * s) - 1.0))
        return z
    if kind == SHARP:
        out = (ax - R0) > 1e-9 * h
        z[out] = np.sign(x[out]) * (R0 + (ax[out] - R0) * np.exp(1j * theta))
        return z
    if kind == TFECS:
        D = rmax - R0
        out = ax > R0
        # int_{R0}^{|x|} q, accumulated over the sorted distinct |x| beyond R0
        us = np.unique(ax[out])
        acc, prev, val = 0.0 + 0.0j, R0, {}
        for u in us:
            re = quad(lambda t: _tfecs_q_scalar(t, R0, D, theta).real, prev, u, epsabs=1e-13, epsrel=1e-13, limit=200)[0]
            im = quad(lambda t: _tfecs_q_scalar(t, R0, D, theta).imag, prev, u, epsabs=1e-13, epsrel=1e-13, limit=200)[0]
            acc += re + 1j * im
            val[u] = acc
            prev = u
        z[out] = np.sign(x[out]) * (R0 + np.array([val[u] for u in ax[out]]))
        return z
    raise ValueError(kind)
