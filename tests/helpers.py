"""Shared test set-up: the same problem built for the oracle and for the HIP
library from one parameter set."""
import numpy as np

from oracle import contour as oc
from oracle import tdse as ot
from paper_1505_06707_amd import workloads as wl

CONTOURS = {"secs": (oc.SECS, 0), "sharp": (oc.SHARP, 1), "off": (oc.OFF, 2), "tfecs": (oc.TFECS, 3)}


def oracle_axis(n, L, R0, theta, kind):
    return ot.Axis(n, L, kind=CONTOURS[kind][0], R0=R0, theta=theta)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def outgoing_state(ax, ay, speed=2.5, inset=3.0):
    """Four Gaussian packets, each `inset` inside R0 on one axis and moving
    outward along it, so that the ECS strips of both axes take real amplitude."""
    psi = np.zeros((ay.n, ax.n), dtype=complex)
    for sx, sy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        x0 = sx * (ax.R0 - inset) if sx else 0.0
        y0 = sy * (ay.R0 - inset) if sy else 0.0
        psi += wl.gaussian_2d(ax.x, ay.x, x0=x0, y0=y0, px=sx * speed, py=sy * speed)
    return psi
