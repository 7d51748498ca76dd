"""Shared test set-up: the same problem built for the oracle and for the HIP
library from one parameter set."""
import numpy as np

from oracle import contour as oc
from oracle import tdse as ot

CONTOURS = {"secs": (oc.SECS, 0), "sharp": (oc.SHARP, 1), "off": (oc.OFF, 2), "tfecs": (oc.TFECS, 3)}


def oracle_axis(n, L, R0, theta, kind):
    return ot.Axis(n, L, kind=CONTOURS[kind][0], R0=R0, theta=theta)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
