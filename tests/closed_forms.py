"""Closed forms used to pin the oracle.  Written from the mathematics, not from
the oracle, so that a mistake in the oracle cannot hide behind them."""
import numpy as np


def free_gaussian(x, t, x0=0.0, k0=0.0):
    """Free evolution (i dpsi/dt = -psi''/2) of pi^{-1/4} exp(-(x-x0)^2/2 + i k0 x),
    the Gaussian packet of Sec. IV (Eq. psi0) displaced by x0."""
    w = 1.0 + 1j * t
    return (np.pi ** -0.25 / np.sqrt(w)
            * np.exp(-(x - x0 - k0 * t) ** 2 / (2 * w) + 1j * k0 * x - 0.5j * k0 ** 2 * t))


def packet_spectrum(k, v0):
    """A_teor(k) = pi^{-1/4} exp(-(k - v0)^2/2), Sec. IV Eq. Ateor: the unitary
    Fourier transform (1/sqrt(2 pi)) int exp(-ikx) psi0(x) dx of the packet."""
    return np.pi ** -0.25 * np.exp(-(k - v0) ** 2 / 2)


def scaled_kinetic_continuous(f, df, d2f, u1, u2, q):
    """K_s f = -1/2 q^{-1/2} d/dx [q^{-1} d/dx (q^{-1/2} f)] written with
    u = ln q:  K_s f = -1/2 q^{-2} [f'' - 2 u' f' + 3/4 u'^2 f - 1/2 u'' f].
    Derived by hand from the operator of Sec. II; u1 = u', u2 = u''."""
    return -0.5 * q ** -2 * (d2f - 2 * u1 * df + 0.75 * u1 ** 2 * f - 0.5 * u2 * f)
