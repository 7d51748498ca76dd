"""Grid, momenta and the unitary DFT of Sec. II (test infrastructure only).

Sec. II, Eq. DVRgrid: on [a, b] the nodes are the cell centres
x_i = a + h (i - 1/2), i = 1..N, h = (b - a)/N.  Here indices are 0-based, so
x_j = a + h (j + 1/2), j = 0..N-1.  We always take a symmetric box a = -L/2,
b = L/2.

Sec. II, Eq. FFTbasis: phi_n(x) = exp(i k_n x)/sqrt(b - a) with
k_n = 2 pi (n-1)/(b-a) for n in [1, N/2] and k_n = -2 pi (N+1-n)/(b-a) for
n in [N/2+1, N].  0-based: k_m = 2 pi m/L for m < N/2, else 2 pi (m - N)/L, so
the Nyquist momentum is negative.

Sec. II, Eq. Fmatrix prints F_{ni} = phi_n(x_i) sqrt(h).  Reading: the forward
("direct") transform carries the conjugate, F_{ni} = phi_n^*(x_i) sqrt(h), so
that F maps a packet moving with +v0 to a spectrum peaked at +v0 (Sec. IV,
Eq. Ateor).  Every use on the hot path is F^-1 g(k^2) F with g even, for which
both signs give the same result.

Sec. II, Eq. DVRbasis: the Lagrange functions xi_i(x) = sqrt(h) sum_n
phi_n^*(x_i) phi_n(x).  The paper states xi_i(x_j) = sqrt(h) delta_ij; summing
the series gives xi_i(x_j) = delta_ij / sqrt(h), which is the value consistent
with the paper's own coefficients psi_i = sqrt(h) psi(x_i) and with the
orthonormality of the xi_i.  The oracle uses the summed value.
"""
import numpy as np
import scipy.fft


def nodes(n, L):
    """Cell-centred nodes x_j = -L/2 + h (j + 1/2) (Sec. II, Eq. DVRgrid)."""
    h = L / n
    return -L / 2 + h * (np.arange(n) + 0.5)


def midpoints(n, L):
    """Cell edges x_{j+1/2} = -L/2 + h (j + 1), j = 0..n-1.

    The last one is the box edge b, which the periodic basis identifies with a.
    They carry q_{i+1/2} of the three-point scheme (Sec. II, Eq. Ks_FD).
    """
    h = L / n
    return -L / 2 + h * (np.arange(n) + 1.0)


def momenta(n, L):
    """k_m in FFT order with a negative Nyquist term (Sec. II, Eq. FFTbasis)."""
    m = np.arange(n)
    return np.where(m < n // 2, 2 * np.pi * m / L, 2 * np.pi * (m - n) / L)


def dft_matrix(n, L):
    """Dense F_{mj} = phi_m^*(x_j) sqrt(h) (Sec. II, Eq. Fmatrix, conjugate
    reading).  For brute-force checks on tiny grids."""
    x = nodes(n, L)
    k = momenta(n, L)
    h = L / n
    return np.exp(-1j * np.outer(k, x)) * np.sqrt(h) / np.sqrt(L)


def _grid_phase(n, L):
    # F_{mj} = exp(-i k_m x_j)/sqrt(n) = exp(-i k_m (a + h/2)) exp(-2 pi i m j/n)/sqrt(n)
    # because k_m h j differs from 2 pi m j / n by a multiple of 2 pi.
    h = L / n
    return np.exp(-1j * momenta(n, L) * (-L / 2 + h / 2))


def forward(psi, L, axis=-1):
    """psi -> F psi along ``axis`` (Sec. II, Eq. Fmatrix), by scipy's FFT
    (a library primitive; ``scipy.fft.set_workers`` sets its thread count)."""
    n = psi.shape[axis]
    ph = _grid_phase(n, L)
    shape = [1] * psi.ndim
    shape[axis] = n
    return scipy.fft.fft(psi, axis=axis, norm="ortho") * ph.reshape(shape)


def inverse(phi, L, axis=-1):
    """phi -> F^-1 phi = F^dagger phi along ``axis`` (Sec. II)."""
    n = phi.shape[axis]
    ph = _grid_phase(n, L)
    shape = [1] * phi.ndim
    shape[axis] = n
    return scipy.fft.ifft(phi * np.conj(ph).reshape(shape), axis=axis, norm="ortho")


def lagrange(i, x_eval, n, L):
    """xi_i(x) = sqrt(h) sum_m phi_m^*(x_i) phi_m(x) (Sec. II, Eq. DVRbasis)."""
    x = nodes(n, L)
    k = momenta(n, L)
    h = L / n
    x_eval = np.atleast_1d(np.asarray(x_eval, dtype=float))
    terms = np.exp(1j * np.outer(x_eval - x[i], k)) / L
    return np.sqrt(h) * terms.sum(axis=1)
