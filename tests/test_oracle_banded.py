"""Pins of the oracle's banded ECS eigen-preconditioner (Sec. III, Eqs.
Prec_eigen_eq, K_l, PreconFFT_ECS)."""
import numpy as np
import pytest

from oracle import banded, contour, sse, tdse
from paper_1505_06707_amd import workloads as wl


@pytest.mark.parametrize("n", [16, 64, 96, 512, 1024])
def test_bands_follow_the_papers_split(n):
    b = banded.bands(n)
    flat = sorted(i for g in b for i in g)
    assert flat == list(range(n))                      # every momentum exactly once
    assert [0] in b and [n // 2] in b                  # k = 0 and Nyquist alone
    for g in b:
        assert g == list(range(g[0], g[0] + len(g)))   # consecutive indices
        if g not in ([0], [n // 2]):
            assert sorted(n - i for i in g) in b            # the mirror band of -k
    widths = sorted(len(g) for g in b if g not in ([0], [n // 2]))
    if n // 2 - 1 >= banded.N_BW:
        assert widths[0] == banded.N_BW and widths[-1] <= 2 * banded.N_BW - 1


def test_without_scaling_it_is_the_plain_fft_preconditioner():
    """q = 1: Q = delta, K_l = diag(k^2/2), so Eq. PreconFFT_ECS reduces to
    Eq. PreconFFT."""
    rng = np.random.default_rng(1)
    ax, ay = tdse.Axis(64, 12.8, kind=contour.OFF, R0=4.0), tdse.Axis(48, 9.6, kind=contour.OFF, R0=3.0)
    op = sse.Operator((ax, ay), np.zeros((48, 64)), 0.7)
    v = rng.normal(size=(48, 64)) + 1j * rng.normal(size=(48, 64))
    got = banded.preconditioner(op)(v)
    assert np.max(np.abs(got - op.precond(v))) < 1e-12 * np.max(np.abs(op.precond(v)))


@pytest.mark.parametrize("kind,theta", [(contour.SECS, 0.5), (contour.TFECS, 0.5)])
def test_blocks_are_complex_orthogonal_and_reconstruct_K_l(kind, theta):
    ab = banded.AxisBands(tdse.Axis(256, 51.2, kind=kind, R0=18.0, theta=theta))
    for b, X, K in zip(ab.bands, ab.X, ab.Kl):
        assert np.max(np.abs(X.T @ X - np.eye(len(b)))) < 1e-10          # X^-1 = X^T
        assert np.allclose(K, K.T, rtol=0, atol=1e-12 * np.max(np.abs(K)) + 1e-300)   # complex symmetric
        assert np.max(np.abs(X.T @ np.diag(ab.lam[b]) @ X - K)) <= 1e-10 * max(1.0, np.max(np.abs(K)))


def test_q_fourier_is_even_and_its_mean():
    ax = tdse.Axis(128, 25.6, kind=contour.TFECS, R0=8.0, theta=0.5)
    d = np.arange(-9, 10)
    Q = banded.q_fourier(ax.q, ax.x, ax.L, d)
    assert np.max(np.abs(Q - Q[::-1])) < 1e-13
    assert abs(Q[9] - np.mean(ax.q ** -2.0)) < 1e-14


@pytest.mark.parametrize("kind,theta,paper", [(contour.SECS, np.pi / 4, 36), (contour.TFECS, 0.5, 79)])
def test_iterations_against_the_papers_counts(kind, theta, paper):
    """Sec. V reports about 36 (SECS) and 79 (TFECS) PCG iterations to 1e-12
    with this preconditioner at N = 1024, h = 0.1, r_s = 40, for right-hand
    sides it does not give.  With a seeded smooth source the banded
    preconditioner must beat the plain one and stay within twice those counts."""
    n, L, R0 = 1024, 102.4, 40.0
    ax = tdse.Axis(n, L, kind=kind, R0=R0, theta=theta)
    V = tdse.softcore(1.0, 2.0, ax.z)
    f = wl.smooth_source(None, n, seed=3)
    for E in (1.0, 2.0):
        op = sse.Operator((ax,), V, E)
        _, it_plain, _ = sse.cocg(op, f, rtol=1e-12, maxit=20000)
        op.precond = banded.preconditioner(op)
        _, it_band, res = sse.cocg(op, f, rtol=1e-12, maxit=20000)
        assert res <= 1e-12
        assert it_band < it_plain and it_band <= 2 * paper


def test_banded_cocg_reaches_the_dense_solution_2d():
    rng = np.random.default_rng(9)
    ax, ay = tdse.Axis(16, 6.4, R0=2.0), tdse.Axis(16, 6.4, kind=contour.TFECS, R0=2.0, theta=0.5)
    V = tdse.softcore(1.0, 0.64, ax.z[None, :], ay.z[:, None])
    op = sse.Operator((ax, ay), V, 0.8)
    f = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    xd = sse.dense_solve(op, f)
    op.precond = banded.preconditioner(op)
    x, it, res = sse.cocg(op, f, rtol=1e-13)
    assert res <= 1e-13
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


def _banded_kinetic_dense(axis, bands):
    """K_a of Eq. K_l in the Fourier basis, block-diagonal over the bands, built
    without the oracle's Toeplitz shortcut: Q = F diag(q^-2) F^dagger with the
    dense F of Eq. Fmatrix, [K_l]_{nm} = 1/2 k_n k_m Q_{nm} inside a band."""
    from oracle import grid
    F = grid.dft_matrix(axis.n, axis.L)
    Q = F @ np.diag(axis.q ** -2.0) @ F.conj().T
    K = np.zeros((axis.n, axis.n), dtype=complex)
    for b in bands:
        idx = np.asarray(b)
        K[np.ix_(idx, idx)] = 0.5 * np.outer(axis.k[idx], axis.k[idx]) * Q[np.ix_(idx, idx)]
    return K


@pytest.mark.parametrize("kind", [contour.SECS, contour.TFECS])
def test_banded_preconditioner_inverts_its_own_operator(kind):
    """P^-1 = F^-1 X^T (Lambda - E)^-1 X F is the exact inverse of
    F^-1 K_a F - E with K_a assembled from the blocks K_l (Eqs. K_l,
    PreconFFT_ECS).  Swapping X and X^T in the apply breaks this identity."""
    rng = np.random.default_rng(21)
    ax = tdse.Axis(64, 12.8, kind=kind, R0=3.5, theta=0.5)
    ay = tdse.Axis(48, 9.6, kind=kind, R0=2.8, theta=0.5)
    E = 0.65
    op = sse.Operator((ax, ay), np.zeros((48, 64)), E)
    Kx = _banded_kinetic_dense(ax, banded.bands(64))
    Ky = _banded_kinetic_dense(ay, banded.bands(48))
    v = rng.normal(size=(48, 64)) + 1j * rng.normal(size=(48, 64))
    s = op._F(v)
    Av = op._Finv(s @ Kx.T + Ky @ s) - E * v
    P = banded.preconditioner(op)
    assert np.linalg.norm(P(Av) - v) / np.linalg.norm(v) < 1e-11
    # the same check with X and X^T swapped in the apply must fail
    ab = [banded.AxisBands(ax), banded.AxisBands(ay)]
    div = ab[0].lam[None, :] + ab[1].lam[:, None] - E
    t = op._F(Av)
    t = ab[0].apply_X(ab[1].apply_X(t, 0, transpose=True), 1, transpose=True)
    t = ab[1].apply_X(ab[0].apply_X(t / div, 1), 0)
    assert np.linalg.norm(op._Finv(t) - v) / np.linalg.norm(v) > 1e-3


# ---- 3D (Eq. PreconFFT_ECS with X = X_x (x) X_y (x) X_z)

def test_3d_without_scaling_it_is_the_plain_fft_preconditioner():
    rng = np.random.default_rng(31)
    axes = (tdse.Axis(32, 6.4, kind=contour.OFF, R0=2.0), tdse.Axis(24, 4.8, kind=contour.OFF, R0=1.5),
            tdse.Axis(16, 3.2, kind=contour.OFF, R0=1.0))
    op = sse.Operator(axes, np.zeros((16, 24, 32)), 0.45)
    v = rng.normal(size=(16, 24, 32)) + 1j * rng.normal(size=(16, 24, 32))
    got = banded.preconditioner(op)(v)
    assert np.max(np.abs(got - op.precond(v))) < 1e-12 * np.max(np.abs(op.precond(v)))


@pytest.mark.parametrize("kind", [contour.SECS, contour.TFECS])
def test_3d_banded_preconditioner_inverts_its_own_operator(kind):
    """P^-1 is the exact inverse of F^-1 (K_x + K_y + K_z) F - E with each
    K_a assembled from the dense Q of Eq. Fmatrix; the apply with X and X^T
    swapped is not."""
    rng = np.random.default_rng(32)
    ax = tdse.Axis(32, 6.4, kind=kind, R0=2.0, theta=0.5)
    ay = tdse.Axis(24, 4.8, kind=kind, R0=1.5, theta=0.5)
    az = tdse.Axis(16, 3.2, kind=kind, R0=1.0, theta=0.5)
    E = 0.65
    op = sse.Operator((ax, ay, az), np.zeros((16, 24, 32)), E)
    K = [_banded_kinetic_dense(a, banded.bands(a.n)) for a in (ax, ay, az)]
    v = rng.normal(size=(16, 24, 32)) + 1j * rng.normal(size=(16, 24, 32))
    s = op._F(v)
    Ks = (np.einsum("ij,zyj->zyi", K[0], s) + np.einsum("ij,zjx->zix", K[1], s)
          + np.einsum("ij,jyx->iyx", K[2], s))
    Av = op._Finv(Ks) - E * v
    P = banded.preconditioner(op)
    assert np.linalg.norm(P(Av) - v) / np.linalg.norm(v) < 1e-11
    ab = [banded.AxisBands(a) for a in (ax, ay, az)]
    div = ab[0].lam[None, None, :] + ab[1].lam[None, :, None] + ab[2].lam[:, None, None] - E
    t = op._F(Av)
    for a in range(3):
        t = ab[a].apply_X(t, 2 - a, transpose=True)
    t = t / div
    for a in range(3):
        t = ab[a].apply_X(t, 2 - a)
    assert np.linalg.norm(op._Finv(t) - v) / np.linalg.norm(v) > 1e-3


def test_3d_banded_cocg_reaches_the_dense_solution():
    """With ECS (SECS, SECS, TFECS) and the soft-core on the contour, COCG
    with the banded P^-1 (complex symmetric: X^T on both sides) converges to
    Gaussian elimination's solution, in fewer iterations than with Eq.
    PreconFFT."""
    axes = (tdse.Axis(16, 6.4, kind=contour.SECS, R0=2.0, theta=0.5),
            tdse.Axis(12, 4.8, kind=contour.SECS, R0=1.5, theta=0.5),
            tdse.Axis(8, 4.0, kind=contour.TFECS, R0=1.2, theta=0.5))
    ax, ay, az = axes
    V = tdse.softcore(1.0, 0.64, ax.z[None, None, :], ay.z[None, :, None], az.z[:, None, None])
    op = sse.Operator(axes, V, 0.8)
    rng = np.random.default_rng(33)
    f = rng.normal(size=(8, 12, 16)) + 1j * rng.normal(size=(8, 12, 16))
    xd = sse.dense_solve(op, f)
    _, it_plain, _ = sse.cocg(op, f, rtol=1e-12)
    op.precond = banded.preconditioner(op)
    x, it, res = sse.cocg(op, f, rtol=1e-12)
    assert res <= 1e-12
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-9
    assert it < it_plain
