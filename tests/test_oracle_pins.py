"""Pins of the FP64 oracle against what the paper and the mathematics fix:
closed forms, invariants, convergence orders, special cases and brute force.
None of these re-types an oracle formula; each would fail for a plausible
mistake (a dropped term, a wrong sign or index, a transposed operand)."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.integrate import quad

from oracle import contour, ecs, grid, sse, tdse
from tests import closed_forms as cf


# ----------------------------------------------------------------- grid, F
def test_grid_is_cell_centred():
    n, L = 64, 12.8
    x = grid.nodes(n, L)
    h = L / n
    assert np.allclose(np.diff(x), h, atol=1e-14)
    assert x[0] == pytest.approx(-L / 2 + h / 2, abs=1e-14)
    assert x[-1] == pytest.approx(L / 2 - h / 2, abs=1e-14)
    assert np.allclose(x, -x[::-1], atol=1e-13)


def test_momenta_cover_one_brillouin_zone_with_negative_nyquist():
    n, L = 16, 3.2
    k = grid.momenta(n, L)
    assert k[0] == 0.0
    assert k[n // 2] == pytest.approx(-np.pi * n / L)   # Nyquist is negative
    assert np.all(np.diff(k[: n // 2]) > 0) and np.all(np.diff(k[n // 2:]) > 0)
    assert sorted(np.round(k * L / (2 * np.pi)).astype(int)) == list(range(-n // 2, n // 2))


def test_F_is_unitary_and_fft_route_equals_dense_matrix():
    n, L = 24, 5.0
    F = grid.dft_matrix(n, L)
    assert np.allclose(F @ F.conj().T, np.eye(n), atol=1e-13)
    rng = np.random.default_rng(0)
    v = rng.normal(size=n) + 1j * rng.normal(size=n)
    assert np.allclose(grid.forward(v, L), F @ v, atol=1e-13)
    assert np.allclose(grid.inverse(F @ v, L), v, atol=1e-13)


def test_forward_transform_of_packet_is_the_analytic_spectrum():
    # Sec. IV: psi0 = pi^{-1/4} exp(-x^2/2 + i v0 x) has A_teor(k) peaked at +v0.
    # (F psi)_m = sum_j h e^{-i k_m x_j} psi(x_j) / sqrt(L h) ~ sqrt(2 pi/(L h)) A(k_m).
    n, L, v0 = 1024, 102.4, 2.0
    x, k = grid.nodes(n, L), grid.momenta(n, L)
    psi0 = np.pi ** -0.25 * np.exp(-x ** 2 / 2 + 1j * v0 * x)
    got = grid.forward(psi0, L)
    want = np.sqrt(2 * np.pi / (L * (L / n))) * cf.packet_spectrum(k, v0)
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))
    assert k[np.argmax(np.abs(got))] == pytest.approx(v0, abs=2 * np.pi / L)


def test_lagrange_functions_are_cardinal():
    # xi_i(x_j) = delta_ij / sqrt(h): the summed series of Eq. DVRbasis.
    n, L = 32, 6.4
    x, h = grid.nodes(n, L), L / n
    for i in (0, 5, 31):
        vals = grid.lagrange(i, x, n, L)
        want = np.zeros(n)
        want[i] = 1 / np.sqrt(h)
        assert np.allclose(vals, want, atol=1e-12)


# ----------------------------------------------------------------- contours
@pytest.mark.parametrize("kind", [contour.SECS, contour.SHARP])
def test_z_is_the_integral_of_q(kind):
    R0, rmax, theta, h = 8.0, 12.8, 0.5, 0.1
    for xv in (-12.7, -9.3, -3.0, 0.4, 7.99, 8.5, 11.0, 12.75):
        def qre(u):
            return contour.q_of_x(np.array([u]), kind, R0, rmax, theta, h)[0].real

        def qim(u):
            return contour.q_of_x(np.array([u]), kind, R0, rmax, theta, h)[0].imag
        pts = [R0, -R0]
        want = quad(qre, 0, xv, points=pts, limit=200)[0] + 1j * quad(qim, 0, xv, points=pts, limit=200)[0]
        got = contour.z_of_x(np.array([xv]), kind, R0, rmax, theta, h)[0]
        assert abs(got - want) < 1e-10


def test_secs_end_angle_and_continuity():
    R0, rmax, theta, h = 40.0, 51.2, np.pi / 4, 0.1
    q = contour.q_of_x(np.array([rmax, -rmax, R0, R0 + 1e-12]), contour.SECS, R0, rmax, theta, h)
    assert np.allclose(q[:2], np.exp(1j * np.pi / 4))     # end angle pi/4 at r_max
    assert np.allclose(q[2:], 1.0)


# ----------------------------------------------------------------- C and K_s
def _axis(n, L, kind=contour.SECS, R0=None, theta=0.5):
    return tdse.Axis(n, L, kind=kind, R0=R0, theta=theta)


def test_remainder_vanishes_where_q_is_one_and_is_symmetric():
    ax = _axis(256, 51.2, R0=20.0)
    C = ax.C.toarray()
    assert np.allclose(C, C.T, atol=0)
    interior = np.where(np.abs(ax.x) < 20.0 - 2 * ax.h)[0]
    assert np.all(C[interior, :] == 0) and np.all(C[:, interior] == 0)
    assert np.any(C != 0)


def test_remainder_for_constant_q_is_scaled_fd_laplacian():
    # Deep inside a region of constant q (sharp contour): K_s = q^-2 K_FD, so
    # C = (q^-2 - 1) K_FD there.
    ax = _axis(128, 25.6, kind=contour.SHARP, R0=6.0, theta=0.4)
    q = np.exp(0.4j)
    C = ax.C.toarray()
    h = ax.h
    rows = np.where(np.abs(ax.x) > 6.0 + 2 * h)[0]
    for j in rows:
        assert C[j, j] == pytest.approx((q ** -2 - 1) / h ** 2, rel=1e-13)
        assert C[j, (j + 1) % ax.n] == pytest.approx(-(q ** -2 - 1) / (2 * h ** 2), rel=1e-13)


def test_matrix_equals_literal_stencil_action():
    ax = _axis(96, 19.2, R0=5.0)
    rng = np.random.default_rng(1)
    v = rng.normal(size=ax.n) + 1j * rng.normal(size=ax.n)
    lit = ecs.apply_Ks(v, ax.q, ax.qm, ax.h) - ecs.apply_KFD(v, ax.h)
    assert np.allclose(ax.C @ v, lit, atol=1e-12)


def test_three_point_Ks_is_second_order_consistent_with_the_scaled_operator():
    # A smooth packet sitting in the SECS region (u = ln q linear there):
    # the three-point K_s approximates -1/2 q^-1/2 d/dx q^-1 d/dx q^-1/2 with O(h^2).
    L, R0, theta = 40.0, 4.0, 0.7
    errs = []
    for n in (400, 800, 1600):
        ax = _axis(n, L, R0=R0, theta=theta)
        x = ax.x
        c, w = 12.0, 1.5
        f = np.exp(-(x - c) ** 2 / (2 * w * w))
        df = -(x - c) / w ** 2 * f
        d2f = ((x - c) ** 2 / w ** 4 - 1 / w ** 2) * f
        D = ax.rmax - R0
        u1 = np.where(np.abs(x) > R0, 1j * theta / D * np.sign(x), 0.0)
        want = cf.scaled_kinetic_continuous(f, df, d2f, u1, 0.0, ax.q)
        got = ecs.apply_Ks(f.astype(complex), ax.q, ax.qm, ax.h)
        sel = np.abs(x - c) < 4 * w
        errs.append(np.max(np.abs(got - want)[sel]))
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.05)


def test_crank_nicolson_has_third_order_local_error():
    ax = _axis(64, 12.8, R0=3.0, theta=0.5)
    C = ax.C.toarray()
    rng = np.random.default_rng(2)
    v = rng.normal(size=ax.n) + 1j * rng.normal(size=ax.n)
    errs = []
    for tau in (0.002, 0.001, 0.0005):
        cn = ecs.CrankNicolson(ax.C, tau).apply(v)
        ex = sla.expm(-1j * tau * C) @ v
        errs.append(np.linalg.norm(cn - ex))
    assert errs[0] / errs[1] == pytest.approx(8.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(8.0, rel=0.05)


# ----------------------------------------------------------------- TDSE step
def _dense_step_1d(ax, V, tau):
    """Literal dense product of the Sec. II scheme, built from the dense F of
    Eq. Fmatrix, diagonal exponentials and a dense CN."""
    F = grid.dft_matrix(ax.n, ax.L)
    Finv = F.conj().T
    Kh = np.diag(np.exp(-1j * ax.k ** 2 / 2 * tau / 2))
    Uh = np.diag(np.exp(-1j * V * tau / 2))
    C = ax.C.toarray()
    I = np.eye(ax.n)
    CN = np.linalg.solve(I + 0.5j * tau * C, I - 0.5j * tau * C)
    return Finv @ Kh @ F @ Uh @ CN @ Uh @ Finv @ Kh @ F


def test_step_equals_dense_brute_force_1d():
    ax = _axis(32, 12.8, R0=3.0, theta=0.5)
    prob = tdse.Problem1D(ax, Zc=1.0, a2=2.0)
    rng = np.random.default_rng(3)
    v = rng.normal(size=ax.n) + 1j * rng.normal(size=ax.n)
    tau, f = 0.05, 0.03
    M = _dense_step_1d(ax, prob.potential(f), tau)
    assert np.allclose(prob.step(v, tau, f), M @ v, atol=1e-13)


def test_step_equals_dense_brute_force_2d():
    ax, ay = _axis(8, 6.4, R0=2.0), _axis(12, 7.2, R0=2.5)
    prob = tdse.Problem2D(ax, ay, Zc=1.0, a2=0.64)
    tau, f = 0.05, 0.02
    Fx, Fy = grid.dft_matrix(ax.n, ax.L), grid.dft_matrix(ay.n, ay.L)
    F = np.kron(Fy, Fx)                     # psi.ravel() has x fastest
    K = (ax.k[None, :] ** 2 + ay.k[:, None] ** 2).ravel() / 2
    Kh = np.diag(np.exp(-1j * K * tau / 2))
    Uh = np.diag(np.exp(-1j * prob.potential(f).ravel() * tau / 2))
    Ix, Iy = np.eye(ax.n), np.eye(ay.n)
    Cx, Cy = ax.C.toarray(), ay.C.toarray()
    CNx = np.linalg.solve(Ix + 0.5j * tau * Cx, Ix - 0.5j * tau * Cx)
    CNy = np.linalg.solve(Iy + 0.5j * tau * Cy, Iy - 0.5j * tau * Cy)
    CN = np.kron(CNy, Ix) @ np.kron(Iy, CNx)
    M = F.conj().T @ Kh @ F @ Uh @ CN @ Uh @ F.conj().T @ Kh @ F
    rng = np.random.default_rng(4)
    v = rng.normal(size=(ay.n, ax.n)) + 1j * rng.normal(size=(ay.n, ax.n))
    assert np.allclose(prob.step(v, tau, f).ravel(), M @ v.ravel(), atol=1e-13)


def test_strang_step_is_second_order_in_time():
    # Global error against exp(-i H T) with H = F^-1 K F + C + U (static U):
    # Strang splitting with a CN factor is second order.
    ax = _axis(48, 14.4, R0=4.0, theta=0.5)
    prob = tdse.Problem1D(ax, Zc=1.0, a2=2.0)
    F = grid.dft_matrix(ax.n, ax.L)
    H = F.conj().T @ np.diag(ax.k ** 2 / 2) @ F + ax.C.toarray() + np.diag(prob.potential(0.0))
    x = ax.x
    v = np.exp(-(x - 1.0) ** 2 + 0.5j * x)
    T = 0.4
    exact = sla.expm(-1j * H * T) @ v
    errs = []
    for nst in (8, 16, 32):
        tau = T / nst
        errs.append(np.linalg.norm(prob.propagate(v, tau, np.zeros(nst)) - exact))
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.1)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.1)


@pytest.mark.parametrize("kind", [contour.OFF, contour.SECS, contour.TFECS])
def test_free_gaussian_matches_closed_form_1d(kind):
    # Before the packet reaches R0, C acts on nothing: SO-FFT is exact for free motion.
    n, L = 512, 102.4
    ax = _axis(n, L, kind=kind, R0=40.0, theta=0.5)
    prob = tdse.Problem1D(ax, Zc=0.0)
    x0, k0, tau, nst = -3.0, 1.0, 0.05, 80
    psi0 = cf.free_gaussian(ax.x, 0.0, x0, k0)
    got = prob.propagate(psi0, tau, np.zeros(nst))
    want = cf.free_gaussian(ax.x, tau * nst, x0, k0)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-12


def test_free_gaussian_matches_closed_form_2d():
    ax, ay = _axis(160, 64.0, R0=26.0), _axis(128, 51.2, R0=20.0)
    prob = tdse.Problem2D(ax, ay, Zc=0.0)
    X, Y = ax.x[None, :], ay.x[:, None]
    g0 = cf.free_gaussian(X, 0.0, 1.0, 0.5) * cf.free_gaussian(Y, 0.0, -0.5, -0.3)
    tau, nst = 0.05, 40
    got = prob.propagate(g0, tau, np.zeros(nst))
    t = tau * nst
    want = cf.free_gaussian(X, t, 1.0, 0.5) * cf.free_gaussian(Y, t, -0.5, -0.3)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-12


def test_norm_is_conserved_without_ecs_and_with_real_potential():
    ax = _axis(256, 51.2, kind=contour.OFF)
    prob = tdse.Problem1D(ax, Zc=1.0, a2=2.0)
    psi0 = cf.free_gaussian(ax.x, 0.0, 0.0, 0.3)
    f = 0.05 * np.sin(0.3 * np.arange(400))
    psi = prob.propagate(psi0, 0.05, f)
    assert abs(np.linalg.norm(psi) / np.linalg.norm(psi0) - 1) < 1e-13


@pytest.mark.parametrize("kind,nst", [(contour.OFF, 200), (contour.SECS, 10)])
def test_time_reversal_recovers_the_initial_state(kind, nst):
    # Every factor, CN included, is inverted exactly by the step with -tau, so
    # running forward and then backward with the field reversed restores psi0.
    # With ECS the backward run undoes a damping of the fast modes in the
    # scaled layer that grows like exp(k^2 t), so it amplifies rounding noise;
    # a short run keeps that amplification below the tolerance.
    ax, ay = _axis(64, 25.6, kind=kind, R0=8.0), _axis(48, 19.2, kind=kind, R0=6.0)
    prob = tdse.Problem2D(ax, ay, Zc=1.0, a2=0.64)
    X, Y = ax.x[None, :], ay.x[:, None]
    psi0 = np.exp(-((X - 1) ** 2 + Y ** 2) / 2 + 1j * (0.8 * X - 0.4 * Y)) * (1 + 0.3j * Y)
    f = 0.05 * np.sin(0.2 * np.arange(nst))
    psi = prob.propagate(psi0, 0.05, f)
    back = prob.propagate(psi, -0.05, f[::-1])
    assert np.linalg.norm(back - psi0) / np.linalg.norm(psi0) < 1e-12
    assert np.linalg.norm(psi - psi0) / np.linalg.norm(psi0) > 1e-2


def test_ecs_absorbs_an_outgoing_packet_without_growth():
    ax = _axis(512, 102.4, R0=40.0, theta=0.5)
    prob = tdse.Problem1D(ax, Zc=0.0)
    psi = cf.free_gaussian(ax.x, 0.0, 0.0, 2.0)
    n0 = np.linalg.norm(psi)
    norms = []
    for _ in range(8):
        psi = prob.propagate(psi, 0.05, np.zeros(100))
        norms.append(np.linalg.norm(psi))
    assert max(norms) <= n0 * (1 + 1e-6)
    assert all(b <= a * (1 + 1e-6) for a, b in zip(norms, norms[1:]))
    # by t = 40 the bulk of the packet (k ~ 2 +- 1) has left through the ECS layer;
    # what remains are its slow components
    assert norms[-1] < 0.4 * n0


# ----------------------------------------------------------------- SSE / PCG
def _sse_1d(n=128, L=25.6, kind=contour.SECS, R0=8.0, E=0.7, Zc=1.0):
    ax = _axis(n, L, kind=kind, R0=R0, theta=0.5)
    V = tdse.softcore(Zc, 2.0, ax.z)
    return ax, sse.Operator((ax,), V, E)


def test_matvec_approximates_the_continuous_operator_on_smooth_functions():
    ax, op = _sse_1d(n=256, L=51.2, R0=20.0, E=0.3)
    x = ax.x
    f = np.exp(-x ** 2 / 2) * (1 + 0.2 * x)
    d2f = np.exp(-x ** 2 / 2) * ((x ** 2 - 1) * (1 + 0.2 * x) - 0.4 * x)
    V = tdse.softcore(1.0, 2.0, x.astype(complex))
    want = -0.5 * d2f + (V - 0.3) * f
    assert np.max(np.abs(op.matvec(f) - want)) < 1e-12


def test_operator_is_complex_symmetric():
    ax, ay = _axis(16, 6.4, R0=2.0), _axis(12, 4.8, R0=1.5)
    V = tdse.softcore(1.0, 0.64, ax.z[None, :], ay.z[:, None])
    op = sse.Operator((ax, ay), V, 0.9)
    A = op.dense()
    assert np.allclose(A, A.T, atol=1e-13)
    assert not np.allclose(A, A.conj().T, atol=1e-6)


def test_preconditioner_is_the_exact_inverse_without_ecs_and_potential():
    ax, op = _sse_1d(kind=contour.OFF, Zc=0.0, E=0.37)
    rng = np.random.default_rng(6)
    v = rng.normal(size=ax.n) + 1j * rng.normal(size=ax.n)
    assert np.allclose(op.precond(op.matvec(v)), v, atol=1e-12)
    x, it, res = sse.cocg(op, v, rtol=1e-12)
    assert it == 1 and res < 1e-12


@pytest.mark.parametrize("dim", [1, 2])
def test_cocg_matches_dense_gaussian_elimination(dim):
    rng = np.random.default_rng(7)
    if dim == 1:
        ax, op = _sse_1d(n=64, L=12.8, R0=4.0, E=0.8)
        f = rng.normal(size=64) + 1j * rng.normal(size=64)
    else:
        ax, ay = _axis(16, 6.4, R0=2.0), _axis(16, 6.4, R0=2.0)
        V = tdse.softcore(1.0, 0.64, ax.z[None, :], ay.z[:, None])
        op = sse.Operator((ax, ay), V, 0.6)
        f = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    x, it, res = sse.cocg(op, f, rtol=1e-13)
    xd = sse.dense_solve(op, f)
    assert res <= 1e-13
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


# The shifted divisor k^2/2 - E - i eta is an option outside the paper
# (eta = 0 is Eq. PreconFFT as printed); these pin the oracle's version of it.
def test_shifted_preconditioner_on_plane_waves():
    """Closed form: a grid plane wave exp(i(k_x x + k_y y)) is an eigenvector of
    the FFT preconditioner with eigenvalue 1/((k_x^2 + k_y^2)/2 - E - i eta)."""
    ax, ay = _axis(32, 12.8, R0=4.0), _axis(16, 6.4, R0=2.0)
    V = tdse.softcore(1.0, 0.64, ax.z[None, :], ay.z[:, None])
    E, eta = 0.8, 0.15
    op = sse.Operator((ax, ay), V, E, eta=eta)
    X, Y = np.meshgrid(ax.x, ay.x)
    for nx_, ny_ in ((0, 0), (3, 1), (-5, 2), (7, -6)):
        kx, ky = 2 * np.pi * nx_ / ax.L, 2 * np.pi * ny_ / ay.L
        v = np.exp(1j * (kx * X + ky * Y))
        want = v / ((kx ** 2 + ky ** 2) / 2 - E - 1j * eta)
        assert np.max(np.abs(op.precond(v) - want)) < 1e-12 * np.max(np.abs(want))


def test_shifted_preconditioner_is_complex_symmetric():
    ax, ay = _axis(8, 3.2, R0=1.0), _axis(6, 2.4, R0=0.8)
    op = sse.Operator((ax, ay), np.zeros((6, 8)), 0.5, eta=0.3)
    n = 48
    P = np.empty((n, n), dtype=complex)
    for j in range(n):
        e = np.zeros(n, dtype=complex)
        e[j] = 1.0
        P[:, j] = op.precond(e.reshape(6, 8)).ravel()
    assert np.allclose(P, P.T, atol=1e-14)
    assert not np.allclose(P, P.conj().T, atol=1e-6)


def test_shifted_cocg_reaches_the_dense_solution():
    """The shift changes the iterations, not the solution of Eq. linsys."""
    rng = np.random.default_rng(8)
    ax, ay = _axis(16, 6.4, R0=2.0), _axis(16, 6.4, R0=2.0)
    V = tdse.softcore(1.0, 0.64, ax.z[None, :], ay.z[:, None])
    f = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    xd = sse.dense_solve(sse.Operator((ax, ay), V, 0.6), f)
    its = []
    for eta in (0.0, 0.1, 0.4):
        x, it, res = sse.cocg(sse.Operator((ax, ay), V, 0.6, eta=eta), f, rtol=1e-13)
        assert res <= 1e-13
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10
        its.append(it)
    assert len(set(its)) > 1   # the shift is in effect



# ---- TFECS contour (Sec. IV, Eq. qTFECS)

def test_tfecs_y_small_s_series():
    """(1 - s)^-2 - (1 + s)^-2 = 4s + 8s^3 + 12s^5 + ..., so y(s) = alpha (8s^3 +
    12s^5 + 16s^7 + 20s^9 + ...): the s^3 onset the paper states."""
    s = np.array([0.01, 0.03, 0.05])
    series = 0.5 * (8 * s ** 3 + 12 * s ** 5 + 16 * s ** 7 + 20 * s ** 9)
    assert np.max(np.abs(contour.tfecs_y(s, 0.5) / series - 1)) < 1e-9
    # and the printed form of Eq. qTFECS, where it does not cancel
    t = np.array([0.3, 0.6, 0.9])
    printed = 0.5 * ((1 - t) ** -2 - (1 + t) ** -2 - 4 * t)
    assert np.max(np.abs(contour.tfecs_y(t, 0.5) / printed - 1)) < 1e-13


def test_tfecs_z_grows_like_the_papers_log_form():
    """z(x_N) ~ sqrt(alpha i) Dx ln(2 Dx/h) (Sec. IV): halving h at fixed Dx adds
    sqrt(alpha i) Dx ln 2, up to O(h^2) terms."""
    alpha, L, R0 = 0.5, 51.2, 20.0
    D = L / 2 - R0
    zN = [contour.z_of_x(np.array([L / 2 - h / 2]), contour.TFECS, R0, L / 2, alpha, h)[0]
          for h in (0.2, 0.1, 0.05)]
    want = np.sqrt(1j * alpha) * D * np.log(2.0)
    e1 = abs((zN[1] - zN[0]) - want) / abs(want)
    e2 = abs((zN[2] - zN[1]) - want) / abs(want)
    assert e1 < 1e-3 and e2 < 3e-4
    assert e1 / e2 == pytest.approx(4.0, rel=0.15)


def test_tfecs_z_derivative_is_q():
    """z(x) = int_0^x q (Eq. ECSintdef): central differences of z give q."""
    alpha, L, R0, h = 0.5, 25.6, 8.0, 0.1
    x = np.array([8.5, 10.0, 11.7, 12.5, -9.3])
    d = 1e-4
    zp = contour.z_of_x(x + d, contour.TFECS, R0, L / 2, alpha, h)
    zm = contour.z_of_x(x - d, contour.TFECS, R0, L / 2, alpha, h)
    q = contour.q_of_x(x, contour.TFECS, R0, L / 2, alpha, h)
    assert np.max(np.abs((zp - zm) / (2 * d) - q) / np.abs(q)) < 1e-6


def test_tfecs_box_edge_decouples_the_scaled_stencil():
    """q is infinite at the box edge, so K_s does not couple through it and C's
    coupling there is minus that of K_FD: C_{N,1} = C_{1,N} = 1/(2h^2)."""
    n, L = 128, 25.6
    ax = _axis(n, L, kind=contour.TFECS, R0=8.0, theta=0.5)
    assert np.isinf(ax.qm[-1].real)
    C = ax.C.toarray()
    c = 1.0 / (2 * ax.h ** 2)
    assert C[n - 1, 0] == c and C[0, n - 1] == c
    assert np.all(np.isfinite(C))


# ---- caller-supplied potential U = V0 + f(t) W on the grid

def test_constant_user_potential_adds_a_global_phase():
    """V0 = c (constant), W = 0: exp(-iUt) commutes with everything, so the
    state is the free one times exp(-i c t)."""
    ax, ay = _axis(64, 25.6, kind=contour.OFF, R0=8.0), _axis(48, 19.2, kind=contour.OFF, R0=6.0)
    psi0 = cf.free_gaussian(ax.x, 0.0, 0.5, 0.7)[None, :] * cf.free_gaussian(ay.x, 0.0, -0.3, 0.2)[:, None]
    c, tau, nst = 0.37 - 0.0j, 0.05, 40
    free = tdse.Problem2D(ax, ay, Zc=0.0).propagate(psi0, tau, np.zeros(nst))
    got = tdse.Problem2D(ax, ay, V0=np.full((48, 64), c), W=np.zeros((48, 64))).propagate(psi0, tau, np.zeros(nst))
    assert np.max(np.abs(got - free * np.exp(-1j * c * tau * nst))) < 1e-12


def test_uniform_field_along_y_shifts_the_mean_momentum():
    """U = f y (W = y, V0 = 0): by Ehrenfest d<p_y>/dt = -f exactly, while the
    packet stays away from the box edges."""
    ax, ay = _axis(64, 38.4, kind=contour.OFF, R0=8.0), _axis(64, 38.4, kind=contour.OFF, R0=8.0)
    psi0 = cf.free_gaussian(ax.x, 0.0, 0.0, 0.0)[None, :] * cf.free_gaussian(ay.x, 0.0, 0.0, 0.0)[:, None]
    f, tau, nst = 0.2, 0.02, 100
    prob = tdse.Problem2D(ax, ay, V0=np.zeros((64, 64)), W=np.broadcast_to(ay.x[:, None], (64, 64)))
    psi = prob.propagate(psi0, tau, np.full(nst, f))
    spec = np.fft.fft(psi, axis=0)
    ky = 2 * np.pi * np.fft.fftfreq(64, d=ay.h)
    py = np.sum(ky[:, None] * np.abs(spec) ** 2) / np.sum(np.abs(spec) ** 2)
    assert abs(py - (-f * tau * nst)) < 1e-10


# ---- soft-core potential at complex coordinates (Sec. II: U(z(x), t))

def test_softcore_hand_values():
    """Values worked out by hand, without a square root routine:
    V0(0) = -Zc/sqrt(a2); (1 + 2i)^2 = -3 + 4i and (1 - 2i)^2 = -3 - 4i, so on
    the principal branch sqrt(-3 +- 4i) = 1 +- 2i and V0 = -1/(1 +- 2i) =
    -(1 -+ 2i)/5; (0.8i)^2 + 0.64 = 0 removes the y term and a2."""
    assert tdse.softcore(1.0, 2.0, np.array([0.0j]))[0] == pytest.approx(-2 ** -0.5, abs=3e-16)
    assert tdse.softcore(1.0, 0.64, np.array([0.0j]), np.array([0.0j]))[0] == pytest.approx(-1.25, abs=1e-15)
    assert tdse.softcore(3.0, 0.25, np.array([0.0j]))[0] == pytest.approx(-6.0, abs=1e-15)
    zx = np.array([1 + 2j, 1 - 2j])
    zy = np.array([0.8j, 0.8j])
    got = tdse.softcore(1.0, 0.64, zx, zy)
    assert np.max(np.abs(got - np.array([-0.2 + 0.4j, -0.2 - 0.4j]))) < 1e-15
    # 1D with (2 + i)^2 = 3 + 4i and a2 = 2: sqrt(5 + 4i) is not simple, but
    # (2 + 1i)^2 + (-6 + 0i) = -3 + 4i, so a2 = -6 reaches the same value
    assert abs(tdse.softcore(2.0, -6.0, np.array([2 + 1j]))[0] - 2 * (-0.2 + 0.4j)) < 1e-15
    # the other branch would give -V0: Re sqrt > 0 is what is fixed here
    assert got[0].real < 0 and got[1].real < 0


def test_softcore_on_the_real_axis_and_far_away():
    """Interior nodes (q = 1, z = x) give the real -Zc/sqrt(x^2 + a2); far out
    along the scaled contour (|z| >> a) V0 approaches -Zc/z (Re z > 0)."""
    ax = _axis(256, 51.2, R0=20.0, theta=0.5)
    inner = np.abs(ax.x) < 20.0
    v = tdse.softcore(1.0, 2.0, ax.z)
    x = ax.x[inner]
    assert np.max(np.abs(v[inner].imag)) == 0.0
    assert np.max(np.abs(v[inner].real * np.sqrt(x * x + 2.0) + 1.0)) < 1e-15
    z = np.array([300.0 * np.exp(0.4j), 500.0 * np.exp(0.7j)])
    w = tdse.softcore(1.0, 0.64, z)
    assert np.max(np.abs(w * z + 1.0)) < 1e-5        # -1/z (1 - a2/(2 z^2) + ...)
