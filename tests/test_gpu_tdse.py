"""GPU parity of the SO-FFT + ECS propagation (HIP library via the C ABI)
against the FP64 oracle, element by element on the same seeded inputs.

Tolerance (FP64 mode): relative L2 <= 1e-10 after the whole run, the bound
the method's FP64 target states; single steps agree to ~1e-14."""
import numpy as np
import pytest

from oracle import tdse as ot
from paper_1505_06707_amd import workloads as wl
from tests.helpers import CONTOURS, oracle_axis, outgoing_state, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _sofft():
    from paper_1505_06707_amd import sofft
    return sofft


def _dev(a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def run_gpu_1d(n, L, R0, theta, kind, charge, a2, psi0, dt, f_mid):
    s = _sofft()
    plan = s.Plan(n, L, R0=R0, theta=theta, contour=CONTOURS[kind][1], charge=charge, a2=a2, dtype=s.C128)
    psi = _dev(psi0.astype(np.complex128))
    f = _dev(np.asarray(f_mid, dtype=np.float64)) if len(f_mid) else None
    plan.propagate(psi, dt, len(f_mid), f)
    torch.cuda.synchronize()
    out = psi.cpu().numpy()
    plan.close()
    return out


def run_gpu_2d(nx, ny, Lx, Ly, R0x, R0y, theta, kind, charge, a2, psi0, dt, f_mid, dtype=None):
    s = _sofft()
    dtype = s.C128 if dtype is None else dtype
    plan = s.Plan([nx, ny], [Lx, Ly], R0=[R0x, R0y], theta=theta, contour=CONTOURS[kind][1],
                  charge=charge, a2=a2, dtype=dtype)
    cdt = np.complex128 if dtype == s.C128 else np.complex64
    psi = _dev(psi0.astype(cdt))
    f = _dev(np.asarray(f_mid, dtype=np.float64)) if len(f_mid) else None
    plan.propagate(psi, dt, len(f_mid), f)
    torch.cuda.synchronize()
    out = psi.cpu().numpy().astype(np.complex128)
    plan.close()
    return out


def oracle_1d(n, L, R0, theta, kind, charge, a2, psi0, dt, f_mid):
    ax = oracle_axis(n, L, R0, theta, kind)
    return ot.Problem1D(ax, Zc=charge, a2=a2).propagate(psi0, dt, f_mid)


def oracle_2d(nx, ny, Lx, Ly, R0x, R0y, theta, kind, charge, a2, psi0, dt, f_mid):
    ax = oracle_axis(nx, Lx, R0x, theta, kind)
    ay = oracle_axis(ny, Ly, R0y, theta, kind)
    return ot.Problem2D(ax, ay, Zc=charge, a2=a2).propagate(psi0, dt, f_mid)


@pytest.mark.parametrize("n", [16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 2048])
def test_1d_parity_all_lengths(n):
    print(f"1D n={n}", flush=True)
    h = 0.2
    L = n * h
    R0 = 0.7 * L / 2
    x = ot.Axis(n, L, R0=R0).x
    psi0 = wl.gaussian_1d(x, x0=0.3, k0=1.5) * (1 + 0.1j * x)
    f = wl.Pulse(E0=0.05, omega=0.3, cycles=2).at_midpoints(0.0, 0.05, 60)
    args = (n, L, R0, 0.5, "secs", 1.0, 2.0, psi0, 0.05, f)
    g = run_gpu_1d(*args)
    o = oracle_1d(*args)
    assert rel_l2(g, o) < TOL64


@pytest.mark.parametrize("kind", ["secs", "sharp", "off", "tfecs"])
def test_1d_parity_contours(kind):
    print(f"1D contour={kind}", flush=True)
    n, L, R0 = 512, 102.4, 30.0
    x = ot.Axis(n, L, R0=R0).x
    psi0 = wl.gaussian_1d(x, x0=-1.0, k0=2.0)
    f = wl.Pulse(E0=0.05, omega=0.2, cycles=2).at_midpoints(0.0, 0.05, 400)
    args = (n, L, R0, 0.4, kind, 1.0, 2.0, psi0, 0.05, f)
    assert rel_l2(run_gpu_1d(*args), oracle_1d(*args)) < TOL64


def test_1d_full_workload_parity():
    """The 1D workload at full size: N = 4096, 4000 steps of the laser pulse."""
    c = wl.TDSE_1D
    print("1D full 4096 x 4000", flush=True)
    x = ot.Axis(c.n, c.L, R0=c.R0).x
    psi0 = wl.gaussian_1d(x)
    f = c.pulse.at_midpoints(0.0, c.dt, c.nsteps)
    args = (c.n, c.L, c.R0, c.theta, "secs", c.charge, c.a2, psi0, c.dt, f)
    g = run_gpu_1d(*args)
    o = oracle_1d(*args)
    assert rel_l2(g, o) < TOL64
    assert np.linalg.norm(g) < np.linalg.norm(psi0)


@pytest.mark.parametrize("nx,ny", [(64, 48), (128, 128), (384, 256), (32, 768), (1024, 16)])
def test_2d_parity_shapes(nx, ny):
    print(f"2D {nx}x{ny}", flush=True)
    h = 0.2
    Lx, Ly = nx * h, ny * h
    R0x, R0y = 0.8 * Lx / 2, 0.75 * Ly / 2
    ax, ay = ot.Axis(nx, Lx, R0=R0x), ot.Axis(ny, Ly, R0=R0y)
    prm = wl.packet_params(seed=nx * 7 + ny)
    psi0 = wl.gaussian_2d(ax.x, ay.x, **prm)
    f = wl.Pulse(E0=0.08, omega=0.3, cycles=2).at_midpoints(0.0, 0.05, 40)
    args = (nx, ny, Lx, Ly, R0x, R0y, 0.5, "secs", 1.0, 0.64, psi0, 0.05, f)
    assert rel_l2(run_gpu_2d(*args), oracle_2d(*args)) < TOL64


def test_2d_tfecs_parity():
    """TFECS on both axes (Eq. qTFECS, alpha = 0.5): a packet driven into the
    scaled strips, with the soft-core potential and the pulse."""
    print("2D TFECS 128x96", flush=True)
    nx, ny, h = 128, 96, 0.2
    Lx, Ly = nx * h, ny * h
    R0x, R0y = 0.7 * Lx / 2, 0.7 * Ly / 2
    ax, ay = ot.Axis(nx, Lx, R0=R0x), ot.Axis(ny, Ly, R0=R0y)
    psi0 = wl.gaussian_2d(ax.x, ay.x, x0=0.5, y0=-0.3, px=2.0, py=-1.5)
    f = wl.Pulse(E0=0.05, omega=0.3, cycles=2).at_midpoints(0.0, 0.05, 120)
    args = (nx, ny, Lx, Ly, R0x, R0y, 0.5, "tfecs", 1.0, 0.64, psi0, 0.05, f)
    g = run_gpu_2d(*args)
    o = oracle_2d(*args)
    assert rel_l2(g, o) < TOL64
    assert np.linalg.norm(g) < np.linalg.norm(psi0)   # the strips absorb


def test_2d_full_size_parity_few_steps():
    """The 2D workload grid (1024^2, h = 0.2, SECS from 80% of the half-width)
    in the launch configuration the benchmark times, for 8 steps."""
    c = wl.TDSE_2D
    print("2D full grid 1024^2 x 8 steps", flush=True)
    ax = ot.Axis(c.n, c.L, R0=c.R0)
    psi0 = wl.gaussian_2d(ax.x, ax.x, **wl.packet_params(seed=1))
    f = c.pulse.at_midpoints(0.0, c.dt, 8)
    args = (c.n, c.n, c.L, c.L, c.R0, c.R0, c.theta, "secs", c.charge, c.a2, psi0, c.dt, f)
    assert rel_l2(run_gpu_2d(*args), oracle_2d(*args)) < TOL64


def test_2d_free_gaussian_closed_form_on_gpu():
    # Independent of the oracle: free spreading of a Gaussian before it reaches R0.
    from tests import closed_forms as cf
    nx, ny, h = 256, 256, 0.2
    L = nx * h
    x = ot.Axis(nx, L, R0=20.0).x
    X, Y = x[None, :], x[:, None]
    g0 = cf.free_gaussian(X, 0.0, 0.5, 0.7) * cf.free_gaussian(Y, 0.0, -0.3, -0.4)
    out = run_gpu_2d(nx, ny, L, L, 20.0, 20.0, 0.5, "secs", 0.0, 0.64, g0, 0.05, np.zeros(40))
    want = cf.free_gaussian(X, 2.0, 0.5, 0.7) * cf.free_gaussian(Y, 2.0, -0.3, -0.4)
    assert rel_l2(out, want) < 1e-12


def test_2d_time_reversal_on_gpu():
    nx, ny, h = 128, 96, 0.2
    Lx, Ly = nx * h, ny * h
    ax, ay = ot.Axis(nx, Lx, R0=10.0), ot.Axis(ny, Ly, R0=7.5)
    psi0 = wl.gaussian_2d(ax.x, ay.x, x0=0.5, y0=-0.2, px=0.3, py=0.1)
    f = 0.05 * np.sin(0.2 * np.arange(10))
    fwd = run_gpu_2d(nx, ny, Lx, Ly, 10.0, 7.5, 0.5, "secs", 1.0, 0.64, psi0, 0.05, f)
    back = run_gpu_2d(nx, ny, Lx, Ly, 10.0, 7.5, 0.5, "secs", 1.0, 0.64, fwd, -0.05, f[::-1])
    # The backward run undoes the damping of fast modes in the thin scaled
    # layer (h = 0.2 here), which amplifies rounding noise to ~1e-11.
    assert rel_l2(back, psi0) < 1e-10
    assert rel_l2(fwd, psi0) > 1e-2


def test_norm2_and_zero_steps():
    s = _sofft()
    plan = s.Plan([128, 64], [25.6, 12.8], R0=[10.0, 5.0], dtype=s.C128)
    rng = np.random.default_rng(3)
    a = rng.normal(size=(64, 128)) + 1j * rng.normal(size=(64, 128))
    psi = _dev(a)
    assert plan.norm2(psi) == pytest.approx(np.sum(np.abs(a) ** 2), rel=1e-14)
    plan.propagate(psi, 0.05, 0, None)
    torch.cuda.synchronize()
    assert np.array_equal(psi.cpu().numpy(), a)
    plan.close()


# ---------------------------------------------------------------- FP32 mode
# complex64 state in HBM, FP64 arithmetic and tables on chip (the state is
# rounded to FP32 once per pass).  Error against the FP64 oracle, stated per
# result; the FP32 target is 1e-5 relative L2.
TOL32 = 1e-5


def test_fp32_2d_tfecs_against_fp64_oracle():
    """complex64 state on the TFECS contour (large |q| near the box edges)."""
    from paper_1505_06707_amd import sofft
    print("2D c64 TFECS 128^2 x 1000", flush=True)
    n, h = 128, 0.2
    L = n * h
    R0 = 0.7 * L / 2
    ax = ot.Axis(n, L, R0=R0)
    psi0 = wl.gaussian_2d(ax.x, ax.x, x0=0.3, y0=-0.2, px=1.5, py=1.0)
    f = wl.Pulse().at_midpoints(0.0, 0.05, 1000)
    args = (n, n, L, L, R0, R0, 0.5, "tfecs", 1.0, 0.64, psi0, 0.05, f)
    g = run_gpu_2d(*args, dtype=sofft.C64)
    o = oracle_2d(*args)
    err = rel_l2(g, o)
    print(f"   rel L2 (c64 vs FP64 oracle) = {err:.3e}", flush=True)
    assert err < TOL32


@pytest.mark.parametrize("n,steps", [(128, 2000), (256, 500)])
def test_fp32_2d_error_against_fp64_oracle(n, steps):
    from paper_1505_06707_amd import sofft
    print(f"2D c64 {n}^2 x {steps}", flush=True)
    h = 0.2
    L = n * h
    R0 = 0.8 * L / 2
    ax = ot.Axis(n, L, R0=R0)
    psi0 = wl.gaussian_2d(ax.x, ax.x, **wl.packet_params(seed=n))
    f = wl.Pulse().at_midpoints(0.0, 0.05, steps)
    args = (n, n, L, L, R0, R0, 0.5, "secs", 1.0, 0.64, psi0, 0.05, f)
    g = run_gpu_2d(*args, dtype=sofft.C64)
    o = oracle_2d(*args)
    err = rel_l2(g, o)
    print(f"   rel L2 (c64 vs FP64 oracle) = {err:.3e}", flush=True)
    assert err < TOL32


def test_fp32_1d_error_against_fp64_oracle():
    from paper_1505_06707_amd import sofft
    c = wl.TDSE_1D
    x = ot.Axis(c.n, c.L, R0=c.R0).x
    psi0 = wl.gaussian_1d(x)
    f = c.pulse.at_midpoints(0.0, c.dt, c.nsteps)
    plan = sofft.Plan(c.n, c.L, R0=c.R0, theta=c.theta, charge=c.charge, a2=c.a2, dtype=sofft.C64)
    psi = _dev(psi0.astype(np.complex64))
    plan.propagate(psi, c.dt, c.nsteps, _dev(f))
    torch.cuda.synchronize()
    g = psi.cpu().numpy().astype(np.complex128)
    plan.close()
    o = oracle_1d(c.n, c.L, c.R0, c.theta, "secs", c.charge, c.a2, psi0, c.dt, f)
    err = rel_l2(g, o)
    print(f"   1D c64 4096 x 4000: rel L2 = {err:.3e}", flush=True)
    assert err < TOL32


# ---------------------------------------------------------------- ECS strips
# Packets started a few units inside R0 and moving outward put real amplitude
# on the exterior strips, so the Crank-Nicolson solve of the remainder C
# (Sec. II, Eq. C_FD and the CN formula) acts on data, at the line lengths the
# full-size grids use: the row pass's PCR with several wavefronts per line
# (512-, 768- and 1024-point rows) and the column pass's edge-slot CN.


# (1024, 64) runs the row pass's XCD row groups (one row per block, 64 rows a
# multiple of 8 groups at complex128 and complex64) and the column pass's
# column-block groups, as the full-size grid does; (1024, 16) keeps the
# identity row map.
STRIP_SHAPES = [(1024, 16), (1024, 64), (16, 1024), (512, 32), (32, 512), (768, 48), (48, 768), (384, 64)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nx,ny", STRIP_SHAPES)
def test_2d_parity_with_amplitude_on_the_strips(nx, ny, dtype):
    s = _sofft()
    print(f"2D strips {nx}x{ny} {dtype}", flush=True)
    h = 0.2
    Lx, Ly = nx * h, ny * h
    R0x, R0y = 0.8 * Lx / 2, 0.8 * Ly / 2
    ax, ay = ot.Axis(nx, Lx, R0=R0x), ot.Axis(ny, Ly, R0=R0y)
    psi0 = outgoing_state(ax, ay)
    f = wl.Pulse(E0=0.08, omega=0.3, cycles=2).at_midpoints(0.0, 0.05, 80)
    args = (nx, ny, Lx, Ly, R0x, R0y, 0.5, "secs", 1.0, 0.64, psi0, 0.05, f)
    o = oracle_2d(*args)
    # the long axis's strips took real amplitude: part of the norm is gone
    strip = (np.abs(ax.x)[None, :] > R0x) | (np.abs(ay.x)[:, None] > R0y)
    assert np.linalg.norm(o[strip]) > 0.05 * np.linalg.norm(o)
    assert np.linalg.norm(o) < 0.97 * np.linalg.norm(psi0)
    g = run_gpu_2d(*args, dtype=s.C128 if dtype == "c128" else s.C64)
    err = rel_l2(g, o)
    print(f"   rel L2 = {err:.3e}", flush=True)
    assert err < (TOL64 if dtype == "c128" else 1e-5)


def test_2d_full_size_parity_amplitude_on_the_strips():
    """The 1024^2 workload grid in the benchmark's launch configuration, with
    packets driven into the x- and y-strips (40 steps)."""
    c = wl.TDSE_2D
    print("2D full grid 1024^2, strips, 40 steps", flush=True)
    ax = ot.Axis(c.n, c.L, R0=c.R0)
    psi0 = outgoing_state(ax, ax, speed=3.0, inset=2.0)
    f = c.pulse.at_midpoints(0.0, c.dt, 40)
    args = (c.n, c.n, c.L, c.L, c.R0, c.R0, c.theta, "secs", c.charge, c.a2, psi0, c.dt, f)
    o = oracle_2d(*args)
    strip = (np.abs(ax.x)[None, :] > c.R0) | (np.abs(ax.x)[:, None] > c.R0)
    assert np.linalg.norm(o[strip]) > 0.1 * np.linalg.norm(o)
    assert rel_l2(run_gpu_2d(*args), o) < TOL64


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_2d_full_workload_against_stored_oracle_checkpoints(dtype):
    """The whole 2D workload (1024^2, 2000 steps of the pulse, packet seed 1)
    against the FP64 oracle's state after 100, 500, 1000 and 2000 steps, stored
    at 8192 seeded grid points with the squared norm of the whole state
    (tests/golden/make_tdse_2d_1024_checkpoints.py, which calls only the
    oracle).  complex128: relative L2 over the samples <= 1e-10; complex64
    (FP32 storage, FP64 arithmetic on chip): <= 1e-5 at every checkpoint."""
    import os
    s = _sofft()
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "tdse_2d_1024_checkpoints.npz"))
    c = wl.TDSE_2D
    ax = ot.Axis(c.n, c.L, R0=c.R0)
    psi0 = wl.gaussian_2d(ax.x, ax.x, **wl.packet_params(int(gold["packet_seed"])))
    f = c.pulse.at_midpoints(0.0, c.dt, int(gold["steps"][-1]))
    dt_ = s.C128 if dtype == "c128" else s.C64
    plan = s.Plan([c.n, c.n], [c.L, c.L], R0=[c.R0, c.R0], theta=c.theta, charge=c.charge, a2=c.a2, dtype=dt_)
    psi = _dev(psi0.astype(np.complex128 if dtype == "c128" else np.complex64))
    fd = _dev(f)
    tol = TOL64 if dtype == "c128" else TOL32
    done = 0
    for k, step in enumerate(gold["steps"]):
        step = int(step)
        print(f"2D 1024^2 {dtype}: steps {done}..{step}", flush=True)
        plan.propagate(psi, c.dt, step - done, fd[done:step])
        done = step
        torch.cuda.synchronize()
        got = psi.cpu().numpy().astype(np.complex128).ravel()[gold["index"]]
        err = rel_l2(got, gold["samples"][k])
        nerr = abs(plan.norm2(psi) - gold["norm2"][k]) / gold["norm2"][k]
        print(f"   step {step}: rel L2 on samples {err:.3e}, norm^2 rel error {nerr:.3e}", flush=True)
        assert err < tol and nerr < tol
    plan.close()
