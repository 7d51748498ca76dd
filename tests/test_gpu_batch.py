"""GPU parity of the batched uneven propagation (sofft_batch_*, via the C ABI).

Every run of a batch is checked element by element: against the FP64 oracle
on small grids (relative L2 <= 1e-10 in FP64, <= 1e-5 for complex64 states),
and against the single-grid path of the same library, which must agree
bit for bit (the same kernels apply the same arithmetic to every line,
whatever the launch shape, graph replay or batch composition).  The full
96-run workload is checked on sampled runs: the smallest against the oracle,
one of every other size against the single-grid path, and all norms."""
import numpy as np
import pytest

from oracle import tdse as ot
from paper_1505_06707_amd import workloads as wl
from tests.helpers import CONTOURS, oracle_axis, outgoing_state, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


def _sofft():
    from paper_1505_06707_amd import sofft
    return sofft


def _runs_small():
    # uneven shapes, several runs per shape, per-run pulses and packets
    spec = [(64, 0), (96, 1), (64, 2), (128, 3), (96, 4), (64, 5), (48, 6)]
    out = []
    for n, seed in spec:
        rng = np.random.default_rng(100 + seed)
        out.append(dict(n=n, pulse=wl.Pulse(E0=float(rng.uniform(0.02, 0.1)), omega=float(rng.uniform(0.2, 0.4)),
                                            cycles=2), packet_seed=seed))
    return out


def _problem(s, n, dtype):
    h = 0.2
    L = n * h
    return s.problem([n, n], [L, L], R0=[0.8 * L / 2] * 2, theta=0.5, charge=1.0, a2=0.64, dtype=dtype)


def _inputs(runs, dt, nsteps):
    psi0, f = [], []
    for r in runs:
        n = r["n"]
        x = ot.Axis(n, n * 0.2).x
        psi0.append(wl.gaussian_2d(x, x, **wl.packet_params(r["packet_seed"])))
        f.append(r["pulse"].at_midpoints(0.0, dt, nsteps))
    return psi0, np.stack(f)


def _batch_run(runs, dtype, dt, nsteps, graph_steps=None, shapes=None, field=True):
    s = _sofft()
    cdt = np.complex128 if dtype == s.C128 else np.complex64
    psi0, f = _inputs(runs, dt, nsteps)
    b = s.Batch([_problem(s, r["n"], dtype) for r in runs])
    if graph_steps is not None:
        b.set_graph_steps(graph_steps)
    if shapes is not None:
        for r in range(len(runs)):
            for p in (0, 1):
                b.set_launch_shape(r, p, *shapes)
    states = [torch.from_numpy(p.astype(cdt)).cuda() for p in psi0]
    fd = torch.from_numpy(f).cuda() if field else None
    norms = b.propagate(states, dt, nsteps, fd)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in states]
    b.close()
    return out, norms, psi0, f


def _single_run(n, dtype, psi0, f, dt):
    s = _sofft()
    cdt = np.complex128 if dtype == s.C128 else np.complex64
    plan = s.Plan([n, n], [n * 0.2] * 2, R0=[0.8 * n * 0.2 / 2] * 2, theta=0.5, charge=1.0, a2=0.64, dtype=dtype)
    psi = torch.from_numpy(psi0.astype(cdt)).cuda()
    fd = torch.from_numpy(np.ascontiguousarray(f)).cuda() if f is not None else None
    plan.propagate(psi, dt, len(f) if f is not None else 0, fd)
    torch.cuda.synchronize()
    out = psi.cpu().numpy()
    plan.close()
    return out


def _oracle(n, psi0, f, dt):
    ax = oracle_axis(n, n * 0.2, 0.8 * n * 0.2 / 2, 0.5, "secs")
    return ot.Problem2D(ax, ax, Zc=1.0, a2=0.64).propagate(psi0, dt, f)


@pytest.mark.parametrize("graph_steps", [0, 8])
def test_batch_matches_oracle_and_single_grid_fp64(graph_steps):
    s = _sofft()
    runs = _runs_small()
    print(f"batch c128 {len(runs)} runs x 40 steps, graph_steps={graph_steps}", flush=True)
    out, norms, psi0, f = _batch_run(runs, s.C128, 0.05, 40, graph_steps=graph_steps)
    for r, run in enumerate(runs):
        single = _single_run(run["n"], s.C128, psi0[r], f[r], 0.05)
        assert np.array_equal(out[r], single), f"run {r} differs from the single-grid path"
        assert abs(norms[r] - np.vdot(single, single).real) <= 1e-12 * norms[r]
    for r in (0, 1, 3, 6):   # one of every shape against the oracle
        o = _oracle(runs[r]["n"], psi0[r], f[r], 0.05)
        err = rel_l2(out[r], o)
        print(f"   run {r} n={runs[r]['n']}: rel L2 vs oracle {err:.2e}", flush=True)
        assert err < TOL64


@pytest.mark.parametrize("shape", [(256, 0), (512, 0), (1024, 0), (256, 3), (512, 1), (1024, 5)])
def test_launch_shapes_agree_bitwise(shape):
    s = _sofft()
    runs = _runs_small()
    print(f"launch shape threads={shape[0]} grid={shape[1]}", flush=True)
    ref, _, _, _ = _batch_run(runs, s.C128, 0.05, 12, graph_steps=0, shapes=(256, 0))
    out, _, _, _ = _batch_run(runs, s.C128, 0.05, 12, graph_steps=4, shapes=shape)
    for r in range(len(runs)):
        assert np.array_equal(out[r], ref[r]), f"run {r}"


def test_batch_fp32_against_oracle():
    s = _sofft()
    runs = _runs_small()[:4]
    print("batch c64 4 runs x 300 steps", flush=True)
    out, norms, psi0, f = _batch_run(runs, s.C64, 0.05, 300)
    for r, run in enumerate(runs):
        o = _oracle(run["n"], psi0[r], f[r], 0.05)
        err = rel_l2(out[r].astype(np.complex128), o)
        print(f"   run {r} n={run['n']}: rel L2 vs oracle {err:.2e}", flush=True)
        assert err < TOL32
        assert abs(norms[r] - np.vdot(o, o).real) < 1e-5 * np.vdot(o, o).real


def test_batch_without_field_and_edge_counts():
    s = _sofft()
    runs = _runs_small()[:3]
    for nsteps in (0, 1, 2, 3):
        out, norms, psi0, f = _batch_run(runs, s.C128, 0.05, nsteps, graph_steps=1, field=False)
        for r, run in enumerate(runs):
            single = _single_run(run["n"], s.C128, psi0[r], np.zeros(nsteps), 0.05)
            if nsteps == 0:
                assert np.array_equal(out[r], psi0[r])
            assert np.array_equal(out[r], single), f"nsteps={nsteps} run {r}"


def test_batch_rejects_bad_arguments():
    s = _sofft()
    p2 = _problem(s, 64, s.C128)
    p1 = s.problem([64], [12.8], dtype=s.C128)
    with pytest.raises(s.SofftError):
        s.Batch([p2, p1])
    with pytest.raises(s.SofftError):
        s.Batch([p2, _problem(s, 64, s.C64)])
    b = s.Batch([p2])
    with pytest.raises(s.SofftError):
        b.set_launch_shape(0, 0, 100, 0)
    with pytest.raises(s.SofftError):
        b.set_graph_steps(-1)
    b.close()


def test_full_batch_workload_sampled():
    """96 uneven complex64 runs x 1000 steps (the batched workload) in the
    launch configuration the benchmark uses (autotuned shapes, graph replays)."""
    s = _sofft()
    runs = wl.batch_runs(seed=2024)
    dt, nsteps = 0.05, 1000
    print(f"full batch: {len(runs)} runs, sizes {sorted(set(r['n'] for r in runs))}, {nsteps} steps", flush=True)
    out, norms, psi0, f = _batch_run(runs, s.C64, dt, nsteps)
    assert np.all(np.isfinite(norms))
    n0 = np.array([np.vdot(p, p).real for p in psi0])
    assert np.all(norms <= n0 * (1 + 1e-6))
    picked = {}
    for r, run in enumerate(runs):
        picked.setdefault(run["n"], r)
    small = picked[min(picked)]
    o = _oracle(runs[small]["n"], psi0[small], f[small], dt)
    err = rel_l2(out[small].astype(np.complex128), o)
    print(f"   run {small} n={runs[small]['n']}: rel L2 vs oracle {err:.2e}", flush=True)
    assert err < TOL32
    for n, r in sorted(picked.items()):
        if n == min(picked):
            continue
        single = _single_run(n, s.C64, psi0[r], f[r], dt)
        assert np.array_equal(out[r], single), f"run {r} (n={n}) differs from the single-grid path"
        print(f"   run {r} n={n}: equal to the single-grid path", flush=True)



def test_batch_mixed_contours_with_tfecs():
    """Runs with the SECS and the TFECS contour (different problem statements,
    hence different classes, even at the same shape) advanced by one batch:
    each run equals its single-grid propagation bit for bit and the oracle."""
    s = _sofft()
    specs = [(64, "secs"), (64, "tfecs"), (96, "tfecs")]
    dt, nsteps = 0.05, 40
    problems, psi0, fs = [], [], []
    for i, (n, kind) in enumerate(specs):
        L = n * 0.2
        problems.append(s.problem([n, n], [L, L], R0=[0.8 * L / 2] * 2, theta=0.5, contour=CONTOURS[kind][1],
                                  charge=1.0, a2=0.64, dtype=s.C128))
        x = ot.Axis(n, L).x
        psi0.append(wl.gaussian_2d(x, x, **wl.packet_params(20 + i)))
        fs.append(wl.Pulse(E0=0.05, omega=0.3, cycles=2).at_midpoints(0.0, dt, nsteps))
    print("batch with SECS and TFECS runs", flush=True)
    b = s.Batch(problems)
    states = [torch.from_numpy(p.astype(np.complex128)).cuda() for p in psi0]
    b.propagate(states, dt, nsteps, torch.from_numpy(np.stack(fs)).cuda())
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in states]
    b.close()
    for i, (n, kind) in enumerate(specs):
        L = n * 0.2
        plan = s.Plan([n, n], [L, L], R0=[0.8 * L / 2] * 2, theta=0.5, contour=CONTOURS[kind][1], charge=1.0, a2=0.64)
        psi = torch.from_numpy(psi0[i].astype(np.complex128)).cuda()
        plan.propagate(psi, dt, nsteps, torch.from_numpy(fs[i]).cuda())
        torch.cuda.synchronize()
        single = psi.cpu().numpy()
        plan.close()
        assert np.array_equal(out[i], single), f"run {i} ({kind}) differs from the single-grid path"
        ax = oracle_axis(n, L, 0.8 * L / 2, 0.5, kind)
        o = ot.Problem2D(ax, ax, Zc=1.0, a2=0.64).propagate(psi0[i], dt, fs[i])
        err = rel_l2(out[i], o)
        print(f"   run {i} n={n} {kind}: rel L2 vs oracle {err:.2e}", flush=True)
        assert err < TOL64


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_batch_large_shapes_against_oracle(dtype):
    """Runs of 512^2, 768^2 and 1024^2 (two of each, launch shapes tuned as in
    the benchmark, steps replayed from the graph) against the oracle, with
    packets driven into the ECS strips of both axes."""
    s = _sofft()
    dt, nsteps = 0.05, 24
    sizes = [512, 768, 1024, 512, 768, 1024]
    problems, psi0, fs = [], [], []
    for i, n in enumerate(sizes):
        L = n * 0.2
        problems.append(_problem(s, n, s.C64 if dtype == "c64" else s.C128))
        ax = ot.Axis(n, L, R0=0.8 * L / 2)
        psi0.append(outgoing_state(ax, ax, speed=2.0 + 0.5 * (i % 3), inset=1.5))
        fs.append(wl.Pulse(E0=0.05 + 0.01 * i, omega=0.3, cycles=2).at_midpoints(0.0, dt, nsteps))
    print(f"batch {dtype} runs {sizes} x {nsteps} steps, strips", flush=True)
    cdt = np.complex64 if dtype == "c64" else np.complex128
    b = s.Batch(problems)
    b.set_graph_steps(8)
    states = [torch.from_numpy(p.astype(cdt)).cuda() for p in psi0]
    b.propagate(states, dt, nsteps, torch.from_numpy(np.stack(fs)).cuda(), norms=False)
    torch.cuda.synchronize()
    out = [t.cpu().numpy().astype(np.complex128) for t in states]
    b.close()
    for i in (0, 1, 2):
        n = sizes[i]
        o = _oracle(n, psi0[i], fs[i], dt)
        err = rel_l2(out[i], o)
        print(f"   run {i} n={n}: rel L2 vs oracle {err:.2e}", flush=True)
        assert err < (TOL32 if dtype == "c64" else TOL64)
