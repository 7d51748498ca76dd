"""sofft_propagate_static (no allocation, static device scratch) against
sofft_propagate (bound workspace): bit-identical results on two calls in a
row, the second on a smaller grid, called through the C ABI; a caller's
potential too large for the static scratch is rejected."""
import ctypes

import numpy as np
import pytest

from paper_1505_06707_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _sofft():
    from paper_1505_06707_amd import sofft
    return sofft


def _case(s, n, dtype, seed, nsteps):
    h = 0.2
    L = n * h
    plan = s.Plan([n, n], [L, L], R0=[0.8 * L / 2] * 2, theta=0.5, charge=1.0, a2=0.64, dtype=dtype)
    x = plan.nodes(0)
    psi0 = wl.gaussian_2d(x, x, **wl.packet_params(seed))
    f = torch.from_numpy(wl.Pulse(E0=0.06, omega=0.2, cycles=2).at_midpoints(0.0, 0.05, nsteps)).cuda()
    cdt = np.complex128 if dtype == s.C128 else np.complex64
    return plan, torch.from_numpy(psi0.astype(cdt)).cuda(), f


@pytest.mark.parametrize("dtype", [0, 1])
def test_static_scratch_matches_workspace_path(dtype):
    s = _sofft()
    L = s.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n, seed, nsteps in ((512, 3, 40), (128, 4, 25)):   # second call: a smaller input
        print(f"no-alloc propagate {n}^2 dtype={dtype} x {nsteps}", flush=True)
        plan, psi, f = _case(s, n, dtype, seed, nsteps)
        ref = psi.clone()
        plan.propagate(ref, 0.05, nsteps, f)
        got = psi.clone()
        assert L.sofft_propagate_static(plan._h, ctypes.c_void_p(got.data_ptr()), 0.05, nsteps,
                                        ctypes.c_void_p(f.data_ptr()), stream) == 0
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy())
        plan.close()


def test_static_scratch_rejects_a_table_beyond_its_size():
    s = _sofft()
    L = s.lib()
    n = 1024
    plan = s.Plan([n, n], [n * 0.2] * 2, R0=[0.8 * n * 0.1] * 2, theta=0.5, charge=1.0, a2=0.64)
    v0 = plan.make_softcore(1.0, 0.64)
    plan.set_potential(v0, None)        # a whole-grid table: 16 MiB > 8 MiB
    psi = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.sofft_propagate_static(plan._h, ctypes.c_void_p(psi.data_ptr()), 0.05, 2, None, stream) == -2
    assert b"static scratch" in L.sofft_last_error()
    plan.close()
