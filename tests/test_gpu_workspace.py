"""The caller-owned workspace of plans and batches (include/sofft.h: ownership
of device memory).  Without a bound workspace of the size the call needs, the
calls fail with SOFFT_EWORKSPACE and leave their outputs untouched; with one
bound by the caller they give exactly what the binding's own workspace gives."""
import ctypes

import numpy as np
import pytest

from paper_1505_06707_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EWORKSPACE = -5


def _sofft():
    from paper_1505_06707_amd import sofft
    return sofft


def _raw_plan(s, n=64, dtype=0):
    p = s.problem([n, n], [n * 0.2] * 2, R0=[0.8 * n * 0.2 / 2] * 2, theta=0.5, charge=1.0, a2=0.64, dtype=dtype)
    h = ctypes.c_void_p()
    assert s.lib().sofft_plan_create(ctypes.byref(p), ctypes.byref(h)) == 0
    return h


def _size(s, h, nE):
    b = ctypes.c_int64()
    assert s.lib().sofft_workspace_size(h, nE, ctypes.byref(b)) == 0
    return b.value


def test_calls_without_workspace_fail_and_enqueue_nothing():
    s = _sofft()
    L = s.lib()
    h = _raw_plan(s)
    print("workspace: unbound plan", flush=True)
    rng = np.random.default_rng(0)
    a = rng.normal(size=(64, 64)) + 1j * rng.normal(size=(64, 64))
    psi = torch.from_numpy(a).cuda()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.sofft_propagate(h, ctypes.c_void_p(psi.data_ptr()), 0.05, 4, None, stream) == EWORKSPACE
    assert b"sofft_plan_bind" in L.sofft_last_error()
    out = ctypes.c_double()
    assert L.sofft_norm2(h, ctypes.c_void_p(psi.data_ptr()), ctypes.byref(out), stream) == EWORKSPACE
    torch.cuda.synchronize()
    assert np.array_equal(psi.cpu().numpy(), a)
    # a workspace for propagation only is too small for a solve
    ws, ptr = s.device_workspace(_size(s, h, 0))
    assert L.sofft_plan_bind(h, ctypes.c_void_p(ptr), _size(s, h, 0)) == 0
    assert L.sofft_plan_bind(h, ctypes.c_void_p(ptr + 8), _size(s, h, 0)) == -1   # misaligned
    E = np.array([0.5])
    x = torch.zeros((1, 64, 64), dtype=torch.complex128, device="cuda")
    st = L.sofft_sse_solve(h, ctypes.c_void_p(psi.data_ptr()), 0, E.ctypes.data_as(ctypes.c_void_p), 1, 0.0,
                           ctypes.c_void_p(x.data_ptr()), 1e-8, 100, None, stream)
    assert st == EWORKSPACE
    assert _size(s, h, 4) > _size(s, h, 1) > _size(s, h, 0)
    L.sofft_plan_destroy(h)
    del ws


def test_caller_workspace_gives_the_same_results():
    s = _sofft()
    L = s.lib()
    n = 128
    print("workspace: caller-bound vs binding-managed", flush=True)
    x = (np.arange(n) + 0.5) * 0.2 - n * 0.1
    psi0 = wl.gaussian_2d(x, x, x0=0.4, y0=-0.2, px=1.0, py=0.5)
    f = wl.Pulse(E0=0.05, omega=0.3, cycles=2).at_midpoints(0.0, 0.05, 30)
    plan = s.Plan([n, n], [n * 0.2] * 2, R0=[0.8 * n * 0.1] * 2, theta=0.5, charge=1.0, a2=0.64)
    ref = torch.from_numpy(psi0).cuda()
    plan.propagate(ref, 0.05, 30, torch.from_numpy(f).cuda())
    h = _raw_plan(s, n)
    nb = _size(s, h, 2)
    ws, ptr = s.device_workspace(nb)
    assert L.sofft_plan_bind(h, ctypes.c_void_p(ptr), nb) == 0
    psi = torch.from_numpy(psi0).cuda()
    fd = torch.from_numpy(f).cuda()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.sofft_propagate(h, ctypes.c_void_p(psi.data_ptr()), 0.05, 30, ctypes.c_void_p(fd.data_ptr()),
                             stream) == 0
    torch.cuda.synchronize()
    assert np.array_equal(psi.cpu().numpy(), ref.cpu().numpy())
    # rebinding other memory rebuilds the phase table there: same result again
    ws2, ptr2 = s.device_workspace(nb)
    assert L.sofft_plan_bind(h, ctypes.c_void_p(ptr2), nb) == 0
    del ws
    psi2 = torch.from_numpy(psi0).cuda()
    assert L.sofft_propagate(h, ctypes.c_void_p(psi2.data_ptr()), 0.05, 30, ctypes.c_void_p(fd.data_ptr()),
                             stream) == 0
    torch.cuda.synchronize()
    assert np.array_equal(psi2.cpu().numpy(), ref.cpu().numpy())
    # a two-energy solve in the caller's workspace equals the managed one
    rhs = torch.from_numpy(-wl.smooth_source(n, n, seed=4)).cuda()
    want, _, _ = plan.sse_solve(rhs, [0.4, 1.1], rtol=1e-8)
    E = np.array([0.4, 1.1])
    out = torch.empty((2, n, n), dtype=torch.complex128, device="cuda")
    st = L.sofft_sse_solve(h, ctypes.c_void_p(rhs.data_ptr()), 0, E.ctypes.data_as(ctypes.c_void_p), 2, 0.0,
                           ctypes.c_void_p(out.data_ptr()), 1e-8, 10000, None, stream)
    assert st == 0
    assert np.array_equal(out.cpu().numpy(), want.cpu().numpy())
    L.sofft_plan_destroy(h)
    plan.close()


def test_batch_needs_its_workspace():
    s = _sofft()
    L = s.lib()
    print("workspace: batch", flush=True)
    probs = (s.Problem * 2)(*[s.problem([n, n], [n * 0.2] * 2, R0=[0.8 * n * 0.1] * 2, dtype=s.C128)
                              for n in (64, 96)])
    h = ctypes.c_void_p()
    assert L.sofft_batch_create(ctypes.cast(probs, ctypes.c_void_p), 2, ctypes.byref(h)) == 0
    states = [torch.zeros((n, n), dtype=torch.complex128, device="cuda") for n in (64, 96)]
    ptrs = (ctypes.c_void_p * 2)(*[t.data_ptr() for t in states])
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.sofft_batch_propagate(h, ctypes.cast(ptrs, ctypes.c_void_p), 0.05, 3, None, None, stream) == EWORKSPACE
    b = ctypes.c_int64()
    assert L.sofft_batch_workspace_size(h, ctypes.byref(b)) == 0
    ws, ptr = s.device_workspace(b.value)
    assert L.sofft_batch_bind(h, ctypes.c_void_p(ptr), b.value - 256) == 0
    assert L.sofft_batch_propagate(h, ctypes.cast(ptrs, ctypes.c_void_p), 0.05, 3, None, None, stream) == EWORKSPACE
    assert L.sofft_batch_bind(h, ctypes.c_void_p(ptr), b.value) == 0
    assert L.sofft_batch_propagate(h, ctypes.cast(ptrs, ctypes.c_void_p), 0.05, 3, None, None, stream) == 0
    torch.cuda.synchronize()
    L.sofft_batch_destroy(h)
    del ws
