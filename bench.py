#!/usr/bin/env python3
"""Benchmark of the SO-FFT + ECS hot path on one MI355X.

One "step" is one split-operator time step (Sec. II: kinetic, potential and
ECS/Crank-Nicolson factors) of the 2D workload: 1024 x 1024 grid, h = 0.2,
complex128, soft-core potential with a 4-cycle dipole pulse, SECS on all four
edges from 80% of the half-width, end angle 0.5.  ``value`` is grid points x
steps per second with the state resident in HBM.  The JSON line also carries
the roofline of the dominant kernel (HIP-event timed), the CPU oracle timed on
a bounded sample, the complex64 mode, and the FFT-preconditioned COCG solve
when the library provides it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point SO-FFT steps/s + PCG time-to-1e-8 residual, plain vs learned/batched"
HBM_PEAK_GBS = 8000.0


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs (profiles/), scaled by the copy-kernel calibration, or None when the
    kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "tdse_2d_1024_c128_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    srcs = [os.path.join(ROOT, "paper_1505_06707_amd", "csrc", n)
            for n in ("tdse.hip", "passes.hpp", "line_fft.hpp", "potential.hpp", "cx.hpp")]
    sha = hashlib.sha256(b"".join(open(p, "rb").read() for p in srcs)).hexdigest()
    k = rec.get("kernels", {}).get(kernel)
    if k is None or rec.get("source_sha256") != sha:
        return None
    return (k["fetch_kib"] * rec["fetch_scale"] + k["write_kib"] * rec["write_scale"]) * 1024


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gpu_tdse(sofft, wl, torch, dtype, steps, warmup, reps=5, seed=1, device_warmup_s=0.3):
    """The 2D workload: the same propagation run untimed for `device_warmup_s`
    seconds (a cold GPU needs a few milliseconds of load to reach its steady
    clocks: without it the first repetitions of 20 steps measure 52 us/step
    against 41 once warm), then `warmup` untimed steps, then `reps`
    repetitions of the same `steps` steps (each from the warmed-up state),
    every one timed with HIP events recorded on the stream the library
    launches on, around the sofft_propagate call.  Returns the median and the
    per-kernel durations."""
    c = wl.TDSE_2D
    plan = sofft.Plan([c.n, c.n], [c.L, c.L], R0=[c.R0, c.R0], theta=c.theta, charge=c.charge,
                      a2=c.a2, dtype=dtype)
    x = plan.nodes(0)
    psi0 = wl.gaussian_2d(x, x, **wl.packet_params(seed))
    cdt = np.complex128 if dtype == sofft.C128 else np.complex64
    f_all = c.pulse.at_midpoints(0.0, c.dt, warmup + steps)
    f_dev = torch.from_numpy(f_all).cuda()
    warm = torch.from_numpy(psi0.astype(cdt)).cuda()
    spare = warm.clone()
    t_end = time.perf_counter() + device_warmup_s
    while time.perf_counter() < t_end:
        plan.propagate(spare, c.dt, min(200, warmup + steps), f_dev[:min(200, warmup + steps)])
        torch.cuda.synchronize()
    del spare
    if warmup:
        plan.propagate(warm, c.dt, warmup, f_dev[:warmup])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev, wall = [], []
    for _ in range(reps):
        psi = warm.clone()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        plan.propagate(psi, c.dt, steps, f_dev[warmup:], stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        wall.append(time.perf_counter() - t0)
        ev.append(e0.elapsed_time(e1) / 1e3)
    result = psi.clone()
    # The same K steps again with every launch bracketed by HIP events on the
    # library's stream, for the per-kernel durations of the roofline.
    psi.copy_(warm)
    plan.timing(True)
    plan.propagate(psi, c.dt, steps, f_dev[warmup:], stream=stream)
    kern = {name: plan.timing_read(k) for name, k in (("row_pass", sofft.KERNEL_ROW),
                                                       ("column_pass", sofft.KERNEL_COL))}
    plan.timing(False)
    plan.close()
    return dict(event_s=float(np.median(ev)), event_all_s=ev, wall_s=float(np.median(wall)), kernels=kern,
                psi=result, npts=c.n * c.n)


def fp32_vs_oracle_checkpoints(sofft, wl, torch):
    """complex64 propagation of the whole 2D workload (2000 steps) against the
    FP64 oracle's stored state at steps 100/500/1000/2000 (8192 seeded points
    and the squared norm; tests/golden/make_tdse_2d_1024_checkpoints.py writes
    them from the oracle alone)."""
    path = os.path.join(ROOT, "tests", "golden", "tdse_2d_1024_checkpoints.npz")
    if not os.path.exists(path):
        return None
    gold = np.load(path)
    c = wl.TDSE_2D
    out = {}
    for name, dt_ in (("c64", sofft.C64), ("c128", sofft.C128)):
        plan = sofft.Plan([c.n, c.n], [c.L, c.L], R0=[c.R0, c.R0], theta=c.theta, charge=c.charge, a2=c.a2,
                          dtype=dt_)
        x = plan.nodes(0)
        psi0 = wl.gaussian_2d(x, x, **wl.packet_params(int(gold["packet_seed"])))
        psi = torch.from_numpy(psi0.astype(np.complex64 if dt_ == sofft.C64 else np.complex128)).cuda()
        f = torch.from_numpy(c.pulse.at_midpoints(0.0, c.dt, int(gold["steps"][-1]))).cuda()
        done, rows = 0, {}
        for k, step in enumerate(gold["steps"]):
            step = int(step)
            plan.propagate(psi, c.dt, step - done, f[done:step])
            done = step
            torch.cuda.synchronize()
            got = psi.cpu().numpy().astype(np.complex128).ravel()[gold["index"]]
            want = gold["samples"][k]
            rows[str(step)] = {"rel_l2_samples": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
                               "norm2_rel_err": float(abs(plan.norm2(psi) - gold["norm2"][k]) / gold["norm2"][k])}
        plan.close()
        out[name] = rows
    out["sampled_points"] = int(len(gold["index"]))
    return out


def gpu_tdse3d(sofft, wl, torch, steps=20, reps=5, device_warmup_s=0.3):
    """The 3D workload (256^3, h = 0.4): per dtype the median of `reps`
    HIP-event timed runs of `steps` steps, the per-launch durations of the
    kinetic and strip passes, and the error against the FP64 oracle's stored
    checkpoints (steps 25/50/100, 8192 sampled points and the norm)."""
    c = wl.TDSE_3D
    gold_path = os.path.join(ROOT, "tests", "golden", "tdse_3d_256_checkpoints.npz")
    gold = np.load(gold_path) if os.path.exists(gold_path) else None
    seed = int(gold["packet_seed"]) if gold is not None else 3
    out = {"workload": f"3D {c.n}^3, h = {c.h}, SECS, soft-core a2 = {c.a2}, pulse along x, dt = {c.dt}"}
    npts = c.n ** 3
    for name, dt_ in (("c128", sofft.C128), ("c64", sofft.C64)):
        S = 16 if dt_ == sofft.C128 else 8
        plan = sofft.Plan([c.n] * 3, [c.L] * 3, R0=[c.R0] * 3, theta=c.theta, charge=c.charge, a2=c.a2, dtype=dt_)
        x = plan.nodes(0)
        cdt = np.complex128 if dt_ == sofft.C128 else np.complex64
        psi0 = torch.from_numpy(wl.gaussian_3d(x, x, x, **wl.packet_params_3d(seed)).astype(cdt)).cuda()
        nf = max(steps, 100)
        f = torch.from_numpy(c.pulse.at_midpoints(0.0, c.dt, nf)).cuda()
        spare = psi0.clone()
        t_end = time.perf_counter() + device_warmup_s
        while time.perf_counter() < t_end:
            plan.propagate(spare, c.dt, 5, f[:5])
            torch.cuda.synchronize()
        del spare
        ev = []
        stream = torch.cuda.current_stream()
        for _ in range(reps):
            psi = psi0.clone()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            plan.propagate(psi, c.dt, steps, f[:steps], stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ev.append(e0.elapsed_time(e1) / 1e3)
        psi = psi0.clone()
        plan.timing(True)
        plan.propagate(psi, c.dt, steps, f[:steps], stream=stream)
        kin = plan.timing_read(sofft.KERNEL_3D_KINETIC)
        strip = plan.timing_read(sofft.KERNEL_3D_STRIP)
        plan.timing(False)
        t = float(np.median(ev))
        kin_us = kin[0] / kin[1] * 1e3
        row = {"us_per_step": t / steps * 1e6, "value": npts * steps / t, "unit": "grid-point-steps/s",
               "kinetic_pass_us": kin_us, "strip_pass_us": strip[0] / strip[1] * 1e3 if strip[1] else None,
               "kinetic_pass_frac": 2 * S * npts / (kin_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
               "step_frac_6S": 6 * S * npts / (t / steps) / 1e9 / HBM_PEAK_GBS}
        if gold is not None:
            psi = psi0.clone()
            done, errs = 0, {}
            for k, step in enumerate(gold["steps"]):
                step = int(step)
                plan.propagate(psi, c.dt, step - done, f[done:step])
                done = step
                torch.cuda.synchronize()
                got = psi.cpu().numpy().astype(np.complex128).ravel()[gold["index"]]
                want = gold["samples"][k]
                errs[str(step)] = {"rel_l2_samples": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
                                   "norm2_rel_err": float(abs(plan.norm2(psi) - gold["norm2"][k]) / gold["norm2"][k])}
            row["vs_fp64_oracle"] = errs
        plan.close()
        out[name] = row
    return out


def gpu_tdse1d(sofft, wl, torch):
    """The 1D workload: 4096 points, 4000 steps in one workgroup (state in LDS/registers)."""
    c = wl.TDSE_1D
    plan = sofft.Plan(c.n, c.L, R0=c.R0, theta=c.theta, charge=c.charge, a2=c.a2)
    psi0 = torch.from_numpy(wl.gaussian_1d(plan.nodes(0))).cuda()
    f = torch.from_numpy(c.pulse.at_midpoints(0.0, c.dt, c.nsteps)).cuda()
    psi = psi0.clone()
    plan.propagate(psi, c.dt, 50, f[:50])     # warm-up
    psi.copy_(psi0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.propagate(psi, c.dt, c.nsteps, f)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.close()
    return {"workload": f"1D n={c.n} c128, {c.nsteps} steps", "time_s": wall, "steps_per_s": c.nsteps / wall,
            "value": c.n * c.nsteps / wall, "unit": "grid-point-steps/s", "us_per_step": wall / c.nsteps * 1e6}


def gpu_pcg(sofft, wl, torch, n_energies=None, seed=0, extras=True, shifted=False):
    """Batched COCG to 1e-8 on the 512^2 stationary workload (Sec. III)."""
    c = wl.SSE_2D
    plan = sofft.Plan([c.n, c.n], [c.L, c.L], R0=[c.R0, c.R0], theta=c.theta, charge=c.charge, a2=c.a2)
    f = torch.from_numpy(-wl.smooth_source(c.n, c.n, seed=seed)).cuda()
    E = c.energies() if n_energies is None else np.linspace(c.E_lo, c.E_hi, n_energies)
    out = torch.empty((len(E), c.n, c.n), dtype=torch.complex128, device="cuda")
    plan.sse_solve(f, E[:4], rtol=c.rtol, out=out[:4])       # warm-up (allocations, code load)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats, code = plan.sse_solve(f, E, rtol=c.rtol, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.timing(True)
    plan.sse_solve(f, E, rtol=c.rtol, out=out)
    kinds = {"row_matvec": sofft.KERNEL_SSE_ROW_MV, "col_matvec": sofft.KERNEL_SSE_COL_MV,
             "row_update_fft": sofft.KERNEL_SSE_ROW_UPD, "col_precond": sofft.KERNEL_SSE_COL_PREC,
             "row_precond_dot": sofft.KERNEL_SSE_ROW_PREC}
    kern = {k: plan.timing_read(v) for k, v in kinds.items()}
    plan.timing(False)
    shifted = pcg_shifted(plan, f, E, c.rtol, out, wall, torch) if shifted else None
    band = pcg_banded(plan, f, E, c.rtol, out, wall, torch) if extras else None
    plan.close()
    its = np.array([s["iterations"] for s in stats])
    res = np.array([s["rel_residual"] for s in stats])
    npts = c.n * c.n
    # algorithmic bytes of the fused passes per point per iteration and energy:
    # K1 4S, K2 3S, K4 7S, K5 2S, K6 3S with S = 16 (complex128)
    per_kernel_S = {"row_matvec": 4, "col_matvec": 3, "row_update_fft": 7, "col_precond": 2, "row_precond_dot": 3}
    total_it = int(its.sum())
    kern_s = sum(v[0] for v in kern.values()) / 1e3
    alg_bytes = 19 * 16 * npts * total_it
    dom = max(kern, key=lambda k: kern[k][0])
    dom_bytes = per_kernel_S[dom] * 16 * npts * total_it
    return {"time_to_tol_s": wall, "energies": int(len(E)), "grid": [c.n, c.n], "rtol": c.rtol,
            "status": int(code), "iterations": {"min": int(its.min()), "mean": float(its.mean()),
                                                 "max": int(its.max()), "total": total_it},
            "max_true_rel_residual": float(res.max()),
            "kernel_time_s": kern_s, "achieved_GBs_all_kernels": alg_bytes / kern_s / 1e9,
            "dominant_kernel": dom, "dominant_GBs": dom_bytes / (kern[dom][0] / 1e3) / 1e9,
            "kernels_ms": {k: v[0] for k, v in kern.items()}, "shifted": shifted, "banded": band}


def gpu_sse1d(sofft, wl, torch):
    """The paper's own stationary example (Sec. V): 1D, N = 1024, h = 0.1,
    r_s = 40, soft-core a2 = 2, PCG to 1e-12 with the banded ECS
    preconditioner; SECS at theta = pi/4 and TFECS at 0.5.  Reported: the
    iterations at E = 1 and 2 beside the paper's printed counts (about 36 and
    79, for a right-hand side it does not give; here the seeded smooth source),
    and the time of 128 energies in [0.05, 2.0] in one launch, plain and banded."""
    out = {"workload": "1D N=1024, h=0.1, R0=40, soft-core a2=2, smooth source (seed 3), rtol 1e-12"}
    f = torch.from_numpy(wl.smooth_source(None, 1024, seed=3)).cuda()
    E = np.linspace(0.05, 2.0, 128)
    for name, kind, theta, paper in (("secs", sofft.SECS, np.pi / 4, 36), ("tfecs", sofft.TFECS, 0.5, 79)):
        plan = sofft.Plan([1024], [102.4], R0=[40.0], theta=theta, contour=kind, charge=1.0, a2=2.0)
        row = {"paper_iterations": paper}
        for banded in (False, True):
            key = "banded" if banded else "plain"
            _, st, code = plan.sse_solve(f, [1.0, 2.0], rtol=1e-12, maxit=20000, banded=banded)
            row[key + "_iterations_E1_E2"] = [st[0]["iterations"], st[1]["iterations"]]
            plan.sse_solve(f, E[:4], rtol=1e-12, maxit=20000, banded=banded)    # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st, code = plan.sse_solve(f, E, rtol=1e-12, maxit=20000, banded=banded)
            torch.cuda.synchronize()
            its = [q["iterations"] for q in st]
            row[key + "_128E"] = {"time_s": time.perf_counter() - t0, "status": int(code),
                                  "iterations_mean": float(np.mean(its)), "iterations_max": int(np.max(its)),
                                  "max_true_rel_residual": float(max(q["rel_residual"] for q in st))}
        plan.close()
        out[name] = row
    return out


def gpu_pcg3d(sofft, wl, torch, seed=0):
    """Batched COCG to 1e-8 on the 3D stationary workload (128^3, 16 energies):
    time to tolerance, iterations, the event-timed line-pass groups and their
    algorithmic bytes; then the same solve with the banded ECS preconditioner."""
    c = wl.SSE_3D
    plan = sofft.Plan([c.n] * 3, [c.L] * 3, R0=[c.R0] * 3, theta=c.theta, charge=c.charge, a2=c.a2)
    f = torch.from_numpy(-wl.smooth_source_3d(c.n, c.n, c.n, seed=seed)).cuda()
    E = c.energies()
    out = torch.empty((len(E), c.n, c.n, c.n), dtype=torch.complex128, device="cuda")
    plan.sse_solve(f, E[:2], rtol=c.rtol, out=out[:2])       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats, code = plan.sse_solve(f, E, rtol=c.rtol, out=out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.timing(True)
    plan.sse_solve(f, E, rtol=c.rtol, out=out)
    kinds = {"xy_matvec": sofft.KERNEL_SSE_ROW_MV, "z_matvec": sofft.KERNEL_SSE_COL_MV,
             "x_update_fft": sofft.KERNEL_SSE_ROW_UPD, "yzy_precond": sofft.KERNEL_SSE_COL_PREC,
             "x_precond_dot": sofft.KERNEL_SSE_ROW_PREC}
    kern = {k: plan.timing_read(v) for k, v in kinds.items()}
    plan.timing(False)
    band = pcg_banded(plan, f, E, c.rtol, out, wall, torch)
    plan.close()
    its = np.array([s["iterations"] for s in stats])
    res = np.array([s["rel_residual"] for s in stats])
    npts = c.n ** 3
    # algorithmic bytes per point, iteration and energy of each pass group
    # (S = 16 B): x+y matvec 4S + 3S, z matvec 3S, update 7S, y/z/y
    # preconditioner 6S, x preconditioner 3S; 26S in all
    per_S = {"xy_matvec": 7, "z_matvec": 3, "x_update_fft": 7, "yzy_precond": 6, "x_precond_dot": 3}
    total_it = int(its.sum())
    kern_s = sum(v[0] for v in kern.values()) / 1e3
    gbs = {k: per_S[k] * 16 * npts * total_it / (v[0] / 1e3) / 1e9 for k, v in kern.items() if v[0] > 0}
    return {"workload": f"3D {c.n}^3, h = {c.h}, SECS, {len(E)} energies in [{c.E_lo}, {c.E_hi}]",
            "time_to_tol_s": wall, "energies": int(len(E)), "rtol": c.rtol, "status": int(code),
            "iterations": {"min": int(its.min()), "mean": float(its.mean()), "max": int(its.max()),
                           "total": total_it},
            "max_true_rel_residual": float(res.max()),
            "us_per_energy_iteration": kern_s / total_it * 1e6,
            "kernel_time_s": kern_s, "achieved_GBs_all_passes": 26 * 16 * npts * total_it / kern_s / 1e9,
            "group_GBs": gbs, "kernels_ms": {k: v[0] for k, v in kern.items()}, "banded": band}


def gpu_pcg_tfecs(sofft, wl, torch, n_energies=32, seed=0, shifted=False):
    """The 512^2 stationary workload on the TFECS contour (Eq. qTFECS, alpha =
    0.5), where the paper finds the plain FFT preconditioner slow: 32 energies
    in [0.05, 2.0] with the paper's divisor, then with tuned shifts."""
    c = wl.SSE_2D
    plan = sofft.Plan([c.n, c.n], [c.L, c.L], R0=[c.R0, c.R0], theta=0.5, contour=sofft.TFECS,
                      charge=c.charge, a2=c.a2)
    f = torch.from_numpy(-wl.smooth_source(c.n, c.n, seed=seed)).cuda()
    E = np.linspace(c.E_lo, c.E_hi, n_energies)
    out = torch.empty((len(E), c.n, c.n), dtype=torch.complex128, device="cuda")
    plan.sse_solve(f, E[:2], rtol=c.rtol, out=out[:2], maxit=50000)    # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats, code = plan.sse_solve(f, E, rtol=c.rtol, out=out, maxit=50000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    shifted = pcg_shifted(plan, f, E, c.rtol, out, wall, torch, every=4) if shifted else None
    band = pcg_banded(plan, f, E, c.rtol, out, wall, torch)
    plan.close()
    its = np.array([q["iterations"] for q in stats])
    return {"workload": f"{c.n}^2 TFECS alpha 0.5, {len(E)} energies in [{c.E_lo}, {c.E_hi}], rtol {c.rtol}",
            "time_to_tol_s": wall, "status": int(code),
            "iterations": {"min": int(its.min()), "mean": float(its.mean()), "max": int(its.max())},
            "max_true_rel_residual": float(max(q["rel_residual"] for q in stats)), "shifted": shifted,
            "banded": band}


def pcg_banded(plan, f, E, rtol, out, plain_s, torch):
    """The same solve with the banded ECS eigen-preconditioner of Eq.
    PreconFFT_ECS (the tables are built by a first small call, outside the
    timed region, as the plan keeps them)."""
    plan.sse_solve(f, E[:1], rtol=rtol, out=out[:1], banded=True, maxit=50000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats, code = plan.sse_solve(f, E, rtol=rtol, out=out, banded=True, maxit=50000)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    its = np.array([q["iterations"] for q in stats])
    return {"time_to_tol_s": t, "status": int(code),
            "iterations": {"min": int(its.min()), "mean": float(its.mean()), "max": int(its.max())},
            "max_true_rel_residual": float(max(q["rel_residual"] for q in stats)), "speedup_vs_plain": plain_s / t}


def pcg_shifted(plan, f, E, rtol, out, plain_s, torch, candidates=(0.02, 0.05, 0.1, 0.2), every=16, probe=24):
    """The same solve with the shifted divisor K - E - i eta (an option beside
    the paper's preconditioner): shifts tuned on every `every`-th energy by short
    batched solves, each energy taking the shift of the nearest tuned one.
    The reported time includes the tuning."""
    sub = E[::every]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eta_sub = plan.sse_tune_shift(f, sub, candidates, probe_iters=probe, rtol=rtol)
    eta = eta_sub[np.abs(E[:, None] - sub[None, :]).argmin(axis=1)]
    t1 = time.perf_counter()
    _, stats, code = plan.sse_solve(f, E, rtol=rtol, out=out, eta=eta)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    its = np.array([s["iterations"] for s in stats])
    res = np.array([s["rel_residual"] for s in stats])
    return {"time_to_tol_s": t2 - t0, "tune_s": t1 - t0, "solve_s": t2 - t1, "status": int(code),
            "candidates": list(candidates), "tuned_on": int(len(sub)), "probe_iters": probe,
            "eta": {f"{e:.3f}": float(v) for e, v in zip(sub, eta_sub)},
            "iterations": {"min": int(its.min()), "mean": float(its.mean()), "max": int(its.max()),
                           "total": int(its.sum())},
            "max_true_rel_residual": float(res.max()), "speedup_vs_plain": plain_s / (t2 - t0)}


def gpu_batch(sofft, wl, torch, steps, seed=2024, warmup=40):
    """96 uneven complex64 runs (256^2 .. 1024^2) advanced together by the
    batched path; aggregate grid-point steps per second."""
    runs = wl.batch_runs(seed=seed)
    dt = 0.05
    probs, states, f_rows = [], [], []
    for r in runs:
        n = r["n"]
        L = n * 0.2
        probs.append(sofft.problem([n, n], [L, L], R0=[0.8 * L / 2] * 2, theta=0.5, charge=1.0, a2=0.64,
                                   dtype=sofft.C64))
    b = sofft.Batch(probs)
    for r, run in enumerate(runs):
        n = run["n"]
        x = (np.arange(n) + 0.5) * 0.2 - n * 0.2 / 2
        states.append(torch.from_numpy(wl.gaussian_2d(x, x, **wl.packet_params(run["packet_seed"]))
                                       .astype(np.complex64)).cuda())
        f_rows.append(run["pulse"].at_midpoints(0.0, dt, steps))
    f = torch.from_numpy(np.stack(f_rows)).cuda()
    fw = f[:, :warmup].contiguous()
    b.propagate(states, dt, warmup, fw, norms=False)   # launch-shape timing, graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norms = b.propagate(states, dt, steps, f, norms=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    npts = sum(run["n"] ** 2 for run in runs)
    shapes = {}
    for r, run in enumerate(runs):
        if run["n"] not in shapes:
            shapes[run["n"]] = {"row": b.launch_shape(r, 0), "col": b.launch_shape(r, 1),
                                "runs": sum(1 for q in runs if q["n"] == run["n"])}
    b.close()
    return {"value": npts * steps / wall, "unit": "grid-point-steps/s", "runs": len(runs), "steps": steps,
            "grid_points": npts, "wall_s": wall, "ms_per_step": wall / steps * 1e3,
            "dtype": "c64 state, f64 arithmetic",
            "algorithmic_GBs": 4 * 8 * npts * steps / wall / 1e9,
            "launch_shapes": {str(k): v for k, v in sorted(shapes.items())}, "graph_steps": 32}


def gpu_learned(sofft, wl, torch, epochs=30, shifted=False):
    """Learned correction on the 1024^2 x 64-energy stationary workload:
    pairs from plain COCG on training sources, training on the GPU, then
    plain COCG and the flexible solve on the evaluation source."""
    from paper_1505_06707_amd.lp_data import init_weights, make_pairs
    c = wl.LEARNED_2D
    plan = sofft.Plan([c.n, c.n], [c.L, c.L], R0=[c.R0, c.R0], theta=c.theta, charge=c.charge, a2=c.a2)
    t0 = time.perf_counter()
    train_src = [torch.from_numpy(-wl.smooth_source(c.n, c.n, seed=sd)).cuda() for sd in (1001, 1002)]
    r, e, Es, pair_its = make_pairs(plan, train_src, [0.2, 0.8, 1.4, 2.0], schedule=(1, 3, 6, 12, 24, 48))
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    lp = sofft.LearnedCorrection()
    lp.set_weights(init_weights(7))
    t0 = time.perf_counter()
    losses = lp.train(plan, r, e, Es, epochs=epochs, batch=4, lr=2e-3, seed=11)
    t_train = time.perf_counter() - t0
    del r, e
    f = torch.from_numpy(-wl.smooth_source(c.n, c.n, seed=0)).cuda()
    E = c.energies()
    out = torch.empty((len(E), c.n, c.n), dtype=torch.complex128, device="cuda")
    plan.sse_solve(f, E[:2], rtol=c.rtol, out=out[:2])    # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st0, code0 = plan.sse_solve(f, E, rtol=c.rtol, out=out)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, st1, code1 = plan.sse_solve_learned(lp, f, E, rtol=c.rtol, patience=30, out=out)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    lp.close()
    shifted = pcg_shifted(plan, f, np.asarray(E, dtype=np.float64), c.rtol, out, t_plain, torch) if shifted else None
    plan.close()
    i0 = np.array([q["iterations"] for q in st0])
    i1 = np.array([q["iterations"] for q in st1])
    return {"workload": f"{c.n}^2 x {len(E)} energies, rtol {c.rtol}", "pairs": int(len(Es)),
            "pair_plain_iterations": int(pair_its), "pairs_s": t_pairs, "train_s": t_train,
            "loss_first_last": [float(losses[0]), float(losses[-1])],
            "plain": {"time_s": t_plain, "status": int(code0), "iterations_mean": float(i0.mean()),
                      "iterations_max": int(i0.max())},
            "learned": {"time_s": t_learned, "status": int(code1), "iterations_mean": float(i1.mean()),
                        "iterations_max": int(i1.max()), "fell_back": int(sum(q["fell_back"] for q in st1)),
                        "max_true_rel_residual": float(max(q["rel_residual"] for q in st1))},
            "gain_time": t_plain / t_learned, "gain_iterations": float(i0.mean() / i1.mean()),
            "shifted_divisor": shifted}


_CPU_CHILD = r"""
import json, os, sys, time
import numpy as np
import scipy.fft
sys.path.insert(0, sys.argv[1])
from oracle import tdse as ot
from paper_1505_06707_amd import workloads as wl
steps, reps, workers = int(sys.argv[2]), int(sys.argv[3]), int(sys.argv[4])
c = wl.TDSE_2D
ax = ot.Axis(c.n, c.L, R0=c.R0, theta=c.theta)
prob = ot.Problem2D(ax, ax, Zc=c.charge, a2=c.a2)
psi0 = wl.gaussian_2d(ax.x, ax.x, **wl.packet_params(1))
f = c.pulse.at_midpoints(0.0, c.dt, steps)
times = []
with scipy.fft.set_workers(workers):
    prob.step(psi0, c.dt, f[0])       # factorisations and tables outside the timing
    for _ in range(reps):
        t0 = time.perf_counter()
        prob.propagate(psi0, c.dt, f)
        times.append(time.perf_counter() - t0)
print(json.dumps({"times": times}))
"""


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _cpu_run(steps, reps, workers, pin):
    import subprocess
    env = dict(os.environ)
    nthreads = "1" if pin else str(workers)
    env.update(OMP_NUM_THREADS=nthreads, OPENBLAS_NUM_THREADS=nthreads, MKL_NUM_THREADS=nthreads)
    pre = (lambda: os.sched_setaffinity(0, {sorted(os.sched_getaffinity(0))[0]})) if pin else None
    r = subprocess.run([sys.executable, "-c", _CPU_CHILD, ROOT, str(steps), str(reps), str(workers)],
                       capture_output=True, text=True, env=env, preexec_fn=pre, timeout=600)
    if r.returncode != 0:
        raise RuntimeError("CPU oracle run failed: " + r.stderr[-2000:])
    return json.loads(r.stdout.strip().splitlines()[-1])["times"]


def cpu_baseline(wl, sample_steps, reps=5):
    """The FP64 oracle on the host, a bounded sample of the same workload: the
    literal four-FFT step (scipy pocketfft + SuperLU) for `sample_steps` steps,
    median of `reps` runs after a warm-up step, in a child process pinned to
    one core (OMP/OpenBLAS at one thread), then the same with scipy.fft's
    workers set to every core the process may use."""
    c = wl.TDSE_2D
    ncores = len(os.sched_getaffinity(0))
    t1 = float(np.median(_cpu_run(sample_steps, reps, 1, pin=True)))
    tn = float(np.median(_cpu_run(sample_steps, reps, ncores, pin=False)))
    npts = c.n * c.n
    return dict(value=npts * sample_steps / t1, unit="grid-point-steps/s", cores=1, kind="oracle",
                sample=f"{sample_steps} steps of the 1024^2 c128 workload (literal four-FFT step, scipy pocketfft + "
                       f"SuperLU), median of {reps} runs of {t1:.2f} s, one pinned core of {ncores} usable "
                       f"({_cpu_model()})",
                cpu_model=_cpu_model(), host_cores=ncores,
                all_cores={"value": npts * sample_steps / tn, "cores": ncores, "median_s": tn,
                           "note": "same oracle, scipy.fft workers = usable cores; SuperLU and the "
                                   "elementwise phases stay single-threaded"})


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions of the K steps (median reported)")
    ap.add_argument("--device-warmup-ms", type=float, default=300.0,
                    help="untimed propagation before the warm-up steps, to bring the GPU to steady clocks")
    ap.add_argument("--cpu-sample-steps", type=int, default=8)
    ap.add_argument("--cpu-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--shifted", action="store_true",
                    help="also time the shifted-divisor option (not the paper's preconditioner)")
    ap.add_argument("--no-pcg-extras", action="store_true",
                    help="only the paper's plain preconditioner in the PCG leg (no banded or TFECS solves)")
    ap.add_argument("--pcg-energies", type=int, default=None)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-1d", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this size (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures a single GPU: the library has no multi-GPU path (batched runs and energies "
              "would shard across GPUs, one process each). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1505_06707_amd import sofft, workloads as wl
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    sofft.lib()
    if args.copy_mib:
        a = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.copy_mib} MiB x 5")
        return

    log(f"TDSE 2D 1024^2 c128: warmup {args.warmup}, {args.reps} x {args.steps} timed steps")
    r64 = gpu_tdse(sofft, wl, torch, sofft.C128, args.steps, args.warmup, reps=args.reps,
                   device_warmup_s=args.device_warmup_ms / 1e3)
    npts = r64["npts"]
    value = npts * args.steps / r64["event_s"]
    ms_per_step = r64["event_s"] / args.steps * 1e3
    log(f"  {ms_per_step * 1e3:.1f} us/step (HIP events, median of {args.reps}; wall "
        f"{r64['wall_s'] / args.steps * 1e6:.1f} us/step), {value / 1e9:.2f} G grid-point-steps/s")

    # roofline of the dominant kernel: algorithmic bytes = read + write of the state
    # (2 x 16 B per grid point) per launch of a row or column pass
    kern = r64["kernels"]
    dom = max(kern, key=lambda k: kern[k][0])
    tot_ms, cnt = kern[dom]
    avg_s = tot_ms / cnt / 1e3
    alg_bytes = 2 * 16 * npts
    achieved = alg_bytes / avg_s / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom), "kernel": dom,
                "avg_launch_us": avg_s * 1e6, "launches": cnt,
                "algorithmic_bytes_per_launch": alg_bytes,
                "kernels_avg_us": {k: v[0] / v[1] * 1e3 for k, v in kern.items() if v[1]},
                "step_frac": 4 * 16 * npts / (r64["event_s"] / args.steps) / 1e9 / HBM_PEAK_GBS}
    log(f"  dominant kernel {dom}: {avg_s * 1e6:.1f} us/launch, {achieved:.0f} GB/s "
        f"({100 * achieved / HBM_PEAK_GBS:.1f}% of HBM peak)")

    fp32 = None
    if not args.no_fp32:
        log("TDSE 2D 1024^2 c64")
        r32 = gpu_tdse(sofft, wl, torch, sofft.C64, args.steps, args.warmup, reps=args.reps,
                       device_warmup_s=args.device_warmup_ms / 1e3)
        a = r64["psi"].cpu().numpy()
        b = r32["psi"].cpu().numpy().astype(np.complex128)
        err = float(np.linalg.norm(b - a) / np.linalg.norm(a))
        fp32 = {"value": npts * args.steps / r32["event_s"], "unit": "grid-point-steps/s",
                "ms_per_step": r32["event_s"] / args.steps * 1e3,
                "rel_l2_vs_fp64_path": err, "steps": args.steps + args.warmup}
        log(f"  c64: {fp32['ms_per_step'] * 1e3:.1f} us/step, rel L2 vs FP64 path {err:.2e}")
        fp32["vs_fp64_oracle"] = fp32_vs_oracle_checkpoints(sofft, wl, torch)
        if fp32["vs_fp64_oracle"]:
            log("  vs FP64 oracle (sampled): " + ", ".join(
                f"{k}: c64 {v['rel_l2_samples']:.2e} / c128 {fp32['vs_fp64_oracle']['c128'][k]['rel_l2_samples']:.2e}"
                for k, v in fp32["vs_fp64_oracle"]["c64"].items()))

    tdse1d = None
    if not args.no_1d:
        log("TDSE 1D 4096 x 4000 steps")
        tdse1d = gpu_tdse1d(sofft, wl, torch)
        log(f"  {tdse1d['time_s'] * 1e3:.1f} ms, {tdse1d['steps_per_s']:.0f} steps/s "
            f"({tdse1d['us_per_step']:.1f} us/step)")

    tdse3d = None
    if not args.no_3d:
        log("TDSE 3D 256^3 (c128, c64)")
        tdse3d = gpu_tdse3d(sofft, wl, torch, device_warmup_s=args.device_warmup_ms / 1e3)
        for k in ("c128", "c64"):
            r = tdse3d[k]
            log(f"  {k}: {r['us_per_step']:.0f} us/step, {r['value'] / 1e9:.2f} G grid-point-steps/s, kinetic pass "
                f"{r['kinetic_pass_us']:.0f} us ({100 * r['kinetic_pass_frac']:.0f}% of HBM peak)"
                + (f", vs oracle {max(v['rel_l2_samples'] for v in r['vs_fp64_oracle'].values()):.1e}"
                   if "vs_fp64_oracle" in r else ""))

    sse1d = None
    if not args.no_pcg and not args.no_1d:
        log("SSE 1D: the paper's example (N=1024, banded PCG to 1e-12), 128 energies per launch")
        sse1d = gpu_sse1d(sofft, wl, torch)
        for k in ("secs", "tfecs"):
            r = sse1d[k]
            log(f"  {k}: E=1,2 banded {r['banded_iterations_E1_E2']} it (paper ~{r['paper_iterations']}), plain "
                f"{r['plain_iterations_E1_E2']}; 128 E: banded {r['banded_128E']['time_s'] * 1e3:.1f} ms, plain "
                f"{r['plain_128E']['time_s'] * 1e3:.1f} ms")

    pcg = None
    if not args.no_pcg:
        log("SSE 512^2 batched COCG to 1e-8")
        pcg = gpu_pcg(sofft, wl, torch, args.pcg_energies, extras=not args.no_pcg_extras, shifted=args.shifted)
        log(f"  {pcg['energies']} energies in {pcg['time_to_tol_s']:.3f} s, iterations "
            f"{pcg['iterations']['min']}..{pcg['iterations']['max']} (mean {pcg['iterations']['mean']:.0f}), "
            f"{pcg['achieved_GBs_all_kernels']:.0f} GB/s over the fused passes")
        if pcg["banded"] is not None:
            bd = pcg["banded"]
            log(f"  banded ECS preconditioner: {bd['time_to_tol_s']:.3f} s, iterations mean "
                f"{bd['iterations']['mean']:.0f}, {bd['speedup_vs_plain']:.2f}x the plain solve")
            log("SSE 512^2 on the TFECS contour, 32 energies")
            pcg["tfecs"] = gpu_pcg_tfecs(sofft, wl, torch, shifted=args.shifted)
            tf = pcg["tfecs"]
            log(f"  plain {tf['time_to_tol_s']:.3f} s (mean {tf['iterations']['mean']:.0f} it); banded "
                f"{tf['banded']['time_to_tol_s']:.3f} s (mean {tf['banded']['iterations']['mean']:.0f} it), "
                f"{tf['banded']['speedup_vs_plain']:.2f}x")

    pcg3d = None
    if not args.no_pcg and not args.no_3d:
        log("SSE 3D 128^3 batched COCG to 1e-8, 16 energies")
        pcg3d = gpu_pcg3d(sofft, wl, torch)
        log(f"  {pcg3d['time_to_tol_s']:.3f} s, iterations {pcg3d['iterations']['min']}.."
            f"{pcg3d['iterations']['max']}, {pcg3d['us_per_energy_iteration']:.0f} us per energy-iteration, "
            f"{pcg3d['achieved_GBs_all_passes']:.0f} GB/s over the passes")
        bd = pcg3d["banded"]
        log(f"  banded ECS preconditioner: {bd['time_to_tol_s']:.3f} s, iterations mean "
            f"{bd['iterations']['mean']:.0f}, {bd['speedup_vs_plain']:.2f}x the plain solve")

    batch = None
    if not args.no_batch:
        log(f"batched uneven TDSE: 96 runs, c64, {args.batch_steps} steps")
        batch = gpu_batch(sofft, wl, torch, args.batch_steps)
        log(f"  {batch['ms_per_step']:.3f} ms/step for {batch['grid_points'] / 1e6:.1f} M points, "
            f"{batch['value'] / 1e9:.2f} G grid-point-steps/s, {batch['algorithmic_GBs']:.0f} GB/s algorithmic")

    learned = None
    if not args.no_learned:
        log("learned correction: 1024^2 x 64 energies (pairs, training, plain vs corrected solve)")
        learned = gpu_learned(sofft, wl, torch, shifted=args.shifted)
        log(f"  plain {learned['plain']['time_s']:.2f} s (mean {learned['plain']['iterations_mean']:.0f} it), "
            f"learned {learned['learned']['time_s']:.2f} s (mean {learned['learned']['iterations_mean']:.0f} it, "
            f"{learned['learned']['fell_back']} fell back); training {learned['train_s']:.1f} s")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU oracle sample: {args.cpu_reps} x {args.cpu_sample_steps} steps, pinned and all cores")
        cpu = cpu_baseline(wl, args.cpu_sample_steps, reps=args.cpu_reps)
        log(f"  {cpu['value'] / 1e6:.2f} M grid-point-steps/s on one core, "
            f"{cpu['all_cores']['value'] / 1e6:.2f} M on {cpu['all_cores']['cores']} ({cpu['cpu_model']})")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "tdse_2d_1024_c128", "grid": [1024, 1024], "h": 0.2, "dt": 0.05,
                   "ecs": "SECS, R0 = 81.92 (80% of half-width), end angle 0.5",
                   "potential": "soft-core a2=0.64 + dipole pulse E0=0.05 w=0.057 4 cycles",
                   "parallelism": "single-gpu"},
        "timing": {"method": "HIP events around sofft_propagate on its stream", "reps": args.reps,
                   "device_warmup_ms": args.device_warmup_ms,
                   "statistic": "median", "per_rep_ms_per_step": [t / args.steps * 1e3 for t in r64["event_all_s"]],
                   "wall_ms_per_step_median": r64["wall_s"] / args.steps * 1e3,
                   "passes_per_call": 2 * args.steps + 2},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp32": fp32,
        "tdse_1d": tdse1d,
        "sse_1d": sse1d,
        "tdse_3d": tdse3d,
        "pcg": pcg,
        "pcg_3d": pcg3d,
        "batch": batch,
        "learned": learned,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
