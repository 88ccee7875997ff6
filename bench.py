"""Benchmark of the GKS step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-adjoint] [--no-3d] [--no-tri]

Workload: 2D TM fields on a 4096 x 4096 Cartesian grid of the unit square, kinetic
non-reflecting sides, eps map of 64 seeded circular inclusions (eps in [1, 4]), Gaussian point
current source at the centre, CFL 0.5, collision time 0.01 dt.  A step is one full GKS time step
(load, gradients, face reconstruction, interface flux, accumulation, boundaries and source)
over the whole grid, with the FP64 energy diagnostic every 100 steps, as in a production run.
Inputs are resident in HBM before timing starts.

One JSON line on stdout:
  value          FP32-mode cell-updates/s (FP32 storage, flux and update)
  fp64           the same run in FP64
  roofline       achieved algorithmic HBM bandwidth of the kernel the timed run uses, the paired
                 kernel (two steps per launch: twice the single step's algorithmic bytes per
                 launch), HIP events around its launches, against the 8 TB/s peak; traffic = HBM
                 bytes per launch from the committed rocprofv3 counter summary (null when the
                 kernel source changed since); single_step_roofline: the same for the single-step
                 kernel (gks_step)
  cpu_baseline   the FP64 oracle on the host cores, on a bounded sample of the same workload
  cart3d         the 3D six-field 384^3 workload (FP32 and FP64): throughput and roofline
  tri2d          the ~4M-triangle workload (FP32 and FP64): throughput and roofline
  adjoint        forward + adjoint step time of the differentiable workload (1024^2 x 8 maps,
                 800 steps, checkpoints every 50) beside the plain FP64 and FP32 steps of the
                 same grids, and the adjoint step's own per-launch time
  cart2d_phm     the 4096^2 workload carried by the PHM fields (Ez, Hx, Hy, psi) with a
                 divergence error to clean (gamma = 1): throughput and roofline
  cart3d_phm     the 384^3 workload on the eight PHM fields (chi = gamma = 1)
  tri2d_phm      the ~4M-triangle workload on the PHM fields (Ez, Hx, Hy, psi), gamma = 1
  tet3d          the tetrahedral workload (1.5M cells around a PEC sphere), FP32 and FP64

Helper modes for the profiles: --profile-kernel PREC runs only step kernels (for rocprofv3);
--profile-pair PREC 20 launches of the paired kernel (gks_run of 40 steps);
--profile-tri PREC runs 20 steps of the triangle workload, --profile-3d PREC 10 steps of the 384^3
workload, --profile-adjoint 10 adjoint steps of the 1024^2 x 8 workload, --profile-phm PREC 20 steps of
the 4096^2 PHM workload, --profile-phm3d PREC 5 steps of the 384^3 PHM workload, --profile-tet PREC 20
steps of the tetrahedral workload; --copy-calibration runs a plain device copy of known size (counter
scale factor).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GKS cell-updates/s (FP32 vs FP64) + % HBM roofline; fwd+adjoint step time"
PEAK_GBS = 8000.0
N = 4096
ENERGY_EVERY = 100
KERNEL_SRC = os.path.join(ROOT, "paper_2412_16845_amd", "csrc", "k_cart2d.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cart2d_step_4096_traffic.txt")
# algorithmic bytes per cell-update: read Ez,Hx,Hy and 1/eps, write Ez,Hx,Hy
BYTES_PER_CELL = {"fp32": 7 * 4, "fp64": 7 * 8}
# with the PHM potential psi: read four fields and 1/eps, write four fields
PHM_BYTES_PER_CELL = {"fp32": 9 * 4, "fp64": 9 * 8}
PHM_STEPS = 300


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload():
    from paper_2412_16845_amd import inputs as I
    return I.tm_dielectric_nr(nx=N, seed=0, nsteps=1000)


def make(torch, wl, precision, energy_every=0, limiter="none"):
    from paper_2412_16845_amd.gks import Solver
    dtype = torch.float64 if precision == "fp64" else torch.float32
    s = Solver("cart2d", n=wl.n, bc=wl.bc, precision=precision, cfl=wl.cfl, tau_over_dt=wl.tau_over_dt,
               energy_every=energy_every, limiter=limiter, phm=wl.extra.get("phm"))
    ei = torch.tensor(wl.epsinv, dtype=dtype, device="cuda")
    s.set_material(ei)
    src = wl.source
    s.set_point_source(src["cells"], src["weights"], src["J0"], src["t0"], src["sigma_t"])
    U = torch.tensor(wl.U0, dtype=dtype, device="cuda")
    return s, U, ei


def time_run(torch, s, U, steps, warmup):
    """Whole-job time of `steps` GKS steps (gks_run with the energy diagnostic)."""
    s.run(U, warmup, t0=0.0, energy=True)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(s.stream)
    s.run(U, steps, t0=warmup * s.dt, energy=True)
    end.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / 1e3, wall


def time_kernel(torch, s, U, launches=200):
    """Average duration of one step-kernel launch on the stream the kernel runs on: a HIP event
    pair around `launches` back-to-back launches, divided by their number (gaps between the
    launches included).  Also returns the mean over event pairs around single launches (up to 50),
    which adds the events' own overhead to every launch."""
    A, B = U, torch.empty_like(U)
    for i in range(10):
        s.step(A, B, t=i * s.dt)
        A, B = B, A
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    for i in range(launches):
        s.step(A, B, t=i * s.dt)
        A, B = B, A
    e1.record(s.stream)
    torch.cuda.synchronize()
    batch = e0.elapsed_time(e1) / 1e3 / launches
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(min(launches, 50))]
    for i, (a, b) in enumerate(evs):
        a.record(s.stream)
        s.step(A, B, t=i * s.dt)
        b.record(s.stream)
        A, B = B, A
    torch.cuda.synchronize()
    pairs = float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3
    return batch, pairs


def time_pair(torch, s, U, launches=200):
    """Average duration of one launch of the paired kernel (two steps per launch, the kernel
    gks_run takes on this grid): a HIP event pair on the solver's stream around gks_run of
    2 x `launches` steps without the energy diagnostic (an even number of launches, so the state
    ends where it began and no copy follows), divided by `launches`."""
    assert launches % 2 == 0
    s.run(U, 20)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.run(U, 2 * launches)
    e1.record(s.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / launches


def kernel_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(precision, kind="step"):
    """HBM bytes per launch from the committed counter summary, if it matches this kernel
    (kind "step": the single-step kernel, "pair": the paired kernel)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        line = line.strip()
        if line.startswith("#") or "=" not in line:
            continue
        k, v = line.split("=", 1)
        kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_sha():
        return None
    key = f"traffic_bytes_per_launch_{precision}" if kind == "step" else f"traffic_bytes_per_launch_pair_{precision}"
    return float(kv[key]) if key in kv else None


def roofline(precision, t_launch):
    ncell = N * N
    alg = BYTES_PER_CELL[precision] * ncell
    achieved = alg / t_launch / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_GBS, 4), "traffic": read_traffic(precision),
            "kernel": "cart2d_step_kernel", "steps_per_launch": 1,
            "algorithmic_bytes_per_launch": alg, "kernel_seconds_per_launch": t_launch}


# arithmetic per 2D cell-update: two flops per multiply-add of the two face operators a cell owns
# (24 + 6 structural non-zeros each with vacuum 1/mu), six differences, and per field the four
# face fluxes and the update
C2_FLOPS_PER_CELL = 2 * 2 * (24 + 6) + 6 + 3 * 6


def roofline_pair(precision, t_launch):
    """The paired kernel: two cell-updates per cell and launch, so its algorithmic bytes are twice
    the single step's; `traffic` is what the counters measured per launch (about one step's
    bytes: the fields are read and written once for both steps).  Its arithmetic is given beside
    it against the non-packed vector peak (the profile summary has its VALU issue fraction)."""
    ncell = N * N
    alg = 2 * BYTES_PER_CELL[precision] * ncell
    achieved = alg / t_launch / 1e9
    tflops = 2 * C2_FLOPS_PER_CELL * ncell / t_launch / 1e12
    peak_alu = 78.6
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_GBS, 4), "traffic": read_traffic(precision, "pair"),
            "kernel": "cart2d_pair_kernel", "steps_per_launch": 2,
            "algorithmic_bytes_per_launch": alg, "kernel_seconds_per_launch": t_launch,
            "vector_alu": {"flops_per_cell_update": C2_FLOPS_PER_CELL, "achieved_tflops": round(tflops, 2),
                           "peak_tflops_non_packed": peak_alu, "frac": round(tflops / peak_alu, 4)}}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads() -> int:
    """Threads the oracle's OpenMP runtime uses in this process."""
    import ctypes
    from oracle import gks_oracle as O
    O.lib()
    try:
        return int(ctypes.CDLL("libgomp.so.1").omp_get_max_threads())
    except OSError:
        return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def oracle_window_rate(wl, dt, max_steps, max_seconds):
    """Cell-updates/s of the FP64 oracle on a 1024 x 1024 window of the workload (its centre,
    with the source and inclusions; cut sides non-reflecting): (rate, steps, seconds)."""
    from oracle import gks_oracle as O
    x0 = y0 = (N - 1024) // 2
    mesh = O.cart_window((N, N, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), [1, 1, 1, 1], (x0, y0, 0),
                         (x0 + 1024, y0 + 1024, 1), 2)
    ei = np.ascontiguousarray(wl.epsinv[0][y0:y0 + 1024, x0:x0 + 1024]).reshape(-1)
    U = O.from_soa(wl.U0[0][:, y0:y0 + 1024, x0:x0 + 1024].reshape(3, -1), "tm2d")
    c = wl.source["cells"][0]
    src = (np.array([(c // N - y0) * 1024 + (c % N - x0)]), np.array([1.0]), 1.0, 0.02, 0.005)
    steps = 0
    t0 = time.perf_counter()
    while True:
        U = O.run(mesh, U, 1, dt, wl.tau_over_dt * dt, epsinv=ei, source=src, t0=steps * dt)
        steps += 1
        el = time.perf_counter() - t0
        if el > max_seconds or steps >= max_steps:
            break
    return 1024 * 1024 * steps / el, steps, el


def cpu_baseline(wl):
    """The FP64 oracle (literal per-face lattice sums) on the host: all cores on a window of the
    benchmark workload, one core on the same window (a child process with one OpenMP thread),
    and the 64 x 64 periodic Gaussian configuration in full (200 steps) on all cores."""
    import subprocess
    from oracle import gks_oracle as O
    from paper_2412_16845_amd import inputs as I
    O.build()
    dt = wl.cfl / N   # c dt = cfl h on the unit square
    rate, steps, el = oracle_window_rate(wl, dt, 40, 12.0)
    threads = oracle_threads()
    code = ("import json, sys; sys.path.insert(0, %r); import bench; "
            "from paper_2412_16845_amd import inputs as I; "
            "r = bench.oracle_window_rate(I.tm_dielectric_nr(nx=bench.N, seed=0, nsteps=1000), %r, 4, 8.0); "
            "print(json.dumps({'rate': r[0], 'steps': r[1], 'seconds': r[2], 'threads': bench.oracle_threads()}))"
            % (ROOT, dt))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = None
    try:
        p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        if p.returncode == 0:
            one = json.loads(p.stdout.strip().splitlines()[-1])
    except (subprocess.TimeoutExpired, ValueError, IndexError):
        one = None
    c1 = I.tm_gaussian_periodic(64, seed=0, nsteps=200)
    mesh = O.cart2d(64, 64, bc=(0, 0, 0, 0))
    U = O.from_soa(c1.U0[0].reshape(3, -1), "tm2d")
    dt1 = c1.cfl / 64
    t0 = time.perf_counter()
    O.run(mesh, U, c1.nsteps, dt1, c1.tau_over_dt * dt1)
    t_c1 = time.perf_counter() - t0
    out = {"value": round(rate, 1), "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"1024x1024 centre window of the 4096x4096 workload, {steps} steps, {el:.1f} s, "
                     f"FP64 literal per-face lattice sums, {threads} OpenMP threads",
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
           "c1_full": {"value": round(64 * 64 * c1.nsteps / t_c1, 1), "unit": "cell-updates/s",
                       "seconds": round(t_c1, 3), "cores": threads,
                       "sample": "64x64 periodic Gaussian pulse, 200 steps (the whole configuration), literal oracle"}}
    if one is not None:
        out["one_core"] = {"value": round(one["rate"], 1), "unit": "cell-updates/s", "cores": one["threads"],
                           "sample": f"the same window, {one['steps']} steps, {one['seconds']:.1f} s, "
                                     f"OMP_NUM_THREADS=1"}
    return out


ADJ_N, ADJ_BATCH, ADJ_STEPS, ADJ_K = 1024, 8, 800, 50
# adjoint step, algorithmic bytes per cell: read lambda' (3) and U^n (3) and 1/eps, write lambda (3)
# in the field type; read and write the FP64 1/eps gradient
ADJ_BYTES_PER_CELL = 7 * 4 + 3 * 4 + 16


def adjoint_leg(torch):
    """The differentiable workload: 8 dielectric maps of 1024 x 1024, probe-box loss after 800
    steps, reverse mode with checkpoints every 50 steps (FP32 fields, FP64 gradient sums),
    timed end to end (forward with checkpoints, then per segment recompute + adjoint steps)
    next to the plain FP64 and FP32 runs of the same grids."""
    from paper_2412_16845_amd import autograd as AG
    from paper_2412_16845_amd import inputs as I
    from paper_2412_16845_amd.gks import Solver
    wl = I.tm_batch_probe(n=ADJ_N, batch=ADJ_BATCH, seed=0, nsteps=ADJ_STEPS)
    ncell = ADJ_N * ADJ_N * ADJ_BATCH

    def solver(prec):
        dtype = torch.float64 if prec == "fp64" else torch.float32
        s = Solver("cart2d", n=wl.n, bc=wl.bc, precision=prec, batch=wl.batch, cfl=wl.cfl,
                   tau_over_dt=wl.tau_over_dt)
        E = torch.tensor(wl.epsinv, dtype=dtype, device="cuda")
        s.set_material(E)
        return s, E, torch.tensor(wl.U0, dtype=dtype, device="cuda")

    def timed(s, fn):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        fn()
        b.record(s.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3

    plain = {}
    for prec in ("fp64", "fp32"):
        s, E, U = solver(prec)
        s.run(U, 50)
        plain[prec] = timed(s, lambda: s.run(U, ADJ_STEPS)) / ADJ_STEPS

        def single_steps():
            A, B = U, torch.empty_like(U)
            for i in range(ADJ_STEPS):
                s.step(A, B, t=i * s.dt)
                A, B = B, A

        plain[prec + "_single"] = timed(s, single_steps) / ADJ_STEPS
        del s, E, U
    s, E, U0 = solver("fp32")
    E.requires_grad_(True)

    def fwd_bwd(nsteps):
        E.grad = None
        UN = AG.run(s, U0, nsteps, E, None, checkpoint_every=ADJ_K)
        AG.probe_energy(s, UN, wl.probe).sum().backward()

    fwd_bwd(2 * ADJ_K)
    t_fb = timed(s, lambda: fwd_bwd(ADJ_STEPS))
    if not torch.isfinite(E.grad).all():
        raise RuntimeError("non-finite permittivity gradient")
    # per-launch duration of the adjoint step (its kernels together) on the solver's stream
    lam = torch.randn_like(U0)
    out = torch.empty_like(U0)
    g = torch.zeros((wl.batch,) + s.grid, dtype=torch.float64, device="cuda")
    Ed = E.detach()
    s.set_material(Ed)
    for _ in range(5):
        s.adjoint_step(U0, lam, out, g)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(50)]
    for e0, e1 in evs:
        e0.record(s.stream)
        s.adjoint_step(U0, lam, out, g)
        e1.record(s.stream)
    torch.cuda.synchronize()
    t_adj = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs])) / 1e3
    alg = ADJ_BYTES_PER_CELL * ncell
    return {"workload": f"tm_batch_probe: 2D TM {ADJ_N}x{ADJ_N} x batch {ADJ_BATCH}, non-reflecting sides, "
                        f"16 dielectric discs per map, probe-box Ez energy after {ADJ_STEPS} steps, "
                        f"checkpoints every {ADJ_K} steps, FP32 fields, FP64 gradient accumulation",
            "fwd_adj_ms_per_step": round(t_fb * 1e3 / ADJ_STEPS, 5),
            "plain_fp64_ms_per_step": round(plain["fp64"] * 1e3, 5),
            "plain_fp32_ms_per_step": round(plain["fp32"] * 1e3, 5),
            "fwd_adj_over_fp64_step": round(t_fb / ADJ_STEPS / plain["fp64"], 3),
            "plain_fp64_single_step_ms": round(plain["fp64_single"] * 1e3, 5),
            "plain_fp32_single_step_ms": round(plain["fp32_single"] * 1e3, 5),
            "fwd_adj_over_fp64_single_step": round(t_fb / ADJ_STEPS / plain["fp64_single"], 3),
            "adjoint_step_us_per_launch": round(t_adj * 1e6, 2),
            "adjoint_roofline": {"bound": "hbm", "achieved": round(alg / t_adj / 1e9, 1), "peak": PEAK_GBS,
                                 "unit": "GB/s", "frac": round(alg / t_adj / 1e9 / PEAK_GBS, 4),
                                 "algorithmic_bytes_per_launch": alg}}


def limited_leg(torch, wl):
    """The 4096^2 workload with minmod-limited slopes (the step for discontinuous data): per-launch
    times of the limited single-step and paired kernels against the same algorithmic bytes."""
    out = {"workload": "tm_dielectric_nr 4096x4096 with limiter = minmod (single-step kernel, 100 timed launches; "
                       "the paired kernel, 50 launches)"}
    ncell = N * N
    for prec in ("fp32", "fp64"):
        s, U, ei = make(torch, wl, prec, limiter="minmod")
        s.run(U, 10)
        t_launch, _ = time_kernel(torch, s, U, launches=100)
        if not torch.isfinite(U).all():
            raise RuntimeError(f"limited {prec} run produced non-finite values")
        t_pair = time_pair(torch, s, U, launches=50)
        alg = BYTES_PER_CELL[prec] * ncell
        out[prec] = {"cell_updates_per_s": round(ncell / t_launch, 1),
                     "roofline": {"bound": "hbm", "achieved": round(alg / t_launch / 1e9, 1), "peak": PEAK_GBS,
                                  "unit": "GB/s", "frac": round(alg / t_launch / 1e9 / PEAK_GBS, 4),
                                  "algorithmic_bytes_per_launch": alg, "kernel_seconds_per_launch": t_launch},
                     "paired_kernel": {"cell_updates_per_s": round(2 * ncell / t_pair, 1),
                                       "kernel_seconds_per_launch": t_pair, "steps_per_launch": 2,
                                       "frac": round(2 * alg / t_pair / 1e9 / PEAK_GBS, 4)}}
        del s, U, ei
        torch.cuda.empty_cache()
    return out


def phm_workload(nsteps=PHM_STEPS):
    from paper_2412_16845_amd import inputs as I
    return I.tm_phm_dielectric_nr(nx=N, seed=0, nsteps=nsteps, gamma=1.0)


def phm_leg(torch):
    """The 4096^2 dielectric workload on the PHM fields (Ez, Hx, Hy, psi), gamma = 1, with a
    divergent Hx bump: whole-run throughput (gks_run with the energy diagnostic, which takes the
    paired kernel) and the per-launch times of the paired and the single-step kernels against
    their algorithmic bytes."""
    wl = phm_workload()
    ncell = N * N
    out = {"workload": f"tm_phm_dielectric_nr: PHM TM fields (Ez, Hx, Hy, psi) 4096x4096, the 4096^2 recipe plus "
                       f"a divergent Hx bump, chi = 0, gamma = 1, CFL 0.4, {PHM_STEPS} steps, energy every 100",
           "cells": ncell}
    for prec in ("fp32", "fp64"):
        s, U, ei = make(torch, wl, prec, energy_every=ENERGY_EVERY)
        el, _ = time_run(torch, s, U, PHM_STEPS, 20)
        if not torch.isfinite(U).all():
            raise RuntimeError(f"PHM {prec} run produced non-finite values")
        t_launch, _ = time_kernel(torch, s, U, launches=100)
        t_pair = time_pair(torch, s, U, launches=100)
        alg = PHM_BYTES_PER_CELL[prec] * ncell
        out[prec] = {"cell_updates_per_s": round(ncell * PHM_STEPS / el, 1),
                     "ms_per_step": round(el * 1e3 / PHM_STEPS, 5),
                     "roofline": {"bound": "hbm", "achieved": round(2 * alg / t_pair / 1e9, 1), "peak": PEAK_GBS,
                                  "unit": "GB/s", "frac": round(2 * alg / t_pair / 1e9 / PEAK_GBS, 4),
                                  "kernel": "cart2d_pair_kernel", "steps_per_launch": 2,
                                  "algorithmic_bytes_per_launch": 2 * alg, "kernel_seconds_per_launch": t_pair},
                     "single_step_roofline": {"bound": "hbm", "achieved": round(alg / t_launch / 1e9, 1),
                                              "peak": PEAK_GBS, "unit": "GB/s",
                                              "frac": round(alg / t_launch / 1e9 / PEAK_GBS, 4),
                                              "kernel": "cart2d_step_kernel", "steps_per_launch": 1,
                                              "algorithmic_bytes_per_launch": alg,
                                              "kernel_seconds_per_launch": t_launch}}
        del s, U, ei
        torch.cuda.empty_cache()
    return out


N_OVERSIZED = 8192


def oversized_leg(torch):
    """The same 2D workload on an 8192 x 8192 grid (1.9 GB per fp32 step, far above the 256 MB
    Infinity Cache): per-launch time of the step kernel against the HBM roofline, so that the
    4096^2 fraction can be checked not to come from cache hits."""
    from paper_2412_16845_amd import inputs as I
    wl = I.tm_dielectric_nr(nx=N_OVERSIZED, seed=0, nsteps=100)
    ncell = N_OVERSIZED * N_OVERSIZED
    out = {"workload": f"tm_dielectric_nr: 2D TM {N_OVERSIZED}x{N_OVERSIZED}, the 4096^2 recipe on a finer grid "
                       f"(step kernel only, 100 timed launches; the paired kernel, 50 launches)", "cells": ncell}
    for prec in ("fp32", "fp64"):
        s, U, ei = make(torch, wl, prec)
        s.run(U, 10)
        t_launch, _ = time_kernel(torch, s, U, launches=100)
        if not torch.isfinite(U).all():
            raise RuntimeError(f"oversized {prec} run produced non-finite values")
        t_pair = time_pair(torch, s, U, launches=50)
        alg = BYTES_PER_CELL[prec] * ncell
        out[prec] = {"cell_updates_per_s": round(ncell / t_launch, 1),
                     "roofline": {"bound": "hbm", "achieved": round(alg / t_launch / 1e9, 1), "peak": PEAK_GBS,
                                  "unit": "GB/s", "frac": round(alg / t_launch / 1e9 / PEAK_GBS, 4),
                                  "algorithmic_bytes_per_launch": alg, "kernel_seconds_per_launch": t_launch},
                     "paired_kernel": {"cell_updates_per_s": round(2 * ncell / t_pair, 1),
                                       "kernel_seconds_per_launch": t_pair, "steps_per_launch": 2,
                                       "frac": round(2 * alg / t_pair / 1e9 / PEAK_GBS, 4)}}
        del s, U, ei
        torch.cuda.empty_cache()
    return out


C3_N, C3_STEPS = 384, 500
# 3D step, algorithmic bytes per cell-update: read six fields and 1/eps, write six fields
C3_BYTES_PER_CELL = {"fp32": 13 * 4, "fp64": 13 * 8}
# arithmetic per 3D cell-update: two flops per multiply-add of the three face operators a cell
# owns (80 + 12 + 12 structural non-zeros each), 18 differences and the six-field update
C3_FLOPS_PER_CELL = 2 * 3 * (80 + 24) + 18 + 6 * 4


def cart3d_leg(torch):
    """The 3D six-field workload: 384^3, dielectric blocks, PEC z walls, non-reflecting x/y
    sides, nu = 1/3, 500 steps (the whole job timed, and each launch with events)."""
    from paper_2412_16845_amd import inputs as I
    from paper_2412_16845_amd.gks import Solver
    wl = I.em_blocks_pec(n=C3_N, seed=0, nsteps=C3_STEPS)
    ncell = C3_N ** 3
    out = {"workload": f"em_blocks_pec: 3D six-field {C3_N}^3, 32 dielectric blocks (eps in [1,6]), PEC z walls, "
                       f"non-reflecting x/y sides, CFL 1/3, tau = 0.01 dt, {C3_STEPS} steps"}
    for prec in ("fp32", "fp64"):
        dtype = torch.float64 if prec == "fp64" else torch.float32
        s = Solver("cart3d", n=wl.n, bc=wl.bc, precision=prec, cfl=wl.cfl, tau_over_dt=wl.tau_over_dt)
        E = torch.tensor(wl.epsinv, dtype=dtype, device="cuda")
        s.set_material(E)
        U = torch.tensor(wl.U0, dtype=dtype, device="cuda")
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        s.run(U, C3_STEPS)
        b.record(s.stream)
        torch.cuda.synchronize()
        t_run = a.elapsed_time(b) / 1e3
        if not torch.isfinite(U).all():
            raise RuntimeError(f"3D {prec} run produced non-finite values")
        t_launch, _ = time_kernel(torch, s, U, launches=30)
        # this kernel is bound by its arithmetic, and arithmetic on nonzero data draws more power:
        # the same launches on a state of unit normal values in every cell
        g = torch.Generator(device="cuda")
        g.manual_seed(11)
        Ur = torch.randn(U.shape, generator=g, dtype=dtype, device="cuda")
        t_rand, _ = time_kernel(torch, s, Ur, launches=30)
        del Ur
        alg = C3_BYTES_PER_CELL[prec] * ncell
        out[prec] = {"value": round(ncell * C3_STEPS / t_run, 1), "unit": "cell-updates/s",
                     "ms_per_step": round(t_run * 1e3 / C3_STEPS, 4),
                     "kernel_us_per_launch_by_state": {"recipe_state": round(t_launch * 1e6, 1),
                                                       "random_state": round(t_rand * 1e6, 1)},
                     "roofline": {"bound": "hbm", "achieved": round(alg / t_launch / 1e9, 1), "peak": PEAK_GBS,
                                  "unit": "GB/s", "frac": round(alg / t_launch / 1e9 / PEAK_GBS, 4),
                                  "algorithmic_bytes_per_launch": alg, "kernel_seconds_per_launch": t_launch},
                     "vector_alu": {"flops_per_cell": C3_FLOPS_PER_CELL,
                                    "achieved_tflops": round(C3_FLOPS_PER_CELL * ncell / t_launch / 1e12, 2),
                                    "peak_tflops_non_packed": 78.6}}
        del s, E, U
        torch.cuda.empty_cache()
    return out


C3_PHM_STEPS = 60
# 3D with the PHM potentials: read eight fields and 1/eps, write eight fields
C3_PHM_BYTES_PER_CELL = {"fp32": 17 * 4, "fp64": 17 * 8}
# two flops per multiply-add of the three face operators a cell owns (168 + 36 + 36 structural
# non-zeros each), 24 differences and the eight-field update
C3_PHM_FLOPS_PER_CELL = 2 * 3 * (168 + 72) + 24 + 8 * 4


def cart3d_phm_leg(torch):
    """The 3D workload on the eight PHM fields: 384^3, dielectric blocks, PEC z walls,
    non-reflecting x/y sides, divergent Ex and Hy bumps, chi = gamma = 1, nu = 0.3 (the 3D PHM step
    grows above it)."""
    from paper_2412_16845_amd import inputs as I
    from paper_2412_16845_amd.gks import Solver
    wl = I.em_phm_blocks_pec(n=C3_N, seed=0, nsteps=C3_PHM_STEPS)
    ncell = C3_N ** 3
    out = {"workload": f"em_phm_blocks_pec: 3D PHM fields (Ex .. Hz, phi, psi) {C3_N}^3, the 384^3 recipe plus "
                       f"divergent Ex and Hy bumps, chi = gamma = 1, CFL 0.3, {C3_PHM_STEPS} steps"}
    for prec in ("fp32", "fp64"):
        dtype = torch.float64 if prec == "fp64" else torch.float32
        s = Solver("cart3d", n=wl.n, bc=wl.bc, precision=prec, cfl=wl.cfl, tau_over_dt=wl.tau_over_dt,
                   phm=wl.extra["phm"])
        E = torch.tensor(wl.epsinv, dtype=dtype, device="cuda")
        s.set_material(E)
        U = torch.tensor(wl.U0, dtype=dtype, device="cuda")
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        s.run(U, C3_PHM_STEPS)
        b.record(s.stream)
        torch.cuda.synchronize()
        t_run = a.elapsed_time(b) / 1e3
        if not torch.isfinite(U).all():
            raise RuntimeError(f"3D PHM {prec} run produced non-finite values")
        t_launch, _ = time_kernel(torch, s, U, launches=20)
        alg = C3_PHM_BYTES_PER_CELL[prec] * ncell
        out[prec] = {"value": round(ncell * C3_PHM_STEPS / t_run, 1), "unit": "cell-updates/s",
                     "ms_per_step": round(t_run * 1e3 / C3_PHM_STEPS, 4),
                     "roofline": {"bound": "hbm", "achieved": round(alg / t_launch / 1e9, 1), "peak": PEAK_GBS,
                                  "unit": "GB/s", "frac": round(alg / t_launch / 1e9 / PEAK_GBS, 4),
                                  "algorithmic_bytes_per_launch": alg, "kernel_seconds_per_launch": t_launch},
                     "vector_alu": {"flops_per_cell": C3_PHM_FLOPS_PER_CELL,
                                    "achieved_tflops": round(C3_PHM_FLOPS_PER_CELL * ncell / t_launch / 1e12, 2),
                                    "peak_tflops_non_packed": 78.6}}
        del s, E, U
        torch.cuda.empty_cache()
    return out


C4_H, C4_STEPS = 6.8e-4, 2000


def tri_bytes_per_cell(prec, nf=3):
    """Compulsory bytes per cell-update of the triangle step with its stored geometry (vacuum),
    nf fields: gradient kernel: fields, 3 neighbour ids, 3 gradient weight vectors, write 2 nf
    gradients; face/update kernel: fields, 2 nf gradients, 3 neighbour ids, 19 geometry values
    (3 x normal, |l|/|Omega|, midpoint minus the neighbour's centroid; 2 midpoint offsets), write
    fields (the neighbours' fields and gradients are gathered from cache)."""
    e = 8 if prec == "fp64" else 4
    grad = nf * e + 3 * 4 + 6 * e + 2 * nf * e
    step = nf * e + 2 * nf * e + 3 * 4 + 19 * e + nf * e
    return grad + step


def tri_leg(torch):
    """The triangle workload: ~4.06M triangles (square with an elliptical PEC hole,
    non-reflecting outer square), Gaussian pulse, 2000 steps, FP32 and FP64."""
    from paper_2412_16845_amd import inputs as I
    from paper_2412_16845_amd.gks import Solver
    wl = I.tri_ellipse_workload(h=C4_H, seed=0, nsteps=C4_STEPS)
    ex = wl.extra
    mesh4 = (ex["verts"], ex["tris"], ex["face_cells"], ex["face_verts"])
    ncell = mesh4[1].shape[0]
    out = {"workload": f"tri_ellipse: 2D TM on {ncell} triangles (jittered-lattice Delaunay mesh, h = {C4_H}, of the "
                       f"unit square minus an elliptical PEC hole; non-reflecting outer square), Gaussian pulse, "
                       f"CFL 0.5 on the smallest inradius, tau = 0.01 dt, {C4_STEPS} steps", "cells": ncell}
    for prec in ("fp32", "fp64"):
        dtype = torch.float64 if prec == "fp64" else torch.float32
        s = Solver("tri2d", tri=mesh4, precision=prec, cfl=wl.cfl, tau_over_dt=wl.tau_over_dt)
        U = torch.tensor(wl.U0, dtype=dtype, device="cuda")
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        s.run(U, C4_STEPS)
        b.record(s.stream)
        torch.cuda.synchronize()
        t_run = a.elapsed_time(b) / 1e3
        if not torch.isfinite(U).all():
            raise RuntimeError(f"triangle {prec} run produced non-finite values")
        t_launch, _ = time_kernel(torch, s, U, launches=100)
        alg = tri_bytes_per_cell(prec) * ncell
        # the same time against the byte models of the two other layouts: geometry rebuilt from
        # vertices on the fly (3 vertex ids, shared coordinates, 3 neighbours, no gradient
        # scratch) and precomputed per-face geometry
        models = {"on_the_fly": 56 if prec == "fp32" else 88, "per_face_geometry": 150 if prec == "fp32" else 250}
        out[prec] = {"value": round(ncell * C4_STEPS / t_run, 1), "unit": "cell-updates/s",
                     "ms_per_step": round(t_run * 1e3 / C4_STEPS, 5), "dt": s.dt,
                     "roofline": {"bound": "hbm", "achieved": round(alg / t_launch / 1e9, 1), "peak": PEAK_GBS,
                                  "unit": "GB/s", "frac": round(alg / t_launch / 1e9 / PEAK_GBS, 4),
                                  "algorithmic_bytes_per_launch": alg, "step_seconds_per_launch": t_launch},
                     "frac_against_other_layouts": {
                         k: {"bytes_per_cell": b, "frac": round(b * ncell / t_launch / 1e9 / PEAK_GBS, 4)}
                         for k, b in models.items()}}
        del s, U
        torch.cuda.empty_cache()
    return out


TRI_PHM_STEPS = 500
C5_TET_N, TET_STEPS = 64, 300


def tet_bytes_per_cell(prec):
    """Compulsory bytes per cell-update of the tetrahedral step (vacuum; about two faces per
    cell): gradient kernel: 6 fields, 4 neighbour ids, 12 weights, write 18 gradients; face
    kernel (per cell: two faces): 2 x (2 cell ids, 12 geometry values, write 6 fluxes) and the
    cell's fields and gradients once; update kernel: 4 face slots, the fluxes once (two faces x 6),
    1/|Omega|, 6 fields, write 6 fields.  Gathered neighbours and face fluxes are counted once."""
    e = 8 if prec == "fp64" else 4
    grad = 6 * e + 4 * 4 + 12 * e + 18 * e
    face = 2 * (2 * 4 + 12 * e + 6 * e) + 24 * e
    upd = 4 * 4 + 12 * e + e + 6 * e + 6 * e
    return grad + face + upd


def tet_leg(torch):
    """The tetrahedral workload: 64^3 jittered cubes of six tetrahedra around a PEC sphere
    (radius 0.15), non-reflecting box sides, Ez pulse, 300 steps, FP32 and FP64."""
    from paper_2412_16845_amd import inputs as I
    from paper_2412_16845_amd.gks import Solver
    wl = I.tet_sphere_workload(n=C5_TET_N, seed=0, nsteps=TET_STEPS)
    ex = wl.extra
    mesh4 = (ex["verts"], ex["tets"], ex["face_cells"], ex["face_verts"])
    ncell = mesh4[1].shape[0]
    out = {"workload": f"tet_sphere: EM3D on {ncell} tetrahedra ({C5_TET_N}^3 jittered cubes of six, PEC sphere of "
                       f"radius 0.15, non-reflecting sides), Ez pulse, CFL 0.5 on the smallest inradius, tau = 0.01 dt, "
                       f"{TET_STEPS} steps", "cells": ncell, "faces": int(mesh4[2].shape[0])}
    for prec in ("fp32", "fp64"):
        dtype = torch.float64 if prec == "fp64" else torch.float32
        s = Solver("tet3d", tet=mesh4, precision=prec, cfl=wl.cfl, tau_over_dt=wl.tau_over_dt)
        U = torch.tensor(wl.U0, dtype=dtype, device="cuda")
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        s.run(U, TET_STEPS)
        b.record(s.stream)
        torch.cuda.synchronize()
        t_run = a.elapsed_time(b) / 1e3
        if not torch.isfinite(U).all():
            raise RuntimeError(f"tetrahedral {prec} run produced non-finite values")
        t_launch, _ = time_kernel(torch, s, U, launches=50)
        alg = tet_bytes_per_cell(prec) * ncell
        out[prec] = {"value": round(ncell * TET_STEPS / t_run, 1), "unit": "cell-updates/s",
                     "ms_per_step": round(t_run * 1e3 / TET_STEPS, 5),
                     "roofline": {"bound": "hbm", "achieved": round(alg / t_launch / 1e9, 1), "peak": PEAK_GBS,
                                  "unit": "GB/s", "frac": round(alg / t_launch / 1e9 / PEAK_GBS, 4),
                                  "algorithmic_bytes_per_launch": alg, "step_seconds_per_launch": t_launch}}
        del s, U
        torch.cuda.empty_cache()
    return out


def tri_phm_leg(torch):
    """The triangle workload on the PHM fields (Ez, Hx, Hy, psi), gamma = 1, with a divergent Hx
    bump (amplitude 0.5, w = 0.05 at (0.8, 0.2)), 500 steps, FP32 and FP64."""
    from paper_2412_16845_amd import inputs as I
    from paper_2412_16845_amd.gks import Solver
    wl = I.tri_ellipse_workload(h=C4_H, seed=0, nsteps=TRI_PHM_STEPS)
    ex = wl.extra
    mesh4 = (ex["verts"], ex["tris"], ex["face_cells"], ex["face_verts"])
    ncell = mesh4[1].shape[0]
    cen = ex["verts"][ex["tris"]].mean(axis=1)
    U0 = np.zeros((1, 4, ncell))
    U0[:, :3] = wl.U0
    U0[0, 1] += 0.5 * np.exp(-((cen[:, 0] - 0.8) ** 2 + (cen[:, 1] - 0.2) ** 2) / (2 * 0.05 ** 2))
    out = {"workload": f"tri_ellipse on the PHM fields (Ez, Hx, Hy, psi): {ncell} triangles, the triangle recipe "
                       f"plus a divergent Hx bump, chi = 0, gamma = 1, {TRI_PHM_STEPS} steps", "cells": ncell}
    for prec in ("fp32", "fp64"):
        dtype = torch.float64 if prec == "fp64" else torch.float32
        s = Solver("tri2d", tri=mesh4, precision=prec, cfl=wl.cfl, tau_over_dt=wl.tau_over_dt, phm=(0.0, 1.0))
        U = torch.tensor(U0, dtype=dtype, device="cuda")
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s.stream)
        s.run(U, TRI_PHM_STEPS)
        b.record(s.stream)
        torch.cuda.synchronize()
        t_run = a.elapsed_time(b) / 1e3
        if not torch.isfinite(U).all():
            raise RuntimeError(f"triangle PHM {prec} run produced non-finite values")
        t_launch, _ = time_kernel(torch, s, U, launches=100)
        alg = tri_bytes_per_cell(prec, 4) * ncell
        out[prec] = {"value": round(ncell * TRI_PHM_STEPS / t_run, 1), "unit": "cell-updates/s",
                     "ms_per_step": round(t_run * 1e3 / TRI_PHM_STEPS, 5),
                     "roofline": {"bound": "hbm", "achieved": round(alg / t_launch / 1e9, 1), "peak": PEAK_GBS,
                                  "unit": "GB/s", "frac": round(alg / t_launch / 1e9 / PEAK_GBS, 4),
                                  "algorithmic_bytes_per_launch": alg, "step_seconds_per_launch": t_launch}}
        del s, U
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-tri", action="store_true")
    ap.add_argument("--no-oversized", action="store_true")
    ap.add_argument("--no-limited", action="store_true")
    ap.add_argument("--no-phm", action="store_true")
    ap.add_argument("--no-tet", action="store_true")
    ap.add_argument("--profile-phm", choices=["fp32", "fp64"])
    ap.add_argument("--profile-phm3d", choices=["fp32", "fp64"])
    ap.add_argument("--profile-tet", choices=["fp32", "fp64"])
    ap.add_argument("--profile-kernel", choices=["fp32", "fp64"])
    ap.add_argument("--profile-pair", choices=["fp32", "fp64"])
    ap.add_argument("--profile-tri", choices=["fp32", "fp64"])
    ap.add_argument("--profile-3d", choices=["fp32", "fp64"])
    ap.add_argument("--profile-adjoint", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the GKS step is measured on one "
              "MI355X and multi-GPU domain decomposition is not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)

    if args.copy_calibration:
        n = 1 << 28   # 1 GiB of float32 read, 1 GiB written
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))
        return

    if args.profile_tri:
        from paper_2412_16845_amd import inputs as I
        from paper_2412_16845_amd.gks import Solver
        twl = I.tri_ellipse_workload(h=C4_H, seed=0, nsteps=20)
        ex = twl.extra
        s = Solver("tri2d", tri=(ex["verts"], ex["tris"], ex["face_cells"], ex["face_verts"]),
                   precision=args.profile_tri, cfl=twl.cfl, tau_over_dt=twl.tau_over_dt)
        U = torch.tensor(twl.U0, dtype=torch.float64 if args.profile_tri == "fp64" else torch.float32, device="cuda")
        s.run(U, 20)
        torch.cuda.synchronize()
        print(json.dumps({"profiled": "tri2d " + args.profile_tri, "steps": 20}))
        return

    if args.profile_3d:
        from paper_2412_16845_amd import inputs as I
        from paper_2412_16845_amd.gks import Solver
        dtype = torch.float64 if args.profile_3d == "fp64" else torch.float32
        w3 = I.em_blocks_pec(n=C3_N, seed=0, nsteps=10)
        s = Solver("cart3d", n=w3.n, bc=w3.bc, precision=args.profile_3d, cfl=w3.cfl, tau_over_dt=w3.tau_over_dt)
        E = torch.tensor(w3.epsinv, dtype=dtype, device="cuda")
        s.set_material(E)
        U = torch.tensor(w3.U0, dtype=dtype, device="cuda")
        s.run(U, 10)
        torch.cuda.synchronize()
        print(json.dumps({"profiled": "cart3d " + args.profile_3d, "steps": 10}))
        return
    if args.profile_adjoint:
        from paper_2412_16845_amd import inputs as I
        from paper_2412_16845_amd.gks import Solver
        wa = I.tm_batch_probe(n=ADJ_N, batch=ADJ_BATCH, seed=0, nsteps=10)
        s = Solver("cart2d", n=wa.n, bc=wa.bc, precision="fp32", batch=wa.batch, cfl=wa.cfl,
                   tau_over_dt=wa.tau_over_dt)
        E = torch.tensor(wa.epsinv, dtype=torch.float32, device="cuda")
        s.set_material(E)
        U = torch.tensor(wa.U0, dtype=torch.float32, device="cuda")
        lam = torch.randn_like(U)
        out = torch.empty_like(U)
        g = torch.zeros((wa.batch,) + s.grid, dtype=torch.float64, device="cuda")
        for _ in range(10):
            s.adjoint_step(U, lam, out, g)
        torch.cuda.synchronize()
        print(json.dumps({"profiled": "adjoint fp32", "steps": 10}))
        return

    if args.profile_tet:
        from paper_2412_16845_amd import inputs as I
        from paper_2412_16845_amd.gks import Solver
        wt = I.tet_sphere_workload(n=C5_TET_N, seed=0, nsteps=20)
        ex = wt.extra
        s = Solver("tet3d", tet=(ex["verts"], ex["tets"], ex["face_cells"], ex["face_verts"]), precision=args.profile_tet,
                   cfl=wt.cfl, tau_over_dt=wt.tau_over_dt)
        U = torch.tensor(wt.U0, dtype=torch.float64 if args.profile_tet == "fp64" else torch.float32, device="cuda")
        s.run(U, 20)
        torch.cuda.synchronize()
        print(json.dumps({"profiled": "tet3d " + args.profile_tet, "steps": 20}))
        return
    if args.profile_phm3d:
        from paper_2412_16845_amd import inputs as I
        from paper_2412_16845_amd.gks import Solver
        dtype = torch.float64 if args.profile_phm3d == "fp64" else torch.float32
        w3 = I.em_phm_blocks_pec(n=C3_N, seed=0, nsteps=5)
        s = Solver("cart3d", n=w3.n, bc=w3.bc, precision=args.profile_phm3d, cfl=w3.cfl, tau_over_dt=w3.tau_over_dt,
                   phm=w3.extra["phm"])
        s.set_material(torch.tensor(w3.epsinv, dtype=dtype, device="cuda"))
        U = torch.tensor(w3.U0, dtype=dtype, device="cuda")
        s.run(U, 5)
        torch.cuda.synchronize()
        print(json.dumps({"profiled": "cart3d phm " + args.profile_phm3d, "steps": 5}))
        return
    if args.profile_phm:
        s, U, _ = make(torch, phm_workload(20), args.profile_phm)
        B = torch.empty_like(U)
        for i in range(20):
            s.step(U, B, t=i * s.dt)
            U, B = B, U
        torch.cuda.synchronize()
        print(json.dumps({"profiled": "phm " + args.profile_phm, "launches": 20}))
        return

    wl = workload()
    if args.profile_pair:
        s, U, _ = make(torch, wl, args.profile_pair)
        s.run(U, 40)   # 20 launches of the paired kernel
        torch.cuda.synchronize()
        print(json.dumps({"profiled": "pair " + args.profile_pair, "launches": 20}))
        return
    if args.profile_kernel:
        s, U, _ = make(torch, wl, args.profile_kernel)
        B = torch.empty_like(U)
        for i in range(20):
            s.step(U, B, t=i * s.dt)
            U, B = B, U
        torch.cuda.synchronize()
        print(json.dumps({"profiled": args.profile_kernel, "launches": 20}))
        return

    res = {}
    for prec in ("fp32", "fp64"):
        log(f"[bench] {prec}: 4096x4096 dielectric box, warmup {args.warmup}, {args.steps} timed steps")
        s, U, ei = make(torch, wl, prec, energy_every=ENERGY_EVERY)
        el, wall = time_run(torch, s, U, args.steps, args.warmup)
        if not torch.isfinite(U).all():
            raise RuntimeError(f"{prec} run produced non-finite values")
        t_pair = time_pair(torch, s, U)
        t_launch, t_pairs = time_kernel(torch, s, U)
        # the recipe's fields are zero away from the source for most of the run; the same launches
        # on a state of unit normal values in every cell show whether the data changes the time
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        Ur = torch.randn(U.shape, generator=g, dtype=U.dtype, device=U.device)
        t_pair_rand = time_pair(torch, s, Ur.clone())
        t_rand, _ = time_kernel(torch, s, Ur)
        res[prec] = {"seconds": el, "wall": wall, "t_launch": t_launch, "t_launch_pairs": t_pairs, "dt": s.dt,
                     "t_launch_random": t_rand, "t_pair": t_pair, "t_pair_random": t_pair_rand}
        log(f"[bench] {prec}: {el * 1e3 / args.steps:.4f} ms/step; paired kernel {t_pair * 1e6:.1f} us/launch "
            f"({t_pair_rand * 1e6:.1f} us from a random state); single-step kernel {t_launch * 1e6:.1f} us/launch "
            f"({t_rand * 1e6:.1f} us from a random state)")
        del Ur
        del s, U, ei
        torch.cuda.empty_cache()

    ncell = N * N
    f32, f64 = res["fp32"], res["fp64"]
    out = {
        "metric": METRIC,
        "value": round(ncell * args.steps / f32["seconds"], 1),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["seconds"] * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "tm_dielectric_nr: 2D TM 4096x4096, non-reflecting sides, 64 dielectric discs "
                               "(eps in [1,4]), Gaussian point source, CFL 0.5, tau = 0.01 dt, energy every 100 steps",
                   "cells": ncell, "precision": "fp32"},
        "roofline": roofline_pair("fp32", f32["t_pair"]),
        "single_step_roofline": roofline("fp32", f32["t_launch"]),
        "fp64": {"value": round(ncell * args.steps / f64["seconds"], 1), "unit": "cell-updates/s",
                 "ms_per_step": round(f64["seconds"] * 1e3 / args.steps, 5), "dtype": "f64",
                 "roofline": roofline_pair("fp64", f64["t_pair"]),
                 "single_step_roofline": roofline("fp64", f64["t_launch"])},
        "kernel_us_per_launch_by_state": {
            prec: {"paired_recipe_state": round(res[prec]["t_pair"] * 1e6, 2),
                   "paired_random_state": round(res[prec]["t_pair_random"] * 1e6, 2),
                   "single_step_recipe_state": round(res[prec]["t_launch"] * 1e6, 2),
                   "single_step_random_state": round(res[prec]["t_launch_random"] * 1e6, 2),
                   "single_step_recipe_state_single_launch_event_pairs": round(res[prec]["t_launch_pairs"] * 1e6, 2)}
            for prec in ("fp32", "fp64")},
    }
    if not args.no_limited:
        log("[bench] limited 2D step: 4096x4096, minmod slopes, fp32 and fp64")
        out["cart2d_limited"] = limited_leg(torch, wl)
    if not args.no_oversized:
        log("[bench] oversized 2D: 8192x8192, step kernel, fp32 and fp64")
        out["cart2d_8192"] = oversized_leg(torch)
    if not args.no_phm:
        log(f"[bench] PHM 2D: 4096x4096 (Ez, Hx, Hy, psi), {PHM_STEPS} steps, fp32 and fp64")
        out["cart2d_phm"] = phm_leg(torch)
        log(f"[bench] PHM 3D: 384^3 (eight fields), {C3_PHM_STEPS} steps, fp32 and fp64")
        out["cart3d_phm"] = cart3d_phm_leg(torch)
        if not args.no_tri:
            log(f"[bench] PHM triangles: ~4M cells (Ez, Hx, Hy, psi), {TRI_PHM_STEPS} steps, fp32 and fp64")
            out["tri2d_phm"] = tri_phm_leg(torch)
    if not args.no_3d:
        log("[bench] 3D: 384^3 six fields, 500 steps, fp32 and fp64")
        out["cart3d"] = cart3d_leg(torch)
    if not args.no_tri:
        log("[bench] triangles: ~4M cells, 2000 steps, fp32 and fp64")
        out["tri2d"] = tri_leg(torch)
    if not args.no_tet:
        log(f"[bench] tetrahedra: {C5_TET_N}^3 x 6 cells around a PEC sphere, {TET_STEPS} steps, fp32 and fp64")
        out["tet3d"] = tet_leg(torch)
    if not args.no_adjoint:
        log("[bench] adjoint: 1024x1024 x 8, 800 steps forward + reverse with checkpoints every 50")
        out["adjoint"] = adjoint_leg(torch)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: oracle on a 1024x1024 window")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
