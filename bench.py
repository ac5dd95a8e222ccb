"""Benchmark of the M1 radiation-moment step on one MI355X.

Headline (`value`): zone-group updates per second of the full step (explicit transport +
implicit interaction update + energy/realizability diagnostics) on the 3-D Cartesian
192^3 zone, 12 group FP64 workload (optically thick core in a thin halo, Planck group
weights), inputs resident in HBM, timed with HIP events on the launch stream over K steps
after W warm-up steps.  Beside it: the same grid with float storage (MIXED), the 2-D
512^2 x 16 periodic blob workload (FP64 and MIXED, options), the spherical 256 x 64 x 128 x 20
workload, the radiation-matter exchange, the adjoint/forward ratio and the step with a
prescribed velocity field on the headline grid; the roofline of the
headline step kernel (algorithmic bytes over its measured duration) and the CPU oracle's rate
on this host's cores (a baseline only).

    python bench.py [--steps K] [--warmup W] [--no-extra] [--no-cpu] [--only NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E nominal
METRIC = "zone-group updates/s + HBM GB/s (FP64 vs FP32); adjoint/forward time ratio"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM traffic of the step kernel on the headline workload, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE counters scaled by the copy-kernel calibration (see the file); it applies only
# while the kernel sources are the ones it was measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_3d_core3d_192x192x192x12_fp64_traffic.json")
KERNEL_SOURCES = ["m1_step_3d.hip", "m1_device.h", "m1_internal.h"]
HEADLINE_KERNEL = "k_step_3d<double, 8, 2, 0, false, true, false>"


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1806_07390_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the headline step kernel, or None when not measured on the
    current kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_digest():
        return None
    return float(t["bytes_per_launch"])


def algorithmic_bytes(ndim, elem):
    """Bytes the step must move per zone-group: read E, F_1..F_D, kappa, sigma, B; write E, F."""
    return (2 * (1 + ndim) + 3) * elem


def device_inputs(w, dtype):
    import torch
    dev = "cuda"
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)
    E = t(w.E)
    F = [t(f) for f in w.F]
    k, s, B = t(w.kappa), t(w.sigma), t(w.B)
    inflow = None if w.inflow is None else torch.from_numpy(w.inflow).to(device=dev, dtype=torch.float64)
    return E, F, k, s, B, inflow


def time_steps(ctx, inputs, dt, steps, warmup, with_diag=True):
    """Average ms per step over `steps` steps (HIP events on the launch stream)."""
    import torch
    E, F, k, s, B, inflow = inputs
    a = (E.clone(), [f.clone() for f in F])
    b = ctx.empty_state()
    diag = ctx.new_diag() if with_diag else None
    step, _ = ctx.stepper(a, b, k, s, B, dt, inflow=inflow, diag=diag)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        step()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return ms, diag


def copy_bandwidth(nbytes=1 << 30, reps=20):
    import torch
    from paper_1806_07390_amd import m1
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        m1.copy_probe(dst, src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        m1.copy_probe(dst, src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2 * nbytes / (ms * 1e-3) / 1e9, ms


def adjoint_ratios(steps=20):
    """Adjoint/forward time ratios on the 2-D 256^2 x 16 FP32-bulk adjoint workload: per step
    (fornax_m1_adjoint given U^{n+1}, as in the checkpointed backward, and recomputing U^{n+1}
    itself, vs fornax_m1_step) and end to end (40-step differentiable run: backward, with the
    checkpoint replay, vs forward; the median of repetitions 3 to 5, after the caching
    allocator has its blocks and the backward pass its bound calls)."""
    import torch
    from paper_1806_07390_amd import m1, workloads as wl
    w = wl.adjoint2d()
    ctx = m1.Context(m1.Config.from_workload(w, precision=m1.MIXED))
    E, F, k, s, B, _ = device_inputs(w, torch.float32)
    fwd_ms, _ = time_steps(ctx, (E, F, k, s, B, None), w.dt, steps, 3, with_diag=False)
    lam = (torch.ones_like(E), [torch.zeros_like(f) for f in F])
    out = ctx.empty_state()
    dk = torch.zeros_like(E)
    U1 = ctx.step(E, F, k, s, B, w.dt)

    def time_adj(adj):
        for _ in range(3):
            adj()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            adj()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    adj_ms = time_adj(ctx.adjointer((E, F), k, s, B, w.dt, lam, out, dk, U1=U1))
    adj_rc_ms = time_adj(ctx.adjointer((E, F), k, s, B, w.dt, lam, out, dk))
    # end to end: 40 steps, checkpoints every 8
    ix, iy, ww = w.extra["window"]
    E0 = E.clone().requires_grad_(True)
    F0 = [f.clone().requires_grad_(True) for f in F]
    kk = k.clone().requires_grad_(True)
    e2e = []
    for rep in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        EN, FN = m1.run_differentiable(ctx, E0, F0, kk, s, B, w.dt, w.steps, ckpt_every=8)
        L = EN[0, iy:iy + ww, ix:ix + ww, :].sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rep >= 2:
            e2e.append((t2 - t1) / (t1 - t0))
    return dict(workload="2-D periodic 256x256 x 16 groups, FP32 bulk, 40 steps, checkpoints every 8",
                forward_ms_per_step=round(fwd_ms, 5), adjoint_ms_per_step=round(adj_ms, 5),
                adjoint_over_forward=round(adj_ms / fwd_ms, 3),
                adjoint_recomputing_step_ms=round(adj_rc_ms, 5),
                adjoint_recomputing_step_over_forward=round(adj_rc_ms / fwd_ms, 3),
                end_to_end_backward_over_forward=round(float(np.median(e2e)), 3),
                end_to_end_runs=[round(v, 3) for v in e2e])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, dt, target_s=20.0, single_s=8.0):
    """The CPU oracle on a bounded sample of the same workload: whole steps of the full grid
    with OpenMP over the host cores this process may use (the reported value), and one step at
    a random sample of zones on one thread."""
    import numpy as np
    from oracle import m1_oracle as orc
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    nthreads = int(omp) if omp and omp.isdigit() and int(omp) > 0 else ncores
    kw = dict(ndim=w.ndim, n=w.n, G=w.G, coord=w.coord, lo=w.lo, hi=w.hi, bc_lo=w.bc_lo, bc_hi=w.bc_hi, c=w.c)
    # one thread: one step at a sample of zones sized to about single_s seconds
    p1 = orc.Problem(nthreads=1, **kw)
    nz = w.zone_groups // w.G
    rng = np.random.default_rng(0)
    nsel = 2000
    zones = np.sort(rng.choice(nz, nsel, replace=False))
    t0 = time.perf_counter()
    orc.step_zones(p1, w.E, w.F, w.kappa, w.sigma, w.B, dt, zones, inflow=w.inflow)
    t1 = time.perf_counter()
    nsel = int(min(nz, max(2000, nsel * single_s / max(t1 - t0, 1e-3))))
    zones = np.sort(rng.choice(nz, nsel, replace=False))
    t0 = time.perf_counter()
    orc.step_zones(p1, w.E, w.F, w.kappa, w.sigma, w.B, dt, zones, inflow=w.inflow)
    t1 = time.perf_counter()
    single = dict(value=nsel * w.G / (t1 - t0), sample=f"one step at {nsel} random zones x {w.G} groups on 1 thread, "
                                                       f"{t1 - t0:.1f} s")
    # all threads: whole steps of the full grid, as many as fit target_s (at least one)
    p = orc.Problem(nthreads=nthreads, **kw)
    t0 = time.perf_counter()
    orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, 1, inflow=w.inflow)
    t1 = time.perf_counter()
    nsteps = max(1, min(200, int(target_s / max(t1 - t0, 1e-3))))
    t0 = time.perf_counter()
    orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, nsteps, inflow=w.inflow)
    t1 = time.perf_counter()
    zgu = w.zone_groups * nsteps / (t1 - t0)
    size = "x".join(str(v) for v in w.n[:w.ndim])
    return dict(value=zgu, unit="zone-group updates/s", cores=nthreads, kind="oracle",
                sample=f"{nsteps} full steps of the {size} x {w.G}-group workload, {nthreads} OpenMP threads, "
                       f"{t1 - t0:.1f} s",
                host_cores_available=ncores, single_thread=single, cpu_model=cpu_model())


def matter_timings(reps=10, steps=10):
    """The radiation-matter energy exchange on the 512^2 x 16 blob radiation with random matter
    (matter2d): the interaction update with the outer solve for T alone (each repetition from
    the same state, HIP events around the call only) and the coupled step (matter
    coefficients at T^n, explicit transport, interaction update) over `steps` steps."""
    import torch
    from paper_1806_07390_amd import m1, workloads as wl
    w = wl.matter2d()
    g = w.groups
    out = {"workload": "2-D periodic 512x512 x 16 groups, blob radiation, random matter T, cv, kappa0 (seed 0)"}
    for prec, name, dtp, el in ((m1.FP64, "fp64", torch.float64, 8), (m1.MIXED, "mixed", torch.float32, 4)):
        ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
        ctx.set_matter_model(g.nu_edge, g.nu_c, g.kg, a_rad=g.a_rad)
        E0, F0 = (torch.from_numpy(w.E).to("cuda", dtp), [torch.from_numpy(f).to("cuda", dtp) for f in w.F])
        sig = torch.from_numpy(w.sigma).to("cuda", dtp)
        cv, k0, T0 = (torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (w.cv, w.kappa0, w.T))
        E, F, T = E0.clone(), [f.clone() for f in F0], T0.clone()
        it = torch.zeros(ctx.nzones, dtype=torch.int32, device="cuda")
        st = torch.cuda.current_stream()
        tot = 0.0
        for r in range(reps + 2):
            E.copy_(E0)
            for f, f0 in zip(F, F0):
                f.copy_(f0)
            T.copy_(T0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            ctx.matter_source(E, F, sig, cv, k0, T, w.dt, iters=it)
            e1.record(st)
            torch.cuda.synchronize()
            if r >= 2:
                tot += e0.elapsed_time(e1)
        ms_src = tot / reps
        iters = it.abs().double().mean().item()
        # coupled steps from the initial state
        E, F, T = E0.clone(), [f.clone() for f in F0], T0.clone()
        Eb, Fb = ctx.empty_state()
        for _ in range(2):
            ctx.matter_step(E, F, sig, cv, k0, T, w.dt, out=(Eb, Fb))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        a, b = (E, F), (Eb, Fb)
        for _ in range(steps):
            ctx.matter_step(a[0], a[1], sig, cv, k0, T, w.dt, out=b)
            a, b = b, a
        e1.record(st)
        torch.cuda.synchronize()
        ms_step = e0.elapsed_time(e1) / steps
        bytes_src = w.zone_groups * (7 * el) + w.n[0] * w.n[1] * 5 * 8
        out[name] = dict(interaction_update_ms=round(ms_src, 5),
                         interaction_update_zgu_per_s=w.zone_groups / (ms_src * 1e-3),
                         interaction_update_algorithmic_GBps=round(bytes_src / (ms_src * 1e-3) / 1e9, 1),
                         mean_newton_iterations=round(iters, 3),
                         coupled_step_ms=round(ms_step, 5),
                         coupled_step_zgu_per_s=w.zone_groups / (ms_step * 1e-3))
        del ctx
        torch.cuda.empty_cache()
    return out


def velocity_timings(steps=10, warmup=3):
    """The step with a prescribed velocity field (fornax_m1_step_velocity: Steps 1 to 4) on the
    192^3 x 12 grid of the headline, a smooth random face velocity up to about 0.1 c with noise,
    FP64 and MIXED.  Algorithmic bytes: the static step's plus the face velocities (3 faces x 3
    components per zone)."""
    import torch
    from paper_1806_07390_amd import m1, workloads as wl
    w = wl.core3d()
    vf = wl.face_velocity(w, amp=0.1, seed=5)
    nu = wl.velocity_edges(w.G)
    out = dict(workload="3-D Cartesian 192^3 x 12 (the headline grid), smooth random face velocity |v| <~ 0.1 c "
                        "plus noise (seed 5), groups edged 0, 0.5 .. 20 (log), 40")
    for prec, name, dtp, el in ((m1.FP64, "fp64", torch.float64, 8), (m1.MIXED, "mixed", torch.float32, 4)):
        ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
        ctx.set_group_edges(nu)
        E, F, k, s, B, _ = device_inputs(w, dtp)
        V = [torch.from_numpy(v).to(device="cuda", dtype=dtp) for v in vf]
        a = (E, F)
        b = ctx.empty_state()
        dg = ctx.new_diag()
        for _ in range(warmup):
            ctx.step_velocity(a[0], a[1], k, s, B, V, w.dt, out=b, diag=dg)
            a, b = b, a
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(steps):
            ctx.step_velocity(a[0], a[1], k, s, B, V, w.dt, out=b, diag=dg)
            a, b = b, a
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        bpz = algorithmic_bytes(3, el) + 9 * el / w.G
        out[name] = dict(ms_per_step=round(ms, 5), zgu_per_s=w.zone_groups / (ms * 1e-3),
                         algorithmic_bytes_per_zone_group=round(bpz, 2),
                         algorithmic_GBps=round(w.zone_groups * bpz / (ms * 1e-3) / 1e9, 1),
                         over_static_step=None)
        del ctx, E, F, k, s, B, V, a, b
        torch.cuda.empty_cache()
    return out


def step_timing(w, prec, dtp, steps, warmup, dt=None):
    """(ms per full step with diagnostics, ms per step-kernel launch alone, final diag) on the
    workload w in precision prec: HIP events on the launch stream."""
    import torch
    from paper_1806_07390_amd import m1
    ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
    dt = w.dt if dt is None else dt
    inp = device_inputs(w, dtp)
    ms, diag = time_steps(ctx, inp, dt, steps, warmup, with_diag=True)
    ms_k, _ = time_steps(ctx, inp, dt, steps, 2, with_diag=False)
    diag = {k: v.cpu() for k, v in diag.items()}
    del ctx, inp
    torch.cuda.empty_cache()
    return ms, ms_k, diag


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", default=None,
                    help="profiling: run only this workload's timed loop (core3d, core3d_mixed, blobs2d, sphere3d, "
                         "options, matter, adjoint, velocity, extras = all after the headline, copy = the copy "
                         "probe alone)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the library has no multi-GPU "
              "path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1806_07390_amd import m1, workloads as wl

    torch.cuda.set_device(0)
    res = {}
    extra = {}
    # ---- headline: 3-D Cartesian 192^3 x 12 groups, FP64 -----------------------------------
    w = wl.core3d()
    if args.only in (None, "core3d"):
        log("headline: core3d", w.n, w.G)
        ms, ms_k, diag = step_timing(w, m1.FP64, torch.float64, args.steps, args.warmup)
        zg = w.zone_groups
        bpz = algorithmic_bytes(w.ndim, 8)
        res["headline"] = dict(ms=ms, value=zg / (ms * 1e-3), ms_kernel=ms_k, achieved=zg * bpz / (ms_k * 1e-3) / 1e9,
                               bpz=bpz, energy=float(diag["energy_total"].item()),
                               n_unrealizable=int(diag["n_unrealizable"].item()))
        h = res["headline"]
        log(f"  {ms:.4f} ms/step, {h['value']:.3e} zgu/s; kernel {ms_k:.4f} ms -> {h['achieved']:.0f} GB/s algorithmic")
    # ---- the same grid with float storage (MIXED) ------------------------------------------
    if args.only in (None, "core3d_mixed"):
        ms, ms_k, _ = step_timing(w, m1.MIXED, torch.float32, args.steps, args.warmup)
        b = algorithmic_bytes(3, 4)
        extra["core3d_192^3x12_mixed"] = dict(ms_per_step=round(ms, 5), zgu_per_s=w.zone_groups / (ms * 1e-3),
                                              kernel_ms=round(ms_k, 5), bytes_per_zone_group=b,
                                              algorithmic_GBps=round(w.zone_groups * b / (ms_k * 1e-3) / 1e9, 1),
                                              kernel="k_step_3d<float, 8, 4, 0, false, false, false>")
        log(f"  core3d mixed: {ms:.4f} ms/step, kernel {ms_k:.4f} ms")
    if not args.no_extra:
        # ---- 2-D 512^2 x 16: FP64 (whole-zone kernel) and MIXED ----------------------------
        if args.only in (None, "extras", "blobs2d"):
            w2 = wl.blobs2d()
            for prec, name, dt_, el in ((m1.FP64, "fp64", torch.float64, 8), (m1.MIXED, "mixed", torch.float32, 4)):
                ms2, ms2k, _ = step_timing(w2, prec, dt_, 100, 300)
                b = algorithmic_bytes(2, el)
                extra[f"blobs2d_512^2x16_{name}"] = dict(ms_per_step=round(ms2, 5), zgu_per_s=w2.zone_groups / (ms2 * 1e-3),
                                                         kernel_ms=round(ms2k, 5),
                                                         algorithmic_GBps=round(w2.zone_groups * b / (ms2k * 1e-3) / 1e9, 1))
                log(f"  blobs2d {name}: {ms2:.4f} ms/step, kernel {ms2k:.4f} ms")
            del w2
        # ---- spherical 256x64x128 x 20 ------------------------------------------------------
        if args.only in (None, "extras", "sphere3d"):
            w4 = wl.sphere3d()
            for prec, name, dt_, el in ((m1.MIXED, "mixed", torch.float32, 4), (m1.FP64, "fp64", torch.float64, 8)):
                ctx = m1.Context(m1.Config.from_workload(w4, precision=prec))
                dt4 = ctx.max_dt(w4.cfl)
                del ctx
                ms4, ms4k, _ = step_timing(w4, prec, dt_, 20, 3, dt=dt4)
                gbs = w4.zone_groups * algorithmic_bytes(3, el) / (ms4k * 1e-3) / 1e9
                extra[f"sphere3d_256x64x128x20_{name}"] = dict(ms_per_step=round(ms4, 5),
                                                               zgu_per_s=w4.zone_groups / (ms4 * 1e-3),
                                                               kernel_ms=round(ms4k, 5), algorithmic_GBps=round(gbs, 1),
                                                               kernel=("k_step_3d<double, 8, 2, 0, true, true, false>" if el == 8 else
                                                                       "k_step_3d<float, 12, 3, 0, true, true, false>"))
                log(f"  sphere3d {name}: {ms4:.4f} ms/step, {gbs:.0f} GB/s")
            del w4
        # ---- the reconstruction and wavespeed options on the 2-D grid ----------------------
        if args.only in (None, "extras", "options"):
            wo = wl.blobs2d()
            inps = {m1.FP64: device_inputs(wo, torch.float64), m1.MIXED: device_inputs(wo, torch.float32)}
            opts = {"fp64_ppm": (m1.FP64, dict(limiter=m1.LIMITER_PPM)),
                    "fp64_m1_speeds": (m1.FP64, dict(wavespeed=m1.WAVESPEED_M1)),
                    "fp64_minmod_tiled": (m1.FP64, dict(limiter=m1.LIMITER_MINMOD))}
            for name, (prec, kw) in opts.items():
                if name == "fp64_minmod_tiled":
                    os.environ["FORNAX_M1_ROWS"] = "0"
                try:
                    ctx = m1.Context(m1.Config.from_workload(wo, precision=prec, **kw))
                finally:
                    os.environ.pop("FORNAX_M1_ROWS", None)
                mso, _ = time_steps(ctx, inps[prec], wo.dt, 50, 20, with_diag=True)
                el = 8 if prec == m1.FP64 else 4
                gbs = wo.zone_groups * algorithmic_bytes(2, el) / (mso * 1e-3) / 1e9
                extra[f"blobs2d_512^2x16_{name}"] = dict(ms_per_step=round(mso, 5),
                                                         zgu_per_s=wo.zone_groups / (mso * 1e-3),
                                                         algorithmic_GBps=round(gbs, 1))
                log(f"  blobs2d {name}: {mso:.4f} ms/step, {gbs:.0f} GB/s")
                del ctx
            del inps, wo
            torch.cuda.empty_cache()
        if args.only in (None, "extras", "matter"):
            extra["matter"] = matter_timings()
            log("  matter:", extra["matter"])
        if args.only in (None, "extras", "adjoint"):
            extra["adjoint"] = adjoint_ratios()
            log("  adjoint:", extra["adjoint"])
        if args.only in (None, "extras", "velocity"):
            extra["velocity"] = velocity_timings()
            if "headline" in res:
                extra["velocity"]["fp64"]["over_static_step"] = round(
                    extra["velocity"]["fp64"]["ms_per_step"] / res["headline"]["ms"], 3)
            if "core3d_192^3x12_mixed" in extra:
                extra["velocity"]["mixed"]["over_static_step"] = round(
                    extra["velocity"]["mixed"]["ms_per_step"] / extra["core3d_192^3x12_mixed"]["ms_per_step"], 3)
            log("  velocity:", extra["velocity"])
        if args.only in (None, "extras", "copy"):
            copy_gbs, copy_ms = copy_bandwidth()
            extra["copy_probe_GBps"] = round(copy_gbs, 1)
            if "headline" in res:
                res["headline"]["frac_of_copy"] = res["headline"]["achieved"] / copy_gbs
            log(f"  copy probe: {copy_gbs:.0f} GB/s")
    if "headline" not in res:
        print(json.dumps(dict(extra=extra)))
        return
    h = res["headline"]
    out = {
        "metric": METRIC,
        "value": h["value"],
        "unit": "zone-group updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3-D Cartesian 192x192x192 zones x 12 groups, FP64, outflow, optically thick core "
                               "(kappa 1e3 within r < 0.2) in a thin halo (1e-2), Planck group weights, seeded noise "
                               "(seed 0)", "zones": list(w.n), "groups": w.G, "zone_groups": w.zone_groups,
                   "dt": w.dt},
        "roofline": {"bound": "hbm", "achieved": round(h["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(h["achieved"] / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": HEADLINE_KERNEL, "bytes_per_zone_group": h["bpz"],
                     "kernel_ms": round(h["ms_kernel"], 5),
                     "frac_of_copy_probe": (round(h["frac_of_copy"], 4) if "frac_of_copy" in h else None)},
        "extra": extra,
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)...")
        out["cpu_baseline"] = cpu_baseline(w, w.dt)
        log("  ", out["cpu_baseline"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
