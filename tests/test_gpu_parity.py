"""GPU parity: the HIP library (through the C interface) against the CPU FP64 oracle on the
same seeded inputs.  Reduced sizes span several blocks and ragged tails; the full workload
sizes are checked on sampled zones of one step, in the launch configuration of bench.py."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import m1_oracle as orc
from paper_1806_07390_amd import workloads as wl
from tests.parity_util import (TOL_FP64, TOL_MIXED_RUN, TOL_MIXED_STEP, check_pointwise, gpu_run, problem_of, rel_l1,
                               to_dev,
                               to_host)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m1():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1806_07390_amd import m1 as mod
    return mod


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dt_of(w, p):
    return w.dt if w.dt is not None else orc.max_dt(p, w.cfl)


def run_pair(m1, w, precision, nsteps, **opts):
    p = problem_of(w, **{k: v for k, v in opts.items() if k in ("limiter", "closure")})
    dt = dt_of(w, p)
    say(f"case {w.name} n={w.n} G={w.G} prec={precision} steps={nsteps} opts={opts}")
    E, F, _ = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, nsteps, inflow=w.inflow)
    cfg = m1.Config.from_workload(w, precision=precision, **opts)
    ctx = m1.Context(cfg)
    Eg, Fg = gpu_run(ctx, w, dt, nsteps)
    e = rel_l1(Eg, Fg, E, F, w.c)
    say(f"  rel-L1 E {e[0]:.2e} F {e[1]:.2e}; element-wise E {e.pE:.2e} F {e.pF:.2e}")
    check_pointwise(e, precision == m1.FP64, w.name)
    return e


# ------------------------------------------------------------------------------------------
def test_slab1d_full_fp64(m1):
    w = wl.slab1d()
    eE, eF = run_pair(m1, w, m1.FP64, w.steps)
    say("slab1d", eE, eF)
    assert eE <= TOL_FP64 and eF <= TOL_FP64


@pytest.mark.parametrize("n", [(64, 64), (45, 37)])
def test_blobs2d_fp64(m1, n):
    w = wl.blobs2d(n=n[0], G=4, steps=20)
    if n[0] != n[1]:
        # ragged, non-square: slice the square input
        w.E = np.ascontiguousarray(w.E[:, : n[1], : n[0]])
        w.F = [np.ascontiguousarray(f[:, : n[1], : n[0]]) for f in w.F]
        w.kappa = np.ascontiguousarray(w.kappa[:, : n[1], : n[0]])
        w.sigma = np.ascontiguousarray(w.sigma[:, : n[1], : n[0]])
        w.B = np.ascontiguousarray(w.B[:, : n[1], : n[0]])
        w.n = (n[0], n[1], 1)
    eE, eF = run_pair(m1, w, m1.FP64, w.steps)
    say("blobs2d", n, eE, eF)
    assert eE <= TOL_FP64 and eF <= TOL_FP64


def test_blobs2d_options_fp64(m1):
    w = wl.blobs2d(n=24, G=3, steps=8)
    for opts in (dict(limiter=m1.LIMITER_MC), dict(limiter=m1.LIMITER_NONE), dict(closure=m1.CLOSURE_EDDINGTON)):
        eE, eF = run_pair(m1, w, m1.FP64, w.steps, **opts)
        assert eE <= TOL_FP64 and eF <= TOL_FP64, opts


def test_core3d_reduced_fp64_and_mixed(m1):
    w = wl.core3d(n=20, G=12, steps=10)
    eE, eF = run_pair(m1, w, m1.FP64, w.steps)
    say("core3d fp64", eE, eF)
    assert eE <= TOL_FP64 and eF <= TOL_FP64
    eE1, eF1 = run_pair(m1, w, m1.MIXED, 1)
    eEn, eFn = run_pair(m1, w, m1.MIXED, w.steps)
    say("core3d mixed", eE1, eF1, eEn, eFn)
    assert eE1 <= TOL_MIXED_STEP and eF1 <= TOL_MIXED_STEP
    assert eEn <= TOL_MIXED_RUN and eFn <= TOL_MIXED_RUN


@pytest.mark.parametrize("case", ["blobs2d", "core3d", "sphere3d"])
def test_mixed_after_100_steps(m1, case):
    """FP32 bulk with FP64 where the error concentrates stays within 1e-4 (rel-L1) of the FP64
    oracle after 100 steps, at reduced sizes of the three workloads."""
    if case == "blobs2d":
        w = wl.blobs2d(n=48, G=16, steps=100)
    elif case == "core3d":
        w = wl.core3d(n=20, G=12, steps=100)
    else:
        w = wl.sphere3d(nr=24, nth=16, nph=16, G=4, steps=100)
    eE, eF = run_pair(m1, w, m1.MIXED, 100)
    say(f"{case} mixed after 100 steps", eE, eF)
    assert eE <= TOL_MIXED_RUN and eF <= TOL_MIXED_RUN


def test_sphere_reduced_fp64_and_mixed(m1):
    w = wl.sphere3d(nr=24, nth=16, nph=16, G=4, steps=20)
    eE, eF = run_pair(m1, w, m1.FP64, w.steps)
    say("sphere fp64", eE, eF)
    assert eE <= TOL_FP64 and eF <= TOL_FP64
    eE1, eF1 = run_pair(m1, w, m1.MIXED, w.steps)
    say("sphere mixed", eE1, eF1)
    assert eE1 <= TOL_MIXED_RUN and eF1 <= TOL_MIXED_RUN


def test_sphere_2d_axisymmetric_fp64(m1):
    w = wl.sphere3d(nr=20, nth=12, nph=1, G=3, steps=15, ndim=2)
    eE, eF = run_pair(m1, w, m1.FP64, w.steps)
    assert eE <= TOL_FP64 and eF <= TOL_FP64


def test_reflect_boundaries_fp64(m1):
    w = wl.blobs2d(n=20, G=2, steps=6)
    w.bc_lo = (wl.BC_REFLECT, wl.BC_OUTFLOW, 0)
    w.bc_hi = (wl.BC_OUTFLOW, wl.BC_REFLECT, 0)
    eE, eF = run_pair(m1, w, m1.FP64, w.steps)
    assert eE <= TOL_FP64 and eF <= TOL_FP64


@pytest.mark.parametrize("case", ["2d", "3d", "sph3d"])
def test_tile_shapes(m1, case):
    """The step kernel's tiling (zone columns per block, planes per block, groups per block)
    changes the work decomposition only: every tiling gives the oracle's result."""
    import os
    if case == "2d":
        # "TXB,TYB,TM,GB[,NW[,V]]": with NW >= 1 a wave holds 64 V/GB zone columns of GB
        # groups (V per lane) and a block NW such waves; with NW = 0 a block holds TXB columns
        w = wl.blobs2d(n=70, G=8, steps=5)
        tiles = ["0,1,1,1", "0,1,7,2,2", "0,1,16,4", "0,1,5,8,1", "0,1,3,1,4", "16,1,8,8,0", "5,1,3,2,0",
                 "0,1,8,8,1,2", "0,1,3,4,2,2", "0,1,6,2,4,2"]
    elif case == "3d":
        w = wl.core3d(n=14, G=6, steps=5)
        tiles = ["4,4,3,6", "6,5,2,2", "5,7,4,3", "8,6,16,1", "6,6,4,6,1,2", "9,7,3,2,1,2"]
    else:
        w = wl.sphere3d(nr=14, nth=10, nph=8, G=4, steps=5)
        tiles = ["4,4,3,4", "6,5,2,2", "7,4,5,1", "5,6,4,4,1,2"]
    p = problem_of(w)
    dt = dt_of(w, p)
    E, F, dg, dEm = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, w.steps, inflow=w.inflow, want_dEm=True)
    for prec, tol in ((m1.FP64, TOL_FP64), (m1.MIXED, TOL_MIXED_RUN)):
        for tile in tiles:
            say(f"case {case} tile {tile} prec {prec}")
            os.environ["FORNAX_M1_TILE"] = tile
            try:
                ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
            finally:
                del os.environ["FORNAX_M1_TILE"]
            Eg, Fg, dgg = gpu_run(ctx, w, dt, w.steps, diag=True)
            e = rel_l1(Eg, Fg, E, F, w.c)
            eE, eF = e
            check_pointwise(e, prec == m1.FP64)
            say("   ", eE, eF)
            assert eE <= tol and eF <= tol, (case, tile, prec)
            # the group sum of dE_matter spans the blocks of a tile's group subsets.  It is a
            # difference of nearly equal energies (after and before the interaction update),
            # so its rounding error scales with E, not with itself
            if prec == m1.FP64:
                atol = 1e-12 * np.abs(E).max()
                assert np.allclose(dgg["dE_matter"], dEm, rtol=1e-10, atol=atol), tile
                assert dgg["energy_total"][0] == pytest.approx(dg["energy_total"], rel=1e-12)
            else:
                assert dgg["energy_total"][0] == pytest.approx(dg["energy_total"], rel=1e-5)


def _c3_case(n=(37, 23, 19), G=8, steps=6, seed=11, bcs="outflow"):
    """A 3-D Cartesian grid for the whole-zone 3-D kernel: x not a multiple of its 14 updated
    columns, y not a multiple of any block's interior rows, a z run shorter than a plane
    window; lognormal E with F up to 0.95 cE in random directions, opacities from the
    free-streaming to the diffusive limit of the HLL flux (tau = kappa dx from 1e-3 to 1e2)."""
    rng = np.random.default_rng(seed)
    n0, n1, n2 = n
    shape = (n2, n1, n0, G)
    E = np.exp(rng.normal(0.0, 1.0, shape))
    f = 0.95 * rng.random(shape)
    d = rng.normal(size=(3,) + shape)
    d /= np.linalg.norm(d, axis=0)
    F = [np.ascontiguousarray(f * E * d[k]) for k in range(3)]
    kappa = 10.0 ** rng.uniform(-3.0, 2.0, shape) * n0
    sigma = 0.3 * kappa * rng.random(shape)
    B = np.exp(rng.normal(0.0, 0.5, shape))
    if bcs == "outflow":
        lo, hi = (wl.BC_OUTFLOW,) * 3, (wl.BC_OUTFLOW,) * 3
    else:  # periodic x, reflect/outflow y, outflow/reflect z
        lo = (wl.BC_PERIODIC, wl.BC_REFLECT, wl.BC_OUTFLOW)
        hi = (wl.BC_PERIODIC, wl.BC_OUTFLOW, wl.BC_REFLECT)
    return wl.Workload("c3case", 3, n, G, wl.CARTESIAN, (0.0, 0.0, 0.0), (1.0, n1 / n0, n2 / n0), lo, hi, 1.0, steps,
                       E, F, kappa, sigma, B, dt=0.3 / (3 * n0))


@pytest.mark.parametrize("bcs", ["outflow", "mixed"])
def test_3d_kernel_tiles(m1, bcs):
    """The whole-zone 3-D kernel at each block height it is built for (y rows per block, z
    planes per block): every one gives the oracle's result element by element, with the energy
    diagnostics and the per-zone interaction energy summed over groups."""
    import os
    w = _c3_case(bcs=bcs)
    p = problem_of(w)
    dt = dt_of(w, p)
    E, F, dg, dEm = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, w.steps, want_dEm=True)
    cases = ((m1.FP64, TOL_FP64, ["8,32", "6,5", "12,3", "8,1", "8,19"]),
             (m1.MIXED, TOL_MIXED_RUN, ["8,32", "4,7", "16,2", "8,64", "12,5"]))
    for prec, tol, tiles in cases:
        for tile in tiles:
            say(f"case 3-D kernel {bcs} tile {tile} prec {prec}")
            os.environ["FORNAX_M1_C3"] = tile
            try:
                ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
            finally:
                del os.environ["FORNAX_M1_C3"]
            Eg, Fg, dgg = gpu_run(ctx, w, dt, w.steps, diag=True)
            e = rel_l1(Eg, Fg, E, F, w.c)
            say(f"  rel-L1 E {e[0]:.2e} F {e[1]:.2e}; element-wise E {e.pE:.2e} F {e.pF:.2e}")
            check_pointwise(e, prec == m1.FP64, f"3-D kernel {tile}")
            assert e[0] <= tol and e[1] <= tol, (tile, prec)
            if prec == m1.FP64:
                atol = 1e-12 * np.abs(E).max()
                assert np.allclose(dgg["dE_matter"], dEm, rtol=1e-10, atol=atol), tile
                assert dgg["energy_total"][0] == pytest.approx(dg["energy_total"], rel=1e-12)
                assert int(dgg["n_unrealizable"][0]) == dg["n_unrealizable"]
            else:
                assert dgg["energy_total"][0] == pytest.approx(dg["energy_total"], rel=1e-5)


def _rows_case(bc, n0=70, n1=40, G=16, steps=4):
    """A 2-D, 16-group grid of the whole-zone kernel's kind: 70 columns (five tiles of 14 updated
    columns) by 40 rows (planes per block not dividing it)."""
    w = wl.blobs2d(n=n0, G=G, steps=steps)
    w.E = np.ascontiguousarray(w.E[:, :n1])
    w.F = [np.ascontiguousarray(f[:, :n1]) for f in w.F]
    w.kappa = np.ascontiguousarray(w.kappa[:, :n1])
    w.sigma = np.ascontiguousarray(w.sigma[:, :n1])
    w.B = np.ascontiguousarray(w.B[:, :n1])
    w.n = (n0, n1, 1)
    if bc == "outflow_reflect":
        w.bc_lo = (wl.BC_REFLECT, wl.BC_OUTFLOW, 0)
        w.bc_hi = (wl.BC_OUTFLOW, wl.BC_REFLECT, 0)
    elif bc == "inflow":
        w.bc_lo = (wl.BC_INFLOW, wl.BC_REFLECT, 0)
        w.bc_hi = (wl.BC_OUTFLOW, wl.BC_OUTFLOW, 0)
        rng = np.random.default_rng(7)
        w.inflow = np.zeros((G, 3))
        w.inflow[:, 0] = rng.uniform(0.2, 1.0, G)
        w.inflow[:, 1] = 0.6 * w.c * w.inflow[:, 0]
        w.inflow[:, 2] = -0.2 * w.c * w.inflow[:, 0]
    return w


@pytest.mark.parametrize("bc", ["periodic", "outflow_reflect", "inflow"])
@pytest.mark.parametrize("lim", ["minmod", "mc", "ppm"])
def test_whole_zone_kernel(m1, bc, lim):
    """The 2-D, 16-group kernel that moves whole zones through LDS gives the oracle's result and
    that of the tiled kernel (FORNAX_M1_ROWS selects either: "NWX,TM" the whole-zone kernel,
    "0" the tiled one), in both precisions: the same arithmetic in the same order, up to where
    the compiler fuses a multiply and an add.  Blocks of 9 planes (the last one 4) and of 3
    (the last one 1: a single plane after the prologue)."""
    import os
    code = {"minmod": m1.LIMITER_MINMOD, "mc": m1.LIMITER_MC, "ppm": m1.LIMITER_PPM}[lim]
    w = _rows_case(bc)
    p = problem_of(w, limiter=code)
    dt = dt_of(w, p)
    E, F, dg, dEm = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, w.steps, inflow=w.inflow, want_dEm=True)
    for prec, tol in ((m1.FP64, TOL_FP64), (m1.MIXED, TOL_MIXED_RUN)):
        say(f"whole-zone kernel bc={bc} lim={lim} prec={prec}")
        ctxs = []
        for rows in ("0", "1,9", "1,3"):
            os.environ["FORNAX_M1_ROWS"] = rows
            try:
                ctxs.append(m1.Context(m1.Config.from_workload(w, precision=prec, limiter=code)))
            finally:
                del os.environ["FORNAX_M1_ROWS"]
        Et, Ft, dgt = gpu_run(ctxs[0], w, dt, w.steps, diag=True)
        for ctx in ctxs[1:]:
            Eg, Fg, dgg = gpu_run(ctx, w, dt, w.steps, diag=True)
            e = rel_l1(Eg, Fg, E, F, w.c)
            eE, eF = e
            check_pointwise(e, prec == m1.FP64)
            say("   ", eE, eF)
            assert eE <= tol and eF <= tol
            tE, tF = rel_l1(Eg, Fg, Et, Ft, w.c)
            say("    vs tiled", tE, tF)
            close = 1e-14 if prec == m1.FP64 else 1e-6
            assert tE <= close and tF <= close
            assert np.allclose(dgg["dE_matter"], dgt["dE_matter"], rtol=0, atol=close * np.abs(Et).max())
            assert dgg["energy_total"][0] == pytest.approx(dgt["energy_total"][0], rel=close)
            assert dgg["max_f"][0] == pytest.approx(dgt["max_f"][0], rel=close)
            assert dgg["n_unrealizable"][0] == dgt["n_unrealizable"][0]
            assert dgg["n_nonpositive"][0] == dgt["n_nonpositive"][0]
            if prec == m1.FP64:
                assert np.allclose(dgg["dE_matter"], dEm, rtol=1e-10, atol=1e-12 * np.abs(E).max())


def test_whole_zone_kernel_diagnostics_each_step(m1):
    """The whole-zone kernel's block partials of the diagnostics, summed by the second launch:
    each of several steps on one context reports the totals of its own output -- the volume
    sum of E, the largest f = |F|/(cE), the realizability and positivity counts -- also when
    the state changes by a large factor between calls and when steps without diagnostics come
    in between, so no partial of an earlier launch carries over."""
    import os
    w = _rows_case("periodic")
    p = problem_of(w)
    dt = dt_of(w, p)
    V = orc.geometry(p)["vol"].reshape(-1)
    os.environ["FORNAX_M1_ROWS"] = "1,9"
    try:
        ctx = m1.Context(m1.Config.from_workload(w, precision=m1.FP64))
    finally:
        del os.environ["FORNAX_M1_ROWS"]
    E0 = to_dev(w.E, torch.float64)
    F0 = [to_dev(f, torch.float64) for f in w.F]
    k, s, B0 = (to_dev(x, torch.float64) for x in (w.kappa, w.sigma, w.B))
    u = 2.0 ** -53
    for scale, plain_before in ((1.0, False), (3.0, True), (0.25, False), (1e3, True)):
        E, F, B = E0 * scale, [f * scale for f in F0], B0 * scale
        if plain_before:
            ctx.step(E, F, k, s, B, dt)
        dg = ctx.new_diag()
        Eo, Fo = ctx.step(E, F, k, s, B, dt, diag=dg)
        torch.cuda.synchronize()
        say(f"fused diagnostics scale={scale}")
        Eh = to_host(Eo).reshape(len(V), -1)
        Fh = [to_host(f).reshape(len(V), -1) for f in Fo[:2]]
        e_ref = float(np.sum(V[:, None] * Eh))
        assert dg["energy_total"].item() == pytest.approx(e_ref, rel=1e-13)
        F2 = Fh[0] ** 2 + Fh[1] ** 2
        cE = w.c * Eh
        pos = Eh > 0
        f_ref = float(np.sqrt((F2[pos] / cE[pos] ** 2).max()))
        assert dg["max_f"].item() == pytest.approx(f_ref, rel=1e-13)
        n_un = int(np.count_nonzero(np.sqrt(F2) > cE * (1 + 8 * u)))
        assert int(dg["n_unrealizable"].item()) == n_un
        assert int(dg["n_nonpositive"].item()) == int(np.count_nonzero(~pos))


@pytest.mark.parametrize("case", ["blobs2d", "reflect2d", "core3d", "sphere3d"])
def test_ssprk2_matches_oracle(m1, case):
    """Shu-Osher SSP-RK2 for the transport (two launches of the step kernel, U* in context
    scratch), the interaction update once per step: the oracle's result in FP64 and MIXED, and
    dE_matter against the averaged U^-."""
    if case == "blobs2d":
        w = wl.blobs2d(n=40, G=16, steps=5)
    elif case == "reflect2d":
        w = _rows_case("outflow_reflect", steps=5)
    elif case == "core3d":
        w = wl.core3d(n=14, G=6, steps=5)
    else:
        w = wl.sphere3d(nr=14, nth=10, nph=8, G=4, steps=5)
    p = problem_of(w, integrator=orc.SSPRK2)
    dt = dt_of(w, p)
    E, F, dg, dEm = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, w.steps, inflow=w.inflow, want_dEm=True)
    Ee, Fe, _ = orc.run(problem_of(w), w.E, w.F, w.kappa, w.sigma, w.B, dt, w.steps, inflow=w.inflow)
    assert rel_l1(Ee, Fe, E, F, w.c)[0] > 1e-9      # the integrators differ
    for prec, tol in ((m1.FP64, TOL_FP64), (m1.MIXED, TOL_MIXED_RUN)):
        ctx = m1.Context(m1.Config.from_workload(w, precision=prec, integrator=m1.SSPRK2))
        Eg, Fg, dgg = gpu_run(ctx, w, dt, w.steps, diag=True)
        e = rel_l1(Eg, Fg, E, F, w.c)
        eE, eF = e
        check_pointwise(e, prec == m1.FP64)
        say(f"ssprk2 {case} prec={prec}", eE, eF)
        assert eE <= tol and eF <= tol
        if prec == m1.FP64:
            assert np.allclose(dgg["dE_matter"], dEm, rtol=1e-10, atol=1e-12 * np.abs(E).max())
            assert dgg["energy_total"][0] == pytest.approx(dg["energy_total"], rel=1e-12)


def test_adjoint_refuses_ssprk2(m1):
    w = wl.adjoint2d(n=16, G=2, steps=1)
    ctx = m1.Context(m1.Config.from_workload(w, precision=m1.FP64, integrator=m1.SSPRK2))
    t = lambda a: to_dev(a, torch.float64)
    z = [torch.zeros_like(t(w.E)) for _ in w.F]
    with pytest.raises(m1.FornaxError) as ei:
        ctx.adjoint(t(w.E), [t(f) for f in w.F], t(w.kappa), t(w.sigma), t(w.B), w.dt, t(w.E), z)
    assert ei.value.code == m1.FORNAX_EUNSUPPORTED


# ------------------------------------------------------------------------------------------
def test_flux_and_source_entry_points(m1):
    w = wl.sphere3d(nr=12, nth=8, nph=8, G=3, steps=1)
    rng = np.random.default_rng(2)
    w.E = w.B * (1 + rng.random(w.E.shape))
    w.F = [0.3 * w.E * rng.uniform(-1, 1, w.E.shape) for _ in range(3)]
    p = problem_of(w)
    ctx = m1.Context(m1.Config.from_workload(w))
    E = to_dev(w.E, torch.float64)
    F = [to_dev(f, torch.float64) for f in w.F]
    k, s, B = (to_dev(x, torch.float64) for x in (w.kappa, w.sigma, w.B))
    inflow = to_dev(w.inflow, torch.float64)
    fl = ctx.flux(E, F, k, s, B, inflow=inflow)
    for d in range(3):
        ref = orc.flux(p, w.E, w.F, w.kappa, w.sigma, w.B, d, inflow=w.inflow)
        got = to_host(fl[d])
        scale = np.abs(ref).max()
        assert np.max(np.abs(got - ref)) <= 1e-13 * scale, d
    Es, Fs, dEm = orc.source(p, w.E, w.F, w.kappa, w.sigma, w.B, 0.05)
    dE = torch.zeros(ctx.nzones, dtype=torch.float64, device="cuda")
    ctx.source(E, F, k, s, B, 0.05, dE_matter=dE)
    assert np.allclose(to_host(E), Es, rtol=1e-14, atol=0)
    for kk in range(3):
        assert np.allclose(to_host(F[kk]), Fs[kk], rtol=1e-14, atol=0)
    assert np.allclose(dE.cpu().numpy(), dEm, rtol=1e-12, atol=1e-15 * np.abs(dEm).max())


def test_diagnostics_match_oracle(m1):
    w = wl.blobs2d(n=40, G=4, steps=3)
    p = problem_of(w)
    E, F, dg, dEm = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, w.dt, w.steps, want_dEm=True)
    ctx = m1.Context(m1.Config.from_workload(w))
    Eg, Fg, dgg = gpu_run(ctx, w, w.dt, w.steps, diag=True)
    assert dgg["energy_total"][0] == pytest.approx(dg["energy_total"], rel=1e-13)
    assert dgg["max_f"][0] == pytest.approx(dg["max_f"], rel=1e-13)
    assert int(dgg["n_unrealizable"][0]) == dg["n_unrealizable"]
    assert int(dgg["n_nonpositive"][0]) == dg["n_nonpositive"]
    assert np.allclose(dgg["dE_matter"], dEm, rtol=1e-10, atol=1e-14 * np.abs(dEm).max())


def test_step_is_deterministic_and_groups_independent(m1):
    w = wl.blobs2d(n=32, G=4, steps=3)
    ctx = m1.Context(m1.Config.from_workload(w))
    a = gpu_run(ctx, w, w.dt, 3)
    b = gpu_run(ctx, w, w.dt, 3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1][0], b[1][0])
    g = 2
    w1 = wl.blobs2d(n=32, G=4, steps=3)
    for nm in ("E", "kappa", "sigma", "B"):
        setattr(w1, nm, np.ascontiguousarray(getattr(w1, nm)[..., g:g + 1]))
    w1.F = [np.ascontiguousarray(f[..., g:g + 1]) for f in w1.F]
    w1.G = 1
    c1 = m1.Context(m1.Config.from_workload(w1))
    o = gpu_run(c1, w1, w1.dt, 3)
    assert np.array_equal(o[0][..., 0], a[0][..., g])


def test_cfl_and_argument_errors(m1):
    w = wl.blobs2d(n=16, G=2, steps=1)
    ctx = m1.Context(m1.Config.from_workload(w))
    assert ctx.max_dt(0.4) == pytest.approx(w.dt, rel=1e-13)
    E = to_dev(w.E, torch.float64)
    F = [to_dev(f, torch.float64) for f in w.F]
    k = to_dev(w.kappa, torch.float64)
    with pytest.raises(m1.FornaxError) as ei:
        ctx.step(E, F, k, k, k, 1.01 * ctx.max_dt(1.0))
    assert ei.value.code == m1.FORNAX_ECFL
    with pytest.raises(m1.FornaxError) as ei:
        ctx.step(E, F, k, k, k, w.dt, out=(E, F))        # aliasing in/out
    assert ei.value.code == m1.FORNAX_EINVAL
    with pytest.raises(TypeError):
        ctx.step(E.float(), F, k, k, k, w.dt)


# ------------------------------------------------------------------------------------------
# full workload sizes: one step, sampled zones against the oracle evaluated zone by zone
# ------------------------------------------------------------------------------------------
def _sampled_step(m1, w, precision, nsample=1500, seed=7):
    p = problem_of(w)
    dt = dt_of(w, p)
    cfg = m1.Config.from_workload(w, precision=precision)
    ctx = m1.Context(cfg)
    say(f"full-size sampled step {w.name} n={w.n} G={w.G} prec={precision}")
    Eg, Fg = gpu_run(ctx, w, dt, 1)
    nz = w.n[0] * w.n[1] * w.n[2]
    rng = np.random.default_rng(seed)
    zones = np.unique(np.concatenate([rng.integers(0, nz, nsample), [0, nz - 1]]))
    Es, Fs, _ = orc.step_zones(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, zones, inflow=w.inflow)
    Eg = Eg.reshape(nz, w.G)[zones]
    Fg = [f.reshape(nz, w.G)[zones] for f in Fg]
    del ctx
    torch.cuda.empty_cache()
    e = rel_l1(Eg, Fg, Es, Fs, w.c)
    say(f"  sampled zones: rel-L1 E {e[0]:.2e} F {e[1]:.2e}; element-wise E {e.pE:.2e} F {e.pF:.2e}")
    check_pointwise(e, precision == m1.FP64, w.name)
    return e


def test_full_size_blobs2d_fp64(m1):
    eE, eF = _sampled_step(m1, wl.blobs2d(), m1.FP64)
    say("blobs2d full", eE, eF)
    assert eE <= TOL_FP64 and eF <= TOL_FP64


def test_full_size_core3d(m1):
    w = wl.core3d()
    eE, eF = _sampled_step(m1, w, m1.FP64)
    assert eE <= TOL_FP64 and eF <= TOL_FP64
    eE, eF = _sampled_step(m1, w, m1.MIXED)
    say("core3d full mixed", eE, eF)
    assert eE <= TOL_MIXED_STEP and eF <= TOL_MIXED_STEP


def test_full_size_sphere(m1):
    w = wl.sphere3d()
    eE, eF = _sampled_step(m1, w, m1.MIXED)
    say("sphere full mixed", eE, eF)
    assert eE <= TOL_MIXED_STEP and eF <= TOL_MIXED_STEP
    eE, eF = _sampled_step(m1, w, m1.FP64)
    assert eE <= TOL_FP64 and eF <= TOL_FP64


@pytest.mark.parametrize("case", ["slab1d", "blobs2d"])
def test_mixed_accuracy_against_the_fp64_closure_threshold(m1, case):
    """MIXED against the FP64 oracle with the closure in double for face states with f >= f*,
    f* in {0.5, 0.9 (the default), infinity (float everywhere)}: the first two meet the run
    bound; the errors are printed for the record."""
    w = wl.slab1d() if case == "slab1d" else wl.blobs2d(n=64, G=16, steps=20)
    p = problem_of(w)
    dt = dt_of(w, p)
    E, F, _ = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, w.steps, inflow=w.inflow)
    errs = {}
    for fstar in (0.5, 0.9, math.inf):
        ctx = m1.Context(m1.Config.from_workload(w, precision=m1.MIXED, f_fp64=fstar))
        Eg, Fg = gpu_run(ctx, w, dt, w.steps)
        errs[fstar] = rel_l1(Eg, Fg, E, F, w.c)
        say(f"mixed {case} {w.steps} steps f*={fstar}: rel-L1 E {errs[fstar][0]:.3e} F {errs[fstar][1]:.3e}")
    for fstar in (0.5, 0.9):
        assert max(errs[fstar]) <= TOL_MIXED_RUN
    assert all(np.isfinite(errs[math.inf]))


@pytest.mark.parametrize("G", [4, 8])
def test_3d_kernel_spherical(m1, G):
    """The whole-zone 3-D kernel on spherical (ln r, theta, phi) grids: inflow at the inner
    radius, polar axes on both theta boundaries (the ghost rows come from the plane shifted by
    n_phi / 2), periodic phi; a grid ragged in every direction (r not a multiple of the 14
    updated columns, theta not of the 12, 8, 7 or 4 updated rows, phi not of the plane count)
    against the oracle element by element, and against the tiled kernel, FP64 and MIXED (4- and
    12-row blocks are built for float only: in FP64 "4,5" and "12,3" run the tiled kernel)."""
    import os
    w = wl.sphere3d(nr=31, nth=17, nph=10, G=G, steps=6)
    rng = np.random.default_rng(G)
    w.E = np.exp(rng.normal(0.0, 0.8, w.E.shape)) * w.B
    p = problem_of(w)
    dt = dt_of(w, p)
    E, F, dg, dEm = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, w.steps, inflow=w.inflow, want_dEm=True)
    for prec, tol in ((m1.FP64, TOL_FP64), (m1.MIXED, TOL_MIXED_RUN)):
        outs = {}
        for c3 in (None, "0", "8,4", "4,5", "12,3"):
            say(f"case spherical 3-D kernel G={G} C3={c3} prec={prec}")
            if c3 is not None:
                os.environ["FORNAX_M1_C3"] = c3
            try:
                ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
            finally:
                os.environ.pop("FORNAX_M1_C3", None)
            Eg, Fg, dgg = gpu_run(ctx, w, dt, w.steps, diag=True)
            e = rel_l1(Eg, Fg, E, F, w.c)
            say(f"  rel-L1 E {e[0]:.2e} F {e[1]:.2e}; element-wise E {e.pE:.2e} F {e.pF:.2e}")
            check_pointwise(e, prec == m1.FP64, f"spherical 3-D kernel {c3}")
            assert e[0] <= tol and e[1] <= tol
            if prec == m1.FP64:
                assert dgg["energy_total"][0] == pytest.approx(dg["energy_total"], rel=1e-12)
                assert int(dgg["n_unrealizable"][0]) == dg["n_unrealizable"]
                assert np.allclose(dgg["dE_matter"], dEm, rtol=1e-10, atol=1e-12 * np.abs(E).max())
            outs[c3] = Eg
        # the default is the 3-D kernel; "0" the tiled kernel
        assert np.array_equal(outs[None], outs["8,4"])
