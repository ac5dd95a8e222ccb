"""GPU parity of the parabolic reconstruction option (FORNAX_LIMITER_PPM) against the CPU
oracle on the same seeded inputs: the step in 1-D, 2-D (the whole-zone kernel in double, the
tiled kernel in float and for other group counts), 3-D and the spherical grid (volume-coordinate
weights), both precisions; the face-flux entry point; and the adjoint, which refuses the
option."""
import sys

import numpy as np
import pytest
import torch

from oracle import m1_oracle as orc
from paper_1806_07390_amd import workloads as wl
from tests.parity_util import TOL_FP64, TOL_MIXED_RUN, gpu_run, problem_of, rel_l1, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m1():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1806_07390_amd import m1 as mod
    return mod


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _case(name):
    if name == "slab1d":
        return wl.slab1d(steps=40)
    if name == "blobs2d":
        return wl.blobs2d(n=40, G=16, steps=6)
    if name == "reflect2d":
        w = wl.blobs2d(n=36, G=5, steps=6)
        w.bc_lo = (wl.BC_REFLECT, wl.BC_OUTFLOW, 0)
        w.bc_hi = (wl.BC_OUTFLOW, wl.BC_REFLECT, 0)
        return w
    if name == "core3d":
        return wl.core3d(n=14, G=6, steps=5)
    return wl.sphere3d(nr=14, nth=10, nph=8, G=4, steps=5)


# The slab's steep pulse makes the parabolic limiter's branch decisions sensitive to rounding:
# perturbing its inputs by 1e-15 (relative, random) changes the oracle's own 40-step result by
# 1.1e-11 rel-L1 (with minmod: 1.5e-15), so an implementation that rounds differently may take
# another branch in a few zone-groups.  Its FP64 bound is 1e-10 instead of 1e-12.
TOL_FP64_PPM_SLAB = 1e-10


@pytest.mark.parametrize("name", ["slab1d", "blobs2d", "reflect2d", "core3d", "sphere3d"])
def test_parabolic_reconstruction_matches_oracle(m1, name):
    w = _case(name)
    p = problem_of(w, limiter=orc.PPM)
    dt = w.dt if w.dt is not None else orc.max_dt(p, w.cfl)
    E, F, dg = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, w.steps, inflow=w.inflow)
    E0, F0, _ = orc.run(problem_of(w), w.E, w.F, w.kappa, w.sigma, w.B, dt, w.steps, inflow=w.inflow)
    assert rel_l1(E0, F0, E, F, w.c)[0] > 1e-10      # the option changes the result
    tol64 = TOL_FP64_PPM_SLAB if name == "slab1d" else TOL_FP64
    for prec, tol in ((m1.FP64, tol64), (m1.MIXED, TOL_MIXED_RUN)):
        ctx = m1.Context(m1.Config.from_workload(w, precision=prec, limiter=m1.LIMITER_PPM))
        Eg, Fg, dgg = gpu_run(ctx, w, dt, w.steps, diag=True)
        eE, eF = rel_l1(Eg, Fg, E, F, w.c)
        say(f"PPM {name} prec={prec}", eE, eF)
        assert eE <= tol and eF <= tol
        assert int(dgg["n_unrealizable"][0]) == dg["n_unrealizable"]
        if prec == m1.FP64:
            assert dgg["energy_total"][0] == pytest.approx(dg["energy_total"], rel=1e-12)


@pytest.mark.parametrize("grid", ["core3d", "sphere3d"])
def test_flux_entry_point_with_parabolic_reconstruction(m1, grid):
    w = wl.core3d(n=12, G=3, steps=1) if grid == "core3d" else wl.sphere3d(nr=12, nth=8, nph=8, G=3, steps=1)
    rng = np.random.default_rng(6)
    w.E = (w.E if grid == "core3d" else w.B) * (1 + rng.random(w.E.shape))
    w.F = [0.3 * w.E * rng.uniform(-1, 1, w.E.shape) for _ in range(3)]
    p = problem_of(w, limiter=orc.PPM)
    ctx = m1.Context(m1.Config.from_workload(w, limiter=m1.LIMITER_PPM))
    E = to_dev(w.E, torch.float64)
    F = [to_dev(f, torch.float64) for f in w.F]
    k, s, B = (to_dev(x, torch.float64) for x in (w.kappa, w.sigma, w.B))
    inflow = None if w.inflow is None else to_dev(w.inflow, torch.float64)
    fl = ctx.flux(E, F, k, s, B, inflow=inflow)
    for d in range(3):
        ref = orc.flux(p, w.E, w.F, w.kappa, w.sigma, w.B, d, inflow=w.inflow)
        ref0 = orc.flux(problem_of(w), w.E, w.F, w.kappa, w.sigma, w.B, d, inflow=w.inflow)
        scale = np.abs(ref).max()
        assert np.max(np.abs(ref - ref0)) > 1e-6 * scale
        assert np.max(np.abs(to_host(fl[d]) - ref)) <= 1e-13 * scale, d


def test_adjoint_refuses_parabolic_reconstruction(m1):
    w = wl.adjoint2d(n=16, G=2, steps=1)
    ctx = m1.Context(m1.Config.from_workload(w, precision=m1.FP64, limiter=m1.LIMITER_PPM))
    t = lambda a: to_dev(a, torch.float64)
    z = [torch.zeros_like(t(w.E)) for _ in w.F]
    with pytest.raises(m1.FornaxError) as ei:
        ctx.adjoint(t(w.E), [t(f) for f in w.F], t(w.kappa), t(w.sigma), t(w.B), w.dt, t(w.E), z)
    assert ei.value.code == m1.FORNAX_EUNSUPPORTED
