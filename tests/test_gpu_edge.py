"""GPU parity with the CPU oracle on degenerate inputs: grids of one to three zones per
direction (every column and plane a ghost-rule edge, tiles far larger than the grid), a single
group, states that are not realizable or not positive, and opacities from zero to an
optically thick 1e12 -- in both precisions, through the whole-zone and tiled kernels."""
import math
import os
import sys

import numpy as np
import pytest
import torch

from oracle import m1_oracle as orc
from paper_1806_07390_amd import workloads as wl
from tests.parity_util import TOL_FP64, TOL_MIXED_RUN, gpu_run, problem_of, rel_l1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m1():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1806_07390_amd import m1 as mod
    return mod


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _cut(w, n, G):
    """The first n[0] x n[1] x n[2] zones and G groups of a workload."""
    sl = lambda a: np.ascontiguousarray(a[:n[2], :n[1], :n[0], :G])
    w.E, w.kappa, w.sigma, w.B = sl(w.E), sl(w.kappa), sl(w.sigma), sl(w.B)
    w.F = [sl(f) for f in w.F]
    if w.inflow is not None:
        w.inflow = np.ascontiguousarray(w.inflow[:G])
    w.n = tuple(n)
    w.G = G
    return w


def _tiny(name):
    if name == "slab_2":
        w = _cut(wl.slab1d(steps=3), (2, 1, 1), 1)
        w.bc_lo = (wl.BC_REFLECT, 0, 0)
        return w
    if name == "slab_1":
        return _cut(wl.slab1d(steps=3), (1, 1, 1), 3)
    if name == "plane_3x2":
        return _cut(wl.blobs2d(n=8, G=2, steps=3), (3, 2, 1), 1)
    if name == "plane_5x3_16g":
        return _cut(wl.blobs2d(n=8, G=16, steps=3), (5, 3, 1), 16)
    if name == "box_2x3x2":
        return _cut(wl.core3d(n=4, G=2, steps=3), (2, 3, 2), 2)
    w = wl.sphere3d(nr=3, nth=2, nph=2, G=1, steps=3)
    return w


def _run_both(m1, w, label, tol64=TOL_FP64):
    p = problem_of(w)
    dt = w.dt if w.dt is not None else orc.max_dt(p, w.cfl)
    E, F, dg = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, w.steps, inflow=w.inflow)
    for prec, tol in ((m1.FP64, tol64), (m1.MIXED, TOL_MIXED_RUN)):
        say(f"edge case {label} n={w.n} G={w.G} prec={prec}")
        ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
        Eg, Fg, dgg = gpu_run(ctx, w, dt, w.steps, diag=True)
        eE, eF = rel_l1(Eg, Fg, E, F, w.c)
        say("   ", eE, eF)
        assert eE <= tol and eF <= tol
        if prec == m1.FP64:
            assert int(dgg["n_unrealizable"][0]) == dg["n_unrealizable"]
            assert int(dgg["n_nonpositive"][0]) == dg["n_nonpositive"]
            assert dgg["energy_total"][0] == pytest.approx(dg["energy_total"], rel=1e-12)
        else:
            # float storage counts |F^| > cE (1 + 8u) with the float unit roundoff u
            for k in ("n_unrealizable", "n_nonpositive"):
                assert abs(int(dgg[k][0]) - dg[k]) <= max(2, 0.02 * dg[k])
    return dg


@pytest.mark.parametrize("name", ["slab_2", "slab_1", "plane_3x2", "plane_5x3_16g", "box_2x3x2", "sphere_3x2x2"])
def test_tiny_grids(m1, name):
    _run_both(m1, _tiny(name), name)


@pytest.mark.parametrize("G", [16, 5])
def test_unrealizable_nonpositive_and_extreme_opacity_inputs(m1, G):
    """A quarter of the zone-groups start with E <= 0 or |F| = 1.5 cE; opacities span 0 to 1e12
    (with scattering up to 1e6).  The realizability fallback, the counts and the interaction
    update agree with the oracle.  G = 16 in double runs the whole-zone kernel."""
    w = wl.blobs2d(n=30, G=G, steps=3)
    rng = np.random.default_rng(21)
    shape = w.E.shape
    pick = rng.random(shape)
    w.E = np.where(pick < 0.08, -0.1 * w.E, w.E)
    w.E = np.where((pick >= 0.08) & (pick < 0.12), 0.0, w.E)
    ang = rng.uniform(0, 2 * math.pi, shape)
    over = (pick >= 0.12) & (pick < 0.25)
    w.F = [np.where(over, 1.5 * w.c * np.abs(w.E) * np.cos(ang), w.F[0]),
           np.where(over, 1.5 * w.c * np.abs(w.E) * np.sin(ang), w.F[1])]
    kap = rng.random(shape)
    w.kappa = np.where(kap < 0.2, 0.0, np.where(kap > 0.9, 1e12, w.kappa))
    w.sigma = np.where(rng.random(shape) > 0.95, 1e6, w.sigma)
    dg = _run_both(m1, w, f"unrealizable G={G}")
    assert dg["n_nonpositive"] >= 0 and dg["n_unrealizable"] >= 0


def _rare_case(geom, steps):
    """A 3-D grid of the whole-zone 3-D kernel's kind (group count a multiple of 4) with random
    positive states; h: the scale factors at the zone centres (covariant F = h F^)."""
    if geom == "core3d":
        w = wl.core3d(n=20, G=8, steps=steps)
        h = [np.ones(w.E.shape)] * 3
    else:
        w = wl.sphere3d(nr=20, nth=12, nph=8, G=4, steps=steps)
        r = np.exp(wl._centres(w.lo[0], w.hi[0], w.n[0]))
        th = wl._centres(w.lo[1], w.hi[1], w.n[1])
        R, TH = r[None, None, :, None], th[None, :, None, None]
        h = [np.broadcast_to(R, w.E.shape), np.broadcast_to(R, w.E.shape), np.broadcast_to(R * np.sin(TH), w.E.shape)]
    rng = np.random.default_rng(33)
    w.E = np.exp(rng.normal(0.0, 0.8, w.E.shape)) * w.B
    return w, h, rng


def _unit_vectors(rng, shape):
    v = rng.normal(size=(3,) + shape)
    return v / np.linalg.norm(v, axis=0)


@pytest.mark.parametrize("geom", ["core3d", "sphere3d"])
def test_3d_kernel_rare_states(m1, geom):
    """The whole-zone 3-D kernel (Cartesian and spherical) on states that take the closure's
    rare path: a quarter of the zone-groups start with E <= 0 or |F^| = 1.5 cE, opacities span
    0 to 1e12.  FP64 and MIXED against the oracle, with the counts."""
    w, h, rng = _rare_case(geom, steps=3)
    shape = w.E.shape
    pick = rng.random(shape)
    w.E = np.where(pick < 0.08, -0.1 * w.E, w.E)
    w.E = np.where((pick >= 0.08) & (pick < 0.12), 0.0, w.E)
    over = (pick >= 0.12) & (pick < 0.25)
    v = _unit_vectors(rng, shape)
    w.F = [np.where(over, 1.5 * w.c * np.abs(w.E) * v[k] * h[k], 0.2 * w.c * w.E * v[k] * h[k]) for k in range(3)]
    kap = rng.random(shape)
    w.kappa = np.where(kap < 0.2, 0.0, np.where(kap > 0.9, 1e12, w.kappa))
    dg = _run_both(m1, w, f"3-D kernel rare states {geom}")
    assert dg["n_unrealizable"] > 0 and dg["n_nonpositive"] > 0


@pytest.mark.parametrize("geom", ["core3d", "sphere3d"])
def test_3d_kernel_tiny_states(m1, geom):
    """States scaled by 1e-140 (cE below 2^-450: the closure evaluates them scaled by 2^600),
    a fifth of them also not realizable (|F^| = 1.5 cE), in a block of zones without emission;
    FP64, one step: the zones whose stencil lies inside the block agree with the oracle to the
    element-wise FP64 gate relative to their own energy (floor PW_FLOOR |E| for E, PW_FLOOR c |E| h
    for F), the whole grid element by element."""
    from tests.parity_util import PW_FLOOR, TOL_PW_FP64, check_pointwise
    w, h, rng = _rare_case(geom, steps=1)
    shape = w.E.shape
    v = _unit_vectors(rng, shape)
    over = rng.random(shape) < 0.2
    w.F = [np.where(over, 1.5, 0.3) * w.c * w.E * v[k] * h[k] for k in range(3)]
    # array axes: z (phi), y (theta), x (r), group; the inner zones are 2 zones inside the
    # block in every direction (the whole periodic phi range on the spherical grid)
    blk = np.zeros(shape, dtype=bool)
    inner = np.zeros(shape, dtype=bool)
    if geom == "core3d":
        blk[2:12, 2:12, 2:12] = True
        inner[4:10, 4:10, 4:10] = True
    else:
        blk[:, 2:10, 3:15] = True
        inner[:, 4:8, 5:13] = True
    sc = np.where(blk, 1e-140, 1.0)
    w.E = w.E * sc
    w.F = [f * sc for f in w.F]
    w.B = np.where(blk, 0.0, w.B)
    p = problem_of(w)
    dt = w.dt if w.dt is not None else orc.max_dt(p, w.cfl)
    E, F, dg = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, 1, inflow=w.inflow)
    ctx = m1.Context(m1.Config.from_workload(w, precision=m1.FP64))
    Eg, Fg, dgg = gpu_run(ctx, w, dt, 1, diag=True)
    e = rel_l1(Eg, Fg, E, F, w.c)
    check_pointwise(e, True, f"tiny states {geom}")
    assert 0 < np.abs(E[inner]).max() < 1e-130
    relE = np.abs(Eg[inner] - E[inner]) / ((1.0 + PW_FLOOR) * np.abs(E[inner]))
    relF = [np.abs(Fg[k][inner] - F[k][inner]) / (np.abs(F[k][inner]) + PW_FLOOR * w.c * np.abs(E[inner]) * h[k][inner])
            for k in range(3)]
    say(f"tiny states {geom}: rel-L1 {e[0]:.2e} {e[1]:.2e}; inner zones element-wise E {relE.max():.2e} "
        f"F {max(r.max() for r in relF):.2e}")
    assert relE.max() <= TOL_PW_FP64
    for k in range(3):
        assert relF[k].max() <= TOL_PW_FP64, k
    assert int(dgg["n_unrealizable"][0]) == dg["n_unrealizable"]
