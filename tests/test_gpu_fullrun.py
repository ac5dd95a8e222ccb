"""GPU parity over whole runs: the workloads' full step counts against the CPU oracle, compared
in rel-L1 and element by element.

* 2-D 512^2 x 16 periodic blobs, 100 steps: the full size, FP64 on the default kernel (the
  whole-zone kernel) and MIXED;
* 3-D core workload, 50 steps, at 96^3 x 12 (the largest grid whose oracle run takes about
  half a minute on the test host's cores; the full 192^3 x 12 needs 8x that) in FP64 and
  MIXED, and its geometry for 100 steps at 64^3 x 12 in MIXED (the after-100-steps gate);
* spherical inflow workload, 100 steps, at 128 x 32 x 64 x 20 (the full 256 x 64 x 128 x 20
  needs 16x the oracle time), FP64 and MIXED.
The full-size 3-D and spherical grids are checked on sampled zones of one step elsewhere."""
import sys

import numpy as np
import pytest
import torch

from oracle import m1_oracle as orc
from paper_1806_07390_amd import workloads as wl
from tests.parity_util import TOL_FP64, TOL_MIXED_RUN, gpu_run, problem_of, rel_l1

pytestmark = pytest.mark.gpu

# element-wise bounds (|x - x_ref| <= tol (|x_ref| + 1e-3 max |E_ref|)), on top of the rel-L1
# gates: FP64 the same 1e-12; MIXED a factor 10 above its rel-L1 gate (float storage rounds
# every zone by 6e-8 each step; the element-wise error is the L1 error's worst zone)
TOL_PW_FP64 = 1e-12
TOL_PW_MIXED_RUN = 1e-3


@pytest.fixture(scope="module")
def m1():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1806_07390_amd import m1 as mod
    return mod


def say(*a):
    print(*a, file=sys.stderr, flush=True)


_oracle_cache = {}


def oracle_run(w, nsteps, key):
    if key not in _oracle_cache:
        p = problem_of(w, nthreads=0)
        dt = w.dt if w.dt is not None else orc.max_dt(p, w.cfl)
        say(f"oracle {key}: {w.n} x {w.G}, {nsteps} steps")
        E, F, dg = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, nsteps, inflow=w.inflow)
        _oracle_cache[key] = (dt, E, F, dg)
    return _oracle_cache[key]


def compare(m1, w, precision, nsteps, key):
    dt, E, F, dg = oracle_run(w, nsteps, key)
    name = "fp64" if precision == m1.FP64 else "mixed"
    say(f"case full run {key} {name}")
    ctx = m1.Context(m1.Config.from_workload(w, precision=precision))
    Eg, Fg, dgg = gpu_run(ctx, w, dt, nsteps, diag=True)
    e = rel_l1(Eg, Fg, E, F, w.c)
    say(f"  {key} {name}: rel-L1 E {e[0]:.3e} F {e[1]:.3e}; element-wise E {e.pE:.3e} F {e.pF:.3e}")
    return e, dg, dgg


def check_fp64(e, dg, dgg):
    assert e[0] <= TOL_FP64 and e[1] <= TOL_FP64
    assert e.pE <= TOL_PW_FP64 and e.pF <= TOL_PW_FP64
    assert float(dgg["energy_total"][0]) == pytest.approx(dg["energy_total"], rel=1e-12)
    assert int(dgg["n_unrealizable"][0]) == dg["n_unrealizable"]
    assert int(dgg["n_nonpositive"][0]) == dg["n_nonpositive"]


def check_mixed(e):
    assert e[0] <= TOL_MIXED_RUN and e[1] <= TOL_MIXED_RUN
    assert e.pE <= TOL_PW_MIXED_RUN and e.pF <= TOL_PW_MIXED_RUN


def test_blobs2d_full_size_100_steps(m1):
    w = wl.blobs2d()
    e, dg, dgg = compare(m1, w, m1.FP64, w.steps, "blobs2d512")
    check_fp64(e, dg, dgg)
    e, _, _ = compare(m1, w, m1.MIXED, w.steps, "blobs2d512")
    check_mixed(e)


def test_core3d_50_steps(m1):
    w = wl.core3d(n=96)
    e, dg, dgg = compare(m1, w, m1.FP64, w.steps, "core3d96")
    check_fp64(e, dg, dgg)
    e, _, _ = compare(m1, w, m1.MIXED, w.steps, "core3d96")
    check_mixed(e)


def test_core3d_geometry_100_steps_mixed(m1):
    w = wl.core3d(n=64, steps=100)
    e, _, _ = compare(m1, w, m1.MIXED, 100, "core3d64x100")
    check_mixed(e)


def test_sphere_100_steps(m1):
    w = wl.sphere3d(nr=128, nth=32, nph=64)
    e, dg, dgg = compare(m1, w, m1.FP64, w.steps, "sphere128")
    check_fp64(e, dg, dgg)
    e, _, _ = compare(m1, w, m1.MIXED, w.steps, "sphere128")
    check_mixed(e)
