"""GPU parity of the step with a prescribed velocity (fornax_m1_step_velocity: advective fluxes,
velocity gradient terms, frequency advection, then the interaction update) and of the lab-frame
moments (fornax_m1_lab_frame), through the C interface, against the CPU oracle on the same
seeded inputs: Cartesian 1-D, 2-D and 3-D grids (ragged, every boundary kind but the axis),
spherical 2-D with inflow and polar axes, spherical 3-D; FP64 element by element within
2e-12 and in rel-L1 within 1e-12, MIXED within its run gates."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import m1_oracle as orc
from paper_1806_07390_amd import workloads as wl
from tests.parity_util import TOL_FP64, TOL_MIXED_RUN, check_pointwise, problem_of, rel_l1, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m1():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1806_07390_amd import m1 as mod
    return mod


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _random_radiation(w, seed, fmax=0.8):
    """Lognormal E; Cartesian grids also get F up to fmax c E in random directions (spherical
    ones start from F = 0, whose covariant components need no scale factors)."""
    rng = np.random.default_rng(seed)
    s = (w.n[2], w.n[1], w.n[0], w.G)
    w.E = np.exp(rng.normal(0.0, 0.8, s))
    if w.coord == wl.CARTESIAN:
        d = rng.normal(size=(w.ndim,) + s)
        d /= np.linalg.norm(d, axis=0)
        f = fmax * rng.random(s)
        w.F = [np.ascontiguousarray(f * w.c * w.E * d[k]) for k in range(w.ndim)]
    else:
        w.F = [np.zeros(s) for _ in range(w.ndim)]
    return w


def case(name):
    if name == "cart1d":
        w = wl.slab1d(n=45, G=6)
        w.bc_lo = (wl.BC_REFLECT, 0, 0)
    elif name == "cart2d":
        w = wl.blobs2d(n=26, G=6)
    elif name == "cart3d":
        from tests.test_gpu_parity import _c3_case
        w = _c3_case(n=(17, 13, 10), G=5, steps=3, seed=4, bcs="mixed")
    elif name == "cart3d_k":
        # a group count of the whole-zone 3-D kernel: Step 1 runs on it, the flux rows' velocity
        # terms in the frequency step
        from tests.test_gpu_parity import _c3_case
        w = _c3_case(n=(17, 13, 10), G=8, steps=3, seed=4, bcs="mixed")
    elif name == "sph2d":
        w = wl.sphere3d(nr=18, nth=10, nph=1, G=4, ndim=2)
    else:
        w = wl.sphere3d(nr=12, nth=8, nph=8, G=3)
    w = _random_radiation(w, seed=len(name))
    w.steps = 3
    return w


def oracle_v(w, vf, nu, dt, nsteps):
    p = problem_of(w)
    return orc.run_v(p, w.E, w.F, w.kappa, w.sigma, w.B, vf, nu, dt, nsteps, inflow=w.inflow, want_dEm=True)


def gpu_v(m1, ctx, w, vf, nu, dt, nsteps):
    dtp = ctx.dtype
    E = to_dev(w.E, dtp)
    F = [to_dev(f, dtp) for f in w.F]
    k, s, B = (to_dev(x, dtp) for x in (w.kappa, w.sigma, w.B))
    inflow = None if w.inflow is None else to_dev(w.inflow, torch.float64)
    V = [to_dev(v, dtp) for v in vf]
    ctx.set_group_edges(nu)
    dg = ctx.new_diag()
    A = (E, F)
    Bst = ctx.empty_state()
    for _ in range(nsteps):
        ctx.step_velocity(A[0], A[1], k, s, B, V, dt, out=Bst, inflow=inflow, diag=dg)
        A, Bst = Bst, A
    torch.cuda.synchronize()
    return to_host(A[0]), [to_host(f) for f in A[1]], {kk: v.cpu().numpy() for kk, v in dg.items()}


@pytest.mark.parametrize("name", ["cart1d", "cart2d", "cart3d", "cart3d_k", "sph2d", "sph3d"])
def test_velocity_step_matches_oracle(m1, name):
    w = case(name)
    vf = wl.face_velocity(w, amp=0.15, seed=3)
    nu = wl.velocity_edges(w.G)
    p = problem_of(w)
    dt = w.dt if w.dt is not None else orc.max_dt(p, 0.4)
    E, F, dg, dEm = oracle_v(w, vf, nu, dt, w.steps)
    # the velocity terms change the result: compare with the static step
    E0, _, _ = orc.run(p, w.E, w.F, w.kappa, w.sigma, w.B, dt, w.steps, inflow=w.inflow)
    assert np.abs(E - E0).max() > 1e-6 * np.abs(E).max()
    for prec in (m1.FP64, m1.MIXED):
        say(f"case velocity {name} n={w.n} G={w.G} prec={prec}")
        ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
        Eg, Fg, dgg = gpu_v(m1, ctx, w, vf, nu, dt, w.steps)
        e = rel_l1(Eg, Fg, E, F, w.c)
        say(f"  rel-L1 E {e[0]:.2e} F {e[1]:.2e}; element-wise E {e.pE:.2e} F {e.pF:.2e}")
        if prec == m1.FP64:
            check_pointwise(e, True, name)
            assert e[0] <= TOL_FP64 and e[1] <= TOL_FP64
            assert float(dgg["energy_total"][0]) == pytest.approx(dg["energy_total"], rel=1e-12)
            assert int(dgg["n_unrealizable"][0]) == dg["n_unrealizable"]
            assert int(dgg["n_nonpositive"][0]) == dg["n_nonpositive"]
            assert float(dgg["max_f"][0]) == pytest.approx(dg["max_f"], rel=1e-10)
            assert np.allclose(dgg["dE_matter"], dEm.ravel(), rtol=1e-10, atol=1e-12 * np.abs(E).max())
        else:
            assert e[0] <= TOL_MIXED_RUN and e[1] <= TOL_MIXED_RUN
            assert e.pE <= 1e-3 and e.pF <= 1e-3
            assert float(dgg["energy_total"][0]) == pytest.approx(dg["energy_total"], rel=1e-5)


def test_velocity_step_48cube_12_groups(m1):
    """A 48^3 x 12 grid (several thousand blocks of each kernel) in FP64 and MIXED."""
    w = _random_radiation(wl.core3d(n=48, G=12), seed=9)
    vf = wl.face_velocity(w, amp=0.1, seed=5)
    nu = wl.velocity_edges(w.G)
    E, F, dg, dEm = oracle_v(w, vf, nu, w.dt, 2)
    for prec in (m1.FP64, m1.MIXED):
        say(f"case velocity core3d48 prec={prec}")
        ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
        Eg, Fg, dgg = gpu_v(m1, ctx, w, vf, nu, w.dt, 2)
        e = rel_l1(Eg, Fg, E, F, w.c)
        say(f"  rel-L1 E {e[0]:.2e} F {e[1]:.2e}; element-wise E {e.pE:.2e} F {e.pF:.2e}")
        if prec == m1.FP64:
            check_pointwise(e, True, "core3d48")
            assert e[0] <= TOL_FP64 and e[1] <= TOL_FP64
            assert float(dgg["energy_total"][0]) == pytest.approx(dg["energy_total"], rel=1e-12)
        else:
            assert e[0] <= TOL_MIXED_RUN and e[1] <= TOL_MIXED_RUN


@pytest.mark.parametrize("name", ["cart3d", "cart3d_k"])
def test_zero_velocity_is_the_static_step(m1, name):
    w = case(name)
    vf = [np.zeros_like(v) for v in wl.face_velocity(w)]
    nu = wl.velocity_edges(w.G)
    ctx = m1.Context(m1.Config.from_workload(w, precision=m1.FP64))
    Eg, Fg, _ = gpu_v(m1, ctx, w, vf, nu, w.dt, 2)
    dtp = ctx.dtype
    E0 = to_dev(w.E, dtp)
    F0 = [to_dev(f, dtp) for f in w.F]
    k, s, B = (to_dev(x, dtp) for x in (w.kappa, w.sigma, w.B))
    Es, Fs = ctx.run(E0, F0, k, s, B, w.dt, 2)
    e = rel_l1(Eg, Fg, to_host(Es), [to_host(f) for f in Fs], w.c)
    assert e.pE <= 1e-13 and e.pF <= 1e-13


@pytest.mark.parametrize("name", ["cart3d", "sph2d", "sph3d"])
def test_lab_frame_matches_oracle(m1, name):
    w = case(name)
    vf = wl.face_velocity(w, amp=0.2, seed=1)
    p = problem_of(w)
    El, Fl = orc.lab_frame(p, w.E, w.F, vf)
    for prec, tol in ((m1.FP64, 1e-13), (m1.MIXED, 2e-6)):
        ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
        E = to_dev(w.E, ctx.dtype)
        F = [to_dev(f, ctx.dtype) for f in w.F]
        Elg, Flg = ctx.lab_frame(E, F, [to_dev(v, ctx.dtype) for v in vf])
        scale = np.abs(El).max()
        assert np.abs(to_host(Elg) - El).max() <= tol * scale
        for k in range(w.ndim):
            assert np.abs(to_host(Flg[k]) - Fl[k]).max() <= tol * w.c * scale


def test_velocity_argument_errors(m1):
    w = case("cart2d")
    vf = wl.face_velocity(w)
    ctx = m1.Context(m1.Config.from_workload(w, precision=m1.FP64))
    dtp = ctx.dtype
    E = to_dev(w.E, dtp)
    F = [to_dev(f, dtp) for f in w.F]
    k, s, B = (to_dev(x, dtp) for x in (w.kappa, w.sigma, w.B))
    V = [to_dev(v, dtp) for v in vf]
    with pytest.raises(m1.FornaxError) as ei:       # no group edges yet
        ctx.step_velocity(E, F, k, s, B, V, w.dt)
    assert ei.value.code == m1.FORNAX_EINVAL
    with pytest.raises(m1.FornaxError):
        ctx.set_group_edges([0.0, 1.0, 1.0, 2.0, 3.0, 4.0, 5.0])
    with pytest.raises(m1.FornaxError):
        ctx.set_group_edges([0.0, 1.0, 2.0, 3.0, 4.0, 5.0, math.inf])
    ctx.set_group_edges(wl.velocity_edges(w.G))
    ctx.step_velocity(E, F, k, s, B, V, w.dt)
    with pytest.raises(m1.FornaxError) as ei:
        ctx.step_velocity(E, F, k, s, B, V, 10.0)     # above the CFL limit
    assert ei.value.code == m1.FORNAX_ECFL
    for kw in (dict(integrator=m1.SSPRK2), dict(limiter=m1.LIMITER_PPM), dict(wavespeed=m1.WAVESPEED_M1)):
        c2 = m1.Context(m1.Config.from_workload(w, precision=m1.FP64, **kw))
        c2.set_group_edges(wl.velocity_edges(w.G))
        with pytest.raises(m1.FornaxError) as ei:
            c2.step_velocity(E, F, k, s, B, V, w.dt)
        assert ei.value.code == m1.FORNAX_EUNSUPPORTED
    torch.cuda.synchronize()


def test_transparent_shock_long_run(m1):
    """The transparent standing shock (spherical 1-D, 120 zones, a beam from the inner boundary,
    no matter, the paper's velocity profile with a shock at r = 100): 2.2 light-crossing times
    (13911 steps) on the GPU in FP64 against the oracle within 1e-10 of the largest E and F,
    with the lab-frame moments from the GPU state; MIXED against the oracle after 200 steps
    within its run gate, and at steady state the comoving jump (> 15 %) and the lab-frame
    continuity (< 3 %) across the shock."""
    n, G = 120, 4
    rin, rmax, rsh, vsh = 10.0, 1000.0, 100.0, 0.1
    w = wl.Workload("shock1d", 1, (n, 1, 1), G, wl.SPHERICAL_LOGR, (math.log(rin), 0.0, 0.0),
                    (math.log(rmax), math.pi, 2 * math.pi), (wl.BC_INFLOW, wl.BC_AXIS, wl.BC_PERIODIC),
                    (wl.BC_OUTFLOW, wl.BC_AXIS, wl.BC_PERIODIC), 1.0, 0, np.full((1, 1, n, G), 1e-8),
                    [np.zeros((1, 1, n, G))], np.zeros((1, 1, n, G)), np.zeros((1, 1, n, G)),
                    np.zeros((1, 1, n, G)))
    Eg = np.array([0.2, 0.4, 0.3, 0.1])
    w.inflow = np.stack([Eg, Eg], axis=1)
    rf = np.exp(np.linspace(math.log(rin), math.log(rmax), n + 1))
    v = np.where(rf < rsh, -0.1 * vsh * rf / rsh, -vsh * (np.sqrt(rmax / rf) - 1) / (math.sqrt(rmax / rsh) - 1))
    vf = [(v / rf).reshape(1, 1, 1, n + 1)]
    nu = np.array([0.0, 1.0, 2.0, 4.0, 8.0])
    p = problem_of(w)
    p.nthreads = 1
    dt = orc.max_dt(p, 0.4)
    nsteps = int(2.2 * (rmax - rin) / dt)
    E, F, dg, _ = oracle_v(w, vf, nu, dt, nsteps)
    say(f"case transparent shock FP64 steps={nsteps}")
    ctx = m1.Context(m1.Config.from_workload(w, precision=m1.FP64))
    Eg_, Fg_, _ = gpu_v(m1, ctx, w, vf, nu, dt, nsteps)
    eE = np.abs(Eg_ - E).max() / np.abs(E).max()
    eF = np.abs(Fg_[0] - F[0]).max() / np.abs(F[0]).max()
    say(f"  max |dE| / max E {eE:.2e}, max |dF| / max F {eF:.2e}")
    assert eE <= 1e-10 and eF <= 1e-10
    El, Fl = orc.lab_frame(p, E, F, vf)
    Elg, Flg = ctx.lab_frame(to_dev(Eg_, torch.float64), [to_dev(Fg_[0], torch.float64)],
                             [to_dev(vf[0], torch.float64)])
    assert np.abs(to_host(Elg) - El).max() <= 1e-9 * np.abs(El).max()
    assert np.abs(to_host(Flg[0]) - Fl[0]).max() <= 1e-9 * np.abs(Fl[0]).max()
    # MIXED: parity over the first 200 steps, the physics at steady state
    E2, F2, _, _ = oracle_v(w, vf, nu, dt, 200)
    ctx = m1.Context(m1.Config.from_workload(w, precision=m1.MIXED))
    Em, Fm, _ = gpu_v(m1, ctx, w, vf, nu, dt, 200)
    e = rel_l1(Em, Fm, E2, F2, w.c)
    say(f"  MIXED 200 steps: rel-L1 E {e[0]:.2e} F {e[1]:.2e}; element-wise E {e.pE:.2e} F {e.pF:.2e}")
    assert e[0] <= TOL_MIXED_RUN and e[1] <= TOL_MIXED_RUN
    Em, Fm, _ = gpu_v(m1, ctx, w, vf, nu, dt, nsteps)
    eE = np.abs(Em - E).max() / np.abs(E).max()
    at = int(np.unravel_index(np.argmax(np.abs(Em - E)), E.shape)[2])
    say(f"  MIXED {nsteps} steps: max |dE| / max E {eE:.2e} at zone {at}")
    h = np.sqrt(np.exp(2 * np.log(rf[:-1] * rf[1:]) / 2))          # geometric-mean radius
    Elm, Flm = ctx.lab_frame(to_dev(Em, torch.float32), [to_dev(Fm[0], torch.float32)],
                             [to_dev(vf[0], torch.float32)])
    s = int(np.searchsorted(rf, rsh)) - 1
    com = Em.sum(-1)[0, 0] * h ** 2
    lab = to_host(Elm)[0, 0] * h ** 2
    assert com[s + 1] / com[s - 1] > 1.15
    assert abs(lab[s + 1] / lab[s - 1] - 1.0) < 0.03


def test_velocity_step_mc_limiter_on_the_3d_kernel(m1):
    """The MC limiter (the 3-D kernel's instantiation that reads the limiter at run time) in the
    velocity step on a grid of the 3-D kernel's kind, FP64 and MIXED, against the oracle."""
    w = case("cart3d_k")
    vf = wl.face_velocity(w, amp=0.15, seed=3)
    nu = wl.velocity_edges(w.G)
    p = problem_of(w, limiter=orc.MC)
    dt = w.dt if w.dt is not None else orc.max_dt(p, 0.4)
    E, F, dg, dEm = orc.run_v(p, w.E, w.F, w.kappa, w.sigma, w.B, vf, nu, dt, w.steps, inflow=w.inflow,
                              want_dEm=True)
    E0, _, _, _ = oracle_v(w, vf, nu, dt, w.steps)
    assert np.abs(E - E0).max() > 1e-8 * np.abs(E).max()     # the limiter changes the result
    for prec in (m1.FP64, m1.MIXED):
        say(f"case velocity cart3d_k MC prec={prec}")
        ctx = m1.Context(m1.Config.from_workload(w, precision=prec, limiter=m1.LIMITER_MC))
        Eg, Fg, dgg = gpu_v(m1, ctx, w, vf, nu, dt, w.steps)
        e = rel_l1(Eg, Fg, E, F, w.c)
        say(f"  rel-L1 E {e[0]:.2e} F {e[1]:.2e}; element-wise E {e.pE:.2e} F {e.pF:.2e}")
        if prec == m1.FP64:
            check_pointwise(e, True, "cart3d_k MC")
            assert e[0] <= TOL_FP64 and e[1] <= TOL_FP64
            assert np.allclose(dgg["dE_matter"], dEm.ravel(), rtol=1e-10, atol=1e-12 * np.abs(E).max())
        else:
            assert e[0] <= TOL_MIXED_RUN and e[1] <= TOL_MIXED_RUN
