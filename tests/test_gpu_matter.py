"""GPU parity of the radiation-matter energy exchange (the outer solve for the matter
temperature with every group's inner backward-Euler update) and of the explicit-only transport,
through the C interface, against the CPU FP64 oracle on the same seeded inputs.

Bounds: the solve stops when Newton's relative step is at most tol = 1e-6, and Newton's
quadratic convergence leaves an error of order that step squared; both sides evaluate the
residual in double with differently rounded series and exponentials (about 1e-15 relative), so
the temperatures agree to about 1e-12 whichever side takes one more iteration.  The tests
bound T, E, F and dE_matter at 1e-9 relative (FP64 states).  MIXED contexts hold float states
and solve in double: compared with the oracle run on the float-rounded inputs, at float
rounding (2e-6)."""
import sys

import numpy as np
import pytest
import torch

from oracle import m1_oracle as orc
from paper_1806_07390_amd import workloads as wl
from tests.parity_util import TOL_FP64, TOL_MIXED_STEP, problem_of, rel_l1, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_MATTER = 1e-9
TOL_MATTER_MIXED = 2e-6


@pytest.fixture(scope="module")
def m1():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1806_07390_amd import m1 as mod
    return mod


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _ctx(m1, w, precision=0, max_newton=30, integrator=0):
    ctx = m1.Context(m1.Config.from_workload(w, precision=precision, integrator=integrator))
    g = w.groups
    ctx.set_matter_model(g.nu_edge, g.nu_c, g.kg, a_rad=g.a_rad, tol=1e-6, max_newton=max_newton)
    return ctx


def _model(w, max_newton=30):
    g = w.groups
    return orc.MatterModel(g.nu_edge, g.nu_c, g.kg, a_rad=g.a_rad, c=w.c, tol=1e-6, max_newton=max_newton)


def _zone_case(nx=24, ny=10, G=16, seed=0, E_scale=1.0, kappa_scale=1.0):
    """A 2-D grid whose zones hold independent random matter and radiation (the interaction
    update is zone-local): temperatures, heat capacities and opacity scales over a few decades,
    radiation out of equilibrium with the matter."""
    w = wl.matter2d(n=nx, G=G, seed=seed, kappa_scale=kappa_scale)
    rng = np.random.default_rng(seed + 7)
    sh = (1, ny, nx)
    w.E = np.ascontiguousarray(E_scale * rng.uniform(0.0, 0.5, sh + (G,)))
    w.F = [np.ascontiguousarray(0.4 * w.E * rng.uniform(-1, 1, sh + (G,))) for _ in range(2)]
    w.sigma = np.ascontiguousarray(rng.uniform(0.0, 3.0, sh + (G,)))
    w.kappa = np.ones(sh + (G,))
    w.B = np.zeros(sh + (G,))
    w.T = np.exp(0.5 * rng.standard_normal(sh))
    w.cv = np.exp(0.7 * rng.standard_normal(sh))
    w.kappa0 = kappa_scale * np.exp(1.5 * rng.standard_normal(sh))
    w.n = (nx, ny, 1)
    return w


def _gpu_source(m1, w, dt, precision=0, max_newton=30):
    ctx = _ctx(m1, w, precision, max_newton)
    dtp = ctx.dtype
    E = to_dev(w.E, dtp)
    F = [to_dev(f, dtp) for f in w.F]
    sig = to_dev(w.sigma, dtp)
    cv, k0, T = (to_dev(x, torch.float64) for x in (w.cv, w.kappa0, w.T))
    dEm = torch.zeros(ctx.nzones, dtype=torch.float64, device="cuda")
    it = torch.zeros(ctx.nzones, dtype=torch.int32, device="cuda")
    ctx.matter_source(E, F, sig, cv, k0, T, dt, dE_matter=dEm, iters=it)
    torch.cuda.synchronize()
    return to_host(E), [to_host(f) for f in F], to_host(T), to_host(dEm), it.cpu().numpy()


def _close(a, b, rel):
    scale = np.abs(b).max()
    return np.abs(a - b).max() <= rel * scale and np.all(np.abs(a - b) <= rel * np.abs(b) + 1e-14 * scale)


@pytest.mark.parametrize("seed,dt,E_scale,kappa_scale", [(1, 0.01, 1.0, 1.0), (2, 0.3, 3.0, 10.0),
                                                          (3, 1e-4, 0.2, 0.01), (4, 5.0, 1.0, 1e4)])
def test_matter_source_matches_oracle_fp64(m1, seed, dt, E_scale, kappa_scale):
    w = _zone_case(seed=seed, E_scale=E_scale, kappa_scale=kappa_scale)
    say(f"matter source fp64 seed={seed} dt={dt}")
    E, F, T, dEm, it = orc.matter_source(_model(w), w.E, w.F, w.sigma, w.cv, w.kappa0, w.T, dt)
    Eg, Fg, Tg, dEg, itg = _gpu_source(m1, w, dt)
    assert np.allclose(Tg.ravel(), T.ravel(), rtol=TOL_MATTER, atol=0)
    assert _close(Eg, E, TOL_MATTER)
    for a, b in zip(Fg, F):
        assert _close(a, b, TOL_MATTER)
    assert np.allclose(dEg, dEm.ravel(), rtol=TOL_MATTER, atol=TOL_MATTER * np.abs(w.cv * w.T).max())
    # the same path (Newton or bisection) in every zone, the same iteration count in nearly all
    assert np.array_equal(np.sign(itg), np.sign(it.ravel()))
    assert np.mean(itg == it.ravel()) >= 0.99
    say("   T", np.abs(Tg.ravel() / T.ravel() - 1).max(), "iters", np.bincount(np.abs(itg)))


def test_matter_source_bisection_matches_oracle(m1):
    w = _zone_case(seed=9, E_scale=2.0)
    E, F, T, dEm, it = orc.matter_source(_model(w, max_newton=0), w.E, w.F, w.sigma, w.cv, w.kappa0, w.T, 0.2)
    Eg, Fg, Tg, dEg, itg = _gpu_source(m1, w, 0.2, max_newton=0)
    assert np.all(itg < 0) and np.all(it < 0)
    assert np.allclose(Tg.ravel(), T.ravel(), rtol=1e-12, atol=0)
    assert _close(Eg, E, TOL_MATTER)


def test_matter_source_mixed(m1):
    w = _zone_case(seed=5, E_scale=1.5)
    dt = 0.05
    # the oracle on the float-rounded states and scattering (the MIXED context's inputs)
    rf = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    E, F, T, dEm, it = orc.matter_source(_model(w), rf(w.E), [rf(f) for f in w.F], rf(w.sigma), w.cv, w.kappa0,
                                         w.T, dt)
    Eg, Fg, Tg, dEg, itg = _gpu_source(m1, w, dt, precision=1)
    assert np.allclose(Tg.ravel(), T.ravel(), rtol=1e-9, atol=0)
    assert _close(Eg, E, TOL_MATTER_MIXED)
    for a, b in zip(Fg, F):
        assert _close(a, b, TOL_MATTER_MIXED)


def test_matter_equilibrium_is_kept(m1):
    """E = B_g(T) from the GPU's own matter coefficients: the solve leaves T and E in place."""
    w = _zone_case(seed=6)
    ctx = _ctx(m1, w)
    cv, k0, T = (to_dev(x, torch.float64) for x in (w.cv, w.kappa0, w.T))
    kap, B = ctx.matter_coeffs(cv, k0, T)
    E = B.clone()
    F = [torch.zeros_like(E) for _ in range(2)]
    T0 = T.clone()
    ctx.matter_source(E, F, to_dev(w.sigma, torch.float64), cv, k0, T, 0.1)
    torch.cuda.synchronize()
    # to round-off: the residual at T^- is a sum of rounding errors, over a derivative >= cv
    assert torch.allclose(T, T0, rtol=1e-12, atol=0)
    assert torch.allclose(E, B, rtol=1e-12, atol=0)


@pytest.mark.parametrize("prec", [0, 1])
def test_matter_coeffs_match_oracle(m1, prec):
    w = _zone_case(seed=4)
    k, B = orc.matter_coeffs(_model(w), w.kappa0, w.T)
    ctx = _ctx(m1, w, prec)
    kg, Bg = ctx.matter_coeffs(*(to_dev(x, torch.float64) for x in (w.cv, w.kappa0, w.T)))
    torch.cuda.synchronize()
    tol = 1e-13 if prec == 0 else 1e-6
    assert _close(to_host(kg), k, tol)
    assert _close(to_host(Bg), B, tol)


@pytest.mark.parametrize("prec", [0, 1])
def test_transport_matches_oracle(m1, prec):
    w = wl.blobs2d(n=40, G=16)
    p = problem_of(w)
    E, F = orc.explicit(p, w.E, w.F, w.kappa, w.sigma, w.dt)
    ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
    dtp = ctx.dtype
    Eo, Fo = ctx.transport(to_dev(w.E, dtp), [to_dev(f, dtp) for f in w.F], to_dev(w.kappa, dtp),
                           to_dev(w.sigma, dtp), w.dt)
    torch.cuda.synchronize()
    eE, eF = rel_l1(to_host(Eo), [to_host(f) for f in Fo], E, F, w.c)
    tol = TOL_FP64 if prec == 0 else TOL_MIXED_STEP
    assert eE <= tol and eF <= tol


def test_transport_then_source_is_the_step_with_ssprk2(m1):
    w = wl.blobs2d(n=30, G=16)
    ctx = m1.Context(m1.Config.from_workload(w, precision=0, integrator=m1.SSPRK2))
    d = lambda a: to_dev(a, torch.float64)
    k, s, B = d(w.kappa), d(w.sigma), d(w.B)
    E1, F1 = ctx.step(d(w.E), [d(f) for f in w.F], k, s, B, w.dt)
    Em, Fm = ctx.transport(d(w.E), [d(f) for f in w.F], k, s, w.dt)
    ctx.source(Em, Fm, k, s, B, w.dt)
    torch.cuda.synchronize()
    eE, eF = rel_l1(to_host(Em), [to_host(f) for f in Fm], to_host(E1), [to_host(f) for f in F1], w.c)
    assert eE <= 1e-15 and eF <= 1e-15


@pytest.mark.parametrize("prec", [0, 1])
def test_coupled_steps_match_oracle(m1, prec):
    """Three steps of transport with the opacities at T^n, then the outer solve, on the
    blob radiation with random matter (2-D periodic, 32^2 x 16)."""
    w = wl.matter2d(n=32, G=16, seed=3)
    p = problem_of(w)
    m = _model(w)
    E, F, T = w.E, w.F, w.T
    for _ in range(3):
        E, F, T, dEm, it = orc.matter_step(p, m, E, F, w.sigma, w.cv, w.kappa0, T, w.dt)
    ctx = _ctx(m1, w, prec)
    dtp = ctx.dtype
    Eg, Fg = to_dev(w.E, dtp), [to_dev(f, dtp) for f in w.F]
    sig = to_dev(w.sigma, dtp)
    cv, k0, Tg = (to_dev(x, torch.float64) for x in (w.cv, w.kappa0, w.T))
    for _ in range(3):
        Eg, Fg = ctx.matter_step(Eg, Fg, sig, cv, k0, Tg, w.dt)
    torch.cuda.synchronize()
    eE, eF = rel_l1(to_host(Eg), [to_host(f) for f in Fg], E, F, w.c)
    eT = np.abs(to_host(Tg) - T).max() / np.abs(T).max()
    say(f"coupled prec={prec}", eE, eF, eT)
    tol = 1e-10 if prec == 0 else 1e-5
    assert eE <= tol and eF <= tol and eT <= tol


def test_full_size_matter_source_sampled(m1):
    """The 512^2 x 16 workload's interaction update on the GPU; the oracle on 4096 sampled
    zones (the update is zone-local)."""
    w = wl.matter2d(n=512, G=16)
    dt = w.dt
    Eg, Fg, Tg, dEg, itg = _gpu_source(m1, w, dt)
    rng = np.random.default_rng(5)
    zs = np.sort(rng.choice(512 * 512, 4096, replace=False))
    G = w.G
    Ez = w.E.reshape(-1, G)[zs]
    Fz = [f.reshape(-1, G)[zs] for f in w.F]
    E, F, T, dEm, it = orc.matter_source(_model(w), Ez, Fz, w.sigma.reshape(-1, G)[zs], w.cv.ravel()[zs],
                                         w.kappa0.ravel()[zs], w.T.ravel()[zs], dt)
    assert np.allclose(Tg.ravel()[zs], T, rtol=TOL_MATTER, atol=0)
    assert _close(Eg.reshape(-1, G)[zs], E, TOL_MATTER)
    for a, b in zip(Fg, F):
        assert _close(a.reshape(-1, G)[zs], b, TOL_MATTER)
