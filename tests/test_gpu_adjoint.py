"""GPU adjoint of the M1 step against the CPU oracle's exact forward-mode derivative (dual
numbers) and central finite differences.

Dot-product identity for one step: <lam_{n+1}, J dU> + ... = <J^T lam_{n+1}, dU> + <g_kappa, dkappa>
with J dU from the oracle (FP64 dual numbers) and J^T lam from fornax_m1_adjoint.  Multi-step
gradients through the checkpointed torch.autograd.Function are checked entry by entry against
oracle JVPs along unit directions and against central differences."""
import sys

import numpy as np
import pytest
import torch

from oracle import m1_oracle as orc
from paper_1806_07390_amd import workloads as wl
from tests.parity_util import problem_of, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m1():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1806_07390_amd import m1 as mod
    return mod


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def one_step_dot(m1, w, precision, seed=3, local=None):
    """Return (lhs, rhs, scale) of the one-step dot-product identity."""
    p = problem_of(w)
    rng = np.random.default_rng(seed)
    shape = w.E.shape
    mask = np.ones(shape)
    if local is not None:
        mask = np.zeros(shape)
        mask[local] = 1.0
    dE = rng.standard_normal(shape) * w.E * mask
    dF = [rng.standard_normal(shape) * w.E * mask for _ in w.F]
    dk = rng.standard_normal(shape) * w.kappa * mask
    E1, F1, dE1, dF1 = orc.jvp(p, w.E, w.F, w.kappa, w.sigma, w.B, w.dt, 1, dE=dE, dF=dF, dkappa=dk)
    lamE = rng.standard_normal(shape)
    lamF = [rng.standard_normal(shape) for _ in w.F]
    lhs = np.sum(lamE * dE1) + sum(np.sum(a * b) for a, b in zip(lamF, dF1))
    ctx = m1.Context(m1.Config.from_workload(w, precision=precision))
    dtp = ctx.dtype
    E = to_dev(w.E, dtp)
    F = [to_dev(f, dtp) for f in w.F]
    k, s, B = (to_dev(x, dtp) for x in (w.kappa, w.sigma, w.B))
    lE, lF, gk = ctx.adjoint(E, F, k, s, B, w.dt, to_dev(lamE, dtp), [to_dev(f, dtp) for f in lamF])
    torch.cuda.synchronize()
    lE, lF, gk = to_host(lE), [to_host(f) for f in lF], to_host(gk)
    rhs = np.sum(lE * dE) + sum(np.sum(a * b) for a, b in zip(lF, dF)) + np.sum(gk * dk)
    scale = (np.sum(np.abs(lE * dE)) + sum(np.sum(np.abs(a * b)) for a, b in zip(lF, dF))
             + np.sum(np.abs(gk * dk)))
    return lhs, rhs, scale


# (lower, upper) boundary rules per direction (x, y).  A direction periodic at both ends wraps
# in the adjoint kernel (no ghost zones); "x_periodic" and "y_periodic" have one wrapping
# direction and ghost zones along the other.
_BCS = {
    "periodic": ((wl.BC_PERIODIC, wl.BC_PERIODIC), (wl.BC_PERIODIC, wl.BC_PERIODIC)),
    "outflow": ((wl.BC_OUTFLOW, wl.BC_OUTFLOW), (wl.BC_OUTFLOW, wl.BC_OUTFLOW)),
    "reflect": ((wl.BC_REFLECT, wl.BC_OUTFLOW), (wl.BC_REFLECT, wl.BC_REFLECT)),
    "x_periodic": ((wl.BC_PERIODIC, wl.BC_OUTFLOW), (wl.BC_PERIODIC, wl.BC_REFLECT)),
    "y_periodic": ((wl.BC_REFLECT, wl.BC_PERIODIC), (wl.BC_OUTFLOW, wl.BC_PERIODIC)),
}


def _set_bcs(w, bc):
    lo, hi = _BCS[bc]
    w.bc_lo = lo + (0,)
    w.bc_hi = hi + (0,)


@pytest.mark.parametrize("bc", list(_BCS))
def test_one_step_dot_product_2d_fp64(m1, bc):
    w = wl.adjoint2d(n=24, G=3, steps=1)
    _set_bcs(w, bc)
    for local in (None, (slice(None), slice(None), slice(0, 3)), (slice(None), slice(20, 24), slice(None))):
        lhs, rhs, scale = one_step_dot(m1, w, m1.FP64, local=local)
        say(bc, local, lhs, rhs, scale)
        assert abs(lhs - rhs) <= 1e-12 * scale


@pytest.mark.parametrize("n0,n1", [(4, 4), (5, 7), (3, 6)])
def test_one_step_dot_product_small_periodic(m1, n0, n1):
    """Periodic grids at the smallest sizes: a direction of four or more zones wraps in the
    adjoint kernel (no ghost zones; its stencils reach around the whole axis), one of three
    keeps its ghost zones and the fold; the dot-product identity holds on each."""
    w = wl.adjoint2d(n=max(n0, n1), G=3, steps=1)
    cut = lambda a: np.ascontiguousarray(a[..., :n1, :n0, :])
    w.E, w.kappa, w.sigma, w.B = cut(w.E), cut(w.kappa), cut(w.sigma), cut(w.B)
    w.F = [cut(f) for f in w.F]
    w.n = (n0, n1, 1)
    for local in (None, (slice(None), slice(0, 1), slice(None))):
        lhs, rhs, scale = one_step_dot(m1, w, m1.FP64, local=local)
        say("small periodic", n0, n1, local, lhs, rhs, scale)
        assert abs(lhs - rhs) <= 1e-12 * scale


@pytest.mark.parametrize("bc", ["outflow", "periodic"])
def test_one_step_dot_product_1d_fp64(m1, bc):
    w = wl.slab1d(n=40, G=2)
    w.dt = 0.4 / 40
    if bc == "periodic":
        w.bc_lo = w.bc_hi = (wl.BC_PERIODIC,) * 3
    for local in (None, (slice(None), slice(None), slice(0, 3)), (slice(None), slice(None), slice(36, 40))):
        lhs, rhs, scale = one_step_dot(m1, w, m1.FP64, local=local)
        say("1d", bc, local, lhs, rhs, scale)
        assert abs(lhs - rhs) <= 1e-12 * scale


def test_one_step_dot_product_options(m1):
    w = wl.adjoint2d(n=16, G=2, steps=1)
    for lim, clo in ((m1.LIMITER_MC, m1.CLOSURE_M1), (m1.LIMITER_NONE, m1.CLOSURE_M1),
                     (m1.LIMITER_MINMOD, m1.CLOSURE_EDDINGTON)):
        p = problem_of(w, limiter=lim, closure=clo)
        rng = np.random.default_rng(11)
        dE = rng.standard_normal(w.E.shape) * w.E
        dk = rng.standard_normal(w.E.shape) * w.kappa
        _, _, dE1, dF1 = orc.jvp(p, w.E, w.F, w.kappa, w.sigma, w.B, w.dt, 1, dE=dE, dkappa=dk)
        lamE = rng.standard_normal(w.E.shape)
        lhs = np.sum(lamE * dE1)
        ctx = m1.Context(m1.Config.from_workload(w, precision=m1.FP64, limiter=lim, closure=clo))
        t = lambda a: to_dev(a, torch.float64)
        z = [torch.zeros_like(t(w.E)) for _ in w.F]
        lE, lF, gk = ctx.adjoint(t(w.E), [t(f) for f in w.F], t(w.kappa), t(w.sigma), t(w.B), w.dt, t(lamE), z)
        rhs = np.sum(to_host(lE) * dE) + np.sum(to_host(gk) * dk)
        scale = np.sum(np.abs(to_host(lE) * dE)) + np.sum(np.abs(to_host(gk) * dk))
        assert abs(lhs - rhs) <= 1e-12 * scale, (lim, clo)


@pytest.mark.parametrize("lim", ["minmod", "mc", "none"])
def test_one_step_dot_product_kappa_only(m1, lim):
    """Perturb kappa alone: the identity then rests on g_kappa only (the interaction source
    through U^{n+1}, and epsilon in optically thick faces), not on the state adjoint."""
    code = {"minmod": m1.LIMITER_MINMOD, "mc": m1.LIMITER_MC, "none": m1.LIMITER_NONE}[lim]
    w = wl.adjoint2d(n=20, G=3, steps=1)
    p = problem_of(w, limiter=code)
    rng = np.random.default_rng(29)
    dk = rng.standard_normal(w.E.shape) * w.kappa
    _, _, dE1, dF1 = orc.jvp(p, w.E, w.F, w.kappa, w.sigma, w.B, w.dt, 1, dkappa=dk)
    lamE = rng.standard_normal(w.E.shape)
    lamF = [rng.standard_normal(w.E.shape) for _ in w.F]
    lhs = np.sum(lamE * dE1) + sum(np.sum(a * b) for a, b in zip(lamF, dF1))
    ctx = m1.Context(m1.Config.from_workload(w, precision=m1.FP64, limiter=code))
    t = lambda a: to_dev(a, torch.float64)
    _, _, gk = ctx.adjoint(t(w.E), [t(f) for f in w.F], t(w.kappa), t(w.sigma), t(w.B), w.dt, t(lamE),
                           [t(f) for f in lamF])
    gk = to_host(gk)
    rhs = np.sum(gk * dk)
    scale = np.sum(np.abs(gk * dk))
    say("kappa-only", lim, lhs, rhs, scale)
    assert scale > 0
    assert abs(lhs - rhs) <= 1e-12 * scale


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adjoint_with_given_next_state(m1, precision):
    """Supplying U^{n+1} (as the checkpointed backward does) gives bit for bit the result of
    the binding's call without it (which runs the step first); a wrong U^{n+1} changes only
    dkappa."""
    prec = m1.FP64 if precision == "fp64" else m1.MIXED
    w = wl.adjoint2d(n=40, G=4, steps=1)
    ctx = m1.Context(m1.Config.from_workload(w, precision=prec))
    dtp = ctx.dtype
    rng = np.random.default_rng(5)
    E = to_dev(w.E, dtp)
    F = [to_dev(f, dtp) for f in w.F]
    k, s, B = (to_dev(x, dtp) for x in (w.kappa, w.sigma, w.B))
    lamE = to_dev(rng.standard_normal(w.E.shape), dtp)
    lamF = [to_dev(rng.standard_normal(w.E.shape), dtp) for _ in w.F]
    U1 = ctx.step(E, F, k, s, B, w.dt)
    a = ctx.adjoint(E, F, k, s, B, w.dt, lamE, lamF)
    b = ctx.adjoint(E, F, k, s, B, w.dt, lamE, lamF, U1=U1)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and all(torch.equal(x, y) for x, y in zip(a[1], b[1]))
    assert torch.equal(a[2], b[2])
    wrong = (U1[0] * 1.5, U1[1])
    c = ctx.adjoint(E, F, k, s, B, w.dt, lamE, lamF, U1=wrong)
    torch.cuda.synchronize()
    assert torch.equal(a[0], c[0]) and not torch.equal(a[2], c[2])


@pytest.mark.parametrize("bc", ["periodic", "reflect", "x_periodic", "y_periodic"])
def test_adjoint_independent_of_tiling(m1, bc):
    """The adjoint kernel's blocks of TXB zone columns by TM planes (FORNAX_M1_ADJ_TILE="TXB,TM" when
    the context is created; the default takes TM from the CU count): one plane per block, the fewest columns, tiles
    that do not divide the grid, all give the default tiling's result -- each zone sums the
    same face contributions in the same order whichever block computes them."""
    import os
    w = wl.adjoint2d(n=40, G=4, steps=1)
    cut = lambda a: np.ascontiguousarray(a[..., :37, :])   # 37 zones along x
    w.E, w.kappa, w.sigma, w.B = cut(w.E), cut(w.kappa), cut(w.sigma), cut(w.B)
    w.F = [cut(f) for f in w.F]
    w.n = (37, 40, 1)
    if bc == "reflect":
        w.bc_lo = (wl.BC_REFLECT, wl.BC_OUTFLOW, 0)
        w.bc_hi = (wl.BC_OUTFLOW, wl.BC_REFLECT, 0)
    elif bc != "periodic":
        _set_bcs(w, bc)
    ctx = m1.Context(m1.Config.from_workload(w, precision=m1.FP64))
    dtp = ctx.dtype
    rng = np.random.default_rng(9)
    E = to_dev(w.E, dtp)
    F = [to_dev(f, dtp) for f in w.F]
    k, s, B = (to_dev(x, dtp) for x in (w.kappa, w.sigma, w.B))
    lamE = to_dev(rng.standard_normal(w.E.shape), dtp)
    lamF = [to_dev(rng.standard_normal(w.E.shape), dtp) for _ in w.F]
    ref = ctx.adjoint(E, F, k, s, B, w.dt, lamE, lamF)
    torch.cuda.synchronize()
    ref = [to_host(ref[0])] + [to_host(f) for f in ref[1]] + [to_host(ref[2])]
    for tile in ("16,1", "16,2", "16,3", "4,5", "7,7", "64,9", "9,40"):
        # the override is read when a context is created
        os.environ["FORNAX_M1_ADJ_TILE"] = tile
        try:
            ctx_t = m1.Context(m1.Config.from_workload(w, precision=m1.FP64))
        finally:
            del os.environ["FORNAX_M1_ADJ_TILE"]
        got = ctx_t.adjoint(E, F, k, s, B, w.dt, lamE, lamF)
        torch.cuda.synchronize()
        del ctx_t
        got = [to_host(got[0])] + [to_host(f) for f in got[1]] + [to_host(got[2])]
        for a, b in zip(got, ref):
            err = np.abs(a - b).max() / np.abs(b).max()
            say("adjoint tile", bc, tile, err)
            assert err <= 1e-14


def test_one_step_dot_product_mixed(m1):
    w = wl.adjoint2d(n=32, G=4, steps=1)
    lhs, rhs, scale = one_step_dot(m1, w, m1.MIXED)
    say("mixed", lhs, rhs, scale)
    assert abs(lhs - rhs) <= 1e-5 * scale


# ------------------------------------------------------------------------------------------
# Finite differences of the FP64 oracle's loss, Richardson-extrapolated:
#   D(h) = (L(x + h) - L(x - h)) / 2h = L' + h^2 L3 / 6 + O(h^4) + rounding   (L3 = d^3 L/dx^3),
#   R = (4 D(h/2) - D(h)) / 3 = L' + O(h^4) + rounding,
# with h = FD_ETA |x|.  Truncation: the loss varies on the scale of x itself (opacities and
# energies enter through ratios), so R's truncation is ~FD_ETA^4 relative, negligible.
# Rounding: a perturbation changes the rounding of every value downstream, and R carries an
# error of about eps |L| / h (eps = 2.2e-16; measured against the dual-number derivative on
# this workload: at most 1.3 eps |L| / h over the 64 entries), so the comparisons add the
# floor 30 eps |L| / h to their relative tolerance; a gradient entry is resolved where it
# stands well above that floor.  Branches: the scheme is piecewise smooth (minmod choice,
# realizability fallback, the epsilon kink, the f clamp), and on the blob workload those
# switches are dense: at h = 1e-3 |x| many quotients differ from the derivative at 1e-4 with
# no rounding to explain it.  h = 1e-5 |x| keeps switches inside [x - h, x + h] rare; a
# quotient that still meets one shows as |D(h) - R| > FD_SMOOTH |R| + floor (a smooth stretch
# gives h^2 L3 / 8, ~1e-11 relative).  Such branch entries are counted and bounded separately:
# the derivative of the branch the forward step takes at x lies between the one-sided
# quotients (L(x) - L(x - h))/h and (L(x + h) - L(x))/h, up to their O(h) truncation.
FD_ETA = 1e-5
FD_SMOOTH = 1e-3
FD_TOL = 1e-5        # adjoint vs R on smooth entries, on top of the rounding floor


def fd_richardson(f, x0, L0):
    """(R, D(h), one-sided quotients, rounding floor) for the scalar function f at x0."""
    h = FD_ETA * abs(x0)
    fp, fm = f(h), f(-h)
    fp2, fm2 = f(0.5 * h), f(-0.5 * h)
    D1 = (fp - fm) / (2 * h)
    D2 = (fp2 - fm2) / h
    R = (4 * D2 - D1) / 3
    one_sided = ((L0 - fm) / h, (fp - L0) / h)
    floor = 30 * 2.2e-16 * abs(L0) / h
    return R, D1, one_sided, floor


def window_loss_grad(m1, w, precision, ckpt_every):
    """GPU gradient of L = sum over the detector window and groups of E_N (autograd)."""
    ix, iy, ww = w.extra["window"]
    ctx = m1.Context(m1.Config.from_workload(w, precision=precision))
    dtp = ctx.dtype
    E0 = to_dev(w.E, dtp).requires_grad_(True)
    F0 = [to_dev(f, dtp).requires_grad_(True) for f in w.F]
    k = to_dev(w.kappa, dtp).requires_grad_(True)
    s, B = to_dev(w.sigma, dtp), to_dev(w.B, dtp)
    EN, FN = m1.run_differentiable(ctx, E0, F0, k, s, B, w.dt, w.steps, ckpt_every=ckpt_every)
    L = EN[0, iy:iy + ww, ix:ix + ww, :].sum()
    L.backward()
    torch.cuda.synchronize()
    return float(L.item()), to_host(k.grad), to_host(E0.grad)


def oracle_loss(p, w, E0, kappa):
    ix, iy, ww = w.extra["window"]
    E, F, _ = orc.run(p, E0, w.F, kappa, w.sigma, w.B, w.dt, w.steps)
    return E[0, iy:iy + ww, ix:ix + ww, :].sum()


def oracle_dloss(p, w, dE=None, dk=None):
    ix, iy, ww = w.extra["window"]
    _, _, dEN, _ = orc.jvp(p, w.E, w.F, w.kappa, w.sigma, w.B, w.dt, w.steps, dE=dE, dkappa=dk)
    return dEN[0, iy:iy + ww, ix:ix + ww, :].sum()


def fd_entry(p, w, kind, e, L0):
    base = (w.kappa if kind == "kappa" else w.E).ravel()[e]

    def f(delta):
        if kind == "kappa":
            kk = w.kappa.copy()
            kk.ravel()[e] += delta
            return oracle_loss(p, w, w.E, kk)
        EE = w.E.copy()
        EE.ravel()[e] += delta
        return oracle_loss(p, w, EE, w.kappa)

    return fd_richardson(f, base, L0)


def test_checkpointed_gradient_matches_oracle_jvp_and_fd(m1):
    """FP64, 32^2 x 4 groups, 40 steps checkpointed every 8, 64 seeded entries (32 of kappa,
    32 of E^0): the GPU gradient equals the oracle's dual-number derivative to 1e-8, and the
    Richardson difference quotient to FD_TOL plus the rounding floor on every smooth entry
    (at least half of the entries stand 100x above that floor); branch entries (at most 8)
    lie between their one-sided quotients."""
    w = wl.adjoint2d(n=32, G=4, steps=40, window=12)
    p = problem_of(w)
    L, gk, gE = window_loss_grad(m1, w, m1.FP64, 8)
    L0 = oracle_loss(p, w, w.E, w.kappa)
    assert L == pytest.approx(L0, rel=1e-12)
    rng = np.random.default_rng(42)
    nz = w.E.size
    ent_k = rng.choice(nz, 32, replace=False)
    ent_E = rng.choice(nz, 32, replace=False)
    worst_jvp, worst_fd, branch, worst_branch, resolved = 0.0, 0.0, [], 0.0, 0
    gscale = max(np.abs(gk).max(), np.abs(gE).max())
    for kind, ents in (("kappa", ent_k), ("E", ent_E)):
        for e in ents:
            d = np.zeros(nz)
            d[e] = 1.0
            d = d.reshape(w.E.shape)
            ref = oracle_dloss(p, w, dE=d if kind == "E" else None, dk=d if kind == "kappa" else None)
            got = (gk if kind == "kappa" else gE).ravel()[e]
            worst_jvp = max(worst_jvp, abs(got - ref) / (abs(ref) + 1e-9 * gscale))
            R, D1, (lo, hi), floor = fd_entry(p, w, kind, e, L0)
            if abs(R) > 100 * floor:
                resolved += 1
            if abs(D1 - R) > FD_SMOOTH * abs(R) + floor:
                branch.append((kind, int(e)))
                # one-sided quotients carry an O(h) truncation: 1e-2 of their size
                slack = 1e-2 * (abs(lo) + abs(hi)) + floor
                worst_branch = max(worst_branch, max(min(lo, hi) - got, got - max(lo, hi), 0.0) / slack)
                continue
            # the excess of |got - R| over the rounding floor, relative to |R|
            worst_fd = max(worst_fd, max(abs(got - R) - floor, 0.0) / abs(R) if R != 0 else 0.0)
    say("checkpointed fp64: worst vs JVP", worst_jvp, "vs Richardson FD", worst_fd, "resolved entries", resolved,
        "branch entries", branch, "worst branch excess", worst_branch)
    assert worst_jvp <= 1e-8
    assert worst_fd <= FD_TOL
    assert resolved >= 32
    assert len(branch) <= 8
    assert worst_branch <= 1.0


def test_full_size_adjoint_entries_vs_fd(m1):
    """256^2 x 16 groups, 40 steps checkpointed every 8, FP32 bulk (the adjoint workload): four
    seeded entries (two of kappa, two of E^0) inside the detector window, GPU gradient against
    the oracle's dual-number derivative to the MIXED adjoint gate 1e-3; where the FP64 oracle's
    Richardson difference quotient at full size is smooth, the dual-number derivative agrees
    with it to FD_TOL and the GPU gradient to 1e-3."""
    w = wl.adjoint2d()
    p = problem_of(w, nthreads=0)
    say("full-size adjoint fd", w.n, w.G, w.steps)
    _, gk, gE = window_loss_grad(m1, w, m1.MIXED, 8)
    L0 = oracle_loss(p, w, w.E, w.kappa)
    ix, iy, ww = w.extra["window"]
    rng = np.random.default_rng(17)

    def pick():
        j = iy + int(rng.integers(0, ww))
        i = ix + int(rng.integers(0, ww))
        g = int(rng.integers(0, w.G))
        return (j * w.n[0] + i) * w.G + g

    for kind in ("kappa", "kappa", "E", "E"):
        e = pick()
        R, D1, _, floor = fd_entry(p, w, kind, e, L0)
        smooth = abs(D1 - R) <= FD_SMOOTH * abs(R) + floor
        d = np.zeros(w.E.size)
        d[e] = 1.0
        d = d.reshape(w.E.shape)
        ref = oracle_dloss(p, w, dE=d if kind == "E" else None, dk=d if kind == "kappa" else None)
        got = (gk if kind == "kappa" else gE).ravel()[e]
        say(f"  {kind} entry {e}: gpu {got:.6e} jvp {ref:.6e} richardson {R:.6e} smooth {smooth}")
        assert got == pytest.approx(ref, rel=1e-3, abs=floor)
        if smooth:
            assert abs(ref - R) <= FD_TOL * abs(R) + floor
            assert abs(got - R) <= 1e-3 * abs(R) + floor


def test_checkpoint_interval_does_not_change_gradient(m1):
    w = wl.adjoint2d(n=24, G=2, steps=12, window=8)
    _, gk1, gE1 = window_loss_grad(m1, w, m1.FP64, 1)
    _, gk8, gE8 = window_loss_grad(m1, w, m1.FP64, 8)
    _, gkA, gEA = window_loss_grad(m1, w, m1.FP64, 12)
    assert np.array_equal(gk1, gk8) and np.array_equal(gE1, gE8)
    assert np.array_equal(gk1, gkA) and np.array_equal(gE1, gEA)


def test_backward_replay_reused_across_runs(m1):
    """One context and one set of coefficient tensors: the replay's bound calls are kept between
    backward passes and pointed at each run's checkpoints.  Runs with different segment mixes
    in a row (8 + 4, 8 + 8, 8 + 4 steps) each give a fresh context's gradient bit for bit."""
    w12 = wl.adjoint2d(n=24, G=2, steps=12, window=8)
    ix, iy, ww = w12.extra["window"]
    ctx = m1.Context(m1.Config.from_workload(w12, precision=m1.FP64))
    dtp = ctx.dtype
    k = to_dev(w12.kappa, dtp).requires_grad_(True)
    s, B = to_dev(w12.sigma, dtp), to_dev(w12.B, dtp)

    def run(nsteps):
        k.grad = None
        E0 = to_dev(w12.E, dtp).requires_grad_(True)
        F0 = [to_dev(f, dtp) for f in w12.F]
        EN, _ = m1.run_differentiable(ctx, E0, F0, k, s, B, w12.dt, nsteps, ckpt_every=8)
        EN[0, iy:iy + ww, ix:ix + ww, :].sum().backward()
        torch.cuda.synchronize()
        return to_host(k.grad), to_host(E0.grad)

    for n in (12, 16, 12):
        gk, gE = run(n)
        _, rk, rE = window_loss_grad(m1, wl.adjoint2d(n=24, G=2, steps=n, window=8), m1.FP64, 1)
        assert np.array_equal(gk, rk) and np.array_equal(gE, rE), n


def test_mixed_gradient_close_to_fp64_oracle(m1):
    w = wl.adjoint2d(n=32, G=4, steps=40, window=12)
    p = problem_of(w)
    _, gk, gE = window_loss_grad(m1, w, m1.MIXED, 8)
    rng = np.random.default_rng(9)
    vk = rng.standard_normal(w.E.shape) * w.kappa
    vE = rng.standard_normal(w.E.shape) * w.E
    ref = oracle_dloss(p, w, dE=vE, dk=vk)
    got = np.sum(gk * vk) + np.sum(gE * vE)
    say("mixed directional derivative", got, ref)
    assert got == pytest.approx(ref, rel=1e-3)


def test_full_size_adjoint_directional_derivative(m1):
    """256^2 zones x 16 groups, 40 steps checkpointed every 8, FP32 bulk: the gradient dotted
    with a random direction equals the oracle's exact directional derivative."""
    w = wl.adjoint2d()
    p = problem_of(w, nthreads=0)
    say("full-size adjoint", w.n, w.G, w.steps)
    _, gk, gE = window_loss_grad(m1, w, m1.MIXED, 8)
    rng = np.random.default_rng(5)
    vk = rng.standard_normal(w.E.shape) * w.kappa
    ref = oracle_dloss(p, w, dk=vk)
    got = np.sum(gk * vk)
    say("full-size kappa directional derivative", got, ref)
    assert got == pytest.approx(ref, rel=1e-3)
