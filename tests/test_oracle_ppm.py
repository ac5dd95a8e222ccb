"""Pins of the oracle's parabolic reconstruction option (Reconstruction subsection, n = 2:
the parabola with three zones' volume averages, the monotonicity resets, the parabola through
the two face states and the zone's average).

What fixes the answer independently of the oracle: volume averages of a quadratic profile
(taken here by scipy quadrature with the volume element of each coordinate) are reconstructed
exactly wherever the quadratic is monotone, in Cartesian zones and along x1 = ln r and
x2 = theta of the spherical grid; a smooth monotone profile converges at third order; a local
extremum of the data gives a constant zone; after the resets every zone's profile is monotone
within the zone; the full step with the option conserves energy and stays realizable.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import m1_oracle as orc
from paper_1806_07390_amd import workloads as wl


def _faces_1d(x_edges, avg, coord=orc.CART, lo=0.0, hi=1.0):
    n = len(avg)
    p = orc.Problem(ndim=1, n=(n,), G=1, c=1.0, limiter=orc.PPM, coord=coord, lo=(lo, 0, 0), hi=(hi, 1, 1))
    E = np.asarray(avg, dtype=np.float64).reshape(1, 1, n, 1)
    out = orc.faces(p, E, [np.zeros_like(E)], 0)
    return out[0, 0, :, 0, 0, 0], out[0, 0, :, 0, 1, 0]


def _cell_avg(f, w, a, b):
    num = quad(lambda x: f(x) * w(x), a, b, epsabs=0, epsrel=2e-14)[0]
    den = quad(w, a, b, epsabs=0, epsrel=2e-14)[0]
    return num / den


def test_cartesian_quadratic_is_exact():
    n = 24
    xe = np.linspace(0.0, 1.0, n + 1)
    q = lambda x: 2.0 + 1.5 * x + 0.7 * x * x          # monotone on [-1, 2]
    avg = [_cell_avg(q, lambda x: 1.0, xe[i], xe[i + 1]) for i in range(n)]
    vl, vh = _faces_1d(xe, avg)
    for i in range(1, n - 1):
        assert vl[i] == pytest.approx(q(xe[i]), rel=1e-13)
        assert vh[i] == pytest.approx(q(xe[i + 1]), rel=1e-13)
    # the closed form of the uniform grid: (2 q_{i-1} + 5 q_i - q_{i+1}) / 6
    a = np.asarray(avg)
    assert np.allclose(vl[1:-1], (2 * a[:-2] + 5 * a[1:-1] - a[2:]) / 6, rtol=1e-13, atol=0)


@pytest.mark.parametrize("axis", [0, 1])
def test_spherical_quadratic_is_exact_in_the_volume_coordinate(axis):
    """Along x1 = ln r (volume element e^{3 x1}) and x2 = theta (|sin x2|) the parabola with
    the zones' volume averages reproduces a quadratic in the coordinate."""
    n = (10, 12, 4)
    lo, hi = (0.0, 0.3, 0.0), (math.log(20.0), 2.6, 2 * math.pi)
    p = orc.Problem(ndim=3, n=n, G=1, c=1.0, limiter=orc.PPM, coord=orc.SPH_LOGR, lo=lo, hi=hi,
                    bc_lo=(orc.OUTFLOW,) * 3, bc_hi=(orc.OUTFLOW,) * 3)
    w = (lambda x: math.exp(3 * x)) if axis == 0 else (lambda x: abs(math.sin(x)))
    q = (lambda x: 3.0 + 0.8 * x + 0.2 * x * x) if axis == 0 else (lambda x: 4.0 - 1.1 * x + 0.15 * x * x)
    na = n[axis]
    xe = np.linspace(lo[axis], hi[axis], na + 1)
    avg = np.array([_cell_avg(q, w, xe[i], xe[i + 1]) for i in range(na)])
    shape = (n[2], n[1], n[0], 1)
    E = np.empty(shape)
    if axis == 0:
        E[...] = avg[None, None, :, None]
    else:
        E[...] = avg[None, :, None, None]
    F = [np.zeros(shape) for _ in range(3)]
    out = orc.faces(p, E, F, axis)
    for i in range(1, na - 1):
        sl = (0, 0, i, 0) if axis == 0 else (0, i, 0, 0)
        assert out[sl + (0, 0)] == pytest.approx(q(xe[i]), rel=1e-12)
        assert out[sl + (1, 0)] == pytest.approx(q(xe[i + 1]), rel=1e-12)


def test_third_order_convergence_on_smooth_data():
    f = lambda x: math.exp(1.3 * x)
    errs = []
    for n in (16, 32, 64, 128):
        xe = np.linspace(0.0, 1.0, n + 1)
        avg = [(math.exp(1.3 * xe[i + 1]) - math.exp(1.3 * xe[i])) / (1.3 * (xe[i + 1] - xe[i])) for i in range(n)]
        vl, vh = _faces_1d(xe, avg)
        e = max(max(abs(vl[i] - f(xe[i])), abs(vh[i] - f(xe[i + 1]))) for i in range(2, n - 2))
        errs.append(e)
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert all(2.8 < r < 3.2 for r in rates), rates


def test_extremum_gives_a_constant_zone_and_profiles_stay_monotone():
    rng = np.random.default_rng(11)
    n = 400
    xe = np.linspace(0.0, 1.0, n + 1)
    avg = np.cumsum(rng.uniform(-0.2, 1.0, n)) + 5.0 + rng.uniform(0, 0.3, n)
    vl, vh = _faces_1d(xe, avg)
    ext = 0
    for i in range(1, n - 1):
        a, b, c = avg[i - 1], avg[i], avg[i + 1]
        if (b - a) * (c - b) <= 0:
            assert vl[i] == b and vh[i] == b
            ext += 1
            continue
        # the final parabola through (vl, average, vh) has no extremum strictly inside the zone:
        # in u = (x - x_i)/dx its slope c1 = vh - vl and curvature term c2 = 3 (vl + vh - 2 b)
        # satisfy |c1| >= |c2| (to rounding)
        c1, c2 = vh[i] - vl[i], 3 * (vl[i] + vh[i] - 2 * b)
        assert abs(c1) >= abs(c2) * (1 - 1e-12) - 1e-12 * abs(b)
        # and the face states lie on the monotone side of the average
        assert (vh[i] - b) * (c - b) >= -1e-12 * abs(b) and (b - vl[i]) * (b - a) >= -1e-12 * abs(b)
    assert 20 < ext < n - 20


def test_step_with_parabolic_reconstruction_conserves_and_stays_realizable():
    w = wl.blobs2d(n=40, G=3, steps=8)
    p = orc.Problem(ndim=2, n=w.n, G=w.G, bc_lo=w.bc_lo, bc_hi=w.bc_hi, c=w.c, limiter=orc.PPM)
    V = orc.geometry(p)["vol"]
    k0 = np.zeros_like(w.kappa)
    e0 = np.sum(V[..., None] * w.E)
    E, F, dg = orc.run(p, w.E, w.F, k0, w.sigma, w.B, w.dt, w.steps)
    assert dg["energy_total"] == pytest.approx(e0, rel=1e-14)
    assert dg["n_unrealizable"] == 0 and dg["n_nonpositive"] == 0
    # a smooth pulse keeps more of its peak with the parabolas than with minmod slopes
    n = 128
    x = (np.arange(n) + 0.5) / n
    E0 = 1e-3 + np.exp(-((x - 0.3) ** 2) / 0.004)
    shape = (1, 1, n, 1)
    z = np.zeros(shape)
    peaks = {}
    for lim in (orc.MINMOD, orc.PPM):
        p1 = orc.Problem(ndim=1, n=(n,), G=1, c=1.0, limiter=lim, bc_lo=(orc.PERIODIC,) * 3,
                         bc_hi=(orc.PERIODIC,) * 3)
        Ee, Fe, _ = orc.run(p1, E0.reshape(shape), [(0.99 * E0).reshape(shape)], z, z, z, 0.4 / n, 80)
        peaks[lim] = Ee.max()
    assert peaks[orc.PPM] > peaks[orc.MINMOD]
