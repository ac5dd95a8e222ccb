"""Seeded synthetic inputs for the M1 radiation-moment step.

This module only draws and lays out input arrays; it holds none of the method's arithmetic
(no geometry, closure, flux or source).  Both the GPU path and the CPU oracle consume what
it returns.  Arrays are float64 NumPy arrays in the layout ``[n2][n1][n0][G]`` (zone-major,
group innermost); flux arrays hold covariant components ``F_k`` (physical components on
Cartesian grids; every spherical workload here starts with ``F = 0``).

Workloads (sizes overridable for reduced parity cases):
  * ``slab1d``   1-D slab, 128 zones, 4 groups, outflow, absorbing right half (200 steps)
  * ``blobs2d``  2-D periodic 512^2, 16 groups, lognormal opacity, 8 Gaussian blobs (100 steps)
  * ``core3d``   3-D 192^3, 12 groups, opaque core in a thin halo, Planck group weights (50 steps)
  * ``sphere3d`` spherical (ln r, theta, phi) 256x64x128, 20 groups, inner inflow (100 steps)
  * ``adjoint2d`` 2-D periodic 256^2, 16 groups, lognormal per zone-group opacity (40 steps)
  * ``matter2d`` the ``blobs2d`` radiation with a matter temperature, heat capacity and
    opacity scale per zone (the radiation-matter energy exchange)

Velocity fields for the velocity-dependent terms (``face_velocity``) hold coordinate
components on the zone faces, ``[ndim][n2'][n1'][n0']`` per face direction (the face
direction's extent one larger); ``velocity_edges`` gives finite group edges in frequency.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# coordinate and boundary codes (same numbering as the C interface)
CARTESIAN, SPHERICAL_LOGR = 0, 1
BC_OUTFLOW, BC_PERIODIC, BC_REFLECT, BC_INFLOW, BC_AXIS = 0, 1, 2, 3, 4


@dataclass
class Workload:
    name: str
    ndim: int
    n: tuple            # (n0, n1, n2)
    G: int
    coord: int
    lo: tuple
    hi: tuple
    bc_lo: tuple
    bc_hi: tuple
    c: float
    steps: int
    E: np.ndarray
    F: list             # ndim arrays
    kappa: np.ndarray
    sigma: np.ndarray
    B: np.ndarray
    dt: float | None = None     # None: cfl * max_dt(1) of the grid
    cfl: float = 0.4
    inflow: np.ndarray | None = None   # [G][1+ndim]: E and physical F of inflow ghosts
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0], self.G)

    @property
    def zone_groups(self):
        return self.n[0] * self.n[1] * self.n[2] * self.G


def _centres(lo, hi, n):
    dx = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * dx


def planck_group_weights(edges):
    """Fraction of a unit Planck spectrum (T = 1) in each group, x = h nu / kT.

    Uses int_x^inf x^3/(e^x - 1) dx = sum_n e^{-n x} (x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4),
    normalised by pi^4/15, so that the weights of groups covering [0, inf) sum to 1.
    """
    def tail(x):
        if math.isinf(x):
            return 0.0
        s = 0.0
        for n in range(1, 2000):
            t = math.exp(-n * x) * (x ** 3 / n + 3 * x ** 2 / n ** 2 + 6 * x / n ** 3 + 6 / n ** 4)
            s += t
            if t < 1e-19 * max(s, 1e-300):
                break
        return s * 15.0 / math.pi ** 4

    return np.array([tail(a) - tail(b) for a, b in zip(edges[:-1], edges[1:])])


def slab1d(n=128, G=4, steps=200):
    """1-D planar slab: Gaussian pulse streaming (F = 0.9 cE) into an absorber at x >= 0.6."""
    c = 1.0
    x = _centres(0.0, 1.0, n)
    w = 0.5 ** np.arange(G)
    E = 1e-6 + np.exp(-(x - 0.3) ** 2 / 0.002)[:, None] * w[None, :]
    E = E.reshape(1, 1, n, G)
    F = [0.9 * c * E]
    kappa = np.where(x >= 0.6, 10.0, 0.0)[:, None] * np.ones(G)[None, :]
    kappa = kappa.reshape(1, 1, n, G)
    sigma = np.zeros_like(E)
    B = np.full_like(E, 1e-6)
    return Workload("slab1d", 1, (n, 1, 1), G, CARTESIAN, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                    (BC_OUTFLOW,) * 3, (BC_OUTFLOW,) * 3, c, steps, E, F, kappa, sigma, B,
                    dt=0.4 / n)


def _blob_state(rng, n, G, c):
    x = _centres(0.0, 1.0, n)
    X, Y = np.meshgrid(x, x, indexing="xy")   # [j][i]
    cen = rng.random((8, 2))
    wid = rng.uniform(0.02, 0.1, 8)
    amp = rng.uniform(0.1, 1.0, (8, G))
    E = np.full((n, n, G), 1e-8)
    for b in range(8):
        dx = X - cen[b, 0]
        dy = Y - cen[b, 1]
        dx -= np.round(dx)      # minimum image on the unit torus
        dy -= np.round(dy)
        d2 = dx * dx + dy * dy
        E += np.exp(-d2 / (2 * wid[b] ** 2))[:, :, None] * amp[b][None, None, :]
    f0 = rng.uniform(0.0, 0.95, (n, n))
    phi = rng.uniform(0.0, 2 * math.pi, (n, n))
    Fx = (f0 * np.cos(phi))[:, :, None] * c * E
    Fy = (f0 * np.sin(phi))[:, :, None] * c * E
    return E.reshape(1, n, n, G), [Fx.reshape(1, n, n, G), Fy.reshape(1, n, n, G)]


def blobs2d(n=512, G=16, steps=100, seed=0):
    """2-D periodic square: lognormal opacity per zone (group factor 2^(g/4)), sigma = kappa/2,
    E = sum of 8 Gaussian blobs + 1e-8, F = f0 c E n^ with f0 ~ U(0, 0.95), random direction."""
    c = 1.0
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, n))
    kappa = np.exp(z)[:, :, None] * (2.0 ** (np.arange(G) / 4.0))[None, None, :]
    kappa = kappa.reshape(1, n, n, G)
    sigma = 0.5 * kappa
    E, F = _blob_state(rng, n, G, c)
    B = np.full_like(E, 1e-8)
    return Workload("blobs2d", 2, (n, n, 1), G, CARTESIAN, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                    (BC_PERIODIC,) * 3, (BC_PERIODIC,) * 3, c, steps, E, F, kappa, sigma, B,
                    dt=0.2 / n)


def core3d(n=192, G=12, steps=50, seed=0):
    """3-D cube, outflow: kappa = 1e3 inside |x - centre| < 0.2, 1e-2 outside, sigma = 0;
    B = Planck group weights at T = 1; E = B + 1e-3 U[0,1); F = 0."""
    c = 1.0
    rng = np.random.default_rng(seed)
    x = _centres(0.0, 1.0, n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2)
    kz = np.where(r < 0.2, 1e3, 1e-2)
    kappa = np.repeat(kz[..., None], G, axis=3)
    sigma = np.zeros_like(kappa)
    edges = np.concatenate([[0.0], np.geomspace(0.5, 20.0, G - 1), [np.inf]])
    Bg = planck_group_weights(edges)
    B = np.broadcast_to(Bg, (n, n, n, G)).copy()
    E = B + 1e-3 * rng.random((n, n, n, G))
    F = [np.zeros_like(E) for _ in range(3)]
    return Workload("core3d", 3, (n, n, n), G, CARTESIAN, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                    (BC_OUTFLOW,) * 3, (BC_OUTFLOW,) * 3, c, steps, E, F, kappa, sigma, B,
                    dt=0.4 / (3 * n))


def sphere3d(nr=256, nth=64, nph=128, G=20, steps=100, rmax=1000.0, ndim=3):
    """Spherical grid, x1 = ln r uniform on [0, ln rmax], theta on [0, pi], phi on [0, 2pi):
    kappa_g = 1e4 r^-3 (1 + g/4) at the zone centre, sigma = 0, B = Planck group weights,
    inner inflow E = B, F^_r = c B / 2; outer outflow; polar axis; periodic phi.
    Initial E = 1e-6 B, F = 0."""
    c = 1.0
    x1 = _centres(0.0, math.log(rmax), nr)
    rc = np.exp(x1)
    edges = np.concatenate([[0.0], np.geomspace(0.1, 30.0, G - 1), [np.inf]])
    Bg = planck_group_weights(edges)
    shape = (nph, nth, nr, G)
    kappa = (1e4 * rc ** -3)[None, None, :, None] * (1.0 + np.arange(G) / 4.0)[None, None, None, :]
    kappa = np.broadcast_to(kappa, shape).copy()
    sigma = np.zeros(shape)
    B = np.broadcast_to(Bg, shape).copy()
    E = 1e-6 * B
    F = [np.zeros(shape) for _ in range(ndim)]
    inflow = np.zeros((G, 1 + ndim))
    inflow[:, 0] = Bg
    inflow[:, 1] = 0.5 * c * Bg
    n = (nr, nth if ndim >= 2 else 1, nph if ndim >= 3 else 1)
    if ndim < 3:
        shape = (n[2], n[1], n[0], G)
        kappa = np.ascontiguousarray(kappa[: n[2], : n[1]])
        sigma = np.zeros(shape)
        B = np.ascontiguousarray(B[: n[2], : n[1]])
        E = 1e-6 * B
        F = [np.zeros(shape) for _ in range(ndim)]
    return Workload("sphere3d", ndim, n, G, SPHERICAL_LOGR, (0.0, 0.0, 0.0), (math.log(rmax), math.pi, 2 * math.pi),
                    (BC_INFLOW, BC_AXIS, BC_PERIODIC), (BC_OUTFLOW, BC_AXIS, BC_PERIODIC), c, steps, E, F,
                    kappa, sigma, B, dt=None, cfl=0.4, inflow=inflow)


def adjoint2d(n=256, G=16, steps=40, seed=0, window=32):
    """2-D periodic: kappa lognormal(0, 0.5) per zone-group, sigma = 0, B = 1e-8; E, F from the
    blob generator (seed + 1); detector = window x window zones at a seeded offset."""
    c = 1.0
    rng = np.random.default_rng(seed)
    kappa = np.exp(0.5 * rng.standard_normal((1, n, n, G)))
    sigma = np.zeros_like(kappa)
    E, F = _blob_state(np.random.default_rng(seed + 1), n, G, c)
    B = np.full_like(E, 1e-8)
    window = min(window, n // 2)
    ix, iy = (int(v) for v in rng.integers(0, n - window + 1, 2))
    wl = Workload("adjoint2d", 2, (n, n, 1), G, CARTESIAN, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                  (BC_PERIODIC,) * 3, (BC_PERIODIC,) * 3, c, steps, E, F, kappa, sigma, B,
                  dt=0.2 / n)
    wl.extra = dict(window=(ix, iy, window), ckpt_every=8)
    return wl


@dataclass
class MatterGroups:
    """Group tables of the matter model: frequency edges [G+1] (first 0, last inf), the
    frequency at which a group's opacity is taken [G] and the group's opacity factor [G]."""

    nu_edge: np.ndarray
    nu_c: np.ndarray
    kg: np.ndarray
    a_rad: float = 1.0


def matter_groups(G=16, lo=0.1, hi=30.0, T1=1.0):
    """Edges 0, G - 1 log-spaced on [lo, hi] (units of k_B T1 / h), inf; opacity frequency the
    geometric mean of a group's edges (lo/2 and 2 hi for the two open groups); opacity factor
    (nu_c / nu_1)^-3 T1^(1/2) with nu_1 = 2.821 T1, the normalisation of the paper's pulse test."""
    inner = np.geomspace(lo, hi, G - 1)
    edges = np.concatenate([[0.0], inner, [np.inf]])
    nu_c = np.empty(G)
    nu_c[0] = 0.5 * inner[0]
    nu_c[1:G - 1] = np.sqrt(inner[:-1] * inner[1:])
    nu_c[G - 1] = 2.0 * inner[-1]
    kg = (nu_c / (2.821 * T1)) ** -3 * math.sqrt(T1)
    return MatterGroups(edges, nu_c, kg)


def matter2d(n=512, G=16, steps=100, seed=0, kappa_scale=1.0):
    """The blobs2d radiation with matter: temperature T = exp(0.3 z1) per zone (z1 ~ N(0,1)),
    heat capacity cv = exp(0.5 z2), opacity scale kappa0 = kappa_scale exp(z3) (the opacity of
    the groups follows from T through the matter model), sigma as in blobs2d."""
    w = blobs2d(n=n, G=G, steps=steps, seed=seed)
    rng = np.random.default_rng(seed + 101)
    z = rng.standard_normal((3, 1, n, n))
    w.name = "matter2d"
    w.T = np.exp(0.3 * z[0])
    w.cv = np.exp(0.5 * z[1])
    w.kappa0 = kappa_scale * np.exp(z[2])
    w.groups = matter_groups(G)
    return w


def face_velocity(w, amp=0.1, seed=0, noise=0.3):
    """A smooth random velocity field on the faces of w's grid plus uncorrelated noise (so that
    the sign of the face velocities and of their differences changes from zone to zone).

    Each component u_i(x) = amp (a_i . s + b_i + 0.4 sin(2 pi k_i . s + p_i) + noise N(0, 1)) with
    s the face position scaled to [0, 1] per axis and a, b, k, p drawn once.  Cartesian grids
    take v^i = c u_i; spherical (ln r, theta, phi) grids v^i = c u_i / r at the face (physical
    speeds up to about amp c, the phi one times sin theta), finite on the polar axis.
    Returns ndim arrays, the d-th [ndim][face extents]."""
    rng = np.random.default_rng(seed + 7919)
    nd = w.ndim
    n = list(w.n)
    A = rng.uniform(-1.0, 1.0, (nd, 3))
    b = rng.uniform(-0.5, 0.5, nd)
    kv = rng.integers(1, 3, (nd, 3))
    ph = rng.uniform(0.0, 2 * math.pi, nd)
    out = []
    for d in range(nd):
        axes = []
        for e in range(3):
            dx = (w.hi[e] - w.lo[e]) / n[e]
            if e == d:
                x = w.lo[e] + dx * np.arange(n[e] + 1)
            else:
                x = w.lo[e] + dx * (np.arange(n[e]) + 0.5)
            axes.append(x)
        X2, X1, X0 = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        X = (X0, X1, X2)
        S = [(X[e] - w.lo[e]) / (w.hi[e] - w.lo[e]) for e in range(3)]
        comps = []
        for i in range(nd):
            lin = sum(A[i, e] * S[e] for e in range(3)) + b[i]
            wave = 0.4 * np.sin(2 * math.pi * sum(kv[i, e] * S[e] for e in range(3)) + ph[i])
            u = amp * (lin + wave + noise * rng.standard_normal(X0.shape))
            if w.coord == SPHERICAL_LOGR:
                u = u / np.exp(X0)
            comps.append(w.c * u)
        out.append(np.ascontiguousarray(np.stack(comps)))
    return out


def velocity_edges(G, lo=0.5, hi=20.0):
    """Finite group edges in frequency: 0, G - 1 log-spaced on [lo, hi], and 2 hi on top."""
    return np.concatenate([[0.0], np.geomspace(lo, hi, G - 1), [2.0 * hi]])

