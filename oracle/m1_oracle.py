"""ctypes wrapper of the CPU FP64 oracle (``oracle/m1_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
CPU-baseline leg of ``bench.py``.  The product library never imports or calls it.

All arrays are float64 NumPy arrays in the layout ``[n2][n1][n0][G]`` (group innermost);
flux components are covariant ``F_k`` (equal to the physical components on Cartesian grids).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "m1_oracle.cpp")
_LIB = os.path.join(_HERE, "libm1_oracle.so")

CART, SPH_LOGR = 0, 1
OUTFLOW, PERIODIC, REFLECT, INFLOW, AXIS = 0, 1, 2, 3, 4
MINMOD, MC, CONST, PPM = 0, 1, 2, 3
EULER, SSPRK2 = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OrcDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("G", ctypes.c_int32),
        ("coord", ctypes.c_int32),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc_lo", ctypes.c_int32 * 3),
        ("bc_hi", ctypes.c_int32 * 3),
        ("limiter", ctypes.c_int32),
        ("closure", ctypes.c_int32),
        ("eps_mode", ctypes.c_int32),
        ("c", ctypes.c_double),
        ("nthreads", ctypes.c_int32),
        ("integrator", ctypes.c_int32),
        ("wavespeed", ctypes.c_int32),
    ]


class OrcDiag(ctypes.Structure):
    _fields_ = [
        ("energy_total", ctypes.c_double),
        ("max_f", ctypes.c_double),
        ("n_unrealizable", ctypes.c_int64),
        ("n_nonpositive", ctypes.c_int64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        d = ctypes.c_double
        vp = ctypes.c_void_p
        _lib.orc_max_dt.restype = d
        _lib.orc_max_dt.argtypes = [P(OrcDesc), d]
        _lib.orc_run.argtypes = [P(OrcDesc), vp, vp, vp, vp, vp, vp, d, ctypes.c_int, vp, vp, vp, P(OrcDiag)]
        _lib.orc_step_zones.argtypes = [P(OrcDesc), vp, vp, vp, vp, vp, vp, d, ctypes.c_int, vp, vp, vp, vp]
        _lib.orc_flux.argtypes = [P(OrcDesc), vp, vp, vp, vp, vp, vp, ctypes.c_int, vp]
        _lib.orc_source.argtypes = [P(OrcDesc), vp, vp, vp, vp, vp, d, vp]
        _lib.orc_jvp.argtypes = [P(OrcDesc), vp, vp, vp, vp, vp, vp, vp, vp, vp, d, ctypes.c_int, vp, vp, vp, vp]
        _lib.orc_geometry.argtypes = [P(OrcDesc), vp, vp, vp, vp, vp, vp, vp, vp]
        _lib.orc_closure.argtypes = [P(OrcDesc), d, vp, vp]
        _lib.orc_m1_speeds.argtypes = [P(OrcDesc), d, d, P(d), P(d)]
        _lib.orc_faces.argtypes = [P(OrcDesc), vp, vp, vp, ctypes.c_int, vp]
        _lib.orc_explicit.argtypes = [P(OrcDesc), vp, vp, vp, vp, vp, d, vp, vp]
        _lib.orc_run_v.argtypes = [P(OrcDesc), vp, vp, vp, vp, vp, vp, vp, vp, d, ctypes.c_int, vp, vp, vp,
                                   P(OrcDiag)]
        _lib.orc_explicit_v.argtypes = [P(OrcDesc), vp, vp, vp, vp, vp, vp, d, vp, vp]
        _lib.orc_freq_adv.argtypes = [P(OrcDesc), vp, vp, vp, vp, d, vp, vp]
        _lib.orc_closure3.argtypes = [P(OrcDesc), d, vp, vp]
        _lib.orc_vel_grad.argtypes = [P(OrcDesc), vp, vp, vp]
        _lib.orc_lab_frame.argtypes = [P(OrcDesc), vp, vp, vp, vp, vp]
        _lib.orc_planck_tail.restype = d
        _lib.orc_planck_tail.argtypes = [d]
        _lib.orc_matter_coeffs.argtypes = [ctypes.c_int, vp, vp, vp, d, ctypes.c_long, vp, vp, vp, vp]
        _lib.orc_matter_source.argtypes = [ctypes.c_int, vp, vp, vp, d, d, d, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_long, vp, vp, vp, vp, vp, vp, d, vp, vp]
    return _lib


@dataclass
class Problem:
    """Grid and method options (the oracle's own description of a problem)."""

    ndim: int
    n: tuple
    G: int
    coord: int = CART
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    bc_lo: tuple = (OUTFLOW, OUTFLOW, OUTFLOW)
    bc_hi: tuple = (OUTFLOW, OUTFLOW, OUTFLOW)
    limiter: int = MINMOD
    closure: int = 0
    eps_mode: int = 0
    c: float = 1.0
    nthreads: int = 0
    integrator: int = EULER
    wavespeed: int = 0          # 0: S = -+c; 1: HLLE bounds from the M1 characteristic speeds
    extra: dict = field(default_factory=dict)

    def desc(self) -> OrcDesc:
        d = OrcDesc()
        d.ndim = self.ndim
        n = list(self.n) + [1] * (3 - len(self.n))
        d.n[:] = n
        d.G = self.G
        d.coord = self.coord
        d.lo[:] = list(self.lo)
        d.hi[:] = list(self.hi)
        d.bc_lo[:] = list(self.bc_lo)
        d.bc_hi[:] = list(self.bc_hi)
        d.limiter = self.limiter
        d.closure = self.closure
        d.eps_mode = self.eps_mode
        d.c = self.c
        d.nthreads = self.nthreads
        d.integrator = self.integrator
        d.wavespeed = self.wavespeed
        return d

    @property
    def shape(self):
        n = list(self.n) + [1] * (3 - len(self.n))
        return (n[2], n[1], n[0], self.G)

    @property
    def nzones(self):
        s = self.shape
        return s[0] * s[1] * s[2]


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _ptrs(arrs):
    arr = (ctypes.c_void_p * 3)()
    for k, a in enumerate(arrs):
        arr[k] = a.ctypes.data if a is not None else None
    return arr


def max_dt(p: Problem, cfl: float) -> float:
    d = p.desc()
    return lib().orc_max_dt(ctypes.byref(d), cfl)


def run(p: Problem, E, F, kappa, sigma, B, dt, nsteps=1, inflow=None, want_dEm=False):
    """nsteps full steps. Returns (E, [F_k], diag dict[, dE_matter])."""
    d = p.desc()
    E = _c(E)
    F = [_c(f) for f in F]
    kappa, sigma, B = _c(kappa), _c(sigma), _c(B)
    inflow = None if inflow is None else _c(inflow)
    Eo = np.empty_like(E)
    Fo = [np.empty_like(E) for _ in range(p.ndim)]
    dEm = np.empty(p.nzones) if want_dEm else None
    diag = OrcDiag()
    lib().orc_run(ctypes.byref(d), _ptr(E), _ptrs(F), _ptr(kappa), _ptr(sigma), _ptr(B), _ptr(inflow), dt, nsteps,
                  _ptr(Eo), _ptrs(Fo), _ptr(dEm), ctypes.byref(diag))
    dg = dict(energy_total=diag.energy_total, max_f=diag.max_f, n_unrealizable=diag.n_unrealizable,
              n_nonpositive=diag.n_nonpositive)
    if want_dEm:
        return Eo, Fo, dg, dEm
    return Eo, Fo, dg


def step_zones(p: Problem, E, F, kappa, sigma, B, dt, zones, inflow=None):
    """One step evaluated at flat zone indices; returns (E1 [nsel,G], [F1_k], Em [nsel,G])."""
    d = p.desc()
    zones = np.ascontiguousarray(zones, dtype=np.int64)
    nsel = zones.size
    E = _c(E)
    F = [_c(f) for f in F]
    kappa, sigma, B = _c(kappa), _c(sigma), _c(B)
    inflow = None if inflow is None else _c(inflow)
    Eo = np.empty((nsel, p.G))
    Fo = [np.empty((nsel, p.G)) for _ in range(p.ndim)]
    Em = np.empty((nsel, p.G))
    lib().orc_step_zones(ctypes.byref(d), _ptr(E), _ptrs(F), _ptr(kappa), _ptr(sigma), _ptr(B), _ptr(inflow), dt,
                         nsel, _ptr(zones), _ptr(Eo), _ptrs(Fo), _ptr(Em))
    return Eo, Fo, Em


def flux(p: Problem, E, F, kappa, sigma, B, d, inflow=None):
    """Face fluxes along direction d: array [faces..., G, 1+ndim] with the d extent n_d+1."""
    desc = p.desc()
    E = _c(E)
    F = [_c(f) for f in F]
    kappa, sigma, B = _c(kappa), _c(sigma), _c(B)
    inflow = None if inflow is None else _c(inflow)
    s = list(p.shape[:3])
    s[2 - d] += 1
    out = np.empty(tuple(s) + (p.G, 1 + p.ndim))
    lib().orc_flux(ctypes.byref(desc), _ptr(E), _ptrs(F), _ptr(kappa), _ptr(sigma), _ptr(B), _ptr(inflow), d,
                   _ptr(out))
    return out


def faces(p: Problem, E, F, d, inflow=None):
    """Face states of every zone along d (after the realizability fallback): array
    [zones..., G, 2, 1+ndim], index 0 of the 2 the lower face."""
    desc = p.desc()
    E = _c(E)
    F = [_c(f) for f in F]
    inflow = None if inflow is None else _c(inflow)
    out = np.empty(tuple(p.shape[:3]) + (p.G, 2, 1 + p.ndim))
    lib().orc_faces(ctypes.byref(desc), _ptr(E), _ptrs(F), _ptr(inflow), d, _ptr(out))
    return out


def source(p: Problem, E, F, kappa, sigma, B, dt):
    """Implicit interaction update alone. Returns (E, [F_k], dE_matter)."""
    desc = p.desc()
    E = _c(E).copy()
    F = [_c(f).copy() for f in F]
    kappa, sigma, B = _c(kappa), _c(sigma), _c(B)
    dEm = np.empty(p.nzones)
    lib().orc_source(ctypes.byref(desc), _ptr(E), _ptrs(F), _ptr(kappa), _ptr(sigma), _ptr(B), dt, _ptr(dEm))
    return E, F, dEm


def jvp(p: Problem, E, F, kappa, sigma, B, dt, nsteps, dE=None, dF=None, dkappa=None, inflow=None):
    """Exact forward-mode derivative: returns (E_N, [F_N], dE_N, [dF_N])."""
    desc = p.desc()
    E = _c(E)
    F = [_c(f) for f in F]
    kappa, sigma, B = _c(kappa), _c(sigma), _c(B)
    dE = None if dE is None else _c(dE)
    dF = None if dF is None else [_c(f) for f in dF]
    dkappa = None if dkappa is None else _c(dkappa)
    inflow = None if inflow is None else _c(inflow)
    Eo = np.empty_like(E)
    Fo = [np.empty_like(E) for _ in range(p.ndim)]
    dEo = np.empty_like(E)
    dFo = [np.empty_like(E) for _ in range(p.ndim)]
    lib().orc_jvp(ctypes.byref(desc), _ptr(E), _ptrs(F), _ptr(dE), _ptrs(dF) if dF is not None else None,
                  _ptr(kappa), _ptr(dkappa), _ptr(sigma), _ptr(B), _ptr(inflow), dt, nsteps, _ptr(Eo), _ptrs(Fo),
                  _ptr(dEo), _ptrs(dFo))
    return Eo, Fo, dEo, dFo


def geometry(p: Problem):
    desc = p.desc()
    n = list(p.n) + [1] * (3 - len(p.n))
    vol = np.empty(p.nzones)
    areas = []
    for d in range(3):
        m = list(n)
        m[d] += 1
        areas.append(np.empty(m[0] * m[1] * m[2]))
    gam = np.zeros(4 * n[1])
    hcell = np.empty(3 * p.nzones)
    c0 = np.empty(n[0])
    c1 = np.empty(n[1])
    lib().orc_geometry(ctypes.byref(desc), _ptr(vol), _ptr(areas[0]), _ptr(areas[1]), _ptr(areas[2]), _ptr(gam),
                       _ptr(hcell), _ptr(c0), _ptr(c1))
    return dict(vol=vol.reshape(n[2], n[1], n[0]),
                area=[a.reshape(*(list(reversed([n[e] + (1 if e == d else 0) for e in range(3)])))) for d, a in
                      enumerate(areas)],
                gamma_theta=gam.reshape(n[1], 4), hcell=hcell.reshape(n[2], n[1], n[0], 3), centroid0=c0,
                centroid1=c1)


def closure(E, Fphys, c=1.0, eddington=False):
    """Physical-component pressure tensor P^ (3x3) of one state (Cartesian scale factors)."""
    p = Problem(ndim=3, n=(1, 1, 1), G=1, c=c, closure=1 if eddington else 0)
    desc = p.desc()
    F = np.ascontiguousarray(np.asarray(Fphys, dtype=np.float64).reshape(3))
    P = np.empty(9)
    lib().orc_closure(ctypes.byref(desc), float(E), _ptr(F), _ptr(P))
    return P.reshape(3, 3)


def m1_speeds(E, Fn, c=1.0, eddington=False):
    """(lambda_-, lambda_+): the oracle's M1 characteristic speeds of one state with physical
    normal flux Fn (the HLLE wavespeed option)."""
    p = Problem(ndim=3, n=(1, 1, 1), G=1, c=c, closure=1 if eddington else 0)
    desc = p.desc()
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().orc_m1_speeds(ctypes.byref(desc), float(E), float(Fn), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def explicit(p: Problem, E, F, kappa, sigma, dt, inflow=None):
    """The explicit transport update alone (U^- = U^n + dt L(U^n)). Returns (E, [F_k])."""
    d = p.desc()
    E = _c(E)
    F = [_c(f) for f in F]
    kappa, sigma = _c(kappa), _c(sigma)
    inflow = None if inflow is None else _c(inflow)
    Eo = np.empty_like(E)
    Fo = [np.empty_like(E) for _ in range(p.ndim)]
    lib().orc_explicit(ctypes.byref(d), E.ctypes.data, _ptrs(F), kappa.ctypes.data, sigma.ctypes.data,
                       None if inflow is None else inflow.ctypes.data, dt, Eo.ctypes.data, _ptrs(Fo))
    return Eo, Fo


# ---- radiation-matter energy exchange (photon case: one outer equation for T) ----

def planck_tail(x: float) -> float:
    """int_x^inf t^3/(e^t - 1) dt."""
    return lib().orc_planck_tail(float(x))


@dataclass
class MatterModel:
    """Group tables of the matter model: frequency edges nu_edge [G+1] (0 and inf allowed),
    opacity frequency nu_c [G] and factor kg [G], radiation constant a_rad, light speed c;
    Newton tolerance on the relative change of T and the Newton iterations before bisection."""

    nu_edge: np.ndarray
    nu_c: np.ndarray
    kg: np.ndarray
    a_rad: float = 1.0
    c: float = 1.0
    tol: float = 1e-6
    max_newton: int = 30

    @property
    def G(self):
        return len(self.nu_c)


def matter_coeffs(m: MatterModel, kappa0, T):
    """kappa_g(T) and B_g(T) per zone-group ([..., G])."""
    kappa0, T = _c(kappa0), _c(T)
    nz = T.size
    kap = np.empty(T.shape + (m.G,))
    B = np.empty_like(kap)
    ne, nc, kg = _c(m.nu_edge), _c(m.nu_c), _c(m.kg)
    lib().orc_matter_coeffs(m.G, ne.ctypes.data, nc.ctypes.data, kg.ctypes.data, m.a_rad, nz, kappa0.ctypes.data,
                            T.ctypes.data, kap.ctypes.data, B.ctypes.data)
    return kap, B


def matter_source(m: MatterModel, E, F, sigma, cv, kappa0, T, dt):
    """Interaction update with the matter energy equation (zone arrays cv, kappa0, T shaped like
    E without its group axis). Returns (E, [F_k], T, dE_matter = u^{n+1} - u^-, iterations)."""
    E = _c(E).copy()
    F = [_c(f).copy() for f in F]
    sigma, cv, kappa0 = _c(sigma), _c(cv), _c(kappa0)
    T = _c(T).copy()
    nz = T.size
    dEm = np.empty(T.shape)
    it = np.empty(T.shape, dtype=np.int32)
    ne, nc, kg = _c(m.nu_edge), _c(m.nu_c), _c(m.kg)
    lib().orc_matter_source(m.G, ne.ctypes.data, nc.ctypes.data, kg.ctypes.data, m.a_rad, m.c, m.tol, m.max_newton,
                            len(F), nz, E.ctypes.data, _ptrs(F), sigma.ctypes.data, cv.ctypes.data,
                            kappa0.ctypes.data, T.ctypes.data, dt, dEm.ctypes.data, it.ctypes.data)
    return E, F, T, dEm, it


def matter_step(p: Problem, m: MatterModel, E, F, sigma, cv, kappa0, T, dt, inflow=None):
    """One step with the matter coupled (Algorithmic Steps 1, 3, 4 for a static medium):
    explicit transport with the opacities at T^n, then the interaction update with the outer
    solve for T^{n+1}. Returns (E, [F_k], T, dE_matter, iterations)."""
    kap, _ = matter_coeffs(m, kappa0, T)
    Em, Fm = explicit(p, E, F, kap, sigma, dt, inflow=inflow)
    return matter_source(m, Em, Fm, sigma, cv, kappa0, T, dt)


# ---- velocity-dependent terms (prescribed velocity) ----

def face_shape(p: Problem, d: int):
    """Shape (n2, n1, n0) of the d-faces, the d extent n_d + 1."""
    s = list(p.shape[:3])
    s[2 - d] += 1
    return tuple(s)


def _vel(p: Problem, vf):
    """The ndim face-velocity arrays, each [ndim, *face_shape(p, d)]: the coordinate
    (contravariant) components v^0..v^{ndim-1} on the d-faces (on spherical grids v^1 = v_r / r,
    v^2 = v_theta / r, v^3 = v_phi / (r sin theta))."""
    vf = [_c(v) for v in vf]
    if len(vf) != p.ndim:
        raise ValueError("one face-velocity array per active direction")
    for d, v in enumerate(vf):
        if v.shape != (p.ndim,) + face_shape(p, d):
            raise ValueError(f"face velocity {d}: shape {v.shape}, expected {(p.ndim,) + face_shape(p, d)}")
    return vf


def run_v(p: Problem, E, F, kappa, sigma, B, vf, nu_edge, dt, nsteps=1, inflow=None, want_dEm=False):
    """nsteps full steps with the velocity terms (Steps 1 to 4). Returns (E, [F_k], diag[, dEm])."""
    d = p.desc()
    E = _c(E)
    F = [_c(f) for f in F]
    kappa, sigma, B = _c(kappa), _c(sigma), _c(B)
    inflow = None if inflow is None else _c(inflow)
    vf = _vel(p, vf)
    nu = _c(nu_edge)
    if nu.shape != (p.G + 1,):
        raise ValueError("nu_edge needs G + 1 entries")
    Eo = np.empty_like(E)
    Fo = [np.empty_like(E) for _ in range(p.ndim)]
    dEm = np.empty(p.nzones) if want_dEm else None
    diag = OrcDiag()
    rc = lib().orc_run_v(ctypes.byref(d), _ptr(E), _ptrs(F), _ptr(kappa), _ptr(sigma), _ptr(B), _ptr(inflow),
                         _ptrs(vf), _ptr(nu), dt, nsteps, _ptr(Eo), _ptrs(Fo), _ptr(dEm), ctypes.byref(diag))
    if rc != 0:
        raise ValueError("velocity step: Euler integrator and finite increasing group edges required")
    dg = dict(energy_total=diag.energy_total, max_f=diag.max_f, n_unrealizable=diag.n_unrealizable,
              n_nonpositive=diag.n_nonpositive)
    if want_dEm:
        return Eo, Fo, dg, dEm
    return Eo, Fo, dg


def explicit_v(p: Problem, E, F, kappa, sigma, vf, dt, inflow=None):
    """Step 1 with the velocity terms alone. Returns (E, [F_k])."""
    d = p.desc()
    E = _c(E)
    F = [_c(f) for f in F]
    kappa, sigma = _c(kappa), _c(sigma)
    inflow = None if inflow is None else _c(inflow)
    vf = _vel(p, vf)
    Eo = np.empty_like(E)
    Fo = [np.empty_like(E) for _ in range(p.ndim)]
    lib().orc_explicit_v(ctypes.byref(d), _ptr(E), _ptrs(F), _ptr(kappa), _ptr(sigma), _ptr(inflow), _ptrs(vf), dt,
                         _ptr(Eo), _ptrs(Fo))
    return Eo, Fo


def freq_adv(p: Problem, E, F, vf, nu_edge, dt):
    """Step 2 alone: (E, [F_k]) after the frequency advection of (E, F)."""
    d = p.desc()
    E = _c(E)
    F = [_c(f) for f in F]
    vf = _vel(p, vf)
    nu = _c(nu_edge)
    Eo = np.empty_like(E)
    Fo = [np.empty_like(E) for _ in range(p.ndim)]
    rc = lib().orc_freq_adv(ctypes.byref(d), _ptr(E), _ptrs(F), _ptrs(vf), _ptr(nu), dt, _ptr(Eo), _ptrs(Fo))
    if rc != 0:
        raise ValueError("frequency advection: finite increasing group edges required")
    return Eo, Fo


def closure3(E, Fphys, c=1.0, eddington=False):
    """Physical-component third moment Q^ [k][j][i] (3x3x3) of one state (Cartesian)."""
    p = Problem(ndim=3, n=(1, 1, 1), G=1, c=c, closure=1 if eddington else 0)
    desc = p.desc()
    F = np.ascontiguousarray(np.asarray(Fphys, dtype=np.float64).reshape(3))
    Q = np.empty(27)
    lib().orc_closure3(ctypes.byref(desc), float(E), _ptr(F), _ptr(Q))
    return Q.reshape(3, 3, 3)


def vel_grad(p: Problem, vf):
    """<v^i_{;j}> [zones..., 3, 3] and <v^k> [zones..., 3] (coordinate components)."""
    d = p.desc()
    vf = _vel(p, vf)
    Vg = np.empty(p.nzones * 9)
    vb = np.empty(p.nzones * 3)
    lib().orc_vel_grad(ctypes.byref(d), _ptrs(vf), _ptr(Vg), _ptr(vb))
    return Vg.reshape(p.shape[:3] + (3, 3)), vb.reshape(p.shape[:3] + (3,))


def lab_frame(p: Problem, E, F, vf):
    """Group-summed lab-frame energy [zones...] and physical flux [ndim][zones...] to O(v/c)."""
    d = p.desc()
    E = _c(E)
    F = [_c(f) for f in F]
    vf = _vel(p, vf)
    El = np.empty(p.nzones)
    Fl = [np.empty(p.nzones) for _ in range(p.ndim)]
    lib().orc_lab_frame(ctypes.byref(d), _ptr(E), _ptrs(F), _ptrs(vf), _ptr(El), _ptrs(Fl))
    return El.reshape(p.shape[:3]), [f.reshape(p.shape[:3]) for f in Fl]

