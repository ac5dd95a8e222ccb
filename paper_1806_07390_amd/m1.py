"""Python binding of libfornax_m1 (ctypes over the C interface in include/fornax_m1.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch provides device memory (tensors) and the current HIP stream.  Importing this module
raises if the library has not been built (``python -m paper_1806_07390_amd.build``).

Arrays are CUDA (HIP) tensors of shape ``(n2, n1, n0, G)`` (group innermost), dtype
float64 for FP64 contexts and float32 for MIXED contexts; flux components are covariant.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfornax_m1.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1806_07390_amd.build` "
                      "(there is no fallback implementation)")

_lib = ctypes.CDLL(LIB_PATH)

FORNAX_OK, FORNAX_EINVAL, FORNAX_ECFL, FORNAX_EDEVICE, FORNAX_ENOMEM, FORNAX_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FORNAX_ESCRATCH = -6
NOALLOC_SCRATCH_BYTES = 16 << 20     # FORNAX_M1_NOALLOC_SCRATCH_BYTES
CARTESIAN, SPHERICAL_LOGR = 0, 1
BC_OUTFLOW, BC_PERIODIC, BC_REFLECT, BC_INFLOW, BC_AXIS = 0, 1, 2, 3, 4
FP64, MIXED = 0, 1
LIMITER_MINMOD, LIMITER_MC, LIMITER_NONE, LIMITER_PPM = 0, 1, 2, 3
CLOSURE_M1, CLOSURE_EDDINGTON = 0, 1
EULER, SSPRK2 = 0, 1
WAVESPEED_LIGHT, WAVESPEED_M1 = 0, 1

EXPORTED = ["fornax_m1_create", "fornax_m1_destroy", "fornax_m1_max_dt", "fornax_m1_step", "fornax_m1_flux",
            "fornax_m1_source", "fornax_m1_adjoint", "fornax_m1_copy_probe", "fornax_m1_strerror",
            "fornax_m1_transport", "fornax_m1_set_matter_model", "fornax_m1_matter_coeffs",
            "fornax_m1_matter_source", "fornax_m1_step_noalloc", "fornax_m1_set_group_edges",
            "fornax_m1_step_velocity", "fornax_m1_lab_frame"]


class Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("ngroups", ctypes.c_int32),
        ("coord", ctypes.c_int32),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc_lo", ctypes.c_int32 * 3),
        ("bc_hi", ctypes.c_int32 * 3),
        ("limiter", ctypes.c_int32),
        ("closure", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("c", ctypes.c_double),
        ("f_fp64", ctypes.c_double),
        ("integrator", ctypes.c_int32),
        ("wavespeed", ctypes.c_int32),
    ]


class State(ctypes.Structure):
    _fields_ = [("E", ctypes.c_void_p), ("F", ctypes.c_void_p * 3)]


class Coeffs(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_void_p), ("sigma", ctypes.c_void_p), ("B", ctypes.c_void_p)]


class MatterModel(ctypes.Structure):
    _fields_ = [("ngroups", ctypes.c_int32), ("nu_edge", ctypes.c_void_p), ("nu_c", ctypes.c_void_p),
                ("kg", ctypes.c_void_p), ("a_rad", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_newton", ctypes.c_int32)]


class Matter(ctypes.Structure):
    _fields_ = [("cv", ctypes.c_void_p), ("kappa0", ctypes.c_void_p), ("T", ctypes.c_void_p)]


class Velocity(ctypes.Structure):
    _fields_ = [("v", ctypes.c_void_p * 3)]


class Diag(ctypes.Structure):
    _fields_ = [("energy_total", ctypes.c_void_p), ("dE_matter", ctypes.c_void_p), ("max_f", ctypes.c_void_p),
                ("n_unrealizable", ctypes.c_void_p), ("n_nonpositive", ctypes.c_void_p)]


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_lib.fornax_m1_create.argtypes = [_P(Desc), _P(_vp)]
_lib.fornax_m1_create.restype = ctypes.c_int
_lib.fornax_m1_destroy.argtypes = [_vp]
_lib.fornax_m1_max_dt.argtypes = [_vp, ctypes.c_double]
_lib.fornax_m1_max_dt.restype = ctypes.c_double
_lib.fornax_m1_step.argtypes = [_vp, _P(State), _P(State), _P(Coeffs), _vp, ctypes.c_double, _P(Diag), _vp]
_lib.fornax_m1_step_noalloc.argtypes = [_vp, _P(State), _P(State), _P(Coeffs), _vp, ctypes.c_double, _P(Diag),
                                        _vp]
_lib.fornax_m1_flux.argtypes = [_vp, _P(State), _P(Coeffs), _vp, _vp * 3, _vp]
_lib.fornax_m1_source.argtypes = [_vp, _P(State), _P(Coeffs), ctypes.c_double, _vp, _vp]
_lib.fornax_m1_adjoint.argtypes = [_vp, _P(State), _P(State), _P(Coeffs), _vp, ctypes.c_double, _P(State), _P(State),
                                    _vp, _vp]
_lib.fornax_m1_copy_probe.argtypes = [_vp, _vp, ctypes.c_int64, _vp]
_lib.fornax_m1_transport.argtypes = [_vp, _P(State), _P(State), _P(Coeffs), _vp, ctypes.c_double, _vp]
_lib.fornax_m1_set_matter_model.argtypes = [_vp, _P(MatterModel)]
_lib.fornax_m1_matter_coeffs.argtypes = [_vp, _P(Matter), _vp, _vp, _vp]
_lib.fornax_m1_matter_source.argtypes = [_vp, _P(State), _vp, _P(Matter), ctypes.c_double, _vp, _vp, _vp]
_lib.fornax_m1_set_group_edges.argtypes = [_vp, _vp]
_lib.fornax_m1_step_velocity.argtypes = [_vp, _P(State), _P(State), _P(Coeffs), _vp, _P(Velocity), ctypes.c_double,
                                         _P(Diag), _vp]
_lib.fornax_m1_lab_frame.argtypes = [_vp, _P(State), _P(Velocity), _vp, _vp * 3, _vp]
_lib.fornax_m1_strerror.argtypes = [ctypes.c_int]
_lib.fornax_m1_strerror.restype = ctypes.c_char_p


class FornaxError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {_lib.fornax_m1_strerror(code).decode()} (code {code})")
        self.code = code


def _check(code, what):
    if code != FORNAX_OK:
        raise FornaxError(code, what)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class Config:
    ndim: int
    n: tuple
    G: int
    coord: int = CARTESIAN
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    bc_lo: tuple = (BC_OUTFLOW,) * 3
    bc_hi: tuple = (BC_OUTFLOW,) * 3
    limiter: int = LIMITER_MINMOD
    closure: int = CLOSURE_M1
    precision: int = FP64
    c: float = 1.0
    f_fp64: float = 0.9
    integrator: int = EULER
    wavespeed: int = WAVESPEED_LIGHT

    @classmethod
    def from_workload(cls, w, precision=FP64, **kw):
        return cls(ndim=w.ndim, n=tuple(w.n), G=w.G, coord=w.coord, lo=tuple(w.lo), hi=tuple(w.hi),
                   bc_lo=tuple(w.bc_lo), bc_hi=tuple(w.bc_hi), c=w.c, precision=precision, **kw)


class Context:
    """A problem description bound to the current HIP device (owns the geometry tables)."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        d = Desc()
        d.ndim = cfg.ndim
        n = list(cfg.n) + [1] * (3 - len(cfg.n))
        d.n[:] = n
        d.ngroups = cfg.G
        d.coord = cfg.coord
        d.lo[:] = list(cfg.lo)
        d.hi[:] = list(cfg.hi)
        d.bc_lo[:] = list(cfg.bc_lo)
        d.bc_hi[:] = list(cfg.bc_hi)
        d.limiter = cfg.limiter
        d.closure = cfg.closure
        d.precision = cfg.precision
        d.c = cfg.c
        d.f_fp64 = cfg.f_fp64
        d.integrator = cfg.integrator
        d.wavespeed = cfg.wavespeed
        self.desc = d
        self.shape = (n[2], n[1], n[0], cfg.G)
        self.nzones = n[0] * n[1] * n[2]
        self.dtype = torch.float64 if cfg.precision == FP64 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        _check(_lib.fornax_m1_create(ctypes.byref(d), ctypes.byref(h)), "fornax_m1_create")
        self._h = h

    def close(self):
        self._bwd_cache = None
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.fornax_m1_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------------------------
    def _check_arr(self, t, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.dtype != self.dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, expected {self.dtype}")
        if tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.shape}, got {tuple(t.shape)}")

    def _state(self, E, F, name="state"):
        self._check_arr(E, f"{name}.E")
        if len(F) != self.cfg.ndim:
            raise ValueError(f"{name}.F needs {self.cfg.ndim} components")
        s = State()
        s.E = E.data_ptr()
        for k, f in enumerate(F):
            self._check_arr(f, f"{name}.F[{k}]")
            s.F[k] = f.data_ptr()
        return s

    def _point(self, s, E, F, name="state"):
        """Point the existing State structure s (held by a bound call) at (E, [F])."""
        t = self._state(E, F, name)
        s.E = t.E
        for k in range(3):
            s.F[k] = t.F[k]

    def _coeffs(self, kappa, sigma, B):
        for t, nm in ((kappa, "kappa"), (sigma, "sigma"), (B, "B")):
            self._check_arr(t, nm)
        c = Coeffs()
        c.kappa, c.sigma, c.B = kappa.data_ptr(), sigma.data_ptr(), B.data_ptr()
        return c

    def _inflow(self, inflow):
        if inflow is None:
            return None
        if inflow.dtype != torch.float64 or inflow.device.type != "cuda" or not inflow.is_contiguous() \
                or tuple(inflow.shape) != (self.cfg.G, 1 + self.cfg.ndim):
            raise ValueError("inflow must be a contiguous float64 CUDA tensor [G][1+ndim]")
        return ctypes.c_void_p(inflow.data_ptr())

    def empty_state(self):
        E = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        return E, [torch.empty_like(E) for _ in range(self.cfg.ndim)]

    # -- entry points ------------------------------------------------------------------------
    def max_dt(self, cfl: float) -> float:
        v = _lib.fornax_m1_max_dt(self._h, cfl)
        if v < 0:
            raise FornaxError(int(v), "fornax_m1_max_dt")
        return v

    def step(self, E, F, kappa, sigma, B, dt, out=None, inflow=None, diag=None, stream=None, noalloc=False):
        """One step; returns (E_out, [F_out]).  diag: dict of preallocated tensors (optional).
        noalloc: through fornax_m1_step_noalloc (scratch in the library's static array)."""
        sin = self._state(E, F, "in")
        if out is None:
            out = self.empty_state()
        sout = self._state(out[0], out[1], "out")
        cf = self._coeffs(kappa, sigma, B)
        dg = None
        if diag is not None:
            dg = Diag()
            dg.energy_total = _ptr(diag.get("energy_total"))
            dg.dE_matter = _ptr(diag.get("dE_matter"))
            dg.max_f = _ptr(diag.get("max_f"))
            dg.n_unrealizable = _ptr(diag.get("n_unrealizable"))
            dg.n_nonpositive = _ptr(diag.get("n_nonpositive"))
        fn, name = ((_lib.fornax_m1_step_noalloc, "fornax_m1_step_noalloc") if noalloc
                    else (_lib.fornax_m1_step, "fornax_m1_step"))
        _check(fn(self._h, ctypes.byref(sin), ctypes.byref(sout), ctypes.byref(cf), self._inflow(inflow), dt,
                  ctypes.byref(dg) if dg is not None else None, _stream(stream)), name)
        return out

    def new_diag(self):
        dev = self.device
        return dict(energy_total=torch.zeros(1, dtype=torch.float64, device=dev),
                    dE_matter=torch.zeros(self.nzones, dtype=torch.float64, device=dev),
                    max_f=torch.zeros(1, dtype=torch.float64, device=dev),
                    n_unrealizable=torch.zeros(1, dtype=torch.int32, device=dev),
                    n_nonpositive=torch.zeros(1, dtype=torch.int32, device=dev))

    def flux(self, E, F, kappa, sigma, B, inflow=None, stream=None):
        """Face fluxes per direction: list of tensors [faces_d..., G, 1+ndim]."""
        sin = self._state(E, F, "in")
        cf = self._coeffs(kappa, sigma, B)
        outs = []
        arr = (ctypes.c_void_p * 3)()
        for d in range(self.cfg.ndim):
            s = list(self.shape[:3])
            s[2 - d] += 1
            t = torch.empty(tuple(s) + (self.cfg.G, 1 + self.cfg.ndim), dtype=self.dtype, device=self.device)
            outs.append(t)
            arr[d] = t.data_ptr()
        _check(_lib.fornax_m1_flux(self._h, ctypes.byref(sin), ctypes.byref(cf), self._inflow(inflow), arr,
                                   _stream(stream)), "fornax_m1_flux")
        return outs

    def source(self, E, F, kappa, sigma, B, dt, dE_matter=None, stream=None):
        """Implicit interaction update in place."""
        s = self._state(E, F, "inout")
        cf = self._coeffs(kappa, sigma, B)
        _check(_lib.fornax_m1_source(self._h, ctypes.byref(s), ctypes.byref(cf), dt, _ptr(dE_matter),
                                     _stream(stream)), "fornax_m1_source")

    def transport(self, E, F, kappa, sigma, dt, out=None, inflow=None, stream=None):
        """The explicit transport alone: returns (E^-, [F^-]) = U^n + dt L(U^n)."""
        sin = self._state(E, F, "in")
        if out is None:
            out = self.empty_state()
        sout = self._state(out[0], out[1], "out")
        for t, nm in ((kappa, "kappa"), (sigma, "sigma")):
            self._check_arr(t, nm)
        cf = Coeffs()
        cf.kappa, cf.sigma, cf.B = kappa.data_ptr(), sigma.data_ptr(), None
        _check(_lib.fornax_m1_transport(self._h, ctypes.byref(sin), ctypes.byref(sout), ctypes.byref(cf),
                                        self._inflow(inflow), dt, _stream(stream)), "fornax_m1_transport")
        return out

    # -- velocity-dependent terms -------------------------------------------------------------
    def face_shape(self, d):
        """Shape (n2, n1, n0) of the d-faces (the d extent n_d + 1)."""
        s = list(self.shape[:3])
        s[2 - d] += 1
        return tuple(s)

    def set_group_edges(self, nu_edge):
        """Group edges in frequency for the velocity step (host array [G+1], copied)."""
        import numpy as np
        ne = np.ascontiguousarray(nu_edge, dtype=np.float64)
        if ne.shape != (self.cfg.G + 1,):
            raise ValueError(f"nu_edge needs {self.cfg.G + 1} entries")
        _check(_lib.fornax_m1_set_group_edges(self._h, ne.ctypes.data), "fornax_m1_set_group_edges")

    def _velocity(self, vf):
        if len(vf) != self.cfg.ndim:
            raise ValueError(f"one face-velocity tensor per active direction ({self.cfg.ndim})")
        vel = Velocity()
        for d, t in enumerate(vf):
            shp = (self.cfg.ndim,) + self.face_shape(d)
            if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != self.dtype \
                    or tuple(t.shape) != shp or not t.is_contiguous():
                raise ValueError(f"face velocity {d} must be a contiguous {self.dtype} CUDA tensor {shp}")
            vel.v[d] = t.data_ptr()
        return vel

    def step_velocity(self, E, F, kappa, sigma, B, vf, dt, out=None, inflow=None, diag=None, stream=None):
        """One step with the velocity terms (fornax_m1_step_velocity); vf: ndim tensors
        [ndim, *face_shape(d)] of coordinate velocity components on the d-faces."""
        sin = self._state(E, F, "in")
        if out is None:
            out = self.empty_state()
        sout = self._state(out[0], out[1], "out")
        cf = self._coeffs(kappa, sigma, B)
        vel = self._velocity(vf)
        dg = None
        if diag is not None:
            dg = Diag()
            dg.energy_total = _ptr(diag.get("energy_total"))
            dg.dE_matter = _ptr(diag.get("dE_matter"))
            dg.max_f = _ptr(diag.get("max_f"))
            dg.n_unrealizable = _ptr(diag.get("n_unrealizable"))
            dg.n_nonpositive = _ptr(diag.get("n_nonpositive"))
        _check(_lib.fornax_m1_step_velocity(self._h, ctypes.byref(sin), ctypes.byref(sout), ctypes.byref(cf),
                                            self._inflow(inflow), ctypes.byref(vel), dt,
                                            ctypes.byref(dg) if dg is not None else None, _stream(stream)),
               "fornax_m1_step_velocity")
        return out

    def lab_frame(self, E, F, vf, stream=None):
        """Group-summed lab-frame energy [zones] and physical flux [ndim][zones] (float64)."""
        sin = self._state(E, F, "in")
        vel = self._velocity(vf)
        El = torch.empty(self.shape[:3], dtype=torch.float64, device=self.device)
        Fl = [torch.empty_like(El) for _ in range(self.cfg.ndim)]
        arr = (ctypes.c_void_p * 3)()
        for d, t in enumerate(Fl):
            arr[d] = t.data_ptr()
        _check(_lib.fornax_m1_lab_frame(self._h, ctypes.byref(sin), ctypes.byref(vel), El.data_ptr(), arr,
                                        _stream(stream)), "fornax_m1_lab_frame")
        return El, Fl

    # -- radiation-matter energy exchange ------------------------------------------------------
    def set_matter_model(self, nu_edge, nu_c, kg, a_rad=1.0, tol=1e-6, max_newton=30):
        """Group tables of the matter model (host arrays; copied into the context)."""
        import numpy as np
        ne = np.ascontiguousarray(nu_edge, dtype=np.float64)
        nc = np.ascontiguousarray(nu_c, dtype=np.float64)
        k = np.ascontiguousarray(kg, dtype=np.float64)
        mm = MatterModel()
        mm.ngroups = len(nc)
        mm.nu_edge, mm.nu_c, mm.kg = ne.ctypes.data, nc.ctypes.data, k.ctypes.data
        mm.a_rad, mm.tol, mm.max_newton = a_rad, tol, max_newton
        _check(_lib.fornax_m1_set_matter_model(self._h, ctypes.byref(mm)), "fornax_m1_set_matter_model")

    def _matter(self, cv, kappa0, T):
        zshape = self.shape[:3]
        for t, nm in ((cv, "cv"), (kappa0, "kappa0"), (T, "T")):
            if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64 \
                    or tuple(t.shape) != zshape or not t.is_contiguous():
                raise ValueError(f"{nm} must be a contiguous float64 CUDA tensor of shape {zshape}")
        m = Matter()
        m.cv, m.kappa0, m.T = cv.data_ptr(), kappa0.data_ptr(), T.data_ptr()
        return m

    def matter_coeffs(self, cv, kappa0, T, stream=None):
        """kappa_g(T), B_g(T) per zone-group (tensors of the context's type)."""
        m = self._matter(cv, kappa0, T)
        kap = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        B = torch.empty_like(kap)
        _check(_lib.fornax_m1_matter_coeffs(self._h, ctypes.byref(m), ctypes.c_void_p(kap.data_ptr()),
                                            ctypes.c_void_p(B.data_ptr()), _stream(stream)), "fornax_m1_matter_coeffs")
        return kap, B

    def matter_source(self, E, F, sigma, cv, kappa0, T, dt, dE_matter=None, iters=None, stream=None):
        """Interaction update with the matter temperature solved for, in place on E, F and T."""
        s = self._state(E, F, "inout")
        self._check_arr(sigma, "sigma")
        m = self._matter(cv, kappa0, T)
        _check(_lib.fornax_m1_matter_source(self._h, ctypes.byref(s), ctypes.c_void_p(sigma.data_ptr()),
                                            ctypes.byref(m), dt, _ptr(dE_matter), _ptr(iters), _stream(stream)),
               "fornax_m1_matter_source")

    def matter_step(self, E, F, sigma, cv, kappa0, T, dt, out=None, inflow=None, dE_matter=None, iters=None,
                    stream=None):
        """One step with the matter coupled (Algorithmic Steps 1, 3 and 4, static medium): the
        opacities at T^n, the explicit transport, then the interaction update with the outer
        solve for T^{n+1} (T updated in place). Returns (E^{n+1}, [F^{n+1}])."""
        kap, _ = self.matter_coeffs(cv, kappa0, T, stream=stream)
        out = self.transport(E, F, kap, sigma, dt, out=out, inflow=inflow, stream=stream)
        self.matter_source(out[0], out[1], sigma, cv, kappa0, T, dt, dE_matter=dE_matter, iters=iters, stream=stream)
        return out

    def adjoint(self, E, F, kappa, sigma, B, dt, lamE, lamF, out=None, dkappa=None, inflow=None, stream=None,
                U1=None):
        """lam_n = J^T lam_{n+1}; dkappa += (dU^{n+1}/dkappa)^T lam_{n+1}. Returns (lamE_n, [lamF_n], dkappa).
        U1: optional (E, [F]) of the step's result from (E, F); when None the step is run first
        (fornax_m1_step into a new state), since the library requires it."""
        if U1 is None:
            U1 = self.step(E, F, kappa, sigma, B, dt, inflow=inflow, stream=stream)
        su = self._state(E, F, "Un")
        s1 = self._state(U1[0], U1[1], "Unp1")
        sl = self._state(lamE, lamF, "lam_np1")
        if out is None:
            out = self.empty_state()
        so = self._state(out[0], out[1], "lam_n")
        if dkappa is None:
            dkappa = torch.zeros(self.shape, dtype=self.dtype, device=self.device)
        self._check_arr(dkappa, "dkappa")
        cf = self._coeffs(kappa, sigma, B)
        _check(_lib.fornax_m1_adjoint(self._h, ctypes.byref(su), ctypes.byref(s1),
                                      ctypes.byref(cf), self._inflow(inflow), dt,
                                      ctypes.byref(sl), ctypes.byref(so), ctypes.c_void_p(dkappa.data_ptr()),
                                      _stream(stream)), "fornax_m1_adjoint")
        return out[0], out[1], dkappa

    def stepper(self, A, Bst, kappa, sigma, B, dt, inflow=None, diag=None, stream=None):
        """Pre-bound ping-pong stepping between two states A = (E, [F]) and Bst: each call of
        the returned function advances one step (A -> Bst, then Bst -> A, ...) with the C
        arguments built once.  Returns (step_fn, current_state_fn)."""
        sa = self._state(A[0], A[1], "A")
        sb = self._state(Bst[0], Bst[1], "B")
        cf = self._coeffs(kappa, sigma, B)
        dg = None
        if diag is not None:
            dg = Diag()
            dg.energy_total = _ptr(diag.get("energy_total"))
            dg.dE_matter = _ptr(diag.get("dE_matter"))
            dg.max_f = _ptr(diag.get("max_f"))
            dg.n_unrealizable = _ptr(diag.get("n_unrealizable"))
            dg.n_nonpositive = _ptr(diag.get("n_nonpositive"))
        infl = self._inflow(inflow)
        st = _stream(stream)
        pa, pb, pc = ctypes.byref(sa), ctypes.byref(sb), ctypes.byref(cf)
        pd = ctypes.byref(dg) if dg is not None else None
        h = self._h
        fn = _lib.fornax_m1_step
        parity = [0]

        def step():
            if parity[0] == 0:
                rc = fn(h, pa, pb, pc, infl, dt, pd, st)
            else:
                rc = fn(h, pb, pa, pc, infl, dt, pd, st)
            if rc != FORNAX_OK:
                raise FornaxError(rc, "fornax_m1_step")
            parity[0] ^= 1

        def current():
            return A if parity[0] == 0 else Bst

        # keep the structures alive with the closure
        step._keep = (sa, sb, cf, dg)
        return step, current

    def bound_step(self, src, dst, kappa, sigma, B, dt, inflow=None, stream=None):
        """Pre-bound fornax_m1_step src -> dst (arguments built once); returns a function."""
        sa = self._state(src[0], src[1], "in")
        sb = self._state(dst[0], dst[1], "out")
        cf = self._coeffs(kappa, sigma, B)
        args = (self._h, ctypes.byref(sa), ctypes.byref(sb), ctypes.byref(cf), self._inflow(inflow), dt, None,
                _stream(stream))
        fn = _lib.fornax_m1_step

        def call():
            rc = fn(*args)
            if rc != FORNAX_OK:
                raise FornaxError(rc, "fornax_m1_step")

        call._keep = (sa, sb, cf)
        call.src = sa      # the input's structure, which _point may re-aim
        return call

    def adjointer(self, U, kappa, sigma, B, dt, lam_in, lam_out, dkappa, inflow=None, stream=None, U1=None):
        """Pre-bound fornax_m1_adjoint call (arguments built once): returns a function that
        computes lam_out = J^T lam_in and accumulates into dkappa for the state U (U1: the
        step's result from U, when the caller holds it; when None each call first runs the step
        into a state held by the returned function)."""
        pre = None
        if U1 is None:
            U1 = self.empty_state()
            pre = self.bound_step((U[0], U[1]), U1, kappa, sigma, B, dt, inflow=inflow, stream=stream)
        su = self._state(U[0], U[1], "Un")
        s1 = self._state(U1[0], U1[1], "Unp1")
        sl = self._state(lam_in[0], lam_in[1], "lam_np1")
        so = self._state(lam_out[0], lam_out[1], "lam_n")
        self._check_arr(dkappa, "dkappa")
        cf = self._coeffs(kappa, sigma, B)
        infl = self._inflow(inflow)
        st = _stream(stream)
        args = (self._h, ctypes.byref(su), ctypes.byref(s1), ctypes.byref(cf), infl, dt,
                ctypes.byref(sl), ctypes.byref(so), ctypes.c_void_p(dkappa.data_ptr()), st)
        fn = _lib.fornax_m1_adjoint

        def call():
            if pre is not None:
                pre()
            rc = fn(*args)
            if rc != FORNAX_OK:
                raise FornaxError(rc, "fornax_m1_adjoint")

        call._keep = (su, s1, sl, so, cf, U1)
        call.Un, call.Unp1 = su, s1      # the structures _point may re-aim
        return call

    def run(self, E, F, kappa, sigma, B, dt, nsteps, inflow=None, diag=None):
        """nsteps steps with ping-pong buffers; returns (E, [F]) (new tensors)."""
        a = (E.clone(), [f.clone() for f in F])
        b = self.empty_state()
        for s in range(nsteps):
            self.step(a[0], a[1], kappa, sigma, B, dt, out=b, inflow=inflow,
                      diag=diag if s == nsteps - 1 else None)
            a, b = b, a
        return a


def copy_probe(dst: torch.Tensor, src: torch.Tensor, stream=None):
    nbytes = src.numel() * src.element_size()
    _check(_lib.fornax_m1_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                                     _stream(stream)), "fornax_m1_copy_probe")


class M1Steps(torch.autograd.Function):
    """N steps of the M1 update as a differentiable function of the initial state and of the
    absorption opacity: (E_N, F_N) = M1Steps.apply(ctx, dt, nsteps, ckpt_every, inflow,
    kappa, sigma, B, E0, *F0).

    Forward: the library's fused step, keeping a copy of the state every `ckpt_every` steps.
    Backward: for each checkpoint segment in reverse, recompute the segment's states from its
    checkpoint and apply fornax_m1_adjoint step by step, accumulating dL/dkappa.  Gradients
    with respect to sigma, B and dt are not provided (None)."""

    @staticmethod
    def forward(fctx, ctx, dt, nsteps, ckpt_every, inflow, kappa, sigma, B, E0, *F0):
        if ckpt_every < 1:
            raise ValueError("ckpt_every must be >= 1")
        a = (E0.detach().clone(), [f.detach().clone() for f in F0])
        b = ctx.empty_state()
        ckpts = []
        step, current = ctx.stepper(a, b, kappa.detach(), sigma.detach(), B.detach(), dt, inflow=inflow)
        for s in range(nsteps):
            if s % ckpt_every == 0:
                cur = current()
                ckpts.append((s, cur[0].clone(), [f.clone() for f in cur[1]]))
            step()
        out = current()
        res = (out[0].clone(),) + tuple(f.clone() for f in out[1])
        # the final state closes the last segment of the replay
        fctx.m1 = (ctx, dt, nsteps, ckpt_every, inflow, ckpts, (out[0].clone(), [f.clone() for f in out[1]]))
        fctx.save_for_backward(kappa, sigma, B)
        return res

    @staticmethod
    def backward(fctx, gE, *gF):
        ctx, dt, nsteps, ckpt_every, inflow, ckpts, final = fctx.m1
        kappa, sigma, B = fctx.saved_tensors
        kappa, sigma, B = kappa.detach(), sigma.detach(), B.detach()
        K = min(ckpt_every, nsteps)
        # The replay's buffers and bound C calls depend only on the context, the segment length
        # and the coefficient arrays: they are kept on the context and reused by later backward
        # passes (binding them costs far more host time than the GPU work of a small step).
        key = (dt, K, None if inflow is None else inflow.data_ptr(), kappa.data_ptr(), sigma.data_ptr(),
               B.data_ptr())
        cache = getattr(ctx, "_bwd_cache", None)
        if cache is None or cache[0] != key:
            # seg[i]: state i of the segment being replayed.  The segment's first state (its
            # checkpoint) and the state that closes it (the next checkpoint, or the final state)
            # are read where they are: the first replay step and adjoint step are pointed at the
            # checkpoint and the last adjoint step at the closing state, so that every adjoint
            # step gets both U^n and U^{n+1}, none recomputes the step, and nothing is copied.
            # seg[0] and seg[K] only hold the bindings' default targets.
            seg = [ctx.empty_state() for _ in range(K + 1)]
            lam = [ctx.empty_state(), ctx.empty_state()]
            dk = torch.empty(ctx.shape, dtype=ctx.dtype, device=ctx.device)
            # every C call of the replay bound once: K-1 steps, K adjoint steps per lambda parity
            steps = [ctx.bound_step(seg[i], seg[i + 1], kappa, sigma, B, dt, inflow=inflow) for i in range(K - 1)]
            adj = [[ctx.adjointer(seg[i], kappa, sigma, B, dt, lam[p], lam[1 - p], dk, inflow=inflow, U1=seg[i + 1])
                    for p in range(2)] for i in range(K)]
            # the coefficient tensors stay referenced while the bound calls hold their pointers
            cache = (key, seg, lam, dk, steps, adj, (kappa, sigma, B, inflow))
            ctx._bwd_cache = cache
        _, seg, lam, dk, steps, adj, _ = cache
        dk.zero_()
        for dst, g in ((lam[0][0], gE),) + tuple((lam[0][1][k], gF[k]) for k in range(len(gF))):
            if g is None:
                dst.zero_()
            else:
                dst.copy_(g)
        ends = [(c[1], c[2]) for c in ckpts[1:]] + [final]
        p = 0
        for j in reversed(range(len(ckpts))):
            s0, E, F = ckpts[j]
            n_in = min(s0 + ckpt_every, nsteps) - s0
            if n_in > 1:
                ctx._point(steps[0].src, E, F, "checkpoint")
            for q in range(2):
                ctx._point(adj[0][q].Un, E, F, "checkpoint")
                ctx._point(adj[n_in - 1][q].Unp1, ends[j][0], ends[j][1], "checkpoint")
            try:
                for i in range(n_in - 1):
                    steps[i]()
                for i in reversed(range(n_in)):
                    adj[i][p]()
                    p ^= 1
            finally:
                # a later (longer) segment reads U^{n+1} of this step from the replay buffers
                for q in range(2):
                    ctx._point(adj[n_in - 1][q].Unp1, seg[n_in][0], seg[n_in][1])
        fctx.m1 = None
        out = lam[p]
        # fresh tensors: the buffers belong to the context's cache
        return (None, None, None, None, None, dk.clone(), None, None, out[0].clone()) + tuple(f.clone() for f in out[1])


def run_differentiable(ctx, E0, F0, kappa, sigma, B, dt, nsteps, ckpt_every=8, inflow=None):
    """Differentiable N-step run (see M1Steps); returns (E_N, [F_N])."""
    out = M1Steps.apply(ctx, dt, nsteps, ckpt_every, inflow, kappa, sigma, B, E0, *F0)
    return out[0], list(out[1:])
