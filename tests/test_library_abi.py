"""The C-ABI library loads on a machine without a GPU, exports every function that
include/fornax_m1.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1806_07390_amd", "libfornax_m1.so")
HEADER = os.path.join(ROOT, "include", "fornax_m1.h")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fornax_m1_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_the_same_entry_points():
    from paper_1806_07390_amd import m1
    assert sorted(m1.EXPORTED) == declared_functions()


def test_argument_checks_need_no_device():
    from paper_1806_07390_amd import m1
    lib = m1._lib
    h = ctypes.c_void_p()
    bad = m1.Desc()
    bad.ndim = 4
    assert lib.fornax_m1_create(ctypes.byref(bad), ctypes.byref(h)) == m1.FORNAX_EINVAL
    d = m1.Desc()
    d.ndim, d.n[:], d.ngroups, d.coord = 2, [8, 8, 1], 4, m1.CARTESIAN
    d.lo[:], d.hi[:] = [0, 0, 0], [1, 1, 1]
    d.bc_lo[:], d.bc_hi[:] = [m1.BC_PERIODIC, m1.BC_OUTFLOW, 0], [m1.BC_OUTFLOW, m1.BC_OUTFLOW, 0]
    d.c = 1.0
    # periodic on one side only
    assert lib.fornax_m1_create(ctypes.byref(d), ctypes.byref(h)) == m1.FORNAX_EINVAL
    d.bc_lo[0] = m1.BC_AXIS       # axis on a Cartesian grid
    assert lib.fornax_m1_create(ctypes.byref(d), ctypes.byref(h)) == m1.FORNAX_EINVAL
    d.bc_lo[0] = m1.BC_OUTFLOW
    d.n[2] = 2                    # inactive direction with more than one zone
    assert lib.fornax_m1_create(ctypes.byref(d), ctypes.byref(h)) == m1.FORNAX_EINVAL
    d.n[2] = 1
    d.c = -1.0
    assert lib.fornax_m1_create(ctypes.byref(d), ctypes.byref(h)) == m1.FORNAX_EINVAL
    d.c = 1.0
    d.wavespeed = 7               # no such wavespeed option
    assert lib.fornax_m1_create(ctypes.byref(d), ctypes.byref(h)) == m1.FORNAX_EINVAL
    d.wavespeed = m1.WAVESPEED_LIGHT
    d.limiter = 4                 # no such limiter
    assert lib.fornax_m1_create(ctypes.byref(d), ctypes.byref(h)) == m1.FORNAX_EINVAL
    d.limiter = m1.LIMITER_MINMOD
    d.integrator = 5              # no such integrator
    assert lib.fornax_m1_create(ctypes.byref(d), ctypes.byref(h)) == m1.FORNAX_EINVAL
    d.integrator = m1.EULER
    # empty grids and groups
    d.n[0] = 0
    assert lib.fornax_m1_create(ctypes.byref(d), ctypes.byref(h)) == m1.FORNAX_EINVAL
    d.n[0] = 8
    d.ngroups = 0
    assert lib.fornax_m1_create(ctypes.byref(d), ctypes.byref(h)) == m1.FORNAX_EINVAL
    # the largest grid the 32-bit zone-group indices allow: (1 + ndim) components of
    # nzones x G entries must stay below 2^31
    d.ngroups = 16
    d.n[:] = [8192, 8192, 1]      # 2^26 zones x 16 groups x 3 components > 2^31
    assert lib.fornax_m1_create(ctypes.byref(d), ctypes.byref(h)) == m1.FORNAX_EUNSUPPORTED
    d.n[:] = [8, 8, 1]
    assert lib.fornax_m1_max_dt(None, 0.4) == m1.FORNAX_EINVAL
    assert lib.fornax_m1_step(None, None, None, None, None, 0.1, None, None) == m1.FORNAX_EINVAL
    assert lib.fornax_m1_copy_probe(None, None, 16, None) == m1.FORNAX_EINVAL
    assert lib.fornax_m1_strerror(m1.FORNAX_ECFL).decode().startswith("time step")
