"""Helpers shared by the GPU parity tests: run a workload through the HIP library and through
the CPU oracle on the same seeded inputs, and compare (relative L1 norms)."""
import json
import os

import numpy as np
import torch

from oracle import m1_oracle as orc

# Tolerances (spec targets): FP64 path vs FP64 oracle after the full run; MIXED path
# (float storage and bulk arithmetic, double closure near f -> 1, double source) vs the FP64
# oracle per step and after many steps.
TOL_FP64 = 1e-12
TOL_MIXED_STEP = 1e-5
TOL_MIXED_RUN = 1e-4

# Element-wise comparison: |x - x_ref| <= tol (|x_ref| + floor) with floor = PW_FLOOR times the
# largest |E_ref| (c times it for the flux components).  The floor keeps zones many decades
# below the field's scale (the 1e-8 floor of the blob workloads, the 1e-6 B start of the
# sphere), whose values come out of sums of neighbour fluxes up to 1e8 times larger, from
# being judged by their own size; every zone within three decades of the peak is judged
# relative to itself.
PW_FLOOR = 1e-3
# element-wise gates: FP64 within 2e-12 (the worst zone of a run sits up to an order of
# magnitude above the rel-L1 norm, which the 1e-12 gate bounds), MIXED within 1e-3 (float
# storage rounds every zone by 6e-8 each step; the worst zone after 100 steps reaches 5e-4 in
# the flux components of the 3-D core workload)
TOL_PW_FP64 = 2e-12
TOL_PW_MIXED = 1e-3


def check_pointwise(e, fp64, what=""):
    """Assert the element-wise errors of a comparison against its precision's gate."""
    tol = TOL_PW_FP64 if fp64 else TOL_PW_MIXED
    assert e.pE <= tol and e.pF <= tol, (what, "element-wise", e.pE, e.pF, tol)


def problem_of(w, **kw):
    p = orc.Problem(ndim=w.ndim, n=w.n, G=w.G, coord=w.coord, lo=w.lo, hi=w.hi, bc_lo=w.bc_lo, bc_hi=w.bc_hi,
                    c=w.c)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


class Errs(tuple):
    """(rel-L1 of E, rel-L1 of F) with the element-wise errors as attributes .pE, .pF."""


def pointwise(E, F, Eref, Fref, c=1.0):
    """max over elements of |x - x_ref| / (|x_ref| + floor), for E and for the flux components
    (floor: PW_FLOOR max |E_ref|, times c for F)."""
    E = np.asarray(E, dtype=np.float64)
    Eref = np.asarray(Eref, dtype=np.float64)
    fl = PW_FLOOR * np.max(np.abs(Eref))
    pE = float(np.max(np.abs(E - Eref) / (np.abs(Eref) + fl))) if Eref.size else 0.0
    pF = 0.0
    for f, fr in zip(F, Fref):
        fr = np.asarray(fr, dtype=np.float64)
        if fr.size:
            pF = max(pF, float(np.max(np.abs(np.asarray(f, dtype=np.float64) - fr) / (np.abs(fr) + c * fl))))
    return pE, pF


def rel_l1(E, F, Eref, Fref, c=1.0):
    """rel-L1 of E, and of the flux components normalised by c sum |E_ref|; the element-wise
    errors (pointwise) ride along as .pE and .pF."""
    E = np.asarray(E, dtype=np.float64)
    Eref = np.asarray(Eref, dtype=np.float64)
    sE = np.sum(np.abs(Eref))
    eE = np.sum(np.abs(E - Eref)) / sE
    eF = max([np.sum(np.abs(np.asarray(f, dtype=np.float64) - fr)) / (c * sE) for f, fr in zip(F, Fref)] + [0.0])
    r = Errs((eE, eF))
    r.pE, r.pF = pointwise(E, F, Eref, Fref, c)
    _log(eE=float(eE), eF=float(eF), pE=r.pE, pF=r.pF)
    return r


def _log(**kw):
    """Append the errors of a comparison, with the running test's name, to the file named by
    PARITY_LOG (when set): the figures quoted for the parity cases."""
    path = os.environ.get("PARITY_LOG")
    if not path:
        return
    kw["test"] = os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0]
    with open(path, "a") as fh:
        fh.write(json.dumps(kw) + "\n")


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def gpu_run(ctx, w, dt, nsteps, diag=False):
    dtp = ctx.dtype
    E = to_dev(w.E, dtp)
    F = [to_dev(f, dtp) for f in w.F]
    k, s, B = (to_dev(x, dtp) for x in (w.kappa, w.sigma, w.B))
    inflow = None if w.inflow is None else to_dev(w.inflow, torch.float64)
    dg = ctx.new_diag() if diag else None
    Eo, Fo = ctx.run(E, F, k, s, B, dt, nsteps, inflow=inflow, diag=dg)
    torch.cuda.synchronize()
    out = (to_host(Eo), [to_host(f) for f in Fo])
    if diag:
        dgh = {kk: v.cpu().numpy() for kk, v in dg.items()}
        return out + (dgh,)
    return out
