"""Helpers shared by the GPU parity tests: run a workload through the HIP library and through
the CPU oracle on the same seeded inputs, and compare (relative L1 norms)."""
import numpy as np
import torch

from oracle import m1_oracle as orc

# Tolerances (spec targets): FP64 path vs FP64 oracle after the full run; MIXED path
# (float storage and bulk arithmetic, double closure near f -> 1, double source) vs the FP64
# oracle per step and after many steps.
TOL_FP64 = 1e-12
TOL_MIXED_STEP = 1e-5
TOL_MIXED_RUN = 1e-4


def problem_of(w, **kw):
    p = orc.Problem(ndim=w.ndim, n=w.n, G=w.G, coord=w.coord, lo=w.lo, hi=w.hi, bc_lo=w.bc_lo, bc_hi=w.bc_hi,
                    c=w.c)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def rel_l1(E, F, Eref, Fref, c=1.0):
    """rel-L1 of E, and of the flux components normalised by c sum |E_ref|."""
    E = np.asarray(E, dtype=np.float64)
    Eref = np.asarray(Eref, dtype=np.float64)
    sE = np.sum(np.abs(Eref))
    eE = np.sum(np.abs(E - Eref)) / sE
    eF = max([np.sum(np.abs(np.asarray(f, dtype=np.float64) - fr)) / (c * sE) for f, fr in zip(F, Fref)] + [0.0])
    return eE, eF


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
