"""The step under HIP graph capture: three steps with diagnostics captured once and replayed
several times, with eager work and synchronisations between the replays, give the eager result
bit for bit on every replay (the step launches kernels only: no allocation, no memset; the
whole-zone kernel's block-arrival counter returns to zero within each launch)."""
import sys

import pytest
import torch

from paper_1806_07390_amd import workloads as wl
from tests.parity_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m1():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1806_07390_amd import m1 as mod
    return mod


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_step_replays_in_a_graph(m1, prec):
    p = m1.FP64 if prec == "fp64" else m1.MIXED
    w = wl.blobs2d(n=70, G=16, steps=3)      # FP64: the whole-zone kernel; MIXED: the tiled one
    ctx = m1.Context(m1.Config.from_workload(w, precision=p))
    dtp = ctx.dtype
    E0 = to_dev(w.E, dtp)
    F0 = [to_dev(f, dtp) for f in w.F]
    k, s, B = (to_dev(x, dtp) for x in (w.kappa, w.sigma, w.B))
    A = (E0.clone(), [f.clone() for f in F0])
    Bs = ctx.empty_state()
    dg = ctx.new_diag()

    def reset():
        A[0].copy_(E0)
        for f, f0 in zip(A[1], F0):
            f.copy_(f0)

    def three_steps():
        ctx.step(A[0], A[1], k, s, B, w.dt, out=Bs, diag=dg)
        ctx.step(Bs[0], Bs[1], k, s, B, w.dt, out=A, diag=dg)
        ctx.step(A[0], A[1], k, s, B, w.dt, out=Bs, diag=dg)

    def snapshot():
        return [Bs[0].clone()] + [f.clone() for f in Bs[1]] + [v.clone() for v in dg.values()]

    three_steps()
    torch.cuda.synchronize()
    ref = snapshot()

    reset()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        three_steps()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    reset()
    with torch.cuda.graph(g):
        three_steps()
    for rep in range(4):
        reset()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = snapshot()
        say(f"graph replay {rep} prec={prec}")
        for a, b in zip(got, ref):
            assert torch.equal(a, b)
        # unrelated eager work between replays
        x = torch.randn(4096, device="cuda")
        assert torch.isfinite(x.sum())
        torch.cuda.synchronize()
