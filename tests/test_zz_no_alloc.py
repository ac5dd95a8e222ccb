"""fornax_m1_step_noalloc (scratch in the library's static device array) against fornax_m1_step
(scratch in the context), through the C interface: the same kernels, so the same outputs and
diagnostics bit for bit, on two calls in a row -- the second on a smaller grid, with the
array still holding the first call's contents -- and a grid whose scratch does not fit the
array is refused before any launch."""
import sys

import numpy as np
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


def _inputs(ctx, w):
    dtp = ctx.dtype
    E = to_dev(w.E, dtp)
    F = [to_dev(f, dtp) for f in w.F]
    k, s, B = (to_dev(x, dtp) for x in (w.kappa, w.sigma, w.B))
    return E, F, k, s, B


def _both(m1, w, precision):
    ctx = m1.Context(m1.Config.from_workload(w, precision=precision))
    E, F, k, s, B = _inputs(ctx, w)
    dref, dna = ctx.new_diag(), ctx.new_diag()
    ref = ctx.step(E, F, k, s, B, w.dt, diag=dref)
    got = ctx.step(E, F, k, s, B, w.dt, diag=dna, noalloc=True)
    torch.cuda.synchronize()
    return ref, got, dref, dna


def _check_equal(ref, got, dref, dna, what):
    assert torch.equal(ref[0], got[0]), what
    for a, b in zip(ref[1], got[1]):
        assert torch.equal(a, b), what
    for key in dref:
        assert torch.equal(dref[key], dna[key]), (what, key)


def test_noalloc_step_matches_step_on_two_calls(m1):
    # first call: the 2-D 512^2 x 16 grid in FP64 (whole-zone kernel, diagnostics partials in the
    # static array)
    w1 = wl.blobs2d(n=512, G=16, steps=1)
    say("case noalloc blobs2d 512x512x16 fp64")
    r1 = _both(m1, w1, m1.FP64)
    _check_equal(*r1, "blobs2d 512")
    assert float(r1[2]["energy_total"].item()) > 0.0
    # second call, smaller: 3-D 40^3 x 12 in MIXED (tiled kernel, partials summed by a second
    # launch, dE_matter partials of split group blocks in the static array)
    w2 = wl.core3d(n=40, G=12, steps=1)
    say("case noalloc core3d 40^3x12 mixed")
    r2 = _both(m1, w2, m1.MIXED)
    _check_equal(*r2, "core3d 40")
    # and the first grid again (the array holds the second call's partials)
    say("case noalloc blobs2d 512x512x16 fp64 again")
    r3 = _both(m1, w1, m1.FP64)
    _check_equal(*r3, "blobs2d 512 again")
    assert torch.equal(r3[1][0], r1[1][0])


def test_noalloc_refuses_scratch_beyond_the_array(m1):
    # SSP-RK2 keeps a whole stage state in the scratch: 3 x 512^2 x 16 doubles (100 MB) do not fit
    w = wl.blobs2d(n=512, G=16, steps=1)
    say("case noalloc ssprk2 512x512x16 refused")
    ctx = m1.Context(m1.Config.from_workload(w, precision=m1.FP64, integrator=m1.SSPRK2))
    E, F, k, s, B = _inputs(ctx, w)
    out = ctx.empty_state()
    out[0].fill_(7.0)
    with pytest.raises(m1.FornaxError) as ei:
        ctx.step(E, F, k, s, B, w.dt, out=out, noalloc=True)
    assert ei.value.code == m1.FORNAX_ESCRATCH
    torch.cuda.synchronize()
    assert bool(torch.all(out[0] == 7.0))   # nothing launched
    # a grid whose stage fits runs, and matches the context-scratch step
    w2 = wl.blobs2d(n=64, G=4, steps=1)
    say("case noalloc ssprk2 64x64x4")
    ctx2 = m1.Context(m1.Config.from_workload(w2, precision=m1.FP64, integrator=m1.SSPRK2))
    E, F, k, s, B = _inputs(ctx2, w2)
    ref = ctx2.step(E, F, k, s, B, w2.dt)
    got = ctx2.step(E, F, k, s, B, w2.dt, noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(ref[0], got[0]) and all(torch.equal(a, b) for a, b in zip(ref[1], got[1]))
    np.testing.assert_array_equal(got[0].cpu().numpy(), ref[0].cpu().numpy())
