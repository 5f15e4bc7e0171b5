"""The allocation-free observables read (hl_read_observables_device_noalloc)
against the allocating device reads (hl_read_density_device,
hl_read_velocity_device, hl_read_wss_device), through the C ABI: two calls in
a row, the first on a context larger than one pass of the fixed scratch (two
passes), the second on a smaller context whose values must not be disturbed
by what the first left in the scratch.  The results must be bit for bit those
of the allocating reads, and the device's free memory must not change across
the allocation-free calls."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_04144_amd as hl
    hl.lib()
    return hl


def _context(hl, geo, prec, order, steps):
    import torch
    ctx = hl.Context(0, prec, order=order)
    d = ctx.add_domain()
    ctx.load_geometry(d, geo)
    ctx.set_tau(d, 0.7)
    ctx.set_inlet_velocity(d, 0, 0.02)
    ctx.set_stream(torch.cuda.current_stream())
    ctx.step(steps)
    return ctx


def _compare(hl, ctx, n):
    import torch
    f64 = dict(dtype=torch.float64, device="cuda")
    ref = [torch.empty(n, **f64), torch.empty((3, n), **f64), torch.empty(n, **f64)]
    ctx.density_device(0, ref[0])
    ctx.velocity_device(0, ref[1])
    ctx.wss_device(0, ref[2])
    torch.cuda.synchronize()
    out = [torch.full_like(r, float("nan")) for r in ref]
    only_u = torch.full_like(ref[1], float("nan"))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ctx.observables_device_noalloc(0, out[0], out[1], out[2])
    ctx.observables_device_noalloc(0, None, only_u, None)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, (free0, free1)
    for r, o in zip(ref, out):
        assert torch.equal(r, o)
    assert torch.equal(only_u, ref[1])
    assert float(ref[0].abs().min()) > 0.5            # a density was written everywhere


def test_noalloc_read_two_calls_large_then_small(hl):
    big = synth.cylinder(nx=42, ny=42, nz=1400, radius=20.0)
    assert big.n > 1_677_696                         # more than one pass of the scratch
    a = _context(hl, big, "f32", hl.HL_ORDER_BRICK | hl.HL_ORDER_BRICK_32, 7)
    print("noalloc read: large context", big.n, "sites", flush=True)
    _compare(hl, a, big.n)
    a.close()
    small = synth.cylinder(nz=16)
    b = _context(hl, small, "f64", hl.HL_ORDER_BRICK | hl.HL_SCHEME_AA, 5)
    print("noalloc read: small context", small.n, "sites", flush=True)
    _compare(hl, b, small.n)
    b.close()


def test_noalloc_read_needs_a_committed_context(hl):
    ctx = hl.Context(0, "f64")
    d = ctx.add_domain()
    ctx.load_geometry(d, synth.cylinder(nz=8))
    with pytest.raises(hl.HLError) as ei:
        ctx.observables_device_noalloc(0, None, None, None)
    assert ei.value.code == hl.HL_E_STATE
    with pytest.raises(hl.HLError) as ei:
        ctx.observables_device_noalloc(3, None, None, None)
    assert ei.value.code == hl.HL_E_RANGE
