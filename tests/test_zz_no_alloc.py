"""The entry point that allocates nothing (dcrf_qp_frank_wolfe_noalloc),
called through the C ABI and checked against dcrf_qp_frank_wolfe on the same
inputs: two calls in a row on one device, the second with a smaller input
(another context with a smaller image and fewer labels), so that the second
runs on the scratch array the first one left behind.

Bars: the same kernels run on the same layouts, so the two entry points
differ only in the order of the splat's floating-point atomics. In FP64
(32x24, L = 3) that leaves every decision equal: marginals within 1e-12,
objectives within 1e-12 relative, step sizes within 1e-10. In FP32 at
500x375, L = 21 (the benchmarked solve), a conditional gradient at a near-tie
may go either way between any two runs, so as for the FP32 trajectory tests:
objectives within 1e-5 relative and marginals within 1e-4 except on a share
below 1e-3. A solve larger than the scratch array is refused with
DCRF_EINVAL.
"""

import numpy as np
import pytest
import torch

from paper_1608_06192_amd import synth

pytestmark = pytest.mark.gpu

KERNELS = [synth.BILATERAL, synth.SPATIAL]


def _ctx(im, dtype):
    from paper_1608_06192_amd import dcrf
    print(f"[case] noalloc {im.H}x{im.W} L={im.L} {dtype}", flush=True)
    c = dcrf.Context(0)
    c.set_image(im.H, im.W, torch.from_numpy(im.rgb).cuda(), KERNELS, dtype=dtype)
    return c


def _compare(im, dtype, iters, ytol, ftol, atol, share=0.0):
    ctx = _ctx(im, dtype)
    phi = torch.from_numpy(im.unary).cuda().to(dtype)
    y0 = torch.softmax(-phi, dim=1)
    ya, yb = y0.clone(), y0.clone()
    ta = ctx.qp_frank_wolfe(phi, None, ya, iters)
    tb = ctx.qp_frank_wolfe_noalloc(phi, None, yb, iters)
    d = (ya - yb).abs()
    off = (d > ytol).double().mean().item()
    print(f"[noalloc] {im.H}x{im.W} L={im.L}: max |dy| {d.max().item():.3g}, share "
          f"beyond {ytol:g}: {off:.3g}", flush=True)
    assert off <= share
    for ra, rb in zip(ta, tb):
        assert abs(ra[0] - rb[0]) <= ftol * abs(ra[0])
        if share == 0.0:
            assert abs(ra[2] - rb[2]) <= atol
    # an explicit mu takes the same path as the null one
    yc = y0.clone()
    mu = torch.from_numpy(synth.potts(im.L)).cuda().to(dtype)
    ctx.qp_frank_wolfe_noalloc(phi, mu, yc, iters, trace=False)
    assert ((yc - yb).abs() > ytol).double().mean().item() <= share


def test_noalloc_matches_frank_wolfe_twice_second_smaller():
    _compare(synth.make("voronoi_500x375_L21"), torch.float32, 12, 1e-4, 1e-5, 0.0,
             share=1e-3)
    _compare(synth.make("rect_32x24_L3"), torch.float64, 20, 1e-12, 1e-12, 1e-10)


def test_noalloc_refuses_what_does_not_fit():
    from paper_1608_06192_amd import dcrf
    import ctypes
    n = ctypes.c_size_t()
    assert dcrf._lib.dcrf_noalloc_scratch_bytes(ctypes.byref(n)) == 0
    im = synth.voronoi_image(600, 800, 21, seed=81)   # 3 N L FP64 values > 64 MiB
    ctx = _ctx(im, torch.float64)
    phi = torch.from_numpy(im.unary).cuda()
    y = torch.softmax(-phi, dim=1)
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.qp_frank_wolfe_noalloc(phi, None, y, 2)
    assert dcrf.STATUS[e.value.status] == "DCRF_EINVAL"
    ctx.qp_frank_wolfe(phi, None, y, 2, trace=False)   # the context is untouched
