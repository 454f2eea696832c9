"""GPU tests of the boundary's memory and error contract:

* a context given a caller workspace of dcrf_workspace_size bytes runs every
  call (filter both ways and exact, Frank-Wolfe, DC_gen, DC_neg, energy,
  rounding, LP subgradient and descent, the unrolled forward and backward,
  the autotuner) and gives the results of a context that allocates for
  itself, up to floating-point summation order; its peak use stays within
  the workspace, and a workspace too small is reported as DCRF_ENOMEM with
  the context still usable;
* the same for a batch of images;
* failures forced from the host: a hash table smaller than the lattice
  (DCRF_ECAPACITY, then a normal build), a non-finite colour and
  non-finite unaries (DCRF_EINVAL, reported by the next synchronising call).
"""

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1608_06192_amd import synth

pytestmark = pytest.mark.gpu

KERNELS = [synth.BILATERAL, synth.SPATIAL]


def dev():
    return torch.device("cuda:0")


def T(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev(), dtype)


def _run_all(ctx, im, dtype, L):
    """every solver entry point once; returns their results"""
    out = {}
    phi = T(im.unary, dtype)
    Y = torch.rand(im.N, L, generator=torch.Generator().manual_seed(1),
                   dtype=torch.float64).to(dev(), dtype)
    out["filter"] = ctx.filter(Y)
    out["adjoint"] = ctx.filter(Y, adjoint=True)
    y0 = torch.softmax(-phi, dim=1)
    y = y0.clone()
    out["fw_trace"] = ctx.qp_frank_wolfe(phi, None, y, 15)
    out["fw"] = y.clone()
    out["dc_gen"] = ctx.dc_gen(phi, None, y, 2, 4)
    out["dc_neg"] = ctx.dc_neg(phi, None, y, 3)
    lab = ctx.round(y)
    out["labels"] = lab
    out["energy"] = ctx.energy(phi, None, lab)
    # the LP sorts its input: both contexts get the same fixed point (the
    # solvers' outputs differ in their last bits, which may reorder
    # near-equal values and give another valid subgradient)
    y_lp = torch.softmax(-phi, dim=1)
    out["lp"] = ctx.lp_subgradient(phi, y_lp)
    yl = y_lp.clone()
    out["lp_descent"] = ctx.lp_descent(phi, yl, 1, 1e-6)
    yT, saved = ctx.fw_forward(phi, None, 5)
    out["fw_forward"] = yT
    ybar = torch.randn(yT.shape, generator=torch.Generator().manual_seed(2),
                       dtype=torch.float64).to(dev(), dtype)
    out["fw_backward"] = ctx.fw_backward(phi, None, 5, saved, ybar)
    return out


def _close(a, b, rtol):
    if isinstance(a, torch.Tensor):
        if a.dtype == torch.int32:
            return torch.equal(a, b)
        return (a - b).abs().max().item() <= rtol * (1.0 + a.abs().max().item())
    if isinstance(a, (list, tuple)):
        return all(_close(x, y, rtol) for x, y in zip(a, b))
    return abs(a - b) <= rtol * (1.0 + abs(a))


def test_workspace_runs_every_call_without_allocating():
    from paper_1608_06192_amd import dcrf
    im = synth.make("voronoi_320x213_L21")
    f64 = torch.float64
    L = im.L
    rgb = torch.from_numpy(im.rgb).to(dev())
    need = dcrf.workspace_size([(im.H, im.W)], L, KERNELS, f64)
    ws = torch.empty(need, dtype=torch.uint8, device=dev())
    print(f"[case] workspace {need / 1e6:.1f} MB for 320x213 L=21 FP64", flush=True)
    a = dcrf.Context(0)
    a.set_image(im.H, im.W, rgb, KERNELS, dtype=f64, workspace=ws)
    b = dcrf.Context(0)
    b.set_image(im.H, im.W, rgb, KERNELS, dtype=f64)
    ra, rb = _run_all(a, im, f64, L), _run_all(b, im, f64, L)
    for k in ra:
        assert _close(ra[k], rb[k], 1e-9), k
    tune = a.autotune(L, reps=1)
    assert tune["dense_chunk"] <= 64
    in_use, peak = a.workspace_used()
    print(f"[workspace] in use {in_use / 1e6:.1f} MB, peak {peak / 1e6:.1f} MB of "
          f"{need / 1e6:.1f} MB", flush=True)
    assert 0 < in_use <= peak <= need
    with pytest.raises(dcrf.DcrfError) as e:   # more than 64 entries per dense chunk
        a.set_tune(splat_chunk=64, dense_chunk=128, blur_vectors_per_thread=1,
                   blur_block=256, blur_group=2)
    assert dcrf.STATUS[e.value.status] == "DCRF_EINVAL"
    # a new image in the same workspace, then back to self-allocation
    im2 = synth.voronoi_image(150, 200, L, seed=71)
    a.set_image(im2.H, im2.W, torch.from_numpy(im2.rgb).to(dev()), KERNELS, dtype=f64,
                workspace=ws)
    y2 = torch.softmax(-T(im2.unary, f64), dim=1)
    a.qp_frank_wolfe(T(im2.unary, f64), None, y2, 5, trace=False)
    a.set_image(im.H, im.W, rgb, KERNELS, dtype=f64)
    with pytest.raises(dcrf.DcrfError):
        a.workspace_used()
    yb = torch.softmax(-T(im.unary, f64), dim=1)
    a.qp_frank_wolfe(T(im.unary, f64), None, yb, 15, trace=False)
    assert _close(yb, rb["fw"], 1e-9)


def test_workspace_too_small_is_reported():
    from paper_1608_06192_amd import dcrf
    im = synth.make("voronoi_320x213_L21")
    rgb = torch.from_numpy(im.rgb).to(dev())
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=dev())
    ctx = dcrf.Context(0)
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.set_image(im.H, im.W, rgb, KERNELS, workspace=ws)
    assert dcrf.STATUS[e.value.status] == "DCRF_ENOMEM"
    ctx.set_image(im.H, im.W, rgb, KERNELS)          # usable: allocates itself
    y = torch.softmax(-T(im.unary, torch.float32), dim=1)
    ctx.qp_frank_wolfe(T(im.unary, torch.float32), None, y, 3, trace=False)


def test_batch_workspace_matches_self_allocation():
    from paper_1608_06192_amd import dcrf
    L = 5
    ims = [synth.voronoi_image(24, 40, L, seed=72), synth.rect_image(33, 17, L, seed=73),
           synth.voronoi_image(45, 29, L, seed=74, regions=6)]
    f64 = torch.float64
    sizes = [(im.H, im.W) for im in ims]
    rgbs = [torch.from_numpy(im.rgb).to(dev()) for im in ims]
    need = dcrf.workspace_size(sizes, L, KERNELS, f64)
    ws = torch.empty(need, dtype=torch.uint8, device=dev())
    res = []
    for w in (ws, None):
        ctx = dcrf.Context(0)
        ctx.set_images(sizes, rgbs, KERNELS, dtype=f64, workspace=w)
        phi = ctx.pack([T(im.unary, f64) for im in ims], L)
        y, saved = ctx.fw_forward(phi, None, 6)
        g, gw = ctx.fw_backward(phi, None, 6, saved, torch.ones_like(y), summed=True)
        yd = ctx.pack([T(O.softmax_neg(im.unary), f64) for im in ims], L)
        h = ctx.dc_neg(phi, None, yd, 3)
        res.append((ctx.unpack(y), ctx.unpack(g), gw, h))
        if w is not None:
            assert ctx.workspace_used()[1] <= need
    (ya, ga, wa, ha), (yb, gb, wb, hb) = res
    for x, z in zip(ya + ga, yb + gb):
        assert _close(x, z, 1e-9)
    assert _close(wa, wb, 1e-9) and _close(ha, hb, 1e-9)


def test_forced_hash_capacity_then_recovery():
    from paper_1608_06192_amd import dcrf
    im = synth.make("rect_32x24_L3")
    rgb = torch.from_numpy(im.rgb).to(dev())
    ctx = dcrf.Context(0)
    ctx.set_hash_capacity(16)
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.set_image(im.H, im.W, rgb, KERNELS, dtype=torch.float64)
    assert dcrf.STATUS[e.value.status] == "DCRF_ECAPACITY"
    z = torch.zeros(im.N, 2, dtype=torch.float64, device=dev())
    st = dcrf._lib.dcrf_filter(ctx._h, z.data_ptr(), z[:, 1:].data_ptr(), 1, 0)
    assert dcrf.STATUS[st] == "DCRF_ESTATE"    # no image is set after the failure
    ctx.set_hash_capacity(0)
    ctx.set_image(im.H, im.W, rgb, KERNELS, dtype=torch.float64)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    Y = np.random.default_rng(3).uniform(-1, 1, size=(im.N, 3))
    g = ctx.filter(T(Y, torch.float64)).cpu().numpy()
    assert np.abs(g - model.Kp(Y)).max() <= 1e-11 * (1 + np.abs(model.Kp(Y)).max())
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.set_hash_capacity(1000)                # not a power of two
    assert dcrf.STATUS[e.value.status] == "DCRF_EINVAL"


def test_non_finite_inputs_are_reported():
    from paper_1608_06192_amd import dcrf
    im = synth.make("rect_32x24_L3")
    f64 = torch.float64
    ctx = dcrf.Context(0)
    bad_rgb = torch.from_numpy(im.rgb).to(dev()).clone()
    bad_rgb[17, 1] = float("nan")
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.set_image(im.H, im.W, bad_rgb, KERNELS, dtype=f64)
    assert dcrf.STATUS[e.value.status] == "DCRF_EINVAL"
    ctx.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev()), KERNELS, dtype=f64)
    phi = T(im.unary, f64)
    phi[5, 2] = float("inf")
    y = torch.softmax(-T(im.unary, f64), dim=1)
    ctx.qp_frank_wolfe(phi, None, y.clone(), 3, trace=False)   # asynchronous: no report
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.sync()
    assert dcrf.STATUS[e.value.status] == "DCRF_EINVAL"
    ctx.sync()                                              # reported once, then clear
    with pytest.raises(dcrf.DcrfError) as e:                # a synchronising call reports
        ctx.qp_frank_wolfe(phi, None, y.clone(), 3)
    assert dcrf.STATUS[e.value.status] == "DCRF_EINVAL"
    good = T(im.unary, f64)
    ctx.qp_frank_wolfe(good, None, y.clone(), 3)             # and the context is usable
    yn = y.clone()
    yn[0, 0] = float("nan")
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.energy(good, None, ctx.round(y)) if False else ctx.dc_neg(good, None, yn, 1)
    assert dcrf.STATUS[e.value.status] == "DCRF_EINVAL"
