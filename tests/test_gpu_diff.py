"""GPU parity of the reverse-mode derivative of unrolled Frank-Wolfe (the
differentiable QP of Sec. 4 with the line search of App. B) against the FP64
oracle's reverse sweep, through the C ABI and through the autograd Function.

Tolerances:
* FP64, same discrete decisions on both sides (checked: the conditional
  gradients s_t and which steps are interior): y_T within 1e-10 absolute,
  step sizes within 1e-9, dl/dphi within 1e-8 of max|dl/dphi| elementwise and
  dl/dw within 1e-8 relative. The two sides differ only by summation order
  (lattice atomics, block reductions), amplified by the 1/(2 a2) of each
  interior step.
* FP32 at 500x375, L=21, 10 iterations against the FP64 oracle: argmin
  near-ties let a few conditional-gradient labels differ (counted, at most
  1e-3 of the decisions); dl/dphi within 1e-4 in relative 2-norm. dl/dw is a
  sum of summands that cancel to about 1e-4 of their absolute sum at this
  workload (the oracle reports that absolute sum), so FP32 rounding of the
  marginals and filter outputs (unit roundoff u = 6e-8) moves it by about u
  times the absolute sum; the bound is 16 u times it.
* Central differences of the GPU's own FP64 loss with every discrete decision
  (s_t, interior step) checked equal at +eps and -eps: 1e-4 relative. Along
  the unaries at 500x375 the direction is masked to a random subset of
  pixels, so that some eps leaves all decisions unchanged; a change of a
  weight moves the gradient of every pixel, so at 500x375 every eps large
  enough to rise above FP64 rounding changes some decisions, and the weight
  directions are checked on a 128x96 image.
"""

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1608_06192_amd import synth

from diffsaved import _a256, saved_offsets, unpack_saved

pytestmark = pytest.mark.gpu

KERNELS = [synth.BILATERAL, synth.SPATIAL]


def dev():
    return torch.device("cuda:0")


def T(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev(), dtype)


def gpu_ctx(im, dtype, kernels=KERNELS):
    from paper_1608_06192_amd import dcrf
    print(f"[case] {im.H}x{im.W} L={im.L} dtype={dtype}", flush=True)
    ctx = dcrf.Context(0)
    ctx.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev()), kernels,
                  dtype=dtype)
    return ctx


def oracle_problem(im, iters, mu, kernels=KERNELS):
    model = O.Model(im.H, im.W, im.rgb, kernels)
    loss, yT, tape, qp, c = O.fw_unrolled_loss(model, im.unary, mu, iters, im.gt)
    ybar = O.cross_entropy_grad(yT, im.gt)
    gphi, gw, gw_abs = O.fw_unrolled_backward(qp, tape, c, ybar, scale=True)
    return dict(model=model, loss=loss, yT=yT, tape=tape, ybar=ybar, gphi=gphi,
                gw=gw, gw_abs=gw_abs)


def gpu_run(ctx, im, mu, iters, dtype, ybar):
    phi, m = T(im.unary, dtype), T(mu, dtype)
    y, saved = ctx.fw_forward(phi, m, iters)
    gphi, gw = ctx.fw_backward(phi, m, iters, saved, T(ybar, dtype))
    torch.cuda.synchronize()
    return y.double().cpu().numpy(), saved, gphi.double().cpu().numpy(), np.array(gw)


def general_mu(L, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.2, 1.5, size=(L, L))
    mu = 0.5 * (mu + mu.T)
    np.fill_diagonal(mu, 0.0)
    return mu


@pytest.mark.parametrize("case", ["rect_32x24_L3", "voronoi_48x40_L5_mu",
                                  "voronoi_320x213_L21",
                                  "voronoi_500x375_L21_diff"])
def test_fw_diff_fp64_matches_oracle(case):
    if case == "rect_32x24_L3":
        im, iters, mu = synth.make(case), 20, synth.potts(3)
    elif case == "voronoi_48x40_L5_mu":
        im, iters, mu = synth.voronoi_image(40, 48, 5, seed=7), 8, general_mu(5, 7)
    else:
        im, iters = synth.make(case), 10
        mu = synth.potts(im.L)
    ref = oracle_problem(im, iters, mu)
    assert any(r["interior"] for r in ref["tape"])
    ctx = gpu_ctx(im, torch.float64)
    y, saved, gphi, gw = gpu_run(ctx, im, mu, iters, torch.float64, ref["ybar"])
    s, stats = unpack_saved(ctx, saved, im.N, im.L, iters, 8)
    for t, r in enumerate(ref["tape"]):
        assert np.array_equal(s[t], r["s"].argmax(1)), f"s_{t}"
        assert bool(stats[t, 3]) == bool(r["interior"]), f"interior {t}"
        assert abs(stats[t, 0] - r["alpha"]) <= 1e-9
    assert np.abs(y - ref["yT"]).max() <= 1e-10
    assert np.abs(gphi - ref["gphi"]).max() <= 1e-8 * np.abs(ref["gphi"]).max()
    assert np.allclose(gw, ref["gw"], rtol=1e-8, atol=0)


def test_fw_diff_fp32_matches_oracle_500x375():
    im = synth.make("voronoi_500x375_L21_diff")
    iters = synth.WORKLOADS["voronoi_500x375_L21_diff"]["iters"]
    mu = synth.potts(im.L)
    ref = oracle_problem(im, iters, mu)
    ctx = gpu_ctx(im, torch.float32)
    y, saved, gphi, gw = gpu_run(ctx, im, mu, iters, torch.float32, ref["ybar"])
    s, stats = unpack_saved(ctx, saved, im.N, im.L, iters, 4)
    differ = sum(int((s[t] != r["s"].argmax(1)).sum())
                 for t, r in enumerate(ref["tape"]))
    frac = differ / (iters * im.N)
    err_phi = np.linalg.norm(gphi - ref["gphi"]) / np.linalg.norm(ref["gphi"])
    err_w = np.abs(gw - ref["gw"])
    bound_w = 16 * 6e-8 * ref["gw_abs"]
    dy = np.abs(y - ref["yT"])
    print(f"[fp32 diff] decisions differing {differ} ({frac:.2e}); "
          f"|dphi| rel {err_phi:.2e}; dw err {err_w} bound {bound_w} "
          f"(rel {err_w / np.abs(ref['gw'])}); "
          f"y max {dy.max():.2e}, share > 1e-4 {(dy > 1e-4).mean():.2e}", flush=True)
    assert frac <= 1e-3
    assert err_phi <= 1e-4
    assert (err_w <= bound_w).all()
    # marginals: FP32 decisions may flip at near-ties, so a share of entries
    # may differ; measured 8.6e-6 of them beyond 1e-4
    assert (dy > 1e-4).mean() <= 1e-3


def _gpu_loss(ctx, phi, mu, iters, gt):
    y, saved = ctx.fw_forward(phi, mu, iters)
    yv = y.double()
    p = yv[torch.arange(yv.shape[0], device=yv.device), gt].clamp_min(1e-12)
    return float(-torch.log(p).mean()), saved


def _decision_changes(ctx, sp, sm, N, L, iters):
    sp_s, sp_st = unpack_saved(ctx, sp, N, L, iters, 8)
    sm_s, sm_st = unpack_saved(ctx, sm, N, L, iters, 8)
    return int((sp_s != sm_s).sum()) + int((sp_st[:, 3] != sm_st[:, 3]).sum())


def _fd_check(ctx, im, iters, directions, eps_list):
    """directions: (name, perturbed-loss function of eps, analytic value)"""
    for name, loss_at, analytic in directions:
        used = None
        for eps in eps_list:
            lp, sp = loss_at(eps)
            lm, sm = loss_at(-eps)
            changes = _decision_changes(ctx, sp, sm, im.N, im.L, iters)
            fd = (lp - lm) / (2 * eps)
            print(f"[fd] {name} eps={eps:g}: fd={fd:.10e} analytic={analytic:.10e}"
                  f" decision changes={changes}", flush=True)
            if changes == 0:
                used = fd
                break
        assert used is not None, f"{name}: decisions change at every eps"
        assert abs(used - analytic) <= 1e-4 * abs(analytic), name


def _fd_setup(im):
    ctx = gpu_ctx(im, torch.float64)
    phi = T(im.unary, torch.float64)
    mu = T(synth.potts(im.L), torch.float64)
    gt = torch.from_numpy(im.gt.astype(np.int64)).to(dev())
    return ctx, phi, mu, gt


def _analytic(ctx, im, phi, mu, iters, gt):
    y, saved = ctx.fw_forward(phi, mu, iters)
    idx = torch.arange(im.N, device=dev())
    ybar = torch.zeros_like(y)
    ybar[idx, gt] = -1.0 / (im.N * y[idx, gt].clamp_min(1e-12))
    ybar[idx, gt] *= (y[idx, gt] > 1e-12).double()
    return ctx.fw_backward(phi, mu, iters, saved, ybar)


def test_fw_diff_central_differences_unaries_500x375():
    im = synth.make("voronoi_500x375_L21_diff")
    iters = synth.WORKLOADS["voronoi_500x375_L21_diff"]["iters"]
    ctx, phi, mu, gt = _fd_setup(im)
    gphi, _ = _analytic(ctx, im, phi, mu, iters, gt)
    rng = np.random.default_rng(5)
    dirs = []
    for k, npix in enumerate((64, 1024)):
        v = np.zeros(im.unary.shape)
        pix = rng.choice(im.N, size=npix, replace=False)
        v[pix] = rng.normal(size=(npix, im.L))
        vt = T(v, torch.float64)
        dirs.append((f"phi[mask {npix} px]",
                     lambda e, vt=vt: _gpu_loss(ctx, phi + e * vt, mu, iters, gt),
                     float((gphi * vt).sum())))
    _fd_check(ctx, im, iters, dirs, (1e-3, 1e-4, 1e-5, 1e-6))


def test_fw_diff_central_differences_weights_128x96():
    im = synth.voronoi_image(96, 128, 21, seed=11)
    iters = 10
    ctx, phi, mu, gt = _fd_setup(im)
    _, gw = _analytic(ctx, im, phi, mu, iters, gt)
    w0 = np.array([k["weight"] for k in KERNELS])

    def at(m):
        def f(e):
            dw = np.zeros(len(KERNELS))
            dw[m] = e
            ctx.set_weights(list(w0 + dw))
            try:
                return _gpu_loss(ctx, phi, mu, iters, gt)
            finally:
                ctx.set_weights(list(w0))
        return f

    dirs = [(f"w{m}", at(m), gw[m]) for m in range(len(KERNELS))]
    _fd_check(ctx, im, iters, dirs, (1e-3, 1e-4, 1e-5, 1e-6))


def test_autograd_function_matches_abi_and_oracle():
    from paper_1608_06192_amd.autograd import unrolled_frank_wolfe
    im, iters, mu_np = synth.make("rect_32x24_L3"), 12, synth.potts(3)
    ref = oracle_problem(im, iters, mu_np)
    ctx = gpu_ctx(im, torch.float64)
    gt = torch.from_numpy(im.gt.astype(np.int64)).to(dev())
    for recompute in (False, True):
        phi = T(im.unary, torch.float64).requires_grad_(True)
        w = torch.tensor([k["weight"] for k in KERNELS], dtype=torch.float64,
                         requires_grad=True)
        y = unrolled_frank_wolfe(ctx, phi, w, T(mu_np, torch.float64), iters,
                                 recompute=recompute)
        p = y[torch.arange(im.N, device=dev()), gt].clamp_min(1e-12)
        loss = -torch.log(p).mean()
        loss.backward()
        assert abs(loss.item() - ref["loss"]) <= 1e-10
        g = phi.grad.cpu().numpy()
        assert np.abs(g - ref["gphi"]).max() <= 1e-8 * np.abs(ref["gphi"]).max()
        assert np.allclose(w.grad.numpy(), ref["gw"], rtol=1e-8, atol=0)


def test_autograd_weights_are_applied():
    """The Function sets the weights it is given: its output equals the
    oracle's at other weights, and the context keeps them afterwards."""
    from paper_1608_06192_amd.autograd import unrolled_frank_wolfe
    im, iters, mu_np = synth.make("rect_32x24_L3"), 6, synth.potts(3)
    w_np = np.array([4.0, 1.5])
    kern = [dict(k, weight=float(w)) for k, w in zip(KERNELS, w_np)]
    model = O.Model(im.H, im.W, im.rgb, kern)
    _, yT, _, _, _ = O.fw_unrolled_loss(model, im.unary, mu_np, iters, im.gt)
    ctx = gpu_ctx(im, torch.float64)
    y = unrolled_frank_wolfe(ctx, T(im.unary, torch.float64),
                             torch.tensor(w_np), T(mu_np, torch.float64), iters)
    assert np.abs(y.cpu().numpy() - yT).max() <= 1e-10


def test_fw_diff_errors():
    from paper_1608_06192_amd import dcrf
    im = synth.make("rect_32x24_L3")
    ctx = gpu_ctx(im, torch.float64)
    phi, mu = T(im.unary, torch.float64), T(synth.potts(3), torch.float64)
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.fw_forward(phi, mu, 0)
    assert dcrf.STATUS[e.value.status] == "DCRF_EINVAL"
    ctx.set_filter_mode("exact")
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.fw_saved_size(3, 4)
    assert dcrf.STATUS[e.value.status] == "DCRF_EUNSUPPORTED"
    ctx.set_filter_mode("lattice")
    s_off, st_off = saved_offsets(ctx, im.N, 3, 4, 8)
    assert ctx.fw_saved_size(3, 4) == _a256(st_off + 4 * 32)


def test_forward_weights_argument_and_summed_gradient():
    # dcrf_fw_forward's weights argument gives the same forward and reverse
    # sweep as setting the weights first; the library's summed weight
    # gradient of a single image equals its per-image gradient
    im = synth.make("rect_32x24_L3")
    ctx = gpu_ctx(im, torch.float64)
    phi = T(im.unary, torch.float64)
    w = [7.0, 2.0]
    ya, sa = ctx.fw_forward(phi, None, 6, w=w)
    ybar = torch.randn(ya.shape, generator=torch.Generator().manual_seed(3),
                       dtype=torch.float64).to(dev())
    ga, wa = ctx.fw_backward(phi, None, 6, sa, ybar)
    gs, ws = ctx.fw_backward(phi, None, 6, sa, ybar, summed=True)
    assert (ga - gs).abs().max().item() <= 1e-10 * ga.abs().max().item()
    assert np.allclose(wa, ws, rtol=1e-10, atol=0)
    ctx2 = gpu_ctx(im, torch.float64)
    ctx2.set_weights(w)
    yb, sb = ctx2.fw_forward(phi, None, 6)
    gb, wb = ctx2.fw_backward(phi, None, 6, sb, ybar)
    assert (ya - yb).abs().max().item() <= 1e-12
    assert (ga - gb).abs().max().item() <= 1e-10 * ga.abs().max().item()
    assert np.allclose(wa, wb, rtol=1e-10, atol=0)
    # and the oracle with those weights
    kern = [dict(synth.BILATERAL, weight=w[0]), dict(synth.SPATIAL, weight=w[1])]
    model = O.Model(im.H, im.W, im.rgb, kern)
    _, yT, tape, qp, c = O.fw_unrolled_loss(model, im.unary, synth.potts(3), 6, im.gt)
    assert np.abs(ya.cpu().numpy() - yT).max() <= 1e-10
    _, gw_o = O.fw_unrolled_backward(qp, tape, c, ybar.cpu().numpy())
    assert np.allclose(wa, gw_o, rtol=1e-8, atol=0)
