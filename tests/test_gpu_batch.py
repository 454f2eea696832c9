"""GPU parity of the batched path: several images of uneven sizes in one
context (concatenated lattices, one launch per stage, per-image step sizes).

Per image, the batch computes the same thing as a context holding that image
alone. The two differ only in the order of floating-point atomics in the
splat. The checks are:
* filter outputs (FP64) against the FP64 oracle per image, within
  1e-11 * (K~|Y| + 2 sum(w) |Y|), and against the single-image GPU context to
  the same bound;
* Frank-Wolfe (FP64) marginals within 1e-10 and per-image objectives within
  1e-10 relative of the oracle, with the same conditional gradients;
* the reverse sweep (FP64) against the oracle's per image: dl/dphi within
  1e-8 of its max, dl/dw within 1e-8 relative;
* the 16-image 240..500 batch (FP64, 10 iterations) against 16 single-image
  GPU runs (1e-10) and, for its two smallest images, against the oracle.
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


def batch_ctx(ims, dtype):
    from paper_1608_06192_amd import dcrf
    print(f"[case] batch of {len(ims)}: " +
          " ".join(f"{im.H}x{im.W}" for im in ims) + f" dtype={dtype}", flush=True)
    ctx = dcrf.Context(0)
    ctx.set_images([(im.H, im.W) for im in ims],
                   [torch.from_numpy(im.rgb).to(dev()) for im in ims], KERNELS,
                   dtype=dtype)
    return ctx


def single_ctx(im, dtype):
    from paper_1608_06192_amd import dcrf
    ctx = dcrf.Context(0)
    ctx.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev()), KERNELS,
                  dtype=dtype)
    return ctx


def small_batch(L=5):
    return [synth.voronoi_image(24, 40, L, seed=31),
            synth.rect_image(33, 17, L, seed=32),
            synth.voronoi_image(45, 29, L, seed=33, regions=6)]


def test_batch_layout():
    ims = small_batch()
    ctx = batch_ctx(ims, torch.float64)
    assert ctx.nimg == 3
    starts = [a for a, _ in ctx.seg]
    assert starts[0] == 0 and all(a % 64 == 0 for a in starts)
    for (a, b), im in zip(ctx.seg, ims):
        assert b - a == im.N
    assert ctx.N == ctx.seg[-1][1]
    for j in range(2):
        assert ctx.seg[j][1] <= ctx.seg[j + 1][0] < ctx.seg[j][1] + 64


@pytest.mark.parametrize("adjoint", [False, True])
def test_batch_filter_matches_oracle_and_single(adjoint):
    ims = small_batch()
    ctx = batch_ctx(ims, torch.float64)
    rng = np.random.default_rng(4)
    Ys = [rng.uniform(-1, 1, size=(im.N, 4)) for im in ims]
    Yp = ctx.pack([T(Y, torch.float64) for Y in Ys], 4)
    out = ctx.filter(Yp, adjoint=adjoint)
    for im, Y, o in zip(ims, Ys, ctx.unpack(out)):
        model = O.Model(im.H, im.W, im.rgb, KERNELS)
        ref = model.Kp(Y, reverse=adjoint)
        bound = 1e-11 * (model.Kp(np.abs(Y)) + 2 * model.w.sum() * np.abs(Y))
        got = o.cpu().numpy()
        assert (np.abs(got - ref) <= bound + 1e-300).all()
        single = single_ctx(im, torch.float64).filter(T(Y, torch.float64),
                                                      adjoint=adjoint)
        assert (np.abs(got - single.cpu().numpy()) <= bound + 1e-300).all()


def _softmax_neg(phi):
    e = np.exp(-(phi - phi.min(axis=1, keepdims=True)))
    return e / e.sum(axis=1, keepdims=True)


def test_batch_fw_fp64_matches_oracle_per_image():
    ims = small_batch()
    L, iters = 5, 15
    mu = synth.potts(L)
    ctx = batch_ctx(ims, torch.float64)
    phi = ctx.pack([T(im.unary, torch.float64) for im in ims], L)
    y = ctx.pack([T(_softmax_neg(im.unary), torch.float64) for im in ims], L)
    traces = ctx.qp_frank_wolfe(phi, T(mu, torch.float64), y, iters)
    assert len(traces) == 3 and all(len(t) == iters for t in traces)
    for j, (im, yj) in enumerate(zip(ims, ctx.unpack(y))):
        model = O.Model(im.H, im.W, im.rgb, KERNELS)
        qp = O.QP(model, im.unary, mu)
        st = O.frank_wolfe(qp, _softmax_neg(im.unary), iters)
        assert np.abs(yj.cpu().numpy() - st.y).max() <= 1e-10
        for t in range(iters):
            obj, _, alpha = st.trace[t]
            assert abs(traces[j][t][0] - obj) <= 1e-10 * abs(obj)
            assert abs(traces[j][t][2] - alpha) <= 1e-9


def test_batch_fw_backward_fp64_matches_oracle_per_image():
    ims = small_batch()
    L, iters = 5, 8
    mu = synth.potts(L)
    ctx = batch_ctx(ims, torch.float64)
    refs = []
    for im in ims:
        model = O.Model(im.H, im.W, im.rgb, KERNELS)
        loss, yT, tape, qp, c = O.fw_unrolled_loss(model, im.unary, mu, iters, im.gt)
        ybar = O.cross_entropy_grad(yT, im.gt)
        gphi, gw = O.fw_unrolled_backward(qp, tape, c, ybar)
        refs.append((yT, ybar, gphi, gw))
    phi = ctx.pack([T(im.unary, torch.float64) for im in ims], L)
    m = T(mu, torch.float64)
    y, saved = ctx.fw_forward(phi, m, iters)
    ybar = ctx.pack([T(r[1], torch.float64) for r in refs], L)
    gphi, gw = ctx.fw_backward(phi, m, iters, saved, ybar)
    assert len(gw) == 3
    for j, (yj, gj, r) in enumerate(zip(ctx.unpack(y), ctx.unpack(gphi), refs)):
        assert np.abs(yj.cpu().numpy() - r[0]).max() <= 1e-10
        assert np.abs(gj.cpu().numpy() - r[2]).max() <= 1e-8 * np.abs(r[2]).max()
        assert np.allclose(gw[j], r[3], rtol=1e-8, atol=0)


def test_batch16_fp64_matches_single_runs_and_oracle():
    ims = synth.make_batch()
    iters = synth.WORKLOADS["voronoi_batch16_L21"]["iters"]
    L = ims[0].L
    mu = synth.potts(L)
    ctx = batch_ctx(ims, torch.float64)
    tune = ctx.autotune(L, reps=2)
    print(f"[autotune] {tune}", flush=True)
    phi = ctx.pack([T(im.unary, torch.float64) for im in ims], L)
    m = T(mu, torch.float64)
    y, _ = ctx.fw_forward(phi, m, iters)
    ys = [t.cpu().numpy() for t in ctx.unpack(y)]
    for j, im in enumerate(ims):
        sc = single_ctx(im, torch.float64)
        yj, _ = sc.fw_forward(T(im.unary, torch.float64), m, iters)
        assert np.abs(ys[j] - yj.cpu().numpy()).max() <= 1e-10, j
    for j in sorted(range(len(ims)), key=lambda j: ims[j].N)[:2]:
        im = ims[j]
        model = O.Model(im.H, im.W, im.rgb, KERNELS)
        _, yT, _, _, _ = O.fw_unrolled_loss(model, im.unary, mu, iters, im.gt)
        assert np.abs(ys[j] - yT).max() <= 1e-10, j


def test_autotune_keeps_results():
    im = synth.make("voronoi_320x213_L21")
    from paper_1608_06192_amd import dcrf
    ctx = single_ctx(im, torch.float64)
    Y = torch.rand(im.N, 21, device=dev(), dtype=torch.float64)
    before = ctx.filter(Y).cpu().numpy()
    tune = ctx.autotune(21, reps=2)
    assert tune["splat_chunk"] in (32, 64, 128)
    assert tune["dense_chunk"] in (16, 32, 64)
    assert tune["splat_stage"] in (0, 1)
    assert tune["blur_vectors_per_thread"] in (1, 2)
    assert tune["blur_group"] in (1, 2, 3)
    assert tune["tiles"] in (0, 1)
    assert tune["blur_block"] in (128, 256)
    after = ctx.filter(Y).cpu().numpy()
    assert np.abs(after - before).max() <= 1e-12 * np.abs(before).max()
    assert isinstance(ctx, dcrf.Context)


def test_batch_unsupported_calls():
    from paper_1608_06192_amd import dcrf
    ims = small_batch()
    ctx = batch_ctx(ims, torch.float64)
    phi = ctx.pack([T(im.unary, torch.float64) for im in ims], 5)
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.set_filter_mode("exact")
    assert dcrf.STATUS[e.value.status] == "DCRF_EUNSUPPORTED"
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.lp_subgradient(phi, torch.full_like(phi, 0.2))
    assert dcrf.STATUS[e.value.status] == "DCRF_EUNSUPPORTED"
