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
  GPU runs (1e-10) and, for its two smallest images, against the oracle;
* the same batch in FP32 (the benchmarked configuration), forward and
  reverse sweep, every image against the oracle and against a single-image
  FP32 context (bars in the test's docstring).
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


_ORACLE_BATCH16 = {}


def _oracle_batch16(ims, mu, iters):
    """The oracle's unrolled forward and backward for every image of the
    16-image batch, computed once per test session on a thread pool (the
    oracle's C parts release the interpreter lock). NumPy's BLAS is held to
    one thread meanwhile: its own thread pool, entered from several
    interpreter threads at once, returns wrong products (measured: an image's
    first conditional gradients differing at hundreds of pixels from a serial
    run), while the oracle's OpenMP loops are safe to run concurrently."""
    import concurrent.futures as cf
    from threadpoolctl import threadpool_limits
    if "refs" not in _ORACLE_BATCH16:
        with threadpool_limits(limits=1, user_api="blas"), cf.ThreadPoolExecutor(8) as ex:
            _ORACLE_BATCH16["refs"] = list(
                ex.map(lambda im: _oracle_unrolled(im, mu, iters), ims))
    return _ORACLE_BATCH16["refs"]


def _oracle_unrolled(im, mu, iters):
    """The oracle's FP64 unrolled forward and reverse sweep for one image:
    upstream gradient (cross entropy to the region labels), dl/dphi, dl/dw,
    the sum of the absolute values of dl/dw's summands, and the conditional
    gradients' labels of every iteration."""
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    _, yT, tape, qp, c = O.fw_unrolled_loss(model, im.unary, mu, iters, im.gt)
    ybar = O.cross_entropy_grad(yT, im.gt)
    gphi, gw, gw_abs = O.fw_unrolled_backward(qp, tape, c, ybar, scale=True)
    s = np.stack([r["s"].argmax(1) for r in tape]).astype(np.int32)
    # per iteration, the gap between the two smallest entries of the
    # oracle's gradient g = c + 2 P relative to max |g|, per pixel: where it
    # is at the level of rounding, either label is a valid conditional
    # gradient
    margin = []
    for r in tape:
        g = c + 2.0 * r["P"]
        g2 = np.partition(g, 1, axis=1)
        margin.append(((g2[:, 1] - g2[:, 0]) / np.abs(g).max(axis=1)).astype(np.float32))
    return dict(ybar=ybar, gphi=gphi, gw=gw, gw_abs=gw_abs, s=s, yT=yT,
                margin=np.stack(margin))


def _first_flips_are_near_ties(s_gpu, r, rel):
    """At the first iteration where the GPU's conditional gradients differ
    from the oracle's (before it both trajectories agree to rounding), every
    differing pixel is a near-tie of the oracle's own gradient (top-two gap
    within rel of max |g|). Returns the number of differing decisions."""
    differ = s_gpu != r["s"]
    n = int(differ.sum())
    if n:
        t = int(np.argmax(differ.any(axis=1)))
        gaps = r["margin"][t][differ[t]]
        assert (gaps <= rel).all(), (t, gaps.max())
    return n


def test_batch16_fp64_fwd_bwd_matches_oracle():
    """The benchmarked batch (16 images of U{240..500}^2, L = 21, autotuned
    launch shapes, 10 unrolled iterations, cross-entropy upstream) in FP64:
    both sides take their argmin decisions in the same precision, so the
    conditional gradients agree except at exact near-ties (top-two gap of
    the oracle's gradient within 1e-9 of its scale, checked at the first
    differing iteration; at most 10 decisions per image). Where every
    decision agrees the whole derivative must match the oracle's: y_T within
    1e-10, dl/dphi within 1e-8 of its max, dl/dw within 1e-8 relative."""
    from diffsaved import unpack_saved
    ims = synth.make_batch()
    iters = synth.WORKLOADS["voronoi_batch16_L21"]["iters"]
    L = ims[0].L
    mu = synth.potts(L)
    refs = _oracle_batch16(ims, mu, iters)
    f64 = torch.float64
    ctx = batch_ctx(ims, f64)
    ctx.autotune(L, reps=2)
    phi = ctx.pack([T(im.unary, f64) for im in ims], L)
    y, saved = ctx.fw_forward(phi, None, iters)
    gphi, gw = ctx.fw_backward(phi, None, iters, saved,
                               ctx.pack([T(r["ybar"], f64) for r in refs], L))
    s_b, _ = unpack_saved(ctx, saved, ctx.N, L, iters, 8)
    for j, (im, r, yj, gj) in enumerate(zip(ims, refs, ctx.unpack(y), ctx.unpack(gphi))):
        a, b = ctx.seg[j]
        nd = _first_flips_are_near_ties(s_b[:, a:b], r, 1e-9)
        print(f"[batch16 fp64] image {j} {im.H}x{im.W}: decisions differing {nd}",
              flush=True)
        assert nd <= 10, j
        if nd:
            continue
        assert np.abs(yj.cpu().numpy() - r["yT"]).max() <= 1e-10, j
        g = gj.cpu().numpy()
        assert np.abs(g - r["gphi"]).max() <= 1e-8 * np.abs(r["gphi"]).max(), j
        assert np.allclose(gw[j], r["gw"], rtol=1e-8, atol=0), j


def test_batch16_fp32_fwd_bwd_matches_single_and_oracle():
    """The batch configuration that bench.py times: 16 Voronoi images of
    sizes U{240..500}^2, L = 21, FP32, autotuned launch shapes, 10 unrolled
    Frank-Wolfe iterations, then the reverse sweep with the cross-entropy
    upstream gradient (the oracle's, so that both sides differentiate the
    same loss).

    Every image, from the batch and from a single-image FP32 context, against
    the FP64 oracle's unrolled backward with the bars of the single-image
    FP32 test: conditional-gradient labels differing on at most 1e-3 of the
    decisions, those of the first differing iteration all near-ties of the
    oracle's gradient (top-two gap within 1e-5 of its scale), dl/dphi within
    2e-4 in relative 2-norm (measured at most 1.2e-4: the pixels whose
    decisions flipped dominate it), dl/dw within 16 u times the sum of the absolute
    values of its summands (u = 6e-8: the weight gradient is a sum that
    cancels to 1e-2 .. 1e-4 of that absolute sum on these images). The
    derivative is also checked to 1e-8 in FP64
    (test_batch16_fp64_fwd_bwd_matches_oracle). Batch against single: the
    two differ only in the order of floating-point atomics, so the same
    decision bar, marginals within 1e-4 except on a share below 1e-3, and
    dl/dphi within 2e-4 in relative 2-norm."""
    from diffsaved import unpack_saved
    ims = synth.make_batch()
    iters = synth.WORKLOADS["voronoi_batch16_L21"]["iters"]
    L = ims[0].L
    mu = synth.potts(L)
    f32 = torch.float32
    refs = _oracle_batch16(ims, mu, iters)
    ctx = batch_ctx(ims, f32)
    tune = ctx.autotune(L, reps=2)
    print(f"[autotune] {tune}", flush=True)
    phi = ctx.pack([T(im.unary, f32) for im in ims], L)
    m = T(mu, f32)
    y, saved = ctx.fw_forward(phi, m, iters)
    ys = [t.double().cpu().numpy() for t in ctx.unpack(y)]
    ybars32 = [T(r["ybar"], f32) for r in refs]
    gphi, gw = ctx.fw_backward(phi, m, iters, saved, ctx.pack(ybars32, L))
    gphis = [t.double().cpu().numpy() for t in ctx.unpack(gphi)]
    s_b, _ = unpack_saved(ctx, saved, ctx.N, L, iters, 4)
    for j, (im, r) in enumerate(zip(ims, refs)):
        a, b = ctx.seg[j]
        sc = single_ctx(im, f32)
        ph = T(im.unary, f32)
        y1, sv1 = sc.fw_forward(ph, m, iters)
        g1, w1 = sc.fw_backward(ph, m, iters, sv1, ybars32[j])
        s_1, _ = unpack_saved(sc, sv1, im.N, L, iters, 4)
        y1 = y1.double().cpu().numpy()
        g1 = g1.double().cpu().numpy()
        bound_w = 16 * 6e-8 * r["gw_abs"]
        nd = iters * im.N
        for name, s_x, g_x, w_x in (("batch", s_b[:, a:b], gphis[j], gw[j]),
                                    ("single", s_1, g1, w1)):
            d_o = _first_flips_are_near_ties(s_x, r, 1e-5)
            e_phi = np.linalg.norm(g_x - r["gphi"]) / np.linalg.norm(r["gphi"])
            err_w = np.abs(np.array(w_x) - r["gw"])
            print(f"[batch16 fp32] image {j} {im.H}x{im.W} {name} vs oracle: "
                  f"decisions differing {d_o}, dphi rel {e_phi:.2e}, dw err "
                  f"{err_w} bound {bound_w}", flush=True)
            assert d_o <= 1e-3 * nd, (j, name)
            assert e_phi <= 2e-4, (j, name)
            assert (err_w <= bound_w).all(), (j, name)
        differ = int((s_b[:, a:b] != s_1).sum())
        share = float((np.abs(ys[j] - y1) > 1e-4).mean())
        e_phi = np.linalg.norm(gphis[j] - g1) / np.linalg.norm(g1)
        print(f"[batch16 fp32] image {j} batch vs single: decisions differing "
              f"{differ}, y share>1e-4 {share:.2e}, dphi rel {e_phi:.2e}", flush=True)
        assert differ <= 1e-3 * nd, j
        assert share <= 1e-3, j
        assert e_phi <= 2e-4, j


def test_batch_summed_weight_gradient():
    # the library's sum over the images equals the per-image gradients
    ims = small_batch()
    L, iters = 5, 6
    ctx = batch_ctx(ims, torch.float64)
    phi = ctx.pack([T(im.unary, torch.float64) for im in ims], L)
    y, saved = ctx.fw_forward(phi, None, iters)
    ybar = torch.randn(y.shape, generator=torch.Generator().manual_seed(5),
                       dtype=torch.float64).to(dev())
    g1, per = ctx.fw_backward(phi, None, iters, saved, ybar)
    g2, tot = ctx.fw_backward(phi, None, iters, saved, ybar, summed=True)
    # two reverse sweeps: equal up to the order of their atomic additions
    # (compared on the images' rows; the rows between images are unspecified)
    for a1, a2 in zip(ctx.unpack(g1), ctx.unpack(g2)):
        assert (a1 - a2).abs().max().item() <= 1e-10 * a1.abs().max().item()
    for m in range(ctx.nk):
        acc = sum(per[j][m] for j in range(len(ims)))
        assert abs(tot[m] - acc) <= 1e-10 * sum(abs(per[j][m]) for j in range(len(ims)))


def test_batch_per_image_calls_match_packed():
    # dcrf_batch_fw_forward / _backward take one array per image and copy
    # them to and from the packed layout: their results are the packed
    # calls' (up to the rounding order of the step-size atomics)
    from paper_1608_06192_amd import dcrf
    ims = [synth.voronoi_image(h, w, 4, seed=40 + j, regions=5)
           for j, (h, w) in enumerate([(20, 30), (17, 23), (25, 19)])]
    ctx = dcrf.Context(0)
    print("[case] per-image batch calls", flush=True)
    ctx.set_images([(x.H, x.W) for x in ims], [torch.from_numpy(x.rgb).to(dev()) for x in ims],
                   KERNELS, dtype=torch.float64)
    phis = [torch.from_numpy(x.unary).to(dev()) for x in ims]
    packed = ctx.pack(phis, 4)
    y, saved = ctx.fw_forward(packed, None, 6)
    ys, saved2 = ctx.batch_fw_forward(phis, None, 6)
    rng = np.random.default_rng(41)
    gys = [torch.from_numpy(rng.normal(size=(x.N, 4))).to(dev()) for x in ims]
    gp, gw = ctx.fw_backward(packed, None, 6, saved, ctx.pack(gys, 4))
    gps, gws, gtot = ctx.batch_fw_backward(phis, None, 6, saved2, gys)
    for j, (a, b) in enumerate(ctx.seg):
        assert (ys[j] - y[a:b]).abs().max().item() <= 1e-12, j
        assert (gps[j] - gp[a:b]).abs().max().item() <= 1e-12 * gp[a:b].abs().max().item(), j
        assert np.allclose(gws[j], gw[j], rtol=1e-12, atol=0), j
    assert np.allclose(gtot, np.sum(gws, axis=0), rtol=1e-14, atol=0)


def _persistent_vs_stages(ctx, run, tune=None):
    """run(ctx) with one launch per stage and with the persistent launch,
    the other launch shapes as in `tune` (default: the defaults)"""
    t = dict(tune or {})
    ctx.set_tune(**dict(t, fw_persistent=0))
    a = run(ctx)
    ctx.set_tune(**dict(t, fw_persistent=1))
    b = run(ctx)
    ctx.set_tune(**dict(t, fw_persistent=0))
    return a, b


def test_persistent_fw_fp64_matches_per_stage_small_batch():
    # the same solve (3 images of uneven sizes, L = 5, 20 iterations, FP64)
    # in one cooperative launch with grid barriers and with one launch per
    # stage: the same arithmetic up to the order of the splat's atomics, so
    # the marginals and every per-image trace entry agree to 1e-10
    ims = small_batch()
    ctx = batch_ctx(ims, torch.float64)
    L = ims[0].L
    phi = ctx.pack([T(im.unary, torch.float64) for im in ims], L)
    y0 = ctx.pack([T(O.softmax_neg(im.unary), torch.float64) for im in ims], L)

    def run(c):
        y = y0.clone()
        tr = c.qp_frank_wolfe(phi, None, y, 20)
        return y.cpu().numpy(), np.asarray(tr, dtype=np.float64)
    (ya, ta), (yb, tb) = _persistent_vs_stages(ctx, run)
    print(f"[persistent small] max |dy| {np.abs(ya - yb).max():.3g}", flush=True)
    assert np.abs(ya - yb).max() <= 1e-10
    assert np.abs(ta - tb).max() <= 1e-10 * np.abs(ta).max()


def test_persistent_fw_fp64_single_image_500x375():
    # one image at the benchmarked size, 30 iterations in FP64, both paths
    from paper_1608_06192_amd import dcrf
    im = synth.make("voronoi_500x375_L21")
    ctx = dcrf.Context(0)
    ctx.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev()), KERNELS,
                  dtype=torch.float64)
    print("[case] persistent 500x375 fp64", flush=True)
    phi = T(im.unary, torch.float64)
    y0 = T(O.softmax_neg(im.unary), torch.float64)

    def run(c):
        y = y0.clone()
        tr = c.qp_frank_wolfe(phi, None, y, 30)
        return y.cpu().numpy(), np.asarray(tr, dtype=np.float64)
    (ya, ta), (yb, tb) = _persistent_vs_stages(ctx, run)
    print(f"[persistent 500x375] max |dy| {np.abs(ya - yb).max():.3g}", flush=True)
    assert np.abs(ya - yb).max() <= 1e-9
    assert np.abs(ta[:, 0] - tb[:, 0]).max() <= 1e-10 * np.abs(ta[:, 0]).max()


def test_persistent_fw_fwd_bwd_fp64_batch16_matches_per_stage():
    """The benchmarked 16-image batch (U{240..500}^2, L = 21, autotuned launch
    shapes with two blur directions per group, the staged splat and no
    tiles, 10 unrolled iterations with checkpoints, then the reverse sweep)
    in FP64 with the forward in one persistent launch and with one launch per
    stage. Where both take the same conditional gradients (FP64 on both
    sides; a differing decision can only come from an exact near-tie, and
    such an image is skipped, at most 2 of 16) y_T and dl/dphi agree within
    1e-10 of their scale and dl/dw, a sum whose terms cancel to about 1e-4 of
    their absolute sum, within 1e-8 relative (the bar of the oracle
    comparison above)."""
    from diffsaved import unpack_saved
    ims = synth.make_batch()
    iters = synth.WORKLOADS["voronoi_batch16_L21"]["iters"]
    L = ims[0].L
    f64 = torch.float64
    ctx = batch_ctx(ims, f64)
    # autotuned shapes, with those the persistent launch takes
    tune = dict(ctx.autotune(L, reps=2), blur_group=2, tiles=0, splat_stage=1)
    phi = ctx.pack([T(im.unary, f64) for im in ims], L)
    rng = np.random.default_rng(3)
    ybar = ctx.pack([T(rng.standard_normal((im.N, L)), f64) for im in ims], L)

    def run(c):
        y, saved = c.fw_forward(phi, None, iters)
        gphi, gw = c.fw_backward(phi, None, iters, saved, ybar)
        s_b, _ = unpack_saved(c, saved, c.N, L, iters, 8)
        return [v.cpu().numpy() for v in c.unpack(y)], \
            [v.cpu().numpy() for v in c.unpack(gphi)], np.asarray(gw), s_b.copy()
    (ya, ga, wa, sa), (yb, gb, wb, sb) = _persistent_vs_stages(ctx, run, tune)
    skipped, wrel = 0, 0.0
    for j in range(len(ims)):
        a, b = ctx.seg[j]
        if not np.array_equal(sa[:, a:b], sb[:, a:b]):
            skipped += 1
            continue
        assert np.abs(ya[j] - yb[j]).max() <= 1e-10, j
        assert np.abs(ga[j] - gb[j]).max() <= 1e-10 * np.abs(ga[j]).max(), j
        wrel = max(wrel, float(np.max(np.abs(wa[j] - wb[j]) / np.abs(wa[j]))))
        assert np.allclose(wa[j], wb[j], rtol=1e-8, atol=0), j
    print(f"[persistent batch16] images skipped for a differing decision: {skipped}; "
          f"dl/dw max rel diff {wrel:.3g}", flush=True)
    assert skipped <= 2
