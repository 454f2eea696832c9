"""GPU parity: the HIP library against the FP64 oracle, through the C ABI.

Tolerances (written next to each check):
* lattice vertex sets and per-pixel vertex keys: bit-exact; weights
  bit-exact in FP64 and equal to the FP64 weight rounded once in FP32;
* filter outputs: |gpu - oracle| <= rtol * (K~|Y| + wsum |Y|) elementwise, i.e.
  relative to the magnitude of the summands (rtol 1e-5 in FP32, 1e-11 in FP64);
* Frank-Wolfe marginals within 1e-4 absolute and objectives within 1e-4
  relative; energies within 1e-5 relative (FP32) / 1e-10 (FP64).
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


def gpu_ctx(im, dtype, kernels=KERNELS, mode="lattice"):
    from paper_1608_06192_amd import dcrf
    print(f"[case] {im.H}x{im.W} dtype={dtype} mode={mode}", flush=True)
    ctx = dcrf.Context(0)
    ctx.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev()), kernels,
                  dtype=dtype)
    if mode != "lattice":
        ctx.set_filter_mode(mode)
    return ctx


def T(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev(), dtype)


def key_table(keys, vid, w):
    """per pixel: sorted list of (vertex key, weight) with weight > 0"""
    out = []
    for a in range(vid.shape[0]):
        out.append(sorted((tuple(keys[v]), float(w[a, k]))
                          for k, v in enumerate(vid[a]) if v >= 0))
    return out


def filter_bound(model, Y, rtol):
    Ya = np.abs(Y)
    return rtol * (model.Kp(Ya) + 2 * model.w.sum() * Ya) + 1e-300


@pytest.mark.parametrize("name,dtype", [("rect_32x24_L3", torch.float64),
                                        ("voronoi_320x213_L21", torch.float32)])
def test_vertex_sets_match_oracle(name, dtype):
    im = synth.make(name)
    ctx = gpu_ctx(im, dtype)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    for m, lat in enumerate(model.lattices):
        d, M = ctx.lattice_info(m)
        assert d == lat.d and M == lat.nv
        gk, gv, gw = ctx.lattice_export(m)
        ok = lat.keys()
        assert set(map(tuple, gk)) == set(map(tuple, ok))
        ov, ow = lat.points()
        if dtype == torch.float32:
            ow = ow.astype(np.float32).astype(np.float64)
        sample = np.arange(0, im.N, max(1, im.N // 4000))
        gt = key_table(gk, gv[sample], gw[sample])
        ot = key_table(ok, ov[sample], ow[sample])
        assert gt == ot


@pytest.mark.parametrize("name,dtype,C,rtol", [
    ("rect_32x24_L3", torch.float64, 3, 1e-11),
    ("rect_32x24_L3", torch.float64, 1, 1e-11),
    ("voronoi_320x213_L21", torch.float32, 21, 1e-5),
    ("voronoi_320x213_L21", torch.float32, 5, 1e-5),
    ("voronoi_500x375_L21", torch.float32, 21, 1e-5),
])
def test_filter_matches_oracle_lattice(name, dtype, C, rtol):
    im = synth.make(name)
    ctx = gpu_ctx(im, dtype)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    rng = np.random.default_rng(C)
    Y = rng.uniform(-1, 1, size=(im.N, C))
    if dtype == torch.float32:
        Y = Y.astype(np.float32).astype(np.float64)
    bound = filter_bound(model, Y, rtol)
    for adjoint in (False, True):
        g = ctx.filter(T(Y, dtype), adjoint=adjoint).cpu().numpy()
        o = model.Kp(Y, reverse=adjoint)
        assert (np.abs(g - o) <= bound).all(), (adjoint, np.abs(g - o).max())


def test_filter_exact_matches_oracle_exact():
    im = synth.make("rect_32x24_L3")
    ctx = gpu_ctx(im, torch.float64)
    model = O.Model(im.H, im.W, im.rgb, KERNELS, mode="exact")
    Y = np.random.default_rng(1).uniform(-1, 1, size=(im.N, 11))
    g = ctx.filter(T(Y, torch.float64), exact=True).cpu().numpy()
    assert np.abs(g - model.Kp(Y)).max() <= 1e-11 * np.abs(model.Kp(np.abs(Y))).max()


@pytest.mark.parametrize("H,W", [(1, 1), (1, 2), (3, 5), (7, 1), (17, 13)])
def test_filter_small_and_ragged_images(H, W):
    im = synth.voronoi_image(H, W, 4, seed=H * 100 + W, regions=3)
    ctx = gpu_ctx(im, torch.float64)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    Y = np.random.default_rng(2).uniform(0, 1, size=(im.N, 4))
    g = ctx.filter(T(Y, torch.float64)).cpu().numpy()
    assert np.abs(g - model.Kp(Y)).max() <= 1e-11 * (1 + np.abs(model.Kp(Y)).max())


@pytest.mark.parametrize("name,dtype,rtol", [
    ("rect_32x24_L3", torch.float64, 1e-11),
    ("voronoi_320x213_L21", torch.float32, 1e-5)])
def test_qp_apply_matches_oracle(name, dtype, rtol):
    im = synth.make(name)
    ctx = gpu_ctx(im, dtype)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    mu = synth.potts(im.L)
    qp = O.QP(model, im.unary, mu)
    y = O.softmax_neg(im.unary)
    if dtype == torch.float32:
        y = y.astype(np.float32).astype(np.float64)
    g = ctx.qp_apply(T(y, dtype), T(mu, dtype)).cpu().numpy()
    o = qp.Q(y)
    scale = np.abs(qp.Q(np.abs(y))) + np.abs(qp.d) * np.abs(y)
    assert (np.abs(g - o) <= rtol * (scale + 1e-30)).all()


@pytest.mark.parametrize("mode", ["lattice", "exact", "separable"])
def test_fw_fp64_matches_oracle(mode):
    # 32x24, L = 3, FP64, 20 iterations, seed 0
    im = synth.make("rect_32x24_L3")
    ctx = gpu_ctx(im, torch.float64, mode=mode)
    mu = synth.potts(im.L)
    model = O.Model(im.H, im.W, im.rgb, KERNELS, mode=mode)
    qp = O.QP(model, im.unary, mu)
    y0 = O.softmax_neg(im.unary)
    st = O.frank_wolfe(qp, y0, 20)
    y = T(y0, torch.float64)
    tr = ctx.qp_frank_wolfe(T(im.unary, torch.float64), T(mu, torch.float64),
                            y, 20)
    yg = y.cpu().numpy()
    assert np.abs(yg - st.y).max() < 1e-9
    for (fo, go, ao), (fg, gg, ag, _) in zip(st.trace, tr):
        assert abs(fg - fo) <= 1e-9 * abs(fo)
        assert abs(ag - ao) <= 1e-8
        assert abs(gg - go) <= 1e-9 * abs(fo)
    lab = ctx.round(y)
    assert (lab.cpu().numpy() == O.round_argmax(st.y)).all()
    e = ctx.energy(T(im.unary, torch.float64), T(mu, torch.float64), lab)
    eo = O.energy(model, im.unary, mu, O.round_argmax(st.y))
    assert abs(e - eo) <= 1e-10 * abs(eo)


WIDE = dict(use_rgb=1, theta_pos=20.0, theta_rgb=30.0, weight=2.0)


@pytest.mark.parametrize("kernels", [[synth.BILATERAL], [synth.SPATIAL, synth.BILATERAL],
                                     [synth.BILATERAL, synth.SPATIAL, WIDE]])
@pytest.mark.parametrize("fw_splat", [0, 1])
def test_fw_fp64_kernel_layouts_and_splat_paths(kernels, fw_splat):
    # the one-hot splat inside the conditional-gradient kernel for lattice
    # sets other than (5-D, 2-D) (one lattice, the pair in the other order,
    # three lattices) and the splat launch of its own: 37x29 (a ragged last
    # tile), L = 5, 20 iterations in FP64 against the oracle
    im = synth.voronoi_image(37, 29, 5, seed=11, regions=6)
    ctx = gpu_ctx(im, torch.float64, kernels=kernels)
    ctx.set_tune(fw_splat=fw_splat)
    mu = synth.potts(im.L)
    model = O.Model(im.H, im.W, im.rgb, [O.Kernel(**k) for k in kernels])
    qp = O.QP(model, im.unary, mu)
    y0 = O.softmax_neg(im.unary)
    st = O.frank_wolfe(qp, y0, 20)
    y = T(y0, torch.float64)
    tr = ctx.qp_frank_wolfe(T(im.unary, torch.float64), T(mu, torch.float64), y, 20)
    assert np.abs(y.cpu().numpy() - st.y).max() < 1e-9
    for (fo, _, ao), (fg, _, ag, _) in zip(st.trace, tr):
        assert abs(fg - fo) <= 1e-9 * abs(fo)
        assert abs(ag - ao) <= 1e-8


def test_fw_fused_and_separate_splat_agree_500x375():
    # the bench workload (500x375, L = 21, 5-D + 2-D lattices) in FP64, 30
    # iterations with the splat inside the conditional-gradient kernel and
    # with a splat launch of its own (the default): the same arithmetic up
    # to the order of the splat's sums, so the trajectories agree to 1e-9
    im = synth.make("voronoi_500x375_L21")
    phi = T(im.unary, torch.float64)
    mu = T(synth.potts(im.L), torch.float64)
    y0 = O.softmax_neg(im.unary)
    out = []
    for fw_splat in (1, 0):
        ctx = gpu_ctx(im, torch.float64)
        ctx.set_tune(fw_splat=fw_splat)
        y = T(y0, torch.float64)
        tr = ctx.qp_frank_wolfe(phi, mu, y, 30)
        out.append((y.cpu().numpy(), tr))
    (ya, ta), (yb, tb) = out
    print(f"[fw splat paths] max |dy| {np.abs(ya - yb).max():.3g}", flush=True)
    assert np.abs(ya - yb).max() < 1e-9
    for ra, rb in zip(ta, tb):
        assert abs(ra[0] - rb[0]) <= 1e-9 * abs(rb[0])


def test_fw_fp64_matches_oracle_320x213():
    # 320x213, L = 21, 50 iterations in FP64 on both sides: every argmin is
    # decided in the same precision, so the whole trajectory must agree
    im = synth.make("voronoi_320x213_L21")
    ctx = gpu_ctx(im, torch.float64)
    mu = synth.potts(im.L)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    qp = O.QP(model, im.unary, mu)
    y0 = O.softmax_neg(im.unary)
    st = O.frank_wolfe(qp, y0, 50)
    y = T(y0, torch.float64)
    tr = ctx.qp_frank_wolfe(T(im.unary, torch.float64), T(mu, torch.float64),
                            y, 50)
    err = np.abs(y.cpu().numpy() - st.y).max()
    print("max |y_gpu - y_oracle| =", err)
    assert err < 1e-8
    for (fo, go, ao), (fg, gg, ag, _) in zip(st.trace, tr):
        assert abs(fg - fo) <= 1e-9 * abs(fo)
        assert abs(ag - ao) <= 1e-7


def _eps_argmin_ok(g, s, rel=1e-5):
    """s[a] is a valid conditional gradient of g up to FP32 rounding: its
    gradient is within rel * scale of the minimum (scale = row max |g|)."""
    gmin = g.min(axis=1)
    scale = np.abs(g).max(axis=1)
    return g[np.arange(g.shape[0]), s] <= gmin + rel * scale


@pytest.mark.parametrize("t0", [0, 10, 30])
def test_fw_fp32_step_matches_oracle_320x213(t0):
    # one FP32 GPU iteration from the oracle's iterate y_t0 (rounded to FP32):
    # the conditional gradient must be a valid argmin of the oracle's
    # gradient at every pixel, and the step size must agree
    im = synth.make("voronoi_320x213_L21")
    ctx = gpu_ctx(im, torch.float32)
    mu = synth.potts(im.L)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    qp = O.QP(model, im.unary, mu)
    yt = O.frank_wolfe(qp, O.softmax_neg(im.unary), t0).y
    yt = yt.astype(np.float32).astype(np.float64)
    yt /= yt.sum(axis=1, keepdims=True)
    yt = yt.astype(np.float32).astype(np.float64)
    st = O.frank_wolfe(qp, yt, 1)
    g = qp.phi - qp.d + 2 * qp.Q(yt)
    y = T(yt, torch.float32)
    tr = ctx.qp_frank_wolfe(T(im.unary, torch.float32), T(mu, torch.float32),
                            y, 1)
    ag = tr[0][2]
    y1 = y.cpu().numpy().astype(np.float64)
    s_gpu = np.argmax(y1 - (1 - ag) * yt, axis=1)
    s_or = st.s_hist[0]
    ok = _eps_argmin_ok(g, s_gpu)
    print(f"t0={t0} alpha gpu={ag:.6g} oracle={st.alphas[0]:.6g} "
          f"s differs at {(s_gpu != s_or).sum()} pixels")
    assert ok.all()
    assert abs(ag - st.alphas[0]) <= 1e-4 * max(1.0, abs(st.alphas[0]))
    assert abs(tr[0][0] - st.trace[0][0]) <= 1e-5 * abs(st.trace[0][0])
    same = s_gpu == s_or
    assert np.abs(y1[same] - st.y[same]).max() < 1e-4


def test_fw_fp32_trajectory_320x213():
    # 320x213, L = 21, FP32 marginals, 50 iterations. FP32 and FP64 may take
    # different (equally valid) conditional gradients at near-ties, so the
    # trajectories are compared through objectives, energies and the share of
    # marginals that agree to 1e-4.
    im = synth.make("voronoi_320x213_L21")
    ctx = gpu_ctx(im, torch.float32)
    mu = synth.potts(im.L)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    qp = O.QP(model, im.unary, mu)
    y0 = O.softmax_neg(im.unary).astype(np.float32).astype(np.float64)
    st = O.frank_wolfe(qp, y0, 50)
    y = T(y0, torch.float32)
    tr = ctx.qp_frank_wolfe(T(im.unary, torch.float32), T(mu, torch.float32),
                            y, 50)
    yg = y.cpu().numpy().astype(np.float64)
    diff = np.abs(yg - st.y)
    print(f"max |dy| = {diff.max():.3g}, share > 1e-4: {(diff > 1e-4).mean():.3g}")
    assert (diff > 1e-4).mean() < 1e-3
    for (fo, _, _), (fg, _, _, _) in zip(st.trace, tr):
        assert abs(fg - fo) <= 1e-4 * abs(fo)
    lab = ctx.round(y)
    e = ctx.energy(T(im.unary, torch.float32), T(mu, torch.float32), lab)
    eo_same = O.energy(model, im.unary, mu, lab.cpu().numpy())
    assert abs(e - eo_same) <= 1e-5 * abs(eo_same)
    eo = O.energy(model, im.unary, mu, O.round_argmax(st.y))
    print(f"energy gpu {e:.8g} oracle {eo:.8g}")
    assert abs(e - eo) <= 1e-4 * abs(eo)


def test_fw_fp32_500x375_bench_configuration():
    # the workload and launch shapes that bench.py times (default tuning):
    # 500x375, L = 21, FP32, 50 iterations from softmax(-phi). Objectives
    # follow the oracle's FP64 trajectory within 1e-4 relative; the marginals
    # stay on the simplex, and FP32 near-ties may change a few conditional
    # gradients, so only the share of marginals off by more than 1e-4 is
    # bounded (as at 320x213)
    im = synth.make("voronoi_500x375_L21")
    ctx = gpu_ctx(im, torch.float32)
    mu = synth.potts(im.L)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    qp = O.QP(model, im.unary, mu)
    y0 = O.softmax_neg(im.unary).astype(np.float32).astype(np.float64)
    st = O.frank_wolfe(qp, y0, 50)
    y = T(y0, torch.float32)
    tr = ctx.qp_frank_wolfe(T(im.unary, torch.float32), T(mu, torch.float32),
                            y, 50)
    yg = y.cpu().numpy().astype(np.float64)
    assert np.abs(yg.sum(axis=1) - 1.0).max() < 1e-5
    assert yg.min() >= -1e-7
    diff = np.abs(yg - st.y)
    print(f"max |dy| = {diff.max():.3g}, share > 1e-4: {(diff > 1e-4).mean():.3g}")
    assert (diff > 1e-4).mean() < 1e-3
    assert len(tr) == 50
    for (fo, _, _), (fg, _, _, _) in zip(st.trace, tr):
        assert abs(fg - fo) <= 1e-4 * abs(fo)


def test_fw_fp32_steps_500x375_bench_configuration():
    # the timed workload (500x375, L = 21, FP32, default launch shapes), one
    # GPU iteration from each oracle iterate y_t0, t0 = 0, 5, ..., 45 (rounded
    # to FP32 and renormalised, the same start on both sides). At every pixel
    # the GPU's conditional gradient must be a valid argmin of the oracle's
    # gradient at that point (up to FP32 rounding of the gradient), and the
    # step size and objective must agree: alpha within 1e-4, f within 1e-5
    # relative. A GPU that mislabels any pixel fails here, whatever the
    # share of pixels involved.
    im = synth.make("voronoi_500x375_L21")
    ctx = gpu_ctx(im, torch.float32)
    mu = synth.potts(im.L)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    qp = O.QP(model, im.unary, mu)
    starts = {}
    y = O.softmax_neg(im.unary)
    Py = qp.Q(y)
    c = qp.phi - qp.d
    for t in range(46):
        if t % 5 == 0:
            starts[t] = y.copy()
        s = O.onehot(np.argmin(c + 2.0 * Py, axis=1), im.L)
        Ps = qp.Q(s)
        al, _, _ = O.fw_step_size(c, y, s, Py, Ps)
        y = y + al * (s - y)
        Py = (1.0 - al) * Py + al * Ps
    phi = T(im.unary, torch.float32)
    mu_t = T(mu, torch.float32)
    for t0, yt in starts.items():
        yt = yt.astype(np.float32).astype(np.float64)
        yt /= yt.sum(axis=1, keepdims=True)
        yt = yt.astype(np.float32).astype(np.float64)
        ref = O.frank_wolfe(qp, yt, 1)
        g = c + 2.0 * qp.Q(yt)
        yg = T(yt, torch.float32)
        tr = ctx.qp_frank_wolfe(phi, mu_t, yg, 1)
        ag = tr[0][2]
        y1 = yg.cpu().numpy().astype(np.float64)
        # s from y1 = (1 - alpha) y + alpha s; alpha >> FP32 rounding here
        assert ag > 1e-4, (t0, ag)
        s_gpu = np.argmax(y1 - (1 - ag) * yt, axis=1)
        s_or = ref.s_hist[0]
        ok = _eps_argmin_ok(g, s_gpu)
        fo = ref.trace[0][0]
        print(f"[fw step 500x375] t0={t0} alpha gpu={ag:.6g} oracle={ref.alphas[0]:.6g}"
              f" f rel err {abs(tr[0][0] - fo) / abs(fo):.2e}; s differs at "
              f"{(s_gpu != s_or).sum()} pixels, non-argmin {(~ok).sum()}", flush=True)
        assert ok.all(), t0
        assert abs(ag - ref.alphas[0]) <= 1e-4 * max(1.0, abs(ref.alphas[0])), t0
        assert abs(tr[0][0] - fo) <= 1e-5 * abs(fo), t0
        same = s_gpu == s_or
        assert np.abs(y1[same] - ref.y[same]).max() < 1e-4, t0


@pytest.mark.parametrize("L,general_mu", [(3, True), (32, False), (40, False),
                                          (40, True)])
def test_fw_fp64_label_counts_and_general_mu(L, general_mu):
    # 32 labels: the largest per-thread register rows; 40: one lane per
    # (pixel, label); a general (non-Potts) symmetric compatibility
    im = synth.voronoi_image(19, 23, L, seed=40 + L, regions=5)
    ctx = gpu_ctx(im, torch.float64)
    rng = np.random.default_rng(L)
    if general_mu:
        mu = rng.uniform(0.2, 2.0, size=(L, L))
        mu = 0.5 * (mu + mu.T)
        np.fill_diagonal(mu, 0.0)
    else:
        mu = synth.potts(L)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    qp = O.QP(model, im.unary, mu)
    y0 = O.softmax_neg(im.unary)
    st = O.frank_wolfe(qp, y0, 8)
    y = T(y0, torch.float64)
    tr = ctx.qp_frank_wolfe(T(im.unary, torch.float64), T(mu, torch.float64),
                            y, 8)
    assert np.abs(y.cpu().numpy() - st.y).max() < 1e-9
    for (fo, _, ao), (fg, _, ag, _) in zip(st.trace, tr):
        assert abs(fg - fo) <= 1e-9 * abs(fo)
        assert abs(ag - ao) <= 1e-8
    g = ctx.filter(T(im.unary, torch.float64)).cpu().numpy()
    assert np.abs(g - model.Kp(im.unary)).max() <= 1e-10 * np.abs(g).max()


def test_energy_random_labels():
    im = synth.make("voronoi_320x213_L21")
    ctx = gpu_ctx(im, torch.float32)
    mu = synth.potts(im.L)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    x = np.random.default_rng(3).integers(0, im.L, size=im.N).astype(np.int32)
    e = ctx.energy(T(im.unary, torch.float32), T(mu, torch.float32),
                   torch.from_numpy(x).to(dev()))
    assert abs(e - O.energy(model, im.unary, mu, x)) <= 1e-5 * abs(e)


def test_dc_gen_fp64_matches_oracle():
    im = synth.make("rect_32x24_L3")
    ctx = gpu_ctx(im, torch.float64)
    mu = synth.potts(im.L)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    qp = O.QP(model, im.unary, mu)
    y0 = O.frank_wolfe(qp, O.softmax_neg(im.unary), 10).y
    yo, ho = O.dc_gen(qp, y0, outer=4, inner=5)
    y = T(y0, torch.float64)
    hg = ctx.dc_gen(T(im.unary, torch.float64), T(mu, torch.float64), y, 4, 5)
    assert np.abs(y.cpu().numpy() - yo).max() < 1e-9
    assert np.allclose(hg, ho, rtol=1e-9, atol=0)


def test_dc_gen_fp32_matches_oracle_320x213():
    # the configuration bench.py times for DC_gen: 320x213, L = 21, FP32,
    # 5 concave-convex steps of 10 Frank-Wolfe iterations from the oracle's
    # 50-iteration QP solution (rounded to FP32, the same start on both
    # sides). The S history follows the oracle's within 1e-4 relative, and
    # the rounded labelling's energy within 1e-4 of the oracle's.
    im = synth.make("voronoi_320x213_L21")
    ctx = gpu_ctx(im, torch.float32)
    mu = synth.potts(im.L)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    qp = O.QP(model, im.unary, mu)
    y0 = O.frank_wolfe(qp, O.softmax_neg(im.unary), 50).y
    y0 = y0.astype(np.float32).astype(np.float64)
    yo, ho = O.dc_gen(qp, y0, outer=5, inner=10)
    y = T(y0, torch.float32)
    hg = ctx.dc_gen(T(im.unary, torch.float32), T(mu, torch.float32), y, 5, 10)
    print("S gpu", hg, "oracle", ho)
    for a, b in zip(hg, ho):
        assert abs(a - b) <= 1e-4 * abs(b)
    assert all(b2 <= b1 + 1e-4 * abs(b1) for b1, b2 in zip(hg, hg[1:]))   # CCCP decreases S
    lab = ctx.round(y)
    e = ctx.energy(T(im.unary, torch.float32), T(mu, torch.float32), lab)
    eo = O.energy(model, im.unary, mu, O.round_argmax(yo))
    print(f"energy gpu {e:.8g} oracle {eo:.8g}")
    assert abs(e - eo) <= 1e-4 * abs(eo)


def test_errors_are_reported_not_fatal():
    from paper_1608_06192_amd import dcrf
    im = synth.make("rect_32x24_L3")
    ctx = gpu_ctx(im, torch.float64)
    mu = T(synth.potts(3), torch.float64)
    bad = torch.full((im.N,), 7, dtype=torch.int32, device=dev())
    with pytest.raises(dcrf.DcrfError) as ei:
        ctx.energy(T(im.unary, torch.float64), mu, bad)
    assert ei.value.status == -1
    with pytest.raises(dcrf.DcrfError) as ei:
        ctx.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev()),
                      [dict(use_rgb=1, theta_pos=0.0, theta_rgb=13, weight=1)])
    assert ei.value.status == -1
    with pytest.raises(dcrf.DcrfError) as ei:
        # tiny theta: coordinates beyond the vertex key range
        ctx.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev()),
                      [dict(use_rgb=1, theta_pos=80, theta_rgb=0.01, weight=1)])
    assert ei.value.status == -3
    # the context stays usable
    ctx.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev()), KERNELS,
                  dtype=torch.float64)
    x = torch.zeros(im.N, dtype=torch.int32, device=dev())
    ctx.energy(T(im.unary, torch.float64), mu, x)


@pytest.mark.parametrize("tune", [
    dict(splat_chunk=16, blur_vectors_per_thread=1, blur_block=64, blur_group=1,
         dense_chunk=16),
    dict(splat_chunk=128, blur_vectors_per_thread=2, blur_block=128, blur_group=2,
         dense_chunk=128),
    dict(splat_chunk=64, blur_vectors_per_thread=1, blur_block=256, blur_group=2,
         dense_chunk=256),
    dict(splat_chunk=64, blur_vectors_per_thread=1, blur_block=256, blur_group=2,
         dense_chunk=32, splat_stage=0),
    dict(splat_chunk=64, blur_vectors_per_thread=1, blur_block=256, blur_group=2,
         dense_chunk=64, splat_stage=1),
    dict(splat_chunk=256, blur_vectors_per_thread=4, blur_block=256, blur_group=3),
    dict(splat_chunk=32, blur_vectors_per_thread=3, blur_block=256, blur_group=3),
    dict(splat_chunk=64, blur_vectors_per_thread=1, blur_block=256, blur_group=2,
         tiles=1),
    dict(splat_chunk=64, blur_vectors_per_thread=2, blur_block=128, blur_group=1,
         tiles=1),
])
@pytest.mark.parametrize("name,dtype,rtol", [("rect_32x24_L3", torch.float64, 1e-11),
                                              ("voronoi_320x213_L21", torch.float32, 1e-5)])
def test_launch_shapes_keep_filter_parity(tune, name, dtype, rtol):
    """Every launch shape (splat chunk length, blur directions per launch,
    vectors per thread, block size) gives the oracle's filter, both ways."""
    im = synth.make(name)
    ctx = gpu_ctx(im, dtype)
    ctx.set_tune(**tune)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    rng = np.random.default_rng(11)
    Y = rng.uniform(-1, 1, size=(im.N, 5))
    for adjoint in (False, True):
        got = ctx.filter(T(Y, dtype), adjoint=adjoint).double().cpu().numpy()
        ref = model.Kp(Y, reverse=adjoint)
        assert (np.abs(got - ref) <= filter_bound(model, Y, rtol)).all(), adjoint


@pytest.mark.parametrize("tiles", [0, 1])
def test_grouped_blur_fw_fp64_matches_oracle(tiles):
    im = synth.make("rect_32x24_L3")
    ctx = gpu_ctx(im, torch.float64)
    ctx.set_tune(splat_chunk=32, blur_vectors_per_thread=2, blur_block=128,
                 blur_group=3, tiles=tiles)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    mu = synth.potts(3)
    qp = O.QP(model, im.unary, mu)
    e = np.exp(-(im.unary - im.unary.min(axis=1, keepdims=True)))
    y0 = e / e.sum(axis=1, keepdims=True)
    st = O.frank_wolfe(qp, y0, 20)
    y = T(y0, torch.float64)
    ctx.qp_frank_wolfe(T(im.unary, torch.float64), T(mu, torch.float64), y, 20)
    assert np.abs(y.cpu().numpy() - st.y).max() <= 1e-10


def test_null_mu_is_potts():
    # a null mu stands for Potts: the same kernels run as for an explicit
    # Potts mu. Results agree to FP64 rounding (the splat's atomics add in a
    # run-dependent order, so bitwise equality is not expected)
    im = synth.make("voronoi_320x213_L21")
    ctx = gpu_ctx(im, torch.float64)
    phi = T(im.unary, torch.float64)
    mu = T(synth.potts(im.L), torch.float64)
    y0 = T(O.softmax_neg(im.unary), torch.float64)
    ya, yb = y0.clone(), y0.clone()
    ta = ctx.qp_frank_wolfe(phi, mu, ya, 12)
    tb = ctx.qp_frank_wolfe(phi, None, yb, 12)
    assert (ya - yb).abs().max().item() <= 1e-12
    for ra, rb in zip(ta, tb):
        assert abs(ra[0] - rb[0]) <= 1e-12 * abs(ra[0])
        assert abs(ra[2] - rb[2]) <= 1e-10
    ha = ctx.dc_gen(phi, mu, ya, 2, 3)
    hb = ctx.dc_gen(phi, None, yb, 2, 3)
    assert (ya - yb).abs().max().item() <= 1e-11
    assert np.allclose(ha, hb, rtol=1e-11, atol=0)
    lab = ctx.round(ya)
    ea, eb = ctx.energy(phi, mu, lab), ctx.energy(phi, None, lab)
    assert abs(ea - eb) <= 1e-12 * abs(ea)
    qa, qb = ctx.qp_apply(y0, mu), ctx.qp_apply(y0, None)
    assert (qa - qb).abs().max().item() <= 1e-12 * qa.abs().max().item()
    im3 = synth.make("rect_32x24_L3")   # another label count
    c3 = gpu_ctx(im3, torch.float64)
    p3 = T(im3.unary, torch.float64)
    y3a = T(O.softmax_neg(im3.unary), torch.float64)
    y3b = y3a.clone()
    c3.qp_frank_wolfe(p3, T(synth.potts(3), torch.float64), y3a, 5, trace=False)
    c3.qp_frank_wolfe(p3, None, y3b, 5, trace=False)
    assert (y3a - y3b).abs().max().item() <= 1e-12


def test_batch_image_lattices_match_oracle():
    # every image of the 16-image batch workload, one context each (FP64):
    # the vertex sets and per-pixel (vertex, weight) tables bit-exact against
    # the oracle's lattices, and the filter K'Y of a random Y within
    # 1e-11 (K~|Y| + 2 wsum |Y|); all images are reported before asserting
    ims = synth.make_batch()
    bad = []
    for j, im in enumerate(ims):
        ctx = gpu_ctx(im, torch.float64)
        model = O.Model(im.H, im.W, im.rgb, KERNELS)
        msg = []
        for m, lat in enumerate(model.lattices):
            d, M = ctx.lattice_info(m)
            gk, gv, gw = ctx.lattice_export(m)
            ok = lat.keys()
            sg, so = set(map(tuple, gk)), set(map(tuple, ok))
            ov, ow = lat.points()
            gt = key_table(gk, gv, gw)
            ot = key_table(ok, ov, ow)
            npix = sum(1 for a, b in zip(gt, ot) if a != b)
            if M != lat.nv or sg != so or npix:
                first = next((a for a in range(im.N) if gt[a] != ot[a]), None)
                msg.append(f"lattice {m}: M gpu {M} oracle {lat.nv}, keys only in gpu "
                           f"{len(sg - so)}, only in oracle {len(so - sg)}, pixels "
                           f"differing {npix}, first {first}")
                if first is not None:
                    msg.append(f"  gpu {gt[first]}\n  oracle {ot[first]}")
        Y = np.random.default_rng(j).uniform(-1, 1, size=(im.N, 3))
        g = ctx.filter(T(Y, torch.float64)).cpu().numpy()
        o = model.Kp(Y)
        nbad = int((np.abs(g - o) > filter_bound(model, Y, 1e-11)).sum())
        if nbad:
            msg.append(f"filter: {nbad} entries off, max |diff| {np.abs(g - o).max():.3g}")
        print(f"[lattice check] image {j} {im.H}x{im.W}: " + ("ok" if not msg else
              "\n".join(msg)), flush=True)
        if msg:
            bad.append(j)
    assert not bad, bad
