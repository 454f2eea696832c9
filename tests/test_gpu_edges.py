"""GPU edge cases against the FP64 oracle, through the C ABI: vertices
shared by thousands of pixels, the largest channel and label counts, a single
label, zero iterations.

Tolerances are those of the other parity tests: filter outputs within
rtol * (K~|Y| + 2 wsum |Y|) elementwise (rtol 1e-11 in FP64, 1e-5 in FP32),
Frank-Wolfe marginals within 1e-9 and objectives within 1e-9 relative (FP64).
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


def gpu_ctx(H, W, rgb, kernels, dtype):
    from paper_1608_06192_amd import dcrf
    print(f"[case] {H}x{W} dtype={dtype} kernels={kernels}", flush=True)
    ctx = dcrf.Context(0)
    ctx.set_image(H, W, torch.from_numpy(rgb).to(dev()), kernels, dtype=dtype)
    return ctx


def filter_bound(model, Y, rtol):
    Ya = np.abs(Y)
    return rtol * (model.Kp(Ya) + 2 * model.w.sum() * Ya) + 1e-300


def flat_image(H, W, colour=(90.0, 140.0, 200.0)):
    return np.tile(np.asarray(colour, np.float32), (H * W, 1))


@pytest.mark.parametrize("theta,dtype,rtol", [
    (400.0, torch.float64, 1e-11),
    (400.0, torch.float32, 1e-5),
    (12.0, torch.float32, 1e-5),
])
def test_filter_vertices_shared_by_thousands_of_pixels(theta, dtype, rtol):
    # one colour everywhere and wide position kernels: a handful of vertices,
    # each in the inverse index of thousands of pixels, so one vertex's
    # entries span many chunks that all add into it
    H, W = 96, 64
    rgb = flat_image(H, W)
    kernels = [dict(use_rgb=1, theta_pos=theta, theta_rgb=13.0, weight=10.0),
               dict(use_rgb=0, theta_pos=theta / 2, theta_rgb=0.0, weight=3.0)]
    model = O.Model(H, W, rgb, kernels)
    lat = O.Lattice(model.feats[0])
    vid, _ = lat.points()
    deg = np.bincount(vid[vid >= 0].ravel(), minlength=lat.nv)
    print(f"bilateral lattice: {lat.nv} vertices, largest degree {deg.max()}")
    assert deg.max() >= 300
    ctx = gpu_ctx(H, W, rgb, kernels, dtype)
    rng = np.random.default_rng(21)
    for C in (1, 21):
        Y = rng.uniform(-1, 1, size=(H * W, C))
        if dtype == torch.float32:
            Y = Y.astype(np.float32).astype(np.float64)
        for adjoint in (False, True):
            got = ctx.filter(T(Y, dtype), adjoint=adjoint).double().cpu().numpy()
            ref = model.Kp(Y, reverse=adjoint)
            err = np.abs(got - ref)
            assert (err <= filter_bound(model, Y, rtol)).all(), (C, adjoint, err.max())


@pytest.mark.parametrize("C,dtype,rtol", [
    (256, torch.float64, 1e-11),
    (255, torch.float64, 1e-11),
    (256, torch.float32, 1e-5),
    (129, torch.float32, 1e-5),
])
def test_filter_largest_channel_counts(C, dtype, rtol):
    # C = 256 is the largest the filter takes: one chunk per splat block and
    # the widest vertex rows; 255 and 129 leave ragged 16-byte vectors
    im = synth.voronoi_image(40, 56, 4, seed=C, regions=7)
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    ctx = gpu_ctx(im.H, im.W, im.rgb, KERNELS, dtype)
    Y = np.random.default_rng(C).uniform(-1, 1, size=(im.N, C))
    if dtype == torch.float32:
        Y = Y.astype(np.float32).astype(np.float64)
    for adjoint in (False, True):
        got = ctx.filter(T(Y, dtype), adjoint=adjoint).double().cpu().numpy()
        ref = model.Kp(Y, reverse=adjoint)
        assert (np.abs(got - ref) <= filter_bound(model, Y, rtol)).all(), adjoint


def test_filter_rejects_too_many_channels():
    from paper_1608_06192_amd import dcrf
    im = synth.make("rect_32x24_L3")
    ctx = gpu_ctx(im.H, im.W, im.rgb, KERNELS, torch.float64)
    with pytest.raises(dcrf.DcrfError) as ei:
        ctx.filter(torch.zeros(im.N, 257, dtype=torch.float64, device=dev()))
    assert ei.value.status == -1


def _fw_pair(im, mu, iters, phi=None, dtype=torch.float64):
    phi = im.unary if phi is None else phi
    model = O.Model(im.H, im.W, im.rgb, KERNELS)
    qp = O.QP(model, phi, mu)
    y0 = O.softmax_neg(phi)
    st = O.frank_wolfe(qp, y0, iters)
    ctx = gpu_ctx(im.H, im.W, im.rgb, KERNELS, dtype)
    y = T(y0, dtype)
    tr = ctx.qp_frank_wolfe(T(phi, dtype), T(mu, dtype), y, iters)
    return st, y.cpu().numpy(), tr


@pytest.mark.parametrize("L", [100, 256])
def test_fw_largest_label_counts(L):
    # L = 256 is the largest label count the solvers take
    im = synth.voronoi_image(12, 10, L, seed=L, regions=4)
    mu = synth.potts(L)
    st, yg, tr = _fw_pair(im, mu, 5)
    assert np.abs(yg - st.y).max() < 1e-9
    for (fo, _, ao), (fg, _, ag, _) in zip(st.trace, tr):
        assert abs(fg - fo) <= 1e-9 * abs(fo)
        assert abs(ag - ao) <= 1e-8


def test_fw_single_label():
    # L = 1: mu = [[0]] makes the pairwise term and d vanish and the only
    # labelling is the constant one, so s = y, the gap is 0 and the objective
    # is sum(phi) at every step. The direction s - y is zero, so every alpha
    # in [0, 1] is a minimiser: only its range is checked.
    im = synth.voronoi_image(9, 14, 1, seed=1, regions=3)
    mu = synth.potts(1)
    phi = np.random.default_rng(1).normal(0.0, 2.0, size=(im.N, 1))
    st, yg, tr = _fw_pair(im, mu, 3, phi=phi)
    assert (yg == 1.0).all()
    assert len(tr) == 3
    scale = np.abs(phi).sum()
    for (fo, go, _), (fg, gg, ag, _) in zip(st.trace, tr):
        assert 0.0 <= ag <= 1.0
        assert abs(fg - phi.sum()) <= 1e-12 * scale
        assert abs(fo - phi.sum()) <= 1e-12 * scale
        assert abs(gg) <= 1e-12 * scale and abs(go) <= 1e-12 * scale


def test_fw_two_labels_and_zero_iterations():
    im = synth.voronoi_image(21, 17, 2, seed=2, regions=4)
    mu = synth.potts(2)
    st, yg, tr = _fw_pair(im, mu, 6)
    assert np.abs(yg - st.y).max() < 1e-9
    for (fo, _, ao), (fg, _, ag, _) in zip(st.trace, tr):
        assert abs(fg - fo) <= 1e-9 * abs(fo)
        assert abs(ag - ao) <= 1e-8
    # zero iterations leave y as it was and return an empty trace
    ctx = gpu_ctx(im.H, im.W, im.rgb, KERNELS, torch.float64)
    y0 = O.softmax_neg(im.unary)
    y = T(y0, torch.float64)
    tr0 = ctx.qp_frank_wolfe(T(im.unary, torch.float64), T(mu, torch.float64),
                             y, 0)
    assert len(tr0) == 0
    assert np.array_equal(y.cpu().numpy(), y0)
