"""GPU parity of the separable filter mode: kernels on position alone by
the exact sum (two one-dimensional convolutions), the others by the lattice.

The oracle's model in mode "separable" sums the spatial kernel exactly
(O(N^2)) and runs its reference lattice for the bilateral one. The bar is the
filter's: |gpu - oracle| <= rtol (Ktilde|Y| + 2 sum(w) |Y|), rtol 1e-11 in
FP64 and 1e-5 in FP32. The Frank-Wolfe and DC_neg trajectories in this mode
are checked beside the lattice and exact modes in test_gpu_parity and
test_gpu_dcneg.
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


def ctx_for(im, dtype, kernels=KERNELS, mode="separable"):
    from paper_1608_06192_amd import dcrf
    print(f"[case] separable {im.H}x{im.W} {dtype} mode={mode}", flush=True)
    c = dcrf.Context(0)
    c.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev()), kernels, dtype=dtype)
    if mode != "lattice":
        c.set_filter_mode(mode)
    return c


def bound(model, Y, rtol):
    Ya = np.abs(Y)
    return rtol * (model.Kp(Ya) + 2 * model.w.sum() * Ya) + 1e-300


@pytest.mark.parametrize("H,W,C,dtype,rtol", [
    (24, 32, 3, torch.float64, 1e-11),
    (37, 29, 5, torch.float64, 1e-11),    # ragged tiles both ways
    (1, 1, 2, torch.float64, 1e-11),
    (1, 70, 4, torch.float64, 1e-11),     # one row
    (90, 1, 4, torch.float64, 1e-11),     # one column
    (120, 160, 21, torch.float32, 1e-5),
])
def test_separable_filter_matches_oracle(H, W, C, dtype, rtol):
    im = synth.voronoi_image(H, W, 4, seed=H * 7 + W, regions=5)
    ctx = ctx_for(im, dtype)
    model = O.Model(im.H, im.W, im.rgb, KERNELS, mode="separable")
    Y = np.random.default_rng(C).uniform(-1, 1, size=(im.N, C))
    if dtype == torch.float32:
        Y = Y.astype(np.float32).astype(np.float64)
    b = bound(model, Y, rtol)
    for adjoint in (False, True):
        g = ctx.filter(T(Y, dtype), adjoint=adjoint, separable=True).cpu().numpy()
        o = model.Kp(Y, reverse=adjoint)
        err = np.abs(g - o)
        print(f"[separable] adjoint={adjoint}: max err / bound {(err / b).max():.3g}",
              flush=True)
        assert (err <= b).all(), adjoint


def test_separable_spatial_only_is_the_exact_filter():
    # with the spatial kernel alone the separable mode is the exact sum:
    # the GPU's separable passes against its own O(N^2) kernel
    im = synth.voronoi_image(33, 45, 3, seed=2, regions=4)
    ctx = ctx_for(im, torch.float64, kernels=[synth.SPATIAL], mode="lattice")
    Y = T(np.random.default_rng(3).uniform(-1, 1, size=(im.N, 6)), torch.float64)
    a = ctx.filter(Y, separable=True)
    b = ctx.filter(Y, exact=True)
    scale = ctx.filter(Y.abs(), exact=True).abs().max().item()
    assert (a - b).abs().max().item() <= 1e-13 * scale


def test_separable_unstaged_passes_match_oracle():
    # a wide spatial kernel (theta 60, so R = the larger side - 1 = 69) and 64
    # channels in FP64: the staged tiles exceed 64 KB of LDS and both passes
    # run one thread per output value
    im = synth.voronoi_image(50, 70, 3, seed=4, regions=4)
    wide = dict(use_rgb=0, theta_pos=60.0, theta_rgb=0.0, weight=2.0)
    ctx = ctx_for(im, torch.float64, kernels=[synth.BILATERAL, wide])
    model = O.Model(im.H, im.W, im.rgb, [synth.BILATERAL, wide], mode="separable")
    Y = np.random.default_rng(5).uniform(-1, 1, size=(im.N, 64))
    g = ctx.filter(T(Y, torch.float64), separable=True).cpu().numpy()
    assert (np.abs(g - model.Kp(Y)) <= bound(model, Y, 1e-11)).all()


def test_separable_energy_and_qp_apply_match_oracle():
    im = synth.voronoi_image(30, 40, 5, seed=6, regions=5)
    ctx = ctx_for(im, torch.float64)
    model = O.Model(im.H, im.W, im.rgb, KERNELS, mode="separable")
    mu = synth.potts(5)
    x = np.random.default_rng(7).integers(0, 5, size=im.N).astype(np.int32)
    e = ctx.energy(T(im.unary, torch.float64), T(mu, torch.float64),
                   torch.from_numpy(x).to(dev()))
    eo = O.energy(model, im.unary, mu, x)
    assert abs(e - eo) <= 1e-10 * abs(eo)
    y = synth.random_simplex_points(im.N, 5, seed=8)
    qp = O.QP(model, im.unary, mu)
    g = ctx.qp_apply(T(y, torch.float64), T(mu, torch.float64)).cpu().numpy()
    o = qp.Q(y)
    assert np.abs(g - o).max() <= 1e-10 * np.abs(o).max()


def test_separable_mode_rejects_what_it_does_not_build():
    from paper_1608_06192_amd import dcrf
    im = synth.voronoi_image(16, 20, 3, seed=9, regions=3)
    ctx = ctx_for(im, torch.float64)
    phi = T(im.unary, torch.float64)
    y = T(O.softmax_neg(im.unary), torch.float64)
    for call in (lambda: ctx.lp_subgradient(phi, y),
                 lambda: ctx.lp_descent(phi, y.clone(), 1, 1e-3),
                 lambda: ctx.fw_forward(phi, None, 2)):
        with pytest.raises(dcrf.DcrfError) as e:
            call()
        assert dcrf.STATUS[e.value.status] == "DCRF_EUNSUPPORTED"
    with pytest.raises(dcrf.DcrfError) as e:
        ctx.filter(y, exact=True, separable=True)
    assert dcrf.STATUS[e.value.status] == "DCRF_EINVAL"


def test_separable_filter_fp32_500x375_sampled_pixels():
    # the timed image: K'Y for Y ~ U[-1, 1]^(N x 21) in FP32, against the
    # oracle at 200 sampled pixels: the exact spatial sum over all N pixels
    # at each sampled pixel, and the oracle's bilateral lattice filter
    im = synth.make("voronoi_500x375_L21")
    ctx = ctx_for(im, torch.float32)
    Y = np.random.default_rng(10).uniform(-1, 1, size=(im.N, 21))
    Y = Y.astype(np.float32).astype(np.float64)
    g = ctx.filter(T(Y, torch.float32), separable=True).cpu().numpy()
    bil, spa = O.Kernel(**synth.BILATERAL), O.Kernel(**synth.SPATIAL)
    fb = O.features(im.H, im.W, im.rgb, bil)
    fs = O.features(im.H, im.W, im.rgb, spa)
    lat = O.Lattice(fb)
    at = np.sort(np.random.default_rng(11).choice(im.N, 200, replace=False))
    Kb = lat.filter(Y)[at]
    Kb_abs = lat.filter(np.abs(Y))[at]
    Ks = O.gauss_exact(fs[at], fs, Y, exclude_same_index=False)
    Ks_abs = O.gauss_exact(fs[at], fs, np.abs(Y), exclude_same_index=False)
    wsum = bil.weight + spa.weight
    o = bil.weight * Kb + spa.weight * Ks - wsum * Y[at]
    b = 1e-5 * (bil.weight * Kb_abs + spa.weight * Ks_abs + wsum * np.abs(Y[at]))
    err = np.abs(g[at] - o)
    print(f"[separable 500x375] max err / bound {(err / b).max():.3g}", flush=True)
    assert (err <= b).all()


def test_separable_with_two_kernels_of_each_kind():
    # two lattice kernels and two position-only ones: the lattice sum is
    # formed first (scaled once the second arrives), the first exact kernel
    # accumulates into it and the second writes the result
    im = synth.voronoi_image(30, 40, 3, seed=12, regions=5)
    ks = [synth.BILATERAL, dict(use_rgb=1, theta_pos=20.0, theta_rgb=30.0, weight=2.0),
          synth.SPATIAL, dict(use_rgb=0, theta_pos=1.5, theta_rgb=0.0, weight=0.7)]
    ctx = ctx_for(im, torch.float64, kernels=ks)
    model = O.Model(im.H, im.W, im.rgb, ks, mode="separable")
    Y = np.random.default_rng(13).uniform(-1, 1, size=(im.N, 5))
    for adjoint in (False, True):
        g = ctx.filter(T(Y, torch.float64), adjoint=adjoint, separable=True).cpu().numpy()
        assert (np.abs(g - model.Kp(Y, reverse=adjoint)) <= bound(model, Y, 1e-11)).all()
