"""Pins of the oracle's reverse-mode derivative of unrolled Frank-Wolfe:
central finite differences in FP64 along random directions of the unaries
and of the kernel weights, with the discrete decisions (conditional
gradients, clipped or interior steps) checked to be the same on both sides
of the difference."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1608_06192_amd import synth


def problem(mode, seed=0, L=3, H=6, W=8):
    im = synth.voronoi_image(H, W, L, seed=seed, regions=3)
    kern = [O.Kernel(1, 4.0, 40.0, 2.0), O.Kernel(0, 1.5, 0.0, 0.7)]
    return im, O.Model(im.H, im.W, im.rgb, kern, mode=mode)


def decisions(tape):
    return [(r["s"].argmax(1).tobytes(), r["interior"]) for r in tape]


@pytest.mark.parametrize("mode", ["exact", "lattice"])
@pytest.mark.parametrize("seed", [0, 1])
def test_fw_gradient_matches_central_differences(mode, seed):
    im, model = problem(mode, seed)
    mu = synth.potts(im.L)
    iters, eps = 6, 1e-6
    loss, yT, tape, qp, c = O.fw_unrolled_loss(model, im.unary, mu, iters, im.gt)
    gphi, gw = O.fw_unrolled_backward(qp, tape, c, O.cross_entropy_grad(yT, im.gt))
    assert any(r["interior"] for r in tape)
    rng = np.random.default_rng(seed)
    for _ in range(3):
        v = rng.normal(size=im.unary.shape)
        lp, _, tp, _, _ = O.fw_unrolled_loss(model, im.unary + eps * v, mu, iters, im.gt)
        lm, _, tm, _, _ = O.fw_unrolled_loss(model, im.unary - eps * v, mu, iters, im.gt)
        assert decisions(tp) == decisions(tm) == decisions(tape)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - (gphi * v).sum()) <= 1e-6 * max(1.0, abs(fd))
    for m in range(2):
        dw = np.zeros(2)
        dw[m] = eps
        lp, _, tp, _, _ = O.fw_unrolled_loss(model.with_weights(model.w + dw),
                                            im.unary, mu, iters, im.gt)
        lm, _, tm, _, _ = O.fw_unrolled_loss(model.with_weights(model.w - dw),
                                            im.unary, mu, iters, im.gt)
        assert decisions(tp) == decisions(tm)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - gw[m]) <= 1e-6 * max(1.0, abs(fd))


def test_fw_gradient_general_mu():
    im, model = problem("exact", 3, L=4)
    rng = np.random.default_rng(3)
    mu = rng.uniform(0.2, 1.5, size=(4, 4))
    mu = 0.5 * (mu + mu.T)
    np.fill_diagonal(mu, 0.0)
    iters, eps = 5, 1e-6
    loss, yT, tape, qp, c = O.fw_unrolled_loss(model, im.unary, mu, iters, im.gt)
    gphi, gw = O.fw_unrolled_backward(qp, tape, c, O.cross_entropy_grad(yT, im.gt))
    v = rng.normal(size=im.unary.shape)
    lp = O.fw_unrolled_loss(model, im.unary + eps * v, mu, iters, im.gt)[0]
    lm = O.fw_unrolled_loss(model, im.unary - eps * v, mu, iters, im.gt)[0]
    assert abs((lp - lm) / (2 * eps) - (gphi * v).sum()) <= 1e-6
    dw = np.array([eps, 0.0])
    lp = O.fw_unrolled_loss(model.with_weights(model.w + dw), im.unary, mu, iters, im.gt)[0]
    lm = O.fw_unrolled_loss(model.with_weights(model.w - dw), im.unary, mu, iters, im.gt)[0]
    assert abs((lp - lm) / (2 * eps) - gw[0]) <= 1e-6 * max(1.0, abs(gw[0]))


def test_fw_gradient_scale_bounds_the_sum():
    """The absolute sum reported with ``scale`` bounds |dl/dw| and leaves the
    gradients unchanged."""
    im, model = problem("lattice", 2)
    mu = synth.potts(im.L)
    loss, yT, tape, qp, c = O.fw_unrolled_loss(model, im.unary, mu, 6, im.gt)
    ybar = O.cross_entropy_grad(yT, im.gt)
    g1, w1 = O.fw_unrolled_backward(qp, tape, c, ybar)
    g2, w2, wabs = O.fw_unrolled_backward(qp, tape, c, ybar, scale=True)
    assert np.array_equal(g1, g2) and np.array_equal(w1, w2)
    assert (wabs >= np.abs(w1)).all() and (wabs > 0).all()
