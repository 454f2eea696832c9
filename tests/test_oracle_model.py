"""Pins of the oracle's model, exact filter and permutohedral lattice.

Each test checks the oracle against something other than itself: a closed
form, a textbook identity, a brute-force count, or an exact invariant of the
lattice. None of them retypes the oracle's formula.
"""

import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O


# ---------------------------------------------------------------- exact sum

def test_exact_two_points_closed_form():
    # |f_a - f_b|^2 = 2 ln 2  =>  k = exp(-ln 2) = 1/2 (eq. gaussiankernel)
    f = np.array([[0.0, 0.0], [math.sqrt(2 * math.log(2)), 0.0]])
    v = np.array([[3.0], [5.0]])
    out = O.gauss_exact(f, f, v, exclude_same_index=False)
    assert np.allclose(out[:, 0], [3.0 + 2.5, 5.0 + 1.5], rtol=0, atol=1e-14)
    out = O.gauss_exact(f, f, v, exclude_same_index=True)
    assert np.allclose(out[:, 0], [2.5, 1.5], rtol=0, atol=1e-14)


def test_exact_identical_features():
    # all features equal: K'1 = (N - 1) per kernel
    f = np.full((7, 3), 0.25)
    out = O.gauss_exact(f, f, np.ones((7, 1)), exclude_same_index=True)
    assert np.allclose(out, 6.0, rtol=0, atol=1e-14)


def test_exact_grid_gaussian_integral():
    # Poisson summation: sum over Z^2 of exp(-|k|^2 h^2 / 2) = 2 pi / h^2 up to
    # terms of order exp(-2 pi^2 / h^2); with h = 1/3 those are ~1e-77.
    theta = 3.0
    H = W = 121
    model = O.Model(H, W, np.zeros((H * W, 3), np.float32),
                    [O.Kernel(0, theta, 0.0, 1.0)], mode="exact")
    centre = (H // 2) * W + W // 2
    f = model.feats[0]
    out = O.gauss_exact(f[centre:centre + 1], f, np.ones((H * W, 1)), False)
    assert abs(out[0, 0] - 2 * math.pi * theta ** 2) < 1e-9


def test_feature_scaling_app_g_form():
    # App. G: w exp(-|p_a - p_b|^2 / sigma) with sigma = 2 theta^2 under our
    # reading. Pixels (0,0) and (4,3) (distance 5), theta = 5: exp(-1/2).
    # Colours differ by (13, 0, 0) with theta_rgb = 13: another exp(-1/2).
    H, W = 4, 5
    rgb = np.zeros((H * W, 3), np.float32)
    b = 3 * W + 4
    rgb[b, 0] = 13.0
    m = O.Model(H, W, rgb, [O.Kernel(1, 5.0, 13.0, 2.0)], mode="exact")
    K = m.dense_K()
    assert abs(K[0, b] - 2.0 * math.exp(-1.0)) < 1e-15
    m2 = O.Model(H, W, rgb, [O.Kernel(0, 5.0, 0.0, 7.0)], mode="exact")
    assert abs(m2.dense_K()[0, b] - 7.0 * math.exp(-0.5)) < 1e-15


def test_exact_Kp_matches_dense_matrix():
    rng = np.random.default_rng(3)
    H, W = 5, 6
    rgb = rng.uniform(0, 255, size=(H * W, 3)).astype(np.float32)
    m = O.Model(H, W, rgb, [O.Kernel(1, 4.0, 30.0, 2.0),
                            O.Kernel(0, 2.0, 0.0, 0.5)], mode="exact")
    Y = rng.normal(size=(H * W, 4))
    assert np.allclose(m.Kp(Y), m.dense_K() @ Y, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------- lattice math

def _elevation(d):
    # the scaled orthonormal basis written as a matrix, independently
    s = (d + 1) * math.sqrt(2.0 / 3.0)
    E = np.zeros((d + 1, d))
    for j in range(d):
        col = np.zeros(d + 1)
        col[: j + 1] = 1.0
        col[j + 1] = -(j + 1)
        E[:, j] = s * col / np.linalg.norm(col)
    return E


@pytest.mark.parametrize("d", [1, 2, 3, 5])
def test_elevation_is_scaled_isometry_onto_hyperplane(d):
    rng = np.random.default_rng(d)
    s = (d + 1) * math.sqrt(2.0 / 3.0)
    for _ in range(200):
        f = rng.normal(0, 5, size=d)
        x = O.elevate(f)
        assert abs(x.sum()) < 1e-12 * (1 + np.abs(x).max())
        assert abs(np.linalg.norm(x) - s * np.linalg.norm(f)) < 1e-11 * s * (
            1 + np.linalg.norm(f))
    E = _elevation(d)
    f = rng.normal(size=d)
    assert np.allclose(O.elevate(f), E @ f, rtol=1e-14, atol=1e-13)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_simplex_contains_point(d):
    # b >= 0, sum b = 1, sum_k b_k v_k = x, each vertex of remainder k,
    # coordinates sum to zero: the simplex of (d+1)A*_d that contains x.
    rng = np.random.default_rng(10 + d)
    for t in range(3000):
        scale = [0.3, 3.0, 40.0][t % 3]
        x = O.elevate(rng.normal(0, scale, size=d))
        v, b = O.simplex(x)
        assert b.min() >= -1e-12 and abs(b.sum() - 1) < 1e-12
        assert np.abs((b[:, None] * v).sum(0) - x).max() < 1e-10 * (1 + scale)
        for k in range(d + 1):
            assert ((v[k] - k) % (d + 1) == 0).all()
            assert v[k].sum() == 0
        # consecutive vertices differ by a 0/1 pattern times (d+1) minus 1
        for k in range(d):
            step = v[k + 1] - v[k]
            assert set(np.unique(step)) <= {1, -d}


@pytest.mark.parametrize("d", [2, 3, 5])
def test_remainder_zero_vertex_is_nearest(d):
    # vertex 0 of the cell is the remainder-0 point (coordinates multiples of
    # d+1, sum 0) nearest to x: brute force over the 3^(d+1) moves of each
    # coordinate by -(d+1), 0, +(d+1) (Conway and Sloane's A_d decoding)
    rng = np.random.default_rng(20 + d)
    D1 = d + 1
    moves = np.array(list(itertools.product([-D1, 0, D1], repeat=D1)))
    moves = moves[moves.sum(1) == 0]
    for _ in range(500):
        x = O.elevate(rng.normal(0, 4, size=d))
        v, b = O.simplex(x)
        c = v[0].astype(float)
        assert (v[0] % D1 == 0).all() and v[0].sum() == 0
        best = min(np.linalg.norm(c + m - x) for m in moves)
        assert np.linalg.norm(c - x) <= best + 1e-9


def _lattice_cloud(d):
    """Points placed on every lattice vertex reachable from 0 with at most one
    +-u_j step per direction (the support of a full blur of a delta)."""
    s2 = ((d + 1) * math.sqrt(2.0 / 3.0)) ** 2
    E = _elevation(d)
    u = np.array([[(d + 1) * (i == j) - 1 for i in range(d + 1)]
                  for j in range(d + 1)], float)
    pts = np.unique(np.array([(np.array(p)[:, None] * u).sum(0)
                              for p in itertools.product([-1, 0, 1],
                                                         repeat=d + 1)]),
                    axis=0)
    f = pts @ E / s2                      # E^T v / s^2 maps back to features
    centre = int(np.where((pts == 0).all(axis=1))[0][0])
    return f, centre


@pytest.mark.parametrize("d", [2, 3, 5])
def test_blur_moments_of_a_delta(d):
    # d+1 passes of [1/4, 1/2, 1/4] along u_0..u_d on a fully occupied
    # neighbourhood: mass 1, mean 0, covariance sum_j u_j u_j^T / 2
    # = (d+1)^2 / 2 (I - 11^T / (d+1)).
    f, centre = _lattice_cloud(d)
    lat = O.Lattice(f)
    Y = np.zeros((f.shape[0], 1))
    Y[centre] = 1.0
    V = lat.blur(lat.splat(Y))[:, 0]
    keys = lat.keys()
    pos = np.concatenate([keys, -keys.sum(1, keepdims=True)], 1).astype(float)
    assert abs(V.sum() - 1.0) < 1e-14
    assert np.abs(V @ pos).max() < 1e-12
    cov = (V[:, None, None] * pos[:, :, None] * pos[:, None, :]).sum(0)
    target = 0.5 * (d + 1) ** 2 * (np.eye(d + 1) - 1.0 / (d + 1))
    assert np.abs(cov - target).max() < 1e-10
    # the reverse order gives the same moments on a full neighbourhood
    V2 = lat.blur(lat.splat(Y), reverse=True)[:, 0]
    assert np.abs(V2 - V).max() < 1e-15


@pytest.mark.parametrize("d", [2, 3])
def test_dense_cloud_calibration(d):
    # uniform density rho: the exact sum is rho (2 pi)^{d/2} in the interior;
    # gamma_d makes the lattice agree on average (to ~0.5%)
    rng = np.random.default_rng(30 + d)
    box = 10.0
    n = int(30 * box ** d) if d == 2 else int(20 * box ** d)
    f = rng.uniform(0, box, size=(n, d))
    lat = O.Lattice(f)
    out = lat.filter(np.ones((n, 1)))[:, 0]
    inner = np.all((f > 4) & (f < box - 4), axis=1)
    ex = O.gauss_exact(f[inner], f, np.ones((n, 1)), False)[:, 0]
    ratio = ex / out[inner]
    assert abs(ratio.mean() - 1.0) < 5e-3
    assert ratio.std() < 2e-2


def test_one_dimensional_lattice_by_hand():
    # d = 1: the lattice is the integer grid of t = 2 f / sqrt(3); splat and
    # slice are linear interpolation, the blur is [1,2,1]/4 twice ([1,4,6,4,1]
    # /16) over the occupied grid points, gamma_1 = sqrt(4 pi / 3) sqrt(2).
    rng = np.random.default_rng(5)
    f = np.concatenate([rng.uniform(0, 3, 40), rng.uniform(10, 11, 5)])
    Y = rng.normal(size=(f.shape[0], 2))
    t = 2.0 * f / math.sqrt(3.0)
    lo = np.floor(t).astype(int)
    fr = t - lo
    occupied = {}
    for a in range(f.shape[0]):
        if 1 - fr[a] > 0:
            occupied.setdefault(lo[a], len(occupied))
        if fr[a] > 0:
            occupied.setdefault(lo[a] + 1, len(occupied))
    V = {k: np.zeros(2) for k in occupied}
    for a in range(f.shape[0]):
        V[lo[a]] += (1 - fr[a]) * Y[a]
        if fr[a] > 0:
            V[lo[a] + 1] += fr[a] * Y[a]
    for _ in range(2):
        V = {k: 0.5 * V[k] + 0.25 * (V.get(k - 1, 0) + V.get(k + 1, 0))
             for k in V}
    g = math.sqrt(4 * math.pi / 3) * math.sqrt(2)
    out = np.array([g * ((1 - fr[a]) * V[lo[a]] +
                         (fr[a] * V[lo[a] + 1] if fr[a] > 0 else 0))
                    for a in range(f.shape[0])])
    lat = O.Lattice(f[:, None])
    assert lat.nv == len(occupied)
    assert np.abs(lat.filter(Y) - out).max() < 1e-12


def test_splat_slice_adjoint_and_filter_adjoint():
    rng = np.random.default_rng(7)
    for d in (2, 5):
        f = rng.normal(0, 2, size=(300, d))
        lat = O.Lattice(f)
        u = rng.normal(size=(300, 3))
        V = rng.normal(size=(lat.nv, 3))
        assert abs((lat.splat(u) * V).sum() - (u * lat.slice(V)).sum()) < 1e-10
        v = rng.normal(size=(300, 3))
        lhs = (u * lat.filter(v)).sum()
        rhs = (lat.filter(u, reverse=True) * v).sum()
        assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_lattice_filter_linear_nonnegative_permutation_invariant():
    rng = np.random.default_rng(8)
    f = rng.normal(0, 1.5, size=(400, 5))
    lat = O.Lattice(f)
    a, b = rng.normal(size=(400, 2)), rng.normal(size=(400, 2))
    assert np.allclose(lat.filter(2 * a - 3 * b),
                       2 * lat.filter(a) - 3 * lat.filter(b), atol=1e-10)
    pos = rng.uniform(0, 1, size=(400, 1))
    assert lat.filter(pos).min() >= 0
    perm = rng.permutation(400)
    lat2 = O.Lattice(f[perm])
    assert lat2.nv == lat.nv
    assert np.allclose(lat2.filter(a[perm]), lat.filter(a)[perm], atol=1e-10)


def test_lattice_collinear_with_exact_on_image():
    # App. A: lattice outputs are a near-constant factor from the exact sums
    from paper_1608_06192_amd import synth
    im = synth.make("rect_32x24_L3")
    kern = [synth.BILATERAL, synth.SPATIAL]
    lat = O.Model(im.H, im.W, im.rgb, kern, mode="lattice")
    ex = O.Model(im.H, im.W, im.rgb, kern, mode="exact")
    Y = np.ones((im.N, 1))
    a, b = lat.Kp(Y)[:, 0], ex.Kp(Y)[:, 0]
    cos = a @ b / np.linalg.norm(a) / np.linalg.norm(b)
    assert cos > 0.99
    assert 0.7 < (b / a).mean() < 1.5


def test_spatial_gaussian_factorises_into_two_one_dimensional_passes():
    # the spatial kernel exp(-((x_a-x_b)^2 + (y_a-y_b)^2) / (2 theta^2))
    # (features p / theta, eq. gaussiankernel with App. G's scaling) is the
    # product of a Gaussian in x and one in y, so K Y is a convolution along
    # the rows followed by one along the columns, each with the taps
    # g(t) = exp(-t^2 / (2 theta^2)); the taps below 2^-60 of the centre
    # (|t| > theta sqrt(120 ln 2)) change no FP64 result
    H, W, theta = 11, 17, 3.0
    rng = np.random.default_rng(0)
    Y = rng.normal(size=(H * W, 3))
    k = O.Kernel(0, theta, 0.0, 1.0)
    f = O.features(H, W, np.zeros((H * W, 3), np.float32), k)
    ref = O.gauss_exact(f, f, Y, exclude_same_index=False)
    R = int(math.ceil(theta * math.sqrt(120 * math.log(2))))
    g = np.exp(-np.arange(-R, R + 1) ** 2 / (2 * theta ** 2))
    img = Y.reshape(H, W, 3)
    rows = np.zeros_like(img)
    for x in range(W):
        for t in range(-R, R + 1):
            if 0 <= x + t < W:
                rows[:, x] += g[t + R] * img[:, x + t]
    both = np.zeros_like(img)
    for yy in range(H):
        for t in range(-R, R + 1):
            if 0 <= yy + t < H:
                both[yy] += g[t + R] * rows[yy + t]
    assert np.allclose(both.reshape(-1, 3), ref, rtol=1e-13, atol=1e-13)


def test_separable_mode_is_exact_spatial_plus_lattice_bilateral():
    # mode "separable": spatial kernels by the exact sum, the others by the
    # lattice; with one kind of kernel it is the exact or the lattice model
    H, W = 9, 12
    rng = np.random.default_rng(1)
    rgb = rng.uniform(0, 255, size=(H * W, 3)).astype(np.float32)
    Y = rng.random((H * W, 4))
    bil = O.Kernel(1, 5.0, 30.0, 2.0)
    spa = O.Kernel(0, 2.0, 0.0, 1.5)
    both = O.Model(H, W, rgb, [bil, spa], mode="separable").Kp(Y)
    lat = O.Model(H, W, rgb, [bil], mode="lattice")
    ex = O.Model(H, W, rgb, [spa], mode="exact")
    assert np.allclose(both, lat.Kp(Y) + ex.Kp(Y), rtol=1e-13, atol=1e-13)
    assert np.allclose(O.Model(H, W, rgb, [spa], mode="separable").Kp(Y), ex.Kp(Y),
                       rtol=1e-14, atol=1e-14)
    assert np.allclose(O.Model(H, W, rgb, [bil], mode="separable").Kp(Y), lat.Kp(Y),
                       rtol=1e-14, atol=1e-14)
