"""Pins of the oracle's solvers: Frank-Wolfe on the convex QP, CCCP on the
generic DC relaxation, the LP subgradient (brute force and divide and
conquer), projected subgradient descent and the simplex projection.

The pins are brute-force minima, an independent LP solver (scipy's HiGHS on
the standard-form LP with one extra variable per pair), independent line
searches and projections, and identities the paper states.
"""

import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1608_06192_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_problem(N=6, L=3, seed=0, w=(4.0, 1.5)):
    """A tiny dense CRF on a 2 x (N/2) image, exact filter."""
    rng = np.random.default_rng(seed)
    H, W = 2, N // 2
    rgb = rng.uniform(0, 255, size=(N, 3)).astype(np.float32)
    kern = [O.Kernel(1, 2.0, 60.0, w[0]), O.Kernel(0, 1.0, 0.0, w[1])]
    model = O.Model(H, W, rgb, kern, mode="exact")
    phi = rng.normal(0, 3.0, size=(N, L))
    return model, phi


def test_energy_two_pixels_by_hand():
    # N = 2, Kbar_12 = w/2: E(x) = phi_1(x_1) + phi_2(x_2) + 2 mu(x_1,x_2) w/2,
    # because eq. labelling-energy sums ordered pairs a != b.
    t = math.sqrt(2 * math.log(2))        # pixel distance giving k = 1/2
    model = O.Model(1, 2, np.zeros((2, 3), np.float32),
                    [O.Kernel(0, 1.0 / t, 0.0, 3.0)], mode="exact")
    phi = np.array([[0.5, 2.0], [1.0, 0.25]])
    mu = synth.potts(2)
    expect = {(0, 0): 1.5, (1, 1): 2.25, (0, 1): 0.75 + 3.0, (1, 0): 3.0 + 3.0}
    for x, e in expect.items():
        assert abs(O.energy(model, phi, mu, np.array(x)) - e) < 1e-14


def test_qp_equals_energy_at_integral_points():
    # eq. energy-ip: the objective equals E at integral y; S_cvx adds
    # sum d (y^2 - y), which vanishes there (eq. cvx-qp-min).
    model, phi = tiny_problem()
    mu = synth.potts(3)
    qp = O.QP(model, phi, mu)
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.integers(0, 3, size=6)
        y = O.onehot(x, 3)
        E = O.energy(model, phi, mu, x)
        assert abs(qp.S(y) - E) < 1e-12 * max(1, abs(E))
        assert abs(qp.S_cvx(y) - E) < 1e-12 * max(1, abs(E))
    # on M, S_cvx <= S since d >= 0 and y^2 <= y
    for _ in range(20):
        y = synth.random_simplex_points(6, 3, int(rng.integers(1 << 30)))
        assert qp.S_cvx(y) <= qp.S(y) + 1e-12


def test_rl_diagonal_is_row_sum_of_abs_psi():
    # eq. RL-diagonal with an explicit Psi built from the dense Kbar
    model, phi = tiny_problem()
    mu = np.array([[0.0, 1.0, 2.0], [1.0, 0.0, -0.5], [2.0, -0.5, 0.0]])
    qp = O.QP(model, phi, mu)
    K = model.dense_K()
    N, L = phi.shape
    for a in range(N):
        for i in range(L):
            dd = sum(abs(mu[i, j] * K[a, b]) for b in range(N) if b != a
                     for j in range(L))
            assert abs(qp.d[a, i] - dd) < 1e-12


def test_fw_step_is_exact_line_minimum():
    # App. B: alpha* minimises S_cvx on the segment; compare with a 10001-point
    # grid of fresh evaluations of S_cvx
    model, phi = tiny_problem(seed=2)
    qp = O.QP(model, phi, synth.potts(3))
    y = O.softmax_neg(phi)
    c = qp.phi - qp.d
    for _ in range(4):
        Py = qp.Q(y)
        s = O.onehot(np.argmin(c + 2 * Py, axis=1), 3)
        alpha, _, _ = O.fw_step_size(c, y, s, Py, qp.Q(s))
        grid = np.linspace(0, 1, 10001)
        vals = np.array([qp.S_cvx(y + t * (s - y)) for t in grid])
        assert qp.S_cvx(y + alpha * (s - y)) <= vals.min() + 1e-9
        assert abs(alpha - grid[vals.argmin()]) <= 2e-4 or alpha in (0.0, 1.0)
        y = y + alpha * (s - y)


def test_fw_invariants_and_bounds():
    # gap >= 0; f non-increasing; recurrence P_y == fresh Q y; the best dual
    # bound max_t (f_t - gap_t) <= min over M of S_cvx <= E_min (Sec. 4:
    # S_cvx is a relaxation; Ravikumar-Lafferty tightness of the QP)
    model, phi = tiny_problem(seed=4)
    mu = synth.potts(3)
    qp = O.QP(model, phi, mu)
    st = O.frank_wolfe(qp, O.softmax_neg(phi), 200)
    f = np.array([t[0] for t in st.trace])
    gap = np.array([t[1] for t in st.trace])
    assert (gap >= -1e-9).all()
    assert (np.diff(f) <= 1e-9).all()
    assert np.abs(st.Py - qp.Q(st.y)).max() < 1e-9
    Emin, xmin = O.brute_force_min(model.dense_K(), phi, mu)
    lower = (f - gap).max()
    assert lower <= qp.S_cvx(st.y) + 1e-9
    assert lower <= Emin + 1e-9
    assert qp.S_cvx(st.y) <= Emin + 1e-9
    assert abs(O.energy(model, phi, mu, xmin) - Emin) < 1e-12


def test_fw_matches_projected_gradient_minimum():
    # an independent solver of the same convex QP: projected gradient with
    # the textbook simplex projection and step 1/Lipschitz
    model, phi = tiny_problem(seed=6)
    qp = O.QP(model, phi, synth.potts(3))
    st = O.frank_wolfe(qp, O.softmax_neg(phi), 2000)
    Qd = np.stack([qp.Q(e.reshape(6, 3)).ravel() for e in np.eye(18)], 1)
    lip = 2 * np.linalg.eigvalsh(0.5 * (Qd + Qd.T)).max()
    y = O.softmax_neg(phi)
    c = qp.phi - qp.d
    for _ in range(20000):
        y = O.project_simplex(y - (c + 2 * qp.Q(y)) / lip)
    f = np.array([t[0] for t in st.trace])
    gap = np.array([t[1] for t in st.trace])
    pg = qp.S_cvx(y)
    # FW's duality bound and value bracket the independent minimum
    assert (f - gap).max() <= pg + 1e-9
    assert pg <= qp.S_cvx(st.y) + 1e-9
    assert qp.S_cvx(st.y) - pg < 1e-4 * abs(pg)


def test_fw_zero_weights_is_unary_argmin():
    # w = 0: d = 0 and the objective is linear; one step reaches argmin phi
    model, phi = tiny_problem(seed=7, w=(0.0, 0.0))
    qp = O.QP(model, phi, synth.potts(3))
    st = O.frank_wolfe(qp, O.softmax_neg(phi), 1)
    assert st.alphas[0] == 1.0
    assert (O.round_argmax(st.y) == np.argmin(phi, axis=1)).all()


def test_dc_gen_monotone_and_above_minimum():
    # Alg. cccp: S(y^{k+1}) <= S(y^k) (Sec. 5.1; App. C: an inexact convex
    # step that decreases the surrogate is enough); S >= E_min on M
    model, phi = tiny_problem(seed=8)
    mu = synth.potts(3)
    qp = O.QP(model, phi, mu)
    st = O.frank_wolfe(qp, O.softmax_neg(phi), 30)
    y, hist = O.dc_gen(qp, st.y, outer=8, inner=10)
    assert (np.diff(hist) <= 1e-9).all()
    Emin, _ = O.brute_force_min(model.dense_K(), phi, mu)
    assert min(hist) >= Emin - 1e-9
    # the surrogate's linear term at y = 1/2 everywhere equals S_cvx's: 2 d/2 = d
    assert np.allclose(qp.phi - 2 * qp.d * 0.5, qp.phi - qp.d)


def nsd_mu(L, seed):
    """A symmetric compatibility that is negative semi-definite on the
    directions with zero sum (the condition of the DC_neg decomposition):
    J - B B^T with a zero-sum-blind constant part J."""
    rng = np.random.default_rng(seed)
    B = rng.normal(0, 0.6, size=(L, 2))
    return np.ones((L, L)) - B @ B.T


def _dcneg_parts(model, phi, mu, y, yk):
    """S's convex part p, concave part q and the CCCP surrogate at y^k
    (tangent of q), evaluated from a dense Kbar (independent of dc_neg)."""
    K = model.dense_K()
    wsum = model.w.sum()
    Kbar = K + wsum * np.eye(K.shape[0])     # dense_K has no self-pairs
    quad = lambda Kx, z: float((z * (Kx @ z @ mu.T)).sum())
    p = float((phi * y).sum()) - wsum * float((y * (y @ mu.T)).sum())
    q = quad(Kbar, y)
    grad = 2.0 * (Kbar @ yk) @ mu.T
    sur = p + quad(Kbar, yk) + float((grad * (y - yk)).sum())
    return p, q, sur


@pytest.mark.parametrize("general", [False, True])
def test_dc_neg_decomposition_and_surrogate(general):
    # eq. QP-concave-CCCP: S = p + q with p convex and q concave on M;
    # the CCCP surrogate (q replaced by its tangent at y^k) equals S at y^k
    # and lies above S on M (the tangent of a concave function)
    model, phi = tiny_problem(N=8, L=3, seed=21)
    L = 3
    mu = nsd_mu(L, 3) if general else synth.potts(L)
    assert np.array_equal(model.dense_K(), model.dense_K().T)
    assert np.abs(np.diag(model.dense_K())).max() == 0.0
    qp = O.QP(model, phi, mu)
    rng = np.random.default_rng(5)
    for _ in range(10):
        y = synth.random_simplex_points(8, L, int(rng.integers(1 << 30)), 0.3)
        yk = synth.random_simplex_points(8, L, int(rng.integers(1 << 30)), 0.3)
        p, q, sur = _dcneg_parts(model, phi, mu, y, yk)
        assert abs(p + q - qp.S(y)) <= 1e-10 * max(1.0, abs(qp.S(y)))
        _, _, tight = _dcneg_parts(model, phi, mu, yk, yk)
        assert abs(tight - qp.S(yk)) <= 1e-10 * max(1.0, abs(qp.S(yk)))
        assert sur >= qp.S(y) - 1e-9


@pytest.mark.parametrize("general", [False, True])
def test_dc_neg_monotone_and_above_minimum(general):
    # Alg. cccp on the DC_neg decomposition (exact filter): S(y^{k+1}) <=
    # S(y^k) and S >= E_min on M (brute force); the surrogate is minimised
    # exactly for Potts and by per-pixel Frank-Wolfe otherwise
    model, phi = tiny_problem(N=8, L=3, seed=22)
    mu = nsd_mu(3, 4) if general else synth.potts(3)
    qp = O.QP(model, phi, mu)
    y0 = O.softmax_neg(phi)
    y, hist = O.dc_neg(qp, y0, outer=12, inner=50)
    assert (np.diff(hist) <= 1e-9).all(), hist
    assert hist[-1] < hist[0]
    Emin, _ = O.brute_force_min(model.dense_K(), phi, mu)
    assert min(hist) >= Emin - 1e-9
    assert np.abs(y.sum(axis=1) - 1).max() < 1e-12 and y.min() >= 0


@pytest.mark.parametrize("general", [False, True])
def test_dc_neg_pixel_problem_matches_slsqp(general):
    # eq. convexpb-onevar solved by an independent method (scipy's SLSQP with
    # the simplex constraints) at random linear terms
    from scipy.optimize import minimize
    L, N = 5, 12
    rng = np.random.default_rng(8)
    mu = nsd_mu(L, 9) if general else synth.potts(L)
    wsum = 2.5
    c = rng.normal(0, 4.0, size=(N, L))
    y0 = synth.random_simplex_points(N, L, 3, 0.0)
    got = O.dcneg_pixel_step(c, y0, mu, wsum, 3000, not general)
    h = lambda z, a: float(c[a] @ z - wsum * z @ mu @ z)
    for a in range(N):
        r = minimize(lambda z: h(z, a), y0[a], method="SLSQP",
                     bounds=[(0, 1)] * L,
                     constraints=[{"type": "eq", "fun": lambda z: z.sum() - 1}],
                     options={"ftol": 1e-14, "maxiter": 500})
        assert abs(got[a].sum() - 1) < 1e-12 and got[a].min() >= 0
        if not general:   # closed form: the exact minimiser
            assert h(got[a], a) <= r.fun + 1e-9, a
            continue
        # Frank-Wolfe: its duality gap brackets the optimum, and after 3000
        # iterations the value is close to it
        grad = c[a] - 2.0 * wsum * mu @ got[a]
        gap = float(grad @ got[a] - grad.min())
        assert r.fun >= h(got[a], a) - gap - 1e-9, a
        assert h(got[a], a) - r.fun <= 1e-4 * max(1.0, abs(r.fun)), a
        assert h(got[a], a) <= h(y0[a], a) + 1e-12, a


def test_dc_neg_zero_weights_is_unary_argmin():
    # w = 0: the per-pixel problems are linear; one step gives argmin phi
    model, phi = tiny_problem(seed=23, w=(0.0, 0.0))
    qp = O.QP(model, phi, synth.potts(3))
    y, _ = O.dc_neg(qp, O.softmax_neg(phi), outer=1)
    assert np.array_equal(y, O.onehot(np.argmin(phi, axis=1), 3))


# ----------------------------------------------------------------------- LP

def test_dnc_nodes_golden_example():
    rows = [tuple(int(v) for v in line.split())
            for line in open(os.path.join(GOLDEN, "dnc_n6_example.txt"))
            if line.strip() and not line.startswith("#")]
    got = list(O.dnc_nodes(6))
    assert [(lo, mid, hi) for (_, lo, mid, hi) in rows] == got


@pytest.mark.parametrize("N", list(range(1, 40)) + [64, 100, 187])
def test_dnc_blocks_cover_upper_triangle_once(N):
    cover = np.zeros((N, N), dtype=int)
    for lo, mid, hi in O.dnc_nodes(N):
        cover[lo:mid, mid:hi] += 1
    assert (cover == np.triu(np.ones((N, N), dtype=int), 1)).all()


def test_lp_dnc_exact_equals_brute_force():
    model, phi = tiny_problem(N=12, L=3, seed=9)
    K = model.dense_K()
    rng = np.random.default_rng(0)
    for sp in (0.0, 0.5):
        y = synth.random_simplex_points(12, 3, int(rng.integers(99)), sp)
        g1, S1 = O.lp_subgradient(phi, y, lambda o: O.lp_pair_sums_brute(K, o))
        g2, S2 = O.lp_subgradient(
            phi, y, lambda o: O.lp_pair_sums_dnc(model, o, "exact"))
        assert np.abs(g1 - g2).max() < 1e-12
        assert abs(S1 - S2) < 1e-11


def test_lp_dnc_sampled_pixels():
    # the sampled evaluation (only the nodes holding a wanted position) gives
    # the brute-force sums at the wanted pixels (exact inner filter), and the
    # full divide and conquer's values there (lattice inner filter)
    model, _ = tiny_problem(N=40, L=3, seed=12)
    K = model.dense_K()
    rng = np.random.default_rng(4)
    for _ in range(3):
        order = rng.permutation(40)
        at = rng.choice(40, size=7, replace=False)
        Ub, Lb = O.lp_pair_sums_brute(K, order)
        Us, Ls = O.lp_pair_sums_dnc(model, order, "exact", at=at)
        assert np.abs(Us[at] - Ub[at]).max() < 1e-12
        assert np.abs(Ls[at] - Lb[at]).max() < 1e-12
    im = synth.voronoi_image(15, 20, 3, seed=5, regions=4)
    lat = O.Model(im.H, im.W, im.rgb, [synth.BILATERAL, synth.SPATIAL])
    order = O.sorted_order(synth.random_simplex_points(im.N, 3, 6, 0.5)[:, 1])
    at = np.array([order[0], order[-1], order[im.N // 2], 17, 123])
    Uf, Lf = O.lp_pair_sums_dnc(lat, order, "lattice")
    Us, Ls = O.lp_pair_sums_dnc(lat, order, "lattice", at=at)
    assert np.array_equal(Us[at], Uf[at]) and np.array_equal(Ls[at], Lf[at])


def test_lp_dnc_c_walk_equals_python_walk():
    # the C walk of the divide and conquer (lattice inner filter, nodes of a
    # level in parallel) is the Python walk node for node: bit-identical
    # sums, for odd and even N, one and two pixels, and ties in the order
    for H, W, L, seed in [(24, 32, 3, 5), (17, 13, 4, 6), (1, 2, 2, 7),
                          (1, 1, 2, 8), (9, 7, 3, 9)]:
        im = synth.voronoi_image(H, W, L, seed=seed, regions=4)
        model = O.Model(im.H, im.W, im.rgb, [synth.BILATERAL, synth.SPATIAL])
        y = synth.random_simplex_points(im.N, L, seed=seed, sparsity=0.5)
        for i in range(L):
            order = O.sorted_order(y[:, i])
            U, Lo = O.lp_pair_sums_dnc(model, order, "lattice")
            U2, Lo2 = O.lp_pair_sums_dnc_c(model, order)
            assert np.array_equal(U, U2) and np.array_equal(Lo, Lo2), (H, W, i)


def test_lp_reformulation_and_integral_energy():
    # eq. simple_S: <g(y), y> equals eq. potts-lp's |.| form; at integral y
    # S_LP = E (Sec. 6)
    model, phi = tiny_problem(N=10, L=3, seed=10)
    K = model.dense_K()
    mu = synth.potts(3)
    rng = np.random.default_rng(1)
    brute = lambda o: O.lp_pair_sums_brute(K, o)
    for sp in (0.0, 0.3, 0.7):
        y = synth.random_simplex_points(10, 3, int(rng.integers(99)), sp)
        _, S = O.lp_subgradient(phi, y, brute)
        assert abs(S - O.S_LP_dense(K, phi, y)) < 1e-11
    for _ in range(10):
        x = rng.integers(0, 3, size=10)
        _, S = O.lp_subgradient(phi, O.onehot(x, 3), brute)
        assert abs(S - O.energy(model, phi, mu, x)) < 1e-11


def test_lp_subgradient_inequality():
    # S_LP is convex and g(y) is a subgradient: S_LP(z) >= S_LP(y) + <g, z - y>
    model, phi = tiny_problem(N=10, L=4, seed=11)
    K = model.dense_K()
    rng = np.random.default_rng(2)
    for _ in range(30):
        y = synth.random_simplex_points(10, 4, int(rng.integers(1 << 20)), 0.3)
        g, S = O.lp_subgradient(phi, y, lambda o: O.lp_pair_sums_brute(K, o))
        for _ in range(5):
            z = synth.random_simplex_points(10, 4, int(rng.integers(1 << 20)))
            assert O.S_LP_dense(K, phi, z) >= S + (g * (z - y)).sum() - 1e-10


def _lp_optimum_highs(K, phi):
    """min phi^T y + sum_{a<b} K_ab sum_i t_ab(i), t >= |y_a(i) - y_b(i)|,
    y in M: the LP of Kleinberg and Tardos with one variable per pair."""
    from scipy.optimize import linprog
    N, L = phi.shape
    pairs = [(a, b) for a in range(N) for b in range(a + 1, N)]
    ny, nt = N * L, len(pairs) * L
    cost = np.concatenate([phi.ravel(),
                           np.repeat([K[a, b] for a, b in pairs], L)])
    A, rhs = [], []
    for p, (a, b) in enumerate(pairs):
        for i in range(L):
            for sgn in (1, -1):
                row = np.zeros(ny + nt)
                row[a * L + i] = sgn
                row[b * L + i] = -sgn
                row[ny + p * L + i] = -1
                A.append(row)
                rhs.append(0.0)
    Aeq = np.zeros((N, ny + nt))
    for a in range(N):
        Aeq[a, a * L:(a + 1) * L] = 1
    res = linprog(cost, A_ub=np.array(A), b_ub=rhs, A_eq=Aeq, b_eq=np.ones(N),
                  bounds=[(0, None)] * (ny + nt), method="highs")
    assert res.status == 0
    return res.fun


def test_lp_descent_approaches_lp_optimum_and_two_label_tightness():
    # Alg. lp_subgrad converges to the LP optimum (checked against HiGHS);
    # with two labels the LP is tight: its optimum equals E_min (Sec. 8)
    for L, seed, beta0 in ((2, 12, 0.2), (3, 13, 2.0)):
        model, phi = tiny_problem(N=6, L=L, seed=seed)
        K = model.dense_K()
        opt = _lp_optimum_highs(K, phi)
        Emin, _ = O.brute_force_min(K, phi, synth.potts(L))
        assert opt <= Emin + 1e-9
        if L == 2:
            assert abs(opt - Emin) < 1e-8
        y0 = O.softmax_neg(phi)
        _, best, best_y, hist = O.lp_descent(
            phi, y0, 3000, beta0, lambda o: O.lp_pair_sums_brute(K, o))
        assert best >= opt - 1e-9
        assert best - opt < 2e-2 * max(1.0, abs(opt))


def _kt_draws(R, L, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, L, size=R).astype(np.int32), rng.random(R)


def test_kt_round_integral_points_and_fallback():
    # an integral y is returned as its labelling; without rounds every pixel
    # takes the argmax and is counted as left over
    rng = np.random.default_rng(0)
    x = rng.integers(0, 4, size=50)
    lab, th = _kt_draws(400, 4, 1)
    got, left = O.kt_round(O.onehot(x, 4), lab, th)
    assert left == 0 and np.array_equal(got, x)
    y = synth.random_simplex_points(50, 4, 2, 0.3)
    got, left = O.kt_round(y, lab[:0], th[:0])
    assert left == 50 and np.array_equal(got, O.round_argmax(y))


def test_kt_round_marginals_and_pairwise_bound():
    # Monte Carlo over independent draws: P(x_a = i) = y_a(i) (labels of
    # marginal 0 never taken), and the expected energy is at most
    # phi^T y + 2 (the LP's pairwise term), the bound behind the factor 2
    model, phi = tiny_problem(N=6, L=3, seed=31)
    K = model.dense_K()
    mu = synth.potts(3)
    y = synth.random_simplex_points(6, 3, 5, 0.4)
    n = 20000
    counts = np.zeros((6, 3))
    E = np.empty(n)
    for k in range(n):
        lab, th = _kt_draws(120, 3, 1000 + k)
        x, left = O.kt_round(y, lab, th)
        assert left == 0
        counts[np.arange(6), x] += 1
        E[k] = O.energy_dense(K, phi, mu, x)
    freq = counts / n
    sigma = np.sqrt(np.maximum(y * (1 - y), 1e-12) / n)
    assert (np.abs(freq - y) <= 5 * sigma + 1e-12).all()
    assert (freq[y == 0] == 0).all()
    unary = float((phi * y).sum())
    pair = O.S_LP_dense(K, phi, y) - unary
    assert E.mean() <= unary + 2 * pair + 5 * E.std() / np.sqrt(n)


def test_present_labels_and_subset_lp():
    # the labels present in a labelling; the LP restricted to all labels is
    # the plain LP; a proper subset keeps the other labels at 0 and its S_LP
    # history is the full problem's S_LP at the scattered points
    rng = np.random.default_rng(3)
    x = rng.choice([0, 2, 3], size=12)
    assert np.array_equal(O.present_labels(O.onehot(x, 5), 0.5), np.unique(x))
    model, phi = tiny_problem(N=12, L=4, seed=33)
    K = model.dense_K()
    pair = lambda o: O.lp_pair_sums_brute(K, o)
    y0 = synth.random_simplex_points(12, 4, 7, 0.0)
    ya, ba, _, ha = O.lp_descent(phi, y0, 4, 0.05, pair)
    yb, bb, _, hb = O.lp_descent_subset(phi, y0, [0, 1, 2, 3], 4, 0.05, pair)
    assert np.allclose(ya, yb, rtol=0, atol=1e-14) and np.allclose(ha, hb, rtol=1e-14)
    S = [1, 3]
    ys, best, by, hs = O.lp_descent_subset(phi, y0, S, 5, 0.05, pair)
    assert (ys[:, [0, 2]] == 0).all() and (by[:, [0, 2]] == 0).all()
    assert np.abs(ys.sum(axis=1) - 1).max() < 1e-12
    y = O.project_simplex(y0[:, S])
    for t in range(5):
        full = np.zeros_like(y0)
        full[:, S] = y
        _, S_full = O.lp_subgradient(phi, full, pair)
        assert abs(S_full - hs[t]) <= 1e-12 * abs(S_full)
        g, _ = O.lp_subgradient(phi[:, S], y, pair)
        y = O.project_simplex(y - 0.05 / (1 + t) * g)


def test_simplex_projection_kkt_and_bisection():
    rng = np.random.default_rng(14)
    V = rng.normal(0, 2, size=(200, 21))
    V[:20, :5] = 0.3                        # ties
    P = O.project_simplex(V)
    assert (P >= 0).all() and np.allclose(P.sum(1), 1, atol=1e-13)
    for v, p in zip(V, P):
        lo, hi = v.min() - 1, v.max()
        for _ in range(200):                 # bisection on sum max(v-t,0) = 1
            mid = 0.5 * (lo + hi)
            if np.maximum(v - mid, 0).sum() > 1:
                lo = mid
            else:
                hi = mid
        assert np.abs(p - np.maximum(v - 0.5 * (lo + hi), 0)).max() < 1e-12
        # nearest point: no feasible random point is closer
        for _ in range(10):
            z = rng.dirichlet(np.ones(21))
            assert np.linalg.norm(v - p) <= np.linalg.norm(v - z) + 1e-12


def _pair_model(H, W, seed, mode="exact"):
    rng = np.random.default_rng(seed)
    rgb = rng.uniform(0, 255, size=(H * W, 3)).astype(np.float32)
    kern = [O.Kernel(1, 2.0, 40.0, 4.0), O.Kernel(0, 1.5, 0.0, 1.5)]
    return O.Model(H, W, rgb, kern, mode=mode), rng


@pytest.mark.parametrize("leaf", [1, 2, 3, 5, 16, 61, 200])
def test_leaf_exact_dnc_with_exact_inner_is_the_brute_force(leaf):
    # exact filters above the cut plus exact pairs inside the leaves count
    # every pair once: the brute-force sums for any cutoff (here N = 60, so
    # 61 and 200 make the whole range one leaf)
    model, rng = _pair_model(6, 10, 1)
    K = model.dense_K()
    order = rng.permutation(60)
    Ub, Lb = O.lp_pair_sums_brute(K, order)
    U, Lo = O.lp_pair_sums_dnc(model, order, "exact", leaf=leaf)
    assert np.allclose(U, Ub, rtol=1e-12, atol=1e-12)
    assert np.allclose(Lo, Lb, rtol=1e-12, atol=1e-12)
    assert O.leaf_level(60, leaf) == (0 if leaf >= 60 else int(np.ceil(np.log2(60 / leaf))))


def test_leaf_exact_dnc_lattice_whole_leaf_and_sampling():
    model, rng = _pair_model(9, 13, 2, mode="lattice")
    N = 117
    order = rng.permutation(N)
    K = _pair_model(9, 13, 2)[0].dense_K()
    Ub, Lb = O.lp_pair_sums_brute(K, order)
    U, Lo = O.lp_pair_sums_dnc(model, order, "lattice", leaf=N)
    assert np.allclose(U, Ub, rtol=1e-12, atol=1e-12)
    assert np.allclose(Lo, Lb, rtol=1e-12, atol=1e-12)
    # sampled evaluation equals the full one at the sampled pixels
    U, Lo = O.lp_pair_sums_dnc(model, order, "lattice", leaf=8)
    at = rng.choice(N, 20, replace=False)
    Us, Ls = O.lp_pair_sums_dnc(model, order, "lattice", at=at, leaf=8)
    assert np.array_equal(Us[at], U[at]) and np.array_equal(Ls[at], Lo[at])


def test_leaf_exact_dnc_is_closer_to_the_exact_sums():
    # the lattice is least accurate on the few points of small nodes; summing
    # those exactly brings U - Lo closer to the brute force
    errs = {}
    for leaf in (0, 16, 64):
        e = []
        for seed in (3, 4, 5):
            model, rng = _pair_model(20, 24, seed, mode="lattice")
            K = _pair_model(20, 24, seed)[0].dense_K()
            order = rng.permutation(480)
            Ub, Lb = O.lp_pair_sums_brute(K, order)
            U, Lo = O.lp_pair_sums_dnc(model, order, "lattice", leaf=leaf)
            e.append(np.linalg.norm((U - Lo) - (Ub - Lb)) / np.linalg.norm(Ub - Lb))
        errs[leaf] = float(np.mean(e))
    print("relative error of U - Lo by leaf cutoff", errs)
    assert errs[64] < errs[16] < errs[0]
