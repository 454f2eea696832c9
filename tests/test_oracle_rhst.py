"""Pins of the oracle's LP for an r-HST metric (App. F, eq. rHST-LP,
Alg. rHST).

The pins: a tree worked out by hand (label sets, path-length metric); the
star tree, whose LP is the Potts LP of Sec. 6 exactly; the identity between
the LP at an integral point and the energy with the tree metric as the label
compatibility (with c_T twice the length of the edge above T); the
subgradient's objective against eq. rHST-LP evaluated directly; its
directional derivative and the subgradient inequality; and the descent
against an independent LP solver (scipy's HiGHS on the standard-form LP),
whose optimum lies below the brute-force minimum energy.
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1608_06192_amd import synth


def tiny_problem(N=6, L=3, seed=0, w=(4.0, 1.5)):
    rng = np.random.default_rng(seed)
    H, W = 2, N // 2
    rgb = rng.uniform(0, 255, size=(N, 3)).astype(np.float32)
    kern = [O.Kernel(1, 2.0, 60.0, w[0]), O.Kernel(0, 1.0, 0.0, w[1])]
    model = O.Model(H, W, rgb, kern, mode="exact")
    phi = rng.normal(0, 3.0, size=(N, L))
    return model, phi


def star(L):
    """root L over leaves 0..L-1, every leaf edge of length 1/2 (so the tree
    metric is the Potts [i != j])"""
    parent = np.array([L] * L + [-1], dtype=np.int32)
    length = np.array([0.5] * L + [0.0])
    return parent, length


def test_hand_worked_tree():
    # labels 0, 1 under node 3 (edges 0.5), node 3 and label 2 under the
    # root 4 (edges 1): d(0,1) = 1, d(0,2) = d(1,2) = 0.5 + 1 + 1 = 2.5
    parent = np.array([3, 3, 4, 4, -1])
    length = np.array([0.5, 0.5, 1.0, 1.0, 0.0])
    M = O.tree_label_sets(parent, 3)
    assert M.tolist() == [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 1, 1]]
    D = O.tree_metric(parent, length, 3)
    assert np.array_equal(D, [[0, 1, 2.5], [1, 0, 2.5], [2.5, 2.5, 0]])
    with pytest.raises(ValueError):
        O.tree_label_sets(np.array([1, 0, -1]), 2)
    # y_a(T) sums the marginals of T's labels
    y = np.array([[0.2, 0.3, 0.5], [0.6, 0.0, 0.4]])
    Y = O.tree_columns(y, M)
    assert np.allclose(Y, [[0.2, 0.3, 0.5, 0.5, 1.0], [0.6, 0.0, 0.4, 0.6, 1.0]],
                       atol=1e-15)


def test_random_hst_is_well_separated():
    # the generator's trees: equal edges from a node to its children, lengths
    # falling by r along every root-to-leaf path, and a metric
    for L, seed in ((5, 0), (21, 1), (21, 2)):
        parent, length = synth.random_hst(L, seed, r=2.0)
        n = parent.shape[0]
        assert (parent == -1).sum() == 1
        kids = {}
        for t in range(n):
            if parent[t] >= 0:
                kids.setdefault(int(parent[t]), []).append(t)
        assert all(t >= L for t in kids)            # labels are leaves
        for p, ch in kids.items():
            assert len({length[t] for t in ch}) == 1
            if parent[p] >= 0:
                assert length[ch[0]] * 2.0 <= length[p] + 1e-15
        D = O.tree_metric(parent, length, L)
        assert np.allclose(D, D.T) and (np.diag(D) == 0).all()
        assert (D[~np.eye(L, dtype=bool)] > 0).all()
        for k in range(L):
            assert (D <= D[:, [k]] + D[[k], :] + 1e-12).all()


def test_star_tree_is_the_potts_lp():
    # the star with c_T = 1 on the leaves (and c = 0 at the root) gives the
    # Potts LP's subgradient and objective exactly; a weight at the root adds
    # a per-pixel constant to g (the projection ignores it) and, for a
    # symmetric Kbar (the exact filter; the lattice's is not quite), 0 to S
    im = synth.voronoi_image(12, 10, 4, seed=5, regions=4)
    kern = [O.Kernel(**synth.BILATERAL), O.Kernel(**synth.SPATIAL)]
    model = O.Model(im.H, im.W, im.rgb, kern)
    pair = lambda o: O.lp_pair_sums_dnc(model, o, "lattice")
    y = synth.random_simplex_points(im.N, 4, seed=3, sparsity=0.3)
    parent, _ = star(4)
    M = O.tree_label_sets(parent, 4)
    c = np.array([1.0] * 4 + [0.0])
    g, S = O.rhst_lp_subgradient(im.unary, y, M, c, pair)
    gp, Sp = O.lp_subgradient(im.unary, y, pair)
    assert np.array_equal(g, gp) and S == Sp
    c[4] = 0.7
    K = O.Model(im.H, im.W, im.rgb, kern, mode="exact").dense_K()
    pair = lambda o: O.lp_pair_sums_brute(K, o)
    y = O.project_simplex(y)
    gp, Sp = O.lp_subgradient(im.unary, y, pair)
    g2, S2 = O.rhst_lp_subgradient(im.unary, y, M, c, pair)
    shift = g2 - gp
    assert np.allclose(shift, shift[:, :1], rtol=0, atol=1e-9)
    assert abs(S2 - Sp) <= 1e-9 * abs(Sp)
    assert np.allclose(O.project_simplex(y - 1e-3 * g2), O.project_simplex(y - 1e-3 * gp),
                       rtol=0, atol=1e-12)


@pytest.mark.parametrize("L,seed", [(3, 0), (5, 1), (6, 2)])
def test_integral_objective_is_the_tree_metric_energy(L, seed):
    # with c_T = 2 x (length of the edge above T), eq. rHST-LP at an integral
    # point is the energy with mu = d^t (the path length between the labels)
    model, phi = tiny_problem(N=8, L=L, seed=seed)
    K = model.dense_K()
    parent, length = synth.random_hst(L, seed + 10)
    M = O.tree_label_sets(parent, L)
    c = 2.0 * length
    D = O.tree_metric(parent, length, L)
    pair = lambda o: O.lp_pair_sums_brute(K, o)
    rng = np.random.default_rng(seed)
    for _ in range(5):
        x = rng.integers(0, L, size=8)
        E = O.energy_dense(K, phi, D, x)
        assert abs(O.S_rhst_dense(K, phi, O.onehot(x, L), M, c) - E) <= 1e-12 * abs(E)
        _, S = O.rhst_lp_subgradient(phi, O.onehot(x, L), M, c, pair)
        assert abs(S - E) <= 1e-12 * abs(E)


def test_subgradient_objective_derivative_and_inequality():
    model, phi = tiny_problem(N=8, L=5, seed=4)
    K = model.dense_K()
    parent, length = synth.random_hst(5, 7)
    M = O.tree_label_sets(parent, 5)
    c = 2.0 * length
    pair = lambda o: O.lp_pair_sums_brute(K, o)
    rng = np.random.default_rng(9)
    y = rng.random((8, 5)) + 0.1
    y /= y.sum(axis=1, keepdims=True)        # interior: no ties among y(T)
    g, S = O.rhst_lp_subgradient(phi, y, M, c, pair)
    assert abs(S - O.S_rhst_dense(K, phi, y, M, c)) <= 1e-12 * abs(S)
    # directional derivative: inside the region where no y(T) order changes
    # the objective is linear with gradient g
    d = rng.normal(size=y.shape)
    d -= d.mean(axis=1, keepdims=True)
    Y, dY = O.tree_columns(y, M), O.tree_columns(d, M)
    gaps = [np.diff(np.sort(Y[:, T])) for T in range(M.shape[0]) if c[T] != 0]
    gap = min(v.min() for v in gaps)
    assert gap > 0
    eps = 0.25 * gap / np.abs(dY).max()
    fd = (O.S_rhst_dense(K, phi, y + eps * d, M, c) - S) / eps
    assert abs(fd - (g * d).sum()) <= 1e-6 * np.abs(g * d).sum()
    # subgradient inequality of a convex function
    for _ in range(50):
        z = O.project_simplex(rng.random((8, 5)) ** 3)
        assert O.S_rhst_dense(K, phi, z, M, c) >= S + (g * (z - y)).sum() - 1e-10


def _rhst_optimum_highs(K, phi, M, c):
    """min phi^T y + sum_{a<b} K_ab sum_T c_T t_ab(T), t >= |y_a(T) - y_b(T)|
    with y_a(T) the sum of y_a over L(T), y in the product of simplices"""
    from scipy.optimize import linprog
    N, L = phi.shape
    nodes = [T for T in range(M.shape[0]) if c[T] != 0]
    pairs = [(a, b) for a in range(N) for b in range(a + 1, N)]
    ny, nt = N * L, len(pairs) * len(nodes)
    cost = np.concatenate([phi.ravel(),
                           [K[a, b] * c[T] for a, b in pairs for T in nodes]])
    A, rhs = [], []
    for p, (a, b) in enumerate(pairs):
        for q, T in enumerate(nodes):
            for sgn in (1, -1):
                row = np.zeros(ny + nt)
                for i in np.nonzero(M[T])[0]:
                    row[a * L + i] = sgn
                    row[b * L + i] = -sgn
                row[ny + p * len(nodes) + q] = -1
                A.append(row)
                rhs.append(0.0)
    Aeq = np.zeros((N, ny + nt))
    for a in range(N):
        Aeq[a, a * L:(a + 1) * L] = 1
    res = linprog(cost, A_ub=np.array(A), b_ub=rhs, A_eq=Aeq, b_eq=np.ones(N),
                  bounds=[(0, None)] * (ny + nt), method="highs")
    assert res.status == 0
    return res.fun


@pytest.mark.parametrize("L,seed,beta0,steps", [(3, 21, 1.0, 20000), (4, 22, 0.1, 3000)])
def test_rhst_descent_approaches_the_lp_optimum(L, seed, beta0, steps):
    # the subgradient method with beta_t = beta0 / (1 + t) closes the gap
    # slowly (at 3000 steps the first case is still 13 % away), hence the
    # step counts
    model, phi = tiny_problem(N=6, L=L, seed=seed)
    K = model.dense_K()
    parent, length = synth.random_hst(L, seed)
    M = O.tree_label_sets(parent, L)
    c = 2.0 * length
    opt = _rhst_optimum_highs(K, phi, M, c)
    Emin, _ = O.brute_force_min(K, phi, O.tree_metric(parent, length, L))
    assert opt <= Emin + 1e-9
    _, best, best_y, hist = O.rhst_lp_descent(
        phi, O.softmax_neg(phi), M, c, steps, beta0, lambda o: O.lp_pair_sums_brute(K, o))
    assert best >= opt - 1e-9
    assert best - opt < 2e-2 * max(1.0, abs(opt))
    assert abs(O.S_rhst_dense(K, phi, best_y, M, c) - best) <= 1e-9 * max(1.0, abs(best))
