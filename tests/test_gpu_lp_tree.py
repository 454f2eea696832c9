"""GPU parity of the LP for an r-HST metric (App. F, eq. rHST-LP, Alg. rHST).

The subtree columns y(T) decide the orders, which are index work and must
agree exactly: the inputs are dyadic marginals (multiples of 1/64), whose
subtree sums are exact in both precisions, so both sides sort identical
values (with many ties). g must then agree within rtol * (|phi| + sum over
the label's weighted subtrees of c_T (|U| + |Lo|)), rtol 1e-10 in FP64 and
1e-5 in FP32, U and Lo being the oracle's two triangular sums per subtree.
"""

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1608_06192_amd import synth

pytestmark = pytest.mark.gpu

KERNELS = [synth.BILATERAL, synth.SPATIAL]
OKERNELS = [O.Kernel(**synth.BILATERAL), O.Kernel(**synth.SPATIAL)]


def dev():
    return torch.device("cuda:0")


def T(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev(), dtype)


def ctx_for(im, dtype, mode="lattice"):
    from paper_1608_06192_amd import dcrf
    print(f"[case] tree LP {im.H}x{im.W} L={im.L} {dtype} {mode}", flush=True)
    c = dcrf.Context(0)
    c.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev()), KERNELS, dtype=dtype)
    if mode != "lattice":
        c.set_filter_mode(mode)
    return c


def dyadic_points(N, L, seed, q=64):
    """rows of multiples of 1/q summing to 1 (a multinomial draw of q units)"""
    g = np.random.default_rng(seed)
    return g.multinomial(q, np.full(L, 1.0 / L), size=N).astype(np.float64) / q


def tree(L, seed):
    parent, length = synth.random_hst(L, seed)
    return parent, 2.0 * length


def oracle_tree(im, y, parent, c, phi, at=None):
    """(g, S, mag) of the oracle, mag being the bound's scale per entry"""
    model = O.Model(im.H, im.W, im.rgb, OKERNELS)
    M = O.tree_label_sets(parent, im.L)
    rec = []

    def pair(order):
        U, Lo = O.lp_pair_sums_dnc(model, order, "lattice")
        rec.append((U, Lo))
        return U, Lo
    g, S = O.rhst_lp_subgradient(phi, y, M, c, pair)
    mag = np.abs(phi).copy()
    weighted = [t for t in range(M.shape[0]) if c[t] != 0]
    for t, (U, Lo) in zip(weighted, rec):
        for k in np.nonzero(M[t])[0]:
            mag[:, k] += c[t] * (np.abs(U) + np.abs(Lo))
    return g, S, mag


@pytest.mark.parametrize("H,W,L,dtype,rtol", [
    (24, 32, 5, torch.float64, 1e-10),
    (13, 11, 7, torch.float64, 1e-10),
    (48, 64, 6, torch.float32, 1e-5),
])
def test_tree_subgradient_matches_oracle(H, W, L, dtype, rtol):
    im = synth.voronoi_image(H, W, L, seed=H * W + L, regions=6)
    y = dyadic_points(im.N, L, seed=L)
    parent, c = tree(L, seed=H + L)
    phi = im.unary.astype(np.float32).astype(np.float64) if dtype == torch.float32 \
        else im.unary
    ctx = ctx_for(im, dtype)
    g, S = ctx.lp_subgradient_tree(T(phi, dtype), T(y, dtype), parent, c)
    go, So, mag = oracle_tree(im, y, parent, c, phi)
    err = np.abs(g.cpu().numpy().astype(np.float64) - go)
    print(f"[tree lp] {H}x{W} L={L} nodes={len(parent)}: max rel err "
          f"{(err / mag).max():.3g}, S gpu {S:.12g} oracle {So:.12g}", flush=True)
    assert (err <= rtol * mag).all()
    assert abs(S - So) <= rtol * (mag * y).sum()


def test_star_tree_is_the_potts_lp_on_the_gpu():
    # the star with unit leaf weights (root weight 0) is the Potts LP: the
    # same pair sums on the same columns, so the two calls agree to the
    # rounding of the atomically summed splat
    im = synth.voronoi_image(40, 30, 4, seed=8, regions=5)
    L = im.L
    ctx = ctx_for(im, torch.float64)
    phi = T(im.unary, torch.float64)
    y = T(synth.random_simplex_points(im.N, L, seed=2, sparsity=0.3), torch.float64)
    parent = [L] * L + [-1]
    c = [1.0] * L + [0.0]
    g, S = ctx.lp_subgradient_tree(phi, y, parent, c)
    gp, Sp = ctx.lp_subgradient(phi, y)
    assert (g - gp).abs().max().item() <= 1e-9 * gp.abs().max().item()
    assert abs(S - Sp) <= 1e-12 * abs(Sp)


def test_tree_integral_objective_is_the_tree_metric_energy():
    # exact filter (symmetric Kbar): at an integral point the objective is
    # the energy with mu = the tree's path lengths (c_T = 2 l_T), the GPU's
    # own dense-mu energy on the other side
    im = synth.voronoi_image(12, 16, 5, seed=4, regions=5)
    L = im.L
    parent, length = synth.random_hst(L, 3)
    D = O.tree_metric(parent, length, L)
    ctx = ctx_for(im, torch.float64, mode="exact")
    phi = T(im.unary, torch.float64)
    x = np.random.default_rng(2).integers(0, L, size=im.N).astype(np.int32)
    _, S = ctx.lp_subgradient_tree(phi, T(O.onehot(x, L), torch.float64), parent,
                                   2.0 * length)
    E = ctx.energy(phi, T(D, torch.float64), torch.from_numpy(x).to(dev()))
    print(f"[tree lp] integral S {S:.12g}, energy {E:.12g}", flush=True)
    assert abs(S - E) <= 1e-10 * abs(E)


def test_tree_descent_fp64_matches_oracle():
    # Alg. rHST's loop, one step at a time from the oracle's iterates: after
    # a projection many pixels hold all their mass inside a subtree, so y(T)
    # is 1 up to rounding there, and the order of those near-ties (which
    # decides the nodes of the divide and conquer, and so the lattice's
    # approximation) follows the last bits of the projection. Each GPU step
    # therefore starts from the oracle's y_t; S(y_t) must agree within 1e-9
    # and y_{t+1} within 1e-9.
    im = synth.voronoi_image(24, 32, 5, seed=17, regions=6)
    L = im.L
    parent, c = tree(L, seed=5)
    model = O.Model(im.H, im.W, im.rgb, OKERNELS)
    M = O.tree_label_sets(parent, L)
    pair = lambda o: O.lp_pair_sums_dnc(model, o, "lattice")
    ctx = ctx_for(im, torch.float64)
    phi = T(im.unary, torch.float64)
    y = O.softmax_neg(im.unary)
    beta0 = 1e-3
    for t in range(3):
        beta = beta0 / (1.0 + t)
        g, S = O.rhst_lp_subgradient(im.unary, y, M, c, pair)
        y_next = O.project_simplex(y - beta * g)
        yg = T(y, torch.float64)
        best_y = torch.empty_like(yg)
        best, hist = ctx.lp_descent_tree(phi, yg, parent, c, 1, beta, best_y=best_y)
        err = np.abs(yg.cpu().numpy() - y_next).max()
        print(f"[tree descent] t={t} S gpu {hist[0]:.12g} oracle {S:.12g}; "
              f"max |dy| {err:.2e}", flush=True)
        assert abs(hist[0] - S) <= 1e-9 * abs(S), t
        assert best == hist[0] and torch.equal(best_y, T(y, torch.float64))
        assert err < 1e-9, t
        y = y_next


def test_tree_subgradient_fp32_500x375_sampled_entries():
    # 500x375, L = 21, FP32, a random 2-HST over the 21 labels: the whole
    # N x L subgradient from one GPU call; the oracle evaluates the columns of
    # the label with the fewest weighted subtrees above it at sampled pixels
    # (both ends and the middle of every subtree order included)
    im = synth.make("voronoi_500x375_L21")
    N, L = im.N, im.L
    parent, c = tree(L, seed=21)
    M = O.tree_label_sets(parent, L)
    y = dyadic_points(N, L, seed=3)
    phi32 = im.unary.astype(np.float32).astype(np.float64)
    ctx = ctx_for(im, torch.float32)
    g, _ = ctx.lp_subgradient_tree(T(phi32, torch.float32), T(y, torch.float32), parent, c)
    g = g.cpu().numpy().astype(np.float64)
    model = O.Model(im.H, im.W, im.rgb, OKERNELS)
    depth = [sum(1 for t in range(len(parent)) if M[t, k] and c[t] != 0) for k in range(L)]
    k = int(np.argmin(depth))
    Y = O.tree_columns(y, M)
    rng = np.random.default_rng(5)
    at = rng.choice(N, 160, replace=False)
    orders = {t: O.sorted_order(Y[:, t]) for t in range(len(parent)) if M[t, k] and c[t] != 0}
    for order in orders.values():
        at = np.concatenate([at, order[[0, 1, N // 2 - 1, N // 2, N - 2, N - 1]]])
    at = np.unique(at)
    go = phi32[at, k].copy()
    mag = np.abs(phi32[at, k])
    for t, order in orders.items():
        U, Lo = O.lp_pair_sums_dnc(model, order, "lattice", at=at)
        go += c[t] * (U[at] - Lo[at])
        mag += c[t] * (np.abs(U[at]) + np.abs(Lo[at]))
    rel = np.abs(g[at, k] - go) / mag
    print(f"[tree lp 500x375] label {k} under {len(orders)} weighted subtrees: "
          f"max rel err {rel.max():.3g}", flush=True)
    assert (rel <= 1e-5).all()


def test_malformed_trees_are_rejected():
    from paper_1608_06192_amd import dcrf
    im = synth.voronoi_image(8, 8, 3, seed=1, regions=3)
    ctx = ctx_for(im, torch.float64)
    phi = T(im.unary, torch.float64)
    y = T(O.softmax_neg(im.unary), torch.float64)
    bad = [
        ([3, 3, 4, 4, 3], [1.0] * 5),          # cycle between 3 and 4, no root
        ([3, 3, 3, -1, -1], [1.0] * 5),        # two roots
        ([1, 3, 3, -1], [1.0] * 4),            # a label's node as a parent
        ([3, 3, 3, -1], [1.0, -1.0, 1.0, 0.0]),  # negative weight
        ([3, 3, 3, 7], [1.0] * 4),             # parent out of range
        ([2, -1], [1.0, 0.0]),                 # fewer nodes than labels
    ]
    for parent, c in bad:
        with pytest.raises(dcrf.DcrfError) as e:
            ctx.lp_subgradient_tree(phi, y, parent, c)
        assert dcrf.STATUS[e.value.status] == "DCRF_EINVAL", parent


def test_tree_with_a_chain_of_single_child_nodes():
    # internal nodes with one child repeat their child's column: the oracle
    # and the GPU must both count every weighted node; labels 0, 1 under node
    # 4, node 4 alone under node 5, node 5 and label 2 and label 3 under the
    # root 6
    im = synth.voronoi_image(18, 22, 4, seed=16, regions=4)
    parent = [4, 4, 6, 6, 5, 6, -1]
    c = [1.0, 1.0, 2.0, 2.0, 0.5, 0.25, 0.0]
    y = dyadic_points(im.N, 4, seed=17)
    ctx = ctx_for(im, torch.float64)
    g, S = ctx.lp_subgradient_tree(T(im.unary, torch.float64), T(y, torch.float64),
                                   parent, c)
    go, So, mag = oracle_tree(im, y, np.array(parent), np.array(c), im.unary)
    assert (np.abs(g.cpu().numpy() - go) <= 1e-10 * mag).all()
    assert abs(S - So) <= 1e-10 * (mag * y).sum()
