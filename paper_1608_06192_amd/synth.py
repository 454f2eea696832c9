"""Seeded synthetic inputs shaped like the paper's segmentation workloads.

This module is the only code shared by the FP64 oracle tests and the GPU path.
It holds none of the method's arithmetic: it only draws images, unaries and
ground truths, in FP64 with NumPy's PCG64, and casts once at the end.

Two generators:

* ``rect_image``: a background plus four painted rectangles, RGB noise
  N(0, 10^2), unaries from N(0,1) logits (the tiny FP64 case).
* ``voronoi_image``: R random Voronoi regions with a mean colour and a label
  each, RGB noise N(0, 8^2), unaries from N(0,1) logits plus a +2 bias on the
  region's label; the region label doubles as a ground truth.

The paper evaluates on PASCAL VOC 2010 (images up to 500x375, 21 classes, with
the unaries of Kraehenbuehl and Koltun) and on Middlebury stereo pairs. Neither
is available here, so these generators stand in for them with the same image
sizes, label count and a piecewise-constant colour structure.

Layouts: ``rgb`` is float32 H*W x 3 in [0, 255], pixel index a = row*W + col;
``unary`` is N x L (float64 here; callers cast); ``gt`` is int32 N.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Image:
    H: int
    W: int
    rgb: np.ndarray      # (N, 3) float32, values in [0, 255]
    unary: np.ndarray    # (N, L) float64, -log softmax of the logits
    gt: np.ndarray       # (N,) int32 region label (voronoi) or argmax logit

    @property
    def N(self) -> int:
        return self.H * self.W

    @property
    def L(self) -> int:
        return self.unary.shape[1]


def _neg_log_softmax(z: np.ndarray) -> np.ndarray:
    zmax = z.max(axis=1, keepdims=True)
    lse = zmax + np.log(np.exp(z - zmax).sum(axis=1, keepdims=True))
    return lse - z


def rect_image(H: int, W: int, L: int, seed: int) -> Image:
    """Background + 4 rectangles, RGB ~ U[0,255]^3 each, noise N(0,10^2)."""
    g = np.random.Generator(np.random.PCG64(seed))
    img = np.empty((H, W, 3), dtype=np.float64)
    img[:] = g.uniform(0.0, 255.0, size=3)
    for _ in range(4):
        r0, r1 = np.sort(g.integers(0, H + 1, size=2))
        c0, c1 = np.sort(g.integers(0, W + 1, size=2))
        img[r0:r1, c0:c1] = g.uniform(0.0, 255.0, size=3)
    img += g.normal(0.0, 10.0, size=img.shape)
    np.clip(img, 0.0, 255.0, out=img)
    z = g.normal(0.0, 1.0, size=(H * W, L))
    unary = _neg_log_softmax(z)
    return Image(H, W, img.reshape(-1, 3).astype(np.float32), unary,
                 np.argmin(unary, axis=1).astype(np.int32))


def voronoi_image(H: int, W: int, L: int, seed: int, regions: int = 32,
                  noise: float = 8.0, bias: float = 2.0) -> Image:
    """Random Voronoi regions; each has a mean RGB and a label."""
    g = np.random.Generator(np.random.PCG64(seed))
    sr = g.uniform(0.0, H, size=regions)
    sc = g.uniform(0.0, W, size=regions)
    mean_rgb = g.uniform(0.0, 255.0, size=(regions, 3))
    lab = g.integers(0, L, size=regions)
    rows, cols = np.mgrid[0:H, 0:W]
    rows = rows.reshape(-1).astype(np.float64)
    cols = cols.reshape(-1).astype(np.float64)
    # nearest seed, lower index wins ties (argmin returns the first minimum)
    best = np.zeros(H * W, dtype=np.int64)
    best_d = np.full(H * W, np.inf)
    for r in range(regions):
        dd = (rows - sr[r]) ** 2 + (cols - sc[r]) ** 2
        take = dd < best_d
        best[take] = r
        best_d[take] = dd[take]
    rgb = mean_rgb[best] + g.normal(0.0, noise, size=(H * W, 3))
    np.clip(rgb, 0.0, 255.0, out=rgb)
    gt = lab[best].astype(np.int32)
    z = g.normal(0.0, 1.0, size=(H * W, L))
    z[np.arange(H * W), gt] += bias
    return Image(H, W, rgb.astype(np.float32), _neg_log_softmax(z), gt)


def batch_sizes(count: int, seed: int, lo: int = 240, hi: int = 500):
    """Image sizes for the uneven batch: H, W ~ U{lo..hi}."""
    g = np.random.Generator(np.random.PCG64(seed))
    H = g.integers(lo, hi + 1, size=count)
    W = g.integers(lo, hi + 1, size=count)
    return [(int(h), int(w)) for h, w in zip(H, W)]


def random_simplex_points(N: int, L: int, seed: int, sparsity: float = 0.0):
    """Random points of the product of simplices (rows >= 0 summing to 1).

    With ``sparsity`` > 0 that fraction of entries is set to exactly zero
    before renormalising, which creates the ties that projections produce.
    Every value is rounded to float32 first so that both precisions see the
    same numbers.
    """
    g = np.random.Generator(np.random.PCG64(seed))
    y = g.exponential(1.0, size=(N, L))
    if sparsity > 0:
        y[g.uniform(size=(N, L)) < sparsity] = 0.0
        empty = y.sum(axis=1) == 0
        y[empty, 0] = 1.0
    y = (y / y.sum(axis=1, keepdims=True)).astype(np.float32).astype(np.float64)
    return y


def potts(L: int) -> np.ndarray:
    """Potts label compatibility [i != j] as an L x L float64 matrix."""
    return 1.0 - np.eye(L)


def random_hst(L: int, seed: int, r: float = 2.0, top: float = 1.0,
               max_children: int = 3):
    """A random r-hierarchically well-separated tree over L labels: the
    labels are split recursively into 2..max_children random groups down
    to single labels; the edges from a node to its children all have one
    length, top / r^depth (so lengths fall by the factor r from the root
    down). Nodes 0..L-1 are the leaves (node k is label k), internal nodes
    follow in creation order, the root first among them.

    Returns (parent, length): int32 parent of every node (-1 for the root)
    and float64 length of the edge from every node to its parent (0 for the
    root)."""
    g = np.random.Generator(np.random.PCG64(seed))
    parent = list(range(L))            # placeholders for the leaves
    length = [0.0] * L
    parent_int, length_int = [], []

    def build(labels, par, depth, edge):
        if len(labels) == 1:
            parent[labels[0]] = par
            length[labels[0]] = edge
            return
        node = L + len(parent_int)
        parent_int.append(par)
        length_int.append(edge)
        k = int(g.integers(2, min(max_children, len(labels)) + 1))
        perm = g.permutation(labels)
        cuts = np.sort(g.choice(np.arange(1, len(labels)), size=k - 1, replace=False))
        child_edge = top / r ** depth
        for part in np.split(perm, cuts):
            build(sorted(int(v) for v in part), node, depth + 1, child_edge)

    build(list(range(L)), -1, 0, 0.0)
    return (np.array(parent + parent_int, dtype=np.int32),
            np.array(length + length_int, dtype=np.float64))


# The workloads used throughout (image sizes, label counts, seeds, iterations).
WORKLOADS = {
    "rect_32x24_L3": dict(kind="rect", H=24, W=32, L=3, seed=0, iters=20),
    "voronoi_320x213_L21": dict(kind="voronoi", H=213, W=320, L=21, seed=1,
                                iters=50, dc_outer=5, dc_inner=10),
    "voronoi_500x375_L21": dict(kind="voronoi", H=375, W=500, L=21, seed=2,
                                qp_iters=50, lp_steps=100),
    "voronoi_500x375_L21_diff": dict(kind="voronoi", H=375, W=500, L=21,
                                     seed=3, iters=10),
    "voronoi_batch16_L21": dict(kind="batch", count=16, size_seed=99,
                                seed0=100, L=21, iters=10),
}

# Kernel parameters of the two-kernel pixel compatibility (bilateral on
# position and RGB, spatial on position).
BILATERAL = dict(use_rgb=1, theta_pos=80.0, theta_rgb=13.0, weight=10.0)
SPATIAL = dict(use_rgb=0, theta_pos=3.0, theta_rgb=0.0, weight=3.0)


def make(name: str) -> Image:
    w = WORKLOADS[name]
    if w["kind"] == "rect":
        return rect_image(w["H"], w["W"], w["L"], w["seed"])
    if w["kind"] == "voronoi":
        return voronoi_image(w["H"], w["W"], w["L"], w["seed"])
    raise ValueError(name)


def make_batch(name: str = "voronoi_batch16_L21"):
    w = WORKLOADS[name]
    sizes = batch_sizes(w["count"], w["size_seed"])
    return [voronoi_image(h, ww, w["L"], w["seed0"] + j)
            for j, (h, ww) in enumerate(sizes)]
