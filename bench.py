"""Benchmark of the dense-CRF hot path on one MI355X.

Workload: a 500x375 synthetic Voronoi image (N = 187,500 pixels), L = 21
labels, FP32, a bilateral kernel (w=10, theta_alpha=80, theta_beta=13) and a
spatial kernel (w=3, theta_gamma=3), Potts compatibility.

A timed step is one Frank-Wolfe iteration on the convex QP relaxation
(gradient, conditional gradient, one lattice filter of the conditional
gradient, exact line search, update), run inside one solve of K iterations
whose per-solve setup (linear term, first filter of y0, final update) is part
of the timed region. `value` is Frank-Wolfe iterations per second.

Beside it the JSON line reports:
* lattice_filter: one dense L=21 lattice filter K'Y (splat, blur, slice) at
  the same shape, timed with HIP events, in algorithmic GB/s;
* roofline: the dominant kernel of the step, its algorithmic bytes per launch
  over its average launch time (HIP events on the library's stream), against
  the 8 TB/s HBM peak;
* cpu_baseline: the FP64 oracle's Frank-Wolfe iterations on the host, one
  thread, over a bounded sample of iterations of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = ("lattice-filter GB/s + Frank-Wolfe QP iters/s @500×375 L=21; "
          "fwd+bwd vs plain")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def lattice_bytes(N, C, e, lattices):
    """Algorithmic bytes of one dense filter call over C channels:
    in + out (2 N C e); per pixel and kernel the d+1 vertex ids (4 B) and
    weights (e B) read by splat and again by slice; per kernel the splat write,
    the d+1 blur passes (read + write each, plus the two neighbour rows and
    the neighbour ids) and the slice read of M x C vertex values."""
    b = 2 * N * C * e
    for d, M in lattices:
        b += 2 * N * (d + 1) * (4 + e)
        b += (2 * (d + 1) + 2) * M * C * e
        b += (d + 1) * 8 * M
    return b


def fw_step_bytes(N, L, e, lattices):
    """Algorithmic bytes of one Frank-Wolfe iteration: k_fw_lmo reads y, P_y,
    P_s, c and writes y, P_y (6 N L e) plus labels; k_fw_slice reads y and
    writes P_s (2 N L e); the one-hot splat and the slice read the per-pixel
    vertex ids and weights; the blur moves the vertex arrays."""
    b = 8 * N * L * e + 2 * N * 4
    for d, M in lattices:
        b += 2 * N * (d + 1) * (4 + e)
        b += (2 * (d + 1) + 2) * M * L * e + (d + 1) * 8 * M
    return b


def lmo_bytes(N, L, e, lattices):
    """k_fw_lmo alone: 6 N L e (y, P_y, P_s, c in; y, P_y out), the labels,
    the vertex ids and weights of the one-hot splat and its N (d+1) scattered
    value updates."""
    b = 6 * N * L * e + 2 * N * 4
    for d, M in lattices:
        b += N * (d + 1) * (4 + e) + N * (d + 1) * e
    return b


def cpu_baseline(im, kernels, mu, iters):
    """The FP64 oracle's Frank-Wolfe on the same image, one host thread."""
    from threadpoolctl import threadpool_limits
    from oracle import oracle as O
    with threadpool_limits(limits=1):
        os.environ["OMP_NUM_THREADS"] = "1"
        model = O.Model(im.H, im.W, im.rgb, kernels)
        qp = O.QP(model, im.unary, mu)
        y0 = O.softmax_neg(im.unary)
        O.frank_wolfe(qp, y0, 1)                    # warm the code paths
        t0 = time.perf_counter()
        O.frank_wolfe(qp, y0, iters)
        dt = time.perf_counter() - t0
    return dict(value=iters / dt, unit="FW iters/s", cores=1, kind="oracle",
                sample=f"{iters} Frank-Wolfe iterations (plus the solve's "
                       f"first filter of y0) of the FP64 oracle on the same "
                       f"500x375 L=21 image, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--filter-reps", type=int, default=200)
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--lp-steps", type=int, default=3)
    ap.add_argument("--lp-beta0", type=float, default=1e-4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "a multi-GPU run is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1608_06192_amd import dcrf, synth

    name = "voronoi_500x375_L21"
    im = synth.make(name)
    kernels = [synth.BILATERAL, synth.SPATIAL]
    mu_np = synth.potts(im.L)
    dev = torch.device("cuda:0")
    f32 = torch.float32
    N, L = im.N, im.L

    ctx = dcrf.Context(0)
    rgb = torch.from_numpy(im.rgb).to(dev)
    ctx.set_image(im.H, im.W, rgb, kernels, dtype=f32)
    lat = [ctx.lattice_info(m) for m in range(2)]
    log(f"[bench] {name}: N={N} L={L} lattices (d, M) = {lat}")

    phi = torch.from_numpy(im.unary).to(dev, f32)
    mu = torch.from_numpy(mu_np).to(dev, f32)
    e = np.exp(-(im.unary - im.unary.min(axis=1, keepdims=True)))
    y0 = torch.from_numpy(e / e.sum(axis=1, keepdims=True)).to(dev, f32)

    # ---- warmup + timed Frank-Wolfe solve ---------------------------------
    y = y0.clone()
    ctx.qp_frank_wolfe(phi, mu, y, args.warmup, trace=False)
    torch.cuda.synchronize()
    y = y0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.qp_frank_wolfe(phi, mu, y, args.steps, trace=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    log(f"[bench] FW {args.steps} iterations: {dt * 1e3:.2f} ms, "
        f"{ms_per_step * 1e3:.1f} us/iter")

    # ---- per-kernel times of the step (HIP events) ------------------------
    ctx.set_profiling(True)
    yp = y0.clone()
    prof_iters = min(args.steps, 200)
    ctx.qp_frank_wolfe(phi, mu, yp, prof_iters, trace=False)
    prof = ctx.profile()
    ctx.set_profiling(False)
    per_iter = {k: (ms / max(n, 1), n) for k, (ms, n) in prof.items() if n}
    log("[bench] per-kernel average launch time (HIP events):")
    for k, (ms, n) in per_iter.items():
        log(f"    {k:16s} {ms * 1e3:9.2f} us  x{n}")

    # ---- the dense lattice filter -----------------------------------------
    Y = torch.rand(N, L, device=dev, dtype=f32)
    out = torch.empty_like(Y)
    for _ in range(10):
        ctx.filter(Y, out=out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.filter_reps):
        ctx.filter(Y, out=out)
    ev1.record()
    torch.cuda.synchronize()
    f_ms = ev0.elapsed_time(ev1) / args.filter_reps
    f_bytes = lattice_bytes(N, L, 4, lat)
    filt = dict(ms=f_ms, GBps=f_bytes / f_ms / 1e6, bytes=f_bytes,
                frac_of_hbm_peak=f_bytes / f_ms / 1e6 / HBM_PEAK_GBPS)
    log(f"[bench] dense filter L=21: {f_ms * 1e3:.1f} us, "
        f"{filt['GBps']:.0f} GB/s algorithmic")

    # ---- LP subgradient steps from the QP solution -------------------------
    lp = None
    if args.lp_steps > 0:
        ylp = y.clone()                       # the timed QP solve's result
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        best, hist = ctx.lp_descent(phi, ylp, args.lp_steps, args.lp_beta0)
        torch.cuda.synchronize()
        lp_ms = (time.perf_counter() - t0) * 1e3 / args.lp_steps
        lp = dict(ms_per_step=lp_ms, steps=args.lp_steps, beta0=args.lp_beta0,
                  S_LP_first=hist[0], S_LP_best=best)
        log(f"[bench] LP subgradient step (divide and conquer, 21 labels, "
            f"{int(np.ceil(np.log2(N)))} levels): {lp_ms:.1f} ms")

    # ---- roofline of the dominant kernel of the step ----------------------
    dom = max(per_iter, key=lambda k: per_iter[k][0] * per_iter[k][1])
    dom_ms = per_iter[dom][0]
    if dom == "k_fw_lmo":
        dom_bytes = lmo_bytes(N, L, 4, lat)
    elif dom == "k_fw_slice":
        dom_bytes = 2 * N * L * 4 + N * 4 + sum(
            N * (d + 1) * 8 + N * (d + 1) * L * 4 for d, M in lat)
    else:  # one blur pass over both lattices
        dom_bytes = sum((4 * M * L * 4 + 2 * M * 4) for d, M in lat)
    achieved = dom_bytes / dom_ms / 1e6
    roofline = dict(bound="hbm", kernel=dom, achieved=achieved,
                    peak=HBM_PEAK_GBPS, unit="GB/s", frac=achieved / HBM_PEAK_GBPS,
                    traffic=None, bytes_per_launch=dom_bytes,
                    avg_launch_us=dom_ms * 1e3)

    res = dict(metric=METRIC, value=args.steps / dt, unit="FW iters/s",
               n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=ms_per_step, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="voronoi 500x375, L=21, FP32, Potts, "
                                    "bilateral w=10 ta=80 tb=13 + spatial "
                                    "w=3 tg=3", H=im.H, W=im.W, L=L,
                           step="one Frank-Wolfe QP iteration",
                           lattice_vertices=[M for d, M in lat]),
               lattice_filter=filt, step_bytes=fw_step_bytes(N, L, 4, lat),
               per_kernel_us={k: v[0] * 1e3 for k, v in per_iter.items()},
               lp=lp, roofline=roofline)
    if not args.no_cpu:
        log(f"[bench] CPU baseline: {args.cpu_iters} oracle FW iterations ...")
        res["cpu_baseline"] = cpu_baseline(im, kernels, mu_np, args.cpu_iters)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
