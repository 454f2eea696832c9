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
  over its average launch time (HIP events carried by the kernel dispatches
  on the library's stream), against the 8 TB/s HBM peak;
* cpu_baseline: the FP64 oracle's Frank-Wolfe iterations on the host's
  cores (and on one thread beside it), over a bounded sample of iterations
  of the same workload;
* dc_neg: microseconds per step of the DC relaxation for negative
  semi-definite compatibilities at the same shape (one filter call and the
  per-pixel closed form per step);
* lp: the LP relaxation's projected subgradient descent (divide and conquer,
  100 steps from the timed QP solution): milliseconds per step and the
  first, best and last S_LP; 20 steps of it with leaf-exact nodes of at
  most 256 positions; the same descent restricted to the labels that
  the QP solution's argmax uses; and Kleinberg-Tardos
  rounding of the best LP point (8 L seeded rounds) with its energy beside
  the argmax's; and the LP for a tree metric (a seeded 2-HST over the 21
  labels, 10 steps): milliseconds per step;
* qp_dc / qp_dcneg: 50 Frank-Wolfe iterations and then the generic DC
  relaxation (5 concave-convex steps of 10 inner iterations) or DC_neg (5
  steps) at 320x213, L=21, FP32, with the energy of the rounded labelling;
* diff: 10 unrolled Frank-Wolfe iterations at 500x375, L=21, FP32 (seed 3):
  forward with checkpoints, reverse sweep, and the plain forward beside them;
* batch: 16 Voronoi images of sizes U{240..500}^2, L=21, FP32, 10 Frank-
  Wolfe iterations each: the batched forward and forward+backward (one launch
  per stage over the concatenated lattices, autotuned launch shapes) against
  16 sequential single-image forwards and forward+backwards; batch.persistent:
  the same with every iteration of the forward in one cooperative launch;
* lattice_error: the lattice filter against the exact O(N^2) sum at 320x213
  (ratio of means, cosine and relative 2-norm error of K'Y for a random Y),
  and the same for the separable mode (spatial kernel exact, bilateral on
  the lattice);
* lattice_filter.separable_ms / separable_fw_iteration_us: the dense filter
  and a Frank-Wolfe iteration in the separable mode at 500x375;
* lattice_filter.fused_splat_fw_iteration_us: a Frank-Wolfe iteration with
  the one-hot splat done pixel by pixel inside the conditional-gradient
  kernel instead of its own vertex-major launch.

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


def class_bytes(name, N, L, e, lattices, group=2):
    """Algorithmic bytes per launch of the kernel class `name` of the
    Frank-Wolfe step (the names of the library's profiling classes):
    * k_fw_lmo_rows: y, P_y, P_s, c in, y and P_y out (6 N L e), the previous
      and the new labels (2 N 4);
    * k_splat_labels_lds / _chunks: the labels (N 4), per lattice the (pixel, weight)
      entries (N (d+1) (4 + e)) and the vertex rows written (M L e);
    * k_fw_slice_rows: y in and P_s out (2 N L e), labels and r (N (4 + e)),
      per lattice the per-pixel vertex ids and weights and the vertex rows
      read;
    * k_blur_group: per launch, over the lattices it covers, each vertex row
      in and out (2 M L e) and the path table (M 3^G 4)."""
    if name == "k_fw_lmo_rows":
        return 6 * N * L * e + 2 * N * 4
    if name in ("k_splat_labels_lds", "k_splat_labels_chunks"):
        return N * 4 + sum(N * (d + 1) * (4 + e) + M * L * e for d, M in lattices)
    if name == "k_fw_slice_rows":
        return 2 * N * L * e + N * (4 + e) + sum(
            N * (d + 1) * (4 + e) + M * L * e for d, M in lattices)
    if name in ("k_blur_group", "k_blur_pass"):
        group = 1 if name == "k_blur_pass" else group
        groups = [-(-(d + 1) // group) for d, M in lattices]
        tot = sum(g * (2 * M * L * e + M * 3 ** group * 4)
                  for g, (d, M) in zip(groups, lattices))
        return tot / max(groups)
    raise KeyError(name)


def cpu_baseline(im, kernels, mu, iters):
    """The FP64 oracle's Frank-Wolfe on the same image on the host's cores:
    its lattice filter runs OpenMP threads (over output elements in the blur
    and slice, over channels in the splat), its other steps are NumPy. Timed
    with every thread the OpenMP runtime offers, then with one thread for
    comparison."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import oracle as O
    model = O.Model(im.H, im.W, im.rgb, kernels)
    qp = O.QP(model, im.unary, mu)
    y0 = O.softmax_neg(im.unary)
    O.frank_wolfe(qp, y0, 1)                    # warm the code paths
    omp = [p["num_threads"] for p in threadpool_info() if p.get("user_api") == "openmp"]
    cores = max(omp) if omp else 1
    t0 = time.perf_counter()
    O.frank_wolfe(qp, y0, iters)
    dt = time.perf_counter() - t0
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        O.frank_wolfe(qp, y0, iters)
        dt1 = time.perf_counter() - t1
    return dict(value=iters / dt, unit="FW iters/s", cores=cores, kind="oracle",
                sample=f"{iters} Frank-Wolfe iterations (plus the solve's "
                       f"first filter of y0) of the FP64 oracle on the same "
                       f"500x375 L=21 image, {dt:.1f} s on {cores} threads",
                one_thread=dict(value=iters / dt1, seconds=dt1))


# ---- profiler summaries ----------------------------------------------------

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fw_step_500x375_L21_hbm_traffic.txt")
CALIB_BYTES = 256 << 20   # the --calib-copy kernel reads and writes 256 MiB


def source_digest():
    """sha256 over the library's kernel sources (file names and contents)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1608_06192_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        h.update(name.encode())
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _short(name):
    """kernel name without namespaces and parameter list (template arguments
    kept, so that instantiations stay apart)"""
    n = name[5:] if name.startswith("void ") else name
    n = n.replace("dcrf::(anonymous namespace)::", "").replace("dcrf::", "")
    depth, out = 0, []
    for ch in n:           # cut at the parameter list: the first '(' outside <>
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            break
        out.append(ch)
    return "".join(out).strip()


def summarize_pmc(fetch_csv, write_csv, command):
    """Write TRAFFIC_FILE from the counter CSVs of two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of `bench.py
    --calib-copy`. The calibration dispatches are those of the plain copy of
    CALIB_BYTES (torch.mul; the counter of its 256 MiB read shows half of it on
    this part), told apart from the cache-flush fill by the kernel's name."""
    import csv
    per = {}
    calib = {}
    for ctr, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != ctr:
                continue
            v = float(r["Counter_Value"])
            k = _short(r["Kernel_Name"])
            if "MulFunctor" in r["Kernel_Name"] and v * 1024 >= 64 * (1 << 20):
                calib.setdefault(ctr, []).append(v)   # the 256 MiB copy (torch.mul)
            elif k.startswith("k_"):
                per.setdefault(k, {}).setdefault(ctr, []).append(v)
    lines = ["# HBM traffic per dispatch of the library's kernels, from the L2-to-memory",
             "# byte counters of rocprofv3 (KiB per dispatch, averaged over dispatches),",
             "# with a plain 256 MiB copy kernel in the same run as calibration.",
             "# Workload: bench.py (voronoi 500x375, L=21, FP32, both kernels).",
             "# Commands (repository root on the GPU host, TMPDIR=/tmp):"]
    lines += ["#   " + c for c in command]
    lines += ["# Summary written by: python bench.py --summarize-pmc <fetch csv> <write csv>",
              f"source_sha256 {source_digest()}"]
    kib = CALIB_BYTES / 1024
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        vals = calib.get(ctr, [])
        avg = sum(vals) / len(vals) if vals else float("nan")
        lines.append(f"calib {ctr} measured_kib {avg:.1f} expected_kib {kib:.1f} "
                     f"dispatches {len(vals)}")
    for k in sorted(per):
        f = per[k].get("FETCH_SIZE", [])
        w = per[k].get("WRITE_SIZE", [])
        if not f or not w:
            continue
        lines.append(f"kernel {k.replace(' ', '')} fetch_kib {sum(f) / len(f):.1f} "
                     f"write_kib {sum(w) / len(w):.1f} dispatches {len(f)}")
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_busy(csv_path, out_path, command):
    """Write a summary of the texture-address (TA) and texture-data (TD) unit
    busy fractions per kernel from one rocprofv3 --pmc run of TA_BUSY_avr,
    TD_TD_BUSY_sum, TCC_BUSY_avr and GRBM_GUI_ACTIVE: busy cycles over the
    active cycles of the dispatch. GRBM_GUI_ACTIVE reads the sum over the 8
    XCDs (a 17.9 us dispatch reads about 472 000, eight windows of about 59 000
    cycles), so the per-XCD cycle count is an eighth of it; TD is summed over
    its 256 instances (one per CU) and averaged here."""
    import csv
    per = {}
    for r in csv.DictReader(open(csv_path)):
        k = _short(r["Kernel_Name"])
        d = per.setdefault(k, {}).setdefault(r.get("Dispatch_Id", r.get("Correlation_Id")), {})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    lines = ["# Vector-memory pipeline busy fractions per dispatch: TA (address",
             "# unit) and TD (data return) busy cycles, and L2 (TCC) busy, over",
             "# the per-XCD active cycles (GRBM_GUI_ACTIVE / 8); averaged over the",
             "# kernel's dispatches. at::native::vectorized_elementwise is the plain",
             "# 256 MiB copy (torch.mul) run beside the library as a reference.",
             "# Workload: bench.py (voronoi 500x375, L=21, FP32, both kernels).",
             "# Command (repository root on the GPU host, TMPDIR=/tmp):"]
    lines += ["#   " + c for c in command]
    lines += ["# Summary written by: python bench.py --summarize-busy <csv> <out>",
              f"{'kernel':40s} {'dispatches':>10s} {'TA busy':>8s} {'TD busy':>8s} "
              f"{'L2 busy':>8s}"]
    rows = []
    for k, ds in per.items():
        ta, td, tcc = [], [], []
        for c in ds.values():
            g = c.get("GRBM_GUI_ACTIVE", 0.0) / 8.0
            if g <= 0:
                continue
            ta.append(c.get("TA_BUSY_avr", 0.0) / g)
            td.append(c.get("TD_TD_BUSY_sum", 0.0) / 256.0 / g)
            tcc.append(c.get("TCC_BUSY_avr", 0.0) / g)
        if ta:
            rows.append((k, len(ta), sum(ta) / len(ta), sum(td) / len(td),
                         sum(tcc) / len(tcc)))
    rows.sort(key=lambda r: -r[1])
    for k, n, a, b, c in rows[:40]:
        lines.append(f"{k[:40]:40s} {n:10d} {100 * a:7.1f}% {100 * b:7.1f}% {100 * c:7.1f}%")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def traffic_bytes(kernel):
    """HBM bytes per launch of `kernel` from TRAFFIC_FILE, each counter scaled
    by expected / measured of the calibration copy; None when the file is
    missing, lacks the kernel, or was taken on other kernel sources."""
    try:
        lines = open(TRAFFIC_FILE).read().split("\n")
    except OSError:
        return None
    rec, calib = {}, {}
    sha = None
    for ln in lines:
        t = ln.split()
        if not t or t[0].startswith("#"):
            continue
        if t[0] == "source_sha256":
            sha = t[1]
        elif t[0] == "calib":
            calib[t[1]] = float(t[5]) / float(t[3])
        elif t[0] == "kernel" and t[1].split("<")[0] == kernel:
            n = int(t[-1])   # the instantiation with the most dispatches
            if not rec or n > rec["n"]:
                rec = dict(fetch=float(t[-5]), write=float(t[-3]), n=n)
    if sha != source_digest() or not rec or len(calib) != 2:
        return None
    return (rec["fetch"] * calib["FETCH_SIZE"] + rec["write"] * calib["WRITE_SIZE"]) * 1024


def summarize_trace(stats_csv, out_path, command, note):
    """Write a kernel-statistics summary (calls, average/min/max microseconds,
    total ms) of a rocprofv3 --kernel-trace --stats run."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# {note}", "#", "# Command (repository root on the GPU host):"]
    lines += ["#   " + c for c in command]
    lines += [f"# Summary written by: python bench.py --summarize-trace <stats csv> "
              f"{os.path.relpath(out_path, ROOT)}", "#",
              f"{'kernel':48s} {'calls':>7s} {'avg us':>9s} {'min us':>9s} "
              f"{'max us':>9s} {'total ms':>9s}"]
    for r in rows[:40]:
        k = _short(r["Name"])
        if "rocprim" in r["Name"]:
            k = "rocprim " + r["Name"].split("::")[-1][:32]
        lines.append(f"{k[:48]:48s} {int(r['Calls']):7d} "
                     f"{float(r['AverageNs']) / 1e3:9.2f} {float(r['MinNs']) / 1e3:9.2f} "
                     f"{float(r['MaxNs']) / 1e3:9.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:9.3f}")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _timed(torch, fn, reps=1):
    """milliseconds per call of fn on the current stream (HIP events)"""
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def extensions(torch, dcrf, synth, dev, kernels):
    f32, f64 = torch.float32, torch.float64
    out = {}

    # -- QP + DC relaxation at 320x213: 50 Frank-Wolfe iterations, then the
    #    concave-convex procedure with 5 outer steps of 10 inner iterations --
    im = synth.make("voronoi_320x213_L21")
    wl = synth.WORKLOADS["voronoi_320x213_L21"]
    ctx = dcrf.Context(0)
    ctx.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev), kernels, dtype=f32)
    phi = torch.from_numpy(im.unary).to(dev, f32)
    mu = None   # the Potts compatibility (a null mu: no host read of it)
    y0 = torch.softmax(-phi, dim=1)
    res_dc = {}

    def qp_dc():
        y = y0.clone()
        ctx.qp_frank_wolfe(phi, mu, y, wl["iters"], trace=False)
        res_dc["hist"] = ctx.dc_gen(phi, mu, y, wl["dc_outer"], wl["dc_inner"])
        res_dc["y"] = y

    t_qd = _timed(torch, qp_dc, 3)
    labels = ctx.round(res_dc["y"])
    energy = ctx.energy(phi, mu, labels)
    out["qp_dc"] = dict(workload="voronoi 320x213 L=21 FP32: 50 FW iterations, then "
                                 "DC_gen 5 x 10", ms=t_qd,
                        S_after_dc=res_dc["hist"][-1], energy=energy)
    log(f"[bench] QP 50 + DC_gen 5x10 at 320x213: {t_qd:.2f} ms, S = "
        f"{res_dc['hist'][-1]:.6g}, E(argmax) = {energy:.6g}")

    # -- DC_neg: 50 Frank-Wolfe iterations, then 5 CCCP steps of the
    #    negative semi-definite decomposition (one filter call each) --------
    res_dn = {}

    def qp_dcneg():
        y = y0.clone()
        ctx.qp_frank_wolfe(phi, mu, y, wl["iters"], trace=False)
        ctx.dc_neg(phi, mu, y, 5, hist=False)
        res_dn["y"] = y

    t_qn = _timed(torch, qp_dcneg, 3)
    yq = y0.clone()
    ctx.qp_frank_wolfe(phi, mu, yq, wl["iters"], trace=False)
    hist_dn = ctx.dc_neg(phi, mu, yq.clone(), 5)
    e_dn = ctx.energy(phi, mu, ctx.round(res_dn["y"]))
    out["qp_dcneg"] = dict(workload="voronoi 320x213 L=21 FP32: 50 FW iterations, then "
                                    "DC_neg 5 steps", ms=t_qn, S_hist=hist_dn,
                           energy=e_dn)
    log(f"[bench] QP 50 + DC_neg 5 at 320x213: {t_qn:.2f} ms, S {hist_dn[0]:.6g} -> "
        f"{hist_dn[-1]:.6g}, E(argmax) = {e_dn:.6g}")

    # -- differentiation: 10 unrolled iterations at 500x375 ------------------
    im = synth.make("voronoi_500x375_L21_diff")
    iters = synth.WORKLOADS["voronoi_500x375_L21_diff"]["iters"]
    ctx = dcrf.Context(0)
    ctx.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev), kernels, dtype=f32)
    phi = torch.from_numpy(im.unary).to(dev, f32)
    mu = None   # the Potts compatibility (a null mu: no host read of it)
    gt = torch.from_numpy(im.gt.astype(np.int64)).to(dev)
    holder = {}

    def fwd():
        holder["y"], holder["saved"] = ctx.fw_forward(phi, mu, iters)

    def bwd():
        y = holder["y"]
        idx = torch.arange(im.N, device=dev)
        g = torch.zeros_like(y)
        g[idx, gt] = -1.0 / (im.N * y[idx, gt].clamp_min(1e-12))
        ctx.fw_backward(phi, mu, iters, holder["saved"], g)

    holder_y0 = torch.softmax(-phi, dim=1)   # start point, set up once

    def plain():
        y = holder_y0.clone()
        ctx.qp_frank_wolfe(phi, mu, y, iters, trace=False)

    t_f = _timed(torch, fwd, 5)
    t_b = _timed(torch, bwd, 3)
    t_p = _timed(torch, plain, 5)
    out["diff"] = dict(workload="voronoi 500x375 L=21 FP32, 10 unrolled FW "
                                "iterations, cross-entropy to the region labels",
                       forward_ms=t_f, backward_ms=t_b, fwd_bwd_ms=t_f + t_b,
                       plain_forward_ms=t_p,
                       fwd_bwd_over_plain=(t_f + t_b) / t_p,
                       checkpoint_MB=ctx.fw_saved_size(im.L, iters) / 1e6)
    log(f"[bench] diff: forward {t_f:.2f} ms, backward {t_b:.2f} ms, "
        f"plain forward {t_p:.2f} ms")
    del ctx, holder

    # -- batch: 16 uneven images -------------------------------------------
    ims = synth.make_batch()
    iters = synth.WORKLOADS["voronoi_batch16_L21"]["iters"]
    L = ims[0].L
    mu = None   # the Potts compatibility (a null mu: no host read of it)
    bctx = dcrf.Context(0)
    bctx.set_images([(x.H, x.W) for x in ims],
                    [torch.from_numpy(x.rgb).to(dev) for x in ims], kernels,
                    dtype=f32)
    tune = bctx.autotune(L, reps=3)
    bphi = bctx.pack([torch.from_numpy(x.unary).to(dev, f32) for x in ims], L)
    bgt = bctx.pack([torch.from_numpy(x.gt.astype(np.float32)).to(dev, f32)[:, None]
                     for x in ims], 1)[:, 0].long()
    segs = bctx.seg
    w_img = torch.zeros(bctx.N, device=dev, dtype=f32)
    for a, b in segs:
        w_img[a:b] = 1.0 / (b - a)
    bh = {}

    def bfwd():
        bh["y"], bh["saved"] = bctx.fw_forward(bphi, mu, iters)

    def bfwdbwd():
        bfwd()
        y = bh["y"]
        idx = torch.arange(bctx.N, device=dev)
        g = torch.zeros_like(y)
        g[idx, bgt] = -w_img / y[idx, bgt].clamp_min(1e-12)
        bctx.fw_backward(bphi, mu, iters, bh["saved"], g)

    sctx = []
    for x in ims:
        c = dcrf.Context(0)
        c.set_image(x.H, x.W, torch.from_numpy(x.rgb).to(dev), kernels, dtype=f32)
        sctx.append((c, torch.from_numpy(x.unary).to(dev, f32),
                     torch.from_numpy(x.gt.astype(np.int64)).to(dev), x.N))

    def seq_fwd():
        for c, p, _, _ in sctx:
            bh[id(c)] = c.fw_forward(p, mu, iters)

    def seq_fwdbwd():
        for c, p, g_t, n in sctx:
            y, saved = c.fw_forward(p, mu, iters)
            idx = torch.arange(n, device=dev)
            g = torch.zeros_like(y)
            g[idx, g_t] = -1.0 / (n * y[idx, g_t].clamp_min(1e-12))
            c.fw_backward(p, mu, iters, saved, g)

    # steady-state batched Frank-Wolfe iterations (one launch per stage over
    # all 16 images): the time of 60 iterations minus that of 10, per
    # iteration, against the algorithmic bytes of one iteration
    blat = [bctx.lattice_info(m) for m in range(len(kernels))]
    yb = torch.empty_like(bphi)

    def bsolve(k):
        yb.copy_(torch.softmax(-bphi, dim=1))
        bctx.qp_frank_wolfe(bphi, mu, yb, k, trace=False)
    t10 = _timed(torch, lambda: bsolve(10), 3)
    t60 = _timed(torch, lambda: bsolve(60), 3)
    it_ms = (t60 - t10) / 50
    npx = sum(x.N for x in ims)
    it_bytes = fw_step_bytes(npx, L, 4, blat)
    t_bf = _timed(torch, bfwd, 3)
    t_bfb = _timed(torch, bfwdbwd, 2)
    t_sf = _timed(torch, seq_fwd, 2)
    t_sfb = _timed(torch, seq_fwdbwd, 1)
    # the same forward (and forward+backward) with all iterations of the
    # forward in one persistent cooperative launch (two blur directions per
    # group, the staged splat, no tiles: the launch shapes it takes)
    ptune = dict(tune, blur_group=2, tiles=0, splat_stage=1)
    bctx.set_tune(**dict(ptune, fw_persistent=0))
    t_sbf = _timed(torch, bfwd, 3)
    bctx.set_tune(**dict(ptune, fw_persistent=1))
    t_pbf = _timed(torch, bfwd, 3)
    t_pbfb = _timed(torch, bfwdbwd, 2)
    t_p10 = _timed(torch, lambda: bsolve(10), 3)
    t_p60 = _timed(torch, lambda: bsolve(60), 3)
    p_it_ms = (t_p60 - t_p10) / 50
    bctx.set_tune(**dict(tune, fw_persistent=0))
    out["batch"] = dict(workload="16 Voronoi images, H and W ~ U{240..500}, "
                                 "L=21, FP32, 10 FW iterations each",
                        pixels=npx, autotune=tune, lattice_vertices=[M for d, M in blat],
                        fw_iteration_ms=it_ms, fw_iteration_bytes=it_bytes,
                        fw_iteration_GBps=it_bytes / it_ms / 1e6,
                        fw_iteration_frac_of_hbm_peak=it_bytes / it_ms / 1e6 / HBM_PEAK_GBPS,
                        batched_forward_ms=t_bf, batched_fwd_bwd_ms=t_bfb,
                        sequential_plain_forward_ms=t_sf,
                        sequential_fwd_bwd_ms=t_sfb,
                        batched_fwd_bwd_over_sequential_forward=t_bfb / t_sf,
                        forward_speedup=t_sf / t_bf,
                        fwd_bwd_speedup=t_sfb / t_bfb,
                        persistent=dict(
                            launch_shapes=ptune,
                            per_stage_forward_ms=t_sbf, forward_ms=t_pbf,
                            fwd_bwd_ms=t_pbfb, fw_iteration_ms=p_it_ms,
                            fw_iteration_GBps=it_bytes / p_it_ms / 1e6))
    log(f"[bench] batch of 16: steady FW iteration {it_ms * 1e3:.1f} us, "
        f"{it_bytes / 1e6:.1f} MB algorithmic = {it_bytes / it_ms / 1e6:.0f} GB/s")
    log(f"[bench] batch of 16 ({npx} px): batched fwd {t_bf:.2f} ms, fwd+bwd "
        f"{t_bfb:.2f} ms; sequential fwd {t_sf:.2f} ms, fwd+bwd {t_sfb:.2f} ms; "
        f"tune {tune}")
    log(f"[bench] batch of 16, one persistent launch per forward: fwd {t_pbf:.2f} ms "
        f"(per-stage {t_sbf:.2f} ms in the same shapes), fwd+bwd {t_pbfb:.2f} ms, "
        f"steady FW iteration {p_it_ms * 1e3:.1f} us")
    del bctx, sctx, bh

    # -- lattice against the exact sum at 320x213 ----------------------------
    im = synth.make("voronoi_320x213_L21")
    ctx = dcrf.Context(0)
    ctx.set_image(im.H, im.W, torch.from_numpy(im.rgb).to(dev), kernels, dtype=f64)
    g = torch.Generator(device="cpu").manual_seed(7)
    Y = torch.rand(im.N, 4, generator=g, dtype=f64).to(dev)
    lat = ctx.filter(Y)
    exact = ctx.filter(Y, exact=True)
    num = float((lat * exact).sum())
    cos = num / float(lat.norm() * exact.norm())
    sep = ctx.filter(Y, separable=True)
    out["lattice_error"] = dict(
        workload="voronoi 320x213, both kernels, K'Y for Y ~ U[0,1]^(N x 4), FP64",
        ratio_of_means=float(lat.mean() / exact.mean()), cosine=cos,
        rel_l2_error=float((lat - exact).norm() / exact.norm()),
        separable_ratio_of_means=float(sep.mean() / exact.mean()),
        separable_cosine=float((sep * exact).sum() / (sep.norm() * exact.norm())),
        separable_rel_l2_error=float((sep - exact).norm() / exact.norm()))
    log(f"[bench] lattice vs exact: {out['lattice_error']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--filter-reps", type=int, default=200)
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--lp-steps", type=int, default=100)
    ap.add_argument("--lp-beta0", type=float, default=1e-6)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB copy kernel (reference for "
                         "the HBM byte counters of a profiler run)")
    ap.add_argument("--no-ext", action="store_true",
                    help="skip the separable-mode, diff, batch and lattice-error "
                         "measurements")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic summary under profiles/ from two "
                         "rocprofv3 --pmc counter CSVs and exit")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("STATS_CSV", "OUT"),
                    help="write a kernel statistics summary from a rocprofv3 "
                         "--stats CSV and exit")
    ap.add_argument("--summarize-busy", nargs=2, metavar=("CSV", "OUT"),
                    help="write a TA/TD busy summary from a rocprofv3 --pmc CSV "
                         "and exit")
    ap.add_argument("--command", action="append", default=[],
                    help="profiler command line to record in a summary")
    ap.add_argument("--note", default="Kernel statistics",
                    help="first line of a trace summary")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args.command)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, args.command, args.note)
        return
    if args.summarize_busy:
        summarize_busy(*args.summarize_busy, args.command)
        return
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
    mu = None   # the Potts compatibility (a null mu: no host read of it)
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
    # cold: each call after a 512 MB write that evicts the L2s and the
    # 256 MB Infinity Cache (median of 5)
    flush = torch.empty(128 << 20, device=dev, dtype=f32)
    cold = []
    for _ in range(5):
        flush.fill_(1.0)
        ev0.record()
        ctx.filter(Y, out=out)
        ev1.record()
        torch.cuda.synchronize()
        cold.append(ev0.elapsed_time(ev1))
    del flush
    c_ms = sorted(cold)[2]
    filt = dict(ms=f_ms, GBps=f_bytes / f_ms / 1e6, bytes=f_bytes,
                frac_of_hbm_peak=f_bytes / f_ms / 1e6 / HBM_PEAK_GBPS,
                cold_ms=c_ms, cold_GBps=f_bytes / c_ms / 1e6,
                cold_frac_of_hbm_peak=f_bytes / c_ms / 1e6 / HBM_PEAK_GBPS)
    log(f"[bench] dense filter L=21: {f_ms * 1e3:.1f} us, "
        f"{filt['GBps']:.0f} GB/s algorithmic; after a 512 MB flush "
        f"{c_ms * 1e3:.1f} us, {filt['cold_GBps']:.0f} GB/s")

    # ---- DC_neg steps at the same size (one filter call per step) ---------
    yd = y.clone()
    ctx.dc_neg(phi, mu, yd, 2, hist=False)
    torch.cuda.synchronize()
    dn_steps = 20
    ev0.record()
    ctx.dc_neg(phi, mu, yd, dn_steps, hist=False)
    ev1.record()
    torch.cuda.synchronize()
    dn_ms = ev0.elapsed_time(ev1) / dn_steps
    log(f"[bench] DC_neg step at 500x375: {dn_ms * 1e3:.1f} us")

    # ---- LP subgradient steps from the QP solution -------------------------
    lp = None
    if args.lp_steps > 0:
        ylp = y.clone()                       # the timed QP solve's result
        ybest = torch.empty_like(y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        best, hist = ctx.lp_descent(phi, ylp, args.lp_steps, args.lp_beta0, best_y=ybest)
        torch.cuda.synchronize()
        lp_ms = (time.perf_counter() - t0) * 1e3 / args.lp_steps
        lp = dict(ms_per_step=lp_ms, steps=args.lp_steps, beta0=args.lp_beta0,
                  S_LP_first=hist[0], S_LP_best=best, S_LP_last=hist[-1],
                  best_step=int(np.argmin(hist)))
        log(f"[bench] LP subgradient step (divide and conquer, 21 labels, "
            f"{int(np.ceil(np.log2(N)))} levels): {lp_ms:.1f} ms")

        # the same descent with leaf-exact nodes of at most 256 positions
        yleaf = y.clone()
        leaf_steps = max(1, args.lp_steps // 5)
        ctx.set_lp_leaf(256)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bleaf, hleaf = ctx.lp_descent(phi, yleaf, leaf_steps, args.lp_beta0)
        torch.cuda.synchronize()
        leaf_ms = (time.perf_counter() - t0) * 1e3 / leaf_steps
        ctx.set_lp_leaf(0)
        lp["leaf_exact"] = dict(leaf=256, steps=leaf_steps, ms_per_step=leaf_ms,
                                S_LP_first=hleaf[0], S_LP_best=bleaf,
                                plain_S_LP_at_same_step=hist[leaf_steps - 1],
                                leaf_S_LP_at_same_step=hleaf[-1])
        log(f"[bench] LP step with leaf-exact nodes (<= 256 positions): {leaf_ms:.1f} ms, "
            f"S_LP after {leaf_steps} steps {hleaf[-1]:.6g} (plain {hist[leaf_steps - 1]:.6g})")

        # the LP on the labels that the QP solution's argmax uses (Sec. 7
        # restricts the LP to the labels present in another method's result)
        sub = ctx.labels_used(ctx.round(y), L)
        ysub = y.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bsub, hsub = ctx.lp_descent_subset(phi, ysub, sub, args.lp_steps, args.lp_beta0)
        torch.cuda.synchronize()
        sub_ms = (time.perf_counter() - t0) * 1e3 / args.lp_steps
        lp["subset"] = dict(labels=len(sub), ms_per_step=sub_ms,
                            S_LP_first=hsub[0], S_LP_best=bsub, S_LP_last=hsub[-1])
        log(f"[bench] LP on the {len(sub)} labels the argmax uses: "
            f"{sub_ms:.1f} ms/step, S_LP {hsub[0]:.6g} -> {bsub:.6g}")

        # Kleinberg-Tardos rounding of the best LP point, 8 L rounds drawn
        # from a seeded generator, against the argmax of the same point
        g = torch.Generator().manual_seed(7)
        R = 8 * L
        rl = torch.randint(0, L, (R,), generator=g, dtype=torch.int32).to(dev)
        rt = torch.rand(R, generator=g, dtype=torch.float64).to(dev, f32)
        kt_reps = 20
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(kt_reps):
            xk, left = ctx.round_kt(ybest, rl, rt)
        kt_ms = (time.perf_counter() - t0) * 1e3 / kt_reps
        lp["kt_round"] = dict(rounds=R, ms=kt_ms, pixels_left=left,
                              energy=ctx.energy(phi, mu, xk),
                              energy_argmax=ctx.energy(phi, mu, ctx.round(ybest)))
        log(f"[bench] KT rounding ({R} rounds): {kt_ms * 1e3:.0f} us per call incl. "
            f"readback, E {lp['kt_round']['energy']:.6g} vs argmax "
            f"{lp['kt_round']['energy_argmax']:.6g}, {left} pixels left")

        # the LP for a tree metric: a seeded 2-HST over the labels, c_T twice
        # the edge length above T, descent from the QP solution
        parent, length = synth.random_hst(L, seed=21)
        c = [2.0 * v for v in length]
        yt = y.clone()
        tree_steps = max(1, args.lp_steps // 10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        btree, htree = ctx.lp_descent_tree(phi, yt, parent, c, tree_steps, args.lp_beta0)
        torch.cuda.synchronize()
        tree_ms = (time.perf_counter() - t0) * 1e3 / tree_steps
        lp["tree"] = dict(nodes=len(parent), weighted_subtrees=int(sum(v > 0 for v in c)),
                          steps=tree_steps, ms_per_step=tree_ms, S_first=htree[0],
                          S_best=btree)
        log(f"[bench] r-HST LP ({len(parent)} nodes): {tree_ms:.1f} ms/step, "
            f"S {htree[0]:.6g} -> {btree:.6g} in {tree_steps} steps")

    if not args.no_ext:
        # the separable mode: the spatial kernel exact by two 1-D passes
        ev0.record()
        for _ in range(20):
            ctx.filter(Y, out=out, separable=True)
        ev1.record()
        torch.cuda.synchronize()
        sep_ms = ev0.elapsed_time(ev1) / 20
        ctx.set_filter_mode("separable")
        ysep = y0.clone()
        ctx.qp_frank_wolfe(phi, mu, ysep, 5, trace=False)
        ysep = y0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.qp_frank_wolfe(phi, mu, ysep, 50, trace=False)
        torch.cuda.synchronize()
        sep_fw_us = (time.perf_counter() - t0) * 1e6 / 50
        ctx.set_filter_mode("lattice")
        filt["separable_ms"] = sep_ms
        filt["separable_fw_iteration_us"] = sep_fw_us
        # the one-hot splat inside the conditional-gradient kernel
        # (pixel-major, runs of equal vertex and label summed per wave)
        ctx.set_tune(fw_splat=1)
        yfu = y0.clone()
        ctx.qp_frank_wolfe(phi, mu, yfu, 5, trace=False)
        yfu = y0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.qp_frank_wolfe(phi, mu, yfu, 100, trace=False)
        torch.cuda.synchronize()
        filt["fused_splat_fw_iteration_us"] = (time.perf_counter() - t0) * 1e6 / 100
        ctx.set_tune(fw_splat=0)
        log(f"[bench] FW iteration with the splat in the LMO kernel: "
            f"{filt['fused_splat_fw_iteration_us']:.1f} us (100 iterations)")
        log(f"[bench] separable mode: dense filter {sep_ms * 1e3:.1f} us, FW iteration "
            f"{sep_fw_us:.1f} us (50 iterations)")
    ext = {} if args.no_ext else extensions(torch, dcrf, synth, dev, kernels)
    if args.calib_copy:
        a = torch.ones(64 << 20, device=dev, dtype=f32)
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)   # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del a, b

    # ---- roofline of the dominant kernel of the step ----------------------
    step_classes = ("k_fw_lmo_rows", "k_splat_labels_lds", "k_splat_labels_chunks",
                    "k_blur_group", "k_blur_pass", "k_fw_slice_rows")
    dom = max((k for k in per_iter if k in step_classes),
              key=lambda k: per_iter[k][0] * per_iter[k][1])
    dom_ms = per_iter[dom][0]
    dom_bytes = class_bytes(dom, N, L, 4, lat)
    achieved = dom_bytes / dom_ms / 1e6
    roofline = dict(bound="hbm", kernel=dom, achieved=achieved,
                    peak=HBM_PEAK_GBPS, unit="GB/s", frac=achieved / HBM_PEAK_GBPS,
                    traffic=traffic_bytes(dom), bytes_per_launch=dom_bytes,
                    avg_launch_us=dom_ms * 1e3)
    # the same for every kernel of the step (the LMO and the slice take
    # nearly the same time, so which one is dominant varies between runs)
    step_rooflines = []
    for k in sorted((k for k in per_iter if k in step_classes),
                    key=lambda k: -per_iter[k][0] * per_iter[k][1]):
        b = class_bytes(k, N, L, 4, lat)
        a = b / per_iter[k][0] / 1e6
        step_rooflines.append(dict(kernel=k, avg_launch_us=per_iter[k][0] * 1e3,
                                   launches_per_step=per_iter[k][1] / prof_iters,
                                   bytes_per_launch=b, achieved=a,
                                   frac=a / HBM_PEAK_GBPS, traffic=traffic_bytes(k)))

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
               dc_neg=dict(workload="voronoi 500x375 L=21 FP32, DC_neg steps from "
                                    "the timed QP solution", us_per_step=dn_ms * 1e3,
                           steps=dn_steps),
               per_kernel_us={k: v[0] * 1e3 for k, v in per_iter.items()},
               lp=lp, roofline=roofline, step_rooflines=step_rooflines, **ext)
    if not args.no_cpu:
        log(f"[bench] CPU baseline: {args.cpu_iters} oracle FW iterations ...")
        res["cpu_baseline"] = cpu_baseline(im, kernels, mu_np, args.cpu_iters)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
