#!/usr/bin/env python3
"""Throughput of the PixelSNE iteration on one MI355X: points x iterations / s.

Workload: 1,000,000 x 128 float32 points from a 100-component Gaussian mixture
with Zipf(1.1) component sizes and per-component variance U(0.5, 2),
perplexity 50 (k = 150), 2048 x 2048 screen, theta = 0.5.  One step is one
full iteration of the method (pixel snap + Morton keys, sort, P-Quadtree,
Barnes-Hut repulsion, Z, sparse attraction + gains/momentum step, screen
scaling) over all points; the one-time setup (kNN, perplexity, P) is timed
separately.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  The roofline figures use algorithmic counts: bytes
the method must move (`attract_bytes`, `tree_bytes`) and flops per visited
and per used cell for the traversal, over the measured pass times.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "points×iters/sec at n=1M (fp32 vs fp64) + time-to-KL within 1%, MLP init vs plain"
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz: the rate of FP64 and of
# non-packed FP32 vector arithmetic (the library is compiled without packed FP32)
VALU_PEAK_TFLOPS = 78.6


# Hardware byte counters per launch of the dominant kernels (rocprofv3 FETCH_SIZE
# and WRITE_SIZE, scaled by what the counters read for a copy of known size),
# valid while the kernel's source file is unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_1M.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(kernel):
    """HBM bytes per iteration of `kernel`'s launches (the entry's note says
    which launches are added) from the committed counter summary, or None if
    there is none or a source the kernel's traffic depends on (its own, and
    the layout it reads) changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            entry = json.load(f)["kernels"].get(kernel)
        if not entry:
            return None
        for path, sha in entry["sources_sha256"].items():
            with open(os.path.join(ROOT, path), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != sha:
                    return None
        return (entry["fetch_kib"] * 1024 * entry["fetch_scale"]
                + entry["write_kib"] * 1024 * entry["write_scale"])
    except (OSError, KeyError, ValueError):
        return None


def tree_bytes(n, n_nodes, sb):
    """Algorithmic HBM bytes of snap + sort + cell build for one iteration:
    read zh and write z (2 sb each), write and read (key, index) once in and
    once out of the sort (4 x 8 B), gather z in sorted order (2 sb) and write
    each cell's count (4 B) and FP64 sums (16 B)."""
    return n * (2 * 2 * sb + 4 * 8 + 2 * sb) + n_nodes * 20


def attract_bytes(n, nnz, sb):
    """Algorithmic HBM bytes of the attraction's row sums for one iteration:
    CSR column word (4 B) and value (sb) per nonzero, row offset (8 B), z_i
    once and z_j compulsory once (2 x 2 sb) and the row sum A_i written
    (2 sb).  The optimiser step that follows is a kernel of its own."""
    return nnz * (4 + sb) + n * (8 + 6 * sb)


def update_bytes(n, sb):
    """Algorithmic HBM bytes of the optimiser step (its own kernel): read the
    row sums A, z, R, u and g, write u, g and the new positions (8 x 2 sb per
    point)."""
    return n * 16 * sb


def traverse_bytes(n, n_nodes, sb):
    """Compulsory HBM bytes of the Barnes-Hut walk: sorted positions (2 sb),
    the permutation and own-leaf index (8 B), R written (2 sb) and Z_i partials,
    and each cell record read once (32 B + 16 B of sums)."""
    return n * (4 * sb + 8) + n_nodes * 48


def pass_metrics(n, nnz, sb, K, ms, pt, vis, used, n_nodes):
    """Per-pass times and their roofline figures for one timed window."""
    per = {k[:-3]: v / K for k, v in pt.items() if k.endswith("_ms")}
    tree_ms = per["snap"] + per["sort"] + per["tree"]
    tb = tree_bytes(n, n_nodes, sb)
    ab = attract_bytes(n, nnz, sb)
    ub = update_bytes(n, sb)
    vb = traverse_bytes(n, n_nodes, sb)
    flops = n * (8.0 * vis + 9.0 * used)
    it_bytes = tb + ab + ub + vb
    return {
        "value": n * K / (ms / 1e3),
        "ms_per_step": ms / K,
        "pass_ms": per,
        "mean_visits": vis,
        "mean_used_cells": used,
        "cells": n_nodes,
        "tree_build": {"ms": tree_ms, "bytes": tb, "GBps": tb / (tree_ms * 1e6),
                       "frac_hbm": tb / (tree_ms * 1e6) / HBM_PEAK_GBS},
        "attract": {"ms": per["attract"], "bytes": ab, "GBps": ab / (per["attract"] * 1e6),
                    "frac_hbm": ab / (per["attract"] * 1e6) / HBM_PEAK_GBS},
        "traverse": {"ms": per["traverse"], "flops": flops,
                     "TFLOPs": flops / (per["traverse"] * 1e9),
                     "frac_valu": flops / (per["traverse"] * 1e9) / VALU_PEAK_TFLOPS},
        # the whole iteration's algorithmic bytes over its wall time
        "iteration": {"bytes": it_bytes, "GBps": it_bytes / (ms / K * 1e6),
                      "frac_hbm": it_bytes / (ms / K * 1e6) / HBM_PEAK_GBS},
    }


def timed_window(ctx, K, profiled=True):
    """K iterations between two events on the caller's stream; with
    `profiled`, the library also records events between the passes."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    if profiled:
        pt = ctx.step_profiled(K).as_dict()
    else:
        ctx.step_async(K)
        pt = None
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), pt


def run_gpu(args):
    import numpy as np
    import torch

    from paper_1611_02568_amd import datagen, pixelsne

    torch.cuda.set_device(0)
    n = args.n
    log(f"[bench] generating {n} x 128 mixture")
    X, _, mix = datagen.zipf_mixture_1m(n=n)
    y0 = torch.as_tensor(datagen.initial_embedding(n, seed=datagen.seed_for(2, 1)))
    Xd = torch.from_numpy(X).cuda()
    torch.cuda.synchronize()

    g = 0 if args.no_graphs else 1
    t0 = time.perf_counter()
    if args.no_fp64:
        log("[bench] setup (kNN, perplexity, P) for the FP32 path")
        ctx64 = None
        ctx32 = pixelsne.Context.from_data(Xd, 50.0, 2048, Y_init=y0, precision=pixelsne.FP32,
                                           graphs=g, opening_fp64=args.opening_fp64)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
    else:
        # the same setup for each path (identical P and initial numbering)
        log("[bench] setup (kNN, perplexity, P), FP32 and FP64 paths")
        ctx32 = pixelsne.Context.from_data(Xd, 50.0, 2048, Y_init=y0, precision=pixelsne.FP32,
                                           graphs=g, opening_fp64=args.opening_fp64)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        ctx64 = pixelsne.Context.from_data(Xd, 50.0, 2048, Y_init=y0, precision=pixelsne.FP64,
                                           graphs=g)
    del Xd
    nnz = ctx32.stats().nnz
    log(f"[bench] setup {setup_s:.2f} s, nnz {nnz} ({nnz / n:.1f} per row)")

    out = {}
    K = args.steps
    for name, ctx, sb in (("fp32", ctx32, 4), ("fp64", ctx64, 8)):
        if name == "fp64" and args.no_fp64:
            continue
        ctx.step(args.warmup)
        saved = ctx.get_state()

        def restore(st):
            ctx.set_state(st["z"], st["s"], u=st["u"], g=st["g"], iteration=st["iteration"])

        # the timed region: K iterations after the warm-up as the library
        # runs them (graph replay), between two events on the caller's stream
        ms, _ = timed_window(ctx, K, profiled=False)
        log(f"[bench] {name}: {K} iterations in {ms:.1f} ms")
        if args.plain_timing:
            out[name] = {"value": n * K / (ms / 1e3), "ms_per_step": ms / K}
            continue
        # the statistics of the window's last tree
        gr = ctx.gradient(1.0)
        vis = gr["visits"].double().mean().item()
        used = gr["used"].double().mean().item()
        del gr
        n_nodes = ctx.stats().n_nodes
        # the same K iterations again from the saved state with HIP events
        # recorded by the library between the passes (per-pass times; the
        # pass-timed iterations launch their kernels directly)
        restore(saved)
        ms_p, pt = timed_window(ctx, K)
        res = pass_metrics(n, nnz, sb, K, ms, pt, vis, used, n_nodes)
        res["iterations"] = [args.warmup + 1, args.warmup + K]
        res["ms_per_step_pass_timed"] = ms_p / K
        log(f"[bench] {name}: passes {json.dumps({k: round(v, 4) for k, v in res['pass_ms'].items()})}")
        # repetitions: the same K iterations again from the saved state
        reps = [ms / K]
        for _ in range(args.reps - 1):
            restore(saved)
            ms_r, _ = timed_window(ctx, K, profiled=False)
            reps.append(ms_r / K)
        res["reps_ms_per_step"] = reps
        res["ms_per_step_mean"] = float(np.mean(reps))
        res["ms_per_step_sd"] = float(np.std(reps, ddof=1)) if len(reps) > 1 else 0.0
        del saved
        # steady state: iterations 981-1000 of the run (untimed iterations up
        # to 980), timed the same way, then again with the pass events
        it = ctx.stats().iteration
        if it < 980:
            ctx.step(980 - it)
        it0 = ctx.stats().iteration
        saved = ctx.get_state()
        ms_s, _ = timed_window(ctx, 20, profiled=False)
        gr = ctx.gradient(1.0)
        vis_s = gr["visits"].double().mean().item()
        used_s = gr["used"].double().mean().item()
        del gr
        n_nodes_s = ctx.stats().n_nodes
        restore(saved)
        _, pt_s = timed_window(ctx, 20)
        del saved
        st = pass_metrics(n, nnz, sb, 20, ms_s, pt_s, vis_s, used_s, n_nodes_s)
        st["iterations"] = [it0 + 1, it0 + 20]
        res["steady_state"] = st
        log(f"[bench] {name}: steady state (iterations {it0 + 1}-{it0 + 20}) "
            f"{st['ms_per_step']:.4f} ms/iteration")
        out[name] = res
        if name == "fp32" and args.ttkl:
            # the network learns from the converged run (>= 1,000 iterations)
            out["time_to_kl"] = time_to_kl(ctx, X, mix, args)
    if "fp64" in out:
        out["fp32_vs_fp64"] = compare_precisions(ctx32, ctx64)
    return out, setup_s, nnz


def compare_precisions(ctx32, ctx64):
    """Error of the FP32 path against the FP64 path on one snapshot (the FP64
    run's final state rounded to FP32, loaded into both), and the final KL of
    each run (exact Z)."""
    import torch

    kl32, kl64 = ctx32.kl(), ctx64.kl()
    st = ctx64.get_state()
    z = st["z"].float()
    ctx64.set_state(z.double(), st["s"])
    ctx32.set_state(z, st["s"])
    g64, g32 = ctx64.gradient(1.0), ctx32.gradient(1.0)

    def rel(k):
        a, b = g32[k].double(), g64[k].double()
        return (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()

    res = {"A_rel": rel("A"), "R_rel": rel("R"), "B_rel": rel("B"),
           "Z_rel": abs(g32["Z"] - g64["Z"]) / g64["Z"],
           "visits_equal_frac": (g32["visits"] == g64["visits"]).double().mean().item(),
           "final_kl_fp32": kl32, "final_kl_fp64": kl64}
    log(f"[bench] fp32 vs fp64: {json.dumps(res)}")
    return res


def time_to_kl(ctx_train, X_train, mix, args):
    """Learned placement: a 128-512-512-2 network trained (BF16 MFMA) on the
    converged 1M run (>= 1,000 iterations) places 200,000 held-out draws of the
    same mixture; the placed embedding is refined by ordinary iterations (no
    exaggeration, momentum 0.8, fresh gains; pixelsne_refine) until its exact
    KL is within 1% of 1,000 plain iterations from a random start, the plain
    method continuing past the 100-iteration refinement budget (fallback).
    Times are GPU times of the iterations (HIP events) plus the placement;
    the shared P setup, the KL checks and the network training (reported on
    its own) are excluded."""
    import torch

    from paper_1611_02568_amd import datagen, pixelsne

    def sync():
        torch.cuda.synchronize()

    r = 2048
    tr = ctx_train.stats()
    assert tr.iteration >= 1000, "the network must learn from a converged run"
    st = ctx_train.get_state()
    s_train = st["s"]
    Y01 = (st["z"] / r).float().contiguous()
    Xd = torch.from_numpy(X_train).cuda()
    net = pixelsne.MLP(128, 512, 512, seed=7)
    net.fit_norm(Xd)
    t0 = time.perf_counter()
    loss = net.train(Xd, Y01, epochs=args.mlp_epochs, batch=4096, lr=1e-3)
    sync()
    t_train = time.perf_counter() - t0
    del Xd, Y01
    Xh, _ = datagen.heldout(mix, n=args.heldout)
    Xhd = torch.from_numpy(Xh).cuda()
    nh = Xh.shape[0]
    yh0 = torch.as_tensor(datagen.initial_embedding(nh, seed=datagen.seed_for(3, 1)))
    hi, _ = pixelsne.knn(Xhd, 30)                  # high-dimensional neighbours for Eq. (14)
    out = {"heldout": nh, "train_points": X_train.shape[0],
           "train_run": {"iteration": tr.iteration, "kl": ctx_train.kl()},
           "mlp": "128-512-512-2 GELU, BF16 MFMA",
           "mlp_epochs": args.mlp_epochs, "mlp_train_s": t_train, "mlp_last_epoch_loss": loss}
    for label, eta in (("eta200", 200.0), ("eta_n_over_12", nh / 12.0)):
        plain = pixelsne.Context.from_data(Xhd, 50.0, r, Y_init=yh0, precision=pixelsne.FP32, eta=eta)
        ms_plain, _ = timed_window(plain, 1000, profiled=False)
        kl_plain = plain.kl()
        prec_plain = plain.neighborhood_precision(hi, [1, 10, 30])
        del plain
        res = {"plain_1000_s": ms_plain / 1e3, "plain_kl": kl_plain, "target_kl": 1.01 * kl_plain,
               "plain_precision_k1_10_30": prec_plain}
        # placed scale: the training run's s, and s times sqrt(n_heldout / n_train)
        # (the embedding's extent grows with the number of points)
        fsq = (nh / X_train.shape[0]) ** 0.5
        for rlabel, reta, fs in (("refine_eta200", 200.0, 1.0),
                                 ("refine_eta200_s_sqrt_n_ratio", 200.0, fsq),
                                 ("refine_eta_n_over_12", nh / 12.0, 1.0),
                                 ("refine_eta_n_over_12_s_sqrt_n_ratio", nh / 12.0, fsq)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            Yp = net.place(Xhd, r, (s_train[0] * fs, s_train[1] * fs))
            e1.record()
            sync()
            t_place = e0.elapsed_time(e1) / 1e3
            placed = pixelsne.Context.from_data(Xhd, 50.0, r, Y_init=Yp, precision=pixelsne.FP32,
                                                exag_iters=0, mom_switch=0, eta=reta)
            rr = placed.refine(1.01 * kl_plain, check_every=10, refine_iters=100, max_iters=1000)
            rr["seconds"] = t_place + rr["iter_ms"] / 1e3 if rr["reached"] else None
            rr["speedup"] = (ms_plain / 1e3 / rr["seconds"]) if rr["seconds"] else None
            rr["precision_k1_10_30"] = placed.neighborhood_precision(hi, [1, 10, 30])
            rr["place_s"] = t_place
            res[rlabel] = rr
            del placed, Yp
        out["plain_" + label] = res
        log(f"[bench] time-to-KL plain {label}: {json.dumps(res)}")
    return out


def r_sweep(args):
    """The paper's central comparison (Section 4.1, Fig. 3, Table 5) on the
    benchmark's FP32 workload (1,000,000 x 128 mixture, perplexity 50): the
    pixel-aligned P-Quadtree at screen sizes r = 512 ... 8,192 against the
    data-driven D-Quadtree of Barnes-Hut-SNE (root on the data, cells split
    until each leaf holds one point, rebuilt every iteration), both walked by
    the same traversal.  Per configuration: wall time per iteration over
    `--steps` iterations after `--warmup` (graph replay), the pass times of
    20 further iterations, mean visited cells per point, the number of cells
    and the exact-Z KL at the end.  Setup (kNN, P) runs for each
    configuration and is not timed."""
    import torch

    from paper_1611_02568_amd import datagen, pixelsne

    torch.cuda.set_device(0)
    n = args.n
    X, _, _ = datagen.zipf_mixture_1m(n=n)
    y0 = torch.as_tensor(datagen.initial_embedding(n, seed=datagen.seed_for(2, 1)))
    Xd = torch.from_numpy(X).cuda()
    out = []
    configs = [("pixel", r) for r in (512, 1024, 2048, 4096, 8192)] + [("data", 2048)]
    for tree, r in configs:
        ctx = pixelsne.Context.from_data(Xd, 50.0, r, Y_init=y0, precision=pixelsne.FP32,
                                         tree=pixelsne.TREE_DATA if tree == "data"
                                         else pixelsne.TREE_PIXEL)
        ctx.step(args.warmup)
        ms, _ = timed_window(ctx, args.steps, profiled=False)
        _, pt = timed_window(ctx, 20)
        per = {k[:-3]: round(v / 20, 4) for k, v in pt.items() if k.endswith("_ms")}
        g = ctx.gradient(1.0)
        st = ctx.stats()
        row = {"tree": tree, "r": r, "ms_per_iter": ms / args.steps,
               "iterations": [args.warmup + 1, args.warmup + args.steps],
               "pass_ms_after": per, "tree_build_ms": per["snap"] + per["sort"] + per["tree"],
               "kl": ctx.kl(), "mean_visits": g["visits"].double().mean().item(),
               "cells": st.n_nodes}
        log(f"[bench] tree sweep {json.dumps(row)}")
        out.append(row)
        del ctx, g
    return out


def three_d(args):
    """The 3-D embedding (voxel octree of depth log2 r; Section 1 notes that
    the method extends to 3-D) on the FP32 workload's data (1,000,000 x 128
    mixture, perplexity 50), FP64 throughout, at cube sides r = 256 and
    1,024, with the step size n / 12 (at this n the default 200 leaves the
    initial blob nearly unchanged for hundreds of iterations).  Per
    configuration: wall time per iteration over `--steps` iterations after
    `--warmup` (one synchronisation at the end), and again over `--steps`
    iterations ending at iteration 500 (the embedding formed), with the mean
    visited cells per point, the cells of the octree and the exact-Z KL at
    each point.  Setup (kNN, P) is not timed."""
    import torch

    from paper_1611_02568_amd import datagen, pixelsne

    torch.cuda.set_device(0)
    n = args.n
    X, _, _ = datagen.zipf_mixture_1m(n=n)
    y0 = torch.as_tensor(datagen.initial_embedding(n, seed=datagen.seed_for(2, 1), dim=3))
    Xd = torch.from_numpy(X).cuda()
    out = []
    def window(ctx, first, last):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(last - first + 1)
        ms = (time.perf_counter() - t0) * 1e3 / (last - first + 1)
        g = ctx.gradient(1.0)
        tr = ctx.export_tree()
        return {"iterations": [first, last], "ms_per_iter": ms,
                "points_iter_per_s": n / (ms * 1e-3),
                "mean_visits": g["visits"].double().mean().item(),
                "cells": int(sum(tr["level_size"])), "kl": ctx.kl()}

    late = max(500, args.warmup + 2 * args.steps)
    for r in (256, 1024):
        ctx = pixelsne.Context3.from_data(Xd, 50.0, r, Y_init=y0, eta=n / 12.0)
        ctx.step(args.warmup)
        row = {"r": r, "eta": n / 12.0,
               "early": window(ctx, args.warmup + 1, args.warmup + args.steps)}
        ctx.step(late - args.steps - (args.warmup + args.steps))
        row["formed"] = window(ctx, late - args.steps + 1, late)
        log(f"[bench] 3-D {json.dumps(row)}")
        out.append(row)
        del ctx
    return out


def time_to_kl_large(args):
    """The 5,000,000 x 100 workload with 1% outliers (perplexity 30, k 90, screen
    4096): a 100-1024-1024-2 network is trained on the converged plain run of a
    seeded 1,000,000-point subsample and places all 5,000,000 points, which are
    refined (no exaggeration, momentum 0.8, fresh gains) until their exact KL is
    within 1% of 1,000 plain iterations from a random start (learning rate 200,
    and n / 12 for comparison).  The placed scale s is the subsample run's
    times sqrt(5,000,000 / 1,000,000).  KL checks every 50 iterations are not
    timed."""
    import numpy as np
    import torch

    from paper_1611_02568_amd import datagen, pixelsne

    def sync():
        torch.cuda.synchronize()

    n, r, u = args.large_n, 4096, 30.0
    log(f"[large] generating {n} x 100 mixture with outliers")
    X, _, _ = datagen.zipf_mixture_outliers(n=n)
    sub = np.sort(np.random.default_rng(datagen.seed_for(4, 3)).choice(n, n // 5, replace=False))
    Xd = torch.from_numpy(X).cuda()
    Xs = Xd[torch.from_numpy(sub).cuda()].contiguous()
    out = {"n": n, "subsample": int(sub.size), "screen": r, "perplexity": u,
           "mlp": "100-1024-1024-2 GELU, BF16 MFMA"}
    t0 = time.perf_counter()
    cs = pixelsne.Context.from_data(Xs, u, r, precision=pixelsne.FP32,
                                    Y_init=torch.as_tensor(datagen.initial_embedding(sub.size, seed=datagen.seed_for(4, 4))))
    cs.step(1000)
    sync()
    out["subsample_run_s"] = time.perf_counter() - t0
    st = cs.get_state()
    s_sub = st["s"]
    Y01 = (st["z"] / r).float().contiguous()
    del cs
    net = pixelsne.MLP(100, 1024, 1024, seed=11)
    net.fit_norm(Xs)
    t0 = time.perf_counter()
    out["mlp_last_epoch_loss"] = net.train(Xs, Y01, epochs=args.mlp_epochs, batch=4096, lr=1e-3)
    sync()
    out["mlp_train_s"] = time.perf_counter() - t0
    del Xs, Y01
    log(f"[large] subsample run and network: {json.dumps(out)}")
    t0 = time.perf_counter()
    y0 = torch.as_tensor(datagen.initial_embedding(n, seed=datagen.seed_for(4, 1)))
    plain = pixelsne.Context.from_data(Xd, u, r, precision=pixelsne.FP32, Y_init=y0)
    sync()
    out["setup_s"] = time.perf_counter() - t0
    rp, col, val = plain.export_P()
    out["nnz"] = int(col.numel())
    t0 = time.perf_counter()
    plain.step(1000)
    sync()
    out["plain_1000_s"] = time.perf_counter() - t0
    kl_plain = plain.kl()
    out["plain_kl"] = kl_plain
    del plain
    log(f"[large] plain eta 200: {out['plain_1000_s']:.2f} s, KL {kl_plain:.4f}")
    # the same with the learning rate n / 12 (a later t-SNE convention) for fairness
    plain = pixelsne.Context.from_P(rp, col, val, r, Y_init=y0, precision=pixelsne.FP32,
                                    eta=n / 12.0)
    t0 = time.perf_counter()
    plain.step(1000)
    sync()
    out["plain_eta_n_over_12_1000_s"] = time.perf_counter() - t0
    kl_plain12 = plain.kl()
    out["plain_eta_n_over_12_kl"] = kl_plain12
    del plain
    log(f"[large] plain eta n/12: {out['plain_eta_n_over_12_1000_s']:.2f} s, KL {kl_plain12:.4f}")
    for label, eta, fs, kref, tref in (
            ("eta200_s_sqrt5", 200.0, 5 ** 0.5, kl_plain, out["plain_1000_s"]),
            ("eta_n_over_12_s_sqrt5", n / 12.0, 5 ** 0.5, kl_plain, out["plain_1000_s"]),
            ("vs_plain_eta_n_over_12", n / 12.0, 5 ** 0.5, kl_plain12,
             out["plain_eta_n_over_12_1000_s"])):
        target = 1.01 * kref
        t0 = time.perf_counter()
        Yp = net.place(Xd, r, (s_sub[0] * fs, s_sub[1] * fs))
        sync()
        t_place = time.perf_counter() - t0
        ctx = pixelsne.Context.from_P(rp, col, val, r, Y_init=Yp, precision=pixelsne.FP32,
                                      exag_iters=0, mom_switch=0, eta=eta)
        del Yp
        k0 = ctx.kl()
        t_it, it, k = 0.0, 0, k0
        while it < 1000:
            t1 = time.perf_counter()
            ctx.step(50)
            sync()
            t_it += time.perf_counter() - t1
            it += 50
            k = ctx.kl()
            if k <= target:
                break
        res = {"kl_placed": k0, "target_kl": target, "iters": it if k <= target else None,
               "kl": k, "seconds": (t_place + t_it) if k <= target else None, "place_s": t_place}
        res["speedup"] = tref / res["seconds"] if res["seconds"] else None
        out[label] = res
        log(f"[large] {label}: {json.dumps(res)}")
        del ctx
    return out


def _oracle_rate(oracle, st, p, P, n, min_seconds, max_iters, chunk):
    """points x iterations / s of oracle.iterate over at least min_seconds
    (or max_iters iterations), in chunks."""
    iters, t = 0, 0.0
    while (t < min_seconds or iters == 0) and iters < max_iters:
        k = min(chunk, max_iters - iters)
        t0 = time.perf_counter()
        oracle.iterate(st, p, P, k)
        t += time.perf_counter() - t0
        iters += k
    return {"value": n * iters / t, "iterations": iters, "seconds": t}


def knn_compare(args):
    """Setup with the exact brute-force kNN against the approximate kNN of
    Section 4.3 (random-projection trees + neighbour exploring) on the
    5,000,000 x 100 workload with 1% outliers (perplexity 30, k 90, screen
    4096): setup time of each, recall of the approximate lists on sampled rows
    against the oracle's exact FP64 kNN of those rows, and the exact-Z KL after
    1,000 iterations from the same start with each P (the paper reports the
    quality of the RP-tree P as close to the exact one)."""
    import numpy as np
    import torch

    import oracle
    from paper_1611_02568_amd import datagen, pixelsne

    torch.cuda.set_device(0)
    n, r, u = args.large_n, 4096, 30.0
    k = int(3 * u)
    X, _, _ = datagen.zipf_mixture_outliers(n=n)
    Xd = torch.from_numpy(X).cuda()
    y0 = torch.as_tensor(datagen.initial_embedding(n, seed=datagen.seed_for(4, 1)))
    out = {"n": n, "k": k, "trees": args.knn_trees, "explore": args.knn_explore}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx, _ = pixelsne.knn_approx(Xd, k, trees=args.knn_trees, explore=args.knn_explore, seed=1)
    torch.cuda.synchronize()
    out["approx_knn_s"] = time.perf_counter() - t0
    rows = np.random.default_rng(15).choice(n, args.knn_rows, replace=False)
    ei, _ = oracle.knn(X, k, rows=rows)
    got = idx.cpu().numpy()[rows]
    out["recall"] = float(np.mean([len(set(a.tolist()) & set(b.tolist())) / k
                                   for a, b in zip(got, ei)]))
    del idx
    log(f"[knn] approximate kNN {out['approx_knn_s']:.2f} s, recall {out['recall']:.4f}")
    ctxs = {}
    for label, trees in (("approx", args.knn_trees), ("exact", 0)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = pixelsne.Context.from_data(Xd, u, r, Y_init=y0, precision=pixelsne.FP32,
                                         knn_trees=trees, knn_explore=args.knn_explore, seed=1)
        torch.cuda.synchronize()
        out[label + "_setup_s"] = time.perf_counter() - t0
        ctx.step(1000)
        out[label + "_kl_own_P"] = ctx.kl()
        ctxs[label] = ctx
        log(f"[knn] {label}: setup {out[label + '_setup_s']:.2f} s, "
            f"KL after 1,000 iterations (its own P) {out[label + '_kl_own_P']:.5f}")
    # both embeddings scored against the exact P: the approximate run's final
    # state loaded into the exact context
    ex = ctxs["exact"]
    out["exact_kl_exact_P"] = out["exact_kl_own_P"]
    st = ctxs["approx"].get_state()
    del ctxs["approx"]
    ex.set_state(st["z"], st["s"], u=st["u"], g=st["g"], iteration=st["iteration"])
    out["approx_kl_exact_P"] = ex.kl()
    log(f"[knn] against the exact P: approx run {out['approx_kl_exact_P']:.5f}, "
        f"exact run {out['exact_kl_exact_P']:.5f}")
    return out


def cpu_baseline(args):
    """The oracle as it stands (FP64, OpenMP over points) on this host's cores,
    on bounded samples of the workloads:
      * the benchmark's shape: 1,000,000 points, screen 2048, theta 0.5, a P of
        the benchmark's row length (258 nonzeros per row; synthetic, from the
        input generators, since the oracle cannot build P from a million
        128-dimensional rows in minutes), the benchmark's initial embedding:
        the first iterations on all cores (the headline figure) and on one
        thread (the paper's own timings are single-threaded);
      * the 2,000 x 50 mixture (its own P, perplexity 30, screen 512), all
        cores and one thread;
      * 70,000 points at the uint8 workload's row length (136, synthetic P),
        screen 1024, all cores and one thread.
    Setup is not timed."""
    import numpy as np

    import oracle
    from paper_1611_02568_amd import datagen

    cores = oracle.num_threads()
    res = {}
    # the benchmark's shape
    n = 1_000_000
    P = datagen.circulant_affinities(n, 129, seed=datagen.seed_for(2, 5))
    y0 = datagen.initial_embedding(n, seed=datagen.seed_for(2, 1))
    p = oracle.params(2048)
    st = oracle.State(y0, 2048)
    res["1m_all"] = _oracle_rate(oracle, st, p, P, n, args.cpu_seconds, 50, 2)
    oracle.set_num_threads(1)
    res["1m_single"] = _oracle_rate(oracle, oracle.State(y0, 2048), p, P, n, 0.0, 1, 1)
    oracle.set_num_threads(cores)
    del P, st
    # the 2,000-point workload
    X, _ = datagen.small_mixture(n=2000)
    P = oracle.build_P(X, 30.0)
    y0 = datagen.initial_embedding(2000, seed=datagen.seed_for(0, 1))
    p = oracle.params(512)
    res["2k_all"] = _oracle_rate(oracle, oracle.State(y0, 512), p, P, 2000, 2.0, 1000, 50)
    oracle.set_num_threads(1)
    res["2k_single"] = _oracle_rate(oracle, oracle.State(y0, 512), p, P, 2000, 2.0, 1000, 50)
    oracle.set_num_threads(cores)
    # 70,000 points, synthetic P of the uint8 workload's row length
    P = datagen.circulant_affinities(70000, 68, seed=datagen.seed_for(1, 5))
    y0 = datagen.initial_embedding(70000, seed=datagen.seed_for(1, 1))
    p = oracle.params(1024)
    res["70k_all"] = _oracle_rate(oracle, oracle.State(y0, 1024), p, P, 70000, 3.0, 200, 5)
    oracle.set_num_threads(1)
    res["70k_single"] = _oracle_rate(oracle, oracle.State(y0, 1024), p, P, 70000, 3.0, 20, 1)
    oracle.set_num_threads(cores)
    head = res["1m_all"]
    return {"value": head["value"], "unit": "points*iters/s", "cores": cores, "kind": "oracle",
            "sample": f"iterations 1-{head['iterations']} of the 1,000,000-point workload from "
                      "its initial embedding (screen 2048, theta 0.5), with a synthetic P of the "
                      "benchmark's row length (258 per row) in place of the kNN P; FP64, "
                      "OpenMP; setup not timed",
            "single_thread": {"value": res["1m_single"]["value"], "cores": 1,
                              "sample": "iteration 1 of the same"},
            "workloads": res}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="minimum all-core oracle time on the 1,000,000-point workload")
    ap.add_argument("--reps", type=int, default=3,
                    help="timed windows of the same iterations (from a saved state)")
    ap.add_argument("--no-ttkl", dest="ttkl", action="store_false",
                    help="skip the learned-placement time-to-KL comparison")
    ap.add_argument("--mlp-epochs", type=int, default=20)
    ap.add_argument("--heldout", type=int, default=200_000)
    ap.add_argument("--plain-timing", action="store_true",
                    help="time the region without per-pass events (for counter runs)")
    ap.add_argument("--opening-fp64", type=int, default=0, choices=(0, 1),
                    help="FP32 path: run the opening test and distances in FP64")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch kernels one by one outside the timed region too")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after the timed region, copy a buffer of this size once (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    ap.add_argument("--large", action="store_true",
                    help="run only the 5M time-to-KL experiment and print its own JSON line")
    ap.add_argument("--large-n", type=int, default=5_000_000)
    ap.add_argument("--knn-compare", action="store_true",
                    help="run only the exact vs approximate kNN setup comparison on the "
                         "5M workload and print its own JSON line")
    ap.add_argument("--knn-trees", type=int, default=16)
    ap.add_argument("--knn-explore", type=int, default=2)
    ap.add_argument("--knn-rows", type=int, default=200)
    ap.add_argument("--r-sweep", action="store_true",
                    help="run only the tree comparison (pixel tree at r = 512 ... 8,192 and the "
                         "data-driven tree) on the FP32 workload and print its own JSON line")
    ap.add_argument("--three-d", action="store_true",
                    help="run only the 3-D embedding (voxel octree) on the FP32 workload's data "
                         "and print its own JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; sharding across GPUs is "
                                   "described, not implemented, so --gpus must be 1"}))
        sys.exit(2)

    if args.r_sweep:
        res = r_sweep(args)
        print(json.dumps({"metric": "ms per iteration and exact-Z KL, pixel-aligned tree at "
                                    "screen sizes r against the data-driven tree",
                          "unit": "ms", "higher_is_better": False, "n_gpus": 1,
                          "data": "synthetic", "dtype": "f32", "steps": args.steps,
                          "warmup": args.warmup, "result": res}), flush=True)
        return

    if args.three_d:
        res = three_d(args)
        print(json.dumps({"metric": "3-D embedding: ms per iteration and exact-Z KL, voxel "
                                    "octree, 1M x 128",
                          "unit": "ms", "higher_is_better": False, "n_gpus": 1,
                          "data": "synthetic", "dtype": "f64", "steps": args.steps,
                          "warmup": args.warmup, "result": res}), flush=True)
        return

    if args.knn_compare:
        res = knn_compare(args)
        print(json.dumps({"metric": "setup seconds, exact vs approximate kNN, 5M x 100",
                          "unit": "s", "higher_is_better": False, "n_gpus": 1,
                          "data": "synthetic", "dtype": "f32", "result": res}), flush=True)
        return

    if args.large:
        import torch
        torch.cuda.set_device(0)
        res = time_to_kl_large(args)
        print(json.dumps({"metric": "time-to-KL within 1%, MLP init vs plain, 5M x 100",
                          "unit": "s", "higher_is_better": False, "n_gpus": 1,
                          "data": "synthetic", "dtype": "f32", "result": res}), flush=True)
        return

    res, setup_s, nnz = run_gpu(args)
    if args.calibrate_copy_mib:
        import torch
        a = torch.ones(args.calibrate_copy_mib * 2**18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    main32 = res["fp32"]
    # dominant kernel of the FP32 iteration
    per = main32.get("pass_ms", {"unmeasured": 0.0})
    dom = max(per, key=per.get)
    if dom == "traverse":
        ach = main32["traverse"]["TFLOPs"]
        roof = {"bound": "alu", "kernel": "k_traverse<float, false, true, false>", "achieved": ach,
                "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / VALU_PEAK_TFLOPS,
                "traffic": None}
    elif dom == "attract":
        ach = main32["attract"]["GBps"]
        roof = {"bound": "hbm", "kernel": "k_attract<float, 0>", "achieved": ach,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": None}
    elif "tree_build" in main32:
        ach = main32["tree_build"]["GBps"]
        roof = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None}
    else:
        roof = None                           # --plain-timing: no per-pass times
    if roof:
        roof["traffic"] = measured_traffic(roof["kernel"])

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(args)

    line = {
        "metric": METRIC,
        "value": main32["value"],
        "unit": "points*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.n:,} x 128 fp32 Zipf(1.1) 100-component Gaussian mixture, "
                               "perplexity 50, k 150, screen 2048x2048, theta 0.5, FP32 path "
                               + ("(FP64 Z, cell sums and opening test)" if args.opening_fp64
                                  else "(FP32 opening test and forces, FP64 Z and cell sums)"),
                   "n": args.n, "D": 128, "perplexity": 50, "k": 150, "screen": 2048,
                   "theta": 0.5, "nnz": nnz},
        "roofline": roof,
        "cpu_baseline": cpu,
        "iteration_roofline": main32.get("iteration"),
        "ms_per_step_reps": main32.get("reps_ms_per_step"),
        "ms_per_step_sd": main32.get("ms_per_step_sd"),
        "steady_state": main32.get("steady_state") and {
            "iterations": main32["steady_state"]["iterations"],
            "value": main32["steady_state"]["value"],
            "ms_per_step": main32["steady_state"]["ms_per_step"],
            "iteration_frac_hbm": main32["steady_state"]["iteration"]["frac_hbm"]},
        "fp64": res.get("fp64") and {"value": res["fp64"]["value"],
                                     "ms_per_step": res["fp64"]["ms_per_step"]},
        "setup_s": setup_s,
        "time_to_kl": res.get("time_to_kl"),
        "fp32_vs_fp64": res.get("fp32_vs_fp64"),
        "passes": {k: v for k, v in res.items() if k in ("fp32", "fp64")},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
