#!/usr/bin/env python3
"""Benchmark: PFE outer (SOC) iterations per second on one MI355X.

Workload: 481x321 synthetic Voronoi image (40 cells, smooth colour gradients,
noise 0.03), RGB + scaled xy features, 8-neighbour heat-kernel graph
(sigma 0.1), d = 10, 10 Split-Bregman iterations per SOC iteration, Jacobi-PCG
to relative residual 1e-6, FP32 vectors with FP64 reductions; lambda = r = c
with the shrink threshold 1/c at the 0.99-quantile of |M Y0|.

One timed step = one SOC iteration (10 inner solves + shrink/Bregman + P/B
update), launched as one persistent kernel; inputs are resident in HBM.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "voronoi481x321_8nbr"
PEAK_HBM_GBS = 8000.0


def progress(msg):
    """A line on stderr when a leg of the benchmark ends (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def shape_label(shape):
    """A readable name of an autotuned launch shape."""
    if shape["persistent"]:
        return "persistent"
    if shape.get("pixel"):
        return f"per-row ({shape['pixel']} workgroup(s) per CU)"
    if shape["strips"]:
        return f"strips ({shape['strips']} wave(s)" + (", one pass per iteration)" if shape.get("one_pass") else ")")
    return "row chunks"


def launch_of(info):
    """Launch of a run from its step flags."""
    if info["workgroups"]:
        return "persistent"
    return "per-row" if info["flags"] & 4 else ("strips" if info["flags"] & 2 else "multi")


def algorithmic_bytes(n, E, d, esz, cg_iters, solves, n_inner, n_outer, pupdate=True):
    """Bytes the method has to move (FP32 values, int32 indices): per CG
    iteration the slot columns and weights, row pointers, diagonal and ten n x d
    vector streams; per inner step the residual or edge update with its split
    state; per SOC iteration the Gram and apply passes.  Summed over n_outer
    SOC iterations (without the P- and B-update when pupdate is False: Split
    Bregman alone)."""
    rowptr = 4 * (n + 1)
    csr = 8 * 2 * E + rowptr                  # column index + weight per directed slot
    nd = n * d * esz
    cg_iter = csr + 2 * n * esz + 10 * nd       # A: r,p_old -> p_new,q ; B: x,p,q,r -> x,r
    first_res = csr + 3 * n * esz + 4 * nd      # P, B, x -> r
    edge_res = csr + 3 * n * esz + 4 * nd + 2 * E * d * esz + 4 * E  # + b read/write per edge
    ortho = 2 * n * esz + 6 * nd                # Gram (Y, B) + apply (Y, B -> P, B)
    per_outer_fixed = first_res + (n_inner - 1) * edge_res + (ortho if pupdate else 0)
    return cg_iters * cg_iter + n_outer * per_outer_fixed


# committed rocprofv3 FETCH_SIZE / WRITE_SIZE records: (workload, launch) ->
# file; persistent records count one k_soc launch, per-row and strip records one
# SOC iteration of the one-launch-per-phase path (all its kernels)
TRAFFIC_FILES = {("voronoi481x321_8nbr", "persistent"): "k_soc_voronoi481x321_traffic.json",
                 ("voronoi1024_r2", "per-row"): "per_row_voronoi1024_r2_traffic.json",
                 ("voronoi_batch64_8nbr", "strips"): "strips_voronoi_batch64_traffic.json"}


def measured_traffic(workload, launch):
    """HBM traffic per SOC iteration from the committed counter runs (scaled by
    the copy-kernel calibration), or None when there is none for the workload
    and launch shape or the kernel source changed since the counters were
    taken."""
    import hashlib
    if (workload, launch) not in TRAFFIC_FILES:
        return None
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES[(workload, launch)])
    src = os.path.join(ROOT, "paper_1612_06496_amd", "csrc", "solver.hip")
    try:
        rec = json.load(open(path))
        cur = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if rec.get("solver_sha256") != cur:
        return None
    return rec.get("traffic_bytes_per_launch", rec.get("traffic_bytes_per_soc"))


def copy_bandwidth(gib):
    """Achievable bandwidth of a plain 16-byte-vector device copy (read + write
    bytes / time), best of 5."""
    import ctypes as C
    import torch
    from paper_1612_06496_amd import _lib as L
    nbytes = int(gib * 2**30) // 64 * 64
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    best = 0.0
    for _ in range(6):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        L.check(L.lib.pfe_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, stream),
                "pfe_stream_copy")
        b.record()
        torch.cuda.synchronize()
        best = max(best, 2 * nbytes / (a.elapsed_time(b) / 1e3) / 1e9)
    del src, dst
    return best


def load_graph(name, seed):
    """(workload, Graph) of a named image or point-cloud workload."""
    import synth
    from paper_1612_06496_amd import Graph
    if name in synth.EDGE_WORKLOADS:
        wl = synth.make_edges_workload(name, seed)
        return wl, Graph.edges(wl.n, wl.src, wl.dst, wl.dist2, wl.sigma)
    wl = synth.make_workload(name, seed)
    return wl, Graph.grid(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)


def training_residuals(workload, seeds, ratios, solves_per_image, cols, rng):
    """Residuals of the PFE solves themselves, the network's training data:
    on each held-out image (seed), solves_per_image Jacobi-PCG inner solves
    split evenly over the lambda/r of the sweep, each contributing `cols`
    randomly chosen columns of its initial residual (rhs - A Y of the solve).
    Returns the open solvers/graphs and groups (solver, lambda, r, n x m
    residual columns) of one system each."""
    import torch

    from paper_1612_06496_amd import Solver
    keep, groups = [], []
    for seed in seeds:
        wl, G = load_graph(workload, seed)
        S = Solver(G, wl.y0, lam=1.0, r=1.0, n_inner=wl.n_inner, tol=wl.tol, maxit=5000, persistent=False,
                   graphs=True)
        c = 1.0 / S.edge_quantile(0.99)
        per_ratio = max(1, solves_per_image // len(ratios))
        for ratio in ratios:
            S.set_penalties(ratio * c, c)
            S.inner_index = 0
            cap = []
            for _ in range(per_ratio):
                R = S.get("resid")
                pick = torch.as_tensor(rng.choice(wl.d, cols, replace=False), device="cuda")
                cap.append(R[:, pick].clone())
                S.step("inner", allow_noconv=True)
                if S.inner_index == wl.n_inner:
                    S.step("outer", allow_noconv=True)     # the P- and B-update closing the SOC iteration
            groups.append((S, ratio * c, c, torch.cat(cap, dim=1)))
        keep.append((G, S))
    return keep, groups


def learned_leg(train_seeds=(1000, 1001, 1002, 1003, 1004), ratios=(1.0, 10.0, 100.0, 1000.0),
                solves_per_image=100, cols_per_solve=2, steps=600, batch_cols=16, lr=3e-3,
                workload="voronoi1024_r2", train_workload=None, n_outer=2):
    """PCG iterations to 1e-6 with the learned preconditioner vs Jacobi, and
    vs FSAI (a classical sparse approximate inverse factor of the same form).

    Training data: 500 PFE inner solves on five held-out images (training
    seeds, 100 solves each, 25 per lambda/r of the sweep), two columns of each
    solve's initial residual.  A training step draws batch_cols columns of one
    (image, lambda/r) system.  The held-out loss per lambda/r is measured on
    the evaluation image's residuals before and after training, next to the
    identity network's (Jacobi).  Evaluation on the evaluation image (seed 0):
    from the same start, one untimed SOC iteration, then n_outer timed ones
    (n_outer x n_inner solves) with each preconditioner in its autotuned launch
    shape (tuned at the first ratio, kept for the others; Jacobi persistent or
    one launch per phase, the factor preconditioners one launch per phase on
    image strips or row chunks, with one or two passes per CG iteration; PCG
    replayed from HIP graphs); the network's factor inference and the FSAI
    factor are timed separately (once per graph and penalties).
    train_workload: the workload of the training images (default: the
    evaluation workload; the network is size-independent)."""
    import numpy as np
    import torch

    import synth
    from paper_1612_06496_amd import Graph, Mpnn, Solver

    t_start = time.perf_counter()
    rng = np.random.default_rng(0)
    keep, groups = training_residuals(train_workload or workload, train_seeds, ratios, solves_per_image,
                                      cols_per_solve, rng)
    t_data = time.perf_counter() - t_start
    progress(f"learned leg: {len(train_seeds) * solves_per_image} training solves in {t_data:.1f} s")
    init = rng.normal(0.0, 0.1, size=Mpnn.NPARAMS).astype(np.float32)
    init[672:] = 0.0
    init[721] = np.log(np.e - 1.0)
    net = Mpnn(init)

    # held-out residuals: the evaluation image's first inner solve per ratio
    wl, G = load_graph(workload, 0)
    Sh = Solver(G, wl.y0, lam=1.0, r=1.0, n_inner=wl.n_inner, tol=wl.tol, maxit=5000, persistent=False)
    c = 1.0 / Sh.edge_quantile(0.99)
    held = []
    for ratio in ratios:
        Sh.set_penalties(ratio * c, c)
        held.append((ratio, Sh.get("resid")))
    ident = Mpnn(None)

    def held_losses(network):
        out = {}
        for ratio, R in held:
            Sh.set_penalties(ratio * c, c)
            out[str(ratio)] = round(network.train_step(Sh, R, 0.0), 5)
        return out

    loss_before, loss_jacobi = held_losses(net), held_losses(ident)
    t0 = time.perf_counter()
    losses = []
    for t in range(steps):
        S, lam, r, R = groups[rng.integers(len(groups))]
        pick = torch.as_tensor(rng.choice(R.shape[1], batch_cols, replace=False), device="cuda")
        S.set_penalties(lam, r)
        losses.append(net.train_step(S, R[:, pick], lr))
    t_train = time.perf_counter() - t0
    loss_after = held_losses(net)
    ident.close()
    Sh.close()
    for G_, S_ in keep:
        S_.close()
        G_.close()
    del keep, groups
    progress(f"learned leg: {steps} training steps in {t_train:.1f} s")
    training = {"train_images": list(train_seeds), "train_solves": len(train_seeds) * solves_per_image,
                "columns_per_solve": cols_per_solve, "train_steps": steps, "batch_columns": batch_cols,
                "data_s": round(t_data, 1), "train_s": round(t_train, 1),
                "held_out_loss": {"jacobi": loss_jacobi, "initial": loss_before, "trained": loss_after}}

    rows = []
    jshape = None     # Jacobi's launch shape, autotuned at the first ratio (the factor path: at every
                      # ratio, its best shape depends on the iteration count)
    for ratio in ratios:
        res = {"lambda_over_r": ratio}
        # FSAI is built for pixel grids (stencil slot layout) only
        for pre in (("jacobi", "fsai", "learned") if wl.kind == "grid" else ("jacobi", "learned")):
            S = Solver(G, wl.y0, lam=ratio * c, r=c, n_inner=wl.n_inner, tol=wl.tol, maxit=5000,
                       persistent=(pre == "jacobi" and (jshape is None or jshape["persistent"] == 1)), graphs=True)
            factor_ms = None
            shape = None
            if pre != "jacobi":
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if pre == "learned":
                    S.set_learned(net)
                else:
                    S.set_fsai()
                torch.cuda.synchronize()
                factor_ms = round((time.perf_counter() - t0) * 1e3, 2)
                shape = [t for t in S.autotune(trials=1) if t["chosen"]][0]
            elif jshape is None:
                shape = jshape = [t for t in S.autotune(trials=1) if t["chosen"]][0]
            else:
                shape = jshape
                S.set_launch_shape(persistent=bool(shape["persistent"]), strips=shape["strips"], team=shape["team"],
                                   row_cache=bool(shape["row_cache"]), second_weight=shape["second_weight"],
                                   pixel=int(shape["pixel"]))
            S.solve(1, allow_noconv=True)
            S.stats(reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = S.solve(n_outer, info=True, allow_noconv=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res[pre] = {"iters_mean": round(info["cg_iters_total"] / max(1, info["solves"]), 2),
                        "iters_max": info["cg_iters_max"], "solves": info["solves"],
                        "ms_per_solve": round(dt * 1e3 / max(1, info["solves"]), 3),
                        "rel_res_max": float(f"{info['rel_res_max']:.3g}"), "status": info["status"]}
            if shape is not None:
                res[pre]["launch"] = shape_label(shape)
            if factor_ms is not None:
                res[pre]["factor_ms"] = factor_ms
                res[pre]["ms_per_solve_amortised"] = round(res[pre]["ms_per_solve"] + factor_ms / max(1, info["solves"]), 3)
            S.close()
        rows.append(res)
        progress(f"learned leg: lambda/r = {ratio} done")
    net.close()
    return {"workload": workload, "train_workload": train_workload or workload, "n": wl.n, "d": wl.d,
            "training": training,
            "run": f"{n_outer} SOC iterations x {wl.n_inner} inner solves per preconditioner and lambda/r",
            "sweep": rows}


def d_sweep_leg(G, wl, dims=(5, 10, 15, 20, 25), steps=10):
    """SOC iterations/s of one image at several embedding dimensions d (one
    context per d, its launch shape autotuned, shrink-active penalties from its
    own initial embedding; one untimed and `steps` timed SOC iterations)."""
    import torch

    import synth
    from paper_1612_06496_amd import Solver
    rows = []
    for d in dims:
        y0 = synth.smooth_y0(wl.H, wl.W, d, 7919)
        S = Solver(G, y0, lam=1.0, r=1.0, n_inner=wl.n_inner, tol=wl.tol, maxit=1000)
        c = 1.0 / S.edge_quantile(0.99)
        S.set_penalties(c, c)
        S.autotune(trials=1)
        S.solve(1)
        S.stats(reset=True)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for _ in range(steps):
            S.solve(1)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop)
        info = S.stats(reset=True)
        rows.append({"d": d, "outer_iters_per_s": round(steps / (ms / 1e3), 1), "ms_per_step": round(ms / steps, 4),
                     "pcg_iters_per_solve": round(info["cg_iters_total"] / max(1, info["solves"]), 2),
                     "launch": launch_of(info)})
        S.close()
        progress(f"d-sweep: d = {d} done")
    return rows


def split_activity(G, wl, S, Y0, c):
    """Share of nonzero entries of the split variable d (edge differences the
    shrink leaves active) in the first Split-Bregman iteration from the state
    the timed SOC iterations ended in.  Measured in a second context that stores
    d (keep_split), loaded with that state, so the timed kernels stay as timed."""
    from paper_1612_06496_amd import Solver
    S2 = Solver(G, Y0, lam=c, r=c, n_inner=wl.n_inner, tol=wl.tol, maxit=1000, keep_split=True, persistent=False)
    for which in ("Y", "P", "B"):
        S2.set(which, S.get(which))
    S2.step("inner")
    frac = S2.monitor()["split_nonzero"]
    S2.close()
    return frac


def host_cpu():
    """CPU model and logical CPU count of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def le_init_leg(G, wl, k=32, tol=1e-12, steps=10, oracle_time=True):
    """The Laplacian-eigenmap initialisation on the device (pfe_le_init,
    d = the workload's d, a block of k vectors from a seeded Gaussian start,
    FP64) timed with HIP events; then the headline measurement repeated from
    that embedding (one untimed and `steps` timed SOC iterations, shrink-active
    penalties from it, autotuned shape).  With oracle_time, the oracle's
    shift-invert Lanczos on the same graph is timed on the host for context."""
    import numpy as np
    import torch

    from paper_1612_06496_amd import Solver, le_init
    X0 = torch.as_tensor(np.random.default_rng(5).normal(size=(wl.n, k)), device="cuda")
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    Y, mu, info = le_init(G, wl.d, X0, tol=tol, max_iter=400)
    stop.record()
    torch.cuda.synchronize()
    ms_le = start.elapsed_time(stop)
    out = {"d": wl.d, "k": k, "tol": tol, "ms": round(ms_le, 2), "iterations": info["iterations"],
           "degree": info["degree"], "residual": float(f"{info['residual']:.3g}"),
           "mu": [float(f"{m:.4g}") for m in mu]}
    progress(f"LE initialisation on the GPU: {ms_le:.1f} ms")
    S = Solver(G, Y.float(), lam=1.0, r=1.0, n_inner=wl.n_inner, tol=wl.tol, maxit=1000)
    c = 1.0 / S.edge_quantile(0.99)
    S.set_penalties(c, c)
    S.autotune(trials=1)
    S.solve(1)
    S.stats(reset=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        S.solve(1)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    st = S.stats(reset=True)
    S.close()
    out["headline_from_le"] = {"lambda": c, "r": c, "ms_per_step": round(ms / steps, 4),
                               "outer_iters_per_s": round(steps / (ms / 1e3), 1),
                               "pcg_iters_per_solve": round(st["cg_iters_total"] / max(1, st["solves"]), 2),
                               "launch": launch_of(st)}
    if oracle_time:
        import oracle as O
        g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
        t0 = time.perf_counter()
        O.le_init(g, wl.d)
        out["oracle_s"] = round(time.perf_counter() - t0, 2)
    return out


def clustering_leg(name="gmm200k_knn16_rcm", steps=3):
    """The general data-clustering configuration (Sec. IV's use beyond images):
    a Gaussian-mixture point cloud's symmetrised exact k-NN graph (edge list,
    general CSR slot layout), d = 20, shrink-active penalties, Jacobi-PCG;
    autotuned launch shape, one untimed and `steps` timed SOC iterations; then
    k-means (K = the mixture's components) on the embedding and its label
    agreement with the mixture components (Hungarian matching)."""
    import numpy as np
    import torch
    from scipy.optimize import linear_sum_assignment

    import synth
    from paper_1612_06496_amd import Graph, Solver, kmeans
    t0 = time.perf_counter()
    wl = synth.make_edges_workload(name, 0)
    t_input = time.perf_counter() - t0
    G = Graph.edges(wl.n, wl.src, wl.dst, wl.dist2, wl.sigma)
    S = Solver(G, wl.y0, lam=1.0, r=1.0, n_inner=wl.n_inner, tol=wl.tol, maxit=1000, graphs=True)
    c = 1.0 / S.edge_quantile(0.99)
    S.set_penalties(c, c)
    tuned = [t for t in S.autotune(trials=1) if t["chosen"]]
    S.solve(1)
    S.stats(reset=True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        S.solve(1)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    info = S.stats(reset=True)
    byt = algorithmic_bytes(G.n, G.n_edges, wl.d, 4, info["cg_iters_total"], info["solves"], wl.n_inner, steps)
    yh = S.get("Yhat")
    K = wl.n_clusters
    rows = np.random.default_rng(0).choice(G.n, K, replace=False)
    labels, _, kit = kmeans(yh, yh[torch.as_tensor(rows, device="cuda")].double(), 300)
    lab = labels.cpu().numpy()
    conf = np.zeros((K, K))
    np.add.at(conf, (lab, np.asarray(wl.labels)), 1)
    ri, ci = linear_sum_assignment(-conf)
    agree = float(conf[ri, ci].sum() / G.n)
    out = {"workload": name, "n": G.n, "edges": G.n_edges, "d": wl.d, "lambda": c, "r": c,
           "input_s": round(t_input, 1), "ms_per_step": round(ms / steps, 3),
           "outer_iters_per_s": round(steps / (ms / 1e3), 2),
           "pcg_iters_per_solve": round(info["cg_iters_total"] / max(1, info["solves"]), 2),
           "algorithmic_gbs": round(byt / (ms / 1e3) / 1e9, 1),
           "frac": round(byt / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
           "launch": launch_of(info),
           "autotuned": tuned[0] if tuned else None,
           "kmeans_iterations": kit, "label_agreement_with_components": round(agree, 4)}
    S.close()
    G.close()
    progress(f"clustering leg ({name}): {ms / steps:.1f} ms per SOC iteration")
    return out


def d_sweep_batched_leg(wl, c, dims=(5, 10, 15, 20, 25), steps=10):
    """The same d-sweep in ONE launch per SOC iteration: copies of the image in
    a block-diagonal union, copy k embedded in dims[k] dimensions (its initial
    embedding padded with zero columns to the largest d; the library keeps
    them zero and orthonormalises each copy on its active block).  One
    lambda = r = c for all copies (a batch shares its penalties); autotuned
    launch shape; one untimed and `steps` timed SOC iterations."""
    import numpy as np
    import torch

    import synth
    from paper_1612_06496_amd import Graph, Solver
    dmax = max(dims)
    parts = [Graph.grid(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma) for _ in dims]
    U = Graph.union(parts)
    for p_ in parts:
        p_.close()
    Y0 = np.zeros((U.n, dmax), dtype=np.float32)
    for k, d in enumerate(dims):
        Y0[k * wl.n:(k + 1) * wl.n, :d] = synth.smooth_y0(wl.H, wl.W, d, 7919)
    S = Solver(U, Y0, lam=c, r=c, n_inner=wl.n_inner, tol=wl.tol, maxit=1000)
    tuned = [t for t in S.autotune(trials=1) if t["chosen"]]
    S.solve(1)
    S.stats(reset=True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        S.solve(1)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    info = S.stats(reset=True)
    mon = S.monitor()
    S.close()
    U.close()
    progress("d-sweep in one launch done")
    return {"dims": list(dims), "images": len(dims), "n": int(len(dims) * wl.n), "d_max": dmax,
            "lambda": c, "r": c, "ms_per_step": round(ms / steps, 4),
            "outer_iters_per_s": round(steps / (ms / 1e3), 1),
            "pcg_iters_per_solve": round(info["cg_iters_total"] / max(1, info["solves"]), 2),
            "constraint": float(f"{mon['constraint']:.3g}"),
            "launch": launch_of(info),
            "autotuned": tuned[0] if tuned else None}


def cpu_baseline(wls, lam, r, n_steps=2, max_images=2):
    """The FP64 oracle on the host, on a bounded sample: n_steps SOC iterations
    of the workload's first max_images images (sparse LU factorisation reported
    separately); for a batch the rate is scaled to the whole batch by its
    vertex count."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O
    sample = wls[:max_images]
    n_all = sum(w.n for w in wls)
    n_sample = sum(w.n for w in sample)
    dt = t_fact = 0.0
    with threadpool_limits(limits=1):
        for wl in sample:
            g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
            Y = O.orthonormalize_init(g, wl.y0)
            t0 = time.perf_counter()
            solve = O.DirectSolver(O.system_matrix(g, lam, r))
            t_fact += time.perf_counter() - t0
            P = np.sqrt(g.D)[:, None] * Y
            B = np.zeros_like(Y)
            t0 = time.perf_counter()
            for _ in range(n_steps):
                Y, P, B = O.soc_outer_step(g, solve, Y, P, B, lam, r, wl.n_inner)
            dt += time.perf_counter() - t0
    scale = n_all / n_sample
    what = (f"{len(sample)} of {len(wls)} images ({n_sample} of {n_all} vertices, rate scaled by vertex count)"
            if len(wls) > 1 else "the whole image")
    return {"value": n_steps / (dt * scale), "unit": "outer iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_steps} SOC iterations x {sample[0].n_inner} inner on {what}; sparse LU solves "
                      f"(factorisation {t_fact:.2f} s once, not in the rate), 1 thread",
            **host_cpu()}


def cpu_cg_per_solve(names=("voronoi481x321_8nbr", "voronoi1024_r2")):
    """The oracle's own FP64 Jacobi-PCG (the GPU's algorithm) on the host: one
    solve to 1e-6 of each image's first inner step (rhs = r/2 D Y0, x0 = Y0,
    Y0 D-orthonormalised, lambda = r = the shrink-active scale), one thread."""
    from threadpoolctl import threadpool_limits

    import oracle as O
    import synth
    out = {}
    with threadpool_limits(limits=1):
        for name in names:
            wl = synth.make_workload(name, 0)
            g = O.build_grid_graph(wl.feat, wl.H, wl.W, wl.stencil, wl.sigma)
            Y = O.orthonormalize_init(g, wl.y0)
            c = O.shrink_active_scale(g, Y)
            A = O.system_matrix(g, c, c).tocsr()
            rhs = 0.5 * c * g.D[:, None] * Y
            t0 = time.perf_counter()
            _, it, _ = O.pcg(A, rhs, Y, 1.0 / A.diagonal(), 1e-6, 5000)
            out[name] = {"s_per_solve": round(time.perf_counter() - t0, 3), "iterations_max": int(it.max()),
                         "d": wl.d}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-gib", type=float, default=2.0, help="size of the copy-bandwidth probe")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-Jacobi PCG comparison")
    ap.add_argument("--multi-launch", action="store_true", help="one launch per phase instead of one per SOC iteration")
    ap.add_argument("--no-graphs", action="store_true",
                    help="one-launch-per-phase PCG launched from the host instead of replayed from HIP graphs")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shape instead of autotuning it before timing")
    ap.add_argument("--learned-workload", default="voronoi1024_r2",
                    help="evaluation graph of the learned-vs-Jacobi leg (an image or a point-cloud workload)")
    ap.add_argument("--learned-train-workload", default=None,
                    help="training graphs of the learned leg (default: the evaluation workload)")
    ap.add_argument("--learned-outer", type=int, default=2, help="timed SOC iterations per preconditioner and ratio")
    ap.add_argument("--stage2-iters", type=int, default=100,
                    help="Split-Bregman iterations of the timed Stage II run after the SOC iterations (0: skip)")
    ap.add_argument("--kmeans-iters", type=int, default=100,
                    help="cap of the timed k-means (Lloyd) run on the final embedding, single images (0: skip)")
    ap.add_argument("--clustering-workload", default="gmm200k_knn16_rcm",
                    help="point-cloud workload of the data-clustering leg ('' to skip; gmm2m_knn16_rcm is the "
                         "2 M-point configuration, its k-NN input takes about a minute to build)")
    ap.add_argument("--no-le", action="store_true",
                    help="skip the Laplacian-eigenmap initialisation leg (and the headline from its embedding)")
    ap.add_argument("--no-d-sweep", action="store_true",
                    help="skip the SOC-iteration rate at d = 5, 10, 15, 20, 25 on the headline image")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="a single-image workload or an image batch (block-diagonal union) from synth")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the solver runs on a "
              "single MI355X (a batch would shard by whole images, one large graph by row bands with a halo "
              "exchange per CG iteration; neither is built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1612_06496_amd import Graph, Solver

    torch.cuda.set_device(0)
    if args.workload in synth.BATCHES:
        wls = synth.make_batch(args.workload, 0)
        parts = [Graph.grid(w.feat, w.H, w.W, w.stencil, w.sigma) for w in wls]
        G = Graph.union(parts)
        del parts
        Y0 = np.concatenate([w.y0 for w in wls])
    else:
        wls = [synth.make_workload(args.workload, 0)]
        G = Graph.grid(wls[0].feat, wls[0].H, wls[0].W, wls[0].stencil, wls[0].sigma)
        Y0 = wls[0].y0
    wl = wls[0]
    S = Solver(G, Y0, lam=1.0, r=1.0, n_inner=wl.n_inner, tol=wl.tol, maxit=1000,
               persistent=not args.multi_launch, graphs=not args.no_graphs)
    # shrink-active penalties: threshold 1/c at the 0.99-quantile of |M Y0|
    c = 1.0 / S.edge_quantile(0.99)
    S.set_penalties(c, c)
    # the launch shape (persistent or one launch per phase, teams, LDS row
    # cache, image strips) is picked by timing each on this graph; untimed
    tuned = None if args.no_autotune else S.autotune(trials=2)
    progress("launch shape picked" if tuned else "launch shape kept")

    for _ in range(args.warmup):
        S.solve(1)
    S.stats(reset=True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):      # one SOC iteration per step
        S.solve(1)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    info = S.stats(reset=True)          # CG iterations of the timed steps
    progress(f"{args.steps} timed SOC iterations: {ms:.1f} ms")
    mon = S.monitor()
    mon["split_nonzero"] = split_activity(G, wl, S, Y0, c)
    ms_per_step = ms / args.steps
    value = args.steps / (ms / 1e3)

    n, E, d = G.n, G.n_edges, wl.d
    byt = algorithmic_bytes(n, E, d, 4, info["cg_iters_total"], info["solves"], wl.n_inner, args.steps)
    achieved = byt / (ms / 1e3) / 1e9
    launch = launch_of(info)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(args.workload, launch),
            "kernel": "k_soc (one SOC iteration per launch)" if info["workgroups"] else
                      "one kernel per phase (bytes and time per SOC iteration)",
            "bytes_per_launch": int(byt / args.steps), "workgroups": info["workgroups"],
            "launch_flags": info["flags"]}
    default = args.workload == WORKLOAD
    line = {
        "metric": "PFE outer iters/sec at 481x321 d=10 (Jacobi-PCG to 1e-6)" if default else
                  f"PFE outer iters/sec on {args.workload} (Jacobi-PCG to {wl.tol:g})",
        "value": round(value, 2),
        "unit": "outer iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "images": len(wls), "n": n, "edges": E, "d": d,
                   "n_inner": wl.n_inner,
                   "tol": wl.tol, "lambda": c, "r": c, "precond": "jacobi",
                   "launch": launch,
                   "graphs": not args.no_graphs,
                   "autotuned": ([t for t in tuned if t["chosen"]] or [None])[0] if tuned else None},
        "pcg_iters_per_solve": round(info["cg_iters_total"] / max(1, info["solves"]), 2),
        "pcg_iters_learned": None,     # filled by the learned-vs-Jacobi leg below
        "monitor": {k: float(f"{v:.6g}") for k, v in mon.items()},
        "wall_s_timed": round(wall, 4),
        "roofline": roof,
    }
    if args.stage2_iters > 0:
        # Stage II of the two-stage procedure: Split Bregman alone with P and B
        # frozen at the values the timed SOC iterations ended with
        torch.cuda.synchronize()
        start.record()
        S.split_bregman(args.stage2_iters)
        stop.record()
        torch.cuda.synchronize()
        ms2 = start.elapsed_time(stop)
        i2 = S.stats(reset=True)
        progress(f"Stage II, {args.stage2_iters} Split-Bregman iterations: {ms2:.1f} ms")
        b2 = algorithmic_bytes(n, E, d, 4, i2["cg_iters_total"], i2["solves"], args.stage2_iters, 1, pupdate=False)
        line["stage2"] = {"iterations": args.stage2_iters, "ms": round(ms2, 3),
                          "sb_iters_per_s": round(args.stage2_iters / (ms2 / 1e3), 1),
                          "pcg_iters_per_solve": round(i2["cg_iters_total"] / max(1, i2["solves"]), 2),
                          "launch": launch_of(i2),
                          "algorithmic_gbs": round(b2 / (ms2 / 1e3) / 1e9, 1),
                          "frac": round(b2 / (ms2 / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
    if args.kmeans_iters > 0 and len(wls) == 1:
        # the segmentation step: k-means on the embedding, initial centroids at
        # seeded rows (the caller's random draw)
        from paper_1612_06496_amd import kmeans
        yh = S.get("Yhat")
        K = wl.n_clusters
        rows = np.random.default_rng(0).choice(n, K, replace=False)
        C0 = yh[torch.as_tensor(rows, device="cuda")].double()
        torch.cuda.synchronize()
        start.record()
        _, _, kit = kmeans(yh, C0, args.kmeans_iters)
        stop.record()
        torch.cuda.synchronize()
        ms3 = start.elapsed_time(stop)
        line["kmeans"] = {"clusters": K, "iterations": kit, "ms": round(ms3, 3),
                          "ms_per_iteration": round(ms3 / max(1, kit), 4)}
        progress(f"k-means, {kit} Lloyd iterations: {ms3:.1f} ms")
    if not args.no_le and default:
        line["le_init"] = le_init_leg(G, wl, oracle_time=not args.no_cpu_baseline)
    if not args.no_d_sweep and default:
        line["d_sweep"] = d_sweep_leg(G, wl)
        batched = d_sweep_batched_leg(wl, c)
        batched["separate_ms_sum"] = round(sum(r_["ms_per_step"] for r_ in line["d_sweep"]), 4)
        line["d_sweep_one_launch"] = batched
    if args.clustering_workload and default:
        line["clustering"] = clustering_leg(args.clustering_workload)
    if not args.no_learned and default:
        leg = learned_leg(workload=args.learned_workload, train_workload=args.learned_train_workload,
                          n_outer=args.learned_outer)
        line["learned_vs_jacobi"] = leg
        line["pcg_iters_learned"] = {str(r["lambda_over_r"]): {"jacobi_mean": r["jacobi"]["iters_mean"],
                                                               "learned_mean": r["learned"]["iters_mean"],
                                                               "jacobi_max": r["jacobi"]["iters_max"],
                                                               "learned_max": r["learned"]["iters_max"],
                                                               "fsai_mean": r.get("fsai", {}).get("iters_mean"),
                                                               "fsai_max": r.get("fsai", {}).get("iters_max")}
                                     for r in leg["sweep"]}
    if args.copy_gib > 0:
        line["copy_gbs"] = round(copy_bandwidth(args.copy_gib), 1)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(wls, c, c)
        line["cpu_baseline"]["value"] = round(line["cpu_baseline"]["value"], 4)
        if default:
            line["cpu_baseline"]["cg_per_solve"] = cpu_cg_per_solve()
        progress("CPU baseline (oracle) done")
    # explicit teardown while the HIP runtime is up (contexts, networks, graphs)
    from paper_1612_06496_amd import close_all
    close_all()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
