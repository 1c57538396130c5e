"""Benchmark of the SF-GRASS hot path on one MI355X.

One step = one full scoring pass over the power-grid workload (1000 x 1000
mesh plus 2% random diagonal shortcuts, 1,000,000 nodes, 2,037,960 edges,
log-normal weights): build the CSR of the scoring graph (the maximum-weight
spanning tree), centre and smooth 16 random vectors with 20 sweeps, score the
1,037,961 off-tree edges, select the top 10%.  Inputs (edge list, random
block, tree mask, candidate list) are resident in HBM before timing.

Prints one JSON line.  ``value`` is off-tree edges scored per second of the
whole step.  ``roofline`` is for the dominant kernel (the smoothing sweep),
timed with events on the stream the library launches on.

    python bench.py [--steps K] [--warmup W] [--dtype f64|f32] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "off-tree edges scored/s + smoothing HBM GB/s (% peak); surrogate vs plain at equal κ"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_powergrid1000_traffic.json")
SWEEP_SRC = os.path.join(ROOT, "paper_2008_07633_amd", "csrc", "smooth.hip")


def sweep_bytes(n: int, nnz: int, k: int, sx: int, sw: int) -> int:
    """Algorithmic bytes of one sweep: rowptr, col+val, deg, read X_t, write X_t+1."""
    return 4 * (n + 1) + nnz * (4 + sw) + n * sw + 2 * n * k * sx


def score_bytes(ncand: int, n: int, k: int, sx: int, sw: int, ss: int) -> int:
    """Algorithmic bytes of the edge pass: cand id, u, v, w, score per candidate, X once."""
    return ncand * (4 + 8 + sw + ss) + n * k * sx


def src_hash(path: str) -> str:
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def cpu_baseline(g, tree, cand, X0, k: int, T: int, omega: float, ksel: int, f64: bool, gs: bool) -> dict:
    """The oracle (single-threaded C, FP64) timed on one full step of the same workload."""
    import oracle

    oracle.build(force=False)
    tmask = tree.cpu().numpy().astype(bool)
    cnp = cand.cpu().numpy()
    wnp = g.w if f64 else g.w.astype(np.float32).astype(np.float64)
    c0 = time.perf_counter()
    Hc = oracle.laplacian_csr(g.n, g.u[tmask], g.v[tmask], wnp[tmask])
    Xc, _ = oracle.center(X0)
    if gs:
        cl, ncl = oracle.color(Hc)
        Xs = oracle.smooth_gs(Hc, Xc, T, omega, cl, ncl)
    else:
        Xs = oracle.smooth(Hc, Xc, T, omega)
    sc = oracle.edge_scores(Xs, g.u[cnp], g.v[cnp], wnp[cnp])
    oracle.select_topk(sc, cnp, ksel)
    c1 = time.perf_counter()
    ncand = int(cnp.size)
    return {"value": round(ncand / (c1 - c0), 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"one full step of the same workload (tree CSR, centring, {T} sweeps of {k} FP64 vectors, "
                      f"{ncand} scores, top-{ksel} sort), single-threaded C, {c1 - c0:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--smoother", choices=["jacobi", "gs"], default="jacobi",
                    help="gs: multicolour Gauss-Seidel (omega 1; colouring of the tree prepared once, like the tree)")
    ap.add_argument("--sweep-reps", type=int, default=10)
    ap.add_argument("--workload", choices=["powergrid", "knn", "chunglu", "mesh", "sigma", "scaling", "pcg"],
                    default="powergrid",
                    help="powergrid: the headline line; the others print their own lines (bench_workloads.py)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2008_07633_amd import sfg as S

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    S.lib()
    dev = torch.device("cuda:0")
    if args.workload != "powergrid":
        import bench_workloads

        bench_workloads.run(args)
        return

    prm = W.workload_params("powergrid")
    k, T, frac, omega = prm["k"], prm["sweeps"], prm["frac"], 0.5
    g = W.workload_graph("powergrid")
    X0 = W.workload_block("powergrid", g.n)
    f64 = args.dtype == "f64"
    wdt = torch.float64 if f64 else torch.float32
    sx = sw = 8 if f64 else 4

    u = torch.from_numpy(g.u).to(dev)
    v = torch.from_numpy(g.v).to(dev)
    w64 = torch.from_numpy(g.w).to(dev)
    w = w64 if f64 else w64.float()
    x0 = torch.from_numpy(X0).to(dev)
    # input preparation, once per graph: spanning tree and off-tree candidate list
    tree, comps = S.sfg_spanning_tree(g.n, u, v, w64)
    assert comps == 1
    cand = torch.nonzero(tree == 0).reshape(-1).to(torch.int32)
    ncand = int(cand.numel())
    ksel = int(math.ceil(frac * ncand))
    nnz = 2 * (g.n - 1)

    # preallocated buffers: the timed step allocates nothing and never synchronises
    ws_csr = torch.empty(S.sfg_workspace_bytes(S.OP_LAPLACIAN_CSR, g.n, g.m, 0, wdt), dtype=torch.uint8, device=dev)
    ws_sm = torch.empty(S.sfg_workspace_bytes(S.OP_SMOOTH, g.n, 0, k, wdt), dtype=torch.uint8, device=dev)
    ws_sel = torch.empty(S.sfg_workspace_bytes(S.OP_SELECT_TOPK, 0, ncand, 0, wdt), dtype=torch.uint8, device=dev)
    H = S.Csr(g.n, nnz, torch.empty(g.n + 1, dtype=torch.int32, device=dev),
              torch.empty(nnz, dtype=torch.int32, device=dev), torch.empty(nnz, dtype=wdt, device=dev),
              torch.empty(nnz, dtype=torch.int32, device=dev), torch.empty(g.n, dtype=wdt, device=dev))
    X = torch.empty((g.n, k), dtype=wdt, device=dev)
    score = torch.empty(ncand, dtype=wdt, device=dev)
    sel = torch.empty(ncand, dtype=torch.uint8, device=dev)
    tau = torch.empty(1, dtype=torch.float64, device=dev)

    gs = args.smoother == "gs"
    if gs:
        omega = 1.0
        S.sfg_laplacian_csr(g.n, u, v, w, mask=tree, ws=ws_csr, out=H, nnz=nnz)
        classes = S.sfg_color(H)

    def step():
        S.sfg_laplacian_csr(g.n, u, v, w, mask=tree, ws=ws_csr, out=H, nnz=nnz)       # a1
        if gs:
            S.sfg_smooth_gs(H, classes, x0, T, omega, storage=wdt, out=X, ws=ws_sm)
        else:
            S.sfg_smooth(H, x0, T, omega, storage=wdt, out=X, ws=ws_sm)                # a2 + a3
        S.sfg_edge_scores(X, u, v, w, cand=cand, out=score)                            # a4
        S.sfg_select_topk(score, ksel, sel=sel, tau=tau, ws=ws_sel, sync=False)         # a5

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = ncand / (ms_step * 1e-3)

    # ---- per-kernel timing with events on the library's stream (torch's current stream)
    def ev_time(fn, reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        fn()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    reps = args.sweep_reps
    def smooth_fn(sweeps):
        if gs:
            return S.sfg_smooth_gs(H, classes, x0, sweeps, omega, storage=wdt, out=X, ws=ws_sm)
        return S.sfg_smooth(H, x0, sweeps, omega, storage=wdt, out=X, ws=ws_sm)

    t_smooth = ev_time(lambda: smooth_fn(T), reps)
    t_one = ev_time(lambda: smooth_fn(1), reps)
    smooth_fn(T)
    # the first sweep also centres (reads the FP64 block); the other T-1 are plain sweeps
    t_sweep = (t_smooth - t_one) / (T - 1)
    # attainable bandwidth on this machine: a plain device copy of 1 GiB
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    t_copy = ev_time(lambda: dst.copy_(src), 5)
    copy_gbs = 2 * src.numel() * 8 / (t_copy * 1e-3) / 1e9
    del src, dst
    t_score = ev_time(lambda: S.sfg_edge_scores(X, u, v, w, cand=cand, out=score), reps)
    t_select = ev_time(lambda: S.sfg_select_topk(score, ksel, sel=sel, tau=tau, ws=ws_sel, sync=False), reps)
    t_csr = ev_time(lambda: S.sfg_laplacian_csr(g.n, u, v, w, mask=tree, ws=ws_csr, out=H, nnz=nnz), reps)

    bsw = sweep_bytes(g.n, nnz, k, sx, sw)
    bsc = score_bytes(ncand, g.n, k, sx, sw, sx)
    # The library sweeps an FP64 block of >= 16 vectors on a tree-like graph in
    # 8-column parts (one launch per part and sweep), so a launch moves its
    # part of X and the whole tree CSR.
    parts = k // 8 if (f64 and k >= 16 and k % 8 == 0 and nnz <= 3 * g.n and not gs) else 1
    b_launch = sweep_bytes(g.n, nnz, k // parts, sx, sw)
    t_launch = t_sweep / parts
    achieved = b_launch / (t_launch * 1e-3) / 1e9
    smoothing_gbs = bsw / (t_sweep * 1e-3) / 1e9

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        ent = tr.get(args.dtype)
        if ent and ent.get("src_hash") == src_hash(SWEEP_SRC) and not gs:
            traffic = ent["hbm_bytes_per_launch"]

    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": (f"k_sweep_color (one Gauss-Seidel sweep: {classes[3]} colour classes of the tree, in place)"
                           if gs else
                           "k_sweep (one damped-Jacobi sweep of an 8-vector column part of the block on the tree)"
                           if parts > 1 else "k_sweep (one damped-Jacobi sweep of the 16-vector block on the tree)"),
                "algorithmic_bytes_per_launch": b_launch, "avg_launch_us": round(t_launch * 1e3, 2),
                "launches_per_sweep": classes[3] if gs else parts,
                # the smoothing rate with the graph counted once per sweep of the whole block
                "smoothing_gbs": round(smoothing_gbs, 1), "smoothing_frac": round(smoothing_gbs / HBM_PEAK_GBS, 4)}

    # ---- CPU baseline: the oracle on one full step of the same workload
    cpu = None if args.no_cpu_baseline else cpu_baseline(g, tree, cand, X0, k, T, omega, ksel, f64, gs)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "powergrid1000x1000+2%diag", "nodes": g.n, "edges": g.m, "off_tree_edges": ncand,
                   "k_sel": ksel, "vectors": k, "sweeps": T, "omega": omega, "embed": "spanning tree",
                   "smoother": "multicolour Gauss-Seidel" if gs else "damped Jacobi", "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "copy_gbs": round(copy_gbs, 1),
        "stages_ms": {"csr": round(t_csr, 4), "smooth": round(t_smooth, 4), "smooth_1sweep": round(t_one, 4),
                      "sweep": round(t_sweep, 4), "score": round(t_score, 4), "select": round(t_select, 4)},
        "edges_scored_per_s_score_kernel": round(ncand / (t_score * 1e-3), 1),
        "score_gbs": round(bsc / (t_score * 1e-3) / 1e9, 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
