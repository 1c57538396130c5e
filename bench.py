"""Benchmark of the SF-GRASS hot path on one MI355X.

Default line: the 200^3 mesh workload (7-point mesh, 8,000,000 nodes,
23,880,000 edges, log-normal(0, 1.5) weights; K=16 vectors, T=20 sweeps,
f=10%).  One step = one full scoring pass in FP64: the CSR of the scoring
graph (the maximum-weight spanning tree), centring plus 20 damped-Jacobi sweeps
of the 16-vector block, scores of the 15,880,001 off-tree edges, selection of
the top 10%.  The edge list, random block, tree mask and candidate list are
resident in HBM before timing; the step allocates nothing and never
synchronises.  The same pass in FP32 (the storage the surrogate comparison
uses) is reported beside it, and the surrogate-versus-plain comparison at
equal condition number (Eq. 2) follows the timed part.

Prints one JSON line.  ``value`` is off-tree edges scored per second of the
whole step.  ``roofline`` is for the dominant kernel (the smoothing sweep):
algorithmic bytes of one launch over its average duration, timed with HIP
events on the stream the library launches on.

    python bench.py [--steps K] [--warmup W] [--dtype f64|f32] [--no-cpu-baseline] [--no-kappa]
    python bench.py --workload powergrid|knn|chunglu|surrogate|sigma|scaling|pcg
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
MALL_BYTES = 256 << 20            # memory-side (Infinity) cache of the MI355X
PART_BUDGET = 192 << 20           # the library sweeps 8-column parts whose working set fits this
SWEEP_SRC = os.path.join(ROOT, "paper_2008_07633_amd", "csrc", "smooth.hip")
HEADLINE = {
    "mesh": {"label": "mesh200x200x200 (7-point, log-normal(0,1.5) weights)",
             "traffic": os.path.join(ROOT, "profiles", "sweep_mesh200_traffic.json")},
    "powergrid": {"label": "powergrid1000x1000+2%diag",
                  "traffic": os.path.join(ROOT, "profiles", "sweep_powergrid1000_traffic.json")},
}


def sweep_bytes(n: int, nnz: int, k: int, sx: int, sw: int) -> int:
    """Algorithmic bytes of one sweep: rowptr, col+val, deg, read X_t, write X_t+1."""
    return 4 * (n + 1) + nnz * (4 + sw) + n * sw + 2 * n * k * sx


def score_bytes(ncand: int, n: int, k: int, sx: int, sw: int, ss: int) -> int:
    """Algorithmic bytes of the edge pass: cand id, u, v, w, score per candidate, X once."""
    return ncand * (4 + 8 + sw + ss) + n * k * sx


def sweep_parts(n: int, nnz: int, k: int, sx: int, sw: int, gs: bool) -> int:
    """Launches per sweep: the library's rule for sweeping an FP64 block in 8-column parts (a sparse
    graph whose whole working set exceeds the memory-side cache while an 8-column part's fits 192 MB)."""
    graph = 4 * (n + 1) + nnz * (4 + sw) + n * sw
    full, part = 2 * n * k * sx + graph, 2 * n * 8 * sx + graph
    if not gs and sx == 8 and k >= 16 and k % 8 == 0 and nnz <= 3 * n and full > MALL_BYTES and part <= PART_BUDGET:
        return k // 8
    return 1


def src_hash(path: str) -> str:
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, tree, cand, X0, k: int, T: int, omega: float, ksel: int, f64: bool, gs: bool) -> dict:
    """The oracle (plain C, FP64) timed on one full step of the same workload: on every host core it may
    use (OpenMP over the rows of each sweep and over the scored edges) and on one thread.  Each row and
    edge is one thread's work in a fixed order, so both give the same bits."""
    import oracle

    oracle.build(force=False)
    tmask = tree.cpu().numpy().astype(bool)
    cnp = cand.cpu().numpy()
    wnp = g.w if f64 else g.w.astype(np.float32).astype(np.float64)
    all_threads = oracle.max_threads()

    def one_step():
        c0 = time.perf_counter()
        Hc = oracle.laplacian_csr(g.n, g.u[tmask], g.v[tmask], wnp[tmask])
        Xc, _ = oracle.center(X0)
        if gs:
            cl, ncl = oracle.color(Hc)
            Xs = oracle.smooth_gs(Hc, Xc, T, omega, cl, ncl)
        else:
            Xs = oracle.smooth(Hc, Xc, T, omega)
        sc = oracle.edge_scores(Xs, g.u[cnp], g.v[cnp], wnp[cnp])
        pos, tau = oracle.select_topk(sc, cnp, ksel)
        return time.perf_counter() - c0, tau

    t_all, tau_all = one_step()
    oracle.set_threads(1)
    t_one, tau_one = one_step()
    oracle.set_threads(all_threads)
    assert tau_one == tau_all
    ncand = int(cnp.size)
    return {"value": round(ncand / t_all, 1), "unit": "edges/s", "cores": all_threads, "kind": "oracle",
            "sample": f"one full step of the same workload (tree CSR by qsort, exact centring, {T} sweeps of {k} "
                      f"FP64 vectors, {ncand} scores, top-{ksel} qsort): {t_all:.2f} s on {all_threads} threads "
                      f"(sweeps and scores split over rows and edges), {t_one:.2f} s on 1 thread",
            "value_1_thread": round(ncand / t_one, 1), "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kappa", action="store_true",
                    help="skip the surrogate-versus-plain comparison at equal condition number")
    ap.add_argument("--smoother", choices=["jacobi", "gs"], default="jacobi",
                    help="gs: multicolour Gauss-Seidel (omega 1; colouring of the tree prepared once, like the tree)")
    ap.add_argument("--sweep-reps", type=int, default=5)
    ap.add_argument("--single-sweep", action="store_true",
                    help="smooth one sweep per launch in node order (sfg_smooth) instead of two per launch in the "
                         "tree's preorder (sfg_smooth_ordered)")
    ap.add_argument("--workload", choices=["mesh", "powergrid", "knn", "chunglu", "surrogate", "sigma", "scaling",
                                           "pcg"], default="mesh",
                    help="mesh: the headline line; powergrid: the same pass on the 1M-node power grid; "
                         "the others print their own lines (bench_workloads.py)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2008_07633_amd import sfg as S

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    S.lib()
    import bench_workloads as BW

    if args.workload not in HEADLINE:
        BW.run(args)
        return
    print(json.dumps(headline(args, S, BW)), flush=True)


def scoring_pass(S, g, u, v, w64, tree, cand, x0, k, T, omega, ksel, wdt, gs, dev, order=None):
    """Preallocated buffers and the step function of one scoring pass in storage ``wdt``.  With ``order``
    (the spanning tree's preorder) the smoothing takes two sweeps per pass (sfg_smooth_ordered)."""
    import torch

    w = w64 if wdt == torch.float64 else w64.float()
    nnz = 2 * (g.n - 1)
    ncand = int(cand.numel())
    ws_csr = torch.empty(S.sfg_workspace_bytes(S.OP_LAPLACIAN_CSR, g.n, g.m, 0, wdt), dtype=torch.uint8, device=dev)
    ws_sm = torch.empty(S.sfg_workspace_bytes(S.OP_SMOOTH_ORDERED if order is not None else S.OP_SMOOTH, g.n, 0, k,
                                              wdt), dtype=torch.uint8, device=dev)
    ws_sel = torch.empty(S.sfg_workspace_bytes(S.OP_SELECT_TOPK, 0, ncand, 0, wdt), dtype=torch.uint8, device=dev)
    H = S.Csr(g.n, nnz, torch.empty(g.n + 1, dtype=torch.int32, device=dev),
              torch.empty(nnz, dtype=torch.int32, device=dev), torch.empty(nnz, dtype=wdt, device=dev),
              torch.empty(nnz, dtype=torch.int32, device=dev), torch.empty(g.n, dtype=wdt, device=dev))
    X = torch.empty((g.n, k), dtype=wdt, device=dev)
    score = torch.empty(ncand, dtype=wdt, device=dev)
    sel = torch.empty(ncand, dtype=torch.uint8, device=dev)
    tau = torch.empty(1, dtype=torch.float64, device=dev)
    classes = None
    if gs:
        S.sfg_laplacian_csr(g.n, u, v, w, mask=tree, ws=ws_csr, out=H, nnz=nnz)
        classes = S.sfg_color(H)

    def csr():
        S.sfg_laplacian_csr(g.n, u, v, w, mask=tree, ws=ws_csr, out=H, nnz=nnz)

    info = {}

    def smooth(sweeps=T):
        if gs:
            return S.sfg_smooth_gs(H, classes, x0, sweeps, omega, storage=wdt, out=X, ws=ws_sm)
        if order is not None:
            return S.sfg_smooth_ordered(H, order, x0, sweeps, omega, storage=wdt, out=X, ws=ws_sm, info=info)
        return S.sfg_smooth(H, x0, sweeps, omega, storage=wdt, out=X, ws=ws_sm)

    def scores():
        S.sfg_edge_scores(X, u, v, w, cand=cand, out=score)

    def select():
        S.sfg_select_topk(score, ksel, sel=sel, tau=tau, ws=ws_sel, sync=False)

    def step():
        csr()          # a1
        smooth()       # a2 + a3
        scores()       # a4
        select()       # a5

    return {"step": step, "csr": csr, "smooth": smooth, "scores": scores, "select": select, "H": H, "X": X,
            "sel": sel, "tau": tau, "classes": classes, "nnz": nnz, "info": info}


def timed_steps(torch, step, steps, warmup):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def headline(args, S, BW) -> dict:
    import torch

    import workloads as W

    name = args.workload
    prm = W.workload_params(name)
    k, T, frac, omega = prm["k"], prm["sweeps"], prm["frac"], 0.5
    g = BW.cached_graph(name)
    X0 = W.workload_block(name, g.n)
    f64 = args.dtype == "f64"
    wdt = torch.float64 if f64 else torch.float32
    sx = sw = 8 if f64 else 4
    dev = torch.device("cuda:0")
    u = torch.from_numpy(g.u).to(dev)
    v = torch.from_numpy(g.v).to(dev)
    w64 = torch.from_numpy(g.w).to(dev)
    x0 = torch.from_numpy(X0).to(dev)
    # input preparation, once per graph: spanning tree and off-tree candidate list
    tree, comps = S.sfg_spanning_tree(g.n, u, v, w64)
    assert comps == 1
    cand = torch.nonzero(tree == 0).reshape(-1).to(torch.int32)
    ncand = int(cand.numel())
    ksel = int(math.ceil(frac * ncand))
    gs = args.smoother == "gs"
    if gs:
        omega = 1.0
    # input preparation too: the tree's preorder, the row order of the two-sweeps-per-pass smoothing
    order = S.sfg_tree_order(g.n, u, v, w64, tree).order if not (args.single_sweep or gs) else None

    P = scoring_pass(S, g, u, v, w64, tree, cand, x0, k, T, omega, ksel, wdt, gs, dev, order)
    ms_step = timed_steps(torch, P["step"], args.steps, args.warmup)
    value = ncand / (ms_step * 1e-3)
    nnz = P["nnz"]

    reps = args.sweep_reps
    t_smooth = BW.ev_time(lambda: P["smooth"](T), reps)
    per_pass = int(P["info"].get("sweeps_per_pass", 1))
    fused = per_pass >= 2
    if fused:
        # a launch takes per_pass sweeps: a call of two passes is the same layout, the centring first pass and
        # one more, so the difference is the T - 2 per_pass sweeps of the remaining launches (a call of a single
        # pass would be too short to take the passes at all)
        t0_sweeps = 2 * per_pass
        t_one = BW.ev_time(lambda: P["smooth"](t0_sweeps), reps)
        assert int(P["info"].get("sweeps_per_pass", 1)) == per_pass, "the two-pass call did not take the passes"
        t_sweep = (t_smooth - t_one) / (T - t0_sweeps)
    else:
        t_one = BW.ev_time(lambda: P["smooth"](1), reps)
        # the first sweep also centres (reads the FP64 block); the other T-1 are plain sweeps
        t_sweep = (t_smooth - t_one) / (T - 1)
    P["smooth"](T)          # X holds the full pass again before the edge pass and selection are timed
    t_score = BW.ev_time(P["scores"], reps)
    t_select = BW.ev_time(P["select"], reps)
    t_csr = BW.ev_time(P["csr"], reps)
    copy = BW.copy_rates(dev)

    bsw = sweep_bytes(g.n, nnz, k, sx, sw)
    bsc = score_bytes(ncand, g.n, k, sx, sw, sx)
    parts = 1 if fused else sweep_parts(g.n, nnz, k, sx, sw, gs)
    # a launch of the fused kernel must move one sweep's bytes (the graph once, X_t in, X_t+2 out): X_t+1 stays
    # on chip.  Its roofline is taken against those bytes; the smoothing rate below counts B_sweep per sweep.
    b_launch = sweep_bytes(g.n, nnz, k // parts, sx, sw)
    t_launch = per_pass * t_sweep / parts
    achieved = b_launch / (t_launch * 1e-3) / 1e9
    smoothing_gbs = bsw / (t_sweep * 1e-3) / 1e9
    working_set = sweep_bytes(g.n, nnz, k // parts, sx, sw)
    # a launch whose working set fits the memory-side cache is not bound by HBM: compare it with the
    # measured copy rate of a buffer that stays in that cache
    in_cache = working_set <= MALL_BYTES
    bound, peak = ("cache", copy["in_cache_copy_gbs"]) if in_cache else ("hbm", HBM_PEAK_GBS)

    traffic = None
    tf = HEADLINE[name]["traffic"]
    if os.path.exists(tf) and not gs:
        ent = json.load(open(tf)).get(args.dtype + (f"_pass{per_pass}" if fused else ""))
        if ent and ent.get("src_hash") == src_hash(SWEEP_SRC):
            traffic = ent["hbm_bytes_per_launch"]
    if gs:
        kname = f"k_sweep_color (one Gauss-Seidel sweep: {P['classes'][3]} colour classes of the tree, in place)"
    elif fused:
        kname = (f"k_sweep_pass<{per_pass}> ({per_pass} damped-Jacobi sweeps of the {k}-vector block on the tree "
                 f"per launch, blocks of 64 rows of the tree's preorder with their {per_pass}-hop neighbourhoods in "
                 f"LDS; bytes: one sweep's)")
    elif parts > 1:
        kname = f"k_sweep (one damped-Jacobi sweep of an 8-vector column part of the {k}-vector block on the tree)"
    else:
        kname = f"k_sweep (one damped-Jacobi sweep of the {k}-vector block on the tree)"
    roofline = {"bound": bound, "achieved": round(achieved, 1), "peak": round(peak, 1), "unit": "GB/s",
                "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": kname,
                "algorithmic_bytes_per_launch": b_launch, "avg_launch_us": round(t_launch * 1e3, 2),
                "launches_per_sweep": P["classes"][3] if gs else (round(1 / per_pass, 4) if fused else parts),
                "working_set_bytes": working_set,
                # the smoothing rate of the metric: T B_sweep / t(T sweeps), the graph and X counted once per sweep;
                # with two sweeps per pass over X it can exceed the HBM peak (it is then the one-sweep-per-pass
                # roofline that is beaten)
                "smoothing_gbs": round(smoothing_gbs, 1), "smoothing_frac_of_hbm_peak":
                    round(smoothing_gbs / HBM_PEAK_GBS, 4)}

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
        "config": {"workload": HEADLINE[name]["label"], "nodes": g.n, "edges": g.m, "off_tree_edges": ncand,
                   "k_sel": ksel, "vectors": k, "sweeps": T, "omega": omega, "embed": "spanning tree",
                   "smoother": "multicolour Gauss-Seidel" if gs else "damped Jacobi", "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": None,
        "copy": copy,
        "stages_ms": {"csr": round(t_csr, 4), "smooth": round(t_smooth, 4),
                      (f"smooth_{2 * per_pass}sweeps" if fused else "smooth_1sweep"): round(t_one, 4),
                      "sweep": round(t_sweep, 4), "score": round(t_score, 4), "select": round(t_select, 4)},
        "edges_scored_per_s_score_kernel": round(ncand / (t_score * 1e-3), 1),
        "score_gbs": round(bsc / (t_score * 1e-3) / 1e9, 1),
    }
    sel_main = P["sel"].clone()
    del P
    torch.cuda.empty_cache()
    if order is not None:
        # the single-sweep kernel in node order, for comparison (the step above does not use it)
        P1 = scoring_pass(S, g, u, v, w64, tree, cand, x0, k, T, omega, ksel, wdt, gs, dev)
        P1["csr"]()
        t1T = BW.ev_time(lambda: P1["smooth"](T), reps)
        t11 = BW.ev_time(lambda: P1["smooth"](1), reps)
        ts1 = (t1T - t11) / (T - 1)
        out["single_sweep"] = {"us": round(ts1 * 1e3, 2), "gbs": round(bsw / (ts1 * 1e-3) / 1e9, 1),
                               "frac": round(bsw / (ts1 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "kernel": "k_sweep (one sweep per launch, node order)"}
        del P1
        torch.cuda.empty_cache()

    # the same pass in FP32 storage and arithmetic (the surrogate comparison's storage)
    if f64 and not gs:
        P32 = scoring_pass(S, g, u, v, w64, tree, cand, x0, k, T, omega, ksel, torch.float32, False, dev, order)
        ms32 = timed_steps(torch, P32["step"], args.steps, args.warmup)
        # P32["sel"] holds the selection of the last timed step, made before these smoothing timings
        pp32 = int(P32["info"].get("sweeps_per_pass", 1))
        if pp32 >= 2:
            t32 = (BW.ev_time(lambda: P32["smooth"](T), reps) - BW.ev_time(lambda: P32["smooth"](2 * pp32),
                                                                             reps)) / (T - 2 * pp32)
            assert int(P32["info"].get("sweeps_per_pass", 1)) == pp32, "the two-pass call did not take the passes"
        else:
            t32 = (BW.ev_time(lambda: P32["smooth"](T), reps) - BW.ev_time(lambda: P32["smooth"](1), reps)) / (T - 1)
        b32 = sweep_bytes(g.n, nnz, k, 4, 4)
        agree = float((P32["sel"].bool() & sel_main.bool()).sum().item()) / max(ksel, 1)
        out["f32"] = {"ms_per_step": round(ms32, 4), "value": round(ncand / (ms32 * 1e-3), 1),
                      "sweep_us": round(t32 * 1e3, 2), "sweep_gbs": round(b32 / (t32 * 1e-3) / 1e9, 1),
                      "sweep_frac_of_hbm_peak": round(b32 / (t32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "selection_agreement_with_f64": round(agree, 6)}
        del P32
        torch.cuda.empty_cache()

    if name == "mesh" and not args.no_kappa and not gs:
        out["equal_kappa"] = BW.equal_kappa_mesh(g, u, v, w64, tree, cand, dev)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, tree, cand, X0, k, T, omega, ksel, f64, gs)
    return out


if __name__ == "__main__":
    main()
