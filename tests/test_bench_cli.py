"""bench.py's command line: it measures one GPU and says so for more; its
oracle leg; and (GPU) the one JSON line of a short run with the contract's fields."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(args, env_extra=None, timeout=120):
    env = dict(os.environ, **(env_extra or {}))
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                          env=env, timeout=timeout, cwd=ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_world_size_above_one_exits_with_a_message():
    r = run([], {"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_workloads():
    r = run(["--help"])
    assert r.returncode == 0
    for w in ("mesh", "powergrid", "knn", "chunglu", "surrogate", "sigma", "scaling", "pcg"):
        assert w in r.stdout


def test_cpu_baseline_leg_on_a_tiny_graph():
    # the oracle leg of the bench, on CPU tensors: the contract's fields and a sample that names what ran
    import math

    import numpy as np
    import torch

    import bench
    import oracle
    import workloads as W

    g = W.grid2d(12, 13, seed=3)
    tree = torch.from_numpy((oracle.max_spanning_forest(g.n, g.u, g.v, g.w)[0] > 0).astype(np.uint8))
    cand = torch.nonzero(tree == 0).reshape(-1).to(torch.int32)
    X0 = W.random_block(g.n, 4, 5)
    ksel = int(math.ceil(0.1 * cand.numel()))
    r = bench.cpu_baseline(g, tree, cand, X0, 4, 3, 0.5, ksel, True, False)
    assert r["kind"] == "oracle" and r["cores"] == oracle.max_threads() and r["unit"] == "edges/s"
    assert r["value"] > 0 and r["value_1_thread"] > 0 and r["cpu_model"]
    assert f"3 sweeps of 4 FP64 vectors, {cand.numel()} scores, top-{ksel}" in r["sample"]


@pytest.mark.gpu
def test_bench_json_line_on_the_gpu():
    # a short run of the default workload in a child process: one JSON line with the contract's fields
    import json

    import torch

    if torch.cuda.device_count() == 0:   # counts devices without initialising the runtime in this process
        pytest.skip("no GPU")
    r = run(["--steps", "2", "--warmup", "1", "--no-cpu-baseline", "--no-kappa", "--sweep-reps", "2"], timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1 and d["higher_is_better"] is True
    assert d["dtype"] == "f64" and d["data"] == "synthetic" and d["cpu_baseline"] is None
    assert d["config"]["workload"].startswith("mesh200x200x200")
    assert d["value"] > 0 and abs(d["value"] * d["ms_per_step"] * 1e-3 - d["config"]["off_tree_edges"]) < 1e-3 * d[
        "config"]["off_tree_edges"]
    roof = d["roofline"]
    # the FP64 tree sweep of the 8M-node mesh moves 2.3 GB: far beyond the memory-side cache
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    # several sweeps per launch in the tree's preorder (k_sweep_pass; one sweep's bytes a launch)
    assert roof["working_set_bytes"] > 256 << 20 and roof["launches_per_sweep"] in (0.25, 0.3333, 0.5)
    assert 0 < roof["frac"] <= 1 and abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    assert "f32" in d and d["f32"]["selection_agreement_with_f64"] > 0.99


@pytest.mark.gpu
def test_bench_power_grid_lines_name_their_bound():
    # several sweeps per launch (the default): X in and out of a launch and the graph, 292 MB, exceed the
    # memory-side cache, so the launch is priced against the HBM peak.  One sweep per launch: the pass sweeps
    # 8-column parts whose working set fits that cache, and its rate is compared with an in-cache copy instead.
    import json

    import torch

    if torch.cuda.device_count() == 0:
        pytest.skip("no GPU")
    for extra, bound, lps in (([], "hbm", (0.25, 0.3333, 0.5)), (["--single-sweep"], "cache", (2,))):
        r = run(["--workload", "powergrid", "--steps", "2", "--warmup", "1", "--no-cpu-baseline", "--sweep-reps",
                 "2"] + extra, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        d = json.loads([ln for ln in r.stdout.splitlines() if ln.strip()][-1])
        roof = d["roofline"]
        assert d["config"]["workload"].startswith("powergrid1000x1000")
        assert roof["bound"] == bound and roof["launches_per_sweep"] in lps, (extra, roof)
        if bound == "cache":
            assert roof["working_set_bytes"] <= 256 << 20 and roof["peak"] == d["copy"]["in_cache_copy_gbs"]
        else:
            assert roof["working_set_bytes"] > 256 << 20 and roof["peak"] == 8000.0
        assert 0 < roof["frac"] <= 1
