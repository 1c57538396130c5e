"""bench.py's command line: it measures one GPU, and says so for more (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(args, env_extra=None):
    env = dict(os.environ, **(env_extra or {}))
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                          env=env, timeout=120, cwd=ROOT)


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
    for w in ("powergrid", "knn", "chunglu", "mesh", "sigma", "scaling", "pcg"):
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
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "edges/s" and r["value"] > 0
    assert f"3 sweeps of 4 FP64 vectors, {cand.numel()} scores, top-{ksel}" in r["sample"]
