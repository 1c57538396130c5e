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
