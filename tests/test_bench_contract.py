"""The benchmark's command-line contract that needs no GPU: more than one GPU
is refused with exit status 2 and a message, before anything touches a
device; every workload name parses."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("workload", ["metric", "plain", "batching", "serve", "divergent", "stack", "inference", "schemes",
                                      "objects", "noops"])
def test_workloads_parse(workload, monkeypatch):
    import bench
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", workload])
    args = bench.parse()
    assert args.workload == workload and args.gpus == 1



def test_default_workload_is_the_metric():
    import bench
    sys.argv = ["bench.py"]
    args = bench.parse()
    assert args.workload == "metric" and args.gpus == 1


@pytest.mark.parametrize("k,cap,g", [(20, 4, 4), (600, 16, 15), (1000, 16, 10), (7, 4, 1), (3, 16, 3), (64, 16, 16)])
def test_graph_length_divides_the_steps(k, cap, g):
    """Captured graphs cover exactly the requested steps."""
    import bench
    assert bench.graph_len(k, cap) == g and k % g == 0
