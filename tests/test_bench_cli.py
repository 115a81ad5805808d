"""The benchmark's command line, without a GPU: a request for more than one
GPU is refused with a message before anything touches a device, and every
workload the benchmark names is one the workload table defines."""
import os
import subprocess
import sys

from paper_1503_02368_amd.workloads import WORKLOADS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.lstrip().startswith("{")


def test_headline_workloads_are_defined():
    for name in ("rmat20_triangles", "rmat18_4cliques", "batch_triangles", "served"):
        assert name in WORKLOADS, name
