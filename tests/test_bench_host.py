"""Host-side logic of the benchmark (CPU): the single-GPU contract, the
algorithmic operation count and the profile bookkeeping."""
import json
import math
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2110_03214_amd import synth  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "single-GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_ops_count_every_search_tree_node():
    """4 ops per node at depths 1..k of each query's tree: F!/(F-p)! nodes at
    depth p; the leaves are the embeddings."""
    W = np.ones((6, 6), np.uint8) - np.eye(6, dtype=np.uint8)
    q = synth.make_queries([0, 1, 1], [0, 1, 2], [3, 6, 7])
    wl = synth.Workload("t", [W], np.zeros(2, np.int32), np.array([0, 0b11], np.uint32), q)
    emb, ops = bench.algorithmic_ops(wl)
    # server 0: F = 6, k = 3; server 1: F = 4, k = 6 and 7 do not fit
    assert emb == math.perm(6, 3)
    assert ops == 4 * (6 + 30 + 120)


def test_profiles_match_the_sources_they_were_taken_on():
    """Every committed counter profile names the kernel sources it measured;
    the benchmark reports its HBM bytes only while they still hash the same."""
    for cfg, name in bench.PMC_PROFILE.items():
        path = os.path.join(ROOT, "profiles", name)
        assert os.path.exists(path), name
        text = open(path).read()
        assert "kernel_source_sha256:" in text and "command" in text
        traffic, source = bench.profiled_traffic(cfg)
        if traffic is not None:
            assert traffic > 0 and source == f"profiles/{name}"
