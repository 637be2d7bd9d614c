"""Host-side logic of the benchmark (CPU): the single-GPU contract, the
algorithmic operation count and the profile bookkeeping."""
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2110_03214_amd import synth  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "single-GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_operation_counts_of_the_three_models():
    """Per-leaf model: (8 + 3B + |Nb[k-1]|) per embedding times 1 + 1/(F-k+1);
    factored model: 3 per embedding + 4 per interior node at depths 1..k-1;
    node model: 4 per node at depths 1..k.  F!/(F-p)! nodes at depth p."""
    W = np.ones((6, 6), np.uint8) - np.eye(6, dtype=np.uint8)  # B = 1
    q = synth.make_queries([0, 1, 1, 0], [0, 1, 2, 1], [3, 6, 7, 2])
    wl = synth.Workload("t", [W], np.zeros(2, np.int32), np.array([0, 0b11], np.uint32), q)
    ops = bench.op_counts(wl)
    # server 0: F = 6 (ring k=3, all-to-all k=2); server 1: F = 4, k = 6 and 7 do not fit
    assert ops["embeddings"] == math.perm(6, 3) + math.perm(6, 2)
    ring3 = math.perm(6, 3) * (8 + 3 + 2) * (1 + 1 / 4)
    a2a2 = math.perm(6, 2) * (8 + 3 + 1) * (1 + 1 / 5)
    assert ops["ops_leaf8d"] == pytest.approx(ring3 + a2a2)
    assert ops["ops_factored"] == 3 * (120 + 30) + 4 * (6 + 30) + 4 * 6
    assert ops["ops_node4"] == 4 * (6 + 30 + 120) + 4 * (6 + 30)
    # a weight of 3 needs two bit-planes
    assert bench.weight_bits(np.array([[0, 3], [3, 0]])) == 2
    assert [bench.last_back_neighbours(0, k) for k in (1, 2, 3, 8)] == [0, 1, 2, 2]
    assert [bench.last_back_neighbours(1, k) for k in (1, 2, 8)] == [0, 1, 7]
    assert [bench.last_back_neighbours(2, k) for k in (1, 2, 8)] == [0, 1, 1]


def test_large_sample_is_eight_topologies_with_all_their_queries():
    sample, topo = bench.large_sample()
    assert len(topo) == 8 and sample.nq == 48
    assert sorted(set(sample.queries["server"].tolist())) == topo
    assert sorted(sample.queries["k"].tolist()) == [6] * 16 + [7] * 16 + [8] * 16


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
