"""Seeded generator: determinism and the workload statistics the configs are
defined by (sizes, NOFIT fraction, embedding totals)."""
import math

import numpy as np

from paper_2110_03214_amd import synth


def _free(n, busy):
    return n - bin(int(busy)).count("1")


def test_determinism():
    a, b = synth.config2(4096), synth.config2(4096)
    for key in a.queries:
        assert np.array_equal(a.queries[key], b.queries[key])
    assert np.array_equal(a.busy, b.busy) and np.array_equal(a.server_topo, b.server_topo)
    for x, y in zip(synth.config3_topologies(8), synth.config3_topologies(8)):
        assert np.array_equal(x, y)
    t1, t2 = synth.config4(5000), synth.config4(5000)
    assert np.array_equal(t1.t_arrival, t2.t_arrival) and np.array_equal(t1.k, t2.k)


def test_topologies_well_formed():
    topos = synth.config2_topologies() + synth.config3_topologies(16) + synth.config1().topologies
    for W in topos:
        assert W.dtype == np.uint8 and (W == W.T).all() and (np.diag(W) == 0).all()
    t0, t1, t2 = synth.config2_topologies()
    assert (t0 > 0).sum() == 32 and set(np.unique(t0)) == {0, 1}
    assert (t1 == 2).sum() == 16 and (t1 == 1).sum() == 16
    assert t2.shape == (6, 6) and (t2 == 2).sum() == 12 and (t2 == 1).sum() == 6
    for W in synth.config3_topologies(32):
        hyper = [(u, v) for u in range(16) for v in range(16) if bin(u ^ v).count("1") == 1]
        assert all(1 <= W[u, v] <= 3 for u, v in hyper)
        off = (W > 0).sum() // 2 - 32
        assert off == 8


def test_config1_shape():
    wl = synth.config1()
    assert wl.nq == 1000 and len(wl.topologies) == 1
    nb = np.array([bin(int(b)).count("1") for b in wl.busy])
    assert nb.min() == 0 and nb.max() == 4
    assert set(wl.queries["k"]) == {4} and set(wl.queries["kind"]) == {synth.RING}


def test_config2_statistics():
    wl = synth.config2()
    assert wl.nq == 65536
    n = np.array([wl.topologies[t].shape[0] for t in wl.server_topo])
    F = np.array([_free(nn, b) for nn, b in zip(n, wl.busy)])
    k = wl.queries["k"].astype(int)
    nofit = (k > F).mean()
    assert abs(nofit - 0.517) < 0.01
    emb = np.array([math.perm(int(f), int(kk)) if kk <= f else 0 for f, kk in zip(F, k)])
    assert abs(emb.mean() / 1725.1 - 1) < 0.03


def test_config3_totals():
    wl = synth.config3()
    assert wl.nq == 1536
    total = sum(math.perm(16, int(k)) for k in wl.queries["k"])
    assert total == 256 * 2 * (math.perm(16, 6) + math.perm(16, 7) + math.perm(16, 8))
    assert abs(total / 2.98e11 - 1) < 0.01


def test_serving_traces():
    t4 = synth.config4(20000)
    assert (np.diff(t4.t_arrival) >= 0).all()
    rate = t4.n / t4.t_arrival[-1]
    assert abs(rate / 46.0 - 1) < 0.05
    pk = np.bincount(t4.k, minlength=9)[1:] / t4.n
    assert abs(pk[1] / pk[0] - 4) < 0.5 and abs(pk[7] / pk[0] - 4) < 0.5
    t5 = synth.config5(20000)
    assert (np.diff(t5.t_arrival) >= 0).all() and t5.k.max() == 8 and t5.k.min() == 1
    assert len(t5.topologies) == 257 and t5.server_topo.shape == (2048,)
