"""The autotuner (mapa_autotune) and the cached tunings it produced: results
never depend on the launch settings, so every candidate the tuner times and
every cached setting must return exactly the default setting's results."""
import numpy as np
import pytest

import oracle
from paper_2110_03214_amd import binding as B
from paper_2110_03214_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    c = B.Context(0)
    yield c
    c.close()


def test_autotune_keeps_the_fastest_and_changes_no_result(ctx):
    wl = synth.config2(8192)
    q, ids = B.load_workload(ctx, wl)
    ref = ctx.query_batch(q)
    best, trials = ctx.autotune(q, reps=1)
    assert len(trials) >= 10
    assert ctx.tuning().as_dict() == best
    assert min(ms for _, ms in trials) > 0
    assert np.array_equal(ctx.query_batch(q), ref)
    assert np.array_equal(ctx.get_busy(ids), wl.busy)  # the tuning runs commit nothing


def test_every_cached_tuning_gives_identical_results(ctx):
    cache = B.load_tuning_cache()
    big = synth.config3(8)   # 8 sixteen-vertex topologies, k = 6..8
    big = big.subset(np.nonzero(big.queries["k"] < 8)[0])
    small = synth.config2(4096)
    qs, _ = B.load_workload(ctx, small)
    qb, _ = B.load_workload(ctx, big)
    qe = qs.copy()
    qe["metric"] = B.METRIC_EFFBW  # the batched topologies weigh 0..2
    ref_s, ref_b = ctx.query_batch(qs, pipeline=True), ctx.query_batch(qb)
    ref_e = ctx.query_batch(qe, pipeline=True)
    for key, entry in sorted(cache.items()):
        print(f"[autotune] cached {key}: {entry['tuning']}", flush=True)
        ctx.set_tuning(**entry["tuning"])
        assert np.array_equal(ctx.query_batch(qs, pipeline=True), ref_s), key
        assert np.array_equal(ctx.query_batch(qb), ref_b), key
        assert np.array_equal(ctx.query_batch(qe, pipeline=True), ref_e), key
    k = big.queries["k"]
    sel = np.nonzero(k == 6)[0]
    ref = oracle.run_workload(big.subset(sel), 16)
    for f in ("count", "key", "agg", "pres", "vertex_mask"):
        assert np.array_equal(ref_b[f][sel], ref[f]), f
