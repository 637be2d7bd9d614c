"""Serving loop on the GPU: every request answered in the continuously
batched mix equals the oracle's answer for that request alone, evaluated
against the busy mask the loop dispatched it with; the loop hands every
allocation back when it stops."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2110_03214_amd import binding as B
from paper_2110_03214_amd import synth

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    c = B.Context(0)
    yield c
    c.close()


def requests_from_trace(tr, ids, mode=0, a=1, b=1):
    r = np.zeros(tr.n, dtype=B.REQUEST_DTYPE)
    r["id"] = np.arange(tr.n)
    r["t_arrival"] = tr.t_arrival
    r["hold"] = tr.hold
    r["server"] = ids[tr.server]
    r["kind"], r["k"], r["mode"], r["a"], r["b"] = tr.kind, tr.k, mode, a, b
    return r


def drain(ctx, n):
    got = []
    total = 0
    import time
    t_end = time.time() + 120
    while total < n and time.time() < t_end:
        c = ctx.serve_poll()
        got.append(c)
        total += len(c)
        if not len(c):
            time.sleep(0.002)
    return np.concatenate(got) if got else np.zeros(0, B.COMPLETION_DTYPE)


def check_against_alone(tr, reqs, comp, max_leaves=2e7, ctx=None, ids=None):
    """Oracle answer of each request alone, on its server's topology with the
    busy mask it was dispatched with.  Requests of more than max_leaves
    embeddings are checked, when a context is given (the serving loop
    stopped), against a single-query GPU batch of that request alone on its
    server with that busy mask (the batch path, which the full large-config
    parity pins to the oracle).  Returns the number of requests checked."""
    order = np.argsort(comp["id"])
    comp = comp[order]
    assert np.array_equal(comp["id"], np.arange(len(reqs)))
    srv = tr.server  # trace server index == topology lookup
    n_of = np.array([tr.topologies[t].shape[0] for t in tr.server_topo[srv]])
    F = n_of - np.array([bin(int(x)).count("1") for x in comp["busy_before"]])
    leaves = np.array([math.perm(int(f), int(k)) if k <= f else 0 for f, k in zip(F, reqs["k"])])
    sel = np.nonzero(leaves <= max_leaves)[0]
    ref = oracle.batch(tr.topologies, tr.server_topo[srv[sel]], comp["busy_before"][sel],
                       reqs["kind"][sel], reqs["k"][sel], reqs["mode"][sel], reqs["a"][sel],
                       reqs["b"][sel], NTHREADS)
    got = comp[sel]
    assert np.array_equal(got["count"], ref["count"])
    assert np.array_equal(got["status"], ref["status"])
    ok = ref["status"] == 0
    for f in ("key", "agg", "pres", "vertex_mask"):
        assert np.array_equal(got[f][ok], ref[f][ok]), f
    for kk in range(1, 9):
        m = ok & (reqs["k"][sel] == kk)
        assert np.array_equal(got["mapping"][m, :kk], ref["mapping"][m, :kk])
    # every granted request is committed, every other is not
    assert ((got["alloc_handle"] >= 0) == ok).all()
    checked = len(sel)
    big = np.nonzero(leaves > max_leaves)[0]
    if ctx is not None and len(big):
        for i in big:
            sid = int(ids[srv[i]])
            ctx.set_busy([sid], [int(comp["busy_before"][i])])
            q = B.pack_queries([sid], [reqs["kind"][i]], [reqs["k"][i]], reqs["mode"][i], 0,
                               reqs["a"][i], reqs["b"][i])
            r = ctx.query_batch(q)[0]
            c = comp[i]
            for f in ("count", "status"):
                assert int(r[f]) == int(c[f]), (i, f)
            assert c["status"] == 0 and c["alloc_handle"] >= 0
            for f in ("key", "agg", "pres", "vertex_mask"):
                assert int(r[f]) == int(c[f]), (i, f)
            kk = int(reqs["k"][i])
            assert np.array_equal(r["mapping"][:kk], c["mapping"][:kk]), i
            checked += 1
        ctx.set_busy(ids, np.zeros(len(ids), np.uint32))
    return checked


def test_serving_mix_equals_alone_batched_config_servers(ctx):
    tr = synth.config4(30000)
    ids = ctx.load_servers(tr.topologies, tr.server_topo)
    reqs = requests_from_trace(tr, ids)
    ctx.serve_start(max_batch=2048, inflight=2, time_unit_us=40.0)
    ctx.serve_submit(reqs)
    comp = drain(ctx, tr.n)
    st = ctx.serve_stop()
    assert len(comp) == tr.n and st["completed"] == tr.n
    assert st["batches"] > 10 and st["mean_batch"] > 1
    assert st["granted"] + st["nofit"] == tr.n
    checked = check_against_alone(tr, reqs, comp)
    assert checked == tr.n
    # the loop released everything it granted
    assert (ctx.get_busy(ids) == 0).all()


def test_serving_mixed_sizes_admission_and_release(ctx):
    tr = synth.config5(6000)
    ids = ctx.load_servers(tr.topologies, tr.server_topo)
    reqs = requests_from_trace(tr, ids)
    # small admission budget: big 16-vertex requests must wait their turn
    ctx.serve_start(max_batch=512, inflight=2, time_unit_us=20.0, admission_items=200000,
                    item_leaves=4096)
    ctx.serve_submit(reqs)
    comp = drain(ctx, tr.n)
    st = ctx.serve_stop()
    assert len(comp) == tr.n and st["completed"] == tr.n
    assert (ctx.get_busy(ids) == 0).all()
    checked = check_against_alone(tr, reqs, comp, max_leaves=2e7, ctx=ctx, ids=ids)
    assert checked == tr.n


def test_serving_as_fast_as_possible_and_restart(ctx):
    tr = synth.config4(5000)
    ids = ctx.load_servers(tr.topologies, tr.server_topo)
    reqs = requests_from_trace(tr, ids)
    for _ in range(2):
        ctx.serve_start(max_batch=4096, inflight=1, time_unit_us=0.0)
        ctx.serve_submit(reqs)
        comp = drain(ctx, tr.n)
        ctx.serve_stop()
        assert len(comp) == tr.n
        check_against_alone(tr, reqs, comp)
        assert (ctx.get_busy(ids) == 0).all()
