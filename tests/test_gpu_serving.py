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


def test_serving_wide_requests_mix_equals_alone(ctx):
    """Requests the batch path does not take (32- and 24-vertex servers, and
    k = 9..10 on a 16-vertex server) are served in the same loop as 8-vertex
    ones: every completion equals that request alone against its busy mask
    (the oracle up to 2e6 embeddings, above that a wide call of the request
    alone, which the wide parity tests pin to the oracle); a request beyond
    the wide kernels' embedding limit is refused on the host; Eq. 2 requests
    ride along on the servers of weights 0..2; the loop hands back
    everything it granted."""
    rng = np.random.default_rng(41)

    def rand_topo(n, wmax, p):
        W = np.zeros((n, n), np.uint8)
        for u in range(n):
            for v in range(u + 1, n):
                if rng.random() < p:
                    W[u, v] = W[v, u] = rng.integers(1, wmax + 1)
        return W

    topos = [rand_topo(8, 2, 0.7), rand_topo(16, 3, 0.5), rand_topo(24, 3, 0.4), rand_topo(32, 2, 0.3)]
    st = np.array([0, 0, 0, 1, 2, 2, 3, 3, 3], np.int32)
    ids = ctx.load_servers(topos, st)
    # wide servers start mostly busy (kept busy throughout), so k = 9..11 stays small
    base = np.zeros(len(st), np.uint32)
    for s, keep_free in ((3, 12), (4, 12), (5, 11), (6, 12), (7, 13), (8, 32)):
        n = topos[st[s]].shape[0]
        free = rng.choice(n, size=keep_free, replace=False)
        base[s] = ((1 << n) - 1) & ~int(np.bitwise_or.reduce(1 << free.astype(np.int64)))
    ctx.set_busy(ids, base)
    nreq = 700
    srv = rng.integers(0, len(st) - 1, size=nreq)  # the all-free 32-vertex server only below
    k = np.where(st[srv] == 0, rng.integers(1, 9, size=nreq),
                 np.where(st[srv] == 1, rng.integers(6, 11, size=nreq), rng.integers(2, 12, size=nreq)))
    r = np.zeros(nreq + 1, dtype=B.REQUEST_DTYPE)
    r["id"] = np.arange(nreq + 1)
    r["t_arrival"][:nreq] = np.cumsum(rng.exponential(1.0, size=nreq))
    r["t_arrival"][nreq] = r["t_arrival"][nreq - 1]
    r["hold"][:nreq] = rng.exponential(6.0, size=nreq)
    r["server"][:nreq] = ids[srv]
    r["kind"][:nreq] = rng.integers(0, 3, size=nreq)
    r["k"][:nreq] = k
    r["mode"][:nreq] = rng.random(nreq) < 0.3
    r["a"], r["b"] = 1, 1
    # Eq. 2 on the servers whose links weigh 0..2 (8- and 32-vertex)
    r["metric"][:nreq] = np.isin(st[srv], (0, 3)) & (rng.random(nreq) < 0.4)
    # 12 of the 32 free accelerators: 32!/20! embeddings, past the wide limit
    r["server"][nreq], r["kind"][nreq], r["k"][nreq], r["hold"][nreq] = ids[8], 1, 12, 1.0
    ctx.serve_start(max_batch=64, inflight=2, time_unit_us=300.0)
    ctx.serve_submit(r)
    comp = drain(ctx, nreq + 1)
    st_ = ctx.serve_stop()
    assert len(comp) == nreq + 1 and st_["completed"] == nreq + 1
    assert np.array_equal(ctx.get_busy(ids), base)
    comp = comp[np.argsort(comp["id"])]
    assert comp["status"][nreq] == B.RES_REFUSED and comp["alloc_handle"][nreq] == -1
    comp, r = comp[:nreq], r[:nreq]
    tsel = st[srv]
    n_of = np.array([topos[t].shape[0] for t in tsel])
    F = n_of - np.array([bin(int(x)).count("1") for x in comp["busy_before"]])
    leaves = np.array([math.perm(int(f), int(kk)) if kk <= f else 0 for f, kk in zip(F, k)])
    small = leaves <= 2e6
    sel = np.nonzero(small)[0]
    ref = oracle.batch(topos, tsel[sel], comp["busy_before"][sel], r["kind"][sel], r["k"][sel],
                       r["mode"][sel], r["a"][sel], r["b"][sel], NTHREADS, metric=r["metric"][sel])
    got = comp[sel]
    for f in ("count", "status"):
        assert np.array_equal(got[f], ref[f]), f
    ok = ref["status"] == 0
    for f in ("key", "agg", "pres", "vertex_mask"):
        assert np.array_equal(got[f][ok], ref[f][ok]), f
    for kk in range(1, 13):
        m = ok & (r["k"][sel] == kk)
        assert np.array_equal(got["mapping"][m, :kk], ref["mapping"][m, :kk]), kk
        assert (got["mapping"][m, kk:] == 0xFF).all()
    assert ((got["alloc_handle"] >= 0) == ok).all()
    big = np.nonzero(~small)[0]
    for i in big:
        sid = int(r["server"][i])
        ctx.set_busy([sid], [int(comp["busy_before"][i])])
        q = B.pack_queries([sid], [r["kind"][i]], [r["k"][i]], r["mode"][i], 0, 1, 1, r["metric"][i])
        alone = ctx.query_batch_wide(q)[0]
        c = comp[i]
        for f in ("count", "status", "key", "agg", "pres", "vertex_mask"):
            assert int(alone[f]) == int(c[f]), (i, f)
        assert np.array_equal(alone["mapping"], c["mapping"]), i
    ctx.set_busy(ids, base)
    wide = (tsel > 0) | (k > 8)
    assert (wide & (comp["status"] == B.RES_OK)).sum() > 100
    assert (k[comp["status"] == B.RES_OK] >= 9).any()
    assert (wide & (r["metric"] == 1) & (comp["status"] == B.RES_OK)).sum() > 20
