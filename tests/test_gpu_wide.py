"""GPU parity for the wide path (mapa_query_batch_wide): servers of 17..32
accelerators and patterns of 9..12 vertices against the oracle bit for bit,
the batch path's answers on servers both paths take, the five-cube's hand
counts, registered patterns, the batch commit rule, the device-pointer form
against the host form, and the embedding limit."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2110_03214_amd import binding as B
from paper_2110_03214_amd import synth

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return t


@pytest.fixture
def ctx(torch):
    c = B.Context(0)
    yield c
    c.close()


def assert_same(gpu, ref, k, label=""):
    k = np.asarray(k)
    for f in ("count", "status"):
        bad = np.nonzero(gpu[f] != ref[f])[0]
        assert bad.size == 0, f"{label} {f} differs at {bad[:5]}: gpu {gpu[f][bad[:5]]} ref {ref[f][bad[:5]]}"
    ok = ref["status"] == 0
    for f in ("key", "agg", "pres", "vertex_mask", "links"):
        bad = np.nonzero(ok & (gpu[f] != ref[f]))[0]
        assert bad.size == 0, f"{label} {f} differs at {bad[:5]}: gpu {gpu[f][bad[:5]]} ref {ref[f][bad[:5]]}"
    for kk in np.unique(k):
        sel = ok & (k == kk)
        assert np.array_equal(gpu["mapping"][sel, :kk], ref["mapping"][sel, :kk]), f"{label} mapping k={kk}"
        assert (gpu["mapping"][sel, kk:] == 0xFF).all()


def random_topology(rng, n, wmax, p_edge):
    W = np.zeros((n, n), np.uint8)
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p_edge:
                W[u, v] = W[v, u] = rng.integers(1, wmax + 1)
    return W


def busy_leaving(rng, n, F):
    free = rng.choice(n, size=F, replace=False)
    return int(((1 << n) - 1) & ~int(np.bitwise_or.reduce(1 << free.astype(np.int64))))


def run_wide(ctx, topos, st, busy, cols, edges=None, metric=0):
    q = synth.make_queries(cols["server"], cols["kind"], cols["k"], cols["mode"], cols.get("commit", 0),
                           cols["a"], cols["b"], metric)
    wl = synth.Workload("wide", topos, np.array(st, np.int32), np.array(busy, np.uint32), q)
    qh, ids = B.load_workload(ctx, wl)
    got = ctx.query_batch_wide(qh)
    srv = wl.queries["server"]
    ref = oracle.batch(topos, wl.server_topo[srv], wl.busy[srv], q["kind"], q["k"], q["mode"], q["a"],
                       q["b"], NTHREADS, metric=q["metric"], edges=edges)
    return got, ref, qh


@pytest.mark.parametrize("wmax", [3, 255])
def test_wide_servers_against_oracle(ctx, wmax):
    """Servers of 17..32 accelerators with 2..11 free, every kind, k = 1..12,
    both modes, several keys; one call."""
    rng = np.random.default_rng(900 + wmax)
    topos = [random_topology(rng, n, wmax, 0.5) for n in (17, 20, 24, 32)]
    st, busy, cols = [], [], {c: [] for c in ("server", "kind", "k", "mode", "a", "b")}
    s = 0
    for t, W in enumerate(topos):
        n = W.shape[0]
        for F in (2, 5, 8, 11):
            st.append(t)
            busy.append(busy_leaving(rng, n, F))
            limit = 2_000_000 if n <= 20 else 20_000  # the oracle memoises PreservedBW up to n = 20
            for kind in range(3):
                for k in range(1, 13):
                    if k <= F and math.perm(F, k) > limit:
                        continue
                    for mode in (0, 1):
                        a, b = [(1, 1), (1, 0), (0, 1), (1024, 3)][int(rng.integers(0, 4))]
                        for c, v in zip(cols, (s, kind, k, mode, a, b)):
                            cols[c].append(v)
            s += 1
    got, ref, qh = run_wide(ctx, topos, st, busy, cols)
    assert_same(got, ref, qh["k"], "wide")
    assert (ref["status"] == 0).sum() > 100
    assert ctx.stats()["self_check_failures"] == 0


def test_wide_effbw_against_oracle(ctx):
    """Eq. 2 on the wide path: servers of 17..32 accelerators whose links
    are PCIe (0), single (1) or double NVLinks (2), every kind, k = 1..12
    (up to 66 pattern edges), both modes; key round(1000 * EffBW), the link
    mix and the mapping of the first best placement, as the oracle."""
    rng = np.random.default_rng(2)
    topos = [random_topology(rng, n, 2, p) for n, p in ((17, 0.6), (24, 0.9), (32, 0.5))]
    st, busy, cols = [], [], {c: [] for c in ("server", "kind", "k", "mode", "a", "b")}
    s = 0
    for t, W in enumerate(topos):
        n = W.shape[0]
        for F in (4, 10, 12):
            st.append(t)
            busy.append(busy_leaving(rng, n, F))
            limit = 2_000_000 if n <= 20 else 50_000
            for kind in range(3):
                for k in range(1, 13):
                    # k = F = 10 stays on the 17-vertex server (10! embeddings)
                    if k <= F and math.perm(F, k) > limit and not (k == F == 10 and n <= 20):
                        continue
                    for mode in (0, 1):
                        for c, v in zip(cols, (s, kind, k, mode, 1, 1)):
                            cols[c].append(v)
            s += 1
    got, ref, qh = run_wide(ctx, topos, st, busy, cols, metric=1)
    assert_same(got, ref, qh["k"], "wide effbw")
    ok = ref["status"] == 0
    assert ok.sum() > 80 and (qh["k"][ok] >= 9).any()
    assert ctx.stats()["self_check_failures"] == 0


def test_wide_effbw_equals_batch_path(ctx):
    """Eq. 2 queries on servers both paths take (cube-mesh 8-GPU graphs of
    weights 0..2, k <= 8) answer identically on the wide and batch calls."""
    rng = np.random.default_rng(3)
    topos = [random_topology(rng, n, 2, 0.7) for n in (8, 12, 16)]
    ids = ctx.load_servers(topos, np.arange(3, dtype=np.int32))
    ctx.set_busy(ids, [busy_leaving(rng, 8, 7), busy_leaving(rng, 12, 9), busy_leaving(rng, 16, 8)])
    cols = [(s, kind, k, mode) for s in range(3) for kind in range(3) for k in range(1, 9) for mode in (0, 1)]
    srv, kind, k, mode = (np.array(c) for c in zip(*cols))
    q = B.pack_queries(ids[srv], kind, k, mode, metric=1)
    base = ctx.query_batch(q)
    wide = ctx.query_batch_wide(q)
    for f in ("count", "status", "key", "agg", "pres", "vertex_mask", "links", "alloc_handle"):
        assert np.array_equal(wide[f], base[f]), f
    assert np.array_equal(wide["mapping"][:, :8], base["mapping"])
    assert (base["status"] == B.RES_OK).sum() > 40


def test_wide_jobs_of_nine_to_twelve(ctx):
    """k = 9..12 on 9..12 free accelerators of 18- and 20-vertex servers,
    up to 12! embeddings per query."""
    rng = np.random.default_rng(912)
    topos = [random_topology(rng, 18, 3, 0.6), random_topology(rng, 20, 7, 0.8)]
    st, busy, cols = [], [], {c: [] for c in ("server", "kind", "k", "mode", "a", "b")}
    s = 0
    for t in range(2):
        for F in (9, 10, 11, 12):
            st.append(t)
            busy.append(busy_leaving(rng, topos[t].shape[0], F))
            for kind in range(3):
                for k in range(9, 13):
                    if k < F and math.perm(F, k) > 4_000_000:
                        continue  # k = F stays: the oracle takes a few seconds for 12!
                    mode = int(rng.integers(0, 2))
                    for c, v in zip(cols, (s, kind, k, mode, 1, 1)):
                        cols[c].append(v)
            s += 1
    got, ref, qh = run_wide(ctx, topos, st, busy, cols)
    assert_same(got, ref, qh["k"], "k9-12")
    assert (ref["status"] == 0).sum() >= 12 and (qh["k"] >= 11).any()
    assert ctx.stats()["self_check_failures"] == 0


def test_wide_path_equals_batch_path_on_small_servers(ctx):
    """On servers both paths take (n <= 16, k <= 8) the wide call answers
    exactly as mapa_query_batch: 8,192 queries of the batched config."""
    wl = synth.config2(8192)
    qh, _ = B.load_workload(ctx, wl)
    base = ctx.query_batch(qh)
    wide = ctx.query_batch_wide(qh)
    for f in ("count", "status", "key", "agg", "pres", "vertex_mask", "alloc_handle"):
        assert np.array_equal(wide[f], base[f]), f
    assert np.array_equal(wide["mapping"][:, :8], base["mapping"])
    assert (wide["mapping"][:, 8:] == 0xFF).all()


def test_five_cube_hand_counts(ctx):
    """Q5 (32 vertices, degree 5, bipartite): LINKED ring k=2: 160; 4-cycles
    80 faces x 8 = 640; heap tree k=3: 32*5*4 = 640; heap tree k=4: 2560;
    no triangle; ALL mode ring k=3: 32*31*30."""
    W = np.zeros((32, 32), np.uint8)
    for u in range(32):
        for b in range(5):
            W[u, u ^ (1 << b)] = 1
    ids = ctx.load_servers([W], np.zeros(1, np.int32))
    q = B.pack_queries(ids[[0] * 6], [0, 0, 2, 2, 1, 0], [2, 4, 3, 4, 3, 3], [1, 1, 1, 1, 1, 0])
    got = ctx.query_batch_wide(q)
    assert list(got["count"]) == [160, 640, 640, 2560, 0, 29760]
    assert got["status"][4] == B.RES_NOFIT


def test_wide_registered_patterns(ctx):
    """Registered application graphs on 24-vertex servers, both modes."""
    rng = np.random.default_rng(24)
    pats = [(5, [(0, 4), (1, 4), (2, 4), (3, 4)]), (6, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5)]),
            (4, []), (8, [(i, (i + 3) % 8) for i in range(8)])]
    kinds = [ctx.create_pattern(k, e) for k, e in pats]
    topos = [random_topology(rng, 24, 3, 0.5)]
    st, busy, cols, edges = [], [], {c: [] for c in ("server", "kind", "k", "mode", "a", "b")}, []
    for s, F in enumerate((6, 8, 9)):
        st.append(0)
        busy.append(busy_leaving(rng, 24, F))
        for (k, e), kind in zip(pats, kinds):
            if math.perm(F, k) > 20_000:
                continue
            for mode in (0, 1):
                for c, v in zip(cols, (s, kind, k, mode, 1, 1)):
                    cols[c].append(v)
                edges.append(e)
    got, ref, qh = run_wide(ctx, topos, st, busy, cols, edges)
    assert_same(got, ref, qh["k"], "wide patterns")


def test_wide_commit_conflict_release(ctx):
    """Per server only the first committing query commits; later committing
    queries of that server get MAPA_RES_CONFLICT; handles release."""
    rng = np.random.default_rng(5)
    W = random_topology(rng, 28, 3, 0.6)
    ids = ctx.load_servers([W, W], np.zeros(2, np.int32))
    ctx.set_busy(ids, [busy_leaving(rng, 28, 10), busy_leaving(rng, 28, 10)])
    before = ctx.get_busy(ids).copy()
    q = B.pack_queries(ids[[0, 0, 1, 0]], [0, 1, 2, 0], [9, 3, 4, 2], commit=[1, 1, 1, 0])
    got = ctx.query_batch_wide(q)
    assert list(got["status"]) == [B.RES_OK, B.RES_CONFLICT, B.RES_OK, B.RES_OK]
    after = ctx.get_busy(ids)
    assert after[0] == before[0] | got["vertex_mask"][0]
    assert after[1] == before[1] | got["vertex_mask"][2]
    assert got["alloc_handle"][1] == -1 and got["alloc_handle"][3] == -1
    ctx.release(got["alloc_handle"][[0, 2]])
    assert np.array_equal(ctx.get_busy(ids), before)


def test_batch_path_refuses_wide_servers(ctx, torch):
    """The batch path answers queries on servers of more than 16
    accelerators with MAPA_RES_INVALID through device pointers (and refuses
    them up front through host pointers); the rest of the batch is served."""
    W = np.ones((24, 24), np.uint8) - np.eye(24, dtype=np.uint8)
    ids = ctx.load_servers([W, np.ones((4, 4), np.uint8) - np.eye(4, dtype=np.uint8)],
                           np.array([0, 1], np.int32))
    q = B.pack_queries(ids, [0, 0], [3, 3])
    with pytest.raises(B.MapaError) as e:
        ctx.query_batch(q)
    assert e.value.code == B.ERR_UNSUPPORTED
    dq = torch.from_numpy(q.view(np.uint8)).to("cuda")
    dr = torch.zeros(2 * 48, dtype=torch.uint8, device="cuda")
    ctx.query_batch(dq, dr, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    got = dr.cpu().numpy().view(B.RESULT_DTYPE)
    assert got["status"][0] == B.RES_INVALID
    assert got["status"][1] == B.RES_OK and got["count"][1] == 24
    wide = ctx.query_batch_wide(q)
    assert list(wide["count"]) == [24 * 23 * 22, 24]


def test_wide_config_full_against_stored_oracle_results(ctx):
    """Every query of the wide benchmark workload (16 seeded 32-vertex
    servers, 12 free accelerators each, ring / all-to-all / tree with k = 9
    and 10), in the call the benchmark times, against the stored oracle
    results field by field (tests/golden/c6_expected.txt, written by
    tests/golden/make_c6_expected.py from the oracle alone)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c6_expected.txt")
    if not os.path.exists(path):
        pytest.skip("tests/golden/c6_expected.txt not generated")
    rows = [[int(x) for x in line.split()] for line in open(path) if not line.startswith("#")]
    wl = synth.config6()
    assert len(rows) == wl.nq
    q, ids = B.load_workload(ctx, wl)
    got = ctx.query_batch_wide(q)
    for i, r in enumerate(rows):
        idx, server, busy, kind, k = r[:5]
        count, status, key, agg, pres, mask = r[5:11]
        assert idx == i and busy == int(wl.busy[server])
        assert (int(wl.queries["kind"][i]), int(wl.queries["k"][i])) == (kind, k)
        g = got[i]
        assert (int(g["count"]), int(g["status"])) == (count, status), i
        assert (int(g["key"]), int(g["agg"]), int(g["pres"]), int(g["vertex_mask"])) == \
            (key, agg, pres, mask), i
        assert tuple(int(x) for x in g["mapping"][:k]) == tuple(r[11:11 + k]), i
        assert (g["mapping"][k:] == 0xFF).all()
    # a second call on the same state answers the same (nothing committed)
    again = ctx.query_batch_wide(q)
    assert np.array_equal(again, got)


def wide_on_device(ctx, torch, q):
    """The device-pointer form on torch's current stream, results copied back."""
    dq = torch.from_numpy(np.ascontiguousarray(q).view(np.uint8).copy()).to("cuda")
    dr = torch.full((len(q) * B.RESULT_WIDE_DTYPE.itemsize,), 0xAB, dtype=torch.uint8, device="cuda")
    ctx.query_batch_wide(dq, dr, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    return dr.cpu().numpy().view(B.RESULT_WIDE_DTYPE), dr


def test_wide_device_pointers_equal_host_form(ctx, torch):
    """Queries and results in device memory, planned on the device: every
    byte of every result equals the host form's, on the wide benchmark
    workload and on mixed 17..32-vertex servers with every kind and k."""
    wl = synth.config6()
    q, _ = B.load_workload(ctx, wl)
    host = ctx.query_batch_wide(q)
    dev, _ = wide_on_device(ctx, torch, q)
    assert dev.tobytes() == host.tobytes()
    rng = np.random.default_rng(77)
    topos = [random_topology(rng, n, w, 0.5) for n, w in ((17, 1), (24, 2), (32, 255))]
    busy = [busy_leaving(rng, W.shape[0], F) for W, F in zip(topos, (9, 7, 6))]
    ids = ctx.load_servers(topos, np.arange(3, dtype=np.int32))
    ctx.set_busy(ids, busy)
    cols = [(s, kind, k, mode) for s in range(3) for kind in range(3) for k in range(1, 10)
            for mode in (0, 1)]
    srv, kind, k, mode = (np.array(c) for c in zip(*cols))
    q2 = B.pack_queries(ids[srv], kind, k, mode, a=rng.integers(0, 5, len(cols)), b=1)
    host2 = ctx.query_batch_wide(q2)
    dev2, _ = wide_on_device(ctx, torch, q2)
    assert dev2.tobytes() == host2.tobytes()
    assert (host2["status"] == B.RES_OK).sum() > 50


def test_wide_device_pointers_malformed_queries(ctx, torch):
    """Malformed queries are answered with MAPA_RES_INVALID on the device
    (no mapping, no handle); the well-formed rest of the batch answers as
    the host form does without them."""
    rng = np.random.default_rng(13)
    W = random_topology(rng, 24, 3, 0.6)
    ids = ctx.load_servers([W], np.zeros(1, np.int32))
    ctx.set_busy(ids, [busy_leaving(rng, 24, 8)])
    q = B.pack_queries(ids[[0] * 14], [0, 1, 2] * 4 + [0, 1], [3, 4, 5, 6] * 3 + [2, 7])
    bad = {1: ("k", 0), 2: ("k", 13), 4: ("server", -1), 5: ("server", 99), 6: ("metric", 1),
           7: ("metric", 3), 8: ("kind", 5), 9: ("kind", B.PATTERN_BASE + 7), 10: ("mode", 2),
           11: ("commit", 2), 12: ("a", -1), 13: ("b", 1025)}
    for i, (f, v) in bad.items():
        q[f][i] = v
    dev, _ = wide_on_device(ctx, torch, q)
    idx = np.array(sorted(bad))
    assert (dev["status"][idx] == B.RES_INVALID).all()
    assert (dev["alloc_handle"][idx] == -1).all() and (dev["mapping"][idx] == 0xFF).all()
    good = np.array([i for i in range(len(q)) if i not in bad])
    host = ctx.query_batch_wide(q[good])
    assert dev[good].tobytes() == host.tobytes()


def test_wide_device_pointers_commit_and_release(ctx, torch):
    """The batch commit rule through device pointers, handles released from
    the device result array in place (alloc_handle at byte 48 of 56)."""
    rng = np.random.default_rng(6)
    W = random_topology(rng, 30, 3, 0.6)
    ids = ctx.load_servers([W, W], np.zeros(2, np.int32))
    ctx.set_busy(ids, [busy_leaving(rng, 30, 10), busy_leaving(rng, 30, 9)])
    before = ctx.get_busy(ids).copy()
    q = B.pack_queries(ids[[0, 1, 0, 1, 0]], [0, 1, 2, 0, 1], [9, 3, 4, 2, 2], commit=[1, 1, 1, 0, 1])
    expect = ctx.query_batch_wide(q)  # host form: commits, then given back
    ctx.release(expect["alloc_handle"][expect["alloc_handle"] >= 0])
    assert np.array_equal(ctx.get_busy(ids), before)
    dev, dr = wide_on_device(ctx, torch, q)
    assert dev.tobytes() == expect.tobytes()
    assert list(dev["status"]) == [B.RES_OK, B.RES_OK, B.RES_CONFLICT, B.RES_OK, B.RES_CONFLICT]
    after = ctx.get_busy(ids)
    assert after[0] == before[0] | dev["vertex_mask"][0] and after[1] == before[1] | dev["vertex_mask"][1]
    ctx.release(dr.view(torch.int64)[6:], stride=56, count=len(q), stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert np.array_equal(ctx.get_busy(ids), before)


def test_wide_embedding_limit(ctx, torch):
    """A batch beyond 2^36 embeddings: the host form refuses it with
    MAPA_ERR_ADMISSION before anything runs; the device form answers every
    well-formed query with MAPA_RES_REFUSED, commits nothing and leaves the
    servers' commit claims free for the next call.  More than
    MAPA_MAX_WIDE_QUERIES queries are refused up front in both forms."""
    W = np.ones((32, 32), np.uint8) - np.eye(32, dtype=np.uint8)
    ids = ctx.load_servers([W, W], np.zeros(2, np.int32))
    q = B.pack_queries(ids[[0, 1, 1]], [0, 1, 0], [12, 3, 0], commit=[1, 1, 0])  # 32!/20! > 2^36
    with pytest.raises(B.MapaError) as e:
        ctx.query_batch_wide(q[:2])
    assert e.value.code == B.ERR_ADMISSION
    dev, _ = wide_on_device(ctx, torch, q)
    assert list(dev["status"]) == [B.RES_REFUSED, B.RES_REFUSED, B.RES_INVALID]
    assert (dev["count"] == 0).all() and (dev["alloc_handle"] == -1).all()
    assert (ctx.get_busy(ids) == 0).all()
    small = B.pack_queries(ids[[0, 1]], [0, 1], [2, 3], commit=[1, 1])
    dev2, _ = wide_on_device(ctx, torch, small)
    assert list(dev2["status"]) == [B.RES_OK, B.RES_OK]
    assert list(dev2["count"]) == [32 * 31, 32 * 31 * 30]
    assert list(ctx.get_busy(ids)) == [int(dev2["vertex_mask"][0]), int(dev2["vertex_mask"][1])]
    many = B.pack_queries(np.full(B.MAX_WIDE_QUERIES + 1, ids[0]), 0, 2)
    with pytest.raises(B.MapaError) as e:
        ctx.query_batch_wide(many)
    assert e.value.code == B.ERR_ADMISSION
