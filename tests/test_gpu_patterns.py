"""GPU parity for registered application graphs (edge lists, Sec. 3.1):
unions of the canonical shapes, sparse and dense random graphs, edgeless
and complete ones, against the oracle bit for bit, through the pipeline and
the fused launch, in both match modes and under both metrics."""
import itertools
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


def random_topology(rng, n, wmax, p_edge):
    W = np.zeros((n, n), np.uint8)
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p_edge:
                W[u, v] = W[v, u] = rng.integers(1, wmax + 1)
    return W


def pattern_set(rng):
    """(k, edges) of every shape family: random graphs of three densities,
    edgeless and complete graphs, canonical shapes renumbered, ring + tree
    unions, stars with the centre last (no earlier neighbour until the end)."""
    pats = []
    for k in range(1, 9):
        for p in (0.25, 0.5, 0.8):
            pats.append((k, [e for e in itertools.combinations(range(k), 2) if rng.random() < p]))
        pats.append((k, []))
        pats.append((k, list(itertools.combinations(range(k), 2))))
        ring = [] if k == 1 else [(0, 1)] if k == 2 else [(i, (i + 1) % k) for i in range(k)]
        tree = [((i - 1) // 2, i) for i in range(1, k)]
        sigma = rng.permutation(k)
        pats.append((k, [(int(sigma[u]), int(sigma[v])) for u, v in ring]))
        pats.append((k, sorted(set(tuple(sorted(e)) for e in ring + tree))))
        pats.append((k, [(i, k - 1) for i in range(k - 1)]))
    return pats


def build_queries(rng, topos, pats, kinds, per_topo, modes=(0, 1), metrics=(0,), max_leaves=2_000_000,
                  fmin=0):
    st, busy, cols, edges = [], [], {c: [] for c in ("server", "kind", "k", "mode", "a", "b", "metric")}, []
    s = 0
    for t, W in enumerate(topos):
        n = W.shape[0]
        for _ in range(per_topo):
            while True:
                b = int(rng.integers(0, 1 << n)) & int(rng.integers(0, 1 << n))
                if n - bin(b).count("1") >= fmin:
                    break
            F = n - bin(b).count("1")
            st.append(t)
            busy.append(b)
            for (k, e), kind in zip(pats, kinds):
                if k <= F and math.perm(F, k) > max_leaves:
                    continue
                for mode in modes:
                    for metric in metrics:
                        a, bb = [(1, 1), (1, 0), (0, 1), (5, 1024)][int(rng.integers(0, 4))]
                        for c, v in zip(cols, (s, kind, k, mode, a, bb, metric)):
                            cols[c].append(v)
                        edges.append(e)
            s += 1
    q = synth.make_queries(cols["server"], cols["kind"], cols["k"], cols["mode"], 0, cols["a"], cols["b"],
                           cols["metric"])
    wl = synth.Workload("patterns", topos, np.array(st, np.int32), np.array(busy, np.uint32), q)
    return wl, edges


def distinct_server_batches(servers):
    occ = {}
    batch_of = np.empty(len(servers), np.int64)
    for i, s in enumerate(servers):
        batch_of[i] = occ.get(int(s), 0)
        occ[int(s)] = batch_of[i] + 1
    return [np.nonzero(batch_of == j)[0] for j in range(int(batch_of.max()) + 1)]


def oracle_answers(wl, edges):
    q = wl.queries
    srv = q["server"]
    return oracle.batch(wl.topologies, wl.server_topo[srv], wl.busy[srv], q["kind"], q["k"], q["mode"],
                        q["a"], q["b"], NTHREADS, q["metric"], edges=edges)


@pytest.mark.parametrize("wmax,nmax", [(3, 9), (15, 9), (3, 12)])
def test_registered_patterns_against_oracle(ctx, wmax, nmax):
    """Every shape family on random topologies (row formats of weights <= 3
    and <= 15; with 12 vertices the variant that scores the last two
    positions from per-candidate tables), one pipeline batch and
    one-query-per-server fused batches."""
    rng = np.random.default_rng(40 + wmax + nmax)
    pats = pattern_set(rng)
    kinds = [ctx.create_pattern(k, e) for k, e in pats]
    assert kinds[0] == B.PATTERN_BASE and kinds[-1] == B.PATTERN_BASE + len(pats) - 1
    topos = [random_topology(rng, int(rng.integers(2, nmax + 1)), wmax, 0.6) for _ in range(5)]
    wl, edges = build_queries(rng, topos, pats, kinds, 2)
    qh, _ = B.load_workload(ctx, wl)
    got = ctx.query_batch(qh)
    ref = oracle_answers(wl, edges)
    assert_same(got, ref, qh["k"], "patterns")
    assert (ref["status"] == 0).sum() > 200
    for sel in distinct_server_batches(qh["server"])[:40]:
        fused = ctx.query_batch(qh[sel])
        assert np.array_equal(fused, got[sel])
    assert ctx.stats()["self_check_failures"] == 0


def test_registered_patterns_sixteen_vertices_every_pair_width(ctx):
    """16-vertex topologies, 2..13 free vertices: the last two positions of
    registered patterns see every candidate count of the table-scored
    variant."""
    rng = np.random.default_rng(1617)
    pats = [p for p in pattern_set(rng) if p[0] >= 2]
    pats = [pats[i] for i in rng.choice(len(pats), size=24, replace=False)]
    kinds = [ctx.create_pattern(k, e) for k, e in pats]
    topos = [random_topology(rng, 16, 3, 0.7) for _ in range(3)]
    st, busy = [], []
    for F in range(2, 14):
        t = int(rng.integers(0, 3))
        free = rng.choice(16, size=F, replace=False)
        st.append(t)
        busy.append(int(0xFFFF & ~int(np.bitwise_or.reduce(1 << free))))
    cols = {c: [] for c in ("server", "kind", "k", "mode", "a", "b")}
    edges = []
    for s, b in enumerate(busy):
        F = 16 - bin(b).count("1")
        for (k, e), kind in zip(pats, kinds):
            if k > F or math.perm(F, k) > 1_000_000:
                continue
            for mode in (0, 1):
                for c, v in zip(cols, (s, kind, k, mode, 1, 1)):
                    cols[c].append(v)
                edges.append(e)
    q = synth.make_queries(cols["server"], cols["kind"], cols["k"], cols["mode"], 0, cols["a"], cols["b"])
    wl = synth.Workload("patterns16", topos, np.array(st, np.int32), np.array(busy, np.uint32), q)
    qh, _ = B.load_workload(ctx, wl)
    got = ctx.query_batch(qh)
    assert_same(got, oracle_answers(wl, edges), qh["k"], "patterns16")
    assert ctx.stats()["self_check_failures"] == 0


def test_registered_patterns_effective_bandwidth(ctx):
    """Eq. 2 on registered patterns (the link-mix tables cover every edge
    count up to 28)."""
    rng = np.random.default_rng(88)
    pats = pattern_set(rng)
    kinds = [ctx.create_pattern(k, e) for k, e in pats]
    topos = [random_topology(rng, int(rng.integers(3, 10)), 2, 0.6) for _ in range(4)]
    wl, edges = build_queries(rng, topos, pats, kinds, 2, metrics=(1,), max_leaves=500_000)
    qh, _ = B.load_workload(ctx, wl)
    got = ctx.query_batch(qh)
    ref = oracle_answers(wl, edges)
    assert_same(got, ref, qh["k"], "patterns effbw")
    assert (ref["status"] == 0).sum() > 100
    assert ctx.stats()["self_check_failures"] == 0


def test_canonical_shapes_registered_equal_the_kinds(ctx):
    """The batched config's queries, re-asked with their ring / all-to-all /
    tree written out as registered patterns, give the same results as the
    built-in kinds (and those equal the oracle's in the kind tests)."""
    wl = synth.config2(8192)
    qh, _ = B.load_workload(ctx, wl)
    ring = lambda k: [] if k == 1 else [(0, 1)] if k == 2 else [(i, (i + 1) % k) for i in range(k)]
    shapes = {0: ring, 1: lambda k: list(itertools.combinations(range(k), 2)),
              2: lambda k: [((i - 1) // 2, i) for i in range(1, k)]}
    table = {(kind, k): ctx.create_pattern(k, shapes[kind](k)) for kind in range(3) for k in range(1, 9)}
    q2 = qh.copy()
    q2["kind"] = [table[(int(a), int(b))] for a, b in zip(qh["kind"], qh["k"])]
    base = ctx.query_batch(qh)
    got = ctx.query_batch(q2)
    assert np.array_equal(got, base)


def test_registered_pattern_invalid_on_device(ctx, torch):
    """Through device pointers a query naming a free pattern slot, or the
    wrong k for a registered one, is answered MAPA_RES_INVALID; the rest of
    the batch is unaffected."""
    W = np.ones((6, 6), np.uint8)
    np.fill_diagonal(W, 0)
    ids = ctx.load_servers([W], np.zeros(3, np.int32))
    kind = ctx.create_pattern(3, [(0, 2)])
    q = B.pack_queries(ids, [kind, kind + 1, kind], [3, 3, 4])
    dq = torch.from_numpy(q.view(np.uint8)).to("cuda")
    dr = torch.zeros(3 * 48, dtype=torch.uint8, device="cuda")
    ctx.query_batch(dq, dr, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    got = dr.cpu().numpy().view(B.RESULT_DTYPE)
    assert got["status"][0] == B.RES_OK and got["count"][0] == 120
    assert got["status"][1] == B.RES_INVALID and got["status"][2] == B.RES_INVALID


def test_linked_search_order_keeps_the_numbering_tie_break(ctx):
    """LINKED search places a registered pattern's vertices in a matching
    order (most constrained first, each next to a placed neighbour); the
    selection must still be the lexicographically first maximum in the
    caller's numbering.  Random renumberings of connected patterns on dense
    topologies with weights 1 (many equal keys) and 1..3, against the oracle
    on the same numbering, through the pipeline and the fused launch."""
    rng = np.random.default_rng(77)
    base = [(4, [(0, 1), (1, 2), (2, 3)]), (5, [(0, 4), (1, 4), (2, 4), (3, 4)]),
            (6, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5), (5, 3), (0, 3)]),
            (7, [(i, 6) for i in range(6)] + [(0, 1)]), (8, [(i, i + 1) for i in range(7)]),
            (6, [(0, 1), (2, 3), (4, 5)])]  # a disconnected one: order per component
    for _ in range(6):  # random connected graphs
        k = int(rng.integers(4, 9))
        perm = rng.permutation(k)
        e = {tuple(sorted((int(perm[i]), int(perm[int(rng.integers(0, i))])))) for i in range(1, k)}
        e |= {tuple(sorted(map(int, rng.choice(k, 2, replace=False)))) for _ in range(int(rng.integers(0, k)))}
        base.append((k, sorted(e)))
    pats = []
    for k, e in base:
        for _ in range(3):
            sigma = rng.permutation(k)
            pats.append((k, [(int(sigma[u]), int(sigma[v])) for u, v in e]))
    kinds = [ctx.create_pattern(k, e) for k, e in pats]
    topos = [random_topology(rng, 10, 1, 0.8), random_topology(rng, 11, 3, 0.7),
             random_topology(rng, 9, 1, 1.0)]
    wl, edges = build_queries(rng, topos, pats, kinds, 2, modes=(1,), max_leaves=3_000_000)
    qh, _ = B.load_workload(ctx, wl)
    print(f"[patterns] {len(qh)} LINKED queries of {len(pats)} renumbered patterns", flush=True)
    got = ctx.query_batch(qh)
    ref = oracle_answers(wl, edges)
    assert_same(got, ref, qh["k"], "renumbered LINKED")
    assert (ref["status"] == 0).sum() > 100
    for sel in distinct_server_batches(qh["server"])[:10]:
        assert np.array_equal(ctx.query_batch(qh[sel]), got[sel])
    assert ctx.stats()["self_check_failures"] == 0
