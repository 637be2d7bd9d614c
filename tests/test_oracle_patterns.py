"""Pins for the oracle's caller-supplied application graphs (a pattern given
as its edge list on vertices 0..k-1, Sec. 3.1: unions of the canonical
shapes, graphs derived from a program).  Values come from combinatorics and
from the definitions of matches (Sec. 3.3), AggBW (Eq. 1) and PreservedBW
(Eq. 3), not from the oracle itself."""
import itertools
import math

import numpy as np
import pytest

from oracle import brute

RING, A2A, TREE = 0, 1, 2
ALL, LINKED = 0, 1


def graph(n, edges, w=1):
    W = np.zeros((n, n), dtype=np.uint8)
    for u, v in edges:
        W[u, v] = W[v, u] = w
    return W


def random_sym(rng, n, wmax, p_edge=1.0):
    W = np.zeros((n, n), dtype=np.uint8)
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p_edge:
                W[u, v] = W[v, u] = rng.integers(0, wmax + 1)
    return W


def random_pattern(rng, k, p):
    return [(u, v) for u, v in itertools.combinations(range(k), 2) if rng.random() < p]


CUBE_Q3 = [(u, u ^ (1 << b)) for u in range(8) for b in range(3) if u < u ^ (1 << b)]
CUBE_MESH = (list(itertools.combinations(range(4), 2)) +
             [(u + 4, v + 4) for u, v in itertools.combinations(range(4), 2)] +
             [(i, i + 4) for i in range(4)])

# |Aut| from theory: a star K_{1,m} permutes its leaves (m!); a path on k >= 2
# vertices has its reversal (2); the edgeless graph on k vertices has k!;
# K_{2,3} swaps within each side (2! 3!); the cube Q3 has 48 symmetries
# (3! axis permutations x 2^3 reflections); the wheel with a 4-cycle rim has
# the rim's dihedral group (8); two disjoint triangles: 2 * 3! * 3! = 72.
AUT_CASES = [
    ("star K1,3", 4, [(0, 1), (0, 2), (0, 3)], 6),
    ("star K1,7", 8, [(0, i) for i in range(1, 8)], 5040),
    ("path P5", 5, [(0, 1), (1, 2), (2, 3), (3, 4)], 2),
    ("path P8", 8, [(i, i + 1) for i in range(7)], 2),
    ("edgeless 5", 5, [], 120),
    ("K2,3", 5, [(u, v) for u in (0, 1) for v in (2, 3, 4)], 12),
    ("cube Q3", 8, CUBE_Q3, 48),
    ("wheel W4", 5, [(0, i) for i in range(1, 5)] + [(1, 2), (2, 3), (3, 4), (4, 1)], 8),
    ("two triangles", 6, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5), (5, 3)], 72),
]


@pytest.mark.parametrize("name,k,edges,aut", AUT_CASES, ids=[c[0] for c in AUT_CASES])
def test_automorphisms_and_self_embeddings(orc, name, k, edges, aut):
    """|Aut(P)| from theory; the LINKED embeddings of P into a host graph
    equal to P are exactly its automorphisms."""
    assert orc.aut_count(None, k, edges) == aut
    r = orc.query(graph(k, edges), 0, 0, k, LINKED, edges=edges)
    assert r["count"] == aut and r["status"] == 0


def test_cube_into_cube_mesh_by_hand(orc):
    """Q3 into the 8-vertex cube-mesh (two K4 joined by rungs i - i+4): Q3 has
    12 edges and no triangle, so each K4 can host at most a 4-cycle (4 edges)
    and all 4 rungs must be used; the two 4-cycles must correspond under the
    rungs, or an odd cycle appears.  3 copies (one per 4-cycle of a K4) x
    |Aut(Q3)| = 144 embeddings."""
    r = orc.query(graph(8, CUBE_MESH), 0, 0, 8, LINKED, edges=CUBE_Q3)
    assert r["count"] == 144


def test_canonical_shapes_given_as_edge_lists(orc):
    """The ring, all-to-all and tree written out as edge lists from their
    definitions (Sec. 3.1), in shuffled order and orientation, give the same
    answer as the canonical kinds, mapping included."""
    shapes = {
        RING: lambda k: [] if k == 1 else [(0, 1)] if k == 2 else [(i, (i + 1) % k) for i in range(k)],
        A2A: lambda k: list(itertools.combinations(range(k), 2)),
        TREE: lambda k: [(i, c) for i in range(k) for c in (2 * i + 1, 2 * i + 2) if c < k],
    }
    rng = np.random.default_rng(5)
    W = random_sym(rng, 9, 3, 0.7)
    for kind, make in shapes.items():
        for k in range(1, 7):
            e = make(k)
            rng.shuffle(e)
            e = [(v, u) if rng.random() < 0.5 else (u, v) for u, v in e]
            for mode in (ALL, LINKED):
                for ab in ((1, 1), (1, 0), (0, 1)):
                    assert orc.query(W, 0b100100, kind, k, mode, *ab) == \
                        orc.query(W, 0b100100, 0, k, mode, *ab, edges=e), (kind, k, mode, ab)


def test_ring_tree_union_is_complete_on_four(orc):
    """A combined application graph: the 4-ring's edges plus the 4-vertex heap
    tree's (0-1, 0-2, 1-3) give every pair, i.e. K4, so the union answers
    exactly as the all-to-all pattern."""
    union = sorted(set(map(tuple, map(sorted, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 1), (0, 2), (1, 3)]))))
    assert union == list(itertools.combinations(range(4), 2))
    rng = np.random.default_rng(9)
    W = random_sym(rng, 8, 3)
    for mode in (ALL, LINKED):
        assert orc.query(W, 0, 0, 4, mode, edges=union) == orc.query(W, 0, A2A, 4, mode)


def test_edgeless_pattern_closed_form(orc):
    """No pattern edge: AggBW is 0 for every map, every injective map is a
    match in both modes (F!/(F-k)!), and under the Greedy key (a, b) = (1, 0)
    every map ties at 0, so the lexicographically first tuple -- the k
    smallest free vertices in increasing order -- is kept."""
    rng = np.random.default_rng(3)
    W = random_sym(rng, 10, 3, 0.5)
    busy = 0b0100010010
    R = [v for v in range(10) if not busy >> v & 1]
    for k in range(1, 6):
        for mode in (ALL, LINKED):
            r = orc.query(W, busy, 0, k, mode, 1, 0, edges=[])
            assert r["count"] == math.perm(len(R), k)
            assert (r["key"], r["agg"], r["mapping"]) == (0, 0, tuple(R[:k]))


def test_star_greedy_closed_form(orc):
    """Star with its centre at vertex 0 and m leaves, Greedy key: AggBW of a
    map is the weight from the centre's host vertex to the m leaves' hosts, so
    the best is, over host vertices v, the sum of the m heaviest weights from
    v to the other free vertices."""
    rng = np.random.default_rng(4)
    for n, m in ((7, 3), (9, 4), (10, 2)):
        W = random_sym(rng, n, 5)
        busy = int(rng.integers(0, 1 << n)) & int(rng.integers(0, 1 << n)) & int(rng.integers(0, 1 << n))
        R = [v for v in range(n) if not busy >> v & 1]
        if len(R) < m + 1:
            continue
        best = max(sum(sorted((int(W[v, u]) for u in R if u != v), reverse=True)[:m]) for v in R)
        r = orc.query(W, busy, 0, m + 1, ALL, 1, 0, edges=[(0, i) for i in range(1, m + 1)])
        assert r["key"] == best == r["agg"]


def test_relabeling_the_pattern_keeps_count_and_key(orc):
    """Renumbering the pattern's vertices changes only which tuple stands for
    a placement: the number of matches and the best key stay, and the kept
    mapping is a match of the renumbered pattern with that AggBW."""
    rng = np.random.default_rng(6)
    for _ in range(6):
        k = int(rng.integers(3, 7))
        e = random_pattern(rng, k, 0.5)
        sigma = rng.permutation(k)
        e2 = [(int(sigma[u]), int(sigma[v])) for u, v in e]
        W = random_sym(rng, 9, 3, 0.6)
        busy = int(rng.integers(0, 8))
        for mode in (ALL, LINKED):
            r1 = orc.query(W, busy, 0, k, mode, 2, 1, edges=e)
            r2 = orc.query(W, busy, 0, k, mode, 2, 1, edges=e2)
            assert (r1["count"], r1["status"], r1.get("key")) == (r2["count"], r2["status"], r2.get("key"))
            if r2["status"] == 0:
                phi = r2["mapping"]
                assert r2["agg"] == sum(int(W[phi[u], phi[v]]) for u, v in e2)
                if mode == LINKED:
                    assert all(W[phi[u], phi[v]] > 0 for u, v in e2)


def test_agreement_with_python_brute_force(orc):
    """Random edge lists on k <= 5 against the independent brute force, every
    busy mask of n <= 5 graphs, both modes, both metrics."""
    rng = np.random.default_rng(31)
    cases = 0
    for n in range(2, 6):
        for _ in range(2):
            W = random_sym(rng, n, 2)
            for k in range(1, n + 1):
                for p in (0.3, 0.7):
                    e = random_pattern(rng, k, p)
                    for busy in range(1 << n):
                        for mode in (ALL, LINKED):
                            for metric, ab in ((0, (1, 1)), (0, (2, 3)), (1, (1, 1))):
                                got = orc.query(W, busy, 0, k, mode, *ab, metric=metric, edges=e)
                                ref = brute.query(W.tolist(), busy, 0, k, mode, *ab, metric, pattern=e)
                                assert got["count"] == ref["count"] and got["status"] == ref["status"]
                                if ref["status"] == 0:
                                    assert (got["key"], got["agg"], got["pres"], got["mapping"]) == \
                                        (ref["key"], ref["agg"], ref["pres"], ref["mapping"])
                                cases += 1
    assert cases > 3000


def test_edge_list_validation(orc):
    W = graph(6, [(0, 1), (1, 2)])
    for e in ([(0, 0)], [(0, 1), (1, 0)], [(0, 4)], [(-1, 2)]):
        assert orc.query(W, 0, 0, 4, edges=e)["status"] == orc.EINVAL, e
    assert orc.aut_count(None, 4, [(0, 1), (0, 1)]) == orc.EINVAL
    # 28 edges (K8) is the most a simple graph on 8 vertices has
    k8 = list(itertools.combinations(range(8), 2))
    assert orc.query(graph(8, k8), 0, 0, 8, LINKED, edges=k8)["count"] == math.factorial(8)
