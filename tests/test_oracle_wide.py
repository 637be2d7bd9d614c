"""Pins for the oracle on wide shapes: servers of 17..32 accelerators and
patterns of 9..12 vertices (the larger jobs of Sec. 5.4).  Values come
from combinatorics and textbook problems, not from the oracle itself."""
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


def busy_leaving(rng, n, F):
    free = rng.choice(n, size=F, replace=False)
    return int(((1 << n) - 1) & ~int(np.bitwise_or.reduce(1 << free.astype(np.int64))))


def q5():
    return graph(32, [(u, u ^ (1 << b)) for u in range(32) for b in range(5) if u < u ^ (1 << b)])


# Heap-numbered binary trees on 9 and 10 vertices: node 3 holds leaves 7, 8
# (and node 4 holds 9 for k = 10), node 2 holds leaves 5, 6; the two subtrees
# of the root differ in size and those of node 1 in shape, so only the leaf
# pairs {7, 8} and {5, 6} can swap: |Aut| = 4 for both.
AUT_WIDE = {RING: {9: 18, 10: 20}, A2A: {9: math.factorial(9), 10: math.factorial(10)},
            TREE: {9: 4, 10: 4}}


@pytest.mark.parametrize("kind", [RING, A2A, TREE])
def test_wide_pattern_automorphisms(orc, kind):
    for k in (9, 10):
        assert orc.aut_count(kind, k) == AUT_WIDE[kind][k]


def test_wide_patterns_into_themselves(orc):
    """LINKED embeddings of the 9- and 10-vertex ring and tree into host
    graphs equal to them (written from the definitions) are |Aut|."""
    hosts = {RING: lambda k: [(i, (i + 1) % k) for i in range(k)],
             TREE: lambda k: [(i, c) for i in range(k) for c in (2 * i + 1, 2 * i + 2) if c < k]}
    for kind, make in hosts.items():
        for k in (9, 10):
            assert orc.query(graph(k, make(k)), 0, kind, k, LINKED)["count"] == AUT_WIDE[kind][k]


def test_five_cube_hand_counts(orc):
    """The 32-vertex hypercube Q5: 80 edges, degree 5, bipartite.
    ring k=2: 2 * 80; 4-cycles are the 2-faces, C(5,2) * 2^3 = 80, times 8
    orders; heap tree k=3 (a 2-path around position 0): 32 * 5 * 4; heap
    tree k=4 (the path 3-1-0-2): 160 ordered middle edges * 4 * 4; no odd
    cycle and no triangle."""
    W = q5()
    assert orc.query(W, 0, RING, 2, LINKED)["count"] == 160
    assert orc.query(W, 0, RING, 4, LINKED)["count"] == 640
    assert orc.query(W, 0, TREE, 3, LINKED)["count"] == 640
    assert orc.query(W, 0, TREE, 4, LINKED)["count"] == 2560
    assert orc.query(W, 0, RING, 3, LINKED)["count"] == 0
    assert orc.query(W, 0, A2A, 3, LINKED)["count"] == 0


@pytest.mark.parametrize("n", [17, 24, 32])
def test_wide_all_mode_counts(orc, n):
    """Every injective map is a match: F!/(F-k)! for any k <= 12."""
    rng = np.random.default_rng(500 + n)
    W = random_sym(rng, n, 3)
    for F in (3, 9, 11, 12):
        busy = busy_leaving(rng, n, F)
        for kind in (RING, A2A, TREE):
            for k in range(1, 13):
                if math.perm(F, k) > 20_000:
                    continue
                r = orc.query(W, busy, kind, k, ALL)
                if k > F:
                    assert r["status"] == 1 and r["count"] == 0
                else:
                    assert r["count"] == math.perm(F, k) and len(r["mapping"]) == k


def held_karp_max_cycle(W, verts):
    m = len(verts)
    NEG = -1 << 60
    dp = [[NEG] * m for _ in range(1 << m)]
    dp[1][0] = 0
    for S in range(1 << m):
        if not S & 1:
            continue
        for j in range(m):
            if dp[S][j] == NEG:
                continue
            for t in range(1, m):
                if S >> t & 1:
                    continue
                v = dp[S][j] + int(W[verts[j], verts[t]])
                if v > dp[S | 1 << t][t]:
                    dp[S | 1 << t][t] = v
    full = (1 << m) - 1
    return max(dp[full][j] + int(W[verts[j], verts[0]]) for j in range(1, m))


def test_wide_greedy_ring_is_max_hamiltonian_cycle(orc):
    """Greedy key, ring with k = F in {9, 10}: the best AggBW is the heaviest
    Hamiltonian cycle on the free vertices (Held-Karp)."""
    rng = np.random.default_rng(77)
    for F in (9, 10):
        n = 18
        W = random_sym(rng, n, 9)
        busy = busy_leaving(rng, n, F)
        R = [v for v in range(n) if not busy >> v & 1]
        r = orc.query(W, busy, RING, F, ALL, 1, 0)
        assert r["key"] == r["agg"] == held_karp_max_cycle(W, R)


def test_wide_greedy_all_to_all_is_heaviest_subset(orc):
    """Greedy key, all-to-all with k = 9 of F = 10: the best AggBW is the
    heaviest induced 9-subset; every order of it scores the same, so the
    kept mapping is that subset in increasing order (the first maximum)."""
    rng = np.random.default_rng(78)
    n = 20
    W = random_sym(rng, n, 5)
    busy = busy_leaving(rng, n, 10)
    R = [v for v in range(n) if not busy >> v & 1]
    best = max(itertools.combinations(R, 9),
               key=lambda S: (sum(int(W[u, v]) for u, v in itertools.combinations(S, 2)),
                              [-x for x in S]))
    r = orc.query(W, busy, A2A, 9, ALL, 1, 0)
    assert r["key"] == sum(int(W[u, v]) for u, v in itertools.combinations(best, 2))
    assert r["mapping"] == tuple(best)


def test_wide_single_vertex_closed_form(orc):
    """k = 1 on 32 vertices, key = PreservedBW = W(R) - d_R(v): the free
    vertex of least weight to the rest, smallest index among ties."""
    rng = np.random.default_rng(79)
    W = random_sym(rng, 32, 4)
    busy = busy_leaving(rng, 32, 20)
    R = [v for v in range(32) if not busy >> v & 1]
    WR = sum(int(W[u, v]) for u, v in itertools.combinations(R, 2))
    d = {v: sum(int(W[v, u]) for u in R) for v in R}
    v = min(R, key=lambda x: (d[x], x))
    r = orc.query(W, busy, RING, 1, ALL, 0, 1)
    assert r["mapping"] == (v,) and r["key"] == WR - d[v]


def test_wide_agreement_with_python_brute_force(orc):
    """Servers of 17..32 vertices with 4..8 free, every kind, k <= 4, both
    modes, three key weightings, and k = 9 on 9..10 free vertices."""
    rng = np.random.default_rng(80)
    for n in (17, 23, 32):
        W = random_sym(rng, n, 3, 0.7)
        for F in (4, 6, 8):
            busy = busy_leaving(rng, n, F)
            for kind in (RING, A2A, TREE):
                for k in range(1, 5):
                    for mode in (ALL, LINKED):
                        for a, b in ((1, 1), (1, 0), (2, 3)):
                            got = orc.query(W, busy, kind, k, mode, a, b)
                            ref = brute.query(W.tolist(), busy, kind, k, mode, a, b)
                            assert got["count"] == ref["count"]
                            if ref["status"] == 0:
                                assert (got["key"], got["agg"], got["pres"], got["mapping"]) == \
                                    (ref["key"], ref["agg"], ref["pres"], ref["mapping"])
    W = random_sym(rng, 20, 2)
    busy = busy_leaving(rng, 20, 9)
    for kind in (RING, TREE):
        got = orc.query(W, busy, kind, 9, ALL, 1, 1)
        ref = brute.query(W.tolist(), busy, kind, 9, ALL, 1, 1)
        assert (got["count"], got["key"], got["mapping"]) == (ref["count"], ref["key"], ref["mapping"])


def test_wide_limits(orc):
    W = q5()
    assert orc.query(W, 0, RING, 13)["status"] == orc.EUNSUP
    assert orc.query(np.zeros((33, 33), np.uint8), 0, RING, 2)["status"] == orc.EUNSUP
    # all 32 bits of the busy mask are vertices: 31 busy leaves one free
    r = orc.query(W, 0x7FFFFFFF, RING, 1, ALL)
    assert r["count"] == 1 and r["mapping"] == (31,)
