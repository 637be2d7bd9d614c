"""Tiny-graph brute force of the MAPA allocation query -- TEST INFRASTRUCTURE.

Written independently of ``mapa_oracle.c`` to cross-check it exhaustively on
small graphs.  Pure Python over ``itertools.permutations``: only for n <= 6.

Definitions (Sec. 3.1-3.5 of the paper):
  * matches: injective maps of the k pattern positions into the free vertices
    (Sec. 3.3); mode LINKED additionally needs W > 0 on every pattern edge;
  * AggBW = sum of W over mapped pattern edges (Eq. 1);
  * PreservedBW = sum of W over pairs of free vertices left unallocated (Eq. 3);
  * key = a*AggBW + b*PreservedBW; the first strict maximum in lexicographic
    order of the mapping tuple wins (Alg. 1 scan with strict '>');
  * bandwidth-sensitive jobs: the key is Eq. 2's predicted effective
    bandwidth of the mapped pattern edges' link mix (x double NVLinks =
    weight 2, y single = 1, z PCIe = 0; coefficients of Table "Values of
    Coefficients"), compared as a float, reported as round(1000 * EffBW).
"""
from __future__ import annotations

import itertools


def edges(kind: int, k: int):
    """Pattern edges: ring (kind 0), all-to-all (kind 1), heap binary tree (kind 2)."""
    if kind == 0:
        if k == 1:
            return []
        if k == 2:
            return [(0, 1)]
        return [(i, (i + 1) % k) for i in range(k)]
    if kind == 1:
        return list(itertools.combinations(range(k), 2))
    if kind == 2:
        return [((i - 1) // 2, i) for i in range(1, k)]
    raise ValueError(kind)


THETA = (16.396, 4.536, 1.556, -20.694, -9.467, 7.615, -7.973,
         12.733, -4.195, -8.413, 62.851, 27.418, -5.114, -46.973)


def effbw(x: int, y: int, z: int) -> float:
    """Eq. 2, feature by feature in the paper's order."""
    feats = (x, y, z, 1 / (x + 1), 1 / (y + 1), 1 / (z + 1), x * y, y * z, z * x,
             1 / (x * y + 1), 1 / (y * z + 1), 1 / (z * x + 1), x * y * z, 1 / (x * y * z + 1))
    return sum(t * f for t, f in zip(THETA, feats))


def query(W, busy: int, kind: int, k: int, mode: int = 0, a: int = 1, b: int = 1,
          metric: int = 0, pattern=None):
    """``pattern``: an explicit edge list on vertices 0..k-1 (``kind`` is then
    ignored), e.g. a union of canonical patterns or a program-derived graph."""
    n = len(W)
    free = [v for v in range(n) if not (busy >> v) & 1]
    E = edges(kind, k) if pattern is None else [tuple(e) for e in pattern]
    count = 0
    best = None
    for phi in itertools.permutations(free, k):
        if mode == 1 and any(W[phi[p]][phi[q]] == 0 for p, q in E):
            continue
        count += 1
        agg = sum(int(W[phi[p]][phi[q]]) for p, q in E)
        left = [v for v in free if v not in phi]
        pres = sum(int(W[u][v]) for u, v in itertools.combinations(left, 2))
        if metric == 1:
            ws = [int(W[phi[p]][phi[q]]) for p, q in E]
            key = effbw(ws.count(2), ws.count(1), ws.count(0))
        else:
            key = a * agg + b * pres
        if best is None or key > best[0]:
            best = (key, phi, agg, pres)
    if best is None:
        return {"count": 0, "status": 1}
    key, phi, agg, pres = best
    if metric == 1:
        key = int(round(1000 * key))
    mask = 0
    for v in phi:
        mask |= 1 << v
    return {"count": count, "status": 0, "key": key, "agg": agg, "pres": pres,
            "mapping": tuple(phi), "vertex_mask": mask}
