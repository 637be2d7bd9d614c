"""CPU oracle for the MAPA allocation query -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU product path never loads it and
shares no code with it.

Two independent implementations live here:

* ``mapa_oracle.c`` (built to ``liboracle.so`` with gcc): plain recursive brute
  force over every injective tuple in lexicographic order, Eq. 1 and Eq. 3
  evaluated literally, Alg. 1's strict-improvement scan.
* ``brute.py``: the same definition with ``itertools.permutations``; slow,
  used to cross-check the C file exhaustively on tiny graphs.

``run_batch_semantics`` adds the batch-level state update (Sec. 3.6): each
query is evaluated against the busy masks at batch entry; afterwards, in array
order, the first query of a server that asked to commit marks its chosen
vertices busy, and any later committing query of the same server is refused
(status CONFLICT).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "mapa_oracle.c")

RING, A2A, TREE = 0, 1, 2
MAX_N, MAX_K = 32, 12
MAX_E = MAX_K * (MAX_K - 1) // 2
MODE_ALL, MODE_LINKED = 0, 1
METRIC_WEIGHTED, METRIC_EFFBW = 0, 1
OK, NOFIT, CONFLICT = 0, 1, 2
EINVAL, EUNSUP = -1, -2


class OrResult(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("key", ctypes.c_int32),
        ("agg", ctypes.c_int32),
        ("pres", ctypes.c_int32),
        ("vertex_mask", ctypes.c_uint32),
        ("mapping", ctypes.c_uint8 * 16),
        ("links", ctypes.c_int32),
    ]


RESULT_DTYPE = np.dtype([
    ("count", np.int64), ("status", np.int32), ("key", np.int32), ("agg", np.int32),
    ("pres", np.int32), ("vertex_mask", np.uint32), ("mapping", np.uint8, 16), ("links", np.int32),
], align=True)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no vectorisation pragmas)."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.or_query.restype = ctypes.c_int
        L.or_query.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.POINTER(OrResult)]
        L.or_batch.restype = ctypes.c_int
        L.or_query_edges.restype = ctypes.c_int
        L.or_query_edges.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.POINTER(OrResult)]
        L.or_batch.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 13 + [ctypes.c_int]
        L.or_effbw.restype = ctypes.c_double
        L.or_effbw.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_pattern_edges.restype = ctypes.c_int
        L.or_pattern_edges.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.or_aut_count.restype = ctypes.c_int
        L.or_aut_count.argtypes = [ctypes.c_int, ctypes.c_int]
        L.or_aut_count_edges.restype = ctypes.c_int
        L.or_aut_count_edges.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        L.or_result_size.restype = ctypes.c_int
        assert L.or_result_size() == RESULT_DTYPE.itemsize == ctypes.sizeof(OrResult)
        _lib = L
    return _lib


def edge_array(edges):
    """Flat int32 array of an edge list [(u, v), ...]."""
    return np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1))


def query(W, busy, kind, k, mode=MODE_ALL, a=1, b=1, metric=METRIC_WEIGHTED, edges=None) -> dict:
    """One query on an n x n weight matrix.  Returns a dict of the result.
    With ``edges`` (a list of (u, v) pairs on vertices 0..k-1) the pattern
    is that graph and ``kind`` is ignored."""
    W = np.ascontiguousarray(np.asarray(W, dtype=np.uint8))
    n = W.shape[0]
    r = OrResult()
    if edges is None:
        lib().or_query(n, W.ctypes.data, int(busy), int(kind), int(k), int(mode), int(a), int(b),
                       int(metric), ctypes.byref(r))
    else:
        e = edge_array(edges)
        lib().or_query_edges(n, W.ctypes.data, int(busy), int(k), len(e) // 2, e.ctypes.data,
                             int(mode), int(a), int(b), int(metric), ctypes.byref(r))
    return {
        "count": r.count, "status": r.status, "key": r.key, "agg": r.agg, "pres": r.pres,
        "vertex_mask": r.vertex_mask, "links": r.links,
        "mapping": tuple(r.mapping[i] for i in range(k) if r.status == OK) if 1 <= k <= MAX_K else (),
    }


def effbw(x, y, z) -> float:
    """Eq. 2 (predicted effective bandwidth) as the oracle evaluates it."""
    return float(lib().or_effbw(int(x), int(y), int(z)))


def pattern_edges(kind, k):
    buf = (ctypes.c_int * (2 * MAX_E))()
    ne = lib().or_pattern_edges(int(kind), int(k), buf)
    if ne < 0:
        raise ValueError("bad pattern")
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(ne)]


def aut_count(kind, k, edges=None) -> int:
    if edges is None:
        return int(lib().or_aut_count(int(kind), int(k)))
    e = edge_array(edges)
    return int(lib().or_aut_count_edges(int(k), len(e) // 2, e.ctypes.data))


def pad_topologies(topologies):
    T = len(topologies)
    tn = np.array([t.shape[0] for t in topologies], dtype=np.int32)
    tw = np.zeros((T, MAX_N, MAX_N), dtype=np.uint8)
    for i, t in enumerate(topologies):
        n = t.shape[0]
        tw[i, :n, :n] = t
    return tn, tw


def batch(topologies, q_topo, q_busy, kind, k, mode, a, b, nthreads: int | None = None,
          metric=None, edges=None):
    """Evaluate queries independently.  Returns a structured numpy array.
    ``edges``, if given, holds per query an edge list (the pattern of that
    query, ``kind`` ignored) or None (the canonical pattern of ``kind``)."""
    tn, tw = pad_topologies(topologies)
    nq = len(q_topo)
    if metric is None:
        metric = np.zeros(nq, np.uint8)
    q_ne = np.full(nq, -1, np.int32)
    q_edges = np.zeros((nq, 2 * MAX_E), np.int32)
    if edges is not None:
        for i, e in enumerate(edges):
            if e is None:
                continue
            flat = edge_array(e)
            q_ne[i] = len(flat) // 2
            q_edges[i, :len(flat)] = flat[:2 * MAX_E]
    cols = [np.ascontiguousarray(np.asarray(x, dtype=dt)) for x, dt in (
        (q_topo, np.int32), (q_busy, np.uint32), (kind, np.uint8), (k, np.uint8),
        (mode, np.uint8), (a, np.int16), (b, np.int16), (metric, np.uint8))]
    out = np.zeros(nq, dtype=RESULT_DTYPE)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    lib().or_batch(nq, tn.ctypes.data, tw.ctypes.data, *[c.ctypes.data for c in cols],
                   q_ne.ctypes.data, q_edges.ctypes.data, out.ctypes.data, int(nthreads))
    return out


def run_workload(wl, nthreads: int | None = None):
    """Evaluate every query of a synth.Workload against its entry busy masks."""
    q = wl.queries
    srv = q["server"]
    return batch(wl.topologies, wl.server_topo[srv], wl.busy[srv], q["kind"], q["k"],
                 q["mode"], q["a"], q["b"], nthreads, q.get("metric"))


def run_batch_semantics(wl, nthreads: int | None = None):
    """Evaluate a batch, then apply commits (see module docstring).

    Returns (results, handles int64 [nq], busy_after uint32 [S])."""
    res = run_workload(wl, nthreads)
    q = wl.queries
    busy = wl.busy.copy()
    handles = np.full(wl.nq, -1, dtype=np.int64)
    seen = set()
    for i in range(wl.nq):
        if not q["commit"][i]:
            continue
        if res["status"][i] < 0:      # malformed query: never claims a server
            continue
        s = int(q["server"][i])
        first = s not in seen
        seen.add(s)
        if res["status"][i] != OK:
            continue
        if not first:
            res["status"][i] = CONFLICT
            continue
        m = int(res["vertex_mask"][i])
        busy[s] |= np.uint32(m)
        handles[i] = (s << 32) | m
    return res, handles, busy
