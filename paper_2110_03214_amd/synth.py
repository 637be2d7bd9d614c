"""Seeded synthetic workloads for the MAPA allocation hot path.

This module only *generates inputs*: server topologies (symmetric weight
matrices whose entries are link counts, 0 = no direct link), busy masks, query
records and request traces.  It holds none of the method's arithmetic (no
pattern edges, no scores, no enumeration), so both the CPU oracle and the GPU
library can consume its output without sharing any computation.

Weight matrices follow the paper's hardware graph (Sec. 3.2): vertices are
accelerators, the label of a pair is its highest link bandwidth.  Following
Table "Peak Bandwidths per link", a pair joined by two NVLinks carries twice the
bandwidth of a single link, so link counts are proportional to bandwidth; a pair
with no direct link is weighted 0 here (the paper routes it over PCIe).

Every stream derives from ``SeedSequence([0x2110_0321, config_id])`` and is
spawned into named children (topology, busy, pattern, arrival, hold) so that a
change to one stream's consumption never perturbs another.

Config ids 1..5 are the five workloads: a tiny single-topology set, a 65,536
state batch, a large 16-vertex enumeration, and two request traces for the
serving loop.  Their exact recipes are documented in each builder below.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import itertools

import numpy as np

SEED_ROOT = 0x2110_0321

# stream slots of the SeedSequence spawn
S_TOPO, S_BUSY, S_PATTERN, S_ARRIVAL, S_HOLD = range(5)

# pattern kinds and modes, as small integers shared by every consumer
RING, ALL_TO_ALL, TREE = 0, 1, 2
MODE_ALL, MODE_LINKED = 0, 1


def streams(config_id: int, n: int = 5):
    ss = np.random.SeedSequence([SEED_ROOT, int(config_id)])
    return [np.random.default_rng(s) for s in ss.spawn(n)]


# ---------------------------------------------------------------------------
# topology edge lists (input data)
# ---------------------------------------------------------------------------

def cube_mesh_edges():
    """8-vertex hybrid cube-mesh: K4 on {0..3}, K4 on {4..7}, rungs i--i+4."""
    e = [(u, v) for u, v in itertools.combinations(range(4), 2)]
    e += [(u + 4, v + 4) for u, v in itertools.combinations(range(4), 2)]
    e += [(i, i + 4) for i in range(4)]
    return e


def two_socket_edges():
    """6-vertex two-socket layout: two K3 cliques joined by rungs i--i+3.

    Returns (clique_edges, cross_edges)."""
    clique = [(0, 1), (0, 2), (1, 2), (3, 4), (3, 5), (4, 5)]
    cross = [(i, i + 3) for i in range(3)]
    return clique, cross


def hypercube_edges(dim: int = 4):
    n = 1 << dim
    return [(u, u ^ (1 << b)) for u in range(n) for b in range(dim) if u < (u ^ (1 << b))]


def _sym(n, edges, weights):
    W = np.zeros((n, n), dtype=np.uint8)
    for (u, v), w in zip(edges, weights):
        W[u, v] = W[v, u] = w
    return W


# ---------------------------------------------------------------------------
# workload container
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    """A batch of allocation queries over device-resident server states.

    topologies  : list of uint8 [n, n] symmetric weight matrices (diag 0)
    server_topo : int32 [S]  topology index of each server
    busy        : uint32 [S] busy mask of each server at batch entry
    queries     : dict of equal-length columns
                  server (int32), kind (uint8), k (uint8), mode (uint8),
                  commit (uint8), a (int16), b (int16)
    """
    name: str
    topologies: list
    server_topo: np.ndarray
    busy: np.ndarray
    queries: dict
    meta: dict = field(default_factory=dict)

    @property
    def nq(self) -> int:
        return int(self.queries["server"].shape[0])

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx)
        q = {key: col[idx].copy() for key, col in self.queries.items()}
        return Workload(self.name + "[sub]", self.topologies, self.server_topo,
                        self.busy, q, dict(self.meta))

    def with_keys(self, a: int, b: int, mode: int | None = None) -> "Workload":
        q = {key: col.copy() for key, col in self.queries.items()}
        q["a"][:] = a
        q["b"][:] = b
        if mode is not None:
            q["mode"][:] = mode
        return Workload(f"{self.name}(a={a},b={b})", self.topologies, self.server_topo,
                        self.busy, q, dict(self.meta))


def make_queries(server, kind, k, mode=MODE_ALL, commit=0, a=1, b=1, metric=0):
    nq = len(server)

    def col(x, dt):
        arr = np.empty(nq, dtype=dt)
        arr[:] = x
        return arr

    return {
        "server": col(server, np.int32),
        "kind": col(kind, np.uint8),
        "k": col(k, np.uint8),
        "mode": col(mode, np.uint8),
        "commit": col(commit, np.uint8),
        "a": col(a, np.int16),
        "b": col(b, np.int16),
        "metric": col(metric, np.uint8),
    }


def random_busy(rng, n: int, nbusy: int) -> int:
    """Uniform nbusy-subset of range(n) as a bit mask."""
    if nbusy <= 0:
        return 0
    chosen = rng.choice(n, size=min(nbusy, n), replace=False)
    m = 0
    for v in chosen:
        m |= 1 << int(v)
    return m


# ---------------------------------------------------------------------------
# configs
# ---------------------------------------------------------------------------

def config1(nq: int = 1000) -> Workload:
    """Tiny: one 8-vertex cube-mesh, edge weights U{1,2}; nq queries, each on
    its own server state with U{0..4} busy vertices; ring k=4, ALL mode,
    key weights (1,1)."""
    rt, rb, _, _, _ = streams(1)
    edges = cube_mesh_edges()
    W = _sym(8, edges, rt.integers(1, 3, size=len(edges)))
    busy = np.array([random_busy(rb, 8, int(rb.integers(0, 5))) for _ in range(nq)],
                    dtype=np.uint32)
    q = make_queries(np.arange(nq), RING, 4)
    return Workload("C1", [W], np.zeros(nq, np.int32), busy, q,
                    {"config": 1})


def config2_topologies():
    """The three topologies of the batched and serving configs:
    0: cube-mesh, all weights 1
    1: cube-mesh, a seeded 8 of its 16 edges weight 2, the rest 1
    2: 6-vertex two-socket: two K3 cliques of weight 2, rungs of weight 1"""
    rt = streams(2)[S_TOPO]
    edges = cube_mesh_edges()
    t0 = _sym(8, edges, [1] * len(edges))
    heavy = set(int(i) for i in rt.permutation(len(edges))[:len(edges) // 2])
    t1 = _sym(8, edges, [2 if i in heavy else 1 for i in range(len(edges))])
    clique, cross = two_socket_edges()
    t2 = _sym(6, clique + cross, [2] * len(clique) + [1] * len(cross))
    return [t0, t1, t2]


def config2(nq: int = 65536) -> Workload:
    """Batched: nq independent server states, topology U over the three above,
    U{0..6} busy vertices (a uniform subset), kind U{ring, a2a, tree},
    k U{2..8}; ALL mode, key weights (1,1)."""
    _, rb, rp, _, _ = streams(2)
    topos = config2_topologies()
    tid = rb.integers(0, 3, size=nq).astype(np.int32)
    nb = rb.integers(0, 7, size=nq)
    busy = np.array([random_busy(rb, topos[t].shape[0], int(b)) for t, b in zip(tid, nb)],
                    dtype=np.uint32)
    kind = rp.integers(0, 3, size=nq)
    k = rp.integers(2, 9, size=nq)
    q = make_queries(np.arange(nq), kind, k)
    return Workload("C2", topos, tid, busy, q, {"config": 2})


def config3_topology(rng) -> np.ndarray:
    """16-vertex: 4-D hypercube edges with weight U{1,2,3}, plus 8 distinct
    extra chords (uniform over the non-hypercube pairs) of weight 1."""
    hc = hypercube_edges(4)
    W = _sym(16, hc, rng.integers(1, 4, size=len(hc)))
    hcs = set(hc)
    others = [(u, v) for u, v in itertools.combinations(range(16), 2) if (u, v) not in hcs]
    pick = rng.choice(len(others), size=8, replace=False)
    for i in pick:
        u, v = others[int(i)]
        W[u, v] = W[v, u] = 1
    return W


def config3_topologies(count: int = 256):
    rt = streams(3)[S_TOPO]
    return [config3_topology(rt) for _ in range(count)]


def config3(ntopo: int = 256, ks=(6, 7, 8), kinds=(RING, ALL_TO_ALL)) -> Workload:
    """Large: ntopo independently seeded 16-vertex topologies, all vertices
    free; for each topology, kinds {ring, a2a} x k in {6,7,8} (1,536 queries
    at full size).  Up to 16!/8! embeddings per query."""
    topos = config3_topologies(ntopo)
    srv, kd, kk = [], [], []
    for t in range(ntopo):
        for kind in kinds:
            for k in ks:
                srv.append(t)
                kd.append(kind)
                kk.append(k)
    q = make_queries(srv, kd, kk)
    return Workload("C3", topos, np.arange(ntopo, dtype=np.int32),
                    np.zeros(ntopo, np.uint32), q, {"config": 3})


def config6_topology(rng) -> np.ndarray:
    """32-vertex: 5-D hypercube edges with weight U{1,2,3}, plus 16 distinct
    extra chords (uniform over the non-hypercube pairs) of weight 1."""
    hc = hypercube_edges(5)
    W = _sym(32, hc, rng.integers(1, 4, size=len(hc)))
    hcs = set(hc)
    others = [(u, v) for u, v in itertools.combinations(range(32), 2) if (u, v) not in hcs]
    pick = rng.choice(len(others), size=16, replace=False)
    for i in pick:
        u, v = others[int(i)]
        W[u, v] = W[v, u] = 1
    return W


def config6(nserv: int = 16, free: int = 12, ks=(9, 10), kinds=(RING, ALL_TO_ALL, TREE)) -> Workload:
    """Wide: nserv independently seeded 32-vertex topologies, each server
    with `free` accelerators free (a uniform subset, the rest busy); kinds x
    ks queries per server (jobs of 9 and 10 accelerators)."""
    rt, rb = streams(6)[S_TOPO], streams(6)[S_BUSY]
    topos = [config6_topology(rt) for _ in range(nserv)]
    busy = np.empty(nserv, np.uint32)
    for t in range(nserv):
        fr = rb.choice(32, size=free, replace=False)
        busy[t] = np.uint32(0xFFFFFFFF & ~int(np.bitwise_or.reduce(1 << fr.astype(np.int64))))
    srv, kd, kk = [], [], []
    for t in range(nserv):
        for kind in kinds:
            for k in ks:
                srv.append(t)
                kd.append(kind)
                kk.append(k)
    q = make_queries(srv, kd, kk)
    return Workload("C6", topos, np.arange(nserv, dtype=np.int32), busy, q, {"config": 6})


# ---------------------------------------------------------------------------
# serving traces
# ---------------------------------------------------------------------------

@dataclass
class Trace:
    """Request trace for the serving loop.

    Each request asks for an allocation at t_arrival; if it is granted the
    allocation is held for ``hold`` time units and then released.
    """
    name: str
    topologies: list
    server_topo: np.ndarray
    t_arrival: np.ndarray      # float64, non-decreasing
    server: np.ndarray         # int32
    kind: np.ndarray           # uint8
    k: np.ndarray              # uint8
    hold: np.ndarray           # float64
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.server.shape[0])

    def head(self, n: int) -> "Trace":
        return Trace(self.name + f"[:{n}]", self.topologies, self.server_topo,
                     self.t_arrival[:n], self.server[:n], self.kind[:n], self.k[:n],
                     self.hold[:n], dict(self.meta))


def config4(nreq: int = 1_000_000, rate: float = 46.0) -> Trace:
    """Serving: 4,096 servers (topology = id mod 3 over the batched config's
    three topologies), all free at t=0; Poisson arrivals at ``rate`` per time
    unit; server U{0..4095}; kind U{3}; k ~ pmf proportional to
    (1,4,1,4,1,1,1,4) over k=1..8; hold Exp(mean 100)."""
    _, _, rp, ra, rh = streams(4)
    topos = config2_topologies()
    S = 4096
    st = (np.arange(S) % 3).astype(np.int32)
    t = np.cumsum(ra.exponential(1.0 / rate, size=nreq))
    server = rp.integers(0, S, size=nreq).astype(np.int32)
    kind = rp.integers(0, 3, size=nreq).astype(np.uint8)
    pmf = np.array([1, 4, 1, 4, 1, 1, 1, 4], dtype=np.float64)
    k = (rp.choice(8, size=nreq, p=pmf / pmf.sum()) + 1).astype(np.uint8)
    hold = rh.exponential(100.0, size=nreq)
    return Trace("C4", topos, st, t, server, kind, k, hold,
                 {"config": 4, "rate": rate})


def config5(nreq: int = 200_000, mean_rate: float = 38.0) -> Trace:
    """Mixed-size serving stress: 1,024 servers of the seeded half-weight-2
    cube-mesh and 1,024 servers of 16-vertex hypercube-plus-chords topologies
    (server 1024+j uses the j mod 256-th topology of the large config);
    two-state Markov-modulated Poisson arrivals (rates 0.5x and 4x the mean
    rate, state sojourns Exp(1000) and Exp(200) time units); k U{1..8};
    kind U{3}; hold Exp(100)."""
    _, _, rp, ra, rh = streams(5)
    cm = config2_topologies()[1]
    big = config3_topologies(256)
    topos = [cm] + big
    S = 2048
    st = np.concatenate([np.zeros(1024, np.int32),
                         1 + (np.arange(1024) % 256).astype(np.int32)])
    lam = (0.5 * mean_rate, 4.0 * mean_rate)
    soj = (1000.0, 200.0)
    times = np.empty(nreq)
    t, state, i = 0.0, 0, 0
    t_switch = ra.exponential(soj[0])
    while i < nreq:
        dt = ra.exponential(1.0 / lam[state])
        if t + dt >= t_switch:
            t = t_switch
            state ^= 1
            t_switch = t + ra.exponential(soj[state])
            continue
        t += dt
        times[i] = t
        i += 1
    server = rp.integers(0, S, size=nreq).astype(np.int32)
    kind = rp.integers(0, 3, size=nreq).astype(np.uint8)
    k = rp.integers(1, 9, size=nreq).astype(np.uint8)
    hold = rh.exponential(100.0, size=nreq)
    return Trace("C5", topos, st, times, server, kind, k, hold,
                 {"config": 5, "mean_rate": mean_rate})



# ---------------------------------------------------------------------------
# job files for the trace simulator (Sec. 5.2)
# ---------------------------------------------------------------------------

def dgx1v_topology() -> np.ndarray:
    """DGX-1 V100 (8 GPUs, hybrid cube-mesh), NVLink counts per pair, 0 = PCIe
    only: the cells the paper's text fixes (GPUs 1-5 double, 1-2 single, 1-6
    and 2-5 PCIe, GPUs 1, 3, 4 one single and two doubles) and the publicly
    documented layout for the rest (every GPU uses its six NVLink ports).
    Vertex index = paper GPU id - 1."""
    double = [(0, 3), (0, 4), (1, 2), (1, 5), (2, 3), (4, 7), (5, 6), (6, 7)]
    single = [(0, 1), (0, 2), (1, 3), (2, 6), (3, 7), (4, 5), (4, 6), (5, 7)]
    return _sym(8, double + single, [2] * len(double) + [1] * len(single))


def torus2d_16_topology(rng) -> np.ndarray:
    """16 GPUs on a 4 x 4 torus (each joined to its four grid neighbours,
    wrapping around), a seeded half of the 32 links double, the rest single;
    every other pair PCIe only."""
    edges = sorted({tuple(sorted((4 * r + c, 4 * r + (c + 1) % 4))) for r in range(4) for c in range(4)} |
                   {tuple(sorted((4 * r + c, 4 * ((r + 1) % 4) + c))) for r in range(4) for c in range(4)})
    heavy = set(int(i) for i in rng.permutation(len(edges))[:len(edges) // 2])
    return _sym(16, edges, [2 if i in heavy else 1 for i in range(len(edges))])


def cubemesh_16_topology(rng) -> np.ndarray:
    """16 GPUs as two 8-GPU hybrid cube-meshes (each with a seeded half of its
    16 links double) joined by single links i--i+8; every other pair PCIe."""
    e8 = cube_mesh_edges()
    edges, w = [], []
    for base in (0, 8):
        heavy = set(int(i) for i in rng.permutation(len(e8))[:len(e8) // 2])
        edges += [(u + base, v + base) for u, v in e8]
        w += [2 if i in heavy else 1 for i in range(len(e8))]
    edges += [(i, i + 8) for i in range(8)]
    w += [1] * 8
    return _sym(16, edges, w)


@dataclass
class JobFiles:
    """Simulations for the trace simulator: simulation i runs job file
    ``jobs[offsets[i]:offsets[i+1]]`` on a server of topology ``sim_topo[i]``
    under policy ``policy[i]`` (0 Preserve, 1 Greedy, 2 lowest ids)."""
    name: str
    topologies: list
    sim_topo: np.ndarray   # int32 per simulation
    policy: np.ndarray     # int32 per simulation
    offsets: np.ndarray    # int32, nsim + 1
    jobs: np.ndarray       # structured: id, arrival, duration, kind, k, sensitive
    meta: dict = field(default_factory=dict)

    @property
    def nsim(self) -> int:
        return int(self.sim_topo.shape[0])

    def subset(self, idx) -> "JobFiles":
        idx = np.asarray(idx)
        parts = [self.jobs[self.offsets[i]:self.offsets[i + 1]] for i in idx]
        off = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int32)
        return JobFiles(self.name + "[sub]", self.topologies, self.sim_topo[idx], self.policy[idx],
                        off, np.concatenate(parts) if parts else self.jobs[:0], dict(self.meta))


JOB_DTYPE = np.dtype([("id", np.int32), ("arrival", np.int32), ("duration", np.int32),
                      ("kind", np.uint8), ("k", np.uint8), ("sensitive", np.uint8),
                      ("reserved", np.uint8)])


def job_file(rng, njobs: int = 300, kmax: int = 5, dmin: int = 100, dmax: int = 1000,
             mean_gap: float = 0.0) -> np.ndarray:
    """One job file: njobs jobs asking U{1..kmax} GPUs (the paper's jobs ask
    1 to 5, uniformly), pattern U{ring, all-to-all, tree}, bandwidth-sensitive
    with probability 1/2, execution time U{dmin..dmax} cycles; all queued at
    cycle 0 (mean_gap = 0, the paper's FIFO job file) or Poisson arrivals
    with that mean gap in cycles."""
    j = np.zeros(njobs, dtype=JOB_DTYPE)
    j["id"] = np.arange(njobs)
    if mean_gap > 0:
        j["arrival"] = np.floor(np.cumsum(rng.exponential(mean_gap, size=njobs))).astype(np.int32)
    j["duration"] = rng.integers(dmin, dmax + 1, size=njobs)
    j["kind"] = rng.integers(0, 3, size=njobs)
    j["k"] = rng.integers(1, kmax + 1, size=njobs)
    j["sensitive"] = rng.integers(0, 2, size=njobs)
    return j


def config7(files_per_topology: int = 16, njobs: int = 300) -> JobFiles:
    """Trace simulation: three hardware graphs (DGX-1 V100; 16-GPU torus-2d;
    16-GPU two-cube-mesh), each with ``files_per_topology`` seeded job files
    of ``njobs`` jobs (job_file defaults), every file run under each of the
    three policies: 3 x files x 3 simulations."""
    rt, _, rp, _, _ = streams(7)
    topos = [dgx1v_topology(), torus2d_16_topology(rt), cubemesh_16_topology(rt)]
    files = [[job_file(rp, njobs) for _ in range(files_per_topology)] for _ in topos]
    sim_topo, policy, parts = [], [], []
    for t in range(len(topos)):
        for f in files[t]:
            for pol in (0, 1, 2):
                sim_topo.append(t)
                policy.append(pol)
                parts.append(f)
    off = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int32)
    return JobFiles("C7", topos, np.array(sim_topo, np.int32), np.array(policy, np.int32), off,
                    np.concatenate(parts), {"config": 7})
