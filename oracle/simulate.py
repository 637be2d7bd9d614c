"""Job-trace simulator of Sec. 5.2 -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` and the CPU-baseline leg of ``bench.py`` may import this
module; the library's simulator (mapa_simulate) shares no code with it.

The paper's simulation framework: a job file lists jobs (id, number of GPUs,
application pattern, bandwidth sensitivity, execution time); a dispatcher
puts each job into a first-in first-out job queue; whenever the hardware has
room for the job at the head of the queue, the allocation policy places it;
the execution engine is cycle based: an allocated job marks its GPUs busy at
its start cycle and, once its execution time has elapsed, frees them again
(the Job Finished Signal that updates the allocator's hardware state) and
the logger records the job with its predicted effective bandwidth (Eq. 2).

Policies (Sec. 4 and the evaluation's comparison policies):
  PRESERVE  Alg. 1: bandwidth-sensitive jobs take the match of largest
            predicted effective bandwidth (Eq. 2), the others the match of
            largest PreservedBW (Eq. 3);
  GREEDY    the match of largest AggBW (Eq. 1);
  BASELINE  the lowest free GPU ids (pattern vertex i on the i-th lowest).
Every match is an injective map into the free GPUs (the hardware graph is
fully connected through the host, Sec. 3.2); ties go to the
lexicographically smallest mapping.

Readings where the paper is silent:
  * within one cycle, finished jobs free their GPUs first, then arrivals
    join the queue, then the head of the queue is placed repeatedly while it
    fits (a job that fits as soon as GPUs free up starts in that cycle);
  * a job that needs more GPUs than its server can ever offer (more than the
    GPUs not reserved at the start) is logged as not placeable when it
    arrives and leaves the queue, so it cannot block the queue forever;
  * the log reports start and finish cycles, the chosen GPUs and mapping,
    AggBW and PreservedBW at the start cycle and round(1000 * EffBW) with
    the link mix (x double NVLinks, y single NVLinks, z PCIe links).
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np

from . import A2A, MODE_ALL, METRIC_EFFBW, METRIC_WEIGHTED, NOFIT, OK, RING, TREE  # noqa: F401
from . import effbw, pattern_edges, query

POLICY_PRESERVE, POLICY_GREEDY, POLICY_BASELINE = 0, 1, 2

LOG_FIELDS = ("id", "status", "start", "finish", "vertex_mask", "mapping", "agg", "pres",
              "effbw_milli", "links")


def round_half_away(v: float) -> int:
    return int(math.floor(abs(v) + 0.5)) * (1 if v >= 0 else -1)


def score_mapping(W, busy, kind, k, mapping):
    """AggBW (Eq. 1), PreservedBW (Eq. 3), link mix and round(1000 * EffBW)
    (Eq. 2) of one mapping placed on a server with busy mask `busy`."""
    n = W.shape[0]
    edges = pattern_edges(kind, k)
    agg = sum(int(W[mapping[p], mapping[q]]) for p, q in edges)
    x = sum(1 for p, q in edges if W[mapping[p], mapping[q]] == 2)
    y = sum(1 for p, q in edges if W[mapping[p], mapping[q]] == 1)
    z = len(edges) - x - y
    chosen = set(mapping)
    left = [v for v in range(n) if not (busy >> v) & 1 and v not in chosen]
    pres = sum(int(W[u, v]) for i, u in enumerate(left) for v in left[i + 1:])
    return agg, pres, x | (y << 8) | (z << 16), round_half_away(1000.0 * effbw(x, y, z))


def place(W, busy, job, policy):
    """The policy's mapping for `job` on free GPUs ~busy (k must fit)."""
    n = W.shape[0]
    k, kind = int(job["k"]), int(job["kind"])
    if policy == POLICY_BASELINE:
        free = [v for v in range(n) if not (busy >> v) & 1]
        return tuple(free[:k]), None
    if policy == POLICY_GREEDY:
        r = query(W, busy, kind, k, MODE_ALL, a=1, b=0)
    elif job["sensitive"]:
        r = query(W, busy, kind, k, MODE_ALL, metric=METRIC_EFFBW)
    else:
        r = query(W, busy, kind, k, MODE_ALL, a=0, b=1)
    assert r["status"] == OK
    return tuple(int(v) for v in r["mapping"]), r


def simulate(W, busy0: int, jobs, policy: int):
    """Run one job file (a sequence of records with id, arrival, duration,
    kind, k, sensitive; arrivals non-decreasing) on one server whose GPUs in
    busy0 stay reserved.  Returns the per-job log, in job-file order, as a
    list of dicts with LOG_FIELDS."""
    W = np.asarray(W, dtype=np.uint8)
    n = W.shape[0]
    capacity = n - bin(busy0).count("1")
    logs = [None] * len(jobs)
    busy = busy0
    queue = deque()
    running = []  # (finish cycle, job index, vertex mask)
    nxt = 0
    t = 0
    while True:
        # Job Finished Signal: jobs whose execution time has elapsed free their GPUs
        still = []
        for fin, j, mask in running:
            if fin <= t:
                busy &= ~mask
            else:
                still.append((fin, j, mask))
        running = still
        # dispatcher: jobs that have arrived join the FIFO queue
        while nxt < len(jobs) and int(jobs[nxt]["arrival"]) <= t:
            job = jobs[nxt]
            if int(job["k"]) > capacity:
                logs[nxt] = {"id": int(job["id"]), "status": NOFIT, "start": -1, "finish": -1,
                             "vertex_mask": 0, "mapping": (), "agg": 0, "pres": 0,
                             "effbw_milli": 0, "links": 0}
            else:
                queue.append(nxt)
            nxt += 1
        # allocation: the head of the queue, as long as it fits
        while queue:
            j = queue[0]
            job = jobs[j]
            k = int(job["k"])
            if k > n - bin(busy).count("1"):
                break
            mapping, r = place(W, busy, job, policy)
            agg, pres, links, eff = score_mapping(W, busy, int(job["kind"]), k, mapping)
            if r is not None:  # the query's own scores agree with the recomputation
                assert (r["agg"], r["pres"]) == (agg, pres)
            mask = 0
            for v in mapping:
                mask |= 1 << v
            busy |= mask
            fin = t + int(job["duration"])
            running.append((fin, j, mask))
            logs[j] = {"id": int(job["id"]), "status": OK, "start": t, "finish": fin,
                       "vertex_mask": mask, "mapping": mapping, "agg": agg, "pres": pres,
                       "effbw_milli": eff, "links": links}
            queue.popleft()
        # next cycle with an event (idle cycles change nothing)
        nexts = [fin for fin, _, _ in running]
        if nxt < len(jobs):
            nexts.append(int(jobs[nxt]["arrival"]))
        if not nexts:
            assert not queue
            break
        t = max(t + 1, min(nexts))
    return logs
