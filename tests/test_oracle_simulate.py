"""Pins of the oracle's job-trace simulator (Sec. 5.2; policies of Sec. 4).

What fixes the simulator independently of its own code:
  * closed forms: jobs that each need the whole server run one after another
    under every policy (start = sum of the earlier durations);
  * hand-derived traces on the DGX-1 V100 (NVLink counts of the worked
    example): lowest-id placement and the cycle a blocked head starts in;
  * the paper's printed numbers: the first 3-GPU ring under Greedy and under
    Preserve (bandwidth-sensitive) on the idle DGX-1 V100 is the "ideal"
    GPUs 1, 3, 4 with one single and two double NVLinks, whose predicted
    effective bandwidth the paper prints as 57.85;
  * a second simulator written differently (it ticks every cycle and places
    jobs with the itertools brute force) agrees job for job on random tiny
    job files under all three policies;
  * invariants on random job files (FIFO start order, no GPU in two running
    jobs, start >= arrival, finish = start + duration);
  * planted mistakes (allocating before freeing, backfilling past a blocked
    head, the Greedy key for insensitive jobs) each fail a pin.
"""
import os
import random
from collections import deque

import numpy as np
import pytest

import oracle
from oracle import brute
from oracle import simulate as sim

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dgx1v():
    rows, on = [], False
    with open(os.path.join(GOLDEN, "dgx1v_worked_example.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line == "nvlink_counts":
                on = True
            elif line == "end":
                on = False
            elif on and line:
                rows.append([int(x) for x in line.split()])
    return np.array(rows, dtype=np.uint8)


def jobs_of(rows):
    """rows: (arrival, duration, kind, k, sensitive); ids count from 0."""
    return [{"id": i, "arrival": a, "duration": d, "kind": kd, "k": k, "sensitive": s}
            for i, (a, d, kd, k, s) in enumerate(rows)]


@pytest.fixture(scope="module", autouse=True)
def _built(orc):
    return orc


def test_whole_server_jobs_run_back_to_back():
    W = dgx1v()
    durs = [7, 3, 11, 1, 5]
    jobs = jobs_of([(0, d, j % 3, 8, j % 2) for j, d in enumerate(durs)])
    for pol in (sim.POLICY_PRESERVE, sim.POLICY_GREEDY, sim.POLICY_BASELINE):
        logs = sim.simulate(W, 0, jobs, pol)
        t = 0
        for d, lg in zip(durs, logs):
            assert (lg["start"], lg["finish"], lg["vertex_mask"]) == (t, t + d, 0xFF)
            t += d


def test_baseline_lowest_ids_and_blocked_head_by_hand():
    W = dgx1v()
    # k=3 (10 cycles), k=2 (5 cycles), k=4 (3 cycles): the third waits for the
    # second to finish at cycle 5, then takes GPUs 3..6
    jobs = jobs_of([(0, 10, oracle.RING, 3, 0), (0, 5, oracle.RING, 2, 0), (0, 3, oracle.RING, 4, 0)])
    logs = sim.simulate(W, 0, jobs, sim.POLICY_BASELINE)
    assert [lg["mapping"] for lg in logs] == [(0, 1, 2), (3, 4), (3, 4, 5, 6)]
    assert [(lg["start"], lg["finish"]) for lg in logs] == [(0, 10), (0, 5), (5, 8)]
    # ring on GPUs 1, 2, 3: links 1-2 single, 2-3 double, 3-1 single
    assert logs[0]["agg"] == 4 and logs[0]["links"] == 1 | (2 << 8)
    # a reserved GPU stays busy; a job larger than the rest is not placeable
    logs = sim.simulate(W, 0b1, jobs_of([(0, 4, oracle.RING, 8, 0), (2, 4, oracle.RING, 2, 0)]),
                        sim.POLICY_BASELINE)
    assert logs[0]["status"] == oracle.NOFIT and logs[0]["start"] == -1
    assert logs[1]["mapping"] == (1, 2) and logs[1]["start"] == 2


def test_paper_ideal_three_gpu_allocation_and_its_effective_bandwidth():
    """Sec. 2.2: GPUs 1, 3, 4 (one single, two double NVLinks) are the ideal
    3-GPU allocation; Sec. 5.1 prints 57.85 GB/s as the predicted effective
    bandwidth of that mix (x = 2, y = 1, z = 0)."""
    W = dgx1v()
    for pol, sens in ((sim.POLICY_GREEDY, 0), (sim.POLICY_PRESERVE, 1)):
        lg = sim.simulate(W, 0, jobs_of([(0, 9, oracle.RING, 3, sens)]), pol)[0]
        assert lg["mapping"] == (0, 2, 3), pol
        assert lg["links"] == 2 | (1 << 8)
        assert lg["effbw_milli"] // 10 == 5785  # printed to two decimals: 57.85
    # Preserve, insensitive 1-GPU job with GPU 1 reserved: every GPU has six
    # NVLinks, so the weight left among the other seven is 24 - 6 = 18 and
    # placing v preserves 18 - (6 - W[v][0]); GPUs 4 and 5 share a double
    # NVLink with GPU 1, so GPU 4 (index 3) preserves 14.  Greedy scores every
    # single GPU 0 and takes the lowest free id, GPU 2.
    lg = sim.simulate(W, 0b1, jobs_of([(0, 9, oracle.RING, 1, 0)]), sim.POLICY_PRESERVE)[0]
    assert lg["mapping"] == (3,) and lg["pres"] == 14
    lg = sim.simulate(W, 0b1, jobs_of([(0, 9, oracle.RING, 1, 0)]), sim.POLICY_GREEDY)[0]
    assert lg["mapping"] == (1,) and lg["pres"] == 13


def tick_reference(W, busy0, jobs, policy):
    """Second simulator: one iteration per cycle, placements by brute force."""
    n = len(W)
    cap = n - bin(busy0).count("1")
    logs = [None] * len(jobs)
    busy, queue, running, nxt, t = busy0, deque(), [], 0, 0
    while nxt < len(jobs) or queue or running:
        for r in [r for r in running if r[0] == t]:
            busy &= ~r[1]
        running = [r for r in running if r[0] != t]
        while nxt < len(jobs) and jobs[nxt]["arrival"] == t:
            if jobs[nxt]["k"] > cap:
                logs[nxt] = ("nofit",)
            else:
                queue.append(nxt)
            nxt += 1
        while queue and jobs[queue[0]]["k"] <= n - bin(busy).count("1"):
            j = queue.popleft()
            job = jobs[j]
            free = [v for v in range(n) if not (busy >> v) & 1]
            if policy == sim.POLICY_BASELINE:
                phi = tuple(free[:job["k"]])
            elif policy == sim.POLICY_GREEDY:
                phi = brute.query(W, busy, job["kind"], job["k"], 0, 1, 0)["mapping"]
            elif job["sensitive"]:
                phi = brute.query(W, busy, job["kind"], job["k"], 0, metric=1)["mapping"]
            else:
                phi = brute.query(W, busy, job["kind"], job["k"], 0, 0, 1)["mapping"]
            m = sum(1 << v for v in phi)
            busy |= m
            running.append((t + job["duration"], m))
            logs[j] = (t, t + job["duration"], phi)
        t += 1
    return logs


def random_topology(rng, n):
    W = np.zeros((n, n), np.uint8)
    for u in range(n):
        for v in range(u + 1, n):
            W[u, v] = W[v, u] = rng.choice([0, 1, 2])
    return W


def random_jobs(rng, count, kmax, arrival_gap=3, dmax=12):
    rows, t = [], 0
    for _ in range(count):
        t += rng.randrange(0, arrival_gap + 1)
        rows.append((t, rng.randrange(1, dmax + 1), rng.randrange(3), rng.randrange(1, kmax + 1),
                     rng.randrange(2)))
    return jobs_of(rows)


@pytest.mark.parametrize("seed", range(6))
def test_agrees_with_cycle_by_cycle_brute_force(seed):
    rng = random.Random(seed)
    n = rng.choice([4, 5, 6])
    W = random_topology(rng, n)
    busy0 = rng.choice([0, 0, 1 << rng.randrange(n)])
    jobs = random_jobs(rng, 14, n)
    for pol in (sim.POLICY_PRESERVE, sim.POLICY_GREEDY, sim.POLICY_BASELINE):
        got = sim.simulate(W, busy0, jobs, pol)
        ref = tick_reference(W, busy0, jobs, pol)
        for lg, r in zip(got, ref):
            if r == ("nofit",):
                assert lg["status"] == oracle.NOFIT
            else:
                assert (lg["start"], lg["finish"], lg["mapping"]) == r, (pol, lg, r)


def check_invariants(W, busy0, jobs, logs):
    n = W.shape[0]
    placed = [(lg, j) for lg, j in zip(logs, jobs) if lg["status"] == oracle.OK]
    starts = [lg["start"] for lg, _ in placed]
    assert starts == sorted(starts), "FIFO: a later job started before an earlier one"
    for lg, j in placed:
        assert lg["start"] >= j["arrival"] and lg["finish"] == lg["start"] + j["duration"]
        assert bin(lg["vertex_mask"]).count("1") == j["k"] and not lg["vertex_mask"] & busy0
    events = sorted({lg["start"] for lg, _ in placed})
    for t in events:
        live = [lg["vertex_mask"] for lg, _ in placed if lg["start"] <= t < lg["finish"]]
        acc = 0
        for m in live:
            assert not acc & m, "a GPU in two running jobs"
            acc |= m
        assert bin(acc).count("1") <= n - bin(busy0).count("1")


@pytest.mark.parametrize("seed", range(3))
def test_invariants_on_random_job_files(seed):
    rng = random.Random(100 + seed)
    W = dgx1v()
    jobs = random_jobs(rng, 60, 5, arrival_gap=2, dmax=30)
    for pol in (sim.POLICY_PRESERVE, sim.POLICY_GREEDY, sim.POLICY_BASELINE):
        logs = sim.simulate(W, 0, jobs, pol)
        check_invariants(W, 0, jobs, logs)
        for lg, j in zip(logs, jobs):  # the logged EffBW is Eq. 2 of the logged link mix
            links = lg["links"]
            x, y, z = links & 255, (links >> 8) & 255, links >> 16
            assert x + y + z == len(brute.edges(j["kind"], j["k"]))
            assert lg["effbw_milli"] == sim.round_half_away(1000 * brute.effbw(x, y, z))


def test_pins_catch_planted_mistakes(monkeypatch):
    W = dgx1v()
    hand = jobs_of([(0, 10, oracle.RING, 3, 0), (0, 5, oracle.RING, 2, 0), (0, 3, oracle.RING, 4, 0)])

    def hand_pin():
        logs = sim.simulate(W, 0, hand, sim.POLICY_BASELINE)
        return [(lg["start"], lg["finish"]) for lg in logs] == [(0, 10), (0, 5), (5, 8)]

    def fifo_pin():
        rng = random.Random(7)
        jobs = random_jobs(rng, 60, 5, arrival_gap=1, dmax=30)
        try:
            check_invariants(W, 0, jobs, sim.simulate(W, 0, jobs, sim.POLICY_BASELINE))
            return True
        except AssertionError:
            return False

    def preserve_pin():
        lg = sim.simulate(W, 0b1, jobs_of([(0, 9, oracle.RING, 1, 0)]), sim.POLICY_PRESERVE)[0]
        return lg["mapping"] == (3,) and lg["pres"] == 14

    assert hand_pin() and fifo_pin() and preserve_pin()

    # 1. free the GPUs of finished jobs one cycle late
    real = sim.simulate

    def late_free(W_, busy0, jobs, policy):
        shifted = [dict(j, duration=j["duration"] + 1) for j in jobs]
        logs = real(W_, busy0, shifted, policy)
        for lg in logs:
            if lg["status"] == oracle.OK:
                lg["finish"] -= 1
        return logs
    monkeypatch.setattr(sim, "simulate", late_free)
    assert not hand_pin()
    monkeypatch.setattr(sim, "simulate", real)

    # 2. backfill: skip a blocked head and place a later job that fits
    class Backfill(deque):
        def __getitem__(self, i):
            return deque.__getitem__(self, len(self) - 1 if i == 0 else i)

        def popleft(self):
            return self.pop()
    monkeypatch.setattr(sim, "deque", Backfill)
    assert not fifo_pin()
    monkeypatch.undo()

    # 3. insensitive jobs under Preserve scored with the Greedy key
    real_query = sim.query

    def greedy_query(W_, busy, kind, k, mode=0, a=1, b=1, metric=0, edges=None):
        if metric == oracle.METRIC_WEIGHTED:
            a, b = 1, 0
        return real_query(W_, busy, kind, k, mode, a, b, metric, edges)
    monkeypatch.setattr(sim, "query", greedy_query)
    assert not preserve_pin()
