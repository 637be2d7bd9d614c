#!/usr/bin/env python3
"""Benchmark of the MAPA allocation hot path on one MI355X.

A step is one pass of the whole hot path over one batch: every query of the
workload is answered (free sets and key constants, pattern tables, every
embedding enumerated and scored, best selected with the fixed tie-break),
every successful query commits its allocation, and every committed
allocation is released again, so each step starts from the same busy state.
Queries, results and busy masks stay in HBM; nothing crosses PCIe inside the
timed region.

Headline workload (default): the large enumeration (256 16-vertex
hypercube-plus-chord topologies, all free, ring and all-to-all patterns with
k = 6, 7, 8: 1,536 queries, 2.98e11 embeddings per batch), the paper's
overhead case of large jobs on 16-accelerator hardware graphs (Sec. 5.4).
``--config 2`` makes the batched config the headline, ``--config 1`` the tiny
one, ``--config 6`` the wide path (32-vertex servers, jobs of 9 and 10).

Beside the headline the default run also reports (each skippable):
  * the batched config (65,536 server states) as a timed batch;
  * the plain form: one query per call with host buffers, on both;
  * the serving forms on the serving trace (1M Poisson requests over 4,096
    servers) and the mixed-size bursty trace (1,024 cube-mesh + 1,024
    16-vertex servers): the continuous-batching loop at 0.5 / 0.8 / 1.0 /
    1.2 x its measured capacity, and the plain serving form (one request per
    device batch, one batch in flight) at the same fractions of its own;
  * the trace simulation of Sec. 5.2 (job files on three hardware graphs under
    the Preserve, Greedy and lowest-id policies) with the oracle's simulator;
  * the CPU oracle on the host (single thread and all cores).

Prints ONE JSON line:  value = embeddings scored per second on the headline
workload, plus queries/s, per-batch p50/p99 latency, the roofline of the
enumeration kernel (integer ALU bound) under three operation counts, and the
CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pattern embeddings scored/sec + allocation queries/sec, p50/p99 latency"
# MI355X vector-ALU ceiling for 32-bit lane operations: the published fp32
# vector rate, 157.3 TFLOP/s, is 256 CUs x 2.4 GHz x 128 lanes x 2 flops per
# FMA, so the vector ALUs retire at most 256 x 128 x 2.4e9 = 78.6e12 32-bit
# lane-ops/s.  This is an upper bound for integer work: mapa_measure_alu_peak
# (independent chains of the leaf loop's integer instruction mix) sustains
# about 46e12.
CU, LANES_PER_CLK, CLK = 256, 128, 2.4e9
ALU_PEAK = CU * LANES_PER_CLK * CLK  # 78.64e12 int32 lane-ops/s
PEAK_NOTE = ("78.64 T = the fp32 vector FMA lane rate (157.3 TFLOP/s / 2 flops): an upper bound "
             "for 32-bit integer lane ops; measured_peak is the integer probe's sustained rate")

# Counter profiles (rocprofv3) of the enumeration kernel, committed under
# profiles/; their figures are reported only while the kernel sources still
# hash to the value the profile was taken on.
KERNEL_SOURCES = tuple("paper_2110_03214_amd/csrc/" + f for f in (
    "device.h", "enumerate.h", "enum_pair12_lds.hip", "enum_pair12_glb.hip", "enum_pair6.hip",
    "enum_plain.hip", "mapa_internal.h"))
WIDE_SOURCES = tuple("paper_2110_03214_amd/csrc/" + f for f in ("wide.hip", "wide.h", "mapa_internal.h"))
PMC_PROFILE = {2: "k_enumerate_batched_65536q_pmc.txt", 3: "k_enumerate_large_1536q_pmc.txt",
               6: "k_wide_search_wide_96q_pmc.txt"}

WORKLOAD_TEXT = {
    1: "tiny: 1,000 states of one 8-vertex cube-mesh (weights 1-2), 0-4 busy, ring k=4",
    2: ("batched: 65,536 server states over three topologies (cube-mesh all-1, cube-mesh half "
        "weight-2, 6-vertex two-socket), 0-6 busy, ring/all-to-all/tree with k in 2..8"),
    3: ("large: 256 16-vertex hypercube+chord topologies (weights 1-3), all free, ring and "
        "all-to-all with k in 6..8 (1,536 queries, 2.98e11 embeddings)"),
    6: ("wide: 16 32-vertex 5-cube+chord topologies (weights 1-3), 12 free accelerators each, "
        "ring/all-to-all/tree with k in 9..10 (96 queries, 1.53e10 embeddings; host buffers)"),
}
SERVING_TEXT = {
    4: "serving: Poisson requests over 4,096 servers of the batched config's three topologies",
    5: "mixed serving: bursty (two-state MMPP) requests over 1,024 cube-mesh and 1,024 16-vertex servers",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- op models

def last_back_neighbours(kind: int, k: int) -> int:
    """|Nb[k-1]|: pattern neighbours of the last position among the earlier
    ones (ring: previous and first; all-to-all: all; tree: the parent)."""
    if k <= 1:
        return 0
    if kind == 0:  # ring
        return 1 if k == 2 else 2
    if kind == 1:  # all-to-all
        return k - 1
    return 1  # binary tree


def weight_bits(W) -> int:
    """B = bits of the largest weight (bit-planes a weighted popcount reads)."""
    return max(1, int(np.max(W)).bit_length())


def op_counts(wl) -> dict:
    """Embeddings and three algorithmic integer-op counts of one pass:
      ops_leaf8d : 8 + 3B + |Nb[k-1]| per embedding, plus that per leaf times
                   1/(F-k+1) for the interior nodes (the per-leaf work of an
                   enumerate-and-score method that scores each embedding on
                   its own: candidate test, edge adds, B plane ANDs, popcounts
                   and shift-adds, the preserved-weight lookup, the key and
                   the select);
      ops_factored : 3 per embedding + 4 per interior node at depths 1..k-1
                   (the factored last two positions: a leaf is one weight-field
                   extract, one multiply-add and one max over terms tabulated
                   once per candidate of its parent);
      ops_node4  : 4 per search-tree node at depths 1..k.
    Counts are for ALL mode (every injective map), the headline mode."""
    q = wl.queries
    n_of = [W.shape[0] for W in wl.topologies]
    B_of = [weight_bits(W) for W in wl.topologies]
    emb = o8d = ofac = onode = 0.0
    cache = {}
    for s, kind, k in zip(q["server"], q["kind"], q["k"]):
        t = int(wl.server_topo[s])
        F = n_of[t] - bin(int(wl.busy[s])).count("1")
        key = (F, int(k), int(kind), B_of[t])
        if key not in cache:
            k_ = int(k)
            if k_ > F:
                cache[key] = (0, 0, 0, 0)
            else:
                leaves = math.perm(F, k_)
                per_leaf = 8 + 3 * B_of[t] + last_back_neighbours(int(kind), k_)
                a = leaves * per_leaf * (1.0 + 1.0 / (F - k_ + 1))
                interior = sum(math.perm(F, p) for p in range(1, k_))
                cache[key] = (leaves, a, 3 * leaves + 4 * interior, 4 * (interior + leaves))
        e, a, f, n = cache[key]
        emb += e
        o8d += a
        ofac += f
        onode += n
    return {"embeddings": int(emb), "ops_leaf8d": o8d, "ops_factored": ofac, "ops_node4": onode}


# ---------------------------------------------------------------- profiles

def kernel_source_hash(cfg: int = 3) -> str:
    """sha256 of the sources of the kernel a workload's roofline is about."""
    h = hashlib.sha256()
    for rel in (WIDE_SOURCES if cfg == 6 else KERNEL_SOURCES):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profile_fields(cfg: int):
    """Key: value header fields of the committed counter profile of a
    workload, or (None, reason) when there is none or the kernel sources have
    changed since it was taken."""
    name = PMC_PROFILE.get(cfg)
    if not name:
        return None, "no counter profile for this workload"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None, f"profiles/{name} missing"
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
    if fields.get("kernel_source_sha256") != kernel_source_hash(cfg):
        return None, f"profiles/{name} was taken on other kernel sources"
    return fields, f"profiles/{name}"


def profiled_traffic(cfg: int):
    """(HBM bytes per enumeration launch, source) from the committed counter
    profile, or (None, reason)."""
    fields, source = profile_fields(cfg)
    if fields is None:
        return None, source
    if "traffic_bytes_per_launch" not in fields:
        return None, f"{source} holds no memory counters"
    return int(fields["traffic_bytes_per_launch"]), source


def profiled_valu_lane_ops(cfg: int):
    """(SQ_INSTS_VALU x 64 per launch, source) from the committed profile."""
    fields, source = profile_fields(cfg)
    if fields is None:
        return None, source
    if "valu_lane_ops_per_launch" not in fields:
        return None, f"{source} holds no instruction counters"
    return float(fields["valu_lane_ops_per_launch"]), source


# ---------------------------------------------------------------- CPU oracle

def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    # at most 16 threads: the host cores one GPU is given, whatever the machine reports
    return max(1, min(16, n))


def large_sample(ntopo: int = 8):
    """The large config's seeded 8-topology sample: 8 of its 256 topologies,
    each with its 6 queries (ring and all-to-all, k = 6, 7, 8), 48 queries."""
    from paper_2110_03214_amd import synth
    wl = synth.config3()
    rng = np.random.default_rng(np.random.SeedSequence([0x2110_0321, 3, 48]))
    topo = np.sort(rng.choice(len(wl.topologies), size=ntopo, replace=False))
    sel = np.nonzero(np.isin(wl.queries["server"], topo))[0]
    return wl.subset(sel), [int(t) for t in topo]


def cpu_baseline(wl, cfg: int, all_core_s: float = 30.0):
    """The oracle (test infrastructure, plain C at -O2, one query per thread,
    static split by query) timed on the host: all cores on the workload's
    sample, one thread on a part of it."""
    import oracle
    oracle.build()
    cores = host_threads()

    def timed(sub, nthreads):
        t0 = time.perf_counter()
        res = oracle.run_workload(sub, nthreads=nthreads)
        return int(res["count"].sum()), time.perf_counter() - t0

    if cfg == 3:
        sample, topo = large_sample()
        n_all, dt_all = timed(sample, cores)
        k6 = np.nonzero(sample.queries["k"] == 6)[0]
        one = sample.subset(k6)
        n_one, dt_one = timed(one, 1)
        desc = (f"all cores: the large config's seeded 8-topology sample (topologies {topo}, "
                f"48 queries, {n_all:.3g} embeddings) in {dt_all:.1f} s; one thread: its 16 "
                f"k=6 queries ({n_one:.3g} embeddings) in {dt_one:.1f} s")
    else:
        # whole queries in a fixed pseudo-random order, up to ~5e8 embeddings
        q = wl.queries
        emb_q = []
        for i in range(wl.nq):
            t = int(wl.server_topo[q["server"][i]])
            F = wl.topologies[t].shape[0] - bin(int(wl.busy[q["server"][i]])).count("1")
            emb_q.append(math.perm(F, int(q["k"][i])) if q["k"][i] <= F else 0)
        order = np.argsort(np.arange(wl.nq) * 2654435761 % (1 << 32), kind="stable")
        sel, total = [], 0
        for i in order:
            if total + emb_q[i] > 5e8 and sel:
                continue
            sel.append(int(i))
            total += emb_q[i]
        sample = wl.subset(np.sort(np.array(sel)))
        n_all, dt_all = timed(sample, cores)
        one = wl.subset(np.sort(np.array(sel[: max(1, len(sel) // 16)])))
        n_one, dt_one = timed(one, 1)
        desc = (f"all cores: {len(sel)} of {wl.nq} queries ({n_all:.3g} embeddings) in "
                f"{dt_all:.1f} s; one thread: {one.nq} of them ({n_one:.3g} embeddings) in "
                f"{dt_one:.1f} s")
    return {"value": n_all / dt_all, "unit": "embeddings/s", "cores": cores, "kind": "oracle",
            "single_thread_value": n_one / dt_one, "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(), "sample": desc + "; static split by query"}


# ---------------------------------------------------------------- GPU forms

def autotune_into(B, ctx, wl, qh, path):
    """Run the library's autotuner on the workload (no commits) and merge the
    chosen tuning into the JSON cache at `path` under the workload's shape
    class."""
    q = qh.copy()
    q["commit"] = 0
    best, trials = ctx.autotune(q, reps=3)
    key = B.shape_class(wl)
    cache = B.load_tuning_cache(path)
    cache[key] = {"tuning": best, "ms": min(ms for _, ms in trials),
                  "default_ms": trials[0][1], "trials": len(trials)}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    log(f"[bench] autotuned {key}: {best} ({trials[0][1]:.4f} -> {cache[key]['ms']:.4f} ms, "
        f"{len(trials)} trials)")
    return key, best


def timed_batch(B, wl, steps, warmup, metric="weighted", wide=False, profile=True, tuning="cache",
                autotune=None, step_pass=True, graph_pass=False):
    """The batched form: `steps` timed steps (query batch with commits, then
    release of every handle) after `warmup` untimed ones, inputs resident in
    HBM.  Kernel time from HIP events on the launch stream over the timed
    region.  Validates after the timed region.  With `step_pass` (the
    default) the step time comes from a first pass of `steps` steps with
    nothing recorded between them (an event record between kernels adds
    ~15 us to a ~0.15 ms step), and per-step latency and kernel time from a
    second pass of `steps` steps with the events.  With `graph_pass`, a third
    pass replays the query batch as a captured HIP graph (MAPA_USE_GRAPH)
    and reports its step time beside the stream-launched one."""
    import torch
    ops = op_counts(wl)
    emb = ops["embeddings"]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ctx = B.Context(0)
    qh, ids = B.load_workload(ctx, wl)
    qh["commit"] = 1
    qh["metric"] = B.METRIC_EFFBW if metric == "effbw" else B.METRIC_WEIGHTED
    if autotune and not wide:
        key, settings = autotune_into(B, ctx, wl, qh, autotune)
        source = f"autotuned in this run, written to {autotune}"
    elif tuning == "cache" and not wide:
        key, settings = B.apply_cached_tuning(ctx, wl)
        source = ("autotuner cache paper_2110_03214_amd/tuning.json" if settings else
                  "library defaults (no cached entry for this shape class)")
    else:
        key, settings, source = None, None, "library defaults"
    tuning_info = {"shape_class": key, "source": source, "settings": ctx.tuning().as_dict()}
    dq = torch.from_numpy(qh.view(np.uint8).copy()).to(dev)
    dr = torch.zeros(wl.nq * B.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    handles = dr.view(torch.int64)[5:]  # alloc_handle: byte 40 of each 48-byte result
    wide_res = [None]

    def step():
        if wide:  # host buffers in and out (16 B per query, 56 B per result)
            wide_res[0] = ctx.query_batch_wide(qh)
            ctx.release(wide_res[0]["alloc_handle"])
            return
        ctx.query_batch(dq, dr, stream=stream)
        ctx.release(handles, stride=48, count=wl.nq, stream=stream)

    for i in range(warmup):
        step()
        if i == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    wall_plain = None
    if step_pass:
        t0 = time.perf_counter()
        for s in range(steps):
            step()
        torch.cuda.synchronize()
        wall_plain = time.perf_counter() - t0
    ctx.profile(profile)
    ctx.reset_stats()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        ev[s][0].record(stream)
        step()
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    st = ctx.stats()
    ctx.profile(False)
    graph_ms = None
    if graph_pass and not wide:
        def gstep():
            ctx.query_batch(dq, dr, stream=stream, graph=True)
            ctx.release(handles, stride=48, count=wl.nq, stream=stream)

        for _ in range(3):  # the first call captures the graph
            gstep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            gstep()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) * 1e3 / steps
    # every step scored every embedding and handed every allocation back
    res = wide_res[0] if wide else dr.cpu().numpy().view(B.RESULT_DTYPE)
    assert int(res["count"].sum()) == emb, (int(res["count"].sum()), emb)
    assert np.array_equal(ctx.get_busy(ids), wl.busy), "release did not restore the entry state"
    assert st["self_check_failures"] == 0
    out = {"wall_s": wall_plain if step_pass else wall, "steps": steps, "embeddings": emb, "ops": ops,
           "queries": wl.nq, "lat_ms": lat, "stats": st, "qh": qh, "tuning": tuning_info,
           "graph_ms_per_step": graph_ms,
           "timing": ("step time from a pass of the steps with nothing recorded between them; "
                      "per-step latency and kernel time from a second pass with HIP events "
                      f"({wall * 1e3 / steps:.4f} ms per step with the events)") if step_pass else
                     "one pass: step time, per-step latency (HIP events around each step) and "
                     "kernel time (HIP events around each enumeration launch)"}
    out["kernel_ms"] = (st["enum_ms"] / st["enum_launches"]) if st["enum_launches"] else None
    out["probe"] = ctx.measure_alu_peak() if profile else None
    return ctx, out


def run_plain(ctx, qh, limit: int):
    """Plain form: one query per call, host pointers, synchronous (launch +
    copy back + sync per query).  Returns queries/s and per-query latency."""
    n = min(limit, len(qh))
    q = qh[:n].copy()
    q["commit"] = 0
    lat = np.empty(n)
    for i in range(min(16, n)):  # warm
        ctx.query_batch(q[i:i + 1])
    emb = 0
    t0 = time.perf_counter()
    for i in range(n):
        t = time.perf_counter()
        r = ctx.query_batch(q[i:i + 1])
        lat[i] = time.perf_counter() - t
        emb += int(r["count"][0])
    wall = time.perf_counter() - t0
    return {"queries": n, "queries_per_s": n / wall, "embeddings_per_s": emb / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3)}


def run_serving(B, cfg: int, nreq: int, plain: bool = False, loads=(0.5, 0.8, 1.0, 1.2)):
    """Serving form on a request trace.  Continuous batching: up to 4,096
    requests of different servers per device batch, two batches in flight.
    Plain: one request per device batch, one batch in flight.  First replays
    the trace with every request due at once to measure the form's capacity,
    then at offered loads that are fractions of it (trace time scaled)."""
    from paper_2110_03214_amd import synth
    tr = synth.config4(nreq) if cfg == 4 else synth.config5(nreq)
    rate_per_unit = nreq / tr.t_arrival[-1]
    out = {"workload": SERVING_TEXT[cfg], "requests": nreq,
           "form": ("plain: one request per device batch, one batch in flight" if plain else
                    "continuous batching: up to 4,096 requests per device batch, two in flight"),
           "runs": []}
    ctx = B.Context(0)
    ids = ctx.load_servers(tr.topologies, tr.server_topo)
    r = np.zeros(tr.n, dtype=B.REQUEST_DTYPE)
    r["id"] = np.arange(tr.n)
    r["t_arrival"], r["hold"], r["server"] = tr.t_arrival, tr.hold, ids[tr.server]
    r["kind"], r["k"], r["a"], r["b"] = tr.kind, tr.k, 1, 1

    def one(unit_us):
        ctx.serve_start(max_batch=1 if plain else 4096, inflight=1 if plain else 2,
                        time_unit_us=unit_us)
        ctx.serve_submit(r)
        got = 0
        while got < tr.n:
            got += len(ctx.serve_poll())
            time.sleep(0.002)
        return ctx.serve_stop()

    cap = one(0.0)
    capacity = cap["requests_per_s"]
    out["capacity_requests_per_s"] = capacity
    for f in loads:
        unit = rate_per_unit / (f * capacity) * 1e6  # us per trace time unit
        st = one(unit)
        out["runs"].append({
            "offered_fraction": f, "offered_requests_per_s": f * capacity,
            "requests_per_s": st["requests_per_s"], "p50_us": st["p50_us"], "p99_us": st["p99_us"],
            "p999_us": st["p999_us"], "wait_p50_us": st["wait_p50_us"],
            "wait_p99_us": st["wait_p99_us"], "turnaround_p50_us": st["turnaround_p50_us"],
            "turnaround_p99_us": st["turnaround_p99_us"], "mean_batch": st["mean_batch"],
            "batches": st["batches"], "mean_batch_us": st["mean_batch_us"],
            "mean_dispatch_us": st["mean_dispatch_us"], "mean_gpu_us": st["mean_gpu_us"],
            "mean_harvest_us": st["mean_harvest_us"], "fused_batches": st["fused_batches"],
            "granted": st["granted"], "nofit": st["nofit"], "host_nofit": st["host_nofit"],
            "admission_waits": st["admission_waits"],
            "embeddings_per_s": st["embeddings_per_s"]})
        log(f"[bench]   {'plain' if plain else 'continuous'} trace {cfg} at {f}x: "
            f"{st['requests_per_s']:.4g} req/s, p50 {st['p50_us']:.0f} us, p99 {st['p99_us']:.0f} us, "
            f"batch {st['mean_batch']:.0f} x {st['mean_batch_us']:.0f} us")
    ctx.close()
    return out


SIM_TOPOLOGY = ("DGX-1 V100 (8 GPUs)", "torus-2d (16 GPUs)", "two cube-meshes (16 GPUs)")
SIM_POLICY = ("preserve", "greedy", "baseline lowest ids")


def run_simulator(B, files_per_topology: int, njobs: int = 300, cpu_sims: int = 3):
    """Trace simulation (Sec. 5.2) of the job-file workload: every job file
    on each hardware graph under each policy, all simulations in one
    mapa_simulate call; plus the oracle's simulator on a few of them and the
    predicted effective bandwidth of the bandwidth-sensitive jobs per
    (hardware graph, policy), the paper's figure of merit."""
    from paper_2110_03214_amd import synth
    jf = synth.config7(files_per_topology, njobs)
    ctx = B.Context(0)
    ids = B.load_jobfiles(ctx, jf)
    warm = jf.subset(np.arange(3))
    ctx.simulate(ids[:3], warm.policy, warm.offsets, warm.jobs)
    t0 = time.perf_counter()
    logs, st = ctx.simulate(ids, jf.policy, jf.offsets, jf.jobs)
    wall = time.perf_counter() - t0
    ctx.close()
    out = {"workload": (f"{jf.nsim} simulations: {files_per_topology} seeded job files of {njobs} "
                        "jobs (1-5 GPUs, ring/all-to-all/tree, half bandwidth-sensitive, all "
                        "queued at cycle 0) on each of 3 hardware graphs, each file under the "
                        "3 policies"),
           "jobs": int(len(jf.jobs)), "wall_s": wall, "jobs_per_s": len(jf.jobs) / wall,
           "rounds": st["rounds"], "device_batches": st["device_batches"],
           "jobs_placed": st["jobs_placed"]}
    eff = {}
    for t, tname in enumerate(SIM_TOPOLOGY):
        eff[tname] = {}
        for p, pname in enumerate(SIM_POLICY):
            sel = [i for i in range(jf.nsim) if jf.sim_topo[i] == t and jf.policy[i] == p]
            v = np.concatenate([logs["effbw_milli"][jf.offsets[i]:jf.offsets[i + 1]][
                (jf.jobs["sensitive"][jf.offsets[i]:jf.offsets[i + 1]] == 1) &
                (jf.jobs["k"][jf.offsets[i]:jf.offsets[i + 1]] >= 2)] for i in sel]) / 1000.0
            eff[tname][pname] = [round(float(x), 3) for x in np.percentile(v, [0, 25, 50, 75, 100])]
    out["effbw_sensitive_min_p25_p50_p75_max_gbps"] = eff
    # the oracle's simulator (test infrastructure) on the first job file of
    # each hardware graph under Preserve
    from oracle import simulate as osim
    pick = [int(np.nonzero((jf.sim_topo == t) & (jf.policy == 0))[0][0]) for t in range(3)][:cpu_sims]
    t0 = time.perf_counter()
    n = 0
    for i in pick:
        a, b = jf.offsets[i], jf.offsets[i + 1]
        osim.simulate(jf.topologies[jf.sim_topo[i]], 0, jf.jobs[a:b], 0)
        n += b - a
    dt = time.perf_counter() - t0
    out["cpu_baseline"] = {"value": n / dt, "unit": "jobs/s", "cores": 1, "kind": "oracle",
                           "sample": f"{len(pick)} simulations ({n} jobs, Preserve) one after another"}
    return out


def roofline(cfg, tb):
    """Roofline of the enumeration kernel from the timed region's HIP-event
    kernel time: the per-leaf operation count (``achieved``/``frac``), the
    factored count and the issued VALU lane-ops of the committed counter
    profile."""
    avg_s = tb["kernel_ms"] / 1e3
    ops = tb["ops"]
    probe = tb["probe"]
    traffic, tsrc = profiled_traffic(cfg)
    valu, vsrc = profiled_valu_lane_ops(cfg)
    r = {"bound": "alu", "achieved": ops["ops_leaf8d"] / avg_s / 1e12, "peak": ALU_PEAK / 1e12,
         "unit": "Tops/s", "frac": ops["ops_leaf8d"] / avg_s / ALU_PEAK, "traffic": traffic,
         "traffic_unit": "HBM bytes per launch", "traffic_source": tsrc,
         "kernel": "k_wide_search" if cfg == 6 else "k_enumerate", "kernel_ms": tb["kernel_ms"],
         "op_model": ("per embedding 8 + 3B + |Nb[k-1]| int ops (B = weight bits), times "
                      "1 + 1/(F-k+1) for the interior nodes"),
         "ops_per_launch": ops["ops_leaf8d"], "embeddings_per_launch": ops["embeddings"],
         "peak_note": PEAK_NOTE, "measured_peak": probe / 1e12 if probe else None,
         "frac_of_measured_peak": ops["ops_leaf8d"] / avg_s / probe if probe else None,
         "items_per_launch": tb["stats"]["last_items"]}
    r["factored_model"] = {
        "model": ("3 int ops per embedding (weight-field extract, multiply-add, max) + 4 per "
                  "interior node at depths 1..k-1"),
        "ops_per_launch": ops["ops_factored"], "achieved": ops["ops_factored"] / avg_s / 1e12,
        "frac": ops["ops_factored"] / avg_s / ALU_PEAK,
        "frac_of_measured_peak": ops["ops_factored"] / avg_s / probe if probe else None}
    r["valu_counters"] = {"source": vsrc}
    if valu:
        r["valu_counters"].update({
            "lane_ops_per_launch": valu, "lane_ops_per_embedding": valu / max(1, ops["embeddings"]),
            "achieved": valu / avg_s / 1e12, "frac": valu / avg_s / ALU_PEAK,
            "frac_of_measured_peak": valu / avg_s / probe if probe else None})
    return r


def batched_summary(tb):
    lat = tb["lat_ms"]
    return {"embeddings_per_s": tb["embeddings"] * tb["steps"] / tb["wall_s"],
            "queries_per_s": tb["queries"] * tb["steps"] / tb["wall_s"],
            "ms_per_step": tb["wall_s"] * 1e3 / tb["steps"], "steps": tb["steps"],
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "kernel_ms": tb["kernel_ms"], "tuning": tb["tuning"], "timing": tb["timing"],
            "hip_graph_ms_per_step": tb["graph_ms_per_step"],
            "launch": "stream launches; hip_graph_ms_per_step replays the same batch as a captured "
                      "HIP graph (MAPA_USE_GRAPH), which the step time does not use"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps of the headline batch")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3, choices=(1, 2, 3, 6),
                    help="headline workload (3: large enumeration)")
    ap.add_argument("--metric", default="weighted", choices=("weighted", "effbw"),
                    help="key of every query: a*AggBW + b*PreservedBW, or the predicted effective "
                         "bandwidth of Eq. 2 (bandwidth-sensitive jobs; needs weights 0..2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="no HIP-event timing of the kernel")
    ap.add_argument("--batched", type=int, default=200,
                    help="timed steps of the batched config beside the headline (0: skip)")
    ap.add_argument("--plain", type=int, default=4096,
                    help="queries timed in the plain one-query-per-call form (0: skip; the "
                         "large config times at most 16)")
    ap.add_argument("--serving", type=int, default=1_000_000,
                    help="requests of the serving trace through the continuous-batching loop "
                         "(0: skip)")
    ap.add_argument("--serving-plain", type=int, default=100_000,
                    help="requests of the serving trace through the plain serving form (0: skip)")
    ap.add_argument("--mixed", type=int, default=20_000,
                    help="requests of the mixed-size trace through the continuous loop (0: skip)")
    ap.add_argument("--mixed-plain", type=int, default=5_000,
                    help="requests of the mixed-size trace through the plain serving form (0: skip)")
    ap.add_argument("--simulate", type=int, default=16,
                    help="job files per hardware graph for the trace simulation (0: skip)")
    ap.add_argument("--tuning", default="cache", choices=("cache", "default"),
                    help="launch settings: the autotuner's cached choice for the workload's shape "
                         "class (paper_2110_03214_amd/tuning.json), or the library defaults")
    ap.add_argument("--autotune", default="",
                    help="run the autotuner on each timed batch workload first and merge its "
                         "choices into this JSON cache file")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this many MiB first, to scale "
                         "hardware memory counters (FETCH_SIZE / WRITE_SIZE) against known bytes")
    ap.add_argument("--only-headline", action="store_true",
                    help="the headline batch alone (for profiling runs)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: every multi-GPU server exists only as a "
                                   "topology graph in the input; run with --gpus 1"}))
        sys.exit(2)

    import torch
    from paper_2110_03214_amd import binding as B
    from paper_2110_03214_amd import synth

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    if args.only_headline:
        args.batched = args.plain = args.serving = args.serving_plain = 0
        args.mixed = args.mixed_plain = args.simulate = 0
        args.no_cpu_baseline = True
    if args.copy_calibration_mib:
        src = torch.empty(args.copy_calibration_mib << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    makers = {1: synth.config1, 2: synth.config2, 3: synth.config3, 6: synth.config6}
    wl = makers[args.config]()
    if args.metric == "effbw":
        wl.queries["metric"][:] = 1
    ops = op_counts(wl)
    log(f"[bench] headline config {args.config}: {wl.nq} queries, {ops['embeddings']:.4g} "
        f"embeddings/step")
    ctx, tb = timed_batch(B, wl, args.steps, args.warmup, args.metric, wide=args.config == 6,
                          profile=not args.no_profile, tuning=args.tuning, autotune=args.autotune,
                          step_pass=True, graph_pass=args.config == 2)
    log(f"[bench] {args.steps} steps in {tb['wall_s']:.3f} s; kernel "
        f"{tb['kernel_ms'] if tb['kernel_ms'] else float('nan'):.3f} ms avg")
    lat = tb["lat_ms"]
    out = {
        "metric": METRIC,
        "value": tb["embeddings"] * args.steps / tb["wall_s"],
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tb["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded generator)",
        "config": {"workload": WORKLOAD_TEXT[args.config], "config_id": args.config,
                   "key": ("a*AggBW + b*PreservedBW, (a, b) = (1, 1)" if args.metric == "weighted"
                           else "predicted effective bandwidth (Eq. 2)"),
                   "queries": wl.nq, "embeddings_per_step": tb["embeddings"],
                   "topologies": len(wl.topologies), "parallelism": "single GPU"},
        "queries_per_s": wl.nq * args.steps / tb["wall_s"],
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "latency_scope": "per batch (every query of a batch completes together)",
        "tuning": tb["tuning"],
        "timing": tb["timing"],
    }
    if tb["graph_ms_per_step"] is not None:
        out["hip_graph_ms_per_step"] = tb["graph_ms_per_step"]
    if tb["kernel_ms"]:
        out["roofline"] = roofline(args.config, tb)
    plain = {}
    if args.plain:
        log("[bench] plain form: one query per call")
        plain[f"config_{args.config}"] = run_plain(ctx, tb["qh"], 16 if args.config == 3 else args.plain)
    ctx.close()
    if args.batched and args.config != 2:
        log("[bench] batched config")
        c2 = synth.config2()
        ctx2, tb2 = timed_batch(B, c2, args.batched, args.warmup, profile=not args.no_profile,
                                tuning=args.tuning, autotune=args.autotune, step_pass=True,
                                graph_pass=True)
        out["batched_config_2"] = batched_summary(tb2)
        out["batched_config_2"]["workload"] = WORKLOAD_TEXT[2]
        if tb2["kernel_ms"]:
            rl = roofline(2, tb2)
            out["batched_config_2"]["roofline"] = {
                k: rl[k] for k in ("achieved", "frac", "kernel_ms", "measured_peak",
                                   "frac_of_measured_peak", "traffic")}
            out["batched_config_2"]["roofline"]["factored_frac"] = rl["factored_model"]["frac"]
        if args.plain:
            plain["config_2"] = run_plain(ctx2, tb2["qh"], args.plain)
        ctx2.close()
    if plain:
        out["plain_one_query_per_call"] = plain
    serving = {}
    if args.serving:
        log(f"[bench] serving trace, continuous batching, {args.serving} requests")
        serving["trace_4_continuous"] = run_serving(B, 4, args.serving)
    if args.serving_plain:
        log(f"[bench] serving trace, plain form, {args.serving_plain} requests")
        serving["trace_4_plain"] = run_serving(B, 4, args.serving_plain, plain=True)
    if args.mixed:
        log(f"[bench] mixed-size trace, continuous batching, {args.mixed} requests")
        serving["trace_5_continuous"] = run_serving(B, 5, args.mixed)
    if args.mixed_plain:
        log(f"[bench] mixed-size trace, plain form, {args.mixed_plain} requests")
        serving["trace_5_plain"] = run_serving(B, 5, args.mixed_plain, plain=True)
    if serving:
        out["serving"] = serving
    if args.simulate:
        log(f"[bench] trace simulation, {args.simulate} job files per hardware graph")
        out["simulation"] = run_simulator(B, args.simulate)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(wl, args.config)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
