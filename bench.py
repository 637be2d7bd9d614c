#!/usr/bin/env python3
"""Benchmark of the MAPA allocation hot path on one MI355X.

A step is one pass of the whole hot path over one batch: every query of the
workload is answered (free sets and key constants, pattern tables, every
embedding enumerated and scored, best selected with the fixed tie-break),
every successful query commits its allocation, and every committed
allocation is released again, so each step starts from the same busy state.
Queries, results and busy masks stay in HBM; nothing crosses PCIe inside the
timed region.

Default workload: the batched config (65,536 server states over three 8- and
6-vertex topologies, 0-6 busy vertices, ring / all-to-all / tree patterns with
k in 2..8).  ``--config 3`` runs the large 16-vertex enumeration and
``--config 1`` the tiny one, ``--config 6`` the wide path (32-vertex servers,
jobs of 9 and 10 accelerators).

Prints ONE JSON line (rank 0):  value = embeddings scored per second, plus
queries/s, per-batch p50/p99 latency, the roofline of the enumeration kernel
(integer ALU bound) and the CPU oracle timed on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pattern embeddings scored/sec + allocation queries/sec, p50/p99 latency"
# MI355X vector-ALU ceiling for 32-bit lane operations: the published fp32
# vector rate, 157.3 TFLOP/s, is 256 CUs x 2.4 GHz x 128 lanes x 2 flops per
# FMA, so the vector ALUs retire at most 256 x 128 x 2.4e9 = 78.6e12 32-bit
# lane-ops/s.  (A 4 SIMD x 16 lane model, 39.3e12, is exceeded in
# measurement: the enumeration kernel itself sustains ~75 int32 lane-ops per
# clock per CU.)
CU, LANES_PER_CLK, CLK = 256, 128, 2.4e9
ALU_PEAK = CU * LANES_PER_CLK * CLK  # 78.64e12 int32 lane-ops/s

# Counter profiles (rocprofv3 FETCH_SIZE / WRITE_SIZE) of the enumeration
# kernel, committed under profiles/; their HBM byte count is reported only
# while the kernel sources still hash to the value the profile was taken on.
KERNEL_SOURCES = tuple("paper_2110_03214_amd/csrc/" + f for f in (
    "device.h", "enumerate.h", "enum_pair12_lds.hip", "enum_pair12_glb.hip", "enum_pair6.hip",
    "enum_plain.hip", "mapa_internal.h"))
WIDE_SOURCES = tuple("paper_2110_03214_amd/csrc/" + f for f in ("wide.hip", "mapa_internal.h"))
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Integer ops charged per node of the search tree (every partial and every
# complete embedding): with the weights of the node's candidates to the
# vertices still free tabulated once per parent, placing one more vertex
# needs one packed-weight read (the weight to the vertex just placed), one
# multiply-add, one add of the tabulated term and one compare/select.  No
# method that scores every embedding separately does less, so the fraction
# of peak this gives is a lower bound on the kernel's ALU use.
OPS_PER_NODE = 4


def algorithmic_ops(wl) -> tuple[int, int]:
    """(embeddings, algorithmic int ops) of one pass over the workload:
    OPS_PER_NODE for every node at depth 1..k of each query's search tree,
    F!/(F-p)! of them at depth p in ALL mode (the leaves are the embeddings)."""
    q = wl.queries
    n_of = [W.shape[0] for W in wl.topologies]
    emb = ops = 0
    cache = {}
    for s, k in zip(q["server"], q["k"]):
        t = int(wl.server_topo[s])
        F = n_of[t] - bin(int(wl.busy[s])).count("1")
        key = (F, int(k))
        if key not in cache:
            if k > F:
                cache[key] = (0, 0)
            else:
                nodes = sum(math.perm(F, p) for p in range(1, int(k) + 1))
                cache[key] = (math.perm(F, int(k)), OPS_PER_NODE * nodes)
        e, o = cache[key]
        emb += e
        ops += o
    return emb, ops


def kernel_source_hash(cfg: int = 2) -> str:
    """sha256 of the sources of the kernel a workload's roofline is about."""
    h = hashlib.sha256()
    for rel in (WIDE_SOURCES if cfg == 6 else KERNEL_SOURCES):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_traffic(cfg: int):
    """(HBM bytes per enumeration launch, profile path) from the committed
    counter profile of this workload, or (None, reason) when there is none or
    the kernel has changed since it was taken."""
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
    if "traffic_bytes_per_launch" not in fields:
        return None, f"profiles/{name} holds no memory counters"
    return int(fields["traffic_bytes_per_launch"]), f"profiles/{name}"


def cpu_baseline(wl, seconds: float = 8.0):
    """The oracle (test infrastructure) timed on the host on a bounded sample."""
    import oracle
    oracle.build()
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(16, cores))
    # bounded sample: whole queries, at most ~5e8 embeddings per pass
    sel, total = [], 0
    emb_q = []
    q = wl.queries
    for i in range(wl.nq):
        t = int(wl.server_topo[q["server"][i]])
        F = wl.topologies[t].shape[0] - bin(int(wl.busy[q["server"][i]])).count("1")
        e = math.perm(F, int(q["k"][i])) if q["k"][i] <= F else 0
        emb_q.append(e)
    order = np.argsort(np.arange(wl.nq) * 2654435761 % (1 << 32), kind="stable")
    for i in order:
        if total + emb_q[i] > 5e8 and sel:
            continue
        sel.append(int(i))
        total += emb_q[i]
    sub = wl.subset(np.sort(np.array(sel)))
    done = passes = 0
    t0 = time.perf_counter()
    while True:
        res = oracle.run_workload(sub, nthreads=cores)
        done += int(res["count"].sum())
        passes += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "embeddings/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sel)} of {wl.nq} queries ({total:.3g} embeddings) x {passes} "
                      f"passes in {dt:.1f} s, static split by query over {cores} threads"}


def run_plain(ctx, B, qh, limit: int = 4096):
    """Plain form: one query per call, host pointers, synchronous (launch +
    copy back + sync per query).  Returns queries/s and per-query latency."""
    n = min(limit, len(qh))
    q = qh[:n].copy()
    q["commit"] = 0
    lat = np.empty(n)
    for i in range(min(64, n)):  # warm
        ctx.query_batch(q[i:i + 1])
    t0 = time.perf_counter()
    for i in range(n):
        t = time.perf_counter()
        ctx.query_batch(q[i:i + 1])
        lat[i] = time.perf_counter() - t
    wall = time.perf_counter() - t0
    return {"queries": n, "queries_per_s": n / wall, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3)}


def run_serving(B, cfg: int, nreq: int, loads=(0.5, 0.8, 1.0, 1.2)):
    """Serving form: a request trace through the continuous-batching loop.
    First replays it as fast as possible to measure capacity, then at offered
    loads that are fractions of that capacity (time unit scaled)."""
    from paper_2110_03214_amd import synth
    tr = synth.config4(nreq) if cfg == 4 else synth.config5(nreq)
    rate_per_unit = nreq / tr.t_arrival[-1]
    out = {"workload": ("serving: Poisson requests over 4,096 servers of the batched config's "
                        "three topologies" if cfg == 4 else
                        "mixed serving: bursty requests over 1,024 cube-mesh and 1,024 16-vertex "
                        "servers"), "requests": nreq, "runs": []}
    ctx = B.Context(0)
    ids = ctx.load_servers(tr.topologies, tr.server_topo)
    r = np.zeros(tr.n, dtype=B.REQUEST_DTYPE)
    r["id"] = np.arange(tr.n)
    r["t_arrival"], r["hold"], r["server"] = tr.t_arrival, tr.hold, ids[tr.server]
    r["kind"], r["k"], r["a"], r["b"] = tr.kind, tr.k, 1, 1

    def one(unit_us):
        ctx.serve_start(max_batch=4096, inflight=2, time_unit_us=unit_us)
        ctx.serve_submit(r)
        got = 0
        while got < tr.n:
            got += len(ctx.serve_poll())
            time.sleep(0.001)
        return ctx.serve_stop()

    cap = one(0.0)
    capacity = cap["requests_per_s"]
    out["capacity_requests_per_s"] = capacity
    for f in loads:
        unit = rate_per_unit / (f * capacity) * 1e6  # us per trace time unit
        st = one(unit)
        out["runs"].append({"offered_fraction": f, "offered_requests_per_s": f * capacity,
                            "requests_per_s": st["requests_per_s"], "p50_us": st["p50_us"],
                            "p99_us": st["p99_us"], "p999_us": st["p999_us"],
                            "mean_batch": st["mean_batch"], "batches": st["batches"],
                            "mean_batch_us": st["mean_batch_us"], "fused_batches": st["fused_batches"],
                            "granted": st["granted"], "nofit": st["nofit"],
                            "embeddings_per_s": st["embeddings_per_s"]})
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="timed steps (default: per config)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=2, choices=(1, 2, 3, 6))
    ap.add_argument("--metric", default="weighted", choices=("weighted", "effbw"),
                    help="key of every query: a*AggBW + b*PreservedBW, or the predicted effective "
                         "bandwidth of Eq. 2 (bandwidth-sensitive jobs; needs weights 0..2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="no HIP-event timing of the kernel")
    ap.add_argument("--plain", type=int, default=4096,
                    help="queries timed in the plain one-query-per-launch form (0: skip)")
    ap.add_argument("--serving-trace", type=int, default=4, choices=(4, 5),
                    help="serving trace: 4 = Poisson requests over the batched config's topologies, "
                         "5 = bursty requests over cube-mesh and 16-vertex servers")
    ap.add_argument("--serving", type=int, default=100000,
                    help="requests of the serving trace timed through the serving loop (0: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this many MiB first, to scale "
                         "hardware memory counters (FETCH_SIZE / WRITE_SIZE) against known bytes")
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
    steps = args.steps or {1: 200, 2: 200, 3: 3, 6: 3}[args.config]
    wl = {1: synth.config1, 2: synth.config2, 3: synth.config3, 6: synth.config6}[args.config]()
    wide = args.config == 6
    emb, ops = algorithmic_ops(wl)
    log(f"[bench] config {args.config}: {wl.nq} queries, {emb:.4g} embeddings/step, "
        f"{ops:.4g} algorithmic ops/step")

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if args.copy_calibration_mib:
        src = torch.empty(args.copy_calibration_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = B.Context(0)
    qh, ids = B.load_workload(ctx, wl)
    qh["commit"] = 1
    qh["metric"] = B.METRIC_EFFBW if args.metric == "effbw" else B.METRIC_WEIGHTED
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

    for i in range(args.warmup):
        step()
        if i == 0:
            torch.cuda.synchronize()
            log("[bench] first step done")
    torch.cuda.synchronize()

    if not args.no_profile:
        ctx.profile(True)
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
    # every step scored every embedding and handed every allocation back
    res = wide_res[0] if wide else dr.cpu().numpy().view(B.RESULT_DTYPE)
    assert int(res["count"].sum()) == emb, (int(res["count"].sum()), emb)
    assert np.array_equal(ctx.get_busy(ids), wl.busy), "release did not restore the entry state"
    assert st["self_check_failures"] == 0
    ctx.profile(False)
    log(f"[bench] {steps} steps in {wall:.3f} s; enumerate {st['enum_ms'] / max(1, st['enum_launches']):.3f} ms avg")

    ms_per_step = wall * 1e3 / steps
    value = emb * steps / wall
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded generator)",
        "config": {"workload": WORKLOAD_TEXT[args.config], "config_id": args.config,
                   "key": ("a*AggBW + b*PreservedBW, (a, b) = (1, 1)" if args.metric == "weighted"
                           else "predicted effective bandwidth (Eq. 2)"),
                   "queries": wl.nq, "embeddings_per_step": emb,
                   "topologies": len(wl.topologies), "parallelism": "single GPU"},
        "queries_per_s": wl.nq * steps / wall,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "latency_scope": "per batch (every query of a batch completes together)",
    }
    if not args.no_profile and st["enum_launches"]:
        avg_s = st["enum_ms"] / st["enum_launches"] / 1e3
        achieved = ops / avg_s
        probe = ctx.measure_alu_peak()
        traffic, source = profiled_traffic(args.config)
        out["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK / 1e12,
                           "unit": "Tops/s", "frac": achieved / ALU_PEAK, "traffic": traffic,
                           "traffic_unit": "HBM bytes per launch", "traffic_source": source,
                           "kernel": "k_wide_search" if wide else "k_enumerate",
                           "kernel_ms": avg_s * 1e3,
                           "ops_per_launch": ops, "items_per_launch": st["last_items"],
                           "measured_peak": probe / 1e12, "frac_of_measured_peak": achieved / probe}
    if args.plain:
        log("[bench] plain form: one query per launch")
        out["plain_one_query_per_launch"] = run_plain(ctx, B, qh, args.plain)
    ctx.close()
    if args.serving and args.config == 2:
        log(f"[bench] serving form, trace {args.serving_trace}")
        out["serving"] = run_serving(B, args.serving_trace, args.serving)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        if args.metric == "effbw":
            wl.queries["metric"][:] = 1
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
