"""ctypes binding of ``libmapa.so`` (C ABI in ``include/mapa.h``).

Argument marshalling only: every step of the allocation path runs in the HIP
library.  There is no fallback; if the library is missing, loading raises.

The raw functions keep the C names (``mapa_create_topology``,
``mapa_set_busy``, ``mapa_query_batch``, ``mapa_release`` ...).  ``Context``
wraps them for numpy host arrays and for device tensors (anything exposing
``data_ptr()``, e.g. torch tensors on a ROCm device).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmapa.so")

MAPA_OK = 0
ERRORS = {
    -1: "MAPA_ERR_INVALID_ARG", -2: "MAPA_ERR_UNSUPPORTED", -3: "MAPA_ERR_OOM",
    -4: "MAPA_ERR_DEVICE", -5: "MAPA_ERR_NOT_BUSY", -6: "MAPA_ERR_UNKNOWN_SERVER",
    -7: "MAPA_ERR_ADMISSION", -8: "MAPA_ERR_NO_DEVICE", -9: "MAPA_ERR_STATE",
}
ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_OOM, ERR_DEVICE, ERR_NOT_BUSY = -1, -2, -3, -4, -5
ERR_UNKNOWN_SERVER, ERR_ADMISSION, ERR_NO_DEVICE, ERR_STATE = -6, -7, -8, -9
RING, ALL_TO_ALL, TREE = 0, 1, 2
PATTERN_BASE, MAX_PATTERNS = 16, 240
ALL_INJECTIVE, LINKED = 0, 1
METRIC_WEIGHTED, METRIC_EFFBW = 0, 1
RES_OK, RES_NOFIT, RES_CONFLICT, RES_INVALID, RES_REFUSED = 0, 1, 2, 3, 4
DEVICE_PTRS = 1
USE_GRAPH = 2
PIPELINE = 4

QUERY_DTYPE = np.dtype([("server", np.int32), ("kind", np.uint8), ("k", np.uint8),
                        ("mode", np.uint8), ("commit", np.uint8), ("a", np.int16),
                        ("b", np.int16), ("metric", np.int32)])
RESULT_DTYPE = np.dtype([("count", np.int64), ("status", np.int32), ("key", np.int32),
                         ("agg", np.int32), ("pres", np.int32), ("vertex_mask", np.uint32),
                         ("mapping", np.uint8, 8), ("links", np.int32),
                         ("alloc_handle", np.int64)])
assert QUERY_DTYPE.itemsize == 16 and RESULT_DTYPE.itemsize == 48
assert RESULT_DTYPE.fields["alloc_handle"][1] == 40
RESULT_WIDE_DTYPE = np.dtype([("count", np.int64), ("status", np.int32), ("key", np.int32),
                              ("agg", np.int32), ("pres", np.int32), ("vertex_mask", np.uint32),
                              ("mapping", np.uint8, 16), ("links", np.int32),
                              ("alloc_handle", np.int64)])
assert RESULT_WIDE_DTYPE.itemsize == 56 and RESULT_WIDE_DTYPE.fields["alloc_handle"][1] == 48
MAX_N_WIDE, MAX_K_WIDE = 32, 12
MAX_WIDE_QUERIES = 16384
NOALLOC_MAX_QUERIES = 65536


class Tuning(ctypes.Structure):
    _fields_ = [("min_leaves_per_item", ctypes.c_int32), ("mean_item_leaves", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("threads_per_block", ctypes.c_int32),
                ("pair_width", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TuneTrial(ctypes.Structure):
    _fields_ = [("tuning", Tuning), ("ms", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_int64), ("enum_launches", ctypes.c_int64),
                ("enum_ms", ctypes.c_double), ("last_items", ctypes.c_int64),
                ("last_split", ctypes.c_int32), ("self_check_failures", ctypes.c_int64),
                ("cu_count", ctypes.c_int32), ("num_servers", ctypes.c_int32),
                ("num_topologies", ctypes.c_int32)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("inflight", ctypes.c_int32),
                ("time_unit_us", ctypes.c_double), ("admission_items", ctypes.c_int64),
                ("item_leaves", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ServeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "requests", "completed", "granted", "nofit", "host_nofit", "batches", "releases",
        "embeddings", "admission_waits")] + [(n, ctypes.c_double) for n in (
            "wall_s", "requests_per_s", "embeddings_per_s", "p50_us", "p99_us", "p999_us",
            "max_us", "mean_batch", "mean_batch_us")] + [("fused_batches", ctypes.c_int64)] + [
                (n, ctypes.c_double) for n in (
                    "wait_p50_us", "wait_p99_us", "turnaround_p50_us", "turnaround_p99_us",
                    "mean_dispatch_us", "mean_gpu_us", "mean_harvest_us")]


REQUEST_DTYPE = np.dtype([("id", np.int64), ("t_arrival", np.float64), ("hold", np.float64),
                          ("server", np.int32), ("kind", np.uint8), ("k", np.uint8),
                          ("mode", np.uint8), ("metric", np.uint8), ("a", np.int16),
                          ("b", np.int16), ("reserved1", np.int32)])
COMPLETION_DTYPE = np.dtype([("id", np.int64), ("count", np.int64), ("alloc_handle", np.int64),
                             ("latency_us", np.float64), ("wait_us", np.float64),
                             ("status", np.int32), ("key", np.int32),
                             ("agg", np.int32), ("pres", np.int32), ("vertex_mask", np.uint32),
                             ("busy_before", np.uint32), ("batch", np.int32),
                             ("server", np.int32), ("mapping", np.uint8, 16)])
assert REQUEST_DTYPE.itemsize == 40 and COMPLETION_DTYPE.itemsize == 88


POLICY_PRESERVE, POLICY_GREEDY, POLICY_BASELINE = 0, 1, 2
JOB_DTYPE = np.dtype([("id", np.int32), ("arrival", np.int32), ("duration", np.int32),
                      ("kind", np.uint8), ("k", np.uint8), ("sensitive", np.uint8),
                      ("reserved", np.uint8)])
JOB_LOG_DTYPE = np.dtype([("id", np.int32), ("status", np.int32), ("start", np.int32),
                          ("finish", np.int32), ("vertex_mask", np.uint32), ("mapping", np.uint8, 8),
                          ("agg", np.int32), ("pres", np.int32), ("effbw_milli", np.int32),
                          ("links", np.int32), ("reserved", np.int32)])
assert JOB_DTYPE.itemsize == 16 and JOB_LOG_DTYPE.itemsize == 48


class SimStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "cycles", "event_cycles", "rounds", "device_batches", "jobs_placed")]


# every symbol include/mapa.h declares, with its ctypes signature
_P, _I32, _U32, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
SIGNATURES = {
    "mapa_last_error": (ctypes.c_char_p, []),
    "mapa_ctx_create": (_I32, [_I32, _SZ, ctypes.POINTER(_P)]),
    "mapa_ctx_destroy": (_I32, [_P]),
    "mapa_create_topology": (_I32, [_P, _I32, _P, _I32, _P, _P]),
    "mapa_create_pattern": (_I32, [_P, _I32, _I32, _P, _P]),
    "mapa_set_busy": (_I32, [_P, _I32, _P, _P, _U32, _P]),
    "mapa_get_busy": (_I32, [_P, _I32, _P, _P]),
    "mapa_query_batch": (_I32, [_P, _P, _I32, _P, _U32, _P]),
    "mapa_query_batch_wide": (_I32, [_P, _P, _I32, _P, _U32, _P]),
    "mapa_query_batch_noalloc": (_I32, [_P, _P, _I32, _P, _P]),
    "mapa_release": (_I32, [_P, _I32, _P, _I32, _U32, _P]),
    "mapa_simulate": (_I32, [_P, _I32, _P, _P, _P, _P, _P, ctypes.POINTER(SimStats)]),
    "mapa_get_tuning": (_I32, [_P, ctypes.POINTER(Tuning)]),
    "mapa_set_tuning": (_I32, [_P, ctypes.POINTER(Tuning)]),
    "mapa_autotune": (_I32, [_P, _P, _I32, _I32, ctypes.POINTER(Tuning), _P, _I32,
                             ctypes.POINTER(_I32)]),
    "mapa_profile": (_I32, [_P, _I32]),
    "mapa_get_stats": (_I32, [_P, ctypes.POINTER(Stats)]),
    "mapa_reset_stats": (_I32, [_P]),
    "mapa_sync": (_I32, [_P]),
    "mapa_measure_alu_peak": (_I32, [_P, ctypes.POINTER(ctypes.c_double)]),
    "mapa_serve_start": (_I32, [_P, ctypes.POINTER(ServeOpts)]),
    "mapa_serve_submit": (_I32, [_P, _P, _I32]),
    "mapa_serve_poll": (_I32, [_P, _P, _I32, ctypes.POINTER(_I32)]),
    "mapa_serve_stop": (_I32, [_P, ctypes.POINTER(ServeStats)]),
}

_lib = None


def lib():
    """Load libmapa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2110_03214_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MapaError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().mapa_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


def check(code, where):
    if code != MAPA_OK:
        raise MapaError(code, where)
    return code


def _ptr(x):
    """Device pointer of a tensor-like, or host pointer of a numpy array."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return ctypes.c_void_p(x.data_ptr())
    return ctypes.c_void_p(x.ctypes.data)


def pack_queries(server, kind, k, mode=ALL_INJECTIVE, commit=0, a=1, b=1, metric=0) -> np.ndarray:
    q = np.zeros(len(server), dtype=QUERY_DTYPE)
    q["server"], q["kind"], q["k"], q["mode"] = server, kind, k, mode
    q["commit"], q["a"], q["b"], q["metric"] = commit, a, b, metric
    return q


class Context:
    """One device context: topologies, device-resident server busy masks,
    batch workspace and enumeration buffer."""

    def __init__(self, device: int = 0, enum_buffer_bytes: int = 0):
        h = ctypes.c_void_p()
        check(lib().mapa_ctx_create(int(device), int(enum_buffer_bytes), ctypes.byref(h)),
              "mapa_ctx_create")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().mapa_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- state ---------------------------------------------------------------
    def create_topology(self, W, num_servers: int):
        W = np.ascontiguousarray(np.asarray(W, dtype=np.uint8))
        n = W.shape[0]
        tid, first = ctypes.c_int32(), ctypes.c_int32()
        check(lib().mapa_create_topology(self.h, n, W.ctypes.data, int(num_servers),
                                         ctypes.byref(tid), ctypes.byref(first)),
              "mapa_create_topology")
        return tid.value, first.value

    def create_pattern(self, k: int, edges) -> int:
        """Register an application graph given as (u, v) pairs on vertices
        0..k-1; returns the kind value that names it in queries/requests."""
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.uint8).reshape(-1))
        kind = ctypes.c_int32()
        check(lib().mapa_create_pattern(self.h, int(k), len(e) // 2, e.ctypes.data if len(e) else None,
                                        ctypes.byref(kind)), "mapa_create_pattern")
        return kind.value

    def load_servers(self, topologies, server_topo) -> np.ndarray:
        """Create one server per entry of server_topo; returns the library's
        server id of each (servers are created grouped by topology)."""
        server_topo = np.asarray(server_topo)
        ids = np.empty(len(server_topo), dtype=np.int32)
        for t, W in enumerate(topologies):
            idx = np.nonzero(server_topo == t)[0]
            _, first = self.create_topology(W, len(idx))
            ids[idx] = first + np.arange(len(idx), dtype=np.int32)
        return ids

    def set_busy(self, server_ids, masks, stream=None):
        if hasattr(server_ids, "data_ptr"):
            check(lib().mapa_set_busy(self.h, int(server_ids.numel()), _ptr(server_ids),
                                      _ptr(masks), DEVICE_PTRS, _stream(stream)), "mapa_set_busy")
            return
        ids = np.ascontiguousarray(server_ids, dtype=np.int32)
        m = np.ascontiguousarray(masks, dtype=np.uint32)
        check(lib().mapa_set_busy(self.h, len(ids), _ptr(ids), _ptr(m), 0, None), "mapa_set_busy")

    def get_busy(self, server_ids) -> np.ndarray:
        ids = np.ascontiguousarray(server_ids, dtype=np.int32)
        out = np.zeros(len(ids), dtype=np.uint32)
        check(lib().mapa_get_busy(self.h, len(ids), _ptr(ids), _ptr(out)), "mapa_get_busy")
        return out

    # -- queries -------------------------------------------------------------
    def query_batch(self, queries, results=None, stream=None, graph: bool = False,
                    pipeline: bool = False):
        """Host numpy QUERY_DTYPE array -> numpy RESULT_DTYPE array (blocking;
        ``pipeline=True``: never the fused small-batch launch), or device byte
        tensors (nq*16 and nq*48 bytes) -> asynchronous (``graph=True``:
        replay a captured HIP graph of the batch)."""
        if hasattr(queries, "data_ptr"):
            nq = queries.numel() * queries.element_size() // QUERY_DTYPE.itemsize
            flags = DEVICE_PTRS | (USE_GRAPH if graph else 0)
            check(lib().mapa_query_batch(self.h, _ptr(queries), int(nq), _ptr(results),
                                         flags, _stream(stream)), "mapa_query_batch")
            return results
        q = np.ascontiguousarray(queries, dtype=QUERY_DTYPE)
        res = np.zeros(len(q), dtype=RESULT_DTYPE) if results is None else results
        check(lib().mapa_query_batch(self.h, _ptr(q), len(q), _ptr(res),
                                     PIPELINE if pipeline else 0, None), "mapa_query_batch")
        return res

    def query_batch_noalloc(self, queries, results, stream=None):
        """Device byte tensors (nq*16 and nq*48 bytes) -> asynchronous batch
        whose workspace is the library's fixed device array (no allocation
        inside the call)."""
        nq = queries.numel() * queries.element_size() // QUERY_DTYPE.itemsize
        check(lib().mapa_query_batch_noalloc(self.h, _ptr(queries), int(nq), _ptr(results),
                                             _stream(stream)), "mapa_query_batch_noalloc")
        return results

    def query_batch_wide(self, queries, results=None, stream=None):
        """Host QUERY_DTYPE array -> RESULT_WIDE_DTYPE array (servers of up to
        32 accelerators, patterns of up to 12 vertices; blocking), or device
        byte tensors (nq*16 and nq*56 bytes) -> asynchronous."""
        if hasattr(queries, "data_ptr"):
            nq = queries.numel() * queries.element_size() // QUERY_DTYPE.itemsize
            check(lib().mapa_query_batch_wide(self.h, _ptr(queries), int(nq), _ptr(results),
                                              DEVICE_PTRS, _stream(stream)), "mapa_query_batch_wide")
            return results
        q = np.ascontiguousarray(queries, dtype=QUERY_DTYPE)
        res = np.zeros(len(q), dtype=RESULT_WIDE_DTYPE) if results is None else results
        check(lib().mapa_query_batch_wide(self.h, _ptr(q), len(q), _ptr(res), 0, None),
              "mapa_query_batch_wide")
        return res

    def release(self, handles, stride: int = 8, count: int | None = None, stream=None):
        if hasattr(handles, "data_ptr"):
            n = count if count is not None else handles.numel() * handles.element_size() // stride
            check(lib().mapa_release(self.h, int(n), _ptr(handles), int(stride), DEVICE_PTRS,
                                     _stream(stream)), "mapa_release")
            return
        h = np.ascontiguousarray(handles, dtype=np.int64)
        check(lib().mapa_release(self.h, len(h), _ptr(h), 8, 0, None), "mapa_release")

    # -- job-trace simulation ------------------------------------------------------
    def simulate(self, servers, policies, offsets, jobs):
        """Run len(servers) simulations (job files jobs[offsets[i]:offsets[i+1]]
        on distinct servers under the given policies).  Returns (logs as a
        JOB_LOG_DTYPE array aligned with jobs, stats dict)."""
        srv = np.ascontiguousarray(servers, dtype=np.int32)
        pol = np.ascontiguousarray(policies, dtype=np.int32)
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        j = np.zeros(len(jobs), dtype=JOB_DTYPE)
        for f in ("id", "arrival", "duration", "kind", "k", "sensitive"):
            j[f] = jobs[f]
        logs = np.zeros(len(j), dtype=JOB_LOG_DTYPE)
        st = SimStats()
        check(lib().mapa_simulate(self.h, len(srv), _ptr(srv), _ptr(pol), _ptr(off),
                                  _ptr(j) if len(j) else None, _ptr(logs) if len(j) else None,
                                  ctypes.byref(st)), "mapa_simulate")
        return logs, {name: getattr(st, name) for name, _ in SimStats._fields_}

    # -- tuning / stats ----------------------------------------------------------
    def tuning(self) -> Tuning:
        t = Tuning()
        check(lib().mapa_get_tuning(self.h, ctypes.byref(t)), "mapa_get_tuning")
        return t

    def set_tuning(self, **kw):
        t = self.tuning()
        for key, v in kw.items():
            setattr(t, key, int(v))
        check(lib().mapa_set_tuning(self.h, ctypes.byref(t)), "mapa_set_tuning")

    def autotune(self, queries, reps: int = 3):
        """Run the library's autotuner on host queries; the context keeps the
        fastest tuning.  Returns (best tuning dict, list of (tuning dict, ms))."""
        q = np.ascontiguousarray(queries, dtype=QUERY_DTYPE)
        cap = 256
        trials = (TuneTrial * cap)()
        best, n = Tuning(), ctypes.c_int32()
        check(lib().mapa_autotune(self.h, _ptr(q), len(q), int(reps), ctypes.byref(best),
                                  ctypes.cast(trials, ctypes.c_void_p), cap, ctypes.byref(n)),
              "mapa_autotune")
        return best.as_dict(), [(trials[i].tuning.as_dict(), trials[i].ms)
                                for i in range(min(cap, n.value))]

    def profile(self, on: bool = True):
        check(lib().mapa_profile(self.h, 1 if on else 0), "mapa_profile")

    def stats(self) -> dict:
        s = Stats()
        check(lib().mapa_get_stats(self.h, ctypes.byref(s)), "mapa_get_stats")
        return {name: getattr(s, name) for name, _ in Stats._fields_}

    def reset_stats(self):
        check(lib().mapa_reset_stats(self.h), "mapa_reset_stats")

    def sync(self):
        check(lib().mapa_sync(self.h), "mapa_sync")

    def measure_alu_peak(self) -> float:
        v = ctypes.c_double()
        check(lib().mapa_measure_alu_peak(self.h, ctypes.byref(v)), "mapa_measure_alu_peak")
        return v.value

    # -- serving loop ----------------------------------------------------------
    def serve_start(self, max_batch=0, inflight=0, time_unit_us=0.0, admission_items=0,
                    item_leaves=0):
        o = ServeOpts(int(max_batch), int(inflight), float(time_unit_us), int(admission_items),
                      int(item_leaves), 0)
        check(lib().mapa_serve_start(self.h, ctypes.byref(o)), "mapa_serve_start")

    def serve_submit(self, reqs):
        r = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
        check(lib().mapa_serve_submit(self.h, _ptr(r), len(r)), "mapa_serve_submit")

    def serve_poll(self, cap: int = 65536) -> np.ndarray:
        """Completions finished since the last poll (a copy; the staging
        buffer is kept between calls)."""
        buf = getattr(self, "_poll_buf", None)
        if buf is None or len(buf) < cap:
            buf = self._poll_buf = np.zeros(cap, dtype=COMPLETION_DTYPE)
        n = ctypes.c_int32()
        check(lib().mapa_serve_poll(self.h, _ptr(buf), cap, ctypes.byref(n)), "mapa_serve_poll")
        return buf[:n.value].copy()

    def serve_stop(self) -> dict:
        st = ServeStats()
        check(lib().mapa_serve_stop(self.h, ctypes.byref(st)), "mapa_serve_stop")
        return {name: getattr(st, name) for name, _ in ServeStats._fields_}


# Autotuned settings per batch shape class, as written by a bench run with
# --autotune: {class key: {"tuning": {...}, "ms": ..., "default_ms": ...}}.
TUNING_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def shape_class(wl) -> str:
    """Key of a synth.Workload's batch shape: accelerators per server, pattern
    sizes, kinds, modes, key metric, widest weight class and the batch size
    (power of two)."""
    q = wl.queries
    topo = wl.server_topo[q["server"]]
    n = [wl.topologies[t].shape[0] for t in np.unique(topo)]
    wmax = max(int(np.max(wl.topologies[t])) for t in np.unique(topo))
    wcls = 3 if wmax <= 3 else 15 if wmax <= 15 else 255
    metric = sorted(set(int(x) for x in q.get("metric", np.zeros(1, np.int32))))
    return (f"n{min(n)}-{max(n)}|k{int(q['k'].min())}-{int(q['k'].max())}|"
            f"kinds{','.join(str(int(k)) for k in np.unique(q['kind']))}|"
            f"mode{','.join(str(int(m)) for m in np.unique(q['mode']))}|"
            f"metric{','.join(map(str, metric))}|w{wcls}|q2^{max(0, int(wl.nq - 1).bit_length())}")


def load_tuning_cache(path: str = TUNING_CACHE) -> dict:
    import json
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def apply_cached_tuning(ctx: Context, wl, path: str = TUNING_CACHE):
    """Set the autotuned tuning cached for the workload's shape class, if any.
    Returns (key, tuning dict or None)."""
    key = shape_class(wl)
    entry = load_tuning_cache(path).get(key)
    if entry:
        ctx.set_tuning(**entry["tuning"])
    return key, (entry or {}).get("tuning")


def load_jobfiles(ctx: Context, jf):
    """Create one server per simulation of a synth.JobFiles; returns the server ids."""
    return ctx.load_servers(jf.topologies, jf.sim_topo)


def _stream(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def load_workload(ctx: Context, wl):
    """Create a synth.Workload's servers in ctx, set their busy masks and
    return its queries translated to library server ids."""
    ids = ctx.load_servers(wl.topologies, wl.server_topo)
    ctx.set_busy(ids, wl.busy)
    q = wl.queries
    return pack_queries(ids[q["server"]], q["kind"], q["k"], q["mode"], q["commit"], q["a"], q["b"],
                        q.get("metric", 0)), ids
