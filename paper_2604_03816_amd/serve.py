"""Continuous-batching serving loop over libqsv's server core (qsv_server_* in
include/qsv.h), plus the plain one-circuit-at-a-time path it is compared with.

The C++ core plans requests on host threads, admits them FIFO by HBM footprint (the
memory model of Eq. 14 against free memory minus a reserve, Eq. 15), and advances all
running requests together in batched, graph-replayed launches.  This module drives it
with an open-loop arrival clock: request i is submitted when the wall clock reaches its
arrival time, whatever the server is doing, and its latency runs from that arrival time
to the moment its result reaches the host.
"""
from __future__ import annotations

import ctypes
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import qsv as Q


class ServerOpts(ctypes.Structure):
    _fields_ = [("capacity_bytes", ctypes.c_size_t), ("reserve_bytes", ctypes.c_size_t),
                ("max_slots", ctypes.c_int), ("passes_per_step", ctypes.c_int), ("grid", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("planner_threads", ctypes.c_int), ("keep_states", ctypes.c_int),
                ("dry_run", ctypes.c_int), ("eps_tol", ctypes.c_double), ("norm_guard", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_longlong), ("n", ctypes.c_int), ("dtype", ctypes.c_int), ("status", ctypes.c_int),
                ("norm", ctypes.c_double), ("zexp", ctypes.c_double * 34), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_finish", ctypes.c_double), ("passes", ctypes.c_longlong),
                ("fused", ctypes.c_longlong), ("requested", ctypes.c_int), ("promoted", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_longlong) for f in (
        "submitted", "admitted", "finished", "rejected", "steps", "graph_replays", "tiles", "admission_waits",
        "peak_running", "peak_used_bytes", "capacity_bytes", "used_bytes", "running", "pending",
        "auto_c64", "auto_c128", "promoted")]


_BOUND = False


def _bind():
    global _BOUND
    if _BOUND:
        return Q.lib()
    L = Q.lib()
    vp, i, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    L.qsv_server_create.argtypes = [ctypes.POINTER(ServerOpts), vp, ctypes.POINTER(vp)]
    L.qsv_server_free.argtypes = [vp]
    L.qsv_server_submit.argtypes = [vp, i, i, ctypes.POINTER(Q.Gate), sz, ctypes.POINTER(Q.PlanOpts),
                                    ctypes.POINTER(ctypes.c_longlong)]
    L.qsv_server_step.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i)]
    L.qsv_server_results.argtypes = [vp, ctypes.POINTER(Result), i, ctypes.POINTER(i)]
    L.qsv_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.qsv_server_get_state.argtypes = [vp, ctypes.c_longlong, vp]
    L.qsv_server_release.argtypes = [vp, ctypes.c_longlong]
    _BOUND = True
    return L


class Server:
    def __init__(self, max_slots: int = 64, passes_per_step: int = 1, use_graph: bool = True,
                 capacity_bytes: int = 0, reserve_bytes: int = 0, planner_threads: int = 4,
                 keep_states: bool = False, dry_run: bool = False, grid: int = 0, stream=None,
                 eps_tol: float = 0.0, norm_guard: float = 0.0):
        L = _bind()
        o = ServerOpts()
        o.capacity_bytes = capacity_bytes
        o.reserve_bytes = reserve_bytes
        o.max_slots = max_slots
        o.passes_per_step = passes_per_step
        o.grid = grid
        o.use_graph = 1 if use_graph else 0
        o.planner_threads = planner_threads
        o.keep_states = 1 if keep_states else 0
        o.dry_run = 1 if dry_run else 0
        o.eps_tol = eps_tol
        o.norm_guard = norm_guard
        h = ctypes.c_void_p()
        sp = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        Q.check(L.qsv_server_create(ctypes.byref(o), sp, ctypes.byref(h)))
        self.h = h
        self._buf = (Result * 256)()

    def submit(self, n: int, dtype: str, gates, **plan_opts) -> int:
        gl = gates if isinstance(gates, (Q.GateList, Q.ArrayGateList)) else Q.GateList(gates)
        rid = ctypes.c_longlong()
        po = Q._opts(**plan_opts) if plan_opts else None
        Q.check(_bind().qsv_server_submit(self.h, n, Q._DT_SERVE[dtype], gl.arr, gl.n,
                                          ctypes.byref(po) if po is not None else None, ctypes.byref(rid)))
        return rid.value

    def step(self):
        r, p = ctypes.c_int(), ctypes.c_int()
        Q.check(_bind().qsv_server_step(self.h, ctypes.byref(r), ctypes.byref(p)))
        return r.value, p.value

    def results(self) -> List[dict]:
        out = []
        while True:
            c = ctypes.c_int()
            Q.check(_bind().qsv_server_results(self.h, self._buf, len(self._buf), ctypes.byref(c)))
            for k in range(c.value):
                r = self._buf[k]
                out.append({"id": r.id, "n": r.n, "dtype": "c64" if r.dtype == 0 else "c128", "status": r.status,
                            "requested": ("c64", "c128", "auto")[r.requested], "promoted": bool(r.promoted),
                            "norm": r.norm, "zexp": np.array(r.zexp[: r.n]), "passes": r.passes, "fused": r.fused,
                            "t_submit": r.t_submit, "t_admit": r.t_admit, "t_finish": r.t_finish})
            if c.value < len(self._buf):
                return out

    def stats(self) -> dict:
        st = ServerStats()
        Q.check(_bind().qsv_server_get_stats(self.h, ctypes.byref(st)))
        return {f[0]: getattr(st, f[0]) for f in st._fields_}

    def get_state(self, rid: int, n: int, dtype: str) -> np.ndarray:
        out = np.empty(1 << n, dtype=np.complex64 if dtype == "c64" else np.complex128)
        Q.check(_bind().qsv_server_get_state(self.h, rid, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def release(self, rid: int) -> None:
        Q.check(_bind().qsv_server_release(self.h, rid))

    def close(self):
        if getattr(self, "h", None):
            _bind().qsv_server_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _percentiles(lat: Sequence[float]) -> dict:
    a = np.sort(np.asarray(lat, dtype=np.float64))
    if a.size == 0:
        return {"p50_ms": None, "p99_ms": None, "mean_ms": None, "max_ms": None}
    return {"p50_ms": float(np.percentile(a, 50) * 1e3), "p99_ms": float(np.percentile(a, 99) * 1e3),
            "mean_ms": float(a.mean() * 1e3), "max_ms": float(a[-1] * 1e3)}


def run_batched(requests, circuits, server: Server, time_limit_s: float = 600.0, closed_loop: bool = False,
                trace_every_s: float = 0.5) -> dict:
    """Open-loop continuous batching: submit each request at its arrival time, step the
    server whenever it has work, record arrival -> result latency.  closed_loop: every
    request arrives at time 0 (the server runs flat out; circuits/s is then its capacity
    for this mix, and latency includes the time spent queued).  The queue is sampled
    every trace_every_s: (time, requests submitted but not finished, running, waiting
    for admission)."""
    N = len(requests)
    arrival = [0.0 if closed_loop else r.arrival_s for r in requests]
    id2req: Dict[int, int] = {}
    lat = [None] * N
    trace = []
    next_trace = 0.0
    t0 = time.perf_counter()
    i = done = 0
    while done < N:
        now = time.perf_counter() - t0
        if now > time_limit_s:
            break
        while i < N and arrival[i] <= now:
            r = requests[i]
            id2req[server.submit(r.n, r.dtype, circuits[i])] = i
            i += 1
        running, pending = server.step()
        tnow = time.perf_counter() - t0
        for res in server.results():
            k = id2req[res["id"]]
            lat[k] = tnow - arrival[k]
            done += 1
        if tnow >= next_trace:
            trace.append([round(tnow, 3), i - done, running, pending])
            next_trace = tnow + trace_every_s
        if running == 0 and pending == 0 and i < N:
            wait = arrival[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.01))
    wall = time.perf_counter() - t0
    got = [x for x in lat if x is not None]
    out = {"completed": len(got), "requests": N, "wall_s": wall,
           "circuits_per_s": len(got) / wall if wall > 0 else None, "closed_loop": closed_loop}
    out.update(_percentiles(got))
    out["server"] = server.stats()
    out["queue_trace"] = {"columns": ["t_s", "in_system", "running", "waiting_admission"], "samples": trace}
    return out


def run_plain(requests, circuits, fuse: bool = False, time_limit_s: float = 600.0) -> dict:
    """One circuit at a time on one stream: each request waits for the previous one,
    then runs its own plan (unfused: one gate per HBM pass, as the paper applies gates)
    and its reductions (norm, per-qubit <Z_i>)."""
    import torch
    N = len(requests)
    lat = []
    states: Dict[tuple, Q.State] = {}
    t0 = time.perf_counter()
    for k, r in enumerate(requests):
        now = time.perf_counter() - t0
        if now > time_limit_s:
            break
        if r.arrival_s > now:
            time.sleep(r.arrival_s - now)
        key = (r.n, r.dtype)
        s = states.get(key)
        if s is None:
            s = states[key] = Q.State(r.n, r.dtype)
        s.reset()
        s.apply(circuits[k], fuse=fuse)
        s.expval([(1.0, ((q, "Z"),)) for q in range(r.n)])
        s.norm()
        lat.append(time.perf_counter() - t0 - r.arrival_s)
    wall = time.perf_counter() - t0
    for s in states.values():
        s.free()
    torch.cuda.empty_cache()
    out = {"completed": len(lat), "requests": N, "wall_s": wall,
           "circuits_per_s": len(lat) / wall if wall > 0 else None}
    out.update(_percentiles(lat))
    return out
