"""Serving: continuous batching of structures through the library's server.

`Server` wraps sn_server_* (include/sn.h): worker threads in the library pack
queued structures into one graph per batch, on their own streams, within an
HBM budget.  `replay` submits a stream of (arrival time, structure) requests at
their arrival times and collects per-request latencies (completion minus
arrival), from which p50/p99 and throughput follow.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np

from ._lib import lib, check, PRECISIONS, Request, Result, SNError
from . import Model


class Server:
    def __init__(self, model: Model, device: int = 0, n_streams: int = 3, precision: str = "fp32",
                 hbm_budget: int = 0, max_batch_atoms: int = 16384, max_batch_structures: int = 256):
        h = C.c_void_p()
        check(lib().sn_server_create(model.handle, device, n_streams, PRECISIONS[precision],
                                     hbm_budget, max_batch_atoms, max_batch_structures, C.byref(h)))
        self.model = model
        self._h = h
        self._live = {}  # ticket -> (inputs and output arrays kept alive until polled)
        self._res = (Result * 256)()

    def submit(self, pos, Z, cell, forces: bool = True) -> int:
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        Z = np.ascontiguousarray(Z, dtype=np.int32)
        cell = np.ascontiguousarray(cell, dtype=np.float64)
        n = len(Z)
        ae = np.zeros(n)
        f = np.zeros((n, 3)) if forces else None
        req = Request(n, pos.ctypes.data, Z.ctypes.data, cell.ctypes.data, ae.ctypes.data,
                      f.ctypes.data if f is not None else None)
        t = C.c_uint64()
        check(lib().sn_server_submit(self._h, C.byref(req), C.byref(t)))
        self._live[t.value] = (ae, f)
        return t.value

    def warmup(self, pos, Z, cell) -> None:
        """Evaluate one structure once on every worker (results dropped), so that the
        workers' workspaces and kernels are ready before traffic arrives."""
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        Z = np.ascontiguousarray(Z, dtype=np.int32)
        cell = np.ascontiguousarray(cell, dtype=np.float64)
        req = Request(len(Z), pos.ctypes.data, Z.ctypes.data, cell.ctypes.data, None, None)
        check(lib().sn_server_warmup(self._h, C.byref(req)))

    def poll(self, timeout_ms: int = 0) -> list:
        n = C.c_int()
        check(lib().sn_server_poll(self._h, self._res, len(self._res), int(timeout_ms), C.byref(n)))
        out = []
        for k in range(n.value):
            r = self._res[k]
            ae, f = self._live.pop(r.ticket)
            out.append(dict(ticket=r.ticket, status=r.status, energy=r.energy,
                            virial=np.array(r.virial[:]).reshape(3, 3), atom_energy=ae, forces=f,
                            t_submit=r.t_submit, t_start=r.t_start, t_done=r.t_done,
                            batch_structures=r.batch_structures, batch_atoms=r.batch_atoms))
        return out

    def pending(self):
        q, r = C.c_int64(), C.c_int64()
        check(lib().sn_server_pending(self._h, C.byref(q), C.byref(r)))
        return q.value, r.value

    def close(self):
        if getattr(self, "_h", None):
            lib().sn_server_free(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server: Server, stream, time_scale: float = 1.0) -> dict:
    """Submit each (arrival_s, structure) at its arrival time; wait for every result.

    Returns per-request results in submission order with `latency` = completion time
    minus the scheduled arrival (queueing included), plus wall time and atom count.
    """
    t0 = time.perf_counter()
    tickets = []
    results = {}
    arrival = {}
    i = 0
    while i < len(stream) or len(results) < len(tickets):
        now = time.perf_counter() - t0
        while i < len(stream) and stream[i][0] * time_scale <= now:
            t_arr, s = stream[i]
            tk = server.submit(s.pos, s.Z, s.cell)
            arrival[tk] = (t_arr * time_scale, time.perf_counter() - t0)
            tickets.append(tk)
            i += 1
        wait_ms = 1
        if i < len(stream):
            wait_ms = max(0, min(5, int((stream[i][0] * time_scale - now) * 1e3)))
        for r in server.poll(timeout_ms=wait_ms):
            r["t_host_done"] = time.perf_counter() - t0
            results[r["ticket"]] = r
    wall = time.perf_counter() - t0
    out = []
    for tk in tickets:
        r = results[tk]
        if r["status"] != 0:
            raise SNError(r["status"], f"request {tk} failed")
        t_arr, t_sub = arrival[tk]
        r["latency"] = r["t_host_done"] - t_arr
        r["service"] = r["t_done"] - r["t_start"]
        out.append(r)
    return dict(results=out, wall=wall)


def latency_summary(rep: dict) -> dict:
    lat = np.array([r["latency"] for r in rep["results"]]) * 1e3
    atoms = sum(len(r["atom_energy"]) for r in rep["results"])
    bs = np.array([r["batch_structures"] for r in rep["results"]])
    return dict(p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), max_ms=float(lat.max()), requests=len(lat),
                atoms=int(atoms), wall_s=rep["wall"], atom_steps_per_s=atoms / rep["wall"],
                mean_batch_structures=float(bs.mean()))
