"""Python driver of the serving core (hs_server_* in libheatst).

The admission by resident bytes, lane management and continuous batching
live in the C++ core; this module owns the device pool (a torch
allocation), keeps request tensors alive while the core uses them, sizes
the classes' lane counts, and replays a Poisson arrival stream to measure
latency and throughput.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass

import numpy as np

from . import heatst as hs


def lane_bytes(n, order=2, nnodes=5, precision=hs.HS_MIXED, **kw) -> int:
    """Device bytes one request of grid n holds while admitted (its fields and
    multigrid hierarchy)."""
    p = hs.Problem(n=n, order=order, nnodes=nnodes, precision=precision, **kw)
    d, keep = p.desc()
    d.lane_memory = 1
    out = C.c_size_t(0)
    hs.check(hs.lib().hs_lane_bytes(C.byref(d), 0, C.byref(out)), "hs_lane_bytes")
    return out.value


def lane_cap(n: int) -> int:
    """Lanes of a size class's batched plan (the most of its requests served
    at once; the budget decides how many are resident).  Small grids are
    bound by launch latency and gain from wide batches; from 255^3 on a few
    lanes already saturate HBM."""
    if n <= 31:
        return 64
    if n <= 63:
        return 32
    if n <= 127:
        return 16
    return 8


def capacities_for_budget(budget_bytes: int, sizes, order=2, nnodes=5, precision=hs.HS_MIXED,
                          cap=lane_cap, **kw) -> dict:
    """Lanes per class: the class cap, or fewer when the budget could never
    hold that many requests of the class at once."""
    out = {}
    for n in sizes:
        per = lane_bytes(n, order, nnodes, precision, **kw)
        out[n] = max(1, min(cap(n), budget_bytes // per))
    return out


def _desc(slots, order, nnodes, precision, tol, max_cycles, inner, nu1, nu2, sweeps, sdc_tol, max_sweeps,
          forcing_c):
    d = hs.ServerDesc()
    d.order, d.nnodes = order, nnodes
    d.mg = hs.MgDesc(nu1, nu2, 6.0 / 7.0, 3, tol, max_cycles, 0, precision, inner[0], inner[1], 1, 0)
    d.sweeps, d.sdc_tol, d.max_sweeps, d.forcing_c = sweeps, sdc_tol, max_sweeps, forcing_c
    items = sorted(slots.items())
    d.nclasses = len(items)
    for i, (n, s) in enumerate(items):
        d.class_n[i] = n
        d.class_slots[i] = s
    return d, items


def pool_bytes(desc):
    """(shared workspace bytes, bytes with every lane of every class in use)."""
    sh, full = C.c_size_t(0), C.c_size_t(0)
    hs.check(hs.lib().hs_server_pool_bytes(C.byref(desc), C.byref(sh), C.byref(full)), "hs_server_pool_bytes")
    return sh.value, full.value


class Server:
    """Continuous-batching server for independent heat solves on one GPU.

    slots: {grid n: lanes of that class's plan}.  budget_bytes: the most
    device memory the server holds (shared workspaces plus the admitted
    requests); the pool is sized to it (or to every lane in use, if less)."""

    def __init__(self, slots: dict, order=2, nnodes=5, precision=hs.HS_MIXED, tol=1e-10,
                 max_cycles=60, inner=(2, 2), nu1=2, nu2=1, sweeps=0, sdc_tol=1e-10, max_sweeps=40,
                 forcing_c=3.0, budget_bytes=None):
        import torch
        L = hs.lib()
        d, items = _desc(slots, order, nnodes, precision, tol, max_cycles, inner, nu1, nu2, sweeps, sdc_tol,
                         max_sweeps, forcing_c)
        shared, full = pool_bytes(d)
        budget = full if budget_bytes is None else int(budget_bytes)
        self.pool_bytes = min(full, budget)
        self.budget_bytes = budget
        self.shared_bytes = shared
        self.pool = torch.empty(self.pool_bytes + 256, dtype=torch.uint8, device="cuda")
        base = (self.pool.data_ptr() + 255) & ~255
        self._h = C.c_void_p()
        hs.check(L.hs_server_create(C.byref(d), C.c_void_p(base), self.pool_bytes, budget,
                                    C.byref(self._h)), "hs_server_create")
        self.slots = dict(items)
        self._keep = {}

    @classmethod
    def for_budget(cls, budget_bytes, sizes, weights=None, order=2, nnodes=5, precision=hs.HS_MIXED, **kw):
        """A server for the grid sizes `sizes` whose resident requests share
        budget_bytes (weights are accepted for symmetry with the request
        stream; admission does not need them)."""
        caps = capacities_for_budget(budget_bytes, sizes, order, nnodes, precision,
                                     tol=kw.get("tol", 1e-10))
        return cls(caps, order=order, nnodes=nnodes, precision=precision, budget_bytes=budget_bytes, **kw)

    def resident(self):
        r, b = C.c_size_t(0), C.c_size_t(0)
        hs.check(hs.lib().hs_server_resident(self._h, C.byref(r), C.byref(b)), "hs_server_resident")
        return r.value, b.value

    def submit(self, n, nu, dt, nsteps, u0, t0=0.0):
        import torch
        u0 = u0.contiguous()
        out = torch.empty_like(u0)
        # the core reads u0 on its own streams: finish torch's pending work on it first
        torch.cuda.current_stream().synchronize()
        tk = C.c_uint64(0)
        hs.check(hs.lib().hs_server_submit(self._h, n, nu, dt, t0, nsteps, C.c_void_p(u0.data_ptr()),
                                           C.c_void_p(out.data_ptr()), C.byref(tk)), "hs_server_submit")
        self._keep[tk.value] = (u0, out)
        return tk.value

    def poll(self, ticket):
        info = hs.RequestInfo()
        s = hs.lib().hs_server_poll(self._h, ticket, C.byref(info))
        hs.check(s, "hs_server_poll")
        return s == hs.HS_OK, info

    def result(self, ticket):
        return self._keep[ticket][1]

    def release(self, ticket):
        self._keep.pop(ticket, None)

    def drain(self):
        hs.check(hs.lib().hs_server_drain(self._h), "hs_server_drain")

    def close(self):
        if getattr(self, "_h", None):
            hs.lib().hs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class StreamResult:
    n_requests: int
    wall_s: float
    solves_per_s: float
    p50_s: float
    p99_s: float
    mean_s: float
    dof_updates: float


def replay(server: Server, requests, u0_of, time_scale=1.0, keep_results=False, progress=None,
           progress_every=30.0):
    """Submit `requests` (inputs.Request) at their arrival times (scaled) and
    wait for all; latency = completion - arrival.  progress(msg), when given,
    is called about every `progress_every` seconds with the counts so far."""
    t_start = time.perf_counter()
    t_note = t_start
    tickets = []

    def note(force=False):
        nonlocal t_note
        now = time.perf_counter()
        if progress is not None and (force or now - t_note >= progress_every):
            t_note = now
            progress(f"replay: {len(tickets)}/{len(requests)} submitted after {now - t_start:.0f} s")

    for r in requests:
        due = t_start + r.arrival * time_scale
        while True:
            dtw = due - time.perf_counter()
            if dtw <= 0:
                break
            time.sleep(min(dtw, 0.002))
            note()
        t_arr = time.perf_counter()
        tk = server.submit(r.n, r.nu, r.dt, r.nsteps, u0_of(r))
        tickets.append((tk, r, t_arr))
    if progress is None:
        server.drain()
    else:
        pending = [tk for tk, _, _ in tickets]
        while pending:
            pending = [tk for tk in pending if not server.poll(tk)[0]]
            if pending:
                time.sleep(0.05)
                note()
    t_end = time.perf_counter()
    lat, infos = [], []
    dof = 0.0
    for tk, r, t_arr in tickets:
        done, info = server.poll(tk)
        assert done
        infos.append(info)
        dof += float(r.n) ** 3 * r.nsteps
    # completion times from the core's clock, arrival from ours: use the core's
    # submit stamp (taken inside submit) as the arrival
    lat = np.array([i.t_done - i.t_submit for i in infos])
    if not keep_results:
        for tk, _, _ in tickets:
            server.release(tk)
    wall = t_end - t_start
    res = StreamResult(len(requests), wall, len(requests) / wall, float(np.percentile(lat, 50)),
                       float(np.percentile(lat, 99)), float(lat.mean()), dof)
    return res, tickets, infos
