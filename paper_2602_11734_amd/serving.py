"""Request-stream drivers for the continuous-batching server and for the plain
one-at-a-time path, with wall-clock arrivals and per-request latency.

Both drivers take requests with arrival times (seconds from the start), replay the
arrivals in real time, and record completion - arrival for every request.  Every
generation step runs in the HIP library; these functions only schedule calls.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import (ERR_DEVICE, QsgsError, params_of, qsgs_generate, qsgs_server_create,
               qsgs_server_destroy, qsgs_server_ready, qsgs_server_reserved_bytes, qsgs_server_submit,
               qsgs_server_take, qsgs_server_tick, qsgs_grid_bytes, qsgs_workspace_bytes)


@dataclass
class StreamResult:
    latencies_s: np.ndarray   # per request, in request order
    makespan_s: float         # first arrival to last completion
    grown: int                # voxels grown over all requests
    max_resident: int = 0
    failed: tuple = ()        # ids of requests the server retired as failed

    def summary(self) -> dict:
        lat = self.latencies_s
        return {"requests": int(len(lat)),
                "realizations_per_s": float(len(lat) / self.makespan_s),
                "voxels_grown_per_s": float(self.grown / self.makespan_s),
                "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_latency_ms": float(lat.mean() * 1e3),
                "makespan_s": float(self.makespan_s),
                "max_resident": int(self.max_resident),
                "failed": len(self.failed)}


def serve_stream(requests, arena_bytes: int, max_slots: int = 64, steps_per_tick: int = 2,
                 keep=None, out=None) -> StreamResult:
    """Continuous batching: requests are submitted when they arrive; every tick admits
    what fits the arena, seeds it, advances all resident requests and retires the
    finished ones.  `keep(rid, host_grid)` receives each result if given; with `out`
    (request id -> device uint8 tensor of at least N bytes) each result is copied into
    out[rid] on the device instead."""
    import torch
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    srv = qsgs_server_create(arena, arena_bytes, max_slots, steps_per_tick)
    n = len(requests)
    done_at = np.zeros(n)
    grown = 0
    finished = 0
    max_res = 0
    nxt = 0
    failed = []
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        resident = queued = 0
        while finished < n:
            now = time.perf_counter() - t0
            fresh = 0
            while nxt < n and requests[nxt].arrival_s <= now:
                r = requests[nxt]
                qsgs_server_submit(srv, r.rid, r.case.dims, params_of(r.case))
                nxt += 1
                fresh += 1
            if resident == 0 and queued == 0 and fresh == 0 and nxt < n:
                # idle: wait for the next arrival
                time.sleep(max(0.0, min(requests[nxt].arrival_s - now, 0.005)))
                continue
            try:
                resident, queued, nready = qsgs_server_tick(srv)
            except QsgsError as e:  # a failed request was retired; the others go on
                if e.status != ERR_DEVICE or not hasattr(e, "counts"):
                    raise
                resident, queued, nready = e.counts
            max_res = max(max_res, resident)
            if nready:
                t_done = time.perf_counter() - t0
                for rid, info in qsgs_server_ready(srv, nready):
                    if info.status < 0:  # failed: nothing to copy out
                        qsgs_server_take(srv, rid, None, check=False)
                        failed.append(rid)
                        done_at[rid] = t_done
                        finished += 1
                        continue
                    if out is not None:
                        dst = out[rid]
                        qsgs_server_take(srv, rid, dst, dst.numel(), dst_on_host=False)
                    elif keep is not None:
                        c = requests[rid].case
                        host = np.empty(c.n, dtype=np.uint8)
                        qsgs_server_take(srv, rid, host)
                        keep(rid, host)
                    else:
                        qsgs_server_take(srv, rid, None)
                    done_at[rid] = t_done
                    grown += info.solid_count - info.n_seeds
                    finished += 1
        makespan = done_at.max() - requests[0].arrival_s
    finally:
        qsgs_server_destroy(srv)
    arrivals = np.array([r.arrival_s for r in requests])
    return StreamResult(done_at - arrivals, makespan, grown, max_res, tuple(failed))


def plain_stream(requests, out=None) -> StreamResult:
    """The plain path: one qsgs_generate per request, first come first served.  With
    `out` (request id -> device uint8 tensor of qsgs_grid_bytes(dims)) each request is
    generated into out[rid]."""
    import torch
    n = len(requests)
    done_at = np.zeros(n)
    grown = 0
    # one workspace and grid sized for the largest request, reused
    gbytes = max(qsgs_grid_bytes(r.case.dims) for r in requests)
    wbytes = max(qsgs_workspace_bytes(r.case.dims, params_of(r.case)) for r in requests)
    grid = torch.empty(gbytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(wbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, r in enumerate(requests):
        now = time.perf_counter() - t0
        if r.arrival_s > now:
            time.sleep(r.arrival_s - now)
        st, info = qsgs_generate(r.case.dims, params_of(r.case),
                                 grid if out is None else out[r.rid], ws, wbytes)
        done_at[k] = time.perf_counter() - t0
        grown += info.solid_count - info.n_seeds
    makespan = done_at.max() - requests[0].arrival_s
    arrivals = np.array([r.arrival_s for r in requests])
    return StreamResult(done_at - arrivals, makespan, grown, 1)


def server_arena_bytes(requests, max_slots: int, budget_bytes: int) -> int:
    """Arena size: the control area plus the budget."""
    return qsgs_server_reserved_bytes(max_slots) + int(budget_bytes)
