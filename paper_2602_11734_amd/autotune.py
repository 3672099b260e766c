"""Autotuner for the launch shape of the item kernels.

Times every candidate (workgroup size x workgroup count of the fused sweep and of the
seeding kernels, graph-captured or plain pass launches) on the given batch by wall
clock, checks on the device that every candidate produces the same grids (the shape
must never change a result), applies the fastest, and caches it per device and
workload size bucket.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import (QsgsError, params_of, qsgs_generate_batch, qsgs_batch_workspace_bytes,
               qsgs_grid_bytes, qsgs_set_tuning, qsgs_tuning)

SWEEP_BLOCKS = (128, 256, 512)
SWEEP_GRIDS = (0, 2560, 3840, 5120)  # 0: one round of resident workgroups
SEED_SHAPES = ((256, 2048), (512, 4096))


def cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "qsgs", "tuning.json")


def bucket_of(cases) -> str:
    total = sum(c.n for c in cases)
    return f"n{len(cases)}_v2^{int(math.log2(max(total, 1)))}"


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0)


def _run(cases, grids, ws, wsb):
    import torch
    dims = [c.dims for c in cases]
    params = [params_of(c) for c in cases]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qsgs_generate_batch(dims, params, grids, ws, wsb)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def autotune(cases, repeats: int = 2, use_cache: bool = True, verbose: bool = False) -> dict:
    """Returns (and applies) the fastest tuning for this batch of cases: every workgroup
    size and count of the sweep and the seeding kernels with graph-captured passes, then
    the fastest of them with plain launches; every candidate must give the same grids.
    The entry reports the candidates' count, the best wall time, the default tuning's
    wall time and the speedup over it."""
    import torch
    key = f"{_device_name()}|{bucket_of(cases)}"
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
        if key in cache:
            qsgs_set_tuning(cache[key]["tuning"])
            return cache[key]
    dims = [c.dims for c in cases]
    params = [params_of(c) for c in cases]
    grids = [torch.empty(qsgs_grid_bytes(d), dtype=torch.uint8, device="cuda") for d in dims]
    wsb = qsgs_batch_workspace_bytes(dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    results = []
    ref = []  # the first candidate's grids, kept on the device

    def trial(t):
        qsgs_set_tuning(t)
        _run(cases, grids, ws, wsb)  # warm-up (and graph capture)
        wall = min(_run(cases, grids, ws, wsb) for _ in range(repeats))
        if not ref:
            ref.extend(gr.clone() for gr in grids)
        elif not all(bool(torch.equal(a[: d[0] * d[1] * d[2]], b[: d[0] * d[1] * d[2]]))
                     for a, b, d in zip(ref, grids, dims)):
            raise QsgsError(-4, f"tuning {t} changed the result")
        results.append((wall, t))
        if verbose:
            print(f"tune {t}: {wall * 1e3:.2f} ms", flush=True)

    try:
        for sb, sg in SEED_SHAPES:
            for b in SWEEP_BLOCKS:
                for g in SWEEP_GRIDS:
                    trial({"grow_block": b, "grow_grid": g, "prune_block": b,
                           "prune_grid": g or 2048, "seed_block": sb, "seed_grid": sg,
                           "steps_per_sync": 0, "graphs": 1})
        best_graph = min(results, key=lambda r: r[0])[1]
        trial({**best_graph, "graphs": 0})
    finally:
        qsgs_set_tuning(None)
    wall, best = min(results, key=lambda r: r[0])
    default_wall = next(r[0] for r in results
                        if r[1]["grow_block"] == 256 and r[1]["grow_grid"] == 0
                        and r[1]["seed_block"] == 256 and r[1]["graphs"] == 1)
    entry = {"tuning": best, "wall_ms": wall * 1e3, "candidates": len(results),
             "default_wall_ms": default_wall * 1e3, "speedup_over_default": default_wall / wall,
             "plain_launch_wall_ms": results[-1][0] * 1e3}
    qsgs_set_tuning(best)
    if use_cache:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        cache[key] = entry
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return entry


__all__ = ["autotune", "cache_path", "bucket_of", "qsgs_tuning"]
