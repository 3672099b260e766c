"""Benchmark: LIETS-QSGS generation at 400^3 on one MI355X.

One step = one pass of the whole path (seeding with diamond spacing, then the growth
loop to the target) for each of the three 400^3 workloads (porosity 0.10, 0.20, 0.30;
S_d 5e-4; G_ref 0.01/0.0025/0.000625; s = 20; key 1).  The value is voxels grown per
second over the timed steps (grown = final solid count - seeds).

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu-baseline]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# 32-bit integer vector ALU: 256 CUs x 128 lanes x 2.4 GHz.  A SIMD issues one wave64
# 32-bit instruction every two cycles (32 lanes per cycle, 4 SIMDs per CU): the rate behind
# the published 157.3 TFLOP/s fp32 vector peak (one FMA = 2 flops per lane)
ALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
# algorithmic integer ops: a Philox4x32-10 block is 10 rounds of two 32x32->64
# products (2 ops each), four XORs and two key additions; a draw extracts a 16-bit
# half and compares it; a front voxel tests its 26 neighbours
OPS_PER_BLOCK, OPS_PER_DRAW, OPS_PER_FRONT = 100, 2, 26


def sweep_pass_ops(log_front, log_draws, log_blocks, final_front):
    """Algorithmic integer ops of every fused-sweep pass of one generation: a running
    pass finds F_t (26 tests per front voxel) and draws for it; the final pass only
    finds F_T."""
    out = [OPS_PER_BLOCK * b + OPS_PER_DRAW * d + OPS_PER_FRONT * f
           for f, d, b in zip(log_front, log_draws, log_blocks)]
    return out + [OPS_PER_FRONT * final_front]


# occupancy bytes per cell of the growth sweep: one bit per cell and plane
OCC_BYTES = 1.0 / 8.0


def step_bytes(log_front, log_new, band_f, band_u, final_front, g=OCC_BYTES):
    """Algorithmic bytes of every growth step of one generation (the list-indexed step's
    own traffic, not the full-field work it avoids): step t reads F_t (4 B per entry) and
    the occupancy of the one-voxel band around F_t (g B per cell), marks and appends New_t
    (g + 8 B per voxel: the mark, the append and its read back), reads the occupancy of
    the band around F_t u New_t to prune (g B per cell) and writes F_{t+1} (4 B per
    entry):  B_t = 4|F_t| + g|band(F_t)| + (g + 8)|New_t| + g|band(F_t u New_t)|
    + 4|F_{t+1}|."""
    fronts = list(log_front) + [final_front]
    return [4 * fronts[t] + g * band_f[t] + (g + 8) * log_new[t] + g * band_u[t] +
            4 * fronts[t + 1] for t in range(len(log_front))]


def step_api_bands(q, torch, case):
    """Per-step band sizes (|band(F_t)|, |band(F_t u New_t)|) of `case`, from a run of
    the step API (the same grid evolution as qsgs_generate) with the grid copied before
    every step.  Outside every timed region."""
    n = case.n
    p = q.params_of(case)
    grid = torch.empty(q.qsgs_grid_bytes(case.dims), dtype=torch.uint8, device="cuda")
    before = torch.empty_like(grid)
    fa = torch.empty(n, dtype=torch.int32, device="cuda")
    fb = torch.empty(n, dtype=torch.int32, device="cuda")
    wsb = q.qsgs_workspace_bytes(case.dims, p)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    sws = torch.empty(q.qsgs_step_workspace_bytes(), dtype=torch.uint8, device="cuda")
    sb = q.qsgs_band_scratch_bytes(case.dims)
    scratch = torch.empty(sb, dtype=torch.uint8, device="cuda")
    st, info = q.qsgs_seed(case.dims, p, grid, fa, n, ws, wsb)
    bf, bu = [], []
    while st == q.OK:
        before.copy_(grid)
        st, info = q.qsgs_grow_step(case.dims, p, grid, fa, fb, n, sws, sws.numel(), info)
        fa, fb = fb, fa
        f, u = q.qsgs_band_sizes(case.dims, before, grid, scratch, sb)
        bf.append(f)
        bu.append(u)
    return bf, bu


KERNEL_SOURCES = ("qsgs_kernels.hip", "qsgs_device.h", "qsgs_internal.h", "qsgs_host.h")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_sweep_400cube_hbm_traffic.md")


def kernel_source_hash() -> str:
    """First 16 hex digits of the SHA-256 of the sweep kernel's sources and launch set-up."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2602_11734_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(launches_per_step: float):
    """HBM bytes per k_sweep launch (scaled FETCH_SIZE + WRITE_SIZE) from the committed
    counter summary, or None when the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    vals = {}
    with open(TRAFFIC_SUMMARY) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])


def _oracle_job(case):
    """One end-to-end oracle generation (runs in a worker process)."""
    from oracle import oracle
    t0 = time.perf_counter()
    r = oracle.generate(case.dims, case.solid_fraction, case.seed_prob, case.g_ref,
                        case.spacing, case.key)
    return r.solid_count - r.n_seeds, time.perf_counter() - t0, r.steps


def host_cpu() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def cpu_baseline(cases, edge: int = 128, max_workers: int = 16):
    """The oracle (plain single-threaded C, as committed) timed on this host's cores on
    a bounded sample of the headline workload: the 400^3 parameter sets (porosity
    0.10 / 0.20 / 0.30, S_d 5e-4, s = 20, G_ref 0.01 / 0.0025 / 0.000625) on an
    edge^3 grid, each generation end to end (seeding and every growth step).  One
    generation in this process gives the one-core rate; then one generation per worker
    process (porosities in turn, keys 1, 2, ...) over all usable cores (at most
    max_workers) gives the all-cores rate, the value.  Runs before the GPU is touched, so
    the workers are plain forks of a process without GPU state."""
    from concurrent.futures import ProcessPoolExecutor
    import dataclasses
    from oracle import oracle
    oracle.build()
    sample = [dataclasses.replace(c, name=f"{c.name}_at_{edge}", dims=(edge,) * 3)
              for c in cases]
    grown1, dt1, steps1 = _oracle_job(sample[1])
    workers = max(1, min(max_workers, len(os.sched_getaffinity(0))))
    jobs = [dataclasses.replace(sample[j % len(sample)], key=1 + j // len(sample))
            for j in range(workers)]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(_oracle_job, jobs))
    wall = time.perf_counter() - t0
    grown_all = sum(r[0] for r in res)
    out = {"value": grown_all / wall, "unit": "voxels/s", "cores": workers, "kind": "oracle",
           "sample": f"{workers} end-to-end oracle generations in parallel processes, one per "
                     f"core: the 400^3 workload's parameters (porosity 0.10/0.20/0.30 in turn, "
                     f"keys 1..) on {edge}^3 grids; {grown_all} voxels grown in {wall:.1f} s",
           "one_core": {"value": grown1 / dt1, "unit": "voxels/s",
                        "sample": f"{sample[1].name}: {steps1} steps, {grown1} voxels grown "
                                  f"in {dt1:.1f} s"},
           "host": host_cpu()}
    # the full 400^3 oracle runs stored with the golden values (timed when they were
    # written, on the build host, one core each), for scale: the full grid no longer
    # fits the caches, which lowers the rate
    gold = os.path.join(ROOT, "tests", "golden", "oracle_runs.json")
    if os.path.exists(gold):
        with open(gold) as f:
            runs = json.load(f)
        full = {}
        for c in cases:
            e = runs.get(c.name)
            if e and e.get("oracle_seconds"):
                full[c.name] = {"voxels_grown": e["solid_count"] - e["n_seeds"],
                                "seconds": e["oracle_seconds"],
                                "voxels_per_s": (e["solid_count"] - e["n_seeds"]) /
                                e["oracle_seconds"]}
        out["stored_full_400_runs_one_core"] = full
    return out


def batched_vs_plain(q, torch):
    """Realizations/s of the batched workload -- the 64-realization mix (edges
    {96..256}) plus the five 500^3 sandstone-like singletons -- as one qsgs_generate_batch
    (one sweep launch per step over all realizations) against one qsgs_generate per
    realization.  The batch runs with the default launch shape (graph-captured passes),
    with plain launches, and with the shape the autotuner picks on this batch; every
    output is compared byte for byte with the plain path's."""
    from paper_2602_11734_amd import autotune
    cases = workloads.config4() + workloads.config4_singletons()
    dims = [c.dims for c in cases]
    params = [q.params_of(c) for c in cases]
    grids = [torch.empty(q.qsgs_grid_bytes(d), dtype=torch.uint8, device="cuda") for d in dims]
    wsb = q.qsgs_batch_workspace_bytes(dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")

    def batch_once():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q.qsgs_generate_batch(dims, params, grids, ws, wsb)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def best_of(k=3):
        batch_once()  # warm-up (graph capture)
        return min(batch_once() for _ in range(k))

    q.qsgs_set_tuning(None)
    t_default = best_of()
    q.qsgs_set_tuning({**q.qsgs_get_tuning().as_dict(), "graphs": 0})
    t_nograph = best_of()
    q.qsgs_set_tuning(None)
    tuned = autotune.autotune(cases, use_cache=True)
    t_tuned = best_of()
    q.qsgs_set_tuning(None)
    # the plain path, one realization at a time, each output compared
    grid1 = torch.empty(max(q.qsgs_grid_bytes(d) for d in dims), dtype=torch.uint8,
                        device="cuda")
    pws = max(q.qsgs_workspace_bytes(d, p) for d, p in zip(dims, params))
    ws1 = torch.empty(pws, dtype=torch.uint8, device="cuda")
    same = True
    t_plain = 0.0
    for c, p, g in zip(cases, params, grids):
        q.qsgs_generate(c.dims, p, grid1, ws1, pws)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q.qsgs_generate(c.dims, p, grid1, ws1, pws)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        same = same and bool(torch.equal(grid1[:c.n], g[:c.n]))
    n = len(cases)
    return {"workload": "64 realizations, edges {96..256}, porosity U[0.05,0.25], s U{4..30}, "
                        "S_d 5e-4, face 0.01 at 4:1:0.25, keys 0..63; plus five 500^3 "
                        "singletons, porosity 0.05..0.25, s = 30, S_d from the grain-size "
                        "formula (d = 225 um), keys 100..104",
            "realizations": n, "voxels": sum(c.n for c in cases),
            "batched_realizations_per_s": n / t_default,
            "batched_plain_launches_realizations_per_s": n / t_nograph,
            "batched_autotuned_realizations_per_s": n / t_tuned,
            "autotune": tuned,
            "plain_realizations_per_s": n / t_plain,
            "speedup": t_plain / min(t_default, t_tuned),
            "graph_speedup": t_nograph / t_default,
            "identical_outputs": same}


def list_vs_full_field(q, torch, case):
    """The paper's central comparison on this GPU: the list-indexed sweep (LIETS,
    Algorithm 3) against the full-field form (Algorithm 2: every cell draws for all its
    directions every step, then a whole-grid fold) on one realization, plus the tile
    sweep with every tile listed every step (no list); outputs compared byte for byte."""
    out = {"workload": case.name}
    grids = {}
    for form, code in (("list_indexed", q.SWEEP_LIST), ("full_field_alg2", q.SWEEP_FIELD),
                       ("all_tiles", q.SWEEP_ALL_TILES)):
        p = q.params_of(case, sweep_form=code)
        b = q.alloc(case.dims, p)
        q.qsgs_generate(case.dims, p, b.grid, b.ws, b.ws_bytes)  # warm-up
        torch.cuda.synchronize()
        q.qsgs_profile_enable(True)
        q.qsgs_profile_read(reset=True)
        t0 = time.perf_counter()
        st, info = q.qsgs_generate(case.dims, p, b.grid, b.ws, b.ws_bytes)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = q.qsgs_profile_read(reset=True)
        q.qsgs_profile_enable(False)
        out[form] = {"generation_ms": wall * 1e3, "sweep_ms": prof["grow_ms"],
                     "steps": info.step,
                     "voxels_grown_per_s": (info.solid_count - info.n_seeds) / wall}
        grids[form] = b.grid[:case.n].clone()
        del b
    li = out["list_indexed"]["sweep_ms"]
    out["alg2_over_list"] = out["full_field_alg2"]["sweep_ms"] / li
    out["all_tiles_over_list"] = out["all_tiles"]["sweep_ms"] / li
    out["identical_outputs"] = all(bool(torch.equal(grids["list_indexed"], g))
                                   for g in grids.values())
    return out


def voxel_list_step_api(q, torch, case):
    """The paper's literal list-indexed loop through the step API: F_t kept as a voxel
    list, one qsgs_grow_step (grow, then prune of F_t + New_t) per step, the host reading
    the loop state after every step.  Compared with qsgs_generate's tile-indexed sweep on
    the same realization; outputs compared byte for byte."""
    p = q.params_of(case)
    n = case.n
    grid = torch.empty(q.qsgs_grid_bytes(case.dims), dtype=torch.uint8, device="cuda")
    fa = torch.empty(n, dtype=torch.int32, device="cuda")
    fb = torch.empty(n, dtype=torch.int32, device="cuda")
    wsb = q.qsgs_workspace_bytes(case.dims, p)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    swsb = q.qsgs_step_workspace_bytes()
    sws = torch.empty(swsb, dtype=torch.uint8, device="cuda")

    def run():
        st, info = q.qsgs_seed(case.dims, p, grid, fa, n, ws, wsb)
        bufs = (fa, fb)
        k = 0
        while st == 0:
            st, info = q.qsgs_grow_step(case.dims, p, grid, bufs[k], bufs[k ^ 1], n, sws, swsb,
                                        info)
            k ^= 1
        return info

    run()  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps_grid = grid[:n].clone()
    b = q.alloc(case.dims, p)
    q.qsgs_generate(case.dims, p, b.grid, b.ws, b.ws_bytes)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q.qsgs_generate(case.dims, p, b.grid, b.ws, b.ws_bytes)
    torch.cuda.synchronize()
    wall_gen = time.perf_counter() - t0
    return {"workload": case.name, "steps": info.step,
            "voxel_list_ms": wall * 1e3, "tile_sweep_ms": wall_gen * 1e3,
            "speedup": wall / wall_gen,
            "identical_outputs": bool(torch.equal(steps_grid, b.grid[:n]))}


def front_rules(q, torch, case):
    """The two front rules on one 400^3 realization: the interface, prune(F_t u New_t),
    against Algorithm 3 as printed, prune(New_t) (failed sources dropped)."""
    out = {"workload": case.name}
    for rule, lit in (("interface", False), ("literal_alg3", True)):
        p = q.params_of(case, literal_front=lit)
        b = q.alloc(case.dims, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, info = q.qsgs_generate(case.dims, p, b.grid, b.ws, b.ws_bytes)
        torch.cuda.synchronize()
        out[rule] = {"generation_ms": (time.perf_counter() - t0) * 1e3,
                     "status": q.STATUS_NAMES[st], "steps": info.step,
                     "solid_fraction": info.solid_count / case.n,
                     "target_fraction": case.solid_fraction}
        del b
    return out


def multiphase(q, torch):
    """Three independent growing phases in sequence on one 400^3 label grid (Sec. 2.1
    steps 1-5): wall time of qsgs_generate_phases and voxels grown per second over all
    phases (each phase's final count minus its cores)."""
    ps = workloads.phase_bench()
    params = [q.params_of(c) for c in ps.phases]
    gb = q.qsgs_grid_bytes(ps.dims)
    wb = q.qsgs_phases_workspace_bytes(ps.dims, params)
    labels = torch.empty(gb, dtype=torch.uint8, device="cuda")
    ws = torch.empty(wb, dtype=torch.uint8, device="cuda")
    q.qsgs_generate_phases(ps.dims, params, labels, ws, wb)  # warm-up
    torch.cuda.synchronize()
    q.qsgs_profile_enable(True)
    q.qsgs_profile_read(reset=True)
    t0 = time.perf_counter()
    st, infos = q.qsgs_generate_phases(ps.dims, params, labels, ws, wb)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = q.qsgs_profile_read(reset=True)
    q.qsgs_profile_enable(False)
    grown = sum(i.solid_count - i.n_seeds for i in infos)
    n = ps.dims[0] * ps.dims[1] * ps.dims[2]
    counts = torch.bincount(labels[:n].to(torch.int64), minlength=len(params) + 1).tolist()
    return {"workload": "400^3, three phases: P 0.50 / 0.15 / 0.05, S_d 5e-4 / 1e-4 / 2e-3, "
                        "s 20 / 10 / 0, face 0.01 / 0.01 / 0.02 at 4:1:0.25, keys 1 / 2 / 3",
            "generation_ms": wall * 1e3, "sweep_ms": prof["grow_ms"],
            "voxels_grown_per_s": grown / wall,
            "phases": [{"count": i.solid_count, "target": i.target_count, "steps": i.step,
                        "status": q.STATUS_NAMES[i.status]} for i in infos],
            "label_counts": counts,
            "counts_match_labels": counts[1:] == [i.solid_count for i in infos]}


def grid_store(q, torch, reqs):
    """One device buffer with a grid slot (qsgs_grid_bytes, 256-byte aligned) per request;
    returns (buffer, {request id: view})."""
    sizes = [(q.qsgs_grid_bytes(r.case.dims) + 255) // 256 * 256 for r in reqs]
    buf = torch.empty(sum(sizes), dtype=torch.uint8, device="cuda")
    views, off = {}, 0
    for r, sz in zip(reqs, sizes):
        views[r.rid] = buf[off:off + sz]
        off += sz
    return buf, views


def served_vs_plain(q, torch, n_requests: int, loads=(0.8, 1.2), light=(0.2, 300)):
    """The request stream of mixed sizes (cube edge U{64..320}, porosity U[0.05,0.30],
    s U{4..30}, S_d U[5e-4,5e-3], face U[0.005,0.02], key = request id) through the
    continuous-batching server and through the plain one-at-a-time path on the same
    Poisson arrivals.  The server's capacity on the mix (every request present at the
    start) sets the rates: `loads` x capacity for n_requests, plus a light load
    (light[0] x capacity, first light[1] requests).  Every served grid is compared byte
    for byte with the plain path's grid of the same request (both kept on the device)."""
    from paper_2602_11734_amd import serving
    budget = 24 << 30
    slots = 64
    arena = serving.server_arena_bytes(None, slots, budget)
    reqs = workloads.config5(n_requests, rate_per_s=1e9)
    cap = serving.serve_stream(reqs, arena, max_slots=slots, steps_per_tick=4).summary()
    capacity = cap["realizations_per_s"]
    out = {"workload": f"{n_requests} requests, edge U{{64..320}}, porosity U[0.05,0.30], "
                       "s U{4..30}, S_d U[5e-4,5e-3], face U[0.005,0.02] at 4:1:0.25, key = "
                       "request id, Poisson arrivals", "arena_budget_bytes": budget,
           "max_slots": slots, "capacity": cap}
    bufs, views_s = grid_store(q, torch, reqs)
    bufp, views_p = grid_store(q, torch, reqs)
    runs = [(f"load_{f:g}", f, n_requests) for f in loads] + [
        (f"light_load_{light[0]:g}", light[0], light[1])]
    for name, frac, nreq in runs:
        rate = frac * capacity
        rq = workloads.config5(n_requests, rate_per_s=rate)[:nreq]
        served = serving.serve_stream(rq, arena, max_slots=slots, steps_per_tick=4,
                                      out=views_s).summary()
        plain = serving.plain_stream(rq, out=views_p).summary()
        torch.cuda.synchronize()
        same = all(bool(torch.equal(views_s[r.rid][:r.case.n], views_p[r.rid][:r.case.n]))
                   for r in rq)
        out[name] = {"rate_per_s": rate, "requests": nreq, "served": served, "plain": plain,
                     "identical_outputs": same}
    del bufs, bufp
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-edge", type=int, default=128,
                    help="grid edge of the oracle's bounded sample (the 400^3 parameters)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the list-indexed vs full-field comparison")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched vs plain realizations/s measurement")
    ap.add_argument("--no-bands", action="store_true",
                    help="skip the step-API runs that measure the band sizes (the algorithmic "
                         "bytes then leave out the band terms; for profiled runs)")
    ap.add_argument("--no-phases", action="store_true",
                    help="skip the three-phase 400^3 generation")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served vs plain request-stream measurement")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--alu-calibration", action="store_true",
                    help="only measure the 32-bit vector ALU issue rate (1..8 waves per SIMD)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain copy kernel over BYTES bytes three times "
                         "(the reference kernel for scaling HBM byte counters)")
    ap.add_argument("--step-api-only", action="store_true",
                    help="only run the voxel-list step API against qsgs_generate on the 400^3 "
                         "porosity-0.20 realization (for profiling k_grow and k_prune)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(independent realizations shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    # the CPU leg first, before anything touches the GPU (its workers are forks)
    cpu = None
    if not (args.no_cpu_baseline or args.copy_calibration or args.alu_calibration
            or args.step_api_only):
        cpu = cpu_baseline(workloads.config3(), edge=args.cpu_edge)

    import torch

    import paper_2602_11734_amd as q

    if not os.path.exists(q.LIB_PATH):
        from paper_2602_11734_amd import build
        build.build_library()
    q.load()
    torch.cuda.set_device(0)
    if args.alu_calibration:
        rates = {w: q.qsgs_alu_rate(w) / 1e12 for w in range(1, 9)}
        print(json.dumps({"alu_lane_ops_per_s_T_by_waves_per_simd": rates,
                          "peak_T": ALU_PEAK_TOPS,
                          "best_frac_of_peak": max(rates.values()) / ALU_PEAK_TOPS}))
        return
    if args.step_api_only:
        print(json.dumps(voxel_list_step_api(q, torch, workloads.config3()[1])))
        return
    if args.copy_calibration:
        # an elementwise kernel that reads and writes BYTES bytes (a DMA copy would
        # not show up as a kernel dispatch)
        src = torch.ones(args.copy_calibration // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calibration, "copies": 3}))
        return
    cases = workloads.config3()
    params = [q.params_of(c) for c in cases]
    bufs = [q.alloc(c.dims, p) for c, p in zip(cases, params)]  # one workspace per case
    stream = torch.cuda.current_stream()

    def one_step(infos):
        for c, p, b in zip(cases, params, bufs):
            st, info = q.qsgs_generate(c.dims, p, b.grid, b.ws, b.ws_bytes, stream=stream)
            if infos is not None:
                infos.append(info.as_dict())

    for _ in range(args.warmup):
        one_step(None)
    torch.cuda.synchronize()

    q.qsgs_profile_enable(True)
    q.qsgs_profile_read(reset=True)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(infos)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = q.qsgs_profile_read(reset=True)
    q.qsgs_profile_enable(False)
    # every timed step repeats the same three generations (deterministic), so the
    # per-step logs of the last one describe all of them
    logs = [q.qsgs_read_step_log(b.ws, b.ws_bytes, stream=stream) +
            q.qsgs_read_step_work(b.ws, b.ws_bytes, stream=stream) for b in bufs]
    runs = [(c.name, infos[k * len(cases) + i], logs[i])
            for k in range(args.steps) for i, c in enumerate(cases)]

    grown = sum(info["solid_count"] - info["n_seeds"] for _, info, _ in runs)
    value = grown / elapsed
    # algorithmic ops and bytes of the timed sweep launches (every pass of every
    # generation: one per step, plus the final prune-only pass)
    ops = [sweep_pass_ops(lg[0], lg[3], lg[4], info["front_size"]) for _, info, lg in runs]
    launches = sum(len(x) for x in ops)
    assert launches == int(prof["grow_launches"]), (launches, prof)
    bands = ({c.name: step_api_bands(q, torch, c) for c in cases} if not args.no_bands else
             {name: ([0] * len(lg[0]), [0] * len(lg[0])) for name, _, lg in runs})
    sbytes = 0.0
    for name, info, lg in runs:
        bf, bu = bands[name]
        assert len(bf) == len(lg[0]) == info["step"], (name, len(bf), len(lg[0]))
        sbytes += sum(step_bytes(lg[0], lg[1], bf, bu, info["front_size"]))
    sops = sum(sum(x) for x in ops)
    sweep_avg_ms = prof["grow_ms"] / max(launches, 1)
    sweep_s = sweep_avg_ms * 1e-3
    sweep_tops = (sops / launches) / sweep_s / 1e12 if launches else 0.0
    sweep_gbs = (sbytes / launches) / sweep_s / 1e9 if launches else 0.0
    traffic = measured_traffic(launches_per_step=launches / args.steps)
    # the issue rate of plain 32-bit ALU instructions measured on this device (five waves
    # per SIMD, the sweep's occupancy), beside the peak derived from the unit counts
    alu_measured = q.qsgs_alu_rate(5) / 1e12

    per_case = {}
    for name, info, lg in runs:
        lf = lg[0]
        per_case.setdefault(name, {"steps": info["step"], "seeds": info["n_seeds"],
                                   "solid": info["solid_count"], "status": info["status"],
                                   "max_front": int(np.max(lf)) if len(lf) else 0})

    out = {
        "metric": "voxels grown/s & %HBM peak at 400^3; realizations/s + p50/p99 latency "
                  "batched vs plain",
        "value": value,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "400^3 uint8 grid, porosity {0.10,0.20,0.30}, S_d 5e-4, "
                               "G_ref 0.01/0.0025/0.000625, diamond spacing s=20, key 1; "
                               "one step = the three generations end to end",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": sweep_tops, "peak": ALU_PEAK_TOPS,
                     "peak_measured_issue": alu_measured,
                     "unit": "Tops/s (int32)", "frac": sweep_tops / ALU_PEAK_TOPS,
                     "traffic": traffic, "kernel": "k_sweep",
                     "avg_launch_ms": sweep_avg_ms, "launches": launches,
                     "ops_per_launch": sops / max(launches, 1),
                     "hbm_algorithmic": {"achieved": sweep_gbs, "peak": HBM_PEAK_GBS,
                                         "unit": "GB/s", "frac": sweep_gbs / HBM_PEAK_GBS,
                                         "bytes_per_launch": sbytes / max(launches, 1),
                                         "occupancy_bytes_per_cell": OCC_BYTES,
                                         "band_terms": not args.no_bands,
                                         "band_cells": {k: [sum(v[0]), sum(v[1])]
                                                        for k, v in bands.items()}}},
        "detail": {"sweep_ms_total": prof["grow_ms"], "seed_ms_total": prof["seed_ms"],
                   "growth_only_voxels_per_s": grown / (prof["grow_ms"] * 1e-3),
                   "n_over_t_per_realization": cases[0].n * 3 * args.steps / elapsed,
                   "realizations": per_case},
    }
    if not args.no_compare:
        out["detail"]["voxel_list_vs_tiles"] = voxel_list_step_api(q, torch, cases[1])
        out["detail"]["list_vs_full_field"] = [
            list_vs_full_field(q, torch, cases[1]),
            list_vs_full_field(q, torch, workloads.config4_singletons()[3])]
        out["detail"]["front_rules"] = front_rules(q, torch, cases[1])
    if not args.no_batch:
        out["detail"]["batched"] = batched_vs_plain(q, torch)
    if not args.no_phases:
        out["detail"]["multiphase"] = multiphase(q, torch)
    if not args.no_serve:
        out["detail"]["serving"] = served_vs_plain(q, torch, args.serve_requests)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
