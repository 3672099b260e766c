"""GPU parity at the full sizes of the batched and served workloads: the oracle's stored
results (tests/golden/oracle_runs.json, written by tests/golden/make_goldens.py from the
oracle alone) for the 64-realization mix (edges 96..256, s 4..30), the 500^3
sandstone-like singletons (s = 30, S_d from the grain-size formula) and requests of the
serving stream (edges up to 320, S_d up to 5e-3) are reproduced through the batched
call and through the continuous-batching server, mixed with small cases, grid SHA-256
and per-step logs compared.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "oracle_runs.json")


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_11734_amd as q
    if not os.path.exists(q.LIB_PATH):
        from paper_2602_11734_amd import build
        build.build_library()
    q.load()
    return q


@pytest.fixture(scope="module")
def gold():
    with open(GOLDEN) as f:
        return json.load(f)


def say(*a):
    print(*a, flush=True)


def case_of(entry):
    c = entry["case"]
    return workloads.Case(**{**c, "dims": tuple(c["dims"]), "g_ref": tuple(c["g_ref"])})


def sha(t, n):
    return hashlib.sha256(t[:n].cpu().numpy().tobytes()).hexdigest()


def check_info(info, e, name):
    assert info.status == e["status"], name
    assert info.n_candidates == e["n_candidates"] and info.n_seeds == e["n_seeds"], name
    assert info.step == e["steps"] and info.solid_count == e["solid_count"], name
    assert info.front_size == e["front_size"], name


def test_golden_groups_present(gold):
    """The stored results cover the whole 64-realization mix, the five 500^3 singletons
    and the serving requests picked for parity."""
    names = set(gold)
    assert {c.name for c in workloads.config4()} <= names
    assert {c.name for c in workloads.config4_singletons()} <= names
    assert {c.name for c in workloads.config5_parity()} <= names


def test_config4_mix_and_singletons_in_one_batch(q, orc, gold):
    """All 64 realizations of the mix, two 500^3 singletons (porosity 0.05 and 0.25) and
    small cases in one qsgs_generate_batch: each equals the oracle's stored (or live, for
    the small cases) run of that realization alone, with its per-step logs."""
    import torch
    big = workloads.config4() + [workloads.config4_singletons()[i] for i in (0, 4)]
    small = workloads.small_cases()[:6]
    cases = big + small
    params = [q.params_of(c) for c in cases]
    dims = [c.dims for c in cases]
    grids = [torch.empty(q.qsgs_grid_bytes(d), dtype=torch.uint8, device="cuda") for d in dims]
    wsb = q.qsgs_batch_workspace_bytes(dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    say("GPU generate_batch: config-4 mix + 2 x 500^3 + small,", len(cases), "realizations")
    st, infos = q.qsgs_generate_batch(dims, params, grids, ws, wsb)
    torch.cuda.synchronize()
    for k, (c, g, info) in enumerate(zip(cases, grids, infos)):
        if c in small:
            ref = orc.generate(c.dims, c.solid_fraction, c.seed_prob, c.g_ref, c.spacing, c.key,
                               max_steps=c.max_steps)
            nx, ny, nz = c.dims
            assert info.status == ref.status and info.step == ref.steps, c.name
            assert np.array_equal(g[:c.n].view(nz, ny, nx).cpu().numpy(), ref.grid), c.name
            continue
        e = gold[c.name]
        check_info(info, e, c.name)
        lf, ln, lc = q.qsgs_read_step_log(ws, wsb, index=k)
        m = min(e["steps"], 4096)
        assert len(lf) == m, c.name
        assert list(lf) == e["log_front"][:m] and list(ln) == e["log_new"][:m], c.name
        assert list(lc) == e["log_count"][:m], c.name
        ld, lb = q.qsgs_read_step_work(ws, wsb, index=k)
        assert list(ld) == e["log_draws"][:m] and list(lb) == e["log_blocks"][:m], c.name
        assert sha(g, c.n) == e["grid_sha256"], c.name


def _serve(q, cases, params, arena_bytes, slots, steps_per_tick, stagger):
    """Runs `cases` through a server; returns {index: (device grid, info)}."""
    import torch
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    srv = q.qsgs_server_create(arena, arena_bytes, slots, steps_per_tick=steps_per_tick)
    out = {}
    max_res = 0
    try:
        free0 = q.qsgs_server_free_bytes(srv)
        pending = list(range(len(cases)))
        ticks = 0
        while len(out) < len(cases):
            for _ in range(stagger if ticks == 0 else (1 if ticks % 3 == 0 else 0)):
                if pending:
                    k = pending.pop(0)
                    q.qsgs_server_submit(srv, k, cases[k].dims, params[k])
            res, queued, nready = q.qsgs_server_tick(srv)
            max_res = max(max_res, res)
            for rid, info in q.qsgs_server_ready(srv):
                dst = torch.empty(q.qsgs_grid_bytes(cases[rid].dims), dtype=torch.uint8,
                                  device="cuda")
                q.qsgs_server_take(srv, rid, dst, dst.numel(), dst_on_host=False)
                out[rid] = (dst, info)
            ticks += 1
            assert ticks < 20000
        assert q.qsgs_server_free_bytes(srv) == free0
    finally:
        q.qsgs_server_destroy(srv)
    return out, max_res


def test_serving_requests_through_the_server(q, gold):
    """The serving stream's parity requests (its first 12 and the 4 heaviest-seeded with
    edge >= 300 and s >= 25), two config-4 realizations and a 500^3 singleton through one
    server whose arena holds only a few of them at once: admission binds, requests
    overlap, and every result equals the oracle's stored run of that request alone."""
    cases = workloads.config5_parity() + [workloads.config4()[i] for i in (0, 1)] + \
        [workloads.config4_singletons()[2]]
    params = [q.params_of(c) for c in cases]
    slots = 8
    # the 500^3 request alone needs about 2.8 GB with its seeding scratch
    arena_bytes = q.qsgs_server_reserved_bytes(slots) + (3 << 30)
    say("GPU server: serving-stream parity requests,", len(cases), "requests")
    out, max_res = _serve(q, cases, params, arena_bytes, slots, 3, stagger=5)
    assert max_res >= 2
    for k, c in enumerate(cases):
        g, info = out[k]
        e = gold[c.name]
        check_info(info, e, c.name)
        assert sha(g, c.n) == e["grid_sha256"], c.name
