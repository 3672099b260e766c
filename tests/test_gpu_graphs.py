"""GPU: graph-captured passes and the autotuner.

Passes issued as launches of captured chunk graphs must give the oracle's results on
every replay (the graphs are cached and replayed by later calls, with other work and
host synchronisation between the replays), the same as plain launches; the autotuner
must pick a launch shape under which the results are unchanged.
"""
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


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
    yield q
    q.qsgs_set_tuning(None)


def say(*a):
    print(*a, flush=True)


def oracle_grids(orc, cases):
    return [orc.generate(c.dims, c.solid_fraction, c.seed_prob, c.g_ref, c.spacing, c.key,
                         max_steps=c.max_steps) for c in cases]


def run_batch(q, cases):
    import torch
    params = [q.params_of(c) for c in cases]
    dims = [c.dims for c in cases]
    grids = [torch.empty(q.qsgs_grid_bytes(d), dtype=torch.uint8, device="cuda") for d in dims]
    wsb = q.qsgs_batch_workspace_bytes(dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    return dims, params, grids, ws, wsb


@pytest.mark.parametrize("graphs", [1, 0], ids=["graphs", "plain_launches"])
def test_batch_replays_match_oracle(q, orc, graphs):
    """One workspace, four batched generations in a row (the later ones replay the cached
    graphs), each checked against the oracle; host-side work and a torch kernel run
    between the replays."""
    import torch
    q.qsgs_set_tuning({**q.qsgs_get_tuning().as_dict(), "graphs": graphs})
    try:
        cases = workloads.small_cases()[:8] + workloads.config1()
        refs = oracle_grids(orc, cases)
        dims, params, grids, ws, wsb = run_batch(q, cases)
        junk = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
        for rep in range(4):
            for g in grids:
                g.fill_(0x5A)  # stale contents must not matter
            say("GPU generate_batch, graphs", graphs, "replay", rep)
            st, infos = q.qsgs_generate_batch(dims, params, grids, ws, wsb)
            torch.cuda.synchronize()
            for c, g, info, ref in zip(cases, grids, infos, refs):
                nx, ny, nz = c.dims
                assert info.status == ref.status and info.step == ref.steps, (c.name, rep)
                assert np.array_equal(g[:c.n].view(nz, ny, nx).cpu().numpy(), ref.grid), \
                    (c.name, rep)
            junk.add_(rep)  # eager work between replays
            torch.cuda.synchronize()
    finally:
        q.qsgs_set_tuning(None)


def test_single_generation_replays_match_oracle(q, orc):
    """qsgs_generate three times in a row on one workspace with graphs on (chunk graphs of
    several lengths are captured by the first call and replayed by the next)."""
    import torch
    q.qsgs_set_tuning(None)
    case = workloads.config1()[0]
    ref = oracle_grids(orc, [case])[0]
    params = q.params_of(case)
    buf = q.alloc(case.dims, params)
    for rep in range(3):
        buf.grid.fill_(0xA5)
        say("GPU generate with graphs, replay", rep)
        st, info = q.qsgs_generate(case.dims, params, buf.grid, buf.ws, buf.ws_bytes)
        torch.cuda.synchronize()
        nx, ny, nz = case.dims
        assert info.step == ref.steps and info.solid_count == ref.solid_count
        assert np.array_equal(buf.grid[:case.n].view(nz, ny, nx).cpu().numpy(), ref.grid)


def test_autotune_keeps_results(q, orc):
    """The autotuner on a small batch (no cache): it reports its candidates and picks a
    shape; the batch generated under that shape equals the oracle."""
    import torch
    from paper_2602_11734_amd import autotune
    cases = workloads.small_cases()[:6] + workloads.config1()
    refs = oracle_grids(orc, cases)
    try:
        say("GPU autotune on", len(cases), "realizations")
        entry = autotune.autotune(cases, repeats=1, use_cache=False)
        assert entry["candidates"] == (len(autotune.SEED_SHAPES) * len(autotune.SWEEP_BLOCKS) *
                                       len(autotune.SWEEP_GRIDS) + 1)
        assert entry["wall_ms"] <= entry["default_wall_ms"]
        t = q.qsgs_get_tuning().as_dict()
        assert t == entry["tuning"]
        dims, params, grids, ws, wsb = run_batch(q, cases)
        q.qsgs_generate_batch(dims, params, grids, ws, wsb)
        torch.cuda.synchronize()
        for c, g, ref in zip(cases, grids, refs):
            nx, ny, nz = c.dims
            assert np.array_equal(g[:c.n].view(nz, ny, nx).cpu().numpy(), ref.grid), c.name
    finally:
        q.qsgs_set_tuning(None)
