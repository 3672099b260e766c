"""GPU: the whole-generation calls that never synchronise with the host.

qsgs_generate_async / qsgs_generate_batch_async enqueue the whole generation and write
qsgs_info to device memory; their results equal the oracle's (and so qsgs_generate's).
One call is captured into a graph with torch.cuda.graph and replayed several times, with
eager work and synchronisation between the replays; every replay equals the oracle.
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
    return q


def say(*a):
    print(*a, flush=True)


def capped(case, steps=400):
    return workloads.Case(**{**case.as_dict(), "max_steps": case.max_steps or steps})


def oracle(orc, c):
    return orc.generate(c.dims, c.solid_fraction, c.seed_prob, c.g_ref, c.spacing, c.key,
                        max_steps=c.max_steps, log_cap=100000)


def check(q, c, grid, info, ref):
    nx, ny, nz = c.dims
    assert info.status == ref.status, c.name
    assert info.step == ref.steps and info.solid_count == ref.solid_count, c.name
    assert info.n_seeds == ref.n_seeds and info.front_size == ref.front_size, c.name
    assert np.array_equal(grid[:c.n].view(nz, ny, nx).cpu().numpy(), ref.grid), c.name


CASES = [capped(c) for c in workloads.small_cases()[:10] + workloads.config1()]


@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_async_generate_matches_oracle(q, orc, case):
    import torch
    params = q.params_of(case)
    buf = q.alloc(case.dims, params)
    d_info = torch.zeros(q.INFO_BYTES, dtype=torch.uint8, device="cuda")
    say("GPU generate_async", case.name, case.dims)
    q.qsgs_generate_async(case.dims, params, buf.grid, buf.ws, buf.ws_bytes, d_info)
    torch.cuda.synchronize()
    info = q.info_from_device(d_info)
    ref = oracle(orc, case)
    check(q, case, buf.grid, info, ref)
    lf, ln, lc = q.qsgs_read_step_log(buf.ws, buf.ws_bytes)
    assert np.array_equal(lf, ref.log_front) and np.array_equal(ln, ref.log_new)


def test_async_batch_matches_oracle(q, orc):
    import torch
    cases = CASES
    params = [q.params_of(c) for c in cases]
    dims = [c.dims for c in cases]
    grids = [torch.empty(q.qsgs_grid_bytes(d), dtype=torch.uint8, device="cuda") for d in dims]
    wsb = q.qsgs_batch_workspace_bytes(dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    d_infos = torch.zeros(q.INFO_BYTES * len(cases), dtype=torch.uint8, device="cuda")
    say("GPU generate_batch_async of", len(cases))
    q.qsgs_generate_batch_async(dims, params, grids, ws, wsb, d_infos)
    torch.cuda.synchronize()
    for k, (c, g) in enumerate(zip(cases, grids)):
        check(q, c, g, q.info_from_device(d_infos, k), oracle(orc, c))


def test_async_rejects_unbounded_steps(q):
    import torch
    case = workloads.config1()[0]  # max_steps 0: unbounded
    params = q.params_of(case)
    buf = q.alloc(case.dims, params)
    d_info = torch.zeros(q.INFO_BYTES, dtype=torch.uint8, device="cuda")
    with pytest.raises(q.QsgsError) as e:
        q.qsgs_generate_async(case.dims, params, buf.grid, buf.ws, buf.ws_bytes, d_info)
    assert e.value.status == q.ERR_INVALID


def test_async_generate_captured_in_a_graph(q, orc):
    """The 64^3 generation captured once into a graph and replayed three times (the grid
    poisoned and a torch kernel run between replays): each replay equals the oracle."""
    import torch
    case = capped(workloads.config1()[0], 64)
    ref = oracle(orc, case)
    params = q.params_of(case)
    buf = q.alloc(case.dims, params)
    d_info = torch.zeros(q.INFO_BYTES, dtype=torch.uint8, device="cuda")
    junk = torch.zeros(1 << 20, dtype=torch.float32, device="cuda")
    # one eager call first: the library's per-device set-up happens outside the capture
    q.qsgs_generate_async(case.dims, params, buf.grid, buf.ws, buf.ws_bytes, d_info)
    torch.cuda.synchronize()
    check(q, case, buf.grid, q.info_from_device(d_info), ref)
    g = torch.cuda.CUDAGraph()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        say("capturing generate_async into a graph")
        with torch.cuda.graph(g, stream=stream):
            q.qsgs_generate_async(case.dims, params, buf.grid, buf.ws, buf.ws_bytes, d_info,
                                  stream=stream)
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    for rep in range(3):
        buf.grid.fill_(0x77)
        d_info.zero_()
        junk.add_(1.0)
        torch.cuda.synchronize()
        say("graph replay", rep)
        g.replay()
        torch.cuda.synchronize()
        check(q, case, buf.grid, q.info_from_device(d_info), ref)
