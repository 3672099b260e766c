"""GPU: the per-step band sizes (the occupancy a growth step reads, used for the
algorithmic byte count of a step) against the oracle's logged band sizes.

The step API advances one step at a time; before each step the grid is copied, and
qsgs_band_sizes(before, after) must equal the oracle's |band(F_t)| and
|band(F_t u New_t)| of that step, for every step.
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


def step_api_bands(q, case):
    """Band sizes of every step of the step-API run of `case`."""
    import torch
    nx, ny, nz = case.dims
    n = nx * ny * nz
    params = q.params_of(case)
    grid = torch.empty(q.qsgs_grid_bytes(case.dims), dtype=torch.uint8, device="cuda")
    wsb = q.qsgs_workspace_bytes(case.dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    sws = torch.empty(q.qsgs_step_workspace_bytes(), dtype=torch.uint8, device="cuda")
    fa = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    fb = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    sb = q.qsgs_band_scratch_bytes(case.dims)
    scratch = torch.empty(sb, dtype=torch.uint8, device="cuda")
    print("GPU step-API bands", case.name, case.dims, flush=True)
    st, info = q.qsgs_seed(case.dims, params, grid, fa, n, ws, wsb)
    bands = []
    while st == q.OK:
        before = grid.clone()
        st, info = q.qsgs_grow_step(case.dims, params, grid, fa, fb, n, sws, sws.numel(), info)
        fa, fb = fb, fa
        bands.append(q.qsgs_band_sizes(case.dims, before, grid, scratch, sb))
    return bands, info


CASES = [workloads.config1()[0]] + [workloads.small_cases()[i] for i in (0, 1, 2, 6, 8, 9)]


@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_band_sizes_match_oracle_logs(q, orc, case):
    bands, info = step_api_bands(q, case)
    ref = orc.generate(case.dims, case.solid_fraction, case.seed_prob, case.g_ref, case.spacing,
                       case.key, max_steps=case.max_steps, log_cap=100000, bands=True)
    assert info.step == ref.steps == len(bands)
    got_f = np.array([b[0] for b in bands], dtype=np.int64)
    got_u = np.array([b[1] for b in bands], dtype=np.int64)
    assert np.array_equal(got_f, ref.log_band)
    assert np.array_equal(got_u, ref.log_band_union)


def test_band_sizes_of_hand_made_grids(q):
    """A single solid voxel inside a 5^3 grid: F = that voxel, band = its 27 cells; a
    voxel grown next to it on the +x face adds the 9 cells of the next x plane."""
    import torch
    dims = (5, 5, 5)
    n = 125
    before = torch.zeros(q.qsgs_grid_bytes(dims), dtype=torch.uint8, device="cuda")
    before[2 + 5 * (2 + 5 * 2)] = 1
    after = before.clone()
    after[3 + 5 * (2 + 5 * 2)] = 1
    sb = q.qsgs_band_scratch_bytes(dims)
    scratch = torch.empty(sb, dtype=torch.uint8, device="cuda")
    assert q.qsgs_band_sizes(dims, before, before, scratch, sb) == (27, 27)
    assert q.qsgs_band_sizes(dims, before, after, scratch, sb) == (27, 36)
    # a corner voxel of the domain: its band is the 2 x 2 x 2 corner block
    c = torch.zeros_like(before)
    c[0] = 1
    assert q.qsgs_band_sizes(dims, c, c, scratch, sb) == (8, 8)
    # an all-solid grid has no front
    full = torch.ones_like(before)
    assert q.qsgs_band_sizes(dims, full[:n].contiguous(), full, scratch, sb) == (0, 0)


def test_alu_rate_is_plausible(q):
    """The measured 32-bit ALU issue rate: positive, below the chip's unit-count peak
    (256 compute units x 128 lanes x 2.4 GHz), rising with waves per SIMD."""
    peak = 256 * 128 * 2.4e9
    r1, r8 = q.qsgs_alu_rate(1), q.qsgs_alu_rate(8)
    assert 0 < r1 < r8 <= 1.05 * peak
