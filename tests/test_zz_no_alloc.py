"""The allocation-free entry point (qsgs_generate_noalloc) against qsgs_generate.

Both run on the GPU through the C ABI; the scratch-array variant must give the same
grid and the same counts as the workspace variant, call after call, when a smaller
grid follows a larger one (the scratch keeps the previous call's contents) and when
the larger one comes again.  Grids beyond the scratch are refused before any launch.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2602_11734_amd as q
    q.load()
    return q


def _by_name(name):
    for c in workloads.small_cases() + workloads.config1():
        if c.name == name:
            return c
    raise KeyError(name)


def _run_both(q, case):
    import torch
    params = q.params_of(case)
    ref_view, ref_info, _ = q.generate(case.dims, params)
    ref = ref_view.cpu().numpy().copy()
    gb = q.qsgs_grid_bytes(case.dims)
    grid = torch.full((gb,), 0xAB, dtype=torch.uint8, device="cuda")
    st, info = q.qsgs_generate_noalloc(case.dims, params, grid)
    torch.cuda.synchronize()
    nx, ny, nz = case.dims
    got = grid[: nx * ny * nz].view(nz, ny, nx).cpu().numpy()
    return st, info.as_dict(), got, ref_info, ref


@pytest.mark.parametrize("names", [("c1_64", "ragged_37x23x19", "c1_64"),
                                   ("spacing2_many", "two_voxels", "no_spacing_dense")])
def test_noalloc_equals_generate_on_consecutive_calls(q, names):
    for name in names:  # the second call is smaller than the first
        case = _by_name(name)
        print("noalloc case", name, case.dims, flush=True)
        st, info, got, ref_info, ref = _run_both(q, case)
        assert st == ref_info["status"]
        for k in ("n_candidates", "n_seeds", "solid_count", "target_count", "front_size",
                  "grown_last_step", "step", "status"):
            assert info[k] == ref_info[k], (name, k, info[k], ref_info[k])
        assert np.array_equal(got, ref), name


def test_noalloc_matches_oracle(q, orc):
    case = workloads.config1()[0]
    import torch
    gb = q.qsgs_grid_bytes(case.dims)
    grid = torch.zeros(gb, dtype=torch.uint8, device="cuda")
    st, info = q.qsgs_generate_noalloc(case.dims, q.params_of(case), grid)
    torch.cuda.synchronize()
    r = orc.generate(case.dims, case.solid_fraction, case.seed_prob, case.g_ref, case.spacing,
                     case.key)
    nx, ny, nz = case.dims
    assert st == r.status and info.solid_count == r.solid_count and info.step == r.steps
    assert np.array_equal(grid[: nx * ny * nz].view(nz, ny, nx).cpu().numpy(), r.grid)


def test_noalloc_refuses_grids_beyond_its_scratch(q):
    import torch
    case = workloads.config3()[1]  # 400^3 needs far more than the scratch
    grid = torch.zeros(16, dtype=torch.uint8, device="cuda")  # never written: refused first
    with pytest.raises(q.QsgsError) as e:
        q.qsgs_generate_noalloc(case.dims, q.params_of(case), grid)
    assert e.value.status == q.ERR_WORKSPACE
    assert "scratch" in q.qsgs_last_error()
    assert int(grid.sum().item()) == 0
    # the workspace entry point is unaffected, and the scratch variant works afterwards
    small = _by_name("ragged_37x23x19")
    st, info, got, ref_info, ref = _run_both(q, small)
    assert info["solid_count"] == ref_info["solid_count"] and np.array_equal(got, ref)
