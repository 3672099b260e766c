"""GPU: a grid at the size limit (N just below 2^31 voxels), where no oracle run fits in a
test.  Properties that hold at any size are checked instead: the run is deterministic, the
grid holds only 0 and 1, its number of solid voxels equals the reported count, the count
reaches the target, and the per-step log is consistent (each step's count is the previous
count plus its new voxels, starting from the seeds).
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

DIMS = (2047, 1024, 1024)  # N = 2 146 435 072 < 2^31 = 2 147 483 648


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


def test_largest_grid_properties(q):
    import torch
    n = DIMS[0] * DIMS[1] * DIMS[2]
    assert n < 2**31
    p = q.make_params(0.8, 5e-4, (0.01, 0.0025, 0.000625), 20, 7)
    wsb = q.qsgs_workspace_bytes(DIMS, p)
    gb = q.qsgs_grid_bytes(DIMS)
    assert wsb > 0 and gb >= n
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    grids = [torch.empty(gb, dtype=torch.uint8, device="cuda") for _ in range(2)]
    infos = []
    for k, g in enumerate(grids):
        print("GPU generate at the size limit", DIMS, "run", k, flush=True)
        st, info = q.qsgs_generate(DIMS, p, g, ws, wsb)
        torch.cuda.synchronize()
        infos.append(info)
        assert st == q.DONE, q.STATUS_NAMES.get(st, st)
    a, b = infos
    assert bytes(a) == bytes(b)
    assert torch.equal(grids[0][:n], grids[1][:n])
    g = grids[0][:n]
    assert int(torch.count_nonzero(g > 1)) == 0
    assert int(torch.count_nonzero(g)) == a.solid_count
    assert a.solid_count >= a.target_count == int(np.ceil(0.8 * n))
    assert 0 < a.n_seeds <= a.n_candidates
    lf, ln, lc = q.qsgs_read_step_log(ws, wsb)
    assert len(lf) == a.step and lc[0] == a.n_seeds
    assert np.array_equal(lc[1:], (lc + ln)[:-1])
    assert lc[-1] + ln[-1] == a.solid_count


def test_largest_batch_matches_oracle(q, orc):
    """The largest batch (4096 realizations, tiny uneven grids and mixed parameters): every
    result equals the oracle's run of that realization alone."""
    import torch
    import workloads
    rng = np.random.default_rng(4096)
    cases = []
    for i in range(4096):
        dims = tuple(int(v) for v in rng.integers(3, 13, size=3))
        cases.append(workloads.Case(f"b{i}", dims, round(float(rng.uniform(0.3, 0.9)), 4),
                                    round(float(rng.uniform(0.0, 0.08)), 4),
                                    workloads.g_from_face(round(float(rng.uniform(0.05, 0.5)), 4)),
                                    int(rng.integers(0, 5)), 9000 + i))
    params = [q.params_of(c) for c in cases]
    dims = [c.dims for c in cases]
    grid_bytes = [q.qsgs_grid_bytes(d) for d in dims]
    buf = torch.empty(sum((b + 255) // 256 * 256 for b in grid_bytes), dtype=torch.uint8,
                      device="cuda")
    grids, off = [], 0
    for b in grid_bytes:
        grids.append(buf[off:off + b])
        off += (b + 255) // 256 * 256
    wsb = q.qsgs_batch_workspace_bytes(dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    print("GPU generate_batch of", len(cases), flush=True)
    st, infos = q.qsgs_generate_batch(dims, params, grids, ws, wsb)
    torch.cuda.synchronize()
    host = buf.cpu().numpy()
    off = 0
    for c, info, b in zip(cases, infos, grid_bytes):
        ref = orc.generate(c.dims, c.solid_fraction, c.seed_prob, c.g_ref, c.spacing, c.key)
        nx, ny, nz = c.dims
        assert info.status == ref.status and info.step == ref.steps, c.name
        assert info.solid_count == ref.solid_count, c.name
        assert np.array_equal(host[off:off + c.n].reshape(nz, ny, nx), ref.grid), c.name
        off += (b + 255) // 256 * 256
