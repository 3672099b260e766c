"""Whole-run pins of the oracle's generation loop (Sec. 2.3 step 5, Algorithm 3)."""
import numpy as np
import pytest

from tests import ref_tiny


def _replay_check(orc, dims, run, key, g_ref, spacing):
    """Reconstruct G_t from the birth map and check every step: a voxel born at
    t+1 has a passing draw from a solid neighbour of G_t (reachability), and no
    void voxel of G_{t+1} has one (completeness)."""
    nx, ny, nz = dims
    n = nx * ny * nz
    birth = run.birth.ravel()
    s_star = run.target_count
    t_ref = [orc.prob_threshold(g) for g in g_ref]
    offs = ref_tiny.OFFSETS
    for t in range(run.steps):
        solid = (birth >= 0) & (birth <= t)
        cnt = int(solid.sum())
        assert cnt == run.log_count[t]
        T = [orc.growth_threshold(tr, cnt, s_star) for tr in t_ref]
        grown = set()
        for a in np.flatnonzero(solid):
            ax, ay, az = a % nx, (a // nx) % ny, a // (nx * ny)
            j = 0
            for d, (dx, dy, dz) in enumerate(offs):
                qx, qy, qz = ax + dx, ay + dy, az + dz
                if not (0 <= qx < nx and 0 <= qy < ny and 0 <= qz < nz):
                    continue
                q = qx + nx * (qy + ny * qz)
                if solid[q]:
                    continue
                if orc.growth_draw(key, int(a), t, j) < T[ref_tiny.CLASSES[d]]:
                    grown.add(int(q))
                j += 1
        born = set(int(v) for v in np.flatnonzero(birth == t + 1))
        assert born == grown, t
    assert int((birth >= 0).sum()) == run.solid_count
    assert run.solid_count <= n


def test_small_run_replays_exactly(orc):
    dims = (14, 11, 9)
    g_ref = (0.02, 0.008, 0.002)
    run = orc.generate(dims, 0.6, 0.01, g_ref, 3, key=41, birth=True, log_cap=10000)
    assert run.status == orc.DONE
    _replay_check(orc, dims, run, 41, g_ref, 3)


@pytest.mark.parametrize("key", [0, 1])
def test_config_like_run_invariants(orc, key):
    dims = (48, 40, 32)
    g_ref = (0.02, 0.005, 0.00125)
    run = orc.generate(dims, 0.7, 0.005, g_ref, 4, key=key, birth=True, log_cap=10000)
    n = 48 * 40 * 32
    assert run.status == orc.DONE
    # overshoot: the last step starts below the target and ends at or above it
    assert run.log_count[-1] < run.target_count <= run.solid_count
    # monotone growth; counts follow the per-step new counts
    counts = np.append(run.log_count, run.solid_count)
    assert np.all(np.diff(counts) >= 0)
    assert np.array_equal(np.diff(counts), run.log_new)
    assert run.log_count[0] == run.n_seeds
    # seeds are the birth-0 voxels, pairwise L1 >= s, and form the first front
    seeds = np.flatnonzero(run.birth.ravel() == 0)
    assert len(seeds) == run.n_seeds
    c = np.stack([seeds % 48, (seeds // 48) % 40, seeds // (48 * 40)], -1)
    dist = np.abs(c[:, None] - c[None]).sum(-1)
    np.fill_diagonal(dist, 99)
    assert dist.min() >= 4
    assert run.log_front[0] == len(seeds)  # isolated seeds are all interface cells
    # final grid equals the birth map, front equals the interface
    assert np.array_equal(run.grid.ravel(), (run.birth.ravel() >= 0).astype(np.uint8))
    assert run.front_size == len(orc.interface(run.grid))
    assert run.solid_count == int(run.grid.sum()) < n


def test_replay_with_overlapping_seeds(orc):
    """s <= 1 allows adjacent seeds, so the first front can exclude buried seeds."""
    dims = (10, 9, 8)
    g_ref = (0.05, 0.02, 0.01)
    run = orc.generate(dims, 0.9, 0.35, g_ref, 0, key=9, birth=True, log_cap=1000)
    _replay_check(orc, dims, run, 9, g_ref, 0)
    g0 = (run.birth >= 0) & (run.birth <= 0)
    assert run.log_front[0] == len(orc.interface(g0.astype(np.uint8)))


def test_status_exhausted_without_seeds(orc):
    run = orc.generate((8, 8, 8), 0.5, 0.0, (0.1, 0.1, 0.1), 0, key=1, log_cap=10)
    assert run.status == orc.EXHAUSTED and run.steps == 0 and run.solid_count == 0


def test_status_max_steps_without_growth(orc):
    run = orc.generate((8, 8, 8), 0.5, 0.01, (0.0, 0.0, 0.0), 0, key=1, max_steps=7,
                       log_cap=10)
    assert run.status == orc.MAXSTEPS and run.steps == 7
    assert run.solid_count == run.n_seeds and run.n_seeds > 0


def test_status_done_when_seeds_reach_target(orc):
    run = orc.generate((6, 6, 6), 0.5, 1.0, (0.1, 0.1, 0.1), 0, key=1, log_cap=10)
    assert run.status == orc.DONE and run.steps == 0 and run.solid_count == 216
    assert run.front_size == 0


def test_full_fill_terminates(orc):
    """phi_s = 1 needs every voxel; growth with p = 1 fills the grid."""
    run = orc.generate((7, 6, 5), 1.0, 0.02, (1.0, 1.0, 1.0), 2, key=3, log_cap=100)
    assert run.status == orc.DONE and run.solid_count == 210 and run.front_size == 0


def test_single_voxel_domain(orc):
    run = orc.generate((1, 1, 1), 1.0, 1.0, (0.5, 0.5, 0.5), 5, key=0, log_cap=4)
    assert run.status == orc.DONE and run.solid_count == 1 and run.steps == 0
    run = orc.generate((1, 1, 1), 1.0, 0.0, (0.5, 0.5, 0.5), 5, key=0, log_cap=4)
    assert run.status == orc.EXHAUSTED and run.solid_count == 0


def _void_neighbour_counts(solid):
    """For every voxel, the number of in-domain void neighbours among its 26
    (array shifts over a zero-padded copy: out-of-domain cells count as solid)."""
    nz, ny, nx = solid.shape
    pad = np.ones((nz + 2, ny + 2, nx + 2), dtype=np.int32)
    pad[1:-1, 1:-1, 1:-1] = solid
    void = 1 - pad
    cnt = np.zeros(solid.shape, dtype=np.int32)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == dy == dz == 0:
                    continue
                cnt += void[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
    return cnt


@pytest.mark.parametrize("dims,spacing,key", [((23, 17, 11), 3, 5), ((40, 9, 30), 6, 2)])
def test_step_work_log_matches_front_counts(orc, dims, spacing, key):
    """The per-step work log: the front F_t is the solid voxels with a void neighbour,
    draws_t sums their void-neighbour counts and blocks_t sums ceil(count / 8), all
    recomputed from G_t (rebuilt from the birth map) with array shifts."""
    nx, ny, nz = dims
    run = orc.generate(dims, 0.7, 0.01, (0.1, 0.03, 0.01), spacing, key, birth=True,
                       log_cap=10000)
    assert run.steps > 2
    for t in range(run.steps):
        solid = ((run.birth >= 0) & (run.birth <= t)).astype(np.int32)
        nv = _void_neighbour_counts(solid)
        front = (solid == 1) & (nv > 0)
        assert int(front.sum()) == run.log_front[t]
        assert int(nv[front].sum()) == run.log_draws[t]
        assert int(((nv[front] + 7) // 8).sum()) == run.log_blocks[t]


def _replay_literal(orc, dims, run, key, g_ref):
    """Birth-map replay of the literal Algorithm 3 front (A <- prune(A_new)): the
    sources of step 0 are the seeds, those of step t >= 1 the cells grown in step t - 1;
    a cell is born at t + 1 iff some source has a passing draw to it (rank over the
    source's void neighbours at the step's start)."""
    nx, ny, nz = dims
    birth = run.birth.ravel()
    s_star = run.target_count
    t_ref = [orc.prob_threshold(g) for g in g_ref]
    offs = ref_tiny.OFFSETS
    for t in range(run.steps):
        solid = (birth >= 0) & (birth <= t)
        cnt = int(solid.sum())
        T = [orc.growth_threshold(tr, cnt, s_star) for tr in t_ref]
        sources = np.flatnonzero(birth == t)
        grown = set()
        for a in sources:
            ax, ay, az = a % nx, (a // nx) % ny, a // (nx * ny)
            j = 0
            for d, (dx, dy, dz) in enumerate(offs):
                qx, qy, qz = ax + dx, ay + dy, az + dz
                if not (0 <= qx < nx and 0 <= qy < ny and 0 <= qz < nz):
                    continue
                q = qx + nx * (qy + ny * qz)
                if solid[q]:
                    continue
                if orc.growth_draw(key, int(a), t, j) < T[ref_tiny.CLASSES[d]]:
                    grown.add(int(q))
                j += 1
        born = set(int(v) for v in np.flatnonzero(birth == t + 1))
        assert born == grown, t


def test_literal_front_replays_exactly(orc):
    dims = (13, 12, 10)
    g_ref = (0.06, 0.02, 0.005)
    run = orc.generate(dims, 0.6, 0.01, g_ref, 2, key=77, birth=True, log_cap=10000,
                       literal_front=True)
    assert run.steps >= 3
    _replay_literal(orc, dims, run, 77, g_ref)


def test_literal_front_dies_out_at_paper_like_parameters(orc):
    """At moderate growth probabilities the literal rule drops failed sources and the
    front empties before the target (the reason for the interface reading)."""
    dims = (48, 48, 48)
    g = (0.01, 0.0025, 0.000625)
    lit = orc.generate(dims, 0.8, 0.001, g, 4, key=3, literal_front=True)
    ref = orc.generate(dims, 0.8, 0.001, g, 4, key=3)
    assert ref.status == orc.DONE
    assert lit.status == orc.EXHAUSTED and lit.solid_count < lit.target_count
    assert lit.n_seeds == ref.n_seeds


def test_literal_front_equals_interface_rule_when_every_draw_passes(orc):
    """With every probability 1 each source grows into all its void neighbours, so an
    old source has none left: prune(A u A_new) = prune(A_new) and the runs coincide."""
    dims = (21, 17, 15)
    for key, sp in ((5, 0), (6, 3)):
        a = orc.generate(dims, 0.9, 0.003, (1.0, 1.0, 1.0), sp, key, log_cap=1000)
        b = orc.generate(dims, 0.9, 0.003, (1.0, 1.0, 1.0), sp, key, log_cap=1000,
                         literal_front=True)
        assert np.array_equal(a.grid, b.grid) and a.steps == b.steps
        assert np.array_equal(a.log_front, b.log_front)


def test_band_logs_equal_dilations_of_the_birth_map(orc):
    """The per-step band sizes the oracle logs (cells within one voxel of F_t, and of
    F_t u New_t) equal scipy dilations of the front and new sets rebuilt from the birth
    map: G_t = {birth <= t}, F_t = G_t minus the cells without a void 26-neighbour,
    New_t = {birth = t + 1}."""
    from scipy import ndimage
    dims = (31, 27, 23)
    r = orc.generate(dims, 0.7, 0.01, (0.05, 0.02, 0.005), 3, 9, birth=True, log_cap=1000,
                     bands=True)
    full = ndimage.generate_binary_structure(3, 3)
    for t in range(r.steps):
        g = (r.birth >= 0) & (r.birth <= t)
        front = g & ndimage.binary_dilation(~g, structure=full, border_value=0)
        new = r.birth == t + 1
        assert int(front.sum()) == r.log_front[t]
        assert int(ndimage.binary_dilation(front, structure=full).sum()) == r.log_band[t]
        assert int(ndimage.binary_dilation(front | new, structure=full).sum()) == \
            r.log_band_union[t]
