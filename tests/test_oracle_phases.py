"""Pins of the oracle's multi-phase generation (Sec. 2.1 steps 1-5): independent growing
phases in sequence, each on the cells no earlier phase holds."""
import numpy as np
import pytest

G1 = (0.02, 0.005, 0.00125)
G2 = (0.03, 0.01, 0.002)


def _phases():
    # (target fraction P^n, core probability, G_ref, spacing, key)
    return [(0.30, 0.004, G1, 4, 11), (0.20, 0.003, G2, 3, 12), (0.15, 0.002, G1, 0, 13)]


def test_one_phase_is_the_single_phase_generation(orc):
    """With one growing phase the label grid is the single-phase grid (0 pore, 1 solid)
    and the phase's result is the single-phase result."""
    for dims, ph in (((24, 20, 17), (0.55, 0.01, G1, 3, 5)),
                     ((33, 9, 21), (0.7, 0.004, G2, 0, 6)),
                     ((16, 16, 16), (0.4, 0.0, G1, 2, 7))):  # no cores: exhausted at once
        labels, res = orc.generate_phases(dims, [ph])
        run = orc.generate(dims, ph[0], ph[1], ph[2], ph[3], ph[4])
        assert np.array_equal(labels, run.grid)
        r = res[0]
        assert (r.n_candidates, r.n_seeds, r.count, r.target_count, r.front_size, r.steps,
                r.status) == (run.n_candidates, run.n_seeds, run.solid_count, run.target_count,
                              run.front_size, run.steps, run.status)


def test_phases_are_disjoint_and_later_phases_leave_earlier_ones(orc):
    dims = (40, 36, 30)
    ph = _phases()
    l2, r2 = orc.generate_phases(dims, ph[:2])
    l3, r3 = orc.generate_phases(dims, ph)
    # phases 1 and 2 are the same with or without phase 3; phase 3 only takes matrix cells
    assert np.array_equal(l3[l2 != 0], l2[l2 != 0])
    assert set(np.unique(l3[l2 == 0]).tolist()) <= {0, 3}
    n = l3.size
    for k, r in enumerate(r3, start=1):
        assert int((l3 == k).sum()) == r.count
        assert r.target_count == orc.target_count(ph[k - 1][0], n)
        if r.status == orc.DONE:
            assert r.count >= r.target_count
    assert [dataclass_tuple(a) for a in r2] == [dataclass_tuple(a) for a in r3[:2]]


def dataclass_tuple(r):
    return (r.n_candidates, r.n_seeds, r.count, r.target_count, r.front_size, r.steps,
            r.status)


def test_cores_only_on_unassigned_cells(orc):
    """Phase 2's candidates are the cells whose core draw passes and that phase 1 does
    not hold (Sec. 2.1 steps 2 and 4)."""
    dims = (30, 28, 26)
    ph = _phases()
    l1, _ = orc.generate_phases(dims, ph[:1])
    _, r2 = orc.generate_phases(dims, ph[:2])
    cand, _ = orc.seed_candidates(dims, ph[1][4], orc.prob_threshold(ph[1][1]))
    free = l1.ravel()[cand] == 0
    assert r2[1].n_candidates == int(free.sum())
    assert r2[1].n_candidates < len(cand)  # phase 1 held some of the drawn cells


@pytest.mark.parametrize("spacing", [0, 3])
def test_later_phase_matches_the_full_field_form(orc, spacing):
    """Phase 2 grown by the list-indexed loop equals phase 2 grown by the full-field
    form (Sec. 2.2, Algorithm 2: every cell of the phase draws per direction and the
    accepted ones are shifted) on the same walled grid, step by step with Eq. (1)."""
    dims = (34, 30, 28)
    nx, ny, nz = dims
    ph = _phases()
    ph2 = (ph[1][0], ph[1][1], ph[1][2], spacing, ph[1][4])
    l1, _ = orc.generate_phases(dims, ph[:1])
    l2, r2 = orc.generate_phases(dims, [ph[0], ph2])
    # full-field regeneration of phase 2: phase-1 cells are walls (value 7)
    g = np.where(l1 == 1, 7, 0).astype(np.uint8)
    cand, prio = orc.seed_candidates(dims, ph2[4], orc.prob_threshold(ph2[1]))
    keep = g.ravel()[cand] == 0
    cand, prio = cand[keep], prio[keep]
    seeded, n_seeds = orc.seed_select(dims, spacing, cand, prio)
    g[seeded == 1] = 1
    assert n_seeds == r2[1].n_seeds
    s_star = orc.target_count(ph2[0], g.size)
    t_ref = [orc.prob_threshold(p) for p in ph2[2]]
    cnt = n_seeds
    t = 0
    while cnt < s_star and t < r2[1].steps:
        T = [orc.growth_threshold(tr, cnt, s_star) for tr in t_ref]
        cnt += orc.step_fullfield(g, t, T, ph2[4])
        t += 1
    assert t == r2[1].steps and cnt == r2[1].count
    assert np.array_equal(g == 1, l2 == 2)
    assert np.array_equal(g == 7, l2 == 1)
