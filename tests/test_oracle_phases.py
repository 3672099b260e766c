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


# ----- interacting phases (Sec. 2.1 step 4: phase n grows into a neighbour held by an
# earlier phase m with the interaction probability I_i^{n,m}) -----

def _zero_interaction(k):
    return np.zeros((k, k, 3))


def test_zero_interaction_is_the_independent_generation(orc):
    """With every I = 0 no cell of another phase is a candidate, so the interacting
    generation is the independent one, label for label and result for result."""
    import workloads
    for ps in workloads.phase_sets():
        ph = [(c.solid_fraction, c.seed_prob, c.g_ref, c.spacing, c.key, c.max_steps)
              for c in ps.phases]
        la, ra = orc.generate_phases(ps.dims, ph)
        lb, rb = orc.generate_phases(ps.dims, ph, _zero_interaction(len(ph)))
        assert np.array_equal(la, lb), ps.name
        assert [dataclass_tuple(a) for a in ra] == [dataclass_tuple(b) for b in rb], ps.name


def _geodesic(seeds, void, other, face_only_other, steps):
    """Growth with probability 1 into unassigned cells through all 26 neighbours and into
    cells of an interacting phase through face neighbours only (or all 26), each step
    from the step's start: a sequence of binary dilations (scipy.ndimage)."""
    from scipy import ndimage
    full = ndimage.generate_binary_structure(3, 3)
    face = ndimage.generate_binary_structure(3, 1)
    s = seeds.copy()
    for _ in range(steps):
        grow_v = ndimage.binary_dilation(s, structure=full, border_value=0) & void & ~s
        st = face if face_only_other else full
        grow_o = ndimage.binary_dilation(s, structure=st, border_value=0) & other & ~s
        s = s | grow_v | grow_o
    return s


@pytest.mark.parametrize("face_only", [True, False])
@pytest.mark.parametrize("steps", [1, 3])
def test_certain_interaction_is_a_geodesic_dilation(orc, face_only, steps):
    """Phase 3 with G = 1 for every class grows into every unassigned neighbour; with
    I^{3,1} = 1 (face class only, or every class) it also takes phase-1 neighbours
    through those directions; phase 2 (I^{3,2} = 0) blocks it.  After k steps phase 3
    is the dilation of its cores computed by scipy, restricted step by step."""
    dims = (26, 22, 19)
    nx, ny, nz = dims
    ph = [(0.30, 0.01, G1, 3, 61), (0.15, 0.006, G2, 2, 62),
          (1.0, 0.003, (1.0, 1.0, 1.0), 0, 63, steps)]
    I = _zero_interaction(3)
    I[2, 0] = (1.0, 0.0, 0.0) if face_only else (1.0, 1.0, 1.0)
    before, _ = orc.generate_phases(dims, ph[:2])
    labels, res = orc.generate_phases(dims, ph, I)
    cand, _ = orc.seed_candidates(dims, 63, orc.prob_threshold(0.003))
    seeds = np.zeros(before.size, bool)
    seeds[cand[before.ravel()[cand] == 0]] = True
    seeds = seeds.reshape(before.shape)
    assert res[2].n_seeds == int(seeds.sum()) > 0
    want = _geodesic(seeds, before == 0, before == 1, face_only, steps)
    assert np.array_equal(labels == 3, want)
    # phase 2 never changes; phase 1 keeps what phase 3 did not take
    assert np.array_equal(labels == 2, before == 2)
    assert np.array_equal(labels == 1, (before == 1) & ~want)
    assert int((labels == 1).sum()) < int((before == 1).sum())  # some cells were converted
    assert res[2].steps == steps and res[2].status == orc.MAXSTEPS
    assert res[2].count == int(want.sum())


def _step_stats(orc, labels0, I_thr, G_thr, keys):
    """Per-direction conversions of a lone phase-n cell at the centre of a 3^3 grid whose
    26 neighbours hold `labels0` (0 or 4 = a cell of phase 1) over many keys."""
    cand = np.zeros(256, np.uint8)
    cand[0] = cand[4] = 1
    thr = np.zeros((256, 3), np.uint64)
    thr[0] = G_thr
    thr[4] = I_thr
    att = np.zeros(52, np.uint64)
    suc = np.zeros(52, np.uint64)
    for key in keys:
        g = np.asarray(labels0, np.uint8).reshape(3, 3, 3).copy()
        g[1, 1, 1] = 1
        _, conv, a, s = orc.step_interacting(g, cand, thr, np.array([13], np.int32), 0, key,
                                             counters=True)
        att += a
        suc += s
        assert len(conv) == int(s.sum())
    return att, suc


def test_interaction_frequencies_per_direction_and_target(orc):
    """One step from a lone cell: every neighbour is a candidate (rank j = direction j),
    an unassigned target converts with the Eq. (1) threshold of its class and a phase-1
    target with I of its class.  26-bin chi-square of the conversion counts against
    those probabilities, over 6000 keys."""
    from scipy import stats
    rng = np.random.default_rng(7)
    lab = np.where(rng.random(27) < 0.5, 4, 0).astype(np.uint8)
    lab[13] = 1
    G = [orc.prob_threshold(p) for p in (0.30, 0.20, 0.10)]
    I = [orc.prob_threshold(p) for p in (0.15, 0.45, 0.05)]
    K = 6000
    att, suc = _step_stats(orc, lab, I, G, range(K))
    obs, exp = [], []
    for d in range(26):
        dx, dy, dz, cls = orc.direction(d)
        v = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)
        other = lab[v] == 4
        idx = d + (26 if other else 0)
        assert att[idx] == K and att[d + (0 if other else 26)] == 0
        p = (I if other else G)[cls] / 2**32
        obs.append(int(suc[idx]))
        exp.append(K * p)
    obs, exp = np.array(obs, float), np.array(exp)
    chi2 = float((((obs - exp) ** 2) / (exp * (1 - exp / K))).sum())
    assert stats.chi2.sf(chi2, 26) > 1e-4, chi2


def test_non_interacting_neighbours_take_no_rank(orc):
    """A neighbour of a phase that phase n does not interact with is no candidate: it
    takes no rank, so the candidates after it draw the ranks the independent rule gives
    them.  Checked on a state where phase-2 cells (label 5) sit between candidates."""
    rng = np.random.default_rng(11)
    lab = rng.choice([0, 4, 5], size=27).astype(np.uint8)
    lab[13] = 1
    cand = np.zeros(256, np.uint8)
    cand[0] = cand[4] = 1
    thr = np.zeros((256, 3), np.uint64)
    thr[0] = [orc.prob_threshold(0.5)] * 3
    thr[4] = [orc.prob_threshold(0.5)] * 3
    for key in range(200):
        g = lab.reshape(3, 3, 3).copy()
        _, conv = orc.step_interacting(g, cand, thr, np.array([13], np.int32), 2, key)
        want = []
        j = 0
        for d in range(26):
            dx, dy, dz, cls = orc.direction(d)
            v = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)
            if lab[v] in (0, 4):
                if orc.growth_draw(key, 13, 2, j) < thr[lab[v], cls]:
                    want.append(v)
                j += 1
        assert sorted(conv.tolist()) == sorted(want)
        assert all(g.ravel()[v] == 1 for v in want)
        assert all(g.ravel()[v] == 5 for v in range(27) if lab[v] == 5)
