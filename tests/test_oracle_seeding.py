"""Pins of the oracle's seeding: candidate draw (Sec. 2.1 step 2) and diamond
(L1) seed spacing (Sec. 2.3, Fig. 1D) with greedy acceptance by priority."""
import itertools

import numpy as np
import pytest

from tests import ref_tiny


def test_candidates_match_bigint_coding(orc):
    dims = (5, 4, 3)
    for key in (0, 1, 2**40 + 3):
        t = orc.prob_threshold(0.3)
        cand, prio = orc.seed_candidates(dims, key, t)
        want = ref_tiny.seed_candidates(dims, key, t)
        assert [int(c) for c in cand] == [c for c, _ in want]
        assert [int(p) for p in prio] == [p for _, p in want]


def test_candidate_count_is_binomial(orc):
    """With s <= 1 the seeds are the candidates and their number is
    Binomial(N, T_seed / 2^32); z-scores over keys stay small and average ~0."""
    dims = (40, 30, 20)
    n = 40 * 30 * 20
    p_prob = 0.01
    t = orc.prob_threshold(p_prob)
    p = t / 2**32
    zs = []
    for key in range(40):
        cand, prio = orc.seed_candidates(dims, key, t)
        grid, k = orc.seed_select(dims, 1, cand, prio)
        assert k == len(cand) == int(grid.sum())
        zs.append((k - n * p) / np.sqrt(n * p * (1 - p)))
    zs = np.array(zs)
    assert np.all(np.abs(zs) < 4.5)
    assert abs(zs.mean()) < 4.0 / np.sqrt(len(zs))
    assert 0.4 < zs.std() < 1.7


def test_extreme_seed_probabilities(orc):
    dims = (6, 5, 4)
    cand, _ = orc.seed_candidates(dims, 3, orc.prob_threshold(1.0))
    assert list(cand) == list(range(120))
    cand, _ = orc.seed_candidates(dims, 3, orc.prob_threshold(0.0))
    assert len(cand) == 0


def _coords(dims, v):
    nx, ny, _ = dims
    return np.stack([v % nx, (v // nx) % ny, v // (nx * ny)], axis=-1)


def _check_spacing_and_maximality(dims, cand, prio, grid, s):
    seeds = np.flatnonzero(grid.ravel())
    cs = _coords(dims, seeds)
    if len(seeds) > 1:
        d = np.abs(cs[:, None, :] - cs[None, :, :]).sum(-1)
        np.fill_diagonal(d, 10**9)
        assert d.min() >= s  # pairwise spacing >= s
    order = sorted(range(len(cand)), key=lambda i: (int(prio[i]), int(cand[i])))
    rank = {int(cand[i]): r for r, i in enumerate(order)}
    seedset = set(int(x) for x in seeds)
    assert seedset <= set(int(c) for c in cand)
    cc = _coords(dims, np.asarray(cand, dtype=np.int64))
    for i, v in enumerate(cand):
        v = int(v)
        if v in seedset:
            continue
        # every rejected candidate lies within s-1 of a seed of smaller key
        dist = np.abs(cs - cc[i]).sum(-1)
        blockers = [int(seeds[k]) for k in np.flatnonzero(dist <= s - 1)]
        assert any(rank[b] < rank[v] for b in blockers)


@pytest.mark.parametrize("s", [2, 3, 4, 7])
def test_spacing_random(orc, s):
    dims = (23, 17, 11)
    for key in range(6):
        cand, prio = orc.seed_candidates(dims, key, orc.prob_threshold(0.05))
        grid, k = orc.seed_select(dims, s, cand, prio)
        assert k == int(grid.sum())
        _check_spacing_and_maximality(dims, cand, prio, grid, s)


def _mis_case(orc, dims, cs, prios, s):
    cand = np.array(cs, dtype=np.int32)
    prio = np.array(prios, dtype=np.uint64)
    grid, _ = orc.seed_select(dims, s, cand, prio)
    got = sorted(int(v) for v in np.flatnonzero(grid.ravel()))
    want = sorted(cs) if s <= 1 else ref_tiny.lexfirst_mis_bruteforce(
        dims, list(zip(cs, prios)), s)
    assert got == want, (cs, prios, s)


def test_spacing_exhaustive_pairs_4cubed(orc):
    """Every candidate pair on a 4^3 grid, every spacing 0..6, both priority orders:
    the pair survives iff its L1 distance is >= s, else only the smaller key."""
    dims = (4, 4, 4)
    for s in range(0, 7):
        for u, v in itertools.combinations(range(64), 2):
            for pu, pv in ((5, 9), (9, 5)):
                cand = np.array([u, v], dtype=np.int32)
                prio = np.array([pu, pv], dtype=np.uint64)
                grid, k = orc.seed_select(dims, s, cand, prio)
                dist = ref_tiny.l1(dims, u, v)
                if s <= 1 or dist >= s:
                    assert k == 2
                else:
                    assert k == 1 and grid.ravel()[u if pu < pv else v] == 1


def test_spacing_bruteforce_small_sets(orc):
    """Candidate sets of size 1..9 on 4^3 and 5x4x3 grids against the brute-force
    lexicographically-first maximal independent set, including equal priorities
    (ties broken by the voxel index)."""
    rng = np.random.default_rng(5)
    for dims in ((4, 4, 4), (5, 4, 3)):
        n = dims[0] * dims[1] * dims[2]
        for trial in range(700):
            k = int(rng.integers(1, 10))
            cs = [int(c) for c in rng.choice(n, size=k, replace=False)]
            if trial % 3 == 0:
                prios = [int(p) for p in rng.integers(0, 3, size=k)]  # many ties
            else:
                prios = [int(p) for p in rng.integers(0, 2**64, size=k, dtype=np.uint64)]
            s = int(rng.integers(0, 7))
            _mis_case(orc, dims, cs, prios, s)


def test_all_triples_4cubed_sampled(orc):
    """A fixed sample of the 41 664 three-candidate sets of a 4^3 grid."""
    dims = (4, 4, 4)
    triples = list(itertools.combinations(range(64), 3))
    rng = np.random.default_rng(6)
    for idx in rng.choice(len(triples), size=1500, replace=False):
        cs = list(triples[idx])
        prios = [int(p) for p in rng.permutation(3)]
        _mis_case(orc, dims, cs, prios, int(rng.integers(2, 7)))


def test_candidate_threshold_is_strict(orc):
    """A voxel is a candidate iff its word 0 is strictly below the threshold:
    with the threshold equal to a voxel's own word it is excluded, one above it
    is included."""
    dims = (4, 3, 2)
    for key in (5, 6):
        for v in (0, 7, 23):
            w0 = ref_tiny.keyed(key, v, 0, 0, 1)[0]
            cand, _ = orc.seed_candidates(dims, key, w0)
            assert v not in set(int(c) for c in cand)
            cand, _ = orc.seed_candidates(dims, key, w0 + 1)
            assert v in set(int(c) for c in cand)
