"""Pins of the oracle's growth step (Sec. 2.2-2.3, Algorithms 2 and 3, Eq. (1))."""
import itertools

import numpy as np
import pytest
from scipy import ndimage

from tests import ref_tiny

ALWAYS, NEVER = 2**32, 0


def _structure(active):
    """3x3x3 dilation structure: centre plus the offsets of the active classes."""
    s = np.zeros((3, 3, 3), dtype=bool)
    s[1, 1, 1] = True
    for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
        c = abs(dx) + abs(dy) + abs(dz) - 1
        if c >= 0 and active[c]:
            s[dz + 1, dy + 1, dx + 1] = True
    return s


PATTERNS = [tuple(bool(b >> c & 1) for c in range(3)) for b in range(8)]


def test_direction_table(orc):
    offs, classes = [], []
    for d in range(26):
        dx, dy, dz, c = orc.direction(d)
        offs.append((dx, dy, dz))
        classes.append(c)
    assert offs == ref_tiny.OFFSETS
    assert len(set(offs)) == 26 and (0, 0, 0) not in offs
    assert classes == ref_tiny.CLASSES
    assert [classes.count(c) for c in range(3)] == [6, 12, 8]
    assert [d for d in range(26) if classes[d] == 0] == [4, 10, 12, 13, 15, 21]
    for d in range(26):  # the set is symmetric: -e_d is direction 25 - d, same class
        dx, dy, dz = offs[d]
        assert offs[25 - d] == (-dx, -dy, -dz) and classes[25 - d] == classes[d]


def _run_both_forms(orc, grid0, steps, T, key):
    """Apply `steps` steps with the list form and the full-field form, checking
    they agree and that the list form's front is the interface after each step."""
    g_list = grid0.copy()
    g_full = grid0.copy()
    front = orc.interface(g_list)
    out = []
    for t in range(steps):
        front, n_new = orc.step_liets(g_list, front, t, T, key)
        n_full = orc.step_fullfield(g_full, t, T, key)
        assert n_new == n_full
        assert np.array_equal(g_list, g_full)
        assert np.array_equal(np.sort(front), orc.interface(g_list))
        out.append(g_list.copy())
    return out


@pytest.mark.parametrize("pattern", PATTERNS)
def test_deterministic_limits_are_dilations(orc, pattern):
    """With p in {0, 1} per class, one step is a binary dilation (no wrap-around)
    by the centre plus the active classes' offsets."""
    T = [ALWAYS if a else NEVER for a in pattern]
    rng = np.random.default_rng(sum(b << i for i, b in enumerate(pattern)))
    for dims in ((9, 7, 5), (4, 11, 6), (1, 8, 3)):
        nx, ny, nz = dims
        g0 = (rng.random((nz, ny, nx)) < 0.06).astype(np.uint8)
        want = g0.astype(bool)
        grids = _run_both_forms(orc, g0, 3, T, key=5)
        for g in grids:
            want = ndimage.binary_dilation(want, structure=_structure(pattern), border_value=0)
            assert np.array_equal(g.astype(bool), want)


def test_parity_invariants_of_single_classes(orc):
    """Edge-only growth keeps x+y+z mod 2; corner-only keeps x-y and y-z mod 2."""
    nx, ny, nz = 10, 9, 8
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    g0 = np.zeros((nz, ny, nx), dtype=np.uint8)
    g0[4, 4, 5] = 1
    g = _run_both_forms(orc, g0, 4, [NEVER, ALWAYS, NEVER], 1)[-1].astype(bool)
    assert np.all(((x + y + z) % 2)[g] == 1)
    g = _run_both_forms(orc, g0, 4, [NEVER, NEVER, ALWAYS], 1)[-1].astype(bool)
    assert np.all(((x - y) % 2)[g] == 1) and np.all(((y - z) % 2)[g] == 0)


def test_exhaustive_small_starts_4cubed(orc):
    """Every 1- and 2-voxel start on 4^3, every class pattern, 3 steps, against
    the scipy dilation (full-field form; the list form is compared on a subset)."""
    dims = (4, 4, 4)
    starts = [(v,) for v in range(64)] + list(itertools.combinations(range(64), 2))
    for i, st in enumerate(starts):
        g0 = np.zeros(64, dtype=np.uint8)
        g0[list(st)] = 1
        g0 = g0.reshape(4, 4, 4)
        for pattern in PATTERNS:
            T = [ALWAYS if a else NEVER for a in pattern]
            want = g0.astype(bool)
            g = g0.copy()
            for t in range(3):
                orc.step_fullfield(g, t, T, 0)
                want = ndimage.binary_dilation(want, structure=_structure(pattern),
                                               border_value=0)
                assert np.array_equal(g.astype(bool), want), (st, pattern, t)
            if i % 97 == 0:
                _run_both_forms(orc, g0, 3, T, 0)


def test_exhaustive_2cubed_states(orc):
    """All 256 states of a 2x2x2 grid, one step, every pattern and a random one."""
    for b in range(256):
        g0 = np.array([(b >> i) & 1 for i in range(8)], dtype=np.uint8).reshape(2, 2, 2)
        for pattern in PATTERNS:
            T = [ALWAYS if a else NEVER for a in pattern]
            g = g0.copy()
            orc.step_fullfield(g, 0, T, 0)
            want = ndimage.binary_dilation(g0.astype(bool), structure=_structure(pattern),
                                           border_value=0)
            assert np.array_equal(g.astype(bool), want)
        T = [2**31, 2**30, 2**29]
        g = g0.copy()
        orc.step_fullfield(g, 2, T, 99)
        assert np.array_equal(g, np.array(ref_tiny.step(g0.tolist(), 2, T, 99), np.uint8))


def test_list_and_fullfield_forms_agree(orc):
    rng = np.random.default_rng(21)
    for trial in range(12):
        nx, ny, nz = (int(v) for v in rng.integers(3, 14, size=3))
        g0 = (rng.random((nz, ny, nx)) < rng.uniform(0.01, 0.3)).astype(np.uint8)
        T = [int(v) for v in rng.integers(0, 2**32, size=3)]
        _run_both_forms(orc, g0, 4, T, key=int(rng.integers(0, 2**63)))


def test_step_matches_target_centred_coding(orc):
    rng = np.random.default_rng(22)
    for trial in range(10):
        nx, ny, nz = (int(v) for v in rng.integers(2, 7, size=3))
        g = (rng.random((nz, ny, nx)) < 0.2).astype(np.uint8)
        key = int(rng.integers(0, 2**63))
        for t in range(3):
            T = [int(v) for v in rng.integers(0, 2**32, size=3)]
            want = np.array(ref_tiny.step(g.tolist(), t, T, key), dtype=np.uint8)
            front = orc.interface(g)
            orc.step_liets(g, front, t, T, key)
            assert np.array_equal(g, want)


def _binom_z(k, n, p):
    return (k - n * p) / np.sqrt(n * p * (1 - p))


def test_single_source_direction_frequencies(orc):
    """One solid voxel in a 3^3 grid: each neighbour grows independently with its
    class probability; per-direction z-scores and a 26-bin chi-square."""
    probs = (0.30, 0.15, 0.05)
    T = [orc.prob_threshold(p) for p in probs]
    p_eff = [t / 2**32 for t in T]
    K = 6000
    counts = np.zeros(26)
    for key in range(K):
        g = np.zeros((3, 3, 3), dtype=np.uint8)
        g[1, 1, 1] = 1
        orc.step_liets(g, np.array([13], np.int32), 0, T, key)
        flat = np.delete(g.ravel(), 13)
        counts += flat
    exp = np.array([K * p_eff[c] for c in ref_tiny.CLASSES])
    var = np.array([K * p_eff[c] * (1 - p_eff[c]) for c in ref_tiny.CLASSES])
    z = (counts - exp) / np.sqrt(var)
    assert np.all(np.abs(z) < 4.5)
    chi2 = float((z**2).sum())
    assert chi2 < 60.0  # 26 dof, p ~ 2e-4


def test_two_source_union_probability(orc):
    """A void cell with a face and an edge solid neighbour grows with probability
    1 - (1 - p_face)(1 - p_edge) (independent draws per source and direction)."""
    T = [orc.prob_threshold(0.2), orc.prob_threshold(0.1), 0]
    pf, pe = T[0] / 2**32, T[1] / 2**32
    p = 1 - (1 - pf) * (1 - pe)
    K = 8000
    hits = 0
    for key in range(K):
        g = np.zeros((1, 3, 3), dtype=np.uint8)  # 3x3x1 slab; target at (1,1)
        g[0, 1, 0] = 1  # face neighbour (-x)
        g[0, 0, 0] = 1  # edge neighbour (-x,-y)
        front = orc.interface(g)
        orc.step_liets(g, front, 5, T, key)
        hits += int(g[0, 1, 1])
    assert abs(_binom_z(hits, K, p)) < 4.5


def test_direction_counters_chi_square(orc):
    """Per-direction success frequencies over a multi-step run on a 24^3 grid,
    attempts counted on void-at-start targets, vs T_class / 2^32."""
    rng = np.random.default_rng(8)
    g = (rng.random((24, 24, 24)) < 0.01).astype(np.uint8)
    T = [orc.prob_threshold(0.12), orc.prob_threshold(0.06), orc.prob_threshold(0.03)]
    front = orc.interface(g)
    att = np.zeros(26)
    suc = np.zeros(26)
    for t in range(6):
        front, _, a, s = orc.step_liets(g, front, t, T, 77, counters=True)
        att += a
        suc += s
    p = np.array([T[c] / 2**32 for c in ref_tiny.CLASSES])
    z = (suc - att * p) / np.sqrt(att * p * (1 - p))
    assert np.all(np.abs(z) < 4.5)
    assert float((z**2).sum()) < 60.0


def test_growth_threshold_is_strict_and_ranked(orc):
    """Source at the centre of 3^3 with every neighbour void: direction d has rank
    d.  With T equal to that draw the neighbour stays void, one above it grows."""
    key, t = 12345, 4
    for d in (0, 4, 9, 13, 25):
        c = ref_tiny.CLASSES[d]
        w = ref_tiny.growth_draw(key, 13, t, d)
        for T_c, grows in ((w, False), (w + 1, True)):
            T = [0, 0, 0]
            T[c] = T_c
            g = np.zeros((3, 3, 3), dtype=np.uint8)
            g[1, 1, 1] = 1
            orc.step_liets(g, np.array([13], np.int32), t, T, key)
            q = d if d < 13 else d + 1
            assert bool(g.ravel()[q]) == grows, (d, T_c)
            g2 = np.zeros((3, 3, 3), dtype=np.uint8)
            g2[1, 1, 1] = 1
            orc.step_fullfield(g2, t, T, key)
            assert np.array_equal(g, g2)


def test_rank_skips_solid_neighbours(orc):
    """With some neighbours already solid the ranks of the remaining void
    directions shift down; the draw used is that of the rank, not of d."""
    key, t = 777, 2
    g = np.zeros((3, 3, 3), dtype=np.uint8)
    g[1, 1, 1] = 1
    g.ravel()[[0, 1, 2]] = 1  # directions 0, 1, 2 are solid
    d = 5
    j = d - 3
    w = ref_tiny.growth_draw(key, 13, t, j)
    T = [0, 0, 0]
    T[ref_tiny.CLASSES[d]] = w + 1
    others = [e for e in range(26) if ref_tiny.CLASSES[e] == ref_tiny.CLASSES[d] and e != d]
    g1 = g.copy()
    orc.step_liets(g1, np.array([13], np.int32), t, T, key)
    assert g1.ravel()[d + 0] == 1  # d < 13 so the flat index is d
    # any other same-class direction grows only if its own rank's draw is below T
    for e in others:
        if e in (0, 1, 2):
            continue
        q = e if e < 13 else e + 1
        je = e - 3
        assert bool(g1.ravel()[q]) == (ref_tiny.growth_draw(key, 13, t, je) < T[ref_tiny.CLASSES[e]])
