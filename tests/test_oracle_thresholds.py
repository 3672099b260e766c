"""Pins of the probability thresholds, the target count and the integer form of Eq. (1)."""
import math

import numpy as np

from tests import ref_tiny


def test_prob_threshold_closed_forms(orc):
    assert orc.prob_threshold(0.0) == 0
    assert orc.prob_threshold(-0.5) == 0
    assert orc.prob_threshold(1.0) == 2**32
    assert orc.prob_threshold(1.5) == 2**32
    assert orc.prob_threshold(0.5) == 2**31
    assert orc.prob_threshold(0.25) == 2**30
    assert orc.prob_threshold(2.0**-32) == 1
    assert orc.prob_threshold(2.0**-33) == 0
    rng = np.random.default_rng(1)
    for p in rng.random(3000):
        t = orc.prob_threshold(float(p))
        assert t == ref_tiny.prob_threshold(float(p))
        # T / 2^32 is the largest multiple of 2^-32 not above p
        assert t / 2**32 <= p < (t + 1) / 2**32


def test_target_count(orc):
    # phi_a < phi_s with phi_a = count / N  <=>  count < S*
    rng = np.random.default_rng(2)
    for _ in range(2000):
        n = int(rng.integers(1, 2**31 - 1))
        phi = float(rng.random())
        s = orc.target_count(phi, n)
        assert s == ref_tiny.target_count(phi, n)
        assert 0 <= s <= n
        assert (s - 1) < phi * n <= s or (s == 0 and phi * n <= 0)
    # values that sit on an integer in binary64 must not round up
    assert orc.target_count(0.8, 200**3) == 6_400_000
    assert orc.target_count(0.7, 64**3) == math.ceil(0.7 * 64**3)
    assert orc.target_count(1.0, 1000) == 1000


def test_eq1_endpoints_and_monotonicity(orc):
    t_ref = orc.prob_threshold(0.01)
    s = 1_000_003
    # factor 20 at phi_a = 0, factor -> 1 as phi_a -> phi_s (Eq. (1))
    assert orc.growth_threshold(t_ref, 0, s) == 20 * t_ref
    last = orc.growth_threshold(t_ref, s - 1, s)
    assert t_ref <= last <= t_ref + math.ceil(19 * t_ref / s)
    prev = None
    for cnt in np.linspace(0, s - 1, 400).astype(np.int64):
        t = orc.growth_threshold(t_ref, int(cnt), s)
        assert t == ref_tiny.growth_threshold(t_ref, int(cnt), s)
        if prev is not None:
            assert t <= prev
        prev = t
    # probability 1 stays 1, probability 0 stays 0, large factors cap at 2^32
    assert orc.growth_threshold(2**32, 0, s) == 2**32
    assert orc.growth_threshold(2**32, s - 1, s) == 2**32
    assert orc.growth_threshold(0, 0, s) == 0
    assert orc.growth_threshold(orc.prob_threshold(0.2), 0, 10) == 2**32


def test_eq1_matches_float_formula(orc):
    """The integer thresholds follow G_ref (phi_s - 0.95 phi_a) / (0.05 phi_s) with
    phi_a = count / N, up to the rounding of S* and of the thresholds."""
    rng = np.random.default_rng(3)
    for _ in range(3000):
        n = int(rng.integers(1000, 2**31 - 1))
        phi_s = float(rng.uniform(0.05, 0.99))
        g = float(rng.uniform(0.0, 0.05))
        s = orc.target_count(phi_s, n)
        cnt = int(rng.integers(0, s))
        phi_a = cnt / n
        p = g * (phi_s - 0.95 * phi_a) / (0.05 * phi_s)
        t = orc.growth_threshold(orc.prob_threshold(g), cnt, s)
        want = min(p, 1.0) * 2**32
        # |T - p 2^32| <= 20 (floor of T_ref, scaled by the factor) + 20 p 2^32 / S*
        # (S* vs phi_s N) + 2
        assert abs(t - want) <= 22 + 20 * want / s + 1e-6 * want
