"""Seeded synthetic workloads: grid sizes and generation parameters only.

This module holds no arithmetic of the method; it only states the inputs (grid
dimensions, target solid fraction, seed probability, reference growth probabilities,
seed spacing and Philox key) of the workloads the library is tested and measured on.
Both the oracle-side tests and the GPU side read their inputs from here.

The paper's timing runs are parameter sets on a cubic grid (Sec. 3.2); its Fontainebleau
benchmark is a 500^3 grid with the seed probability S_d = 6 phi_s Delta^3 / (pi d^3),
Delta = 4 um per voxel and grain diameter d = 200-250 um (Sec. 3.3).  No dataset is read.
"""
from __future__ import annotations

import math
from dataclasses import asdict, dataclass

import numpy as np

# face : edge : corner reference probabilities (4 : 1 : 0.25)
RATIOS = (1.0, 0.25, 0.0625)


@dataclass(frozen=True)
class Case:
    name: str
    dims: tuple  # (nx, ny, nz)
    solid_fraction: float
    seed_prob: float
    g_ref: tuple
    spacing: int
    key: int
    max_steps: int = 0

    @property
    def n(self) -> int:
        return self.dims[0] * self.dims[1] * self.dims[2]

    def as_dict(self) -> dict:
        return asdict(self)


def g_from_face(face: float) -> tuple:
    return tuple(face * r for r in RATIOS)


def fontainebleau_seed_prob(solid_fraction: float, grain_um: float = 225.0,
                            voxel_um: float = 4.0) -> float:
    """S_d = 6 phi_s Delta^3 / (pi d^3) (Sec. 3.3)."""
    return 6.0 * solid_fraction * voxel_um**3 / (math.pi * grain_um**3)


def config1() -> list[Case]:
    """64^3, solid fraction 0.70, S_d 0.005, G_ref 0.02/0.005/0.00125, s = 4, key 0."""
    return [Case("c1_64", (64, 64, 64), 0.70, 0.005, (0.02, 0.005, 0.00125), 4, 0)]


def config2() -> list[Case]:
    """200^3, porosity 0.20, S_d 0.001, G_ref 0.01/0.0025/0.000625, s = 10, keys 0..4."""
    return [Case(f"c2_200_k{k}", (200, 200, 200), 0.80, 0.001, (0.01, 0.0025, 0.000625), 10, k)
            for k in range(5)]


def config3() -> list[Case]:
    """400^3 (the paper's timing size), porosity {0.10, 0.20, 0.30}, S_d 5e-4,
    G_ref 0.01/0.0025/0.000625, s = 20, key 1."""
    return [Case(f"c3_400_p{int(round(p * 100)):02d}", (400, 400, 400), round(1.0 - p, 10), 5e-4,
                 (0.01, 0.0025, 0.000625), 20, 1) for p in (0.10, 0.20, 0.30)]


def config4(seed: int = 0) -> list[Case]:
    """64 realizations: cube edges from {96,128,160,192,256}, porosity U[0.05,0.25],
    s uniform in [4,30], G_ref face 0.01 at 4:1:0.25, keys 0..63.  The seed probability
    is not given for this mix; config 3's 5e-4 is used."""
    rng = np.random.default_rng(seed)
    edges = rng.choice([96, 128, 160, 192, 256], size=64)
    por = rng.uniform(0.05, 0.25, size=64)
    sp = rng.integers(4, 31, size=64)
    return [Case(f"c4_r{k:02d}", (int(e), int(e), int(e)), float(1.0 - p), 5e-4,
                 g_from_face(0.01), int(s), k) for k, (e, p, s) in enumerate(zip(edges, por, sp))]


def config4_singletons() -> list[Case]:
    """500^3 sandstone-like singletons: porosity 0.05..0.25 in 5 steps, s = 30, S_d from
    the Fontainebleau formula at d = 225 um, G_ref face 0.01 at 4:1:0.25."""
    out = []
    for i, p in enumerate((0.05, 0.10, 0.15, 0.20, 0.25)):
        phi = round(1.0 - p, 10)
        out.append(Case(f"c4_500_p{int(round(p * 100)):02d}", (500, 500, 500), phi,
                        fontainebleau_seed_prob(phi), g_from_face(0.01), 30, 100 + i))
    return out


@dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    case: Case


def config5(n_requests: int = 1000, rate_per_s: float = 100.0, seed: int = 0) -> list[Request]:
    """Poisson stream of generation requests: cube edge U{64..320}, porosity
    U[0.05,0.30], s U{4..30}, S_d U[5e-4, 5e-3], face U[0.005, 0.02] at 4:1:0.25,
    key = request id."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    edges = rng.integers(64, 321, size=n_requests)
    por = rng.uniform(0.05, 0.30, size=n_requests)
    sp = rng.integers(4, 31, size=n_requests)
    sd = rng.uniform(5e-4, 5e-3, size=n_requests)
    face = rng.uniform(0.005, 0.02, size=n_requests)
    return [Request(i, float(t[i]),
                    Case(f"c5_q{i:04d}", (int(edges[i]),) * 3, float(1.0 - por[i]), float(sd[i]),
                         g_from_face(float(face[i])), int(sp[i]), i))
            for i in range(n_requests)]


def config5_parity(n_first: int = 12, n_large: int = 4) -> list[Case]:
    """Requests of the config-5 stream checked against the oracle at full size: the first
    ``n_first`` requests, and the ``n_large`` requests with cube edge >= 300 and spacing
    >= 25 that have the largest seed probabilities (the heaviest seeding in the mix)."""
    stream = config5()
    large = [r for r in stream if r.case.dims[0] >= 300 and r.case.spacing >= 25]
    large.sort(key=lambda r: -r.case.seed_prob)
    picked = {r.rid: r for r in stream[:n_first]}
    for r in large[:n_large]:
        picked[r.rid] = r
    return [picked[k].case for k in sorted(picked)]


def many_small_cases(n: int = 80, seed: int = 2602) -> list[Case]:
    """More small realizations than one wavefront of the step-end planner handles at
    once (edges U{6..28}, porosity U[0.1, 0.5], S_d U[0.002, 0.05], face U[0.02, 0.2],
    s U{0..6}, keys 5000 + i)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        dims = tuple(int(v) for v in rng.integers(6, 29, size=3))
        out.append(Case(f"many_{i:03d}", dims, round(1.0 - float(rng.uniform(0.1, 0.5)), 6),
                        round(float(rng.uniform(0.002, 0.05)), 6),
                        g_from_face(round(float(rng.uniform(0.02, 0.2)), 6)),
                        int(rng.integers(0, 7)), 5000 + i))
    return out


def small_cases() -> list[Case]:
    """Small and ragged grids (several sweep tiles, odd extents) and the method's
    degenerate cases, for element-by-element parity with the oracle.  The last one holds
    fronts of about 1 200 voxels per 64 x 8 x 4 tile for five steps, more than one chunk of the
    sweep's 512-voxel queue."""
    g = (0.02, 0.005, 0.00125)
    return [
        Case("ragged_37x23x19", (37, 23, 19), 0.65, 0.01, g, 3, 7),
        Case("flat_96x80x1", (96, 80, 1), 0.6, 0.004, (0.05, 0.02, 0.01), 5, 3),
        Case("thin_1x1x300", (1, 1, 300), 0.7, 0.02, (0.2, 0.0, 0.0), 2, 5),
        Case("no_spacing_dense", (40, 30, 20), 0.8, 0.2, (0.03, 0.01, 0.002), 0, 11),
        Case("spacing1_dense", (33, 17, 25), 0.75, 0.3, (0.03, 0.01, 0.002), 1, 12),
        Case("large_spacing", (50, 45, 40), 0.7, 0.01, g, 25, 13),
        Case("spacing2_many", (48, 48, 48), 0.6, 0.05, (0.01, 0.01, 0.01), 2, 14),
        Case("prob_one", (21, 19, 17), 0.9, 0.002, (1.0, 1.0, 1.0), 4, 15),
        Case("face_only", (30, 30, 30), 0.5, 0.003, (0.3, 0.0, 0.0), 5, 16),
        Case("corner_only", (30, 30, 30), 0.4, 0.003, (0.0, 0.0, 0.3), 5, 17),
        Case("full_fill", (20, 18, 16), 1.0, 0.01, (0.5, 0.3, 0.2), 3, 18),
        Case("no_seeds", (24, 24, 24), 0.5, 0.0, g, 4, 19),
        Case("no_growth_cap", (24, 24, 24), 0.5, 0.01, (0.0, 0.0, 0.0), 4, 20, max_steps=9),
        Case("step_cap", (32, 32, 32), 0.9, 0.002, g, 4, 21, max_steps=3),
        Case("all_seeds", (16, 16, 16), 0.5, 1.0, g, 0, 22),
        Case("single_voxel", (1, 1, 1), 1.0, 1.0, g, 0, 23),
        Case("key_high_bits", (45, 41, 39), 0.7, 0.006, g, 6, 0xFFFF_FFFF_0000_0001),
        Case("two_voxels", (2, 1, 1), 1.0, 0.5, (0.5, 0.5, 0.5), 0, 24),
        Case("dense_front_64x64x32", (64, 64, 32), 0.97, 0.6, (0.02, 0.01, 0.002), 0, 25),
    ]


@dataclass(frozen=True)
class PhaseSet:
    """A multi-phase generation (Sec. 2.1 steps 1-5): growing phases in order, phase
    n = index + 1; each Case gives that phase's target fraction P^n (solid_fraction),
    core probability (seed_prob), growth probabilities, spacing, key and step cap."""
    name: str
    dims: tuple
    phases: tuple


def _ph(sf, sd, g, s, key, max_steps=0) -> Case:
    return Case(f"phase_k{key}", (0, 0, 0), sf, sd, g, s, key, max_steps)


def phase_sets() -> list[PhaseSet]:
    """Small multi-phase cases for element-by-element parity: three phases over several
    tiles; a ragged grid; a phase whose target the earlier phases make unreachable
    (exhausted); a phase without cores; a phase stopped by its step cap."""
    g1, g2, g3 = (0.02, 0.005, 0.00125), (0.03, 0.01, 0.002), (0.01, 0.0025, 0.000625)
    return [
        PhaseSet("mp3_40x36x30", (40, 36, 30),
                 (_ph(0.30, 0.004, g1, 4, 11), _ph(0.20, 0.003, g2, 3, 12),
                  _ph(0.15, 0.002, g1, 0, 13))),
        PhaseSet("mp2_97x70x45", (97, 70, 45),
                 (_ph(0.50, 0.002, g3, 6, 21), _ph(0.30, 0.001, g1, 4, 22))),
        PhaseSet("mp2_blocked_48x40x33", (48, 40, 33),
                 (_ph(0.70, 0.003, g1, 3, 31), _ph(0.50, 0.002, g1, 2, 32))),
        PhaseSet("mp3_nocores_20", (20, 20, 20),
                 (_ph(0.40, 0.01, g1, 2, 41), _ph(0.30, 0.0, g1, 2, 42),
                  _ph(0.20, 0.02, g2, 0, 43))),
        PhaseSet("mp2_cap_33x29x31", (33, 29, 31),
                 (_ph(0.35, 0.003, g1, 3, 51, 4), _ph(0.25, 0.004, g2, 2, 52, 3))),
    ]


def phase_bench() -> PhaseSet:
    """Three-phase 400^3 medium: a grain phase as in the paper's timing runs (P 0.50,
    S_d 5e-4, s = 20, G_ref 0.01 / 0.0025 / 0.000625), a sparse second mineral (P 0.15,
    S_d 1e-4, s = 10) and a fine-grained third phase (P 0.05, S_d 2e-3, no spacing,
    face 0.02); keys 1, 2, 3."""
    g = (0.01, 0.0025, 0.000625)
    return PhaseSet("mp3_400", (400, 400, 400),
                    (_ph(0.50, 5e-4, g, 20, 1), _ph(0.15, 1e-4, g, 10, 2),
                     _ph(0.05, 2e-3, g_from_face(0.02), 0, 3)))
