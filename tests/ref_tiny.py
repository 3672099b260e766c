"""Pure-Python second coding of the integer definitions, for tiny grids only.

Written independently of ``oracle/qsgs_oracle.c`` (different loop structure:
target-centred growth, big-int Philox, itertools direction order) so that the
two codings can pin each other on small inputs.  Test infrastructure only.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 block (Salmon et al., SC'11) with Python integers."""
    x = [int(c) & MASK32 for c in ctr]
    k = [int(key[0]) & MASK32, int(key[1]) & MASK32]
    for _ in range(10):
        p0 = 0xD2511F53 * x[0]
        p1 = 0xCD9E8D57 * x[2]
        x = [((p1 >> 32) ^ x[1] ^ k[0]) & MASK32, p1 & MASK32,
             ((p0 >> 32) ^ x[3] ^ k[1]) & MASK32, p0 & MASK32]
        k = [(k[0] + 0x9E3779B9) & MASK32, (k[1] + 0xBB67AE85) & MASK32]
    return tuple(x)


def keyed(key: int, c0: int, c1: int, c2: int, c3: int):
    return philox4x32_10((c0, c1, c2, c3), (key & MASK32, key >> 32))


# The 26-neighbourhood, dz slowest and dx fastest, centre removed.
OFFSETS = [(dx, dy, dz) for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3)
           if (dx, dy, dz) != (0, 0, 0)]
CLASSES = [abs(dx) + abs(dy) + abs(dz) - 1 for dx, dy, dz in OFFSETS]


def prob_threshold(p: float) -> int:
    if not p > 0:
        return 0
    return min(1 << 32, math.floor(Fraction(p) * (1 << 32)))


def target_count(phi_s: float, n: int) -> int:
    return min(n, max(0, math.ceil(phi_s * float(n))))


def growth_threshold(t_ref: int, cnt: int, s_star: int) -> int:
    return min(1 << 32, (t_ref * (20 * s_star - 19 * cnt)) // s_star)


def growth_draw(key: int, a: int, t: int, j: int) -> int:
    block, word, half = j // 8, (j // 2) % 4, j % 2
    hi = keyed(key, a, t, block, 2)[word]
    lo = keyed(key, a, t, block, 3)[word]
    h = (hi >> (16 * half)) & 0xFFFF
    lo16 = (lo >> (16 * half)) & 0xFFFF
    return (h << 16) | lo16


def _inside(dims, x, y, z):
    nx, ny, nz = dims
    return 0 <= x < nx and 0 <= y < ny and 0 <= z < nz


def step(grid, t: int, T, key: int):
    """One growth step, target-centred: a void cell q becomes solid iff some solid
    neighbour a = q - e_d draws below the threshold of class(d)."""
    nz, ny, nx = len(grid), len(grid[0]), len(grid[0][0])
    dims = (nx, ny, nz)

    def solid(x, y, z):
        return grid[z][y][x] == 1

    def rank(ax, ay, az, d):
        r = 0
        for e in range(d):
            ex, ey, ez = OFFSETS[e]
            if _inside(dims, ax + ex, ay + ey, az + ez) and not solid(ax + ex, ay + ey, az + ez):
                r += 1
        return r

    out = [[[grid[z][y][x] for x in range(nx)] for y in range(ny)] for z in range(nz)]
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if solid(x, y, z):
            continue
        for d, (dx, dy, dz) in enumerate(OFFSETS):
            ax, ay, az = x - dx, y - dy, z - dz
            if not _inside(dims, ax, ay, az) or not solid(ax, ay, az):
                continue
            a = ax + nx * (ay + ny * az)
            if growth_draw(key, a, t, rank(ax, ay, az, d)) < T[CLASSES[d]]:
                out[z][y][x] = 1
                break
    return out


def seed_candidates(dims, key: int, t_seed: int):
    nx, ny, nz = dims
    cands = []
    for v in range(nx * ny * nz):
        w = keyed(key, v, 0, 0, 1)
        if w[0] < t_seed:
            cands.append((v, (w[1] << 32) | w[2]))
    return cands


def l1(dims, u: int, v: int) -> int:
    nx, ny, _ = dims
    ux, uy, uz = u % nx, (u // nx) % ny, u // (nx * ny)
    vx, vy, vz = v % nx, (v // nx) % ny, v // (nx * ny)
    return abs(ux - vx) + abs(uy - vy) + abs(uz - vz)


def lexfirst_mis_bruteforce(dims, cands, spacing: int):
    """The unique independent set S such that every candidate outside S conflicts
    with a member of S of smaller (priority, v) -- found by trying every subset."""
    items = sorted(cands, key=lambda c: (c[1], c[0]))
    n = len(items)

    def conflict(i, j):
        return 0 < l1(dims, items[i][0], items[j][0]) <= spacing - 1

    found = []
    for mask in range(1 << n):
        members = [i for i in range(n) if mask >> i & 1]
        if any(conflict(i, j) for i, j in itertools.combinations(members, 2)):
            continue
        ok = True
        for i in range(n):
            if mask >> i & 1:
                continue
            if not any(conflict(i, j) and j < i for j in members):
                ok = False
                break
        if ok:
            found.append(sorted(items[i][0] for i in members))
    assert len(found) == 1, "fixed point must be unique"
    return found[0]
