"""ctypes binding of the CPU oracle (``qsgs_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain single-threaded reference the
GPU library is checked against; only ``tests/``, the package smoke check and the
benchmark's CPU-baseline leg import this module.  It imports nothing from the GPU
package.

Shapes follow the paper's grid convention: a grid is a uint8 array of shape
``(nz, ny, nx)`` in C order (0 = pore, 1 = solid), voxel ``v = x + nx*(y + ny*z)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsgs_oracle.c")
_HDR = os.path.join(_HERE, "qsgs_oracle.h")
_LIB = os.path.join(_HERE, "liborc.so")

DONE, EXHAUSTED, MAXSTEPS = 1, 2, 3
STATUS_NAMES = {DONE: "done", EXHAUSTED: "exhausted", MAXSTEPS: "max_steps"}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liborc.so`` (single-threaded, -O2)."""
    stale = not os.path.exists(_LIB) or any(
        os.path.getmtime(p) > os.path.getmtime(_LIB) for p in (_SRC, _HDR))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("solid_fraction", ctypes.c_double), ("seed_prob", ctypes.c_double),
                ("g_ref", ctypes.c_double * 3), ("spacing", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("key", ctypes.c_uint64),
                ("front_rule", ctypes.c_int32), ("unused", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int64), ("n_seeds", ctypes.c_int64),
                ("solid_count", ctypes.c_int64), ("target_count", ctypes.c_int64),
                ("front_size", ctypes.c_int64), ("steps", ctypes.c_int32),
                ("status", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        i32, i64, u32, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        vp = ctypes.c_void_p
        _lib.orc_philox4x32_10.argtypes = [vp, vp, vp]
        _lib.orc_direction.argtypes = [i32, P(i32), P(i32), P(i32), P(i32)]
        _lib.orc_prob_threshold.argtypes = [ctypes.c_double]
        _lib.orc_prob_threshold.restype = u64
        _lib.orc_target_count.argtypes = [ctypes.c_double, i64]
        _lib.orc_target_count.restype = i64
        _lib.orc_growth_threshold.argtypes = [u64, i64, i64]
        _lib.orc_growth_threshold.restype = u64
        _lib.orc_growth_draw.argtypes = [u64, i32, u32, i32]
        _lib.orc_growth_draw.restype = u32
        _lib.orc_seed_candidates.argtypes = [i32, i32, i32, u64, u64, vp, vp, i64]
        _lib.orc_seed_candidates.restype = i64
        _lib.orc_seed_select.argtypes = [i32, i32, i32, i32, i64, vp, vp, vp]
        _lib.orc_seed_select.restype = i64
        _lib.orc_interface.argtypes = [i32, i32, i32, vp, vp]
        _lib.orc_interface.restype = i64
        _lib.orc_step_liets.argtypes = [i32, i32, i32, vp, vp, i64, u32, vp, u64, vp, P(i64),
                                        vp, vp, vp, vp]
        _lib.orc_step_liets.restype = i64
        _lib.orc_step_fullfield.argtypes = [i32, i32, i32, vp, u32, vp, u64]
        _lib.orc_step_fullfield.restype = i64
        _lib.orc_generate.argtypes = [i32, i32, i32, P(_Params), vp, P(_Result), vp, vp, vp, vp,
                                      vp, vp, vp, vp, i32]
        _lib.orc_generate.restype = i32
        _lib.orc_generate_phases.argtypes = [i32, i32, i32, i32, P(_Params), vp, P(_Result)]
        _lib.orc_generate_phases.restype = i32
        _lib.orc_step_interacting.argtypes = [i32, i32, i32, vp, vp, vp, vp, i64, u32, u64, vp,
                                              P(i64), vp, vp, vp, vp]
        _lib.orc_step_interacting.restype = i64
        _lib.orc_generate_phases_interacting.argtypes = [i32, i32, i32, i32, P(_Params), vp, vp,
                                                         P(_Result)]
        _lib.orc_generate_phases_interacting.restype = i32
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key) -> tuple[int, int, int, int]:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return tuple(int(x) for x in out)


def direction(d: int) -> tuple[int, int, int, int]:
    v = [ctypes.c_int32() for _ in range(4)]
    lib().orc_direction(d, *[ctypes.byref(x) for x in v])
    return tuple(x.value for x in v)


def prob_threshold(p: float) -> int:
    return int(lib().orc_prob_threshold(float(p)))


def target_count(phi_s: float, n: int) -> int:
    return int(lib().orc_target_count(float(phi_s), int(n)))


def growth_threshold(t_ref: int, cnt: int, s_star: int) -> int:
    return int(lib().orc_growth_threshold(int(t_ref), int(cnt), int(s_star)))


def growth_draw(key: int, a: int, t: int, j: int) -> int:
    return int(lib().orc_growth_draw(int(key), int(a), int(t), int(j)))


def seed_candidates(dims, key: int, t_seed: int):
    nx, ny, nz = dims
    n = nx * ny * nz
    cand = np.zeros(max(n, 1), dtype=np.int32)
    prio = np.zeros(max(n, 1), dtype=np.uint64)
    k = lib().orc_seed_candidates(nx, ny, nz, int(key), int(t_seed), _ptr(cand), _ptr(prio), n)
    return cand[:k].copy(), prio[:k].copy()


def seed_select(dims, spacing: int, cand: np.ndarray, prio: np.ndarray):
    nx, ny, nz = dims
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    prio = np.ascontiguousarray(prio, dtype=np.uint64)
    grid = np.zeros((nz, ny, nx), dtype=np.uint8)
    k = lib().orc_seed_select(nx, ny, nz, int(spacing), len(cand), _ptr(cand), _ptr(prio),
                              _ptr(grid))
    return grid, int(k)


def interface(grid: np.ndarray) -> np.ndarray:
    nz, ny, nx = grid.shape
    g = np.ascontiguousarray(grid, dtype=np.uint8)
    out = np.zeros(max(g.size, 1), dtype=np.int32)
    k = lib().orc_interface(nx, ny, nz, _ptr(g), _ptr(out))
    return out[:k].copy()


def step_liets(grid: np.ndarray, front: np.ndarray, t: int, T, key: int, counters: bool = False):
    """One list-indexed step in place on ``grid``; returns (next front, n_new[, att, succ])."""
    assert grid.flags.c_contiguous and grid.dtype == np.uint8
    nz, ny, nx = grid.shape
    n = grid.size
    A = np.ascontiguousarray(front, dtype=np.int32)
    Tarr = np.asarray(T, dtype=np.uint64)
    A_next = np.zeros(max(n, 1), dtype=np.int32)
    mask = np.zeros(max(len(A), 1), dtype=np.uint32)
    new = np.zeros(max(n, 1), dtype=np.int32)
    att = np.zeros(26, dtype=np.uint64) if counters else None
    suc = np.zeros(26, dtype=np.uint64) if counters else None
    n_new = ctypes.c_int64()
    k = lib().orc_step_liets(nx, ny, nz, _ptr(grid), _ptr(A), len(A), int(t), _ptr(Tarr),
                             int(key), _ptr(A_next), ctypes.byref(n_new), _ptr(mask), _ptr(new),
                             _ptr(att), _ptr(suc))
    if counters:
        return A_next[:k].copy(), int(n_new.value), att, suc
    return A_next[:k].copy(), int(n_new.value)


def step_fullfield(grid: np.ndarray, t: int, T, key: int) -> int:
    assert grid.flags.c_contiguous and grid.dtype == np.uint8
    nz, ny, nx = grid.shape
    Tarr = np.asarray(T, dtype=np.uint64)
    return int(lib().orc_step_fullfield(nx, ny, nz, _ptr(grid), int(t), _ptr(Tarr), int(key)))


@dataclass
class OracleRun:
    grid: np.ndarray
    n_candidates: int
    n_seeds: int
    solid_count: int
    target_count: int
    front_size: int
    steps: int
    status: int
    birth: np.ndarray | None = None
    log_front: np.ndarray | None = None
    log_new: np.ndarray | None = None
    log_count: np.ndarray | None = None
    log_draws: np.ndarray | None = None
    log_blocks: np.ndarray | None = None
    log_band: np.ndarray | None = None
    log_band_union: np.ndarray | None = None


def generate(dims, solid_fraction: float, seed_prob: float, g_ref, spacing: int, key: int,
             max_steps: int = 0, birth: bool = False, log_cap: int = 0,
             literal_front: bool = False, bands: bool = False) -> OracleRun:
    """``literal_front``: the next sources are this step's new cells with a void
    neighbour (Algorithm 3 as printed) instead of the whole interface.  ``bands``: also
    log the sizes of the one-voxel bands around F_t and around F_t u New_t."""
    nx, ny, nz = dims
    p = _Params(float(solid_fraction), float(seed_prob), (ctypes.c_double * 3)(*g_ref),
                int(spacing), int(max_steps), int(key), 1 if literal_front else 0, 0)
    res = _Result()
    grid = np.zeros((nz, ny, nx), dtype=np.uint8)
    b = np.zeros((nz, ny, nx), dtype=np.int32) if birth else None
    lf = np.zeros(max(log_cap, 1), dtype=np.int64) if log_cap else None
    ln = np.zeros(max(log_cap, 1), dtype=np.int64) if log_cap else None
    lc = np.zeros(max(log_cap, 1), dtype=np.int64) if log_cap else None
    ld = np.zeros(max(log_cap, 1), dtype=np.int64) if log_cap else None
    lb = np.zeros(max(log_cap, 1), dtype=np.int64) if log_cap else None
    lbf = np.zeros(max(log_cap, 1), dtype=np.int64) if (log_cap and bands) else None
    lbu = np.zeros(max(log_cap, 1), dtype=np.int64) if (log_cap and bands) else None
    lib().orc_generate(nx, ny, nz, ctypes.byref(p), _ptr(grid), ctypes.byref(res), _ptr(b),
                       _ptr(lf), _ptr(ln), _ptr(lc), _ptr(ld), _ptr(lb), _ptr(lbf), _ptr(lbu),
                       int(log_cap))
    m = min(res.steps, log_cap)
    cut = (lambda a: a[:m].copy() if a is not None else None)
    return OracleRun(grid, res.n_candidates, res.n_seeds, res.solid_count, res.target_count,
                     res.front_size, res.steps, res.status, b, cut(lf), cut(ln), cut(lc),
                     cut(ld), cut(lb), cut(lbf), cut(lbu))


@dataclass
class PhaseResult:
    n_candidates: int
    n_seeds: int
    count: int
    target_count: int
    front_size: int
    steps: int
    status: int


def _phase_params(phases):
    k = len(phases)
    arr = (_Params * k)()
    for i, ph in enumerate(phases):
        sf, sd, g, sp, key = ph[:5]
        ms = ph[5] if len(ph) > 5 else 0
        lit = 1 if (len(ph) > 6 and ph[6]) else 0
        arr[i] = _Params(float(sf), float(sd), (ctypes.c_double * 3)(*g), int(sp), int(ms),
                         int(key), lit, 0)
    return arr


def generate_phases(dims, phases, interact=None) -> tuple[np.ndarray, list[PhaseResult]]:
    """Growing phases in sequence (Sec. 2.1 steps 1-5).  ``phases`` is a sequence of
    (solid_fraction, seed_prob, g_ref, spacing, key[, max_steps[, literal_front]]) tuples,
    phase n = index + 1; returns the label grid (0 = matrix, n = phase n) and one result
    per phase.  ``interact`` (optional): array [n_phases, n_phases, 3] of the
    phase-interaction probabilities I_c^{n,m} (index [n - 1, m - 1, c], read for m < n);
    None means independent phases."""
    nx, ny, nz = dims
    k = len(phases)
    arr = _phase_params(phases)
    res = (_Result * k)()
    labels = np.zeros((nz, ny, nx), dtype=np.uint8)
    if interact is None:
        lib().orc_generate_phases(nx, ny, nz, k, arr, _ptr(labels), res)
    else:
        I = np.ascontiguousarray(interact, dtype=np.float64)
        assert I.shape == (k, k, 3)
        lib().orc_generate_phases_interacting(nx, ny, nz, k, arr, _ptr(I), _ptr(labels), res)
    out = [PhaseResult(r.n_candidates, r.n_seeds, r.solid_count, r.target_count, r.front_size,
                       r.steps, r.status) for r in res]
    return labels, out


def step_interacting(labels: np.ndarray, cand, thr, front: np.ndarray, t: int, key: int,
                     counters: bool = False):
    """One growth step of the phase held as label 1 on ``labels`` (in place), with the
    candidate table ``cand`` (256 flags) and thresholds ``thr`` (256 x 3); returns (next
    front, converted cells[, attempts, successes]) -- counters 52 entries each: index d
    for unassigned targets, 26 + d for targets of other phases."""
    assert labels.flags.c_contiguous and labels.dtype == np.uint8
    nz, ny, nx = labels.shape
    n = labels.size
    A = np.ascontiguousarray(front, dtype=np.int32)
    c = np.ascontiguousarray(cand, dtype=np.uint8)
    T = np.ascontiguousarray(thr, dtype=np.uint64).reshape(-1)
    assert c.size == 256 and T.size == 768
    A_next = np.zeros(max(n, 1), dtype=np.int32)
    conv = np.zeros(max(n, 1), dtype=np.int32)
    mask = np.zeros(max(len(A), 1), dtype=np.uint32)
    att = np.zeros(52, dtype=np.uint64) if counters else None
    suc = np.zeros(52, dtype=np.uint64) if counters else None
    nn = ctypes.c_int64()
    k = lib().orc_step_interacting(nx, ny, nz, _ptr(labels), _ptr(c), _ptr(T), _ptr(A), len(A),
                                   int(t), int(key), _ptr(A_next), ctypes.byref(nn), _ptr(conv),
                                   _ptr(mask), _ptr(att), _ptr(suc))
    out = (A_next[:nn.value].copy(), conv[:k].copy())
    return out + (att, suc) if counters else out
