"""Planted mistakes in the CPU oracle: each must break at least one oracle pin.

Every case below rewrites one spot of ``oracle/qsgs_oracle.c`` into a plausible mistake
(a wrong constant, a comparison, an index, an order, a dropped term), compiles the copy with
gcc into a temporary library, binds it through a private copy of ``oracle/oracle.py`` and
runs the oracle pins of ``tests/test_oracle_*.py`` against it (every parametrization, the
tests that need more than the oracle left out) until one of them fails.  The unmodified
source, built the same way, passes all of them.  Mistakes are planted in the oracle on the
CPU only; nothing here touches the GPU library.

Each rewrite keeps every memory access in bounds (the index changes stay inside the grid),
so a mutant fails by its results, never by a crash.
"""
from __future__ import annotations

import importlib.util
import inspect
import itertools
import os
import shutil
import subprocess
import sys
import time

import pytest

from tests import (test_oracle_growth, test_oracle_phases, test_oracle_philox,
                   test_oracle_run, test_oracle_seeding, test_oracle_thresholds)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_DIR = os.path.join(ROOT, "oracle")
PIN_MODULES = [test_oracle_thresholds, test_oracle_philox, test_oracle_seeding,
               test_oracle_growth, test_oracle_run, test_oracle_phases]

_ROW_BOUND = "  if (qx < 0 || qx >= nx || qy < 0 || qy >= ny || qz < 0 || qz >= nz) return -1;\n"
_LIN = "(int64_t)qx + (int64_t)nx * ((int64_t)qy + (int64_t)ny * (int64_t)qz)"

# (name, what the mistake is, original text, planted text); the original occurs once.
MUTANTS = [
    ("philox_multiplier", "a wrong Philox round multiplier",
     "M0 = 0xD2511F53u", "M0 = 0xD2511F55u"),
    ("philox_round_key", "the wrong key word mixed into a Philox round",
     "uint32_t y0 = hi1 ^ x1 ^ k0;", "uint32_t y0 = hi1 ^ x1 ^ k1;"),
    ("philox_weyl", "a wrong key schedule constant",
     "W1 = 0xBB67AE85u", "W1 = 0xBB67AE87u"),
    ("threshold_rounding", "P32(p) rounded up instead of down",
     "return (uint64_t)floor(p * 4294967296.0);", "return (uint64_t)ceil(p * 4294967296.0);"),
    ("target_rounding", "S* rounded down instead of up",
     "double t = ceil(phi_s * (double)n);", "double t = floor(phi_s * (double)n);"),
    ("eq1_coefficient", "a wrong coefficient in Eq. (1)",
     "(20 * s_star - 19 * cnt)", "(20 * s_star - 18 * cnt)"),
    ("eq1_stale_count", "Eq. (1) never sees the grown count",
     "    cnt += n_new;\n", "\n"),
    ("class_permuted", "face, edge and corner classes permuted",
     "*cls = abs(x) + abs(y) + abs(z) - 1;", "*cls = (abs(x) + abs(y) + abs(z)) % 3;"),
    ("axis_swap", "x and y swapped in the neighbour's index",
     "  return " + _LIN + ";", "  return (int64_t)qy + (int64_t)ny * ((int64_t)qx + "
     "(int64_t)nx * (int64_t)qz);"),
    ("row_spill", "the x boundary missed: neighbours spill into the next row",
     _ROW_BOUND,
     "  if (qy < 0 || qy >= ny || qz < 0 || qz >= nz) return -1;\n"
     "  if (" + _LIN + " < 0 || " + _LIN + " >= (int64_t)nx * ny * nz) return -1;\n"),
    ("growth_not_strict", "a growth draw accepted at the threshold (<= for <)",
     "if ((uint64_t)w < T[cls]) {", "if ((uint64_t)w <= T[cls]) {"),
    ("rank_off_by_one", "every rank one too high",
     "int32_t j = popcount32(m & ((1u << d) - 1u));\n      uint32_t w",
     "int32_t j = popcount32(m & ((1u << d) - 1u)) + 1;\n      uint32_t w"),
    ("rank_by_direction", "draws ranked by direction instead of by void neighbour",
     "int32_t j = popcount32(m & ((1u << d) - 1u));\n      uint32_t w",
     "int32_t j = d;\n      uint32_t w"),
    ("draw_halves_swapped", "the two 16-bit halves of a draw swapped",
     "return (h << 16) | l;", "return (l << 16) | h;"),
    ("draw_block_index", "a wrong Philox block for a rank",
     "(uint32_t)(j >> 3), ORC_TAG_GROW_HI, hi);", "(uint32_t)(j >> 2), ORC_TAG_GROW_HI, hi);"),
    ("old_front_dropped", "the old front dropped from the next front",
     "  for (int64_t i = 0; i < nA; ++i)\n"
     "    if (has_void_neighbour(nx, ny, nz, grid, A[i])) A_next[kept++] = A[i];\n", ""),
    ("new_cells_not_listed", "the step's new cells left out of the next front",
     "  for (int64_t k = 0; k < added; ++k)\n"
     "    if (has_void_neighbour(nx, ny, nz, grid, new_scratch[k])) "
     "A_next[kept++] = new_scratch[k];\n", ""),
    ("fullfield_in_place", "the full-field form ranks on the half-updated grid",
     "if (r >= 0 && (grid[r] == 0 || grid[r] == 2)) ++j;", "if (r >= 0 && grid[r] == 0) ++j;"),
    ("seed_not_strict", "a core accepted at the seed threshold (<= for <)",
     "if ((uint64_t)w[0] < t_seed) {", "if ((uint64_t)w[0] <= t_seed) {"),
    ("seed_counter", "a wrong counter for the core draw",
     "philox_keyed(key, (uint32_t)v, 0u, 0u, ORC_TAG_SEED, w);",
     "philox_keyed(key, (uint32_t)v, 1u, 0u, ORC_TAG_SEED, w);"),
    ("seed_priority_words", "the priority's two words swapped",
     "prio[k] = ((uint64_t)w[1] << 32) | (uint64_t)w[2];",
     "prio[k] = ((uint64_t)w[2] << 32) | (uint64_t)w[1];"),
    ("spacing_radius", "the diamond's radius one too large",
     "const int32_t r = spacing - 1;", "const int32_t r = spacing;"),
    ("priority_order", "candidates accepted by descending priority",
     "return x->prio < y->prio ? -1 : 1;", "return x->prio > y->prio ? -1 : 1;"),
    ("tie_order", "priority ties broken by descending voxel index",
     "return x->v < y->v ? -1 : 1;", "return x->v > y->v ? -1 : 1;"),
    ("cores_on_other_phases", "cores placed on cells another phase holds",
     "    if (grid[A[i]] == 0) {\n", "    if (1) {\n"),
    ("interaction_uses_eq1", "conversions of another phase's cells take Eq. (1)",
     "uint64_t T = thr[3 * labels[q] + cls];", "uint64_t T = thr[cls];"),
    ("literal_front_unpruned", "Alg. 3's front keeps new cells without a void neighbour",
     "if (has_void_neighbour(nx, ny, nz, grid, added[k])) A_next[nA_next++] = added[k];",
     "A_next[nA_next++] = added[k];"),
]


def _pins():
    """(label, callable(orc)) for every oracle pin that needs nothing but the oracle."""
    out = []
    for mod in PIN_MODULES:
        for name, fn in sorted(vars(mod).items()):
            if not name.startswith("test_") or not callable(fn):
                continue
            params = list(inspect.signature(fn).parameters)
            if not params or params[0] != "orc":
                continue
            grids = {}
            for mark in getattr(fn, "pytestmark", []):
                if mark.name != "parametrize":
                    continue
                names = [s.strip() for s in mark.args[0].split(",")] \
                    if isinstance(mark.args[0], str) else list(mark.args[0])
                grids[tuple(names)] = list(mark.args[1])
            if set(params[1:]) != {n for k in grids for n in k}:
                continue  # needs another fixture
            keys = list(grids)
            for combo in itertools.product(*(grids[k] for k in keys)):
                kw = {}
                for k, v in zip(keys, combo):
                    kw.update(zip(k, v if len(k) > 1 else (v,)))
                label = f"{mod.__name__.split('.')[-1]}::{name}" + (f"{kw}" if kw else "")
                out.append((label, lambda orc, fn=fn, kw=kw: fn(orc, **kw)))
    return out


PINS = _pins()
# seconds per pin on the unmodified oracle, taken by the control test: the mutants try
# the cheap pins first (the order changes only how soon a mutant is caught)
_COST: dict = {}


def _bind(src_text: str, where: str, tag: str):
    """Compile src_text as the oracle in directory where; a private binding of it."""
    os.makedirs(where, exist_ok=True)
    shutil.copy(os.path.join(ORACLE_DIR, "qsgs_oracle.h"), where)
    src = os.path.join(where, "qsgs_oracle.c")
    with open(src, "w") as f:
        f.write(src_text)
    lib = os.path.join(where, "liborc_%s.so" % tag)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", lib, src, "-lm"])
    spec = importlib.util.spec_from_file_location("oracle_%s" % tag,
                                                  os.path.join(ORACLE_DIR, "oracle.py"))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod  # (its dataclasses look the module up)
    spec.loader.exec_module(mod)
    mod.build = lambda force=False: lib
    mod._lib = None
    return mod


def _first_failing_pin(mod):
    for label, pin in sorted(PINS, key=lambda p: _COST.get(p[0], 0.0)):
        try:
            pin(mod)
        except AssertionError:
            return label
        except pytest.skip.Exception:
            continue
    return None


@pytest.fixture(scope="module")
def source():
    with open(os.path.join(ORACLE_DIR, "qsgs_oracle.c")) as f:
        return f.read()


def test_pins_collected():
    # the pins of every module take part, parametrized ones in every combination
    mods = {label.split("::")[0] for label, _ in PINS}
    assert mods == {m.__name__.split(".")[-1] for m in PIN_MODULES}
    assert len(PINS) >= 60


def test_unmodified_oracle_passes_every_pin(source, tmp_path):
    mod = _bind(source, str(tmp_path), "control")
    for label, pin in PINS:
        t0 = time.perf_counter()
        pin(mod)  # raises on a failing pin
        _COST[label] = time.perf_counter() - t0


@pytest.mark.parametrize("name,what,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_breaks_a_pin(source, tmp_path, name, what, old, new):
    assert source.count(old) == 1, f"the site of '{name}' is not unique in the oracle"
    mod = _bind(source.replace(old, new), str(tmp_path), name)
    caught = _first_failing_pin(mod)
    assert caught is not None, f"no pin fails when the oracle has {what}"
