"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qsgs.h")


@pytest.fixture(scope="module")
def q():
    import paper_2602_11734_amd as q
    from paper_2602_11734_amd import build
    build.build_library(force=False)
    q.load()
    return q


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qsgs_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(q):
    names = declared_functions()
    assert len(names) >= 10
    lib = ctypes.CDLL(q.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(q.SIGNATURES), "binding and header disagree"


def test_version(q):
    assert "gfx950" in q.qsgs_version()


def test_size_queries(q):
    p = q.make_params(0.7, 0.005, (0.02, 0.005, 0.00125), 4, 0)
    assert q.qsgs_grid_bytes((64, 64, 64)) == 64**3 + 8  # N + 8 padding, multiple of 4
    assert q.qsgs_grid_bytes((3, 1, 1)) == 12
    assert q.qsgs_grid_bytes((0, 4, 4)) == 0
    assert q.qsgs_grid_bytes((2**11, 2**10, 2**10)) == 0  # N = 2^31
    ws = q.qsgs_workspace_bytes((64, 64, 64), p)
    n = 64**3
    assert ws >= 17 * n  # candidates, sorted candidates + priorities, status
    assert q.qsgs_step_workspace_bytes() >= 4096
    # a larger spacing needs fewer buckets, never more bytes
    p2 = q.make_params(0.7, 0.005, (0.02, 0.005, 0.00125), 30, 0)
    assert q.qsgs_workspace_bytes((64, 64, 64), p2) <= ws


@pytest.mark.parametrize("bad", [
    dict(solid_fraction=0.0), dict(solid_fraction=1.5), dict(solid_fraction=float("nan")),
    dict(seed_prob=-0.1), dict(seed_prob=1.01), dict(g_ref=(0.1, float("inf"), 0.0)),
    dict(g_ref=(0.1, 0.2, -0.3)), dict(spacing=-1),
])
def test_invalid_params_rejected_before_launch(q, bad):
    base = dict(solid_fraction=0.7, seed_prob=0.01, g_ref=(0.1, 0.05, 0.01), spacing=3, key=1)
    base.update(bad)
    p = q.make_params(**base)
    assert q.qsgs_workspace_bytes((8, 8, 8), p) == 0
    info = q.qsgs_info()
    st = q.load().qsgs_generate(ctypes.byref(q.make_dims((8, 8, 8))), ctypes.byref(p), 256,
                                256, 1 << 20, ctypes.byref(info), None)
    assert st == q.ERR_INVALID
    assert q.qsgs_last_error()


def test_sweep_form_flag_checked(q):
    for form in (q.SWEEP_LIST, q.SWEEP_FIELD, q.SWEEP_ALL_TILES):
        p = q.make_params(0.7, 0.01, (0.1, 0.05, 0.01), 3, 1, sweep_form=form)
        assert q.qsgs_workspace_bytes((8, 8, 8), p) > 0
    p.sweep_form = 3
    assert q.qsgs_workspace_bytes((8, 8, 8), p) == 0
    p.sweep_form = -1
    assert q.qsgs_workspace_bytes((8, 8, 8), p) == 0
    p.sweep_form = 0
    p.front_rule = 7
    assert q.qsgs_workspace_bytes((8, 8, 8), p) == 0
    # the full-field form has no front: the literal front rule is refused with it
    p = q.make_params(0.7, 0.01, (0.1, 0.05, 0.01), 3, 1, sweep_form=q.SWEEP_FIELD,
                      literal_front=True)
    assert q.qsgs_workspace_bytes((8, 8, 8), p) == 0
    p.sweep_form = q.SWEEP_ALL_TILES
    assert q.qsgs_workspace_bytes((8, 8, 8), p) > 0


def test_interaction_arguments_checked_before_launch(q):
    """Interaction probabilities outside [0, 1] and an interacting phase in the full-field
    form are refused before anything runs (device pointers here are dummies)."""
    import numpy as np
    ph = [q.make_params(0.3, 0.01, (0.1, 0.05, 0.01), 2, 1),
          q.make_params(0.2, 0.01, (0.1, 0.05, 0.01), 2, 2)]
    dims = (16, 16, 16)
    wb = q.qsgs_phases_workspace_bytes(dims, ph)
    assert wb > q.qsgs_workspace_bytes(dims, ph[0])  # walls and interaction planes, table
    I = np.zeros((2, 2, 3))
    I[1, 0] = (0.5, 1.5, 0.0)
    with pytest.raises(q.QsgsError) as e:
        q.qsgs_generate_phases_interacting(dims, ph, I, 256, 256, wb, stream=0)
    assert e.value.status == q.ERR_INVALID and "interaction" in str(e.value)
    I[1, 0] = (0.5, 0.5, 0.0)
    ph[1].sweep_form = q.SWEEP_FIELD
    with pytest.raises(q.QsgsError) as e:
        q.qsgs_generate_phases_interacting(dims, ph, I, 256, 256, wb, stream=0)
    assert e.value.status == q.ERR_INVALID and "full-field" in str(e.value)
    with pytest.raises(q.QsgsError):
        q.qsgs_generate_phases_interacting(dims, ph, np.zeros((3, 3, 3)), 256, 256, wb, stream=0)


def test_front_rule_flag_checked(q):
    p = q.make_params(0.7, 0.01, (0.1, 0.05, 0.01), 3, 1)
    p.front_rule = 7
    info = q.qsgs_info()
    st = q.load().qsgs_generate(ctypes.byref(q.make_dims((8, 8, 8))), ctypes.byref(p), 256,
                                256, 1 << 20, ctypes.byref(info), None)
    assert st == q.ERR_INVALID and "front_rule" in q.qsgs_last_error()
    p.front_rule = 1  # the literal rule: whole-generation calls only
    assert q.qsgs_workspace_bytes((8, 8, 8), p) > 0
    st = q.load().qsgs_grow_step(ctypes.byref(q.make_dims((8, 8, 8))), ctypes.byref(p), 256,
                                 512, 1024, 100, 256, 1 << 20, ctypes.byref(info), None)
    assert st == q.ERR_INVALID and "front_rule" in q.qsgs_last_error()


def test_invalid_dims_and_pointers(q):
    p = q.make_params(0.7, 0.01, (0.1, 0.05, 0.01), 3, 1)
    info = q.qsgs_info()
    lib = q.load()
    for dims in ((0, 8, 8), (8, -1, 8), (2**11, 2**10, 2**10)):
        st = lib.qsgs_generate(ctypes.byref(q.make_dims(dims)), ctypes.byref(p), 256, 256,
                               1 << 20, ctypes.byref(info), None)
        assert st == q.ERR_INVALID
    d = ctypes.byref(q.make_dims((8, 8, 8)))
    assert lib.qsgs_generate(d, ctypes.byref(p), None, 256, 1 << 20, ctypes.byref(info),
                             None) == q.ERR_INVALID
    assert lib.qsgs_generate(d, ctypes.byref(p), 258, 256, 1 << 20, ctypes.byref(info),
                             None) == q.ERR_INVALID  # misaligned grid
    assert "aligned" in q.qsgs_last_error()
    assert lib.qsgs_generate(d, ctypes.byref(p), 256, 256, 16, ctypes.byref(info),
                             None) == q.ERR_WORKSPACE
    assert lib.qsgs_grow_step(d, ctypes.byref(p), 256, 512, 512, 100, 256, 1 << 20,
                              ctypes.byref(info), None) == q.ERR_INVALID  # same buffers
    assert lib.qsgs_grow_step(d, ctypes.byref(p), 256, 512, 1024, 100, 256, 16,
                              ctypes.byref(info), None) == q.ERR_WORKSPACE
    bad_info = q.qsgs_info()
    bad_info.front_size = 200
    assert lib.qsgs_grow_step(d, ctypes.byref(p), 256, 512, 1024, 100, 256, 1 << 20,
                              ctypes.byref(bad_info), None) == q.ERR_INVALID
    assert lib.qsgs_seed(d, ctypes.byref(p), 256, None, 100, 256, 1 << 30, ctypes.byref(info),
                         None) == q.ERR_INVALID


def test_phases_arguments_checked(q):
    """Multi-phase queries and argument checks (nothing is launched)."""
    dims = (16, 16, 16)
    p1 = q.make_params(0.3, 0.01, (0.1, 0.05, 0.01), 3, 1)
    p2 = q.make_params(0.2, 0.01, (0.1, 0.05, 0.01), 30, 2)
    w1, w2 = q.qsgs_workspace_bytes(dims, p1), q.qsgs_workspace_bytes(dims, p2)
    # one phase at a time, plus the walls and interaction planes and the interaction table
    assert q.qsgs_phases_workspace_bytes(dims, [p1, p2]) > max(w1, w2)
    assert q.qsgs_phases_workspace_bytes(dims, [p1, p2]) < max(w1, w2) + 64 * 1024
    assert w1 < q.qsgs_phases_workspace_bytes(dims, [p1]) < w1 + 64 * 1024
    bad = q.make_params(1.5, 0.01, (0.1, 0.05, 0.01), 3, 1)
    assert q.qsgs_phases_workspace_bytes(dims, [p1, bad]) == 0
    lib = q.load()
    d = ctypes.byref(q.make_dims(dims))
    arr = (q.qsgs_params * 2)(p1, p2)
    infos = (q.qsgs_info * 2)()
    assert lib.qsgs_phases_workspace_bytes(d, 0, arr) == 0
    assert lib.qsgs_phases_workspace_bytes(d, 253, arr) == 0
    assert lib.qsgs_generate_phases(d, 0, arr, 256, 256, 1 << 24, infos, None) == q.ERR_INVALID
    assert lib.qsgs_generate_phases(d, 2, arr, None, 256, 1 << 24, infos, None) == q.ERR_INVALID
    assert lib.qsgs_generate_phases(d, 2, arr, 258, 256, 1 << 24, infos, None) == q.ERR_INVALID
    assert "aligned" in q.qsgs_last_error()
    assert lib.qsgs_generate_phases(d, 2, arr, 256, 256, 16, infos, None) == q.ERR_WORKSPACE
    arr_bad = (q.qsgs_params * 2)(p1, bad)
    assert lib.qsgs_generate_phases(d, 2, arr_bad, 256, 256, 1 << 24, infos,
                                    None) == q.ERR_INVALID


def test_finished_state_is_a_noop(q):
    """A grow step on a state whose status is already terminal returns it untouched
    without launching anything (so it runs on a machine without a GPU)."""
    p = q.make_params(0.7, 0.01, (0.1, 0.05, 0.01), 3, 1)
    info = q.qsgs_info()
    info.status = q.DONE
    info.front_size = 5
    st = q.load().qsgs_grow_step(ctypes.byref(q.make_dims((8, 8, 8))), ctypes.byref(p), 256, 512,
                                 1024, 100, 256, 1 << 20, ctypes.byref(info), None)
    assert st == q.DONE and info.front_size == 5


def test_package_fails_loudly_without_library(tmp_path):
    import paper_2602_11734_amd as q
    saved = q._lib
    q._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            q.load(str(tmp_path / "missing.so"))
    finally:
        q._lib = saved


def test_seed_prob_from_grain(q):
    """S_d = 6 phi_s delta^3 / (pi d^3) (Sec. 3.3): a grain of diameter d holds
    pi d^3 / (6 delta^3) voxels, so phi_s N / that volume cores give the fraction phi_s."""
    import math
    v = q.qsgs_seed_prob_from_grain(0.8, 225.0, 4.0)
    assert abs(v - 6 * 0.8 * 64 / (math.pi * 225.0**3)) < 1e-18
    assert abs(v - 8.584e-6) < 1e-9
    # one grain per voxel-sized sphere volume: d = delta (6/pi)^(1/3) gives phi_s
    d = 4.0 * (6 / math.pi) ** (1 / 3)
    assert abs(q.qsgs_seed_prob_from_grain(0.3, d, 4.0) - 0.3) < 1e-12
    assert q.qsgs_seed_prob_from_grain(1.0, 1.0, 10.0) == 1.0  # capped
    for bad in ((1.2, 200.0, 4.0), (0.5, 0.0, 4.0), (0.5, 200.0, -1.0)):
        with pytest.raises(q.QsgsError):
            q.qsgs_seed_prob_from_grain(*bad)


def test_noalloc_refuses_oversized_grids_before_touching_a_device(q):
    """The allocation-free entry point checks the generation's scratch need against its
    fixed scratch first: a 400^3 generation is refused without any HIP call."""
    p = q.make_params(0.8, 5e-4, (0.01, 0.0025, 0.000625), 20, 1)
    info = q.qsgs_info()
    st = q.load().qsgs_generate_noalloc(ctypes.byref(q.make_dims((400, 400, 400))),
                                        ctypes.byref(p), 256, ctypes.byref(info), None)
    assert st == q.ERR_WORKSPACE
    assert "scratch" in q.qsgs_last_error()
    assert q.qsgs_workspace_bytes((400, 400, 400), p) > 128 << 20


def test_band_sizes_arguments_checked(q):
    """The band-size utility: scratch size query and argument checks before any launch."""
    lib = q.load()
    assert q.qsgs_band_scratch_bytes((10, 10, 10)) >= 1000 + 16
    assert q.qsgs_band_scratch_bytes((0, 10, 10)) == 0
    d = ctypes.byref(q.make_dims((10, 10, 10)))
    out = (ctypes.c_uint64 * 2)()
    sb = q.qsgs_band_scratch_bytes((10, 10, 10))
    assert lib.qsgs_band_sizes(d, None, 256, 512, sb, out, None) == q.ERR_INVALID
    assert lib.qsgs_band_sizes(d, 256, 256, 512, sb, None, None) == q.ERR_INVALID
    assert lib.qsgs_band_sizes(d, 256, 256, 512, 16, out, None) == q.ERR_WORKSPACE
    assert lib.qsgs_band_sizes(d, 256, 256, 516, sb, out, None) == q.ERR_INVALID  # alignment
    bad = ctypes.byref(q.make_dims((0, 1, 1)))
    assert lib.qsgs_band_sizes(bad, 256, 256, 512, sb, out, None) == q.ERR_INVALID


def test_async_arguments_checked(q):
    """The calls without host synchronisation: a step cap outside [1, 4096], a NULL or
    misaligned info, a short workspace: errors before any launch."""
    lib = q.load()
    d = ctypes.byref(q.make_dims((8, 8, 8)))
    for steps in (0, -1, 4097):
        p = q.make_params(0.7, 0.01, (0.1, 0.05, 0.01), 3, 1, max_steps=steps)
        assert lib.qsgs_generate_async(d, ctypes.byref(p), 256, 256, 1 << 20, 1024,
                                       None) == q.ERR_INVALID
        assert "max_steps" in q.qsgs_last_error()
    p = q.make_params(0.7, 0.01, (0.1, 0.05, 0.01), 3, 1, max_steps=10)
    assert lib.qsgs_generate_async(d, ctypes.byref(p), 256, 256, 1 << 20, None,
                                   None) == q.ERR_INVALID
    assert lib.qsgs_generate_async(d, ctypes.byref(p), 256, 256, 1 << 20, 1028,
                                   None) == q.ERR_INVALID  # misaligned info
    assert lib.qsgs_generate_async(d, ctypes.byref(p), 256, 256, 16, 1024,
                                   None) == q.ERR_WORKSPACE
