"""GPU parity: the HIP library through its C ABI against the CPU oracle, bit-exact.

Small and ragged grids and the degenerate cases are compared with live oracle runs;
the 200^3 and 400^3 workloads are compared with the oracle's stored results
(tests/golden/oracle_runs.json, written by tests/golden/make_goldens.py).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "oracle_runs.json")


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_11734_amd as q
    if not os.path.exists(q.LIB_PATH):
        from paper_2602_11734_amd import build
        build.build_library()
    q.load()
    return q


def say(*a):
    print(*a, flush=True)


def run_gpu(q, case, literal_front=False):
    import torch
    say("GPU generate", case.name, case.dims, "key", case.key,
        "literal front" if literal_front else "")
    params = q.params_of(case, literal_front=literal_front)
    grid, info, buf = q.generate(case.dims, params)
    torch.cuda.synchronize()
    logs = q.qsgs_read_step_log(buf.ws, buf.ws_bytes) + q.qsgs_read_step_work(buf.ws,
                                                                               buf.ws_bytes)
    return grid.cpu().numpy(), info, logs


def run_oracle(orc, case, **kw):
    return orc.generate(case.dims, case.solid_fraction, case.seed_prob, case.g_ref, case.spacing,
                        case.key, max_steps=case.max_steps, log_cap=100000, **kw)


SMALL = workloads.small_cases() + workloads.config1()


@pytest.mark.parametrize("case", SMALL, ids=[c.name for c in SMALL])
def test_generate_matches_oracle(q, orc, case):
    got, info, (lf, ln, lc, ld, lb) = run_gpu(q, case)
    ref = run_oracle(orc, case)
    assert info["status"] == ref.status
    assert info["n_candidates"] == ref.n_candidates
    assert info["n_seeds"] == ref.n_seeds
    assert info["step"] == ref.steps
    assert info["solid_count"] == ref.solid_count
    assert info["target_count"] == ref.target_count
    assert info["front_size"] == ref.front_size
    assert np.array_equal(lf, ref.log_front)
    assert np.array_equal(ln, ref.log_new)
    assert np.array_equal(lc, ref.log_count)
    assert np.array_equal(ld, ref.log_draws)
    assert np.array_equal(lb, ref.log_blocks)
    assert np.array_equal(got, ref.grid)


FORM_CASES = SMALL[::3] + workloads.config1()
FORM_NAMES = {1: "full_field", 2: "all_tiles"}


def expected_blocks(ref, case, form):
    """High-half Philox blocks per step: the list forms draw one per eight ranks of each
    front voxel (the oracle's count); the full-field form draws four for every cell of
    the grid every step (Algorithm 2's work)."""
    if form == 1:
        n = case.dims[0] * case.dims[1] * case.dims[2]
        return np.full(len(ref.log_blocks), 4 * n, dtype=np.int64)
    return ref.log_blocks


@pytest.mark.parametrize("form", [1, 2], ids=["full_field", "all_tiles"])
@pytest.mark.parametrize("case", FORM_CASES, ids=[c.name for c in FORM_CASES])
def test_sweep_forms_match_oracle(q, orc, case, form):
    """The full-field form (every cell draws every step, Algorithm 2) and the all-tiles
    sweep reach the same grid, logs and draw counts as the list-indexed form and the
    oracle; the full-field form's Philox work is four blocks per cell per step."""
    import torch
    say("GPU generate", FORM_NAMES[form], case.name, case.dims, "key", case.key)
    params = q.params_of(case, sweep_form=form)
    grid, info, buf = q.generate(case.dims, params)
    torch.cuda.synchronize()
    lf, ln, lc = q.qsgs_read_step_log(buf.ws, buf.ws_bytes)
    ld, lb = q.qsgs_read_step_work(buf.ws, buf.ws_bytes)
    ref = run_oracle(orc, case)
    assert info["status"] == ref.status and info["step"] == ref.steps
    assert info["solid_count"] == ref.solid_count and info["front_size"] == ref.front_size
    assert info["n_seeds"] == ref.n_seeds
    assert np.array_equal(lf, ref.log_front) and np.array_equal(ln, ref.log_new)
    assert np.array_equal(lc, ref.log_count)
    assert np.array_equal(ld, ref.log_draws)
    assert np.array_equal(lb, expected_blocks(ref, case, form))
    assert np.array_equal(grid.cpu().numpy(), ref.grid)


def test_generate_is_deterministic(q):
    import torch
    case = workloads.small_cases()[0]
    a, ia, _ = run_gpu(q, case)
    # a second, separately allocated workspace; a busy stream in between
    x = torch.randn(1 << 22, device="cuda")
    (x * 2).sum()
    b, ib, _ = run_gpu(q, case)
    assert ia == ib and np.array_equal(a, b)


def _step_api_run(q, orc, case, front_cap=None, check_every_step=True):
    """qsgs_seed + qsgs_grow_step, compared with the oracle's own steps each step."""
    import torch
    nx, ny, nz = case.dims
    n = nx * ny * nz
    params = q.params_of(case)
    cap = n if front_cap is None else front_cap
    grid = torch.empty(q.qsgs_grid_bytes(case.dims), dtype=torch.uint8, device="cuda")
    fa = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    fb = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    wsb = q.qsgs_workspace_bytes(case.dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    sws = torch.empty(q.qsgs_step_workspace_bytes(), dtype=torch.uint8, device="cuda")
    say("GPU seed", case.name)
    st, info = q.qsgs_seed(case.dims, params, grid, fa, cap, ws, wsb)

    # oracle side, step by step from its own seeds
    tseed = orc.prob_threshold(case.seed_prob)
    cand, prio = orc.seed_candidates(case.dims, case.key, tseed)
    g_ref, _ = orc.seed_select(case.dims, case.spacing, cand, prio)
    front_ref = orc.interface(g_ref)
    s_star = orc.target_count(case.solid_fraction, n)
    t_ref = [orc.prob_threshold(g) for g in case.g_ref]
    cnt = int(g_ref.sum())
    assert info.n_seeds == cnt and info.n_candidates == len(cand)
    assert np.array_equal(grid[:n].view(nz, ny, nx).cpu().numpy(), g_ref)
    assert np.array_equal(np.sort(fa[: info.front_size].cpu().numpy()), front_ref)

    t = 0
    while st == q.OK:
        T = [orc.growth_threshold(tr, cnt, s_star) for tr in t_ref]
        front_ref, n_new = orc.step_liets(g_ref, front_ref, t, T, case.key)
        cnt += n_new
        say("GPU grow_step", case.name, "t", t)
        st, info = q.qsgs_grow_step(case.dims, params, grid, fa, fb, cap, sws, sws.numel(), info)
        fa, fb = fb, fa
        assert info.step == t + 1 and info.solid_count == cnt
        assert info.grown_last_step == n_new
        if check_every_step or st != q.OK:
            assert np.array_equal(grid[:n].view(nz, ny, nx).cpu().numpy(), g_ref), t
            assert np.array_equal(np.sort(fa[: info.front_size].cpu().numpy()), np.sort(front_ref)), t
        t += 1
    ref = run_oracle(orc, case)
    assert st == ref.status and info.step == ref.steps
    assert np.array_equal(g_ref, ref.grid)
    return grid, info


@pytest.mark.parametrize("idx", [0, 4, 7, 16])
def test_step_api_matches_oracle_each_step(q, orc, idx):
    cases = workloads.small_cases()
    _step_api_run(q, orc, cases[idx])


def test_step_api_config1(q, orc):
    _step_api_run(q, orc, workloads.config1()[0])


def test_capacity_error_restores_state(q, orc):
    """A front buffer too small for F_t + New_t: the step reports QSGS_ERR_CAPACITY,
    leaves the grid as it was, and succeeds when retried with room."""
    import torch
    case = workloads.config1()[0]
    nx, ny, nz = case.dims
    n = nx * ny * nz
    params = q.params_of(case)
    grid = torch.empty(q.qsgs_grid_bytes(case.dims), dtype=torch.uint8, device="cuda")
    wsb = q.qsgs_workspace_bytes(case.dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    sws = torch.empty(q.qsgs_step_workspace_bytes(), dtype=torch.uint8, device="cuda")
    small = 3000
    fa = torch.empty(n, dtype=torch.int32, device="cuda")
    fb = torch.empty(n, dtype=torch.int32, device="cuda")
    say("GPU seed (capacity test)")
    st, info = q.qsgs_seed(case.dims, params, grid, fa, small, ws, wsb)
    assert st == q.OK and info.front_size <= small
    before = grid.clone()
    front_before = fa[: info.front_size].clone()
    saved = q.qsgs_info.from_buffer_copy(info)
    say("GPU grow_step with a small front buffer")
    with pytest.raises(q.QsgsError) as e:
        q.qsgs_grow_step(case.dims, params, grid, fa, fb, small, sws, sws.numel(), info)
    assert e.value.status == q.ERR_CAPACITY
    assert torch.equal(grid, before)
    assert torch.equal(fa[: info.front_size], front_before)
    assert bytes(info) == bytes(saved)
    say("GPU grow_step retry")
    st, info = q.qsgs_grow_step(case.dims, params, grid, fa, fb, n, sws, sws.numel(), info)
    # the retried step equals the oracle's first step
    ref = run_oracle(orc, case, birth=True)
    g1 = ((ref.birth >= 0) & (ref.birth <= 1)).astype(np.uint8)
    assert np.array_equal(grid[:n].view(nz, ny, nx).cpu().numpy(), g1)


def test_seed_capacity_error(q):
    import torch
    case = workloads.config1()[0]
    params = q.params_of(case)
    grid = torch.empty(q.qsgs_grid_bytes(case.dims), dtype=torch.uint8, device="cuda")
    wsb = q.qsgs_workspace_bytes(case.dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    fa = torch.full((16,), -7, dtype=torch.int32, device="cuda")
    say("GPU seed with a 10-entry front buffer")
    with pytest.raises(q.QsgsError) as e:
        q.qsgs_seed(case.dims, params, grid, fa, 10, ws, wsb)
    assert e.value.status == q.ERR_CAPACITY
    assert torch.all(fa[10:] == -7)


def _golden():
    if not os.path.exists(GOLDEN):
        return {}
    with open(GOLDEN) as f:
        return json.load(f)


def _golden_check(q, entry):
    import torch
    c = entry["case"]
    case = workloads.Case(**{**c, "dims": tuple(c["dims"]), "g_ref": tuple(c["g_ref"])})
    got, info, (lf, ln, lc, ld, lb) = run_gpu(q, case, entry.get("literal_front", False))
    assert info["status"] == entry["status"]
    assert info["n_candidates"] == entry["n_candidates"]
    assert info["n_seeds"] == entry["n_seeds"]
    assert info["step"] == entry["steps"]
    assert info["solid_count"] == entry["solid_count"]
    assert info["front_size"] == entry["front_size"]
    assert list(lf) == entry["log_front"]
    assert list(ln) == entry["log_new"]
    assert list(lc) == entry["log_count"]
    assert list(ld) == entry["log_draws"]
    assert list(lb) == entry["log_blocks"]
    assert hashlib.sha256(got.tobytes()).hexdigest() == entry["grid_sha256"]
    del got
    torch.cuda.empty_cache()


GOLD_NAMES = sorted(_golden().keys())


@pytest.mark.parametrize("name", GOLD_NAMES)
def test_full_size_matches_oracle_golden(q, name):
    _golden_check(q, _golden()[name])


def test_batch_matches_oracle(q, orc):
    """Uneven realizations (sizes, spacing, degenerate cases) in one batch: each result
    equals the oracle's run of that realization alone."""
    import torch
    cases = workloads.small_cases() + workloads.config1()
    # the three growth forms in turn: the tile forms share the sweep launches, the
    # full-field realizations share the full-field launches of the same passes
    forms = [k % 3 for k in range(len(cases))]
    params = [q.params_of(c, sweep_form=f) for c, f in zip(cases, forms)]
    dims = [c.dims for c in cases]
    grids = [torch.empty(q.qsgs_grid_bytes(d), dtype=torch.uint8, device="cuda") for d in dims]
    wsb = q.qsgs_batch_workspace_bytes(dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    say("GPU generate_batch of", len(cases))
    st, infos = q.qsgs_generate_batch(dims, params, grids, ws, wsb)
    torch.cuda.synchronize()
    for k, (c, g, info) in enumerate(zip(cases, grids, infos)):
        ref = run_oracle(orc, c)
        nx, ny, nz = c.dims
        got = g[: nx * ny * nz].view(nz, ny, nx).cpu().numpy()
        assert info.status == ref.status, c.name
        assert info.step == ref.steps and info.solid_count == ref.solid_count, c.name
        assert info.n_seeds == ref.n_seeds and info.front_size == ref.front_size, c.name
        assert np.array_equal(got, ref.grid), c.name
        lf, ln, lc = q.qsgs_read_step_log(ws, wsb, index=k)
        assert np.array_equal(lf, ref.log_front[: len(lf)]) and len(lf) == min(ref.steps, 4096)
        assert np.array_equal(ln, ref.log_new[: len(ln)])
        assert np.array_equal(lc, ref.log_count[: len(lc)])
        ld, lb = q.qsgs_read_step_work(ws, wsb, index=k)
        assert np.array_equal(ld, ref.log_draws[: len(ld)])
        assert np.array_equal(lb, expected_blocks(ref, c, forms[k])[: len(lb)])


def test_large_batch_matches_oracle(q, orc):
    """A batch of more realizations than a wavefront (80): the step end plans it with
    block-wide scans.  Every result equals the oracle's run of that realization alone."""
    import torch
    cases = workloads.many_small_cases()
    params = [q.params_of(c) for c in cases]
    dims = [c.dims for c in cases]
    grids = [torch.empty(q.qsgs_grid_bytes(d), dtype=torch.uint8, device="cuda") for d in dims]
    wsb = q.qsgs_batch_workspace_bytes(dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    say("GPU generate_batch of", len(cases))
    st, infos = q.qsgs_generate_batch(dims, params, grids, ws, wsb)
    torch.cuda.synchronize()
    for c, g, info in zip(cases, grids, infos):
        ref = run_oracle(orc, c)
        nx, ny, nz = c.dims
        assert info.status == ref.status and info.step == ref.steps, c.name
        assert np.array_equal(g[: nx * ny * nz].view(nz, ny, nx).cpu().numpy(), ref.grid), c.name


def test_batch_reuses_workspace(q, orc):
    """Two batches in a row on one workspace, the second smaller and with other keys."""
    import torch
    base = workloads.small_cases()[:6]
    for rnd, cases in enumerate((base, base[1:4])):
        cases = [workloads.Case(**{**c.as_dict(), "key": c.key + 1000 * rnd}) for c in cases]
        params = [q.params_of(c) for c in cases]
        dims = [c.dims for c in cases]
        grids = [torch.empty(q.qsgs_grid_bytes(d), dtype=torch.uint8, device="cuda")
                 for d in dims]
        if rnd == 0:
            wsb = q.qsgs_batch_workspace_bytes(dims, params)
            ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        assert q.qsgs_batch_workspace_bytes(dims, params) <= wsb
        say("GPU generate_batch round", rnd)
        q.qsgs_generate_batch(dims, params, grids, ws, wsb)
        for c, g in zip(cases, grids):
            ref = run_oracle(orc, c)
            nx, ny, nz = c.dims
            assert np.array_equal(g[: nx * ny * nz].view(nz, ny, nx).cpu().numpy(), ref.grid)


def test_server_results_equal_solo_runs(q, orc):
    """Requests of mixed sizes through the continuous-batching server with an arena
    small enough that admission has to wait: every result equals the oracle's run of
    that request alone, and the arena is fully returned at the end."""
    import torch
    cases = workloads.small_cases()[:10] + workloads.config1()
    reserved = q.qsgs_server_reserved_bytes(4)
    # the 64^3 request needs ~30 N bytes with its seeding scratch: admission binds
    arena_bytes = reserved + 40 * 64**3
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    srv = q.qsgs_server_create(arena, arena_bytes, 4, steps_per_tick=2)
    try:
        free0 = q.qsgs_server_free_bytes(srv)
        pending = list(enumerate(cases))
        results = {}
        ticks = 0
        max_resident = 0
        while len(results) < len(cases):
            # three requests arrive together (they share the device), the rest staggered
            for _ in range(3 if ticks == 0 else (1 if ticks % 2 == 0 else 0)):
                if pending:
                    rid, c = pending.pop(0)
                    q.qsgs_server_submit(srv, rid, c.dims, q.params_of(c))
            say("server tick", ticks)
            res, queued, nready = q.qsgs_server_tick(srv)
            max_resident = max(max_resident, res)
            for rid, info in q.qsgs_server_ready(srv):
                c = cases[rid]
                nx, ny, nz = c.dims
                out = np.empty(nx * ny * nz, dtype=np.uint8)
                q.qsgs_server_take(srv, rid, out)
                results[rid] = (out.reshape(nz, ny, nx), info)
            ticks += 1
            assert ticks < 2000
        assert max_resident >= 2  # requests overlapped on the device
        assert q.qsgs_server_free_bytes(srv) == free0
    finally:
        q.qsgs_server_destroy(srv)
    for rid, c in enumerate(cases):
        grid, info = results[rid]
        ref = run_oracle(orc, c)
        assert info.status == ref.status and info.step == ref.steps, c.name
        assert info.solid_count == ref.solid_count, c.name
        assert np.array_equal(grid, ref.grid), c.name


def test_server_mixes_front_rules(q, orc):
    """Requests with either front rule share the server's launches: each result equals
    the oracle's run of that request alone with its rule."""
    import torch
    cases = workloads.small_cases()[:8] + workloads.config1()
    lit = [k % 2 == 1 for k in range(len(cases))]
    reserved = q.qsgs_server_reserved_bytes(len(cases))
    arena_bytes = reserved + 64 * 64**3
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    srv = q.qsgs_server_create(arena, arena_bytes, len(cases), steps_per_tick=3)
    results = {}
    try:
        for rid, (c, f) in enumerate(zip(cases, lit)):
            q.qsgs_server_submit(srv, rid, c.dims, q.params_of(c, literal_front=f))
        ticks = 0
        while len(results) < len(cases):
            say("server tick (mixed front rules)", ticks)
            q.qsgs_server_tick(srv)
            for rid, info in q.qsgs_server_ready(srv):
                nx, ny, nz = cases[rid].dims
                out = np.empty(nx * ny * nz, dtype=np.uint8)
                q.qsgs_server_take(srv, rid, out)
                results[rid] = (out.reshape(nz, ny, nx), info)
            ticks += 1
            assert ticks < 2000
    finally:
        q.qsgs_server_destroy(srv)
    for rid, (c, f) in enumerate(zip(cases, lit)):
        grid, info = results[rid]
        ref = run_oracle(orc, c, literal_front=f)
        assert info.status == ref.status and info.step == ref.steps, c.name
        assert info.solid_count == ref.solid_count, c.name
        assert np.array_equal(grid, ref.grid), c.name


def test_server_rejects_oversized_request(q):
    import torch
    reserved = q.qsgs_server_reserved_bytes(2)
    arena = torch.empty(reserved + (1 << 20), dtype=torch.uint8, device="cuda")
    srv = q.qsgs_server_create(arena, arena.numel(), 2)
    try:
        c = workloads.config1()[0]
        with pytest.raises(q.QsgsError) as e:
            q.qsgs_server_submit(srv, 1, c.dims, q.params_of(c))
        assert e.value.status == q.ERR_CAPACITY
    finally:
        q.qsgs_server_destroy(srv)


def test_tuning_does_not_change_results(q, orc):
    case = workloads.small_cases()[0]
    ref = run_oracle(orc, case)
    try:
        for t in ({"grow_block": 64, "grow_grid": 8, "prune_block": 512, "prune_grid": 64,
                   "seed_block": 128, "seed_grid": 16, "steps_per_sync": 1},
                  {"grow_block": 512, "grow_grid": 4096, "prune_block": 128, "prune_grid": 1024,
                   "seed_block": 512, "seed_grid": 4096, "steps_per_sync": 5}):
            q.qsgs_set_tuning(t)
            got, info, _ = run_gpu(q, case)
            assert np.array_equal(got, ref.grid) and info["step"] == ref.steps
    finally:
        q.qsgs_set_tuning(None)
    with pytest.raises(q.QsgsError):
        q.qsgs_set_tuning({"grow_block": 100, "grow_grid": 8, "prune_block": 64,
                           "prune_grid": 8, "seed_block": 64, "seed_grid": 8,
                           "steps_per_sync": 0})


# ----- multi-phase generation (Sec. 2.1 steps 1-5) -----

def _phase_tuples(ps):
    return [(c.solid_fraction, c.seed_prob, c.g_ref, c.spacing, c.key, c.max_steps)
            for c in ps.phases]


PHASES = workloads.phase_sets()


# every set with the list-indexed sweep; two sets with the full-field and all-tiles forms
PHASE_RUNS = [(ps, 0) for ps in PHASES] + [(ps, f) for f in (1, 2) for ps in PHASES[:2]]


@pytest.mark.parametrize("ps,form", PHASE_RUNS,
                         ids=[f"{p.name}-{['list', 'full_field', 'all_tiles'][f]}"
                              for p, f in PHASE_RUNS])
def test_phases_match_oracle(q, orc, ps, form):
    """Independent phases in sequence: labels and per-phase results equal the
    oracle's, with each growth form."""
    import torch
    say("GPU generate_phases", ps.name, ps.dims, "form", form)
    params = [q.params_of(c, sweep_form=form) for c in ps.phases]
    labels, infos = q.generate_phases(ps.dims, params)
    torch.cuda.synchronize()
    ref, res = orc.generate_phases(ps.dims, _phase_tuples(ps))
    for info, r in zip(infos, res):
        assert (info["n_candidates"], info["n_seeds"], info["solid_count"], info["target_count"],
                info["front_size"], info["step"], info["status"]) == \
               (r.n_candidates, r.n_seeds, r.count, r.target_count, r.front_size, r.steps,
                r.status)
    assert np.array_equal(labels.cpu().numpy(), ref)


def test_phases_with_literal_front_match_oracle(q, orc):
    """A later phase under Algorithm 3's literal front rule on a walled grid (the sweep
    instance for both): labels and per-phase results equal the oracle's."""
    import torch
    ps = PHASES[0]
    tuples = [t + (k == 1,) for k, t in enumerate(_phase_tuples(ps))]
    params = [q.params_of(c, literal_front=(k == 1)) for k, c in enumerate(ps.phases)]
    say("GPU generate_phases (phase 2 literal front)", ps.name)
    labels, infos = q.generate_phases(ps.dims, params)
    torch.cuda.synchronize()
    ref, res = orc.generate_phases(ps.dims, tuples)
    for info, r in zip(infos, res):
        assert (info["solid_count"], info["step"], info["status"], info["front_size"]) == \
               (r.count, r.steps, r.status, r.front_size)
    assert np.array_equal(labels.cpu().numpy(), ref)


def test_one_phase_equals_generate(q):
    import torch
    case = workloads.small_cases()[0]
    say("GPU generate_phases (one phase) vs generate", case.name)
    labels, infos = q.generate_phases(case.dims, [q.params_of(case)])
    torch.cuda.synchronize()
    got = labels.cpu().numpy().copy()
    grid, info, _ = q.generate(case.dims, q.params_of(case))
    torch.cuda.synchronize()
    assert np.array_equal(got, grid.cpu().numpy())
    assert infos[0]["solid_count"] == info["solid_count"] and infos[0]["step"] == info["step"]


def test_phases_at_400_cube_properties(q):
    """The three-phase 400^3 medium (too large for the oracle): phase 1 equals the
    single-phase generation with its parameters; phases 1-2 are the same with and
    without phase 3; phase 3 takes only matrix cells; label counts equal the reported
    per-phase counts; every phase reports a terminal status."""
    import torch
    ps = workloads.phase_bench()
    params = [q.params_of(c) for c in ps.phases]
    say("GPU generate_phases", ps.name, "three phases")
    l3, i3 = q.generate_phases(ps.dims, params)
    torch.cuda.synchronize()
    a3 = l3.cpu().numpy().copy()
    del l3
    say("GPU generate_phases", ps.name, "two phases")
    l2, i2 = q.generate_phases(ps.dims, params[:2])
    torch.cuda.synchronize()
    a2 = l2.cpu().numpy().copy()
    del l2
    say("GPU generate", ps.name, "phase 1 alone")
    g1, info1, _ = q.generate(ps.dims, params[0])
    torch.cuda.synchronize()
    assert np.array_equal(a3 == 1, g1.cpu().numpy() == 1)
    assert info1["solid_count"] == i3[0]["solid_count"]
    assert np.array_equal(a3[a2 != 0], a2[a2 != 0])
    assert set(np.unique(a3[a2 == 0]).tolist()) <= {0, 3}
    counts = np.bincount(a3.ravel(), minlength=4)
    assert len(counts) == 4
    for k in range(3):
        assert counts[k + 1] == i3[k]["solid_count"]
        assert i3[k]["status"] in (q.DONE, q.EXHAUSTED)
        if k < 2:
            assert i3[k] == i2[k]


# ----- the literal Algorithm 3 front rule, prune(New_t) -----

LIT = workloads.small_cases()[::2] + workloads.config1()


# every case with the list-indexed sweep, one with the all-tiles sweep (the full-field
# form has no front and refuses the literal rule)
LIT_RUNS = [(c, 0) for c in LIT] + [(LIT[0], 2)]


@pytest.mark.parametrize("case,form", LIT_RUNS,
                         ids=[f"{c.name}-{['list', 'full_field', 'all_tiles'][f]}"
                              for c, f in LIT_RUNS])
def test_literal_front_matches_oracle(q, orc, case, form):
    import torch
    say("GPU generate (literal front)", case.name, case.dims, "form", form)
    params = q.params_of(case, sweep_form=form, literal_front=True)
    grid, info, buf = q.generate(case.dims, params)
    torch.cuda.synchronize()
    lf, ln, lc = q.qsgs_read_step_log(buf.ws, buf.ws_bytes)
    ld, lb = q.qsgs_read_step_work(buf.ws, buf.ws_bytes)
    ref = run_oracle(orc, case, literal_front=True)
    assert info["status"] == ref.status and info["step"] == ref.steps
    assert info["solid_count"] == ref.solid_count and info["front_size"] == ref.front_size
    assert np.array_equal(lf, ref.log_front) and np.array_equal(ln, ref.log_new)
    assert np.array_equal(lc, ref.log_count)
    assert np.array_equal(ld, ref.log_draws) and np.array_equal(lb, ref.log_blocks)
    assert np.array_equal(grid.cpu().numpy(), ref.grid)


def test_batch_mixes_front_rules(q, orc):
    """Realizations with either front rule in one batch: each equals its oracle run."""
    import torch
    cases = workloads.small_cases() + workloads.config1()
    lit = [k % 2 == 0 for k in range(len(cases))]
    params = [q.params_of(c, literal_front=f) for c, f in zip(cases, lit)]
    dims = [c.dims for c in cases]
    grids = [torch.empty(q.qsgs_grid_bytes(d), dtype=torch.uint8, device="cuda") for d in dims]
    wsb = q.qsgs_batch_workspace_bytes(dims, params)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    say("GPU generate_batch (mixed front rules) of", len(cases))
    st, infos = q.qsgs_generate_batch(dims, params, grids, ws, wsb)
    torch.cuda.synchronize()
    for c, f, g, info in zip(cases, lit, grids, infos):
        ref = run_oracle(orc, c, literal_front=f)
        nx, ny, nz = c.dims
        got = g[: nx * ny * nz].view(nz, ny, nx).cpu().numpy()
        assert info.status == ref.status and info.step == ref.steps, c.name
        assert info.solid_count == ref.solid_count and info.front_size == ref.front_size, c.name
        assert np.array_equal(got, ref.grid), c.name


def test_phases_at_the_label_limit(q, orc):
    """252 phases (the largest label) on a small grid: labels, counts and statuses equal
    the oracle's; the late phases find few free cells and exhaust."""
    import torch
    dims = (23, 19, 17)
    g = (0.05, 0.02, 0.005)
    tuples = [(0.004, 0.002, g, k % 4, 900 + k, 6) for k in range(252)]
    params = [q.make_params(*t[:5], max_steps=t[5]) for t in tuples]
    say("GPU generate_phases, 252 phases", dims)
    labels, infos = q.generate_phases(dims, params)
    torch.cuda.synchronize()
    ref, res = orc.generate_phases(dims, tuples)
    assert np.array_equal(labels.cpu().numpy(), ref)
    assert int(ref.max()) > 200
    for info, r in zip(infos, res):
        assert (info["solid_count"], info["step"], info["status"], info["n_seeds"]) == \
               (r.count, r.steps, r.status, r.n_seeds)


# ----- interacting phases (Sec. 2.1 step 4) -----

def _interaction(k, pairs):
    I = np.zeros((k, k, 3))
    for (n, m), v in pairs.items():
        I[n - 1, m - 1] = v
    return I


INTERACT_RUNS = [
    # (name, phase set, interaction {(n, m): (face, edge, corner)}, growth form)
    ("mp3_zero", PHASES[0], {}, 0),
    ("mp3_mixed", PHASES[0], {(2, 1): (0.3, 0.1, 0.05), (3, 1): (0.2, 0.0, 0.0),
                              (3, 2): (0.1, 0.1, 0.1)}, 0),
    ("mp3_mixed_all_tiles", PHASES[0], {(2, 1): (0.3, 0.1, 0.05), (3, 1): (0.2, 0.0, 0.0),
                                        (3, 2): (0.1, 0.1, 0.1)}, 2),
    ("mp2_ragged_strong", PHASES[1], {(2, 1): (0.6, 0.4, 0.2)}, 0),
    ("mp2_blocked_certain", PHASES[2], {(2, 1): (1.0, 1.0, 1.0)}, 0),
    ("mp2_cap_face_only", PHASES[4], {(2, 1): (1.0, 0.0, 0.0)}, 0),
]


@pytest.mark.parametrize("name,ps,pairs,form", INTERACT_RUNS, ids=[r[0] for r in INTERACT_RUNS])
def test_interacting_phases_match_oracle(q, orc, name, ps, pairs, form):
    """Phases that convert cells of earlier phases: labels and per-phase results equal
    the oracle's interacting generation."""
    import torch
    k = len(ps.phases)
    I = _interaction(k, pairs)
    say("GPU generate_phases_interacting", name, ps.dims, "form", form)
    params = [q.params_of(c, sweep_form=form) for c in ps.phases]
    labels, infos = q.generate_phases(ps.dims, params, interact=I)
    torch.cuda.synchronize()
    ref, res = orc.generate_phases(ps.dims, _phase_tuples(ps), I)
    for info, r in zip(infos, res):
        assert (info["n_candidates"], info["n_seeds"], info["solid_count"], info["target_count"],
                info["front_size"], info["step"], info["status"]) == \
               (r.n_candidates, r.n_seeds, r.count, r.target_count, r.front_size, r.steps,
                r.status), name
    assert np.array_equal(labels.cpu().numpy(), ref), name


def test_interacting_phase_with_literal_front_matches_oracle(q, orc):
    import torch
    ps = PHASES[0]
    I = _interaction(3, {(2, 1): (0.4, 0.2, 0.1), (3, 2): (0.3, 0.3, 0.3)})
    tuples = [t + (k == 2,) for k, t in enumerate(_phase_tuples(ps))]
    params = [q.params_of(c, literal_front=(k == 2)) for k, c in enumerate(ps.phases)]
    say("GPU generate_phases_interacting (phase 3 literal front)", ps.name)
    labels, infos = q.generate_phases(ps.dims, params, interact=I)
    torch.cuda.synchronize()
    ref, res = orc.generate_phases(ps.dims, tuples, I)
    for info, r in zip(infos, res):
        assert (info["solid_count"], info["step"], info["status"], info["front_size"]) == \
               (r.count, r.steps, r.status, r.front_size)
    assert np.array_equal(labels.cpu().numpy(), ref)
