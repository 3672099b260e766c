"""LIETS-QSGS porous-media generation on MI355X (gfx950).

A thin ctypes binding of ``libqsgs.so`` (C ABI in ``include/qsgs.h``): every function
below marshals arguments and calls the library of the same name.  Device memory and
streams come from torch (``torch.empty(..., device="cuda")`` and
``torch.cuda.current_stream()``); every step of the method runs in the HIP kernels.
There is no CPU fallback: using the package without the built library raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libqsgs.so")

OK, DONE, EXHAUSTED, MAXSTEPS = 0, 1, 2, 3
# growth forms of the whole-generation calls (qsgs_params.sweep_form)
SWEEP_LIST, SWEEP_FIELD, SWEEP_ALL_TILES = 0, 1, 2
ERR_INVALID, ERR_CAPACITY, ERR_WORKSPACE, ERR_DEVICE = -1, -2, -3, -4
STATUS_NAMES = {OK: "ok", DONE: "done", EXHAUSTED: "exhausted", MAXSTEPS: "max_steps",
                ERR_INVALID: "invalid", ERR_CAPACITY: "capacity", ERR_WORKSPACE: "workspace",
                ERR_DEVICE: "device"}


class QsgsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class qsgs_dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class qsgs_params(ctypes.Structure):
    _fields_ = [("solid_fraction", ctypes.c_double), ("seed_prob", ctypes.c_double),
                ("g_ref", ctypes.c_double * 3), ("spacing", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("key", ctypes.c_uint64),
                ("sweep_form", ctypes.c_int32), ("front_rule", ctypes.c_int32)]


class qsgs_info(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int64), ("n_seeds", ctypes.c_int64),
                ("solid_count", ctypes.c_int64), ("target_count", ctypes.c_int64),
                ("front_size", ctypes.c_int64), ("grown_last_step", ctypes.c_int64),
                ("step", ctypes.c_int32), ("status", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class qsgs_tuning(ctypes.Structure):
    _fields_ = [("grow_block", ctypes.c_int32), ("grow_grid", ctypes.c_int32),
                ("prune_block", ctypes.c_int32), ("prune_grid", ctypes.c_int32),
                ("seed_block", ctypes.c_int32), ("seed_grid", ctypes.c_int32),
                ("steps_per_sync", ctypes.c_int32), ("graphs", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


# Every symbol the header declares, with its ctypes signature.
_P = ctypes.POINTER
_VP, _SZ, _I64, _I32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64, ctypes.c_int32
SIGNATURES = {
    "qsgs_grid_bytes": (_SZ, [_P(qsgs_dims)]),
    "qsgs_workspace_bytes": (_SZ, [_P(qsgs_dims), _P(qsgs_params)]),
    "qsgs_step_workspace_bytes": (_SZ, []),
    "qsgs_seed": (ctypes.c_int, [_P(qsgs_dims), _P(qsgs_params), _VP, _VP, _I64, _VP, _SZ,
                                 _P(qsgs_info), _VP]),
    "qsgs_grow_step": (ctypes.c_int, [_P(qsgs_dims), _P(qsgs_params), _VP, _VP, _VP, _I64, _VP,
                                      _SZ, _P(qsgs_info), _VP]),
    "qsgs_generate": (ctypes.c_int, [_P(qsgs_dims), _P(qsgs_params), _VP, _VP, _SZ,
                                     _P(qsgs_info), _VP]),
    "qsgs_generate_noalloc": (ctypes.c_int, [_P(qsgs_dims), _P(qsgs_params), _VP,
                                             _P(qsgs_info), _VP]),
    "qsgs_batch_workspace_bytes": (_SZ, [_I32, _VP, _VP]),
    "qsgs_generate_batch": (ctypes.c_int, [_I32, _VP, _VP, _VP, _VP, _SZ, _VP, _VP]),
    "qsgs_phases_workspace_bytes": (_SZ, [_P(qsgs_dims), _I32, _VP]),
    "qsgs_generate_phases": (ctypes.c_int, [_P(qsgs_dims), _I32, _VP, _VP, _VP, _SZ, _VP,
                                            _VP]),
    "qsgs_generate_phases_interacting": (ctypes.c_int, [_P(qsgs_dims), _I32, _VP, _VP, _VP,
                                                        _VP, _SZ, _VP, _VP]),
    "qsgs_read_step_log": (_I64, [_VP, _SZ, _I32, _VP, _VP, _VP, _I64, _VP]),
    "qsgs_read_step_work": (_I64, [_VP, _SZ, _I32, _VP, _VP, _I64, _VP]),
    "qsgs_generate_async": (ctypes.c_int, [_P(qsgs_dims), _P(qsgs_params), _VP, _VP, _SZ,
                                           _VP, _VP]),
    "qsgs_generate_batch_async": (ctypes.c_int, [_I32, _VP, _VP, _VP, _VP, _SZ, _VP, _VP]),
    "qsgs_band_scratch_bytes": (_SZ, [_P(qsgs_dims)]),
    "qsgs_alu_scratch_bytes": (_SZ, [_I32]),
    "qsgs_alu_rate": (ctypes.c_int, [_I32, _VP, _SZ, _P(ctypes.c_double), _VP]),
    "qsgs_band_sizes": (ctypes.c_int, [_P(qsgs_dims), _VP, _VP, _VP, _SZ, _VP, _VP]),
    "qsgs_server_reserved_bytes": (_SZ, [_I32]),
    "qsgs_server_create": (ctypes.c_int, [_VP, _SZ, _I32, _I32, _VP, _P(_VP)]),
    "qsgs_server_submit": (ctypes.c_int, [_VP, _I64, _P(qsgs_dims), _P(qsgs_params)]),
    "qsgs_server_tick": (ctypes.c_int, [_VP, _P(_I32), _P(_I32), _P(_I32)]),
    "qsgs_server_ready": (_I32, [_VP, _VP, _VP, _I32]),
    "qsgs_server_take": (ctypes.c_int, [_VP, _I64, _VP, _SZ, _I32]),
    "qsgs_server_free_bytes": (_SZ, [_VP]),
    "qsgs_server_destroy": (None, [_VP]),
    "qsgs_set_tuning": (ctypes.c_int, [_P(qsgs_tuning)]),
    "qsgs_get_tuning": (None, [_P(qsgs_tuning)]),
    "qsgs_profile_enable": (None, [_I32]),
    "qsgs_profile_read": (None, [_VP, _I32]),
    "qsgs_last_error": (ctypes.c_char_p, []),
    "qsgs_version": (ctypes.c_char_p, []),
    "qsgs_seed_prob_from_grain": (ctypes.c_double, [ctypes.c_double, ctypes.c_double,
                                                    ctypes.c_double]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libqsgs.so (built by ``__graft_entry__.build()``); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


# ----- argument marshalling helpers -----

def make_dims(dims) -> qsgs_dims:
    if isinstance(dims, qsgs_dims):
        return dims
    nx, ny, nz = (int(v) for v in dims)
    return qsgs_dims(nx, ny, nz)


def make_params(solid_fraction: float, seed_prob: float, g_ref, spacing: int, key: int,
                max_steps: int = 0, sweep_form: int = SWEEP_LIST,
                literal_front: bool = False) -> qsgs_params:
    """``sweep_form``: SWEEP_LIST (the list-indexed sweep), SWEEP_FIELD (full-field steps,
    Algorithm 2) or SWEEP_ALL_TILES; ``literal_front``: Algorithm 3's front rule
    prune(New_t) instead of the interface."""
    g = (ctypes.c_double * 3)(*[float(v) for v in g_ref])
    return qsgs_params(float(solid_fraction), float(seed_prob), g, int(spacing), int(max_steps),
                       int(key) & 0xFFFFFFFFFFFFFFFF, int(sweep_form),
                       1 if literal_front else 0)


def params_of(case, sweep_form: int = SWEEP_LIST, literal_front: bool = False) -> qsgs_params:
    return make_params(case.solid_fraction, case.seed_prob, case.g_ref, case.spacing, case.key,
                       case.max_steps, sweep_form, literal_front)


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(status: int) -> int:
    if status < 0:
        raise QsgsError(status, qsgs_last_error())
    return status


# ----- the C ABI, one function each -----

def qsgs_grid_bytes(dims) -> int:
    return int(load().qsgs_grid_bytes(ctypes.byref(make_dims(dims))))


def qsgs_workspace_bytes(dims, params: qsgs_params) -> int:
    return int(load().qsgs_workspace_bytes(ctypes.byref(make_dims(dims)), ctypes.byref(params)))


def qsgs_step_workspace_bytes() -> int:
    return int(load().qsgs_step_workspace_bytes())


def qsgs_seed(dims, params, grid, front, front_cap: int, ws, ws_bytes: int,
              info: qsgs_info | None = None, stream=None) -> tuple[int, qsgs_info]:
    info = info if info is not None else qsgs_info()
    st = load().qsgs_seed(ctypes.byref(make_dims(dims)), ctypes.byref(params), _ptr(grid),
                          _ptr(front), int(front_cap), _ptr(ws), int(ws_bytes),
                          ctypes.byref(info), _stream(stream))
    return _check(st), info


def qsgs_grow_step(dims, params, grid, front_in, front_out, front_cap: int, ws, ws_bytes: int,
                   info: qsgs_info, stream=None) -> tuple[int, qsgs_info]:
    st = load().qsgs_grow_step(ctypes.byref(make_dims(dims)), ctypes.byref(params), _ptr(grid),
                               _ptr(front_in), _ptr(front_out), int(front_cap), _ptr(ws),
                               int(ws_bytes), ctypes.byref(info), _stream(stream))
    return _check(st), info


def qsgs_generate(dims, params, grid, ws, ws_bytes: int, info: qsgs_info | None = None,
                  stream=None) -> tuple[int, qsgs_info]:
    info = info if info is not None else qsgs_info()
    st = load().qsgs_generate(ctypes.byref(make_dims(dims)), ctypes.byref(params), _ptr(grid),
                              _ptr(ws), int(ws_bytes), ctypes.byref(info), _stream(stream))
    return _check(st), info


def qsgs_generate_noalloc(dims, params, grid, info: qsgs_info | None = None,
                          stream=None) -> tuple[int, qsgs_info]:
    """Whole generation in the library's own scratch (no workspace argument)."""
    info = info if info is not None else qsgs_info()
    st = load().qsgs_generate_noalloc(ctypes.byref(make_dims(dims)), ctypes.byref(params),
                                      _ptr(grid), ctypes.byref(info), _stream(stream))
    return _check(st), info


def qsgs_read_step_log(ws, ws_bytes: int, index: int = 0, max_entries: int = 65536,
                       stream=None):
    import numpy as np
    front = np.zeros(max_entries, np.int64)
    grown = np.zeros(max_entries, np.int64)
    count = np.zeros(max_entries, np.int64)
    n = load().qsgs_read_step_log(_ptr(ws), int(ws_bytes), int(index), front.ctypes.data,
                                  grown.ctypes.data, count.ctypes.data, int(max_entries),
                                  _stream(stream))
    n = _check(int(n))
    return front[:n].copy(), grown[:n].copy(), count[:n].copy()


def qsgs_read_step_work(ws, ws_bytes: int, index: int = 0, max_entries: int = 65536,
                        stream=None):
    """Per-step (draws, Philox high blocks) of a generation's growth sweep."""
    import numpy as np
    draws = np.zeros(max_entries, np.int64)
    blocks = np.zeros(max_entries, np.int64)
    n = load().qsgs_read_step_work(_ptr(ws), int(ws_bytes), int(index), draws.ctypes.data,
                                   blocks.ctypes.data, int(max_entries), _stream(stream))
    n = _check(int(n))
    return draws[:n].copy(), blocks[:n].copy()


INFO_BYTES = ctypes.sizeof(qsgs_info)


def qsgs_generate_async(dims, params: qsgs_params, grid, ws, ws_bytes: int, d_info,
                        stream=None) -> None:
    """Enqueues a whole generation without host synchronisation; d_info is a device
    buffer of at least INFO_BYTES bytes (read it with info_from_device)."""
    _check(load().qsgs_generate_async(ctypes.byref(make_dims(dims)), ctypes.byref(params),
                                      _ptr(grid), _ptr(ws), int(ws_bytes), _ptr(d_info),
                                      _stream(stream)))


def qsgs_generate_batch_async(dims_list, params_list, grids, ws, ws_bytes: int, d_infos,
                              stream=None) -> None:
    n = len(dims_list)
    d = (qsgs_dims * n)(*[make_dims(x) for x in dims_list])
    p = (qsgs_params * n)(*params_list)
    g = (ctypes.c_void_p * n)(*[_ptr(x) for x in grids])
    _check(load().qsgs_generate_batch_async(n, d, p, g, _ptr(ws), int(ws_bytes), _ptr(d_infos),
                                            _stream(stream)))


def info_from_device(d_info, index: int = 0) -> qsgs_info:
    """The qsgs_info at `index` of a device buffer written by the async calls (copies it
    to the host; the caller synchronises first)."""
    raw = bytes(d_info[index * INFO_BYTES:(index + 1) * INFO_BYTES].cpu().numpy().tobytes())
    return qsgs_info.from_buffer_copy(raw)


def qsgs_alu_rate(waves_per_simd: int = 8, stream=None) -> float:
    """32-bit vector ALU lane operations per second measured on the current device."""
    import torch
    n = int(load().qsgs_alu_scratch_bytes(int(waves_per_simd)))
    if n == 0:
        raise QsgsError(ERR_INVALID, "waves_per_simd must be in [1, 8]")
    scratch = torch.empty(n, dtype=torch.uint8, device="cuda")
    out = ctypes.c_double()
    _check(load().qsgs_alu_rate(int(waves_per_simd), _ptr(scratch), n, ctypes.byref(out),
                                _stream(stream)))
    return out.value


def qsgs_band_scratch_bytes(dims) -> int:
    return int(load().qsgs_band_scratch_bytes(ctypes.byref(make_dims(dims))))


def qsgs_band_sizes(dims, before, after, scratch, scratch_bytes: int, stream=None):
    """(|band(F_t)|, |band(F_t u New_t)|) of the step that took grid `before` to `after`."""
    out = (ctypes.c_uint64 * 2)()
    _check(load().qsgs_band_sizes(ctypes.byref(make_dims(dims)), _ptr(before), _ptr(after),
                                  _ptr(scratch), int(scratch_bytes), out, _stream(stream)))
    return int(out[0]), int(out[1])


def qsgs_batch_workspace_bytes(dims_list, params_list) -> int:
    n = len(dims_list)
    d = (qsgs_dims * n)(*[make_dims(x) for x in dims_list])
    p = (qsgs_params * n)(*params_list)
    return int(load().qsgs_batch_workspace_bytes(n, d, p))


def qsgs_generate_batch(dims_list, params_list, grids, ws, ws_bytes: int, stream=None):
    """Batched generation; returns (status, list of qsgs_info)."""
    n = len(dims_list)
    d = (qsgs_dims * n)(*[make_dims(x) for x in dims_list])
    p = (qsgs_params * n)(*params_list)
    g = (ctypes.c_void_p * n)(*[_ptr(x) for x in grids])
    infos = (qsgs_info * n)()
    st = load().qsgs_generate_batch(n, d, p, g, _ptr(ws), int(ws_bytes), infos, _stream(stream))
    return _check(st), list(infos)


def qsgs_phases_workspace_bytes(dims, phases) -> int:
    n = len(phases)
    p = (qsgs_params * n)(*phases)
    return int(load().qsgs_phases_workspace_bytes(ctypes.byref(make_dims(dims)), n, p))


def qsgs_generate_phases(dims, phases, labels, ws, ws_bytes: int, stream=None):
    """Multi-phase generation; returns (status, list of qsgs_info, one per phase)."""
    n = len(phases)
    p = (qsgs_params * n)(*phases)
    infos = (qsgs_info * n)()
    st = load().qsgs_generate_phases(ctypes.byref(make_dims(dims)), n, p, _ptr(labels),
                                     _ptr(ws), int(ws_bytes), infos, _stream(stream))
    return _check(st), list(infos)


def qsgs_generate_phases_interacting(dims, phases, interact, labels, ws, ws_bytes: int,
                                     stream=None):
    """Multi-phase generation with interacting phases; ``interact`` is None or an array
    [n_phases, n_phases, 3] of I_c^{n,m} (index [n - 1, m - 1, c], read for m < n).
    Returns (status, list of qsgs_info, one per phase)."""
    import numpy as np
    n = len(phases)
    p = (qsgs_params * n)(*phases)
    infos = (qsgs_info * n)()
    I = None
    if interact is not None:
        I = np.ascontiguousarray(interact, dtype=np.float64)
        if I.shape != (n, n, 3):
            raise QsgsError(ERR_INVALID, f"interact must have shape ({n}, {n}, 3)")
    st = load().qsgs_generate_phases_interacting(
        ctypes.byref(make_dims(dims)), n, p, None if I is None else I.ctypes.data, _ptr(labels),
        _ptr(ws), int(ws_bytes), infos, _stream(stream))
    return _check(st), list(infos)


def qsgs_server_reserved_bytes(max_slots: int) -> int:
    return int(load().qsgs_server_reserved_bytes(int(max_slots)))


def qsgs_server_create(arena, arena_bytes: int, max_slots: int, steps_per_tick: int = 1,
                       stream=None) -> int:
    h = ctypes.c_void_p()
    _check(load().qsgs_server_create(_ptr(arena), int(arena_bytes), int(max_slots),
                                     int(steps_per_tick), _stream(stream), ctypes.byref(h)))
    return h.value


def qsgs_server_submit(server: int, request_id: int, dims, params: qsgs_params) -> None:
    _check(load().qsgs_server_submit(server, int(request_id), ctypes.byref(make_dims(dims)),
                                     ctypes.byref(params)))


def qsgs_server_tick(server: int) -> tuple[int, int, int]:
    """(resident, queued, ready).  A tick that retired a failed request raises
    QsgsError(ERR_DEVICE) with the counts in ``.counts``; the server stays usable."""
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    try:
        _check(load().qsgs_server_tick(server, ctypes.byref(a), ctypes.byref(b),
                                       ctypes.byref(c)))
    except QsgsError as e:
        e.counts = (a.value, b.value, c.value)
        raise
    return a.value, b.value, c.value


def qsgs_server_ready(server: int, max_n: int = 4096):
    ids = (ctypes.c_int64 * max_n)()
    infos = (qsgs_info * max_n)()
    n = load().qsgs_server_ready(server, ids, infos, int(max_n))
    return [(ids[k], infos[k]) for k in range(n)]


def qsgs_server_take(server: int, request_id: int, dst=None, dst_bytes: int = 0,
                     dst_on_host: bool = False, check: bool = True) -> int:
    """Copies out (or drops, dst=None) a finished request's grid; returns the status
    (raises on an error unless check=False, e.g. to drop a failed request)."""
    if dst is not None and hasattr(dst, "ctypes"):  # numpy array on the host
        ptr, dst_on_host, dst_bytes = dst.ctypes.data, True, dst.nbytes
    else:
        ptr = _ptr(dst)
    st = load().qsgs_server_take(server, int(request_id), ptr, int(dst_bytes),
                                 1 if dst_on_host else 0)
    return _check(st) if check else st


def qsgs_server_free_bytes(server: int) -> int:
    return int(load().qsgs_server_free_bytes(server))


def qsgs_server_destroy(server: int) -> None:
    load().qsgs_server_destroy(server)


def qsgs_set_tuning(tuning: qsgs_tuning | dict | None) -> None:
    if isinstance(tuning, dict):
        tuning = qsgs_tuning(**{"graphs": 1, **tuning})
    _check(load().qsgs_set_tuning(ctypes.byref(tuning) if tuning is not None else None))


def qsgs_get_tuning() -> qsgs_tuning:
    t = qsgs_tuning()
    load().qsgs_get_tuning(ctypes.byref(t))
    return t


def qsgs_profile_enable(enable: bool) -> None:
    load().qsgs_profile_enable(1 if enable else 0)


def qsgs_profile_read(reset: bool = False) -> dict:
    out = (ctypes.c_double * 5)()
    load().qsgs_profile_read(out, 1 if reset else 0)
    return {"grow_launches": out[0], "grow_ms": out[1], "prune_launches": out[2],
            "prune_ms": out[3], "seed_ms": out[4]}


def qsgs_last_error() -> str:
    return load().qsgs_last_error().decode()


def qsgs_seed_prob_from_grain(solid_fraction: float, grain_diameter: float,
                              voxel_size: float) -> float:
    """S_d = 6 phi_s delta^3 / (pi d^3) (Sec. 3.3); raises on invalid arguments."""
    v = float(load().qsgs_seed_prob_from_grain(float(solid_fraction), float(grain_diameter),
                                               float(voxel_size)))
    if v < 0:
        raise QsgsError(ERR_INVALID, "solid_fraction in [0, 1], grain and voxel size > 0")
    return v


def qsgs_version() -> str:
    return load().qsgs_version().decode()


# ----- convenience: torch-allocated buffers -----

@dataclass
class Buffers:
    """Device buffers for one grid size; reused across calls of the same size."""
    dims: tuple
    grid: object
    ws: object
    ws_bytes: int
    extra: dict = field(default_factory=dict)

    def view(self):
        nx, ny, nz = self.dims
        return self.grid[: nx * ny * nz].view(nz, ny, nx)


def alloc(dims, params: qsgs_params, device: str = "cuda") -> Buffers:
    import torch
    dims = tuple(int(v) for v in dims)
    gb = qsgs_grid_bytes(dims)
    wb = qsgs_workspace_bytes(dims, params)
    if gb == 0 or wb == 0:
        raise QsgsError(ERR_INVALID, qsgs_last_error() or "invalid dims or params")
    grid = torch.empty(gb, dtype=torch.uint8, device=device)
    ws = torch.empty(wb, dtype=torch.uint8, device=device)
    return Buffers(dims, grid, ws, wb)


def generate(dims, params: qsgs_params, buffers: Buffers | None = None, stream=None):
    """Run qsgs_generate; returns (grid view [nz, ny, nx] uint8 on the device, info dict)."""
    if buffers is None or buffers.ws_bytes < qsgs_workspace_bytes(dims, params):
        buffers = alloc(dims, params)
    st, info = qsgs_generate(dims, params, buffers.grid, buffers.ws, buffers.ws_bytes,
                             stream=stream)
    d = info.as_dict()
    d["status_name"] = STATUS_NAMES[st]
    return buffers.view(), d, buffers


def generate_phases(dims, phases, stream=None, device: str = "cuda", interact=None):
    """Run qsgs_generate_phases (or, with ``interact``, qsgs_generate_phases_interacting);
    returns (label grid view [nz, ny, nx] uint8 on the device: n for phase n, 0 for the
    matrix; list of per-phase info dicts)."""
    import torch
    dims = tuple(int(v) for v in dims)
    gb = qsgs_grid_bytes(dims)
    wb = qsgs_phases_workspace_bytes(dims, phases)
    if gb == 0 or wb == 0:
        raise QsgsError(ERR_INVALID, qsgs_last_error() or "invalid dims or phases")
    labels = torch.empty(gb, dtype=torch.uint8, device=device)
    ws = torch.empty(wb, dtype=torch.uint8, device=device)
    if interact is None:
        _, infos = qsgs_generate_phases(dims, phases, labels, ws, wb, stream=stream)
    else:
        _, infos = qsgs_generate_phases_interacting(dims, phases, interact, labels, ws, wb,
                                                    stream=stream)
    out = []
    for info in infos:
        d = info.as_dict()
        d["status_name"] = STATUS_NAMES[d["status"]]
        out.append(d)
    nx, ny, nz = dims
    return labels[: nx * ny * nz].view(nz, ny, nx), out
