// qsgs_api.hip -- host side of libqsgs: seeding, single steps, whole generations and
// batches (C ABI in include/qsgs.h), all driven through the shared Engine.
#include <array>

#include "qsgs_host.h"

using namespace qsgs;
using namespace qsgs::host;

namespace {

constexpr size_t kStepWorkspace = 1024 * 1024;

// Workspace of qsgs_generate / qsgs_generate_batch: the persistent part, the sweep
// state (tile lists and stamps) of every realization, then the seeding scratch of
// the whole batch.
struct GenLayout {
  PersistLayout P;
  std::vector<size_t> sweep;
  size_t itab = 0;  // multi-phase grids: the interaction table of the growing phase
  size_t seed = 0, total = 0;
  SeedLayout S;
};

GenLayout gen_layout(const std::vector<Spec>& specs, bool with_sweep, bool walls = false) {
  GenLayout G;
  G.P = persist_layout(specs.size(), specs.size() == 1 ? kLogCapSingle : kLogCapBatch);
  size_t off = G.P.total;
  if (with_sweep) {
    for (const Spec& s : specs) {
      G.sweep.push_back(off);
      off = align_up(off + sweep_state_bytes(s.g, walls));
    }
  }
  if (walls) {
    G.itab = off;
    off = align_up(off + sizeof(InteractTable));
  }
  G.seed = off;
  G.S = seed_layout(specs, true);
  G.total = off + G.S.total;
  return G;
}

qsgs_status make_specs(int32_t count, const qsgs_dims* dims, const qsgs_params* params,
                       uint8_t* const* grids, std::vector<Spec>* specs) {
  if (count < 1 || (uint32_t)count > kMaxBatch)
    return fail(QSGS_ERR_INVALID, "count must be in [1, %u]", kMaxBatch);
  if (!dims || !params || !grids) return fail(QSGS_ERR_INVALID, "NULL array argument");
  specs->resize((size_t)count);
  for (int32_t r = 0; r < count; ++r) {
    QSGS_TRY(check_dims(&dims[r], &(*specs)[r].g));
    QSGS_TRY(check_params(&params[r]));
    QSGS_TRY(check_grid(grids[r]));
    (*specs)[r].bk = make_buckets((*specs)[r].g, params[r].spacing);
  }
  return QSGS_OK;
}

// no_alloc: the call may not allocate (the allocation-free entry point): transfers go
// through pageable host memory instead of the pinned staging buffer, and no timing
// events are recorded.
// itab (walls only, may be null): the interaction table of the phase being grown, with
// ihi_max[c] the largest high half of its thresholds per class.
// async: the call never synchronises with the host (graph capture): infos is device
// memory, written by the last kernel; every params[r].max_steps is in [1, 4096] and the
// loop runs max(max_steps) + 1 passes.
qsgs_status generate_impl(int32_t count, const qsgs_dims* dims, const qsgs_params* params,
                          uint8_t* const* grids, void* ws, size_t ws_bytes, qsgs_info* infos,
                          hipStream_t s, bool walls = false, bool no_alloc = false,
                          const InteractTable* itab = nullptr,
                          const uint32_t* ihi_max = nullptr, bool async = false) {
  std::vector<Spec> specs;
  QSGS_TRY(make_specs(count, dims, params, grids, &specs));
  if (!ws || !infos) return fail(QSGS_ERR_INVALID, "d_ws and info must not be NULL");
  int32_t steps_cap = 0;
  if (async) {
    for (int32_t r = 0; r < count; ++r) {
      if (params[r].max_steps < 1 || params[r].max_steps > kMaxAsyncSteps)
        return fail(QSGS_ERR_INVALID, "the calls without host synchronisation need max_steps "
                                      "in [1, %d] (realization %d has %d)",
                    kMaxAsyncSteps, r, params[r].max_steps);
      steps_cap = std::max(steps_cap, params[r].max_steps);
    }
    if (((uintptr_t)infos & 7u) != 0) return fail(QSGS_ERR_INVALID, "d_info not 8-byte aligned");
  }
  const GenLayout G = gen_layout(specs, true, walls);
  if (ws_bytes < G.total)
    return fail(QSGS_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", G.total, ws_bytes);
  Engine E;
  E.bind(ws, G.P, (size_t)count, s, walls, count == 1 ? 2u * kBlock : 0u);
  E.no_events = no_alloc || async;
  E.async = async;
  E.stage = (no_alloc || async) ? nullptr
                                : thread_pinned_stage(Engine::stage_bytes((size_t)count));
  std::vector<size_t> group;
  for (int32_t r = 0; r < count; ++r) {
    E.init_sweep_record((size_t)r, specs[r], &params[r], grids[r], at<void>(ws, G.sweep[r]),
                        walls);
    group.push_back((size_t)r);
  }
  if (walls && itab) {
    InteractTable* d_itab = at<InteractTable>(ws, G.itab);
    QSGS_HIP(hipMemcpyAsync(d_itab, itab, sizeof(InteractTable), hipMemcpyHostToDevice, s));
    for (int32_t r = 0; r < count; ++r) {
      E.reals[r].itab = d_itab;
      for (int c = 0; c < 3; ++c) E.reals[r].ihi_max[c] = ihi_max[c];
    }
  }
  E.attach_scratch(group, at<void>(ws, G.seed), G.S);
  const bool profiling = prof_on() && !no_alloc && !async;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (profiling) {
    prof_release_all();
    e0 = prof_event();
    e1 = prof_event();
    QSGS_HIP(hipEventRecord(e0, s));
  }
  QSGS_TRY(E.upload_header());
  QSGS_TRY(E.upload_control());
  QSGS_TRY(E.upload(0, E.reals.size()));
  QSGS_TRY(E.seed_core(at<void>(ws, G.seed), G.S));
  QSGS_TRY(E.sweep_start(group));
  if (async) {
    QSGS_TRY(E.run_sweep_fixed((uint32_t)steps_cap + 1u));
    QSGS_TRY(E.export_grids());
    hipLaunchKernelGGL(k_info_out, dim3((count + 255) / 256), dim3(256), 0, s, E.args, infos);
    QSGS_LAUNCHED("k_info_out");
    return QSGS_OK;
  }
  if (profiling) QSGS_HIP(hipEventRecord(e1, s));
  QSGS_TRY(E.run_sweep_loop());
  QSGS_TRY(E.export_grids());
  std::vector<Real> fin;
  QSGS_TRY(E.read_all(&fin));
  if (profiling) {
    float ms = 0.f;
    QSGS_HIP(hipEventElapsedTime(&ms, e0, e1));
    std::lock_guard<std::mutex> lk(prof().mu);
    prof().seed_ms += ms;
  }
  int32_t worst = QSGS_OK;
  for (int32_t r = 0; r < count; ++r) {
    const Ctl& c = fin[r].ctl;
    if (c.status == kStatusOverflow || c.bad_entry)
      return fail(QSGS_ERR_DEVICE, "internal front overflow in realization %d", r);
    fill_info(c, &infos[r]);
    worst = std::max(worst, c.status);
  }
  return (qsgs_status)worst;
}

// Scratch of the allocation-free entry point: the generation workspace of one call,
// held in device memory by the code object (each device that runs the library holds its
// own copy until the process ends).  Host code never passes `scratch` itself to a kernel
// or a copy (in host code the name is a stand-in, not a device address): it uses the
// device address hipGetSymbolAddress returns, taken once per device.
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;

struct NoAllocDevice {
  std::mutex mu;   // serialises the calls that share this device's scratch
  void* ptr = nullptr;
};

NoAllocDevice* no_alloc_devices() {
  static NoAllocDevice d[kMaxDevices];
  return d;
}

}  // namespace

extern "C" {

qsgs_status qsgs_generate_noalloc(const qsgs_dims* dims, const qsgs_params* params,
                                  uint8_t* d_grid, qsgs_info* info, void* stream) {
  last_error().clear();
  std::vector<Spec> specs;
  QSGS_TRY(make_specs(1, dims, params, &d_grid, &specs));
  if (!info) return fail(QSGS_ERR_INVALID, "info must not be NULL");
  const size_t need = gen_layout(specs, true).total;
  if (need > kNoAllocScratchBytes)
    return fail(QSGS_ERR_WORKSPACE,
                "qsgs_generate_noalloc: this grid needs %zu bytes of scratch, more than the "
                "%zu it holds; use qsgs_generate with a workspace of "
                "qsgs_workspace_bytes() bytes",
                need, kNoAllocScratchBytes);
  int dev = 0;
  QSGS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(QSGS_ERR_DEVICE, "device %d outside [0, %d)", dev, kMaxDevices);
  NoAllocDevice& D = no_alloc_devices()[dev];
  std::lock_guard<std::mutex> lk(D.mu);
  if (!D.ptr) {  // first call on this device (it is current): the array's device address
    void* p = nullptr;
    QSGS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(QSGS_ERR_DEVICE, "hipGetSymbolAddress returned NULL for the scratch");
    D.ptr = p;
  }
  return generate_impl(1, dims, params, &d_grid, D.ptr, kNoAllocScratchBytes, info,
                       (hipStream_t)stream, false, true);
}

size_t qsgs_grid_bytes(const qsgs_dims* dims) {
  Geometry g{};
  if (check_dims(dims, &g) != QSGS_OK) return 0;
  return grid_bytes(g);
}

size_t qsgs_batch_workspace_bytes(int32_t count, const qsgs_dims* dims,
                                  const qsgs_params* params) {
  if (count < 1 || !dims || !params) return 0;
  std::vector<Spec> specs((size_t)count);
  for (int32_t r = 0; r < count; ++r) {
    if (check_dims(&dims[r], &specs[r].g) != QSGS_OK || check_params(&params[r]) != QSGS_OK)
      return 0;
    specs[r].bk = make_buckets(specs[r].g, params[r].spacing);
  }
  return gen_layout(specs, true).total;
}

size_t qsgs_workspace_bytes(const qsgs_dims* dims, const qsgs_params* params) {
  return qsgs_batch_workspace_bytes(1, dims, params);
}

size_t qsgs_step_workspace_bytes(void) { return kStepWorkspace; }

qsgs_status qsgs_seed(const qsgs_dims* dims, const qsgs_params* params, uint8_t* d_grid,
                      int32_t* d_front, int64_t front_cap, void* d_ws, size_t ws_bytes,
                      qsgs_info* info, void* stream) {
  last_error().clear();
  if (!d_front || front_cap < 0) return fail(QSGS_ERR_INVALID, "bad d_front / front_cap");
  std::vector<Spec> specs;
  QSGS_TRY(make_specs(1, dims, params, &d_grid, &specs));
  if (!d_ws || !info) return fail(QSGS_ERR_INVALID, "d_ws and info must not be NULL");
  const GenLayout G = gen_layout(specs, false);
  if (ws_bytes < G.total)
    return fail(QSGS_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", G.total, ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  Engine E;
  E.bind(d_ws, G.P, 1, s);
  E.stage = thread_pinned_stage(Engine::stage_bytes(1));
  E.init_record(0, specs[0], params, d_grid, d_front, nullptr,
                (uint32_t)std::min<int64_t>(front_cap, (int64_t)UINT32_MAX));
  E.attach_scratch({0}, at<void>(d_ws, G.seed), G.S);
  QSGS_TRY(E.upload_header());
  QSGS_TRY(E.upload(0, 1));
  QSGS_TRY(E.seed_core(at<void>(d_ws, G.seed), G.S));
  QSGS_TRY(E.seed_fronts());
  Ctl h{};
  QSGS_TRY(E.read_ctl(0, &h));
  if (h.status == kStatusOverflow)
    return fail(QSGS_ERR_CAPACITY, "initial front needs more than front_cap = %lld entries",
                (long long)front_cap);
  fill_info(h, info);
  return QSGS_OK;
}

qsgs_status qsgs_grow_step(const qsgs_dims* dims, const qsgs_params* params, uint8_t* d_grid,
                           int32_t* d_front_in, int32_t* d_front_out, int64_t front_cap,
                           void* d_ws, size_t ws_bytes, qsgs_info* info, void* stream) {
  last_error().clear();
  Geometry g{};
  QSGS_TRY(check_dims(dims, &g));
  QSGS_TRY(check_params(params));
  if (params->front_rule != 0)
    return fail(QSGS_ERR_INVALID, "front_rule 1 is for the whole-generation calls");
  QSGS_TRY(check_grid(d_grid));
  if (!d_front_in || !d_front_out || d_front_in == d_front_out || front_cap < 0)
    return fail(QSGS_ERR_INVALID, "bad front buffers / front_cap");
  if (!d_ws || !info) return fail(QSGS_ERR_INVALID, "d_ws and info must not be NULL");
  const PersistLayout P = persist_layout(1, 0);
  if (ws_bytes < kStepWorkspace || P.total > kStepWorkspace)
    return fail(QSGS_ERR_WORKSPACE, "step workspace needs %zu bytes, got %zu", kStepWorkspace,
                ws_bytes);
  if (info->front_size < 0 || info->front_size > front_cap || info->solid_count < 0 ||
      info->solid_count > (int64_t)g.n || info->step < 0)
    return fail(QSGS_ERR_INVALID, "info does not describe a valid state");
  if (info->status >= QSGS_DONE && info->status <= QSGS_MAXSTEPS) return (qsgs_status)info->status;
  hipStream_t s = (hipStream_t)stream;
  Engine E;
  E.bind(d_ws, P, 1, s);
  E.stage = thread_pinned_stage(Engine::stage_bytes(1));
  E.init_record(0, Spec{g, Buckets{}}, params, d_grid, d_front_in, d_front_out,
                (uint32_t)std::min<int64_t>(front_cap, (int64_t)UINT32_MAX));
  Real& R = E.reals[0];
  R.phase = kPhaseGrow;
  R.ctl.cnt = (uint64_t)info->solid_count;
  R.ctl.front_size = (uint32_t)info->front_size;
  R.ctl.step = info->step;
  R.ctl.n_cand = (uint32_t)info->n_candidates;
  R.ctl.n_seeds = (uint32_t)info->n_seeds;
  QSGS_TRY(E.upload(0, 1));
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, E.args, 0u);
  QSGS_LAUNCHED("k_ctl_init");
  hipLaunchKernelGGL(k_loop_resume, dim3(1), dim3(1), 0, s, E.args);
  QSGS_LAUNCHED("k_loop_resume");
  QSGS_TRY(E.step(nullptr));
  Ctl h{};
  QSGS_TRY(E.read_ctl(0, &h));
  if (h.bad_entry) return fail(QSGS_ERR_INVALID, "front entry outside the grid");
  if (h.status == kStatusOverflow) {
    hipLaunchKernelGGL(k_rollback, dim3(2048), dim3(kBlock), 0, s, d_grid, g.n);
    QSGS_LAUNCHED("k_rollback");
    QSGS_HIP(hipStreamSynchronize(s));
    return fail(QSGS_ERR_CAPACITY, "front would exceed front_cap = %lld entries",
                (long long)front_cap);
  }
  fill_info(h, info);
  return (qsgs_status)h.status;
}

qsgs_status qsgs_generate(const qsgs_dims* dims, const qsgs_params* params, uint8_t* d_grid,
                          void* d_ws, size_t ws_bytes, qsgs_info* info, void* stream) {
  last_error().clear();
  return generate_impl(1, dims, params, &d_grid, d_ws, ws_bytes, info, (hipStream_t)stream);
}

qsgs_status qsgs_generate_async(const qsgs_dims* dims, const qsgs_params* params,
                                uint8_t* d_grid, void* d_ws, size_t ws_bytes, qsgs_info* d_info,
                                void* stream) {
  last_error().clear();
  return generate_impl(1, dims, params, &d_grid, d_ws, ws_bytes, d_info, (hipStream_t)stream,
                       false, false, nullptr, nullptr, true);
}

qsgs_status qsgs_generate_batch_async(int32_t count, const qsgs_dims* dims,
                                      const qsgs_params* params, uint8_t* const* d_grids,
                                      void* d_ws, size_t ws_bytes, qsgs_info* d_infos,
                                      void* stream) {
  last_error().clear();
  return generate_impl(count, dims, params, d_grids, d_ws, ws_bytes, d_infos,
                       (hipStream_t)stream, false, false, nullptr, nullptr, true);
}

qsgs_status qsgs_generate_batch(int32_t count, const qsgs_dims* dims, const qsgs_params* params,
                                uint8_t* const* d_grids, void* d_ws, size_t ws_bytes,
                                qsgs_info* infos, void* stream) {
  last_error().clear();
  return generate_impl(count, dims, params, d_grids, d_ws, ws_bytes, infos, (hipStream_t)stream);
}

// Multi-phase generation: phases grown in sequence on one label grid.  While phase k
// grows, its cells are 1 (and the step marks 2 / 3), unassigned cells 0 and the cells of
// phase m < k the value 3 + m, which the seeding and the sweep treat as walls.
constexpr int32_t kMaxPhases = 252;
constexpr uint32_t kWallBase = 3;

size_t qsgs_phases_workspace_bytes(const qsgs_dims* dims, int32_t n_phases,
                                   const qsgs_params* phases) {
  if (!dims || !phases || n_phases < 1 || n_phases > kMaxPhases) return 0;
  Geometry g{};
  if (check_dims(dims, &g) != QSGS_OK) return 0;
  size_t m = 0;
  for (int32_t k = 0; k < n_phases; ++k) {  // one phase at a time, with the walls plane
    if (check_params(&phases[k]) != QSGS_OK) return 0;
    m = std::max(m, gen_layout({Spec{g, make_buckets(g, phases[k].spacing)}}, true, true).total);
  }
  return m;
}

qsgs_status qsgs_generate_phases(const qsgs_dims* dims, int32_t n_phases,
                                 const qsgs_params* phases, uint8_t* d_labels, void* d_ws,
                                 size_t ws_bytes, qsgs_info* infos, void* stream) {
  last_error().clear();
  return qsgs_generate_phases_interacting(dims, n_phases, phases, nullptr, d_labels, d_ws,
                                          ws_bytes, infos, stream);
}

qsgs_status qsgs_generate_phases_interacting(const qsgs_dims* dims, int32_t n_phases,
                                             const qsgs_params* phases, const double* interact,
                                             uint8_t* d_labels, void* d_ws, size_t ws_bytes,
                                             qsgs_info* infos, void* stream) {
  last_error().clear();
  if (!dims || !phases || !d_labels || !d_ws || !infos)
    return fail(QSGS_ERR_INVALID, "dims, phases, d_labels, d_ws and infos must not be NULL");
  if (n_phases < 1 || n_phases > kMaxPhases)
    return fail(QSGS_ERR_INVALID, "n_phases %d outside [1, %d]", n_phases, kMaxPhases);
  Geometry g{};
  QSGS_TRY(check_dims(dims, &g));
  for (int32_t k = 0; k < n_phases; ++k) QSGS_TRY(check_params(&phases[k]));
  // the interaction tables: phase k + 1 may convert earlier phase m + 1 (grid byte 4 + m)
  std::vector<InteractTable> tabs;
  std::vector<std::array<uint32_t, 3>> hmax;
  std::vector<bool> interacts((size_t)n_phases, false);
  if (interact) {
    tabs.resize((size_t)n_phases);
    hmax.assign((size_t)n_phases, {0u, 0u, 0u});
    for (int32_t k = 0; k < n_phases; ++k) {
      InteractTable& T = tabs[(size_t)k];
      std::memset(&T, 0, sizeof T);
      for (int32_t m = 0; m < k; ++m) {
        const double* I = interact + 3 * ((size_t)k * (size_t)n_phases + (size_t)m);
        bool any = false;
        for (int c = 0; c < 3; ++c) {
          if (!is_prob(I[c]))
            return fail(QSGS_ERR_INVALID, "interaction of phase %d with phase %d, class %d, "
                        "must be in [0, 1]", k + 1, m + 1, c);
          any = any || I[c] > 0.0;
        }
        if (!any) continue;
        const uint32_t b = kWallBase + 1u + (uint32_t)m;
        T.bits[b >> 5] |= 1u << (b & 31u);
        for (int c = 0; c < 3; ++c) {
          const uint64_t thr = prob_threshold(I[c]);
          T.thr[6 * b + c] = (uint32_t)(thr >> 16);
          T.thr[6 * b + 3 + c] = (uint32_t)(thr & 0xFFFFu);
          hmax[(size_t)k][c] = std::max(hmax[(size_t)k][c], (uint32_t)(thr >> 16));
        }
        interacts[(size_t)k] = true;
      }
      if (interacts[(size_t)k] && phases[k].sweep_form == QSGS_SWEEP_FIELD)
        return fail(QSGS_ERR_INVALID, "phase %d interacts with an earlier phase: the "
                    "full-field form does not convert other phases", k + 1);
    }
  }
  if (reinterpret_cast<uintptr_t>(d_labels) % 4 != 0)
    return fail(QSGS_ERR_INVALID, "d_labels must be 4-byte aligned");
  const size_t need = qsgs_phases_workspace_bytes(dims, n_phases, phases);
  if (ws_bytes < need)
    return fail(QSGS_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", need, ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  const size_t gb = grid_bytes(g);
  const uint32_t words = (uint32_t)(gb / 4);
  const dim3 mg(std::min<uint32_t>(2048u, (words + 255u) / 256u)), mb(256);
  QSGS_HIP(hipMemsetAsync(d_labels, 0, gb, s));
  int32_t worst = QSGS_OK;
  for (int32_t k = 0; k < n_phases; ++k) {
    const bool it = interacts[(size_t)k];
    const qsgs_status st =
        generate_impl(1, dims, &phases[k], &d_labels, d_ws, ws_bytes, &infos[k], s, true, false,
                      it ? &tabs[(size_t)k] : nullptr, it ? hmax[(size_t)k].data() : nullptr);
    if (st < 0) return st;
    worst = std::max(worst, (int32_t)st);
    ByteMap m{};  // the phase's cells become walls for the phases after it
    for (int b = 0; b < 256; ++b) m.lut[b] = (uint8_t)b;
    m.lut[1] = (uint8_t)(kWallBase + 1 + k);
    hipLaunchKernelGGL(k_map_bytes, mg, mb, 0, s, (uint32_t*)d_labels, words, m);
    QSGS_LAUNCHED("k_map_bytes");
  }
  ByteMap m{};  // walls 3 + n -> label n
  for (int b = 0; b < 256; ++b) m.lut[b] = (uint8_t)b;
  for (int32_t k = 1; k <= n_phases; ++k) m.lut[kWallBase + k] = (uint8_t)k;
  hipLaunchKernelGGL(k_map_bytes, mg, mb, 0, s, (uint32_t*)d_labels, words, m);
  QSGS_LAUNCHED("k_map_bytes");
  QSGS_HIP(hipStreamSynchronize(s));
  return (qsgs_status)worst;
}

}  // extern "C"

namespace {

// Reads up to max_entries per-step log entries (kLogWords words each) of realization
// `index` of a generation workspace; returns the number of entries or an error.
int64_t read_log(const void* d_ws, size_t ws_bytes, int32_t index, int64_t max_entries,
                 void* stream, std::vector<uint64_t>* out) {
  if (!d_ws) return fail(QSGS_ERR_INVALID, "d_ws is NULL");
  if (ws_bytes < sizeof(WsHeader)) return fail(QSGS_ERR_WORKSPACE, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  WsHeader h{};
  QSGS_HIP(hipMemcpyAsync(&h, d_ws, sizeof h, hipMemcpyDeviceToHost, s));
  QSGS_HIP(hipStreamSynchronize(s));
  if (h.magic != kMagic) return fail(QSGS_ERR_INVALID, "workspace holds no generation");
  if (index < 0 || (uint32_t)index >= h.count)
    return fail(QSGS_ERR_INVALID, "realization index %d outside [0, %u)", index, h.count);
  Ctl c{};
  const char* base = static_cast<const char*>(d_ws);
  QSGS_HIP(hipMemcpyAsync(&c, base + h.reals + sizeof(Real) * index + offsetof(Real, ctl),
                          sizeof c, hipMemcpyDeviceToHost, s));
  QSGS_HIP(hipStreamSynchronize(s));
  const int64_t n = std::min<int64_t>({(int64_t)c.step, max_entries, (int64_t)h.log_cap});
  if (n <= 0) return 0;
  out->resize(kLogWords * (size_t)n);
  QSGS_HIP(hipMemcpyAsync(out->data(),
                          base + h.logs + sizeof(uint64_t) * kLogWords * h.log_cap * index,
                          sizeof(uint64_t) * out->size(), hipMemcpyDeviceToHost, s));
  QSGS_HIP(hipStreamSynchronize(s));
  return n;
}

}  // namespace

extern "C" {

int64_t qsgs_read_step_log(const void* d_ws, size_t ws_bytes, int32_t index, int64_t* front,
                           int64_t* grown, int64_t* count, int64_t max_entries, void* stream) {
  last_error().clear();
  std::vector<uint64_t> buf;
  const int64_t n = read_log(d_ws, ws_bytes, index, max_entries, stream, &buf);
  for (int64_t t = 0; t < n; ++t) {
    if (front) front[t] = (int64_t)buf[kLogWords * t];
    if (grown) grown[t] = (int64_t)buf[kLogWords * t + 1];
    if (count) count[t] = (int64_t)buf[kLogWords * t + 2];
  }
  return n;
}

int64_t qsgs_read_step_work(const void* d_ws, size_t ws_bytes, int32_t index, int64_t* draws,
                            int64_t* blocks, int64_t max_entries, void* stream) {
  last_error().clear();
  std::vector<uint64_t> buf;
  const int64_t n = read_log(d_ws, ws_bytes, index, max_entries, stream, &buf);
  for (int64_t t = 0; t < n; ++t) {
    if (draws) draws[t] = (int64_t)buf[kLogWords * t + 3];
    if (blocks) blocks[t] = (int64_t)buf[kLogWords * t + 4];
  }
  return n;
}

qsgs_status qsgs_set_tuning(const qsgs_tuning* t) {
  last_error().clear();
  Tuning n;
  if (t) {
    const uint32_t blocks[3] = {(uint32_t)t->grow_block, (uint32_t)t->prune_block,
                                (uint32_t)t->seed_block};
    const uint32_t grids[3] = {(uint32_t)t->grow_grid, (uint32_t)t->prune_grid,
                               (uint32_t)t->seed_grid};
    for (int k = 0; k < 3; ++k) {
      if (blocks[k] < 64 || blocks[k] > (uint32_t)kMaxBlock || blocks[k] % 64)
        return fail(QSGS_ERR_INVALID, "block sizes must be multiples of 64 in [64, %d]",
                    kMaxBlock);
      if (k == 0 && grids[k] == 0) continue;  // growth grid: one resident round
      if (grids[k] < 8 || grids[k] > kMaxSweepGrid || grids[k] % 8)
        return fail(QSGS_ERR_INVALID, "grid sizes must be multiples of 8 in [8, %u]",
                    kMaxSweepGrid);
    }
    if (t->steps_per_sync < 0 || t->steps_per_sync > 1024)
      return fail(QSGS_ERR_INVALID, "steps_per_sync must be in [0, 1024]");
    if (t->graphs != 0 && t->graphs != 1) return fail(QSGS_ERR_INVALID, "graphs must be 0 or 1");
    n.graphs = t->graphs != 0;
    n.grow_block = blocks[0];
    n.grow_block_auto = false;
    n.prune_block = blocks[1];
    n.seed_block = blocks[2];
    n.grow_grid = grids[0];
    n.prune_grid = grids[1];
    n.seed_grid = grids[2];
    n.steps_per_sync = t->steps_per_sync;
  }
  std::lock_guard<std::mutex> lk(tuning_mu());
  tuning_ref() = n;
  return QSGS_OK;
}

void qsgs_get_tuning(qsgs_tuning* t) {
  if (!t) return;
  const Tuning c = current_tuning();
  t->grow_block = (int32_t)c.grow_block;
  t->grow_grid = (int32_t)c.grow_grid;
  t->prune_block = (int32_t)c.prune_block;
  t->prune_grid = (int32_t)c.prune_grid;
  t->seed_block = (int32_t)c.seed_block;
  t->seed_grid = (int32_t)c.seed_grid;
  t->steps_per_sync = c.steps_per_sync;
  t->graphs = c.graphs ? 1 : 0;
}

void qsgs_profile_enable(int32_t enable) {
  std::lock_guard<std::mutex> lk(prof().mu);
  prof().enabled = enable != 0;
}

void qsgs_profile_read(double out[5], int32_t reset) {
  Profile& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  out[0] = p.grow_launches;
  out[1] = p.grow_ms;
  out[2] = p.prune_launches;
  out[3] = p.prune_ms;
  out[4] = p.seed_ms;
  if (reset) {
    p.grow_launches = p.grow_ms = p.prune_launches = p.prune_ms = 0;
    p.seed_ms = 0;
  }
}

const char* qsgs_last_error(void) { return last_error().c_str(); }

const char* qsgs_version(void) { return "qsgs 0.3.0 gfx950"; }

double qsgs_seed_prob_from_grain(double solid_fraction, double grain_diameter,
                                 double voxel_size) {
  if (!(solid_fraction >= 0.0 && solid_fraction <= 1.0) || !(grain_diameter > 0.0) ||
      !(voxel_size > 0.0) || !std::isfinite(grain_diameter) || !std::isfinite(voxel_size))
    return -1.0;
  const double r = voxel_size / grain_diameter;
  const double pi = 3.14159265358979323846;
  return std::min(1.0, 6.0 * solid_fraction * r * r * r / pi);
}

}  // extern "C"
