// qsgs_server.hip -- continuous-batching generation server (C ABI in include/qsgs.h).
//
// Requests of different sizes queue on the host; each tick admits queued requests in
// arrival order while a slot is free and their footprint (grid + tile lists) fits
// the free part of the caller's device arena, seeds them, and advances every resident
// realization by a few growth steps with the same per-step kernels that serve batches,
// so the growth steps of all resident requests share each launch.  Finished requests
// keep their grid in the arena until the caller takes it.
#include <deque>
#include <map>
#include <unordered_map>

#include "qsgs_host.h"

using namespace qsgs;
using namespace qsgs::host;

struct qsgs_server {
  // First-fit allocator over [lo, hi) of the arena, in 256-byte units.
  struct Arena {
    std::map<size_t, size_t> free_;  // offset -> size
    size_t lo = 0, hi = 0, used = 0;
    void reset(size_t l, size_t h) {
      lo = l;
      hi = h;
      free_.clear();
      if (h > l) free_[l] = h - l;
      used = 0;
    }
    bool alloc(size_t bytes, size_t* off) {
      bytes = align_up(bytes);
      for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= bytes) {
          *off = it->first;
          const size_t rest = it->second - bytes;
          const size_t at_ = it->first + bytes;
          free_.erase(it);
          if (rest) free_[at_] = rest;
          used += bytes;
          return true;
        }
      }
      return false;
    }
    void release(size_t off, size_t bytes) {
      bytes = align_up(bytes);
      used -= bytes;
      auto it = free_.emplace(off, bytes).first;
      auto next = std::next(it);
      if (next != free_.end() && it->first + it->second == next->first) {
        it->second += next->second;
        free_.erase(next);
      }
      if (it != free_.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
          prev->second += it->second;
          free_.erase(it);
        }
      }
    }
  };

  struct Request {
    int64_t id = 0;
    qsgs_dims dims{};
    qsgs_params params{};
    Spec spec{};
    size_t grid_off = 0, front_off = 0;
    int32_t slot = -1;
    bool failed = false;  // finished with an error: no grid is kept
    qsgs_info info{};
  };

  hipStream_t s = nullptr;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int32_t steps_per_tick = 1;
  Engine eng;
  Arena heap;
  std::deque<Request> queue;
  std::vector<int64_t> slot_req;  // request id per slot, -1 when free
  std::unordered_map<int64_t, Request> resident;
  std::deque<int64_t> ready;      // finished, grid not yet taken
  std::unordered_map<int64_t, Request> done;
  std::vector<Real> recs;         // the records as the last tick left them
  char* stage = nullptr;          // the engine's pinned staging (owned by the server)

  static size_t front_bytes(const Geometry& g) { return sweep_state_bytes(g, false); }
  static size_t footprint(const Geometry& g) { return align_up(grid_bytes(g)) + front_bytes(g); }
};

namespace {

// Upper bound of the passes one tick runs when every resident request is far from done.
constexpr uint64_t kMaxPassesPerTick = 16;

qsgs_status server_admit(qsgs_server* S, std::vector<size_t>* group) {
  // Admit in arrival order while a slot is free and grid + fronts fit.
  while (!S->queue.empty()) {
    auto free_slot = std::find(S->slot_req.begin(), S->slot_req.end(), (int64_t)-1);
    if (free_slot == S->slot_req.end()) break;
    qsgs_server::Request& q = S->queue.front();
    size_t g_off = 0, f_off = 0;
    if (!S->heap.alloc(align_up(grid_bytes(q.spec.g)), &g_off)) break;
    if (!S->heap.alloc(qsgs_server::front_bytes(q.spec.g), &f_off)) {
      S->heap.release(g_off, align_up(grid_bytes(q.spec.g)));
      break;
    }
    q.grid_off = g_off;
    q.front_off = f_off;
    q.slot = (int32_t)(free_slot - S->slot_req.begin());
    *free_slot = q.id;
    group->push_back((size_t)q.slot);
    S->resident.emplace(q.id, q);
    S->queue.pop_front();
  }
  return QSGS_OK;
}

}  // namespace

extern "C" {

size_t qsgs_server_reserved_bytes(int32_t max_slots) {
  if (max_slots < 1) return 0;
  return persist_layout((size_t)max_slots, 0).total;
}

qsgs_status qsgs_server_create(void* d_arena, size_t arena_bytes, int32_t max_slots,
                               int32_t steps_per_tick, void* stream, qsgs_server** out) {
  last_error().clear();
  if (!out) return fail(QSGS_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!d_arena || (uintptr_t)d_arena % kAlign)
    return fail(QSGS_ERR_INVALID, "d_arena must be a 256-byte aligned device pointer");
  if (max_slots < 1 || (uint32_t)max_slots > kMaxBatch)
    return fail(QSGS_ERR_INVALID, "max_slots in [1, %u]", kMaxBatch);
  if (steps_per_tick < 1 || steps_per_tick > 1024)
    return fail(QSGS_ERR_INVALID, "steps_per_tick in [1, 1024]");
  const PersistLayout P = persist_layout((size_t)max_slots, 0);
  if (arena_bytes < P.total)
    return fail(QSGS_ERR_WORKSPACE, "arena needs at least %zu bytes", P.total);
  auto* S = new qsgs_server();
  S->s = (hipStream_t)stream;
  S->arena = static_cast<char*>(d_arena);
  S->arena_bytes = arena_bytes;
  S->steps_per_tick = steps_per_tick;
  S->eng.bind(d_arena, P, (size_t)max_slots, S->s);
  if (hipHostMalloc((void**)&S->stage, Engine::stage_bytes((size_t)max_slots),
                    hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    S->stage = nullptr;  // pageable copies
  }
  S->eng.stage = S->stage;
  S->heap.reset(P.total, arena_bytes);
  S->slot_req.assign((size_t)max_slots, -1);
  qsgs_status st = S->eng.upload_header();
  if (st == QSGS_OK) st = S->eng.upload_control();
  if (st == QSGS_OK) st = S->eng.upload(0, (size_t)max_slots);  // every slot empty
  if (st != QSGS_OK) {
    (void)hipStreamSynchronize(S->s);  // the uploads read the staging buffer
    if (S->stage) (void)hipHostFree(S->stage);
    delete S;
    return st;
  }
  *out = S;
  return QSGS_OK;
}

qsgs_status qsgs_server_submit(qsgs_server* S, int64_t request_id, const qsgs_dims* dims,
                               const qsgs_params* params) {
  last_error().clear();
  if (!S) return fail(QSGS_ERR_INVALID, "server is NULL");
  qsgs_server::Request q;
  QSGS_TRY(check_dims(dims, &q.spec.g));
  QSGS_TRY(check_params(params));
  if (S->resident.count(request_id) || S->done.count(request_id))
    return fail(QSGS_ERR_INVALID, "request id %lld is in use", (long long)request_id);
  for (const auto& r : S->queue)
    if (r.id == request_id)
      return fail(QSGS_ERR_INVALID, "request id %lld is in use", (long long)request_id);
  q.spec.bk = make_buckets(q.spec.g, params->spacing);
  q.id = request_id;
  q.dims = *dims;
  q.params = *params;
  const size_t need = qsgs_server::footprint(q.spec.g) + seed_layout({q.spec}, true).total;
  if (need > S->heap.hi - S->heap.lo)
    return fail(QSGS_ERR_CAPACITY, "request needs %zu arena bytes, the arena holds %zu", need,
                S->heap.hi - S->heap.lo);
  S->queue.push_back(q);
  return QSGS_OK;
}

qsgs_status qsgs_server_tick(qsgs_server* S, int32_t* n_resident, int32_t* n_queued,
                             int32_t* n_ready) {
  last_error().clear();
  if (!S) return fail(QSGS_ERR_INVALID, "server is NULL");
  Engine& E = S->eng;
  std::vector<size_t> group;
  QSGS_TRY(server_admit(S, &group));
  // The seeding scratch of the admitted group; if it does not fit, the newest
  // admissions go back to the head of the queue.
  size_t scratch_off = 0, scratch_bytes = 0;
  while (!group.empty()) {
    std::vector<Spec> specs;
    for (size_t slot : group) specs.push_back(S->resident.at(S->slot_req[slot]).spec);
    const SeedLayout L = seed_layout(specs, true);
    if (S->heap.alloc(L.total, &scratch_off)) {
      scratch_bytes = L.total;
      for (size_t k = 0; k < group.size(); ++k) {
        qsgs_server::Request& q = S->resident.at(S->slot_req[group[k]]);
        E.init_sweep_record(group[k], q.spec, &q.params,
                            reinterpret_cast<uint8_t*>(S->arena + q.grid_off),
                            S->arena + q.front_off, false);
      }
      E.attach_scratch(group, S->arena + scratch_off, L);
      for (size_t slot : group) QSGS_TRY(E.upload(slot, 1));
      QSGS_TRY(E.seed_core(S->arena + scratch_off, L));
      QSGS_TRY(E.sweep_start(group));
      break;
    }
    const size_t slot = group.back();
    group.pop_back();
    qsgs_server::Request q = S->resident.at(S->slot_req[slot]);
    S->resident.erase(q.id);
    S->slot_req[slot] = -1;
    S->heap.release(q.front_off, qsgs_server::front_bytes(q.spec.g));
    S->heap.release(q.grid_off, align_up(grid_bytes(q.spec.g)));
    q.slot = -1;
    S->queue.push_front(q);
  }
  if (scratch_bytes) S->heap.release(scratch_off, scratch_bytes);  // stream-ordered reuse

  // Passes this tick: at least steps_per_tick, and up to the fewest any resident request
  // is expected to need before it stops (its remaining count over its last growth, plus
  // the final pass; steps_per_tick for one without growth seen yet), so that a lone
  // request does not pay a host round trip every few passes while a full table still
  // retires requests promptly.
  if (!S->resident.empty()) {
    uint64_t passes = kMaxPassesPerTick;
    for (size_t slot = 0; slot < S->slot_req.size(); ++slot) {
      if (S->slot_req[slot] < 0) continue;
      uint64_t need = (uint64_t)S->steps_per_tick;  // no growth seen yet
      if (slot < S->recs.size() && S->recs[slot].phase == kPhaseGrow) {
        const Ctl& c = S->recs[slot].ctl;
        if (c.mode == kModeFinal)
          need = 1;
        else if (c.step > 0 && c.last_new > 0)
          need = (c.s_star > c.cnt ? (c.s_star - c.cnt) : 0) / c.last_new + 2;
        else if (c.step > 0)
          need = kMaxPassesPerTick;  // growing without new voxels yet: not near its end
      }
      passes = std::min(passes, need);
    }
    passes = std::max<uint64_t>(passes, (uint64_t)S->steps_per_tick);
    std::vector<bool> live(S->slot_req.size());
    for (size_t slot = 0; slot < live.size(); ++slot) live[slot] = S->slot_req[slot] >= 0;
    bool tiles = false, field = false;
    E.forms_in_use(&tiles, &field, &live);
    QSGS_TRY(E.run_passes((uint32_t)passes, nullptr, tiles, field));
    QSGS_TRY(E.export_grids());  // the requests that stopped: byte grids from their planes
  }

  // Retire finished requests: their fronts return to the arena, the grid waits.
  std::vector<Real>& recs = S->recs;
  int64_t failed_id = -1;
  QSGS_TRY(E.read_all(&recs));
  for (size_t slot = 0; slot < S->slot_req.size(); ++slot) {
    const int64_t id = S->slot_req[slot];
    if (id < 0) continue;
    const Real& R = recs[slot];
    if (R.phase != kPhaseGrow || R.ctl.status == 0) continue;
    qsgs_server::Request q = S->resident.at(id);
    S->resident.erase(id);
    S->slot_req[slot] = -1;
    fill_info(R.ctl, &q.info);
    S->heap.release(q.front_off, qsgs_server::front_bytes(q.spec.g));
    q.slot = -1;
    if (R.ctl.status == kStatusOverflow || R.ctl.bad_entry) {
      // an internal list overflowed: the request fails, its grid is released at once,
      // and the other requests of this tick are still retired
      S->heap.release(q.grid_off, align_up(grid_bytes(q.spec.g)));
      q.failed = true;
      q.info.status = QSGS_ERR_DEVICE;
      if (failed_id < 0) failed_id = id;
    }
    S->done.emplace(id, q);
    S->ready.push_back(id);
  }
  if (n_resident) *n_resident = (int32_t)S->resident.size();
  if (n_queued) *n_queued = (int32_t)S->queue.size();
  if (n_ready) *n_ready = (int32_t)S->ready.size();
  if (failed_id >= 0)
    return fail(QSGS_ERR_DEVICE, "internal front overflow in request %lld", (long long)failed_id);
  return QSGS_OK;
}

int32_t qsgs_server_ready(qsgs_server* S, int64_t* ids, qsgs_info* infos, int32_t max) {
  if (!S || max <= 0) return 0;
  int32_t n = 0;
  for (int64_t id : S->ready) {
    if (n >= max) break;
    if (ids) ids[n] = id;
    if (infos) infos[n] = S->done.at(id).info;
    ++n;
  }
  return n;
}

qsgs_status qsgs_server_take(qsgs_server* S, int64_t request_id, void* dst, size_t dst_bytes,
                             int32_t dst_on_host) {
  last_error().clear();
  if (!S) return fail(QSGS_ERR_INVALID, "server is NULL");
  auto it = S->done.find(request_id);
  if (it == S->done.end())
    return fail(QSGS_ERR_INVALID, "request %lld is not finished", (long long)request_id);
  const qsgs_server::Request& q = it->second;
  const size_t n = q.spec.g.n;
  if (q.failed) {  // its grid was released when it failed
    S->ready.erase(std::find(S->ready.begin(), S->ready.end(), request_id));
    S->done.erase(it);
    return fail(QSGS_ERR_DEVICE, "request %lld failed (internal front overflow)",
                (long long)request_id);
  }
  if (dst) {
    if (dst_bytes < n) return fail(QSGS_ERR_INVALID, "dst needs %zu bytes", n);
    QSGS_HIP(hipMemcpyAsync(dst, S->arena + q.grid_off, n,
                            dst_on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, S->s));
    QSGS_HIP(hipStreamSynchronize(S->s));
  }
  S->heap.release(q.grid_off, align_up(grid_bytes(q.spec.g)));
  S->ready.erase(std::find(S->ready.begin(), S->ready.end(), request_id));
  S->done.erase(it);
  return QSGS_OK;
}

size_t qsgs_server_free_bytes(const qsgs_server* S) {
  if (!S) return 0;
  return (S->heap.hi - S->heap.lo) - S->heap.used;
}

void qsgs_server_destroy(qsgs_server* S) {
  if (!S) return;
  (void)hipStreamSynchronize(S->s);  // destroy cannot report; pending work must finish first
  if (S->stage) (void)hipHostFree(S->stage);
  delete S;
}

}  // extern "C"
