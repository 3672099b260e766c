// qsgs_host.h -- host-side engine of libqsgs, shared by the C-ABI translation units.
//
// An Engine drives a table of realization records in device memory: it seeds the
// records marked for seeding, advances every growing record by one step per call,
// and reads the records back.  The single-grid entry points, the batched entry point
// and the serving loop all run through it.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "qsgs.h"
#include "qsgs_internal.h"

namespace qsgs {
namespace host {

inline std::string& last_error() {
  static thread_local std::string e;
  return e;
}

inline qsgs_status fail(qsgs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error() = buf;
  return s;
}

#define QSGS_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::qsgs::host::fail(QSGS_ERR_DEVICE, "%s failed: %s", #call,                 \
                                hipGetErrorString(e_));                                  \
  } while (0)

#define QSGS_LAUNCHED(what)                                                              \
  do {                                                                                   \
    hipError_t e_ = hipGetLastError();                                                   \
    if (e_ != hipSuccess)                                                                \
      return ::qsgs::host::fail(QSGS_ERR_DEVICE, "launch of %s failed: %s", what,        \
                                hipGetErrorString(e_));                                  \
  } while (0)

#define QSGS_TRY(expr)              \
  do {                              \
    qsgs_status st_ = (expr);       \
    if (st_ != QSGS_OK) return st_; \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int32_t kDefaultMaxSteps = 1 << 20;
constexpr uint32_t kRoundsPerCheck = 8;
constexpr uint32_t kLogCapSingle = 65536;  // per-step log entries of a batch of one
constexpr uint32_t kLogCapBatch = 4096;    // per realization in larger batches
constexpr uint64_t kMagic = 0x51534753574B5331ull;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// ----- integer constants (Sec. 2.1 step 2, Sec. 2.3 step 5, Eq. (1)) -----

// min(2^32, floor(p 2^32)); p * 2^32 is exact in binary64.
inline uint64_t prob_threshold(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return kOne32;
  return (uint64_t)std::floor(p * 4294967296.0);
}

// S* = ceil(phi_s N) evaluated in binary64, clamped to [0, N].
inline uint64_t target_count(double phi_s, uint64_t n) {
  double t = std::ceil(phi_s * (double)n);
  if (t < 0.0) t = 0.0;
  if (t > (double)n) t = (double)n;
  return (uint64_t)t;
}

inline bool is_prob(double p) { return std::isfinite(p) && p >= 0.0 && p <= 1.0; }

inline qsgs_status check_dims(const qsgs_dims* d, Geometry* g) {
  if (!d) return fail(QSGS_ERR_INVALID, "dims is NULL");
  if (d->nx < 1 || d->ny < 1 || d->nz < 1)
    return fail(QSGS_ERR_INVALID, "dims must be >= 1 (got %d x %d x %d)", d->nx, d->ny, d->nz);
  const int64_t n = (int64_t)d->nx * d->ny * d->nz;
  if (n >= (int64_t)1 << 31)
    return fail(QSGS_ERR_INVALID, "nx*ny*nz = %lld must be < 2^31", (long long)n);
  g->nx = d->nx;
  g->ny = d->ny;
  g->nz = d->nz;
  g->nxy = (uint32_t)d->nx * (uint32_t)d->ny;
  g->n = (uint32_t)n;
  g->div_nx.init((uint32_t)d->nx);
  g->div_ny.init((uint32_t)d->ny);
  return QSGS_OK;
}

inline qsgs_status check_params(const qsgs_params* p) {
  if (!p) return fail(QSGS_ERR_INVALID, "params is NULL");
  if (!(std::isfinite(p->solid_fraction) && p->solid_fraction > 0.0 && p->solid_fraction <= 1.0))
    return fail(QSGS_ERR_INVALID, "solid_fraction must be in (0, 1]");
  if (!is_prob(p->seed_prob)) return fail(QSGS_ERR_INVALID, "seed_prob must be in [0, 1]");
  for (int c = 0; c < 3; ++c)
    if (!is_prob(p->g_ref[c])) return fail(QSGS_ERR_INVALID, "g_ref[%d] must be in [0, 1]", c);
  if (p->spacing < 0) return fail(QSGS_ERR_INVALID, "spacing must be >= 0");
  if (p->sweep_form < QSGS_SWEEP_LIST || p->sweep_form > QSGS_SWEEP_ALL_TILES)
    return fail(QSGS_ERR_INVALID, "sweep_form must be 0 (list), 1 (full field) or 2 (all tiles)");
  if (p->front_rule != 0 && p->front_rule != 1)
    return fail(QSGS_ERR_INVALID, "front_rule must be 0 or 1");
  if (p->front_rule == 1 && p->sweep_form == QSGS_SWEEP_FIELD)
    return fail(QSGS_ERR_INVALID, "the full-field form has no front: front_rule must be 0");
  return QSGS_OK;
}

inline qsgs_status check_grid(const uint8_t* grid) {
  if (!grid) return fail(QSGS_ERR_INVALID, "d_grid is NULL");
  if ((uintptr_t)grid % 4 != 0) return fail(QSGS_ERR_INVALID, "d_grid must be 4-byte aligned");
  return QSGS_OK;
}

// N bytes of voxels, rounded up to a multiple of 4 for the 32-bit claim atomics, plus
// 8 bytes of padding read (never written) by the 8-byte neighbourhood windows.
inline size_t grid_bytes(const Geometry& g) { return ((size_t)g.n + 8 + 3) / 4 * 4; }

inline Tiles make_tiles(const Geometry& g) {
  Tiles t{};
  t.ntx = (uint32_t)((g.nx + kTileX - 1) / kTileX);
  t.nty = (uint32_t)((g.ny + kTileY - 1) / kTileY);
  t.ntz = (uint32_t)((g.nz + kTileZ - 1) / kTileZ);
  t.n = t.ntx * t.nty * t.ntz;  // <= N: every tile holds a voxel
  t.div_ntx.init(t.ntx);
  t.div_nty.init(t.nty);
  return t;
}

// Device memory of the fused sweep per realization: the two tile maps (one bit per tile
// each) and the occupancy planes (S, M0, M1, and W and X on a multi-phase grid) of
// ntx * ny * nz 64-bit words each.
inline size_t map_bytes(const Geometry& g) {
  return 2 * sizeof(uint32_t) * (size_t)tile_map_words(make_tiles(g).n);
}
inline uint32_t plane_words(const Geometry& g) {
  return make_tiles(g).ntx * (uint32_t)g.ny * (uint32_t)g.nz;
}
// S, M0, M1; on a multi-phase grid also W and X
inline size_t plane_bytes(const Geometry& g, bool walls) {
  return sizeof(uint64_t) * (size_t)plane_words(g) * (walls ? 5 : 3);
}
inline size_t sweep_state_bytes(const Geometry& g, bool walls) {
  return align_up(map_bytes(g)) + align_up(plane_bytes(g, walls));
}

inline Buckets make_buckets(const Geometry& g, int32_t spacing) {
  Buckets b{};
  if (spacing <= 1) return b;
  const uint32_t e = (uint32_t)(spacing - 1);
  b.edge.init(e);
  b.nbx = (uint32_t)(((uint64_t)g.nx + e - 1) / e);
  b.nby = (uint32_t)(((uint64_t)g.ny + e - 1) / e);
  b.nbz = (uint32_t)(((uint64_t)g.nz + e - 1) / e);
  b.nb = b.nbx * b.nby * b.nbz;
  b.radius = spacing - 1;
  return b;
}

inline Ctl make_ctl(const Geometry& g, const qsgs_params* p) {
  Ctl c{};
  c.s_star = target_count(p->solid_fraction, g.n);
  for (int k = 0; k < 3; ++k) c.t_ref[k] = prob_threshold(p->g_ref[k]);
  c.max_steps = p->max_steps > 0 ? p->max_steps : kDefaultMaxSteps;
  return c;
}

inline void fill_info(const Ctl& c, qsgs_info* info) {
  info->n_candidates = c.n_cand;
  info->n_seeds = c.n_seeds;
  info->solid_count = (int64_t)c.cnt;
  info->target_count = (int64_t)c.s_star;
  info->front_size = c.front_size;
  info->grown_last_step = c.last_new;
  info->step = c.step;
  info->status = c.status;
}

struct Spec {
  Geometry g;
  Buckets bk;
};

// Host-readable description at the start of a workspace (for the step-log reader).
struct WsHeader {
  uint64_t magic;
  uint32_t count, log_cap;
  uint64_t reals, logs;
};

// Fixed part of a workspace: header, batch control, realization records, offset
// table, round counters and per-step logs.
struct PersistLayout {
  size_t hdr = 0, bctl = 0, reals = 0, off = 0, live = 0, logs = 0, total = 0;
  size_t rec = 0, desc = 0;
  uint32_t log_cap = 0;
};

inline PersistLayout persist_layout(size_t count, uint32_t log_cap) {
  PersistLayout L;
  L.log_cap = log_cap;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t a = off;
    off = align_up(off + bytes);
    return a;
  };
  L.hdr = take(sizeof(WsHeader));
  L.bctl = take(sizeof(BatchCtl));
  L.reals = take(sizeof(Real) * count);
  L.off = take(sizeof(uint64_t) * (count + 1));
  L.live = take(sizeof(uint32_t) * kMaxRounds);
  L.logs = take(sizeof(uint64_t) * kLogWords * (size_t)log_cap * count);
  L.rec = take(sizeof(WgRec) * kMaxSweepGrid);
  L.desc = take(sizeof(WgDesc) * kMaxSweepGrid);
  L.total = off;
  return L;
}

// Seeding scratch of a group of realizations (offsets relative to its base): the
// candidate lists, the spacing buckets and the bucket-sorted candidates.
struct SeedLayout {
  std::vector<size_t> cand;
  size_t counts = 0, cursor = 0, sums = 0, sorted_v = 0, sorted_r = 0, prio = 0, status = 0,
         total = 0;
  uint32_t total_buckets = 0;
};

inline SeedLayout seed_layout(const std::vector<Spec>& specs, bool with_cand = true) {
  SeedLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t a = off;
    off = align_up(off + bytes);
    return a;
  };
  uint64_t tb = 0, sorted = 0;
  for (const Spec& s : specs) {
    tb += s.bk.nb;
    if (s.bk.nb) sorted += s.g.n;
  }
  L.total_buckets = (uint32_t)tb;
  const size_t nscan = (size_t)tb + 1;
  L.counts = take(sizeof(uint32_t) * nscan);
  L.cursor = take(sizeof(uint32_t) * nscan);
  size_t sums = 0;
  for (size_t m = nscan; m > 1;) {
    m = (m + kScanBlock - 1) / kScanBlock;
    sums += m + 1;
  }
  L.sums = take(sizeof(uint32_t) * (sums + 8));
  L.sorted_v = take(sizeof(int32_t) * sorted);
  L.sorted_r = take(sizeof(uint32_t) * sorted);
  L.prio = take(sizeof(uint64_t) * sorted);
  L.status = take(sorted);
  for (const Spec& s : specs)
    L.cand.push_back(with_cand ? take(sizeof(int32_t) * s.g.n) : (size_t)-1);
  L.total = off;
  return L;
}

// Pinned host memory for an engine's small transfers: a pageable copy is staged by the
// runtime and costs a host round trip each; from pinned memory copies are plain DMA and
// several share one synchronization.  One buffer per thread for the calls that bind an
// engine for their own duration (each of them synchronizes before it returns), grown
// when a call needs more; nullptr when pinned memory cannot be had (the engine then
// copies from pageable memory).
inline char* thread_pinned_stage(size_t bytes) {
  thread_local char* p = nullptr;
  thread_local size_t n = 0;
  if (bytes > n) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    if (hipHostMalloc((void**)&p, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return nullptr;
    }
    n = bytes;
  }
  return p;
}

// Launch shape of the item kernels (block = threads per workgroup, a multiple of 64 up
// to 512; grid = workgroups, a multiple of 8) and the steps issued between host reads.
struct Tuning {
  uint32_t grow_block = kBlock, grow_grid = 0;  // 0: one round of resident sweep workgroups
  // the whole-generation calls on one realization take 512-thread sweep workgroups (eight
  // waves share a share's tiles; measured faster there, slower for batches of many)
  bool grow_block_auto = true;
  uint32_t prune_block = kBlock, prune_grid = 2048;
  uint32_t seed_block = kBlock, seed_grid = 2048;
  int32_t steps_per_sync = 0;  // 0: adaptive
  bool graphs = true;          // passes as launches of captured chunk graphs
};

// LDS is granted to a workgroup in whole granules of this many bytes (gfx950: 128 of them
// per compute unit).  The runtime's occupancy query divides the bytes exactly and so can
// promise one workgroup per compute unit more than the granules allow: measured, 26 880
// bytes (21 granules) fit six workgroups and 26 881 five, though the query says six up to
// 27 306; 32 000 bytes fit five and 32 001 four.
constexpr size_t kLdsGranule = 1280;

// Workgroups of one k_sweep variant (block threads each) that a compute unit of device
// dev holds at once: the runtime's occupancy (registers, waves) capped by the LDS
// granules; 0 when the runtime cannot say.
template <bool kWalls, bool kLiteral>
int sweep_per_cu(int dev, uint32_t block) {
  int per_cu = 0, lds_cu = 0;
  hipFuncAttributes fa{};
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep<kWalls, kLiteral>,
                                                   (int)block,
                                                   sweep_lds_bytes(block)) != hipSuccess ||
      hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_sweep<kWalls, kLiteral>)) !=
          hipSuccess ||
      hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
          hipSuccess ||
      per_cu <= 0 || lds_cu <= 0) {
    (void)hipGetLastError();
    return 0;
  }
  const size_t wg = (fa.sharedSizeBytes + sweep_lds_bytes(block) + kLdsGranule - 1) /
                    kLdsGranule * kLdsGranule;
  return std::min<int>(per_cu, (int)((size_t)lds_cu / wg));
}

// Workgroups of k_sweep (block threads each; the variants for grids with other phases'
// cells when walls) that the current device holds at once: one round of them takes every
// list share at the same time, and no share waits for a slot.  2048 when the runtime
// cannot say.
// Computed once per device, block size and variant pair (the later calls may be under
// graph capture).
inline uint32_t resident_sweep_grid(uint32_t block, bool walls) {
  static std::mutex mu;
  static std::map<std::tuple<int, uint32_t, bool>, uint32_t> known;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 2048;
  }
  std::lock_guard<std::mutex> lk(mu);
  const auto it = known.find({dev, block, walls});
  if (it != known.end()) return it->second;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0) {
    (void)hipGetLastError();
    return 2048;
  }
  const int per_cu = walls ? std::min(sweep_per_cu<true, false>(dev, block),
                                      sweep_per_cu<true, true>(dev, block))
                           : std::min(sweep_per_cu<false, false>(dev, block),
                                      sweep_per_cu<false, true>(dev, block));
  if (per_cu <= 0) return 2048;
  const uint32_t n = (uint32_t)cus * (uint32_t)per_cu;
  const uint32_t g = std::max<uint32_t>(kNumXcd, n / kNumXcd * kNumXcd);
  known[{dev, block, walls}] = g;
  return g;
}

inline std::mutex& tuning_mu() {
  static std::mutex m;
  return m;
}
inline Tuning& tuning_ref() {
  static Tuning t;
  return t;
}
inline Tuning current_tuning() {
  std::lock_guard<std::mutex> lk(tuning_mu());
  return tuning_ref();
}

// ----- kernel timing -----
struct Profile {
  std::mutex mu;
  bool enabled = false;
  double grow_launches = 0, grow_ms = 0, prune_launches = 0, prune_ms = 0, seed_ms = 0;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
};
inline Profile& prof() {
  static Profile p;
  return p;
}
inline bool prof_on() {
  std::lock_guard<std::mutex> lk(prof().mu);
  return prof().enabled;
}
inline hipEvent_t prof_event() {
  Profile& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (p.used == p.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p.pool.push_back(e);
  }
  return p.pool[p.used++];
}
inline void prof_release_all() {
  std::lock_guard<std::mutex> lk(prof().mu);
  prof().used = 0;
}

// ----- captured pass chunks -----
// Executable graphs of captured chunks of passes, keyed by everything the passes launch
// with (device, kernel arguments, launch shapes, kernel choice, chunk length).  A graph
// is reused only by launches identical to the ones it captured.  Kept for the life of
// the process; at most kMaxGraphs, later configurations launch their kernels directly.
constexpr size_t kMaxGraphs = 64;
struct GraphCache {
  std::mutex mu;
  std::map<std::string, hipGraphExec_t> exec;
};
inline GraphCache& graph_cache() {
  static GraphCache c;
  return c;
}
// The calling thread's capture stream on the current device (a graph is captured on it
// and launched on the caller's stream, which may be the null stream).
inline hipStream_t capture_stream() {
  thread_local std::map<int, hipStream_t> streams;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  streams[dev] = cs;
  return cs;
}

// ----- the engine -----
struct Engine {
  hipStream_t s = nullptr;
  void* ws = nullptr;  // base of the persistent part
  PersistLayout P;
  std::vector<Real> reals;  // host mirror of the records
  BatchArgs args{};
  Tuning tune;
  WsHeader hdr{};
  uint32_t sweep_grid = 2048;
  bool no_events = false;  // the call may not allocate: no timing events
  // the call never synchronises with the host (it may be captured into a graph): host
  // data reaches the device as kernel arguments, the spacing rounds run a fixed number
  // of times and the passes a fixed number of times
  bool async = false;
  // pinned staging (see thread_pinned_stage): uploads, then readbacks, each in its own
  // region; nullptr for pageable copies
  char* stage = nullptr;
  static size_t stage_bytes(size_t count) {
    return 4 * kStageSlot + 2 * align_up(sizeof(Real) * count) + kStageSlot;
  }
  static constexpr size_t kStageSlot = 256;
  char* st_up_hdr() { return stage; }
  char* st_up_ctl() { return stage + kStageSlot; }
  char* st_up_reals() { return stage + 2 * kStageSlot; }
  char* st_dn_bctl() { return st_up_reals() + align_up(sizeof(Real) * reals.size()); }
  char* st_dn_ctl() { return st_dn_bctl() + kStageSlot; }
  char* st_dn_reals() { return st_dn_ctl() + kStageSlot; }
  char* st_dn_live() { return st_dn_reals() + align_up(sizeof(Real) * reals.size()); }

  // Binds the engine to a persistent region of `count` records at `base`.
  // walls: the records' grids may hold other phases' cells (the sweep variants for them);
  // auto_grow_block: the sweep workgroup size when the tuning leaves it to the call.
  void bind(void* base, const PersistLayout& L, size_t count, hipStream_t stream,
            bool walls = false, uint32_t auto_grow_block = 0) {
    ws = base;
    P = L;
    s = stream;
    tune = current_tuning();
    if (tune.grow_block_auto && auto_grow_block) tune.grow_block = auto_grow_block;
    reals.assign(count, Real{});
    args = BatchArgs{};
    args.reals = at<Real>(base, L.reals);
    args.count = (uint32_t)count;
    args.off = at<uint64_t>(base, L.off);
    args.bctl = at<BatchCtl>(base, L.bctl);
    args.live = at<uint32_t>(base, L.live);
    args.rec = at<WgRec>(base, L.rec);
    args.desc = at<WgDesc>(base, L.desc);
    const uint32_t g =
        tune.grow_grid ? tune.grow_grid : resident_sweep_grid(tune.grow_block, walls);
    const uint32_t want = std::max<uint32_t>(g, 2 * (uint32_t)count);
    sweep_grid = std::min<uint32_t>(kMaxSweepGrid, (want + kNumXcd - 1) / kNumXcd * kNumXcd);
    args.sweep_grid = sweep_grid;
  }

  // Control block, plan index and the zeroed tail counters: once per engine.
  // n bytes of host data to device address dst: a copy, or (async) kernel arguments
  qsgs_status put(void* dst, const void* src, size_t n) {
    if (!async) {
      QSGS_HIP(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s));
      return QSGS_OK;
    }
    const size_t words = (n + 3) / 4;
    for (size_t w0 = 0; w0 < words; w0 += 256) {
      WordBlob b{};
      b.n = (uint32_t)std::min<size_t>(256, words - w0);
      std::memcpy(b.w, static_cast<const char*>(src) + 4 * w0,
                  std::min<size_t>(4 * (size_t)b.n, n - 4 * w0));
      hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, s,
                         reinterpret_cast<uint32_t*>(static_cast<char*>(dst) + 4 * w0), b);
      QSGS_LAUNCHED("k_put_words");
    }
    return QSGS_OK;
  }

  qsgs_status upload_control() {
    BatchCtl b{};
    b.grid = sweep_grid;
    const void* src = &b;
    if (stage) src = std::memcpy(st_up_ctl(), &b, sizeof b);
    QSGS_TRY(put(args.bctl, src, sizeof b));
    return QSGS_OK;
  }

  dim3 rgrid() const { return dim3(((uint32_t)reals.size() + 255) / 256); }

  uint64_t* log_of(size_t r) const {
    if (P.log_cap == 0) return nullptr;
    return at<uint64_t>(ws, P.logs) + (size_t)kLogWords * P.log_cap * r;
  }

  // Fills record r for a new realization (to be seeded).  For the fused sweep,
  // `sweep` is the realization's sweep_state_bytes region (two tile lists of 2 x tiles
  // entries, parts in the first half and spills in the second, then the stamps); the
  // step-by-step path passes its caller's front buffers instead.
  void init_record(size_t r, const Spec& sp, const qsgs_params* p, uint8_t* grid, int32_t* f0,
                   int32_t* f1, uint32_t cap) {
    Real& R = reals[r];
    R = Real{};
    R.g = sp.g;
    R.bk = sp.bk;
    R.tl = make_tiles(sp.g);
    R.grid = grid;
    R.f0 = f0;
    R.f1 = f1;
    R.cap = cap;
    R.log = log_of(r);
    R.log_cap = P.log_cap;
    R.k0 = (uint32_t)p->key;
    R.k1 = (uint32_t)(p->key >> 32);
    R.t_seed = prob_threshold(p->seed_prob);
    R.spacing = p->spacing;
    R.phase = kPhaseSeed;
    R.ctl = make_ctl(sp.g, p);
  }

  void init_sweep_record(size_t r, const Spec& sp, const qsgs_params* p, uint8_t* grid,
                         void* sweep, bool walls) {
    init_record(r, sp, p, grid, nullptr, nullptr, 0);
    reals[r].maps = at<uint32_t>(sweep, 0);
    reals[r].planes = at<uint64_t>(sweep, align_up(map_bytes(sp.g)));
    reals[r].pwords = plane_words(sp.g);
    reals[r].walls = walls ? 1u : 0u;
    reals[r].form = (uint32_t)p->sweep_form;
    reals[r].literal = (uint32_t)p->front_rule;
  }

  qsgs_status upload_header() {
    hdr = WsHeader{kMagic, (uint32_t)reals.size(), P.log_cap, P.reals, P.logs};
    const void* src = &hdr;
    if (stage) src = std::memcpy(st_up_hdr(), &hdr, sizeof hdr);
    QSGS_TRY(put(at<void>(ws, P.hdr), src, sizeof hdr));
    return QSGS_OK;
  }

  qsgs_status upload(size_t first, size_t n) {
    if (n == 0) return QSGS_OK;
    const void* src = reals.data() + first;
    if (stage)
      src = std::memcpy(st_up_reals() + sizeof(Real) * first, reals.data() + first,
                        sizeof(Real) * n);
    QSGS_TRY(put(args.reals + first, src, sizeof(Real) * n));
    return QSGS_OK;
  }

  qsgs_status offsets(ItemKind kind) {
    if (reals.size() == 1 && kind != kItemsPrune) return QSGS_OK;  // kernels count directly
    hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, s, args, (uint32_t)kind);
    QSGS_LAUNCHED("k_offsets");
    return QSGS_OK;
  }

  qsgs_status scan(uint32_t* data, uint32_t n, uint32_t* sums) {
    const uint32_t nb = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanBlock), 0, s, data, n, sums);
    QSGS_LAUNCHED("k_scan_local");
    if (nb > 1) {
      QSGS_TRY(scan(sums, nb, sums + nb + 1));
      hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanBlock), 0, s, data, n, sums);
      QSGS_LAUNCHED("k_scan_add");
    }
    return QSGS_OK;
  }

  // Points the seeding records `group` at a scratch region laid out by `L` (their
  // candidate lists and bucket offsets); call before uploading the records.
  void attach_scratch(const std::vector<size_t>& group, void* scratch, const SeedLayout& L) {
    uint32_t boff = 0;
    for (size_t k = 0; k < group.size(); ++k) {
      Real& R = reals[group[k]];
      // without a candidate slice the candidates (then the seeds) go to f0
      R.cand = L.cand[k] == (size_t)-1 ? R.f0 : at<int32_t>(scratch, L.cand[k]);
      R.boff = boff;
      boff += R.bk.nb;
    }
    args.counts = at<uint32_t>(scratch, L.counts);
    args.cursor = at<uint32_t>(scratch, L.cursor);
    args.sorted_v = at<int32_t>(scratch, L.sorted_v);
    args.sorted_r = at<uint32_t>(scratch, L.sorted_r);
    args.sorted_prio = at<uint64_t>(scratch, L.prio);
    args.status = at<uint8_t>(scratch, L.status);
  }

  // a1-a2 for every record in the seeding phase: candidates, spacing, seed lists.
  qsgs_status seed_core(void* scratch, const SeedLayout& L) {
    const dim3 sg(tune.seed_grid), sb(tune.seed_block);
    hipLaunchKernelGGL(k_ctl_init, dim3(16), dim3(256), 0, s, args, 1u);
    QSGS_LAUNCHED("k_ctl_init");
    QSGS_TRY(offsets(kItemsQuads));
    hipLaunchKernelGGL(k_seed_draw, sg, sb, 0, s, args);
    QSGS_LAUNCHED("k_seed_draw");
    const uint32_t tb = L.total_buckets;
    hipLaunchKernelGGL(k_fill_u32, dim3(std::min<uint32_t>(1024, tb / 256 + 1)), dim3(256), 0, s,
                       args.counts, 0u, tb + 1);
    QSGS_LAUNCHED("k_fill_u32");
    QSGS_TRY(offsets(kItemsCand));
    if (tb > 0) {
      hipLaunchKernelGGL(k_bucket_count, sg, sb, 0, s, args);
      QSGS_LAUNCHED("k_bucket_count");
      QSGS_TRY(scan(args.counts, tb + 1, at<uint32_t>(scratch, L.sums)));
      QSGS_HIP(hipMemcpyAsync(args.cursor, args.counts, sizeof(uint32_t) * (tb + 1),
                              hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL(k_bucket_scatter, sg, sb, 0, s, args, tb);
    QSGS_LAUNCHED("k_bucket_scatter");
    if (tb > 0 && async) {  // a fixed number of rounds, checked on the device
      for (uint32_t round = 0; round < kAsyncRounds; ++round) {
        hipLaunchKernelGGL(k_luby_round, sg, sb, 0, s, args, round);
        QSGS_LAUNCHED("k_luby_round");
        hipLaunchKernelGGL(k_luby_kill, sg, sb, 0, s, args);
        QSGS_LAUNCHED("k_luby_kill");
      }
      hipLaunchKernelGGL(k_seed_settled, dim3(1), dim3(256), 0, s, args, kAsyncRounds);
      QSGS_LAUNCHED("k_seed_settled");
      hipLaunchKernelGGL(k_collect_seeds, sg, sb, 0, s, args);
      QSGS_LAUNCHED("k_collect_seeds");
    } else if (tb > 0) {
      uint32_t round = 0;
      for (;;) {
        for (uint32_t k = 0; k < kRoundsPerCheck; ++k, ++round) {
          hipLaunchKernelGGL(k_luby_round, sg, sb, 0, s, args, round);
          QSGS_LAUNCHED("k_luby_round");
          hipLaunchKernelGGL(k_luby_kill, sg, sb, 0, s, args);
          QSGS_LAUNCHED("k_luby_kill");
        }
        uint32_t live = 0;
        void* dst = stage ? (void*)st_dn_live() : (void*)&live;
        QSGS_HIP(hipMemcpyAsync(dst, args.live + round - 1, sizeof live, hipMemcpyDeviceToHost, s));
        QSGS_HIP(hipStreamSynchronize(s));
        if (stage) std::memcpy(&live, st_dn_live(), sizeof live);
        if (live == 0) break;
        if (round + kRoundsPerCheck > kMaxRounds)
          return fail(QSGS_ERR_DEVICE, "seed spacing did not settle in %u rounds", kMaxRounds);
      }
      hipLaunchKernelGGL(k_collect_seeds, sg, sb, 0, s, args);
      QSGS_LAUNCHED("k_collect_seeds");
    }
    return QSGS_OK;
  }

  // a3 for the step-by-step path: F_0 = interface(G_0) into front buffer 0, step 0.
  qsgs_status seed_fronts() {
    const dim3 sg(tune.seed_grid), sb(tune.seed_block);
    QSGS_TRY(offsets(kItemsSeeds));
    hipLaunchKernelGGL(k_front_init, sg, sb, 0, s, args);
    QSGS_LAUNCHED("k_front_init");
    hipLaunchKernelGGL(k_loop_init, rgrid(), dim3(256), 0, s, args);
    QSGS_LAUNCHED("k_loop_init");
    return QSGS_OK;
  }

  // One growth step of every growing record (a4-a6).
  qsgs_status step(std::vector<hipEvent_t>* ev) {
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
    QSGS_TRY(offsets(kItemsGrow));
    if (ev) {
      e0 = prof_event();
      e1 = prof_event();
      e2 = prof_event();
      e3 = prof_event();
      QSGS_HIP(hipEventRecord(e0, s));
    }
    hipLaunchKernelGGL(k_grow, dim3(tune.grow_grid ? tune.grow_grid : 2048u),
                       dim3(tune.grow_block), 0, s, args);
    QSGS_LAUNCHED("k_grow");
    if (ev) QSGS_HIP(hipEventRecord(e1, s));
    QSGS_TRY(offsets(kItemsPrune));
    if (ev) QSGS_HIP(hipEventRecord(e2, s));
    hipLaunchKernelGGL(k_prune, dim3(tune.prune_grid), dim3(tune.prune_block), 0, s, args);
    QSGS_LAUNCHED("k_prune");
    if (ev) {
      QSGS_HIP(hipEventRecord(e3, s));
      ev->push_back(e0);
      ev->push_back(e1);
      ev->push_back(e2);
      ev->push_back(e3);
    }
    hipLaunchKernelGGL(k_step_end, rgrid(), dim3(256), 0, s, args);
    QSGS_LAUNCHED("k_step_end");
    return QSGS_OK;
  }

  qsgs_status read_bctl(BatchCtl* h) {
    void* dst = stage ? (void*)st_dn_bctl() : (void*)h;
    QSGS_HIP(hipMemcpyAsync(dst, args.bctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, s));
    QSGS_HIP(hipStreamSynchronize(s));
    if (stage) std::memcpy(h, st_dn_bctl(), sizeof(BatchCtl));
    return QSGS_OK;
  }

  // The batch control block and realization 0's loop state, with one synchronization.
  qsgs_status read_bctl_ctl0(BatchCtl* hb, Ctl* hc) {
    void* db = stage ? (void*)st_dn_bctl() : (void*)hb;
    void* dc = stage ? (void*)st_dn_ctl() : (void*)hc;
    QSGS_HIP(hipMemcpyAsync(db, args.bctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, s));
    QSGS_HIP(hipMemcpyAsync(dc, &args.reals[0].ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    QSGS_HIP(hipStreamSynchronize(s));
    if (stage) {
      std::memcpy(hb, st_dn_bctl(), sizeof(BatchCtl));
      std::memcpy(hc, st_dn_ctl(), sizeof(Ctl));
    }
    return QSGS_OK;
  }
  qsgs_status read_ctl(size_t r, Ctl* h) {
    void* dst = stage ? (void*)st_dn_ctl() : (void*)h;
    QSGS_HIP(hipMemcpyAsync(dst, &args.reals[r].ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    QSGS_HIP(hipStreamSynchronize(s));
    if (stage) std::memcpy(h, st_dn_ctl(), sizeof(Ctl));
    return QSGS_OK;
  }

  qsgs_status read_all(std::vector<Real>* out) {
    out->resize(reals.size());
    void* dst = stage ? (void*)st_dn_reals() : (void*)out->data();
    QSGS_HIP(hipMemcpyAsync(dst, args.reals, sizeof(Real) * reals.size(), hipMemcpyDeviceToHost,
                            s));
    QSGS_HIP(hipStreamSynchronize(s));
    if (stage) std::memcpy(out->data(), st_dn_reals(), sizeof(Real) * reals.size());
    return QSGS_OK;
  }

  // Loop state of the fused sweep for the freshly seeded records `group`: their first
  // tile lists (the tiles of their seeds; every tile for the all-tiles form), their
  // occupancy planes and the plan of the first pass.
  qsgs_status sweep_start(const std::vector<size_t>& group) {
    QSGS_TRY(offsets(kItemsSeeds));
    hipLaunchKernelGGL(k_seed_tiles, dim3(tune.seed_grid), dim3(tune.seed_block), 0, s, args);
    QSGS_LAUNCHED("k_seed_tiles");
    bool any_all_tiles = false;
    for (size_t r : group) any_all_tiles = any_all_tiles || reals[r].form == kFormAllTiles;
    if (any_all_tiles) {
      QSGS_TRY(offsets(kItemsVoxels));
      hipLaunchKernelGGL(k_full_tiles, dim3(tune.seed_grid), dim3(tune.seed_block), 0, s, args);
      QSGS_LAUNCHED("k_full_tiles");
    }
    QSGS_TRY(offsets(kItemsPack));
    hipLaunchKernelGGL(k_pack_planes, dim3(tune.seed_grid), dim3(tune.seed_block), 0, s, args);
    QSGS_LAUNCHED("k_pack_planes");
    hipLaunchKernelGGL(k_sweep_prepare, dim3(1), dim3(1024), 0, s, args);
    QSGS_LAUNCHED("k_sweep_prepare");
    return QSGS_OK;
  }

  // Writes the byte grid of every realization whose loop has stopped since the last
  // call, from its solid plane.
  qsgs_status export_grids() {
    QSGS_TRY(offsets(kItemsExport));
    hipLaunchKernelGGL(k_export_planes, dim3(tune.seed_grid), dim3(tune.seed_block), 0, s, args);
    QSGS_LAUNCHED("k_export_planes");
    hipLaunchKernelGGL(k_export_done, rgrid(), dim3(256), 0, s, args);
    QSGS_LAUNCHED("k_export_done");
    return QSGS_OK;
  }

  // Which passes the records need: `tiles` when a record in a tile-sweep form may still
  // be growing, `field` when one in the full-field form may.  A caller that keeps some
  // slots empty passes their records' flags as false through `live`.
  void forms_in_use(bool* tiles, bool* field, const std::vector<bool>* live = nullptr) const {
    *tiles = *field = false;
    for (size_t r = 0; r < reals.size(); ++r) {
      if (live && !(*live)[r]) continue;
      if (reals[r].form == kFormField)
        *field = true;
      else
        *tiles = true;
    }
  }

  // One pass over every record with a pending pass: the fused tile sweep (front of step t
  // and its growth; k_sweep_end ends the step) and/or the full-field step (every cell;
  // k_field_fold, then k_field_end ends the step).
  qsgs_status sweep_pass(std::vector<hipEvent_t>* ev, bool tiles = true, bool field = false) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ev) {
      e0 = prof_event();
      e1 = prof_event();
      QSGS_HIP(hipEventRecord(e0, s));
    }
    if (tiles) {
      bool walls = false, literal = false;
      for (const Real& R : reals) {
        walls = walls || R.walls != 0;
        literal = literal || R.literal != 0;
      }
      auto kernel = walls ? (literal ? k_sweep<true, true> : k_sweep<true, false>)
                          : (literal ? k_sweep<false, true> : k_sweep<false, false>);
      hipLaunchKernelGGL(kernel, dim3(sweep_grid), dim3(tune.grow_block),
                         sweep_lds_bytes(tune.grow_block), s, args);
      QSGS_LAUNCHED("k_sweep");
    }
    if (field) {
      QSGS_TRY(offsets(kItemsField));
      hipLaunchKernelGGL(k_field_step, dim3(tune.seed_grid), dim3(tune.seed_block), 0, s, args);
      QSGS_LAUNCHED("k_field_step");
    }
    if (ev) {
      QSGS_HIP(hipEventRecord(e1, s));
      ev->push_back(e0);
      ev->push_back(e1);
    }
    if (tiles) {
      hipLaunchKernelGGL(k_sweep_end, dim3(1), dim3(1024), 0, s, args);
      QSGS_LAUNCHED("k_sweep_end");
    }
    if (field) {
      hipLaunchKernelGGL(k_field_fold, dim3(tune.seed_grid), dim3(tune.seed_block), 0, s, args);
      QSGS_LAUNCHED("k_field_fold");
      hipLaunchKernelGGL(k_field_end, dim3(1), dim3(1024), 0, s, args, tiles ? 0u : 1u);
      QSGS_LAUNCHED("k_field_end");
    }
    return QSGS_OK;
  }

  // n passes.  With graphs on (and no timing events), as launches of captured chunk
  // graphs of 16, 8, 4, 2 and 1 passes; otherwise every kernel launched on its own.
  qsgs_status run_passes(uint32_t n, std::vector<hipEvent_t>* ev, bool tiles, bool field) {
    if (ev || !tune.graphs || no_events) {
      for (uint32_t k = 0; k < n; ++k) QSGS_TRY(sweep_pass(ev, tiles, field));
      return QSGS_OK;
    }
    for (uint32_t k = 16; k > 0; k >>= 1) {
      while (n >= k) {
        hipGraphExec_t g = nullptr;
        QSGS_TRY(chunk_graph(k, tiles, field, &g));
        if (g) {
          QSGS_HIP(hipGraphLaunch(g, s));
        } else {
          for (uint32_t i = 0; i < k; ++i) QSGS_TRY(sweep_pass(nullptr, tiles, field));
        }
        n -= k;
      }
    }
    return QSGS_OK;
  }

  // The cached executable graph of k passes with the current launch configuration,
  // captured on first use; *out = nullptr when no graph can be had (capture refused,
  // cache full): the caller then launches the passes directly.
  qsgs_status chunk_graph(uint32_t k, bool tiles, bool field, hipGraphExec_t* out) {
    *out = nullptr;
    bool walls = false, literal = false;
    for (const Real& R : reals) {
      walls = walls || R.walls != 0;
      literal = literal || R.literal != 0;
    }
    int dev = 0;
    QSGS_HIP(hipGetDevice(&dev));
    const uint32_t cfg[10] = {(uint32_t)dev, k, sweep_grid, tune.grow_block,
                              (uint32_t)sweep_lds_bytes(tune.grow_block), tune.seed_grid,
                              tune.seed_block,
                              (tiles ? 1u : 0u) | (field ? 2u : 0u) | (walls ? 4u : 0u) |
                                  (literal ? 8u : 0u),
                              (uint32_t)reals.size(), 0u};
    std::string key(reinterpret_cast<const char*>(cfg), sizeof cfg);
    key.append(reinterpret_cast<const char*>(&args), sizeof args);
    GraphCache& C = graph_cache();
    {
      std::lock_guard<std::mutex> lk(C.mu);
      auto it = C.exec.find(key);
      if (it != C.exec.end()) {
        *out = it->second;
        return QSGS_OK;
      }
      if (C.exec.size() >= kMaxGraphs) return QSGS_OK;
    }
    hipStream_t cs = capture_stream();
    if (!cs) return QSGS_OK;
    const hipStream_t caller = s;
    s = cs;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
      s = caller;
      (void)hipGetLastError();
      return QSGS_OK;
    }
    qsgs_status st = QSGS_OK;
    for (uint32_t i = 0; i < k && st == QSGS_OK; ++i) st = sweep_pass(nullptr, tiles, field);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    s = caller;
    if (st != QSGS_OK || ec != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      last_error().clear();
      return QSGS_OK;  // launch directly instead
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess || !ex) {
      (void)hipGetLastError();
      return QSGS_OK;
    }
    std::lock_guard<std::mutex> lk(C.mu);
    auto it = C.exec.find(key);
    if (it != C.exec.end()) {  // another thread captured the same chunk meanwhile
      (void)hipGraphExecDestroy(ex);
      *out = it->second;
      return QSGS_OK;
    }
    if (C.exec.size() >= kMaxGraphs) {
      (void)hipGraphExecDestroy(ex);  // never launched
      return QSGS_OK;
    }
    C.exec.emplace(key, ex);
    *out = ex;
    return QSGS_OK;
  }

  // The sweep loop without host reads: `passes` passes (those after every record has
  // stopped find nothing to do), launched one by one.
  qsgs_status run_sweep_fixed(uint32_t passes) {
    bool tiles = false, field = false;
    forms_in_use(&tiles, &field);
    for (uint32_t k = 0; k < passes; ++k) QSGS_TRY(sweep_pass(nullptr, tiles, field));
    return QSGS_OK;
  }

  // Fused-sweep loop until every record has stopped.  A realization takes steps + 1
  // passes (the last one only prunes and folds).  For a single realization the chunk
  // length follows the remaining count over the last step's growth, plus the final pass
  // (passes after the stop find nothing to do and cost two empty launches, less than a
  // round trip to the host).
  qsgs_status run_sweep_loop() {
    bool tiles = false, field = false;
    forms_in_use(&tiles, &field);
    const bool profiling = prof_on() && !no_events;
    std::vector<hipEvent_t> ev;
    BatchCtl b{};
    Ctl c{};
    const bool single = tune.steps_per_sync <= 0 && reals.size() == 1;
    auto read_state = [&]() { return single ? read_bctl_ctl0(&b, &c) : read_bctl(&b); };
    QSGS_TRY(read_state());
    while (b.running > 0) {
      uint32_t chunk = tune.steps_per_sync > 0 ? (uint32_t)tune.steps_per_sync : 8u;
      if (single) {
        chunk = 16;
        if (c.mode == kModeFinal)
          chunk = 1;
        else if (c.step > 0 && c.last_new > 0)
          chunk = (uint32_t)std::max<uint64_t>(
              1, std::min<uint64_t>(16, (c.s_star - c.cnt) / c.last_new + 2));
        else if (c.step > 0)
          chunk = 4;
      }
      QSGS_TRY(run_passes(chunk, profiling ? &ev : nullptr, tiles, field));
      QSGS_TRY(read_state());
    }
    if (profiling && !ev.empty()) {
      std::vector<Real> fin;
      QSGS_TRY(read_all(&fin));
      size_t active = 0;
      for (const Real& R : fin) active = std::max(active, (size_t)R.ctl.step + 1);
      const size_t n = std::min(active, ev.size() / 2);
      double ms_total = 0;
      for (size_t i = 0; i < n; ++i) {
        float a = 0.f;
        QSGS_HIP(hipEventElapsedTime(&a, ev[2 * i], ev[2 * i + 1]));
        ms_total += a;
      }
      std::lock_guard<std::mutex> lk(prof().mu);
      prof().grow_launches += (double)n;
      prof().grow_ms += ms_total;
    }
    return QSGS_OK;
  }

  // Accumulates the durations of the first `active` timed steps.
  qsgs_status record_profile(const std::vector<hipEvent_t>& ev, size_t active) {
    double grow_ms = 0, prune_ms = 0;
    const size_t n = std::min(active, ev.size() / 4);
    for (size_t i = 0; i < n; ++i) {
      float a = 0.f, c = 0.f;
      QSGS_HIP(hipEventElapsedTime(&a, ev[4 * i], ev[4 * i + 1]));
      QSGS_HIP(hipEventElapsedTime(&c, ev[4 * i + 2], ev[4 * i + 3]));
      grow_ms += a;
      prune_ms += c;
    }
    std::lock_guard<std::mutex> lk(prof().mu);
    prof().grow_launches += (double)n;
    prof().grow_ms += grow_ms;
    prof().prune_launches += (double)n;
    prof().prune_ms += prune_ms;
    return QSGS_OK;
  }
};

}  // namespace host
}  // namespace qsgs
