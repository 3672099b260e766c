// qsgs_api.hip -- host side of libqsgs: the C ABI declared in include/qsgs.h.
//
// Validates arguments, computes the integer constants of the path (T_seed, T_ref,
// S*), lays out the caller's workspace, enqueues the kernels and drives the growth
// loop in chunks of steps with one control-block read per chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qsgs.h"
#include "qsgs_internal.h"

using namespace qsgs;

namespace {

thread_local std::string g_last_error;

qsgs_status fail(qsgs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define QSGS_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(QSGS_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));       \
  } while (0)

#define QSGS_LAUNCHED(what)                                                              \
  do {                                                                                   \
    hipError_t e_ = hipGetLastError();                                                   \
    if (e_ != hipSuccess)                                                                \
      return fail(QSGS_ERR_DEVICE, "launch of %s failed: %s", what, hipGetErrorString(e_)); \
  } while (0)

constexpr uint32_t kGrid = 2048;  // persistent grid for list kernels: 8 XCDs x 256
constexpr size_t kAlign = 256;
constexpr int32_t kDefaultMaxSteps = 1 << 20;
constexpr uint32_t kRoundsPerCheck = 8;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ----- integer constants (Sec. 2.1 step 2, Sec. 2.3 step 5, Eq. (1)) -----

// min(2^32, floor(p 2^32)); p * 2^32 is exact in binary64.
uint64_t prob_threshold(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return kOne32;
  return (uint64_t)std::floor(p * 4294967296.0);
}

// S* = ceil(phi_s N) evaluated in binary64, clamped to [0, N].
uint64_t target_count(double phi_s, uint64_t n) {
  double t = std::ceil(phi_s * (double)n);
  if (t < 0.0) t = 0.0;
  if (t > (double)n) t = (double)n;
  return (uint64_t)t;
}

bool is_prob(double p) { return std::isfinite(p) && p >= 0.0 && p <= 1.0; }

qsgs_status check_dims(const qsgs_dims* d, Geometry* g) {
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

qsgs_status check_params(const qsgs_params* p) {
  if (!p) return fail(QSGS_ERR_INVALID, "params is NULL");
  if (!(std::isfinite(p->solid_fraction) && p->solid_fraction > 0.0 && p->solid_fraction <= 1.0))
    return fail(QSGS_ERR_INVALID, "solid_fraction must be in (0, 1]");
  if (!is_prob(p->seed_prob)) return fail(QSGS_ERR_INVALID, "seed_prob must be in [0, 1]");
  for (int c = 0; c < 3; ++c)
    if (!is_prob(p->g_ref[c])) return fail(QSGS_ERR_INVALID, "g_ref[%d] must be in [0, 1]", c);
  if (p->spacing < 0) return fail(QSGS_ERR_INVALID, "spacing must be >= 0");
  return QSGS_OK;
}

Buckets make_buckets(const Geometry& g, int32_t spacing) {
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

// Workspace layout for qsgs_seed / qsgs_generate.  The front lists of the growth
// loop reuse the seeding regions: r1 holds the candidates, then the seed list, then
// front buffer 0; r2 holds the bucket-sorted candidates, then front buffer 1.
struct Layout {
  size_t ctl, live, log, r1, r2, prio, status, counts, cursor, sums, total;
  uint32_t scan_levels[4];
  uint32_t n_levels;
};

Layout make_layout(const Geometry& g, const Buckets& b) {
  Layout L{};
  size_t off = 0;
  L.ctl = off;
  off = align_up(off + sizeof(Ctl));
  L.live = off;
  off = align_up(off + sizeof(uint32_t) * kMaxRounds);
  L.log = off;
  off = align_up(off + sizeof(uint64_t) * 3 * kLogCap);
  L.r1 = off;
  off = align_up(off + sizeof(int32_t) * (size_t)g.n);
  L.r2 = off;
  off = align_up(off + sizeof(int32_t) * (size_t)g.n);
  L.prio = off;
  off = align_up(off + sizeof(uint64_t) * (size_t)g.n);
  L.status = off;
  off = align_up(off + (size_t)g.n);
  const uint32_t nscan = b.nb ? b.nb + 1 : 0;
  L.counts = off;
  off = align_up(off + sizeof(uint32_t) * nscan);
  L.cursor = off;
  off = align_up(off + sizeof(uint32_t) * nscan);
  L.sums = off;
  L.n_levels = 0;
  size_t sums = 0;
  for (uint32_t m = nscan; m > 1 && L.n_levels < 4;) {
    m = (m + kScanBlock - 1) / kScanBlock;
    L.scan_levels[L.n_levels++] = m;
    sums += m;
  }
  off = align_up(off + sizeof(uint32_t) * (sums + 8));
  L.total = off;
  return L;
}

constexpr size_t kStepWorkspace = 64 * 1024;

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// ----- profiling -----
struct Profile {
  std::mutex mu;
  bool enabled = false;
  double grow_launches = 0, grow_ms = 0, prune_launches = 0, prune_ms = 0, seed_ms = 0;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
};
Profile g_prof;

bool prof_on() {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  return g_prof.enabled;
}

hipEvent_t prof_event() {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (g_prof.used == g_prof.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_prof.pool.push_back(e);
  }
  return g_prof.pool[g_prof.used++];
}

void prof_release_all() {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.used = 0;
}

// ----- pieces of the path -----

qsgs_status scan_exclusive(uint32_t* data, uint32_t n, uint32_t* sums, hipStream_t s) {
  // Recursive scan: per-block scans, a scan of the block totals, then the add-back.
  const uint32_t nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanBlock), 0, s, data, n, sums);
  QSGS_LAUNCHED("k_scan_local");
  if (nb > 1) {
    qsgs_status st = scan_exclusive(sums, nb, sums + nb + 1, s);
    if (st != QSGS_OK) return st;
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanBlock), 0, s, data, n, sums);
    QSGS_LAUNCHED("k_scan_add");
  }
  return QSGS_OK;
}

// a1 + a2: candidates, spacing and the seed list (left in the r1 region).
qsgs_status run_seeding(const Geometry& g, const qsgs_params* p, uint8_t* grid, void* ws,
                        const Layout& L, const Buckets& bk, hipStream_t s) {
  Ctl* ctl = at<Ctl>(ws, L.ctl);
  const uint32_t k0 = (uint32_t)p->key, k1 = (uint32_t)(p->key >> 32);
  int32_t* r1 = at<int32_t>(ws, L.r1);
  SeedArgs sa{g, grid, r1, ctl, prob_threshold(p->seed_prob), k0, k1};
  hipLaunchKernelGGL(k_seed_draw, dim3(kGrid), dim3(kBlock), 0, s, sa);
  QSGS_LAUNCHED("k_seed_draw");
  if (p->spacing <= 1) {
    MarkArgs ma{grid, r1, ctl};
    hipLaunchKernelGGL(k_mark_all_seeds, dim3(kGrid), dim3(kBlock), 0, s, ma);
    QSGS_LAUNCHED("k_mark_all_seeds");
    return QSGS_OK;
  }
  BucketArgs ba{};
  ba.g = g;
  ba.bk = bk;
  ba.cand = r1;
  ba.counts = at<uint32_t>(ws, L.counts);
  ba.cursor = at<uint32_t>(ws, L.cursor);
  ba.offsets = ba.counts;
  ba.sorted_v = at<int32_t>(ws, L.r2);
  ba.sorted_prio = at<uint64_t>(ws, L.prio);
  ba.status = at<uint8_t>(ws, L.status);
  ba.live = at<uint32_t>(ws, L.live);
  ba.ctl = ctl;
  ba.k0 = k0;
  ba.k1 = k1;
  const uint32_t nscan = bk.nb + 1;
  hipLaunchKernelGGL(k_fill_u32, dim3(256), dim3(kBlock), 0, s, ba.counts, 0u, nscan);
  QSGS_LAUNCHED("k_fill_u32");
  hipLaunchKernelGGL(k_bucket_count, dim3(kGrid), dim3(kBlock), 0, s, ba);
  QSGS_LAUNCHED("k_bucket_count");
  qsgs_status st = scan_exclusive(ba.counts, nscan, at<uint32_t>(ws, L.sums), s);
  if (st != QSGS_OK) return st;
  QSGS_HIP(hipMemcpyAsync(ba.cursor, ba.counts, sizeof(uint32_t) * nscan,
                          hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_bucket_scatter, dim3(kGrid), dim3(kBlock), 0, s, ba);
  QSGS_LAUNCHED("k_bucket_scatter");
  uint32_t round = 0;
  for (;;) {
    for (uint32_t k = 0; k < kRoundsPerCheck; ++k, ++round) {
      hipLaunchKernelGGL(k_luby_round, dim3(kGrid), dim3(kBlock), 0, s, ba, round);
      QSGS_LAUNCHED("k_luby_round");
    }
    uint32_t live = 0;
    QSGS_HIP(hipMemcpyAsync(&live, ba.live + round - 1, sizeof live, hipMemcpyDeviceToHost, s));
    QSGS_HIP(hipStreamSynchronize(s));
    if (live == 0) break;
    if (round + kRoundsPerCheck > kMaxRounds)
      return fail(QSGS_ERR_DEVICE, "seed spacing did not settle in %u rounds", kMaxRounds);
  }
  hipLaunchKernelGGL(k_collect_seeds, dim3(kGrid), dim3(kBlock), 0, s, ba, r1, grid);
  QSGS_LAUNCHED("k_collect_seeds");
  return QSGS_OK;
}

qsgs_status read_ctl(const Ctl* d_ctl, Ctl* h, hipStream_t s) {
  QSGS_HIP(hipMemcpyAsync(h, d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  QSGS_HIP(hipStreamSynchronize(s));
  return QSGS_OK;
}

void fill_info(const Ctl& c, qsgs_info* info) {
  info->n_candidates = c.n_cand;
  info->n_seeds = c.n_seeds;
  info->solid_count = (int64_t)c.cnt;
  info->target_count = (int64_t)c.s_star;
  info->front_size = c.front_size;
  info->grown_last_step = c.last_new;
  info->step = c.step;
  info->status = c.status;
}

qsgs_status common_checks(const qsgs_dims* dims, const qsgs_params* params, const uint8_t* grid,
                          Geometry* g) {
  qsgs_status st = check_dims(dims, g);
  if (st != QSGS_OK) return st;
  st = check_params(params);
  if (st != QSGS_OK) return st;
  if (!grid) return fail(QSGS_ERR_INVALID, "d_grid is NULL");
  if ((uintptr_t)grid % 4 != 0) return fail(QSGS_ERR_INVALID, "d_grid must be 4-byte aligned");
  return QSGS_OK;
}

CtlInit make_init(const Geometry& g, const qsgs_params* p) {
  CtlInit init{};
  init.s_star = target_count(p->solid_fraction, g.n);
  for (int c = 0; c < 3; ++c) init.t_ref[c] = prob_threshold(p->g_ref[c]);
  init.max_steps = p->max_steps > 0 ? p->max_steps : kDefaultMaxSteps;
  return init;
}

}  // namespace

extern "C" {

size_t qsgs_grid_bytes(const qsgs_dims* dims) {
  Geometry g{};
  if (check_dims(dims, &g) != QSGS_OK) return 0;
  return ((size_t)g.n + 3) / 4 * 4;
}

size_t qsgs_workspace_bytes(const qsgs_dims* dims, const qsgs_params* params) {
  Geometry g{};
  if (check_dims(dims, &g) != QSGS_OK || check_params(params) != QSGS_OK) return 0;
  return make_layout(g, make_buckets(g, params->spacing)).total;
}

size_t qsgs_step_workspace_bytes(void) { return kStepWorkspace; }

qsgs_status qsgs_seed(const qsgs_dims* dims, const qsgs_params* params, uint8_t* d_grid,
                      int32_t* d_front, int64_t front_cap, void* d_ws, size_t ws_bytes,
                      qsgs_info* info, void* stream) {
  g_last_error.clear();
  Geometry g{};
  qsgs_status st = common_checks(dims, params, d_grid, &g);
  if (st != QSGS_OK) return st;
  if (!d_front || front_cap < 0) return fail(QSGS_ERR_INVALID, "bad d_front / front_cap");
  if (!d_ws || !info) return fail(QSGS_ERR_INVALID, "d_ws and info must not be NULL");
  const Buckets bk = make_buckets(g, params->spacing);
  const Layout L = make_layout(g, bk);
  if (ws_bytes < L.total)
    return fail(QSGS_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", L.total, ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  Ctl* ctl = at<Ctl>(d_ws, L.ctl);
  CtlInit init = make_init(g, params);
  hipLaunchKernelGGL(k_ctl_init, dim3(16), dim3(kBlock), 0, s, ctl, init, at<uint32_t>(d_ws, L.live),
                     kMaxRounds);
  QSGS_LAUNCHED("k_ctl_init");
  st = run_seeding(g, params, d_grid, d_ws, L, bk, s);
  if (st != QSGS_OK) return st;
  const uint32_t cap = (uint32_t)std::min<int64_t>(front_cap, (int64_t)UINT32_MAX);
  FrontInitArgs fa{g, d_grid, at<int32_t>(d_ws, L.r1), d_front, cap, ctl};
  hipLaunchKernelGGL(k_front_init, dim3(kGrid), dim3(kBlock), 0, s, fa);
  QSGS_LAUNCHED("k_front_init");
  hipLaunchKernelGGL(k_loop_init, dim3(1), dim3(1), 0, s, ctl, 0u);
  QSGS_LAUNCHED("k_loop_init");
  Ctl h{};
  st = read_ctl(ctl, &h, s);
  if (st != QSGS_OK) return st;
  if (h.overflow)
    return fail(QSGS_ERR_CAPACITY, "initial front needs more than front_cap = %lld entries",
                (long long)front_cap);
  fill_info(h, info);
  return QSGS_OK;
}

qsgs_status qsgs_grow_step(const qsgs_dims* dims, const qsgs_params* params, uint8_t* d_grid,
                           int32_t* d_front_in, int32_t* d_front_out, int64_t front_cap,
                           void* d_ws, size_t ws_bytes, qsgs_info* info, void* stream) {
  g_last_error.clear();
  Geometry g{};
  qsgs_status st = common_checks(dims, params, d_grid, &g);
  if (st != QSGS_OK) return st;
  if (!d_front_in || !d_front_out || d_front_in == d_front_out || front_cap < 0)
    return fail(QSGS_ERR_INVALID, "bad front buffers / front_cap");
  if (!d_ws || !info) return fail(QSGS_ERR_INVALID, "d_ws and info must not be NULL");
  if (ws_bytes < kStepWorkspace)
    return fail(QSGS_ERR_WORKSPACE, "step workspace needs %zu bytes, got %zu", kStepWorkspace,
                ws_bytes);
  if (info->front_size < 0 || info->front_size > front_cap || info->solid_count < 0 ||
      info->solid_count > (int64_t)g.n || info->step < 0)
    return fail(QSGS_ERR_INVALID, "info does not describe a valid state");
  if (info->status >= QSGS_DONE && info->status <= QSGS_MAXSTEPS) return (qsgs_status)info->status;
  hipStream_t s = (hipStream_t)stream;
  Ctl* ctl = at<Ctl>(d_ws, 0);
  CtlInit init = make_init(g, params);
  init.cnt = (uint64_t)info->solid_count;
  init.front_size = (uint32_t)info->front_size;
  init.cur = 0;
  init.step = info->step;
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl, init, (uint32_t*)nullptr, 0u);
  QSGS_LAUNCHED("k_ctl_init");
  hipLaunchKernelGGL(k_loop_resume, dim3(1), dim3(1), 0, s, ctl);
  QSGS_LAUNCHED("k_loop_resume");
  const uint32_t cap = (uint32_t)std::min<int64_t>(front_cap, (int64_t)UINT32_MAX);
  StepArgs sa{g, d_grid, d_front_in, d_front_out, cap, ctl, (uint32_t)params->key,
              (uint32_t)(params->key >> 32)};
  hipLaunchKernelGGL(k_grow, dim3(kGrid), dim3(kBlock), 0, s, sa);
  QSGS_LAUNCHED("k_grow");
  hipLaunchKernelGGL(k_prune, dim3(kGrid), dim3(kBlock), 0, s, sa);
  QSGS_LAUNCHED("k_prune");
  hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, s, ctl, (uint64_t*)nullptr, 0u);
  QSGS_LAUNCHED("k_step_end");
  Ctl h{};
  st = read_ctl(ctl, &h, s);
  if (st != QSGS_OK) return st;
  if (h.bad_entry) return fail(QSGS_ERR_INVALID, "front entry outside the grid");
  if (h.status == kStatusOverflow) {
    hipLaunchKernelGGL(k_rollback, dim3(kGrid), dim3(kBlock), 0, s, d_grid, g.n);
    QSGS_LAUNCHED("k_rollback");
    QSGS_HIP(hipStreamSynchronize(s));
    return fail(QSGS_ERR_CAPACITY, "front would exceed front_cap = %lld entries",
                (long long)front_cap);
  }
  const int32_t before = info->step;
  const int64_t n_seeds = info->n_seeds, n_cand = info->n_candidates;
  fill_info(h, info);
  info->n_seeds = n_seeds;
  info->n_candidates = n_cand;
  (void)before;
  return (qsgs_status)h.status;
}

qsgs_status qsgs_generate(const qsgs_dims* dims, const qsgs_params* params, uint8_t* d_grid,
                          void* d_ws, size_t ws_bytes, qsgs_info* info, void* stream) {
  g_last_error.clear();
  Geometry g{};
  qsgs_status st = common_checks(dims, params, d_grid, &g);
  if (st != QSGS_OK) return st;
  if (!d_ws || !info) return fail(QSGS_ERR_INVALID, "d_ws and info must not be NULL");
  const Buckets bk = make_buckets(g, params->spacing);
  const Layout L = make_layout(g, bk);
  if (ws_bytes < L.total)
    return fail(QSGS_ERR_WORKSPACE, "workspace needs %zu bytes, got %zu", L.total, ws_bytes);
  hipStream_t s = (hipStream_t)stream;
  const bool prof = prof_on();
  hipEvent_t seed_beg = nullptr, seed_end = nullptr;
  if (prof) {
    prof_release_all();
    seed_beg = prof_event();
    seed_end = prof_event();
    QSGS_HIP(hipEventRecord(seed_beg, s));
  }
  Ctl* ctl = at<Ctl>(d_ws, L.ctl);
  CtlInit init = make_init(g, params);
  hipLaunchKernelGGL(k_ctl_init, dim3(16), dim3(kBlock), 0, s, ctl, init,
                     at<uint32_t>(d_ws, L.live), kMaxRounds);
  QSGS_LAUNCHED("k_ctl_init");
  st = run_seeding(g, params, d_grid, d_ws, L, bk, s);
  if (st != QSGS_OK) return st;
  int32_t* f0 = at<int32_t>(d_ws, L.r1);
  int32_t* f1 = at<int32_t>(d_ws, L.r2);
  FrontInitArgs fa{g, d_grid, f0, f1, g.n, ctl};
  hipLaunchKernelGGL(k_front_init, dim3(kGrid), dim3(kBlock), 0, s, fa);
  QSGS_LAUNCHED("k_front_init");
  hipLaunchKernelGGL(k_loop_init, dim3(1), dim3(1), 0, s, ctl, 1u);
  QSGS_LAUNCHED("k_loop_init");
  if (prof) QSGS_HIP(hipEventRecord(seed_end, s));

  StepArgs sa{g, d_grid, f0, f1, g.n, ctl, (uint32_t)params->key, (uint32_t)(params->key >> 32)};
  uint64_t* log = at<uint64_t>(d_ws, L.log);
  std::vector<hipEvent_t> ev;  // per launched step: grow begin/end, prune end
  Ctl h{};
  st = read_ctl(ctl, &h, s);
  if (st != QSGS_OK) return st;
  while (h.status == 0) {
    // Steps per chunk: the remaining count over the last step's growth bounds the
    // steps left while growth slows down, so chunks rarely run past the end.
    uint32_t chunk = 16;
    if (h.step > 0 && h.last_new > 0) {
      const uint64_t left = h.s_star - h.cnt;
      chunk = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(16, left / h.last_new));
    } else if (h.step > 0) {
      chunk = 4;
    }
    for (uint32_t k = 0; k < chunk; ++k) {
      hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
      if (prof) {
        e0 = prof_event();
        e1 = prof_event();
        e2 = prof_event();
        QSGS_HIP(hipEventRecord(e0, s));
      }
      hipLaunchKernelGGL(k_grow, dim3(kGrid), dim3(kBlock), 0, s, sa);
      QSGS_LAUNCHED("k_grow");
      if (prof) QSGS_HIP(hipEventRecord(e1, s));
      hipLaunchKernelGGL(k_prune, dim3(kGrid), dim3(kBlock), 0, s, sa);
      QSGS_LAUNCHED("k_prune");
      if (prof) QSGS_HIP(hipEventRecord(e2, s));
      hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, s, ctl, log, kLogCap);
      QSGS_LAUNCHED("k_step_end");
      if (prof) {
        ev.push_back(e0);
        ev.push_back(e1);
        ev.push_back(e2);
      }
    }
    st = read_ctl(ctl, &h, s);
    if (st != QSGS_OK) return st;
  }
  if (h.status == kStatusOverflow || h.bad_entry)
    return fail(QSGS_ERR_DEVICE, "internal front overflow");
  if (prof) {
    float ms = 0.f;
    QSGS_HIP(hipEventElapsedTime(&ms, seed_beg, seed_end));
    double grow_ms = 0, prune_ms = 0;
    const size_t active = std::min<size_t>((size_t)h.step, ev.size() / 3);
    for (size_t i = 0; i < active; ++i) {
      float a = 0.f, b = 0.f;
      QSGS_HIP(hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]));
      QSGS_HIP(hipEventElapsedTime(&b, ev[3 * i + 1], ev[3 * i + 2]));
      grow_ms += a;
      prune_ms += b;
    }
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.seed_ms += ms;
    g_prof.grow_launches += (double)active;
    g_prof.grow_ms += grow_ms;
    g_prof.prune_launches += (double)active;
    g_prof.prune_ms += prune_ms;
  }
  fill_info(h, info);
  return (qsgs_status)h.status;
}

int64_t qsgs_read_step_log(const void* d_ws, size_t ws_bytes, int64_t* front, int64_t* grown,
                           int64_t* count, int64_t max_entries, void* stream) {
  g_last_error.clear();
  if (!d_ws) return fail(QSGS_ERR_INVALID, "d_ws is NULL");
  // The control block and the log sit at the same offsets for every size.
  const Geometry g0{1, 1, 1, 1, 1, {}, {}};
  const Layout L = make_layout(g0, Buckets{});
  if (ws_bytes < L.log + sizeof(uint64_t) * 3 * kLogCap)
    return fail(QSGS_ERR_WORKSPACE, "workspace too small to hold a step log");
  hipStream_t s = (hipStream_t)stream;
  Ctl h{};
  qsgs_status st = read_ctl(reinterpret_cast<const Ctl*>(static_cast<const char*>(d_ws) + L.ctl),
                            &h, s);
  if (st != QSGS_OK) return st;
  int64_t n = std::min<int64_t>({(int64_t)h.step, max_entries, (int64_t)kLogCap});
  if (n <= 0) return 0;
  std::vector<uint64_t> buf(3 * (size_t)n);
  QSGS_HIP(hipMemcpyAsync(buf.data(), static_cast<const char*>(d_ws) + L.log,
                          sizeof(uint64_t) * buf.size(), hipMemcpyDeviceToHost, s));
  QSGS_HIP(hipStreamSynchronize(s));
  for (int64_t t = 0; t < n; ++t) {
    if (front) front[t] = (int64_t)buf[3 * t];
    if (grown) grown[t] = (int64_t)buf[3 * t + 1];
    if (count) count[t] = (int64_t)buf[3 * t + 2];
  }
  return n;
}

void qsgs_profile_enable(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.enabled = enable != 0;
}

void qsgs_profile_read(double out[5], int32_t reset) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  out[0] = g_prof.grow_launches;
  out[1] = g_prof.grow_ms;
  out[2] = g_prof.prune_launches;
  out[3] = g_prof.prune_ms;
  out[4] = g_prof.seed_ms;
  if (reset) {
    g_prof.grow_launches = g_prof.grow_ms = g_prof.prune_launches = g_prof.prune_ms = 0;
    g_prof.seed_ms = 0;
  }
}

const char* qsgs_last_error(void) { return g_last_error.c_str(); }

const char* qsgs_version(void) { return "qsgs 0.1.0 gfx950"; }

}  // extern "C"
