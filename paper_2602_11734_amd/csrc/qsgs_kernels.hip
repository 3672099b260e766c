// qsgs_kernels.hip -- gfx950 kernels of libqsgs: seeding (Sec. 2.1 step 2), diamond
// seed spacing (Sec. 2.3, Fig. 1D), the list-indexed growth sweep and front
// compaction (Sec. 2.3 steps 2-5, Algorithm 3) with the thresholds of Eq. (1).
//
// All kernels serve a batch of realizations.  Item kernels walk an offset table in
// wavefront-sized chunks; each chunk belongs to one realization, whose record is
// read with scalar loads.  The item range is cut into 8 contiguous parts, one per
// XCD, so neighbouring front entries (neighbouring voxels) share one XCD's L2.
#include "qsgs_internal.h"

namespace qsgs {

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

__device__ __forceinline__ uint32_t atomic_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Items of one realization for an offset table of the given kind.
__device__ __forceinline__ uint64_t items_of(const Real& R, uint32_t kind) {
  const Ctl& c = R.ctl;
  const bool seeding = R.phase == kPhaseSeed;
  const bool growing = R.phase == kPhaseGrow && c.status == 0;
  switch (kind) {
    case kItemsVoxels: return seeding ? R.g.n : 0;
    case kItemsCand: return seeding ? c.n_cand : 0;
    case kItemsSeeds: return seeding ? c.n_seeds : 0;
    case kItemsGrow: return growing ? c.front_size : 0;
    case kItemsPrune:
      return (growing && !c.overflow) ? (uint64_t)c.front_size + c.new_count : 0;
    default: return (growing && c.mode != kModeIdle) ? c.n_list : 0;
  }
}

// Calls body(r, local) for every chunk of kWave items; `local` is this lane's index in
// realization r's (padded) item range.  A batch walks the offset table; a single
// realization takes its item count directly.  The chunk range is cut into 8
// contiguous parts, one per XCD, so neighbouring list entries share one XCD's L2.
template <typename Body>
__device__ __forceinline__ void for_each_chunk(const BatchArgs& A, uint32_t kind, Body&& body) {
  const bool single = A.count == 1;
  const uint64_t total = single ? (items_of(A.reals[0], kind) + kWave - 1) / kWave * kWave
                                : uniform64(A.off[A.count]);
  const uint64_t nchunks = total / kWave;
  const uint32_t wib = uniform(threadIdx.x / kWave);
  const uint32_t wpb = blockDim.x / kWave;
  const uint32_t xcd = blockIdx.x % kNumXcd;
  const uint64_t per = (nchunks + kNumXcd - 1) / kNumXcd;
  const uint64_t c_beg = min(nchunks, (uint64_t)xcd * per);
  const uint64_t c_end = min(nchunks, c_beg + per);
  const uint64_t stride = (uint64_t)(gridDim.x / kNumXcd) * wpb;
  uint32_t r = 0;
  uint64_t lo = 0, hi = single ? total : 0;
  for (uint64_t c = c_beg + (uint64_t)(blockIdx.x / kNumXcd) * wpb + wib; c < c_end; c += stride) {
    const uint64_t item0 = c * kWave;
    if (item0 < lo || item0 >= hi) {
      uint32_t a = 0, b = A.count;  // largest r with off[r] <= item0
      while (b - a > 1) {
        const uint32_t mid = (a + b) >> 1;
        if (uniform64(A.off[mid]) <= item0) a = mid; else b = mid;
      }
      r = a;
      lo = uniform64(A.off[r]);
      hi = uniform64(A.off[r + 1]);
    }
    body(r, (uint32_t)(item0 - lo) + lane_id());
  }
}

// ---------------------------------------------------------------------------
// Neighbourhood of one voxel.  Each of the nine rows (dy, dz) of the 3x3x3 block
// around (x, y, z) is read with one 8-byte load; off-grid neighbours do not exist
// (the domain is not periodic).  `mark` is the value voxels grown during the current step carry.
// Bit d of `voidm` is set for an in-domain neighbour that was void at the step's
// start (value 0 or `mark`), bit d of `grown` for one already grown during this step
// (value `mark`), bit d of `zero` for value 0.
// ---------------------------------------------------------------------------
struct Nbhd {
  uint32_t voidm, grown, zero;
};

// Global-address-space views of device pointers that live in memory (so loads are
// emitted as global rather than flat memory instructions).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gptr(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// Eight grid bytes from the dword-aligned address at or below p (p >= 0); the grid
// buffer carries 8 bytes of padding, so the window never leaves it.
__device__ __forceinline__ uint64_t window8(const uint8_t* __restrict__ grid, int32_t p) {
  const auto* w = gptr(reinterpret_cast<const uint32_t*>(grid + (p & ~3)));
  return (uint64_t)w[0] | ((uint64_t)w[1] << 32);
}

__device__ __forceinline__ Nbhd load_neighbourhood(const uint8_t* __restrict__ grid,
                                                   const Geometry& g, uint32_t a, uint32_t x,
                                                   uint32_t y, uint32_t z,
                                                   uint8_t mark = kGrown) {
  const bool xm = x > 0, xp = x + 1 < (uint32_t)g.nx;
  const bool ym = y > 0, yp = y + 1 < (uint32_t)g.ny;
  const bool zm = z > 0, zp = z + 1 < (uint32_t)g.nz;
  // All nine row windows are loaded unconditionally so that they are in flight
  // together; a row outside the domain reads the voxel's own row and is masked below.
  uint64_t w[9];
  int32_t sh[9];
  bool rin[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int dz = k / 3 - 1, dy = k % 3 - 1;
    rin[k] = (dz < 0 ? zm : (dz > 0 ? zp : true)) && (dy < 0 ? ym : (dy > 0 ? yp : true));
    const int32_t p = (int32_t)a - 1 + (rin[k] ? dy * g.nx + dz * (int32_t)g.nxy : 0);
    const int32_t pa = p < 0 ? 0 : p;
    sh[k] = (p - (pa & ~3)) * 8;  // -8 only for p = -1
    w[k] = window8(grid, pa);
  }
  Nbhd r{0u, 0u, 0u};
  int d = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    // bytes x-1, x, x+1 of the row
    const uint32_t bytes3 = sh[k] >= 0 ? (uint32_t)(w[k] >> sh[k]) : (uint32_t)(w[k] << 8);
    const int dz = k / 3 - 1, dy = k % 3 - 1;
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      if (dx == 0 && dy == 0 && dz == 0) continue;
      const bool in = rin[k] && (dx < 0 ? xm : (dx > 0 ? xp : true));
      const uint32_t b = (bytes3 >> (8 * (dx + 1))) & 0xFFu;
      r.voidm |= (uint32_t)(in && (b == kVoid || b == mark)) << d;
      r.grown |= (uint32_t)(in && b == mark) << d;
      r.zero |= (uint32_t)(in && b == kVoid) << d;
      ++d;
    }
  }
  return r;
}

__device__ __forceinline__ int32_t dir_offset(const Geometry& g, int d) {
  return (dir_field(kDirDX, d) - 1) + (dir_field(kDirDY, d) - 1) * g.nx +
         (dir_field(kDirDZ, d) - 1) * (int32_t)g.nxy;
}

__device__ __forceinline__ void coords_of(const Geometry& g, uint32_t v, uint32_t& x, uint32_t& y,
                                          uint32_t& z) {
  const uint32_t yz = g.div_nx.div(v);
  x = v - yz * (uint32_t)g.nx;
  z = g.div_ny.div(yz);
  y = yz - z * (uint32_t)g.ny;
}

__device__ __forceinline__ uint32_t bucket_of(const Buckets& bk, uint32_t x, uint32_t y,
                                              uint32_t z) {
  return bk.edge.div(x) + bk.nbx * (bk.edge.div(y) + bk.nby * bk.edge.div(z));
}

// ---------------------------------------------------------------------------
// Set-up.
// ---------------------------------------------------------------------------
__global__ void k_ctl_init(BatchArgs A, uint32_t zero_live) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nthr = gridDim.x * blockDim.x;
  if (tid == 0) {
    A.bctl->running = 0;
    A.bctl->n_sorted = 0;
    A.bctl->blocks_done = 0;
  }
  if (zero_live)
    for (uint32_t i = tid; i < kMaxRounds; i += nthr) A.live[i] = 0;
}

// Offset table: each realization's item count of the given kind, rounded up to a
// multiple of kWave, exclusive-scanned by one workgroup (up to 1024 threads).
__device__ void block_offsets(const BatchArgs& A, uint32_t kind) {
  __shared__ uint64_t wave_tot[1024 / kWave];
  __shared__ uint64_t carry;
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < A.count; base += blockDim.x) {
    const uint32_t r = base + threadIdx.x;
    uint64_t v = 0;
    if (r < A.count) v = (items_of(A.reals[r], kind) + kWave - 1) / kWave * kWave;
    uint64_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint64_t t = __shfl_up(incl, o, kWave);
      if (lane >= (uint32_t)o) incl += t;
    }
    if (lane == kWave - 1) wave_tot[wv] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t acc = carry;
      for (uint32_t w = 0; w < nw; ++w) {
        const uint64_t t = wave_tot[w];
        wave_tot[w] = acc;
        acc += t;
      }
      carry = acc;
    }
    __syncthreads();
    if (r < A.count) A.off[r] = wave_tot[wv] + incl - v;
    __syncthreads();
  }
  if (threadIdx.x == 0) A.off[A.count] = carry;
  __syncthreads();
}

// The prune table also restarts the count of running realizations that k_step_end
// accumulates.
__global__ __launch_bounds__(1024) void k_offsets(BatchArgs A, uint32_t kind) {
  if (kind == kItemsPrune && threadIdx.x == 0) A.bctl->running = 0;
  block_offsets(A, kind);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = value;
}

// Exclusive scan, kScanBlock items per workgroup; each workgroup also writes its total.
__global__ __launch_bounds__(kScanBlock) void k_scan_local(uint32_t* data, uint32_t n,
                                                           uint32_t* sums) {
  __shared__ uint32_t wave_tot[kScanBlock / kWave];
  const uint32_t i = blockIdx.x * kScanBlock + threadIdx.x;
  const uint32_t v = i < n ? data[i] : 0u;
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, kWave);
    if (lane >= (uint32_t)off) incl += t;
  }
  if (lane == kWave - 1) wave_tot[wv] = incl;
  __syncthreads();
  if (wv == 0) {
    const uint32_t t = lane < kScanBlock / kWave ? wave_tot[lane] : 0u;
    uint32_t ti = t;
#pragma unroll
    for (int off = 1; off < kScanBlock / kWave; off <<= 1) {
      const uint32_t u = __shfl_up(ti, off, kWave);
      if (lane >= (uint32_t)off) ti += u;
    }
    if (lane < kScanBlock / kWave) wave_tot[lane] = ti - t;  // exclusive wave offsets
    if (lane == kScanBlock / kWave - 1) sums[blockIdx.x] = ti;
  }
  __syncthreads();
  if (i < n) data[i] = incl - v + wave_tot[wv];
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(uint32_t* data, uint32_t n,
                                                         const uint32_t* sums) {
  const uint32_t i = blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) data[i] += sums[blockIdx.x];
}

// ---------------------------------------------------------------------------
// a1: seed candidates (items: voxels).  Voxel v draws the block at (v, 0, 0, 1);
// word 0 below T_seed makes it a candidate (Sec. 2.1 step 2).  The grid is zeroed
// in the same pass; candidates are appended with one atomic per wavefront.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBlock) void k_seed_draw(BatchArgs A) {
  for_each_chunk(A, kItemsVoxels, [&](uint32_t r, uint32_t v) {
    Real& R = A.reals[r];
    bool cand = false;
    if (v < R.g.n) {
      const U4 w = philox10(v, 0u, 0u, kTagSeed, R.k0, R.k1);
      cand = (uint64_t)w.x < R.t_seed;
      R.grid[v] = kVoid;
    }
    const uint32_t pos = wave_append_flag(cand, &R.ctl.n_cand);
    if (cand) R.cand[pos] = (int32_t)v;  // capacity N: cannot overflow
  });
}

// ---------------------------------------------------------------------------
// a2: diamond spacing.  Candidates of a realization with s >= 2 are bucketed by
// (x, y, z) / (s - 1) into that realization's slice of the batch's bucket arrays;
// every conflict (L1 distance 1..s-1) lies in the 27 surrounding buckets.
// Without spacing (s <= 1) every candidate becomes a seed directly.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBlock) void k_bucket_count(BatchArgs A) {
  for_each_chunk(A, kItemsCand, [&](uint32_t r, uint32_t i) {
    const Real& R = A.reals[r];
    if (i < R.ctl.n_cand && R.bk.nb != 0) {
      uint32_t x, y, z;
      coords_of(R.g, (uint32_t)R.cand[i], x, y, z);
      atomicAdd(&A.counts[R.boff + bucket_of(R.bk, x, y, z)], 1u);
    }
  });
}

__global__ __launch_bounds__(kMaxBlock) void k_bucket_scatter(BatchArgs A, uint32_t total_buckets) {
  if (blockIdx.x == 0 && threadIdx.x == 0) A.bctl->n_sorted = A.counts[total_buckets];
  for_each_chunk(A, kItemsCand, [&](uint32_t r, uint32_t i) {
    Real& R = A.reals[r];
    if (i >= R.ctl.n_cand) return;
    const uint32_t v = (uint32_t)R.cand[i];
    if (R.bk.nb == 0) {  // no spacing: the candidate list is the seed list
      R.grid[v] = kSolid;
      if (i == 0) R.ctl.n_seeds = R.ctl.n_cand;
      return;
    }
    uint32_t x, y, z;
    coords_of(R.g, v, x, y, z);
    const uint32_t pos = atomicAdd(&A.cursor[R.boff + bucket_of(R.bk, x, y, z)], 1u);
    const U4 w = philox10(v, 0u, 0u, kTagSeed, R.k0, R.k1);
    A.sorted_v[pos] = (int32_t)v;
    A.sorted_r[pos] = r;
    A.sorted_prio[pos] = ((uint64_t)w.y << 32) | (uint64_t)w.z;
    A.status[pos] = kLive;
  });
}

// One priority round over all bucket-sorted candidates.  A live candidate that sees
// an accepted conflicting candidate dies; one whose key (priority, v) is below every
// live conflicting candidate's key is accepted.  Statuses only move forward, and a
// stale read can only delay a decision, never change it, so in-place updates
// reproduce the greedy acceptance in ascending key order.
__global__ __launch_bounds__(kMaxBlock) void k_luby_round(BatchArgs A, uint32_t round) {
  const uint32_t n = A.bctl->n_sorted;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    bool still_live = false;
    if (i < n && A.status[i] == kLive) {
      const Real& R = A.reals[A.sorted_r[i]];
      const Buckets bk = R.bk;
      const uint32_t v = (uint32_t)A.sorted_v[i];
      const uint64_t p = A.sorted_prio[i];
      uint32_t x, y, z;
      coords_of(R.g, v, x, y, z);
      const int32_t bx = (int32_t)bk.edge.div(x), by = (int32_t)bk.edge.div(y),
                    bz = (int32_t)bk.edge.div(z);
      bool killed = false, minimal = true;
      for (int32_t cz = max(bz - 1, 0); cz <= min(bz + 1, (int32_t)bk.nbz - 1) && !killed; ++cz)
        for (int32_t cy = max(by - 1, 0); cy <= min(by + 1, (int32_t)bk.nby - 1) && !killed; ++cy)
          for (int32_t cx = max(bx - 1, 0); cx <= min(bx + 1, (int32_t)bk.nbx - 1) && !killed;
               ++cx) {
            const uint32_t b =
                R.boff + (uint32_t)cx + bk.nbx * ((uint32_t)cy + bk.nby * (uint32_t)cz);
            const uint32_t e = A.counts[b + 1];
            for (uint32_t j = A.counts[b]; j < e; ++j) {
              if (j == i) continue;
              const uint32_t w = (uint32_t)A.sorted_v[j];
              uint32_t wx, wy, wz;
              coords_of(R.g, w, wx, wy, wz);
              const int32_t dist = abs((int32_t)wx - (int32_t)x) + abs((int32_t)wy - (int32_t)y) +
                                   abs((int32_t)wz - (int32_t)z);
              if (dist > bk.radius) continue;
              const uint8_t st = A.status[j];
              if (st == kAccepted) {
                killed = true;
                break;
              }
              if (st == kLive) {
                const uint64_t q = A.sorted_prio[j];
                if (q < p || (q == p && w < v)) minimal = false;
              }
            }
          }
      if (killed)
        A.status[i] = kDead;
      else if (minimal)
        A.status[i] = kAccepted;
      else
        still_live = true;
    }
    wave_append_flag(still_live, &A.live[round]);
  }
}

// Accepted candidates become seeds: 1 in the grid, appended to the realization's
// seed list (which reuses its candidate list).
__global__ __launch_bounds__(kMaxBlock) void k_collect_seeds(BatchArgs A) {
  const uint32_t n = A.bctl->n_sorted;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (A.status[i] != kAccepted) continue;
    Real& R = A.reals[A.sorted_r[i]];
    const int32_t v = A.sorted_v[i];
    R.grid[v] = kSolid;
    R.cand[atomicAdd(&R.ctl.n_seeds, 1u)] = v;
  }
}

// ---------------------------------------------------------------------------
// a3: initial front F_0 = interface(G_0) (Sec. 2.3 step 2), compacted from the seed
// list into front buffer 0; then the loop state for step 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBlock) void k_front_init(BatchArgs A) {
  for_each_chunk(A, kItemsSeeds, [&](uint32_t r, uint32_t i) {
    Real& R = A.reals[r];
    bool keep = false;
    uint32_t v = 0;
    if (i < R.ctl.n_seeds) {
      v = (uint32_t)R.cand[i];
      uint32_t x, y, z;
      coords_of(R.g, v, x, y, z);
      keep = load_neighbourhood(R.grid, R.g, v, x, y, z).zero != 0;
    }
    const uint32_t pos = wave_append_flag(keep, &R.ctl.out_count);
    if (keep) {
      if (pos < R.cap)
        R.f0[pos] = (int32_t)v;
      else
        R.ctl.overflow = 1u;
    }
  });
}

__device__ __forceinline__ void set_status_and_thresholds(Ctl& c) {
  int32_t status = 0;
  if (c.cnt >= c.s_star)
    status = kStatusDone;
  else if (c.front_size == 0)
    status = kStatusExhausted;
  else if (c.step >= c.max_steps)
    status = kStatusMaxSteps;
  c.status = status;
  if (status == 0)
    for (int k = 0; k < 3; ++k) c.T[k] = eq1_threshold(c.t_ref[k], c.cnt, c.s_star);
}

__global__ void k_loop_init(BatchArgs A) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= A.count || A.reals[r].phase != kPhaseSeed) return;
  A.reals[r].phase = kPhaseGrow;
  Ctl& c = A.reals[r].ctl;
  if (c.overflow) {
    c.status = kStatusOverflow;
    return;
  }
  c.cnt = c.n_seeds;
  c.front_size = c.out_count;
  c.out_count = 0;
  c.new_count = 0;
  c.step = 0;
  c.cur = 0;
  set_status_and_thresholds(c);
  if (c.status == 0) atomicAdd(&A.bctl->running, 1u);
}

// Loop state supplied by the host (qsgs_grow_step): status and thresholds only.
__global__ void k_loop_resume(BatchArgs A) {
  Ctl& c = A.reals[0].ctl;
  set_status_and_thresholds(c);
}

// Draws of source voxel a at step t (Sec. 2.3 step 3; the draw rule is stated in qsgs.h):
// its in-domain void neighbours (at the step's start) take the draws of ranks
// j = 0, 1, ... in ascending direction; a passing draw claims the neighbour with a
// 32-bit atomicOr that writes `mark` into its grid byte.  Returns the directions this
// thread claimed first (the neighbour was still 0).
__device__ __forceinline__ uint32_t grow_draws(const Real& R, const Geometry& g, uint32_t a,
                                               uint32_t t, const Nbhd& nb, uint64_t T0,
                                               uint64_t T1, uint64_t T2, uint8_t mark) {
  uint32_t claims = 0;
  uint32_t m = nb.voidm;
  uint32_t j = 0;
  int32_t hi_block = -1, lo_block = -1;
  U4 H{0, 0, 0, 0}, L{0, 0, 0, 0};
  while (m) {
    const int d = __builtin_ctz(m);
    m &= m - 1u;
    if (!((nb.grown >> d) & 1u)) {  // a target already grown this step needs no draw
      const int32_t blk = (int32_t)(j >> 3);
      if (blk != hi_block) {
        H = philox10(a, t, (uint32_t)blk, kTagGrowHi, R.k0, R.k1);
        hi_block = blk;
      }
      const uint32_t wh = pick(H, (j >> 1) & 3u);
      const uint32_t h = (j & 1u) ? (wh >> 16) : (wh & 0xFFFFu);
      const int cls = dir_field(kDirClass, d);
      const uint64_t Tc = cls == 0 ? T0 : (cls == 1 ? T1 : T2);
      const uint32_t th = (uint32_t)(Tc >> 16);  // 65536 when Tc = 2^32
      bool pass = h < th;
      if (h == th) {  // high halves tie: decide on the low halves
        if (blk != lo_block) {
          L = philox10(a, t, (uint32_t)blk, kTagGrowLo, R.k0, R.k1);
          lo_block = blk;
        }
        const uint32_t wl = pick(L, (j >> 1) & 3u);
        const uint32_t l = (j & 1u) ? (wl >> 16) : (wl & 0xFFFFu);
        pass = l < (uint32_t)(Tc & 0xFFFFu);
      }
      if (pass) {
        const uint32_t q = (uint32_t)((int32_t)a + dir_offset(g, d));
        const uint32_t sh = (q & 3u) * 8u;
        const uint32_t old = atomicOr((uint32_t*)(R.grid + (q & ~3u)), (uint32_t)mark << sh);
        if (((old >> sh) & 0xFFu) == kVoid) claims |= 1u << d;
      }
    }
    ++j;
  }
  return claims;
}

// ---------------------------------------------------------------------------
// a4: growth sweep of step t (items: F_t of running realizations).  One thread per
// front voxel a: its in-domain void neighbours (at the step's start) take the draws
// of ranks j = 0, 1, ... in ascending direction; a passing draw claims the
// neighbour with a 32-bit atomicOr on the grid word (value 2 = grown this step),
// and the first claimer appends it after F_t in the same list.  Sources are F_t
// only (Jacobi step).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBlock) void k_grow(BatchArgs A) {
  for_each_chunk(A, kItemsGrow, [&](uint32_t r, uint32_t i) {
    Real& R = A.reals[r];
    Ctl& c = R.ctl;
    const uint32_t t = (uint32_t)c.step;
    const uint32_t nf = c.front_size;
    int32_t* __restrict__ fin = c.cur ? R.f1 : R.f0;
    const Geometry g = R.g;
    uint32_t a = 0, claims = 0;
    if (i < nf) {
      a = (uint32_t)fin[i];
      if (a >= g.n) {
        c.bad_entry = 1u;
      } else {
        const uint64_t T0 = c.T[0], T1 = c.T[1], T2 = c.T[2];
        uint32_t x, y, z;
        coords_of(g, a, x, y, z);
        const Nbhd nb = load_neighbourhood(R.grid, g, a, x, y, z);
        claims = grow_draws(R, g, a, t, nb, T0, T1, T2, kGrown);
      }
    }
    uint32_t pos = wave_append((uint32_t)__builtin_popcount(claims), &c.new_count);
    while (claims) {
      const int d = __builtin_ctz(claims);
      claims &= claims - 1u;
      const uint32_t slot = nf + pos;
      if (slot < R.cap)
        fin[slot] = (int32_t)((int32_t)a + dir_offset(g, d));
      else
        c.overflow = 1u;
      ++pos;
    }
  });
}

// ---------------------------------------------------------------------------
// a5: prune and compaction (Sec. 2.3 step 4), items: F_t + New_t.  F_{t+1} = the
// entries that still have an in-domain void neighbour, appended with one atomic per
// wavefront.  New voxels are folded from 2 to 1 here.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBlock) void k_prune(BatchArgs A) {
  for_each_chunk(A, kItemsPrune, [&](uint32_t r, uint32_t i) {
    Real& R = A.reals[r];
    Ctl& c = R.ctl;
    const uint32_t nf = c.front_size;
    const uint32_t n_in = nf + c.new_count;
    const int32_t* __restrict__ fin = c.cur ? R.f1 : R.f0;
    int32_t* __restrict__ fout = c.cur ? R.f0 : R.f1;
    const Geometry g = R.g;
    bool keep = false;
    uint32_t v = 0;
    if (i < n_in) {
      v = (uint32_t)fin[i];
      if (v < g.n) {
        uint32_t x, y, z;
        coords_of(g, v, x, y, z);
        keep = load_neighbourhood(R.grid, g, v, x, y, z).zero != 0;
        if (i >= nf) R.grid[v] = kSolid;
      }
    }
    const uint32_t pos = wave_append_flag(keep, &c.out_count);
    if (keep) {
      if (pos < R.cap)
        fout[pos] = (int32_t)v;
      else
        c.overflow = 1u;
    }
  });
}

// ---------------------------------------------------------------------------
// a6: end of step t, one thread per realization: log, count update, front swap,
// loop status and the thresholds of step t+1 from the new count (Eq. (1)).
// ---------------------------------------------------------------------------
__global__ void k_step_end(BatchArgs A) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= A.count) return;
  Real& R = A.reals[r];
  Ctl& c = R.ctl;
  if (R.phase != kPhaseGrow || c.status != 0) return;
  if (c.overflow) {
    c.status = kStatusOverflow;
    return;
  }
  const uint32_t t = (uint32_t)c.step;
  const uint32_t grown = c.new_count;
  if (R.log && t < R.log_cap) {
    R.log[3 * (uint64_t)t + 0] = c.front_size;
    R.log[3 * (uint64_t)t + 1] = grown;
    R.log[3 * (uint64_t)t + 2] = c.cnt;
  }
  c.cnt += grown;
  c.last_new = grown;
  c.front_size = c.out_count;
  c.out_count = 0;
  c.new_count = 0;
  c.cur ^= 1u;
  c.step = (int32_t)t + 1;
  set_status_and_thresholds(c);
  if (c.status == 0) atomicAdd(&A.bctl->running, 1u);
}

// Undo a step that overflowed its front capacity: grown voxels (2) back to void.
__global__ __launch_bounds__(kBlock) void k_rollback(uint8_t* grid, uint32_t n) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    if (grid[v] == kGrown) grid[v] = kVoid;
}


// ---------------------------------------------------------------------------
// Fused sweep (qsgs_generate*, server).  One pass over L_t = F_{t-1} + New_{t-1}
// does the prune of step t-1 and the growth of step t, which read the same
// neighbourhoods (the state at the start of step t): entries flagged new are folded
// from the previous step's mark to 1, entries with an in-domain void neighbour form
// F_t, and in a running pass each of them draws for its void neighbours.  Voxels
// grown in step t carry mark 2 + (t & 1), so marks of consecutive steps differ.
//
// Output without contended atomics: every active realization r gets G_r workgroups;
// workgroup k reads the k-th equal share of r's chunks (through the segment table of
// the input plan) and appends L_{t+1} entries to the k-th part of r's other list
// buffer with an LDS counter.  Its part's fill and its kept count go to per-workgroup
// slots; a part that fills up spills into the second half of the buffer through r's
// tail counter.  The last workgroup to finish (ticket) ends the step for every
// realization (a6: log, count, status, Eq. (1) thresholds of the next step) and
// builds the next plan.
// ---------------------------------------------------------------------------

// Block-wide exclusive scan of n values val(i), handing out(i, prefix); returns the
// total.  Every thread of the block calls it; blockDim.x <= 1024.
template <typename Val, typename Out>
__device__ uint32_t block_scan_u32(uint32_t n, Val val, Out out) {
  __shared__ uint32_t wt[1024 / kWave];
  __shared__ uint32_t carry;
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < n; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < n ? val(i) : 0u;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o, kWave);
      if (lane >= (uint32_t)o) incl += t;
    }
    if (lane == kWave - 1) wt[wv] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t acc = carry;
      for (uint32_t w = 0; w < nw; ++w) {
        const uint32_t t = wt[w];
        wt[w] = acc;
        acc += t;
      }
      carry = acc;
    }
    __syncthreads();
    if (i < n) out(i, wt[wv] + incl - v);
    __syncthreads();
  }
  const uint32_t total = carry;
  __syncthreads();
  return total;
}

__device__ __forceinline__ bool sweep_active(const Real& R) {
  return R.phase == kPhaseGrow && R.ctl.status == 0 && R.ctl.mode != kModeIdle;
}

// Chunk prefix and workgroup assignment of plan q, whose segment table and
// realization ranges are complete.  G_r = max(1, floor((G - B) n_r / n)) for an
// active realization with n_r > 0 chunks (B of them, n chunks in all), so that
// sum G_r <= G.  One workgroup.
__device__ void plan_assign(const BatchArgs& A, uint32_t q) {
  const SweepPlan& P = A.plan[q];
  const uint32_t S = P.rseg[A.count];
  const uint32_t chunks = block_scan_u32(
      S, [&](uint32_t i) { return (atomic_load(&P.seg[i].fill) + kWave - 1) / (uint32_t)kWave; },
      [&](uint32_t i, uint32_t x) { P.segchunk[i] = x; });
  if (threadIdx.x == 0) P.segchunk[S] = chunks;
  __syncthreads();
  auto nch = [&](uint32_t r) -> uint32_t {
    return sweep_active(A.reals[r]) ? P.segchunk[P.rseg[r + 1]] - P.segchunk[P.rseg[r]] : 0u;
  };
  const uint32_t total = block_scan_u32(A.count, nch, [](uint32_t, uint32_t) {});
  const uint32_t busy = block_scan_u32(
      A.count, [&](uint32_t r) { return nch(r) > 0 ? 1u : 0u; }, [](uint32_t, uint32_t) {});
  const uint64_t avail = (uint64_t)A.bctl->grid - busy;
  const uint32_t nwg = block_scan_u32(
      A.count,
      [&](uint32_t r) -> uint32_t {
        const uint32_t n = nch(r);
        if (n == 0) return 0u;
        return (uint32_t)max<uint64_t>(1, avail * n / total);
      },
      [&](uint32_t r, uint32_t x) { P.wgoff[r] = x; });
  if (threadIdx.x == 0) P.wgoff[A.count] = nwg;
  __syncthreads();
}

// Loop state of step 0 for every freshly seeded realization (L_0 = its seed list,
// at the start of list buffer 0), and the input plan of the next pass: realizations
// already growing keep their segments, new ones get one segment, finished ones none.
// One workgroup.
__global__ __launch_bounds__(1024) void k_sweep_prepare(BatchArgs A) {
  const uint32_t qi = A.bctl->plan, qo = qi ^ 1u;
  const SweepPlan& I = A.plan[qi];
  const SweepPlan& O = A.plan[qo];
  if (threadIdx.x == 0) {
    A.bctl->blocks_done = 0;
    A.bctl->running = 0;
  }
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < A.count; r += blockDim.x) {
    Real& R = A.reals[r];
    if (R.phase != kPhaseSeed) continue;
    R.phase = kPhaseGrow;
    Ctl& c = R.ctl;
    c.cnt = c.n_seeds;
    c.n_list = c.n_seeds;
    c.cur = 0;
    c.step = 0;
    c.kept = 0;
    c.out_count = 0;
    c.new_count = 0;
    c.front_size = 0;
    c.status = c.overflow ? kStatusOverflow : 0;
    c.mode = kModeIdle;
    if (c.status == 0) {
      if (c.cnt < c.s_star && c.max_steps > 0) {
        c.mode = kModeRun;
        for (int k = 0; k < 3; ++k) c.T[k] = eq1_threshold(c.t_ref[k], c.cnt, c.s_star);
      } else {
        c.mode = kModeFinal;
      }
      c.bad_entry = 0;
      c.last_new = 0;
      // mark as new for the table rebuild below (seed lists need no fold)
      c.pad0 = 1;
    }
  }
  __syncthreads();
  auto entries = [&](uint32_t r) -> uint32_t {
    const Real& R = A.reals[r];
    if (!sweep_active(R)) return 0u;
    return R.ctl.pad0 ? 1u : I.rseg[r + 1] - I.rseg[r];
  };
  const uint32_t S = block_scan_u32(A.count, entries,
                                    [&](uint32_t r, uint32_t x) { O.rseg[r] = x; });
  if (threadIdx.x == 0) O.rseg[A.count] = S;
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < A.count; r += blockDim.x) {
    Real& R = A.reals[r];
    if (!sweep_active(R)) continue;
    atomicAdd(&A.bctl->running, 1u);
    uint32_t o = O.rseg[r];
    if (R.ctl.pad0) {
      O.seg[o] = SegEntry{r, 0u, R.ctl.n_list, 0u};
      R.ctl.pad0 = 0;
    } else {
      for (uint32_t e = I.rseg[r]; e < I.rseg[r + 1]; ++e) O.seg[o++] = I.seg[e];
    }
  }
  __syncthreads();
  plan_assign(A, qo);
  if (threadIdx.x == 0) A.bctl->plan = qo;
}

// End of a pass for realization r: kept = |F_t|, out = |L_{t+1}|.
__device__ void sweep_end(const BatchArgs& A, uint32_t r, uint32_t kept, uint32_t out) {
  Real& R = A.reals[r];
  Ctl& c = R.ctl;
  const uint32_t bad = atomic_load(&c.overflow) | atomic_load(&c.bad_entry);
  if (bad) {
    c.status = kStatusOverflow;
    c.mode = kModeIdle;
    return;
  }
  const uint32_t grown = out - kept;
  c.front_size = kept;
  c.n_list = out;
  c.cur ^= 1u;
  if (c.mode == kModeRun && kept > 0) {
    const uint32_t t = (uint32_t)c.step;
    if (R.log && t < R.log_cap) {
      R.log[3 * (uint64_t)t + 0] = kept;
      R.log[3 * (uint64_t)t + 1] = grown;
      R.log[3 * (uint64_t)t + 2] = c.cnt;
    }
    c.cnt += grown;
    c.last_new = grown;
    c.step = (int32_t)t + 1;
    if (c.cnt < c.s_star && c.step < c.max_steps) {
      for (int k = 0; k < 3; ++k) c.T[k] = eq1_threshold(c.t_ref[k], c.cnt, c.s_star);
    } else {
      c.mode = kModeFinal;  // one more pass: fold this step's marks, report F_T
    }
    atomicAdd(&A.bctl->running, 1u);
  } else {
    // a final pass, or a running pass that found F_t empty: the loop has stopped
    c.status = c.cnt >= c.s_star ? kStatusDone : (kept == 0 ? kStatusExhausted : kStatusMaxSteps);
    c.mode = kModeIdle;
  }
}

// Wave-wide exclusive prefix of cnt; *total receives the wave's sum.
__device__ __forceinline__ uint32_t wave_prefix(uint32_t cnt, uint32_t* total) {
  const uint32_t lane = lane_id();
  uint32_t incl = cnt;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t v = __shfl_up(incl, off, kWave);
    if (lane >= (uint32_t)off) incl += v;
  }
  *total = __shfl(incl, kWave - 1, kWave);
  return incl - cnt;
}

__global__ __launch_bounds__(kMaxBlock) void k_sweep(BatchArgs A) {
  __shared__ uint32_t s_fill, s_commit, s_kept;
  const uint32_t G = gridDim.x;
  const uint32_t p = uniform(A.bctl->plan);
  const SweepPlan& P = A.plan[p];
  const SweepPlan& Q = A.plan[p ^ 1u];
  // logical workgroup index: XCD x (workgroups b with b % 8 == x) holds [x G/8, (x+1) G/8)
  const uint32_t beta = (blockIdx.x % kNumXcd) * (G / kNumXcd) + blockIdx.x / kNumXcd;
  const uint32_t nwg = uniform(P.wgoff[A.count]);
  if (threadIdx.x == 0) {
    s_fill = 0;
    s_commit = 0;
    s_kept = 0;
  }
  __syncthreads();
  uint32_t r = 0, k = 0, part_base = 0;
  if (beta < nwg) {
    uint32_t a = 0, b = A.count;  // largest r with wgoff[r] <= beta
    while (b - a > 1) {
      const uint32_t mid = (a + b) >> 1;
      if (uniform(P.wgoff[mid]) <= beta) a = mid; else b = mid;
    }
    r = a;
    k = beta - uniform(P.wgoff[r]);
    const uint32_t Gr = uniform(P.wgoff[r + 1]) - uniform(P.wgoff[r]);
    Real& R = A.reals[r];
    Ctl& c = R.ctl;
    const Geometry g = R.g;
    const uint32_t sb = uniform(P.rseg[r]), se = uniform(P.rseg[r + 1]);
    const uint32_t ch0 = uniform(P.segchunk[sb]);
    const uint64_t nch = uniform(P.segchunk[se]) - ch0;
    const uint32_t c_lo = ch0 + (uint32_t)(nch * k / Gr);
    const uint32_t c_hi = ch0 + (uint32_t)(nch * (k + 1) / Gr);
    const uint64_t half = g.n;
    part_base = (uint32_t)(half * k / Gr);
    const uint32_t part_cap = (uint32_t)(half * (k + 1) / Gr) - part_base;
    const uint32_t t = (uint32_t)c.step;
    const bool run = c.mode == kModeRun;
    const uint8_t mark = (uint8_t)(kGrown + (t & 1u));
    const uint64_t T0 = c.T[0], T1 = c.T[1], T2 = c.T[2];
    const int32_t* __restrict__ lin = c.cur ? R.f1 : R.f0;
    int32_t* __restrict__ lout = c.cur ? R.f0 : R.f1;
    const uint32_t wib = uniform(threadIdx.x / kWave), wpb = blockDim.x / kWave;
    uint32_t s = sb;
    if (c_lo + wib < c_hi) {  // first segment of this wave: largest s with segchunk[s] <= chunk
      uint32_t a = sb, b = se;
      while (b - a > 1) {
        const uint32_t mid = (a + b) >> 1;
        if (uniform(P.segchunk[mid]) <= c_lo + wib) a = mid; else b = mid;
      }
      s = a;
    }
    for (uint32_t ch = c_lo + wib; ch < c_hi; ch += wpb) {
      while (uniform(P.segchunk[s + 1]) <= ch) ++s;
      const SegEntry seg = P.seg[s];
      const uint32_t idx = (ch - uniform(P.segchunk[s])) * kWave + lane_id();
      uint32_t v = 0, claims = 0;
      bool keep = false;
      if (idx < seg.fill) {
        const uint32_t raw = (uint32_t)lin[seg.base + idx];
        v = raw & ~kNewFlag;
        if (v >= g.n) {
          atomicOr(&c.bad_entry, 1u);
        } else {
          if (raw & kNewFlag) R.grid[v] = kSolid;  // grown last step: fold its mark
          uint32_t x, y, z;
          coords_of(g, v, x, y, z);
          const Nbhd nb = load_neighbourhood(R.grid, g, v, x, y, z, mark);
          keep = nb.voidm != 0;
          if (keep && run) claims = grow_draws(R, g, v, t, nb, T0, T1, T2, mark);
        }
      }
      const uint32_t cnt = (keep ? 1u : 0u) + (uint32_t)__builtin_popcount(claims);
      uint32_t total = 0;
      uint32_t pos = wave_prefix(cnt, &total);
      const uint64_t kmask = __ballot(keep);
      uint32_t dst = 0;
      if (lane_id() == kWave - 1 && total) {
        const uint32_t base = atomicAdd(&s_fill, total);
        if (base + total <= part_cap) {
          atomicMax(&s_commit, base + total);
          dst = part_base + base;
        } else {  // the part is full: spill into the tail half
          const uint32_t tb = atomicAdd(&A.tailfill[r], total);
          if (tb + total <= g.n)
            dst = g.n + tb;
          else
            dst = 0xFFFFFFFFu;
        }
      }
      if (lane_id() == 0 && kmask) atomicAdd(&s_kept, (uint32_t)__popcll(kmask));
      dst = __shfl(dst, kWave - 1, kWave);
      if (dst == 0xFFFFFFFFu) {
        if (cnt) atomicOr(&c.overflow, 1u);
        continue;
      }
      pos += dst;
      if (keep) lout[pos++] = (int32_t)v;
      while (claims) {
        const int d = __builtin_ctz(claims);
        claims &= claims - 1u;
        lout[pos++] = (int32_t)((uint32_t)((int32_t)v + dir_offset(g, d)) | kNewFlag);
      }
    }
  }
  __syncthreads();
  if (beta < nwg && threadIdx.x == 0) {
    Q.seg[P.wgoff[r] + r + k] = SegEntry{r, part_base, s_commit, 0u};
    A.wgkept[beta] = s_kept;
  }
}

// End of a fused pass (one workgroup of 1024 threads, launched after k_sweep): sums
// every workgroup's kept count and part fill per realization in LDS, writes the tail
// segments, ends the step for every active realization (a6: log, count, status,
// Eq. (1) thresholds of the next step) and builds the next plan.
__global__ __launch_bounds__(1024) void k_sweep_end(BatchArgs A) {
  __shared__ uint32_t acc_kept[kMaxBatch];
  __shared__ uint32_t acc_out[kMaxBatch];
  const uint32_t p = A.bctl->plan;
  const SweepPlan& P = A.plan[p];
  const SweepPlan& Q = A.plan[p ^ 1u];
  for (uint32_t r = threadIdx.x; r < A.count; r += blockDim.x) {
    acc_kept[r] = 0;
    acc_out[r] = A.tailfill[r];
  }
  if (threadIdx.x == 0) A.bctl->running = 0;
  __syncthreads();
  const uint32_t nwg = P.wgoff[A.count];
  for (uint32_t w = threadIdx.x; w < nwg; w += blockDim.x) {
    uint32_t a = 0, b = A.count;  // realization of logical workgroup w
    while (b - a > 1) {
      const uint32_t mid = (a + b) >> 1;
      if (P.wgoff[mid] <= w) a = mid; else b = mid;
    }
    atomicAdd(&acc_kept[a], A.wgkept[w]);
    atomicAdd(&acc_out[a], Q.seg[w + a].fill);
  }
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < A.count; r += blockDim.x) {
    const uint32_t w0 = P.wgoff[r], w1 = P.wgoff[r + 1];
    Q.seg[w1 + r] = SegEntry{r, A.reals[r].g.n, A.tailfill[r], 0u};
    A.tailfill[r] = 0;
    Q.rseg[r] = w0 + r;
    if (sweep_active(A.reals[r])) sweep_end(A, r, acc_kept[r], acc_out[r]);
  }
  if (threadIdx.x == 0) Q.rseg[A.count] = nwg + A.count;
  __syncthreads();
  plan_assign(A, p ^ 1u);
  if (threadIdx.x == 0) A.bctl->plan = p ^ 1u;
}

}  // namespace qsgs
