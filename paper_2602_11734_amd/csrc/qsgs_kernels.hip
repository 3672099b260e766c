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

// Global and LDS views of generic pointers.  A generic (flat) access counts against both
// the vector-memory and the LDS wait counters, so every later wait for an LDS access
// would also wait for it; the fused sweep keeps its global stores and atomics in flight
// across LDS work, so it makes them global accesses, and its LDS reads LDS ones.
typedef __attribute__((address_space(1))) uint8_t g_u8;
typedef __attribute__((address_space(1))) int32_t g_i32;
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) uint64_t g_u64;
typedef __attribute__((address_space(3))) uint32_t l_u32;
__device__ __forceinline__ uint32_t global_or(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_or((g_u32*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// (the old value unused: a fire-and-forget atomic)
__device__ __forceinline__ void global_or_nr(uint32_t* p, uint32_t v) {
  (void)__hip_atomic_fetch_or((g_u32*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Items of one realization for an offset table of the given kind.
__device__ __forceinline__ uint64_t items_of(const Real& R, uint32_t kind) {
  const Ctl& c = R.ctl;
  const bool seeding = R.phase == kPhaseSeed;
  const bool growing = R.phase == kPhaseGrow && c.status == 0;
  switch (kind) {
    case kItemsVoxels: return seeding ? R.g.n : 0;
    case kItemsQuads: return seeding ? (R.g.n + 3u) / 4u : 0;
    case kItemsCand: return seeding ? c.n_cand : 0;
    case kItemsSeeds: return seeding ? c.n_seeds : 0;
    case kItemsGrow: return growing ? c.front_size : 0;
    case kItemsPrune:
      return (growing && !c.overflow) ? (uint64_t)c.front_size + c.new_count : 0;
    case kItemsPack: return (seeding && R.planes) ? R.pwords : 0;
    case kItemsExport: return (R.phase == kPhaseGrow && c.export_state == 1u) ? R.pwords : 0;
    case kItemsField:
      return (growing && R.form == kFormField && c.mode != kModeIdle) ? R.pwords : 0;
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
  const uint32_t incl = wave_incl_sum(v);
  if (lane == kWave - 1) wave_tot[wv] = incl;
  __syncthreads();
  if (wv == 0) {
    const uint32_t t = lane < kScanBlock / kWave ? wave_tot[lane] : 0u;
    const uint32_t ti = wave_incl_sum(t);
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

// Wave-wide exclusive prefix of cnt; *total receives the wave's sum.
__device__ __forceinline__ uint32_t wave_prefix(uint32_t cnt, uint32_t* total) {
  const uint32_t incl = wave_incl_sum(cnt);
  *total = __builtin_amdgcn_readlane(incl, kWave - 1);
  return incl - cnt;
}

// Orders LDS accesses of the lanes of one wavefront (a wave executes in lockstep; this
// keeps the compiler from moving LDS accesses across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// a1: seed candidates (items: voxels).  Voxel v draws the block at (v, 0, 0, 1);
// word 0 below T_seed makes it a candidate (Sec. 2.1 step 2).  The grid is zeroed
// in the same pass; candidates are buffered per wavefront in LDS and appended in bulk.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBlock) void k_seed_draw(BatchArgs A) {
  // the record's fields, read once per realization (the byte stores below could alias
  // the record, which would otherwise force a reload of every field per chunk)
  // (pointers are made wave-uniform so that they sit in scalar registers: a vector copy
  // would make each chunk wait for the previous chunk's stores)
  typedef __attribute__((address_space(1))) uint8_t gbyte;
  typedef __attribute__((address_space(1))) uint32_t gword;
  uint32_t cr = 0xFFFFFFFFu, n = 0, k0 = 0, k1 = 0, tiles = 0;
  bool walls = false;
  uint64_t t_seed = 0;
  gbyte* grid = nullptr;
  gword* maps = nullptr;
  int32_t* cand_list = nullptr;
  uint32_t* n_cand = nullptr;
  // Candidates collect in a per-wavefront LDS buffer and go to the realization's list
  // with one atomic per flush: one global counter per realization would otherwise take
  // an atomic from every chunk that holds a candidate, all on one address.
  constexpr uint32_t kSeedBuf = 512;
  __shared__ int32_t s_cbuf[kMaxBlock / kWave][kSeedBuf];
  int32_t* cbuf = s_cbuf[threadIdx.x / kWave];
  uint32_t nbuf = 0;  // (wave-uniform)
  auto flush = [&]() {
    if (nbuf == 0) return;
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(n_cand, nbuf);
    base = uniform((uint32_t)__builtin_amdgcn_readfirstlane(base));
    wave_sync();  // the buffer's entries are written
    for (uint32_t k = lane_id(); k < nbuf; k += kWave) cand_list[base + k] = cbuf[k];
    wave_sync();  // and read before the buffer is reused
    nbuf = 0;
  };
  // each lane takes the four voxels 4i .. 4i + 3: four independent blocks in flight and
  // one word store of the grid (byte stores only for the last, partial group, so that
  // the grid's padding is never written)
  for_each_chunk(A, kItemsQuads, [&](uint32_t r, uint32_t i) {
    if (r != cr) {
      flush();  // (the previous realization's candidates)
      Real& R = A.reals[r];
      n = uniform(R.g.n);
      k0 = uniform(R.k0);
      k1 = uniform(R.k1);
      t_seed = uniform64(R.t_seed);
      grid = (gbyte*)uniform64((uint64_t)R.grid);
      maps = (gword*)uniform64((uint64_t)R.maps);
      tiles = 2u * tile_map_words(uniform(R.tl.n));  // map words (both halves)
      walls = uniform(R.walls) != 0;
      cand_list = (int32_t*)uniform64((uint64_t)R.cand);
      n_cand = &R.ctl.n_cand;
      cr = r;
    }
    const uint32_t v0 = 4u * i;
    uint32_t cand = 0;  // bit k: voxel v0 + k is a candidate
    if (v0 < n) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t v = v0 + (uint32_t)k;
        const U4 w = philox10(v, 0u, 0u, kTagSeed, k0, k1);
        if (v < n && (uint64_t)w.x < t_seed) cand |= 1u << k;
      }
      const bool whole = v0 + 4u <= n;
      if (walls) {  // a later phase: cores only on cells no earlier phase holds
        uint32_t occ = 0;  // bit k: voxel v0 + k holds another phase
        if (whole) {
          const uint32_t b = *(const gword*)(grid + v0);
#pragma unroll
          for (int k = 0; k < 4; ++k) occ |= (((b >> (8 * k)) & 0xFFu) != kVoid ? 1u : 0u) << k;
        } else {
          for (uint32_t k = 0; v0 + k < n; ++k) occ |= (grid[v0 + k] != kVoid ? 1u : 0u) << k;
        }
        cand &= ~occ;
      } else if (whole) {
        *(gword*)(grid + v0) = 0u;  // kVoid x 4
      } else {
        for (uint32_t k = 0; v0 + k < n; ++k) grid[v0 + k] = kVoid;
      }
      if (maps)  // fused sweep: no tile listed yet (both map halves; fewer words than voxels)
        for (uint32_t k = 0; k < 4u && v0 + k < tiles; ++k) maps[v0 + k] = 0;
    }
    if (__ballot(cand != 0)) {
      uint32_t tot;
      uint32_t pos = nbuf + wave_prefix((uint32_t)__builtin_popcount(cand), &tot);
      while (cand) {
        const int k = __builtin_ctz(cand);
        cand &= cand - 1u;
        cbuf[pos++] = (int32_t)(v0 + (uint32_t)k);
      }
      nbuf += uniform(tot);
      if (nbuf > kSeedBuf - 4u * kWave) flush();  // room for one more chunk's four per lane
    }
  });
  flush();  // (capacity N: the list cannot overflow)
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

// Conflicting candidates of candidate i (L1 distance 1..radius) in neighbouring bucket
// k (0..26: offsets (k % 3 - 1, k / 3 % 3 - 1, k / 9 - 1)) of i's bucket; a bucket outside
// the grid or whose nearest point lies beyond the radius is skipped.  visit(j, w) returns
// false to stop early.  Eight candidates' loads are in flight at a time.
template <typename Visit>
__device__ __forceinline__ void scan_bucket(const BatchArgs& A, const Real& R, uint32_t i,
                                            uint32_t v, uint32_t k, Visit&& visit) {
  const Buckets bk = R.bk;
  uint32_t x, y, z;
  coords_of(R.g, v, x, y, z);
  const int32_t bx = (int32_t)bk.edge.div(x), by = (int32_t)bk.edge.div(y),
                bz = (int32_t)bk.edge.div(z);
  const int32_t cx = bx + (int32_t)(k % 3) - 1, cy = by + (int32_t)(k / 3 % 3) - 1,
                cz = bz + (int32_t)(k / 9) - 1;
  if (cx < 0 || cy < 0 || cz < 0 || cx >= (int32_t)bk.nbx || cy >= (int32_t)bk.nby ||
      cz >= (int32_t)bk.nbz)
    return;
  // L1 distance from the candidate to bucket c along one axis (bucket c covers
  // [c E, (c + 1) E - 1])
  const int32_t E = (int32_t)bk.edge.d;
  auto gap = [E](int32_t c, int32_t b0, int32_t p) -> int32_t {
    return c < b0 ? p - ((c + 1) * E - 1) : (c > b0 ? c * E - p : 0);
  };
  if (gap(cx, bx, (int32_t)x) + gap(cy, by, (int32_t)y) + gap(cz, bz, (int32_t)z) > bk.radius)
    return;
  const uint32_t b = R.boff + (uint32_t)cx + bk.nbx * ((uint32_t)cy + bk.nby * (uint32_t)cz);
  const uint32_t e = A.counts[b + 1];
  for (uint32_t j0 = A.counts[b]; j0 < e; j0 += 8) {
    uint32_t wv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) wv[u] = j0 + u < e ? (uint32_t)A.sorted_v[j0 + u] : 0u;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t j = j0 + u;
      if (j >= e || j == i) continue;
      const uint32_t w = wv[u];
      uint32_t wx, wy, wz;
      coords_of(R.g, w, wx, wy, wz);
      const int32_t dist = abs((int32_t)wx - (int32_t)x) + abs((int32_t)wy - (int32_t)y) +
                           abs((int32_t)wz - (int32_t)z);
      if (dist > bk.radius) continue;
      if (!visit(j, w)) return;
    }
  }
}

// One priority round over all bucket-sorted candidates, in two launches.  Decide: a
// live candidate whose key (priority, v) is below the key of every conflicting
// candidate that is still live (or accepted in this round) is accepted.  Kill: every
// candidate accepted in this round marks its live conflicting candidates dead.  A
// candidate is accepted exactly when no conflicting candidate with a smaller key is
// still in play, so the rounds reproduce the greedy acceptance in ascending key order.
// Each candidate takes half a wavefront: lane k < 27 of the half scans neighbouring
// bucket k (a lane stops at its first smaller key), and a ballot combines the lanes.
// Any candidate left live sets the round's flag (the host stops when it stays 0).
__global__ __launch_bounds__(kMaxBlock) void k_luby_round(BatchArgs A, uint32_t round) {
  const uint32_t n = A.bctl->n_sorted;
  const uint32_t lane = lane_id(), half = lane >> 5, k = lane & 31u;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t nwaves = gridDim.x * blockDim.x / kWave;
  for (uint32_t base = 2 * wave; base < n; base += 2 * nwaves) {
    const uint32_t i = base + half;
    const bool live = i < n && A.status[i] == kLive;
    bool smaller = false;
    if (live && k < 27u) {
      const Real& R = A.reals[A.sorted_r[i]];
      const uint32_t v = (uint32_t)A.sorted_v[i];
      const uint64_t p = A.sorted_prio[i];
      scan_bucket(A, R, i, v, k, [&](uint32_t j, uint32_t w) {
        const uint8_t st = A.status[j];
        if (st == kLive || st == kAcceptedNew) {
          const uint64_t q = A.sorted_prio[j];
          if (q < p || (q == p && w < v)) {
            smaller = true;
            return false;
          }
        }
        return true;
      });
    }
    const uint64_t bal = __ballot(smaller);
    const bool beaten = ((bal >> (32u * half)) & 0xFFFFFFFFull) != 0;
    if (live && k == 0) {
      if (beaten)
        A.live[round] = 1u;
      else
        A.status[i] = kAcceptedNew;
    }
  }
}

__global__ __launch_bounds__(kMaxBlock) void k_luby_kill(BatchArgs A) {
  const uint32_t n = A.bctl->n_sorted;
  const uint32_t lane = lane_id(), half = lane >> 5, k = lane & 31u;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t nwaves = gridDim.x * blockDim.x / kWave;
  for (uint32_t base = 2 * wave; base < n; base += 2 * nwaves) {
    const uint32_t i = base + half;
    const bool fresh = i < n && A.status[i] == kAcceptedNew;
    if (fresh && k < 27u) {
      const Real& R = A.reals[A.sorted_r[i]];
      scan_bucket(A, R, i, (uint32_t)A.sorted_v[i], k, [&](uint32_t j, uint32_t) {
        if (A.status[j] == kLive) A.status[j] = kDead;
        return true;
      });
    }
    if (fresh && k == 0) A.status[i] = kAccepted;
  }
}

// Accepted candidates become seeds: 1 in the grid, appended to the realization's
// seed list (which reuses its candidate list).  The accepted lanes of a wavefront are
// grouped by realization, one atomic per group.
__global__ __launch_bounds__(kMaxBlock) void k_collect_seeds(BatchArgs A) {
  const uint32_t n = A.bctl->n_sorted;
  const uint32_t lane = lane_id();
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const bool acc = i < n && A.status[i] == kAccepted;
    const uint32_t r = acc ? A.sorted_r[i] : 0xFFFFFFFFu;
    uint64_t pending = __ballot(acc);
    while (pending) {
      const uint32_t leader = (uint32_t)__builtin_ctzll(pending);
      const uint32_t rl = uniform(__shfl(r, (int)leader, kWave));
      const bool mine = acc && r == rl;
      const uint64_t m = __ballot(mine);
      uint32_t slot = 0;
      if (lane == leader) slot = atomicAdd(&A.reals[rl].ctl.n_seeds, (uint32_t)__popcll(m));
      slot = __shfl(slot, (int)leader, kWave) + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      if (mine) {
        Real& R = A.reals[rl];
        const int32_t v = A.sorted_v[i];
        R.grid[v] = kSolid;
        R.cand[slot] = v;
      }
      pending &= ~m;
    }
  }
}

// The all-tiles form lists every tile, in every pass (no map is kept).
__global__ __launch_bounds__(kMaxBlock) void k_full_tiles(BatchArgs A) {
  for_each_chunk(A, kItemsVoxels, [&](uint32_t r, uint32_t i) {
    Real& R = A.reals[r];
    if (R.form == kFormAllTiles && i == 0) R.ctl.n_list = R.tl.n;
  });
}

// The fused sweep's first list: the tiles holding a seed, as bits of map half 0 (zeroed
// with the grid), and their number (a tile counts once: for the first seed that set
// its bit).
__global__ __launch_bounds__(kMaxBlock) void k_seed_tiles(BatchArgs A) {
  for_each_chunk(A, kItemsSeeds, [&](uint32_t r, uint32_t i) {
    Real& R = A.reals[r];
    if (R.form != kFormList) return;  // (uniform per wavefront)
    bool fresh = false;
    if (i < R.ctl.n_seeds) {
      uint32_t x, y, z;
      coords_of(R.g, (uint32_t)R.cand[i], x, y, z);
      const uint32_t u = x / kTileX + R.tl.ntx * (y / kTileY + R.tl.nty * (z / kTileZ));
      const uint32_t bit = 1u << (u & 31u);
      fresh = (atomicOr(&R.maps[u >> 5], bit) & bit) == 0u;
    }
    wave_append_flag(fresh, &R.ctl.n_list);
  });
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

// Directions of each class as 26-bit masks (bit d).
constexpr uint32_t class_mask(int cls) {
  uint32_t m = 0;
  for (int d = 0; d < 26; ++d)
    if ((int)((kDirClass >> (2 * d)) & 3u) == cls) m |= 1u << d;
  return m;
}
constexpr uint32_t kEdgeDirs = class_mask(1), kCornerDirs = class_mask(2);

// Eq. (1) thresholds of one step split for the 32-bit draws (H << 16 | L): a draw
// passes iff H < hi, or H == hi and L < lo.  T = 2^32 gives hi = 65536 (always passes).
// (Named fields, not arrays: a dynamically indexed array would live in scratch memory.)
struct DrawThresholds {
  uint32_t hi_face, hi_edge, hi_corner, lo_face, lo_edge, lo_corner;
};

__device__ __forceinline__ DrawThresholds draw_thresholds(uint64_t T0, uint64_t T1, uint64_t T2) {
  return DrawThresholds{(uint32_t)(T0 >> 16),     (uint32_t)(T1 >> 16),
                        (uint32_t)(T2 >> 16),     (uint32_t)(T0 & 0xFFFFu),
                        (uint32_t)(T1 & 0xFFFFu), (uint32_t)(T2 & 0xFFFFu)};
}

// Linear offsets of the 26 directions for one geometry, computed on the fly.
struct DirOffsetCalc {
  const Geometry& g;
  __device__ __forceinline__ int32_t operator()(int d) const { return dir_offset(g, d); }
};
// The same from a table (26 entries, e.g. in LDS).
struct DirOffsetTable {
  const int32_t* off;
  __device__ __forceinline__ int32_t operator()(int d) const { return off[d]; }
};

// High-half threshold of direction d: from its class, or from a 26-entry table.
struct DirThresholdCalc {
  uint32_t hf, he, hc;
  __device__ __forceinline__ uint32_t operator()(int d) const {
    return ((kCornerDirs >> d) & 1u) ? hc : (((kEdgeDirs >> d) & 1u) ? he : hf);
  }
};
struct DirThresholdTable {
  const uint32_t* hi;
  __device__ __forceinline__ uint32_t operator()(int d) const { return hi[d]; }
};


// Draws of source voxel a at step t (Sec. 2.3 step 3; the draw rule is stated in qsgs.h):
// its in-domain void neighbours (at the step's start) take the draws of ranks
// j = 0, 1, ... in ascending direction; a passing draw claims the neighbour with a
// 32-bit atomicOr that writes `mark` into its grid byte.  Returns the directions this
// thread claimed first (the neighbour was still 0).  Ranks are taken eight at a time,
// one Philox block per eight, with the word and half of each rank fixed by unrolling;
// a block's claim atomics are all issued before their results are read.  Targets in
// `skip` (already grown this step) take their rank but need no claim.  The key and
// grid pointer are passed by value: read through the record they would be reloaded
// after every claim atomic.
template <typename DirOffset, typename DirThreshold>
__device__ __forceinline__ uint32_t grow_draws(uint8_t* __restrict__ grid, uint32_t k0,
                                               uint32_t k1, DirOffset doff, DirThreshold dhi,
                                               uint32_t a, uint32_t t, uint32_t voidm,
                                               uint32_t skip, DrawThresholds th, uint8_t mark) {
  // values, selected per draw with v_cndmask (a select of field addresses would put
  // the thresholds in scratch memory)
  const uint32_t lf = th.lo_face, le = th.lo_edge, lc = th.lo_corner;
  uint32_t claims = 0;
  uint32_t m = voidm;
  for (uint32_t blk = 0; m; ++blk) {
    const U4 H = philox10(a, t, blk, kTagGrowHi, k0, k1);
    uint32_t dir[8];
    bool pass[8], tie[8];
    bool any_tie = false;
#pragma unroll
    for (int sl = 0; sl < 8; ++sl) {
      dir[sl] = 0;
      pass[sl] = false;
      tie[sl] = false;
      if (m) {
        const int d = __builtin_ctz(m);
        m &= m - 1u;
        dir[sl] = (uint32_t)d;
        const uint32_t w = sl < 2 ? H.x : (sl < 4 ? H.y : (sl < 6 ? H.z : H.w));
        const uint32_t h = (sl & 1) ? (w >> 16) : (w & 0xFFFFu);
        const uint32_t hi = dhi(d);
        pass[sl] = h < hi;
        tie[sl] = h == hi;
      }
      any_tie |= tie[sl];
    }
    if (any_tie) {  // high halves tie (rare): decide those slots on the low halves
      const U4 L = philox10(a, t, blk, kTagGrowLo, k0, k1);
#pragma unroll
      for (int sl = 0; sl < 8; ++sl) {
        if (tie[sl]) {
          const uint32_t wl = sl < 2 ? L.x : (sl < 4 ? L.y : (sl < 6 ? L.z : L.w));
          const uint32_t l = (sl & 1) ? (wl >> 16) : (wl & 0xFFFFu);
          const uint32_t d = dir[sl];
          const uint32_t lo =
              ((kCornerDirs >> d) & 1u) ? lc : (((kEdgeDirs >> d) & 1u) ? le : lf);
          pass[sl] = l < lo;
        }
      }
    }
    uint32_t old[8], shift[8];
#pragma unroll
    for (int sl = 0; sl < 8; ++sl) {
      old[sl] = 0;
      shift[sl] = 0;
      pass[sl] = pass[sl] && !((skip >> dir[sl]) & 1u);
      if (pass[sl]) {
        const uint32_t q = (uint32_t)((int32_t)a + doff((int)dir[sl]));
        shift[sl] = (q & 3u) * 8u;
        old[sl] = atomicOr((uint32_t*)(grid + (q & ~3u)), (uint32_t)mark << shift[sl]);
      }
    }
#pragma unroll
    for (int sl = 0; sl < 8; ++sl)
      if (pass[sl] && ((old[sl] >> shift[sl]) & 0xFFu) == kVoid) claims |= 1u << dir[sl];
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
// A wavefront's appends to one realization's list go through an LDS buffer and reach the
// list's counter with one atomic per flush (per-chunk atomics on one counter serialize).
constexpr uint32_t kListBuf = 512;

__global__ __launch_bounds__(kMaxBlock) void k_grow(BatchArgs A) {
  __shared__ int32_t s_lbuf[kMaxBlock / kWave][kListBuf];
  int32_t* lbuf = s_lbuf[threadIdx.x / kWave];
  uint32_t nbuf = 0, cr = 0xFFFFFFFFu;  // (wave-uniform)
  auto flush = [&]() {
    if (nbuf == 0) return;
    Real& R = A.reals[cr];
    Ctl& c = R.ctl;
    int32_t* __restrict__ fin = c.cur ? R.f1 : R.f0;
    const uint32_t nf = c.front_size;
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(&c.new_count, nbuf);
    base = uniform((uint32_t)__builtin_amdgcn_readfirstlane(base));
    wave_sync();  // the buffer's entries are written
    for (uint32_t k = lane_id(); k < nbuf; k += kWave) {
      const uint32_t slot = nf + base + k;
      if (slot < R.cap)
        fin[slot] = lbuf[k];
      else
        c.overflow = 1u;
    }
    wave_sync();  // and read before the buffer is reused
    nbuf = 0;
  };
  for_each_chunk(A, kItemsGrow, [&](uint32_t r, uint32_t i) {
    if (r != cr) {
      flush();
      cr = r;
    }
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
        const DrawThresholds th = draw_thresholds(c.T[0], c.T[1], c.T[2]);
        uint32_t x, y, z;
        coords_of(g, a, x, y, z);
        const Nbhd nb = load_neighbourhood(R.grid, g, a, x, y, z);
        claims = grow_draws(R.grid, uniform(R.k0), uniform(R.k1), DirOffsetCalc{g},
                            DirThresholdCalc{th.hi_face, th.hi_edge, th.hi_corner}, a, t,
                            nb.voidm, nb.grown, th, kGrown);
      }
    }
    if (__ballot(claims != 0) == 0) return;
    uint32_t tot;
    uint32_t pos = wave_prefix((uint32_t)__builtin_popcount(claims), &tot);
    tot = uniform(tot);
    if (nbuf + tot > kListBuf) flush();
    if (tot > kListBuf) {  // (a chunk with more claims than the buffer holds: direct)
      uint32_t base = 0;
      if (lane_id() == 0) base = atomicAdd(&c.new_count, tot);
      pos += uniform((uint32_t)__builtin_amdgcn_readfirstlane(base));
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
      return;
    }
    pos += nbuf;
    while (claims) {
      const int d = __builtin_ctz(claims);
      claims &= claims - 1u;
      lbuf[pos++] = (int32_t)((int32_t)a + dir_offset(g, d));
    }
    nbuf += tot;
  });
  flush();
}

// ---------------------------------------------------------------------------
// a5: prune and compaction (Sec. 2.3 step 4), items: F_t + New_t.  F_{t+1} = the
// entries that still have an in-domain void neighbour, appended through the
// wavefront's LDS buffer.  New voxels are folded from 2 to 1 here.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBlock) void k_prune(BatchArgs A) {
  __shared__ int32_t s_lbuf[kMaxBlock / kWave][kListBuf];
  int32_t* lbuf = s_lbuf[threadIdx.x / kWave];
  uint32_t nbuf = 0, cr = 0xFFFFFFFFu;  // (wave-uniform)
  auto flush = [&]() {
    if (nbuf == 0) return;
    Real& R = A.reals[cr];
    Ctl& c = R.ctl;
    int32_t* __restrict__ fout = c.cur ? R.f0 : R.f1;
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(&c.out_count, nbuf);
    base = uniform((uint32_t)__builtin_amdgcn_readfirstlane(base));
    wave_sync();  // the buffer's entries are written
    for (uint32_t k = lane_id(); k < nbuf; k += kWave) {
      if (base + k < R.cap)
        fout[base + k] = lbuf[k];
      else
        c.overflow = 1u;
    }
    wave_sync();  // and read before the buffer is reused
    nbuf = 0;
  };
  for_each_chunk(A, kItemsPrune, [&](uint32_t r, uint32_t i) {
    if (r != cr) {
      flush();
      cr = r;
    }
    Real& R = A.reals[r];
    Ctl& c = R.ctl;
    const uint32_t nf = c.front_size;
    const uint32_t n_in = nf + c.new_count;
    const int32_t* __restrict__ fin = c.cur ? R.f1 : R.f0;
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
    const uint64_t km = __ballot(keep);
    if (km == 0) return;
    if (nbuf + kWave > kListBuf) flush();
    if (keep)
      lbuf[nbuf + __builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u))] =
          (int32_t)v;
    nbuf += (uint32_t)__popcll(km);
  });
  flush();
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
    uint64_t* e = R.log + kLogWords * (uint64_t)t;
    e[0] = c.front_size;
    e[1] = grown;
    e[2] = c.cnt;
    e[3] = 0;  // the step-by-step path does not count its work
    e[4] = 0;
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
// Fused sweep (qsgs_generate*, server), indexed by active tiles.
//
// F_t is exactly the interface of the grid at the start of step t (the solid voxels
// with an in-domain void neighbour): a voxel of F_{t-1} keeps a void neighbour only
// if it had one, since the void set only shrinks, and a voxel grown in step t-1
// joins F_t iff it has one.  The list carried from step to step therefore names
// 64 x 8 x 4 tiles rather than voxels: the list of step t, a bitmap over the tiles,
// holds every tile that contains a voxel of F_t (a superset is harmless).  A pass
// stages each listed tile with its one-voxel halo from the occupancy planes (S, the
// marks of the previous step, the walls) by coalesced row loads, finds F_t in the tile
// with 64-bit row masks, compacts those voxels into an LDS queue (wavefront prefix),
// and every queued voxel draws for its void neighbours (Sec. 2.3 step 3, Eq. (1)),
// claiming winners with a 32-bit atomicOr on the step's mark plane.  A voxel of
// F_{t+1} either was in F_t or was grown in step t, so the next bitmap gets the tiles
// that had a front voxel and the tiles that received a claim (an atomicOr each).  The
// previous step's marks are folded into S by the wavefront that stages their tile
// (listed, because a claim lists its tile); until then every reader counts them as
// solid, so stale reads never change a decision.
//
// Every realization with a pending pass gets G_r workgroups; workgroup k takes the k-th
// equal share of r's listed tiles, in index order, from a descriptor written by the
// previous step end.  Its front count, growth count, draws and blocks go to a
// per-workgroup record; k_sweep_end then ends the step for every realization (log,
// count, status, Eq. (1) thresholds of the next step) and writes the next shares.
// ---------------------------------------------------------------------------

// Bitwise or / sum of a value over the 64 lanes of the wavefront (every lane gets it;
// every lane must be active).  The 64-bit sum adds the low and high 16-bit halves apart.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  return __builtin_amdgcn_readlane(wave_incl_or(v), kWave - 1);
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  return __builtin_amdgcn_readlane(wave_incl_sum(v), kWave - 1);
}
__device__ __forceinline__ unsigned long long wave_sum64(uint32_t v) {
  const uint32_t lo = wave_sum(v & 0xFFFFu), hi = wave_sum(v >> 16);
  return ((unsigned long long)hi << 16) + lo;
}


// A realization with a pending tile-sweep pass, or (field_active) a pending full-field step.
__device__ __forceinline__ bool sweep_active(const Real& R) {
  return R.phase == kPhaseGrow && R.ctl.status == 0 && R.ctl.mode != kModeIdle &&
         R.form != kFormField;
}
__device__ __forceinline__ bool field_active(const Real& R) {
  return R.phase == kPhaseGrow && R.ctl.status == 0 && R.ctl.mode != kModeIdle &&
         R.form == kFormField;
}

// Byte grid <-> occupancy planes of the fused sweep.  Items are plane words; a chunk of
// 64 words is handled word by word, lane b taking voxel x = 64 ix + b of the word's row,
// so every grid access of the wavefront is one coalesced 64-byte row piece.

// After seeding: S = the seeds (byte 1), M0 = M1 = 0, W = cells of other phases (bytes
// above 1, multi-phase generation only).
// Flags of the four bytes of v (bit k: byte k) equal to 1, resp. above 1: a byte test
// without carries between bytes (each byte's low seven bits plus 0x7F stay below 0x100),
// then the four flag bits (7, 15, 23, 31) gathered by one multiply whose partial
// products land on distinct bits.
__device__ __forceinline__ uint32_t bytes_eq1(uint32_t v) {
  const uint32_t t = v ^ 0x01010101u;  // zero where the byte is 1
  const uint32_t z = ~(((t & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | t | 0x7F7F7F7Fu);
  return ((z >> 7) * 0x00204081u) >> 21 & 0xFu;
}
__device__ __forceinline__ uint32_t bytes_gt1(uint32_t v) {
  const uint32_t u = v & 0xFEFEFEFEu;  // non-zero where the byte is above 1
  const uint32_t nz = (((u & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | u) & 0x80808080u;
  return ((nz >> 7) * 0x00204081u) >> 21 & 0xFu;
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The four low bits of n as bytes 0 / 1 (the inverse of bytes_eq1 on 0 / 1 bytes).
__device__ __forceinline__ uint32_t bits_to_bytes(uint32_t n) {
  return (n * 0x00204081u) & 0x01010101u;
}

__global__ __launch_bounds__(kMaxBlock) void k_pack_planes(BatchArgs A) {
  const uint32_t lane = lane_id();
  for_each_chunk(A, kItemsPack, [&](uint32_t r, uint32_t i) {
    const Real& R = A.reals[r];
    const uint32_t pw = uniform(R.pwords);
    const uint32_t w0 = i - lane;
    if (w0 >= pw) return;  // (uniform) padding of the item range
    const uint32_t nw = min((uint32_t)kWave, pw - w0);
    const uint32_t nx = (uint32_t)uniform((uint32_t)R.g.nx), ntx = uniform(R.tl.ntx);
    const FastDiv dntx = R.tl.div_ntx;
    const __attribute__((address_space(1))) uint8_t* grid =
        (const __attribute__((address_space(1))) uint8_t*)uniform64((uint64_t)R.grid);
    // the phases an interacting phase may convert (bit b: grid byte b)
    const InteractTable* it = (const InteractTable*)uniform64((uint64_t)R.itab);
    uint64_t s_mine = 0, w_mine = 0, x_mine = 0;
    if ((nx & 15u) == 0u && ((uintptr_t)grid & 15u) == 0u && !it) {
      // (uniform) rows of aligned 16-byte chunks: each lane packs its own word from four
      // 16-byte loads
      if (lane < nw) {
        const uint32_t w = w0 + lane;
        const uint32_t row = dntx.div(w);
        const uint32_t x0 = (w - row * ntx) * (uint32_t)kTileX;
        const uint32_t nc = min((uint32_t)kTileX, nx - x0) >> 4;  // chunks in the domain
        typedef const __attribute__((address_space(1))) u32x4 g4;
        g4* p = (g4*)(grid + (size_t)row * nx + x0);
        u32x4 v[4];
#pragma unroll
        for (uint32_t c = 0; c < 4u; ++c) {
          v[c] = u32x4{0u, 0u, 0u, 0u};
          if (c < nc) v[c] = p[c];
        }
#pragma unroll
        for (uint32_t c = 0; c < 4u; ++c) {
          const uint32_t q[4] = {v[c].x, v[c].y, v[c].z, v[c].w};
#pragma unroll
          for (uint32_t k = 0; k < 4u; ++k) {
            s_mine |= (uint64_t)bytes_eq1(q[k]) << (16u * c + 4u * k);
            w_mine |= (uint64_t)bytes_gt1(q[k]) << (16u * c + 4u * k);
          }
        }
      }
    } else {
    for (uint32_t j = 0; j < nw; ++j) {
      const uint32_t w = w0 + j;
      const uint32_t row = dntx.div(w);
      const uint32_t x = (w - row * ntx) * (uint32_t)kTileX + lane;
      const uint32_t b = x < nx ? (uint32_t)grid[row * nx + x] : 0u;
      const uint64_t sm = __ballot(b == kSolid);
      const uint64_t wm = __ballot(b > kSolid);
      const uint64_t xm = it ? __ballot(b > kSolid && ((it->bits[b >> 5] >> (b & 31u)) & 1u))
                             : 0ull;
      if (lane == j) {
        s_mine = sm;
        w_mine = wm;
        x_mine = xm;
      }
    }
    }
    if (lane < nw) {
      uint64_t* P = (uint64_t*)uniform64((uint64_t)R.planes);
      P[(size_t)kPlaneS * pw + w0 + lane] = s_mine;
      P[(size_t)kPlaneM0 * pw + w0 + lane] = 0ull;
      P[(size_t)kPlaneM1 * pw + w0 + lane] = 0ull;
      if (R.walls) P[(size_t)kPlaneW * pw + w0 + lane] = w_mine;
      if (it) P[(size_t)kPlaneX * pw + w0 + lane] = x_mine;
    }
  });
}

// After the last pass of a realization (every mark folded into S): byte = S bit, or, on
// a multi-phase grid, 1 where S is set and the byte unchanged elsewhere.
__global__ __launch_bounds__(kMaxBlock) void k_export_planes(BatchArgs A) {
  const uint32_t lane = lane_id();
  for_each_chunk(A, kItemsExport, [&](uint32_t r, uint32_t i) {
    const Real& R = A.reals[r];
    const uint32_t pw = uniform(R.pwords);
    const uint32_t w0 = i - lane;
    if (w0 >= pw) return;  // (uniform)
    const uint32_t nw = min((uint32_t)kWave, pw - w0);
    const uint32_t nx = (uint32_t)uniform((uint32_t)R.g.nx), ntx = uniform(R.tl.ntx);
    const FastDiv dntx = R.tl.div_ntx;
    const bool walls = uniform(R.walls) != 0;
    __attribute__((address_space(1))) uint8_t* grid =
        (__attribute__((address_space(1))) uint8_t*)uniform64((uint64_t)R.grid);
    const uint64_t* S = (const uint64_t*)uniform64((uint64_t)R.planes);
    const uint64_t mine = lane < nw ? S[w0 + lane] : 0ull;
    if ((nx & 15u) == 0u && ((uintptr_t)grid & 15u) == 0u) {
      // (uniform) rows of aligned 16-byte chunks: each lane writes its own word's bytes
      // with four 16-byte stores
      if (lane < nw) {
        const uint32_t w = w0 + lane;
        const uint32_t row = dntx.div(w);
        const uint32_t x0 = (w - row * ntx) * (uint32_t)kTileX;
        const uint32_t nc = min((uint32_t)kTileX, nx - x0) >> 4;
        typedef __attribute__((address_space(1))) u32x4 g4;
        g4* p = (g4*)(grid + (size_t)row * nx + x0);
        for (uint32_t c = 0; c < nc; ++c) {
          const uint32_t b16 = (uint32_t)(mine >> (16u * c));
          u32x4 v = u32x4{bits_to_bytes(b16 & 0xFu), bits_to_bytes((b16 >> 4) & 0xFu),
                          bits_to_bytes((b16 >> 8) & 0xFu), bits_to_bytes((b16 >> 12) & 0xFu)};
          if (walls) {  // kSolid where S is set, the byte unchanged elsewhere
            const u32x4 o = p[c];
            v.x |= o.x & ~(v.x * 0xFFu);
            v.y |= o.y & ~(v.y * 0xFFu);
            v.z |= o.z & ~(v.z * 0xFFu);
            v.w |= o.w & ~(v.w * 0xFFu);
          }
          p[c] = v;
        }
      }
      return;
    }
    const uint32_t mlo = (uint32_t)mine, mhi = (uint32_t)(mine >> 32);
    for (uint32_t j = 0; j < nw; ++j) {
      const uint32_t w = w0 + j;
      const uint32_t row = dntx.div(w);
      const uint32_t x = (w - row * ntx) * (uint32_t)kTileX + lane;
      const uint32_t half = lane < 32u ? (uint32_t)__builtin_amdgcn_readlane(mlo, j)
                                       : (uint32_t)__builtin_amdgcn_readlane(mhi, j);
      const uint32_t bit = (half >> (lane & 31u)) & 1u;
      if (x < nx) {
        if (!walls)
          grid[row * nx + x] = (uint8_t)bit;
        else if (bit)
          grid[row * nx + x] = kSolid;
      }
    }
  });
}

// ----- calls that never synchronise with the host (graph capture) -----

// Host data carried by value in the kernel arguments: a copy node would read host memory
// when a captured graph is replayed, a kernel argument is part of the graph.
__global__ void k_put_words(uint32_t* __restrict__ dst, WordBlob b) {
  for (uint32_t i = threadIdx.x; i < b.n; i += blockDim.x) dst[i] = b.w[i];
}

// After a fixed number of spacing rounds: if candidates are still undecided, every
// realization of the call fails (its loop state reports an internal error).
__global__ void k_seed_settled(BatchArgs A, uint32_t rounds) {
  if (rounds == 0 || A.live[rounds - 1] == 0) return;
  for (uint32_t r = threadIdx.x; r < A.count; r += blockDim.x) A.reals[r].ctl.overflow = 1u;
}

// Each realization's loop state as a qsgs_info in device memory.
__global__ void k_info_out(BatchArgs A, qsgs_info* __restrict__ out) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= A.count) return;
  const Ctl& c = A.reals[r].ctl;
  qsgs_info i;
  i.n_candidates = c.n_cand;
  i.n_seeds = c.n_seeds;
  i.solid_count = (int64_t)c.cnt;
  i.target_count = (int64_t)c.s_star;
  i.front_size = c.front_size;
  i.grown_last_step = c.last_new;
  i.step = c.step;
  i.status = (c.status == kStatusOverflow || c.bad_entry) ? (int32_t)QSGS_ERR_DEVICE : c.status;
  out[r] = i;
}

// The grids of the realizations exported by the last k_export_planes are written.
__global__ void k_export_done(BatchArgs A) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < A.count && A.reals[r].ctl.export_state == 1u) A.reals[r].ctl.export_state = 2u;
}

// Exclusive prefix sums of a[0..n) in place (LDS), with a[n] = the total, which is
// returned.  One workgroup, every thread calling; each thread takes a contiguous run.
__device__ uint32_t lds_exclusive_scan(uint32_t* a, uint32_t n) {
  __shared__ uint32_t wt[1024 / kWave];
  __shared__ uint32_t s_total;
  __syncthreads();  // a[] is complete
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
  const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
  const uint32_t lo = min(n, threadIdx.x * per), hi = min(n, lo + per);
  uint32_t sum = 0;
  for (uint32_t i = lo; i < hi; ++i) sum += a[i];
  const uint32_t incl = wave_incl_sum(sum);
  if (lane == kWave - 1) wt[wv] = incl;
  __syncthreads();
  if (wv == 0) {  // the first wave scans the wave totals (at most 16)
    const uint32_t t = lane < nw ? wt[lane] : 0u;
    const uint32_t ti = wave_incl_sum(t);
    if (lane < nw) wt[lane] = ti - t;
    if (lane == nw - 1) s_total = ti;
  }
  __syncthreads();
  uint32_t run = wt[wv] + incl - sum;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
  const uint32_t total = s_total;
  if (threadIdx.x == 0) a[n] = total;
  __syncthreads();
  return total;
}

// Exclusive prefix sums of a[0..n) and b[0..n) in place, as lds_exclusive_scan (one pass,
// one set of barriers); a[n], b[n] = the totals.
__device__ void lds_exclusive_scan2(uint32_t* a, uint32_t* b, uint32_t n) {
  __shared__ uint32_t wt[2][1024 / kWave];
  __shared__ uint32_t s_total[2];
  __syncthreads();  // a[], b[] are complete
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
  const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
  const uint32_t lo = min(n, threadIdx.x * per), hi = min(n, lo + per);
  uint32_t sa = 0, sb = 0;
  for (uint32_t i = lo; i < hi; ++i) {
    sa += a[i];
    sb += b[i];
  }
  const uint32_t ia = wave_incl_sum(sa), ib = wave_incl_sum(sb);
  if (lane == kWave - 1) {
    wt[0][wv] = ia;
    wt[1][wv] = ib;
  }
  __syncthreads();
  if (wv == 0) {  // the first wave scans the wave totals (at most 16)
    const uint32_t ta = lane < nw ? wt[0][lane] : 0u, tb = lane < nw ? wt[1][lane] : 0u;
    const uint32_t xa = wave_incl_sum(ta), xb = wave_incl_sum(tb);
    if (lane < nw) {
      wt[0][lane] = xa - ta;
      wt[1][lane] = xb - tb;
    }
    if (lane == nw - 1) {
      s_total[0] = xa;
      s_total[1] = xb;
    }
  }
  __syncthreads();
  uint32_t ra = wt[0][wv] + ia - sa, rb = wt[1][wv] + ib - sb;
  for (uint32_t i = lo; i < hi; ++i) {
    const uint32_t va = a[i], vb = b[i];
    a[i] = ra;
    b[i] = rb;
    ra += va;
    rb += vb;
  }
  if (threadIdx.x == 0) {
    a[n] = s_total[0];
    b[n] = s_total[1];
  }
  __syncthreads();
}

// Position of the j-th (from 0) set bit of w (j < popcount(w)): a binary search for the
// lowest q with j + 1 set bits at or below it, on popcounts of prefixes.
__device__ __forceinline__ uint32_t select_bit(uint32_t w, uint32_t j) {
  uint32_t q = 0;  // invariant: at most j set bits below q
#pragma unroll
  for (uint32_t s = 16; s; s >>= 1)
    if ((uint32_t)__builtin_popcount(w & ((1u << (q + s)) - 1u)) <= j) q += s;
  return q;
}

// LDS arrays of plan_shares (one workgroup).  info[r]: bit 0 a tile pass of r is
// pending, bit 1 the all-tiles form, bit 2 the map half that lists the pass's tiles;
// tn[r]: its tiles; maps[r]: its maps.  The rest is plan_shares' own: n (listed tiles),
// wo (first word of r in the scanned word space), np (listed tiles before r in that
// space), wg (first logical workgroup of r), ulo (first tile of each share of a mapped
// realization).
struct PlanArrays {
  uint8_t* info;
  uint32_t* tn;
  uint32_t** maps;
  uint32_t* n;
  uint32_t* wo;
  uint32_t* np;
  uint32_t* wg;
  uint32_t* ulo;
  uint32_t* sum;  // 4 words
};

// The next pass's shares (one workgroup of 1 024 threads, every thread calling).  A
// pending realization's listed tiles are the set bits of its map half; its G_r
// workgroups (G_r = max(1, floor((G - B) n_r / n)) for n_r > 0 listed tiles, B such
// realizations, n tiles in all, so sum G_r <= G) take equal shares of them in index
// order: share k holds listed tiles floor(n_r k / G_r) .. floor(n_r (k + 1) / G_r) - 1,
// from the tile of its first one to the tile of the next share's first one.  The
// all-tiles form takes equal ranges of every tile.  With clear_other the other map half
// of each pending realization (the previous pass's list) is cleared for the pass after.
// Writes every logical workgroup's WgDesc and each pending realization's n_list; returns
// the number of workgroups with a share.  Each thread reads a contiguous run of the map
// words, kChunk at a time with the loads issued together (held from the first reading to
// the second when the run is one chunk).
__device__ uint32_t plan_shares(const BatchArgs& A, const PlanArrays& L, bool clear_other) {
  constexpr uint32_t kChunk = 8;
  const uint32_t tid = threadIdx.x, count = A.count, G = A.sweep_grid;
  auto mapped = [&](uint32_t r) { return (L.info[r] & 3u) == 1u; };
  // words of every mapped realization in one space, realization by realization
  for (uint32_t r = tid; r < count; r += blockDim.x) {
    L.wo[r] = mapped(r) ? tile_map_words(L.tn[r]) : 0u;
    L.n[r] = (L.info[r] & 3u) == 3u ? L.tn[r] : 0u;
  }
  const uint32_t W = lds_exclusive_scan(L.wo, count);
  const uint32_t per = (W + blockDim.x - 1u) / blockDim.x;
  const uint32_t g0 = min(W, tid * per), g1 = min(W, g0 + per);
  uint32_t r0 = 0;  // the realization of word g0: the last r with wo[r] <= g0 < wo[r + 1]
  if (g0 < g1) {
    uint32_t hi = count;
    while (hi - r0 > 1) {
      const uint32_t mid = (r0 + hi) >> 1;
      if (L.wo[mid] <= g0) r0 = mid; else hi = mid;
    }
    while (L.wo[r0 + 1] <= g0) ++r0;  // (realizations without words share their start)
  }
  // the words c0 .. c0 + kChunk - 1 of the run (0 past its end), their realizations and
  // their indices in their maps; r, rbase, rend follow the realization of the next word
  uint32_t wv[kChunk], wr[kChunk], wl[kChunk];
  auto load_chunk = [&](uint32_t c0, uint32_t& r, uint32_t& rbase, uint32_t& rend) {
#pragma unroll
    for (uint32_t k = 0; k < kChunk; ++k) {
      const uint32_t g = c0 + k;
      wv[k] = 0;
      wr[k] = r;
      wl[k] = 0;
      if (g < g1) {
        while (g >= rend) {
          ++r;
          rbase = rend;
          rend = L.wo[r + 1];
        }
        const uint32_t mw = tile_map_words(L.tn[r]), half = (L.info[r] >> 2) & 1u;
        wr[k] = r;
        wl[k] = g - rbase;
        wv[k] = ((const g_u32*)L.maps[r])[half * mw + wl[k]];
      }
    }
  };
  // 1. listed tiles per realization (and the other halves cleared)
  uint32_t run_total = 0;
  const bool one_chunk = g1 - g0 <= kChunk;
  if (g0 < g1) {
    uint32_t r = r0, rbase = L.wo[r0], rend = L.wo[r0 + 1];
    uint32_t cr = r0, part = 0;
    for (uint32_t c0 = g0; c0 < g1; c0 += kChunk) {
      load_chunk(c0, r, rbase, rend);
#pragma unroll
      for (uint32_t k = 0; k < kChunk; ++k) {
        if (c0 + k >= g1) break;
        if (wr[k] != cr) {
          if (part) atomicAdd(&L.n[cr], part);
          part = 0;
          cr = wr[k];
        }
        const uint32_t pop = (uint32_t)__builtin_popcount(wv[k]);
        part += pop;
        run_total += pop;
        if (clear_other) {
          const uint32_t mw = tile_map_words(L.tn[cr]), half = (L.info[cr] >> 2) & 1u;
          ((g_u32*)L.maps[cr])[(half ^ 1u) * mw + wl[k]] = 0u;
        }
      }
    }
    if (part) atomicAdd(&L.n[cr], part);
  }
  __syncthreads();
  // 2. workgroups per realization, listed tiles before each mapped realization
  for (uint32_t r = tid; r < count; r += blockDim.x) {
    L.np[r] = mapped(r) ? L.n[r] : 0u;
    if (L.info[r] & 1u) A.reals[r].ctl.n_list = L.n[r];
  }
  if (tid < 4) L.sum[tid] = 0;
  __syncthreads();
  {
    uint32_t tot = 0, busy = 0;
    for (uint32_t r = tid; r < count; r += blockDim.x) {
      const uint32_t nr = (L.info[r] & 1u) ? L.n[r] : 0u;
      tot += nr;
      busy += nr ? 1u : 0u;
    }
    tot = wave_sum(tot);
    busy = wave_sum(busy);
    if (lane_id() == 0) {
      if (tot) atomicAdd(&L.sum[0], tot);
      if (busy) atomicAdd(&L.sum[1], busy);
    }
  }
  __syncthreads();
  const uint32_t total = L.sum[0];
  const uint64_t avail = (uint64_t)G - L.sum[1];
  for (uint32_t r = tid; r < count; r += blockDim.x) {
    const uint32_t nr = (L.info[r] & 1u) ? L.n[r] : 0u;
    L.wg[r] = nr ? max(1u, floor_div53(avail * nr, total)) : 0u;
  }
  lds_exclusive_scan2(L.np, L.wg, count);
  const uint32_t nwg = L.wg[count];
  // 3. the first tile of every share of a mapped realization, from the words' side: the
  // word holding listed tiles [pre, pre + pop) of r holds the first one of exactly the
  // shares k in [ceil(pre G_r / n_r), ceil((pre + pop) G_r / n_r))
  __shared__ uint32_t s_wave_tot[1024 / kWave];
  const uint32_t before = wave_incl_sum(run_total) - run_total;
  if (lane_id() == kWave - 1) s_wave_tot[tid / kWave] = before + run_total;
  __syncthreads();
  uint32_t gp = before;  // listed tiles of mapped realizations before this thread's run
  for (uint32_t v = 0; v < tid / kWave; ++v) gp += s_wave_tot[v];
  if (g0 < g1) {
    uint32_t r = r0, rbase = L.wo[r0], rend = L.wo[r0 + 1];
    // the realization of the words in hand and the first share not yet placed
    uint32_t cr = kNoReal, nr = 0, w0 = 0, Gr = 0, npr = 0, knext = 0;
    for (uint32_t c0 = g0; c0 < g1; c0 += kChunk) {
      if (!one_chunk) load_chunk(c0, r, rbase, rend);  // (a run of one chunk is still held)
#pragma unroll
      for (uint32_t k = 0; k < kChunk; ++k) {
        if (c0 + k >= g1) break;
        const uint32_t rr = wr[k], word = wv[k];
        const uint32_t pop = (uint32_t)__builtin_popcount(word);
        if (rr != cr) {
          cr = rr;
          nr = L.n[rr];
          w0 = L.wg[rr];
          Gr = L.wg[rr + 1] - w0;
          npr = L.np[rr];
          knext = Gr ? floor_div53((uint64_t)(gp - npr) * Gr + nr - 1u, nr) : 0u;
        }
        if (pop && Gr) {
          const uint32_t pre = gp - npr;
          const uint32_t k1 = min(Gr, floor_div53((uint64_t)(pre + pop) * Gr + nr - 1u, nr));
          for (uint32_t ks = knext; ks < k1; ++ks)
            L.ulo[w0 + ks] =
                32u * wl[k] + select_bit(word, floor_div53((uint64_t)nr * ks, Gr) - pre);
          knext = k1;
        }
        gp += pop;
      }
    }
  }
  __syncthreads();
  // 4. the share of every logical workgroup
  for (uint32_t beta = tid; beta < G; beta += blockDim.x) {
    WgDesc d{kNoReal, 0u, 0u, 0u};
    if (beta < nwg) {
      uint32_t lo = 0, hi = count;  // the last r with wg[r] <= beta
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (L.wg[mid] <= beta) lo = mid; else hi = mid;
      }
      const uint32_t r = lo, k = beta - L.wg[r], Gr = L.wg[r + 1] - L.wg[r];
      const uint64_t nr = L.n[r], tn = L.tn[r];
      const uint32_t c0 = floor_div53(nr * k, Gr), c1 = floor_div53(nr * (k + 1), Gr);
      if (L.info[r] & 2u)  // all tiles
        d = WgDesc{r, c0, c1, c1 - c0};
      else
        d = WgDesc{r, L.ulo[beta], k + 1 < Gr ? L.ulo[beta + 1] : (uint32_t)tn, c1 - c0};
    }
    A.desc[beta] = d;
  }
  return nwg;
}

// Loop state of step 0 for every freshly seeded realization (its first map: the tiles of
// its seeds, in half 0), and the shares of the next pass over every realization with a
// pending one.  One workgroup.
__global__ __launch_bounds__(1024) void k_sweep_prepare(BatchArgs A) {
  __shared__ uint8_t s_info[kMaxBatch];
  __shared__ uint32_t s_tn[kMaxBatch], s_n[kMaxBatch];
  __shared__ uint32_t* s_maps[kMaxBatch];
  __shared__ uint32_t s_wo[kMaxBatch + 1], s_np[kMaxBatch + 1], s_wg[kMaxBatch + 1];
  __shared__ uint32_t s_ulo[kMaxSweepGrid], s_sum[4];
  if (threadIdx.x == 0) {
    A.bctl->running = 0;
  }
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < A.count; r += blockDim.x) {
    Real& R = A.reals[r];
    if (R.phase == kPhaseSeed) {
      R.phase = kPhaseGrow;
      Ctl& c = R.ctl;
      c.cnt = c.n_seeds;
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
      }
    }
    const bool tiles = sweep_active(R);
    if (tiles || field_active(R)) atomicAdd(&A.bctl->running, 1u);
    s_info[r] = (uint8_t)((tiles ? 1u : 0u) | (R.form == kFormAllTiles ? 2u : 0u) |
                          (R.ctl.cur & 1u) << 2);
    s_tn[r] = R.tl.n;
    s_maps[r] = R.maps;
  }
  __syncthreads();
  const PlanArrays L{s_info, s_tn, s_maps, s_n, s_wo, s_np, s_wg, s_ulo, s_sum};
  const uint32_t nwg = plan_shares(A, L, false);
  if (threadIdx.x == 0) A.bctl->nwg = nwg;
}

// Loop state that the end of a pass reads for realization r, loaded at once (the sweep
// that wrote it has finished).
struct EndIn {
  uint32_t active;   // a tile-sweep pass was pending (sweep_active)
  uint32_t all;      // the all-tiles form
  uint32_t bad;      // overflow | bad_entry
  uint32_t mode, cur, log_cap, tn;
  int32_t step, max_steps;
  uint64_t cnt, s_star, t_ref[3];
  uint64_t* log;
  uint32_t* maps;
};

__device__ __forceinline__ EndIn end_load(const BatchArgs& A, uint32_t r) {
  const Real& R = A.reals[r];
  const Ctl& c = R.ctl;
  EndIn in;
  in.active = sweep_active(R) ? 1u : 0u;
  in.all = R.form == kFormAllTiles ? 1u : 0u;
  in.bad = c.overflow | c.bad_entry;
  in.mode = c.mode;
  in.cur = c.cur;
  in.log_cap = R.log_cap;
  in.tn = R.tl.n;
  in.step = c.step;
  in.max_steps = c.max_steps;
  in.cnt = c.cnt;
  in.s_star = c.s_star;
  for (int k = 0; k < 3; ++k) in.t_ref[k] = c.t_ref[k];
  in.log = R.log;
  in.maps = R.maps;
  return in;
}

// End of a pass for realization r (a6): kept = |F_t|, grown = voxels grown in the pass,
// draws and blocks = its work.  Writes the step log, the count, the status and the
// Eq. (1) thresholds of the next step.  Returns whether a pass is still pending (the
// realization keeps running, or a final pass follows).
__device__ bool pass_end(const BatchArgs& A, uint32_t r, const EndIn& in, uint32_t kept,
                         uint32_t grown, uint64_t draws, uint64_t blocks) {
  Ctl& c = A.reals[r].ctl;
  if (in.bad) {
    c.status = kStatusOverflow;
    c.mode = kModeIdle;
    return false;
  }
  c.front_size = kept;
  c.cur = in.cur ^ 1u;
  if (in.mode == kModeRun && kept > 0) {
    const uint32_t t = (uint32_t)in.step;
    if (in.log && t < in.log_cap) {
      uint64_t* e = in.log + kLogWords * (uint64_t)t;
      e[0] = kept;
      e[1] = grown;
      e[2] = in.cnt;
      e[3] = draws;
      e[4] = blocks;
    }
    const uint64_t cnt = in.cnt + grown;
    c.cnt = cnt;
    c.last_new = grown;
    c.step = (int32_t)t + 1;
    if (cnt < in.s_star && (int32_t)t + 1 < in.max_steps) {
      for (int k = 0; k < 3; ++k) c.T[k] = eq1_threshold(in.t_ref[k], cnt, in.s_star);
    } else {
      c.mode = kModeFinal;  // one more pass: fold this step's marks, report F_T
    }
    return true;
  }
  // a final pass, or a running pass that found F_t empty: the loop has stopped, and the
  // grid is written from the solid plane
  c.status = in.cnt >= in.s_star ? kStatusDone : (kept == 0 ? kStatusExhausted : kStatusMaxSteps);
  c.mode = kModeIdle;
  c.export_state = 1u;
  return false;
}

// Directions (26-bit masks) whose step leaves the voxel's tile on each side.
constexpr uint32_t dir_mask_where(int field, int val) {
  uint32_t m = 0;
  for (int d = 0; d < 26; ++d)
    if ((int)((pack_direction_field(field) >> (2 * d)) & 3u) == val) m |= 1u << d;
  return m;
}
constexpr uint32_t kDxNeg = dir_mask_where(0, 0), kDxPos = dir_mask_where(0, 2);
constexpr uint32_t kDyNeg = dir_mask_where(1, 0), kDyPos = dir_mask_where(1, 2);
constexpr uint32_t kDzNeg = dir_mask_where(2, 0), kDzPos = dir_mask_where(2, 2);

// The draw rule of grow_draws for the tile sweep, for one block `blk` of a voxel whose
// void mask has had the ranks of its earlier blocks removed (m: ranks 8 blk onward):
// a rank goes further only when its high half is at or below its threshold's; a
// passing rank claims its target with a 32-bit atomicOr of the target's bit in the
// step's mark plane `mark32` (issued at once; the old words are checked after the block,
// and a rank that did not claim keeps an all-ones word, which never counts).  The
// source is voxel a, x coordinate xa, whose row starts at 32-bit word `rb` of a plane;
// drow[d] is the row offset of direction d in 32-bit words.  The directions of passing
// ranks are returned in *passed (for the tiles they reach).  Returns the number of
// voxels this thread claimed first.
// `lds_key` holds the key again for the rare tie path: read through a volatile LDS load,
// the low-half block cannot be hoisted out of that path and computed for every block.
// Interacting phases (kInteract, itab != null): dhi[d] is the largest high half any
// target of direction d can have (unassigned, or a cell of a phase the growing one may
// convert); a rank at or below it reads its target's grid byte b -- 0 for an unassigned
// cell, 3 + m for a cell of phase m, as at the phase's start -- and is decided against
// that target's own threshold (Eq. (1) for b = 0, the interaction table otherwise).
template <bool kInteract>
__device__ __forceinline__ uint32_t sweep_block(uint32_t* __restrict__ mark32, uint32_t k0,
                                                uint32_t k1, const uint32_t* lds_key,
                                                const int32_t* drow, const uint32_t* dhi,
                                                uint32_t a, uint32_t rb, uint32_t xa, uint32_t t,
                                                uint32_t blk, uint32_t m, const U4 H,
                                                DrawThresholds th, uint32_t* passed,
                                                const Geometry& g,
                                                const uint8_t* __restrict__ labels,
                                                const InteractTable* __restrict__ itab) {
  const bool inter = kInteract && itab != nullptr;
  // 1. every rank of the block against dhi of its direction, without branches: with
  // independent phases a high half below it passes and one equal to it ties; with
  // interacting phases every rank at or below it is decided in step 2 (slot mask `slow`)
  uint32_t pass = 0, slow = 0;
  uint32_t mm = m;
#pragma unroll
  for (int sl = 0; sl < 8; ++sl) {
    const uint32_t d = (uint32_t)__builtin_ctz(mm | 0x80000000u);  // 31: no rank left
    mm &= mm - 1u;
    const bool valid = d < 26u;
    const uint32_t w = sl < 2 ? H.x : (sl < 4 ? H.y : (sl < 6 ? H.z : H.w));
    const uint32_t h = (sl & 1) ? (w >> 16) : (w & 0xFFFFu);
    const uint32_t hi = dhi[d];
    if (!inter) pass |= valid && h < hi ? 1u << d : 0u;
    slow |= valid && (inter ? h <= hi : h == hi) ? 1u << sl : 0u;
  }
  // 2. (rare) high-half ties, decided on the low half, and interacting targets
  if (slow) {
    const uint32_t lf = th.lo_face, le = th.lo_edge, lc = th.lo_corner;
    bool have_lo = false;
    U4 L{0, 0, 0, 0};
    if (!inter) {  // every slow rank is a tie: the low-half block is needed, drawn once here
      const uint32_t kl0 = *(const volatile l_u32*)&lds_key[0];
      const uint32_t kl1 = *(const volatile l_u32*)&lds_key[1];
      L = philox10(a, t, blk, kTagGrowLo, kl0, kl1);
      have_lo = true;
    }
    uint32_t m2 = m;
#pragma unroll
    for (int sl = 0; sl < 8; ++sl) {
      const uint32_t d = (uint32_t)__builtin_ctz(m2 | 0x80000000u);
      m2 &= m2 - 1u;
      if (((slow >> sl) & 1u) == 0u) continue;
      const uint32_t w = sl < 2 ? H.x : (sl < 4 ? H.y : (sl < 6 ? H.z : H.w));
      const uint32_t h = (sl & 1) ? (w >> 16) : (w & 0xFFFFu);
      const uint32_t cls = ((kCornerDirs >> d) & 1u) ? 2u : (((kEdgeDirs >> d) & 1u) ? 1u : 0u);
      uint32_t hi = cls == 2u ? th.hi_corner : (cls == 1u ? th.hi_edge : th.hi_face);
      uint32_t lo = cls == 2u ? lc : (cls == 1u ? le : lf);
      if (inter) {  // the target's own threshold
        const int32_t off = (dir_field(kDirDX, (int)d) - 1) +
                            (dir_field(kDirDY, (int)d) - 1) * g.nx +
                            (dir_field(kDirDZ, (int)d) - 1) * (int32_t)g.nxy;
        const uint32_t b = ((const g_u8*)labels)[(uint32_t)((int32_t)a + off)];
        if (b != kVoid) {
          const g_u32* thr = (const g_u32*)itab->thr;
          hi = thr[6u * b + cls];
          lo = thr[6u * b + 3u + cls];
        }
      }
      bool ok = h < hi;
      if (h == hi) {  // high halves tie: decide on the low half
        if (!have_lo) {
          const uint32_t kl0 = *(const volatile l_u32*)&lds_key[0];
          const uint32_t kl1 = *(const volatile l_u32*)&lds_key[1];
          L = philox10(a, t, blk, kTagGrowLo, kl0, kl1);
          have_lo = true;
        }
        const uint32_t wl = sl < 2 ? L.x : (sl < 4 ? L.y : (sl < 6 ? L.z : L.w));
        const uint32_t l = (sl & 1) ? (wl >> 16) : (wl & 0xFFFFu);
        ok = l < lo;
      }
      if (ok) pass |= 1u << d;
    }
  }
  // 3. the claims of the passing ranks, issued together; a claim's old word is checked
  // once all are out (a slot without a claim keeps an all-ones word, which never counts)
  uint32_t old[8], bits[8];
  uint32_t pm = pass;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    old[k] = 0xFFFFFFFFu;
    bits[k] = 0xFFFFFFFFu;
    if (pm) {
      const uint32_t d = (uint32_t)__builtin_ctz(pm);
      pm &= pm - 1u;
      const uint32_t xq = xa + (uint32_t)dir_field(kDirDX, (int)d) - 1u;  // in the domain
      bits[k] = 1u << (xq & 31u);
      old[k] = global_or(mark32 + (uint32_t)((int32_t)rb + drow[d]) + (xq >> 5), bits[k]);
    }
  }
  uint32_t grown = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) grown += (old[k] & bits[k]) == 0u;
  *passed = pass;
  return grown;
}

// m without its k lowest set bits (k < popcount(m) <= 26): a binary search for the lowest q
// with k set bits below q + 1, on popcounts of prefixes.
__device__ __forceinline__ uint32_t drop_low_ranks(uint32_t m, uint32_t k) {
  if (k == 0) return m;
  uint32_t q = 0;  // invariant: fewer than k set bits below q
#pragma unroll
  for (uint32_t s = 16; s; s >>= 1)
    if ((uint32_t)__builtin_popcount(m & ((1u << (q + s)) - 1u)) < k) q += s;
  return m & (~0u << (q + 1u));
}

// Smallest of the eight 16-bit high halves of a block (two per word).
__device__ __forceinline__ uint32_t min_half(const U4& H) {
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  const u16x2 a = __builtin_elementwise_min(__builtin_bit_cast(u16x2, H.x),
                                            __builtin_bit_cast(u16x2, H.y));
  const u16x2 b = __builtin_elementwise_min(__builtin_bit_cast(u16x2, H.z),
                                            __builtin_bit_cast(u16x2, H.w));
  const u16x2 c = __builtin_elementwise_min(a, b);
  return min((uint32_t)c.x, (uint32_t)c.y);
}

// Front voxels of a tile queued at once (a tile with more takes them in chunks).
constexpr uint32_t kQueueCap = 512;
// The front compaction's pieces: kPiecesPerRow lanes per interior row, kPieceBits each.
constexpr uint32_t kPieceBits = kTileRows * kTileX / kWave;
constexpr uint32_t kPiecesPerRow = kTileX / kPieceBits;
constexpr uint64_t kPieceMask = kPieceBits == 64 ? ~0ull : (1ull << (kPieceBits % 64)) - 1ull;
static_assert(kTileX == 64 && kHaloRows <= kWave && kWave % kTileRows == 0 && kPieceBits <= 32,
              "a tile row is one 64-bit word; a lane stages one halo row and compacts one piece");
static_assert(kTileRows <= 32, "interior rows are 5-bit fields of the queue entries");
// Entries of a wavefront's ring of kept blocks: fewer than 64 wait between rounds, and one
// reject iteration adds at most 64.
constexpr uint32_t kRing = 2 * kWave;

// A block of ranks, self-contained so that it can wait across tiles: the voxel (its index
// in the grid), its void mask (direction order) and the block index.
struct RingEntry {
  uint32_t a;
  uint32_t mb;  // void mask | block << 26
};

// LDS image of one tile at the step's start.  Halo row h = hy + (kTileY + 2) hz covers
// y = y0 - 1 + hy, z = z0 - 1 + hz; interior row i = jy + kTileY jz is halo row
// (jy + 1) + (kTileY + 2) (jz + 1).  Bit i of a row mask is voxel x0 + i.
struct TileImage {
  // Halo row h as a 66-bit window of "in-domain candidate at the step's start" (in none
  // of S, the previous step's marks and the walls, except convertible cells of other
  // phases) in three words: bit i of the window (word i / 32, bit i % 32) is voxel
  // x0 - 1 + i, i < 66.
  uint32_t win[kHaloRows][3];
  uint64_t S[kTileRows];     // solid (interior rows)
  uint16_t qo[kQueueCap];    // the queue of front voxels (interior row << 6 | x - x0)
  // the wavefront's blocks to draw (phase A) and its kept blocks with their high-half
  // Philox words (phase B); both outlive the tile
  RingEntry bring[kRing] __attribute__((aligned(8)));
  RingEntry kring[kRing] __attribute__((aligned(8)));
  U4 kH[kRing] __attribute__((aligned(16)));
};

static_assert(kQueueCap <= 1024 && kQueueCap % kWave == 0, "queue slots are 10-bit fields");

// Words of a workgroup's LDS copy of the next map (the tiles of kMarkWords * 32 indices).
constexpr uint32_t kMarkWords = 64;

// Four images (one workgroup of 256 threads) plus the workgroup's own LDS must stay
// within a sixth of the compute unit's 160 KiB, so that six workgroups fit.  LDS is
// granted in granules of 1280 bytes: a sixth holds 21 of them, 26880 bytes, for the
// images and the static arrays (tile block, directions, counters, marks).
static_assert(4 * sizeof(TileImage) + 544 + 4 * kMarkWords <= 26880, "tile image too large");

// The 26-bit void mask (direction order) of front voxel (xl, jy, jz) of the image: the
// three bits x - 1, x, x + 1 of each of the nine neighbouring rows are bits xl..xl + 2
// of the row's window, concatenated in row order with the centre bit dropped.
// (Bits xl..xl + 2 lie in words xl / 32 and xl / 32 + 1 of the window: one funnel shift
// of that word pair per row.)
__device__ __forceinline__ uint32_t tile_void_mask(const TileImage& T, int xl, int jy, int jz) {
  const uint32_t* w0 = &T.win[jy + (kTileY + 2) * jz][xl >> 5];
  uint32_t acc = 0;
#pragma unroll
  for (int kz = 0; kz < 3; ++kz)
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      const uint32_t* wr = w0 + 3 * (ky + (kTileY + 2) * kz);
      const uint32_t w = __builtin_amdgcn_alignbit(wr[1], wr[0], (uint32_t)xl);
      acc |= (w & 7u) << (3 * (ky + 3 * kz));
    }
  return (acc & 0x1FFFu) | ((acc >> 1) & 0x3FFE000u);
}

// Sets the wave's issue priority (0..3; the builtin takes an immediate).
__device__ __forceinline__ void set_wave_priority(uint32_t p) {
  switch (p) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
  }
}

// Dynamic LDS of k_sweep: one TileImage per wavefront.
size_t sweep_lds_bytes(uint32_t block) { return sizeof(TileImage) * (block / kWave); }

// Each wavefront sweeps whole tiles on its own (no workgroup barrier per tile); the
// workgroup resolves its share of list entries into LDS 64 at a time.  The pass reads
// and writes the occupancy planes only (kPlane*), never the byte grid.  kWalls: the
// grids may hold other phases' cells (multi-phase generation, plane W), which are
// neither void nor sources.  kLiteral: a realization with the literal front rule takes
// as sources, from its second step on, only the voxels grown in the previous step
// (its marks that its tile's fold has not yet moved into S).
// At most 80 VGPRs: six waves per SIMD, which the per-wave LDS images (6.1 KB each)
// allow at the default 256-thread workgroup; the variants for other phases' cells may
// take up to 96 (five waves per SIMD; the resident grid follows what they need).
template <bool kWalls, bool kLiteral>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(kWalls ? 5 : 6)))
void k_sweep(BatchArgs A) {
  extern __shared__ __align__(16) unsigned char sweep_lds[];
  __shared__ uint32_t s_tiles[kWave];
  __shared__ int32_t s_drow[26];
  __shared__ uint32_t s_dhi[32];  // 26..31: 0, read for the empty slots of a block
  __shared__ uint32_t s_key[2];
  __shared__ uint32_t s_kept, s_grown, s_draws, s_blocks, s_next, s_nb;
  __shared__ uint32_t s_marks[kMarkWords];
  const uint32_t G = gridDim.x;
  // logical workgroup index: XCD x (workgroups b with b % 8 == x) holds [x G/8, (x+1) G/8)
  const uint32_t beta = (blockIdx.x % kNumXcd) * (G / kNumXcd) + blockIdx.x / kNumXcd;
  const WgDesc D = A.desc[beta];  // (uniform) this workgroup's share, written with the plan
  const uint32_t lane = lane_id(), wib = uniform(threadIdx.x / kWave);
  TileImage& T = reinterpret_cast<TileImage*>(sweep_lds)[wib];
  if (threadIdx.x == 0) {
    s_kept = 0;
    s_grown = 0;
    s_draws = 0;
    s_blocks = 0;
  }
  for (uint32_t w = threadIdx.x; w < kMarkWords; w += blockDim.x) s_marks[w] = 0;
  const uint32_t r = uniform(D.r);
  // the next map's words [mark_lo / 32, mark_lo / 32 + kMarkWords) are set in LDS when
  // they hold every tile this workgroup can list, then or-ed into the map at the end
  uint32_t mark_lo = 0;
  bool lds_marks = false;
  uint32_t* map_flush = nullptr;
  if (r != kNoReal) {
    Real& R = A.reals[r];
    Ctl& c = R.ctl;
    const Geometry g = R.g;
    const Tiles tl = R.tl;
    const uint32_t ntx = tl.ntx;
    if (threadIdx.x < 26u) {  // plane row offset of direction d in 32-bit words (read after
                              // the first barrier)
      const int d = (int)threadIdx.x;
      s_drow[d] = ((dir_field(kDirDY, d) - 1) + (dir_field(kDirDZ, d) - 1) * g.ny) *
                  (int32_t)(2u * ntx);
    }
    const uint32_t k0 = uniform(R.k0), k1 = uniform(R.k1);
    if (threadIdx.x == 0) {  // read after the first barrier
      s_key[0] = k0;
      s_key[1] = k1;
    }
    const uint32_t u_lo = uniform(D.u_lo), u_hi = uniform(D.u_hi), n_share = uniform(D.n);
    const uint32_t t = uniform((uint32_t)c.step);
    const bool run = uniform(c.mode) == kModeRun;
    // the planes: S, the previous step's marks M[(t - 1) & 1] (folded into S by the
    // owner of their tile during this pass), this step's marks M[t & 1] and the walls
    const uint32_t pw = uniform(R.pwords);
    uint64_t* __restrict__ plS = (uint64_t*)uniform64((uint64_t)R.planes);
    const uint64_t* __restrict__ plP = plS + (size_t)pw * (kPlaneM0 + ((t + 1u) & 1u));
    uint32_t* __restrict__ mark32 = (uint32_t*)(plS + (size_t)pw * (kPlaneM0 + (t & 1u)));
    const uint64_t* __restrict__ plW =
        kWalls && uniform(R.walls) != 0 ? plS + (size_t)pw * kPlaneW : nullptr;
    // interacting phases: the cells of other phases this one may convert, and the table
    const InteractTable* __restrict__ itab =
        kWalls ? (const InteractTable*)uniform64((uint64_t)R.itab) : nullptr;
    const uint64_t* __restrict__ plX = itab ? plS + (size_t)pw * kPlaneX : nullptr;
    const uint8_t* __restrict__ labels = R.grid;
    // all ones where the solid rows are the previous step's new voxels only
    const uint64_t lit = kLiteral && uniform(R.literal) != 0 && t > 0 ? ~0ull : 0ull;
    const DrawThresholds th =
        draw_thresholds(uniform64(c.T[0]), uniform64(c.T[1]), uniform64(c.T[2]));
    if (threadIdx.x < 26u) {  // read after the first barrier
      uint32_t hf = th.hi_face, he = th.hi_edge, hc = th.hi_corner;
      if (itab) {  // the largest high half a target of each class can have
        hf = max(hf, R.ihi_max[0]);
        he = max(he, R.ihi_max[1]);
        hc = max(hc, R.ihi_max[2]);
      }
      const uint32_t d = threadIdx.x;
      s_dhi[d] = ((kCornerDirs >> d) & 1u) ? hc : (((kEdgeDirs >> d) & 1u) ? he : hf);
    } else if (threadIdx.x < 32u) {
      s_dhi[threadIdx.x] = 0u;
    }
    // the tile maps: listed for this pass (read), listed for the next (set here)
    const bool full = uniform(R.form) == kFormAllTiles;
    const uint32_t mw = tile_map_words(tl.n);
    uint32_t* const maps = (uint32_t*)uniform64((uint64_t)R.maps);
    const g_u32* __restrict__ map_in = (const g_u32*)(maps + (uniform(c.cur) ? mw : 0u));
    uint32_t* __restrict__ map_out = maps + (uniform(c.cur) ? 0u : mw);
    {
      const uint32_t reach = ntx * tl.nty + ntx + 1u;  // index distance of a neighbour tile
      mark_lo = (u_lo > reach ? u_lo - reach : 0u) & ~31u;
      lds_marks = !full && (uint64_t)u_hi + reach - mark_lo <= 32ull * kMarkWords;
      map_flush = map_out + (mark_lo >> 5);
    }
    uint32_t kept_w = 0, draws_l = 0, blocks_l = 0;
    uint32_t grown = 0;  // voxels grown by this lane's claims
    uint32_t taken = 0;  // listed tiles of the share in the blocks before this one
    // the next map's bit of tile un
    auto mark_tile = [&](uint32_t un) __attribute__((always_inline)) {
      if (lds_marks)
        atomicOr(&s_marks[(un - mark_lo) >> 5], 1u << (un & 31u));
      else
        global_or_nr(map_out + (un >> 5), 1u << (un & 31u));
    };
    // Phase B of step 5 (below): the wavefront's kept blocks wait in a ring across tiles,
    // entries [head, tail), and are decided 64 at a time, so that every round but the
    // share's last is full.  Each entry is drawn again, its ranks decided exactly and
    // claimed; a passing rank whose target leaves the entry's tile lists the target's tile
    // (first claim or not: the target was void).
    uint32_t head = 0, tail = 0;  // (uniform)
    auto decide_round = [&](uint32_t n) __attribute__((always_inline)) {  // the n <= 64 entries from head
      wave_sync();
      if (lane < n) {
        const uint32_t slot = (head + lane) & (kRing - 1u);
        const RingEntry e = T.kring[slot];
        const U4 H = T.kH[slot];
        const uint32_t blk = e.mb >> 26;
        const uint32_t m = drop_low_ranks(e.mb & 0x3FFFFFFu, 8u * blk);  // earlier blocks'
        const uint32_t q = g.div_nx.div(e.a);  // row y + ny z of the voxel
        const uint32_t ex = e.a - q * (uint32_t)g.nx, ez = g.div_ny.div(q);
        const uint32_t ey = q - ez * (uint32_t)g.ny;
        uint32_t passed = 0;
        grown += sweep_block<kWalls>(mark32, k0, k1, s_key, s_drow, s_dhi, e.a, q * (2u * ntx),
                                     ex, t, blk, m, H, th, &passed, g, labels, itab);
        if (!full) {  // (the all-tiles form lists every tile anyway)
          const uint32_t xl = ex % kTileX, jy = ey % kTileY, jz = ez % kTileZ;
          const uint32_t leave = (xl == 0 ? kDxNeg : 0u) | (xl == kTileX - 1 ? kDxPos : 0u) |
                                 (jy == 0 ? kDyNeg : 0u) | (jy == kTileY - 1 ? kDyPos : 0u) |
                                 (jz == 0 ? kDzNeg : 0u) | (jz == kTileZ - 1 ? kDzPos : 0u);
          uint32_t out = passed & leave;
          while (out) {
            const int d = __builtin_ctz(out);
            out &= out - 1u;
            // the target (in the domain: its claim was issued)
            const uint32_t xn = ex + (uint32_t)dir_field(kDirDX, d) - 1u,
                           yn = ey + (uint32_t)dir_field(kDirDY, d) - 1u,
                           zn = ez + (uint32_t)dir_field(kDirDZ, d) - 1u;
            mark_tile(xn / kTileX + ntx * (yn / kTileY + tl.nty * (zn / kTileZ)));
          }
        }
      }
      head += n;
      wave_sync();
    };
    // Phase A: the wavefront's blocks to draw wait in a ring across tiles too, entries
    // [bhead, btail), and are drawn 64 at a time.  A block is kept (goes to the ring of
    // phase B) only if one of its high half-words is at or below the largest high-half
    // threshold: no rank of any other block can pass.
    uint32_t hmax = max(th.hi_face, max(th.hi_edge, th.hi_corner));
    if (itab) hmax = max(hmax, max(R.ihi_max[0], max(R.ihi_max[1], R.ihi_max[2])));
    uint32_t bhead = 0, btail = 0;  // (uniform)
    auto reject_round = [&](uint32_t n) __attribute__((always_inline)) {  // the n <= 64 entries from bhead
      wave_sync();
      RingEntry e{0u, 0u};
      U4 H{0u, 0u, 0u, 0u};
      bool keep = false;
      if (lane < n) {
        e = T.bring[(bhead + lane) & (kRing - 1u)];
        H = philox10(e.a, t, e.mb >> 26, kTagGrowHi, k0, k1);
        // only the block's ranks count: slots past the voxel's last void are masked
        const uint32_t rk = min(8u, (uint32_t)__builtin_popcount(e.mb & 0x3FFFFFFu) - 8u * (e.mb >> 26));
        U4 Hm = H;
        Hm.x |= rk >= 2u ? 0u : (rk == 1u ? 0xFFFF0000u : ~0u);
        Hm.y |= rk >= 4u ? 0u : (rk == 3u ? 0xFFFF0000u : ~0u);
        Hm.z |= rk >= 6u ? 0u : (rk == 5u ? 0xFFFF0000u : ~0u);
        Hm.w |= rk >= 8u ? 0u : (rk == 7u ? 0xFFFF0000u : ~0u);
        keep = min_half(Hm) <= hmax;
      }
      bhead += n;
      const uint64_t kept = __ballot(keep);
      if (kept) {
        if (keep) {  // (phase B reads the block's words instead of drawing them again)
          const uint32_t slot = (tail + __builtin_amdgcn_mbcnt_hi(
                                            (uint32_t)(kept >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)kept, 0u))) &
                                (kRing - 1u);
          T.kring[slot] = e;
          T.kH[slot] = H;
        }
        tail += (uint32_t)__popcll(kept);
        if (tail - head >= (uint32_t)kWave) decide_round(kWave);
      }
      wave_sync();
    };
    for (uint32_t ub = u_lo; ub < u_hi; ub += kWave) {
      __syncthreads();  // the previous block of tiles is consumed
      if (threadIdx.x < (uint32_t)kWave) {
        // the block's listed tiles, in index order (every tile for the all-tiles form)
        const uint32_t u = ub + lane;
        bool listed = u < u_hi;
        if (listed && !full) listed = ((map_in[u >> 5] >> (u & 31u)) & 1u) != 0u;
        const uint64_t lm = __ballot(listed);
        if (listed)
          s_tiles[__builtin_amdgcn_mbcnt_hi((uint32_t)(lm >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)lm, 0u))] = u;
        if (lane == 0) s_nb = (uint32_t)__popcll(lm);
      }
      if (threadIdx.x == 0) s_next = 0;
      __syncthreads();
      const uint32_t nb = uniform(s_nb);
      // each wavefront takes the block's next tile when it is done with one
      for (;;) {
        uint32_t jn = 0;
        if (lane == 0) jn = atomicAdd(&s_next, 1u);
        const uint32_t j = uniform((uint32_t)__builtin_amdgcn_readfirstlane(jn));
        if (j >= nb) break;
        // The compute unit's arbiter favours older waves: of its resident workgroups
        // the last dispatched would finish long after the first.  A wave's priority
        // falls as its workgroup's share is taken, so workgroups that are behind get
        // issue slots first and all finish together.
        set_wave_priority(3u - min(3u, 4u * (taken + j) / max(n_share, 1u)));
        const uint32_t u = uniform(s_tiles[j]);
        if (u >= tl.n) {
          if (lane == 0) atomicOr(&c.bad_entry, 1u);
          continue;
        }
        const uint32_t q1 = tl.div_ntx.div(u);
        const uint32_t iz = tl.div_nty.div(q1);
        const int32_t x0 = (int32_t)(u - q1 * tl.ntx) * kTileX;
        const int32_t y0 = (int32_t)(q1 - iz * tl.nty) * kTileY;
        const int32_t z0 = (int32_t)iz * kTileZ;
        wave_sync();  // the previous tile's image is no longer read
        // 1. stage the tile and its one-voxel halo from the planes: lane h < kHaloRows takes
        // halo row h (y = y0 - 1 + h % (kTileY + 2), z = z0 - 1 + h / (kTileY + 2)) and loads
        // the row's words ix - 1, ix and ix + 1 of S, of the previous step's marks and of the
        // walls; bit 63 of word ix - 1 is voxel x0 - 1 and bit 0 of word ix + 1 voxel
        // x0 + 64.  A row outside the domain loads a clamped row and is masked.
        const uint32_t ix = (uint32_t)x0 / (uint32_t)kTileX;
        const bool has_l = ix > 0, has_r = ix + 1u < ntx;  // (uniform)
        // voxels of word ix inside the domain in x (uniform)
        const uint64_t xin = (uint32_t)g.nx - (uint32_t)x0 >= (uint32_t)kTileX
                                 ? ~0ull
                                 : (1ull << ((uint32_t)g.nx - (uint32_t)x0)) - 1ull;
        const int32_t hy_ = (int32_t)(lane % (kTileY + 2)), hz_ = (int32_t)(lane / (kTileY + 2));
        const int32_t yh = y0 - 1 + hy_, zh = z0 - 1 + hz_;
        const bool rin = lane < (uint32_t)kHaloRows && yh >= 0 && yh < g.ny && zh >= 0 &&
                         zh < g.nz;
        const uint32_t wb = ((uint32_t)min(max(yh, 0), g.ny - 1) +
                             (uint32_t)g.ny * (uint32_t)min(max(zh, 0), g.nz - 1)) * ntx + ix;
        const uint32_t wl = has_l ? wb - 1u : wb, wr = has_r ? wb + 1u : wb;
        // (global loads: a flat load would also hold up every wait on LDS)
        typedef const __attribute__((address_space(1))) uint64_t gq;
        const uint64_t sC = ((gq*)plS)[wb], pC = ((gq*)plP)[wb];
        const uint64_t sL = ((gq*)plS)[wl], pL = ((gq*)plP)[wl];
        const uint64_t sR = ((gq*)plS)[wr], pR = ((gq*)plP)[wr];
        uint64_t oC = sC | pC, oL = sL | pL, oR = sR | pR;  // occupied at the step's start
        if (kWalls && plW) {  // other phases' cells are not candidates, unless convertible
          uint64_t wC = ((gq*)plW)[wb], wL = ((gq*)plW)[wl], wR = ((gq*)plW)[wr];
          if (plX) {
            wC &= ~((gq*)plX)[wb];
            wL &= ~((gq*)plX)[wl];
            wR &= ~((gq*)plX)[wr];
          }
          oC |= wC;
          oL |= wL;
          oR |= wR;
        }
        {
          const uint64_t vm = rin ? ~oC & xin : 0ull;
          const uint32_t vl = rin && has_l ? (uint32_t)(~oL >> 63) : 0u;
          const uint32_t vr = rin && has_r ? (uint32_t)(~oR & 1ull) : 0u;
          if (lane < (uint32_t)kHaloRows) {
            T.win[lane][0] = (uint32_t)vm << 1 | vl;
            T.win[lane][1] = (uint32_t)(vm >> 31);
            T.win[lane][2] = (uint32_t)(vm >> 63) | vr << 1;
          }
        }
        // interior row i < kTileRows is halo row (i % kTileY + 1) + (kTileY + 2) (i / kTileY
        // + 1): its words come from that lane.  Solid = S | previous marks (literal rule:
        // the previous marks not yet in S); the tile's owner folds the previous marks of its
        // rows into S (a plain store: S only gains bits the readers already count as solid
        // through the marks).
        {
          const uint32_t hi = (lane % kTileY + 1u) + (kTileY + 2u) * (lane / kTileY + 1u);
          const uint32_t src = lane < (uint32_t)kTileRows ? hi : lane;
          const uint64_t s_i = (uint64_t)(uint32_t)__shfl((int)(uint32_t)(sC >> 32), (int)src, kWave) << 32 |
                               (uint32_t)__shfl((int)(uint32_t)sC, (int)src, kWave);
          const uint64_t p_i = (uint64_t)(uint32_t)__shfl((int)(uint32_t)(pC >> 32), (int)src, kWave) << 32 |
                               (uint32_t)__shfl((int)(uint32_t)pC, (int)src, kWave);
          const bool in_i = __shfl((int)rin, (int)src, kWave) != 0;
          const uint32_t wb_i = (uint32_t)__shfl((int)wb, (int)src, kWave);
          if (lane < (uint32_t)kTileRows) {
            const uint64_t fresh = p_i & ~s_i;  // grown in the previous step
            uint64_t sm = (s_i | p_i) & xin;
            if (kLiteral) sm = (fresh & lit) | (sm & ~lit);
            T.S[lane] = in_i ? sm : 0ull;
            if (in_i && fresh != 0ull) ((g_u64*)plS)[wb_i] = s_i | p_i;
          }
        }
        wave_sync();
        // 2. front rows (solid with a void neighbour) and their prefix
        uint64_t F = 0;
        if (lane < (uint32_t)kTileRows) {
          const int jy = (int)lane % kTileY, jz = (int)lane / kTileY;
          uint64_t D = 0;
#pragma unroll
          for (int kz = 0; kz < 3; ++kz)
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
              const int h = (jy + ky) + (kTileY + 2) * (jz + kz);
              const uint64_t lo = (uint64_t)T.win[h][1] << 32 | T.win[h][0],
                             hi = T.win[h][2];
              // x - 1 neighbours: lo; x: V; x + 1 neighbours: window shifted down by two
              D |= lo | (lo >> 1) | (hi << 63) | (lo >> 2) | (hi << 62);
            }
          F = T.S[lane] & D;
        }
        // 3. compact the front voxels into the queue: the 64 lanes split the tile's
        // kTileRows x 64 front bits into pieces of kPieceBits, lane L taking bits
        // kPieceBits (L % kPiecesPerRow) onwards of interior row L / kPiecesPerRow (in
        // row-major order the lanes' pieces follow each other), so one wave prefix places
        // every piece
        const uint32_t prow = lane / kPiecesPerRow, poff = (lane % kPiecesPerRow) * kPieceBits;
        const uint64_t Fr =
            (uint64_t)(uint32_t)__shfl((int)(uint32_t)(F >> 32), (int)prow, kWave) << 32 |
            (uint32_t)__shfl((int)(uint32_t)F, (int)prow, kWave);
        const uint32_t piece = (uint32_t)((Fr >> poff) & kPieceMask);
        uint32_t nq_l;
        uint32_t pos = wave_prefix((uint32_t)__builtin_popcount(piece), &nq_l);
        const uint32_t nq = uniform(nq_l);
        kept_w += nq;
        if (!run || nq == 0) continue;
        // steps 4 and 5 take the queue kQueueCap voxels at a time, in queue order
        for (uint32_t cb = 0; cb < nq; cb += kQueueCap) {
          const uint32_t nc = min(nq - cb, kQueueCap);
          wave_sync();  // the previous chunk's queue is consumed
          {
            uint32_t p = pos - cb;  // (modulo 2^32: positions before the chunk wrap)
            for (uint32_t c = piece; c; c &= c - 1u, ++p)
              if (p < kQueueCap)
                T.qo[p] = (uint16_t)(prow << 6 | (poff + (uint32_t)__builtin_ctz(c)));
          }
          wave_sync();
          // 4. each front voxel's void mask and its blocks of ranks (eight ranks a block);
          // the blocks enter the wavefront's ring of phase A, block by block
          for (uint32_t kb = 0; kb < nc; kb += kWave) {
            const uint32_t k = kb + lane;
            uint32_t nb = 0, va = 0, vm = 0;
            if (k < nc) {
              const uint32_t ent = T.qo[k];
              const uint32_t i = ent >> 6, xl = ent & 63u;
              vm = tile_void_mask(T, (int)xl, (int)(i % kTileY), (int)(i / kTileY));
              const uint32_t nv = (uint32_t)__builtin_popcount(vm);
              nb = (nv + 7u) >> 3;
              draws_l += nv;
              blocks_l += nb;
              va = ((uint32_t)x0 + xl) + ((uint32_t)y0 + i % kTileY) * (uint32_t)g.nx +
                   ((uint32_t)z0 + i / kTileY) * g.nxy;
            }
            for (uint32_t blk = 0;; ++blk) {
              const bool has = blk < nb;
              const uint64_t bal = __ballot(has);
              if (!bal) break;
              if (has)
                T.bring[(btail + __builtin_amdgcn_mbcnt_hi(
                                     (uint32_t)(bal >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))) &
                        (kRing - 1u)] = RingEntry{va, vm | blk << 26};
              btail += (uint32_t)__popcll(bal);
              // 5. draws and claims (Sec. 2.3 step 3, Eq. (1)): phase A as soon as 64
              // blocks wait, phase B as soon as 64 kept blocks wait
              if (btail - bhead >= (uint32_t)kWave) reject_round(kWave);
            }
          }
        }
        // 6. list the tiles that may hold F_{t+1} for the next pass, by setting their bits
        // in the next map (an atomic whose old value is not needed: nothing waits for it):
        // this tile (it has front voxels) here, the tiles its claims reach in decide_round
        if (!full && lane == 0) mark_tile(u);
      }
      taken += nb;
    }
    // the share's last, partial rounds
    if (btail != bhead) reject_round(btail - bhead);
    if (tail != head) decide_round(tail - head);
    const uint32_t grown_w = wave_sum(grown);
    const uint32_t draws_w = wave_sum(draws_l), blocks_w = wave_sum(blocks_l);
    if (lane == 0) {
      if (kept_w) atomicAdd(&s_kept, kept_w);
      if (grown_w) atomicAdd(&s_grown, grown_w);
      if (draws_w) atomicAdd(&s_draws, draws_w);
      if (blocks_w) atomicAdd(&s_blocks, blocks_w);
    }
  }
  __syncthreads();
  if (lds_marks) {  // (uniform)
    for (uint32_t w = threadIdx.x; w < kMarkWords; w += blockDim.x) {
      const uint32_t v = s_marks[w];
      if (v) global_or_nr(map_flush + w, v);
    }
  }
  if (r != kNoReal && threadIdx.x == 0)
    A.rec[beta] = WgRec{r, s_kept, s_grown, s_draws, s_blocks, {0u, 0u, 0u}};
}

template __global__ void k_sweep<false, false>(BatchArgs A);
template __global__ void k_sweep<true, false>(BatchArgs A);
template __global__ void k_sweep<false, true>(BatchArgs A);
template __global__ void k_sweep<true, true>(BatchArgs A);


// End of a fused pass (one workgroup of 1024 threads, launched after k_sweep): sums the
// workgroup records per realization in LDS, ends the step of every realization with a
// pending pass (a6: log, count, status, Eq. (1) thresholds of the next step) and writes
// the shares of the next pass (plan_shares, which also clears each continuing
// realization's map of this pass).  Its loads of records and loop state are issued
// together at the start.
__global__ __launch_bounds__(1024) void k_sweep_end(BatchArgs A) {
  constexpr uint32_t kRecPerThread = kMaxSweepGrid / 1024;
  __shared__ uint8_t s_info[kMaxBatch];
  __shared__ uint32_t s_tn[kMaxBatch], s_sum[4];
  __shared__ uint32_t* s_maps[kMaxBatch];
  // the per-realization sums, then plan_shares' arrays
  constexpr size_t kSumBytes = (2 * sizeof(uint32_t) + 2 * sizeof(unsigned long long)) * kMaxBatch;
  constexpr size_t kPlanBytes = sizeof(uint32_t) * (kMaxBatch + 3 * (kMaxBatch + 1) + kMaxSweepGrid);
  __shared__ __align__(16) unsigned char s_raw[kSumBytes > kPlanBytes ? kSumBytes : kPlanBytes];
  unsigned long long* acc_draws = reinterpret_cast<unsigned long long*>(s_raw);
  unsigned long long* acc_blocks = acc_draws + kMaxBatch;
  uint32_t* acc_kept = reinterpret_cast<uint32_t*>(acc_blocks + kMaxBatch);
  uint32_t* acc_grown = acc_kept + kMaxBatch;
  uint32_t* p_n = reinterpret_cast<uint32_t*>(s_raw);
  uint32_t* p_wo = p_n + kMaxBatch;
  uint32_t* p_np = p_wo + kMaxBatch + 1;
  uint32_t* p_wg = p_np + kMaxBatch + 1;
  uint32_t* p_ulo = p_wg + kMaxBatch + 1;
  const uint32_t tid = threadIdx.x, lane = lane_id();
  const uint32_t count = A.count, G = A.sweep_grid;
  // one round of loads: control, the first 1024 realizations, every workgroup record
  const uint32_t nwg = A.bctl->nwg;
  EndIn in0{};
  if (tid < count) in0 = end_load(A, tid);
  WgRec rec[kRecPerThread];
#pragma unroll
  for (uint32_t u = 0; u < kRecPerThread; ++u) {
    const uint32_t w = tid + 1024u * u;
    rec[u] = WgRec{kNoReal, 0u, 0u, 0u, 0u, {0u, 0u, 0u}};
    if (w < G) rec[u] = A.rec[w];
  }
  for (uint32_t r = tid; r < count; r += blockDim.x) {
    acc_kept[r] = 0;
    acc_grown[r] = 0;
    acc_draws[r] = 0;
    acc_blocks[r] = 0;
  }
  if (tid < 4) s_sum[tid] = 0;
  __syncthreads();
  // per-realization sums (the records of workgroups w < nwg): workgroups are ordered by
  // realization, so a wavefront whose records belong to one realization adds once
#pragma unroll
  for (uint32_t u = 0; u < kRecPerThread; ++u) {
    if (1024u * u >= nwg) break;  // (uniform)
    const bool in = tid + 1024u * u < nwg;
    if (__ballot(in) == 0) continue;  // (uniform)
    const uint32_t rr = in ? rec[u].r : kNoReal;
    const uint32_t kept = in ? rec[u].kept : 0u, grown = in ? rec[u].grown : 0u;
    const uint32_t draws = in ? rec[u].draws : 0u, blocks = in ? rec[u].blocks : 0u;
    const uint32_t a0 = __shfl(rr, 0, kWave);  // lane 0 holds the wave's first record
    if (__ballot(in && rr != a0) == 0) {
      const uint32_t sk = wave_sum(kept), sg = wave_sum(grown);
      const unsigned long long sd = wave_sum64(draws), sb = wave_sum64(blocks);
      if (lane == 0) {
        atomicAdd(&acc_kept[a0], sk);
        atomicAdd(&acc_grown[a0], sg);
        atomicAdd(&acc_draws[a0], sd);
        atomicAdd(&acc_blocks[a0], sb);
      }
    } else if (in) {
      atomicAdd(&acc_kept[rr], kept);
      atomicAdd(&acc_grown[rr], grown);
      atomicAdd(&acc_draws[rr], (unsigned long long)draws);
      atomicAdd(&acc_blocks[rr], (unsigned long long)blocks);
    }
  }
  __syncthreads();
  // the step ends
  uint32_t pending_n = 0;
  for (uint32_t r = tid; r < count; r += blockDim.x) {
    const EndIn in = r == tid ? in0 : end_load(A, r);
    const bool pending = in.active && pass_end(A, r, in, acc_kept[r], acc_grown[r],
                                                acc_draws[r], acc_blocks[r]);
    pending_n += pending ? 1u : 0u;
    s_info[r] = (uint8_t)((pending ? 1u : 0u) | (in.all ? 2u : 0u) | ((in.cur ^ 1u) & 1u) << 2);
    s_tn[r] = in.tn;
    s_maps[r] = in.maps;
  }
  pending_n = wave_sum(pending_n);
  if (lane == 0 && pending_n) atomicAdd(&s_sum[0], pending_n);
  __syncthreads();
  const uint32_t running = s_sum[0];
  const PlanArrays L{s_info, s_tn, s_maps, p_n, p_wo, p_np, p_wg, p_ulo, s_sum};
  const uint32_t nwg_next = plan_shares(A, L, true);
  if (tid == 0) {
    A.bctl->nwg = nwg_next;
    A.bctl->running = running;
  }
}

// ---------------------------------------------------------------------------
// Full-field growth step (Sec. 2.2, Algorithm 2): the baseline the list-indexed sweep is
// measured against.  Every step visits every cell of the grid: each cell draws for all
// its directions (rand over the whole field, Algorithm 2 line 4; here the four high-half
// Philox blocks of the cell, 32 draws covering its at most 26 ranks), the draws of solid
// cells that fall below their direction's threshold claim the neighbour (the solid mask
// and the shift, lines 5-6), and a second pass over the whole field folds the claims into
// the solid phase (line 8).  The draws are the ones of the draw rule (rank j of the
// cell's void neighbours), so the grids equal the list-indexed ones step for step; only
// the work differs.  Items: plane words (kItemsField); a wavefront takes a chunk of 64
// words one at a time, lane b handling voxel x = 64 ix + b of the word's row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBlock) void k_field_step(BatchArgs A) {
  const uint32_t lane = lane_id();
  uint32_t cr = 0xFFFFFFFFu;  // (wave-uniform) realization of the counts below
  uint32_t front_l = 0, grown_l = 0, draws_l = 0;
  auto flush = [&]() {
    const uint32_t f = wave_sum(front_l), gsum = wave_sum(grown_l), d = wave_sum(draws_l);
    if (lane == 0 && cr != 0xFFFFFFFFu) {
      Ctl& c = A.reals[cr].ctl;
      if (f) atomicAdd(&c.ff_front, f);
      if (gsum) atomicAdd(&c.ff_grown, gsum);
      if (d) atomicAdd((unsigned long long*)&c.ff_draws, (unsigned long long)d);
    }
    front_l = grown_l = draws_l = 0;
  };
  for_each_chunk(A, kItemsField, [&](uint32_t r, uint32_t i) {
    if (r != cr) {
      flush();
      cr = r;
    }
    const Real& R = A.reals[r];
    const uint32_t pw = uniform(R.pwords);
    const uint32_t w0 = i - lane;
    if (w0 >= pw) return;  // (uniform)
    const uint32_t nw = min((uint32_t)kWave, pw - w0);
    const Geometry g = R.g;
    const uint32_t ntx = uniform(R.tl.ntx);
    const FastDiv dntx = R.tl.div_ntx;
    const uint32_t t = uniform((uint32_t)R.ctl.step);
    const bool run = uniform(R.ctl.mode) == kModeRun;
    const uint32_t k0 = uniform(R.k0), k1 = uniform(R.k1);
    const DrawThresholds th = draw_thresholds(uniform64(R.ctl.T[0]), uniform64(R.ctl.T[1]),
                                              uniform64(R.ctl.T[2]));
    uint64_t* const planes = (uint64_t*)uniform64((uint64_t)R.planes);
    const g_u64* __restrict__ S = (const g_u64*)planes;
    const g_u64* __restrict__ W = uniform(R.walls) != 0 ? S + (size_t)pw * kPlaneW : nullptr;
    uint32_t* __restrict__ mark32 = (uint32_t*)(planes + (size_t)pw * kPlaneM0);
    // occupied (solid or another phase's cell) word of the plane(s)
    auto occ = [&](uint32_t w) -> uint64_t { return W ? (S[w] | W[w]) : S[w]; };
    for (uint32_t j = 0; j < nw; ++j) {
      const uint32_t w = w0 + j;
      const uint32_t row = dntx.div(w);  // y + ny z
      const uint32_t ix = w - row * ntx;
      const uint32_t z = g.div_ny.div(row), y = row - z * (uint32_t)g.ny;
      const uint32_t x = ix * (uint32_t)kTileX + lane;
      const bool inx = x < (uint32_t)g.nx;
      // in-domain neighbours in x of this lane's voxel: bit 0 = x - 1, bit 1 = x, bit 2 = x + 1
      const uint32_t in3 = (x > 0 ? 1u : 0u) | 2u | (x + 1u < (uint32_t)g.nx ? 4u : 0u);
      uint32_t acc = 0;  // void neighbours, 3 bits per row (dy, dz), row order
      bool solid = false;
#pragma unroll
      for (int kz = 0; kz < 3; ++kz)
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
          const int32_t yy = (int32_t)y + ky - 1, zz = (int32_t)z + kz - 1;
          if (yy < 0 || yy >= g.ny || zz < 0 || zz >= g.nz) continue;  // (uniform)
          const uint32_t rw = ((uint32_t)yy + (uint32_t)g.ny * (uint32_t)zz) * ntx + ix;
          const uint64_t wm = occ(rw);
          const uint64_t wl = ix > 0 ? occ(rw - 1u) : 0ull;
          const uint64_t wr = ix + 1u < ntx ? occ(rw + 1u) : 0ull;
          // 66-bit window: bit 0 = voxel 64 ix - 1, bit k + 1 = voxel 64 ix + k
          const uint64_t lo = wm << 1 | wl >> 63, hi2 = wm >> 63 | (wr & 1ull) << 1;
          uint32_t b3 = (uint32_t)(lo >> lane) & 7u;
          if (lane >= 62u) b3 = (b3 | (uint32_t)(hi2 << (64u - lane))) & 7u;
          acc |= (~b3 & in3 & 7u) << (3 * (ky + 3 * kz));
          if (ky == 1 && kz == 1) solid = ((S[rw] >> lane) & 1ull) != 0;
        }
      const uint32_t vm = inx ? ((acc & 0x1FFFu) | ((acc >> 1) & 0x3FFE000u)) : 0u;
      solid = solid && inx;
      if (solid && vm) {
        ++front_l;
        draws_l += (uint32_t)__builtin_popcount(vm);
      }
      if (!run || !inx) continue;
      // every cell draws its 32 ranks; the solid mask applies to the result
      const uint32_t a = x + (uint32_t)g.nx * row;
      uint32_t m = vm, pass = 0;
#pragma unroll
      for (uint32_t blk = 0; blk < 4; ++blk) {
        const U4 H = philox10(a, t, blk, kTagGrowHi, k0, k1);
        // (every cell's blocks are drawn, used or not: the full-field work of Algorithm 2)
        asm volatile("" ::"v"(H.x), "v"(H.y), "v"(H.z), "v"(H.w));
        bool have_lo = false;
        U4 L{0, 0, 0, 0};
#pragma unroll
        for (int sl = 0; sl < 8; ++sl) {
          if (!m) break;
          const int d = __builtin_ctz(m);
          m &= m - 1u;
          const uint32_t wv = sl < 2 ? H.x : (sl < 4 ? H.y : (sl < 6 ? H.z : H.w));
          const uint32_t h = (sl & 1) ? (wv >> 16) : (wv & 0xFFFFu);
          const bool corner = ((kCornerDirs >> d) & 1u) != 0, edge = ((kEdgeDirs >> d) & 1u) != 0;
          const uint32_t hi = corner ? th.hi_corner : (edge ? th.hi_edge : th.hi_face);
          bool ok = h < hi;
          if (h == hi) {  // high halves tie: the low half decides
            if (!have_lo) {
              L = philox10(a, t, blk, kTagGrowLo, k0, k1);
              have_lo = true;
            }
            const uint32_t wl2 = sl < 2 ? L.x : (sl < 4 ? L.y : (sl < 6 ? L.z : L.w));
            const uint32_t l = (sl & 1) ? (wl2 >> 16) : (wl2 & 0xFFFFu);
            ok = l < (corner ? th.lo_corner : (edge ? th.lo_edge : th.lo_face));
          }
          if (ok) pass |= 1u << d;
        }
      }
      if (!solid) continue;
      // claims: the target's bit in the mark plane; the first setter owns the voxel
      while (pass) {
        const int d = __builtin_ctz(pass);
        pass &= pass - 1u;
        const uint32_t xq = x + (uint32_t)dir_field(kDirDX, d) - 1u;
        const uint32_t yq = y + (uint32_t)dir_field(kDirDY, d) - 1u;
        const uint32_t zq = z + (uint32_t)dir_field(kDirDZ, d) - 1u;
        const uint32_t q32 = ((yq + (uint32_t)g.ny * zq) * ntx) * 2u + (xq >> 5);
        const uint32_t bit = 1u << (xq & 31u);
        grown_l += (global_or(mark32 + q32, bit) & bit) == 0u;
      }
    }
  });
  flush();
}

// Full-field step, second pass (Algorithm 2 line 8): S |= claims, the mark plane cleared.
__global__ __launch_bounds__(kMaxBlock) void k_field_fold(BatchArgs A) {
  for_each_chunk(A, kItemsField, [&](uint32_t r, uint32_t i) {
    const Real& R = A.reals[r];
    const uint32_t pw = R.pwords;
    if (i >= pw) return;
    g_u64* P = (g_u64*)R.planes;
    const uint64_t m = P[(size_t)kPlaneM0 * pw + i];
    if (m) {
      P[(size_t)kPlaneS * pw + i] |= m;
      P[(size_t)kPlaneM0 * pw + i] = 0ull;
    }
  });
}

// End of a full-field step for every realization with a pending one (one workgroup):
// the step's log, count, loop rule and next thresholds, as at the end of a tile pass.
// reset_running: this pass runs no tile sweep, whose step end restarts the count of
// running realizations.
__global__ __launch_bounds__(1024) void k_field_end(BatchArgs A, uint32_t reset_running) {
  if (reset_running) {
    if (threadIdx.x == 0) A.bctl->running = 0;
    __syncthreads();
  }
  for (uint32_t r = threadIdx.x; r < A.count; r += blockDim.x) {
    Real& R = A.reals[r];
    if (!field_active(R)) continue;
    Ctl& c = R.ctl;
    const uint32_t front = c.ff_front, grown = c.ff_grown;
    const uint64_t draws = c.ff_draws;
    c.ff_front = 0;
    c.ff_grown = 0;
    c.ff_draws = 0;
    // the step's high-half blocks: four for every cell of the field
    const uint64_t blocks = c.mode == kModeRun ? 4ull * R.g.n : 0ull;
    if (pass_end(A, r, end_load(A, r), front, grown, draws, blocks))
      atomicAdd(&A.bctl->running, 1u);
  }
}

// Relabelling of a whole grid (multi-phase generation, Sec. 2.1 steps 4-5): every byte b
// becomes lut[b].  n_words 32-bit words (the grid's padding included: lut[0] must be 0).
__global__ __launch_bounds__(256) void k_map_bytes(uint32_t* __restrict__ words,
                                                   uint32_t n_words, ByteMap m) {
  __shared__ uint32_t t[256];
  t[threadIdx.x] = m.lut[threadIdx.x];
  __syncthreads();
  for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n_words; i += gridDim.x * 256u) {
    const uint32_t x = words[i];
    words[i] = t[x & 255u] | t[(x >> 8) & 255u] << 8 | t[(x >> 16) & 255u] << 16 |
               t[x >> 24] << 24;
  }
}

}  // namespace qsgs
