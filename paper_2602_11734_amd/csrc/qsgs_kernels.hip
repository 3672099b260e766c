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

// Calls body(r, local) for every chunk of kWave items of the current offset table;
// `local` is this lane's index within realization r's (padded) item range.
template <typename Body>
__device__ __forceinline__ void for_each_chunk(const BatchArgs& A, Body&& body) {
  const uint64_t total = uniform64(A.off[A.count]);
  const uint64_t nchunks = total / kWave;
  const uint32_t wib = uniform(threadIdx.x / kWave);
  const uint32_t wpb = blockDim.x / kWave;
  const uint32_t xcd = blockIdx.x % kNumXcd;
  const uint64_t per = (nchunks + kNumXcd - 1) / kNumXcd;
  const uint64_t c_beg = min(nchunks, (uint64_t)xcd * per);
  const uint64_t c_end = min(nchunks, c_beg + per);
  const uint64_t stride = (uint64_t)(gridDim.x / kNumXcd) * wpb;
  uint32_t r = 0;
  uint64_t lo = 0, hi = 0;
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
// Neighbourhood of one voxel.  The nine rows (dy, dz) of the 3x3x3 block around
// (x, y, z) are read with byte loads; off-grid neighbours do not exist (the domain
// is not periodic).  Bit d of `voidm` is set for an in-domain neighbour that is not
// solid at the step's start (grid value 0 or 2), bit d of `grown` for one already
// grown during this step (value 2), bit d of `zero` for value 0.
// ---------------------------------------------------------------------------
struct Nbhd {
  uint32_t voidm, grown, zero;
};

__device__ __forceinline__ Nbhd load_neighbourhood(const uint8_t* __restrict__ grid,
                                                   const Geometry& g, uint32_t a, uint32_t x,
                                                   uint32_t y, uint32_t z) {
  Nbhd r{0u, 0u, 0u};
  const bool xm = x > 0, xp = x + 1 < (uint32_t)g.nx;
  const bool ym = y > 0, yp = y + 1 < (uint32_t)g.ny;
  const bool zm = z > 0, zp = z + 1 < (uint32_t)g.nz;
  int d = 0;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const bool row_in = (dz < 0 ? zm : (dz > 0 ? zp : true)) &&
                          (dy < 0 ? ym : (dy > 0 ? yp : true));
      const int32_t row = (int32_t)a + dy * g.nx + dz * (int32_t)g.nxy;
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        const bool in = row_in && (dx < 0 ? xm : (dx > 0 ? xp : true));
        if (in) {
          const uint8_t b = grid[row + dx];
          r.voidm |= (uint32_t)(b != kSolid) << d;
          r.grown |= (uint32_t)(b == kGrown) << d;
          r.zero |= (uint32_t)(b == kVoid) << d;
        }
        ++d;
      }
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
// multiple of kWave, exclusive-scanned (one workgroup).  The prune table also
// restarts the count of running realizations that k_step_end accumulates.
__global__ __launch_bounds__(1024) void k_offsets(BatchArgs A, uint32_t kind) {
  __shared__ uint64_t wave_tot[1024 / kWave];
  __shared__ uint64_t carry;
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
  if (threadIdx.x == 0) {
    carry = 0;
    if (kind == kItemsPrune) A.bctl->running = 0;
  }
  __syncthreads();
  for (uint32_t base = 0; base < A.count; base += blockDim.x) {
    const uint32_t r = base + threadIdx.x;
    uint64_t v = 0;
    if (r < A.count) {
      const Real& R = A.reals[r];
      const Ctl& c = R.ctl;
      const bool seeding = R.phase == kPhaseSeed;
      const bool growing = R.phase == kPhaseGrow && c.status == 0;
      switch (kind) {
        case kItemsVoxels: v = seeding ? R.g.n : 0; break;
        case kItemsCand: v = seeding ? c.n_cand : 0; break;
        case kItemsSeeds: v = seeding ? c.n_seeds : 0; break;
        case kItemsGrow: v = growing ? c.front_size : 0; break;
        default: v = (growing && !c.overflow) ? (uint64_t)c.front_size + c.new_count : 0;
      }
      v = (v + kWave - 1) / kWave * kWave;
    }
    uint64_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint64_t t = __shfl_up(incl, o, kWave);
      if (lane >= (uint32_t)o) incl += t;
    }
    if (lane == kWave - 1) wave_tot[wv] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t s = carry;
      for (uint32_t w = 0; w < nw; ++w) {
        const uint64_t t = wave_tot[w];
        wave_tot[w] = s;
        s += t;
      }
      carry = s;
    }
    __syncthreads();
    if (r < A.count) A.off[r] = wave_tot[wv] + incl - v;
    __syncthreads();
  }
  if (threadIdx.x == 0) A.off[A.count] = carry;
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
  for_each_chunk(A, [&](uint32_t r, uint32_t v) {
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
  for_each_chunk(A, [&](uint32_t r, uint32_t i) {
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
  for_each_chunk(A, [&](uint32_t r, uint32_t i) {
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
  for_each_chunk(A, [&](uint32_t r, uint32_t i) {
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

// ---------------------------------------------------------------------------
// a4: growth sweep of step t (items: F_t of running realizations).  One thread per
// front voxel a: its in-domain void neighbours (at the step's start) take the draws
// of ranks j = 0, 1, ... in ascending direction; a passing draw claims the
// neighbour with a 32-bit atomicOr on the grid word (value 2 = grown this step),
// and the first claimer appends it after F_t in the same list.  Sources are F_t
// only (Jacobi step).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMaxBlock) void k_grow(BatchArgs A) {
  for_each_chunk(A, [&](uint32_t r, uint32_t i) {
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
              const uint32_t old =
                  atomicOr((uint32_t*)(R.grid + (q & ~3u)), (uint32_t)kGrown << sh);
              if (((old >> sh) & 0xFFu) == kVoid) claims |= 1u << d;
            }
          }
          ++j;
        }
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
  for_each_chunk(A, [&](uint32_t r, uint32_t i) {
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

}  // namespace qsgs
