// qsgs_kernels.hip -- gfx950 kernels of libqsgs: seeding (Sec. 2.1 step 2), diamond
// seed spacing (Sec. 2.3, Fig. 1D), the list-indexed growth sweep and front
// compaction (Sec. 2.3 steps 2-5, Algorithm 3) with the thresholds of Eq. (1).
//
// Layout: the caller's uint8 grid (v = x + nx*(y + ny*z)), int32 front lists, and a
// device control block that carries the loop state between kernels so the growth
// loop runs without host round trips.
#include "qsgs_internal.h"

namespace qsgs {

// ---------------------------------------------------------------------------
// Neighbourhood of one voxel.  The nine rows (dy, dz) of the 3x3x3 block around
// (x, y, z) are read with byte loads; off-grid neighbours do not exist (the domain
// is not periodic).  Bit d of `voidm` is set for an in-domain neighbour that is
// not solid at the step's start (grid value 0 or 2), bit d of `grown` for one
// already grown during this step (value 2), bit d of `zero` for value 0.
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

// ---------------------------------------------------------------------------
// Control block initialisation (one workgroup).
// ---------------------------------------------------------------------------
__global__ void k_ctl_init(Ctl* ctl, CtlInit init, uint32_t* live, uint32_t n_live) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->cnt = init.cnt;
    ctl->s_star = init.s_star;
    for (int c = 0; c < 3; ++c) {
      ctl->t_ref[c] = init.t_ref[c];
      ctl->T[c] = 0;
    }
    ctl->front_size = init.front_size;
    ctl->new_count = 0;
    ctl->out_count = 0;
    ctl->cur = init.cur;
    ctl->step = init.step;
    ctl->status = 0;
    ctl->max_steps = init.max_steps;
    ctl->overflow = 0;
    ctl->bad_entry = 0;
    ctl->last_new = 0;
    ctl->n_cand = 0;
    ctl->n_seeds = 0;
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_live; i += gridDim.x * blockDim.x)
    live[i] = 0;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = value;
}

// ---------------------------------------------------------------------------
// a1: seed candidates.  Every voxel draws the block at (v, 0, 0, 1); word 0 below
// T_seed makes v a candidate (Sec. 2.1 step 2).  The grid is zeroed in the same
// pass, and candidates are appended with one atomic per wavefront.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_seed_draw(SeedArgs A) {
  const XcdSplit sp(A.g.n);
  for (uint32_t base = sp.begin; base < sp.end; base += sp.stride) {
    const uint32_t v = base + threadIdx.x;
    const bool valid = v < sp.end;
    bool cand = false;
    if (valid) {
      const U4 w = philox10(v, 0u, 0u, kTagSeed, A.k0, A.k1);
      cand = (uint64_t)w.x < A.t_seed;
      A.grid[v] = kVoid;
    }
    const uint32_t pos = wave_append_flag(cand, &A.ctl->n_cand);
    if (cand) A.cand[pos] = (int32_t)v;  // capacity N: cannot overflow
  }
}

// s <= 1: every candidate is a seed.
__global__ __launch_bounds__(kBlock) void k_mark_all_seeds(MarkArgs A) {
  const uint32_t n = A.ctl->n_cand;
  const XcdSplit sp(n);
  for (uint32_t base = sp.begin; base < sp.end; base += sp.stride) {
    const uint32_t i = base + threadIdx.x;
    if (i < sp.end) A.grid[A.list[i]] = kSolid;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) A.ctl->n_seeds = n;
}

// ---------------------------------------------------------------------------
// a2: diamond spacing.  Candidates are bucketed by (x, y, z) / B with B = s - 1, so
// every conflict (L1 distance 1..s-1) lies in one of the 27 surrounding buckets.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bucket_of(const Buckets& bk, uint32_t x, uint32_t y,
                                              uint32_t z) {
  return bk.edge.div(x) + bk.nbx * (bk.edge.div(y) + bk.nby * bk.edge.div(z));
}

__device__ __forceinline__ void coords_of(const Geometry& g, uint32_t v, uint32_t& x, uint32_t& y,
                                          uint32_t& z) {
  const uint32_t yz = g.div_nx.div(v);
  x = v - yz * (uint32_t)g.nx;
  z = g.div_ny.div(yz);
  y = yz - z * (uint32_t)g.ny;
}

__global__ __launch_bounds__(kBlock) void k_bucket_count(BucketArgs A) {
  const uint32_t n = A.ctl->n_cand;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    uint32_t x, y, z;
    coords_of(A.g, (uint32_t)A.cand[i], x, y, z);
    atomicAdd(&A.counts[bucket_of(A.bk, x, y, z)], 1u);
  }
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
    uint32_t t = lane < kScanBlock / kWave ? wave_tot[lane] : 0u;
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

__global__ __launch_bounds__(kBlock) void k_bucket_scatter(BucketArgs A) {
  const uint32_t n = A.ctl->n_cand;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t v = (uint32_t)A.cand[i];
    uint32_t x, y, z;
    coords_of(A.g, v, x, y, z);
    const uint32_t pos = atomicAdd(&A.cursor[bucket_of(A.bk, x, y, z)], 1u);
    const U4 w = philox10(v, 0u, 0u, kTagSeed, A.k0, A.k1);
    A.sorted_v[pos] = (int32_t)v;
    A.sorted_prio[pos] = ((uint64_t)w.y << 32) | (uint64_t)w.z;
    A.status[pos] = kLive;
  }
}

// One priority round.  A live candidate that sees an accepted conflicting candidate
// dies; one whose key (priority, v) is below every live conflicting candidate's key
// is accepted.  Statuses only move forward, and a stale read can only delay a
// decision, never change it, so in-place updates reproduce the greedy order.
__global__ __launch_bounds__(kBlock) void k_luby_round(BucketArgs A, uint32_t round) {
  const uint32_t n = A.ctl->n_cand;
  const int32_t r = A.bk.radius;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    bool still_live = false;
    if (i < n && A.status[i] == kLive) {
      const uint32_t v = (uint32_t)A.sorted_v[i];
      const uint64_t p = A.sorted_prio[i];
      uint32_t x, y, z;
      coords_of(A.g, v, x, y, z);
      const int32_t bx = (int32_t)A.bk.edge.div(x), by = (int32_t)A.bk.edge.div(y),
                    bz = (int32_t)A.bk.edge.div(z);
      bool killed = false, minimal = true;
      for (int32_t cz = max(bz - 1, 0); cz <= min(bz + 1, (int32_t)A.bk.nbz - 1) && !killed; ++cz)
        for (int32_t cy = max(by - 1, 0); cy <= min(by + 1, (int32_t)A.bk.nby - 1) && !killed;
             ++cy)
          for (int32_t cx = max(bx - 1, 0); cx <= min(bx + 1, (int32_t)A.bk.nbx - 1) && !killed;
               ++cx) {
            const uint32_t b = (uint32_t)cx + A.bk.nbx * ((uint32_t)cy + A.bk.nby * (uint32_t)cz);
            const uint32_t e = A.offsets[b + 1];
            for (uint32_t j = A.offsets[b]; j < e; ++j) {
              if (j == i) continue;
              const uint32_t w = (uint32_t)A.sorted_v[j];
              uint32_t wx, wy, wz;
              coords_of(A.g, w, wx, wy, wz);
              const int32_t dist = abs((int32_t)wx - (int32_t)x) + abs((int32_t)wy - (int32_t)y) +
                                   abs((int32_t)wz - (int32_t)z);
              if (dist > r) continue;
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
      if (killed) {
        A.status[i] = kDead;
      } else if (minimal) {
        A.status[i] = kAccepted;
      } else {
        still_live = true;
      }
    }
    wave_append_flag(still_live, &A.live[round]);
  }
}

// Accepted candidates become seeds: 1 in the grid, appended to the seed list.
__global__ __launch_bounds__(kBlock) void k_collect_seeds(BucketArgs A, int32_t* seeds,
                                                          uint8_t* grid) {
  const uint32_t n = A.ctl->n_cand;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const bool acc = i < n && A.status[i] == kAccepted;
    const uint32_t pos = wave_append_flag(acc, &A.ctl->n_seeds);
    if (acc) {
      const int32_t v = A.sorted_v[i];
      grid[v] = kSolid;
      seeds[pos] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// a3: initial front F_0 = interface(G_0) (Sec. 2.3 step 2), compacted from the seed
// list; then the loop state for step 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_front_init(FrontInitArgs A) {
  const uint32_t n = A.ctl->n_seeds;
  const XcdSplit sp(n);
  for (uint32_t base = sp.begin; base < sp.end; base += sp.stride) {
    const uint32_t i = base + threadIdx.x;
    bool keep = false;
    if (i < sp.end) {
      const uint32_t v = (uint32_t)A.seeds[i];
      uint32_t x, y, z;
      coords_of(A.g, v, x, y, z);
      keep = load_neighbourhood(A.grid, A.g, v, x, y, z).zero != 0;
    }
    const uint32_t pos = wave_append_flag(keep, &A.ctl->out_count);
    if (keep) {
      if (pos < A.cap)
        A.out[pos] = A.seeds[i];
      else
        A.ctl->overflow = 1u;
    }
  }
}

__device__ __forceinline__ void set_status_and_thresholds(Ctl* ctl) {
  int32_t status = 0;
  if (ctl->cnt >= ctl->s_star)
    status = kStatusDone;
  else if (ctl->front_size == 0)
    status = kStatusExhausted;
  else if (ctl->step >= ctl->max_steps)
    status = kStatusMaxSteps;
  ctl->status = status;
  if (status == 0)
    for (int c = 0; c < 3; ++c) ctl->T[c] = eq1_threshold(ctl->t_ref[c], ctl->cnt, ctl->s_star);
}

__global__ void k_loop_init(Ctl* ctl, uint32_t cur) {
  ctl->cnt = ctl->n_seeds;
  ctl->front_size = ctl->out_count;
  ctl->out_count = 0;
  ctl->new_count = 0;
  ctl->step = 0;
  ctl->cur = cur;
  set_status_and_thresholds(ctl);
}

// Loop state supplied by the host (qsgs_grow_step): only the status and thresholds.
__global__ void k_loop_resume(Ctl* ctl) { set_status_and_thresholds(ctl); }

// ---------------------------------------------------------------------------
// a4: growth sweep of step t.  One thread per front voxel a: its in-domain void
// neighbours (at the step's start) take the draws of ranks j = 0, 1, ... in
// ascending direction; a passing draw claims the neighbour with a 32-bit atomicOr
// on the grid word (value 2 = grown this step), and the first claimer appends it
// after F_t in the same list.  Sources are F_t only (Jacobi step).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_grow(StepArgs A) {
  Ctl* ctl = A.ctl;
  if (ctl->status != 0) return;
  const uint32_t t = (uint32_t)ctl->step;
  const uint32_t nf = ctl->front_size;
  int32_t* __restrict__ fin = ctl->cur ? A.f1 : A.f0;
  const uint64_t T0 = ctl->T[0], T1 = ctl->T[1], T2 = ctl->T[2];
  const XcdSplit sp(nf);
  for (uint32_t base = sp.begin; base < sp.end; base += sp.stride) {
    const uint32_t i = base + threadIdx.x;
    uint32_t a = 0, claims = 0;
    if (i < sp.end) {
      a = (uint32_t)fin[i];
      if (a >= A.g.n) {
        ctl->bad_entry = 1u;
      } else {
        uint32_t x, y, z;
        coords_of(A.g, a, x, y, z);
        const Nbhd nb = load_neighbourhood(A.grid, A.g, a, x, y, z);
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
              H = philox10(a, t, (uint32_t)blk, kTagGrowHi, A.k0, A.k1);
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
                L = philox10(a, t, (uint32_t)blk, kTagGrowLo, A.k0, A.k1);
                lo_block = blk;
              }
              const uint32_t wl = pick(L, (j >> 1) & 3u);
              const uint32_t l = (j & 1u) ? (wl >> 16) : (wl & 0xFFFFu);
              pass = l < (uint32_t)(Tc & 0xFFFFu);
            }
            if (pass) {
              const uint32_t q = (uint32_t)((int32_t)a + dir_offset(A.g, d));
              const uint32_t sh = (q & 3u) * 8u;
              const uint32_t old = atomicOr((uint32_t*)(A.grid + (q & ~3u)), (uint32_t)kGrown << sh);
              if (((old >> sh) & 0xFFu) == kVoid) claims |= 1u << d;
            }
          }
          ++j;
        }
      }
    }
    const uint32_t cnt = (uint32_t)__builtin_popcount(claims);
    uint32_t pos = wave_append(cnt, &ctl->new_count);
    while (claims) {
      const int d = __builtin_ctz(claims);
      claims &= claims - 1u;
      const uint32_t slot = nf + pos;
      if (slot < A.cap)
        fin[slot] = (int32_t)((int32_t)a + dir_offset(A.g, d));
      else
        ctl->overflow = 1u;
      ++pos;
    }
  }
}

// ---------------------------------------------------------------------------
// a5: prune and compaction (Sec. 2.3 step 4): F_{t+1} = the entries of F_t and New_t
// that still have an in-domain void neighbour, appended with one atomic per wave.
// New voxels are folded from 2 to 1 here.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_prune(StepArgs A) {
  Ctl* ctl = A.ctl;
  if (ctl->status != 0 || ctl->overflow) return;
  const uint32_t nf = ctl->front_size;
  const uint32_t n_in = nf + ctl->new_count;
  const int32_t* __restrict__ fin = ctl->cur ? A.f1 : A.f0;
  int32_t* __restrict__ fout = ctl->cur ? A.f0 : A.f1;
  const XcdSplit sp(n_in);
  for (uint32_t base = sp.begin; base < sp.end; base += sp.stride) {
    const uint32_t i = base + threadIdx.x;
    bool keep = false;
    uint32_t v = 0;
    if (i < sp.end) {
      v = (uint32_t)fin[i];
      if (v < A.g.n) {
        uint32_t x, y, z;
        coords_of(A.g, v, x, y, z);
        keep = load_neighbourhood(A.grid, A.g, v, x, y, z).zero != 0;
        if (i >= nf) A.grid[v] = kSolid;
      }
    }
    const uint32_t pos = wave_append_flag(keep, &ctl->out_count);
    if (keep) {
      if (pos < A.cap)
        fout[pos] = (int32_t)v;
      else
        ctl->overflow = 1u;
    }
  }
}

// ---------------------------------------------------------------------------
// a6: end of step t (one thread): log, count update, front swap, DEF-9 status and
// the thresholds of step t+1 from the new count (Eq. (1)).
// ---------------------------------------------------------------------------
__global__ void k_step_end(Ctl* ctl, uint64_t* log, uint32_t log_cap) {
  if (ctl->status != 0) return;
  if (ctl->overflow) {
    ctl->status = kStatusOverflow;
    return;
  }
  const uint32_t t = (uint32_t)ctl->step;
  const uint32_t grown = ctl->new_count;
  if (log && t < log_cap) {
    log[3 * t + 0] = ctl->front_size;
    log[3 * t + 1] = grown;
    log[3 * t + 2] = ctl->cnt;
  }
  ctl->cnt += grown;
  ctl->last_new = grown;
  ctl->front_size = ctl->out_count;
  ctl->out_count = 0;
  ctl->new_count = 0;
  ctl->cur ^= 1u;
  ctl->step = (int32_t)t + 1;
  set_status_and_thresholds(ctl);
}

// Undo a step that overflowed its front capacity: grown voxels (2) back to void.
__global__ __launch_bounds__(kBlock) void k_rollback(uint8_t* grid, uint32_t n) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    if (grid[v] == kGrown) grid[v] = kVoid;
}

}  // namespace qsgs
