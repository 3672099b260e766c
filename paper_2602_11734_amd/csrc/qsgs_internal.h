// qsgs_internal.h -- types shared by the kernels and the host side of libqsgs.
//
// Every entry point runs a batch of realizations (one for qsgs_generate, qsgs_seed
// and qsgs_grow_step).  A realization is described by a Real record in device
// memory; per-step kernels walk the concatenation of all realizations' item lists
// through an offset table in which each realization's range is padded to a
// multiple of the wavefront size, so every wavefront serves one realization.
#pragma once

#include "qsgs_device.h"

namespace qsgs {

// floor(a / d) for a < 2^31 as (a * m) >> s with m = ceil(2^s / d), s = 31 + ceil(log2 d):
// the error a (m - 2^s/d) / 2^s < 2^31 / 2^s = 2^-ceil(log2 d) <= 1/d never crosses an
// integer, and m < 2^32 for every d in [1, 2^31).
struct FastDiv {
  uint32_t d, m, s;
  __host__ void init(uint32_t divisor) {
    d = divisor;
    uint32_t l = 0;
    while ((1ull << l) < (uint64_t)divisor) ++l;
    s = 31u + l;
    m = (uint32_t)(((1ull << s) + divisor - 1ull) / divisor);
  }
  __host__ __device__ __forceinline__ uint32_t div(uint32_t a) const {
    return (uint32_t)(((uint64_t)a * m) >> s);
  }
};

struct Geometry {
  int32_t nx, ny, nz;
  uint32_t nxy, n;
  FastDiv div_nx, div_ny;
};

// Spacing buckets: cubes of edge B = s - 1 over the grid; conflicts (L1 <= radius = s - 1)
// lie within one bucket step in each axis.  nb = 0 when there is no spacing (s <= 1).
struct Buckets {
  FastDiv edge;
  uint32_t nbx, nby, nbz, nb;
  int32_t radius;
};

// Loop status codes on the device (the public values plus an internal overflow code).
constexpr int32_t kStatusDone = 1, kStatusExhausted = 2, kStatusMaxSteps = 3,
                  kStatusOverflow = 100;

// Seed candidate states during the spacing rounds.
constexpr uint8_t kLive = 0, kAccepted = 1, kDead = 2;

constexpr int kScanBlock = 1024;       // items per workgroup of the bucket scan
constexpr uint32_t kMaxRounds = 4096;  // spacing rounds (a safety cap; typical runs use < 40)

// Loop state of one realization, carried between kernels.
struct Ctl {
  uint64_t cnt;         // solid count at the start of step `step`
  uint64_t s_star;      // target count S*
  uint64_t t_ref[3];    // reference thresholds (face, edge, corner)
  uint64_t T[3];        // Eq. (1) thresholds of step `step`
  uint32_t front_size;  // |F_t|, held in front buffer `cur`
  uint32_t new_count;   // |New_t| appended during the step
  uint32_t out_count;   // |F_{t+1}| written during the step
  uint32_t cur;         // front buffer (0 or 1) holding F_t
  int32_t step;         // t
  int32_t status;       // 0 while running
  int32_t max_steps;
  uint32_t overflow;    // a list append would have passed its capacity
  uint32_t bad_entry;   // a front entry outside [0, N)
  uint32_t last_new;    // |New| of the last completed step
  uint32_t n_cand;      // seed candidates
  uint32_t n_seeds;     // accepted seeds
};

// Phase of a realization record: an empty slot, waiting for the seeding kernels,
// or in the growth loop (finished ones keep this phase with a non-zero status).
constexpr uint32_t kPhaseEmpty = 0, kPhaseSeed = 1, kPhaseGrow = 2;

// One realization of a batch.
struct Real {
  Geometry g;
  Buckets bk;
  uint8_t* grid;        // caller's grid, qsgs_grid_bytes bytes
  int32_t* f0;          // front buffers, cap entries each
  int32_t* f1;
  int32_t* cand;        // candidates, then the seed list (N entries)
  uint64_t* log;        // per-step log (3 words per step) or null
  uint32_t log_cap;
  uint32_t cap;
  uint32_t boff;        // first bucket of this realization in the batch's bucket arrays
  uint32_t k0, k1;      // Philox key
  uint64_t t_seed;
  int32_t spacing;
  uint32_t phase;
  Ctl ctl;
};

// Batch-wide state.
struct BatchCtl {
  uint32_t running;     // realizations still growing after the last step end
  uint32_t n_sorted;    // bucket-sorted candidates of the spacing rounds
  uint32_t pad[2];
};

// What an offset table counts per realization.
enum ItemKind : uint32_t {
  kItemsVoxels = 0,  // every voxel (seed draw)
  kItemsCand = 1,    // seed candidates
  kItemsSeeds = 2,   // accepted seeds (front construction)
  kItemsGrow = 3,    // F_t of running realizations
  kItemsPrune = 4,   // F_t + New_t of running realizations
};

struct BatchArgs {
  Real* reals;
  uint32_t count;
  uint64_t* off;        // count + 1 item offsets (multiples of kWave)
  BatchCtl* bctl;
  uint32_t* live;       // per-round count of undecided candidates
  // bucket-sorted candidates of all realizations with spacing
  uint32_t* counts;     // per-bucket counts, scanned in place into offsets
  uint32_t* cursor;
  int32_t* sorted_v;
  uint32_t* sorted_r;
  uint64_t* sorted_prio;
  uint8_t* status;
};

__global__ void k_ctl_init(BatchArgs A, uint32_t zero_live);
__global__ void k_offsets(BatchArgs A, uint32_t kind);
__global__ void k_fill_u32(uint32_t* p, uint32_t value, uint32_t n);
__global__ void k_scan_local(uint32_t* data, uint32_t n, uint32_t* sums);
__global__ void k_scan_add(uint32_t* data, uint32_t n, const uint32_t* sums);
__global__ void k_seed_draw(BatchArgs A);
__global__ void k_bucket_count(BatchArgs A);
__global__ void k_bucket_scatter(BatchArgs A, uint32_t total_buckets);
__global__ void k_luby_round(BatchArgs A, uint32_t round);
__global__ void k_collect_seeds(BatchArgs A);
__global__ void k_front_init(BatchArgs A);
__global__ void k_loop_init(BatchArgs A);
__global__ void k_loop_resume(BatchArgs A);
__global__ void k_grow(BatchArgs A);
__global__ void k_prune(BatchArgs A);
__global__ void k_step_end(BatchArgs A);
__global__ void k_rollback(uint8_t* grid, uint32_t n);

}  // namespace qsgs
