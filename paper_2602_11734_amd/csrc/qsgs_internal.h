// qsgs_internal.h -- types shared by the kernels and the host side of libqsgs.
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
// lie within one bucket step in each axis.
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

constexpr int kScanBlock = 1024;        // items per workgroup of the bucket scan
constexpr uint32_t kMaxRounds = 4096;  // spacing rounds (a safety cap; typical runs use < 40)
constexpr uint32_t kLogCap = 65536;    // steps recorded in the per-step log

// Device control block: the growth loop's state, carried between kernels.
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

struct CtlInit {
  uint64_t cnt, s_star, t_ref[3];
  uint32_t front_size, cur;
  int32_t step, max_steps;
};

struct SeedArgs {
  Geometry g;
  uint8_t* grid;
  int32_t* cand;
  Ctl* ctl;
  uint64_t t_seed;
  uint32_t k0, k1;
};

struct MarkArgs {
  uint8_t* grid;
  const int32_t* list;
  Ctl* ctl;
};

struct BucketArgs {
  Geometry g;
  Buckets bk;
  const int32_t* cand;
  uint32_t* counts;         // per-bucket counts, scanned in place into offsets
  uint32_t* cursor;         // scatter cursors (a copy of the offsets)
  const uint32_t* offsets;  // == counts after the scan; nb + 1 entries
  int32_t* sorted_v;
  uint64_t* sorted_prio;
  uint8_t* status;
  uint32_t* live;           // per-round count of undecided candidates
  Ctl* ctl;
  uint32_t k0, k1;
};

struct FrontInitArgs {
  Geometry g;
  const uint8_t* grid;
  const int32_t* seeds;
  int32_t* out;
  uint32_t cap;
  Ctl* ctl;
};

struct StepArgs {
  Geometry g;
  uint8_t* grid;
  int32_t* f0;
  int32_t* f1;
  uint32_t cap;
  Ctl* ctl;
  uint32_t k0, k1;
};

__global__ void k_ctl_init(Ctl* ctl, CtlInit init, uint32_t* live, uint32_t n_live);
__global__ void k_fill_u32(uint32_t* p, uint32_t value, uint32_t n);
__global__ void k_seed_draw(SeedArgs A);
__global__ void k_mark_all_seeds(MarkArgs A);
__global__ void k_bucket_count(BucketArgs A);
__global__ void k_scan_local(uint32_t* data, uint32_t n, uint32_t* sums);
__global__ void k_scan_add(uint32_t* data, uint32_t n, const uint32_t* sums);
__global__ void k_bucket_scatter(BucketArgs A);
__global__ void k_luby_round(BucketArgs A, uint32_t round);
__global__ void k_collect_seeds(BucketArgs A, int32_t* seeds, uint8_t* grid);
__global__ void k_front_init(FrontInitArgs A);
__global__ void k_loop_init(Ctl* ctl, uint32_t cur);
__global__ void k_loop_resume(Ctl* ctl);
__global__ void k_grow(StepArgs A);
__global__ void k_prune(StepArgs A);
__global__ void k_step_end(Ctl* ctl, uint64_t* log, uint32_t log_cap);
__global__ void k_rollback(uint8_t* grid, uint32_t n);

}  // namespace qsgs
