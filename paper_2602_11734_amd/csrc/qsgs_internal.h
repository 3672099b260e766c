// qsgs_internal.h -- types shared by the kernels and the host side of libqsgs.
//
// Every entry point runs a batch of realizations (one for qsgs_generate, qsgs_seed
// and qsgs_grow_step).  A realization is described by a Real record in device
// memory; per-step kernels walk the concatenation of all realizations' item lists
// through an offset table in which each realization's range is padded to a
// multiple of the wavefront size, so every wavefront serves one realization.
#pragma once

#include "qsgs.h"
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

// Tiles of the fused sweep: 64 x 8 x 4 voxels (x, y, z; a tile row is one 64-bit plane
// word).  Tile (ix, iy, iz) has id ix + ntx (iy + nty iz).
constexpr int kTileX = 64, kTileY = 8, kTileZ = 4;
constexpr int kTileRows = kTileY * kTileZ;                // 32 interior rows
constexpr int kHaloRows = (kTileY + 2) * (kTileZ + 2);    // 60 rows with the halo

struct Tiles {
  uint32_t ntx, nty, ntz, n;
  FastDiv div_ntx, div_nty;
};

// Occupancy bit planes of the fused sweep.  A plane holds one bit per voxel in rows of
// ntx 64-bit words: word ix + ntx (y + ny z), bit b is voxel x = 64 ix + b (bits past
// nx stay 0), so a 64 x 8 x 4 tile's interior is 32 whole words.
//   S        solid at the start of the current step (the seeds, then every folded mark);
//   M0, M1   claims of the steps with t even / odd; the pass of step t claims into
//            M[t & 1] and folds the tile's bits of M[(t - 1) & 1] into S.  Solid at the
//            start of step t is S | M[(t - 1) & 1] whether or not the fold has happened.
//            A mark plane keeps bits of earlier steps (never cleared); such cells are
//            also in S, so they are never void and never claimed again;
//   W        (multi-phase generation) cells of other phases: neither void nor sources.
//   X        (interacting phases) cells of the other phases that the growing phase may
//            convert (Sec. 2.1 step 4): candidates like unassigned cells, with their own
//            thresholds.
constexpr uint32_t kPlaneS = 0, kPlaneM0 = 1, kPlaneM1 = 2, kPlaneW = 3, kPlaneX = 4;

// Interaction table of a growing phase (device memory, Sec. 2.1 step 4): for grid byte
// b = 3 + m (a cell of earlier phase m), thr[6 b + c] and thr[6 b + 3 + c] are the high
// and low 16-bit halves of P32(I_c^{n,m}) (c = face, edge, corner; a threshold of 2^32 is
// high half 65536), and bit b of bits marks the phases it may convert.
struct InteractTable {
  uint32_t thr[256 * 6];
  uint32_t bits[8];
};

// Per-step log of a realization: |F_t|, voxels grown in step t, the solid count at the
// start of step t, the step's draws and its high-half Philox blocks.
constexpr uint32_t kLogWords = 5;

// Loop status codes on the device (the public values plus an internal overflow code).
constexpr int32_t kStatusDone = 1, kStatusExhausted = 2, kStatusMaxSteps = 3,
                  kStatusOverflow = 100;

// Seed candidate states during the spacing rounds (kAcceptedNew: accepted in the
// current round, its conflicting candidates not yet marked dead).
constexpr uint8_t kLive = 0, kAccepted = 1, kDead = 2, kAcceptedNew = 3;

constexpr uint32_t kMaxSweepGrid = 8192;  // workgroups of a fused sweep launch (at most)
constexpr uint32_t kMaxBatch = 4096;      // realizations per batch / server slots
constexpr int kScanBlock = 1024;       // items per workgroup of the bucket scan
constexpr uint32_t kMaxRounds = 4096;  // spacing rounds (a safety cap; typical runs use < 40)
constexpr uint32_t kAsyncRounds = 64;  // spacing rounds of the calls without host checks
constexpr int32_t kMaxAsyncSteps = 4096;  // step cap of the calls without host checks

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
  // fused sweep (qsgs_generate*, server): the active tile list of step t in buffer
  // `cur` and the mode of the next pass over it
  uint32_t n_list;      // tiles in the list
  uint32_t mode;        // kModeIdle / kModeRun / kModeFinal
  uint32_t kept;
  uint32_t pad0;
  uint32_t export_state;  // fused sweep: 0 running, 1 stopped (grid to be written), 2 written
  // full-field form: the current step's front, growth and draws, summed by its step kernel
  uint32_t ff_front;
  uint32_t ff_grown;
  uint32_t pad1;
  uint64_t ff_draws;
};

// Growth forms of the whole-generation path: the list-indexed tile sweep (LIETS), the
// full-field step of every cell (Algorithm 2), and the tile sweep over every tile.
constexpr uint32_t kFormList = 0, kFormField = 1, kFormAllTiles = 2;

// Pass modes of the fused sweep: a running pass finds F_t in its tiles and grows from
// it; a final pass only counts F_T and folds the last step's marks (clean 0/1 grid).
constexpr uint32_t kModeIdle = 0, kModeRun = 1, kModeFinal = 2;

// Phase of a realization record: an empty slot, waiting for the seeding kernels,
// or in the growth loop (finished ones keep this phase with a non-zero status).
constexpr uint32_t kPhaseEmpty = 0, kPhaseSeed = 1, kPhaseGrow = 2;

// One realization of a batch.
struct Real {
  Geometry g;
  Buckets bk;
  uint8_t* grid;        // caller's grid, qsgs_grid_bytes bytes
  int32_t* f0;          // front buffers, cap entries each (step API)
  int32_t* f1;
  uint32_t* maps;       // fused sweep: two tile bitmaps of tile_map_words(tiles) words each,
                        // the tiles listed for the pass (half cur) and for the next
  Tiles tl;
  uint32_t form;        // kFormList, kFormField (full-field steps) or kFormAllTiles
  int32_t* cand;        // candidates, then the seed list (N entries)
  uint64_t* log;        // per-step log (3 words per step) or null
  uint32_t log_cap;
  uint32_t cap;         // entries of f0 / f1 (the fused sweep: 2 x tiles, two halves)
  uint32_t boff;        // first bucket of this realization in the batch's bucket arrays
  uint32_t k0, k1;      // Philox key
  uint64_t t_seed;
  int32_t spacing;
  uint32_t phase;
  uint32_t walls;       // the grid holds other phases' cells (bytes >= 4): never cores,
                        // sources or targets; seeding keeps the grid instead of clearing it
  uint32_t literal;     // front rule: the next sources are only this step's new voxels
  // fused sweep: occupancy bit planes of pwords 64-bit words each (see kPlane*)
  uint64_t* planes;
  uint32_t pwords;
  uint32_t pad2;
  // interacting phases: the table of the growing phase (null: independent), and per
  // class the largest high half of its interaction thresholds
  const InteractTable* itab;
  uint32_t ihi_max[3];
  uint32_t pad3;
  Ctl ctl;
};

// Batch-wide state.
struct BatchCtl {
  uint32_t running;     // realizations still growing after the last step end
  uint32_t n_sorted;    // bucket-sorted candidates of the spacing rounds
  uint32_t pad0[2];
  uint32_t grid;        // workgroups of every fused sweep launch
  uint32_t nwg;         // workgroups with a share in the current plan
  uint32_t pad[2];
};

// What one logical workgroup of a fused pass found (written by the workgroup at its end,
// summed per realization by k_sweep_end).
struct WgRec {
  uint32_t r;        // realization
  uint32_t kept;     // front voxels found
  uint32_t grown;    // voxels grown
  uint32_t draws;    // draws made
  uint32_t blocks;   // high-half Philox blocks computed
  uint32_t pad[3];
};

// The share of one logical workgroup in the next fused pass, written with the plan so
// that the workgroup starts from a single load: the listed tiles of realization r with
// index in [u_lo, u_hi), n of them (every tile of the range for the all-tiles form).
constexpr uint32_t kNoReal = 0xFFFFFFFFu;
struct WgDesc {
  uint32_t r;  // realization, or kNoReal: no share in this pass
  uint32_t u_lo, u_hi;
  uint32_t n;
};

// 32-bit words of one tile bitmap of a realization with `tiles` tiles.
__host__ __device__ constexpr uint32_t tile_map_words(uint32_t tiles) {
  return (tiles + 31u) / 32u;
}

// What an offset table counts per realization.
enum ItemKind : uint32_t {
  kItemsVoxels = 0,  // every voxel (seed draw)
  kItemsCand = 1,    // seed candidates
  kItemsSeeds = 2,   // accepted seeds (front construction)
  kItemsGrow = 3,    // F_t of running realizations
  kItemsPrune = 4,   // F_t + New_t of running realizations
  kItemsList = 5,    // listed tiles of realizations with a pending fused pass
  kItemsQuads = 6,   // every aligned group of four voxels (seed draw)
  kItemsPack = 7,    // plane words of freshly seeded realizations (byte grid -> planes)
  kItemsExport = 8,  // plane words of stopped realizations whose grid is not yet written
  kItemsField = 9,   // plane words of full-field realizations with a pending step
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
  // fused sweep
  uint32_t sweep_grid;  // workgroups of every fused sweep launch (a multiple of 8)
  WgRec* rec;           // per logical workgroup of the current pass (kMaxSweepGrid)
  WgDesc* desc;         // per logical workgroup of the next pass (kMaxSweepGrid)
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
__global__ void k_luby_kill(BatchArgs A);
__global__ void k_collect_seeds(BatchArgs A);
__global__ void k_front_init(BatchArgs A);
__global__ void k_loop_init(BatchArgs A);
__global__ void k_loop_resume(BatchArgs A);
__global__ void k_grow(BatchArgs A);
__global__ void k_prune(BatchArgs A);
__global__ void k_step_end(BatchArgs A);
__global__ void k_rollback(uint8_t* grid, uint32_t n);
__global__ void k_seed_tiles(BatchArgs A);
__global__ void k_full_tiles(BatchArgs A);
__global__ void k_sweep_prepare(BatchArgs A);
__global__ void k_pack_planes(BatchArgs A);
__global__ void k_export_planes(BatchArgs A);
__global__ void k_export_done(BatchArgs A);
// up to 256 words of host data carried in kernel arguments
struct WordBlob {
  uint32_t n;
  uint32_t w[256];
};
__global__ void k_put_words(uint32_t* dst, WordBlob b);
__global__ void k_seed_settled(BatchArgs A, uint32_t rounds);
__global__ void k_info_out(BatchArgs A, qsgs_info* out);
__global__ void k_field_step(BatchArgs A);
__global__ void k_field_fold(BatchArgs A);
__global__ void k_field_end(BatchArgs A, uint32_t reset_running);
// dynamic LDS: sweep_lds_bytes(blockDim.x); kWalls: the grids may hold other phases' cells;
// kLiteral: some realizations take only the previous step's new voxels as sources
template <bool kWalls, bool kLiteral> __global__ void k_sweep(BatchArgs A);
size_t sweep_lds_bytes(uint32_t block);
__global__ void k_sweep_end(BatchArgs A);

// Byte relabelling table of k_map_bytes (passed by value).
struct ByteMap {
  uint8_t lut[256];
};
__global__ void k_map_bytes(uint32_t* words, uint32_t n_words, ByteMap m);

}  // namespace qsgs
