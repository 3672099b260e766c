/*
 * qsgs_oracle.c -- CPU oracle for LIETS-QSGS (arXiv 2602.11734).
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow, single-threaded reference the GPU
 * library is checked against.  Loaded only by the tests, the package smoke check
 * and the benchmark's CPU-baseline leg.  It shares no code with the GPU library.
 *
 * Everything is integer: 32-bit Philox words compared against 32-bit thresholds,
 * so a result is a bit-exact function of (dims, parameters, key).
 *
 * Where the paper is silent or ambiguous the oracle takes one reading; each is
 * named at the function that applies it.
 */
#include "qsgs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11).  Each round multiplies counter words 0 and 2 by */
/* two odd 32-bit constants, keeps both 32-bit halves of the products, mixes */
/* the high halves with the other two words and the round key, and permutes; */
/* the key is advanced by two Weyl constants between rounds.                 */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_keyed(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         uint32_t out[4]) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t k[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
  orc_philox4x32_10(ctr, k, out);
}

/* ------------------------------------------------------------------------ */
/* Directions.  The paper's growth tries every neighbour direction i with its */
/* own probability (Sec. 2.1 step 3, Sec. 2.2 step 3) and describes QSGS by a */
/* seed probability and three directional growth probabilities (Sec. 1).  In  */
/* 3D that is the 26-neighbourhood in three classes: 6 face, 12 edge, 8       */
/* corner neighbours.                                                         */
/* ------------------------------------------------------------------------ */
void orc_direction(int32_t d, int32_t* dx, int32_t* dy, int32_t* dz, int32_t* cls) {
  int32_t k = d < 13 ? d : d + 1; /* skip the centre, k = 13 */
  int32_t x = k % 3 - 1, y = (k / 3) % 3 - 1, z = k / 9 - 1;
  *dx = x; *dy = y; *dz = z;
  *cls = abs(x) + abs(y) + abs(z) - 1;
}

/* Neighbour of voxel (x,y,z) in direction d, or -1 when it lies outside the
 * domain (the domain is not periodic: the list-indexed growth only considers
 * neighbours "inside the domain", Algorithm 3). */
static int64_t neighbour(int32_t nx, int32_t ny, int32_t nz, int32_t x, int32_t y, int32_t z,
                         int32_t d) {
  int32_t dx, dy, dz, c;
  orc_direction(d, &dx, &dy, &dz, &c);
  int32_t qx = x + dx, qy = y + dy, qz = z + dz;
  if (qx < 0 || qx >= nx || qy < 0 || qy >= ny || qz < 0 || qz >= nz) return -1;
  return (int64_t)qx + (int64_t)nx * ((int64_t)qy + (int64_t)ny * (int64_t)qz);
}

static void coords(int32_t nx, int32_t ny, int64_t v, int32_t* x, int32_t* y, int32_t* z) {
  *x = (int32_t)(v % nx);
  *y = (int32_t)((v / nx) % ny);
  *z = (int32_t)(v / ((int64_t)nx * ny));
}

/* ------------------------------------------------------------------------ */
/* Probabilities as integer thresholds.  The paper accepts when a uniform     */
/* draw "does not exceed" a probability (Sec. 2.1 steps 2-3) and writes "<" in */
/* Algorithms 2 and 3; on a continuum the two differ on a null set.  Here a   */
/* 32-bit word w is accepted iff w < T with T = floor(p 2^32), so the event   */
/* has probability exactly T / 2^32.  p * 2^32 is exact in binary64.          */
/* ------------------------------------------------------------------------ */
uint64_t orc_prob_threshold(double p) {
  if (!(p > 0.0)) return 0;
  if (p >= 1.0) return (uint64_t)1 << 32;
  return (uint64_t)floor(p * 4294967296.0);
}

/* Sec. 2.3 step 5: iterate while phi_a < phi_s with phi_a = count / N.  For an
 * integer count that is count < ceil(phi_s N), evaluated in binary64. */
int64_t orc_target_count(double phi_s, int64_t n) {
  double t = ceil(phi_s * (double)n);
  if (t < 0.0) t = 0.0;
  if (t > (double)n) t = (double)n;
  return (int64_t)t;
}

/* Eq. (1): G_i(phi) = G_i,ref (phi_s - 0.95 phi_a) / (0.05 phi_s), i.e. the
 * reference probability times 20 - 19 phi_a / phi_s.  With phi_a / phi_s read as
 * count / S* the factor is (20 S* - 19 count) / S*, and the threshold is the
 * exact floor of T_ref times that factor, capped at 2^32 (probability 1).
 * count is the solid count at the start of the step (phi_a is recomputed after
 * each iteration, Algorithm 3). */
uint64_t orc_growth_threshold(uint64_t t_ref, int64_t cnt, int64_t s_star) {
  unsigned __int128 num = (unsigned __int128)(20 * s_star - 19 * cnt);
  unsigned __int128 t = ((unsigned __int128)t_ref * num) / (unsigned __int128)s_star;
  if (t > ((unsigned __int128)1 << 32)) t = (unsigned __int128)1 << 32;
  return (uint64_t)t;
}

/* Growth draw.  The paper draws an independent uniform per candidate neighbour
 * and direction (Sec. 2.3 step 3).  Here the draws of source a at step t are
 * assigned to its void in-domain neighbours in ascending direction order: the
 * j-th such neighbour receives the 32-bit value (H << 16) | L, where H and L
 * are the same 16-bit half (j & 1) of word (j >> 1) & 3 of two Philox blocks at
 * counters (a, t, j >> 3, TAG_GROW_HI) and (a, t, j >> 3, TAG_GROW_LO). */
uint32_t orc_growth_draw(uint64_t key, int32_t a, uint32_t t, int32_t j) {
  uint32_t hi[4], lo[4];
  philox_keyed(key, (uint32_t)a, t, (uint32_t)(j >> 3), ORC_TAG_GROW_HI, hi);
  philox_keyed(key, (uint32_t)a, t, (uint32_t)(j >> 3), ORC_TAG_GROW_LO, lo);
  int word = (j >> 1) & 3, shift = (j & 1) * 16;
  uint32_t h = (hi[word] >> shift) & 0xFFFFu;
  uint32_t l = (lo[word] >> shift) & 0xFFFFu;
  return (h << 16) | l;
}

/* ------------------------------------------------------------------------ */
/* Seeding (Sec. 2.1 step 2): every cell draws a uniform and becomes a core   */
/* when the draw does not exceed the seed probability.  Cell v uses the block */
/* at counter (v, 0, 0, TAG_SEED): word 0 decides candidacy, words 1 and 2    */
/* form its 64-bit priority for the spacing rule.                             */
/* ------------------------------------------------------------------------ */
int64_t orc_seed_candidates(int32_t nx, int32_t ny, int32_t nz, uint64_t key, uint64_t t_seed,
                            int32_t* cand, uint64_t* prio, int64_t cap) {
  int64_t n = (int64_t)nx * ny * nz, k = 0;
  for (int64_t v = 0; v < n; ++v) {
    uint32_t w[4];
    philox_keyed(key, (uint32_t)v, 0u, 0u, ORC_TAG_SEED, w);
    if ((uint64_t)w[0] < t_seed) {
      if (k < cap) {
        cand[k] = (int32_t)v;
        prio[k] = ((uint64_t)w[1] << 32) | (uint64_t)w[2];
      }
      ++k;
    }
  }
  return k;
}

typedef struct {
  uint64_t prio;
  int32_t v;
} keyed_cand;

static int cmp_keyed(const void* a, const void* b) {
  const keyed_cand* x = (const keyed_cand*)a;
  const keyed_cand* y = (const keyed_cand*)b;
  if (x->prio != y->prio) return x->prio < y->prio ? -1 : 1;
  if (x->v != y->v) return x->v < y->v ? -1 : 1;
  return 0;
}

/* Seed spacing (Sec. 2.3, Fig. 1D): the minimum allowed seed distance s is
 * enforced with a diamond (octahedral, L1) exclusion zone.  Two candidates
 * conflict when 0 < |u - v|_1 <= s - 1, so accepted seeds are pairwise at L1
 * distance >= s; s <= 1 imposes nothing.  The paper does not fix the order in
 * which candidates are accepted; the reading here is greedy acceptance in
 * ascending (priority, v): a candidate is accepted iff no already accepted seed
 * lies in its diamond of radius s - 1. */
int64_t orc_seed_select(int32_t nx, int32_t ny, int32_t nz, int32_t spacing, int64_t n_cand,
                        const int32_t* cand, const uint64_t* prio, uint8_t* grid) {
  if (spacing <= 1) {
    for (int64_t i = 0; i < n_cand; ++i) grid[cand[i]] = 1;
    return n_cand;
  }
  keyed_cand* order = (keyed_cand*)malloc(sizeof(keyed_cand) * (size_t)(n_cand > 0 ? n_cand : 1));
  for (int64_t i = 0; i < n_cand; ++i) {
    order[i].prio = prio[i];
    order[i].v = cand[i];
  }
  qsort(order, (size_t)n_cand, sizeof(keyed_cand), cmp_keyed);
  const int32_t r = spacing - 1;
  int64_t accepted = 0;
  for (int64_t i = 0; i < n_cand; ++i) {
    int32_t x, y, z;
    coords(nx, ny, order[i].v, &x, &y, &z);
    int blocked = 0;
    for (int32_t dz = -r; dz <= r && !blocked; ++dz) {
      int32_t rz = r - abs(dz);
      for (int32_t dy = -rz; dy <= rz && !blocked; ++dy) {
        int32_t ry = rz - abs(dy);
        for (int32_t dx = -ry; dx <= ry; ++dx) {
          int32_t qx = x + dx, qy = y + dy, qz = z + dz;
          if (qx < 0 || qx >= nx || qy < 0 || qy >= ny || qz < 0 || qz >= nz) continue;
          int64_t q = (int64_t)qx + (int64_t)nx * ((int64_t)qy + (int64_t)ny * qz);
          if (grid[q] == 1) { blocked = 1; break; }
        }
      }
    }
    if (!blocked) {
      grid[order[i].v] = 1;
      ++accepted;
    }
  }
  free(order);
  return accepted;
}

/* ------------------------------------------------------------------------ */
/* Active front (Sec. 2.3 step 2): the solid cells with at least one void     */
/* neighbour.  Algorithm 3 starts from all solid cells instead; cells with no */
/* void neighbour have no candidate, so both starts give the same growth.     */
/* ------------------------------------------------------------------------ */
static int has_void_neighbour(int32_t nx, int32_t ny, int32_t nz, const uint8_t* grid,
                              int64_t v) {
  int32_t x, y, z;
  coords(nx, ny, v, &x, &y, &z);
  for (int32_t d = 0; d < 26; ++d) {
    int64_t q = neighbour(nx, ny, nz, x, y, z, d);
    if (q >= 0 && grid[q] == 0) return 1;
  }
  return 0;
}

int64_t orc_interface(int32_t nx, int32_t ny, int32_t nz, const uint8_t* grid, int32_t* out) {
  int64_t n = (int64_t)nx * ny * nz, k = 0;
  for (int64_t v = 0; v < n; ++v)
    if (grid[v] == 1 && has_void_neighbour(nx, ny, nz, grid, v)) out[k++] = (int32_t)v;
  return k;
}

/* Void-at-step-start in-domain neighbours of a, one bit per direction. */
static uint32_t void_mask(int32_t nx, int32_t ny, int32_t nz, const uint8_t* grid, int64_t a) {
  int32_t x, y, z;
  coords(nx, ny, a, &x, &y, &z);
  uint32_t m = 0;
  for (int32_t d = 0; d < 26; ++d) {
    int64_t q = neighbour(nx, ny, nz, x, y, z, d);
    if (q >= 0 && grid[q] == 0) m |= 1u << d;
  }
  return m;
}

/* Cells of the one-voxel band around a list of cells: the cells within Chebyshev
 * distance 1 of a listed cell, counted once each (stamp[q] == mark marks a counted cell;
 * the caller passes a mark not yet in stamp). */
static int64_t band_count(int32_t nx, int32_t ny, int32_t nz, const int32_t* cells, int64_t k,
                          uint32_t* stamp, uint32_t mark) {
  int64_t c = 0;
  for (int64_t i = 0; i < k; ++i) {
    int32_t x, y, z;
    coords(nx, ny, cells[i], &x, &y, &z);
    for (int32_t dz = -1; dz <= 1; ++dz)
      for (int32_t dy = -1; dy <= 1; ++dy)
        for (int32_t dx = -1; dx <= 1; ++dx) {
          const int32_t X = x + dx, Y = y + dy, Z = z + dz;
          if (X < 0 || Y < 0 || Z < 0 || X >= nx || Y >= ny || Z >= nz) continue;
          const int64_t q = X + (int64_t)nx * (Y + (int64_t)ny * Z);
          if (stamp[q] != mark) {
            stamp[q] = mark;
            ++c;
          }
        }
  }
  return c;
}

static int popcount32(uint32_t m) {
  int c = 0;
  while (m) { m &= m - 1; ++c; }
  return c;
}

/* ------------------------------------------------------------------------ */
/* One list-indexed growth iteration (Sec. 2.3 steps 3-4, Algorithm 3).      */
/*   for each direction d: N_d = neighbours of A inside the domain,          */
/*   C_d = the void ones, one draw per candidate, accepted cells are set and */
/*   collected in A_new; afterwards A <- prune(A u A_new) and phi_a updates. */
/* Readings: new cells act as sources only from the next iteration (Sec. 2.3 */
/* step 5), so C_d is taken from the state at the start of the iteration --  */
/* a cell already grown by an earlier direction this iteration is marked 2   */
/* and is not collected twice; the pruned front is the union of the old     */
/* front and A_new (the front must keep "solid cells with at least one void */
/* neighbour", and only then does the scheme match the full-field one).      */
/* ------------------------------------------------------------------------ */
int64_t orc_step_liets(int32_t nx, int32_t ny, int32_t nz, uint8_t* grid, const int32_t* A,
                       int64_t nA, uint32_t t, const uint64_t T[3], uint64_t key,
                       int32_t* A_next, int64_t* n_new, uint32_t* mask_scratch,
                       int32_t* new_scratch, uint64_t* attempts, uint64_t* successes) {
  /* C_d membership for every source and direction, from the iteration's start. */
  for (int64_t i = 0; i < nA; ++i) mask_scratch[i] = void_mask(nx, ny, nz, grid, A[i]);

  int64_t added = 0;
  for (int32_t d = 0; d < 26; ++d) {
    int32_t dx, dy, dz, cls;
    orc_direction(d, &dx, &dy, &dz, &cls);
    for (int64_t i = 0; i < nA; ++i) {
      uint32_t m = mask_scratch[i];
      if (!((m >> d) & 1u)) continue; /* neighbour outside the domain or not void */
      int32_t j = popcount32(m & ((1u << d) - 1u));
      uint32_t w = orc_growth_draw(key, A[i], t, j);
      if (attempts) attempts[d] += 1;
      if ((uint64_t)w < T[cls]) {
        if (successes) successes[d] += 1;
        int64_t q = (int64_t)A[i] + dx + (int64_t)nx * (dy + (int64_t)ny * dz);
        if (grid[q] == 0) {
          grid[q] = 2;
          new_scratch[added++] = (int32_t)q;
        }
      }
    }
  }
  for (int64_t k = 0; k < added; ++k) grid[new_scratch[k]] = 1;

  /* prune(A u A_new): keep the cells that still have a void neighbour. */
  int64_t kept = 0;
  for (int64_t i = 0; i < nA; ++i)
    if (has_void_neighbour(nx, ny, nz, grid, A[i])) A_next[kept++] = A[i];
  for (int64_t k = 0; k < added; ++k)
    if (has_void_neighbour(nx, ny, nz, grid, new_scratch[k])) A_next[kept++] = new_scratch[k];
  *n_new = added;
  return kept;
}

/* ------------------------------------------------------------------------ */
/* One full-field growth iteration (Sec. 2.2, Algorithm 2): for every         */
/* direction, each solid cell of the iteration's start draws, the accepted    */
/* ones are shifted by one cell in that direction (without wrap-around) and  */
/* OR-ed into the phase.  The draw of (a, d) is the one the list form uses.  */
/* ------------------------------------------------------------------------ */
int64_t orc_step_fullfield(int32_t nx, int32_t ny, int32_t nz, uint8_t* grid, uint32_t t,
                           const uint64_t T[3], uint64_t key) {
  int64_t n = (int64_t)nx * ny * nz;
  for (int32_t d = 0; d < 26; ++d) {
    int32_t dx, dy, dz, cls;
    orc_direction(d, &dx, &dy, &dz, &cls);
    for (int64_t a = 0; a < n; ++a) {
      if (grid[a] != 1) continue; /* solid_mask: solid at the iteration's start */
      int32_t x, y, z;
      coords(nx, ny, a, &x, &y, &z);
      int64_t q = neighbour(nx, ny, nz, x, y, z, d);
      /* shifted off the grid, or not void at the iteration's start (solid, or a cell of
       * another phase: value 2 = grown this step, still void at the start) */
      if (q < 0 || (grid[q] != 0 && grid[q] != 2)) continue;
      /* rank of d among a's void-at-start neighbours */
      int32_t j = 0;
      for (int32_t e = 0; e < d; ++e) {
        int64_t r = neighbour(nx, ny, nz, x, y, z, e);
        if (r >= 0 && (grid[r] == 0 || grid[r] == 2)) ++j;
      }
      if ((uint64_t)orc_growth_draw(key, (int32_t)a, t, j) < T[cls]) grid[q] = 2;
    }
  }
  int64_t grown = 0;
  for (int64_t v = 0; v < n; ++v)
    if (grid[v] == 2) { grid[v] = 1; ++grown; }
  return grown;
}

/* ------------------------------------------------------------------------ */
/* Whole generation on a grid that holds 0 (void, open to the phase) and     */
/* possibly cells of other phases (any value other than 0, 1 and 2): those   */
/* are never cores, sources or targets.  Candidates on them are dropped.     */
/* ------------------------------------------------------------------------ */
static int32_t generate_on(int32_t nx, int32_t ny, int32_t nz, const orc_params* p,
                           uint8_t* grid, orc_result* res, int32_t* birth, int64_t* log_front,
                           int64_t* log_new, int64_t* log_count, int64_t* log_draws,
                           int64_t* log_blocks, int64_t* log_band, int64_t* log_band_union,
                           int32_t log_cap);

/* ------------------------------------------------------------------------ */
/* Whole generation: seeding, front construction, then list-indexed steps    */
/* while phi_a < phi_s and A is not empty (Sec. 2.3 step 5, Algorithm 3).    */
/* Readings: no trimming of the last step's overshoot; an empty front with   */
/* count < S* ends the run as "exhausted"; a step cap ends it as "max steps". */
/* The step log also records the step's work: draws = one per (front cell,   */
/* void neighbour) pair (Sec. 2.3 step 3), blocks = Philox blocks of the     */
/* high halves, one per eight ranks of a front cell (the draw rule).         */
/* ------------------------------------------------------------------------ */
int32_t orc_generate(int32_t nx, int32_t ny, int32_t nz, const orc_params* p, uint8_t* grid,
                     orc_result* res, int32_t* birth, int64_t* log_front, int64_t* log_new,
                     int64_t* log_count, int64_t* log_draws, int64_t* log_blocks,
                     int64_t* log_band, int64_t* log_band_union, int32_t log_cap) {
  memset(grid, 0, (size_t)nx * ny * nz);
  return generate_on(nx, ny, nz, p, grid, res, birth, log_front, log_new, log_count, log_draws,
                     log_blocks, log_band, log_band_union, log_cap);
}

static int32_t generate_on(int32_t nx, int32_t ny, int32_t nz, const orc_params* p,
                           uint8_t* grid, orc_result* res, int32_t* birth, int64_t* log_front,
                           int64_t* log_new, int64_t* log_count, int64_t* log_draws,
                           int64_t* log_blocks, int64_t* log_band, int64_t* log_band_union,
                           int32_t log_cap) {
  const int64_t n = (int64_t)nx * ny * nz;
  const int64_t s_star = orc_target_count(p->solid_fraction, n);
  const uint64_t t_seed = orc_prob_threshold(p->seed_prob);
  uint64_t t_ref[3];
  for (int c = 0; c < 3; ++c) t_ref[c] = orc_prob_threshold(p->g_ref[c]);
  const int32_t max_steps = p->max_steps > 0 ? p->max_steps : ORC_DEFAULT_MAX_STEPS;

  int32_t* A = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* A_next = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* added = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  uint32_t* mask = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
  uint64_t* prio = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  /* band sizes of the step log (cells within one voxel of F_t, of F_t u New_t) */
  uint32_t* stamp =
      (log_band || log_band_union) ? (uint32_t*)calloc((size_t)n, sizeof(uint32_t)) : NULL;

  int64_t n_drawn = orc_seed_candidates(nx, ny, nz, p->key, t_seed, A, prio, n);
  int64_t n_cand = 0; /* cores only on cells still open (Sec. 2.1 step 4) */
  for (int64_t i = 0; i < n_drawn; ++i)
    if (grid[A[i]] == 0) {
      A[n_cand] = A[i];
      prio[n_cand] = prio[i];
      ++n_cand;
    }
  int64_t n_seeds = orc_seed_select(nx, ny, nz, p->spacing, n_cand, A, prio, grid);
  if (birth)
    for (int64_t v = 0; v < n; ++v) birth[v] = grid[v] == 1 ? 0 : -1;

  int64_t cnt = n_seeds;
  int64_t nA = orc_interface(nx, ny, nz, grid, A);
  int32_t t = 0;
  while (cnt < s_star && nA > 0 && t < max_steps) {
    uint64_t T[3];
    for (int c = 0; c < 3; ++c) T[c] = orc_growth_threshold(t_ref[c], cnt, s_star);
    int64_t n_new = 0;
    int64_t nA_next = orc_step_liets(nx, ny, nz, grid, A, nA, (uint32_t)t, T, p->key, A_next,
                                     &n_new, mask, added, NULL, NULL);
    if (p->front_rule == 1) {
      /* Algorithm 3 as printed: only this step's new cells that still have a void
       * neighbour are the next step's sources (failed sources are dropped) */
      nA_next = 0;
      for (int64_t k = 0; k < n_new; ++k)
        if (has_void_neighbour(nx, ny, nz, grid, added[k])) A_next[nA_next++] = added[k];
    }
    if (t < log_cap) {
      if (log_front) log_front[t] = nA;
      if (log_new) log_new[t] = n_new;
      if (log_count) log_count[t] = cnt;
      /* the masks of the step's sources, as orc_step_liets took them */
      int64_t draws = 0, blocks = 0;
      for (int64_t i = 0; i < nA; ++i) {
        int c = popcount32(mask[i]);
        draws += c;
        blocks += (c + 7) / 8;
      }
      if (log_draws) log_draws[t] = draws;
      if (log_blocks) log_blocks[t] = blocks;
      if (stamp) { /* A still holds F_t, `added` New_t */
        const uint32_t m1 = 2u * (uint32_t)t + 1u, m2 = m1 + 1u;
        const int64_t bf = band_count(nx, ny, nz, A, nA, stamp, m1);
        const int64_t bu = band_count(nx, ny, nz, A, nA, stamp, m2) +
                           band_count(nx, ny, nz, added, n_new, stamp, m2);
        if (log_band) log_band[t] = bf;
        if (log_band_union) log_band_union[t] = bu;
      }
    }
    if (birth)
      for (int64_t k = 0; k < n_new; ++k) birth[added[k]] = t + 1;
    cnt += n_new;
    int32_t* tmp = A; A = A_next; A_next = tmp;
    nA = nA_next;
    ++t;
  }

  res->n_candidates = n_cand;
  res->n_seeds = n_seeds;
  res->solid_count = cnt;
  res->target_count = s_star;
  res->front_size = nA;
  res->steps = t;
  res->status = cnt >= s_star ? ORC_DONE : (nA == 0 ? ORC_EXHAUSTED : ORC_MAXSTEPS);
  free(A); free(A_next); free(added); free(mask); free(prio); free(stamp);
  return res->status;
}

/* ------------------------------------------------------------------------ */
/* Multi-phase generation (Sec. 2.1 steps 1-5): the growing phases 1..K are  */
/* generated one after another on the cells no earlier phase holds, each     */
/* with its own core probability, growth probabilities, spacing, key and     */
/* target fraction P^n of the whole domain (S*_n = ceil(P^n N), Eq. (1) with */
/* the phase's own count).  Phases are independent: a phase grows only into */
/* unassigned cells.  Cells left unassigned form the matrix phase (label 0). */
/* While phase n grows, phase m < n is held as the value 3 + m, which the    */
/* single-phase rules treat as neither void nor solid.                       */
/* ------------------------------------------------------------------------ */
int32_t orc_generate_phases(int32_t nx, int32_t ny, int32_t nz, int32_t n_phases,
                            const orc_params* phases, uint8_t* labels, orc_result* results) {
  const int64_t n = (int64_t)nx * ny * nz;
  memset(labels, 0, (size_t)n);
  int32_t worst = ORC_DONE;
  for (int32_t k = 0; k < n_phases; ++k) {
    const int32_t st = generate_on(nx, ny, nz, &phases[k], labels, &results[k], NULL, NULL,
                                   NULL, NULL, NULL, NULL, NULL, NULL, 0);
    if (st > worst) worst = st;
    for (int64_t v = 0; v < n; ++v)
      if (labels[v] == 1) labels[v] = (uint8_t)(3 + (k + 1));
  }
  for (int64_t v = 0; v < n; ++v)
    if (labels[v] >= 4) labels[v] = (uint8_t)(labels[v] - 3);
  return worst;
}
/* ------------------------------------------------------------------------ */
/* Interacting phases (Sec. 2.1 step 4): the n-th growing phase also grows   */
/* into a neighbour held by an earlier phase m, with the phase-interaction   */
/* probability I_i^{n,m} of the direction's class.                           */
/* Readings: while phase n grows, the label grid holds 0 (unassigned), 1     */
/* (phase n) and 3 + m (earlier phase m).  A neighbour is a candidate target */
/* of a phase-n cell when it is unassigned, or when it belongs to a phase m  */
/* that phase n interacts with (I^{n,m} > 0 for some class).  The j-th       */
/* candidate neighbour of a source (ascending d) takes the draw of rank j    */
/* (the single-phase draw rule).  An unassigned target passes with the       */
/* Eq. (1) threshold of the step, a target of phase m with P32(I_c^{n,m}),   */
/* not scaled by Eq. (1) (the interaction probability is given as such).     */
/* A passing draw converts the target to phase n; it counts towards phase   */
/* n's fraction.  Candidates, labels and thresholds are those of the step's  */
/* start (Jacobi, as for one phase); the front is the set of phase-n cells   */
/* with a candidate neighbour.  With every I = 0 nothing but unassigned      */
/* cells is a candidate, and the phases are the independent ones.            */
/* ------------------------------------------------------------------------ */

/* Candidate targets of phase-n cell a: one bit per direction. */
static uint32_t candidate_mask(int32_t nx, int32_t ny, int32_t nz, const uint8_t* labels,
                               const uint8_t cand[256], int64_t a) {
  int32_t x, y, z;
  coords(nx, ny, a, &x, &y, &z);
  uint32_t m = 0;
  for (int32_t d = 0; d < 26; ++d) {
    int64_t q = neighbour(nx, ny, nz, x, y, z, d);
    if (q >= 0 && cand[labels[q]]) m |= 1u << d;
  }
  return m;
}

int64_t orc_step_interacting(int32_t nx, int32_t ny, int32_t nz, uint8_t* labels,
                             const uint8_t cand[256], const uint64_t thr[768],
                             const int32_t* A, int64_t nA, uint32_t t, uint64_t key,
                             int32_t* A_next, int64_t* n_next, int32_t* converted,
                             uint32_t* mask_scratch, uint64_t* attempts,
                             uint64_t* successes) {
  const int64_t n = (int64_t)nx * ny * nz;
  /* the step's start: every source's candidates, and every cell's label */
  for (int64_t i = 0; i < nA; ++i)
    mask_scratch[i] = candidate_mask(nx, ny, nz, labels, cand, A[i]);
  uint8_t* claimed = (uint8_t*)calloc((size_t)n, 1);
  int64_t added = 0;
  for (int32_t d = 0; d < 26; ++d) {
    int32_t dx, dy, dz, cls;
    orc_direction(d, &dx, &dy, &dz, &cls);
    for (int64_t i = 0; i < nA; ++i) {
      uint32_t m = mask_scratch[i];
      if (!((m >> d) & 1u)) continue;
      int32_t j = popcount32(m & ((1u << d) - 1u));
      int64_t q = (int64_t)A[i] + dx + (int64_t)nx * (dy + (int64_t)ny * dz);
      uint64_t T = thr[3 * labels[q] + cls]; /* labels are untouched during the step */
      if (attempts) attempts[d + 26 * (labels[q] != 0)] += 1;
      if ((uint64_t)orc_growth_draw(key, A[i], t, j) < T) {
        if (successes) successes[d + 26 * (labels[q] != 0)] += 1;
        if (!claimed[q]) {
          claimed[q] = 1;
          converted[added++] = (int32_t)q;
        }
      }
    }
  }
  for (int64_t k = 0; k < added; ++k) labels[converted[k]] = 1;
  free(claimed);
  /* the next front: cells of A and converted cells with a candidate neighbour left */
  int64_t kept = 0;
  for (int64_t i = 0; i < nA; ++i)
    if (candidate_mask(nx, ny, nz, labels, cand, A[i])) A_next[kept++] = A[i];
  for (int64_t k = 0; k < added; ++k)
    if (candidate_mask(nx, ny, nz, labels, cand, converted[k])) A_next[kept++] = converted[k];
  *n_next = kept;
  return added;
}

/* Phase-n generation on a label grid with the candidate table `cand` and the
 * interaction thresholds of the labels 3 + m in `thr` (entries 3..767); entries 0..2
 * (unassigned cells) take the Eq. (1) thresholds of each step.  Seeding as for an
 * independent phase: cores only on unassigned cells. */
static int32_t grow_phase_interacting(int32_t nx, int32_t ny, int32_t nz, const orc_params* p,
                                      uint8_t* labels, const uint8_t cand[256], uint64_t thr[768],
                                      orc_result* res) {
  const int64_t n = (int64_t)nx * ny * nz;
  const int64_t s_star = orc_target_count(p->solid_fraction, n);
  const uint64_t t_seed = orc_prob_threshold(p->seed_prob);
  uint64_t t_ref[3];
  for (int c = 0; c < 3; ++c) t_ref[c] = orc_prob_threshold(p->g_ref[c]);
  const int32_t max_steps = p->max_steps > 0 ? p->max_steps : ORC_DEFAULT_MAX_STEPS;

  int32_t* A = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* A_next = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* conv = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  uint32_t* mask = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
  uint64_t* prio = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);

  int64_t n_drawn = orc_seed_candidates(nx, ny, nz, p->key, t_seed, A, prio, n);
  int64_t n_cand = 0;
  for (int64_t i = 0; i < n_drawn; ++i)
    if (labels[A[i]] == 0) {
      A[n_cand] = A[i];
      prio[n_cand] = prio[i];
      ++n_cand;
    }
  int64_t n_seeds = orc_seed_select(nx, ny, nz, p->spacing, n_cand, A, prio, labels);

  int64_t cnt = n_seeds, nA = 0;
  for (int64_t v = 0; v < n; ++v)
    if (labels[v] == 1 && candidate_mask(nx, ny, nz, labels, cand, v)) A[nA++] = (int32_t)v;
  int32_t t = 0;
  while (cnt < s_star && nA > 0 && t < max_steps) {
    for (int c = 0; c < 3; ++c) thr[c] = orc_growth_threshold(t_ref[c], cnt, s_star);
    int64_t nA_next = 0;
    int64_t added = orc_step_interacting(nx, ny, nz, labels, cand, thr, A, nA, (uint32_t)t,
                                         p->key, A_next, &nA_next, conv, mask, NULL, NULL);
    if (p->front_rule == 1) { /* Algorithm 3 as printed: only the new cells */
      nA_next = 0;
      for (int64_t k = 0; k < added; ++k)
        if (candidate_mask(nx, ny, nz, labels, cand, conv[k])) A_next[nA_next++] = conv[k];
    }
    cnt += added;
    int32_t* tmp = A; A = A_next; A_next = tmp;
    nA = nA_next;
    ++t;
  }
  res->n_candidates = n_cand;
  res->n_seeds = n_seeds;
  res->solid_count = cnt;
  res->target_count = s_star;
  res->front_size = nA;
  res->steps = t;
  res->status = cnt >= s_star ? ORC_DONE : (nA == 0 ? ORC_EXHAUSTED : ORC_MAXSTEPS);
  free(A); free(A_next); free(conv); free(mask); free(prio);
  return res->status;
}

int32_t orc_generate_phases_interacting(int32_t nx, int32_t ny, int32_t nz, int32_t n_phases,
                                        const orc_params* phases, const double* interact,
                                        uint8_t* labels, orc_result* results) {
  const int64_t n = (int64_t)nx * ny * nz;
  memset(labels, 0, (size_t)n);
  int32_t worst = ORC_DONE;
  for (int32_t k = 0; k < n_phases; ++k) {
    /* phase k + 1 grows; earlier phase m + 1 is held as label 4 + m */
    uint8_t cand[256];
    uint64_t thr[768];
    memset(cand, 0, sizeof cand);
    memset(thr, 0, sizeof thr);
    cand[0] = 1;
    for (int32_t m = 0; m < k; ++m) {
      const double* I = interact + ((size_t)k * (size_t)n_phases + (size_t)m) * 3;
      if (I[0] > 0.0 || I[1] > 0.0 || I[2] > 0.0) {
        cand[4 + m] = 1;
        for (int c = 0; c < 3; ++c) thr[3 * (4 + m) + c] = orc_prob_threshold(I[c]);
      }
    }
    const int32_t st =
        grow_phase_interacting(nx, ny, nz, &phases[k], labels, cand, thr, &results[k]);
    if (st > worst) worst = st;
    for (int64_t v = 0; v < n; ++v)
      if (labels[v] == 1) labels[v] = (uint8_t)(3 + (k + 1));
  }
  for (int64_t v = 0; v < n; ++v)
    if (labels[v] >= 4) labels[v] = (uint8_t)(labels[v] - 3);
  return worst;
}
