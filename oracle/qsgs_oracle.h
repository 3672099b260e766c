/*
 * qsgs_oracle.h -- CPU oracle for LIETS-QSGS (Wang & Al Kobaisi, "Ultra-Fast 3D
 * Porous Media Generation: a GPU-Accelerated List-Indexed Explicit Time-Stepping
 * QSGS Algorithm", arXiv 2602.11734).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, single-threaded reference
 * that the GPU library is checked against.  Only the test-suite, the package's
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant with the GPU library, and the GPU library
 * never calls it.
 *
 * Conventions (the integer definitions both sides implement independently):
 *   grid      uint8 [nz][ny][nx], v = x + nx*(y + ny*z); 0 = pore, 1 = solid.
 *             The domain is not periodic: off-grid neighbours do not exist.
 *   direction d = 0..25 enumerates the 26-neighbourhood in the order of
 *             k = (dx+1) + 3(dy+1) + 9(dz+1), k != 13, d = k - (k > 13);
 *             class(d) = |dx|+|dy|+|dz|-1 (0 face, 1 edge, 2 corner).
 *   draws     Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) keyed by the
 *             64-bit realization key; counters are listed at each function.
 *
 * Parity status: every function here is pinned by the CPU tests (known-answer
 * vectors, closed forms, brute force, scipy dilation, statistics), except where
 * a function's comment says "parity unpinned".
 */
#ifndef QSGS_ORACLE_H
#define QSGS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Counter tags (word 3 of the Philox counter) separating the draw streams. */
#define ORC_TAG_SEED    1u
#define ORC_TAG_GROW_HI 2u
#define ORC_TAG_GROW_LO 3u

#define ORC_DONE      1
#define ORC_EXHAUSTED 2
#define ORC_MAXSTEPS  3
#define ORC_DEFAULT_MAX_STEPS (1 << 20)

typedef struct {
  double   solid_fraction; /* phi_s, target solid volume fraction (1 - porosity) */
  double   seed_prob;      /* S_d, seed (core) probability                        */
  double   g_ref[3];       /* G_ref for the face, edge, corner classes             */
  int32_t  spacing;        /* s: minimum pairwise L1 seed distance; s <= 1 = none  */
  int32_t  max_steps;      /* <= 0 selects ORC_DEFAULT_MAX_STEPS                    */
  uint64_t key;            /* Philox key: k0 = low 32 bits, k1 = high 32 bits      */
  int32_t  front_rule;     /* 0: A <- prune(A u A_new) (the interface); 1: the     */
                           /* literal Algorithm 3 rule A <- prune(A_new)           */
  int32_t  unused;
} orc_params;

typedef struct {
  int64_t n_candidates, n_seeds, solid_count, target_count, front_size;
  int32_t steps, status;
} orc_result;

/* Philox4x32-10 block function. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Directions: offsets and class of direction d (0..25). */
void orc_direction(int32_t d, int32_t* dx, int32_t* dy, int32_t* dz, int32_t* cls);

/* Probability -> 32-bit threshold: min(2^32, floor(p * 2^32)); event iff w < T. */
uint64_t orc_prob_threshold(double p);

/* Target solid count S* = ceil(phi_s * N), the loop runs while count < S*. */
int64_t orc_target_count(double phi_s, int64_t n);

/* Eq. (1) at solid count cnt < S*: floor(T_ref * (20 S* - 19 cnt) / S*), capped at 2^32. */
uint64_t orc_growth_threshold(uint64_t t_ref, int64_t cnt, int64_t s_star);

/* Growth draw for the j-th void direction of source a at step t (32-bit value). */
uint32_t orc_growth_draw(uint64_t key, int32_t a, uint32_t t, int32_t j);

/* Seed candidates {v : w0(v) < t_seed} in ascending v, with 64-bit priorities. */
int64_t orc_seed_candidates(int32_t nx, int32_t ny, int32_t nz, uint64_t key, uint64_t t_seed,
                            int32_t* cand, uint64_t* prio, int64_t cap);

/* Greedy seed acceptance in ascending (priority, v); writes 1 at seeds into a zeroed grid. */
int64_t orc_seed_select(int32_t nx, int32_t ny, int32_t nz, int32_t spacing, int64_t n_cand,
                        const int32_t* cand, const uint64_t* prio, uint8_t* grid);

/* Interface: solid voxels with at least one in-domain void 26-neighbour, ascending v. */
int64_t orc_interface(int32_t nx, int32_t ny, int32_t nz, const uint8_t* grid, int32_t* out);

/* One growth step in the list-indexed form (Algorithm 3).  Returns |A_next|. */
int64_t orc_step_liets(int32_t nx, int32_t ny, int32_t nz, uint8_t* grid, const int32_t* A,
                       int64_t nA, uint32_t t, const uint64_t T[3], uint64_t key,
                       int32_t* A_next, int64_t* n_new, uint32_t* mask_scratch,
                       int32_t* new_scratch, uint64_t* attempts, uint64_t* successes);

/* One growth step in the full-field form (Algorithm 2).  Returns the number grown. */
int64_t orc_step_fullfield(int32_t nx, int32_t ny, int32_t nz, uint8_t* grid, uint32_t t,
                           const uint64_t T[3], uint64_t key);

/* Whole generation (seeding, then the list-indexed loop).  Optional outputs may be NULL:
 * birth[v] = step at which v became solid (0 for seeds, -1 for pore), and per-step logs
 * of |F_t|, |New_t|, the solid count at the start of step t, the step's draws (one per
 * front cell and void neighbour), its high-half Philox blocks (one per eight ranks of a
 * front cell), and the sizes of the one-voxel bands (cells within Chebyshev distance 1)
 * around F_t and around F_t u New_t -- the occupancy the step reads -- log_cap entries
 * each. */
int32_t orc_generate(int32_t nx, int32_t ny, int32_t nz, const orc_params* p, uint8_t* grid,
                     orc_result* res, int32_t* birth, int64_t* log_front, int64_t* log_new,
                     int64_t* log_count, int64_t* log_draws, int64_t* log_blocks,
                     int64_t* log_band, int64_t* log_band_union, int32_t log_cap);

/* Multi-phase generation (Sec. 2.1 steps 1-5), independent phases in sequence:
 * labels[v] = n for a cell of growing phase n (1..n_phases), 0 for the matrix phase.
 * Phase n draws its cores only on cells no earlier phase holds and grows only into
 * such cells; results[n - 1] reports it as orc_generate would (solid_count = the
 * phase's cell count).  1 <= n_phases <= 252.  Returns the largest status. */
int32_t orc_generate_phases(int32_t nx, int32_t ny, int32_t nz, int32_t n_phases,
                            const orc_params* phases, uint8_t* labels, orc_result* results);

/* One growth step of phase n on a label grid with interacting phases (Sec. 2.1 step 4).
 * labels: 0 unassigned, 1 the growing phase n, 3 + m a cell of earlier phase m.
 * cand[l] != 0: a neighbour of label l is a candidate target (label 0 always; 3 + m when
 * phase n interacts with phase m).  thr[3 l + c]: the threshold of such a target for
 * direction class c (label 0: the step's Eq. (1) thresholds; 3 + m: P32(I_c^{n,m})).
 * The j-th candidate neighbour of a source in A (ascending d) takes the draw of rank j
 * (orc_growth_draw); a passing draw converts the target to label 1.  Candidates, labels
 * and thresholds are those of the step's start.  Returns the number of converted cells
 * (listed in `converted`, capacity N); A_next receives the cells of A and the converted
 * cells that still have a candidate neighbour (*n_next of them).  mask_scratch holds nA
 * entries.  attempts / successes (52 entries each, may be NULL): per direction d, index
 * d for unassigned targets and 26 + d for targets of other phases. */
int64_t orc_step_interacting(int32_t nx, int32_t ny, int32_t nz, uint8_t* labels,
                             const uint8_t cand[256], const uint64_t thr[768],
                             const int32_t* A, int64_t nA, uint32_t t, uint64_t key,
                             int32_t* A_next, int64_t* n_next, int32_t* converted,
                             uint32_t* mask_scratch, uint64_t* attempts, uint64_t* successes);

/* Multi-phase generation with interacting phases (Sec. 2.1 steps 1-5): as
 * orc_generate_phases, but phase n also grows into cells of an earlier phase m with the
 * phase-interaction probability interact[3 ((n - 1) n_phases + (m - 1)) + c] of the
 * direction's class c (face, edge, corner), not scaled by Eq. (1); entries with m >= n
 * are not read.  A phase n with I^{n,m} > 0 for some class treats phase m's cells as
 * candidate targets; a converted cell joins phase n and counts towards its fraction.
 * results[n - 1].solid_count is phase n's count when it stopped (later phases may convert
 * some of its cells).  With every I = 0 the result equals orc_generate_phases. */
int32_t orc_generate_phases_interacting(int32_t nx, int32_t ny, int32_t nz, int32_t n_phases,
                                        const orc_params* phases, const double* interact,
                                        uint8_t* labels, orc_result* results);

#ifdef __cplusplus
}
#endif
#endif
