/*
 * qsgs.h -- C ABI of libqsgs: LIETS-QSGS porous-media generation on MI355X (gfx950).
 *
 * The method is the list-indexed explicit time-stepping (LIETS) formulation of QSGS
 * (Wang & Al Kobaisi, arXiv 2602.11734): seeds are drawn with a seed probability
 * (Sec. 2.1 step 2) and spaced by a diamond (L1) exclusion zone (Sec. 2.3, Fig. 1D);
 * then, while the solid fraction is below its target and the active front is not
 * empty, every front voxel tries each of its 26 neighbours with the directional
 * growth probability of Eq. (1), and the front is rebuilt from the old front and
 * the newly solid voxels (Sec. 2.3 steps 2-5, Algorithm 3).
 *
 * Integer definitions (bit-exact, shared by contract with the CPU oracle):
 *   grid       uint8, voxel v = x + nx*(y + ny*z), 0 = pore, 1 = solid; not periodic.
 *   directions d = 0..25: k = (dx+1) + 3(dy+1) + 9(dz+1), k != 13, d = k - (k > 13);
 *              class = |dx|+|dy|+|dz|-1 (0 face, 1 edge, 2 corner).
 *   draws      Philox4x32-10 (Salmon et al., SC'11), key = the 64-bit params.key
 *              (word 0 = low 32 bits).  Seeding of v: counter (v, 0, 0, 1), v is a
 *              candidate iff word0 < floor(S_d 2^32), its priority is (word1<<32|word2, v).
 *              Growth at step t from solid a: the j-th in-domain void neighbour of a
 *              (ascending d) draws (H<<16)|L, H and L being the 16-bit half (j&1) of word
 *              (j>>1)&3 of the blocks at counters (a, t, j>>3, 2) and (a, t, j>>3, 3);
 *              the neighbour grows iff the draw < T_class.
 *   thresholds T_ref = min(2^32, floor(G_ref 2^32)); S* = ceil(phi_s N) in binary64;
 *              Eq. (1) at solid count c < S*: T = min(2^32, floor(T_ref (20 S* - 19 c) / S*)).
 *   spacing    candidates at L1 distance 1..s-1 conflict; seeds = greedy acceptance in
 *              ascending priority (lexicographically-first maximal independent set).
 *   front      F_t = solid voxels with an in-domain void 26-neighbour (a set; the order
 *              of a front list is unspecified).
 *   loop       while count < S* and F non-empty and step < max_steps.
 *
 * Conventions for every function:
 *   - Functions never throw; they return a qsgs_status.  Values >= 0 are normal
 *     outcomes, values < 0 are errors, and qsgs_last_error() describes the last error
 *     raised on the calling thread.
 *   - Device pointers are caller-owned device memory (hipMalloc or torch allocations);
 *     the library never allocates or frees device memory on these paths.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued on it;
 *     functions that return host-visible results (every qsgs_info output) synchronise it.
 *   - Calls that share a workspace, grid or front buffer must not overlap in time.
 */
#ifndef QSGS_H
#define QSGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QSGS_OK = 0,            /* a growth step ran; the loop may continue                    */
  QSGS_DONE = 1,          /* solid count >= S* (target solid fraction reached)           */
  QSGS_EXHAUSTED = 2,     /* the front is empty while the count is below the target      */
  QSGS_MAXSTEPS = 3,      /* params.max_steps growth steps were taken                    */
  QSGS_ERR_INVALID = -1,  /* bad argument; nothing was launched                          */
  QSGS_ERR_CAPACITY = -2, /* a front list would exceed front_cap; state left unchanged   */
  QSGS_ERR_WORKSPACE = -3,/* ws_bytes below the size the query functions return          */
  QSGS_ERR_DEVICE = -4    /* a HIP runtime error; the message names the call             */
} qsgs_status;

typedef struct {
  int32_t nx, ny, nz;     /* each >= 1 and nx*ny*nz < 2^31                                */
} qsgs_dims;

/* Growth forms of the whole-generation calls (qsgs_params.sweep_form).  All three give
 * the same grids; they differ in the work done per step. */
#define QSGS_SWEEP_LIST 0      /* list-indexed tile sweep (LIETS, Sec. 2.3, Algorithm 3): */
                               /* only tiles that may hold the front are visited          */
#define QSGS_SWEEP_FIELD 1     /* full-field steps (Sec. 2.2, Algorithm 2): every cell of */
                               /* the grid draws for all its directions every step, then  */
                               /* a whole-grid pass folds the claims into the solid phase */
#define QSGS_SWEEP_ALL_TILES 2 /* the tile sweep with every tile listed every step        */

typedef struct {
  double   solid_fraction;/* phi_s in (0, 1]: target solid volume fraction = 1 - porosity */
  double   seed_prob;     /* S_d in [0, 1]: seed (core) probability, Sec. 2.1 step 2       */
  double   g_ref[3];      /* G_ref of the face, edge and corner classes, each in [0, 1]    */
  int32_t  spacing;       /* s >= 0: minimum pairwise L1 seed distance; s <= 1 = none       */
  int32_t  max_steps;     /* growth step cap; <= 0 selects 2^20                             */
  uint64_t key;           /* Philox key of the realization                                  */
  int32_t  sweep_form;    /* whole-generation calls only: QSGS_SWEEP_LIST (0),              */
                          /* QSGS_SWEEP_FIELD (1) or QSGS_SWEEP_ALL_TILES (2).  Results are   */
                          /* identical; the full-field form is the baseline the list-indexed */
                          /* one is measured against.  Ignored by qsgs_seed / qsgs_grow_step. */
  int32_t  front_rule;    /* whole-generation calls only: 0 = the next front is the        */
                          /* interface, prune(F_t u New_t) (Sec. 2.3 steps 2 and 4: failed   */
                          /* sources stay); 1 = Algorithm 3 as printed, prune(New_t): only   */
                          /* this step's new voxels are the next sources.  qsgs_grow_step    */
                          /* and the full-field form reject 1 (QSGS_ERR_INVALID).            */
} qsgs_params;

typedef struct {
  int64_t n_candidates;   /* voxels whose seed draw passed                                 */
  int64_t n_seeds;        /* accepted seeds (after spacing)                                 */
  int64_t solid_count;    /* solid voxels now                                               */
  int64_t target_count;   /* S* = ceil(phi_s N)                                             */
  int64_t front_size;     /* |F_t| now                                                      */
  int64_t grown_last_step;/* |New| of the last step taken                                   */
  int32_t step;           /* growth steps taken so far (t)                                  */
  int32_t status;         /* a qsgs_status value >= 0 (QSGS_ERR_DEVICE for a failed       */
                          /* server request)                                                */
} qsgs_info;

/* Bytes a grid buffer needs: N + 8 rounded up to a multiple of 4.  The voxels occupy the
 * first N bytes; the padding lets the growth kernels claim voxels with 32-bit atomics and
 * read rows with 8-byte loads.  The library never changes the padding's value (the
 * claim atomics OR zero into it).  0 for invalid dims. */
size_t qsgs_grid_bytes(const qsgs_dims* dims);

/* Workspace bytes for qsgs_seed and qsgs_generate with these dims and parameters
 * (seed-candidate lists, spacing buckets, the two front lists used by qsgs_generate,
 * loop control and the per-step log).  0 for invalid arguments. */
size_t qsgs_workspace_bytes(const qsgs_dims* dims, const qsgs_params* params);

/* Workspace bytes for qsgs_grow_step (loop control only; independent of the size). */
size_t qsgs_step_workspace_bytes(void);

/* Seeding (Sec. 2.1 step 2; spacing Sec. 2.3 / Fig. 1D) and the initial active front
 * (Sec. 2.3 step 2).
 *   d_grid   device, qsgs_grid_bytes(dims) bytes, 4-byte aligned; overwritten: 1 at seeds,
 *            0 elsewhere.
 *   d_front  device int32[front_cap]; receives F_0 (linear voxel indices, any order).
 *   d_ws     device workspace of ws_bytes >= qsgs_workspace_bytes(dims, params).
 *   info     host; on return: n_candidates, n_seeds, solid_count = n_seeds, target_count,
 *            front_size = |F_0|, grown_last_step = 0, step = 0, status = the loop status
 *            of the initial state (QSGS_OK if growth should run).
 * Errors: QSGS_ERR_INVALID (bad dims/params/pointers), QSGS_ERR_WORKSPACE,
 * QSGS_ERR_CAPACITY (|F_0| > front_cap; d_front untouched beyond front_cap),
 * QSGS_ERR_DEVICE.  Synchronises `stream`. */
qsgs_status qsgs_seed(const qsgs_dims* dims, const qsgs_params* params, uint8_t* d_grid,
                      int32_t* d_front, int64_t front_cap, void* d_ws, size_t ws_bytes,
                      qsgs_info* info, void* stream);

/* One growth step t (Sec. 2.3 steps 3-4, Algorithm 3, Eq. (1)).
 *   d_grid      device grid holding G_t (values 0/1); becomes G_{t+1}.
 *   d_front_in  device int32[front_cap] holding F_t in its first info->front_size
 *               entries (as written by qsgs_seed or a previous qsgs_grow_step).  The
 *               step appends this step's new voxels after them (entries beyond
 *               front_size are scratch); entries [0, front_size) are preserved.
 *   d_front_out device int32[front_cap], must not overlap d_front_in; receives F_{t+1}.
 *   d_ws        device workspace, ws_bytes >= qsgs_step_workspace_bytes().
 *   info        host, in: step, solid_count, front_size (as returned by the previous call);
 *               out: updated fields, grown_last_step = |New_t|, status per the loop rule.  When the
 *               input status is already >= 1 (done, exhausted, max steps) nothing runs.
 * Errors: QSGS_ERR_INVALID, QSGS_ERR_WORKSPACE, QSGS_ERR_DEVICE, and QSGS_ERR_CAPACITY
 * when |F_t| + |New_t| > front_cap: the grid is restored to G_t, info is unchanged, and
 * the call can be retried with larger buffers (front_cap >= N never overflows).
 * Synchronises `stream`. */
qsgs_status qsgs_grow_step(const qsgs_dims* dims, const qsgs_params* params, uint8_t* d_grid,
                           int32_t* d_front_in, int32_t* d_front_out, int64_t front_cap,
                           void* d_ws, size_t ws_bytes, qsgs_info* info, void* stream);

/* Whole generation: qsgs_seed, then growth steps until the loop rule stops (Sec. 2.3 step 5).
 * The loop runs on the device; the host reads the loop status once per chunk of steps.
 *   d_grid  device, qsgs_grid_bytes(dims) bytes, 4-byte aligned; receives the final grid.
 *   d_ws    device workspace, ws_bytes >= qsgs_workspace_bytes(dims, params); on return it
 *           holds the per-step log read by qsgs_read_step_log.
 *   info    host; receives the final counts, steps and status (DONE/EXHAUSTED/MAXSTEPS).
 * Errors: QSGS_ERR_INVALID, QSGS_ERR_WORKSPACE, QSGS_ERR_DEVICE.  Synchronises `stream`. */
qsgs_status qsgs_generate(const qsgs_dims* dims, const qsgs_params* params, uint8_t* d_grid,
                          void* d_ws, size_t ws_bytes, qsgs_info* info, void* stream);

/* Allocation-free whole generation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same result as qsgs_generate; the workspace is a scratch array of 128 MiB that the
 * library holds in device memory, one per device it runs on, for the life of the process.
 * The call allocates nothing: no device memory, no pinned host memory, no events (its
 * small control transfers go through pageable host memory).
 *   d_grid  device, qsgs_grid_bytes(dims) bytes, 4-byte aligned; receives the final grid.
 *   info    host; receives the final counts, steps and status.
 * Every call on one device uses that device's scratch and leaves its contents behind
 * (each call re-initialises what it reads).  Calls on one device from several host
 * threads are serialised by the library; work of this entry point enqueued on one device
 * from several processes does not share a scratch.  The per-step log is not readable
 * (qsgs_read_step_log needs the caller's workspace).
 * Errors: QSGS_ERR_INVALID, QSGS_ERR_WORKSPACE when the generation needs more scratch
 * than 128 MiB (qsgs_workspace_bytes(dims, params) > 134217728: roughly N above 6 million
 * voxels with spacing; nothing is launched), QSGS_ERR_DEVICE.  Synchronises `stream`. */
qsgs_status qsgs_generate_noalloc(const qsgs_dims* dims, const qsgs_params* params,
                                  uint8_t* d_grid, qsgs_info* info, void* stream);

/* Batched generation (many independent realizations, e.g. for uncertainty
 * quantification, Sec. 1): `count` realizations of possibly different sizes and
 * parameters share one persistent launch per kernel per growth step, addressed
 * through a per-realization offset table.  Each result is bit-identical to
 * qsgs_generate of the same realization alone.
 *   dims, params  host arrays of `count` entries, 1 <= count <= 4096.
 *   d_grids       host array of `count` device grid pointers (qsgs_grid_bytes each,
 *                 4-byte aligned).
 *   d_ws          device workspace, ws_bytes >= qsgs_batch_workspace_bytes(count, dims, params).
 *   infos         host array of `count` results.
 * Returns the largest per-realization status (DONE, EXHAUSTED or MAXSTEPS) or an error:
 * QSGS_ERR_INVALID (any bad entry; nothing launched), QSGS_ERR_WORKSPACE,
 * QSGS_ERR_DEVICE.  Synchronises `stream`. */
size_t qsgs_batch_workspace_bytes(int32_t count, const qsgs_dims* dims,
                                  const qsgs_params* params);
qsgs_status qsgs_generate_batch(int32_t count, const qsgs_dims* dims, const qsgs_params* params,
                                uint8_t* const* d_grids, void* d_ws, size_t ws_bytes,
                                qsgs_info* infos, void* stream);

/* Whole generations that never synchronise with the host, for capture into a HIP graph
 * (Sec. 2.3, the same loop as qsgs_generate / qsgs_generate_batch and bit-identical
 * results): every transfer, launch and decision is enqueued on `stream` and the results
 * land in device memory, so the whole call can be recorded once and replayed.
 *   d_grid(s), d_ws, ws_bytes  as for qsgs_generate / qsgs_generate_batch (same sizes).
 *   d_info(s)   device, 8-byte aligned, one qsgs_info per realization; written by the
 *               last kernel of the call.  status is DONE, EXHAUSTED or MAXSTEPS, or
 *               QSGS_ERR_DEVICE (an internal list overflow, or a seed spacing that had
 *               not settled after 64 priority rounds, which qsgs_generate never limits).
 *   params[r].max_steps  must be in [1, 4096]: without host reads the call runs exactly
 *               max(max_steps) + 1 sweep passes (passes after a realization has stopped
 *               find nothing to do and cost two short launches each).
 * The per-step log is readable afterwards with qsgs_read_step_log as usual.  Graph-
 * captured pass chunks (qsgs_tuning.graphs) and kernel timing are not used.  Returns
 * QSGS_OK once everything is enqueued, or QSGS_ERR_INVALID / QSGS_ERR_WORKSPACE (nothing
 * launched) / QSGS_ERR_DEVICE (a launch failed).  Does not synchronise `stream`. */
qsgs_status qsgs_generate_async(const qsgs_dims* dims, const qsgs_params* params,
                                uint8_t* d_grid, void* d_ws, size_t ws_bytes, qsgs_info* d_info,
                                void* stream);
qsgs_status qsgs_generate_batch_async(int32_t count, const qsgs_dims* dims,
                                      const qsgs_params* params, uint8_t* const* d_grids,
                                      void* d_ws, size_t ws_bytes, qsgs_info* d_infos,
                                      void* stream);

/* Multi-phase generation (Sec. 2.1 steps 1-5): growing phases 1..n_phases are generated
 * one after another on one label grid, each with its own parameters (core probability
 * seed_prob, target fraction P^n = solid_fraction of the whole domain, growth
 * probabilities, spacing, key, max_steps, full_field).  Phases are independent: phase n
 * draws its cores only on cells no earlier phase holds and grows only into such cells
 * (cells of other phases are neither sources nor targets); Eq. (1) uses the phase's own
 * count and S*_n = ceil(P^n N).  Cells left unassigned form the matrix phase.  With one
 * phase the result equals qsgs_generate.
 *   n_phases  1..252.
 *   phases    host array of n_phases parameter sets, phase n = index + 1.
 *   d_labels  device, qsgs_grid_bytes(dims) bytes, 4-byte aligned; overwritten with
 *             labels: n for a cell of phase n, 0 for the matrix (padding 0).
 *   d_ws      device workspace, ws_bytes >= qsgs_phases_workspace_bytes(...).
 *   infos     host array of n_phases results, as qsgs_generate reports them per phase
 *             (solid_count = the phase's cell count when it stopped).
 * Returns the largest per-phase status or an error (QSGS_ERR_INVALID: nothing launched;
 * QSGS_ERR_WORKSPACE; QSGS_ERR_DEVICE).  On an error the labels are unspecified.  The
 * per-step log of the workspace holds the last phase's steps.  Synchronises `stream`. */
size_t qsgs_phases_workspace_bytes(const qsgs_dims* dims, int32_t n_phases,
                                   const qsgs_params* phases);
qsgs_status qsgs_generate_phases(const qsgs_dims* dims, int32_t n_phases,
                                 const qsgs_params* phases, uint8_t* d_labels, void* d_ws,
                                 size_t ws_bytes, qsgs_info* infos, void* stream);

/* Multi-phase generation with interacting phases (Sec. 2.1 step 4): as qsgs_generate_phases,
 * but growing phase n also converts a neighbour that belongs to an earlier phase m, with the
 * phase-interaction probability of the direction's class.
 *   interact  host, 3 * n_phases * n_phases doubles: interact[3 ((n-1) n_phases + (m-1)) + c]
 *             = I_c^{n,m} in [0, 1] for class c (0 face, 1 edge, 2 corner), read for m < n;
 *             NULL = every I is 0 (qsgs_generate_phases).
 * Rules (the library's reading of the step): while phase n grows, a neighbour is a
 * candidate target when it is unassigned, or when it belongs to a phase m with
 * I_c^{n,m} > 0 for some class c.  The j-th candidate neighbour of a phase-n cell
 * (ascending direction) takes the draw of rank j (the draw rule above); an unassigned
 * target passes below the Eq. (1) threshold of the step, a phase-m target below
 * floor(I_c^{n,m} 2^32) (not scaled by Eq. (1)).  A converted cell belongs to phase n and
 * counts towards its target fraction; the front is the set of phase-n cells with a
 * candidate neighbour.  infos[m - 1].solid_count is phase m's count when it stopped (a
 * later phase may convert some of its cells).  With every I = 0 the result equals
 * qsgs_generate_phases.  A phase that interacts with an earlier one may not use
 * QSGS_SWEEP_FIELD (QSGS_ERR_INVALID).  Workspace: qsgs_phases_workspace_bytes.  Other
 * arguments and errors as qsgs_generate_phases.  Synchronises `stream`. */
qsgs_status qsgs_generate_phases_interacting(const qsgs_dims* dims, int32_t n_phases,
                                             const qsgs_params* phases, const double* interact,
                                             uint8_t* d_labels, void* d_ws, size_t ws_bytes,
                                             qsgs_info* infos, void* stream);

/* Copies the per-step log of realization `index` of the last qsgs_generate or
 * qsgs_generate_batch that used this workspace into host arrays (any may be NULL):
 * front[t] = |F_t|, grown[t] = |New_t|, count[t] = solid count at the start of step t,
 * for t < min(steps, max_entries, log capacity) where the capacity is 65536 steps for a
 * single generation and 4096 per realization in a batch.  Returns the number of
 * entries written (>= 0) or a negative qsgs_status.  Synchronises `stream`. */
int64_t qsgs_read_step_log(const void* d_ws, size_t ws_bytes, int32_t index, int64_t* front,
                           int64_t* grown, int64_t* count, int64_t max_entries, void* stream);

/* The work of each logged step (same entries and return value as qsgs_read_step_log; any
 * array may be NULL): draws[t] = number of draws of step t, one per front voxel and
 * in-domain void neighbour (Sec. 2.3 step 3), blocks[t] = Philox blocks of the high
 * halves, one per eight draws of a front voxel (the draw rule above).  These are the
 * integer work of the growth sweep.  Synchronises `stream`. */
int64_t qsgs_read_step_work(const void* d_ws, size_t ws_bytes, int32_t index, int64_t* draws,
                            int64_t* blocks, int64_t max_entries, void* stream);

/* Continuous-batching server.  Generation requests of different sizes are queued on
 * the host; each tick admits queued requests in arrival order while a slot is free and
 * their footprint -- grid (qsgs_grid_bytes) plus the sweep state (two tile lists and
 * the tile stamps, about N / 100 bytes) -- fits the free part of the caller's device
 * arena (the HBM budget), seeds them (with transient seeding scratch from the same
 * arena), then advances every resident realization in shared launches by at least
 * `steps_per_tick` growth steps, and by up to 16 while every resident request is
 * expected (from its remaining count over its last growth) to need that many before it
 * stops, so that few host round trips fall on a lightly loaded server.  A finished
 * request's grid stays in the arena until qsgs_server_take copies it out.  Each
 * result is bit-identical to qsgs_generate of the same request alone.  A server is
 * used from one thread; its stream orders all of its work.
 *   qsgs_server_reserved_bytes  arena bytes the server keeps for its control area.
 *   qsgs_server_create   d_arena: device, 256-byte aligned, arena_bytes long, owned by
 *                        the caller until qsgs_server_destroy; max_slots in [1, 4096];
 *                        steps_per_tick in [1, 1024].
 *   qsgs_server_submit   queues one request; QSGS_ERR_INVALID for bad dims/params or an
 *                        id in use, QSGS_ERR_CAPACITY if it cannot fit the arena even
 *                        when alone.
 *   qsgs_server_tick     one scheduling tick; reports resident, queued and finished
 *                        (not yet taken) requests.  Synchronises the stream.  If a
 *                        request fails (an internal list overflow), it is retired with
 *                        info.status = QSGS_ERR_DEVICE and its arena space released, the
 *                        tick still retires the others, and then returns QSGS_ERR_DEVICE.
 *   qsgs_server_ready    ids and infos of finished requests, oldest first (at most max).
 *   qsgs_server_take     copies the N-byte grid of a finished request to dst (host
 *                        memory if dst_on_host, else device; dst may be NULL to drop it)
 *                        and releases its arena space; for a failed request it copies
 *                        nothing, forgets the request and returns QSGS_ERR_DEVICE.
 *   qsgs_server_free_bytes  arena bytes not held by requests. */
typedef struct qsgs_server qsgs_server;
size_t qsgs_server_reserved_bytes(int32_t max_slots);
qsgs_status qsgs_server_create(void* d_arena, size_t arena_bytes, int32_t max_slots,
                               int32_t steps_per_tick, void* stream, qsgs_server** out);
qsgs_status qsgs_server_submit(qsgs_server* server, int64_t request_id, const qsgs_dims* dims,
                               const qsgs_params* params);
qsgs_status qsgs_server_tick(qsgs_server* server, int32_t* n_resident, int32_t* n_queued,
                             int32_t* n_ready);
int32_t qsgs_server_ready(qsgs_server* server, int64_t* ids, qsgs_info* infos, int32_t max);
qsgs_status qsgs_server_take(qsgs_server* server, int64_t request_id, void* dst,
                             size_t dst_bytes, int32_t dst_on_host);
size_t qsgs_server_free_bytes(const qsgs_server* server);
void qsgs_server_destroy(qsgs_server* server);

/* Launch shape of the item kernels (seed, growth and prune passes): threads per
 * workgroup (`*_block`, a multiple of 64 in [64, 512]) and workgroups (`*_grid`, a
 * multiple of 8 so that each of the 8 XCDs gets an equal share), plus the growth steps
 * issued between two host reads of the loop state (`steps_per_sync`, 0 = adaptive).
 * The shape never changes a result: every output is a function of the inputs only.
 * grow_grid = 0 sizes the growth sweep to one round of the workgroups the device holds
 * at once (1536 of 256 threads on an MI355X: 256 compute units x 6; 768 of 512 threads);
 * the step API's growth kernel then takes 2048.  `graphs` = 1 issues the passes of the
 * whole-generation
 * calls and of server ticks as HIP graph launches of captured chunks of 16, 8, 4, 2 or 1
 * passes (kernel nodes only; the executable graphs are cached per launch configuration
 * and workspace for the life of the process, at most 64 of them, and reused by later
 * calls with the same configuration); 0 launches every kernel on its own.  Graphs are
 * never used while kernel timing is enabled or by qsgs_generate_noalloc.
 * qsgs_set_tuning applies process-wide to calls that start afterwards (NULL restores the
 * defaults: 256 threads, and 512 for the growth sweep of a whole-generation call on one
 * realization; growth grid 0, 2048 for prune and seeding; adaptive; graphs on); a tuning
 * set here applies as given to every call.  QSGS_ERR_INVALID for a bad shape. */
typedef struct {
  int32_t grow_block, grow_grid;
  int32_t prune_block, prune_grid;
  int32_t seed_block, seed_grid;
  int32_t steps_per_sync;
  int32_t graphs;
} qsgs_tuning;

qsgs_status qsgs_set_tuning(const qsgs_tuning* tuning);
void qsgs_get_tuning(qsgs_tuning* tuning);

/* The occupancy one growth step reads, for the algorithmic byte count of a step.  A
 * step tests the 26 neighbours of every voxel of F_t (Sec. 2.3 step 3), then keeps the
 * voxels of F_t u New_t that still have a void neighbour (Sec. 2.3 step 4): it reads the
 * one-voxel band (in-domain cells within Chebyshev distance 1) around F_t and around
 * F_t u New_t.  From the grid before a step (d_before) and after it (d_after), both N
 * bytes in the layout of qsgs_grid_bytes (0 = void, any other value solid), computes
 *   out[0] = |band(F_t)|, F_t = solid cells of d_before with an in-domain void neighbour;
 *   out[1] = |band(F_t u New_t)|, New_t = cells void in d_before and solid in d_after.
 *   d_scratch  device, 8-byte aligned, >= qsgs_band_scratch_bytes(dims); overwritten.
 *   out        host uint64_t[2].
 * A measurement utility (two passes over the grid), not part of the growth path.
 * Errors: QSGS_ERR_INVALID, QSGS_ERR_WORKSPACE, QSGS_ERR_DEVICE.  Synchronises `stream`. */
size_t qsgs_band_scratch_bytes(const qsgs_dims* dims);
qsgs_status qsgs_band_sizes(const qsgs_dims* dims, const uint8_t* d_before,
                            const uint8_t* d_after, void* d_scratch, size_t scratch_bytes,
                            uint64_t* out, void* stream);

/* Measured issue rate of plain 32-bit vector ALU instructions on the current device, for
 * the ALU roof of the growth sweep (a measurement utility): eight independent chains of
 * xor / add per lane, waves_per_simd (1..8) wavefronts per SIMD on every compute unit,
 * best of two timed runs after a warm-up.  *lane_ops_per_s receives the 32-bit lane
 * operations per second.  d_scratch: device, >= qsgs_alu_scratch_bytes(waves_per_simd)
 * bytes (0 for a bad argument).  Synchronises `stream`. */
size_t qsgs_alu_scratch_bytes(int32_t waves_per_simd);
qsgs_status qsgs_alu_rate(int32_t waves_per_simd, void* d_scratch, size_t scratch_bytes,
                          double* lane_ops_per_s, void* stream);

/* Kernel timing for measurement.  While enabled (enable != 0), qsgs_generate records HIP
 * events around each growth-sweep and prune launch on its stream and accumulates their
 * durations; qsgs_profile_read returns (and with reset != 0 clears) the totals:
 * out[0] = grow launches, out[1] = grow milliseconds, out[2] = prune launches,
 * out[3] = prune milliseconds, out[4] = seeding milliseconds (draw to first front). */
void qsgs_profile_enable(int32_t enable);
void qsgs_profile_read(double out[5], int32_t reset);

/* Description of the last error on the calling thread ("" if none).  The pointer stays
 * valid until the next library call on this thread. */
const char* qsgs_last_error(void);

/* Library version string, e.g. "qsgs 0.3.0 gfx950". */
const char* qsgs_version(void);

/* Seed probability for a granular medium of grain diameter d and voxel size delta (same
 * unit): S_d = 6 phi_s delta^3 / (pi d^3), the expected number of grains per voxel times
 * one (Sec. 3.3, the rule used for the Fontainebleau samples).  Returns -1 for
 * arguments outside phi_s in [0, 1], d > 0, delta > 0, and min(result, 1) otherwise. */
double qsgs_seed_prob_from_grain(double solid_fraction, double grain_diameter,
                                 double voxel_size);

#ifdef __cplusplus
}
#endif
#endif /* QSGS_H */
