/* lf.h -- C ABI of the MI355X (gfx950) layered-field library.
 *
 * Implements the method of Zayer, Mlakar, Steinberger, Seidel, "Layered
 * Fields for Natural Tessellations on Surfaces": a sparse field matrix with
 * one layer per cell (plus a base layer) is evolved on a triangle mesh by
 * explicit Euler steps (Algorithm 1, equations (11)-(13)); cells are read
 * off as labels, re-seeded Lloyd-style (Section 5) and turned into a dual
 * triangle mesh (Sections 5.1-5.2).
 *
 * Conventions
 *  - Every function returns lf_status; nothing throws or longjmps across the
 *    ABI.  On failure lf_last_error() returns a message (thread-local, owned
 *    by the library, valid until the next call on the same thread).
 *  - Field matrix U = Phi^T: CSR, one row per vertex, one column per layer;
 *    columns 0..n_s-1 are the cells in seed order, column n_s is the base
 *    layer.  Row pointers and column ids are int32, values float32, columns
 *    ascending within a row, stored values > 0.
 *  - "Host or device" buffers: arguments documented with `is_device_ptr`
 *    take caller-owned memory; device pointers must stay valid until the
 *    call returns (all calls synchronise with the context stream before
 *    returning).
 *  - Handles are created and destroyed explicitly by their owner.  A context
 *    serves one host thread at a time; calls on one context serialise on its
 *    stream.
 *  - All device state lives in the GPU's HBM and is allocated by the library.
 */
#ifndef LF_H
#define LF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LF_OK = 0,
  LF_EINVAL = 1,    /* invalid argument (ids out of range, duplicate seeds, ...) */
  LF_ENOMEM = 2,    /* device or host allocation failed; state unchanged */
  LF_EDEVICE = 3,   /* HIP runtime error */
  LF_ECAPACITY = 4, /* storage could not be grown / a row exceeded the row limit */
  LF_EBUSY = 5,
  LF_ENOSYS = 6
} lf_status;

typedef enum { LF_OP_GRAPH = 0, LF_OP_COTAN = 1 } lf_operator;

/* Constants of the update (Section 3.1; values of Section 7 where given).
 * w: penalty between cells (0.2); a: gradient coefficient (0.04, a ratio of
 * 5 to w); e: band interaction (1.0); mu: mobility (0.1); dt: Euler step
 * (5.0); theta: entries below theta after normalisation are dropped (1e-3;
 * 0 keeps every positive entry); tau: dual-mesh threshold (0.25).
 * base_mode 0: the base layer couples to cells through the gradient term
 * and an antisymmetric band term only; 1: the base is an ordinary layer.
 * capacity_hint: initial size, in entries, of the overflow area that holds
 * the rows with more than three entries (the library keeps the fields as
 * fixed-width rows of three entries; 0 = max(4096, n_v / 16)); it grows on
 * demand. */
typedef struct {
  double w, a, e, mu, dt, theta, tau;
  int32_t base_mode;
  int32_t pad_;
  int64_t capacity_hint;
} lf_params;

typedef struct lf_ctx lf_ctx;
typedef struct lf_mesh lf_mesh;
typedef struct lf_fields lf_fields;

const char* lf_last_error(void);
void lf_params_default(lf_params* p);

/* Context on one GPU.  hip_stream: a hipStream_t to run on (for example
 * torch.cuda.current_stream().cuda_stream), or NULL for a library-owned
 * stream. */
lf_status lf_ctx_create(int32_t device, void* hip_stream, lf_ctx** out);
lf_status lf_ctx_destroy(lf_ctx* ctx);

/* Mesh and its operator (Section 3.2, "Laplacian computation"): the
 * Laplacian is computed once on the GPU.  V: float64[n_v*3] host positions;
 * F: int32[n_f*3] host triangles (copied in).  LF_EINVAL on ids out of
 * range or a face repeating a vertex; LF_EINVAL for a zero-area face with
 * the cotangent operator.  Graph: L_ij = 1 per edge; cotangent: L_ij =
 * (cot alpha + cot beta)/2; both with L_ii = -sum_j L_ij. */
lf_status lf_mesh_create(lf_ctx* ctx, const double* V, int32_t n_v, const int32_t* F,
                         int32_t n_f, int32_t op, lf_mesh** out);
lf_status lf_mesh_destroy(lf_mesh* mesh);
/* Operator export (diagonal included, columns ascending), size query with
 * NULL buffers: *nnz is always written.  rowptr int32[n_v+1], col int32[nnz],
 * val float32[nnz]. */
lf_status lf_mesh_operator(lf_mesh* mesh, int64_t* nnz, int32_t* rowptr, int32_t* col,
                           float* val, int32_t is_device_ptr);

/* Fields (Algorithm 1, first line; Initialization paragraph): seeds
 * int32[n_s] host array of distinct vertex ids; a seed holds 1 in its own
 * layer, every other vertex 1 in the base layer.  params may be NULL for the
 * defaults. */
lf_status lf_fields_create(lf_mesh* mesh, const int32_t* seeds, int32_t n_s,
                           const lf_params* params, lf_fields** out);
lf_status lf_fields_destroy(lf_fields* f);
/* Fields from seeds grown into regions (Algorithm 1, first line; the
 * Initialization paragraph of Section 3.2 suggests a vertex and its immediate
 * neighbours): every vertex within `rings` edges of a seed starts with 1 in
 * the layer of its nearest seed, ties to the lowest seed index, a seed always
 * in its own layer; every other vertex with 1 in the base layer.  rings = 0
 * is lf_fields_create; rings = 1 gives the 1-ring seeds.  Edges are those of
 * the mesh's triangles.  Regions grow on the GPU, one launch per ring.
 * lf_fields_reset (and so Lloyd rounds) grows the new seeds by the same
 * rings.  LF_EINVAL for rings outside [0, 1024] or invalid seeds. */
lf_status lf_fields_create_rings(lf_mesh* mesh, const int32_t* seeds, int32_t n_s, int32_t rings,
                                 const lf_params* params, lf_fields** out);
/* Fields from initial regions (Algorithm 1, first line: "seeds and/or
 * initial regions"): cell k starts as the vertices
 * region_vertices[region_ptr[k] .. region_ptr[k+1]), each with 1 in layer k;
 * every other vertex starts with 1 in the base layer.  Host arrays:
 * region_ptr int32[n_s+1] from 0, region_vertices int32[region_ptr[n_s]].
 * Regions must be non-empty and disjoint (LF_EINVAL otherwise).  A 1-ring
 * seed is the region {s} + its neighbours.  The seed of cell k (kept by a
 * Lloyd round whose line misses, and the dual vertex's position) is the
 * region's first vertex. */
lf_status lf_fields_create_regions(lf_mesh* mesh, const int32_t* region_ptr,
                                   const int32_t* region_vertices, int32_t n_s,
                                   const lf_params* params, lf_fields** out);
/* Re-initialise from new regions (same count). */
lf_status lf_fields_reset_regions(lf_fields* f, const int32_t* region_ptr,
                                  const int32_t* region_vertices);
/* Re-initialise from new seeds (same count), as after a Lloyd re-seeding;
 * fields made by lf_fields_create_rings grow the seeds by their rings, fields
 * made from regions start from the single seed vertices. */
lf_status lf_fields_reset(lf_fields* f, const int32_t* seeds);
/* Current seeds, int32[n_s] host. */
lf_status lf_fields_seeds(lf_fields* f, int32_t* seeds);

/* Per-pair coefficients (equation (2) carries a, w, e per pair of layers;
 * Section 3.1 fixes one value each and foresees varying them, e.g. to model
 * natural processes).  Layer l (cells 0..n_s-1, then the base) has type
 * layer_types[l] in [0, n_types), host int32[n_s+1]; a pair of layers
 * (j, l), j != l, takes a, w, e from host
 * table[3 * (t_j * n_types + t_l) + 0, 1, 2] (double, finite, rounded to
 * float32).  In base_mode 0 a pair with the base keeps the base reading:
 * no w, and the base's e against a cell is the negated entry.  One type
 * whose entry is (a, w, e) of the params is the scalar model.  n_types = 0
 * (NULL arrays) returns to the scalars of the params.  The update then
 * costs O(n^2) table reads per row of n active layers.  Applies from the
 * next step; the fields are not touched.  LF_EINVAL for types out of range,
 * entries that are not finite in float32 or n_types above 65536; LF_ENOMEM
 * when the table does not fit.  For a batch, the layers are those of lf_batch_fields. */
lf_status lf_fields_set_coefficients(lf_fields* f, int32_t n_types, const int32_t* layer_types,
                                     const double* table);

/* n_steps explicit Euler steps of Algorithm 1 (Jacobi form): field
 * Laplacian L_t = Phi L^T (row form: L U), rows of interest, update with
 * clamping to [0,1], column normalisation, then the theta prune.  Runs on the
 * context stream and waits for it; a step whose rows overflow the overflow
 * area is detected on the GPU, the area grows by 20% or more and the step is
 * replayed, so results never depend on capacities.  LF_ECAPACITY if a
 * vertex touches more layers than the row limit (64) or storage cannot
 * grow; the steps before the failing one stay done, and the fields hold
 * their state from before it. */
lf_status lf_step(lf_fields* f, int32_t n_steps);
/* lf_step without waiting: enqueues the first min(n_steps, 256) steps on
 * the context stream and returns at once (the GPU works while the caller
 * does).  The next call on these fields -- lf_sync, an export, labels, a
 * step, any other lf_fields / lf_lloyd / lf_dual / lf_batch call on them --
 * first waits for those steps, books them (growing storage and stepping
 * again what an overflow stopped) and runs the remaining steps; it returns
 * their errors.  lf_fields_destroy waits only for the enqueued steps. */
lf_status lf_step_async(lf_fields* f, int32_t n_steps);
/* Convergence (the paper's fields "until converged", Sections 4 and 7,
 * made concrete).  A step changes a row when the row's label (argmax over
 * the cells) or its set of layers at or above params.tau changes.  The
 * fields have converged at the end of the first whole chunk of check_every
 * (<= 256) steps in which no step changed any row and no value moved by
 * more than eps.  (With the theta prune the values can end in a period-2
 * oscillation of size about theta, and the first steps from seeds are
 * quiet for a few steps, so eps should exceed theta and check_every that
 * start-up; 1e-2 and 32 are safe.)  Runs up to max_steps steps; *steps_done
 * counts the steps run, *converged_at is the step (1-based, within this
 * call) that ended the quiet chunk, or 0. */
lf_status lf_step_until(lf_fields* f, int32_t max_steps, double eps, int32_t check_every,
                        int64_t* steps_done, int64_t* converged_at);
/* Change made by the last completed step: rows it changed (label or layers
 * at or above tau) and max |U_{t+1} - U_t| over all (vertex, layer) pairs
 * (0 before any step).  The step kernel measures these on every step of
 * lf_step_until and on the last step of every chunk of lf_step (at most 256
 * steps; so always for the last step of a call). */
lf_status lf_last_change(lf_fields* f, int64_t* changed_rows, double* max_delta);
/* Completes what lf_step_async left (see there), then waits for the
 * context stream. */
lf_status lf_sync(lf_fields* f);
/* Work-class ordering of the step's rows: every `every` steps (first 128
 * steps after an initialisation), lf_step re-orders the rows within tiles of
 * tile_rows consecutive rows by work class -- rows inside a cell (one layer,
 * and every neighbour the same single layer) first, then rows whose
 * neighbourhood holds 2, 3, or more layers (`classes` = 2 keeps only the
 * first split) -- so that wavefronts hold rows of one class; wavefronts of
 * rows inside a cell are written without the merge and update.  The order is
 * invisible at the boundary and the results do not depend on it.  Off by
 * default: on the meshes measured it costs more (the rows of a wavefront no
 * longer gather neighbours from a few cache lines) than the short path saves.
 * every = 0 keeps the current order.  tile_rows: a multiple of 256 in
 * [256, 4096]; classes in [2, 4].  lf_fields_reorders returns how many
 * re-orderings have happened. */
lf_status lf_fields_set_reorder(lf_fields* f, int32_t every, int32_t tile_rows, int32_t classes);
lf_status lf_fields_reorders(lf_fields* f, int64_t* n);
/* on = 1: lf_step (and lf_step_until) runs whole chunks of 256 steps from a
 * HIP graph captured on first use (the chunk's kernels only; the counters'
 * copies to the host stay outside), one graph per starting buffer, captured
 * again when storage grows or the coefficients change; chunks of other
 * lengths, and launches timed by lf_step_timing, are launched one by one.
 * Needs a stream other than the legacy default stream.  on = 0 (the
 * default): every launch one by one.  Results are identical either way. */
lf_status lf_fields_use_graphs(lf_fields* f, int32_t on);

/* Export U.  Size query with NULL buffers (*nnz always written).  rowptr
 * int32[n_v+1], col int32[nnz], val float32[nnz]; host or device. */
lf_status lf_fields_export(lf_fields* f, int64_t* nnz, int32_t* rowptr, int32_t* col,
                           float* val, int32_t is_device_ptr);
/* Import U (teacher forcing, resume).  Must be canonical: rowptr monotone
 * from 0, columns ascending in [0, n_s], values in (0, 1].  LF_EINVAL
 * otherwise (checked on the GPU). */
lf_status lf_fields_import(lf_fields* f, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                           const float* val, int32_t is_device_ptr);

/* Sharp labels (Figure 10, Section 7): per vertex, the cell layer with the
 * largest value (lowest id on ties), -1 when the vertex holds no cell.
 * labels int32[n_v], host or device. */
lf_status lf_labels(lf_fields* f, int32_t* labels, int32_t is_device_ptr);

/* One Lloyd-like re-seeding (Section 5) from the current fields: per cell,
 * area-weighted centroid of the barycentres of the faces having a vertex in
 * the cell's support and the area-weighted mean normal; the line through
 * the centroid along it is intersected with those faces; the closest hit
 * wins (lower face id on ties) and the new seed is that face's vertex
 * nearest the hit (lower id on ties); a miss keeps the seed.  Colliding
 * seeds: the lowest cell id keeps the vertex, the others (and movers onto a
 * staying seed) keep their old seed.  Geometry in float64.  Writes
 * seeds_out int32[n_s] and status int32[n_s] (0 hit, 1 miss, 2 collision;
 * may be NULL), host.  Does not re-initialise the fields. */
lf_status lf_lloyd_reseed(lf_fields* f, int32_t* seeds_out, int32_t* status);
/* Lloyd-like iterations (Section 5, Figure 11): `rounds` times, re-seed
 * (lf_lloyd_reseed), re-initialise the fields from the new seeds
 * (lf_fields_reset) and run steps_per_round steps (lf_step).  Writes the
 * final seeds to host seeds_out int32[n_s] (may be NULL); with rounds = 0 it
 * only copies the current seeds.  Errors as the calls it makes; the fields
 * are those of the last completed call. */
lf_status lf_lloyd(lf_fields* f, int32_t rounds, int32_t steps_per_round, int32_t* seeds_out);

/* Dual mesh (Sections 5.1-5.2) from the current fields with threshold tau:
 * A_v = Phibar Phibar^T, A_t = (Phibar Mbar)(Phibar Mbar)^T, candidates
 * A_t and not A_v confirmed by isoline crossings on their common faces,
 * confirmed candidates whose cells share two or more A_v neighbours are
 * dropped, triangles are the 3-cliques of the curated adjacency, spurious
 * triangles over a cell of three mutually adjacent neighbours are removed,
 * orientation is propagated across edges from each component's lowest
 * triangle.  Size query with NULL buffers: n_tri and adj_nnz are always
 * written.  tris int32[3*n_tri]; adj_rowptr int32[n_s+1], adj_col
 * int32[adj_nnz]; host. */
lf_status lf_dual_mesh(lf_fields* f, double tau, int64_t* n_tri, int32_t* tris, int64_t* adj_nnz,
                       int32_t* adj_rowptr, int32_t* adj_col);
/* Intermediate matrices of the last lf_dual_mesh call, for inspection:
 * which 0 = A_v, 1 = A_t; candidates as pairs with state 0 rejected, 1 kept,
 * 2 dropped by the shared-neighbour rule.  Size query with NULL buffers. */
lf_status lf_dual_matrix(lf_fields* f, int32_t which, int64_t* nnz, int32_t* rowptr,
                         int32_t* col);
lf_status lf_dual_candidates(lf_fields* f, int64_t* n_cand, int32_t* pairs, int32_t* state);

/* Counters since creation or the last reset: nnz of U, sum over steps of the
 * rows-of-interest sizes (|skeleton|), steps taken, zero-sum columns,
 * storage growth events. */
lf_status lf_stats(lf_fields* f, int64_t* nnz_u, int64_t* skeleton_total, int64_t* steps,
                   int64_t* empty_columns, int64_t* grow_events);

/* Entries read and written by the completed steps: the sums over steps of
 * nnz(U_t) and nnz(U_{t+1}) (for the algorithmic byte count of a step:
 * operator once, U_t in, U_{t+1} out). */
lf_status lf_traffic(lf_fields* f, int64_t* entries_in, int64_t* entries_out);

/* Device time of the step kernels, measured with HIP events on the
 * context stream around step launches while enabled: enable = 1 times every
 * launch, enable = k > 1 every k-th (the events cost a few microseconds of
 * wall time per timed launch), 0 stops, -1 only reads.  Total in ms and
 * number of launches timed since timing was last switched on. */
lf_status lf_step_timing(lf_fields* f, int32_t enable, double* total_ms, int64_t* launches);

/* ---- batches: many independent meshes advanced by the same launches ------
 * A batch is the disjoint union of its meshes: mesh m's vertices follow
 * those of meshes 0..m-1, its cells take layers off_m .. off_m + n_s[m] - 1
 * (off_m = sum of the earlier n_s), and all meshes share one base layer
 * above every cell.  Every row then computes exactly what it computes in a
 * solo run of its mesh (same operands, same order of operations), so each
 * mesh's fields are bit-identical to a solo run, while one step kernel per
 * time step covers the whole batch.  All meshes use one operator type and
 * one parameter set.  Inputs are host arrays, copied in. */
typedef struct lf_batch lf_batch;
lf_status lf_batch_create(lf_ctx* ctx, int32_t n_meshes, const double* const* V,
                          const int32_t* n_v, const int32_t* const* F, const int32_t* n_f,
                          int32_t op, const int32_t* const* seeds, const int32_t* n_s,
                          const lf_params* params, lf_batch** out);
lf_status lf_batch_destroy(lf_batch* b);
/* The batch's field object: step it with lf_step, time it with
 * lf_step_timing, read counters with lf_stats. */
lf_status lf_batch_fields(lf_batch* b, lf_fields** f);
/* Fields of one mesh in its own numbering (vertex ids from 0, cells 0..n_s-1,
 * base n_s), size query with NULL buffers as for lf_fields_export; host. */
lf_status lf_batch_export(lf_batch* b, int32_t mesh, int64_t* nnz, int32_t* rowptr,
                          int32_t* col, float* val);
/* Labels of one mesh in its own numbering (-1 where no cell), host. */
lf_status lf_batch_labels(lf_batch* b, int32_t mesh, int32_t* labels);

/* ---- serving: a continuous-batching job loop -------------------------------
 * Jobs (a mesh, seeds and a recipe) are queued on submission and admitted
 * while the HBM they will hold fits the budget and an active slot is free.
 * A job runs `steps` Euler steps, then `lloyd_rounds` times (re-seed,
 * re-initialise, `steps` steps), then labels and optionally the dual mesh
 * (with conv_eps > 0, each phase stops at convergence instead).  The steps of
 * all active jobs advance together: each step launch covers the slices of
 * every job that is stepping (one grouped kernel over their independent
 * field objects), in ticks of `chunk` launches; jobs join at the tick after
 * their admission and leave at the end of a phase.  Admission (mesh,
 * operator, fields) and the work between phases (re-seeding, labels, dual
 * mesh) run on a host worker thread per job, on the job's own stream, while
 * the others keep stepping.  A job's fields stay resident from admission to
 * completion, and its memory is released as soon as it finishes, which lets
 * queued jobs in.  Each job computes exactly what it computes alone.  The
 * caller drives the loop with lf_server_poll, which does not wait for the
 * GPU. */
typedef struct lf_server lf_server;
typedef struct {
  const double* V;     /* float64[n_v*3] */
  const int32_t* F;    /* int32[n_f*3] */
  const int32_t* seeds;/* int32[n_s] */
  int32_t n_v, n_f, n_s, op;
  int32_t steps, lloyd_rounds, dual_mesh, pad_;
  lf_params params;
  double conv_eps;     /* > 0: a phase ends at convergence (lf_step_until's rule */
  int32_t conv_every;  /*      with eps = conv_eps, check_every = conv_every); steps
                        *      is then the cap */
  int32_t n_types;     /* > 0: per-pair coefficients, as lf_fields_set_coefficients */
  const int32_t* layer_types;  /* int32[n_s+1] (NULL when n_types = 0) */
  const double* table;         /* double[n_types*n_types*3] */
} lf_job;
/* hbm_budget: bytes the active jobs may hold; max_active: concurrent jobs;
 * chunk: step launches per tick (1..256). */
lf_status lf_server_create(int32_t device, int64_t hbm_budget, int32_t max_active, int32_t chunk,
                           lf_server** out);
lf_status lf_server_destroy(lf_server* s);
/* Copies the job's inputs and queues it; *id identifies it.  LF_ENOMEM when
 * the job alone exceeds the budget. */
lf_status lf_server_submit(lf_server* s, const lf_job* job, int64_t* id);
/* Admits, issues and books work; returns the queue, active and finished
 * counts. */
lf_status lf_server_poll(lf_server* s, int32_t* n_queued, int32_t* n_active, int32_t* n_done);
/* Result of a finished job (LF_EBUSY while it runs): seeds int32[n_s] (final
 * seeds), labels int32[n_v] (may be NULL), n_tri and tris int32[3*n_tri]
 * (size query with tris NULL; 0 without dual mesh), latency_ms from
 * submission to completion, queue_ms spent waiting for admission, steps run.
 * Host buffers. */
/* Cancels a queued or active job: a queued job leaves the queue; an active
 * job's chunk in flight completes, then its memory is released at once.  A
 * cancelled job counts as done for lf_server_poll, its lf_server_result
 * fails with LF_EINVAL, and lf_server_release frees it.  LF_EINVAL for an
 * unknown or finished job. */
lf_status lf_server_cancel(lf_server* s, int64_t id);
lf_status lf_server_result(lf_server* s, int64_t id, int32_t* seeds, int32_t* labels,
                           int64_t* n_tri, int32_t* tris, double* latency_ms, double* queue_ms,
                           int64_t* steps);
/* Frees a finished job's results. */
lf_status lf_server_release(lf_server* s, int64_t id);
/* Bytes charged to the budget by active jobs and the peak so far: per job
 * the larger of an estimate from its size (used for admission) and what its
 * mesh and fields actually hold (storage growth included). */
lf_status lf_server_memory(lf_server* s, int64_t* in_use, int64_t* peak);
/* Times of a job on the host's monotonic clock (CLOCK_MONOTONIC, ms):
 * submission, admission (fields ready) and completion (0 until reached). */
lf_status lf_server_times(lf_server* s, int64_t id, double* submit_ms, double* admit_ms,
                          double* done_ms);
/* Ticks issued and grouped step launches made so far. */
lf_status lf_server_stats(lf_server* s, int64_t* ticks, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif
