/*
 * apsp.h — all-pairs shortest paths by blocked Floyd–Warshall on AMD
 * Instinct MI355X (gfx950).  C ABI of libapsp.so.
 *
 * The method (Rucci, De Giusti, Naiouf, "Blocked All-Pairs Shortest Paths
 * Algorithm on Intel Xeon Phi KNL Processor: A Case Study"):
 *   - Section "Floyd-Warshall Algorithm": the input is an N x N matrix D
 *     holding the direct distance between every pair of nodes; after N
 *     iterations (iteration k relaxes every pair through node k) D holds the
 *     shortest distances, and a second matrix P is produced when paths must
 *     be reconstructed.
 *   - Section "Data Locality": D is split into BS x BS blocks and processed
 *     in R = N/BS rounds; each round first closes the diagonal block, then
 *     the rest of its block row and block column, then every other block.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *   Layout     dist is row-major n x n, contiguous (leading dimension n).
 *              It is read as the weight matrix and overwritten in place by
 *              the distance matrix.  pred (optional) is row-major n x n
 *              int32, output only.
 *   Weights    int32: "no edge" is APSP_INF_INT32; float32: +inf.  The
 *              diagonal must be 0.  int32 weights must satisfy
 *              |w| <= apsp_weight_bound(n) so that no path length gets near
 *              the sentinel.  float32 weights must not be NaN or -inf.
 *   Output     dist(i,j) is the least total weight over all i->j paths,
 *              APSP_INF_INT32 / +inf when j is unreachable from i.
 *              pred(i,j) is the vertex just before j on a shortest i->j
 *              path; when several shortest paths end differently, the
 *              smallest such vertex.  pred(i,i) = pred(i,j unreachable) =
 *              APSP_NO_PRED.  (The paper's P records the last intermediate
 *              node added, which depends on the evaluation order; this
 *              canonical form does not, so blocked and unblocked schedules
 *              agree exactly.)
 *   Arithmetic int32 results are exact.  float32 results are exact when the
 *              weights are integers (every partial sum is then an integer
 *              well below 2^24); otherwise sums are rounded to float32 in
 *              the blocked order, within a relative 1e-6 of the exact value
 *              for short-hop paths.
 *   Memory     Pointers named dist/pred/packed_* are DEVICE pointers owned by
 *              the caller.  The library may allocate internal device
 *              workspace (kept per device and stream and reused -- the work
 *              matrix, a second stream and its events, and about 0.5 MiB of
 *              phase-1 closure scratch per stream that solves run on;
 *              released by apsp_release_workspace).
 *   Streams    apsp_solve* and apsp_batch_plan_execute enqueue work on the
 *              given hipStream_t (NULL = the legacy default stream) and
 *              return without waiting.  Argument errors are detected on the
 *              host before anything is enqueued.  Data-dependent outcomes
 *              (invalid weights, negative cycles) are written, when asked
 *              for, to a device status word (apsp_options_t.d_status).
 *   Errors     Functions never abort and never throw across the ABI.
 *              APSP_ERROR_HIP means a HIP runtime call failed; its code is
 *              available from apsp_last_hip_error() on the calling thread.
 *   Threads    apsp_solve* may be called concurrently from several threads
 *              on different streams.  Server calls are thread-safe.
 */
#ifndef APSP_H
#define APSP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define APSP_INF_INT32 1073741823 /* INT32_MAX / 2 : no edge / unreachable (int32) */
#define APSP_NO_PRED (-1)

typedef enum { APSP_INT32 = 0, APSP_FLOAT32 = 1 } apsp_dtype_t;

typedef enum {
    APSP_SUCCESS = 0,
    APSP_ERROR_INVALID_ARGUMENT = 1, /* bad pointer, size, dtype or option (host check) */
    APSP_ERROR_INVALID_VALUE = 2,    /* weights violate the preconditions above */
    APSP_ERROR_NEGATIVE_CYCLE = 3,   /* a cycle of negative total weight exists */
    APSP_ERROR_OUT_OF_MEMORY = 4,    /* device/host allocation or HBM budget */
    APSP_ERROR_HIP = 5,              /* a HIP runtime call failed */
    APSP_ERROR_QUEUE_FULL = 6,       /* server: admission queue is full */
    APSP_ERROR_NOT_READY = 7,        /* server: request still running */
    APSP_ERROR_CANCELLED = 8,        /* server: request cancelled or server destroyed */
    APSP_ERROR_TIMEOUT = 9,          /* server: wait timed out; single-launch barrier wait ran out */
    APSP_ERROR_UNKNOWN_TICKET = 10   /* server: no such (unreleased) request */
} apsp_status_t;

/* Short human-readable name of a status code (static storage). */
const char *apsp_status_string(apsp_status_t status);

/* hipError_t of the last failed HIP call made by the library on this thread. */
int apsp_last_hip_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int apsp_version(void);

/* Largest |w| accepted for int32 weights at size n: floor((2^28-1)/(n-1)).
 * Keeps every path length within +-2^28 and every intermediate sum of the
 * kernels free of overflow. */
int64_t apsp_weight_bound(int64_t n);

/* ------------------------------------------------------------------ single
 *
 * apsp_solve: one graph, blocked Floyd–Warshall (the paper's Sections
 * "Floyd-Warshall Algorithm" and "Data Locality"), three phases per round:
 *   phase 1  close the BS x BS diagonal block (k sequential, one workgroup)
 *   phase 2  update the block row and block column against it
 *   phase 3  min-plus update of every remaining block from its row's and
 *            column's panel blocks.
 *   dist   device, n*n elements of dtype, in place (weights in, distances out)
 *   pred   device, n*n int32 or NULL (no predecessors)
 *   n      number of vertices, 0 <= n <= 65536 (0 is a no-op)
 * Returns APSP_SUCCESS once the work is enqueued.
 */
apsp_status_t apsp_solve(void *dist, int32_t *pred, int64_t n, apsp_dtype_t dtype,
                         hipStream_t stream);

typedef struct {
    int32_t validate;      /* nonzero: check the weight preconditions on the device first;
                              on failure the solve is skipped and d_status gets
                              APSP_ERROR_INVALID_VALUE (dist/pred unchanged) */
    int32_t block_size;    /* 0 = automatic; else 64, 128 or 256 (256 with predecessors only
                              on the float32 route, see arith: its distance rounds take
                              256-wide blocks, its fallback recurrence 128-wide ones) */
    int32_t thread_tile;   /* 0 = automatic; 8 (8 x 8 register blocks, throughput) or
                              4 (4 x 4, latency-bound small solves; block size 64 only) */
    int32_t schedule;      /* 0 = automatic: for n >= 4096 (3072 for the fp64-key
                              recurrence), phase 3 of round r is split so that
                              phases 1-2 of round r+1 run beside most of it on a library-owned
                              second stream; 1 = one stream, rounds in order; 2 = the
                              two-stream split at any size with at least three rounds
                              (the device-gated fallback passes always run in order);
                              3 = every round in one launch: the blocked schedule over
                              small blocks (32-wide for int32 up to a padded order of 768,
                              else 64-wide) as a graph of tasks that workgroups take in
                              dependency order, each waiting only for the blocks it reads
                              (no co-residency needed, so concurrent solves are fine) --
                              automatic (0) for distance solves up to a padded
                              order of 4096 (directly or under use_graph; not in a
                              stepper or apsp_solve_noalloc).  3 requires distances only,
                              n <= 16384, block_size 0 or 64, thread_tile 0 or 4 and, for
                              int32 weights, arith 0 or 1 (int32 arithmetic), else
                              APSP_ERROR_INVALID_ARGUMENT; the values equal those of the
                              other schedules bit for bit */
    int32_t use_graph;     /* nonzero: capture the launch sequence once per shape into a
                              hipGraph and replay it (fewer launch gaps for small n) */
    int32_t arith;         /* Distances only, int32 weights (ignored for float32 weights):
                              0 = automatic (float32 arithmetic above n = 4096, and at
                              4096 where the single launch does not apply), 1 = int32
                              arithmetic, 2 = float32 arithmetic at any n.  float32
                              arithmetic holds the integers exactly while every operand
                              stays below 2^23 in magnitude, which the kernels check; if one
                              does not, the device redoes the solve in int32 arithmetic.
                              Either way the result is the exact int32 result.
                              With predecessors (either dtype): 0 = automatic (the float32
                              route from n = 4096), 1 = the exact fp64-key recurrence,
                              2 = the float32 route at any n: exact float32 distances, then
                              the canonical predecessors read off one float32 min-plus
                              product of (D(i,v) 2^S + v) with (W(v,j) 2^S), S = bits of
                              n - 1.  The device checks that every key involved is exact
                              (weights and distances small enough, the winning key's
                              distance equal to D(i,j)); if not, it runs the recurrence on
                              the original weights instead.  The results are the same. */
    int32_t *d_status;     /* device int32 or NULL: receives APSP_SUCCESS,
                              APSP_ERROR_INVALID_VALUE or APSP_ERROR_NEGATIVE_CYCLE, or
                              APSP_ERROR_TIMEOUT if a wait inside a dataflow kernel (the
                              single launch, the phase-1 closure) ran out (a second or
                              more; every wait is for work that running workgroups hold,
                              so only a faulty device gets there; dist is then partly
                              updated) */
    int32_t *d_arith;      /* device int32 or NULL: receives 1 if the result came from float32
                              arithmetic (with predecessors: the float32 route held), 0 if
                              from int32 arithmetic (the recurrence) */
    int32_t phase1;        /* 0 = automatic: the dataflow closure (3) for 4-byte distances
                              with 128- or 256-wide blocks, the one-step-per-barrier kernel
                              elsewhere; 1 = always the one-step-per-barrier kernel;
                              2 = always the blocked closure of the diagonal block inside
                              one 256-thread workgroup (four 64-wide sub-rounds; requires
                              block_size 256; applies to the rounds on 4-byte distances,
                              the fp64-key recurrence keeps the stepwise kernel); with 2
                              or 3 the two-stream split issues the rest of phase 3 as one
                              launch per round instead of two;
                              3 = the dataflow closure: the diagonal block solved by the
                              blocked schedule over 32-wide sub-blocks, one workgroup per
                              sub-block in one launch (requires block_size 128 or 256;
                              applies to the rounds on 4-byte distances, the fp64-key
                              recurrence keeps the stepwise kernel, and is their automatic
                              choice for 128- and 256-wide blocks, where the two-stream
                              split then issues the rest of phase 3 as one launch per
                              round; with real-valued float32 weights it rounds otherwise
                              than the stepwise kernel, within float32 rounding, and every
                              path -- direct, hipGraph, stepper, noalloc -- takes it alike) */
} apsp_options_t;

/* apsp_solve with options (NULL options = defaults = apsp_solve). */
apsp_status_t apsp_solve_ex(void *dist, int32_t *pred, int64_t n, apsp_dtype_t dtype,
                            hipStream_t stream, const apsp_options_t *options);

/* apsp_solve_ex for callers that cannot allocate memory (code under hipGraph
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, but every work matrix lives in a static device
 * array of apsp_noalloc_scratch_bytes() bytes (one per device, held until the
 * process ends) instead of library-allocated memory, and the call makes no
 * hipMalloc, hipFree, stream, event or graph creation.
 *   - The rounds run in order on the caller's stream: options->schedule must
 *     be 0 or 1 and options->use_graph 0 (else APSP_ERROR_INVALID_ARGUMENT).
 *   - Sizes whose work memory would exceed the array (any n <= 2048 fits)
 *     return APSP_ERROR_INVALID_ARGUMENT with nothing enqueued.
 *   - All calls on one device share that device's array, and its contents
 *     are whatever the last call left (each solve initialises every word it
 *     reads): calls whose work overlaps in time on one device race, so
 *     serialise them (one stream, or events).
 *   - No per-launch profiling (apsp_profile_*) is recorded for these calls.
 * Arguments, layout and data-dependent outcomes are those of apsp_solve_ex. */
apsp_status_t apsp_solve_noalloc(void *dist, int32_t *pred, int64_t n, apsp_dtype_t dtype,
                                 hipStream_t stream, const apsp_options_t *options);
/* Size in bytes of apsp_solve_noalloc's static per-device array. */
int64_t apsp_noalloc_scratch_bytes(void);

/* ---------------------------------------------------------------- steppers
 *
 * A solve issued a few rounds at a time (round-level preemption, for
 * serving: large solves yield the device between slices).  The rounds are
 * the blocked algorithm's rounds over k-blocks (Section "Data Locality":
 * diagonal block, its block row and column, then the remaining blocks);
 * the state between steps lives in device memory.  The launch sequence of
 * a solve never depends on the data (every data-dependent
 * choice is a device word), so apsp_stepper_begin records the whole
 * sequence of apsp_solve_ex for (dist, pred, stream) without issuing
 * anything, and apsp_stepper_step issues the next `rounds` rounds of it
 * (rounds <= 0: everything left), the distance state staying in device
 * memory between steps.  Round counts include the device-gated fallback
 * passes, which cost one near-empty launch per kernel when skipped.  The
 * result after the last step is the result of apsp_solve_ex with the same
 * options (use_graph ignored), bit for bit.
 *
 * The stepper owns its work memory (allocated at create for any alignment
 * of dist) and its second stream, so slices of several steppers and any
 * other work may interleave on one device, even on one caller stream.
 * Steps are issued on the stream given to begin.  dist/pred must stay
 * valid until the last step's work completes.  A stepper is not
 * thread-safe.  begin while a previous solve is not fully issued returns
 * APSP_ERROR_NOT_READY.  destroy synchronises the stepper's streams first.
 */
typedef struct apsp_stepper apsp_stepper_t;
apsp_status_t apsp_stepper_create(int64_t n, apsp_dtype_t dtype, int32_t want_pred,
                                  const apsp_options_t *options, apsp_stepper_t **out);
apsp_status_t apsp_stepper_begin(apsp_stepper_t *stepper, void *dist, int32_t *pred, hipStream_t stream);
/* *done (optional) = 1 once the whole solve has been issued. */
apsp_status_t apsp_stepper_step(apsp_stepper_t *stepper, int32_t rounds, int32_t *done);
/* Rounds in the recorded solve (-1 for NULL; 0 before begin). */
int64_t apsp_stepper_rounds(const apsp_stepper_t *stepper);
/* Waits for the stepper's streams, then frees it (always, also on an error:
 * APSP_ERROR_HIP if a wait or the release of its memory failed). */
apsp_status_t apsp_stepper_destroy(apsp_stepper_t *stepper);

/* ---------------------------------------------------------------- profiling
 *
 * Per-kernel timing of the single-graph path for benchmarks: between
 * apsp_profile_begin and apsp_profile_end every phase kernel the library
 * launches (from any thread) is bracketed by two hipEvents on its own
 * stream.  apsp_profile_end waits for the recorded events, fills *out with
 * launch counts, summed and largest durations, and the number of
 * (i, j, k) relaxations each kind performed, then stops recording.
 */
typedef struct {
    int64_t launches;
    double total_ms;
    double max_ms;
    double updates; /* (i,j,k) relaxations summed over the launches */
} apsp_kernel_time_t;

typedef struct {
    apsp_kernel_time_t phase1;       /* diagonal block closure */
    apsp_kernel_time_t phase2;       /* block row / block column products */
    apsp_kernel_time_t phase3;       /* remaining-block products (all, or all but the next
                                        round's block row/column under the two-stream schedule) */
    apsp_kernel_time_t other;        /* set-up and wrap-up passes */
    apsp_kernel_time_t phase3_cross; /* two-stream schedule: the next round's block row/column */
    apsp_kernel_time_t pred_product; /* predecessors read off the float32 key product */
    apsp_kernel_time_t phase1_blocked; /* the phase-1 launches (also counted in phase1) that
                                          were the blocked closure of the diagonal block */
    apsp_kernel_time_t single_launch;  /* the single-launch schedule's kernel (all rounds) */
    apsp_kernel_time_t phase1_flow;    /* the phase-1 launches (also counted in phase1) that
                                          were the dataflow closure */
} apsp_profile_t;

apsp_status_t apsp_profile_begin(void);
apsp_status_t apsp_profile_end(apsp_profile_t *out);

/* Measures one 32-bit VALU instruction rate of the device at its actual
 * clock, in lane-instructions per second over the whole device (every CU
 * busy, 8 wavefronts per SIMD, 8 independent accumulators per lane, a loop
 * body of nothing but the measured instructions), in steady state (launches
 * of N and 3N iterations, rate from the differences, best of three pairs).
 *   kind 0  the float32 min-plus step of the phase-3 kernels: two v_add_f32
 *           and one v_min3_f32 per two (i,j,k) relaxations
 *   kind 1  v_add_f32      kind 2  v_min3_f32     kind 3  v_add_u32
 *   kind 4  v_min_f32      kind 5  the int32 step: two v_add_u32, one v_min3_i32
 * *elapsed_ms receives the duration of the longer launch.  Synchronises the
 * device; allocates 16 bytes of device memory for the duration of the call. */
apsp_status_t apsp_probe_valu(int32_t kind, double *lane_instr_per_s, double *elapsed_ms);

/* Release the calling device's internal workspace, cached graphs and
 * per-stream helpers (second streams and their events, closure scratch);
 * later solves make them again.  Must not overlap with solves in flight
 * on that device. */
apsp_status_t apsp_release_workspace(void);

/* ------------------------------------------------------------------ paths
 *
 * Path reconstruction (the paper keeps the path matrix so that shortest
 * paths, not only their lengths, can be recovered; Section "Floyd-Warshall
 * Algorithm").  For each query t the vertices of the shortest path from
 * src[t] to dst[t] are read from the canonical predecessor matrix.
 *   pred     device, n x n int32, as written by apsp_solve with predecessors
 *   src, dst device int32[q], vertex ids
 *   paths    device int32[q * max_len]: query t's path, src[t] first and
 *            dst[t] last, at paths[t * max_len ...]
 *   lengths  device int32[q]: number of vertices on the path (1 when
 *            src == dst), 0 when dst is unreachable, APSP_PATH_TOO_LONG when
 *            the path has more than max_len vertices, APSP_PATH_BAD_QUERY
 *            for a vertex id outside [0, n), APSP_PATH_BROKEN when the
 *            chain leaves [0, n) or exceeds n - 1 hops (pred was not
 *            produced by apsp_solve).
 * Enqueued on stream; every walk is bounded by n steps and max_len writes.
 */
#define APSP_PATH_TOO_LONG (-1)
#define APSP_PATH_BAD_QUERY (-2)
#define APSP_PATH_BROKEN (-3)
apsp_status_t apsp_paths(const int32_t *pred, int64_t n, const int32_t *src, const int32_t *dst, int32_t q,
                         int32_t *paths, int32_t max_len, int32_t *lengths, hipStream_t stream);

/* The paper's form of the path matrix (Section "Floyd-Warshall Algorithm":
 * P holds an intermediate vertex of the shortest path, from which the path
 * is rebuilt recursively), derived from the canonical predecessor matrix:
 * out(i, j) = pred(i, j) when that is an intermediate vertex (not i), else
 * APSP_NO_PRED (direct edge, i == j, or unreachable).  Rebuilding
 * path(i, j) = path(i, out(i, j)) + path(out(i, j), j) yields a shortest
 * path (sub-paths of shortest paths are shortest; with ties the second half
 * may differ from the one apsp_paths reads), in at most 2n - 3 calls.  The
 * paper's matrix records the most recently added intermediate vertex, which
 * depends on the evaluation order; this one does not.  pred, out: device
 * n x n int32 (out may equal pred).
 */
apsp_status_t apsp_pred_to_intermediate(const int32_t *pred, int64_t n, int32_t *out, hipStream_t stream);

/* ----------------------------------------------------------------- batched
 *
 * Many independent graphs of uneven size, solved by one persistent fused
 * launch that runs all three phases of every graph: each 256-thread
 * workgroup pulls graphs, largest first, from a device work counter; graphs
 * with n > 64 are solved by a whole workgroup with 64- or 128-wide k-blocks
 * (the team configuration of the graph's size class, see autotuning),
 * graphs with n <= 64 by a single wavefront in registers.  int32 distance
 * batches run as two launches, the graphs whose weights rule float32
 * arithmetic out (any negative weight, or |w|(n-1) >= 2^23) in int32
 * arithmetic, the others in float32 (exact).  Same conventions and results
 * as apsp_solve, graph by graph.
 *
 *   ns          host, sizes of the batch graphs, 1 <= ns[b] <= 1024
 *   offsets     host, element offset of graph b in the packed buffers;
 *               offsets[b] % 4 == 0; graphs must not overlap
 *   packed_dist device, 16-byte aligned; graph b occupies
 *               [offsets[b], offsets[b] + ns[b]^2), row-major with leading
 *               dimension ns[b]; weights in, distances out
 *   packed_pred device int32, 16-byte aligned, same offsets; required when
 *               the plan was made with want_pred, NULL otherwise
 *   d_status    device int32[batch] or NULL: per graph APSP_SUCCESS or
 *               APSP_ERROR_NEGATIVE_CYCLE
 * A plan owns the device copy of the metadata, the per-workgroup work
 * matrices and the work counters (device memory of about
 * 2 x CUs x (64- or 128-padded max n)^2 x 4 or 8 bytes).  It may be executed any
 * number of times, also from a captured hipGraph, but executions of one plan
 * must not overlap in time (use one plan per concurrent stream).  The plan
 * must outlive the work it enqueued.
 */
typedef struct apsp_batch_plan apsp_batch_plan_t;

apsp_status_t apsp_batch_plan_create(const int32_t *ns, const int64_t *offsets, int32_t batch,
                                     apsp_dtype_t dtype, int32_t want_pred,
                                     apsp_batch_plan_t **out_plan);
apsp_status_t apsp_batch_plan_execute(const apsp_batch_plan_t *plan, void *packed_dist,
                                      int32_t *packed_pred, int32_t *d_status, hipStream_t stream);
apsp_status_t apsp_batch_plan_destroy(apsp_batch_plan_t *plan);

/* As apsp_batch_plan_create, with the team configuration of each graph
 * (n > 64) forced: team_config[b] = 0 wavefront-private 64 x 64 tiles with
 * 8 x 8 registers per lane, 1 workgroup 64 x 64 tiles with 4 x 4 per thread,
 * 2 workgroup 128 x 128 tiles with 8 x 8 per thread and 128-wide k-blocks,
 * 3 (distances) the work matrix padded to 64 only, 128-wide k-blocks with a
 * 64-wide last block and tiles of 128 or 64 rows by 128 or 64 columns,
 * -1 = the tuning table's choice for the graph's size class.  NULL = all -1.
 * A distance batch whose graphs above 64 vertices all have configuration 1
 * or 3 runs in a kernel that holds only those two (and the n <= 64 path):
 * one launch, no register spills.  Otherwise configuration 3 runs as 2. */
apsp_status_t apsp_batch_plan_create_ex(const int32_t *ns, const int64_t *offsets, int32_t batch,
                                        apsp_dtype_t dtype, int32_t want_pred, const int8_t *team_config,
                                        apsp_batch_plan_t **out_plan);

/* ------------------------------------------------------------- autotuning
 *
 * The batched launch picks a team configuration (tile size and per-thread
 * register block, see apsp_batch_plan_create_ex; 3 for distances by default)
 * per graph from a table
 * indexed by (dtype, predecessors, size class), 8 size classes n in
 * (64,128], (128,192], (192,256], (256,320], (320,384], (384,448],
 * (448,512], (512,1024].  The table starts from
 * built-in defaults, is read from the JSON file named by the environment
 * variable APSP_TUNE_TABLE on first use, and can be measured on the current
 * device: apsp_batch_autotune builds one synthetic batch with
 * graphs_per_class graphs in every size class (0 = CU count) and, class by
 * class (coordinate descent, the other classes at their current choice),
 * times the whole batch with each configuration for that class (reps timed
 * executions, 0 = 3) and keeps the fastest (configuration 3 only for
 * distances).  ms_out[class * 4 + config] (32 doubles; 0 where not timed)
 * (when not NULL) receives the per-execution milliseconds of each trial.
 * It allocates device memory and synchronises its own stream.
 */
apsp_status_t apsp_batch_autotune(apsp_dtype_t dtype, int32_t want_pred, int32_t graphs_per_class,
                                  int32_t reps, double *ms_out);
/* As apsp_batch_autotune, on a synthetic batch with the caller's graph sizes
 * (host ns[batch], 1 <= ns[b] <= 1024): tunes the classes the workload
 * actually has, in its own mix.  Classes without graphs keep their entry. */
apsp_status_t apsp_batch_autotune_sizes(const int32_t *ns, int32_t batch, apsp_dtype_t dtype,
                                        int32_t want_pred, int32_t reps, double *ms_out);
/* Team configuration the table gives a graph of n vertices (-1: n <= 64, one wavefront; 0..3 as
 * for apsp_batch_plan_create_ex). */
int32_t apsp_batch_config(int64_t n, apsp_dtype_t dtype, int32_t want_pred);
apsp_status_t apsp_tune_save(const char *path);
apsp_status_t apsp_tune_load(const char *path);

/* create + execute; the plan is freed by a later library call once the
 * stream has passed it (no synchronisation here). */
apsp_status_t apsp_solve_batched(void *packed_dist, int32_t *packed_pred, const int32_t *ns,
                                 const int64_t *offsets, int32_t batch, apsp_dtype_t dtype,
                                 hipStream_t stream);

/* ------------------------------------------------------------------ server
 *
 * A request loop on one GPU with continuous batching.  apsp_server_submit
 * copies the host weights (n x n, row-major, dtype) into library-owned
 * pinned memory and queues the request; a scheduler thread admits queued
 * requests in arrival order whenever the device-memory budget
 * (hbm_budget_bytes) and the resident-request limit (max_inflight) allow,
 * and launches them without waiting for earlier work: requests admitted
 * together with n <= batch_max_n are coalesced per (dtype, predecessors)
 * into one batched fused launch, larger ones run apsp_solve on one of
 * n_streams streams, so work of different requests overlaps on the device.
 * Results (distances, and predecessors when asked for) stay resident in
 * device memory until apsp_server_release, which returns their bytes to the
 * budget.  Each result equals what apsp_solve computes for that request
 * alone.  A request whose footprint exceeds the whole budget is refused at
 * submit with APSP_ERROR_OUT_OF_MEMORY; a full queue gives
 * APSP_ERROR_QUEUE_FULL.  Latency = completion observed by the scheduler
 * (event polled every 50 us) minus entry into apsp_server_submit.
 * All calls are thread-safe; apsp_server_destroy must not overlap other
 * calls on the same server except waits already blocked in
 * apsp_server_wait (they return APSP_ERROR_CANCELLED).
 */
typedef struct apsp_server apsp_server_t;

typedef struct {
    int64_t hbm_budget_bytes; /* device bytes the server may hold (0 = 1/2 of free memory) */
    int32_t max_inflight;     /* requests resident at once (0 = 64) */
    int32_t n_streams;        /* HIP streams used for large requests (0 = 8) */
    int32_t max_queue;        /* pending requests before submit fails (0 = 4096) */
    int32_t batch_max_n;      /* requests with n <= this are coalesced into batched launches
                                 (0 = 512, negative = never; at most 1024) */
    int32_t slice_rounds;     /* 0: a large request's whole solve is issued at admission;
                                 > 0: it is issued this many rounds at a time (a stepper,
                                 see apsp_stepper_*), the next slice once the last one has
                                 finished, so later requests are not queued behind it */
} apsp_server_config_t;

typedef struct {
    const void *weights; /* host, n rows of n elements of dtype, row-major, leading dimension ld */
    int64_t n;
    int64_t ld;          /* elements between row starts (0 = n) */
    apsp_dtype_t dtype;
    int32_t want_pred;
    int32_t borrow;      /* 0: weights are copied during submit; nonzero: weights are pinned host
                            memory (hipHostMalloc) that stays valid and unchanged until the
                            request completes, uploaded directly without a host copy */
} apsp_request_t;

typedef struct {
    int64_t submitted, completed, failed, cancelled;
    int64_t queued, inflight;
    int64_t bytes_in_use;
    double p50_latency_ms, p99_latency_ms; /* submit -> result ready, completed requests */
    double solves_per_s;                   /* completed / (last completion - first submit) */
    double p50_small_ms, p99_small_ms;     /* the same for requests coalesced into batched launches */
    double p50_large_ms, p99_large_ms;     /* ... and for the others (0 when there were none) */
} apsp_server_stats_t;

apsp_status_t apsp_server_create(const apsp_server_config_t *config, apsp_server_t **out);
apsp_status_t apsp_server_submit(apsp_server_t *server, const apsp_request_t *request,
                                 uint64_t *ticket);
apsp_status_t apsp_server_poll(apsp_server_t *server, uint64_t ticket);
apsp_status_t apsp_server_wait(apsp_server_t *server, uint64_t ticket, int64_t timeout_us);
/* Device pointers of a finished request's resident results (valid until release). */
apsp_status_t apsp_server_result(apsp_server_t *server, uint64_t ticket, const void **d_dist,
                                 const int32_t **d_pred);
/* Copy a finished request's results to host memory (h_pred may be NULL). */
apsp_status_t apsp_server_copy_result(apsp_server_t *server, uint64_t ticket, void *h_dist,
                                      int32_t *h_pred);
apsp_status_t apsp_server_release(apsp_server_t *server, uint64_t ticket);
apsp_status_t apsp_server_stats(apsp_server_t *server, apsp_server_stats_t *stats);
/* Cancels pending and running requests (their tickets report CANCELLED) and frees all. */
apsp_status_t apsp_server_destroy(apsp_server_t *server);

#ifdef __cplusplus
}
#endif

#endif /* APSP_H */
