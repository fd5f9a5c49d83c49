/*
 * gltrsv -- GrowLocal-scheduled sparse triangular solves on AMD MI355X
 * (gfx950).  C ABI of the shared library libgltrsv.so.
 *
 * The library solves A x = b for a sparse, non-singular, triangular A by
 * forward substitution (lower-triangular A, Eq. (2.1) of Boehnlein, Papp,
 * Steiner, Matzoros and Yzelman, "Efficient parallel scheduling for sparse
 * triangular solvers", arxiv 2503.05408) or backward substitution (upper-
 * triangular A, its mirror, Sec. 2.2), for one or several right-hand sides,
 * executed on the GPU under a bulk-synchronous schedule (Definition 2.1)
 * built by the GrowLocal scheduler (Algorithm 3.1, optionally block-parallel,
 * Sec. 3.1, or after Funnel coarsening, Sec. 4) and laid out in the
 * schedule's order (Sec. 5).  One system, many systems in one launch, and a
 * continuous-batching server share the same kernels.
 *
 * Conventions shared by every call:
 *  - Return value: 0 (GLTRSV_OK) on success, a negative GLTRSV_E* code on
 *    failure.  Nothing is thrown across the ABI.  gltrsv_last_error() returns
 *    a text for the last failure of the calling thread.
 *  - Matrices are CSR with int64 row pointers, int32 column indices and
 *    binary64 values, in host memory owned by the caller; the library copies
 *    what it needs.  Within each row the columns ascend strictly and the
 *    diagonal is the last stored entry of a lower-triangular A (the first of
 *    an upper-triangular one, see gltrsv_plan_opts.triangle); it must be
 *    non-zero (the matrix is non-singular, Sec. 2.2).  Every stored entry is
 *    an edge of the DAG (Sec. 2.2), explicit zeros included.
 *  - Vectors passed to solve calls are device pointers (hipMalloc'd or torch
 *    CUDA tensors), caller-owned, n binary64 values in the original row
 *    numbering.
 *  - Streams are hipStream_t values passed as void* (NULL = default stream).
 *    Solve calls are asynchronous with respect to the host.
 *  - Results: every x_i is computed as acc <- b_i; acc <- acc - (A_ij * x_j)
 *    for the stored off-diagonals of row i in stored order, each operation
 *    rounded on its own (no fused multiply-add), then x_i <- acc / A_ii with
 *    one correctly rounded division.  The result is therefore bit-identical
 *    for every schedule, every core count and every execution form
 *    (persistent, plain, semi-asynchronous, several right-hand sides,
 *    batched, served).
 */
#ifndef GLTRSV_H
#define GLTRSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define GLTRSV_OK          0
#define GLTRSV_EINVAL     -1   /* null pointer, negative size, bad option    */
#define GLTRSV_ENOTLOWER  -2   /* an entry on the wrong side of the diagonal
                                  (above it; below it for GLTRSV_UPPER)    */
#define GLTRSV_ESINGULAR  -3   /* diagonal missing, not last, or zero        */
#define GLTRSV_EUNSORTED  -4   /* off-diagonal columns not strictly rising   */
#define GLTRSV_ERANGE     -5   /* index out of range, or n too large         */
#define GLTRSV_ENOMEM     -6   /* host or device allocation failed           */
#define GLTRSV_EAGAIN     -7   /* server: request does not fit the budget    */
#define GLTRSV_EHIP       -8   /* a HIP runtime call failed                  */
#define GLTRSV_ETIMEDOUT  -9   /* a device-side wait exceeded its spin limit */
#define GLTRSV_ENOTSUP   -10   /* not supported on this device/build         */
#define GLTRSV_ENOENT    -11   /* server: no pending request with this ticket */

/* Text for the last error on the calling thread (never NULL). */
const char *gltrsv_last_error(void);

/* Library version, e.g. "0.1.0". */
const char *gltrsv_version(void);

/* ---------------------------------------------------------------- inputs */
typedef struct gltrsv_csr {
    int64_t n;               /* rows = columns                                */
    int64_t nnz;             /* stored entries, diagonal included             */
    const int64_t *row_ptr;  /* [n+1], row_ptr[0] = 0, row_ptr[n] = nnz       */
    const int32_t *col;      /* [nnz]                                         */
    const double *val;       /* [nnz]; may be NULL for pattern-only calls     */
} gltrsv_csr;

/* Checks the conventions above for a lower-triangular A (plan creation
 * checks an upper-triangular one itself).  Returns GLTRSV_OK or the first
 * violation (ENOTLOWER, ESINGULAR, EUNSORTED, ERANGE, EINVAL).  n is limited
 * to 2^30 - 1 rows (the device stream packs a row index into 30 bits). */
int gltrsv_check_csr(const gltrsv_csr *A);

/* ------------------------------------------------------------- schedules */
#define GLTRSV_SCHED_GROWLOCAL 0   /* Algorithm 3.1                           */
#define GLTRSV_SCHED_WAVEFRONT 1   /* level sets: one superstep per wavefront */
#define GLTRSV_SCHED_AUTO      2   /* both; keep the lower predicted time     */
#define GLTRSV_SCHED_GIVEN     3   /* plan info only: schedule passed in      */

/* gltrsv_plan_opts.triangle */
#define GLTRSV_LOWER 0
#define GLTRSV_UPPER 1

/* Stream filling (gltrsv_plan_opts.pack), Sec. 5 reorder plus packing:
 *  AUTO   -- device for systems with at least 2^20 stored entries, else host;
 *  HOST   -- one host pass over the entries;
 *  DEVICE -- device kernels: row lengths, a wavefront prefix scan of them
 *            staged through LDS, and the scatter of the entries. */
#define GLTRSV_PACK_AUTO   0
#define GLTRSV_PACK_HOST   1
#define GLTRSV_PACK_DEVICE 2

typedef struct gltrsv_plan_opts {
    int32_t k;              /* cores of the BSP schedule (Def. 2.1), >= 1     */
    double L;               /* barrier cost in weight units (Sec. 3, Eq. 3.1) */
    double alpha0;          /* first superstep length parameter, >= 1         */
    double growth;          /* alpha growth factor, > 1                       */
    double accept;          /* worthy iff beta >= accept * best beta          */
    int32_t schedule_kind;  /* GLTRSV_SCHED_*                                 */
    int32_t reorder;        /* 1 (default): the device stream is in the
                               schedule order of Sec. 5; b/x always stay in
                               the original numbering (see gltrsv_solve).
                               0: the plan also keeps A in the caller's CSR
                               order for gltrsv_solve_unordered (the
                               no-reorder comparison of Sec. 5 / Table 7.3);
                               12 nnz + 12 n more device bytes                */
    int32_t block_size;     /* device threads per workgroup: 0 or 256 (the
                               kernels are compiled for 256-thread
                               workgroups; any other value is ENOTSUP)       */
    int32_t grid_blocks;    /* workgroups of the persistent kernel;
                               0 = all that can be co-resident (<= 2048)      */
    int32_t cooperative;    /* 1: launch the kernels whose workgroups wait
                               for each other (gltrsv_solve, the wave-core
                               gltrsv_solve_async) with
                               hipLaunchCooperativeKernel, which checks the
                               grid against the co-resident capacity (about
                               20-40 us more per launch).  0 (default): a
                               plain launch of the same grid.  Neither keeps
                               kernels on other streams from delaying some
                               workgroups (measured on MI355X); the
                               persistent kernels do not need that (their
                               waves claim and steal work, see
                               gltrsv_plan_set_steal_wait) and the
                               lane-core semi-asynchronous kernels claim
                               chunks in order                                */
    int32_t analysis_threads; /* host threads of the GrowLocal analysis: the
                               iterations of one superstep (Algorithm 3.1)
                               start from the same state and run
                               concurrently; 0 = automatic (1 below 2e5 rows,
                               else up to 8).  The schedule does not depend
                               on it.                                        */
    int32_t pack;             /* GLTRSV_PACK_*: where the packed stream is
                               filled (the layout of tasks, chunks and lanes
                               is always computed on the host); the stream is
                               the same either way                           */
    int32_t blocks;           /* block-parallel scheduling (Sec. 3.1) when > 1:
                               the rows are cut into that many diagonal
                               blocks of equal row count (block b = rows
                               [floor(b n/B), floor((b+1) n/B))), each block
                               is scheduled by GrowLocal as a DAG of its own
                               (edges from earlier blocks dropped) with the
                               weights of the full rows, on separate host
                               threads, and block b's supersteps follow those
                               of blocks 0..b-1; 0 or 1 = the whole matrix   */
    int32_t triangle;         /* GLTRSV_LOWER (forward substitution, Eq. (2.1))
                               or GLTRSV_UPPER (backward substitution, its
                               mirror, Sec. 2.2): A is upper-triangular with
                               the diagonal FIRST in every row and rising
                               columns; x_i = (b_i - sum_{j>i} A_ij x_j) /
                               A_ii for i = n-1 .. 0, the sum as a running
                               subtraction in stored order.  The schedule is
                               built on the reversed numbering (row i is
                               vertex n-1-i) so GrowLocal runs in the solve's
                               direction; gltrsv_schedule and
                               gltrsv_plan_schedule report it per row.       */
    int32_t funnel_max_weight; /* > 0: Funnel coarsening (Sec. 4) before
                               GrowLocal: the long edges of triangles are
                               removed (approximate transitive reduction),
                               the DAG is cut into in-funnels (Algorithm 4.1:
                               reverse topological order, largest vertex
                               first, a parent joins once all its children
                               have) of at most this weight (stored entries;
                               a single vertex may exceed it), GrowLocal
                               schedules the coarsened DAG and every row
                               takes its part's core and superstep; overrides
                               `blocks`.  0 = off                            */
    int32_t exec_hint;        /* the execution AUTO predicts: 0 = persistent
                               (barriers; per superstep 3 us plus the larger
                               of 0.18 us per entry of its longest task and
                               its entries at 4e4 entries/us), 1 =
                               semi-asynchronous (gltrsv_solve_async: the
                               larger of the critical path -- rows of a task
                               one after another at 0.18 us per entry, a
                               parent in another task adding 1.5 us -- and
                               all entries at 4e4 entries/us, plus 10 us),
                               2 = one workgroup (gltrsv_solve_local): the
                               plan also builds that form's layout and
                               prefers it; AUTO predicts 0.1 us per group
                               (four entries of every lane, see
                               gltrsv_solve_local).  2 needs core_width 1
                               and, unless schedule_kind is WAVEFRONT,
                               k <= 64 (EINVAL otherwise); a WAVEFRONT
                               schedule is then dealt onto 64 cores, row r
                               of a level going to core r mod 64           */
    int32_t core_width;       /* lanes per BSP core in gltrsv_solve,
                               gltrsv_solve_plain and gltrsv_solve_async:
                               1 (0 = default) = a core is one lane of a
                               wavefront; 64 = a core is a whole wavefront:
                               the lanes gather and multiply 64 entries of a
                               row at once and the wave subtracts the
                               products in stored order (the same bits), for
                               rows of many entries.  k then counts
                               wavefronts (the device holds 1,024 at one per
                               SIMD).  Several right-hand sides, batches and
                               the server keep one lane per core.           */
} gltrsv_plan_opts;

/* Fills the paper's parameters: k = 22 (the core count of the main
 * experiments, Sec. 7.1), L = 500 (Sec. 3, footnote), alpha0 = 20 and
 * growth 1.5 (Sec. 3), accept = 0.97 (proof of Theorem 3.1, Appendix B),
 * GrowLocal, defaults for the device fields. */
void gltrsv_default_opts(gltrsv_plan_opts *opts);

/* Wavefronts (Sec. 1, Fig. 1.1; Sec. 6.2): level[i] = 1 for a row with no
 * off-diagonal, else 1 + the largest level among its columns.  level may be
 * NULL.  *nlevels = number of wavefronts (= vertices on a longest path).
 * Host only. */
int gltrsv_levels(const gltrsv_csr *A, int32_t *level, int32_t *nlevels);

/* Builds the BSP schedule of A (Def. 2.1) with opts->schedule_kind:
 *  GROWLOCAL -- Algorithm 3.1 with Rule I: cores filled in order; core 0
 *     takes up to floor(alpha) vertices, every later core up to the weight of
 *     core 0; the smallest-ID vertex exclusive to the core first, else the
 *     smallest-ID vertex free at the barrier; beta of Eq. (3.1); alpha grows
 *     by opts->growth while the iteration stays worthy; the last worthy
 *     iteration becomes the superstep.  Vertex weight = stored entries of the
 *     row (Sec. 2.2).
 *  WAVEFRONT -- superstep = level - 1, core = rank of the row in its level.
 *  AUTO -- builds both and keeps the one with the lower predicted device time
 *     (gltrsv_plan_info.predicted_us); under the literal rules GrowLocal puts
 *     a DAG whose ready vertices are all exclusive to core 1 (one source, e.g.
 *     a natural-order grid) in a single serial superstep, which AUTO avoids.
 * Outputs (host arrays of n int32, caller-owned): core[i] in [0, k) (for
 * WAVEFRONT in [0, widest level)), superstep[i] in [0, S), *S = supersteps.
 * Host only; does not touch the GPU. */
int gltrsv_schedule(const gltrsv_csr *A, const gltrsv_plan_opts *opts,
                    int32_t *core, int32_t *superstep, int32_t *S);

/* Permutation of Sec. 5: perm[t] = the row at position t when rows are
 * listed by superstep, then core, then original index.  Host only. */
int gltrsv_reorder(int64_t n, const int32_t *core, const int32_t *superstep, int32_t *perm);

/* ------------------------------------------------------------------ plans */
typedef struct gltrsv_plan gltrsv_plan;

typedef struct gltrsv_plan_info {
    int64_t n, nnz;
    int32_t supersteps;     /* S of the schedule                             */
    int32_t wavefronts;     /* number of levels of the DAG                    */
    int64_t tasks;          /* non-empty (superstep, core) pairs              */
    int64_t chunks;         /* 64-task device work units                      */
    int64_t stream_slots;   /* packed entries incl. padding (>= nnz)          */
    int64_t device_bytes;   /* device memory held by the plan                 */
    int64_t analysis_ns;    /* host time of plan creation                     */
    uint64_t pattern_key;   /* hash of (n, row_ptr, col)                      */
    int32_t grid_blocks;    /* persistent-kernel workgroups                   */
    int32_t block_size;     /* threads per workgroup                          */
    int64_t max_task_rows;  /* longest row sequence on one core in a superstep */
    int32_t schedule_kind;  /* the schedule built (AUTO resolves to one)      */
    double predicted_us;    /* cost-model prediction of one solve in the
                               execution named by opts.exec_hint              */
    int32_t device_packed;  /* 1 if the stream was filled on the device       */
    int32_t async_grid_blocks; /* workgroups of gltrsv_solve_async            */
    int32_t exec_form;      /* preferred execution form of gltrsv_solve_auto
                               (GLTRSV_EXEC_*)                                */
    int32_t core_width;     /* lanes per core of gltrsv_solve / _plain /
                               _async                                         */
    int64_t local_groups;   /* plans built with exec_hint 2: the groups one
                               lane of gltrsv_solve_local steps through (its
                               serial path); else 0                           */
    int64_t local_records;  /* ... and the records they are cut into          */
    int64_t local_far;      /* ... and the operands read from x in global
                               memory rather than from LDS                    */
    int32_t row_dpp;        /* core width 64: 1 if the wave-core solves
                               subtract a row's products through DPP lane
                               broadcasts (systems averaging at least 8
                               stored off-diagonals a row), 0 if through
                               readlane; the bits are the same either way     */
} gltrsv_plan_info;

/* Analyses A (checks, schedule, Sec. 5 order) and uploads the packed matrix
 * to the current HIP device.  The values of A are captured; the matrix data
 * of a plan never changes afterwards.  Solves on one plan must not overlap
 * in time, whatever their streams: they share the plan's barrier and error
 * words (and, for in-place semi-asynchronous solves, its copy of b).  Use one
 * plan per concurrent stream, or a batch.  Batches and servers only read a
 * plan's matrix data and may use it meanwhile.
 * *out is owned by the library until gltrsv_plan_destroy. */
int gltrsv_plan_create(const gltrsv_csr *A, const gltrsv_plan_opts *opts, gltrsv_plan **out);

int gltrsv_plan_info_get(const gltrsv_plan *plan, gltrsv_plan_info *out);

/* Copies the plan's schedule to host arrays of n int32 (any may be NULL). */
int gltrsv_plan_schedule(const gltrsv_plan *plan, int32_t *core, int32_t *superstep, int32_t *perm);

int gltrsv_plan_destroy(gltrsv_plan *plan);

/* ----------------------------------------------------------------- solves */
/* Persistent solve: one launch runs every superstep; between supersteps
 * (Def. 2.1) the waves wait for a device-scope count of the superstep's
 * completed chunks (or wavefront-core tasks).  Each chunk is claimed once
 * per solve; a workgroup that has waited long for a superstep runs its
 * unclaimed chunks itself (gltrsv_plan_set_steal_wait), so the solve needs
 * no co-residency and other work on the device only delays it.  b and x are
 * device arrays in the original numbering; b may alias x (in-place solve).
 * Reading b and writing x fuse the permutation of Sec. 5. */
int gltrsv_solve(gltrsv_plan *plan, const double *b, double *x, void *stream);

/* Baseline: one kernel launch per superstep; the kernel boundary is the
 * barrier.  Same arguments and results as gltrsv_solve. */
int gltrsv_solve_plain(gltrsv_plan *plan, const double *b, double *x, void *stream);

/* The same schedule without the reorder of Sec. 5: A stays in the caller's
 * CSR order on the device and each lane walks its task's rows through the
 * row pointers, one launch per superstep (compare gltrsv_solve_plain, which
 * reads the reordered, lane-interleaved stream).  Same arguments and the
 * same bits as gltrsv_solve.  Needs a plan created with opts.reorder = 0
 * (GLTRSV_ENOTSUP otherwise). */
int gltrsv_solve_unordered(gltrsv_plan *plan, const double *b, double *x, void *stream);

/* As gltrsv_plan_create, but with the schedule of an earlier analysis of
 * the same pattern (gltrsv_plan_schedule or gltrsv_schedule: core[n] and
 * superstep[n] per row, host arrays, caller-owned) instead of running the
 * scheduler: analysis results can be kept and reused across processes.  The
 * schedule is checked against Definition 2.1 (EINVAL with a description
 * otherwise); opts supply the triangle, packing and device settings. */
int gltrsv_plan_create_with_schedule(const gltrsv_csr *A, const gltrsv_plan_opts *opts, const int32_t *core,
                                     const int32_t *superstep, gltrsv_plan **out);

/* Device-side error word of the last persistent solve on this plan (0 = none,
 * 1 = spin limit hit).  Synchronises the plan's last stream. */
int gltrsv_plan_device_status(gltrsv_plan *plan, int32_t *status);

/* Watchdog of the plan's device-side waits (the persistent kernel's
 * superstep waits, the semi-asynchronous readiness waits): the number of
 * polls a wait may take before the solve gives up and sets the error word
 * that gltrsv_plan_device_status reports (default 5,000,000; measured on
 * MI355X a poll takes 0.14 us or more, so at least 0.7 s).  A small
 * value forces that path from the host, e.g. to test error handling: every
 * wave still leaves the kernel normally.  polls >= 1, else EINVAL. */
int gltrsv_plan_set_spin_limit(gltrsv_plan *plan, int64_t polls);

/* How long a workgroup of the persistent solve (gltrsv_solve, lane and
 * wavefront cores) waits for a superstep to complete before it robs the
 * workgroups of the launch that have not started yet: it marks them robbed
 * and claims and runs their chunks (or tasks) of that superstep, and a
 * robbed workgroup claims its own before running them once it starts.  So
 * the solve advances whenever any workgroup runs, and workgroups kept from
 * starting by other work on the device cannot stall it; with every
 * workgroup resident nothing is claimed.  Default 200 us; 0 robs at the
 * first wait.  The result is the same bits either way.  microseconds in
 * 0..2^40, else EINVAL. */
int gltrsv_plan_set_steal_wait(gltrsv_plan *plan, int64_t microseconds);

/* Diagnostic: every 7th workgroup (index 3 mod 7) of the persistent solve
 * (gltrsv_solve) and of the semi-asynchronous solves (gltrsv_solve_async,
 * gltrsv_solve_multi) waits `microseconds` before it starts, so the robbing
 * of workgroups that have not started runs without other work on the
 * device (for tests; 0 = off, the default).  The semi-asynchronous kernels
 * run a static order; a wave that has waited 200 us for values while a
 * workgroup of its launch has not started runs that workgroup's earliest
 * unrun chunk (or task) itself, then its own again (a chunk run twice stores
 * the same bits).  microseconds in 0..1e7, else EINVAL. */
int gltrsv_plan_set_start_delay(gltrsv_plan *plan, int64_t microseconds);

/* ---------------------------------------------------------------- batches */
/* Many independent systems in one persistent launch (the schedules compose:
 * systems share no data, so each advances through its own supersteps,
 * Sec. 3.1 and Def. 2.1).  Waves claim `per_claim` 64-task chunks at a time
 * from whichever system has an open superstep; the wave that completes a
 * superstep opens the next one.  No grid-wide barrier is used, so the launch
 * needs no co-residency. */
typedef struct gltrsv_batch gltrsv_batch;

typedef struct gltrsv_batch_opts {
    int32_t per_claim;     /* chunks claimed per atomic, >= 1                 */
    int32_t grid_blocks;   /* 0 = occupancy-sized grid                        */
    int32_t use_graph;     /* 1: the reset + solve kernels are captured once
                              into a hipGraph per stream and replayed         */
    int32_t async_exec;    /* 1: semi-asynchronous execution (as
                              gltrsv_solve_async): no superstep barriers;
                              chunks of each system claimed in order, at most
                              four supersteps of average width ahead of the
                              completed ones; x filled with the
                              not-yet-computed mark first, so b[i] must not
                              alias x[i] (EINVAL).  If every plan was created
                              with core_width = 64 the systems run on
                              wavefront cores: their tasks in one global
                              order (supersteps of all systems by relative
                              depth s / S, each system's order kept), wave w
                              taking every W-th; a wave that waits long while
                              a workgroup of the launch has not started runs
                              that workgroup's earliest task in its place, so
                              no co-residency is needed; per_claim is then
                              unused                                          */
} gltrsv_batch_opts;

void gltrsv_default_batch_opts(gltrsv_batch_opts *opts);

/* Binds `count` plans (library-owned, created on the current device; they
 * must outlive the batch).  Plans with n = 0 are skipped. */
int gltrsv_batch_create(gltrsv_plan *const *plans, int32_t count, const gltrsv_batch_opts *opts,
                        gltrsv_batch **out);

/* Solves system i with b[i] -> x[i] (host arrays of `count` device pointers,
 * original numbering, b[i] may alias x[i]), asynchronously on `stream`.  Calls
 * on one batch must not overlap (they share its device state). */
int gltrsv_batch_solve(gltrsv_batch *batch, const double *const *b, double *const *x, void *stream);

/* 0, or 1 if a wave went without work longer than the idle limit (~10 s).
 * Synchronises the last stream. */
int gltrsv_batch_status(gltrsv_batch *batch, int32_t *status);

int gltrsv_batch_info(const gltrsv_batch *batch, int32_t *systems, int32_t *grid_blocks);

int gltrsv_batch_destroy(gltrsv_batch *batch);

/* One-shot form: create, solve, synchronise `stream`, destroy. */
int gltrsv_solve_batched(gltrsv_plan *const *plans, const double *const *b, double *const *x, int32_t count,
                         void *stream);

/* gltrsv_solve_batched for callers that cannot allocate (code that must not
 * call hipMalloc, serving loops that allocate nothing per request): the same
 * kernels, launch configuration and results, with the batch's device state
 * (system descriptors, superstep state words, per-superstep done counters,
 * finished and error words) in a fixed device array that the library holds
 * for each GPU it runs on until the process ends, instead of buffers it
 * allocates per call.  The call allocates no memory on the device or the
 * host (no hipMalloc, hipFree or hipHostMalloc).  Limits: at most 1,024
 * systems with n > 0 and at most 4 MiB of state (256 bytes per system plus
 * 4 bytes per superstep of every system, about 9.4e5 supersteps in all);
 * a larger batch returns GLTRSV_ERANGE.  Arguments, vector rules (b[i] may
 * equal x[i]; no other overlap), synchronisation of `stream` and error codes
 * as gltrsv_solve_batched.  All calls on one GPU share that GPU's array:
 * calls from several host threads of a process are serialised by the
 * library (each holds the array until its solve has finished); the array
 * keeps the last call's contents, which the next call clears on the device
 * before use. */
int gltrsv_solve_batched_noalloc(gltrsv_plan *const *plans, const double *const *b, double *const *x,
                                 int32_t count, void *stream);

/* ---------------------------------------------------------------- serving */
/* Continuous batching of solve requests against resident plans.  A worker
 * thread owned by the server runs the batched kernel in time quanta; every
 * admitted request advances through its supersteps in whichever quanta it
 * is on the device, and requests submitted meanwhile join at the next
 * quantum.  Results are bit-identical to gltrsv_solve (same per-row
 * operations), alone or in any mix. */
typedef struct gltrsv_server gltrsv_server;

typedef struct gltrsv_server_opts {
    int64_t budget_bytes;   /* in-flight budget: 16 n + 4 S + 64 bytes per
                               request (its b and x plus its counters)        */
    int32_t max_slots;      /* requests on the device at once                 */
    int32_t per_claim;      /* chunks claimed per atomic                      */
    double quantum_us;      /* device time per launch before new admissions   */
    int32_t counter_words;  /* capacity of the per-superstep counter arena    */
    int32_t grid_blocks;    /* 0 = occupancy-sized grid                       */
    int32_t async_exec;     /* 1: semi-asynchronous execution (see
                               gltrsv_batch_opts.async_exec); a request's b
                               must then not alias its x (EINVAL at submit)   */
} gltrsv_server_opts;

typedef struct gltrsv_server_stats {
    int64_t submitted, completed, failed, launches, rows_completed, queued, inflight_bytes;
    int64_t cancelled;
} gltrsv_server_stats;

void gltrsv_default_server_opts(gltrsv_server_opts *opts);

/* Creates a server on the current device and starts its worker thread. */
int gltrsv_server_create(const gltrsv_server_opts *opts, gltrsv_server **out);

/* Queues the solve b -> x with `plan` (device pointers, original numbering;
 * b must be fully written before the call and b, x and the plan must stay
 * valid until gltrsv_server_poll has reported the ticket or
 * gltrsv_server_cancel has returned for it; the server reads nothing of the
 * plan after that).  Returns GLTRSV_EAGAIN when the request
 * would exceed the in-flight budget (retry after completions), ERANGE if it
 * can never fit.  Thread-safe. */
int gltrsv_server_submit(gltrsv_server *server, gltrsv_plan *plan, const double *b, double *x, uint64_t *ticket);

/* Moves up to `max` completed tickets (and, if done_ns is not NULL, the
 * gltrsv_clock_ns time at which the server saw each complete) to the caller;
 * *ndone receives the count.  A completed ticket's x is final and visible to
 * any later stream work.  Thread-safe. */
int gltrsv_server_poll(gltrsv_server *server, uint64_t *tickets, int64_t *done_ns, int32_t max, int32_t *ndone);

int gltrsv_server_get_stats(gltrsv_server *server, gltrsv_server_stats *out);

/* Withdraws a request that has not completed.  A queued request is removed
 * at once; for one already on the device the call blocks until the worker
 * has dropped it at the next quantum boundary (the worker stops scheduling
 * its chunks; chunks already claimed finish first).  Either way, when the
 * call returns the device no longer touches the request's b, x or plan (the
 * caller may free them), the ticket is never reported by gltrsv_server_poll,
 * its budget is released, and its x is left partly written (undefined).
 * GLTRSV_ENOENT if no pending request has this ticket (unknown, completed or
 * cancelled).  Thread-safe; must not be called from a thread that the
 * server's progress depends on. */
int gltrsv_server_cancel(gltrsv_server *server, uint64_t ticket);

/* Monotonic host clock used for completion times, in nanoseconds. */
int64_t gltrsv_clock_ns(void);

/* Waits until every accepted request has completed, then frees the server. */
int gltrsv_server_destroy(gltrsv_server *server);

/* Semi-asynchronous solve (the paper's future-work direction, Sec. 8): the
 * same schedule, stream and per-row arithmetic as gltrsv_solve (so the same
 * bits), with the barriers replaced by per-row readiness.  x is first filled
 * with a signalling-NaN mark that no computed value can equal (every x_i is
 * the result of a division); a lane that gathers the mark reads again until
 * the value is there.  Waves run the chunks in schedule order, so the solve
 * always progresses.  b and x: device, n values each, original numbering;
 * b == x (in place) is allowed and uses a plan-owned copy of b (allocated on
 * the first such call); b and x must otherwise not overlap.  Asynchronous on
 * `stream`; a wait that exceeds the spin limit is reported by
 * gltrsv_plan_device_status (GLTRSV_ETIMEDOUT). */
int gltrsv_solve_async(gltrsv_plan *plan, const double *b, double *x, void *stream);

/* Several right-hand sides (SpTRSM): solves A X = B for nrhs columns, B and X
 * row-major n x nrhs (element (i, r) at [i * nrhs + r]), device memory,
 * original numbering, not overlapping (EINVAL).  Column r of X is bit-for-bit
 * the gltrsv_solve result for column r of B.  Semi-asynchronous (as
 * gltrsv_solve_async); each launch walks the stream once for up to 4
 * columns, so the matrix bytes and the gathers' memory requests are shared
 * by those columns.  Asynchronous on `stream`; errors are reported by
 * gltrsv_plan_device_status. */
int gltrsv_solve_multi(gltrsv_plan *plan, const double *b, double *x, int32_t nrhs, void *stream);

/* One-workgroup solve, for plans created with opts.exec_hint = 2: the BSP
 * machine of Definition 2.1 is one wavefront of one workgroup, lane c being
 * core c (k <= 64), and the wave's program order is the barrier between
 * supersteps (a value one lane writes to LDS is seen by every later LDS read
 * of the wave), so a superstep costs no device-wide synchronisation at all.
 * Every lane's rows of a superstep run in the order of Sec. 5, in groups of
 * four stream entries (a row starts a new group: b_i and the diagonal, then
 * the off-diagonals in stored order as a running subtraction, Eq. (2.1), and
 * the division where the row ends); a superstep takes as many groups as its
 * busiest lane.  The results of the last 128 groups stay in LDS; older
 * operands, b and the copy of every result to x are handled by a second wave
 * that streams the plan's records through an LDS FIFO.  One launch of one
 * 128-thread workgroup with about 160 KB of LDS.  For the narrow,
 * dependency-bound systems where the device-wide forms wait on memory round
 * trips between waves.  Same arguments and the same bits as gltrsv_solve (b
 * may alias x); GLTRSV_ENOTSUP for a plan without the layout.  Errors are
 * reported by gltrsv_plan_device_status. */
int gltrsv_solve_local(gltrsv_plan *plan, const double *b, double *x, void *stream);

/* Copies a plan's one-workgroup layout to host memory for inspection:
 * rec (rec_bytes bytes) receives the records one after another, info
 * (records x 4 uint32: bytes copied, FIFO byte offset, records that must be
 * computed before the copy, 0) the per-record copy data.  rec_bytes and
 * records must equal the layout's (see gltrsv_plan_local_size), else
 * EINVAL; ENOTSUP without a layout.  Record format: a 32-byte header
 * (uint32 groups, fills, drains, records drained before compute,
 * FIFO offset of the next record, records drained before the fills, 0, 0);
 * per group 64 lanes x 4 doubles as [2][64][2] (entries 2h, 2h+1 of lane l
 * at byte 1024 h + 16 l) and 64 lanes x 4 uint16 LDS slots (bit 15: row
 * header on entry 0, row end on entry 1); fills {uint32 slot | bit 31 for
 * x, int32 row} (slot <- b[row] or x[row]); drains {uint32 slot, int32 row}
 * (x[row] <- slot once computed).  LDS slots (8 bytes each, in blocks of
 * 64): 0..8191 the ring (the row ending in group g on lane c at
 * (g mod 128) * 64 + c), 8192 holds +0.0, the FIFO of 96,768 bytes from
 * slot 8256; records start at multiples of 512 FIFO bytes and their fill
 * i goes to the i-th slot after the copied bytes, rounded up to 512.
 * Synchronous. */
int gltrsv_plan_local_size(const gltrsv_plan *plan, int64_t *rec_bytes, int64_t *records);
/* The same layout built on the host from a schedule (core[n] < 64 and
 * superstep[n] per row, host arrays, checked against Definition 2.1) in the
 * order of Sec. 5, without a plan or a device: with rec or info NULL it
 * stores the sizes in *rec_bytes and *records; otherwise those must hold
 * them and rec/info receive the layout.  triangle: GLTRSV_LOWER or
 * GLTRSV_UPPER (as opts.triangle).  Host only. */
int gltrsv_local_layout(const gltrsv_csr *A, int32_t triangle, const int32_t *core, const int32_t *superstep,
                        void *rec, int64_t *rec_bytes, uint32_t *info, int64_t *records);

/* The per-wave record streams that the semi-asynchronous solve of a
 * wave-core plan (opts.core_width = 64) reads, built on the host from a
 * schedule (core[n] and superstep[n] per row, host arrays, checked against
 * Definition 2.1) for `waves` waves (1 .. 4 x 2048; a plan uses 4 x its
 * grid), without a plan or a device.  Tasks are the runs of one core in a
 * superstep, numbered superstep by superstep in the order of Sec. 5 with
 * each superstep's tasks longest first; wave v runs tasks v, v + waves,
 * ...  Its stream, [sbeg[v], sbeg[v + 1] - 1) of scol/sval followed by one
 * 0xFFFFFFFF word, holds those tasks' rows one after another as records: a
 * header (scol = 0x80000000 | row, with 0x40000000 also set on a task's
 * first row; sval = the diagonal) and the row's off-diagonals in stored
 * order (scol = the column, or 0x40000000 | d for the row d positions
 * earlier in the same task when d < 64; sval = A_ij).  Task t's header is
 * at stask[t].  The arrays end with 0xFFFFFFFF slots (value 0) that the
 * kernel reads past a stream's end.  With any of scol, sval, sbeg, stask
 * NULL it stores the sizes in *slots (scol/sval slots, padding included)
 * and *tasks; otherwise those must hold them, sbeg has waves + 1 entries,
 * and the arrays receive the streams.  triangle: GLTRSV_LOWER or
 * GLTRSV_UPPER (as opts.triangle; rows and columns are the matrix's own).
 * Host only. */
int gltrsv_wave_streams(const gltrsv_csr *A, int32_t triangle, const int32_t *core, const int32_t *superstep,
                        int64_t waves, uint32_t *scol, double *sval, int64_t *sbeg, int64_t *stask, int64_t *slots,
                        int64_t *tasks);
int gltrsv_plan_local_records(const gltrsv_plan *plan, void *rec, int64_t rec_bytes, uint32_t *info, int64_t records);

/* ------------------------------------------------------- execution forms */
/* The single-system forms give the same bits; which is fastest depends on
 * the matrix and its schedule (many short supersteps favour the
 * semi-asynchronous form, a few wide ones the persistent form, a narrow
 * system with a k <= 64 schedule the one-workgroup form). */
#define GLTRSV_EXEC_PERSISTENT 0   /* gltrsv_solve       */
#define GLTRSV_EXEC_PLAIN      1   /* gltrsv_solve_plain */
#define GLTRSV_EXEC_ASYNC      2   /* gltrsv_solve_async */
#define GLTRSV_EXEC_LOCAL      3   /* gltrsv_solve_local (plans with exec_hint 2) */
#define GLTRSV_EXEC_FORMS      4

/* Solves with the plan's preferred form: the one given to
 * gltrsv_plan_set_exec or found by gltrsv_plan_tune, initially the form that
 * opts.exec_hint names (persistent, semi-asynchronous or one workgroup).
 * Arguments as for gltrsv_solve (b may alias x). */
int gltrsv_solve_auto(gltrsv_plan *plan, const double *b, double *x, void *stream);

/* Sets the preferred form (GLTRSV_EXEC_*, else EINVAL; LOCAL only for a
 * plan with that layout, else ENOTSUP), e.g. from a stored tuning result. */
int gltrsv_plan_set_exec(gltrsv_plan *plan, int32_t form);

/* Times the plan's forms and makes the fastest the preferred one (an
 * autotuner; the cost-model choice of opts.exec_hint is a prediction, this
 * is a measurement).  Each form solves b -> x once untimed, then `reps`
 * times (>= 1) between two HIP events on `stream`.  b and x: device, n
 * values each, caller-owned, not overlapping (EINVAL); x ends holding the
 * solution.  us_out (host, GLTRSV_EXEC_FORMS doubles, may be NULL) receives
 * the mean microseconds per solve in GLTRSV_EXEC_* order (-1 for the
 * one-workgroup form of a plan without its layout), *best (may be NULL) the
 * chosen form.  Synchronises `stream`.  If a device-side wait ran out
 * during the measurement the preference is left unchanged and the call
 * returns GLTRSV_ETIMEDOUT. */
int gltrsv_plan_tune(gltrsv_plan *plan, const double *b, double *x, int32_t reps, void *stream, double *us_out,
                     int32_t *best);

/* Plain device-to-device copy of `bytes` (a multiple of 16) from src to dst
 * (device pointers, caller-owned, non-overlapping), asynchronous on `stream`.
 * The achievable-bandwidth reference for the solve kernels and the
 * calibration kernel for memory-traffic counters. */
int gltrsv_copy_probe(const void *src, void *dst, int64_t bytes, void *stream);

/* The solve's memory traffic with its dependencies taken out: streams the
 * plan's packed entries once and gathers x (device, n values, original
 * numbering) at every column one solve reads from memory, with no barrier
 * and no row waiting for another; a measured floor for gltrsv_solve on the
 * same plan.  Writes y[i] (device, n values) = the running sum in stored
 * order of A_ij * x_j over the off-diagonals of row i, where 1.0 stands in
 * for x_j at the entries the solve keeps on chip (columns among the last
 * 16 rows of the same (superstep, core) task); with x = ones, y[i] is
 * exactly the left-to-right sum of row i's off-diagonals.  Rows without
 * off-diagonals get 0.  Asynchronous on `stream`. */
int gltrsv_plan_gather_probe(gltrsv_plan *plan, const double *x, double *y, void *stream);

/* Copies the plan's packed stream to host memory: word[slots] (uint32)
 * and value[slots] (double), slots = gltrsv_plan_info.stream_slots (any
 * other count is EINVAL).  Entry t of lane l of chunk c is at
 * chunk_base[c] + 64 t + l.  Word encoding: bit 31 set = row header (bits
 * 0..29 = original row, value = the diagonal), 0xFFFFFFFF = padding, bit 30
 * set = a column of the same task that many rows back (< 16), otherwise the
 * column itself.  Synchronous. */
int gltrsv_plan_stream(const gltrsv_plan *plan, uint32_t *word, double *value, int64_t slots);

/* Diagnostics of builds compiled with GLTRSV_TRACE (otherwise returns
 * GLTRSV_ENOTSUP): copies up to `count` int64 wall-clock stamps of the last
 * persistent solve, laid out [superstep][workgroup][3] = start of work, end
 * of work, end of the barrier.  Synchronises the plan's last stream. */
int gltrsv_debug_trace(gltrsv_plan *plan, int64_t *out, int64_t count);

#ifdef __cplusplus
}
#endif
#endif /* GLTRSV_H */
