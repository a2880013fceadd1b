/*
 * sptrsv.h -- C ABI of libsptrsv, sparse triangular solves on MI355X (gfx950).
 *
 * Method: R. Li, "On Parallel Solution of Sparse Triangular Linear Systems in
 * CUDA" (arXiv:1710.04985).  The library solves  T x = b  with T a sparse
 * lower or upper triangle in CSR form (Sec. 3, eq. (1)), after a setup
 * ("analysis") phase that computes the level sets of the dependency DAG
 * (Sec. 4.1, Sec. 4.4), on the host or on the device.  Solve schedules:
 *   - level-scheduled (Sec. 4.1, Algorithm LEVR): one kernel launch per level;
 *   - self-scheduled (Sec. 4.2, Algorithm SLFR): one persistent launch whose
 *     waves take rows in level order and wait on per-row readiness instead of
 *     a global synchronisation between levels;
 *   - block: level by level inside one workgroup per independent system;
 *   - column-wise (Sec. 3.2; Algorithms LEVC and SLFC): finished unknowns
 *     push their updates into the rows that depend on them.
 * Transposed solves, several right-hand sides, batches of independent
 * triangles, the gradient with respect to the values, HIP graph capture and
 * an autotuner complete the interface.
 *
 * Conventions shared by every entry point
 *   - Indices are int32, 0-based.  The diagonal is stored INSIDE each row
 *     (the paper keeps it in a separate vector d); its position in the row is
 *     free.  Columns need not be sorted.
 *   - Matrix arrays (row_ptr, col_idx, vals) and vectors (b, x, B, X, ...)
 *     are DEVICE pointers owned by the caller.  row_ptr and col_idx are read
 *     during analysis only.  vals is gathered into the handle's own level-
 *     ordered copy during analysis and by sptrsv_update_values; the solves
 *     never read the caller's vals, so the caller must call
 *     sptrsv_update_values after changing them.
 *   - Every function returns an int status: SPTRSV_OK (0) or a negative
 *     sptrsv_status.  Handles are opaque and owned by the library until
 *     sptrsv_destroy.
 *   - Solves are asynchronous on the given HIP stream (NULL = default stream).
 *     The first solve with a given schedule builds and uploads its work
 *     tables (chunks, per-wavefront lists; for the column-wise solves the
 *     push lists and their scratch; for T^T its analysis) with synchronous
 *     copies; later solves with that schedule perform no allocation, host
 *     synchronisation or memset, so they can be captured in a HIP graph.
 *     sptrsv_graph_capture prepares all of this itself.  The calls of one
 *     handle that use its scratch (ticket, status, flags, epoch, the
 *     position-ordered solution, accumulators, gathered values: solves,
 *     value updates, tuning) are serialized across streams: the library
 *     records an event after each, and a call issued on a different stream
 *     than the previous one first makes its stream wait for that event.
 *     Under graph capture nothing is recorded or waited for: the capturing
 *     stream orders the graph, and the caller orders graph launches against
 *     other work on the handle.
 *   - n = 0 is valid and every solve on it is a no-op.
 *   - Dependencies are taken from the pattern (Sec. 4.4): an explicitly
 *     stored zero off-diagonal still counts as a dependency.
 */
#ifndef SPTRSV_H_
#define SPTRSV_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sptrsv_handle_s *sptrsv_handle_t;
typedef struct sptrsv_graph_s *sptrsv_graph_t;

typedef enum {
    SPTRSV_OK = 0,
    SPTRSV_ERR_INVALID_ARG = -1,    /* null pointer, n < 0, bad enum, bad option */
    SPTRSV_ERR_BAD_ROWPTR = -2,     /* row_ptr[0] != 0, row_ptr[n] != nnz, or decreasing */
    SPTRSV_ERR_BAD_COLIDX = -3,     /* column index outside [0, n) */
    SPTRSV_ERR_NOT_TRIANGULAR = -4, /* entry on the wrong side of the diagonal */
    SPTRSV_ERR_DUPLICATE = -5,      /* a column appears twice in one row */
    SPTRSV_ERR_MISSING_DIAG = -6,   /* no stored diagonal (and unit_diag == 0) */
    SPTRSV_ERR_ZERO_PIVOT = -7,     /* stored diagonal exactly 0.0 (and unit_diag == 0) */
    SPTRSV_ERR_HIP = -8,            /* a HIP runtime call failed */
    SPTRSV_ERR_OOM = -9,            /* device or host allocation failed */
    SPTRSV_ERR_TIMEOUT = -10,       /* self-scheduled wait exceeded its spin limit */
    SPTRSV_ERR_NOT_SUPPORTED = -11, /* valid request the library does not implement */
    SPTRSV_ERR_BUSY = -12,          /* sptrsv_destroy: graphs captured from the handle are
                                       still alive (destroy them first) */
    SPTRSV_ERR_TOO_LARGE = -13,     /* sptrsv_solve_noalloc: the schedule needs more than
                                       SPTRSV_NOALLOC_SCRATCH_BYTES of scratch */
    SPTRSV_ERR_NOT_RESIDENT = -14   /* a static schedule found its persistent grid not all
                                       resident (other work held the GPU): it drained without
                                       a result; the ticket schedule (ASSIGN_TICKET) needs no
                                       residency */
} sptrsv_status;

typedef enum { SPTRSV_F64 = 0, SPTRSV_F32 = 1 } sptrsv_dtype;
typedef enum { SPTRSV_LOWER = 0, SPTRSV_UPPER = 1 } sptrsv_uplo;

typedef enum {
    SPTRSV_ALGO_AUTO = 0,   /* sptrsv_tune's timed choice, or before any tuning a rule on
                               features of the pattern (deterministic, no trials): the
                               block schedule with the whole system in LDS for one
                               system with one lane per row, at most 64 rows per level
                               and small enough for LDS; else self-scheduled.  For the
                               self-scheduled solve (also when chosen explicitly),
                               options left unset follow the pattern too: the ticket
                               schedule when levels average at most 4,096 rows, no row
                               exceeds 64 entries and no slot width was set, else the
                               XCD-regional static one; two wavefronts per CU for rows
                               of more than 64 entries or levels averaging more than
                               8,192 rows; 32-byte slots for rows of more than 64
                               entries.  No rule changes the result bits. */
    SPTRSV_ALGO_LEVEL = 1,  /* level-scheduled: one launch per level (Sec. 4.1) */
    SPTRSV_ALGO_SELF = 2,   /* self-scheduled: one persistent launch (Sec. 4.2) */
    SPTRSV_ALGO_BLOCK = 3,  /* level-scheduled inside one workgroup per independent
                               system (each system of a batched handle; the whole
                               triangle otherwise): the level barrier is a workgroup
                               barrier, not a launch; a system's whole level-ordered
                               copy, or else its x, is kept in LDS when the largest system
                               fits (SPTRSV_OPT_BLOCK_RESIDENT).  One right-hand side
                               (several: the level-scheduled solve is used). */
    SPTRSV_ALGO_COLUMN_LEVEL = 4, /* column-wise, level-scheduled (Sec. 3.2 sweep, Sec. 4.1
                               LEVC): one launch per level; each finished x_k is pushed
                               into the accumulators of the rows depending on it with
                               agent-scope atomic adds */
    SPTRSV_ALGO_COLUMN_SELF = 5   /* column-wise, self-scheduled (Sec. 4.2 SLFC): one
                               persistent launch; a row starts once its arrival counter
                               reaches its dependency count.  Both column forms add
                               updates in an order fixed by timing: results agree with
                               the row-wise solves to rounding, not bit for bit.  One
                               right-hand side (several: the row-wise self-scheduled
                               solve is used).  Never chosen by ALGO_AUTO. */
} sptrsv_algo;

typedef enum {
    SPTRSV_SYNC_VALUE = 0,  /* self-scheduled readiness carried by x itself: x is
                               pre-filled with a signalling-NaN sentinel and each
                               x_i is published by one agent-scope atomic store */
    SPTRSV_SYNC_FLAG = 1    /* per-row ready flags stamped with a per-solve epoch,
                               agent-scope release/acquire (Sec. 4.2 counters,
                               without the per-solve reset) */
} sptrsv_sync;

typedef enum {
    SPTRSV_OPT_ALGO = 0,          /* sptrsv_algo */
    SPTRSV_OPT_GROUP = 1,         /* lanes per row G in {1,2,4,...,64}; 0 = by row length */
    SPTRSV_OPT_ENTRIES_PER_LANE = 2, /* target entries per lane when GROUP = 0 (default 4) */
    SPTRSV_OPT_SYNC = 3,          /* sptrsv_sync (self-scheduled only) */
    SPTRSV_OPT_SPIN_LIMIT = 4,    /* max polls of one dependency before TIMEOUT (>= 1) */
    SPTRSV_OPT_GRID = 5,          /* persistent workgroups; 0 = one wavefront per CU (if
                                     unset, see SPTRSV_ALGO_AUTO) */
    SPTRSV_OPT_TIMING = 6,        /* 1 = record HIP events around the main solve kernel */
    SPTRSV_OPT_WG = 7,            /* threads per workgroup for the row kernels (64..256,
                                     default 64) */
    SPTRSV_OPT_ROWS_PER_LANE = 8, /* rows one lane owns when a row gets one lane (1..4,
                                     default 1): fewer, larger work chunks */
    SPTRSV_OPT_ASSIGN = 9,        /* sptrsv_assign: how self-scheduled wavefronts get chunks
                                     (if unset, by the pattern: see SPTRSV_ALGO_AUTO) */
    SPTRSV_OPT_POLL = 10,         /* how a waiting lane polls its dependencies (value sync):
                                     1 (default) = two rounds in flight over all of its
                                     slots, so a value is seen soon after it lands; 0 = one
                                     round at a time over the pending slots only (less
                                     polling traffic, better when most dependencies are
                                     already available) */
    SPTRSV_OPT_XP_STRIDE = 11,    /* 1 (default; if unset, by the pattern: see
                                     SPTRSV_ALGO_AUTO), 2, 4, 8 or 16: elements between
                                     consecutive values of the position-ordered solution
                                     the self-scheduled static schedules (one right-hand
                                     side) publish and poll.  Wider slots put fewer values on a
                                     cache line under concurrent stores and polls: faster
                                     where dependencies are scattered, slower where polls
                                     coalesce.  The autotuner tries packed values and 32- and
                                     64-byte slots.  Ignored by the other schedules */
    SPTRSV_OPT_MULTI_ROWS = 12,   /* several right-hand sides, static schedules: rows each
                                     group of a row's lanes owns in a chunk (1, 2 or 4; 0 =
                                     default, 1: the fastest on every pattern and column
                                     count measured).  A wavefront issues the gathers of all
                                     its rows before it waits on any.  Results do not depend
                                     on it */
    SPTRSV_OPT_RESIDENCY_LIMIT = 13, /* polls a wavefront of a static (persistent-grid)
                                     schedule waits at its start for the rest of the grid to
                                     sign in (default 2^20); the grid gives up with
                                     SPTRSV_ERR_NOT_RESIDENT if it never fills.  0 makes every
                                     wavefront but the last to arrive give up at once (a test
                                     hook that forces the failure) */
    SPTRSV_OPT_BLOCK_RESIDENT = 14, /* SPTRSV_ALGO_BLOCK: 1 (default) keeps each system's whole
                                     level-ordered copy (b/x, 1/diagonal, off-diagonal values,
                                     16-bit local indices) in LDS when every system fits (at
                                     most 65,535 rows and off-diagonals per system and the
                                     device's per-workgroup LDS), so its levels touch no global
                                     memory; 0 keeps only x there and streams the row data.
                                     Same results either way */
    SPTRSV_OPT_COOPERATIVE = 15   /* how the persistent grids of the static schedules (and of
                                     ALGO_COLUMN_SELF) are launched: 0 (default) = an
                                     ordinary launch; the grid is at most half of what the
                                     occupancy figure allows, so it is resident as soon as the
                                     GPU has room, and its wavefronts check that at their start
                                     (SPTRSV_OPT_RESIDENCY_LIMIT); 1 = a cooperative launch,
                                     whose co-residency guarantee costs about 16 us per solve
                                     (measured on MI355X).  Same results either way */
} sptrsv_option;

typedef enum {
    SPTRSV_ASSIGN_STATIC = 0,     /* chunk c goes to wavefront c mod W of an all-resident
                                     persistent grid (SPTRSV_OPT_COOPERATIVE), pipelined
                                     four chunks deep; value sync, one or several right-hand
                                     sides.  The launch is captured by sptrsv_graph_capture
                                     (which prepares the per-wavefront chunk lists); under a
                                     capture the caller opens itself, the ticket form is used
                                     unless those lists already exist.  A grid that other work
                                     keeps from becoming resident drains with
                                     SPTRSV_ERR_NOT_RESIDENT. */
    SPTRSV_ASSIGN_TICKET = 1,     /* wavefronts claim chunks from an atomic ticket: needs no
                                     co-residency, costs one serialised atomic per chunk */
    SPTRSV_ASSIGN_XCD = 2         /* as STATIC, but each level's chunks are cut into 8
                                     contiguous regions, region r going to the wavefronts of
                                     workgroups r, r+8, ... (dispatched to one XCD), so that
                                     most dependencies are produced under the same L2; needs
                                     a grid that is a multiple of 8 workgroups (else as
                                     STATIC) */
} sptrsv_assign;

/* ---------------------------------------------------------------------- */
/* Analysis (setup phase, Sec. 4.4): validates the triangle, computes the
 * levels lev(i) = 1 + max lev(j) over stored off-diagonals j of row i
 * (0-based: rows without dependencies are level 0), the level sets
 * (jlev = rows ordered by (level, row), ilev = level pointers) and the
 * dependency counts, and builds the level-ordered device copy of the
 * matrix the kernels stream.
 *   n, nnz     matrix order and stored entries (diagonal included)
 *   row_ptr    device int32[n+1];  col_idx device int32[nnz]
 *   vals       device double[nnz] (F64) or float[nnz] (F32)
 *   uplo       SPTRSV_LOWER: forward substitution; SPTRSV_UPPER: backward
 *   unit_diag  nonzero: the diagonal is 1, stored diagonal entries ignored
 *              (and may be absent)
 *   stream     stream for the device copies; the call synchronises it
 *   out        receives the new handle (NULL on failure)
 * Errors: INVALID_ARG, BAD_ROWPTR, BAD_COLIDX, NOT_TRIANGULAR, DUPLICATE,
 * MISSING_DIAG, ZERO_PIVOT, HIP, OOM.  Blocking: copies the pattern to the
 * host, computes there, uploads the result (the host route of
 * sptrsv_analyze_ex).  row_ptr / col_idx / vals may be freed afterwards. */
int sptrsv_analyze(int32_t n, int32_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                   const void *vals, sptrsv_dtype dtype, sptrsv_uplo uplo, int unit_diag,
                   hipStream_t stream, sptrsv_handle_t *out);

/* Where the setup phase runs (Table 1 compares the two routes). */
typedef enum {
    SPTRSV_SETUP_HOST = 0,    /* pattern copied to the host, analysed there, plan uploaded */
    SPTRSV_SETUP_DEVICE = 1   /* analysed in device memory: validity check and dependency
                                 counts, a sync-free max-plus sweep for the levels (the
                                 self-scheduled solve of Sec. 4.2 with max(level)+1 in
                                 place of the dot product), stable radix sorts for jlev and
                                 the level-ordered layout; only nlev, ilev and the row
                                 pointers of that layout come to the host */
} sptrsv_setup;

/* sptrsv_analyze with a choice of route.  Results (levels, jlev, ilev,
 * depcnt, the plan, every solve) are identical for both routes.  The device
 * route handles patterns whose rows hold strictly increasing columns; any
 * other pattern, and every invalid one, goes through the host route, which
 * also names the validation error.  The device route keeps a device copy of
 * the pattern and downloads it, with the plan, the first time something
 * needs them on the host (the block plan, export, sptrsv_tune); the analysis
 * of T^T stays on the device.  Errors as for sptrsv_analyze, plus INVALID_ARG for an
 * unknown route and TIMEOUT (level sweep; cannot happen on a valid
 * triangle).  Blocking. */
int sptrsv_analyze_ex(int32_t n, int32_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                      const void *vals, sptrsv_dtype dtype, sptrsv_uplo uplo, int unit_diag,
                      int setup, hipStream_t stream, sptrsv_handle_t *out);

/* Route the handle's analysis took (sptrsv_setup) and its wall time in
 * milliseconds (host clock around the whole analysis call).  Either
 * pointer may be NULL. */
int sptrsv_get_setup(sptrsv_handle_t h, int32_t *route, double *ms);

/* Batched analysis of `count` independent triangles of one dtype/uplo, solved
 * together as their block-diagonal concatenation (rows and columns of system
 * s offset by the sizes of systems 0..s-1).  n, nnz: host int32[count];
 * row_ptr, col_idx, vals: host arrays of device pointers, one per system.
 * The solves take b and x as the concatenation of the systems' vectors.
 * The concatenation shares one level structure, so one launch serves all
 * systems (levels of different systems interleave).  Errors as for
 * sptrsv_analyze, reported for the first failing system. */
int sptrsv_analyze_batched(int32_t count, const int32_t *n, const int32_t *nnz,
                           const int32_t *const *row_ptr, const int32_t *const *col_idx,
                           const void *const *vals, sptrsv_dtype dtype, sptrsv_uplo uplo,
                           int unit_diag, hipStream_t stream, sptrsv_handle_t *out);

/* sptrsv_analyze_batched with a choice of route (sptrsv_setup).  The device
 * route concatenates the systems in device memory and analyses the
 * concatenation there (only nlev, ilev and row pointers come to the host);
 * a system whose pattern it does not take, and every invalid one, goes
 * through the host route, which names the error.  Same plan, bit for bit,
 * on both routes. */
int sptrsv_analyze_batched_ex(int32_t count, const int32_t *n, const int32_t *nnz,
                              const int32_t *const *row_ptr, const int32_t *const *col_idx,
                              const void *const *vals, sptrsv_dtype dtype, sptrsv_uplo uplo,
                              int unit_diag, int setup, hipStream_t stream, sptrsv_handle_t *out);

/* Re-gather new values for the same pattern (the caller's vals, device).
 * Asynchronous on `stream`; a zero pivot is reported through
 * sptrsv_get_status after the stream has been synchronised. */
int sptrsv_update_values(sptrsv_handle_t h, const void *vals, hipStream_t stream);

/* Batched form: vals is a host array of `count` device pointers. */
int sptrsv_update_values_batched(sptrsv_handle_t h, const void *const *vals, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Solve T x = b (forward for lower, backward for upper; Sec. 3).
 * b, x: device vectors of n elements of the handle's dtype.  b == x (in
 * place) is allowed; partial overlap is not.  Asynchronous. */
int sptrsv_solve(sptrsv_handle_t h, const void *b, void *x, hipStream_t stream);

/* sptrsv_solve for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same schedule, kernels and result (bit for bit) as sptrsv_solve, but the
 * position-ordered solution the kernels publish and poll lives in a
 * library-owned static device array of SPTRSV_NOALLOC_SCRATCH_BYTES (64
 * MiB) per GPU, held until the process ends, instead of the handle's
 * buffer, and the call allocates nothing (no hipMalloc, hipFree, event or
 * library allocation).  Needs n * slot stride * value bytes <= 64 MiB
 * (FP64 packed: up to 8,388,608 rows), else SPTRSV_ERR_TOO_LARGE.  The work
 * tables of the handle's current schedule must already exist: the analysis
 * builds those of the default schedule and sptrsv_tune those of its choice
 * (as does any earlier sptrsv_solve or graph capture with that schedule);
 * otherwise SPTRSV_ERR_NOT_SUPPORTED, as for column-wise schedules not yet
 * prepared.  One exception: a static self-scheduled schedule whose
 * per-wavefront lists do not exist yet runs as the ticket schedule, whose
 * result bits are the same (and which ignores SPTRSV_OPT_XP_STRIDE).  The
 * current device must be the handle's (else INVALID_ARG).
 * All calls on one GPU share the array, which keeps the last call's
 * contents (each solve reinitialises what it reads): calls that overlap in
 * time on one GPU race; order them on one stream.  Asynchronous. */
#define SPTRSV_NOALLOC_SCRATCH_BYTES (64u << 20)
int sptrsv_solve_noalloc(sptrsv_handle_t h, const void *b, void *x, hipStream_t stream);

/* Solve T^T x = b.  Uses the analysis of T^T (the column-wise view of
 * Sec. 3.2: rows of T^T are the columns of T, levels from the reversed
 * sweep); built on first use, which then blocks, or in advance by
 * sptrsv_prepare_transpose.  A handle analysed on the device route builds it
 * on the device as well (the transposed pattern by a stable radix sort of
 * the entries by column, then the same device analysis). */
int sptrsv_solve_transpose(sptrsv_handle_t h, const void *b, void *x, hipStream_t stream);

/* Build the analysis of T^T now (blocking). */
int sptrsv_prepare_transpose(sptrsv_handle_t h, hipStream_t stream);

/* Several right-hand sides, column-major: column r of B starts at B + r*ld.
 * nrhs >= 1, ld >= n.  Each row of T is read once for all columns, and each
 * column is computed as the one-lane-per-row single-RHS solve (equal to
 * sptrsv_solve with GROUP = 1, bit for bit).  Exception: on a pattern with
 * rows longer than 64 entries, unless GROUP = 1, the columns are solved by
 * the single-RHS schedule (each equal to sptrsv_solve on it, bit for bit),
 * since one lane per long row and column would walk the whole row: with a
 * static assignment and outside a stream capture all columns in one launch
 * over a chunk table that repeats every level once per column (grid, if
 * unset, 4 wavefronts per CU from 8 columns, else 2; position-ordered
 * solution n * nrhs slots), otherwise one after another.  B == X allowed.
 * transpose != 0 solves T^T X = B. */
int sptrsv_solve_multi(sptrsv_handle_t h, int32_t nrhs, int32_t ld, const void *B, void *X,
                       int transpose, hipStream_t stream);

/* Gradient of the solve with respect to the stored values (the adjoint of
 * x = T^{-1} b on the pattern): grad_vals[k] = -grad_b[i] * x[j] for each
 * stored entry k = (i, j) of the caller's CSR, in the caller's entry order;
 * 0 for stored diagonal entries when unit_diag.  grad_b = T^{-T} g comes from
 * sptrsv_solve_transpose.  row_ptr / col_idx are the caller's device arrays
 * given to sptrsv_analyze (for a batched handle: NULL, the concatenated
 * pattern kept by the handle is used and grad_vals is concatenated). */
int sptrsv_grad_vals(sptrsv_handle_t h, const int32_t *row_ptr, const int32_t *col_idx,
                     const void *grad_b, const void *x, void *grad_vals, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Options and information */
int sptrsv_set_option(sptrsv_handle_t h, sptrsv_option key, int64_t value);
int sptrsv_get_option(sptrsv_handle_t h, sptrsv_option key, int64_t *value);

/* Time short trials of the candidate schedules on (b, x) -- both device
 * vectors of n elements, x overwritten -- and keep the fastest (rows per
 * lane, sync, persistent grid, assignment, polling mode, slot width; and the
 * algorithm when ALGO is AUTO, else only candidates of the fixed ALGO; the
 * column-wise solves only when fixed).  The lanes of each row (GROUP and
 * ENTRIES_PER_LANE) stay as set, so every candidate computes the same bits:
 * the tuned result does not depend on which candidate timing picks.
 * Results are cached per pattern hash in the process.  Changing a schedule
 * option afterwards drops the tuned choice. */
int sptrsv_tune(sptrsv_handle_t h, const void *b, void *x, hipStream_t stream);

/* Autotuner for solves with nrhs >= 2 right-hand sides (column-major, column
 * stride ld >= n): times the self-scheduled solve over persistent grids of
 * 1, 2, 4 and 8 wavefronts per CU, static and XCD-regional assignment and
 * both polling modes (and the level-scheduled solve, unless the algorithm
 * option excludes it) on the caller's B and X, and keeps the fastest for
 * this nrhs.  Without it, options left unset follow the column count: 2, 4
 * or 8 wavefronts per CU from 2, 8 or 16 columns, XCD-regional assignment up
 * to 4 columns and round-robin beyond, one row per lane group.  Does nothing
 * where sptrsv_solve_multi solves with the single-RHS schedule (long
 * rows).  B != X.
 * Blocking.  Changing a schedule option discards the choice. */
int sptrsv_tune_multi(sptrsv_handle_t h, int32_t nrhs, int32_t ld, const void *B, void *X,
                      hipStream_t stream);

/* Measures the producer-to-consumer hop of the self-scheduled solves: two
 * wavefronts on different CUs bounce a counter through two device words,
 * each side publishing with an agent-scope atomic store and polling the
 * other's with agent-scope atomic loads; *ns_per_hop = elapsed time / (2 *
 * (iters - 1)) (the first round trip warms up).  same_xcd != 0 places the
 * peer workgroup eight workgroups after the first, which the dispatcher
 * sends to the same XCD, else on the next XCD.  iters >= 2.  Uses the
 * current device and its null stream; allocates and frees 256 bytes; waits
 * for the whole device (so that no other work skews the figure).  A hop
 * multiplied by the level count bounds a self-scheduled solve from below.
 * Errors: INVALID_ARG, HIP, OOM, TIMEOUT (a wait exceeded 2^26 polls). */
int sptrsv_probe_hop(int same_xcd, int32_t iters, double *ns_per_hop);

/* n, nnz, nlev of T; the algorithm and lanes per row the next solve uses
 * (resolved if AUTO); any pointer may be NULL. */
int sptrsv_get_info(sptrsv_handle_t h, int32_t *n, int64_t *nnz, int32_t *nlev,
                    int32_t *algo, int32_t *group);

/* The schedule the next solve will use (resolved: the autotuner's choice if
 * current, else the options): sptrsv_algo, lanes per row (0 = by row
 * length), entries per lane of the length rule, sptrsv_sync, rows per lane,
 * persistent workgroups (0 = default), sptrsv_assign, polling mode
 * (SPTRSV_OPT_POLL).  Any pointer may be NULL. */
int sptrsv_get_schedule(sptrsv_handle_t h, int32_t *algo, int32_t *group,
                        int32_t *entries_per_lane, int32_t *sync, int32_t *rows_per_lane,
                        int32_t *grid, int32_t *assign, int32_t *poll);

/* SPTRSV_OPT_XP_STRIDE of the schedule the next solve uses (the
 * autotuner's choice if one is current, else the option). */
int sptrsv_get_xp_stride(sptrsv_handle_t h, int32_t *stride);

/* Copy the analysis to HOST buffers (any may be NULL): level int32[n],
 * ilev int32[nlev+1], jlev int32[n] (rows by (level, row)), depcnt int32[n]
 * (stored off-diagonals per row).  transpose != 0 exports the analysis of
 * T^T (built if needed). */
int sptrsv_export_analysis(sptrsv_handle_t h, int transpose, int32_t *level, int32_t *ilev,
                           int32_t *jlev, int32_t *depcnt);

/* Device-side status of the last solves: synchronises the handle's last
 * stream, returns SPTRSV_OK, SPTRSV_ERR_NOT_RESIDENT, SPTRSV_ERR_TIMEOUT or
 * SPTRSV_ERR_ZERO_PIVOT (in that order of precedence when several were
 * raised), and clears it. */
int sptrsv_get_status(sptrsv_handle_t h);

/* Accumulated duration of the main solve kernels recorded while
 * SPTRSV_OPT_TIMING = 1 (milliseconds, HIP events on the solve stream) and
 * the number of launches timed; synchronises.  reset != 0 clears both.
 * The handle keeps at most 1024 pending event pairs: the next timed solve
 * first folds them into the totals, waiting for the oldest to finish. */
int sptrsv_kernel_time(sptrsv_handle_t h, double *ms, int64_t *count, int reset);

const char *sptrsv_status_string(int status);

/* Frees the handle and everything it owns, after the work it issued has
 * finished.  Returns SPTRSV_ERR_BUSY, and frees nothing, while graphs
 * captured from the handle are alive: their kernels use its buffers. */
int sptrsv_destroy(sptrsv_handle_t h);

/* ---------------------------------------------------------------------- */
/* HIP graph of one solve (or transposed solve) on fixed b/x pointers:
 * captured once on `stream`, replayed by sptrsv_graph_launch.  The handle's
 * options are frozen into the graph.  The graph uses the handle's buffers:
 * the handle cannot be destroyed while it lives (SPTRSV_ERR_BUSY), and a
 * position-ordered solution buffer that later calls replace (several
 * right-hand sides, wider slots) stays allocated until the graph is
 * destroyed.  b and x must stay allocated while the graph may be launched. */
int sptrsv_graph_capture(sptrsv_handle_t h, const void *b, void *x, int transpose,
                         hipStream_t stream, sptrsv_graph_t *out);
int sptrsv_graph_launch(sptrsv_graph_t g, hipStream_t stream);
int sptrsv_graph_destroy(sptrsv_graph_t g);

/* ---------------------------------------------------------------------- */
/* Host-only analysis (no device memory, no GPU needed): the same validation,
 * levels, level sets and dependency counts sptrsv_analyze computes, on HOST
 * arrays.  level/jlev/depcnt: int32[n]; ilev: int32[n+1] capacity (nlev+1
 * used); nlev: out.  Returns the validation status (vals not inspected, so
 * no ZERO_PIVOT). */
int sptrsv_analyze_host(int32_t n, int32_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                        sptrsv_uplo uplo, int unit_diag, int32_t *level, int32_t *ilev,
                        int32_t *jlev, int32_t *depcnt, int32_t *nlev);

#ifdef __cplusplus
}
#endif
#endif /* SPTRSV_H_ */
