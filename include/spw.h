/*
 * spw.h -- sparse wide/tall matrix-vector products on AMD Instinct MI355X (gfx950).
 *
 * The operations are those of Eckstein & Matyasfalvi, "Efficient Distributed-
 * Memory Parallel Matrix-Vector Multiplication with Wide or Tall Unstructured
 * Sparse Matrices" (arXiv:1812.00904), Section I: for a sparse A in R^{m x n},
 * y = A x (x in R^n, y in R^m) and u^T = v^T A (v in R^m, u in R^n).  A is very
 * wide (m << n) and stored column-major (CSC), or very tall (m >> n) and stored
 * row-major (CSR): Section II handles the tall case by swapping the roles of
 * rows and columns, and so does this library.  The work of one product is
 * split among GPU workgroups by equal runs of nonzeros that may cut a column
 * (Section II); cut columns are completed by summing the partial dot products
 * of the chunks that share them (Section IV-A), and A x sums per-workgroup
 * partial y vectors in a fixed order (Section III).  Results are bit-identical
 * from run to run.
 *
 * Conventions for every entry point:
 *   - All functions return spw_status; nothing is thrown across this boundary.
 *     On a non-OK status spw_last_error() returns a message for the calling
 *     thread, naming the first offending argument or position.
 *   - Indices are 0-based.  Host arrays passed to spw_create are copied; the
 *     caller may free them on return.  A matrix is immutable after creation.
 *   - Vector arguments (x, y, v, u, X, Y, V, U) are DEVICE pointers owned by the
 *     caller, on the device the matrix lives on, not aliasing one another.
 *     Outputs are overwritten, not accumulated into.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Products are
 *     asynchronous on that stream; outputs are valid once it has synchronized.
 *     Calls on one matrix handle must be ordered (one stream at a time): the
 *     handle owns the scratch (partial sums, carries) that a call uses.
 *   - Products never allocate device memory, except the first multi-RHS call
 *     with a block width larger than any before it on that handle (which grows
 *     the handle's scratch once, synchronously).
 */
#ifndef SPW_H
#define SPW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPW_OK = 0,
    SPW_ERR_INVALID_ARG = 1,   /* NULL pointer, negative size, bad enum, k < 1, ld < k ... */
    SPW_ERR_BAD_MATRIX = 2,    /* ptr not monotone / wrong ends, index out of range or not strictly increasing */
    SPW_ERR_OUT_OF_MEMORY = 3, /* device or host allocation failed */
    SPW_ERR_BUDGET = 4,        /* serving: registering or admitting would exceed the HBM budget */
    SPW_ERR_DEVICE = 5,        /* a HIP runtime call or kernel launch failed */
    SPW_ERR_UNSUPPORTED = 6,   /* valid request this library version does not implement (e.g. nnz >= 2^31) */
    SPW_ERR_BUSY = 7,          /* serving: queue full; products: the matrix has work in flight on another stream */
    SPW_ERR_TIMEOUT = 8,       /* serving: wait timed out (the request stays queued) */
    SPW_ERR_SHUTDOWN = 9       /* serving: server is shutting down */
} spw_status;

typedef enum { SPW_CSC = 0 /* wide, column-major */, SPW_CSR = 1 /* tall, row-major */ } spw_format;

typedef enum { SPW_F64 = 0, SPW_F32 = 1, SPW_BF16 = 2 } spw_dtype;

/* How the work of one product is divided among the GPU's workers. */
typedef enum {
    SPW_PART_NONZERO = 0,  /* equal runs of nonzeros (Section II), the default */
    SPW_PART_COLUMN = 1,   /* equal numbers of columns of the long dimension: the column
                              partitioning the paper compares against (Section VI); same
                              results, kept for that comparison */
    SPW_PART_MERGE = 2     /* merge path: equal runs of (nonzeros + columns), so that
                              workers whose share holds many short or empty columns
                              (many outputs to write) take fewer nonzeros */
} spw_partition;

typedef struct spw_matrix_s *spw_matrix;

/* Creation options.  Zero-initialise, set struct_size = sizeof(spw_create_opts),
 * or call spw_create_opts_default.  NULL opts means defaults.
 *   value_storage : F64 (default), F32 or BF16 -- the stored nonzero values are
 *                   rounded once from the given binary64 values, to nearest even
 *                   (BF16 directly from binary64, no double rounding); a value
 *                   that overflows the storage type is SPW_ERR_BAD_MATRIX.
 *                   Products promote stored values exactly to binary64.
 *   chunk_nnz     : nonzeros per column-dot chunk: 0 = automatic (1024, or the
 *                   tuner's choice with autotune), 512 or 1024; any other value is
 *                   SPW_ERR_UNSUPPORTED.  Smaller chunks give small matrices more
 *                   workers (Section II's P grows as the chunk shrinks).
 *   relabel       : -1 automatic, 0 off, 1 on.  On: rows are renumbered inside
 *                   the library by descending nonzero count, so the most used
 *                   entries of the short vector share cache lines; results are
 *                   returned in the caller's numbering.
 *   validate      : 1 (default) checks the arrays in O(nnz); 0 trusts them.
 *   panel_rows    : rows per on-chip accumulation panel for A x (0 = automatic).
 *   device        : HIP device ordinal, -1 = the current device.
 *   partition     : SPW_PART_NONZERO (default), SPW_PART_COLUMN or SPW_PART_MERGE.
 *                   With column partitioning each worker of the single-vector
 *                   products (a wave of the column dots, a workgroup of a scatter
 *                   row panel) owns an equal number of consecutive columns, the
 *                   first `cols mod P` workers one more; with merge-path
 *                   partitioning each owns a consecutive run of about equal
 *                   (nonzeros + columns): column-dot workers take whole chunks
 *                   (a chunk costs its nonzeros plus the columns starting in it),
 *                   scatter workgroups split their panel's column-ordered
 *                   nonzeros on the merge-path diagonals.  Column dots give
 *                   bit-identical results in every mode, the scatter product the
 *                   same up to rounding order.
 *   transpose     : 1 also keeps the transpose (the column-dot storage of A^T),
 *                   which the tiled multi-RHS plan of the long-to-short direction
 *                   (CSC A x, CSR v^T A) reads; 0 does not; -1 (default) keeps it
 *                   only with autotune (so the tuner can choose that plan).
 *                   Without it those blocks run scatter passes.  It is stored in
 *                   blocks of 2^18 long-side indices; a tiled call over more
 *                   than one block allocates (once, on first use) binary64
 *                   partial sums of blocks x short side x k entries and adds
 *                   them in block order.
 *   canonicalize  : 0 (default) rejects indices that are not strictly increasing
 *                   inside a column (row) and, in spw_create_coo, repeated
 *                   (row, column) pairs; 1 sorts each column (row) by index and
 *                   sums the values of a repeated index in the order they were
 *                   given.  Indices out of range are rejected either way.
 *   wg_size       : threads per workgroup of the single-vector column dots (v^T A
 *                   of a CSC matrix, A x of a CSR one): 0 = automatic (512, or 1024
 *                   for binary32 vectors with binary32 / bfloat16 values, or the
 *                   tuner's choice), 256, 512 or 1024 (1024 takes effect with
 *                   chunks of 512, or with binary32 vectors and 4- or 2-byte
 *                   values; 512 is used otherwise).  Smaller workgroups run two to a CU.  Results are
 *                   bit-identical whatever the workgroup size (it only changes
 *                   which wave reduces which chunk); the chunk size moves the
 *                   chunk boundaries, so columns cut by them can round
 *                   differently (both within the stated bounds).
 *   autotune      : 0 (default) off.  1: at creation, time the column dots for
 *                   every chunk size and workgroup size not fixed above (binary64
 *                   and binary32 vectors) and keep the fastest; on the first
 *                   multi-RHS call of each (direction, vector type, k) not under
 *                   graph capture, time the multi-RHS plans (spw_plan) on the
 *                   caller's own buffers and stream (that call synchronizes the
 *                   stream) and keep the fastest.  Choices are recorded per matrix
 *                   fingerprint in the tuning cache (spw_tune_cache_path), and a
 *                   recorded choice is taken without timing. */
typedef struct {
    uint32_t struct_size;
    spw_dtype value_storage;
    int32_t chunk_nnz;
    int32_t relabel;
    int32_t validate;
    int32_t panel_rows;
    int32_t device;
    int32_t transpose;
    spw_partition partition;
    int32_t canonicalize;
    int32_t wg_size;
    int32_t autotune;
    int32_t reserved[3];
} spw_create_opts;

/* Read-only description of a created matrix. */
typedef struct {
    uint32_t struct_size;
    spw_format format;
    spw_dtype value_storage;
    int64_t m, n, nnz;            /* as given by the caller */
    int64_t inner_rows;           /* short dimension (m for CSC, n for CSR) */
    int64_t inner_cols;           /* long dimension */
    int64_t chunk_nnz;            /* transpose-product chunk size */
    int64_t n_chunks;             /* number of chunks (the paper's P) */
    int64_t n_zones;              /* columns cut by a chunk boundary (the paper's z) */
    int64_t n_panels;             /* row panels used by A x (long-dimension scatter) */
    int64_t panel_rows;
    int64_t mv_workgroups;        /* workgroups (partial vectors) of the scatter product */
    int64_t index_bytes;          /* bytes per stored row index (2 or 4) */
    int32_t relabeled;            /* rows renumbered by frequency */
    int32_t device;
    int64_t device_bytes;         /* device memory held by the handle */
    int32_t has_transpose;        /* the transpose is kept (see spw_create_opts.transpose) */
    spw_partition partition;
    int64_t workers;              /* P: workers of the single-vector column dots (waves) */
    int64_t worker_max_nnz;       /* nonzeros owned by the busiest / idlest of them; the paper's */
    int64_t worker_min_nnz;       /* imbalance is P * (max - min) / nnz (Section VI) */
    int32_t wg_size_f64;          /* column-dot workgroup size used with binary64 vectors */
    int32_t wg_size_f32;          /* ... and with binary32 vectors */
    int32_t tuned;                /* 1: chunk and workgroup sizes came from the tuner (timed or cached) */
    uint64_t fingerprint;         /* the key of the matrix's tuning-cache records */
} spw_matrix_info;

/* ---------------------------------------------------------------- matrices */

spw_status spw_create_opts_default(spw_create_opts *opts);

/* Create a matrix from host arrays.
 *   fmt == SPW_CSC: ptr has n+1 entries, column j holds positions ptr[j]..ptr[j+1]-1,
 *                   idx[p] is the row (0 <= idx < m), strictly increasing inside a column.
 *   fmt == SPW_CSR: ptr has m+1 entries, row i holds ptr[i]..ptr[i+1]-1, idx[p] is the
 *                   column (0 <= idx < n), strictly increasing inside a row.
 *   ptr[0] == 0, ptr nondecreasing, ptr[last] == nnz.  val has nnz entries.
 *   nnz == 0 is valid (all products are zero); m or n may be 0.
 * Limits of this version: nnz < 2^31, short dimension < 2^31.
 * Errors: SPW_ERR_INVALID_ARG (NULL out/ptr, NULL idx/val with nnz > 0, negative sizes),
 *         SPW_ERR_BAD_MATRIX (validation), SPW_ERR_OUT_OF_MEMORY, SPW_ERR_DEVICE,
 *         SPW_ERR_UNSUPPORTED. */
spw_status spw_create(spw_matrix *out, spw_format fmt, int64_t m, int64_t n, int64_t nnz,
                      const int64_t *ptr, const int32_t *idx, const double *val,
                      const spw_create_opts *opts);

/* Create a matrix from coordinate triples, the input form of the paper's
 * nonzero-partitioned driver (Section V: a stream of (row, column, value)
 * triples in column-major order).  Any order is accepted: the triples are
 * sorted on the host into the compressed arrays of fmt (SPW_CSC: by column,
 * then row; SPW_CSR: by row, then column), which then go through spw_create
 * with opts.
 *   rows, cols : nnz int32 entries each, 0 <= rows[p] < m, 0 <= cols[p] < n
 *   val        : nnz binary64 entries
 * Errors: as spw_create, plus SPW_ERR_BAD_MATRIX for an index out of range or
 * a (row, column) pair given twice (duplicates are not summed). */
spw_status spw_create_coo(spw_matrix *out, spw_format fmt, int64_t m, int64_t n, int64_t nnz,
                          const int32_t *rows, const int32_t *cols, const double *val,
                          const spw_create_opts *opts);

/* Release the matrix and its device memory (waits for the device first).  NULL is a no-op. */
spw_status spw_destroy(spw_matrix A);

spw_status spw_info(spw_matrix A, spw_matrix_info *out);

/* --------------------------------------------------------------- products */

typedef enum { SPW_OP_MV = 0 /* y := A x */, SPW_OP_VTM = 1 /* u^T := v^T A */ } spw_op;

/* Calls are asynchronous on `stream` (a hipStream_t; NULL = the default
 * stream); results are valid once the stream reaches the end of the call's
 * work.  A matrix's scratch serves one stream at a time: a product or solver
 * call on another stream than the previous call's while that call's work is
 * still pending returns SPW_ERR_BUSY (nothing is enqueued).  Work captured into
 * a graph, and work the server issues, is ordered by its owner and not checked.
 */

/* y := A x (Section I; for CSC, Section III's nonzero-split product).
 * x: device, n entries of type vdt; y: device, m entries of type vdt.
 * vdt: SPW_F64 or SPW_F32 (binary32 vectors).  Whatever the vector and
 * storage types, every product and sum is formed in binary64 (products of
 * binary32 or bfloat16 values with binary32 entries are exact there), carries
 * and partial vectors are binary64, and each output is rounded once to vdt. */
spw_status spw_mv(spw_matrix A, spw_dtype vdt, const void *x, void *y, void *stream);

/* u^T := v^T A (Section I; for CSC, Section IV-A's per-column dot with zone sums).
 * v: device, m entries of type vdt; u: device, n entries of type vdt. */
spw_status spw_vtm(spw_matrix A, spw_dtype vdt, const void *v, void *u, void *stream);

/* Multi-right-hand-side forms, one pass over A for k vectors (1 <= k <= 64).
 * X: device, row-major n x k with leading dimension ldx >= k (X[j*ldx + c]);
 * Y: device, row-major m x k, ldy >= k.  Column c of Y equals spw_mv on column c
 * of X up to rounding order.  For the scatter direction (CSC A x, CSR v^T A)
 * with 2 <= k <= 15 the first call allocates a partial-sum workspace of
 * min(k, 8) * mv_workgroups * panel_rows doubles, kept with the matrix. */
spw_status spw_mv_batch(spw_matrix A, spw_dtype vdt, int32_t k, const void *X, int64_t ldx,
                        void *Y, int64_t ldy, void *stream);

/* V: device, row-major m x k (ldv >= k); U: device, row-major n x k (ldu >= k). */
spw_status spw_vtm_batch(spw_matrix A, spw_dtype vdt, int32_t k, const void *V, int64_t ldv,
                         void *U, int64_t ldu, void *stream);

/* How a multi-RHS call (k >= 2) runs.  Every plan gives each column within the
 * binary64 / binary32 bounds of the oracle; SINGLE and PASSES give every
 * column bit-identical to a single-vector call on it.
 *   SPW_PLAN_AUTO   : the library's rule, or the tuner's choice (autotune)
 *   SPW_PLAN_SINGLE : k passes of the single-vector kernels, one per column
 *   SPW_PLAN_PASSES : passes of up to 8 columns that each read the matrix once
 *                     (column dots with one chunk load per pass, or the
 *                     scatter product with one partial-sum slot per column)
 *   SPW_PLAN_TILE   : the tiled column dots, all k columns in one pass; for the
 *                     scatter direction (A x of a CSC matrix, v^T A of a CSR
 *                     one) they run over the kept transpose
 * The fixed rule: scatter direction PASSES below k = 16 (or without a kept
 * transpose), TILE from 16; column-dot direction PASSES up to k = 6, TILE
 * above.  Column dots with an output leading dimension of 2^18 or more always
 * take TILE. */
typedef enum { SPW_PLAN_AUTO = 0, SPW_PLAN_SINGLE = 1, SPW_PLAN_PASSES = 2, SPW_PLAN_TILE = 3 } spw_plan;

/* The plan a k-column call of op with vector type vdt takes now (never
 * SPW_PLAN_AUTO); *tuned = 1 when it was chosen by timing (or set, or read
 * from the tuning cache).  Host only; does not tune. */
spw_status spw_batch_plan(spw_matrix A, spw_op op, spw_dtype vdt, int32_t k, spw_plan *plan, int32_t *tuned);
/* Fixes the plan of k-column calls of op with vector type vdt on this matrix
 * (SPW_PLAN_AUTO returns to the rule / tuner).  SPW_ERR_UNSUPPORTED for
 * SPW_PLAN_TILE in the scatter direction when the transpose is not kept. */
spw_status spw_set_batch_plan(spw_matrix A, spw_op op, spw_dtype vdt, int32_t k, spw_plan plan);

/* ------------------------------------------------------------- a solver */

/* Conjugate gradients on the least-squares problem min ||b - A x||_2 (CGLS):
 * the first-order use of the two products that Section VII describes, where
 * each iteration alternates one y := A p with one u^T := r^T A and a few
 * vector updates and inner products.  The paper names conjugate gradients
 * without fixing a variant; this is the Hestenes-Stiefel form as arranged by
 * Bjorck (1996, Section 7.4): r_0 = b - A x_0, s_0 = p_0 = A^T r_0,
 * gamma_0 = ||s_0||^2, then for k = 0 .. iters-1: q = A p_k,
 * alpha = gamma_k / ||q||^2, x += alpha p_k, r -= alpha q, s = A^T r,
 * gamma_{k+1} = ||s||^2, p_{k+1} = s + (gamma_{k+1} / gamma_k) p_k.  A step
 * whose denominator is exactly zero (the iterate already solves the normal
 * equations) has size zero.  The product with A is taken of s_k and q = A p_k
 * formed by linearity, q_k = A s_k + beta_k q_{k-1} (equal in exact
 * arithmetic), so that the update of p and x can run before the product with
 * A^T; every 50th iteration takes q_k = A p_k with a product of its own
 * (after forming p_k), so rounding does not accumulate in that recurrence.  Inner products are summed in a fixed order, so a call is bit-identical
 * from run to run.
 *   vdt   : SPW_F64 (SPW_ERR_UNSUPPORTED otherwise)
 *   b     : device, m binary64 entries (not written)
 *   x     : device, n binary64 entries: x_0 on entry, x_iters when the stream
 *           reaches the end of the call's work
 *   iters : >= 0
 *   hist  : NULL, or host array of 2*(iters+1) doubles that receives
 *           hist[k] = ||A^T r_k||^2 and hist[iters+1+k] = ||r_k||^2 for
 *           k = 0 .. iters; the call then waits for the stream before returning.
 *           Without hist the call only enqueues work on the stream, the same
 *           launches on every call with the same arguments, so a caller can
 *           capture it in a graph (after one call has grown the workspace).
 * Workspace (2m + 2n doubles and the history) is kept with the matrix until
 * spw_destroy and counted in device_bytes.  Calls on one matrix must not
 * overlap (they share that workspace and the products' scratch). */
spw_status spw_cgls(spw_matrix A, spw_dtype vdt, const void *b, void *x, int32_t iters, double *hist,
                    void *stream);

/* ----------------------------------------------------------------- serving */

/* A server keeps many created matrices resident and serves product requests
 * submitted from any thread.  Queued requests for the same matrix, operation
 * and vector type are merged into one group (continuous batching: requests
 * that arrive while earlier groups run join the next group) and issued on one
 * of a few HIP streams, at most `depth` groups per stream.  A group's columns
 * run as passes of up to 8 columns (column dots or the scatter product, by
 * direction) that each read the matrix once, and every column is reduced
 * exactly as a lone single-vector call would reduce it: a request's output is
 * bit-identical whatever else it was batched with.  The memory a matrix holds
 * (spw_matrix_info.device_bytes, after its scratch -- carries, renumbered
 * inputs and the scatter product's partial sums -- grows to 8 columns at
 * registration) is charged to the server's HBM budget. */
typedef struct spw_server_s *spw_server;

/* Zero-initialise and set struct_size, or call spw_serve_opts_default. */
typedef struct {
    uint32_t struct_size;
    int32_t max_inflight;      /* requests queued or running; submit beyond it is SPW_ERR_BUSY (4096) */
    int64_t hbm_budget_bytes;  /* device bytes registered matrices may hold (64 GiB) */
    int32_t streams;           /* HIP streams, default priority, 1..16 (4) */
    int32_t depth;             /* groups in flight per stream (2) */
    int32_t max_batch_cols;    /* columns merged into one group (64) */
    int32_t device;            /* HIP device ordinal, -1 = current (-1) */
    int32_t start_paused;      /* 1: issue nothing until spw_serve_resume (0) */
    int32_t reserved[7];
} spw_serve_opts;

/* One request: k columns, laid out as for spw_mv_batch / spw_vtm_batch
 * (row-major, leading dimensions ldi, ldo >= k).  in/out are device buffers
 * owned by the caller that must stay valid until the request completes. */
typedef struct {
    uint32_t struct_size;
    int32_t matrix;            /* handle returned by spw_serve_register */
    spw_op op;
    spw_dtype vdt;             /* SPW_F64 or SPW_F32 */
    int32_t k;                 /* 1..64 */
    const void *in;
    int64_t ldi;
    void *out;
    int64_t ldo;
    uint64_t tag;              /* the caller's; not interpreted */
} spw_request;

/* Counters since creation.  Latency is host time from submit to the moment
 * the completion thread sees the request's group finish. */
typedef struct {
    uint32_t struct_size;
    int64_t submitted, completed, rejected_busy;
    int64_t groups;            /* groups issued */
    int64_t merged_requests;   /* requests that shared a group with others */
    int64_t passes;            /* kernel passes over a matrix */
    int64_t inflight;          /* queued or running now */
    int64_t registered;
    int64_t hbm_budget_bytes, hbm_used_bytes;
    double latency_p50_us, latency_p99_us, latency_mean_us;
    double model_bytes;        /* sum over completed requests of the algorithmic bytes:
                                  nnz*(value bytes + 4) + 4*(long dim + 1) + k*(m + n)*vector bytes */
    double busy_seconds;       /* first submit to last completion */
    double gbps;               /* model_bytes / busy_seconds / 1e9 */
} spw_server_stats;

spw_status spw_serve_opts_default(spw_serve_opts *opts);
/* Starts the dispatcher and one completion thread per stream.  NULL opts means
 * defaults.  SPW_ERR_INVALID_ARG for bad options, SPW_ERR_DEVICE without a GPU. */
spw_status spw_serve_create(spw_server *out, const spw_serve_opts *opts);
/* Makes A resident in the server and returns its handle (0, 1, ...).  The
 * caller keeps ownership of A and must not destroy it or use it outside the
 * server until the server is destroyed.  SPW_ERR_BUDGET when A would exceed
 * the budget (A stays usable; its scratch may have grown). */
spw_status spw_serve_register(spw_server s, spw_matrix A, int32_t *handle);
/* Queues a request; *ticket identifies it.  SPW_ERR_BUSY at max_inflight,
 * SPW_ERR_SHUTDOWN while the server is being destroyed, SPW_ERR_INVALID_ARG
 * for a bad request (checked before queueing), SPW_ERR_UNSUPPORTED for an
 * output leading dimension of 2^18 or more on the column-dot side (v^T A of
 * a CSC matrix, A x of a CSR matrix). */
spw_status spw_serve_submit(spw_server s, const spw_request *r, uint64_t *ticket);
/* Starts issuing when the server was created paused (no-op otherwise). */
spw_status spw_serve_resume(spw_server s);
/* *done = 1 when the request has completed (its output is valid). Returns the
 * request's error if it failed on the device. */
spw_status spw_serve_poll(spw_server s, uint64_t ticket, int32_t *done);
/* Blocks until the request completes, or timeout_us passes (< 0: no limit):
 * SPW_ERR_TIMEOUT then, and the request stays queued or running. */
spw_status spw_serve_wait(spw_server s, uint64_t ticket, int64_t timeout_us);
spw_status spw_serve_stats(spw_server s, spw_server_stats *out);
/* Stops accepting requests, runs everything queued (also when paused), waits
 * for it, and frees the server's threads and streams.  NULL is a no-op. */
spw_status spw_serve_destroy(spw_server s);

/* ---------------------------------------------------------- host-only helpers */

/* Tuning cache (the autotuner's records; see spw_create_opts.autotune).  A
 * record is (matrix fingerprint, key, value); keys are 1..63 printable
 * characters without blanks.  Records live in memory for the process and, when
 * a cache file is set, in that file (text: a header line, then one
 * "<16 hex digits> <key> <value>" line per record, rewritten whole after each
 * new record).  The environment variable SPW_TUNE_CACHE names the file unless
 * spw_tune_cache_path is called first.
 *   spw_tune_cache_path  : use `path` (NULL: memory only) and load its records
 *   spw_tune_cache_clear : forget the records held in memory (not the file)
 *   spw_tune_cache_put   : record a value (SPW_ERR_DEVICE if the file cannot be written)
 *   spw_tune_cache_get   : *found = 1 and *value when recorded, else *found = 0
 *   spw_matrix_fingerprint : the key spw_create uses for a matrix: a 64-bit FNV-1a
 *                   hash of format, value storage, shape and 4,097 evenly spaced
 *                   entries of ptr and of idx (values do not enter it). */
spw_status spw_tune_cache_path(const char *path);
spw_status spw_tune_cache_clear(void);
spw_status spw_tune_cache_put(uint64_t fingerprint, const char *key, int32_t value);
spw_status spw_tune_cache_get(uint64_t fingerprint, const char *key, int32_t *value, int32_t *found);
spw_status spw_matrix_fingerprint(spw_format fmt, spw_dtype storage, int64_t m, int64_t n, int64_t nnz,
                                  const int64_t *ptr, const int32_t *idx, uint64_t *out);

/* Rounds n binary64 values the way spw_create stores them for `storage`
 * (nearest, ties to even) and returns them promoted back to binary64, so that
 * a caller can form the exact matrix a product uses.  in/out are host arrays
 * (may be the same).  SPW_ERR_BAD_MATRIX names the first value that overflows. */
spw_status spw_round_values(spw_dtype storage, int64_t n, const double *in, double *out);

/* The chunk / zone plan the transpose product uses, computed on the host from a
 * column pointer array (no device needed).  Chunk c holds positions
 * [c*chunk_nnz, min((c+1)*chunk_nnz, nnz)).  A zone is a column cut by a chunk
 * boundary (Section II's overlap zone); its chunk set S_k is the contiguous run
 * zone_first[k]..zone_last[k] (Table I).  chunk_owned[c] is the first column
 * whose start lies in chunk c (chunk_owned[n_chunks] = n).  Pass NULL arrays to
 * query the counts; otherwise arrays must hold n_chunks+1 / n_zones entries. */
spw_status spw_plan_zones(int64_t n, const int64_t *ptr, int64_t chunk_nnz,
                          int64_t *n_chunks, int64_t *n_zones, int64_t *chunk_owned,
                          int64_t *zone_col, int64_t *zone_first, int64_t *zone_last);

/* -------------------------------------------------------------- profiling */

/* When enabled (per process), every kernel launch of the library is bracketed
 * by HIP events on the launch stream; spw_profile_read returns, per kernel
 * name, the launch count and total milliseconds of the launches completed
 * since the last reset (it synchronizes those events).  Off by default. */
spw_status spw_profile_enable(int32_t on);
/* Restricts the timing to kernels whose name begins with `prefix` (for
 * example "vtm_wave"), so that the events of the other launches do not slow
 * a timed loop; NULL or "" times every launch (the default).  The prefix is
 * copied. */
spw_status spw_profile_select(const char *prefix);
spw_status spw_profile_reset(void);
/* Fills up to `cap` entries; *count receives the number of distinct kernels. */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
} spw_profile_entry;
spw_status spw_profile_read(spw_profile_entry *entries, int32_t cap, int32_t *count);

/* ------------------------------------------------------------ bandwidth probe */

/* The HBM ceilings the products are measured against, with the library's
 * own kernels: a read-only stream over `bytes` of device memory at src
 * (16-byte non-temporal loads, eight in flight per thread, four 512-thread
 * workgroups per CU) and, when dst is not NULL, a copy of the same bytes to
 * dst.  One untimed run, then `reps` timed runs (HIP events on `stream`); the
 * medians go to *read_ms and *copy_ms.  Nothing is written to src; dst
 * receives the copy.  src and dst are device buffers of at least `bytes`,
 * 16-byte aligned; bytes is a positive multiple of 16.  Waits for the stream.
 * Errors: SPW_ERR_INVALID_ARG, SPW_ERR_OUT_OF_MEMORY (an 8-KB result buffer),
 * SPW_ERR_DEVICE. */
spw_status spw_probe_bandwidth(const void *src, void *dst, int64_t bytes, int32_t reps, double *read_ms,
                               double *copy_ms, void *stream);

/* ----------------------------------------------------------------- errors */

const char *spw_last_error(void);
const char *spw_status_string(spw_status s);

#ifdef __cplusplus
}
#endif
#endif /* SPW_H */
