/*
 * lb.h -- C ABI of the load-balanced sparse library for AMD MI355X (gfx950).
 *
 * The library implements the load-balancing programming model of Osama,
 * Porumbescu and Owens, "A Programming Model for GPU Load Balancing"
 * (PPoPP'23): a sparse matrix is a tile set whose tiles are rows and whose
 * work atoms are nonzeros (Sec. 3.1, Sec. 4.1 CSR listing); a schedule maps
 * tiles and atoms to GPU threads (Sec. 3.2, Sec. 4.2, Sec. 5.2); the
 * computation consumes the per-thread ranges (Sec. 3.3, Sec. 4.3).  The
 * computation offered here is CSR sparse matrix-vector product y = A x
 * (Sec. 1, Sec. 4.3 SpMV listing), its multi-right-hand-side form Y = A X
 * (Sec. 5.3 SpMM listing), its backward pass, and a batched form; and, on
 * the same schedules, the graph traversals of Sec. 5.3 (SSSP) and Sec. 6
 * (BFS).  Device-side, include/lb_schedule.hpp exposes the tile sets and
 * schedules to HIP kernels written by the user.
 *
 * Conventions for every entry point:
 *  - Device buffers, the workspace and the stream are owned by the caller.
 *    The library allocates no device memory in these calls and keeps no
 *    device state between them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on `stream` unless stated otherwise.
 *  - Index arrays are int32.  rows + nnz must stay below 2^31 - 1 (merge-path
 *    coordinates are int32); larger inputs return LB_ERR_OVERFLOW.
 *  - Every host-checkable precondition is checked before any launch; on
 *    error nothing is launched and the outputs are untouched.
 *  - Device-only preconditions (row_offsets[0] == 0, non-decreasing,
 *    row_offsets[rows] == nnz, 0 <= col_idx < cols) are not checked by the
 *    compute calls; violating them is undefined behaviour.  lb_validate_csr
 *    checks them (synchronously) for debugging.
 *  - Errors are status codes; nothing throws across this boundary.
 *  - Outputs that are accumulated with hardware float atomics -- dx of
 *    lb_spmv_backward, y of lb_spmv_csc, and the workspace of lb_spgemm_*
 *    (its large-row accumulators) -- must be ordinary device allocations
 *    (hipMalloc, coarse-grained): those atomics are not guaranteed on
 *    fine-grained memory (host-coherent, managed or host-registered).
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_ABI_VERSION 4
#define LB_API __attribute__((visibility("default")))

typedef enum lb_status_t {
    LB_OK = 0,
    LB_ERR_INVALID_ARG = 1,          /* null pointer with nonzero extent, negative size, bad field */
    LB_ERR_UNSUPPORTED = 2,          /* dtype / schedule / parameter combination not built */
    LB_ERR_OVERFLOW = 3,             /* rows + nnz (or a batch's totals) exceed int32 coordinates */
    LB_ERR_WORKSPACE_TOO_SMALL = 4,  /* workspace_bytes below lb_workspace_size() */
    LB_ERR_HIP = 5,                  /* a HIP call or launch failed; see lb_last_hip_error() */
    LB_ERR_INVALID_CSR = 6,          /* lb_validate_csr found a violated device-only precondition */
    LB_ERR_NOT_CONVERGED = 7,        /* a traversal still had a frontier after max_iterations */
    LB_ERR_SCRATCH_LIMIT = 8         /* lb_spmv_noalloc: the call needs more than its static scratch */
} lb_status_t;

/* Element types.  LB_BF16 buffers hold bfloat16 bit patterns (the upper 16
 * bits of an IEEE binary32).  LB_F64 is declared for the ABI but not built. */
typedef enum lb_dtype_t { LB_F32 = 0, LB_BF16 = 1, LB_F64 = 2 } lb_dtype_t;

/* Schedules (Sec. 4.2, Sec. 5.2).  One identifier selects one (Sec. 6.2). */
typedef enum lb_sched_kind_t {
    LB_THREAD_MAPPED = 0,  /* tile r -> one thread, grid-stride over tiles (Sec. 4.2 listing) */
    LB_GROUP_MAPPED = 1,   /* tiles -> groups of G lanes (Sec. 5.2.2, Sec. 5.2.3) */
    LB_MERGE_PATH = 2,     /* rows + nnz split evenly over threads (Sec. 5.2.1) */
    LB_AUTO = 3,           /* heuristic of Sec. 6.2 (alpha = 500, beta = 10000), or a tuned pick */
    LB_WORK_QUEUE = 4      /* group-mapped, G tiles per group, rounds handed to a persistent grid by
                              a device work queue (Sec. 5.1 persistent mode, infinite_range) */
} lb_sched_kind_t;

/* A CSR matrix in device memory (Sec. 4.1): row_offsets[rows + 1],
 * col_idx[nnz], values[nnz] of value_dtype.  row_offsets may be NULL only
 * when rows == 0; col_idx and values may be NULL only when nnz == 0. */
typedef struct lb_csr_t {
    int64_t rows;
    int64_t cols;
    int64_t nnz;
    const int32_t *row_offsets;
    const int32_t *col_idx;
    const void *values;
    lb_dtype_t value_dtype;
} lb_csr_t;

/* Schedule parameters.  A zero field takes the default noted.
 *  group_size        LB_GROUP_MAPPED: lanes per group, a power of two in
 *                    [1, 1024] (default 64, one wavefront).
 *                    LB_WORK_QUEUE: as group-mapped with tiles_per_group =
 *                    group_size (default 64); a persistent grid (grid_size, 0 =
 *                    resident blocks) claims rounds of G-tile chunks from a
 *                    counter in the workspace (256 bytes), so blocks that meet
 *                    short rows take more work.  lb_spmv, lb_sssp and lb_bfs.
 *  tiles_per_group   LB_GROUP_MAPPED: 1 = one tile per group at a time, lanes
 *                    stride its atoms (Sec. 5.2.2); equal to group_size = the
 *                    group takes that many tiles, prefix-sums their sizes in
 *                    LDS and its lanes walk the flattened atoms, each finding
 *                    its tile by binary search (Sec. 5.2.3).  Default 1.
 *  items_per_thread  LB_MERGE_PATH: merge items (row ends + nonzeros) per
 *                    thread, one of 4, 8, 12, 16 (default 8).
 *  block_size        threads per block: thread-mapped 64..1024 (default 256);
 *                    merge-path one of 128, 256, 512 (default 256).  When
 *                    both are 0 in lb_spmv or lb_spmm with k = 1 (one column
 *                    band), a matrix with rows + nnz <= 256 * 2048 gets the
 *                    shortest unit of 128 x 4, 256 x 4 and 256 x 8 items
 *                    that gives at most 256 units, which lb_spmv runs as
 *                    one launch; lb_resolve_schedule reports the choice.  SpMM
 *                    and batched passes take up to 8 columns of X at a
 *                    time, fewer for large block_size * items_per_thread;
 *                    group-mapped derived from group_size (ignored).
 *  grid_size         blocks; 0 = one block per chunk of work.
 *  x_bands           LB_MERGE_PATH in lb_spmv: 1 or 2 (default 1).  With 2,
 *                    every merge-path unit is consumed by two blocks placed on
 *                    different XCDs (blocks are dealt to the 8 XCDs round
 *                    robin), one for the columns below ceil(cols / 2) and one
 *                    for the rest, so each XCD's L2 caches only its half of x;
 *                    y is the sum of the two halves' row sums, added in that
 *                    order (deterministic).  Pays when x is larger than one
 *                    XCD's L2 (4 MiB) and its columns are scattered; costs a
 *                    second read of col_idx (served mostly by the Infinity
 *                    Cache) and a rows-sized buffer in the workspace.  Other
 *                    entry points accept only 0 or 1.
 *  vector_width      LB_MERGE_PATH in lb_spmv with one band: 1 or 4 (default
 *                    1).  With 4 each lane loads four consecutive nonzeros
 *                    (one 16-byte column load, one 16- or 8-byte value load)
 *                    instead of one: more bytes in flight per instruction,
 *                    which pays on matrices with local columns (stencils);
 *                    on scattered columns it costs the x gathers' line
 *                    sharing.  Runs the one-nonzero form when nnz < 4 or
 *                    col_idx / values are not 16- / 16- (BF16: 8-) byte
 *                    aligned; items_per_thread must be a multiple of 4.
 *                    Other entry points accept only 0 or 1. */
typedef struct lb_schedule_t {
    lb_sched_kind_t kind;
    int32_t group_size;
    int32_t tiles_per_group;
    int32_t items_per_thread;
    int32_t block_size;
    int32_t grid_size;
    int32_t x_bands;
    int32_t vector_width;
} lb_schedule_t;

/* Independent CSR matrices stored back to back (a block-diagonal matrix).
 *  row_offsets   int32[total_rows + 1]: the block-diagonal matrix's offsets
 *                into the concatenated nonzeros (matrix b's rows occupy
 *                [mat_row_base[b], mat_row_base[b+1])).
 *  col_idx       int32[total_nnz], local to each matrix: in [0, n_b).
 *  values        total_nnz elements of value_dtype.
 *  mat_row_base, mat_nnz_base, mat_col_base: int64[count + 1] device arrays,
 *                prefix sums of m_b, nnz_b and n_b (first entry 0).
 *  The host-side totals duplicate the last prefix entries so the library
 *  can size work without reading device memory. */
typedef struct lb_batch_t {
    int64_t count;
    int64_t total_rows;
    int64_t total_cols;
    int64_t total_nnz;
    const int32_t *row_offsets;
    const int32_t *col_idx;
    const void *values;
    lb_dtype_t value_dtype;
    const int64_t *mat_row_base;
    const int64_t *mat_nnz_base;
    const int64_t *mat_col_base;
} lb_batch_t;

/* A row-sorted COO matrix in device memory: entry j is (row_idx[j],
 * col_idx[j], values[j]); row_idx is non-decreasing (a device-only
 * precondition), entries of one row in any column order, repeated
 * (row, col) pairs are summed.  Pointers may be NULL only when nnz == 0. */
typedef struct lb_coo_t {
    int64_t rows;
    int64_t cols;
    int64_t nnz;
    const int32_t *row_idx;
    const int32_t *col_idx;
    const void *values;
    lb_dtype_t value_dtype;
} lb_coo_t;

/* A CSC matrix in device memory: column c's entries are
 * [col_offsets[c], col_offsets[c+1]) with rows row_idx[j] and values[j]. */
typedef struct lb_csc_t {
    int64_t rows;
    int64_t cols;
    int64_t nnz;
    const int32_t *col_offsets;
    const int32_t *row_idx;
    const void *values;
    lb_dtype_t value_dtype;
} lb_csc_t;

/* Version of this header the library was built from (LB_ABI_VERSION). */
LB_API int lb_abi_version(void);

/* Static, human-readable text for a status code. */
LB_API const char *lb_status_string(lb_status_t status);

/* Text of the most recent HIP failure on the calling thread ("" if none). */
LB_API const char *lb_last_hip_error(void);

/* Resolve LB_AUTO and zero fields of *in into concrete parameters for the
 * matrix A and k right-hand sides.  Host-only; reads no device memory.
 * LB_AUTO follows Sec. 6.2: merge-path unless (rows < 500 or cols < 500) and
 * nnz < 10000, in which case thread-mapped when the mean row length is below
 * 8, else group-mapped with the next power of two of the mean row length
 * (at most 64) as group size.  A schedule stored by lb_autotune for the
 * matrix (bound by lb_autotune or lb_autotune_lookup) takes precedence. */
LB_API lb_status_t lb_resolve_schedule(const lb_csr_t *A, int32_t k, const lb_schedule_t *in,
                                       lb_schedule_t *out);

/* Device workspace bytes that lb_spmv (k == 1), lb_spmm (k >= 1) or
 * lb_spmv_backward (k == 0) need for A under schedule s.  Host-only. */
LB_API lb_status_t lb_workspace_size(const lb_csr_t *A, const lb_schedule_t *s, int32_t k,
                                     size_t *bytes);

/* y = A x (Sec. 1; Sec. 4.3 SpMV listing).  x: cols elements of x_dtype
 * (must equal A->value_dtype); y: rows float32, overwritten (rows with no
 * nonzeros get 0).  Products and sums are float32 for both input types.
 * For a fixed schedule the result is bit-reproducible run to run (no
 * atomics).  workspace: device memory of at least lb_workspace_size(A, s, 1)
 * bytes (may be NULL when that is 0), contents on entry irrelevant. */
LB_API lb_status_t lb_spmv(const lb_csr_t *A, const void *x, lb_dtype_t x_dtype, float *y,
                           const lb_schedule_t *s, void *workspace, size_t workspace_bytes,
                           void *stream);

/* ---- Planned y = A x for a pattern used many times (an iterative solver, a
 * serving loop).  A plan is built once per sparsity pattern; the values and
 * x may change between calls.  Rows are split in two classes by length:
 *  - short rows (fewer than long_min nonzeros) run the merge path of
 *    lb_spmv (Sec. 5.2.1) over the whole matrix with the long rows' work
 *    left out: the split at every unit boundary is computed once, in the
 *    plan, and only the units in which a short row closes are launched.
 *    The unit where a row closes owns it whole: its block also sums the
 *    row's nonzeros that lie in earlier units, so no carries remain and
 *    with one band (and no long rows) the call is a single launch;
 *  - long rows run a panel schedule: x is cut into panels of panel_cols
 *    columns; each panel is served by panel_blocks blocks, each of which
 *    stages the panel of x in LDS once and consumes an equal share of the
 *    long rows' segments whose columns fall in the panel (a segment is
 *    contiguous in its row, as the row's columns are sorted).  The segments
 *    are cut into tasks of at most 252 nonzeros; a task spanning at most G
 *    aligned groups of four nonzeros runs on a group of G lanes, G = 64, 32,
 *    16 or 8 (the group-mapped schedule, Sec. 5.2.2, with the group size
 *    matched to the tile), one 16-byte group per lane, so x is read from LDS
 *    instead of the cache hierarchy.  Each task's sum is stored, and a long
 *    row's result is the sum of its tasks in (panel, task) order.
 * No atomics: for a fixed plan the result is bit-reproducible run to run.
 *
 * The plan lives in a device buffer owned by the caller, read-only for the
 * calls (several calls may share it).  lb_spmv_plan_build synchronizes
 * `stream` and copies row_offsets (and a few plan tables) through host
 * memory.  Call it first with buffer == NULL: it fills the output fields
 * of *plan (plan_bytes is an upper bound then) and returns
 * LB_ERR_WORKSPACE_TOO_SMALL without touching the device beyond reading
 * row_offsets and a sample of col_idx; then call it with a buffer of at
 * least plan_bytes to build.
 * Long rows must have strictly increasing columns (LB_ERR_INVALID_CSR
 * otherwise, checked by the build); short rows have no such requirement.
 *
 * Inputs of lb_spmv_plan_t (0 = default):
 *  block_size, items_per_thread  the short rows' merge path, as for lb_spmv
 *                                (default: 256 x 12 when the columns are
 *                                local and four nonzeros per lane are
 *                                used; else 128 x 8 with two bands and
 *                                128 x 4 with one); W = their product;
 *  x_bands       1 or 2, as for lb_spmv (default: 2 when x has at least
 *                4 MiB and the columns are scattered -- the median column
 *                span of up to 1024 sampled rows exceeds cols / 16 -- else 1);
 *  long_min      rows with at least this many nonzeros are long; at least
 *                W (a long row then never lies strictly inside one merge-path
 *                unit); default max(W, 16 * panels); -1 = no long rows;
 *  panel_cols    columns per panel, a multiple of 64 up to 40960 (float32
 *                x) or 81920 (BF16 x): 160 KiB, the LDS of one compute
 *                unit; default that maximum;
 *  panel_blocks  blocks per panel; default max(1, floor(CUs / panels)) for
 *                the compute units of the device the plan is built on (one
 *                round of one resident block per CU);
 *  vector_width  1 or 4: the short rows' consume loads one or four
 *                consecutive nonzeros per lane and load (4: one band only;
 *                used when col_idx and the values are aligned to their
 *                4-vectors and nnz >= 4, else 1); default 4 when the
 *                columns are local (the sampled median span is at most
 *                cols / 16) and one band is used, else 1;
 *  streams       2: the long rows' launch runs on a second stream
 *                of the same device, owned by the library (one per device,
 *                created on first use, default priority), concurrently with
 *                the short rows' launch; events order it after the work
 *                already on `stream` and before the finishing launch, so
 *                the call stays asynchronous and ordered on `stream` (and
 *                can be captured in a HIP graph from `stream`); calls from
 *                several host threads take turns on that stream.  1: all
 *                launches on `stream` (default).
 * Outputs: the matrix shape and dtype the plan was built for, its counts,
 * plan_bytes (device bytes of the plan) and workspace_bytes (device bytes
 * each lb_spmv_planned call needs). */
typedef struct lb_spmv_plan_t {
    int32_t block_size;
    int32_t items_per_thread;
    int32_t x_bands;
    int32_t long_min;
    int32_t panel_cols;
    int32_t panel_blocks;
    int32_t streams;
    int32_t vector_width;
    lb_dtype_t value_dtype;
    int64_t rows;
    int64_t cols;
    int64_t nnz;
    int64_t long_nnz;    /* nonzeros in long rows */
    int32_t long_rows;   /* rows with at least long_min nonzeros */
    int32_t panels;      /* ceil(cols / panel_cols) */
    int32_t tasks;       /* long-row tasks (one stored sum each) */
    int32_t units;       /* merge-path units of W items over the whole matrix */
    int32_t active_units;/* units holding short-row work */
    size_t plan_bytes;
    size_t workspace_bytes;
    const void *buffer;  /* the device buffer the plan was built in */
} lb_spmv_plan_t;

LB_API lb_status_t lb_spmv_plan_build(const lb_csr_t *A, lb_spmv_plan_t *plan, void *buffer, size_t buffer_bytes,
                                      void *stream);

/* y = A x with a plan built for A's pattern (rows, cols, nnz, value dtype
 * and row_offsets must be those of the build; col_idx those of the build
 * for the long rows).  x of A->value_dtype; y rows float32, overwritten.
 * workspace: at least plan->workspace_bytes of device memory (the carries
 * of the merge-path units, the second column band's row sums and the long
 * rows' task sums), contents on entry irrelevant.  Asynchronous. */
LB_API lb_status_t lb_spmv_planned(const lb_csr_t *A, const lb_spmv_plan_t *plan, const void *x,
                                   lb_dtype_t x_dtype, float *y, void *workspace, size_t workspace_bytes,
                                   void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lb_spmv
 * with the same arguments minus the workspace.  The scratch that lb_spmv
 * takes from its workspace (merge-path split, carries and, with two column
 * bands, the second band's row sums; the work queue's counter) comes from a
 * static device array of LB_NOALLOC_SCRATCH_BYTES per GPU, held from the
 * library's first call on that GPU until the process ends.  A call whose
 * lb_workspace_size(A, s, 1) exceeds it returns LB_ERR_SCRATCH_LIMIT before
 * any launch (the merge-path default needs about 20 bytes per 2048 rows +
 * nonzeros; two column bands add 4 bytes per row: a 2M-row, 65M-nonzero
 * matrix fits).  The call makes no hipMalloc, hipFree or other allocating
 * call; its first call on a GPU looks up that GPU's address of the array.
 * Every call on one GPU shares the array: calls that overlap in time on one
 * GPU (different streams, or host threads) race and give undefined results;
 * calls ordered on one stream are safe.  Same numerics as lb_spmv: for the
 * same schedule the result is bit-identical to lb_spmv's. */
#define LB_NOALLOC_SCRATCH_BYTES (16u << 20)
LB_API lb_status_t lb_spmv_noalloc(const lb_csr_t *A, const void *x, lb_dtype_t x_dtype, float *y,
                                   const lb_schedule_t *s, void *stream);

/* Y = A X with k right-hand sides (Sec. 5.3 SpMM listing, reading its
 * B(nz, col) as B(col_idx[nz], col)).  X row-major cols x k with leading
 * dimension ldx >= k; Y row-major rows x k float32 with ldy >= k,
 * overwritten.  1 <= k <= 64.  Same numerics and workspace rules as lb_spmv
 * (workspace from lb_workspace_size(A, s, k)). */
LB_API lb_status_t lb_spmm(const lb_csr_t *A, const void *X, lb_dtype_t x_dtype, int32_t k,
                           int64_t ldx, float *Y, int64_t ldy, const lb_schedule_t *s,
                           void *workspace, size_t workspace_bytes, void *stream);

/* Backward of y = A x.  dx = A^T dy (cols float32, zeroed by the call and
 * accumulated with float atomics: not bit-reproducible; dx must be
 * coarse-grained device memory) and
 * dvalues[j] = dy[row(j)] * x[col_idx[j]] (nnz float32, a single rounding
 * of the exact product).  Either output may be NULL to skip it.  x is read
 * only for dvalues.  Runs over the merge-path split of A (s->kind must be
 * LB_MERGE_PATH or LB_AUTO); workspace from lb_workspace_size(A, s, 0). */
LB_API lb_status_t lb_spmv_backward(const lb_csr_t *A, const void *x, lb_dtype_t x_dtype,
                                    const float *dy, float *dx, float *dvalues,
                                    const lb_schedule_t *s, void *workspace,
                                    size_t workspace_bytes, void *stream);

/* Backward without atomics, for a pattern reused across calls (a training
 * loop): lb_transpose_pattern builds A^T's pattern once --
 * at_row_offsets[cols + 1], at_col_idx[nnz] (the rows of A) and perm[nnz]
 * (entry p of A^T is entry perm[p] of A).  The result is the canonical
 * CSC of A: a row of A^T lists its entries in their order in A (so by
 * increasing row of A), the same for every build; it is computed by a
 * stable radix sort of the entries by column (digits of at most 7 bits:
 * three passes for cols <= 2^21), with block-local histograms, tiles
 * sorted in LDS and written as runs, and no global atomics.  Workspace from lb_transpose_workspace_size (24 bytes per
 * nonzero plus the histograms).  cols + nnz < 2^31 - 1.
 * lb_spmv_backward_transposed then computes dvalues as lb_spmv_backward
 * does (bit-exact) and dx = A^T dy by the merge-path SpMV on A^T, which
 * reads the current values of A through perm (a gather, no atomics, no
 * permuted copy); dx is bit-reproducible (the transpose is canonical).  s as for
 * lb_spmv_backward (merge-path block_size / items_per_thread); workspace
 * from lb_backward_transposed_workspace_size. */
LB_API lb_status_t lb_transpose_workspace_size(const lb_csr_t *A, size_t *bytes);
LB_API lb_status_t lb_transpose_pattern(const lb_csr_t *A, int32_t *at_row_offsets, int32_t *at_col_idx,
                                        int32_t *perm, void *workspace, size_t workspace_bytes, void *stream);
LB_API lb_status_t lb_backward_transposed_workspace_size(const lb_csr_t *A, const lb_schedule_t *s,
                                                         size_t *bytes);
LB_API lb_status_t lb_spmv_backward_transposed(const lb_csr_t *A, const int32_t *at_row_offsets,
                                               const int32_t *at_col_idx, const int32_t *perm, const void *x,
                                               lb_dtype_t x_dtype, const float *dy, float *dx, float *dvalues,
                                               const lb_schedule_t *s, void *workspace, size_t workspace_bytes,
                                               void *stream);

/* Workspace bytes for lb_batched_spmm with k right-hand sides.  Host-only. */
LB_API lb_status_t lb_batched_workspace_size(const lb_batch_t *B, const lb_schedule_t *s,
                                             int32_t k, size_t *bytes);

/* For every matrix b of the batch, Y_b = A_b X_b.  X holds the matrices'
 * right-hand sides back to back, row-major total_cols x k; Y row-major
 * total_rows x k float32, overwritten.  One launch splits the single merge
 * path of sum(m_b + nnz_b) items into units, one persistent launch (Sec. 5.1
 * persistent ranges) consumes every unit of every matrix, and one launch
 * adds the carries (per pass of up to 8 columns).  s->kind must be
 * LB_MERGE_PATH or LB_AUTO.  1 <= k <= 64. */
LB_API lb_status_t lb_batched_spmm(const lb_batch_t *B, const void *X, lb_dtype_t x_dtype,
                                   int32_t k, float *Y, const lb_schedule_t *s, void *workspace,
                                   size_t workspace_bytes, void *stream);

/* The merge-path split (Sec. 5.2.1): for t in [0, num_units], the number of
 * row ends out_row[t] and of nonzeros out_nz[t] that precede diagonal
 * d_t = min(t * items_per_unit, rows + nnz) of the merge of the row-end list
 * row_offsets[1..rows] with the nonzero indices 0..nnz-1, where row end r is
 * taken before nonzero j when row_offsets[r+1] <= j.  Device arrays;
 * out_row/out_nz hold num_units + 1 int32 each. */
LB_API lb_status_t lb_merge_path_partition(const int32_t *row_offsets, int64_t rows, int64_t nnz,
                                           int64_t items_per_unit, int64_t num_units,
                                           int32_t *out_row, int32_t *out_nz, void *stream);

/* Group-mapped tile lookup (Sec. 5.2.3 get_tile): for groups of
 * tiles_per_group consecutive tiles of A, write for every nonzero j the
 * index, within its group, of the tile that owns it, found by binary search
 * in the group's LDS prefix sum of tile sizes.  owner: nnz int32, device.
 * tiles_per_group must be a power of two in [2, 1024]. */
LB_API lb_status_t lb_group_tile_owner(const lb_csr_t *A, int32_t tiles_per_group, int32_t *owner,
                                       void *stream);

/* Time candidate schedules for A with k right-hand sides on `stream`
 * (synchronizing) using the caller's x/X, y/Y and workspace (at least
 * lb_autotune_workspace_size bytes), store the fastest in a process-wide
 * cache and return it in *best.  A cache entry is keyed by the shape, k,
 * the value dtype and a fingerprint of the sparsity pattern (Sec. 6.2
 * picks a schedule per matrix), and belongs to the device it was timed on
 * (lb_autotune_device_tag) and to this ABI version.  The call also binds A
 * (its row_offsets and col_idx pointers and shape) to the fingerprint, so
 * LB_AUTO on A resolves to the stored pick; a matrix without a binding
 * gets the Sec. 6.2 rule.  If the environment variable LB_AUTOTUNE_CACHE
 * names a file, the cache is loaded from it (entries of this device and ABI
 * version; others are kept in the file untouched) and saved to it. */
LB_API lb_status_t lb_autotune_workspace_size(const lb_csr_t *A, int32_t k, size_t *bytes);
LB_API lb_status_t lb_autotune(const lb_csr_t *A, const void *X, lb_dtype_t x_dtype, int32_t k,
                               float *Y, void *workspace, size_t workspace_bytes,
                               lb_schedule_t *best, void *stream);

/* The pattern fingerprint the tuning cache uses: FNV-1a (64-bit) over rows,
 * cols, nnz, every row offset and col_idx at 4096 evenly spaced positions.
 * Synchronizes `stream`.  Values do not enter it. */
LB_API lb_status_t lb_pattern_fingerprint(const lb_csr_t *A, uint64_t *fingerprint, void *stream);

/* Host only: bind A to `fingerprint` (so LB_AUTO on A uses a tuned pick for
 * it) and report whether the cache holds one for k right-hand sides:
 * *found = 1 and *out = the pick, or *found = 0.  With a cache file this
 * reuses an earlier process's tuning at the cost of one fingerprint. */
LB_API lb_status_t lb_autotune_lookup(const lb_csr_t *A, int32_t k, uint64_t fingerprint, int32_t *found,
                                      lb_schedule_t *out);

/* The device identity tuning entries are stored under: "<arch>:<CUs>" of the
 * current device (e.g. "gfx950:256"), "none:0" without a device. */
LB_API const char *lb_autotune_device_tag(void);

/* Same for a batch (merge-path items_per_thread and block_size). */
LB_API lb_status_t lb_batched_autotune(const lb_batch_t *B, const void *X, lb_dtype_t x_dtype,
                                       int32_t k, float *Y, void *workspace,
                                       size_t workspace_bytes, lb_schedule_t *best, void *stream);

/* Forget every tuned schedule and binding (process-wide). */
LB_API void lb_autotune_clear(void);

/* Debug check of the device-only CSR preconditions; synchronizes `stream`.
 * Returns LB_OK or LB_ERR_INVALID_CSR. */
LB_API lb_status_t lb_validate_csr(const lb_csr_t *A, void *stream);

/* ---- Other tile sets (Sec. 3.1 names CSR, CSC and COO; Sec. 5.2.1: a
 * format needs only an iterator counting atoms per tile).
 *
 * COO: y = A x (rows float32, overwritten; rows without entries get 0),
 * x of A->value_dtype.  LB_MERGE_PATH (as for CSR: block_size 128/256/512,
 * items_per_thread 4/8/12/16): entry j is the (j + row_idx[j])-th item of
 * the merge of row ends and entries, so the split is one search over the
 * entries and equals the CSR split of the same matrix; consume and carry
 * fix-up as for CSR, bit-reproducible.  LB_THREAD_MAPPED and LB_GROUP_MAPPED
 * (tiles_per_group 1, group_size a power of two in [8, 1024]) find each
 * row's entries by binary search of row_idx.  LB_AUTO = the Sec. 6.2 rule.
 * rows + nnz < 2^31 - 1.  Workspace from lb_coo_workspace_size. */
LB_API lb_status_t lb_coo_workspace_size(const lb_coo_t *A, const lb_schedule_t *s, size_t *bytes);
LB_API lb_status_t lb_spmv_coo(const lb_coo_t *A, const void *x, lb_dtype_t x_dtype, float *y,
                               const lb_schedule_t *s, void *workspace, size_t workspace_bytes,
                               void *stream);

/* The COO merge-path split (test hook): out_row[t], out_nz[t] for t in
 * [0, num_units] at diagonals min(t * items_per_unit, rows + nnz). */
LB_API lb_status_t lb_coo_merge_path_partition(const int32_t *row_idx, int64_t rows, int64_t nnz,
                                               int64_t items_per_unit, int64_t num_units,
                                               int32_t *out_row, int32_t *out_nz, void *stream);

/* CSC: y = A x with columns as tiles: entry j adds values[j] * x[c] into
 * y[row_idx[j]].  x is float32 (values float32 or BF16); y (rows float32,
 * coarse-grained device memory) is zeroed by the call and accumulated with
 * float atomics, so it is not bit-reproducible run to run.  Each block first sums its unit's products
 * per row in LDS, so a row hit from many columns costs one atomic per
 * block.  LB_MERGE_PATH or LB_AUTO (the merge-path split of the columns;
 * block_size/items_per_thread as for CSR, default 512 x 8 here: larger
 * units combine more).  cols + nnz < 2^31 - 1.  Workspace from
 * lb_csc_workspace_size. */
LB_API lb_status_t lb_csc_workspace_size(const lb_csc_t *A, const lb_schedule_t *s, size_t *bytes);
LB_API lb_status_t lb_spmv_csc(const lb_csc_t *A, const void *x, lb_dtype_t x_dtype, float *y,
                               const lb_schedule_t *s, void *workspace, size_t workspace_bytes,
                               void *stream);

/* ---- Sparse matrix-matrix product C = A B (Gustavson; Sec. 5.3 names it as
 * the extension of SpMM: a kernel sizing each output row, an allocation, a
 * multiply kernel).  A is rows x cols, B is A->cols x n (B->rows must equal
 * A->cols), both float32.  Row i of C holds every column reached by a
 * product A[i, j] * B[j, c], ascending (structural: kept even if the sum is
 * 0), with value sum_j A[i, j] * B[j, c] in float32.  Rows are accumulated
 * by product count: up to 32 products an 8-lane group, up to 256 one
 * wavefront, up to 4096 one block
 * (both sort (column, product index) in LDS and sum in product order:
 * deterministic), beyond that a dense slot per block of a work queue (float
 * atomics: summation order varies run to run).
 * lb_spgemm_count (synchronizing) writes C's row offsets (A->rows + 1,
 * device) and *c_nnz (host); the caller allocates col_idx and values of
 * *c_nnz entries; lb_spgemm_compute fills them.  Both take the workspace of
 * lb_spgemm_workspace_size (contents on entry irrelevant): per-row counts
 * and tier lists (about 40 bytes per row of A) plus the large-row slots, a
 * dense float accumulator and bitmap over B's columns each, as many as
 * 1 GiB holds (32 to 512 slots).  nnz(C) must fit int32 (else
 * LB_ERR_OVERFLOW from the count). */
LB_API lb_status_t lb_spgemm_workspace_size(const lb_csr_t *A, const lb_csr_t *B, size_t *bytes);
LB_API lb_status_t lb_spgemm_count(const lb_csr_t *A, const lb_csr_t *B, int32_t *c_row_offsets, int64_t *c_nnz,
                                   void *workspace, size_t workspace_bytes, void *stream);
LB_API lb_status_t lb_spgemm_compute(const lb_csr_t *A, const lb_csr_t *B, const int32_t *c_row_offsets,
                                     int32_t *c_col_idx, float *c_values, void *workspace, size_t workspace_bytes,
                                     void *stream);

/* ---- Graph traversal on the same schedules (Sec. 5.3 SSSP example; BFS,
 * named in Sec. 6).
 * The graph G is a square CSR read as adjacency: vertex u's out-edges are
 * the atoms of tile u, edge j goes to col_idx[j] and (SSSP) weighs
 * values[j], float32 and >= 0 (negative or NaN weights are undefined
 * behaviour; the oracle-checked result assumes them absent).
 * Each iteration takes the current frontier (a device list of vertex ids:
 * an indexed tile set) and relaxes every out-edge of its vertices under the
 * schedule s; the vertices that improve form the next frontier, each listed
 * once.  The host launches again while the frontier holds vertices (Sec. 5.3), reading
 * the frontier size from the device once per batch of iterations, so these
 * calls synchronize `stream`.
 * Schedules: LB_THREAD_MAPPED (a thread per frontier vertex, block_size as
 * for SpMV), LB_WORK_QUEUE (group_size in [8, 1024]: frontier chunks handed
 * out by a device work queue), LB_GROUP_MAPPED with group_size a power of two in [8, 1024]
 * and tiles_per_group 1 (a group per vertex) or group_size (LDS prefix sum
 * and get_tile over the group's vertices), LB_AUTO = the rule of Sec. 6.2
 * as for SpMV (merge-path unless (rows < 500 or cols < 500) and
 * nnz < 10000; then thread-mapped, or group-mapped with at least 8 lanes).
 * LB_MERGE_PATH (256 threads x 8
 * merge items per unit; other block_size / items_per_thread values return
 * LB_ERR_UNSUPPORTED): per iteration the frontier's out-degrees are
 * prefix-summed on the device, the merge of those offsets with the
 * frontier's edges is split into equal units (Sec. 5.2.1) and a persistent
 * launch walks them.  grid_size 0 = the resident grid (CUs x occupancy).
 * max_iterations 0 = rows + 1 (enough for any graph with weights >= 0); a
 * frontier still non-empty after max_iterations returns
 * LB_ERR_NOT_CONVERGED (the outputs then hold upper bounds).
 * *iterations (host, may be NULL) receives the number of non-empty
 * frontiers processed.  source in [0, rows). */

/* Workspace bytes for lb_sssp / lb_bfs on G (about 4 * rows int32, plus the
 * merge-path split over at most rows + nnz items).  Host-only. */
LB_API lb_status_t lb_traversal_workspace_size(const lb_csr_t *G, size_t *bytes);

/* Single-source shortest paths: dist (rows float32, overwritten) receives
 * the least solution of dist[source] = 0, dist[v] = min over edges (u, v, w)
 * of fl32(dist[u] + w): every offer is one float32 addition and the kept
 * value an atomic minimum, so the result is unique (bit-exact, any
 * schedule, any run); +inf where no path exists.  G->value_dtype must be
 * LB_F32. */
LB_API lb_status_t lb_sssp(const lb_csr_t *G, int64_t source, float *dist, const lb_schedule_t *s,
                           int32_t max_iterations, int32_t *iterations, void *workspace,
                           size_t workspace_bytes, void *stream);

/* Breadth-first search: depth (rows int32, overwritten) receives the least
 * number of edges from source, -1 where unreachable.  G->values is not read
 * (may be NULL). */
LB_API lb_status_t lb_bfs(const lb_csr_t *G, int64_t source, int32_t *depth, const lb_schedule_t *s,
                          int32_t max_iterations, int32_t *iterations, void *workspace,
                          size_t workspace_bytes, void *stream);

/* Measurement hooks (not part of the method): the ceilings a kernel of this
 * library is compared with.
 *  lb_probe_stream_read: reads `bytes` (a multiple of 16, 16-byte aligned
 *    device buffer) with non-temporal 16-byte loads and writes one partial
 *    sum per thread to out[grid * 256] (grid = 0 picks CUs x 8); the
 *    streaming-read ceiling of HBM.
 *  lb_probe_gather: sum over j of x[idx[j]] for j in [0, n), x of cols
 *    floats, one partial sum per thread to out[grid * 256]; with a matrix's
 *    col_idx as idx it times the x gather alone, the floor of an SpMV kernel
 *    on that matrix that gathers the same way.  bands = 1: idx read
 *    non-temporally in a grid stride over all XCDs; bands = 2, 4 or 8: the
 *    gather of a banded merge path (x_bands = 2): chunks of 2048 entries go
 *    to `bands` blocks on different XCDs, each reading the whole chunk and
 *    gathering only the entries of its band of x (columns [b * cb, (b + 1) *
 *    cb), cb = ceil(cols / bands)), XCD x serving band x mod bands (grid
 *    rounded down to a multiple of 8, at least 8).
 *  lb_probe_copy: copies `bytes` (a multiple of 16, both buffers 16-byte
 *    aligned, not overlapping) from src to dst with 16-byte loads and
 *    stores; a copy of known size under this kernel's own name, against
 *    which hardware traffic counters are calibrated.
 * All are asynchronous on `stream`; idx values must lie in [0, cols). */
LB_API lb_status_t lb_probe_stream_read(const void *buf, size_t bytes, float *out, int32_t grid, void *stream);
LB_API lb_status_t lb_probe_copy(const void *src, void *dst, size_t bytes, void *stream);
LB_API lb_status_t lb_probe_gather(const int32_t *idx, int64_t n, const float *x, int64_t cols, float *out,
                                   int32_t grid, int32_t bands, void *stream);
LB_API int32_t lb_probe_default_grid(void);

/* Kernel timing.  While enabled, every launch made by this library records a
 * pair of HIP events on its stream.  lb_profile_read synchronizes those
 * events and returns, for the kernel family `name` ("merge_partition",
 * "merge_consume", "merge_fixup", "thread_mapped", "group_mapped",
 * "backward", "batched_consume", "batched_fixup", "fill", "coo_partition",
 * "coo_consume", "coo_fixup", "coo_tiles", "transpose", "merge_finish",
 * "spgemm_products", "spgemm_count_t0" .. "spgemm_count_t3",
 * "spgemm_compute_t0" .. "spgemm_compute_t3" (one per row tier),
 * "work_queue", "traversal_init",
 * "sssp_advance", "bfs_advance"), the summed
 * duration in milliseconds and the launch count since the last reset. */
LB_API void lb_profile_enable(int on);
LB_API void lb_profile_reset(void);
LB_API lb_status_t lb_profile_read(const char *name, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
