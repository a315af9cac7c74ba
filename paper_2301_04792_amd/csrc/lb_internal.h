// Host-side interface between the C ABI (lb_api.cpp) and the kernel files.
// Every launcher enqueues work on `stream` and returns the launch status; it
// assumes its arguments were validated by the caller.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lb.h"

namespace lbk {

struct csr_dev {
    int32_t rows, cols, nnz;
    const int32_t *ro;
    const int32_t *ci;
    const void *val;
    lb_dtype_t dt;
};

// ---- kernel timing (lb_profile_*) ---------------------------------------------------
bool profiling_enabled();
void profile_mark(hipStream_t s, const char *name, bool begin);

struct prof_scope {
    hipStream_t s;
    const char *name;
    bool on;
    prof_scope(hipStream_t st, const char *n) : s(st), name(n), on(profiling_enabled()) {
        if (on) profile_mark(s, name, true);
    }
    ~prof_scope() {
        if (on) profile_mark(s, name, false);
    }
};

inline size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Instantiated merge-path configurations (block_size, items_per_thread).
#define LB_MERGE_CONFIGS(X) \
    X(128, 4) X(128, 8) X(128, 12) X(128, 16) \
    X(256, 4) X(256, 8) X(256, 12) X(256, 16) \
    X(512, 4) X(512, 8) X(512, 12) X(512, 16)

// ---- merge-path split ---------------------------------------------------------------
// Work units of W merge items; T = ceil((rows + nnz) / W) units.
inline int64_t merge_units(int64_t rows, int64_t nnz, int64_t W) { return (rows + nnz + W - 1) / W; }
// Up to this many units a one-band lb_spmv runs as one launch whose blocks
// find their own split and own whole rows (a row longer than a unit is
// summed by the block where it closes, at most kSelfSplitUnits * W
// nonzeros): one block per CU at most.
constexpr int64_t kSelfSplitUnits = 256;

// Workspace: part_i[T+1], part_j[T+1], carry_row[T], carry_val[T * kc].
struct merge_ws {
    int32_t *part_i;
    int32_t *part_j;
    int32_t *carry_row;
    float *carry_val;
};
inline size_t merge_ws_bytes(int64_t T, int kc) {
    return 2 * align256(static_cast<size_t>(T + 1) * 4) + align256(static_cast<size_t>(T) * 4) +
           align256(static_cast<size_t>(T) * 4 * kc);
}
// Two column bands: carries for 2T (unit, band) pairs, then the second
// band's row sums (rows floats).
inline size_t merge_banded_ws_bytes(int64_t T, int64_t rows) {
    return merge_ws_bytes(2 * T, 1) + align256(static_cast<size_t>(rows) * 4);
}
inline merge_ws merge_ws_carve(void *base, int64_t T) {
    char *p = static_cast<char *>(base);
    merge_ws w;
    w.part_i = reinterpret_cast<int32_t *>(p);
    p += align256(static_cast<size_t>(T + 1) * 4);
    w.part_j = reinterpret_cast<int32_t *>(p);
    p += align256(static_cast<size_t>(T + 1) * 4);
    w.carry_row = reinterpret_cast<int32_t *>(p);
    p += align256(static_cast<size_t>(T) * 4);
    w.carry_val = reinterpret_cast<float *>(p);
    return w;
}

// The split at every unit boundary.  With row_base (a batch's int64 row
// prefix sums, count + 1 entries) it also writes part_mat[t], the matrix
// owning row min(part_i[t], rows - 1).
hipError_t merge_partition(const int32_t *ro, int32_t rows, int32_t nnz, int32_t W, int32_t T,
                           int32_t *part_i, int32_t *part_j, hipStream_t s, const int64_t *row_base = nullptr,
                           int32_t count = 0, int32_t *part_mat = nullptr);

// True if (block, items) is an instantiated merge-path configuration.
bool merge_config_supported(int block, int items);

// Deterministic carry fix-up: for each run of equal carry_row entries (rows
// < rows only), adds the run's carry_val sums (kc columns, row-major with
// leading dimension ldy) to y.
hipError_t launch_fixup(int64_t T, int32_t rows, int32_t kc, const int32_t *carry_row,
                        const float *carry_val, float *y, int64_t ldy, hipStream_t s, const char *tag);

// bands 1 or 2 (column bands of x, one per half of the XCDs); the workspace
// is merge_ws_bytes(T, 1) for one band, merge_banded_ws_bytes(T, rows) for two.
// With vperm (one band), nonzero j's value is A.val[vperm[j]] and x is float32.
// vec 4 (one band, no vperm): four consecutive nonzeros per lane and load;
// the one-nonzero form runs instead when nnz < 4 or col_idx / values are
// not aligned to their vectors.
hipError_t merge_spmv(const csr_dev &A, const void *x, float *y, int block, int items, int bands, void *ws,
                      hipStream_t s, const int32_t *vperm = nullptr, int vec = 1);

// ---- planned SpMV (k_plan.hip) ----------------------------------------------------------
// Long rows: a block of kPanelBlock threads stages kPanelBytes of x (one
// panel, the whole 160 KiB LDS of a CU: one resident block per CU, 16
// wavefronts) in LDS, R blocks per panel; a task is at most kPanelTask nonzeros
// of one (row, panel) segment (252: any such range lies in 64 aligned groups
// of four); a task of at most G groups runs on G lanes (G = 64, 32, 16, 8:
// its class), one group per lane; a wavefront works on kPanelBatch steps of
// 64 / G tasks at a time.
constexpr int kPanelBlock = 1024;
constexpr int kPanelTask = 252;
constexpr int kPanelBatch = 4;
constexpr int kPanelBytes = 163840;
constexpr int kPanelClasses = 4;
// The class of a task spanning ng aligned groups: G = 64 >> class.
inline int panel_class(int64_t ng) { return ng > 32 ? 0 : (ng > 16 ? 1 : (ng > 8 ? 2 : 3)); }

// An active unit of the short rows' merge path, as its block needs it: the
// split at both ends, the nonzeros whose products it sums [ja, jb), the
// first nonzero h0 of row i0's head [h0, j0) (h0 = j0: none) and flags
// (bit 0: row i0 is long, its y is not this block's; bit 1: every row that
// closes in the unit has at most kRowPerThreadMax of its nonzeros in it).
struct alignas(16) plan_unit {
    int32_t i0, i1, j0, j1, ja, jb, h0, flags;
};
constexpr int kRowPerThreadMax = 16;

// A task: nonzeros [a0, a0 + len) of one segment; its sum goes to part[out].
struct alignas(16) panel_task {
    int32_t a0, len, out, pad;
};

// The plan as the kernels see it (device pointers into the plan buffer).
struct plan_dev {
    int32_t rows;
    int32_t T, NA;       // merge-path units, active units
    int32_t NL, NP;      // long rows, panels
    int32_t R;           // blocks per panel
    int32_t P;           // columns per panel
    int32_t long_min;
    int32_t bands, block, items;
    int32_t vec;         // 4: the short rows' consume loads four nonzeros per lane (one band)
    int32_t streams;     // 2: the long rows' launch on the library's second stream
    int32_t ntasks;
    const int32_t *part_i, *part_j;  // the split at every unit boundary, T + 1 each (written by the build)
    const plan_unit *units;          // NA records, one per active unit, in unit order
    const int32_t *LR;               // NL long row ids, ascending
    const uint32_t *long_bits;       // ceil(rows / 32) words: bit r % 32 of word r / 32 set for a long row r
    const int32_t *row_task;         // NL + 1: long row q's task sums are part[row_task[q] .. row_task[q + 1])
    const int32_t *pcls_off;         // NP * 4 + 1: panel p's class-k tasks are [pcls_off[4p + k], pcls_off[4p + k + 1])
    const panel_task *tasks;         // ntasks, grouped by panel, then class
};

// Plan buffer: a 256-byte header (build flags), then the tables above, each
// 256-byte aligned; NA_cap entries are reserved for the unit records and
// ntask_cap for the tasks (the last table); the split (part_i, part_j) and
// sb (NL x (NP + 1) segment bounds) are written by the build on the device
// and read back.
struct plan_layout {
    size_t flags, part_i, part_j, units, LR, long_bits, row_task, pcls_off, tasks, sb, total;
};
inline plan_layout plan_layout_of(int64_t T, int64_t NA_cap, int64_t NL, int64_t NP, int64_t ntask_cap,
                                  int64_t rows) {
    plan_layout L{};
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t at = o;
        o += align256(bytes);
        return at;
    };
    L.flags = take(4);
    L.part_i = take(static_cast<size_t>(T + 1) * 4);
    L.part_j = take(static_cast<size_t>(T + 1) * 4);
    L.units = take(static_cast<size_t>(NA_cap) * sizeof(plan_unit));
    L.LR = take(static_cast<size_t>(NL) * 4);
    L.long_bits = take(static_cast<size_t>((rows + 31) / 32) * 4);
    L.row_task = take(static_cast<size_t>(NL + 1) * 4);
    L.pcls_off = take(static_cast<size_t>(NP * kPanelClasses + 1) * 4);
    L.sb = take(static_cast<size_t>(NL) * (NP + 1) * 4);
    L.tasks = take(static_cast<size_t>(ntask_cap) * sizeof(panel_task));  // last: no other offset depends on it
    L.total = o;
    return L;
}

// Per-call workspace: y_hi[rows] (two bands), part[ntasks].
struct plan_ws {
    float *y_hi;
    float *part;
};
inline size_t plan_ws_bytes(int bands, int64_t rows, int64_t ntasks) {
    return (bands == 2 ? align256(static_cast<size_t>(rows) * 4) : 0) + align256(static_cast<size_t>(ntasks) * 4);
}
inline plan_ws plan_ws_carve(void *base, const plan_dev &pl) {
    char *p = static_cast<char *>(base);
    plan_ws w{};
    if (pl.bands == 2) {
        w.y_hi = reinterpret_cast<float *>(p);
        p += align256(static_cast<size_t>(pl.rows) * 4);
    }
    w.part = reinterpret_cast<float *>(p);
    return w;
}

// True if P columns per panel are supported for x of type xt.
bool panel_cols_ok(int64_t P, lb_dtype_t xt);
// Segment bounds of the long rows (flags bit 0: a long row's columns do not strictly increase).
hipError_t plan_segments_launch(int32_t NL, int32_t NP, int32_t P, const int32_t *LR, const int32_t *ro,
                                const int32_t *ci, int32_t *sb, int32_t *flags, hipStream_t s);
// The short rows' merge-path consume over the active units (k_merge.hip).
hipError_t merge_spmv_planned_consume(const csr_dev &A, const plan_dev &pl, const void *x, float *y, float *y_hi,
                                      hipStream_t s);
// y = A x with a built plan; ws holds plan_ws_bytes(...).
hipError_t planned_spmv(const csr_dev &A, const plan_dev &pl, const void *x, float *y, void *ws, hipStream_t s);

hipError_t merge_spmm(const csr_dev &A, const void *X, int32_t k, int64_t ldx, float *Y, int64_t ldy,
                      int block, int items, void *ws, hipStream_t s);

// combine_dx (dx only): products are summed per target in LDS before the
// global atomics (for scatters whose targets repeat within a unit).
hipError_t merge_backward(const csr_dev &A, const void *x, const float *dy, float *dx, float *dvalues,
                          int block, int items, void *ws, hipStream_t s, bool combine_dx = false);

// ---- batched ------------------------------------------------------------------------
struct batch_dev {
    int32_t count, total_rows, total_cols, total_nnz;
    const int32_t *ro;
    const int32_t *ci;
    const void *val;
    lb_dtype_t dt;
    const int64_t *row_base;
    const int64_t *nnz_base;
    const int64_t *col_base;
};
size_t batched_ws_bytes(const batch_dev &B, int block, int items, int k);
hipError_t batched_spmm(const batch_dev &B, const void *X, int32_t k, float *Y, int block, int items,
                        void *ws, hipStream_t s);

// ---- thread- and group-mapped ---------------------------------------------------------
hipError_t thread_mapped_spmv(const csr_dev &A, const void *x, float *y, int block, int grid,
                              hipStream_t s);
hipError_t thread_mapped_spmm(const csr_dev &A, const void *X, int32_t k, int64_t ldx, float *Y,
                              int64_t ldy, int block, int grid, hipStream_t s);
// ticket non-null: the work-queue form (tiles_per_group == group_size, a
// persistent grid claiming rounds from *ticket, which the call zeroes first).
hipError_t group_mapped_spmv(const csr_dev &A, const void *x, float *y, int group_size,
                             int tiles_per_group, int grid, int32_t *ticket, hipStream_t s);
hipError_t group_tile_owner(const csr_dev &A, int tiles_per_group, int32_t *owner, hipStream_t s);

// ---- transposed backward (k_transpose.hip) ------------------------------------------------
// Workspace of transpose_pattern (ranks and scan tile sums).
size_t transpose_ws_bytes(int64_t cols, int64_t nnz);
// A^T's offsets (cols + 1), column indices (= rows of A) and the A entry of each A^T entry.
hipError_t transpose_pattern(const csr_dev &A, int32_t *at_ro, int32_t *at_ci, int32_t *perm, void *ws,
                             hipStream_t s);
size_t backward_transposed_ws_bytes(int64_t rows, int64_t cols, int64_t nnz, int block, int items);
// dvalues (dvalues-only merge pass over A) and dx = A^T dy (merge-path SpMV on A^T reading A's values through perm).
hipError_t backward_transposed(const csr_dev &A, const int32_t *at_ro, const int32_t *at_ci, const int32_t *perm,
                               const void *x, const float *dy, float *dx, float *dvalues, int block, int items,
                               void *ws, hipStream_t s);

// ---- SpGEMM (k_spgemm.hip) ---------------------------------------------------------------
// C = A B with A m x k and B k x n (float32 values).
struct spgemm_dev {
    int32_t m, k, n, a_nnz;
    const int32_t *a_ro, *a_ci;
    const float *a_val;
    const int32_t *b_ro, *b_ci;
    const float *b_val;
};
// Blocks of the large-row tier, each with a dense n-column slot (n floats and
// n / 32 + n / 1024 bitmap words): as many as 1 GiB holds, from 32 to 512.
inline int64_t spgemm_slots(int64_t n) {
    const int64_t per = n * 4 + ((n + 31) / 32 + ((n + 31) / 32 + 31) / 32) * 4 + 512;
    const int64_t s = (int64_t(1) << 30) / (per > 0 ? per : 1);
    return s < 32 ? 32 : (s > 512 ? 512 : s);
}
size_t spgemm_ws_bytes(int64_t m, int64_t n);
// Per-row column counts turned into C's row offsets (m + 1, int32 where the
// total fits); *total_host receives nnz(C).  Synchronizes s.
hipError_t spgemm_count(const spgemm_dev &P, int32_t *c_ro, int64_t *total_host, void *ws, hipStream_t s);
hipError_t spgemm_compute(const spgemm_dev &P, const int32_t *c_ro, int32_t *c_ci, float *c_val, void *ws,
                          hipStream_t s);

// ---- COO and CSC ---------------------------------------------------------------------------
// A row-sorted COO matrix: row_idx[nnz] non-decreasing, col_idx[nnz], values[nnz].
struct coo_dev {
    int32_t rows, cols, nnz;
    const int32_t *ri;
    const int32_t *ci;
    const void *val;
    lb_dtype_t dt;
};
// The merge-path split of a COO (bit-equal to the CSR split of the same matrix).
hipError_t coo_partition(const int32_t *row_idx, int32_t rows, int32_t nnz, int32_t W, int32_t T, int32_t *part_i,
                         int32_t *part_j, hipStream_t s);
// kind: LB_MERGE_PATH (block/items a LB_MERGE_CONFIGS pair, workspace merge_ws_bytes(T, 1)),
// LB_THREAD_MAPPED (block threads) or LB_GROUP_MAPPED (group lanes, one row per group).
hipError_t coo_spmv(const coo_dev &A, const void *x, float *y, lb_sched_kind_t kind, int group, int block, int items,
                    int grid, void *ws, hipStream_t s);

// ---- graph traversal (SSSP, BFS) ---------------------------------------------------------
#define LB_TRAVERSAL_GROUPS(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024)

struct trav_cfg {
    lb_sched_kind_t kind;  // LB_THREAD_MAPPED, LB_GROUP_MAPPED, LB_MERGE_PATH or LB_WORK_QUEUE
    int group;             // group-mapped: lanes per group
    int tiles_per_group;   // group-mapped: 1 or group
    int block;             // thread-mapped: threads per block
    int grid;              // 0 = resident grid
};

// Merge-path units of a frontier: at most (n + nnz) merge items of 2048.
inline int64_t trav_merge_units(int64_t n, int64_t nnz) { return (n + nnz + 2047) / 2048; }

// Workspace: stamp[n], two frontier queues of n vertex ids, counters (three
// rotating frontier sizes, the count of non-empty frontiers, two rotating
// work-queue tickets);
// for merge-path also the frontier's offsets[n + 1], per-tile degree sums,
// {E_f, T_f} and the split at every unit boundary.
struct trav_ws {
    int32_t *stamp;
    int32_t *queue[2];
    int32_t *counters;
    int32_t *offs;
    int32_t *tile_sum;
    int32_t *meta;
    int32_t *part_i;
    int32_t *part_j;
};
inline size_t trav_ws_bytes(int64_t n, int64_t nnz) {
    const size_t q = align256(static_cast<size_t>(n) * 4);
    const size_t units = static_cast<size_t>(trav_merge_units(n, nnz)) + 1;
    return 3 * q + 256 + align256(static_cast<size_t>(n + 1) * 4) + align256(static_cast<size_t>(n / 2048 + 2) * 4) +
           256 + 2 * align256(units * 4);
}
inline trav_ws trav_ws_carve(void *base, int64_t n, int64_t nnz) {
    char *p = static_cast<char *>(base);
    const size_t q = align256(static_cast<size_t>(n) * 4);
    const size_t units = static_cast<size_t>(trav_merge_units(n, nnz)) + 1;
    trav_ws w;
    w.stamp = reinterpret_cast<int32_t *>(p);
    w.queue[0] = reinterpret_cast<int32_t *>(p + q);
    w.queue[1] = reinterpret_cast<int32_t *>(p + 2 * q);
    w.counters = reinterpret_cast<int32_t *>(p + 3 * q);
    p += 3 * q + 256;
    w.offs = reinterpret_cast<int32_t *>(p);
    p += align256(static_cast<size_t>(n + 1) * 4);
    w.tile_sum = reinterpret_cast<int32_t *>(p);
    p += align256(static_cast<size_t>(n / 2048 + 2) * 4);
    w.meta = reinterpret_cast<int32_t *>(p);
    p += 256;
    w.part_i = reinterpret_cast<int32_t *>(p);
    p += align256(units * 4);
    w.part_j = reinterpret_cast<int32_t *>(p);
    return w;
}
bool traversal_group_supported(int g);
// Synchronize s (the host reads the frontier size once per batch of
// iterations).  *converged is false when max_iter iterations left a frontier.
hipError_t sssp(const csr_dev &G, int32_t source, float *dist, const trav_cfg &c, int32_t max_iter,
                int32_t *iterations, bool *converged, void *ws, hipStream_t s);
hipError_t bfs(const csr_dev &G, int32_t source, int32_t *depth, const trav_cfg &c, int32_t max_iter,
               int32_t *iterations, bool *converged, void *ws, hipStream_t s);

// ---- measurement probes -----------------------------------------------------------------
hipError_t probe_stream_read(const void *buf, size_t bytes, float *out, int grid, hipStream_t s);
hipError_t probe_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
hipError_t probe_gather(const int32_t *idx, int64_t n, const float *x, int32_t cb, float *out, int grid, int bands,
                        hipStream_t s);

// ---- utilities ------------------------------------------------------------------------
hipError_t fill_f32(float *p, int64_t n, float v, hipStream_t s);
// out[i] = a[i * n / count] for i < count (0 when n == 0).
hipError_t gather_samples(const int32_t *a, int64_t n, int32_t count, int32_t *out, hipStream_t s);
// out[i] = a[pos[i]] for i < count (device arrays).
hipError_t gather_at(const int32_t *a, const int32_t *pos, int32_t count, int32_t *out, hipStream_t s);
// Writes violation flags (bit 0: offsets, bit 1: columns) into *flags_dev.
hipError_t validate_csr(const csr_dev &A, int32_t *flags_dev, hipStream_t s);

}  // namespace lbk
