// SpMV on the other tile sets the paper's library carries (Sec. 3.1: CSR,
// CSC, COO).  Merge-path needs only a way to count atoms per tile
// (Sec. 5.2.1), so the CSR machinery carries over:
//
//  * COO, sorted by row.  Nonzero j is the (j + row_idx[j])-th item of the
//    same merge of row ends and nonzeros that CSR uses, so the split at a
//    diagonal is one search over the nonzeros (group_coo_search) and equals
//    the CSR split of the same matrix bit for bit.  The consume stages the
//    unit's row indices in LDS and derives each of its rows' ends from them
//    (upper_bound), then runs the CSR consume's walk, block segmented scan
//    and carries; the CSR fix-up completes rows cut by unit boundaries.
//    Thread- and group-mapped run on coo_tile_set (lb_schedule.hpp), whose
//    atoms-per-tile iterator is a binary search of the row indices.
//  * CSC: tiles are columns, atoms their nonzeros; y = A x scatters
//    values[j] * x[c] into y[row_idx[j]].  That is the backward kernel's
//    dx = A^T dy with the column offsets as its "row offsets" (see
//    lb_api.cpp), so it runs over the merge-path split of the columns.
#include "lb_device.h"
#include "lb_internal.h"
#include "lb_schedule.hpp"

namespace lbk {
using namespace lb;

namespace {

constexpr int PG = 16;  // lanes per unit boundary in the split search

__global__ __launch_bounds__(256) void coo_partition_kernel(const int32_t *__restrict__ row_idx, int32_t rows,
                                                            int32_t nnz, int32_t W, int32_t T,
                                                            int32_t *__restrict__ part_i,
                                                            int32_t *__restrict__ part_j) {
    const int64_t t = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / PG;
    const bool live = t <= T;  // uniform per group; every lane still takes part in the ballots
    const int64_t total = static_cast<int64_t>(rows) + nnz;
    const int64_t tt = live ? t : T;
    const int32_t d = static_cast<int32_t>(tt * W < total ? tt * W : total);
    const int32_t j = group_coo_search<PG>(row_idx, rows, nnz, d);
    if (live && (threadIdx.x & (PG - 1)) == 0) {
        part_i[t] = d - j;
        part_j[t] = j;
    }
}

template <int BLOCK, int ITEMS, typename VT>
__global__ __launch_bounds__(BLOCK) void coo_spmv_consume(
    int32_t rows, int32_t nnz, const int32_t *__restrict__ ri, const int32_t *__restrict__ ci,
    const VT *__restrict__ val, const VT *__restrict__ x, float *__restrict__ y, const int32_t *__restrict__ part_i,
    const int32_t *__restrict__ part_j, int32_t *__restrict__ carry_row, float *__restrict__ carry_val) {
    constexpr int W = BLOCK * ITEMS;
    __shared__ int32_t s_row[W];  // the unit's row indices
    __shared__ int32_t s_buf[W];  // row ends [0, nrows), then products [nrows, nrows + nnzs)
    __shared__ seg_t s_wave[BLOCK / kWave];

    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int32_t i0 = part_i[b], j0 = part_j[b];
    const int32_t i1 = part_i[b + 1], j1 = part_j[b + 1];
    const int32_t nrows = i1 - i0, nnzs = j1 - j0;
    int32_t *s_re = s_buf;
    float *s_pv = reinterpret_cast<float *>(s_buf + nrows);

    // Stream loads unconditional with indices clamped into the unit (nnz >= 1
    // here), so every lane's loads are in flight together.
    const int32_t nz_last = nnzs > 0 ? j1 - 1 : (j0 < nnz ? j0 : nnz - 1);
    int32_t r[ITEMS], c[ITEMS];
    VT v[ITEMS];
    float xv[ITEMS];
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        const int32_t jk = j0 + tid + u * BLOCK;
        const int32_t jc = jk < nz_last ? jk : nz_last;
        r[u] = ld_stream(ri + jc);
        c[u] = ld_stream(ci + jc);
        v[u] = ld_stream(val + jc);
    }
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) xv[u] = to_f32(x[c[u]]);
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        const int k = tid + u * BLOCK;
        if (k < nnzs) {
            s_row[k] = r[u];
            s_pv[k] = to_f32(v[u]) * xv[u];
        }
    }
    __syncthreads();
    // Row i0 + q (q < nrows) ends after the unit's entries with row <= i0 + q.
    for (int32_t q = tid; q < nrows; q += BLOCK) {
        const int32_t row = i0 + q;
        int32_t lo = 0, hi = nnzs;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (s_row[mid] <= row)
                lo = mid + 1;
            else
                hi = mid;
        }
        s_re[q] = lo;
    }
    __syncthreads();

    // From here on, the CSR consume: thread diagonal, walk, segmented scan.
    const int32_t total = nrows + nnzs;
    const int32_t d = tid * ITEMS < total ? tid * ITEMS : total;
    const int32_t dend = d + ITEMS < total ? d + ITEMS : total;
    int32_t lo = d - nnzs > 0 ? d - nnzs : 0;
    int32_t hi = d < nrows ? d : nrows;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (s_re[mid] + mid < d)
            lo = mid + 1;
        else
            hi = mid;
    }
    int32_t it = lo, jt = d - lo;
    float acc = 0.f;
    int32_t first = -1;
    float first_sum = 0.f;
    for (int32_t q = d; q < dend; ++q) {
        if (it < nrows && s_re[it] <= jt) {
            if (first < 0) {
                first = it;
                first_sum = acc;
            } else {
                y[i0 + it] = acc;
            }
            acc = 0.f;
            ++it;
        } else {
            acc += s_pv[jt];
            ++jt;
        }
    }
    seg_t tot;
    const seg_t in = block_seg_scan_excl<BLOCK>(seg_t{acc, first >= 0}, s_wave, tot);
    if (first >= 0) y[i0 + first] = first_sum + in.v;
    if (tid == 0) {
        carry_row[b] = i1;
        carry_val[b] = tot.v;
    }
}

template <typename VT>
__global__ __launch_bounds__(256) void coo_thread_spmv(coo_tile_set ts, const int32_t *__restrict__ ci,
                                                       const VT *__restrict__ val, const VT *__restrict__ x,
                                                       float *__restrict__ y) {
    const thread_mapped<coo_tile_set> sch{ts};
    for (int64_t p : sch.tiles()) {
        float acc = 0.f;
        for (int64_t j : sch.atoms(p)) acc += to_f32(val[j]) * to_f32(x[ci[j]]);
        y[p] = acc;
    }
}

template <int G, typename VT>
__global__ __launch_bounds__(group_block<G>::BLOCK) void coo_group_spmv(coo_tile_set ts, const int32_t *__restrict__ ci,
                                                                        const VT *__restrict__ val,
                                                                        const VT *__restrict__ x, float *__restrict__ y) {
    constexpr int BLOCK = group_block<G>::BLOCK;
    __shared__ float s_red[BLOCK / kWave];
    const group_mapped<G, coo_tile_set> sch{ts};
    for (int64_t p : sch.tiles()) {  // uniform across the group (the block when G > 64)
        const tile_ref t = sch.ts.tile(p);
        float acc = 0.f;
        for (int64_t j : sch.atoms(t)) acc += to_f32(val[j]) * to_f32(x[ci[j]]);
        float sum;
        if constexpr (G <= kWave)
            sum = group_sum<G>(acc);
        else
            sum = block_sum<BLOCK>(acc, s_red);
        if (sch.lane() == 0) y[p] = sum;
    }
}

template <int BLOCK, int ITEMS, typename VT>
hipError_t run_coo_merge(const coo_dev &A, const void *x, float *y, void *ws, hipStream_t s) {
    constexpr int W = BLOCK * ITEMS;
    const int64_t T = merge_units(A.rows, A.nnz, W);
    merge_ws w = merge_ws_carve(ws, T);
    hipError_t e = coo_partition(A.ri, A.rows, A.nnz, W, static_cast<int32_t>(T), w.part_i, w.part_j, s);
    if (e != hipSuccess) return e;
    {
        prof_scope p(s, "coo_consume");
        hipLaunchKernelGGL((coo_spmv_consume<BLOCK, ITEMS, VT>), dim3(static_cast<uint32_t>(T)), dim3(BLOCK), 0, s,
                           A.rows, A.nnz, A.ri, A.ci, static_cast<const VT *>(A.val), static_cast<const VT *>(x), y,
                           w.part_i, w.part_j, w.carry_row, w.carry_val);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_fixup(T, A.rows, 1, w.carry_row, w.carry_val, y, 1, s, "coo_fixup");
}

// Blocks for `work` items at `per_block` per block, capped by a caller grid
// and at 2^20 blocks (grid-stride kernels; blocks x threads stays below 2^32).
int64_t grid_for(int64_t work, int64_t per_block, int grid) {
    int64_t g = (work + per_block - 1) / per_block;
    if (grid > 0 && g > grid) g = grid;
    if (g > (int64_t(1) << 20)) g = int64_t(1) << 20;
    return g < 1 ? 1 : g;
}

template <typename VT>
hipError_t run_coo_tiles(const coo_dev &A, const void *x, float *y, lb_sched_kind_t kind, int group, int block,
                         int grid, hipStream_t s) {
    prof_scope p(s, "coo_tiles");
    const coo_tile_set ts{A.ri, A.rows, A.nnz};
    const VT *xv = static_cast<const VT *>(x);
    const VT *vv = static_cast<const VT *>(A.val);
    if (kind == LB_THREAD_MAPPED) {
        hipLaunchKernelGGL(coo_thread_spmv<VT>, dim3(static_cast<uint32_t>(grid_for(A.rows, block, grid))),
                           dim3(block), 0, s, ts, A.ci, vv, xv, y);
        return hipGetLastError();
    }
#define LB_G(G)                                                                                             \
    if (group == G) {                                                                                       \
        const dim3 g(static_cast<uint32_t>(grid_for(A.rows, group_block<G>::GPB, grid)));                   \
        hipLaunchKernelGGL((coo_group_spmv<G, VT>), g, dim3(group_block<G>::BLOCK), 0, s, ts, A.ci, vv, xv, y); \
        return hipGetLastError();                                                                           \
    }
    LB_TRAVERSAL_GROUPS(LB_G)
#undef LB_G
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t coo_partition(const int32_t *row_idx, int32_t rows, int32_t nnz, int32_t W, int32_t T, int32_t *part_i,
                         int32_t *part_j, hipStream_t s) {
    prof_scope p(s, "coo_partition");
    const int64_t blocks = ((static_cast<int64_t>(T) + 1) * PG + 255) / 256;
    hipLaunchKernelGGL(coo_partition_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, row_idx, rows, nnz,
                       W, T, part_i, part_j);
    return hipGetLastError();
}

hipError_t coo_spmv(const coo_dev &A, const void *x, float *y, lb_sched_kind_t kind, int group, int block, int items,
                    int grid, void *ws, hipStream_t s) {
    if (kind != LB_MERGE_PATH) {
        if (A.dt == LB_BF16) return run_coo_tiles<bf16_bits>(A, x, y, kind, group, block, grid, s);
        return run_coo_tiles<float>(A, x, y, kind, group, block, grid, s);
    }
#define X(B, I)                                                                       \
    if (block == B && items == I) {                                                   \
        if (A.dt == LB_BF16) return run_coo_merge<B, I, bf16_bits>(A, x, y, ws, s);   \
        return run_coo_merge<B, I, float>(A, x, y, ws, s);                            \
    }
    LB_MERGE_CONFIGS(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace lbk
