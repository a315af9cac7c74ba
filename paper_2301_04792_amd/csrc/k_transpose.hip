// Backward of y = A x without atomics: dx = A^T dy as a merge-path SpMV over
// the transposed pattern.  A training loop keeps one sparsity pattern across
// steps, so the transpose is built once (transpose_pattern) and each
// backward runs the forward's merge-path kernels on A^T, reading the current
// values of A through the pattern's permutation (val[perm[p]], gathered in
// the consume kernel's setup); dvalues comes from the backward kernel's
// dvalues-only pass.
//
// Transpose of a CSR pattern A (rows x cols): A^T has a row per column of A.
//   1. count:   per nonzero e of row r, rank[e] = atomicAdd(&cnt[col[e]], 1)
//               (cnt lives in the output offsets array);
//   2. scan:    exclusive prefix of the counts into at_row_offsets (per tile
//               of 2048 counts, then the tile totals in one block, then the
//               tile prefixes added);
//   3. scatter: e goes to position at_row_offsets[col[e]] + rank[e]:
//               at_col_idx = r, perm = e.
// The ranks come from atomics, so the order inside a row of A^T varies from
// build to build (any order is a valid CSR; dx's summation order follows it).
#include "lb_device.h"
#include "lb_internal.h"
#include "lb_schedule.hpp"

namespace lbk {
using namespace lb;

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kRowGroup = 64;  // one wavefront per row of A in the count and scatter passes

__global__ __launch_bounds__(256) void transpose_count(csr_tile_set ts, const int32_t *__restrict__ ci,
                                                       int32_t *__restrict__ cnt, int32_t *__restrict__ rank) {
    const group_mapped<kRowGroup, csr_tile_set> sch{ts};
    for (int64_t r : sch.tiles())
        for (int64_t e : sch.atoms(sch.ts.tile(r))) rank[e] = atomicAdd(cnt + ci[e], 1);
}

// In-tile exclusive prefix of a[0, n) in place; the tile total to tile_sum.
__global__ __launch_bounds__(kScanThreads) void scan_tiles(int32_t *__restrict__ a, int64_t n,
                                                           int32_t *__restrict__ tile_sum) {
    __shared__ int32_t s_wave[kScanThreads / kWave];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t sum = 0;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        v[u] = base + u < n ? a[base + u] : 0;
        sum += v[u];
    }
    const int32_t incl = block_scan_incl<kScanThreads>(sum, s_wave);
    int32_t run = incl - sum;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        if (base + u < n) a[base + u] = run;
        run += v[u];
    }
    if (threadIdx.x == kScanThreads - 1) tile_sum[blockIdx.x] = incl;
}

// One block: exclusive prefix of the nb tile totals in place; a[n] = total.
__global__ __launch_bounds__(1024) void scan_totals(int32_t *__restrict__ tile_sum, int32_t nb,
                                                    int32_t *__restrict__ a, int64_t n) {
    __shared__ int32_t s_wave[1024 / kWave];
    __shared__ int32_t s_total;
    int32_t carry = 0;
    for (int32_t c = 0; c < nb; c += 1024) {  // uniform across the block
        const int32_t idx = c + static_cast<int32_t>(threadIdx.x);
        const int32_t v = idx < nb ? tile_sum[idx] : 0;
        const int32_t incl = block_scan_incl<1024>(v, s_wave);
        if (idx < nb) tile_sum[idx] = carry + incl - v;
        if (threadIdx.x == 1023) s_total = incl;
        __syncthreads();
        carry += s_total;
        __syncthreads();
    }
    if (threadIdx.x == 0) a[n] = carry;
}

__global__ __launch_bounds__(256) void scan_add(int32_t *__restrict__ a, int64_t n,
                                                const int32_t *__restrict__ tile_pre) {
    for (int64_t p : grid_stride_range(0, n)) a[p] += tile_pre[p / kScanTile];
}

__global__ __launch_bounds__(256) void transpose_scatter(csr_tile_set ts, const int32_t *__restrict__ ci,
                                                         const int32_t *__restrict__ rank,
                                                         const int32_t *__restrict__ at_ro,
                                                         int32_t *__restrict__ at_ci, int32_t *__restrict__ perm) {
    const group_mapped<kRowGroup, csr_tile_set> sch{ts};
    for (int64_t r : sch.tiles()) {
        for (int64_t e : sch.atoms(sch.ts.tile(r))) {
            const int32_t pos = at_ro[ci[e]] + rank[e];
            at_ci[pos] = static_cast<int32_t>(r);
            perm[pos] = static_cast<int32_t>(e);
        }
    }
}

int64_t capped_blocks(int64_t work, int64_t per_block) {
    const int64_t g = (work + per_block - 1) / per_block;
    return g < 1 ? 1 : (g > 8192 ? 8192 : g);
}

}  // namespace

size_t transpose_ws_bytes(int64_t cols, int64_t nnz) {
    return align256(static_cast<size_t>(nnz) * 4) + align256(static_cast<size_t>(cols / kScanTile + 2) * 4);
}

hipError_t transpose_pattern(const csr_dev &A, int32_t *at_ro, int32_t *at_ci, int32_t *perm, void *ws,
                             hipStream_t s) {
    prof_scope p(s, "transpose");
    char *w = static_cast<char *>(ws);
    int32_t *rank = reinterpret_cast<int32_t *>(w);
    int32_t *tile_sum = reinterpret_cast<int32_t *>(w + align256(static_cast<size_t>(A.nnz) * 4));
    const csr_tile_set ts{A.ro, A.rows, A.nnz};
    const int64_t n = A.cols;
    hipError_t e = fill_f32(reinterpret_cast<float *>(at_ro), n + 1, 0.f, s);  // +0.0f is all zero bits
    if (e != hipSuccess) return e;
    constexpr int GPB = group_block<kRowGroup>::GPB;
    const int64_t want = (static_cast<int64_t>(A.rows) + GPB - 1) / GPB;  // grid-stride: capped at 2^20 blocks
    const uint32_t rb = static_cast<uint32_t>(want < 1 ? 1 : (want > (int64_t(1) << 20) ? int64_t(1) << 20 : want));
    hipLaunchKernelGGL(transpose_count, dim3(rb), dim3(256), 0, s, ts, A.ci, at_ro, rank);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb > 0)
        hipLaunchKernelGGL(scan_tiles, dim3(static_cast<uint32_t>(nb)), dim3(kScanThreads), 0, s, at_ro, n, tile_sum);
    hipLaunchKernelGGL(scan_totals, dim3(1), dim3(1024), 0, s, tile_sum, static_cast<int32_t>(nb), at_ro, n);
    if (n > 0)
        hipLaunchKernelGGL(scan_add, dim3(static_cast<uint32_t>(capped_blocks(n, 256))), dim3(256), 0, s, at_ro, n,
                           tile_sum);
    hipLaunchKernelGGL(transpose_scatter, dim3(rb), dim3(256), 0, s, ts, A.ci, rank, at_ro, at_ci, perm);
    return hipGetLastError();
}

size_t backward_transposed_ws_bytes(int64_t rows, int64_t cols, int64_t nnz, int block, int items) {
    const int64_t W = static_cast<int64_t>(block) * items;
    const size_t a = merge_ws_bytes(merge_units(rows, nnz, W), 1);  // dvalues pass over A
    const size_t b = merge_ws_bytes(merge_units(cols, nnz, W), 1);  // SpMV over A^T
    return a > b ? a : b;
}

hipError_t backward_transposed(const csr_dev &A, const int32_t *at_ro, const int32_t *at_ci, const int32_t *perm,
                               const void *x, const float *dy, float *dx, float *dvalues, int block, int items,
                               void *ws, hipStream_t s) {
    if (dvalues) {
        const hipError_t e = merge_backward(A, x, dy, nullptr, dvalues, block, items, ws, s);
        if (e != hipSuccess) return e;
    }
    if (!dx) return hipSuccess;
    // A^T with A's values (of A's type) read through perm; x of this SpMV is dy
    const csr_dev AT{A.cols, A.rows, A.nnz, at_ro, at_ci, A.val, A.dt};
    return merge_spmv(AT, dy, dx, block, items, 1, ws, s, perm);
}

}  // namespace lbk
