// Backward of y = A x over the merge-path split, for gfx950.
//
//   dvalues[j] = dy[row(j)] * x[col_idx[j]]     (one product per nonzero)
//   dx[c]     += values[j] * dy[row(j)]         (scatter: dx = A^T dy)
//
// Both need each nonzero's row.  Block b owns the same merge-path unit as
// in the forward pass; its threads walk their ITEMS merge items inside the
// LDS copy of the block's row ends and label every nonzero they pass with
// its row (the atom -> tile map that group-mapped gets from get_tile).  The
// block then streams its nonzeros coalesced: dvalues is written in order,
// and dx receives hardware float atomics (atomic order varies, so dx is not
// bit-reproducible run to run; dvalues is).
//
// COMBINE (the CSC product, where the scatter targets are A's rows and a
// long row of A is hit by a large share of all nonzeros): the block first
// sums its products per target in an LDS hash table (linear probing over a
// power of two of slots, at least 2W and at most 4096; a product whose probe
// finds neither its key nor a free slot goes straight to global memory),
// then issues one global atomic per distinct target.  Many blocks adding
// into the same few addresses is what bounds the plain scatter there.
#include "lb_device.h"
#include "lb_internal.h"

namespace lbk {
using namespace lb;

template <int BLOCK, int ITEMS, typename VT, bool WANT_DX, bool WANT_DV, bool COMBINE = false>
__global__ __launch_bounds__(BLOCK) void merge_backward_kernel(
    int32_t rows, int32_t nnz, const int32_t *__restrict__ ro, const int32_t *__restrict__ ci, const VT *__restrict__ val,
    const VT *__restrict__ x, const float *__restrict__ dy, float *__restrict__ dx, float *__restrict__ dvalues,
    const int32_t *__restrict__ part_i, const int32_t *__restrict__ part_j) {
    static_assert(!COMBINE || (WANT_DX && !WANT_DV), "combining is for the dx scatter alone");
    constexpr int W = BLOCK * ITEMS;
    // a power of two >= 2W, at most 4096
    constexpr int SLOTS = !COMBINE ? 1 : (2 * W <= 1024 ? 1024 : (2 * W <= 2048 ? 2048 : 4096));
    __shared__ int32_t s_buf[W];  // row ends [0, nrows), then row labels [nrows, nrows + nnzs)
    __shared__ int32_t s_key[SLOTS];
    __shared__ float s_sum[SLOTS];

    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    if constexpr (COMBINE) {
        for (int q = tid; q < SLOTS; q += BLOCK) {
            s_key[q] = -1;
            s_sum[q] = 0.f;
        }
    }
    const int32_t i0 = part_i[b], j0 = part_j[b];
    const int32_t i1 = part_i[b + 1], j1 = part_j[b + 1];
    const int32_t nrows = i1 - i0, nnzs = j1 - j0;
    int32_t *s_re = s_buf;
    int32_t *s_row = s_buf + nrows;
    // Row ends, and this thread's share of the nonzero streams: unconditional
    // loads with indices clamped into the unit (see k_merge.hip).
    const int32_t re_last = i1 > i0 ? i1 : i0 + 1 <= rows ? i0 + 1 : rows;
    const int32_t nz_last = nnzs > 0 ? j1 - 1 : (j0 < nnz ? j0 : nnz - 1);
    int32_t re[ITEMS], cc[ITEMS];
    VT vv[ITEMS];
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        const int32_t k = tid + u * BLOCK;
        const int32_t rk = i0 + 1 + k;
        const int32_t jk = j0 + k;
        re[u] = ro[rk < re_last ? rk : re_last];
        cc[u] = ld_stream(ci + (jk < nz_last ? jk : nz_last));
        if constexpr (WANT_DX) vv[u] = ld_stream(val + (jk < nz_last ? jk : nz_last));
    }
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        const int k = tid + u * BLOCK;
        if (k < nrows) s_re[k] = re[u] - j0;
    }
    __syncthreads();

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
    for (int32_t q = d; q < dend; ++q) {
        if (it < nrows && s_re[it] <= jt)
            ++it;
        else
            s_row[jt++] = it;
    }
    __syncthreads();

    float g[ITEMS], xv[ITEMS];
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        const int k = tid + u * BLOCK;
        // labels exist for k < nnzs; other lanes read a valid row and discard it
        const int32_t lab = nnzs > 0 ? s_row[k < nnzs ? k : nnzs - 1] : 0;
        const int32_t r = i0 + lab < rows ? i0 + lab : rows - 1;
        g[u] = dy[r];
        if constexpr (WANT_DV) xv[u] = to_f32(x[cc[u]]);
    }
    if constexpr (COMBINE) {
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            const int k = tid + u * BLOCK;
            if (k < nnzs) {
                const int32_t key = cc[u];
                const float p = to_f32(vv[u]) * g[u];
                uint32_t h = (static_cast<uint32_t>(key) * 2654435761u) & (SLOTS - 1);
                bool placed = false;
                for (int probe = 0; probe < SLOTS && !placed; ++probe) {
                    const int32_t prev = atomicCAS(s_key + h, -1, key);
                    if (prev == -1 || prev == key) {
                        atomicAdd(s_sum + h, p);
                        placed = true;
                    }
                    h = (h + 1) & (SLOTS - 1);
                }
                if (!placed) unsafeAtomicAdd(dx + key, p);
            }
        }
        __syncthreads();
        for (int q = tid; q < SLOTS; q += BLOCK) {
            const int32_t key = s_key[q];
            if (key >= 0) unsafeAtomicAdd(dx + key, s_sum[q]);
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        const int k = tid + u * BLOCK;
        if (k < nnzs) {
            const int64_t j = static_cast<int64_t>(j0) + k;
            if constexpr (WANT_DV) dvalues[j] = g[u] * xv[u];
            if constexpr (WANT_DX) unsafeAtomicAdd(dx + cc[u], to_f32(vv[u]) * g[u]);
        }
    }
}

template <int BLOCK, int ITEMS, typename VT>
static hipError_t run_backward(const csr_dev &A, const void *x, const float *dy, float *dx, float *dvalues, void *ws,
                               hipStream_t s, bool combine) {
    constexpr int W = BLOCK * ITEMS;
    const int64_t T = merge_units(A.rows, A.nnz, W);
    merge_ws w = merge_ws_carve(ws, T);
    hipError_t e = merge_partition(A.ro, A.rows, A.nnz, W, static_cast<int32_t>(T), w.part_i, w.part_j, s);
    if (e != hipSuccess) return e;
    prof_scope p(s, "backward");
    const dim3 g(static_cast<uint32_t>(T));
    const VT *xv = static_cast<const VT *>(x);
    const VT *vv = static_cast<const VT *>(A.val);
    if (dx && !dvalues && combine)
        hipLaunchKernelGGL((merge_backward_kernel<BLOCK, ITEMS, VT, true, false, true>), g, dim3(BLOCK), 0, s, A.rows,
                           A.nnz, A.ro, A.ci, vv, xv, dy, dx, dvalues, w.part_i, w.part_j);
    else if (dx && dvalues)
        hipLaunchKernelGGL((merge_backward_kernel<BLOCK, ITEMS, VT, true, true>), g, dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci, vv,
                           xv, dy, dx, dvalues, w.part_i, w.part_j);
    else if (dx)
        hipLaunchKernelGGL((merge_backward_kernel<BLOCK, ITEMS, VT, true, false>), g, dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci,
                           vv, xv, dy, dx, dvalues, w.part_i, w.part_j);
    else
        hipLaunchKernelGGL((merge_backward_kernel<BLOCK, ITEMS, VT, false, true>), g, dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci,
                           vv, xv, dy, dx, dvalues, w.part_i, w.part_j);
    return hipGetLastError();
}

hipError_t merge_backward(const csr_dev &A, const void *x, const float *dy, float *dx, float *dvalues, int block,
                          int items, void *ws, hipStream_t s, bool combine_dx) {
#define X_(B, I)                                                                                             \
    if (block == B && items == I) {                                                                          \
        if (A.dt == LB_BF16) return run_backward<B, I, bf16_bits>(A, x, dy, dx, dvalues, ws, s, combine_dx); \
        return run_backward<B, I, float>(A, x, dy, dx, dvalues, ws, s, combine_dx);                          \
    }
    LB_MERGE_CONFIGS(X_)
#undef X_
    return hipErrorInvalidValue;
}

}  // namespace lbk
