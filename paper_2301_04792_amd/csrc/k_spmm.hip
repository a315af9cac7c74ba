// Merge-path SpMM (Sec. 5.3) and the batched persistent form, for gfx950.
//
// Y[r, :] = sum_j values[j] * X[col_idx[j], :].  The SpMM listing of
// Sec. 5.3 wraps the SpMV loop in a loop over B's columns; here the column
// loop sits inside the atom loop instead, so each nonzero's (col, value) is
// read once per pass and KC (<= 8) contiguous columns of X are gathered per
// nonzero.  k > KC runs ceil(k / KC) passes over the matrix.
//
// The merge-path split and carry handling are those of k_merge.hip, with KC
// partial sums per thread and per carry.
//
// Batched: matrices stored back to back form one block-diagonal matrix whose
// merged sequence of sum(m_b) row ends and sum(nnz_b) nonzeros is cut into
// units of W items.  One persistent launch (grid = CUs x resident blocks)
// loops over the units (Sec. 5.1 persistent ranges; every block leaves once
// the unit index passes the last unit).  Each unit's split is searched
// inside the kernel by two wavefronts (64-ary search, as in the partition
// kernel).  A nonzero's X row is col_base[b] + col_idx[j] for the matrix b
// that owns its row; each thread tracks b as it walks rows.
#include "lb_device.h"
#include "lb_internal.h"

namespace lbk {
using namespace lb;

template <int BLOCK, int ITEMS, int KC, bool BATCHED, typename VT>
__global__ __launch_bounds__(BLOCK) void merge_spmm_consume(
    int32_t rows, int32_t nnz, int32_t T, const int32_t *__restrict__ ro, const int32_t *__restrict__ ci,
    const VT *__restrict__ val, const VT *__restrict__ X, int64_t ldx, float *__restrict__ Y, int64_t ldy,
    const int32_t *__restrict__ part_i, const int32_t *__restrict__ part_j, int32_t *__restrict__ carry_row,
    float *__restrict__ carry_val, int32_t count, const int64_t *__restrict__ row_base,
    const int64_t *__restrict__ col_base) {
    constexpr int W = BLOCK * ITEMS;
    __shared__ int32_t s_buf[W];  // row ends [0, nrows), then column indices [nrows, nrows + nnzs)
    __shared__ float s_val[W];
    __shared__ seg_t s_wave[BLOCK / kWave];
    __shared__ int32_t s_split[4];

    const int tid = threadIdx.x;
    for (int64_t u = blockIdx.x; u < T; u += gridDim.x) {  // one unit per block without BATCHED
        int32_t i0, j0, i1, j1;
        if constexpr (BATCHED) {
            const int64_t total = static_cast<int64_t>(rows) + nnz;
            const int w = wave_id();
            if (w < 2) {
                const int64_t d64 = (u + w) * W < total ? (u + w) * W : total;
                const int32_t d = static_cast<int32_t>(d64);
                const int32_t i = wave_merge_search(ro, rows, nnz, d);
                if (lane_id() == 0) {
                    s_split[2 * w] = i;
                    s_split[2 * w + 1] = d - i;
                }
            }
            __syncthreads();
            i0 = s_split[0];
            j0 = s_split[1];
            i1 = s_split[2];
            j1 = s_split[3];
        } else {
            i0 = part_i[u];
            j0 = part_j[u];
            i1 = part_i[u + 1];
            j1 = part_j[u + 1];
        }
        const int32_t nrows = i1 - i0, nnzs = j1 - j0;
        int32_t *s_re = s_buf;
        int32_t *s_col = s_buf + nrows;
        // unconditional loads, indices clamped into the unit (see k_merge.hip)
        const int32_t re_last = i1 > i0 ? i1 : i0 + 1 <= rows ? i0 + 1 : rows;
        const int32_t nz_last = nnzs > 0 ? j1 - 1 : (j0 < nnz ? j0 : nnz - 1);
        int32_t re[ITEMS], cc[ITEMS];
        VT vv[ITEMS];
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            const int32_t k = tid + q * BLOCK;
            const int32_t rk = i0 + 1 + k;
            const int32_t jk = j0 + k;
            re[q] = ro[rk < re_last ? rk : re_last];
            cc[q] = ld_stream(ci + (jk < nz_last ? jk : nz_last));
            vv[q] = ld_stream(val + (jk < nz_last ? jk : nz_last));
        }
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            const int k = tid + q * BLOCK;
            if (k < nrows) s_re[k] = re[q] - j0;
            if (k < nnzs) {
                s_col[k] = cc[q];
                s_val[k] = to_f32(vv[q]);
            }
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

        // Matrix owning the current row (batched only).
        int32_t mat = 0;
        int64_t next_base = 0x7fffffffffffffffLL, cbase = 0;
        if constexpr (BATCHED) {
            const int64_t r0 = static_cast<int64_t>(i0) + it;
            // first matrix with row_base[b + 1] > r0
            int32_t blo = 0, bhi = count;
            while (blo < bhi) {
                const int32_t mid = (blo + bhi) >> 1;
                if (row_base[mid + 1] <= r0)
                    blo = mid + 1;
                else
                    bhi = mid;
            }
            mat = blo < count ? blo : count - 1;
            next_base = row_base[mat + 1];
            cbase = col_base[mat];
        }

        float acc[KC];
        float first_sum[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = first_sum[c] = 0.f;
        int32_t first = -1;
        for (int32_t q = d; q < dend; ++q) {
            if (it < nrows && s_re[it] <= jt) {
                float *yrow = Y + static_cast<int64_t>(i0 + it) * ldy;
                if (first < 0) {
                    first = it;
#pragma unroll
                    for (int c = 0; c < KC; ++c) first_sum[c] = acc[c];
                } else {
#pragma unroll
                    for (int c = 0; c < KC; ++c) yrow[c] = acc[c];
                }
#pragma unroll
                for (int c = 0; c < KC; ++c) acc[c] = 0.f;
                ++it;
                if constexpr (BATCHED) {
                    while (static_cast<int64_t>(i0) + it >= next_base && mat + 1 < count) {
                        ++mat;
                        next_base = row_base[mat + 1];
                        cbase = col_base[mat];
                    }
                }
            } else {
                const float v = s_val[jt];
                const VT *xr = X + (cbase + s_col[jt]) * ldx;
#pragma unroll
                for (int c = 0; c < KC; ++c) acc[c] += v * to_f32(xr[c]);
                ++jt;
            }
        }

        const int flag = first >= 0;
        float in[KC];
        float tot[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            seg_t t;
            in[c] = block_seg_scan_excl<BLOCK>(seg_t{acc[c], flag}, s_wave, t).v;
            tot[c] = t.v;
        }
        if (first >= 0) {
            float *yrow = Y + static_cast<int64_t>(i0 + first) * ldy;
#pragma unroll
            for (int c = 0; c < KC; ++c) yrow[c] = first_sum[c] + in[c];
        }
        if (tid == 0) {
            carry_row[u] = i1;
#pragma unroll
            for (int c = 0; c < KC; ++c) carry_val[u * KC + c] = tot[c];
        }
        __syncthreads();  // LDS is reused by the next unit
    }
}

template <int BLOCK, int ITEMS, int KC, typename VT>
static hipError_t run_spmm_pass(const csr_dev &A, const VT *X, int64_t ldx, float *Y, int64_t ldy, void *ws,
                                bool partitioned, hipStream_t s) {
    constexpr int W = BLOCK * ITEMS;
    const int64_t T = merge_units(A.rows, A.nnz, W);
    merge_ws w = merge_ws_carve(ws, T);
    if (!partitioned) {
        hipError_t e = merge_partition(A.ro, A.rows, A.nnz, W, static_cast<int32_t>(T), w.part_i, w.part_j, s);
        if (e != hipSuccess) return e;
    }
    {
        prof_scope p(s, "merge_consume");
        hipLaunchKernelGGL((merge_spmm_consume<BLOCK, ITEMS, KC, false, VT>), dim3(static_cast<uint32_t>(T)),
                           dim3(BLOCK), 0, s, A.rows, A.nnz, static_cast<int32_t>(T), A.ro, A.ci,
                           static_cast<const VT *>(A.val), X, ldx, Y, ldy, w.part_i, w.part_j, w.carry_row,
                           w.carry_val, 0, nullptr, nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_fixup(T, A.rows, KC, w.carry_row, w.carry_val, Y, ldy, s, "merge_fixup");
}

template <int BLOCK, int ITEMS, typename VT>
static hipError_t run_spmm(const csr_dev &A, const VT *X, int32_t k, int64_t ldx, float *Y, int64_t ldy, void *ws,
                           hipStream_t s) {
    int32_t c0 = 0;
    bool partitioned = false;
    while (c0 < k) {
        const int32_t left = k - c0;
        hipError_t e;
        if (left >= 8)
            e = run_spmm_pass<BLOCK, ITEMS, 8, VT>(A, X + c0, ldx, Y + c0, ldy, ws, partitioned, s), c0 += 8;
        else if (left >= 4)
            e = run_spmm_pass<BLOCK, ITEMS, 4, VT>(A, X + c0, ldx, Y + c0, ldy, ws, partitioned, s), c0 += 4;
        else if (left >= 2)
            e = run_spmm_pass<BLOCK, ITEMS, 2, VT>(A, X + c0, ldx, Y + c0, ldy, ws, partitioned, s), c0 += 2;
        else
            e = run_spmm_pass<BLOCK, ITEMS, 1, VT>(A, X + c0, ldx, Y + c0, ldy, ws, partitioned, s), c0 += 1;
        if (e != hipSuccess) return e;
        partitioned = true;  // the split depends only on the matrix
    }
    return hipSuccess;
}

// W = BLOCK * ITEMS <= 4096 keeps the two LDS arrays within 32 KB.
#define LB_MERGE_CONFIGS(X) \
    X(128, 4) X(128, 8) X(128, 12) X(128, 16) \
    X(256, 4) X(256, 8) X(256, 12) X(256, 16) \
    X(512, 4) X(512, 8)

hipError_t merge_spmm(const csr_dev &A, const void *X, int32_t k, int64_t ldx, float *Y, int64_t ldy, int block,
                      int items, void *ws, hipStream_t s) {
#define X_(B, I)                                                                                               \
    if (block == B && items == I) {                                                                            \
        if (A.dt == LB_BF16)                                                                                   \
            return run_spmm<B, I, bf16_bits>(A, static_cast<const bf16_bits *>(X), k, ldx, Y, ldy, ws, s);     \
        return run_spmm<B, I, float>(A, static_cast<const float *>(X), k, ldx, Y, ldy, ws, s);                 \
    }
    LB_MERGE_CONFIGS(X_)
#undef X_
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ batched

// Resident blocks per CU for the persistent grid, from the occupancy API.
template <typename K>
static int persistent_grid(K kernel, int block, int64_t units) {
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) {
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0);
    }
    int64_t g = static_cast<int64_t>(cus) * (per_cu > 0 ? per_cu : 1);
    if (g > units) g = units;
    return static_cast<int>(g < 1 ? 1 : g);
}

size_t batched_ws_bytes(const batch_dev &B, int block, int items, int k) {
    const int64_t T = merge_units(B.total_rows, B.total_nnz, static_cast<int64_t>(block) * items);
    const int kc = k >= 8 ? 8 : (k >= 4 ? 4 : (k >= 2 ? 2 : 1));
    return merge_ws_bytes(T, kc);
}

template <int BLOCK, int ITEMS, int KC, typename VT>
static hipError_t run_batched_pass(const batch_dev &B, const VT *X, int32_t k, float *Y, void *ws, hipStream_t s) {
    constexpr int W = BLOCK * ITEMS;
    const int64_t T = merge_units(B.total_rows, B.total_nnz, W);
    merge_ws w = merge_ws_carve(ws, T);
    auto kern = merge_spmm_consume<BLOCK, ITEMS, KC, true, VT>;
    const int grid = persistent_grid(kern, BLOCK, T);
    {
        prof_scope p(s, "batched_consume");
        hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), 0, s, B.total_rows, B.total_nnz, static_cast<int32_t>(T),
                           B.ro, B.ci, static_cast<const VT *>(B.val), X, static_cast<int64_t>(k), Y,
                           static_cast<int64_t>(k), nullptr, nullptr, w.carry_row, w.carry_val, B.count, B.row_base,
                           B.col_base);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_fixup(T, B.total_rows, KC, w.carry_row, w.carry_val, Y, k, s, "batched_fixup");
}

template <int BLOCK, int ITEMS, typename VT>
static hipError_t run_batched(const batch_dev &B, const VT *X, int32_t k, float *Y, void *ws, hipStream_t s) {
    int32_t c0 = 0;
    while (c0 < k) {
        const int32_t left = k - c0;
        hipError_t e;
        if (left >= 8)
            e = run_batched_pass<BLOCK, ITEMS, 8, VT>(B, X + c0, k, Y + c0, ws, s), c0 += 8;
        else if (left >= 4)
            e = run_batched_pass<BLOCK, ITEMS, 4, VT>(B, X + c0, k, Y + c0, ws, s), c0 += 4;
        else if (left >= 2)
            e = run_batched_pass<BLOCK, ITEMS, 2, VT>(B, X + c0, k, Y + c0, ws, s), c0 += 2;
        else
            e = run_batched_pass<BLOCK, ITEMS, 1, VT>(B, X + c0, k, Y + c0, ws, s), c0 += 1;
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t batched_spmm(const batch_dev &B, const void *X, int32_t k, float *Y, int block, int items, void *ws,
                        hipStream_t s) {
#define X_(B_, I)                                                                                           \
    if (block == B_ && items == I) {                                                                        \
        if (B.dt == LB_BF16) return run_batched<B_, I, bf16_bits>(B, static_cast<const bf16_bits *>(X), k, Y, ws, s); \
        return run_batched<B_, I, float>(B, static_cast<const float *>(X), k, Y, ws, s);                    \
    }
    LB_MERGE_CONFIGS(X_)
#undef X_
    return hipErrorInvalidValue;
}

}  // namespace lbk
