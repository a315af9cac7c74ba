// Merge-path SpMM (Sec. 5.3) and the batched persistent form, for gfx950.
//
// Y[r, :] = sum_j values[j] * X[col_idx[j], :].  The SpMM listing of
// Sec. 5.3 wraps the SpMV loop in a loop over B's columns; here the column
// loop sits inside the atom loop instead: a pass handles KC contiguous
// columns of X, gathering KC values per nonzero, and k > KC runs
// ceil(k / KC) passes over the matrix.
//
// Per unit (the merge-path split and carry handling of k_merge.hip), two
// consumers:
//  * one column (merge_spmm_consume with KC = 1): the products
//    values[j] * X[col_idx[j]] of every nonzero are staged in LDS with all
//    loads of a lane issued before the first wait, then the threads walk
//    their merge items over LDS (the SpMV consumer's scheme);
//  * wider passes (merge_spmm_walk): LDS holds the row ends and each
//    nonzero's X row and value; a lane gathers a nonzero's KC values when its
//    walk reaches it and keeps only its KC partial sums live, which keeps
//    occupancy high (staging KC products per nonzero needed so many registers
//    that occupancy fell to 4-5 waves and k = 8 ran ~1.7x slower).
//  Both finish with one segmented scan over all KC columns.  A pass takes
//  KC = 8 columns (4 when 2 * W words would exceed 48 KB of LDS); k > KC runs
//  ceil(k / KC) passes.
//
// Batched: matrices stored back to back form one block-diagonal matrix
// whose merged sequence of sum(m_b) row ends and sum(nnz_b) nonzeros is cut
// into units of W items by the split launch.  One persistent launch (grid =
// CUs x resident blocks) then loops over the units (Sec. 5.1 persistent
// ranges; every block leaves once its unit index passes the last unit).
// A nonzero's X row is col_base[b] + col_idx[j] for the matrix b that owns
// it: two wavefronts find the matrices of the unit's first and last rows;
// only a unit that straddles matrices searches the owner per nonzero.
#include "lb_device.h"
#include "lb_internal.h"

namespace lbk {
using namespace lb;

// Columns per pass: the walk consumer keeps 2 * W words in LDS and KC sums
// per lane, so a pass takes 8 columns unless 2 * W words exceed 48 KB.
template <int BLOCK, int ITEMS>
struct spmm_shape {
    static constexpr int W = BLOCK * ITEMS;
    static constexpr int KC = 2 * W * 4 <= 49152 ? 8 : 4;
};

// Number of entries of the sorted int64 array a[0..n) that are <= key, by
// one wavefront (64-ary search); every lane returns it.
__device__ __forceinline__ int32_t wave_count_le(const int64_t *__restrict__ a, int32_t n, int64_t key) {
    const int lane = lane_id();
    int32_t lo = 0, hi = n;  // a[r] <= key for r < lo, a[r] > key for r >= hi
    while (__ballot(hi - lo > kWave) != 0) {
        const int32_t step = (hi - lo + kWave - 1) / kWave;
        const int32_t r = lo + (lane + 1) * step - 1;
        const bool le = r < hi && a[r] <= key;
        const int32_t c = __popcll(__ballot(le));
        const int32_t rc = lo + (c + 1) * step - 1;
        hi = rc < hi ? rc : hi;
        lo = lo + c * step;
    }
    const int32_t r = lo + lane;
    return lo + __popcll(__ballot(r < hi && a[r] <= key));
}

// KC consecutive values of one X row; VECX: the row start is aligned to the
// load width (16 bytes, or 4 * KC bytes for narrower rows), so whole vectors
// are read.
template <int KC, bool VECX>
__device__ __forceinline__ void load_row(const float *p, float (&o)[KC]) {
    if constexpr (VECX && KC % 4 == 0) {
        typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int c = 0; c < KC; c += 4) {
            const f4 v = *reinterpret_cast<const f4 *>(p + c);
            o[c] = v.x, o[c + 1] = v.y, o[c + 2] = v.z, o[c + 3] = v.w;
        }
    } else if constexpr (VECX && KC == 2) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        const f2 v = *reinterpret_cast<const f2 *>(p);
        o[0] = v.x, o[1] = v.y;
    } else {
#pragma unroll
        for (int c = 0; c < KC; ++c) o[c] = p[c];
    }
}

template <int KC, bool VECX>
__device__ __forceinline__ void load_row(const bf16_bits *p, float (&o)[KC]) {
    if constexpr (VECX && KC % 8 == 0) {
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int c = 0; c < KC; c += 8) {
            const u4 v = *reinterpret_cast<const u4 *>(p + c);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) o[c + 2 * e] = __uint_as_float(w[e] << 16), o[c + 2 * e + 1] = __uint_as_float(w[e] & 0xffff0000u);
        }
    } else if constexpr (VECX && KC == 4) {
        typedef uint32_t u2 __attribute__((ext_vector_type(2)));
        const u2 v = *reinterpret_cast<const u2 *>(p);
        o[0] = __uint_as_float(v.x << 16), o[1] = __uint_as_float(v.x & 0xffff0000u);
        o[2] = __uint_as_float(v.y << 16), o[3] = __uint_as_float(v.y & 0xffff0000u);
    } else if constexpr (VECX && KC == 2) {
        const uint32_t v = *reinterpret_cast<const uint32_t *>(p);
        o[0] = __uint_as_float(v << 16), o[1] = __uint_as_float(v & 0xffff0000u);
    } else {
#pragma unroll
        for (int c = 0; c < KC; ++c) o[c] = to_f32(p[c]);
    }
}

template <int BLOCK, int ITEMS, int KC, bool BATCHED, bool VECX, typename VT>
__global__ __launch_bounds__(BLOCK) void merge_spmm_consume(
    int32_t rows, int32_t nnz, int32_t T, const int32_t *__restrict__ ro, const int32_t *__restrict__ ci,
    const VT *__restrict__ val, const VT *__restrict__ X, int64_t ldx, float *__restrict__ Y, int64_t ldy,
    const int32_t *__restrict__ part_i, const int32_t *__restrict__ part_j, int32_t *__restrict__ carry_row,
    float *__restrict__ carry_val, const int32_t *__restrict__ part_mat, const int64_t *__restrict__ nnz_base,
    const int64_t *__restrict__ col_base) {
    constexpr int W = BLOCK * ITEMS;
    __shared__ float s_buf[W * KC];  // row ends (int) [0, nrows), then products [nrows + k * KC + c]
    __shared__ float s_wv[BLOCK / kWave * KC];
    __shared__ int s_wf[BLOCK / kWave];

    const int tid = threadIdx.x;
    // XCD-aware order for the persistent launch: blocks are dealt round-robin
    // to the 8 XCDs (block b runs on XCD b % 8), so XCD x takes the contiguous
    // eighth [x * per, (x + 1) * per) of the units and its L2 holds only the
    // X rows of its own matrices.  Without BATCHED: one unit per block.
    int32_t u, u_end, u_step;
    if constexpr (BATCHED) {
        const int32_t per = (T + kXcds - 1) / kXcds;
        const int32_t xcd = blockIdx.x % kXcds;
        u = xcd * per + blockIdx.x / kXcds;
        u_end = (xcd + 1) * per < T ? (xcd + 1) * per : T;
        u_step = gridDim.x / kXcds;  // the grid is a multiple of kXcds
    } else {
        u = blockIdx.x, u_end = T, u_step = gridDim.x;
    }
    for (; u < u_end; u += u_step) {
        const int32_t i0 = part_i[u], j0 = part_j[u], i1 = part_i[u + 1], j1 = part_j[u + 1];
        const int32_t nrows = i1 - i0, nnzs = j1 - j0;
        int32_t *s_re = reinterpret_cast<int32_t *>(s_buf);
        float *s_pv = s_buf + nrows;

        int32_t mat_lo = 0, mat_hi = 0;
        if constexpr (BATCHED) mat_lo = part_mat[u], mat_hi = part_mat[u + 1];

        // Unconditional loads with indices clamped into the unit.  A row of
        // X wider than one 16-byte load is split over LPN adjacent lanes so
        // that a single instruction fetches it whole (one request per row).
        constexpr int LPN = (VECX && KC * sizeof(VT) > 16) ? static_cast<int>(KC * sizeof(VT) / 16) : 1;
        constexpr int VPL = KC / LPN;  // X values per lane
        constexpr int SLOTS = ITEMS * LPN;
        const int32_t re_last = i1 > i0 ? i1 : i0 + 1 <= rows ? i0 + 1 : rows;
        const int32_t nz_last = nnzs > 0 ? j1 - 1 : (j0 < nnz ? j0 : nnz - 1);
        int32_t re[ITEMS], cc[SLOTS];
        VT vv[SLOTS];
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            const int32_t rk = i0 + 1 + tid + q * BLOCK;
            re[q] = ro[rk < re_last ? rk : re_last];
        }
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
            const int32_t jk = j0 + (tid + q * BLOCK) / LPN;
            cc[q] = ld_stream(ci + (jk < nz_last ? jk : nz_last));
            vv[q] = ld_stream(val + (jk < nz_last ? jk : nz_last));
        }
        int32_t xrow[SLOTS];  // X row of each slot's nonzero (the batch's total columns fit int32)
        if constexpr (BATCHED) {
            if (mat_lo == mat_hi) {
                const int32_t cb = static_cast<int32_t>(col_base[mat_lo]);
#pragma unroll
                for (int q = 0; q < SLOTS; ++q) xrow[q] = cb + cc[q];
            } else {
#pragma unroll
                for (int q = 0; q < SLOTS; ++q) {
                    const int32_t jk = j0 + (tid + q * BLOCK) / LPN;
                    const int64_t j = jk < nz_last ? jk : nz_last;
                    int32_t lo = mat_lo, hi = mat_hi;  // nnz_base[mat_lo] <= j
                    while (lo < hi) {
                        const int32_t mid = (lo + hi + 1) >> 1;
                        if (nnz_base[mid] <= j)
                            lo = mid;
                        else
                            hi = mid - 1;
                    }
                    xrow[q] = static_cast<int32_t>(col_base[lo]) + cc[q];
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) xrow[q] = cc[q];
        }
        float g[SLOTS][VPL];
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
            const int part = (tid + q * BLOCK) % LPN;
            load_row<VPL, VECX>(X + static_cast<int64_t>(xrow[q]) * ldx + part * VPL, g[q]);
        }
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            const int k = tid + q * BLOCK;
            if (k < nrows) s_re[k] = re[q] - j0;
        }
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
            const int sl = tid + q * BLOCK;
            const int k = sl / LPN, part = sl % LPN;
            if (k < nnzs) {
                const float v = to_f32(vv[q]);
#pragma unroll
                for (int c = 0; c < VPL; ++c) s_pv[k * KC + part * VPL + c] = v * g[q][c];
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

        float acc[KC], first_sum[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = first_sum[c] = 0.f;
        int32_t first = -1;
        for (int32_t q = d; q < dend; ++q) {
            if (it < nrows && s_re[it] <= jt) {
                if (first < 0) {
                    first = it;
#pragma unroll
                    for (int c = 0; c < KC; ++c) first_sum[c] = acc[c];
                } else {
                    float *yrow = Y + static_cast<int64_t>(i0 + it) * ldy;
#pragma unroll
                    for (int c = 0; c < KC; ++c) yrow[c] = acc[c];
                }
#pragma unroll
                for (int c = 0; c < KC; ++c) acc[c] = 0.f;
                ++it;
            } else {
#pragma unroll
                for (int c = 0; c < KC; ++c) acc[c] += s_pv[jt * KC + c];
                ++jt;
            }
        }

        float in[KC], tot[KC];
        block_seg_scan_excl_kc<BLOCK, KC>(acc, first >= 0, in, tot, s_wv, s_wf);
        if (first >= 0) {
            float *yrow = Y + static_cast<int64_t>(i0 + first) * ldy;
#pragma unroll
            for (int c = 0; c < KC; ++c) yrow[c] = first_sum[c] + in[c];
        }
        if (tid == 0) {
            carry_row[u] = i1;
#pragma unroll
            for (int c = 0; c < KC; ++c) carry_val[static_cast<int64_t>(u) * KC + c] = tot[c];
        }
        // the scan ended with a barrier: LDS is free for the next unit
    }
}

// Wide-pass consumer that gathers X inside the walk: LDS holds only the row
// ends, the nonzeros' X rows (global row index) and values, so a lane keeps
// just its KC partial sums live and occupancy stays high; each nonzero's KC
// values are fetched when the walk reaches it.
template <int BLOCK, int ITEMS, int KC, bool BATCHED, bool VECX, typename VT>
__global__ __launch_bounds__(BLOCK) void merge_spmm_walk(
    int32_t rows, int32_t nnz, int32_t T, const int32_t *__restrict__ ro, const int32_t *__restrict__ ci,
    const VT *__restrict__ val, const VT *__restrict__ X, int64_t ldx, float *__restrict__ Y, int64_t ldy,
    const int32_t *__restrict__ part_i, const int32_t *__restrict__ part_j, int32_t *__restrict__ carry_row,
    float *__restrict__ carry_val, const int32_t *__restrict__ part_mat, const int64_t *__restrict__ nnz_base,
    const int64_t *__restrict__ col_base) {
    constexpr int W = BLOCK * ITEMS;
    __shared__ int32_t s_buf[W];  // row ends [0, nrows), then X rows of the nonzeros [nrows, nrows + nnzs)
    __shared__ float s_val[W];
    __shared__ float s_wv[BLOCK / kWave * KC];
    __shared__ int s_wf[BLOCK / kWave];

    const int tid = threadIdx.x;
    int32_t u, u_end, u_step;
    if constexpr (BATCHED) {
        const int32_t per = (T + kXcds - 1) / kXcds;
        const int32_t xcd = blockIdx.x % kXcds;
        u = xcd * per + blockIdx.x / kXcds;
        u_end = (xcd + 1) * per < T ? (xcd + 1) * per : T;
        u_step = gridDim.x / kXcds;
    } else {
        u = blockIdx.x, u_end = T, u_step = gridDim.x;
    }
    for (; u < u_end; u += u_step) {
        const int32_t i0 = part_i[u], j0 = part_j[u], i1 = part_i[u + 1], j1 = part_j[u + 1];
        const int32_t nrows = i1 - i0, nnzs = j1 - j0;
        int32_t *s_re = s_buf;
        int32_t *s_xr = s_buf + nrows;
        int32_t mat_lo = 0, mat_hi = 0;
        if constexpr (BATCHED) mat_lo = part_mat[u], mat_hi = part_mat[u + 1];

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
        if constexpr (BATCHED) {
            if (mat_lo == mat_hi) {
                const int32_t cb = static_cast<int32_t>(col_base[mat_lo]);
#pragma unroll
                for (int q = 0; q < ITEMS; ++q) cc[q] += cb;
            } else {
#pragma unroll
                for (int q = 0; q < ITEMS; ++q) {
                    const int32_t jk = j0 + tid + q * BLOCK;
                    const int64_t j = jk < nz_last ? jk : nz_last;
                    int32_t lo = mat_lo, hi = mat_hi;  // nnz_base[mat_lo] <= j
                    while (lo < hi) {
                        const int32_t mid = (lo + hi + 1) >> 1;
                        if (nnz_base[mid] <= j)
                            lo = mid;
                        else
                            hi = mid - 1;
                    }
                    cc[q] += static_cast<int32_t>(col_base[lo]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            const int k = tid + q * BLOCK;
            if (k < nrows) s_re[k] = re[q] - j0;
            if (k < nnzs) {
                s_xr[k] = cc[q];
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

        float acc[KC], first_sum[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = first_sum[c] = 0.f;
        int32_t first = -1;
        for (int32_t q = d; q < dend; ++q) {
            if (it < nrows && s_re[it] <= jt) {
                if (first < 0) {
                    first = it;
#pragma unroll
                    for (int c = 0; c < KC; ++c) first_sum[c] = acc[c];
                } else {
                    float *yrow = Y + static_cast<int64_t>(i0 + it) * ldy;
#pragma unroll
                    for (int c = 0; c < KC; ++c) yrow[c] = acc[c];
                }
#pragma unroll
                for (int c = 0; c < KC; ++c) acc[c] = 0.f;
                ++it;
            } else {
                float g[KC];
                load_row<KC, VECX>(X + static_cast<int64_t>(s_xr[jt]) * ldx, g);
                const float v = s_val[jt];
#pragma unroll
                for (int c = 0; c < KC; ++c) acc[c] += v * g[c];
                ++jt;
            }
        }

        float in[KC], tot[KC];
        block_seg_scan_excl_kc<BLOCK, KC>(acc, first >= 0, in, tot, s_wv, s_wf);
        if (first >= 0) {
            float *yrow = Y + static_cast<int64_t>(i0 + first) * ldy;
#pragma unroll
            for (int c = 0; c < KC; ++c) yrow[c] = first_sum[c] + in[c];
        }
        if (tid == 0) {
            carry_row[u] = i1;
#pragma unroll
            for (int c = 0; c < KC; ++c) carry_val[static_cast<int64_t>(u) * KC + c] = tot[c];
        }
    }
}

// Resident blocks (CUs x occupancy) for the persistent launch.
template <typename K>
static int resident_grid(K kernel, int block) {
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) {
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0);
    }
    return cus * (per_cu > 0 ? per_cu : 1);
}

struct spmm_problem {
    int32_t rows, nnz;
    const int32_t *ro, *ci;
    const void *val;
    int32_t count;
    const int64_t *row_base, *nnz_base, *col_base;
};

template <int BLOCK, int ITEMS, int KC, bool BATCHED, bool VECX, typename VT>
static hipError_t spmm_launch(const spmm_problem &P, const merge_ws &w, const int32_t *part_mat, int64_t T,
                              const VT *X, int64_t ldx, float *Y, int64_t ldy, hipStream_t s) {
    // one column: products staged in LDS (like SpMV); wider: gathers in the walk
    auto kern = [] {
        if constexpr (KC > 1)
            return merge_spmm_walk<BLOCK, ITEMS, KC, BATCHED, VECX, VT>;
        else
            return merge_spmm_consume<BLOCK, ITEMS, KC, BATCHED, VECX, VT>;
    }();
    int64_t grid = T;
    if (BATCHED) {  // a multiple of kXcds, at most the resident blocks
        const int resident = resident_grid(kern, BLOCK);
        const int64_t per = (T + kXcds - 1) / kXcds;
        const int64_t slots = per < resident / kXcds ? per : resident / kXcds;
        grid = kXcds * (slots > 0 ? slots : 1);
    }
    prof_scope p(s, BATCHED ? "batched_consume" : "merge_consume");
    hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(grid)), dim3(BLOCK), 0, s, P.rows, P.nnz,
                       static_cast<int32_t>(T), P.ro, P.ci, static_cast<const VT *>(P.val), X, ldx, Y, ldy, w.part_i,
                       w.part_j, w.carry_row, w.carry_val, part_mat, P.nnz_base, P.col_base);
    return hipGetLastError();
}

template <int BLOCK, int ITEMS, int KC, bool BATCHED, typename VT>
static hipError_t spmm_pass(const spmm_problem &P, const merge_ws &w, const int32_t *part_mat, int64_t T, const VT *X,
                            int64_t ldx, float *Y, int64_t ldy, hipStream_t s) {
    // whole-vector X rows: the pass's first column and the row stride keep
    // every row start aligned to the vector width
    constexpr size_t vbytes = KC * sizeof(VT) < 16 ? KC * sizeof(VT) : 16;
    const bool vecx = KC > 1 && reinterpret_cast<uintptr_t>(X) % vbytes == 0 &&
                      (static_cast<size_t>(ldx) * sizeof(VT)) % vbytes == 0;
    const hipError_t e = vecx ? spmm_launch<BLOCK, ITEMS, KC, BATCHED, true, VT>(P, w, part_mat, T, X, ldx, Y, ldy, s)
                              : spmm_launch<BLOCK, ITEMS, KC, BATCHED, false, VT>(P, w, part_mat, T, X, ldx, Y, ldy, s);
    if (e != hipSuccess) return e;
    return launch_fixup(T, P.rows, KC, w.carry_row, w.carry_val, Y, ldy, s, BATCHED ? "batched_fixup" : "merge_fixup");
}

// One split launch, then passes of at most KC columns.
template <int BLOCK, int ITEMS, bool BATCHED, typename VT>
static hipError_t run_spmm(const spmm_problem &P, const VT *X, int32_t k, int64_t ldx, float *Y, int64_t ldy, void *ws,
                           hipStream_t s) {
    constexpr int W = BLOCK * ITEMS;
    constexpr int KC = spmm_shape<BLOCK, ITEMS>::KC;
    const int64_t T = merge_units(P.rows, P.nnz, W);
    const merge_ws w = merge_ws_carve(ws, T);
    // batched: the matrix of every unit boundary, after the carries (kc = 8 wide)
    int32_t *part_mat = BATCHED ? reinterpret_cast<int32_t *>(static_cast<char *>(ws) + merge_ws_bytes(T, 8)) : nullptr;
    hipError_t e = merge_partition(P.ro, P.rows, P.nnz, W, static_cast<int32_t>(T), w.part_i, w.part_j, s,
                                   BATCHED ? P.row_base : nullptr, P.count, part_mat);
    for (int32_t c0 = 0; c0 < k && e == hipSuccess;) {
        const int32_t left = k - c0;
        if (KC >= 8 && left >= 8) {
            e = spmm_pass<BLOCK, ITEMS, (KC >= 8 ? 8 : 1), BATCHED, VT>(P, w, part_mat, T, X + c0, ldx, Y + c0, ldy, s);
            c0 += 8;
        } else if (KC >= 4 && left >= 4) {
            e = spmm_pass<BLOCK, ITEMS, (KC >= 4 ? 4 : 1), BATCHED, VT>(P, w, part_mat, T, X + c0, ldx, Y + c0, ldy, s);
            c0 += 4;
        } else if (KC >= 2 && left >= 2) {
            e = spmm_pass<BLOCK, ITEMS, (KC >= 2 ? 2 : 1), BATCHED, VT>(P, w, part_mat, T, X + c0, ldx, Y + c0, ldy, s);
            c0 += 2;
        } else {
            e = spmm_pass<BLOCK, ITEMS, 1, BATCHED, VT>(P, w, part_mat, T, X + c0, ldx, Y + c0, ldy, s);
            c0 += 1;
        }
    }
    return e;
}

template <bool BATCHED>
static hipError_t dispatch(const spmm_problem &P, lb_dtype_t dt, const void *X, int32_t k, int64_t ldx, float *Y,
                           int64_t ldy, int block, int items, void *ws, hipStream_t s) {
#define X_(B, I)                                                                                                  \
    if (block == B && items == I) {                                                                               \
        if (dt == LB_BF16)                                                                                        \
            return run_spmm<B, I, BATCHED, bf16_bits>(P, static_cast<const bf16_bits *>(X), k, ldx, Y, ldy, ws, s); \
        return run_spmm<B, I, BATCHED, float>(P, static_cast<const float *>(X), k, ldx, Y, ldy, ws, s);           \
    }
    LB_MERGE_CONFIGS(X_)
#undef X_
    return hipErrorInvalidValue;
}

hipError_t merge_spmm(const csr_dev &A, const void *X, int32_t k, int64_t ldx, float *Y, int64_t ldy, int block,
                      int items, void *ws, hipStream_t s) {
    const spmm_problem P{A.rows, A.nnz, A.ro, A.ci, A.val, 0, nullptr, nullptr, nullptr};
    return dispatch<false>(P, A.dt, X, k, ldx, Y, ldy, block, items, ws, s);
}

size_t batched_ws_bytes(const batch_dev &B, int block, int items, int k) {
    (void)k;  // carries are sized for 8 columns so the boundary matrices follow at a fixed offset
    const int64_t T = merge_units(B.total_rows, B.total_nnz, static_cast<int64_t>(block) * items);
    return merge_ws_bytes(T, 8) + align256(static_cast<size_t>(T + 1) * 4);
}

hipError_t batched_spmm(const batch_dev &B, const void *X, int32_t k, float *Y, int block, int items, void *ws,
                        hipStream_t s) {
    const spmm_problem P{B.total_rows, B.total_nnz, B.ro, B.ci, B.val, B.count, B.row_base, B.nnz_base, B.col_base};
    return dispatch<true>(P, B.dt, X, k, static_cast<int64_t>(k), Y, static_cast<int64_t>(k), block, items, ws, s);
}

}  // namespace lbk
