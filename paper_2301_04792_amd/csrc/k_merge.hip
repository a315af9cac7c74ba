// Merge-path SpMV for gfx950 (Sec. 5.2.1).
//
// Merge-path treats a row end and a nonzero as one unit of work each and
// cuts the merged sequence of rows + nnz units into equal pieces.  With the
// row-end list R[r] = row_offsets[r + 1] and the nonzero list N[j] = j, row
// end r is taken before nonzero j when R[r] <= j, so row end r sits at
// merged position r + row_offsets[r + 1]; the split at diagonal d is
//   i(d) = #{ r : row_offsets[r + 1] + r < d },  j(d) = d - i(d).
//
// Three launches:
//  1. merge_partition_kernel: the split at every unit boundary d_t = t * W
//     (W = BLOCK * ITEMS), one group of 16 lanes per boundary doing a 16-ary
//     search (each round the lanes probe 16 evenly spaced rows and a ballot
//     narrows the range 16-fold: 6 rounds for 2M rows instead of 21).
//  2. merge_spmv_consume: block b owns units [d_b, d_{b+1}): rows
//     [i_b, i_{b+1}) end in it and nonzeros [j_b, j_{b+1}) are consumed in
//     it.  Setup stages the block's row ends and the products
//     values[j] * x[col_idx[j]] in LDS (coalesced, non-temporal streams);
//     each thread searches its own diagonal tid * ITEMS inside that LDS
//     window and walks ITEMS merge items: a row end closes a row ("complete"
//     tile), the trailing open row is its carry ("partial" tile).  A block
//     segmented scan of the carries (wave64 shuffles + LDS across waves)
//     supplies each thread the partial sum earlier threads hold for the first
//     row it closes.  The block's own trailing partial goes to carry[b].
//  3. merge_fixup: rows that cross block boundaries receive the carries of
//     the blocks before them, summed in block order (deterministic; no
//     atomics on y).
//
// Column bands (XCD-aware form, x_bands = 2).  x of a large matrix with
// scattered columns does not fit one XCD's L2, so its gathers miss to the
// Infinity Cache.  With two bands every unit is consumed twice, by two
// blocks that the round-robin dealing of blocks to XCDs puts on different
// XCDs: one multiplies only the nonzeros with col < cb, the other only the
// rest, so each XCD's L2 holds half of x.  The band-0 block writes its row
// sums to y, the band-1 block to a rows-sized buffer; merge_finish_banded
// then adds, per row, the buffer and the carries of both bands (stored
// interleaved, unit-major, so carry_row stays non-decreasing), in place of
// the fix-up.  Both blocks read the
// whole unit's col_idx and values (the second read mostly hits the Infinity
// Cache, so these loads are temporal; loading values only for the block's
// own band was measured slower, as it waits for the column first) and
// gather only their own band's x.
#include "lb_device.h"
#include "lb_internal.h"

namespace lbk {
using namespace lb;

// ------------------------------------------------------------------ partition

// One group of PG lanes per unit boundary (group_merge_search).  16 lanes
// measured faster than 32 or 64: more boundaries per wavefront outweigh the
// extra search levels (6 instead of 4 on 2M rows).
constexpr int kPartitionGroup = 16;

// With row_base (a batch's row prefix sums, count + 1 entries) the group also
// records in part_mat[t] the matrix that owns row min(i_t, rows - 1).
template <int PG>
__global__ __launch_bounds__(256) void merge_partition_kernel(const int32_t *__restrict__ ro,
                                                              int32_t rows, int32_t nnz, int32_t W,
                                                              int32_t T, int32_t *__restrict__ part_i,
                                                              int32_t *__restrict__ part_j,
                                                              const int64_t *__restrict__ row_base,
                                                              int32_t count, int32_t *__restrict__ part_mat) {
    const int64_t t = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / PG;
    const bool live = t <= T;  // uniform per group; every lane still takes part in the ballots
    const int64_t total = static_cast<int64_t>(rows) + nnz;
    const int64_t tt = live ? t : T;
    const int32_t d = static_cast<int32_t>(tt * W < total ? tt * W : total);
    const int32_t i = group_merge_search<PG>(ro, rows, nnz, d);
    int32_t mat = 0;
    if (row_base) {  // uniform across the grid
        const int64_t r = i < rows ? i : rows - 1;
        mat = group_count_le<PG>(row_base, count + 1, r) - 1;  // last b with row_base[b] <= r
        mat = mat < 0 ? 0 : (mat > count - 1 ? count - 1 : mat);
    }
    if (live && (threadIdx.x & (PG - 1)) == 0) {
        part_i[t] = i;
        part_j[t] = d - i;
        if (row_base) part_mat[t] = mat;
    }
}

hipError_t merge_partition(const int32_t *ro, int32_t rows, int32_t nnz, int32_t W, int32_t T,
                           int32_t *part_i, int32_t *part_j, hipStream_t s, const int64_t *row_base, int32_t count,
                           int32_t *part_mat) {
    prof_scope p(s, "merge_partition");
    const int64_t blocks = ((static_cast<int64_t>(T) + 1) * kPartitionGroup + 255) / 256;
    hipLaunchKernelGGL(merge_partition_kernel<kPartitionGroup>, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s,
                       ro, rows, nnz, W, T, part_i, part_j, row_base, count, part_mat);
    return hipGetLastError();
}

// ------------------------------------------------------------------ consume

// One block per unit (the hardware dispatcher balances blocks over CUs):
// the kernel stays at ~20 VGPRs and full occupancy, which hides the stream
// and gather latency better than a register prefetch pipeline that costs
// occupancy.
// BANDS = 1: block b consumes unit b.  BANDS = 2: block b consumes band
// (b mod 8) mod 2 of unit (b / 8) * 4 + (b mod 8) / 2, the grid has
// 8 * ceil(T / 4) blocks and those past the last unit return at once; every
// (unit, band) pair has exactly one block whatever the hardware's dealing.
// VPERM (one band only): nonzero j's value is val[vperm[j]], gathered in the
// same setup as x (the backward's SpMV on A^T reads A's values through the
// transposed pattern's permutation without a permuted copy).
// VEC = 4 (one band, no VPERM): each lane loads four consecutive nonzeros
// with one 16-byte column load and one 16- (float) or 8-byte (BF16) value
// load, from groups aligned to 4 in the arrays, so a lane has four times
// the bytes in flight per instruction.  The x gathers of a wavefront then
// stride by 4 nonzeros, which costs the line sharing that lane-consecutive
// gathers get from long sorted rows, so this form pays only where columns
// are local (a stencil).  The launcher requires nnz >= 4 and aligned
// col_idx / values.
// PLAN (planned SpMV, short rows only): block b takes the b-th active unit
// (T is then the number of active units) and reads its record from the
// plan (the split, the product range, the head, the long flag); each
// block owns the short rows that close in its unit, whole: it adds the head
// of its first row i0 (the nonzeros [ro[i0], j0) before the unit, summed
// by the whole block and handed to thread 0's walk) and leaves out its open
// row i1 (that row is owned by the unit where it closes).  So no carries
// exist and every short row has one writer.  Long rows (at least long_min
// nonzeros) are left out too: as long_min >= W only i0 can be long among
// the closing rows, and then the block neither writes y[i0] nor reads its
// head.  The nonzeros whose products the walk sums are the one range
// [ja, jb).  With units == nullptr (a small one-band lb_spmv, no plan) the
// block finds its unit's split itself, every unit is launched, and no row
// is treated as long.
template <int BLOCK, int ITEMS, typename VT, typename XT, int BANDS, bool VPERM = false, int VEC = 1,
          bool PLAN = false>
__global__ __launch_bounds__(BLOCK) void merge_spmv_consume(
    int32_t rows, int32_t nnz, const int32_t *__restrict__ ro, const int32_t *__restrict__ ci, const VT *__restrict__ val,
    const XT *__restrict__ x, float *__restrict__ y, const int32_t *__restrict__ part_i,
    const int32_t *__restrict__ part_j, int32_t *__restrict__ carry_row, float *__restrict__ carry_val,
    int32_t T, int32_t cb, float *__restrict__ y_hi, const int32_t *__restrict__ vperm,
    const plan_unit *__restrict__ units = nullptr) {
    static_assert(BANDS == 1 || BANDS == 2, "one or two column bands");
    static_assert(!(VPERM && BANDS != 1), "permuted values with one band only");
    static_assert(VEC == 1 || (VEC == 4 && BANDS == 1 && !VPERM && ITEMS % 4 == 0), "vector loads: one band");
    static_assert(!PLAN || !VPERM, "planned form: own values");
    constexpr int W = BLOCK * ITEMS;
    __shared__ int32_t s_buf[W];  // row ends [0, nrows), then products [nrows, nrows + nnzs)
    __shared__ seg_t s_wave[BLOCK / kWave];
    __shared__ float s_head[PLAN ? BLOCK / kWave : 1];

    const int tid = threadIdx.x;
    int b = blockIdx.x, band = 0;
    if constexpr (BANDS == 2) {
        const int xcd = static_cast<int>(blockIdx.x % kXcds);
        band = xcd & 1;
        b = static_cast<int>(blockIdx.x / kXcds) * (kXcds / 2) + xcd / 2;
        if (b >= T) return;  // uniform across the block, before any barrier
        if (band == 1) y = y_hi;
    }
    // the unit's split; planned: its record (one load), which also gives
    // [ja, jb), the nonzeros whose products this block sums, row i0's head
    // [h0, j0) and skip_first (row i0 is long, its y is not written here)
    int32_t i0, i1, j0, j1, ja, jb, h0;
    bool skip_first = false, short_rows = false;
    if constexpr (PLAN) {
        if (units) {
            const plan_unit u = units[b];
            i0 = u.i0, i1 = u.i1, j0 = u.j0, j1 = u.j1, ja = u.ja, jb = u.jb, h0 = u.h0;
            skip_first = (u.flags & 1) != 0;
            short_rows = (u.flags & 2) != 0;
        } else {
            // no plan (a small matrix, one launch): wavefronts 0 and 1 find
            // the split at the unit's two ends; every unit is launched and
            // owns the rows that close in it, no row is treated as long
            __shared__ int32_t s_split[4];
            if (wave_id() < 2) {
                const int64_t dd = static_cast<int64_t>(b + wave_id()) * W;
                const int32_t d = static_cast<int32_t>(dd < static_cast<int64_t>(rows) + nnz ? dd : rows + nnz);
                const int32_t i = wave_merge_search(ro, rows, nnz, d);
                if (lane_id() == 0) s_split[2 * wave_id()] = i, s_split[2 * wave_id() + 1] = d - i;
            }
            __syncthreads();
            i0 = s_split[0], j0 = s_split[1], i1 = s_split[2], j1 = s_split[3];
            if (i0 == i1) return;  // uniform: no row closes in this unit
            h0 = ro[i0];
            ja = j0;
            jb = i1 < rows ? (ro[i1] < j1 ? ro[i1] : j1) : j1;
        }
    } else {
        i0 = part_i[b], j0 = part_j[b];
        i1 = part_i[b + 1], j1 = part_j[b + 1];
        ja = j0, jb = j1, h0 = j0;
    }
    const int32_t nrows = i1 - i0, nnzs = j1 - j0;
    int32_t *s_re = s_buf;
    float *s_pv = reinterpret_cast<float *>(s_buf + nrows);

    // Setup: row ends relative to j0 (in [0, nnzs]) and products, coalesced;
    // consecutive lanes take consecutive nonzeros so that the x gathers of a
    // long row with sorted columns share cache lines.  Every stream load is
    // issued before the first wait, then every gather, then the LDS writes
    // (nrows <= W, so ITEMS row ends per thread cover the unit).
    // Loads are unconditional with indices clamped into the unit (repeats hit
    // the same cache line), so the compiler's wait counts stay exact and all
    // ITEMS gathers of a lane are in flight together.
    const int32_t re_last = i1 > i0 ? i1 : i0 + 1 <= rows ? i0 + 1 : rows;  // a valid row_offsets index
    // nonzero loads are clamped into [nz_first, nz_last], valid indices
    const int32_t nz_last = jb > ja ? jb - 1 : (ja < nnz ? ja : nnz - 1);
    const int32_t nz_first = ja < nz_last ? ja : nz_last;
    int32_t re[ITEMS], c[ITEMS];
    float pv[ITEMS];
    // planned: each thread's first nonzero of row i0's head goes out before
    // the stream loads, its x gather right after them
    const bool has_head = PLAN && h0 + tid < j0;
    int32_t hc = 0;
    VT hv{};
    float hx = 0.f;
    if (has_head) {
        hc = ci[h0 + tid];
        hv = val[h0 + tid];
    }
    auto head_gather = [&]() {
        if (has_head && (BANDS == 1 || (hc >= cb) == (band == 1))) hx = to_f32(x[hc]);
    };
    if constexpr (VEC == 4) {
        using vec_t = typename vec4_of<VT>::type;
        typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
        // groups [vs, vs + 4) with vs a multiple of 4: the block's W / 4
        // groups start at base; a group is used when it lies inside the
        // array (vs <= last_full) and holds a nonzero of the unit
        const int32_t base = j0 & ~3;
        const int32_t last_full = (nnz & ~3) - 4;  // >= 0: nnz >= 4
        const int32_t vmax = last_full < (nz_last & ~3) ? last_full : (nz_last & ~3);
        VT v[ITEMS];
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            const int32_t rk = i0 + 1 + tid + u * BLOCK;
            re[u] = ro[rk < re_last ? rk : re_last];
        }
#pragma unroll
        for (int q = 0; q < ITEMS / 4; ++q) {
            const int32_t vs = base + 4 * (tid + q * BLOCK);
            const int32_t vc = vs <= vmax ? vs : vmax;
            const i32x4 c4 = ld_stream(reinterpret_cast<const i32x4 *>(ci + vc));
            const vec_t v4 = ld_stream(reinterpret_cast<const vec_t *>(val + vc));
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                c[4 * q + e] = c4[e];
                v[4 * q + e] = v4[e];
            }
        }
        head_gather();
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) pv[u] = to_f32(v[u]) * to_f32(x[c[u]]);
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            const int k = tid + u * BLOCK;
            if (k < nrows) s_re[k] = re[u] - j0;
            const int32_t vs = base + 4 * (tid + (u / 4) * BLOCK);
            const int32_t kp = vs + (u % 4) - j0;
            if (vs <= vmax && kp >= 0 && kp < nnzs) s_pv[kp] = PLAN && (kp + j0 < ja || kp + j0 >= jb) ? 0.f : pv[u];
        }
        // nonzeros past the used groups (the unit running past base + W, or
        // the array's last nnz mod 4 entries): at most 3
        const int32_t cov_end = base + W < vmax + 4 ? base + W : vmax + 4;
        const int32_t g = (cov_end > j0 ? cov_end : j0) + tid;
        if (tid < 3 && g < j1)
            s_pv[g - j0] = PLAN && (g < ja || g >= jb) ? 0.f : to_f32(val[g]) * to_f32(x[ci[g]]);
    } else if constexpr (BANDS == 1) {
        VT v[ITEMS];
        float xv[ITEMS];
        int32_t vp[VPERM ? ITEMS : 1];
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            const int32_t k = tid + u * BLOCK;
            const int32_t rk = i0 + 1 + k;
            const int32_t jk = j0 + k;
            const int32_t jc = jk < nz_first ? nz_first : (jk < nz_last ? jk : nz_last);
            re[u] = ro[rk < re_last ? rk : re_last];
            c[u] = ld_stream(ci + jc);
            if constexpr (VPERM)
                vp[u] = ld_stream(vperm + jc);
            else
                v[u] = ld_stream(val + jc);
        }
        head_gather();
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            if constexpr (VPERM) v[u] = val[vp[u]];
            xv[u] = to_f32(x[c[u]]);
        }
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            pv[u] = to_f32(v[u]) * xv[u];
            if constexpr (PLAN) {
                const int32_t jk = j0 + tid + u * BLOCK;
                if (jk < ja || jk >= jb) pv[u] = 0.f;
            }
        }
    } else {
        // band 0 takes col < cb, band 1 col >= cb: x is gathered only for a
        // nonzero of the block's own band
        VT v[ITEMS];
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            const int32_t k = tid + u * BLOCK;
            const int32_t rk = i0 + 1 + k;
            const int32_t jk = j0 + k;
            const int32_t jc = jk < nz_first ? nz_first : (jk < nz_last ? jk : nz_last);
            re[u] = ro[rk < re_last ? rk : re_last];
            c[u] = ci[jc];
            v[u] = val[jc];
        }
        head_gather();
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            bool mine = (c[u] >= cb) == (band == 1);
            if constexpr (PLAN) {
                const int32_t jk = j0 + tid + u * BLOCK;
                mine = mine && jk >= ja && jk < jb;
            }
            pv[u] = mine ? to_f32(v[u]) * to_f32(x[c[u]]) : 0.f;
        }
    }
    if constexpr (VEC == 1) {
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            const int k = tid + u * BLOCK;
            if (k < nrows) s_re[k] = re[u] - j0;
            if (k < nnzs) s_pv[k] = pv[u];
        }
    }
    if constexpr (PLAN) {
        // this thread's share of row i0's head, in its band (hx is 0 outside it)
        float head = has_head ? to_f32(hv) * hx : 0.f;
        constexpr int HU = 8;  // head nonzeros in flight per thread
        for (int32_t j = h0 + tid + BLOCK; j < j0; j += HU * BLOCK) {  // heads longer than the block
            int32_t cj[HU];
            float vj[HU];
#pragma unroll
            for (int k = 0; k < HU; ++k) {
                const int32_t jk = j + k * BLOCK;
                cj[k] = jk < j0 ? ci[jk] : -1;
                vj[k] = jk < j0 ? to_f32(val[jk]) : 0.f;
            }
#pragma unroll
            for (int k = 0; k < HU; ++k)
                if (cj[k] >= 0 && (BANDS == 1 || (cj[k] >= cb) == (band == 1))) head += vj[k] * to_f32(x[cj[k]]);
        }
        head = group_sum_dpp<kWave>(head);
        if (lane_id() == kWave - 1) s_head[wave_id()] = head;
    }
    __syncthreads();

    // Planned unit whose rows each hold at most kRowPerThreadMax of its
    // nonzeros (flag bit 1, from the plan): every row closes here and no
    // row is long enough to need balancing, so thread t sums rows t, t +
    // BLOCK, ... straight from LDS, left to right (row i0 after its head),
    // with no search, walk or scan.
    if constexpr (PLAN) {
        if (short_rows) {  // uniform across the block
            for (int32_t k = tid; k < nrows; k += BLOCK) {
                float acc = 0.f;
                if (k == 0) {
#pragma unroll
                    for (int w = 0; w < BLOCK / kWave; ++w) acc += s_head[w];
                }
                const int32_t lo = k == 0 ? 0 : s_re[k - 1], hi = s_re[k];
                for (int32_t j = lo; j < hi; ++j) acc += s_pv[j];
                if (!(k == 0 && skip_first)) y[i0 + k] = acc;
            }
            return;
        }
    }

    // Thread diagonal inside the block's window: local row end k sits at
    // local merged position k + s_re[k].
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

    // Walk: complete rows are written; the first one waits for the carry-in.
    // Planned: thread 0 starts with row i0's head, in wavefront order.
    float acc = 0.f;
    if constexpr (PLAN) {
        if (tid == 0) {
#pragma unroll
            for (int k = 0; k < BLOCK / kWave; ++k) acc += s_head[k];
        }
    }
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
    if (first >= 0 && !(skip_first && first == 0)) y[i0 + first] = first_sum + in.v;
    if constexpr (!PLAN) {
        if (tid == 0) {
            carry_row[b * BANDS + band] = i1;  // the row still open at the block's end (rows if none)
            carry_val[b * BANDS + band] = tot.v;
        }
    }
}

// Two bands, after the consume: one wavefront per unit v.  The rows that
// close in v, [part_i[v], part_i[v+1]), get the second band's sums
// (y += y_hi); the first of them, i0 = part_i[v], also gets the carries of
// the units before v that ended inside row i0.  Those carries are the run of
// entries equal to i0 that ends at carry index 2v - 1 (unit v-1 always ended
// in row i0), read backwards 64 at a time until a chunk is not all i0.
// Each row has exactly one writer and a fixed summation order.
__global__ __launch_bounds__(256) void merge_finish_banded(int32_t T, const int32_t *__restrict__ part_i,
                                                           const int32_t *__restrict__ carry_row,
                                                           const float *__restrict__ carry_val,
                                                           float *__restrict__ y, const float *__restrict__ y_hi) {
    const int lane = lane_id();
    const int64_t v = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
    if (v >= T) return;  // uniform across the wavefront
    const int32_t i0 = part_i[v], i1 = part_i[v + 1];
    if (i0 >= i1) return;  // no row closes in this unit: its carry goes to a later one
    // the first 64 rows' sums are loaded before the carry chain, which they
    // do not depend on
    const int32_t r0 = i0 + lane;
    const float first = r0 < i1 ? y[r0] + y_hi[r0] : 0.f;
    float carried = 0.f;
    for (int64_t hi = 2 * v;; hi -= kWave) {  // carry entries [0, 2v) precede unit v
        const int64_t q = hi - 1 - lane;
        const bool match = q >= 0 && carry_row[q] == i0;
        carried += group_sum<kWave>(match ? carry_val[q] : 0.f);
        if (__popcll(__ballot(match)) < kWave) break;  // the run started inside this chunk
    }
    if (r0 < i1) y[r0] = lane == 0 ? first + carried : first;
    for (int32_t r = r0 + kWave; r < i1; r += kWave) y[r] = y[r] + y_hi[r];
}

// ------------------------------------------------------------------ fix-up

// One wavefront per chunk of 64 consecutive carry entries.  carry_row is
// non-decreasing, so entries of one row form a run.  The runs that start in
// the chunk are summed by its wavefront: inside the chunk by a segmented scan
// (fixed butterfly), and the chunk's last run, when it goes on past the
// chunk, by reading on 64 entries at a time, adding each chunk in order.  A
// run that began in an earlier chunk belongs to that chunk's wavefront.  The
// run total is added to its row of y (kc columns).  Deterministic: no
// atomics, one writer per row.
__global__ __launch_bounds__(256) void merge_fixup(int32_t T, int32_t rows, int32_t kc,
                                                   const int32_t *__restrict__ carry_row,
                                                   const float *__restrict__ carry_val,
                                                   float *__restrict__ y, int64_t ldy) {
    const int lane = lane_id();
    const int64_t base = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave * kWave;
    if (base >= T) return;  // uniform across the wavefront
    const int64_t b = base + lane;
    const bool in = b < T;
    const int32_t r = in ? carry_row[b] : -1;
    const bool head = in && (b == 0 || carry_row[b - 1] != r);
    const bool tail = in && (b + 1 == T || carry_row[b + 1] != r);
    // the last lane's run goes on into the next chunk
    const bool open = __ballot(lane == kWave - 1 && in && !tail) != 0;
    const int32_t r_open = __shfl(r, kWave - 1);
    for (int32_t c = 0; c < kc; ++c) {
        const seg_t sc = group_seg_scan_incl<kWave>(seg_t{in ? carry_val[b * kc + c] : 0.f, head});
        // sc.f: some run starts at or before this lane inside the chunk, so
        // a tail lane with sc.f ends a run that this chunk owns
        if (tail && sc.f && r < rows) y[static_cast<int64_t>(r) * ldy + c] += sc.v;
        if (open) {
            const bool owned = __shfl(static_cast<int>(sc.f), kWave - 1) != 0;
            if (owned && r_open < rows) {  // uniform
                float total = __shfl(sc.v, kWave - 1);
                for (int64_t s = base + kWave;; s += kWave) {
                    const int64_t q = s + lane;
                    const bool match = q < T && carry_row[q] == r_open;
                    total += group_sum<kWave>(match ? carry_val[q * kc + c] : 0.f);
                    // the run is contiguous: it ends inside this chunk unless every lane matched
                    if (__popcll(__ballot(match)) < kWave) break;
                }
                if (lane == 0) y[static_cast<int64_t>(r_open) * ldy + c] += total;
            }
        }
    }
}

hipError_t launch_fixup(int64_t T, int32_t rows, int32_t kc, const int32_t *carry_row,
                        const float *carry_val, float *y, int64_t ldy, hipStream_t s, const char *tag) {
    if (T <= 0) return hipSuccess;
    prof_scope p(s, tag);
    const int64_t blocks = (T + 255) / 256;  // one wavefront per 64 entries
    hipLaunchKernelGGL(merge_fixup, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s,
                       static_cast<int32_t>(T), rows, kc, carry_row, carry_val, y, ldy);
    return hipGetLastError();
}

// ------------------------------------------------------------------ dispatch

// The four-nonzero load form needs whole aligned groups: nnz >= 4, col_idx
// 16-byte aligned and the values aligned to their 4-element vector.
static bool vector_loads_ok(const csr_dev &A) {
    const uintptr_t va = A.dt == LB_BF16 ? 8 : 16;
    return A.nnz >= 4 && reinterpret_cast<uintptr_t>(A.ci) % 16 == 0 && reinterpret_cast<uintptr_t>(A.val) % va == 0;
}

template <int BLOCK, int ITEMS, typename VT>
static hipError_t run_merge_spmv(const csr_dev &A, const void *x, float *y, int bands, const int32_t *vperm, int vec,
                                 void *ws, hipStream_t s) {
    constexpr int W = BLOCK * ITEMS;
    const int64_t T = merge_units(A.rows, A.nnz, W);
    const bool two = bands == 2;
    merge_ws w = merge_ws_carve(ws, two ? 2 * T : T);
    float *y_hi = two ? reinterpret_cast<float *>(static_cast<char *>(ws) + merge_ws_bytes(2 * T, 1)) : nullptr;
    if (!two && !vperm && T <= kSelfSplitUnits) {
        // a small matrix: one launch, no split launch, no carries, no fix-up
        prof_scope p(s, "merge_consume");
        const VT *val = static_cast<const VT *>(A.val);
        const int32_t cb = static_cast<int32_t>((A.cols + 1) / 2);
        if (vec == 4 && vector_loads_ok(A))
            hipLaunchKernelGGL((merge_spmv_consume<BLOCK, ITEMS, VT, VT, 1, false, 4, true>),
                               dim3(static_cast<uint32_t>(T)), dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci, val,
                               static_cast<const VT *>(x), y, nullptr, nullptr, nullptr, nullptr,
                               static_cast<int32_t>(T), cb, nullptr, nullptr, nullptr);
        else
            hipLaunchKernelGGL((merge_spmv_consume<BLOCK, ITEMS, VT, VT, 1, false, 1, true>),
                               dim3(static_cast<uint32_t>(T)), dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci, val,
                               static_cast<const VT *>(x), y, nullptr, nullptr, nullptr, nullptr,
                               static_cast<int32_t>(T), cb, nullptr, nullptr, nullptr);
        return hipGetLastError();
    }
    hipError_t e = merge_partition(A.ro, A.rows, A.nnz, W, static_cast<int32_t>(T), w.part_i, w.part_j, s);
    if (e != hipSuccess) return e;
    {
        prof_scope p(s, "merge_consume");
        const VT *val = static_cast<const VT *>(A.val);
        const int32_t cb = static_cast<int32_t>((A.cols + 1) / 2);
        if (vperm) {  // x is float32 (the backward's dy) whatever the value type
            hipLaunchKernelGGL((merge_spmv_consume<BLOCK, ITEMS, VT, float, 1, true>), dim3(static_cast<uint32_t>(T)),
                               dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci, val, static_cast<const float *>(x), y,
                               w.part_i, w.part_j, w.carry_row, w.carry_val, static_cast<int32_t>(T), cb, y_hi, vperm);
        } else if (vec == 4 && vector_loads_ok(A)) {
            hipLaunchKernelGGL((merge_spmv_consume<BLOCK, ITEMS, VT, VT, 1, false, 4>), dim3(static_cast<uint32_t>(T)),
                               dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci, val, static_cast<const VT *>(x), y,
                               w.part_i, w.part_j, w.carry_row, w.carry_val, static_cast<int32_t>(T), cb, y_hi,
                               nullptr);
        } else if (two) {
            const int64_t per = kXcds / 2;  // units per row of kXcds blocks
            const int64_t grid = (T + per - 1) / per * kXcds;
            hipLaunchKernelGGL((merge_spmv_consume<BLOCK, ITEMS, VT, VT, 2>), dim3(static_cast<uint32_t>(grid)),
                               dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci, val, static_cast<const VT *>(x), y,
                               w.part_i, w.part_j, w.carry_row, w.carry_val, static_cast<int32_t>(T), cb, y_hi,
                               nullptr);
        } else {
            hipLaunchKernelGGL((merge_spmv_consume<BLOCK, ITEMS, VT, VT, 1>), dim3(static_cast<uint32_t>(T)),
                               dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci, val, static_cast<const VT *>(x), y,
                               w.part_i, w.part_j, w.carry_row, w.carry_val, static_cast<int32_t>(T), cb, y_hi,
                               nullptr);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (two) {
        prof_scope p(s, "merge_finish");
        const int64_t g = (T + 3) / 4;  // a wavefront per unit
        hipLaunchKernelGGL(merge_finish_banded, dim3(static_cast<uint32_t>(g)), dim3(256), 0, s,
                           static_cast<int32_t>(T), w.part_i, w.carry_row, w.carry_val, y, y_hi);
        return hipGetLastError();
    }
    return launch_fixup(T, A.rows, 1, w.carry_row, w.carry_val, y, 1, s, "merge_fixup");
}

template <int BLOCK, int ITEMS, typename VT>
static hipError_t run_planned_consume(const csr_dev &A, const plan_dev &pl, const void *x, float *y, float *y_hi,
                                      hipStream_t s) {
    prof_scope p(s, "merge_consume");
    const VT *val = static_cast<const VT *>(A.val);
    const VT *xx = static_cast<const VT *>(x);
    const int32_t cb = static_cast<int32_t>((A.cols + 1) / 2);
    if (pl.bands == 2) {
        const int64_t per = kXcds / 2;
        const int64_t grid = (pl.NA + per - 1) / per * kXcds;
        hipLaunchKernelGGL((merge_spmv_consume<BLOCK, ITEMS, VT, VT, 2, false, 1, true>),
                           dim3(static_cast<uint32_t>(grid)), dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci, val, xx, y,
                           pl.part_i, pl.part_j, nullptr, nullptr, pl.NA, cb, y_hi, nullptr, pl.units);
    } else if (pl.vec == 4 && vector_loads_ok(A)) {
        hipLaunchKernelGGL((merge_spmv_consume<BLOCK, ITEMS, VT, VT, 1, false, 4, true>),
                           dim3(static_cast<uint32_t>(pl.NA)), dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci, val, xx,
                           y, pl.part_i, pl.part_j, nullptr, nullptr, pl.NA, cb, nullptr, nullptr, pl.units);
    } else {
        hipLaunchKernelGGL((merge_spmv_consume<BLOCK, ITEMS, VT, VT, 1, false, 1, true>),
                           dim3(static_cast<uint32_t>(pl.NA)), dim3(BLOCK), 0, s, A.rows, A.nnz, A.ro, A.ci, val, xx,
                           y, pl.part_i, pl.part_j, nullptr, nullptr, pl.NA, cb, nullptr, nullptr, pl.units);
    }
    return hipGetLastError();
}

hipError_t merge_spmv_planned_consume(const csr_dev &A, const plan_dev &pl, const void *x, float *y, float *y_hi,
                                      hipStream_t s) {
#define X(B, I)                                                                              \
    if (pl.block == B && pl.items == I) {                                                    \
        if (A.dt == LB_BF16) return run_planned_consume<B, I, bf16_bits>(A, pl, x, y, y_hi, s); \
        return run_planned_consume<B, I, float>(A, pl, x, y, y_hi, s);                      \
    }
    LB_MERGE_CONFIGS(X)
#undef X
    return hipErrorInvalidValue;
}

bool merge_config_supported(int block, int items) {
#define X(B, I) if (block == B && items == I) return true;
    LB_MERGE_CONFIGS(X)
#undef X
    return false;
}

hipError_t merge_spmv(const csr_dev &A, const void *x, float *y, int block, int items, int bands, void *ws,
                      hipStream_t s, const int32_t *vperm, int vec) {
    if (bands != 1 && bands != 2) return hipErrorInvalidValue;
    if (vec != 1 && vec != 4) return hipErrorInvalidValue;
    if ((vperm || vec == 4) && bands != 1) return hipErrorInvalidValue;
    if (vperm && vec != 1) return hipErrorInvalidValue;
#define X(B, I)                                                                                     \
    if (block == B && items == I) {                                                                 \
        if (A.dt == LB_BF16) return run_merge_spmv<B, I, bf16_bits>(A, x, y, bands, vperm, vec, ws, s); \
        return run_merge_spmv<B, I, float>(A, x, y, bands, vperm, vec, ws, s);                      \
    }
    LB_MERGE_CONFIGS(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace lbk
