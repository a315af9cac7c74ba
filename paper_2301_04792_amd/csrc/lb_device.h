// Device-side vocabulary of the load-balancing model for gfx950 (wave64).
//
//  * element loads: float32 and BF16 bit patterns widened to float; the
//    nonzero streams (col_idx, values) are read with non-temporal loads so
//    they do not evict the gathered x from L2;
//  * ranges, tile sets and the thread- and group-mapped schedules come from
//    the public header lb_schedule.hpp;
//  * the merge-path split search (Sec. 5.2.1);
//  * wave64 collectives: group sums, prefix sums and the segmented scan that
//    merge-path and group-mapped use to combine partial tile results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lb_schedule.hpp"  // ranges, tile sets, thread- and group-mapped schedules, int scans

namespace lb {

constexpr int kXcds = 8;  // accelerator dies of an MI355X; workgroups are dealt to them round-robin

// Rounds per work-queue claim so that a whole launch makes at most about
// kMaxClaims claims on its one counter (rounds: rounds of the launch).
constexpr int64_t kMaxClaims = 4096;
__device__ __forceinline__ int64_t claim_batch(int64_t rounds) {
    const int64_t b = rounds / kMaxClaims;
    return b < 1 ? 1 : b;
}

using bf16_bits = uint16_t;

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(bf16_bits v) {
    return __uint_as_float(static_cast<uint32_t>(v) << 16);
}

// Streamed once: keep out of the caches' retained set.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) {
    return __builtin_nontemporal_load(p);
}

// Four consecutive elements as one vector load (16 bytes of float, 8 of BF16).
template <typename T>
struct vec4_of;
template <>
struct vec4_of<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct vec4_of<bf16_bits> {
    typedef uint16_t type __attribute__((ext_vector_type(4)));
};

// ---------------------------------------------------------------- merge-path split (Sec. 5.2.1)

// Count of the positions r in [lo, hi) with key(r) < d, where key is
// increasing, every r < lo counts and no r >= hi does; found by an aligned
// group of G lanes (G a power of two <= 64) with a G-ary search: each step
// the G lanes probe G evenly spaced positions and a ballot narrows the range
// G-fold.  All lanes of the wavefront must execute it (the ballot spans the
// wavefront); every lane of a group returns the same value.
template <int G, typename Key>
__device__ __forceinline__ int32_t group_count_below(int32_t lo, int32_t hi, int32_t d, Key key) {
    const int gl = threadIdx.x & (G - 1);
    const int shift = (threadIdx.x & (kWave - 1)) & ~(G - 1);
    const uint64_t gmask = G >= 64 ? ~0ull : ((1ull << (G & 63)) - 1);
    for (;;) {
        const bool wide = hi - lo > G;
        if (__ballot(wide) == 0) break;  // every group of the wavefront has narrowed down
        const int32_t step = wide ? (hi - lo + G - 1) / G : 1;
        const int32_t r = lo + (gl + 1) * step - 1;
        const bool below = wide && r < hi && key(r) < d;  // true on a prefix of the group
        const int32_t c = __popcll((__ballot(below) >> shift) & gmask);
        if (wide) {
            const int32_t rc = lo + (c + 1) * step - 1;  // first probe not below d
            hi = rc < hi ? rc : hi;
            lo = lo + c * step;
        }
    }
    const int32_t r = lo + gl;
    const bool below = r < hi && key(r) < d;
    return lo + __popcll((__ballot(below) >> shift) & gmask);
}

// Number of row ends of the merge of row_offsets[1..rows] with the nonzero
// indices 0..nnz-1 that precede diagonal d: row end r is the
// (r + row_offsets[r + 1])-th merge item.  Rows below d - nnz end before d
// and rows at or past d cannot.
template <int G>
__device__ __forceinline__ int32_t group_merge_search(const int32_t *__restrict__ ro, int32_t rows, int32_t nnz,
                                                      int32_t d) {
    const int32_t lo = d - nnz > 0 ? d - nnz : 0;
    const int32_t hi = d < rows ? d : rows;
    return group_count_below<G>(lo, hi, d, [ro](int32_t r) { return ro[r + 1] + r; });
}

// The same split for a row-sorted COO: nonzero j is the (j + row_idx[j])-th
// merge item (the rows before it have ended, its own row has not), so the
// nonzeros preceding d are counted directly; the row ends are d minus that.
// Nonzeros below d - rows precede d and those at or past d cannot.
template <int G>
__device__ __forceinline__ int32_t group_coo_search(const int32_t *__restrict__ row_idx, int32_t rows, int32_t nnz,
                                                    int32_t d) {
    const int32_t lo = d - rows > 0 ? d - rows : 0;
    const int32_t hi = d < nnz ? d : nnz;
    return group_count_below<G>(lo, hi, d, [row_idx](int32_t j) { return row_idx[j] + j; });
}

template <int G>
__device__ __forceinline__ int32_t group_count_le(const int64_t *__restrict__ a, int32_t n, int64_t key) {
    const int gl = threadIdx.x & (G - 1);
    const int shift = (threadIdx.x & (kWave - 1)) & ~(G - 1);
    const uint64_t gmask = G >= 64 ? ~0ull : ((1ull << (G & 63)) - 1);
    int32_t lo = 0, hi = n;  // a[r] <= key for r < lo, a[r] > key for r >= hi
    for (;;) {
        const bool wide = hi - lo > G;
        if (__ballot(wide) == 0) break;
        const int32_t step = wide ? (hi - lo + G - 1) / G : 1;
        const int32_t r = lo + (gl + 1) * step - 1;
        const bool le = wide && r < hi && a[r] <= key;
        const int32_t c = __popcll((__ballot(le) >> shift) & gmask);
        if (wide) {
            const int32_t rc = lo + (c + 1) * step - 1;
            hi = rc < hi ? rc : hi;
            lo = lo + c * step;
        }
    }
    const int32_t r = lo + gl;
    return lo + __popcll((__ballot(r < hi && a[r] <= key) >> shift) & gmask);
}

__device__ __forceinline__ int32_t wave_merge_search(const int32_t *__restrict__ ro, int32_t rows, int32_t nnz,
                                                     int32_t d) {
    return group_merge_search<kWave>(ro, rows, nnz, d);
}

// ---------------------------------------------------------------- wave64 collectives

// Sum over aligned groups of G lanes (G a power of two <= 64); every lane of
// the group gets the total.  Fixed butterfly order: deterministic.
template <int G>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

// Sum over aligned groups of G lanes (G = 8, 16, 32 or 64) with DPP lane
// moves, which run on the VALU instead of the LDS crossbar that __shfl_xor
// (ds_bpermute) occupies.  The group's last lane gets the total (for G <= 16
// every lane of the group does).  Steps: swaps inside quads (quad_perm
// [1,0,3,2] and [2,3,0,1]), the mirror inside each half-row of 8 lanes, the
// mirror inside each row of 16, then lane 15 of rows 0 and 2 added into rows
// 1 and 3 (row_bcast15, row mask 0b1010) and lane 31 into rows 2 and 3
// (row_bcast31, row mask 0b1100).  Fixed order: deterministic.
template <int G>
__device__ __forceinline__ float group_sum_dpp(float v) {
    static_assert(G == 8 || G == 16 || G == 32 || G == 64, "groups of 8 to 64 lanes");
    auto mov = [](float a, auto ctrl, auto row_mask) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), decltype(ctrl)::value,
                                                          decltype(row_mask)::value, 0xF, false));
    };
    using qp_1032 = std::integral_constant<int, 0xB1>;
    using qp_2301 = std::integral_constant<int, 0x4E>;
    using half_mirror = std::integral_constant<int, 0x141>;
    using mirror = std::integral_constant<int, 0x140>;
    using bcast15 = std::integral_constant<int, 0x142>;
    using bcast31 = std::integral_constant<int, 0x143>;
    using all_rows = std::integral_constant<int, 0xF>;
    v += mov(v, qp_1032{}, all_rows{});
    v += mov(v, qp_2301{}, all_rows{});
    v += mov(v, half_mirror{}, all_rows{});
    if constexpr (G >= 16) v += mov(v, mirror{}, all_rows{});
    if constexpr (G >= 32) v += mov(v, bcast15{}, std::integral_constant<int, 0xA>{});
    if constexpr (G >= 64) v += mov(v, bcast31{}, std::integral_constant<int, 0xC>{});
    return v;
}

// A segmented-scan element: value and "a segment starts here" flag.  The
// operator drops everything before a flagged element:
//   (va, fa) . (vb, fb) = (fb ? vb : va + vb, fa | fb)
// Merge-path uses it with flag = "this thread finished a row", so the scan
// of the threads' trailing partial sums gives each thread the partial sum
// that earlier threads hold for the row it finishes first.
struct seg_t {
    float v;
    int f;
};

__device__ __forceinline__ seg_t seg_combine(seg_t a, seg_t b) {
    return {b.f ? b.v : a.v + b.v, a.f | b.f};
}

// Inclusive segmented scan over aligned groups of G lanes (G <= 64).
template <int G>
__device__ __forceinline__ seg_t group_seg_scan_incl(seg_t x) {
    const int gl = threadIdx.x & (G - 1);
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
        const float v = __shfl_up(x.v, off, G);
        const int f = __shfl_up(x.f, off, G);
        if (gl >= off) x = seg_combine(seg_t{v, f}, x);
    }
    return x;
}

// Block-wide inclusive segmented scan; s_wave holds BLOCK/64 entries.  All
// threads of the block must call it.  Ends with a barrier so s_wave can be
// reused.  Also returns the block total.
template <int BLOCK>
__device__ __forceinline__ seg_t block_seg_scan_incl(seg_t x, seg_t *s_wave, seg_t &total) {
    constexpr int NW = BLOCK / kWave;
    const int lane = lane_id(), w = wave_id();
    seg_t inc = group_seg_scan_incl<kWave>(x);
    if (lane == kWave - 1) s_wave[w] = inc;
    __syncthreads();
    seg_t pre{0.f, 0};
    seg_t tot{0.f, 0};
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const seg_t s = s_wave[k];
        if (k < w) pre = seg_combine(pre, s);
        tot = seg_combine(tot, s);
    }
    __syncthreads();
    total = tot;
    return w ? seg_combine(pre, inc) : inc;
}

// Block-wide exclusive segmented scan (lane 0 of the block gets {0, 0}).
template <int BLOCK>
__device__ __forceinline__ seg_t block_seg_scan_excl(seg_t x, seg_t *s_wave, seg_t &total) {
    constexpr int NW = BLOCK / kWave;
    const int lane = lane_id(), w = wave_id();
    const seg_t inc = group_seg_scan_incl<kWave>(x);
    if (lane == kWave - 1) s_wave[w] = inc;
    __syncthreads();
    seg_t pre{0.f, 0};
    seg_t tot{0.f, 0};
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const seg_t s = s_wave[k];
        if (k < w) pre = seg_combine(pre, s);
        tot = seg_combine(tot, s);
    }
    __syncthreads();
    total = tot;
    const float pv = __shfl_up(inc.v, 1, kWave);
    const int pf = __shfl_up(inc.f, 1, kWave);
    return lane ? seg_combine(pre, seg_t{pv, pf}) : pre;
}

// Block-wide exclusive segmented scan of KC values sharing one flag per
// thread (the same operator as seg_t), in one pass: KC values per shuffle
// step and one LDS exchange, so two barriers whatever KC is.  s_wv holds
// BLOCK/64 * KC floats, s_wf BLOCK/64 ints.  ex[c] = exclusive prefix,
// tot[c] = block total; ends with a barrier.
template <int BLOCK, int KC>
__device__ __forceinline__ void block_seg_scan_excl_kc(const float (&v)[KC], int flag, float (&ex)[KC],
                                                       float (&tot)[KC], float *s_wv, int *s_wf) {
    constexpr int NW = BLOCK / kWave;
    const int lane = lane_id(), w = wave_id();
    float inc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) inc[c] = v[c];
    int f = flag;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int pf = __shfl_up(f, off, kWave);
        float pv[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) pv[c] = __shfl_up(inc[c], off, kWave);
        if (lane >= off) {
#pragma unroll
            for (int c = 0; c < KC; ++c) inc[c] = f ? inc[c] : pv[c] + inc[c];
            f |= pf;
        }
    }
    if (lane == kWave - 1) {
        s_wf[w] = f;
#pragma unroll
        for (int c = 0; c < KC; ++c) s_wv[w * KC + c] = inc[c];
    }
    __syncthreads();
    float pre[KC], all[KC];
    int pre_f = 0, all_f = 0;
#pragma unroll
    for (int c = 0; c < KC; ++c) pre[c] = all[c] = 0.f;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int fk = s_wf[k];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            const float vk = s_wv[k * KC + c];
            if (k < w) pre[c] = fk ? vk : pre[c] + vk;
            all[c] = fk ? vk : all[c] + vk;
        }
        if (k < w) pre_f |= fk;
        all_f |= fk;
    }
    __syncthreads();
    // exclusive within the wavefront: the inclusive value of the lane before
    const int ef = __shfl_up(f, 1, kWave);
#pragma unroll
    for (int c = 0; c < KC; ++c) {
        const float ev = __shfl_up(inc[c], 1, kWave);
        ex[c] = lane ? (ef ? ev : pre[c] + ev) : pre[c];
        tot[c] = all[c];
    }
    (void)pre_f;
    (void)all_f;
}

// Block-wide sum (all threads call; every thread gets the total).  s_red
// holds BLOCK/64 floats.  Waves are added in index order: deterministic.
template <int BLOCK>
__device__ __forceinline__ float block_sum(float v, float *s_red) {
    constexpr int NW = BLOCK / kWave;
    v = group_sum<kWave>(v);
    if (lane_id() == 0) s_red[wave_id()] = v;
    __syncthreads();
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < NW; ++k) t += s_red[k];
    __syncthreads();
    return t;
}

}  // namespace lb
