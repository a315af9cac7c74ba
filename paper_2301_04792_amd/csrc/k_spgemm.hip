// C = A B, Gustavson's row-by-row sparse product (Sec. 5.3 names it as the
// extension of SpMM: one kernel sizes each output row, the output is
// allocated, a second kernel multiplies).  Row i of C is the union of the
// rows of B selected by row i of A, each scaled by the A entry.
//
// Work per row is its product count p_i = sum over A entries of the length
// of the selected B row, which ranges from a few to millions on power-law
// inputs.  Rows are sorted into four tiers by p_i, each with its own
// accumulator:
//   tier 0 (p_i <= 32):    an 8-lane group per row, the same with a fixed
//                           32-element network, eight rows per wavefront;
//   tier 1 (p_i <= 256):   one wavefront per row; the products, keyed by
//                           (column, product index), are bitonic-sorted in
//                           the wavefront's LDS; equal columns are then
//                           adjacent, in product order;
//   tier 2 (p_i <= 4096):  one block per row, the same in block LDS;
//   tier 3 (larger):       blocks of a work queue (32 to 512, as many as
//                           1 GiB of slots holds), each owning a slot of
//                           global memory with a dense float accumulator
//                           and a two-level column bitmap; products are
//                           enumerated by the group_mapped_scan schedule
//                           over the row's A entries (tiles) and their B
//                           rows (atoms); the columns come out ascending by
//                           walking the bitmap.
// The count pass runs the same tiers without values and writes each row's
// column count; an int64 scan turns them into C's row offsets.  Tiers 1 and
// 2 sum each column's products in product order (deterministic); tier 3
// adds them with float atomics (order varies run to run).
#include "lb_device.h"
#include "lb_internal.h"
#include "lb_schedule.hpp"

namespace lbk {
using namespace lb;

namespace {

constexpr int kTier0 = 32;  // an 8-lane group per row, 8 rows per wavefront
constexpr int kTier1 = 256;
constexpr int kTier2 = 4096;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr uint64_t kPad = ~0ull;  // sorts after every real key

struct gemm_args {
    int32_t m, n;
    const int32_t *a_ro, *a_ci;
    const float *a_val;
    const int32_t *b_ro, *b_ci;
    const float *b_val;
    const int64_t *prod;   // products per row
    int32_t *lists;        // tier lists: [0, m) tier 1, [m, 2m) tier 2, [2m, 3m) tier 3, [3m, 4m) tier 0
    int32_t *list_len;     // counters of tiers 1, 2, 3, the tier-3 work-queue ticket, the tier-0 counter
    int32_t *c_ro;         // count pass: per-row column counts; compute pass: C's row offsets
    int32_t *c_ci;
    float *c_val;
    float *slot_acc;       // tier 3: slots x n floats
    uint32_t *slot_bits;   // tier 3: slots x (n/32 words + n/1024 summary words)
    int64_t slot_words;    // words per slot bitmap (level 0 then level 1)
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int32_t next_pow2(int32_t v) {
    int32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// ---------------------------------------------------------------- products per row and tiers

// A wavefront per row of A (rows of eight or more entries on average).
__global__ __launch_bounds__(256) void gemm_products_rows(gemm_args g, int64_t *__restrict__ prod) {
    const group_mapped<kWave, csr_tile_set> sch{{g.a_ro, g.m, 0}};
    for (int64_t i : sch.tiles()) {
        int64_t p = 0;
        for (int64_t e : sch.atoms(sch.ts.tile(i))) {
            const int32_t j = g.a_ci[e];
            p += g.b_ro[j + 1] - g.b_ro[j];
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) p += __shfl_xor(p, off, kWave);
        if (sch.lane() == 0) prod[i] = p;
    }
}

// For short rows: group_mapped_scan over A's rows: a wavefront takes 64 rows and strides
// their flattened entries, so short and long rows share the lanes; each
// step sums its entries' B row lengths per row (a segmented sum over the
// lanes) into the rows' LDS counters (exact, int64).
__global__ __launch_bounds__(256) void gemm_products(gemm_args g, int64_t *__restrict__ prod) {
    using sched = group_mapped_scan<kWave, csr_tile_set>;
    __shared__ typename sched::storage s_st[sched::GPB];
    __shared__ unsigned long long s_cnt[sched::GPB][kWave];
    const int gi = threadIdx.x / kWave, gl = lane_id();
    sched sch(csr_tile_set{g.a_ro, g.m, 0}, s_st);
    for (int64_t round : sch.rounds()) {  // uniform across the block
        s_cnt[gi][gl] = 0;
        const int32_t total = sch.load(round);  // ends with a barrier: the counters are clear
        const int32_t steps = (total + kWave - 1) / kWave;
        for (int32_t st = 0; st < steps; ++st) {  // uniform within the wavefront
            const int32_t at = st * kWave + gl;
            int32_t q = kWave;  // past the last row: inactive lane
            unsigned long long v = 0;
            if (at < total) {
                q = sch.get_tile(at);
                const int32_t j = g.a_ci[sch.atom(at, q)];
                v = static_cast<unsigned long long>(g.b_ro[j + 1] - g.b_ro[j]);
            }
            // the step's atoms are in row order: sum each run of equal q over
            // the lanes, then its last lane adds the run to the row's counter
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const unsigned long long v2 = __shfl_up(v, off, kWave);
                const int32_t q2 = __shfl_up(q, off, kWave);
                if (gl >= off && q2 == q) v += v2;
            }
            const int32_t qn = __shfl_down(q, 1, kWave);
            if (q < kWave && (gl == kWave - 1 || qn != q)) s_cnt[gi][q] += v;
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        const int64_t i = (round + gi) * kWave + gl;
        if (i < g.m) prod[i] = static_cast<int64_t>(s_cnt[gi][gl]);
        sch.done();
    }
}

// Rows into their tier's list.  A block takes kClassRows consecutive rows
// in two passes: it counts its rows per tier (per wavefront, then in LDS),
// reserves its stretch of each list with one atomicAdd per tier, and writes
// each wavefront's rows from its own offset in that stretch.  (One atomic per
// wavefront and tier put ~16k atomics on the one counter of a 1M-row
// matrix whose rows share a tier, ~200 µs of serialized atomics.)
constexpr int kClassRows = 1024;

__device__ __forceinline__ int gemm_tier_of(int64_t p) {
    return p < 0 ? -1 : (p <= kTier0 ? 3 : (p <= kTier1 ? 0 : (p <= kTier2 ? 1 : 2)));
}

__global__ __launch_bounds__(256) void gemm_classify(gemm_args g) {
    __shared__ int32_t s_cnt[4][4];  // [wavefront][list]
    __shared__ int32_t s_base[4];
    const int w = wave_id(), lane = lane_id();
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kClassRows;
    const int64_t r1 = r0 + kClassRows < g.m ? r0 + kClassRows : g.m;
    // pass 1: this wavefront's rows per list (list t holds tier t + 1 for t < 3, tier 0 for t = 3)
    int32_t cnt[4] = {0, 0, 0, 0};
    for (int64_t i0 = r0 + w * kWave; i0 < r1; i0 += 256) {  // uniform per wavefront
        const int64_t i = i0 + lane;
        const int t = gemm_tier_of(i < r1 ? g.prod[i] : -1);
#pragma unroll
        for (int q = 0; q < 4; ++q) cnt[q] += __popcll(__ballot(t == q));
    }
    if (lane == 0)
        for (int q = 0; q < 4; ++q) s_cnt[w][q] = cnt[q];
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        const int32_t total = s_cnt[0][q] + s_cnt[1][q] + s_cnt[2][q] + s_cnt[3][q];
        s_base[q] = total > 0 ? atomicAdd(g.list_len + (q == 3 ? 4 : q), total) : 0;
    }
    __syncthreads();
    // pass 2: the same rows in the same order, each list from this wavefront's offset
    int32_t off[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        off[q] = s_base[q];
        for (int v = 0; v < w; ++v) off[q] += s_cnt[v][q];
    }
    for (int64_t i0 = r0 + w * kWave; i0 < r1; i0 += 256) {
        const int64_t i = i0 + lane;
        const int t = gemm_tier_of(i < r1 ? g.prod[i] : -1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t mask = __ballot(t == q);
            if (t == q)
                g.lists[static_cast<int64_t>(q) * g.m + off[q] + __popcll(mask & ((1ull << lane) - 1))] =
                    static_cast<int32_t>(i);
            off[q] += __popcll(mask);
        }
    }
}

// ---------------------------------------------------------------- tiers 1 and 2: sort in LDS

// Bitonic sort of key[0, np2) (np2 a power of two) with its values, by
// threads [t0, t0 + nt) of the block; sync() orders LDS between steps.
template <bool VALUES, typename Sync>
__device__ __forceinline__ void lds_bitonic(uint64_t *key, float *val, int32_t np2, int t, int nt, Sync sync) {
    for (int32_t k = 2; k <= np2; k <<= 1) {
        for (int32_t j = k >> 1; j > 0; j >>= 1) {
            for (int32_t x = t; x < np2 / 2; x += nt) {
                const int32_t lo = 2 * j * (x / j) + (x % j);
                const int32_t hi = lo + j;
                const bool up = (lo & k) == 0;
                const uint64_t a = key[lo], b = key[hi];
                if ((a > b) == up) {
                    key[lo] = b;
                    key[hi] = a;
                    if constexpr (VALUES) {
                        const float va = val[lo];
                        val[lo] = val[hi];
                        val[hi] = va;
                    }
                }
            }
            sync();
        }
    }
}

// Tier 0: an 8-lane group per row (p <= 32), eight rows per wavefront; all
// groups run the same 32-element sort network, so the wavefront stays in
// step (a group whose rows ran out is masked off).
template <bool COMPUTE>
__global__ __launch_bounds__(kBlock) void gemm_tier0(gemm_args g) {
    constexpr int GL = 8;
    constexpr int GPB = kBlock / GL;
    __shared__ uint64_t s_key[GPB][kTier0];
    __shared__ float s_val[GPB][COMPUTE ? kTier0 : 1];
    const int gl = threadIdx.x & (GL - 1), gi = threadIdx.x / GL;
    const int shift = lane_id() & ~(GL - 1);  // the group's first lane in the wavefront
    uint64_t *key = s_key[gi];
    float *val = s_val[gi];
    const int32_t rows = g.list_len[4];
    const int64_t groups = static_cast<int64_t>(gridDim.x) * GPB;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * GPB + gi; r < rows; r += groups) {
        const int32_t i = g.lists[3 * static_cast<int64_t>(g.m) + r];
        const int32_t p = static_cast<int32_t>(g.prod[i]);
        const int32_t a0 = g.a_ro[i], a1 = g.a_ro[i + 1];
        int32_t base = 0;
        for (int32_t c0 = a0; c0 < a1; c0 += GL) {
            const int32_t e = c0 + gl;
            int32_t j = 0, len = 0;
            if (e < a1) {
                j = g.a_ci[e];
                len = g.b_ro[j + 1] - g.b_ro[j];
            }
            const int32_t incl = group_scan_incl<GL>(len);
            const int32_t start = base + incl - len;
            if (len > 0) {
                const int32_t f0 = g.b_ro[j];
                const float a = COMPUTE ? g.a_val[e] : 0.f;
                for (int32_t t = 0; t < len; ++t) {
                    const int32_t q = start + t;
                    key[q] = (static_cast<uint64_t>(g.b_ci[f0 + t]) << 32) | static_cast<uint32_t>(q);
                    if constexpr (COMPUTE) val[q] = a * g.b_val[f0 + t];
                }
            }
            base += __shfl(incl, GL - 1, GL);
        }
        for (int32_t q = p + gl; q < kTier0; q += GL) key[q] = kPad;
        wave_sync();
        lds_bitonic<COMPUTE>(key, val, kTier0, gl, GL, wave_sync);
        int32_t rank = 0;
        float carry = 0.f;
        const int32_t out0 = COMPUTE ? g.c_ro[i] : 0;
        for (int32_t c0 = 0; c0 < p; c0 += GL) {
            const int32_t q = c0 + gl;
            const bool in = q < p;
            const uint32_t col = in ? static_cast<uint32_t>(key[q] >> 32) : 0xffffffffu;
            const uint32_t prev = q > 0 && in ? static_cast<uint32_t>(key[q - 1] >> 32) : 0xffffffffu;
            const bool head = in && (q == 0 || col != prev);
            const uint32_t hm = static_cast<uint32_t>((__ballot(head) >> shift) & 0xffu);
            if constexpr (COMPUTE) {
                const bool tail = in && (q == p - 1 || static_cast<uint32_t>(key[q + 1] >> 32) != col);
                seg_t sv = group_seg_scan_incl<GL>(seg_t{in ? val[q] : 0.f, head});
                if (!sv.f) sv.v += carry;
                const int32_t my_rank = rank + __popc(hm & ((2u << gl) - 1)) - 1;
                if (tail) {
                    g.c_ci[out0 + my_rank] = static_cast<int32_t>(col);
                    g.c_val[out0 + my_rank] = sv.v;
                }
                carry = __shfl(sv.v, GL - 1, GL);
            }
            rank += __popc(hm);
        }
        if constexpr (!COMPUTE) {
            if (gl == 0) g.c_ro[i] = rank;
        }
        wave_sync();
    }
}

// Tier 1: a wavefront per row.
template <bool COMPUTE>
__global__ __launch_bounds__(kBlock) void gemm_tier1(gemm_args g) {
    __shared__ uint64_t s_key[kWavesPerBlock][kTier1];
    __shared__ float s_val[kWavesPerBlock][COMPUTE ? kTier1 : 1];
    const int lane = lane_id(), w = wave_id();
    uint64_t *key = s_key[w];
    float *val = s_val[w];
    const int32_t rows = g.list_len[0];
    const int64_t waves = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + w; r < rows; r += waves) {
        const int32_t i = g.lists[r];
        const int32_t p = static_cast<int32_t>(g.prod[i]);
        const int32_t a0 = g.a_ro[i], a1 = g.a_ro[i + 1];
        // expand: 64 A entries at a time; lane l writes its entry's products
        int32_t base = 0;
        for (int32_t c0 = a0; c0 < a1; c0 += kWave) {
            const int32_t e = c0 + lane;
            int32_t j = 0, len = 0;
            if (e < a1) {
                j = g.a_ci[e];
                len = g.b_ro[j + 1] - g.b_ro[j];
            }
            const int32_t incl = group_scan_incl<kWave>(len);
            const int32_t start = base + incl - len;
            if (len > 0) {
                const int32_t f0 = g.b_ro[j];
                const float a = COMPUTE ? g.a_val[e] : 0.f;
                for (int32_t t = 0; t < len; ++t) {
                    const int32_t q = start + t;
                    key[q] = (static_cast<uint64_t>(g.b_ci[f0 + t]) << 32) | static_cast<uint32_t>(q);
                    if constexpr (COMPUTE) val[q] = a * g.b_val[f0 + t];
                }
            }
            base += __shfl(incl, kWave - 1);
        }
        const int32_t np2 = next_pow2(p > 1 ? p : 1);
        for (int32_t q = p + lane; q < np2; q += kWave) key[q] = kPad;
        wave_sync();
        lds_bitonic<COMPUTE>(key, val, np2, lane, kWave, wave_sync);
        // runs of equal columns: count them, or sum each run and write it
        int32_t rank = 0;  // columns written so far
        float carry = 0.f; // open run's partial sum from earlier chunks
        const int32_t out0 = COMPUTE ? g.c_ro[i] : 0;
        for (int32_t c0 = 0; c0 < p; c0 += kWave) {
            const int32_t q = c0 + lane;
            const bool in = q < p;
            const uint32_t col = in ? static_cast<uint32_t>(key[q] >> 32) : 0xffffffffu;
            const uint32_t prev = q > 0 && in ? static_cast<uint32_t>(key[q - 1] >> 32) : 0xffffffffu;
            const bool head = in && (q == 0 || col != prev);
            const uint64_t hm = __ballot(head);
            if constexpr (COMPUTE) {
                const bool tail = in && (q == p - 1 || static_cast<uint32_t>(key[q + 1] >> 32) != col);
                seg_t sv = group_seg_scan_incl<kWave>(seg_t{in ? val[q] : 0.f, head});
                if (!sv.f) sv.v += carry;  // the run began in an earlier chunk
                const int32_t my_rank = rank + __popcll(hm & ((2ull << lane) - 1)) - 1;
                if (tail) {
                    g.c_ci[out0 + my_rank] = static_cast<int32_t>(col);
                    g.c_val[out0 + my_rank] = sv.v;
                }
                carry = __shfl(sv.v, kWave - 1);
            }
            rank += __popcll(hm);
        }
        if constexpr (!COMPUTE) {
            if (lane == 0) g.c_ro[i] = rank;
        }
        wave_sync();
    }
}

// Tier 2: a block per row.
template <bool COMPUTE>
__global__ __launch_bounds__(kBlock) void gemm_tier2(gemm_args g) {
    __shared__ uint64_t s_key[kTier2];
    __shared__ float s_val[COMPUTE ? kTier2 : 1];
    __shared__ int32_t s_wi[kBlock / kWave];
    __shared__ seg_t s_ws[kBlock / kWave];
    __shared__ int32_t s_int;
    __shared__ float s_float;
    const int tid = threadIdx.x;
    const int32_t rows = g.list_len[1];
    auto bsync = [] { __syncthreads(); };
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {  // uniform across the block
        const int32_t i = g.lists[static_cast<int64_t>(g.m) + r];
        const int32_t p = static_cast<int32_t>(g.prod[i]);
        const int32_t a0 = g.a_ro[i], a1 = g.a_ro[i + 1];
        int32_t base = 0;
        for (int32_t c0 = a0; c0 < a1; c0 += kBlock) {
            const int32_t e = c0 + tid;
            int32_t j = 0, len = 0;
            if (e < a1) {
                j = g.a_ci[e];
                len = g.b_ro[j + 1] - g.b_ro[j];
            }
            const int32_t incl = block_scan_incl<kBlock>(len, s_wi);
            const int32_t start = base + incl - len;
            if (len > 0) {
                const int32_t f0 = g.b_ro[j];
                const float a = COMPUTE ? g.a_val[e] : 0.f;
                for (int32_t t = 0; t < len; ++t) {
                    const int32_t q = start + t;
                    s_key[q] = (static_cast<uint64_t>(g.b_ci[f0 + t]) << 32) | static_cast<uint32_t>(q);
                    if constexpr (COMPUTE) s_val[q] = a * g.b_val[f0 + t];
                }
            }
            if (tid == kBlock - 1) s_int = incl;
            __syncthreads();
            base += s_int;
            __syncthreads();
        }
        const int32_t np2 = next_pow2(p > 1 ? p : 1);
        for (int32_t q = p + tid; q < np2; q += kBlock) s_key[q] = kPad;
        __syncthreads();
        lds_bitonic<COMPUTE>(s_key, s_val, np2, tid, kBlock, bsync);
        int32_t rank = 0;
        float carry = 0.f;
        const int32_t out0 = COMPUTE ? g.c_ro[i] : 0;
        for (int32_t c0 = 0; c0 < p; c0 += kBlock) {  // uniform across the block
            const int32_t q = c0 + tid;
            const bool in = q < p;
            const uint32_t col = in ? static_cast<uint32_t>(s_key[q] >> 32) : 0xffffffffu;
            const uint32_t prev = q > 0 && in ? static_cast<uint32_t>(s_key[q - 1] >> 32) : 0xffffffffu;
            const bool head = in && (q == 0 || col != prev);
            const int32_t hincl = block_scan_incl<kBlock>(head ? 1 : 0, s_wi);
            if constexpr (COMPUTE) {
                const bool tail = in && (q == p - 1 || static_cast<uint32_t>(s_key[q + 1] >> 32) != col);
                seg_t tot;
                seg_t sv = block_seg_scan_incl<kBlock>(seg_t{in ? s_val[q] : 0.f, head}, s_ws, tot);
                if (!sv.f) sv.v += carry;
                if (tail) {
                    g.c_ci[out0 + rank + hincl - 1] = static_cast<int32_t>(col);
                    g.c_val[out0 + rank + hincl - 1] = sv.v;
                }
                if (tid == kBlock - 1) s_float = sv.v;
            }
            if (tid == kBlock - 1) s_int = hincl;
            __syncthreads();
            rank += s_int;
            if constexpr (COMPUTE) carry = s_float;
            __syncthreads();
        }
        if constexpr (!COMPUTE) {
            if (tid == 0) g.c_ro[i] = rank;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- tier 3: dense slot per block

template <bool COMPUTE>
__global__ __launch_bounds__(kBlock) void gemm_tier3(gemm_args g) {
    using sched = group_mapped_scan<kBlock, indexed_tile_set>;
    __shared__ typename sched::storage s_st[1];
    __shared__ int32_t s_wi[kBlock / kWave];
    __shared__ int32_t s_slot;
    __shared__ int32_t s_int;
    const int tid = threadIdx.x;
    const int64_t nw0 = (static_cast<int64_t>(g.n) + 31) / 32;  // level-0 words: a bit per column
    float *acc = g.slot_acc + static_cast<int64_t>(blockIdx.x) * g.n;
    uint32_t *bits = g.slot_bits + static_cast<int64_t>(blockIdx.x) * g.slot_words;
    uint32_t *summary = bits + nw0;  // level 1: a bit per level-0 word
    const queue_rounds rows{g.list_len + 3, &s_slot, 1, g.list_len[2]};
    for (int64_t r : rows) {  // uniform across the block
        const int32_t i = g.lists[2 * static_cast<int64_t>(g.m) + r];
        const int32_t a0 = g.a_ro[i], a1 = g.a_ro[i + 1];
        // the row's A entries are the tiles; entry e selects B row a_ci[e]
        sched sch(indexed_tile_set{g.a_ci + a0, g.b_ro, a1 - a0}, s_st);
        int32_t mine = 0;  // columns this thread set first (count pass)
        const int64_t chunks = (static_cast<int64_t>(a1 - a0) + kBlock - 1) / kBlock;
        for (int64_t c = 0; c < chunks; ++c) {
            const int32_t total = sch.load(c);
            for (int64_t at : sch.atoms(total)) {
                const int32_t q = sch.get_tile(static_cast<int32_t>(at));
                const int32_t f = sch.atom(static_cast<int32_t>(at), q);
                const int32_t col = g.b_ci[f];
                const uint32_t bit = 1u << (col & 31);
                const uint32_t old = atomicOr(bits + (col >> 5), bit);
                if (old == 0) atomicOr(summary + (col >> 10), 1u << ((col >> 5) & 31));
                if constexpr (COMPUTE) {
                    const int32_t e = a0 + static_cast<int32_t>(c) * kBlock + q;
                    atomicAdd(acc + col, g.a_val[e] * g.b_val[f]);
                } else {
                    if (!(old & bit)) ++mine;
                }
            }
            sch.done();
        }
        __threadfence();
        __syncthreads();
        // walk the bitmap in column order: per summary word (32 level-0 words,
        // 1024 columns) a thread counts, the block scans, then it emits
        const int64_t nw1 = (nw0 + 31) / 32;
        int32_t written = 0;
        const int32_t out0 = COMPUTE ? g.c_ro[i] : 0;
        for (int64_t s0 = 0; s0 < nw1; s0 += kBlock) {  // uniform across the block
            const int64_t s = s0 + tid;
            const uint32_t sw = s < nw1 ? summary[s] : 0u;
            int32_t cnt = 0;
            if constexpr (COMPUTE) {
                for (uint32_t m = sw; m; m &= m - 1) cnt += __popc(bits[s * 32 + __ffs(m) - 1]);
            }
            const int32_t incl = block_scan_incl<kBlock>(cnt, s_wi);
            int32_t pos = written + incl - cnt;
            for (uint32_t m = sw; m; m &= m - 1) {
                const int64_t wi = s * 32 + __ffs(m) - 1;
                uint32_t word = bits[wi];
                if constexpr (COMPUTE) {
                    for (; word; word &= word - 1) {
                        const int32_t col = static_cast<int32_t>(wi * 32 + __ffs(word) - 1);
                        g.c_ci[out0 + pos] = col;
                        g.c_val[out0 + pos] = acc[col];
                        acc[col] = 0.f;
                        ++pos;
                    }
                }
                bits[wi] = 0u;
            }
            if (s < nw1) summary[s] = 0u;
            if (tid == kBlock - 1) s_int = incl;
            __syncthreads();
            written += s_int;
            __syncthreads();
        }
        if constexpr (!COMPUTE) {
            const int32_t incl = block_scan_incl<kBlock>(mine, s_wi);
            if (tid == kBlock - 1) g.c_ro[i] = incl;
        }
        __threadfence();
        __syncthreads();
    }
}

// ---------------------------------------------------------------- int64 scan of the row counts

constexpr int kScanTile = 2048;

// Per tile of 2048 counts (int32, in c_ro): in-tile exclusive prefix (int64) and the tile total.
__global__ __launch_bounds__(256) void gemm_scan_tiles(const int32_t *__restrict__ cnt, int64_t m,
                                                       int64_t *__restrict__ pre, int64_t *__restrict__ tile_sum) {
    __shared__ int64_t s_w[256 / kWave];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * 8;
    int64_t v[8];
    int64_t sum = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        v[u] = base + u < m ? cnt[base + u] : 0;
        sum += v[u];
    }
    int64_t incl = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int64_t o = __shfl_up(incl, off, kWave);
        if (lane_id() >= off) incl += o;
    }
    if (lane_id() == kWave - 1) s_w[wave_id()] = incl;
    __syncthreads();
    for (int k = 0; k < wave_id(); ++k) incl += s_w[k];
    int64_t run = incl - sum;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if (base + u < m) pre[base + u] = run;
        run += v[u];
    }
    if (threadIdx.x == 255) tile_sum[blockIdx.x] = incl;
}

// One thread: exclusive prefix of the tile totals (few: m / 2048) and the grand total.
__global__ void gemm_scan_totals(int64_t *__restrict__ tile_sum, int64_t nb, int64_t *__restrict__ total) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t run = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t t = tile_sum[b];
        tile_sum[b] = run;
        run += t;
    }
    *total = run;
}

// C's row offsets (int32) where the total fits; the host checks the total first.
__global__ __launch_bounds__(256) void gemm_scan_write(const int64_t *__restrict__ pre,
                                                       const int64_t *__restrict__ tile_pre,
                                                       const int64_t *__restrict__ total, int64_t m,
                                                       int32_t *__restrict__ c_ro) {
    for (int64_t i : grid_stride_range(0, m)) c_ro[i] = static_cast<int32_t>(pre[i] + tile_pre[i / kScanTile]);
    if (blockIdx.x == 0 && threadIdx.x == 0) c_ro[m] = static_cast<int32_t>(*total);
}

int64_t capped(int64_t work, int64_t per) {
    const int64_t b = (work + per - 1) / per;
    return b < 1 ? 1 : (b > 4096 ? 4096 : b);
}

}  // namespace

// ---------------------------------------------------------------- workspace

struct gemm_ws {
    int64_t *prod, *pre, *tile_sum, *total;
    int32_t *lists, *list_len;
    float *slot_acc;
    uint32_t *slot_bits;
    int64_t slot_words;
};

static gemm_ws gemm_carve(void *base, int64_t m, int64_t n) {
    char *p = static_cast<char *>(base);
    gemm_ws w;
    w.prod = reinterpret_cast<int64_t *>(p);
    p += align256(static_cast<size_t>(m) * 8);
    w.pre = reinterpret_cast<int64_t *>(p);
    p += align256(static_cast<size_t>(m) * 8);
    w.tile_sum = reinterpret_cast<int64_t *>(p);
    p += align256(static_cast<size_t>(m / kScanTile + 2) * 8);
    w.total = reinterpret_cast<int64_t *>(p);
    p += 256;
    w.lists = reinterpret_cast<int32_t *>(p);
    p += align256(static_cast<size_t>(4 * m) * 4);
    w.list_len = reinterpret_cast<int32_t *>(p);
    p += 256;
    w.slot_words = (n + 31) / 32 + ((n + 31) / 32 + 31) / 32;
    w.slot_acc = reinterpret_cast<float *>(p);
    p += align256(static_cast<size_t>(spgemm_slots(n)) * n * 4);
    w.slot_bits = reinterpret_cast<uint32_t *>(p);
    return w;
}

size_t spgemm_ws_bytes(int64_t m, int64_t n) {
    const int64_t words = (n + 31) / 32 + ((n + 31) / 32 + 31) / 32;
    return 2 * align256(static_cast<size_t>(m) * 8) + align256(static_cast<size_t>(m / kScanTile + 2) * 8) + 256 +
           align256(static_cast<size_t>(4 * m) * 4) + 256 + align256(static_cast<size_t>(spgemm_slots(n)) * n * 4) +
           align256(static_cast<size_t>(spgemm_slots(n)) * words * 4);
}

static hipError_t gemm_pass(const spgemm_dev &P, int32_t *c_ro, int32_t *c_ci, float *c_val, void *ws, bool compute,
                            hipStream_t s) {
    const gemm_ws w = gemm_carve(ws, P.m, P.n);
    gemm_args g{P.m, P.n, P.a_ro, P.a_ci, P.a_val, P.b_ro, P.b_ci, P.b_val, w.prod, w.lists, w.list_len,
                c_ro, c_ci, c_val, w.slot_acc, w.slot_bits, w.slot_words};
    hipError_t e = fill_f32(reinterpret_cast<float *>(w.list_len), 5, 0.f, s);  // +0.0f is all zero bits
    if (e != hipSuccess) return e;
    {
        prof_scope p(s, "spgemm_products");
        // short rows (fewer than 8 entries on average) share wavefronts; longer ones get one each
        if (P.m > 0 && static_cast<int64_t>(P.a_nnz) < 8 * static_cast<int64_t>(P.m)) {
            constexpr int RPB = group_block<kWave>::BLOCK;  // rows per block round: 4 groups of 64
            hipLaunchKernelGGL(gemm_products, dim3(static_cast<uint32_t>(capped(P.m, RPB))), dim3(256), 0, s, g,
                               w.prod);
        } else {
            constexpr int GPB = group_block<kWave>::GPB;  // grid-stride: at most 2^16 blocks
            const int64_t want = (static_cast<int64_t>(P.m) + GPB - 1) / GPB;
            hipLaunchKernelGGL(gemm_products_rows, dim3(static_cast<uint32_t>(want < 65536 ? want : 65536)), dim3(256),
                               0, s, g, w.prod);
        }
        const int64_t cb = (static_cast<int64_t>(P.m) + kClassRows - 1) / kClassRows;
        hipLaunchKernelGGL(gemm_classify, dim3(static_cast<uint32_t>(cb < 1 ? 1 : cb)), dim3(256), 0, s, g);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // tier-3 slots start clear (the kernel clears what it used)
    const int64_t slots = spgemm_slots(P.n);
    e = fill_f32(reinterpret_cast<float *>(w.slot_bits), slots * w.slot_words, 0.f, s);
    if (e == hipSuccess && compute) e = fill_f32(w.slot_acc, slots * P.n, 0.f, s);
    if (e != hipSuccess) return e;
    // one launch per tier (each reads its list's length on the device)
    const uint32_t grid12 = static_cast<uint32_t>(capped(P.m, 1) < 2048 ? capped(P.m, 1) : 2048);
    const char *names[2][4] = {{"spgemm_count_t0", "spgemm_count_t1", "spgemm_count_t2", "spgemm_count_t3"},
                               {"spgemm_compute_t0", "spgemm_compute_t1", "spgemm_compute_t2", "spgemm_compute_t3"}};
    const int c = compute ? 1 : 0;
    {
        prof_scope p(s, names[c][0]);
        if (compute)
            hipLaunchKernelGGL(gemm_tier0<true>, dim3(grid12), dim3(kBlock), 0, s, g);
        else
            hipLaunchKernelGGL(gemm_tier0<false>, dim3(grid12), dim3(kBlock), 0, s, g);
    }
    {
        prof_scope p(s, names[c][1]);
        if (compute)
            hipLaunchKernelGGL(gemm_tier1<true>, dim3(grid12), dim3(kBlock), 0, s, g);
        else
            hipLaunchKernelGGL(gemm_tier1<false>, dim3(grid12), dim3(kBlock), 0, s, g);
    }
    {
        prof_scope p(s, names[c][2]);
        if (compute)
            hipLaunchKernelGGL(gemm_tier2<true>, dim3(grid12), dim3(kBlock), 0, s, g);
        else
            hipLaunchKernelGGL(gemm_tier2<false>, dim3(grid12), dim3(kBlock), 0, s, g);
    }
    {
        prof_scope p(s, names[c][3]);
        if (compute)
            hipLaunchKernelGGL(gemm_tier3<true>, dim3(static_cast<uint32_t>(slots)), dim3(kBlock), 0, s, g);
        else
            hipLaunchKernelGGL(gemm_tier3<false>, dim3(static_cast<uint32_t>(slots)), dim3(kBlock), 0, s, g);
    }
    e = hipGetLastError();
    return e;
}

hipError_t spgemm_count(const spgemm_dev &P, int32_t *c_ro, int64_t *total_host, void *ws, hipStream_t s) {
    hipError_t e = gemm_pass(P, c_ro, nullptr, nullptr, ws, false, s);
    if (e != hipSuccess) return e;
    const gemm_ws w = gemm_carve(ws, P.m, P.n);
    const int64_t nb = (static_cast<int64_t>(P.m) + kScanTile - 1) / kScanTile;
    if (nb > 0)
        hipLaunchKernelGGL(gemm_scan_tiles, dim3(static_cast<uint32_t>(nb)), dim3(256), 0, s, c_ro,
                           static_cast<int64_t>(P.m), w.pre, w.tile_sum);
    hipLaunchKernelGGL(gemm_scan_totals, dim3(1), dim3(64), 0, s, w.tile_sum, nb, w.total);
    hipLaunchKernelGGL(gemm_scan_write, dim3(static_cast<uint32_t>(capped(P.m, 256))), dim3(256), 0, s, w.pre,
                       w.tile_sum, w.total, static_cast<int64_t>(P.m), c_ro);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(total_host, w.total, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

hipError_t spgemm_compute(const spgemm_dev &P, const int32_t *c_ro, int32_t *c_ci, float *c_val, void *ws,
                          hipStream_t s) {
    return gemm_pass(P, const_cast<int32_t *>(c_ro), c_ci, c_val, ws, true, s);
}

}  // namespace lbk
