// Backward of y = A x without atomics: dx = A^T dy as a merge-path SpMV over
// the transposed pattern.  A training loop keeps one sparsity pattern across
// steps, so the transpose is built once (transpose_pattern) and each
// backward runs the forward's merge-path kernels on A^T, reading the current
// values of A through the pattern's permutation (val[perm[p]], gathered in
// the consume kernel's setup); dvalues comes from the backward kernel's
// dvalues-only pass.
//
// Transpose of a CSR pattern A (rows x cols) without global atomics: a
// stable least-significant-digit radix sort of the nonzeros by column.
// Entry e of row r carries (key = col[e], e, r); every pass sorts by the
// next digit of the key and keeps the order of equal digits, so after the
// last pass the entries are ordered by (column, position in A) = (column,
// row): the canonical CSC, the same for every build.  Each pass:
//   1. count:   each block counts the digits of its tile of kRadixTile
//               entries in LDS (one histogram row per wavefront) and stores
//               the tile's histogram digit-major, hist[d * blocks + b];
//   2. scan:    exclusive prefix of hist: the first output position of
//               (digit d, block b);
//   3. scatter: each wavefront holds a contiguous eighth of the tile in
//               registers and ranks its entries among equal digits in order
//               (lanes holding the same digit find each other with one
//               ballot per digit bit); the block then places the tile in LDS
//               sorted by digit and writes each digit's run to consecutive
//               output positions, so the stores are coalesced runs instead of
//               scattered words.
// The first pass reads col_idx directly and finds each entry's row among
// row ends staged in LDS.  Digits have at most kRadixMaxBits bits (three passes for up to
// 2^21 columns).  at_row_offsets[c] = the first sorted position with key >=
// c, counted per block of columns.  Every count is an LDS add within one block;
// every position is computed, not claimed.
#include <limits.h>

#include "lb_device.h"
#include "lb_internal.h"
#include "lb_schedule.hpp"

namespace lbk {
using namespace lb;

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kRadixThreads = 512;
constexpr int kRadixWaves = kRadixThreads / kWave;
constexpr int kRadixPerLane = 8;
constexpr int kRadixPerWave = kRadixPerLane * kWave;     // entries per wavefront per tile
constexpr int kRadixTile = kRadixWaves * kRadixPerWave;  // entries per block
constexpr int kRadixMaxBits = 7;
constexpr int kRadixBins = 1 << kRadixMaxBits;

struct radix_src {
    const int32_t *key, *e, *r;  // first pass: key = col_idx, e and r null
};
struct radix_dst {
    int32_t *key, *e, *r;
};

__global__ __launch_bounds__(kRadixThreads) void radix_count(int64_t nnz, const int32_t *__restrict__ key,
                                                             int shift, int bits, int32_t nblk,
                                                             int32_t *__restrict__ hist) {
    __shared__ int32_t h[kRadixWaves][kRadixBins];
    const int nb = 1 << bits;
    const int w = wave_id(), lane = lane_id();
    for (int d = lane; d < nb; d += kWave) h[w][d] = 0;
    const int64_t s0 = static_cast<int64_t>(blockIdx.x) * kRadixTile + static_cast<int64_t>(w) * kRadixPerWave;
    const int64_t s1 = s0 + kRadixPerWave < nnz ? s0 + kRadixPerWave : nnz;
    int32_t k[kRadixPerLane];
#pragma unroll
    for (int s = 0; s < kRadixPerLane; ++s) {  // every load in flight before the first add
        const int64_t i = s0 + s * kWave + lane;
        k[s] = i < s1 ? key[i] : -1;
    }
#pragma unroll
    for (int s = 0; s < kRadixPerLane; ++s)
        if (k[s] >= 0) atomicAdd(&h[w][(k[s] >> shift) & (nb - 1)], 1);
    __syncthreads();
    for (int d = threadIdx.x; d < nb; d += kRadixThreads) {
        int32_t c = 0;
#pragma unroll
        for (int k = 0; k < kRadixWaves; ++k) c += h[k][d];
        hist[static_cast<int64_t>(d) * nblk + blockIdx.x] = c;
    }
}

template <bool FIRST, bool LAST>
__global__ __launch_bounds__(kRadixThreads) void radix_scatter(int64_t nnz, int32_t rows,
                                                               const int32_t *__restrict__ ro, radix_src src,
                                                               radix_dst dst, int shift, int bits, int32_t nblk,
                                                               const int32_t *__restrict__ hist,
                                                               int32_t *__restrict__ at_ro) {
    __shared__ int32_t s_key[kRadixTile], s_e[kRadixTile], s_r[kRadixTile];
    __shared__ int32_t wh[kRadixWaves][kRadixBins];  // per wavefront: running count, then its first local slot
    __shared__ int32_t s_start[kRadixBins], s_gbase[kRadixBins], s_wave[kRadixWaves];
    const int nb = 1 << bits;
    const int w = wave_id(), lane = lane_id();
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kRadixTile;
    const int32_t tlen = static_cast<int32_t>(t0 + kRadixTile < nnz ? kRadixTile : nnz - t0);
    const int64_t s0 = t0 + static_cast<int64_t>(w) * kRadixPerWave;
    const int64_t s1 = s0 + kRadixPerWave < nnz ? s0 + kRadixPerWave : nnz;
    for (int d = lane; d < nb; d += kWave) wh[w][d] = 0;

    int32_t key[kRadixPerLane], ev[kRadixPerLane], rv[kRadixPerLane];
#pragma unroll
    for (int s = 0; s < kRadixPerLane; ++s) {
        const int64_t i = s0 + s * kWave + lane;
        const bool valid = i < s1;
        key[s] = valid ? src.key[i] : 0;
        ev[s] = FIRST ? static_cast<int32_t>(i) : (valid ? src.e[i] : 0);
        rv[s] = FIRST ? 0 : (valid ? src.r[i] : 0);
    }
    if constexpr (FIRST) {
        // rows of the entries [s0, s1): row(i) = the last r with ro[r] <= i.
        // rc = row(s0) comes from a wavefront search; every later row that
        // starts inside (s0, s1) marks its start in LDS (the largest such row
        // wins where empty rows share a start), and a running maximum over
        // the marks, from rc, gives each entry its row.
        if (s0 < s1) {  // uniform across the wavefront
            const int32_t rc = group_count_below<kWave>(0, rows, static_cast<int32_t>(s0) + 1,
                                                        [ro](int32_t r) { return ro[r + 1]; });
            int32_t *mark = s_key + w * kRadixPerWave;  // free until the tile is placed
#pragma unroll
            for (int k = 0; k < kRadixPerLane; ++k) mark[k * kWave + lane] = -1;
            for (int32_t r0 = rc + 1;; r0 += kRadixPerWave) {  // r0 uniform
                int32_t st[kRadixPerLane];
#pragma unroll
                for (int k = 0; k < kRadixPerLane; ++k) {
                    const int32_t r = r0 + k * kWave + lane;
                    st[k] = r < rows ? ro[r] : INT_MAX;
                }
#pragma unroll
                for (int k = 0; k < kRadixPerLane; ++k)
                    if (st[k] > s0 && st[k] < s1) atomicMax(&mark[st[k] - s0], r0 + k * kWave + lane);
                // rows go on past this window when its last row still starts inside
                if (__ballot(lane == kWave - 1 && st[kRadixPerLane - 1] < s1) == 0) break;
            }
            int32_t carry = rc;
#pragma unroll
            for (int s = 0; s < kRadixPerLane; ++s) {
                int32_t v = mark[s * kWave + lane];
                v = v > carry ? v : carry;
#pragma unroll
                for (int off = 1; off < kWave; off <<= 1) {
                    const int32_t u = __shfl_up(v, off);
                    if (lane >= off) v = u > v ? u : v;
                }
                rv[s] = v;
                carry = __shfl(v, kWave - 1);
            }
        }
    }
    // ranks among equal digits within this wavefront's entries, in order
    const uint64_t below = (1ull << lane) - 1;
    int32_t lrank[kRadixPerLane];
#pragma unroll
    for (int s = 0; s < kRadixPerLane; ++s) {
        const bool valid = s0 + s * kWave + lane < s1;
        const int d = (key[s] >> shift) & (nb - 1);
        uint64_t same = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool set = (d >> b) & 1;
            const uint64_t m = __ballot(set);
            same &= set ? m : ~m;
        }
        const int rank = __popcll(same & below);
        const int32_t pre = wh[w][d];
        lrank[s] = pre + rank;
        if (valid && rank == 0) wh[w][d] = pre + __popcll(same);
    }
    __syncthreads();
    // per digit: the wavefronts' first local slots and the tile's count
    static_assert(kRadixBins <= kRadixThreads, "one digit per thread");
    int32_t mine = 0;  // thread d: digit d's count in the tile
    if (static_cast<int>(threadIdx.x) < nb) {
        const int d = threadIdx.x;
#pragma unroll
        for (int v = 0; v < kRadixWaves; ++v) {
            const int32_t c = wh[v][d];
            wh[v][d] = mine;
            mine += c;
        }
        s_gbase[d] = hist[static_cast<int64_t>(d) * nblk + blockIdx.x];
    }
    // exclusive prefix of the tile's digit counts: each digit's first local slot
    const int32_t incl = block_scan_incl<kRadixThreads>(mine, s_wave);
    if (threadIdx.x < kRadixBins) s_start[threadIdx.x] = incl - mine;
    __syncthreads();
    // the tile in LDS, sorted by digit (stable)
#pragma unroll
    for (int s = 0; s < kRadixPerLane; ++s) {
        if (s0 + s * kWave + lane < s1) {
            const int d = (key[s] >> shift) & (nb - 1);
            const int32_t lp = s_start[d] + wh[w][d] + lrank[s];
            s_key[lp] = key[s];
            s_e[lp] = ev[s];
            s_r[lp] = rv[s];
        }
    }
    __syncthreads();
    // each digit's run to its consecutive output positions; the last pass
    // writes no keys but the first position of every column whose first
    // entry is not the first of its run (the run starts: transpose_run_starts)
    for (int32_t j = threadIdx.x; j < tlen; j += kRadixThreads) {
        const int32_t k = s_key[j];
        const int d = (k >> shift) & (nb - 1);
        const int32_t g = s_gbase[d] + (j - s_start[d]);
        if constexpr (LAST) {
            if (j > s_start[d] && s_key[j - 1] != k) at_ro[k] = g;
        } else {
            dst.key[g] = k;
        }
        dst.e[g] = s_e[j];
        dst.r[g] = s_r[j];
    }
}

// The first entry of each (digit, block) run of the last pass: if its column
// differs from the entry before it, it is that column's first position.
// Columns are read through perm (the last pass writes no keys).
__global__ __launch_bounds__(256) void transpose_run_starts(int64_t runs, int64_t nnz,
                                                            const int32_t *__restrict__ start,
                                                            const int32_t *__restrict__ ci,
                                                            const int32_t *__restrict__ perm,
                                                            int32_t *__restrict__ at_ro) {
    for (int64_t q : grid_stride_range(0, runs)) {
        const int64_t g = start[q];
        const int64_t g1 = q + 1 < runs ? start[q + 1] : nnz;
        if (g >= g1) continue;  // an empty run
        const int32_t k = ci[perm[g]];
        if (g == 0 || ci[perm[g - 1]] != k) at_ro[k] = static_cast<int32_t>(g);
    }
}

__global__ __launch_bounds__(256) void fill_i32(int32_t *__restrict__ a, int64_t n, int32_t v) {
    for (int64_t p : grid_stride_range(0, n)) a[p] = v;
}

// Suffix minimum of a[0, n) in place, in tiles of kScanTile: a[p] = min
// over a[p..].  Empty columns (still INT_MAX) get the next column's start.
__global__ __launch_bounds__(kScanThreads) void suffix_min_tiles(int32_t *__restrict__ a, int64_t n,
                                                                 int32_t *__restrict__ tile_min) {
    __shared__ int32_t s[kScanThreads];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t m = INT_MAX;
#pragma unroll
    for (int u = kScanItems - 1; u >= 0; --u) {
        v[u] = base + u < n ? a[base + u] : INT_MAX;
        m = v[u] < m ? v[u] : m;
        v[u] = m;
    }
    s[threadIdx.x] = m;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {  // inclusive suffix min over the threads
        const int32_t o = threadIdx.x + off < kScanThreads ? s[threadIdx.x + off] : INT_MAX;
        __syncthreads();
        if (o < s[threadIdx.x]) s[threadIdx.x] = o;
        __syncthreads();
    }
    const int32_t after = threadIdx.x + 1 < kScanThreads ? s[threadIdx.x + 1] : INT_MAX;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u)
        if (base + u < n) a[base + u] = v[u] < after ? v[u] : after;
    if (threadIdx.x == 0) tile_min[blockIdx.x] = s[0];
}

// One block: tile_min[t] = min over the tiles after t (exclusive suffix).
__global__ __launch_bounds__(1024) void suffix_min_totals(int32_t *__restrict__ tile_min, int32_t nb) {
    __shared__ int32_t s[1024];
    int32_t later = INT_MAX;  // min of the tiles after this chunk
    for (int32_t c0 = ((nb - 1) / 1024) * 1024; c0 >= 0; c0 -= 1024) {  // uniform, last chunk first
        const int32_t idx = c0 + static_cast<int32_t>(threadIdx.x);
        const int32_t v = idx < nb ? tile_min[idx] : INT_MAX;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t o = threadIdx.x + off < 1024 ? s[threadIdx.x + off] : INT_MAX;
            __syncthreads();
            if (o < s[threadIdx.x]) s[threadIdx.x] = o;
            __syncthreads();
        }
        const int32_t after = threadIdx.x + 1 < 1024 ? s[threadIdx.x + 1] : INT_MAX;
        if (idx < nb) tile_min[idx] = after < later ? after : later;
        const int32_t chunk = s[0];
        __syncthreads();
        later = chunk < later ? chunk : later;
    }
}

__global__ __launch_bounds__(256) void suffix_min_apply(int32_t *__restrict__ a, int64_t n,
                                                        const int32_t *__restrict__ tile_after) {
    for (int64_t p : grid_stride_range(0, n)) {
        const int32_t t = tile_after[p / kScanTile];
        if (t < a[p]) a[p] = t;
    }
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

// One block: exclusive prefix of the nb tile totals in place.
__global__ __launch_bounds__(1024) void scan_totals(int32_t *__restrict__ tile_sum, int32_t nb) {
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
}

__global__ __launch_bounds__(256) void scan_add(int32_t *__restrict__ a, int64_t n,
                                                const int32_t *__restrict__ tile_pre) {
    for (int64_t p : grid_stride_range(0, n)) a[p] += tile_pre[p / kScanTile];
}

int64_t capped_blocks(int64_t work, int64_t per_block) {
    const int64_t g = (work + per_block - 1) / per_block;
    return g < 1 ? 1 : (g > 8192 ? 8192 : g);
}

// Exclusive prefix of a[0, n) in place (tile_sum: n / kScanTile + 1 ints).
hipError_t scan_exclusive(int32_t *a, int64_t n, int32_t *tile_sum, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_tiles, dim3(static_cast<uint32_t>(nb)), dim3(kScanThreads), 0, s, a, n, tile_sum);
    hipLaunchKernelGGL(scan_totals, dim3(1), dim3(1024), 0, s, tile_sum, static_cast<int32_t>(nb));
    hipLaunchKernelGGL(scan_add, dim3(static_cast<uint32_t>(capped_blocks(n, 256))), dim3(256), 0, s, a, n, tile_sum);
    return hipGetLastError();
}

// Digit bits per pass and passes for keys in [0, cols).
struct radix_plan {
    int bits, passes, digit;
};
radix_plan radix_plan_of(int64_t cols) {
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < cols) ++bits;
    const int passes = (bits + kRadixMaxBits - 1) / kRadixMaxBits;
    return {bits, passes, (bits + passes - 1) / passes};
}

struct transpose_ws {
    int32_t *xk, *xe, *xr, *yk, *ye, *yr, *hist, *tile_sum;
    int64_t nblk;
};
// Entries and ints of each workspace part: three ping-pong pairs of nnz
// (key, e, r), the digit histograms, the scan tiles (of the histograms or of
// at_row_offsets, whichever is longer).
struct transpose_sizes {
    int64_t nblk, hist_n, tiles;
};
transpose_sizes transpose_sizes_of(int64_t cols, int64_t nnz) {
    const radix_plan rp = radix_plan_of(cols);
    transpose_sizes z;
    z.nblk = (nnz + kRadixTile - 1) / kRadixTile;
    z.hist_n = (int64_t(1) << rp.digit) * z.nblk;
    const int64_t m = z.hist_n > cols + 1 ? z.hist_n : cols + 1;
    z.tiles = m / kScanTile + 2;
    return z;
}
transpose_ws transpose_layout(void *ws, int64_t cols, int64_t nnz) {
    const transpose_sizes z = transpose_sizes_of(cols, nnz);
    transpose_ws L{};
    L.nblk = z.nblk;
    char *w = static_cast<char *>(ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        int32_t *p = reinterpret_cast<int32_t *>(w + off);
        off += align256(bytes);
        return p;
    };
    const size_t a = static_cast<size_t>(nnz) * 4;
    L.xk = take(a), L.xe = take(a), L.xr = take(a);
    L.yk = take(a), L.ye = take(a), L.yr = take(a);
    L.hist = take(static_cast<size_t>(z.hist_n) * 4);
    L.tile_sum = take(static_cast<size_t>(z.tiles) * 4);
    return L;
}

template <bool FIRST, bool LAST>
void launch_scatter(int32_t nblk, const csr_dev &A, const radix_src &src, const radix_dst &dst, int shift, int bits,
                    const int32_t *hist, int32_t *at_ro, hipStream_t s) {
    hipLaunchKernelGGL((radix_scatter<FIRST, LAST>), dim3(static_cast<uint32_t>(nblk)), dim3(kRadixThreads), 0, s,
                       static_cast<int64_t>(A.nnz), A.rows, A.ro, src, dst, shift, bits, nblk, hist, at_ro);
}

}  // namespace

size_t transpose_ws_bytes(int64_t cols, int64_t nnz) {
    const transpose_sizes z = transpose_sizes_of(cols, nnz);
    return 6 * align256(static_cast<size_t>(nnz) * 4) + align256(static_cast<size_t>(z.hist_n) * 4) +
           align256(static_cast<size_t>(z.tiles) * 4);
}

hipError_t transpose_pattern(const csr_dev &A, int32_t *at_ro, int32_t *at_ci, int32_t *perm, void *ws,
                             hipStream_t s) {
    prof_scope p(s, "transpose");
    const int64_t n = A.cols, nnz = A.nnz;
    const transpose_ws L = transpose_layout(ws, n, nnz);
    const radix_plan rp = radix_plan_of(n);
    // at_ro: INT_MAX for the columns, nnz at the end; the last pass and the
    // run starts write every column's first position, the suffix minimum
    // gives the empty columns theirs
    hipLaunchKernelGGL(fill_i32, dim3(static_cast<uint32_t>(capped_blocks(n, 256))), dim3(256), 0, s, at_ro, n,
                       static_cast<int32_t>(INT_MAX));
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(256), 0, s, at_ro + n, int64_t(1), static_cast<int32_t>(nnz));
    hipError_t e = hipSuccess;
    if (nnz > 0) {
        radix_src src{A.ci, nullptr, nullptr};
        const int32_t nblk = static_cast<int32_t>(L.nblk);
        int64_t runs = 0;
        for (int pass = 0; pass < rp.passes; ++pass) {
            const int shift = pass * rp.digit;
            const int bits = rp.bits - shift < rp.digit ? rp.bits - shift : rp.digit;
            const bool first = pass == 0, last = pass + 1 == rp.passes;
            radix_dst dst = pass % 2 == 0 ? radix_dst{L.xk, L.xe, L.xr} : radix_dst{L.yk, L.ye, L.yr};
            if (last) dst = radix_dst{nullptr, perm, at_ci};
            runs = (int64_t(1) << bits) * L.nblk;
            hipLaunchKernelGGL(radix_count, dim3(static_cast<uint32_t>(nblk)), dim3(kRadixThreads), 0, s, nnz, src.key,
                               shift, bits, nblk, L.hist);
            e = scan_exclusive(L.hist, runs, L.tile_sum, s);
            if (e != hipSuccess) return e;
            if (first && last)
                launch_scatter<true, true>(nblk, A, src, dst, shift, bits, L.hist, at_ro, s);
            else if (first)
                launch_scatter<true, false>(nblk, A, src, dst, shift, bits, L.hist, at_ro, s);
            else if (last)
                launch_scatter<false, true>(nblk, A, src, dst, shift, bits, L.hist, at_ro, s);
            else
                launch_scatter<false, false>(nblk, A, src, dst, shift, bits, L.hist, at_ro, s);
            src = radix_src{dst.key, dst.e, dst.r};
        }
        hipLaunchKernelGGL(transpose_run_starts, dim3(static_cast<uint32_t>(capped_blocks(runs, 256))), dim3(256), 0,
                           s, runs, nnz, L.hist, A.ci, perm, at_ro);
    }
    const int64_t m = n + 1;
    const int64_t nt = (m + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(suffix_min_tiles, dim3(static_cast<uint32_t>(nt)), dim3(kScanThreads), 0, s, at_ro, m,
                       L.tile_sum);
    hipLaunchKernelGGL(suffix_min_totals, dim3(1), dim3(1024), 0, s, L.tile_sum, static_cast<int32_t>(nt));
    hipLaunchKernelGGL(suffix_min_apply, dim3(static_cast<uint32_t>(capped_blocks(m, 256))), dim3(256), 0, s, at_ro, m,
                       L.tile_sum);
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
