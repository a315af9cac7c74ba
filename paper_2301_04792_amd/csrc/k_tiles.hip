// Tile-per-thread and tile-per-group schedules for gfx950.
//
// thread-mapped (Sec. 4.2 listing, Sec. 4.3 SpMV listing): tile r goes to
//   global thread r, threads stride by the grid, a thread walks its tile's
//   atoms in order.  A wavefront waits for its longest row (Sec. 1).
// group-mapped (Sec. 5.2.2, Sec. 5.2.3): a group of G lanes (G a power of
//   two; G <= 64 packs 64/G groups into a wavefront, G = 64 is one
//   wavefront, G > 64 is a whole block) owns tiles.
//   * tiles_per_group = 1: the group takes one tile at a time and its lanes
//     stride the tile's atoms by G; the lane partials are summed across the
//     group (wave64 butterfly; LDS across waves for G > 64).
//   * tiles_per_group = G: the group takes G consecutive tiles, writes their
//     atom counts to LDS and prefix-sums them; the lanes then walk the
//     group's flattened atoms G at a time and each finds its atom's tile by
//     binary search in the prefix sums (get_tile).  Per-tile sums come from
//     a segmented scan over each step's G lanes keyed by tile; the last lane
//     of each tile's run adds the run total to the tile's LDS accumulator.
//   Imbalance across groups is left to the hardware dispatcher: one group
//   per tile chunk, no grid stride unless grid_size caps the launch.
#include "lb_device.h"
#include "lb_internal.h"

namespace lbk {
using namespace lb;

// ------------------------------------------------------------------ thread-mapped

template <typename VT, typename XT>
__global__ __launch_bounds__(1024) void thread_mapped_spmv_kernel(csr_tile_set ts, const int32_t *__restrict__ ci,
                                                                  const VT *__restrict__ val,
                                                                  const XT *__restrict__ x,
                                                                  float *__restrict__ y) {
    const thread_mapped_schedule sched{ts};
    for (int64_t row : sched.tiles()) {
        // four independent partial sums keep four gathers in flight
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        const step_range atoms = sched.atoms(row);
        int64_t j = atoms.b;
        for (; j + 3 < atoms.e; j += 4) {
            a0 += to_f32(ld_stream(val + j)) * to_f32(x[ld_stream(ci + j)]);
            a1 += to_f32(ld_stream(val + j + 1)) * to_f32(x[ld_stream(ci + j + 1)]);
            a2 += to_f32(ld_stream(val + j + 2)) * to_f32(x[ld_stream(ci + j + 2)]);
            a3 += to_f32(ld_stream(val + j + 3)) * to_f32(x[ld_stream(ci + j + 3)]);
        }
        for (; j < atoms.e; ++j) a0 += to_f32(ld_stream(val + j)) * to_f32(x[ld_stream(ci + j)]);
        y[row] = (a0 + a1) + (a2 + a3);
    }
}

// Blocks for `work` items at `per_block` per block, capped by a caller grid
// and at kMaxBlocks: the kernels loop with a grid stride, and a launch must
// keep blocks x threads below 2^32 (a group per row with 1024 lanes reaches
// that at 4M rows).
constexpr int64_t kMaxBlocks = int64_t(1) << 20;
static int64_t blocks_for(int64_t work, int64_t per_block, int grid) {
    int64_t g = (work + per_block - 1) / per_block;
    if (grid > 0 && g > grid) g = grid;
    if (g > kMaxBlocks) g = kMaxBlocks;
    return g < 1 ? 1 : g;
}

hipError_t thread_mapped_spmv(const csr_dev &A, const void *x, float *y, int block, int grid,
                              hipStream_t s) {
    prof_scope p(s, "thread_mapped");
    const csr_tile_set ts{A.ro, A.rows, A.nnz};
    const dim3 g(static_cast<uint32_t>(blocks_for(A.rows, block, grid)));
    if (A.dt == LB_BF16)
        hipLaunchKernelGGL((thread_mapped_spmv_kernel<bf16_bits, bf16_bits>), g, dim3(block), 0, s, ts, A.ci,
                           static_cast<const bf16_bits *>(A.val), static_cast<const bf16_bits *>(x), y);
    else
        hipLaunchKernelGGL((thread_mapped_spmv_kernel<float, float>), g, dim3(block), 0, s, ts, A.ci,
                           static_cast<const float *>(A.val), static_cast<const float *>(x), y);
    return hipGetLastError();
}

// Thread-mapped SpMM: a thread owns one (row, column) pair of Y.
template <typename VT, typename XT>
__global__ __launch_bounds__(1024) void thread_mapped_spmm_kernel(csr_tile_set ts, const int32_t *__restrict__ ci,
                                                                  const VT *__restrict__ val,
                                                                  const XT *__restrict__ X, int32_t k,
                                                                  int64_t ldx, float *__restrict__ Y,
                                                                  int64_t ldy) {
    for (int64_t q : grid_stride_range(0, ts.num_tiles * k)) {
        const int64_t row = q / k;
        const int32_t col = static_cast<int32_t>(q - row * k);
        float a0 = 0.f, a1 = 0.f;
        int64_t j = ts.atoms_begin(row);
        const int64_t e = ts.atoms_end(row);
        for (; j + 1 < e; j += 2) {
            a0 += to_f32(val[j]) * to_f32(X[static_cast<int64_t>(ci[j]) * ldx + col]);
            a1 += to_f32(val[j + 1]) * to_f32(X[static_cast<int64_t>(ci[j + 1]) * ldx + col]);
        }
        if (j < e) a0 += to_f32(val[j]) * to_f32(X[static_cast<int64_t>(ci[j]) * ldx + col]);
        Y[row * ldy + col] = a0 + a1;
    }
}

hipError_t thread_mapped_spmm(const csr_dev &A, const void *X, int32_t k, int64_t ldx, float *Y,
                              int64_t ldy, int block, int grid, hipStream_t s) {
    prof_scope p(s, "thread_mapped");
    const csr_tile_set ts{A.ro, A.rows, A.nnz};
    const dim3 g(static_cast<uint32_t>(blocks_for(static_cast<int64_t>(A.rows) * k, block, grid)));
    if (A.dt == LB_BF16)
        hipLaunchKernelGGL((thread_mapped_spmm_kernel<bf16_bits, bf16_bits>), g, dim3(block), 0, s, ts, A.ci,
                           static_cast<const bf16_bits *>(A.val), static_cast<const bf16_bits *>(X), k, ldx, Y,
                           ldy);
    else
        hipLaunchKernelGGL((thread_mapped_spmm_kernel<float, float>), g, dim3(block), 0, s, ts, A.ci,
                           static_cast<const float *>(A.val), static_cast<const float *>(X), k, ldx, Y, ldy);
    return hipGetLastError();
}

// ------------------------------------------------------------------ group-mapped, one tile per group

// Group shape (lb_schedule.hpp): groups of up to one wavefront are packed
// 256 lanes to a block; a larger group is exactly one block.

template <int G, typename VT, typename XT>
__global__ __launch_bounds__(group_block<G>::BLOCK) void group_mapped_tile_kernel(
    csr_tile_set ts, const int32_t *__restrict__ ci, const VT *__restrict__ val, const XT *__restrict__ x,
    float *__restrict__ y) {
    constexpr int BLOCK = group_block<G>::BLOCK;
    constexpr int GPB = group_block<G>::GPB;
    const int gl = threadIdx.x & (G - 1);
    if constexpr (G <= kWave) {
        const int64_t g0 = static_cast<int64_t>(blockIdx.x) * GPB + threadIdx.x / G;
        const int64_t ng = static_cast<int64_t>(gridDim.x) * GPB;
        for (int64_t row = g0; row < ts.num_tiles; row += ng) {
            const int32_t b = ts.atoms_begin(row), e = ts.atoms_end(row);
            float a0 = 0.f, a1 = 0.f;
            int32_t j = b + gl;
            for (; j + G < e; j += 2 * G) {
                a0 += to_f32(ld_stream(val + j)) * to_f32(x[ld_stream(ci + j)]);
                a1 += to_f32(ld_stream(val + j + G)) * to_f32(x[ld_stream(ci + j + G)]);
            }
            if (j < e) a0 += to_f32(ld_stream(val + j)) * to_f32(x[ld_stream(ci + j)]);
            const float sum = group_sum<G>(a0 + a1);
            if (gl == 0) y[row] = sum;
        }
    } else {
        __shared__ float s_red[BLOCK / kWave];
        for (int64_t row = blockIdx.x; row < ts.num_tiles; row += gridDim.x) {  // block-uniform
            const int32_t b = ts.atoms_begin(row), e = ts.atoms_end(row);
            float a0 = 0.f, a1 = 0.f;
            int32_t j = b + gl;
            for (; j + G < e; j += 2 * G) {
                a0 += to_f32(ld_stream(val + j)) * to_f32(x[ld_stream(ci + j)]);
                a1 += to_f32(ld_stream(val + j + G)) * to_f32(x[ld_stream(ci + j + G)]);
            }
            if (j < e) a0 += to_f32(ld_stream(val + j)) * to_f32(x[ld_stream(ci + j)]);
            const float sum = block_sum<BLOCK>(a0 + a1, s_red);
            if (threadIdx.x == 0) y[row] = sum;
        }
    }
}

// ------------------------------------------------------------------ group-mapped, G tiles per group

// The schedule is the public group_mapped_scan (lb_schedule.hpp), the same
// one the graph traversals run on: per round, the group's G rows are
// prefix-summed in LDS and its lanes stride the flattened nonzeros, each
// finding its row with get_tile.  Per-row sums: a segmented scan over the
// lanes of each step, whose segment tails add into the row's LDS
// accumulator in step order (deterministic).
template <int G, bool QUEUE, typename VT, typename XT>
__global__ __launch_bounds__(group_block<G>::BLOCK) void group_mapped_scan_kernel(
    csr_tile_set ts, const int32_t *__restrict__ ci, const VT *__restrict__ val, const XT *__restrict__ x,
    float *__restrict__ y, int32_t *__restrict__ ticket) {
    using sched = group_mapped_scan<G, csr_tile_set>;
    constexpr int BLOCK = sched::BLOCK;
    constexpr int GPB = sched::GPB;
    __shared__ typename sched::storage s_st[GPB];
    __shared__ float s_acc[GPB][G];
    __shared__ int32_t s_key[G > kWave ? BLOCK : 1];
    __shared__ seg_t s_wave[BLOCK / kWave];

    __shared__ int32_t s_slot;

    const int gl = threadIdx.x & (G - 1);
    const int gi = threadIdx.x / G;
    sched sch(ts, s_st);
    auto round_body = [&](int64_t round) {  // called by every thread of the block
        const int64_t t0 = (round + gi) * G;
        s_acc[gi][gl] = 0.f;
        const int32_t total = sch.load(round);  // ends with a barrier: s_acc is clear
        const int32_t steps = (total + G - 1) / G;
        for (int32_t st = 0; st < steps; ++st) {  // uniform within the group
            const int32_t a = st * G + gl;
            int32_t key = G;  // past the last tile: inactive lane
            float p = 0.f;
            if (a < total) {
                key = sch.get_tile(a);
                const int32_t j = sch.atom(a, key);
                p = to_f32(ld_stream(val + j)) * to_f32(x[ld_stream(ci + j)]);
            }
            if constexpr (G <= kWave) {
                const int32_t prev = __shfl_up(key, 1, G);
                const int32_t next = __shfl_down(key, 1, G);
                const seg_t r = group_seg_scan_incl<G>(seg_t{p, gl == 0 || prev != key});
                const bool tail = gl == G - 1 || next != key;
                if (tail && key < G) s_acc[gi][key] += r.v;
                __builtin_amdgcn_wave_barrier();
            } else {
                s_key[threadIdx.x] = key;
                __syncthreads();
                const int32_t prev = threadIdx.x ? s_key[threadIdx.x - 1] : -1;
                const int32_t next = threadIdx.x + 1 < BLOCK ? s_key[threadIdx.x + 1] : -1;
                seg_t tot;
                const seg_t r = block_seg_scan_incl<BLOCK>(seg_t{p, prev != key}, s_wave, tot);
                if (next != key && key < G) s_acc[0][key] += r.v;
                __syncthreads();
            }
        }
        __syncthreads();
        if (t0 + gl < ts.num_tiles) y[t0 + gl] = s_acc[gi][gl];
        sch.done();
    };
    if constexpr (QUEUE) {  // persistent grid, rounds claimed from the work queue
        const int64_t rounds = ((ts.num_tiles + G - 1) / G + GPB - 1) / GPB;
        for (int64_t round : sch.queued_rounds(ticket, &s_slot, claim_batch(rounds))) round_body(round);
    } else {
        for (int64_t round : sch.rounds()) round_body(round);  // uniform across the block
    }
}

template <typename K>
static int resident_blocks(K kernel, int block) {
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) {
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0);
    }
    return cus * (per_cu > 0 ? per_cu : 1);
}

template <int G, typename VT>
static hipError_t launch_group(const csr_dev &A, const void *x, float *y, int K, int grid, int32_t *ticket,
                               hipStream_t s) {
    constexpr int BLOCK = group_block<G>::BLOCK;
    constexpr int GPB = group_block<G>::GPB;
    const csr_tile_set ts{A.ro, A.rows, A.nnz};
    if (K == 1) {
        const dim3 g(static_cast<uint32_t>(blocks_for(A.rows, GPB, grid)));
        hipLaunchKernelGGL((group_mapped_tile_kernel<G, VT, VT>), g, dim3(BLOCK), 0, s, ts, A.ci,
                           static_cast<const VT *>(A.val), static_cast<const VT *>(x), y);
    } else if (ticket) {  // work queue: zero the counter, then a persistent grid
        const hipError_t e = fill_f32(reinterpret_cast<float *>(ticket), 1, 0.f, s);  // +0.0f is all zero bits
        if (e != hipSuccess) return e;
        const auto kern = group_mapped_scan_kernel<G, true, VT, VT>;
        const int64_t nchunks = (static_cast<int64_t>(A.rows) + G - 1) / G;
        const int64_t g = grid > 0 ? grid : resident_blocks(kern, BLOCK);
        const int64_t need = (nchunks + GPB - 1) / GPB;
        hipLaunchKernelGGL(kern, dim3(static_cast<uint32_t>(g < need ? g : (need > 0 ? need : 1))), dim3(BLOCK), 0,
                           s, ts, A.ci, static_cast<const VT *>(A.val), static_cast<const VT *>(x), y, ticket);
    } else {
        const int64_t nchunks = (static_cast<int64_t>(A.rows) + G - 1) / G;
        const dim3 g(static_cast<uint32_t>(blocks_for(nchunks, GPB, grid)));
        hipLaunchKernelGGL((group_mapped_scan_kernel<G, false, VT, VT>), g, dim3(BLOCK), 0, s, ts, A.ci,
                           static_cast<const VT *>(A.val), static_cast<const VT *>(x), y, nullptr);
    }
    return hipGetLastError();
}

#define LB_GROUP_SIZES(X) X(1) X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024)

hipError_t group_mapped_spmv(const csr_dev &A, const void *x, float *y, int group_size, int tiles_per_group,
                             int grid, int32_t *ticket, hipStream_t s) {
    prof_scope p(s, ticket ? "work_queue" : "group_mapped");
#define X(G)                                                                                           \
    if (group_size == G) {                                                                             \
        if (A.dt == LB_BF16) return launch_group<G, bf16_bits>(A, x, y, tiles_per_group, grid, ticket, s); \
        return launch_group<G, float>(A, x, y, tiles_per_group, grid, ticket, s);                      \
    }
    LB_GROUP_SIZES(X)
#undef X
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ get_tile test hook

template <int G>
__global__ __launch_bounds__(group_block<G>::BLOCK) void group_tile_owner_kernel(csr_tile_set ts,
                                                                                 int32_t *__restrict__ owner) {
    using sched = group_mapped_scan<G, csr_tile_set>;
    __shared__ typename sched::storage s_st[sched::GPB];
    sched sch(ts, s_st);
    for (int64_t round : sch.rounds()) {
        const int32_t total = sch.load(round);
        for (int64_t a : sch.atoms(total)) {
            const int32_t q = sch.get_tile(static_cast<int32_t>(a));
            owner[sch.atom(static_cast<int32_t>(a), q)] = q;
        }
        sch.done();
    }
}

hipError_t group_tile_owner(const csr_dev &A, int tiles_per_group, int32_t *owner, hipStream_t s) {
    const csr_tile_set ts{A.ro, A.rows, A.nnz};
#define X(G)                                                                                           \
    if (tiles_per_group == G) {                                                                        \
        const int64_t nchunks = (static_cast<int64_t>(A.rows) + G - 1) / G;                            \
        const dim3 g(static_cast<uint32_t>(blocks_for(nchunks, group_block<G>::GPB, 0)));              \
        hipLaunchKernelGGL((group_tile_owner_kernel<G>), g, dim3(group_block<G>::BLOCK), 0, s, ts, owner); \
        return hipGetLastError();                                                                      \
    }
    LB_GROUP_SIZES(X)
#undef X
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ utilities

__global__ __launch_bounds__(256) void fill_kernel(float *__restrict__ p, int64_t n, float v) {
    for (int64_t i : grid_stride_range(0, n)) p[i] = v;
}

hipError_t fill_f32(float *p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    prof_scope pr(s, "fill");
    hipLaunchKernelGGL(fill_kernel, dim3(static_cast<uint32_t>(blocks_for(n, 256, 8192))), dim3(256), 0, s, p,
                       n, v);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void sample_kernel(const int32_t *__restrict__ a, int64_t n, int32_t count,
                                                     int32_t *__restrict__ out) {
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < count) out[i] = n > 0 ? a[static_cast<int64_t>(i) * n / count] : 0;
}

__global__ __launch_bounds__(256) void gather_at_kernel(const int32_t *__restrict__ a, const int32_t *__restrict__ pos,
                                                        int32_t count, int32_t *__restrict__ out) {
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < count) out[i] = a[pos[i]];
}

hipError_t gather_at(const int32_t *a, const int32_t *pos, int32_t count, int32_t *out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_at_kernel, dim3(static_cast<uint32_t>((count + 255) / 256)), dim3(256), 0, s, a, pos,
                       count, out);
    return hipGetLastError();
}

hipError_t gather_samples(const int32_t *a, int64_t n, int32_t count, int32_t *out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(sample_kernel, dim3(static_cast<uint32_t>((count + 255) / 256)), dim3(256), 0, s, a, n, count,
                       out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void validate_kernel(csr_tile_set ts, int32_t cols, const int32_t *__restrict__ ci,
                                                       int32_t *__restrict__ flags) {
    int32_t f = 0;
    for (int64_t r : grid_stride_range(0, ts.num_tiles + 1)) {
        const int32_t o = ts.row_offsets[r];
        if (r == 0 && o != 0) f |= 1;
        if (r == ts.num_tiles && o != ts.num_atoms) f |= 1;
        if (r < ts.num_tiles && ts.row_offsets[r + 1] < o) f |= 1;
    }
    for (int64_t j : grid_stride_range(0, ts.num_atoms)) {
        const int32_t c = ci[j];
        if (c < 0 || c >= cols) f |= 2;
    }
    if (f) atomicOr(flags, f);
}

hipError_t validate_csr(const csr_dev &A, int32_t *flags_dev, hipStream_t s) {
    const csr_tile_set ts{A.ro, A.rows, A.nnz};
    const int64_t work = (A.rows + 1) > A.nnz ? A.rows + 1 : A.nnz;
    hipLaunchKernelGGL(validate_kernel, dim3(static_cast<uint32_t>(blocks_for(work, 256, 4096))), dim3(256), 0, s,
                       ts, A.cols, A.ci, flags_dev);
    return hipGetLastError();
}

}  // namespace lbk
