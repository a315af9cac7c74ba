// Graph traversal written on the public schedules of lb_schedule.hpp: the
// SSSP example of Sec. 5.3 and BFS (named in Sec. 6).  A graph is a CSR
// tile set read as adjacency: vertex u's out-edges are the atoms of tile u,
// edge e goes to col_idx[e] and weighs w[e].
//
// Iteration i takes frontier F_i, a compacted list of vertex ids (the tiles
// of an indexed_tile_set), and relaxes every out-edge of its vertices under
// the chosen schedule; the vertices that improve form F_{i+1}, each listed
// once.  The host launches again while the frontier holds vertices (Sec. 5.3).
//  * SSSP: dist is float32.  The offer dist[u] + w is one float32 addition
//    and an atomic minimum on the bit pattern keeps the smaller value
//    (non-negative floats order like their int32 bit patterns).  A vertex
//    joins F_{i+1} at most once: it carries the iteration that last queued
//    it, so nothing is cleared between iterations.
//  * BFS: depth is int32, -1 = unvisited; the compare-and-swap from -1 to
//    i + 1 that succeeds claims the vertex.
// Appends are aggregated per block: the merge-path advance places a unit's
// new vertices with a block prefix sum and one atomicAdd; the other
// schedules stage them in an LDS buffer and reserve its stretch with one
// atomicAdd per block (per round for the prefix-sum form).  Pushes past the
// buffer fall back to one atomicAdd per wavefront.
//
// Under merge-path an iteration is five launches (degree scan, split,
// consume; see below); under the other schedules one.  Each advance launch
// is persistent (the resident grid) and reads the frontier size from device
// memory, so the host enqueues a batch of
// iterations without waiting and reads the size once per batch to stop.
// Three rotating counters: launch i reads counter i % 3, appends to
// (i + 1) % 3 and zeroes (i + 2) % 3, the one launch i + 1 appends to (and
// launch i - 1 last read), so no memset and no host round trip is needed.
#include <math.h>

#include "lb_device.h"
#include "lb_internal.h"
#include "lb_schedule.hpp"

namespace lbk {
using namespace lb;

namespace {

constexpr int32_t kUnvisited = -1;

struct trav_args {
    const int32_t *ro;
    const int32_t *ci;
    const float *w;
    float *dist;        // SSSP
    int32_t *depth;     // BFS
    int32_t *stamp;     // SSSP: iteration that last queued each vertex
    const int32_t *q_in;
    int32_t *q_out;
    const int32_t *cnt_in;
    int32_t *cnt_out;
    int32_t *cnt_clear;
    int32_t *rounds;    // non-empty frontiers processed
    int32_t *ticket;        // work queue of this launch (LB_WORK_QUEUE)
    int32_t *ticket_clear;  // the next launch's work queue, zeroed here
    int32_t iter;
};

// Appends v for every active lane with `want`; every active lane of the
// wavefront calls it (inactive lanes take no part in the ballot).
__device__ __forceinline__ void frontier_push(bool want, int32_t v, int32_t *q_out, int32_t *cnt_out) {
    const uint64_t m = __ballot(want);
    if (m == 0) return;
    const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
    int32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(cnt_out, __popcll(m));
    base = __shfl(base, leader);
    if (want) q_out[base + __popcll(m & ((1ull << lane_id()) - 1))] = v;
}

// Block-staged appends for the thread- and group-mapped advances: a push
// takes its slot in an LDS buffer from an LDS counter (one LDS atomic per
// wavefront), and flush() reserves the buffer's stretch of the next
// frontier with one global atomic per block, then copies it out.  Pushes
// past the buffer's capacity go straight to the frontier.  One global atomic
// per wavefront and step put every wavefront of the grid on the one frontier
// counter; staging takes that counter off the critical path.
template <int CAP>
struct staged_frontier {
    int32_t *buf;  // LDS, CAP entries
    int32_t *n;    // LDS: entries pushed (may exceed CAP: the rest went straight out)
    int32_t *base; // LDS: the block's first slot in the frontier
    // every thread of the block calls it, before the first push
    __device__ void start() {
        if (threadIdx.x == 0) *n = 0;
        __syncthreads();
    }
    // every active lane of the wavefront calls it
    __device__ void push(bool want, int32_t v, int32_t *q_out, int32_t *cnt_out) {
        const uint64_t m = __ballot(want);
        if (m == 0) return;
        const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
        int32_t pos0 = 0;
        if (lane_id() == leader) pos0 = atomicAdd(n, __popcll(m));
        pos0 = __shfl(pos0, leader);
        const int32_t pos = pos0 + __popcll(m & ((1ull << lane_id()) - 1));
        const bool spill = want && pos >= CAP;
        if (want && !spill) buf[pos] = v;
        frontier_push(spill, v, q_out, cnt_out);
    }
    // every thread of the block calls it; the buffer is empty afterwards
    __device__ void flush(int32_t *q_out, int32_t *cnt_out) {
        __syncthreads();
        const int32_t k = *n < CAP ? *n : CAP;
        if (threadIdx.x == 0) *base = k > 0 ? atomicAdd(cnt_out, k) : 0;
        __syncthreads();
        for (int32_t i = threadIdx.x; i < k; i += blockDim.x) q_out[*base + i] = buf[i];
        __syncthreads();
        if (threadIdx.x == 0) *n = 0;
        __syncthreads();
    }
};
constexpr int kStageCap = 2048;

// Relaxes edge e of a vertex whose distance is du; returns true when the
// target v must join the next frontier.
template <bool BFS>
__device__ __forceinline__ bool relax(const trav_args &t, float du, int32_t e, int32_t &v) {
    v = t.ci[e];
    if constexpr (BFS) {
        // a stale read can only show -1 for a claimed vertex: the CAS decides
        if (t.depth[v] != kUnvisited) return false;
        return atomicCAS(t.depth + v, kUnvisited, t.iter + 1) == kUnvisited;
    } else {
        const float offer = du + t.w[e];
        // distances only decrease, so a stale read is >= the current value:
        // an offer that does not beat it cannot beat the current one
        if (!(offer < t.dist[v])) return false;
        const int32_t old = atomicMin(reinterpret_cast<int32_t *>(t.dist) + v, __float_as_int(offer));
        if (!(offer < __int_as_float(old))) return false;
        return atomicExch(t.stamp + v, t.iter) != t.iter;
    }
}

__device__ __forceinline__ int32_t frontier_size(const trav_args &t) {
    const int32_t nf = *t.cnt_in;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *t.cnt_clear = 0;
        *t.ticket_clear = 0;
        if (nf > 0) *t.rounds += 1;
    }
    return nf;
}

template <bool BFS>
__device__ __forceinline__ float tile_dist(const trav_args &t, int32_t u) {
    if constexpr (BFS)
        return 0.f;
    else
        return t.dist[u];
}

template <bool BFS>
__global__ __launch_bounds__(1024) void advance_thread_kernel(trav_args t) {
    __shared__ int32_t s_buf[kStageCap];
    __shared__ int32_t s_n, s_base;
    staged_frontier<kStageCap> out{s_buf, &s_n, &s_base};
    out.start();
    const int32_t nf = frontier_size(t);
    const thread_mapped<indexed_tile_set> sch{{t.q_in, t.ro, nf}};
    for (int64_t p : sch.tiles()) {
        const tile_ref tile = sch.ts.tile(p);
        const float du = tile_dist<BFS>(t, tile.id);
        for (int64_t e : sch.atoms(tile)) {
            int32_t v;
            const bool want = relax<BFS>(t, du, static_cast<int32_t>(e), v);
            out.push(want, v, t.q_out, t.cnt_out);
        }
    }
    out.flush(t.q_out, t.cnt_out);
}

template <int G, bool BFS>
__global__ __launch_bounds__(group_block<G>::BLOCK) void advance_group_kernel(trav_args t) {
    __shared__ int32_t s_buf[kStageCap];
    __shared__ int32_t s_n, s_base;
    staged_frontier<kStageCap> out{s_buf, &s_n, &s_base};
    out.start();
    const int32_t nf = frontier_size(t);
    const group_mapped<G, indexed_tile_set> sch{{t.q_in, t.ro, nf}};
    for (int64_t p : sch.tiles()) {
        const tile_ref tile = sch.ts.tile(p);
        const float du = tile_dist<BFS>(t, tile.id);
        for (int64_t e : sch.atoms(tile)) {
            int32_t v;
            const bool want = relax<BFS>(t, du, static_cast<int32_t>(e), v);
            out.push(want, v, t.q_out, t.cnt_out);
        }
    }
    out.flush(t.q_out, t.cnt_out);
}

template <int G, bool BFS, bool QUEUE>
__global__ __launch_bounds__(group_block<G>::BLOCK) void advance_scan_kernel(trav_args t) {
    using sched = group_mapped_scan<G, indexed_tile_set>;
    __shared__ typename sched::storage st[sched::GPB];
    __shared__ int32_t s_slot;
    __shared__ int32_t s_buf[kStageCap];
    __shared__ int32_t s_n, s_base;
    staged_frontier<kStageCap> out{s_buf, &s_n, &s_base};
    out.start();
    const int32_t nf = frontier_size(t);
    sched sch(indexed_tile_set{t.q_in, t.ro, nf}, st);
    auto round_body = [&](int64_t round) {  // called by every thread of the block
        const int32_t total = sch.load(round);
        for (int64_t a : sch.atoms(total)) {
            const int32_t q = sch.get_tile(static_cast<int32_t>(a));
            const int32_t u = sch.tile(q);
            const int32_t e = sch.atom(static_cast<int32_t>(a), q);
            int32_t v;
            const bool want = relax<BFS>(t, tile_dist<BFS>(t, u), e, v);
            out.push(want, v, t.q_out, t.cnt_out);
        }
        out.flush(t.q_out, t.cnt_out);  // per round: the buffer never holds more than one round
        sch.done();
    };
    if constexpr (QUEUE) {
        const int64_t rounds = ((static_cast<int64_t>(nf) + G - 1) / G + sched::GPB - 1) / sched::GPB;
        for (int64_t round : sch.queued_rounds(t.ticket, &s_slot, claim_batch(rounds))) round_body(round);
    } else {
        for (int64_t round : sch.rounds()) round_body(round);  // uniform across the block
    }
}

// ---------------------------------------------------------------- merge-path over the frontier
//
// The frontier as a tile set for merge-path (Sec. 5.2.1) needs its "row
// offsets": offs[p] = out-degrees of frontier entries [0, p).  Per
// iteration: (1) per tile of kScanTile entries, the in-tile exclusive
// prefix sums and the tile total; (2) one block scans the tile totals and
// records the frontier's edge count E_f and unit count T_f; (3) the tile
// prefixes are added in; (4) the split at every unit boundary of the merge
// of offs[1..nf] with the edges 0..E_f-1 (the SpMV split); (5) a persistent
// consume: each unit stages its frontier entries in LDS and each thread
// walks kMergeItems merge items, relaxing the edges it meets; the unit's new
// frontier vertices are appended with one atomic per block (a block prefix
// sum of the threads' counts), not one per wavefront and merge item.  Every
// grid is sized for the largest frontier (every vertex); blocks past the
// frontier's work leave at once.

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kMergeBlock = 256;
constexpr int kMergeItems = 8;
constexpr int kMergeW = kMergeBlock * kMergeItems;
constexpr int kPartGroup = 16;

__global__ __launch_bounds__(kScanThreads) void frontier_scan_tiles(const int32_t *__restrict__ q,
                                                                    const int32_t *__restrict__ cnt_in,
                                                                    const int32_t *__restrict__ ro,
                                                                    int32_t *__restrict__ offs,
                                                                    int32_t *__restrict__ tile_sum) {
    __shared__ int32_t s_wave[kScanThreads / kWave];
    const int32_t nf = *cnt_in;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    if (base >= nf) return;  // uniform across the block
    int32_t deg[kScanItems];
    int32_t sum = 0;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const int64_t p = base + threadIdx.x * kScanItems + u;
        int32_t dg = 0;
        if (p < nf) {
            const int32_t v = q[p];
            dg = ro[v + 1] - ro[v];
        }
        deg[u] = dg;
        sum += dg;
    }
    const int32_t incl = block_scan_incl<kScanThreads>(sum, s_wave);
    int32_t run = incl - sum;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const int64_t p = base + threadIdx.x * kScanItems + u;
        if (p < nf) offs[p] = run;
        run += deg[u];
    }
    if (threadIdx.x == kScanThreads - 1) tile_sum[blockIdx.x] = incl;
}

// One block: exclusive prefix of the tile totals (in place), then
// offs[nf] = E_f, meta = {E_f, T_f}.
__global__ __launch_bounds__(1024) void frontier_scan_totals(const int32_t *__restrict__ cnt_in,
                                                             int32_t *__restrict__ tile_sum,
                                                             int32_t *__restrict__ offs,
                                                             int32_t *__restrict__ meta) {
    __shared__ int32_t s_wave[1024 / kWave];
    __shared__ int32_t s_total;
    const int32_t nf = *cnt_in;
    const int32_t nb = (nf + kScanTile - 1) / kScanTile;
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
    if (threadIdx.x == 0) {
        offs[nf] = carry;
        meta[0] = carry;
        meta[1] = (nf + carry + kMergeW - 1) / kMergeW;
    }
}

__global__ __launch_bounds__(256) void frontier_scan_add(const int32_t *__restrict__ cnt_in,
                                                         const int32_t *__restrict__ tile_pre,
                                                         int32_t *__restrict__ offs) {
    const int32_t nf = *cnt_in;
    for (int64_t p : grid_stride_range(0, nf)) offs[p] += tile_pre[p / kScanTile];
}

// Split at boundaries t in [0, T_f]: one group of kPartGroup lanes each.
__global__ __launch_bounds__(256) void frontier_partition(const int32_t *__restrict__ cnt_in,
                                                          const int32_t *__restrict__ offs,
                                                          const int32_t *__restrict__ meta,
                                                          int32_t *__restrict__ part_i,
                                                          int32_t *__restrict__ part_j) {
    const int32_t nf = *cnt_in, ef = meta[0], T = meta[1];
    const int64_t first = static_cast<int64_t>(blockIdx.x) * (256 / kPartGroup);
    if (nf == 0 || first > T) return;  // uniform across the block
    const int64_t t = first + threadIdx.x / kPartGroup;
    const bool live = t <= T;  // uniform per group; every lane still takes part in the ballots
    const int64_t total = static_cast<int64_t>(nf) + ef;
    const int64_t tt = live ? t : T;
    const int32_t d = static_cast<int32_t>(tt * kMergeW < total ? tt * kMergeW : total);
    const int32_t i = group_merge_search<kPartGroup>(offs, nf, ef, d);
    if (live && (threadIdx.x & (kPartGroup - 1)) == 0) {
        part_i[t] = i;
        part_j[t] = d - i;
    }
}

template <bool BFS>
__global__ __launch_bounds__(kMergeBlock) void advance_merge_kernel(trav_args t, const int32_t *__restrict__ offs,
                                                                    const int32_t *__restrict__ meta,
                                                                    const int32_t *__restrict__ part_i,
                                                                    const int32_t *__restrict__ part_j) {
    // frontier entries touched by the unit: row ends relative to j0, the
    // edge id of atom j of entry k is s_base[k] + j, and the entry's distance
    __shared__ int32_t s_end[kMergeW + 1];
    __shared__ int32_t s_base[kMergeW + 1];
    __shared__ float s_du[BFS ? 1 : kMergeW + 1];
    __shared__ int32_t s_wave[kMergeBlock / kWave];
    __shared__ int32_t s_out;
    const int32_t nf = frontier_size(t);
    const int32_t T = nf > 0 ? meta[1] : 0;
    const int tid = threadIdx.x;
    for (int32_t u = blockIdx.x; u < T; u += gridDim.x) {  // uniform across the block
        const int32_t i0 = part_i[u], j0 = part_j[u];
        const int32_t i1 = part_i[u + 1], j1 = part_j[u + 1];
        const int32_t nrows = i1 - i0, nnzs = j1 - j0;
        const int32_t last = i1 < nf ? i1 : nf - 1;  // the entry holding the unit's trailing atoms
        for (int32_t k = tid; k <= last - i0; k += kMergeBlock) {
            const int32_t p = i0 + k;
            const int32_t v = t.q_in[p];
            s_end[k] = offs[p + 1] - j0;
            s_base[k] = t.ro[v] - offs[p];
            if constexpr (!BFS) s_du[k] = t.dist[v];
        }
        __syncthreads();
        // this thread's merge items [d, dend) of the unit's nrows + nnzs
        const int32_t total = nrows + nnzs;
        const int32_t d = tid * kMergeItems < total ? tid * kMergeItems : total;
        const int32_t dend = d + kMergeItems < total ? d + kMergeItems : total;
        int32_t lo = d - nnzs > 0 ? d - nnzs : 0;
        int32_t hi = d < nrows ? d : nrows;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (s_end[mid] + mid < d)
                lo = mid + 1;
            else
                hi = mid;
        }
        int32_t it = lo, jt = d - lo;
        bool want[kMergeItems];
        int32_t nv[kMergeItems];
        int32_t mine = 0;
#pragma unroll
        for (int s = 0; s < kMergeItems; ++s) {
            want[s] = false;
            nv[s] = 0;
            if (d + s < dend) {
                if (it < nrows && s_end[it] <= jt) {
                    ++it;  // entry it's edges are done
                } else {
                    const int32_t j = j0 + jt;
                    want[s] = relax<BFS>(t, BFS ? 0.f : s_du[it], s_base[it] + j, nv[s]);
                    ++jt;
                }
            }
            mine += want[s] ? 1 : 0;
        }
        // the unit's new frontier vertices go out with one atomic per block:
        // a block prefix sum of the threads' counts places each thread's run
        const int32_t incl = block_scan_incl<kMergeBlock>(mine, s_wave);
        if (tid == kMergeBlock - 1) s_out = incl > 0 ? atomicAdd(t.cnt_out, incl) : 0;
        __syncthreads();
        int32_t pos = s_out + incl - mine;
#pragma unroll
        for (int s = 0; s < kMergeItems; ++s)
            if (want[s]) t.q_out[pos++] = nv[s];
        __syncthreads();
    }
}

template <bool BFS>
__global__ __launch_bounds__(256) void traversal_init_kernel(int32_t n, int32_t source, float *dist,
                                                             int32_t *depth, int32_t *stamp, int32_t *q0,
                                                             int32_t *counters) {
    for (int64_t v : grid_stride_range(0, n)) {
        if constexpr (BFS) {
            depth[v] = v == source ? 0 : kUnvisited;
        } else {
            dist[v] = v == source ? 0.f : INFINITY;
            stamp[v] = -1;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        q0[0] = source;
        counters[0] = 1;  // F_0 = {source}
        counters[1] = 0;
        counters[2] = 0;
        counters[3] = 0;  // rounds
        counters[4] = 0;  // work-queue tickets of the first two launches
        counters[5] = 0;
    }
}

template <typename K>
int resident_blocks(K kernel, int block) {
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess) {
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0);
    }
    return cus * (per_cu > 0 ? per_cu : 1);
}

template <typename K>
hipError_t launch_advance(K kernel, int block, int grid, const trav_args &t, hipStream_t s) {
    const int g = grid > 0 ? grid : resident_blocks(kernel, block);
    hipLaunchKernelGGL(kernel, dim3(static_cast<uint32_t>(g)), dim3(block), 0, s, t);
    return hipGetLastError();
}

template <bool BFS>
hipError_t advance_merge(const csr_dev &G, const trav_cfg &c, const trav_ws &w, const trav_args &t, hipStream_t s) {
    const int64_t n = G.rows;
    const int64_t scan_blocks = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(frontier_scan_tiles, dim3(static_cast<uint32_t>(scan_blocks)), dim3(kScanThreads), 0, s,
                       t.q_in, t.cnt_in, G.ro, w.offs, w.tile_sum);
    hipLaunchKernelGGL(frontier_scan_totals, dim3(1), dim3(1024), 0, s, t.cnt_in, w.tile_sum, w.offs, w.meta);
    const int64_t add_blocks = (n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048;
    hipLaunchKernelGGL(frontier_scan_add, dim3(static_cast<uint32_t>(add_blocks)), dim3(256), 0, s, t.cnt_in,
                       w.tile_sum, w.offs);
    const int64_t tmax = trav_merge_units(n, G.nnz);
    const int64_t part_blocks = ((tmax + 1) * kPartGroup + 255) / 256;
    hipLaunchKernelGGL(frontier_partition, dim3(static_cast<uint32_t>(part_blocks)), dim3(256), 0, s, t.cnt_in,
                       w.offs, w.meta, w.part_i, w.part_j);
    const int grid = c.grid > 0 ? c.grid : resident_blocks(advance_merge_kernel<BFS>, kMergeBlock);
    hipLaunchKernelGGL(advance_merge_kernel<BFS>, dim3(static_cast<uint32_t>(grid)), dim3(kMergeBlock), 0, s, t,
                       w.offs, w.meta, w.part_i, w.part_j);
    return hipGetLastError();
}

template <bool BFS>
hipError_t advance(const csr_dev &G, const trav_cfg &c, const trav_ws &w, const trav_args &t, hipStream_t s) {
    prof_scope p(s, BFS ? "bfs_advance" : "sssp_advance");
    if (c.kind == LB_MERGE_PATH) return advance_merge<BFS>(G, c, w, t, s);
    if (c.kind == LB_THREAD_MAPPED) return launch_advance(advance_thread_kernel<BFS>, c.block, c.grid, t, s);
#define LB_G(G)                                                                                               \
    if (c.group == G) {                                                                                       \
        if (c.kind == LB_WORK_QUEUE)                                                                          \
            return launch_advance(advance_scan_kernel<G, BFS, true>, group_block<G>::BLOCK, c.grid, t, s);     \
        if (c.tiles_per_group == 1)                                                                           \
            return launch_advance(advance_group_kernel<G, BFS>, group_block<G>::BLOCK, c.grid, t, s);          \
        return launch_advance(advance_scan_kernel<G, BFS, false>, group_block<G>::BLOCK, c.grid, t, s);        \
    }
    LB_TRAVERSAL_GROUPS(LB_G)
#undef LB_G
    return hipErrorInvalidValue;
}

template <bool BFS>
hipError_t run_traversal(const csr_dev &G, int32_t source, float *dist, int32_t *depth, const trav_cfg &c,
                         int32_t max_iter, int32_t *iterations, bool *converged, void *ws, hipStream_t s) {
    const trav_ws w = trav_ws_carve(ws, G.rows, G.nnz);
    {
        prof_scope p(s, "traversal_init");
        const int64_t blocks = (static_cast<int64_t>(G.rows) + 255) / 256;
        hipLaunchKernelGGL(traversal_init_kernel<BFS>, dim3(static_cast<uint32_t>(blocks < 8192 ? blocks : 8192)),
                           dim3(256), 0, s, G.rows, source, dist, depth, w.stamp, w.queue[0], w.counters);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    trav_args t{G.ro, G.ci, static_cast<const float *>(G.val), dist, depth, w.stamp,
                nullptr, nullptr, nullptr, nullptr, nullptr, w.counters + 3, nullptr, nullptr, 0};
    int32_t launched = 0, batch = 4;
    int32_t host[4] = {0, 0, 0, 0};
    *converged = false;
    for (;;) {
        for (int k = 0; k < batch && launched < max_iter; ++k, ++launched) {
            t.iter = launched;
            t.q_in = w.queue[launched & 1];
            t.q_out = w.queue[(launched + 1) & 1];
            t.cnt_in = w.counters + launched % 3;
            t.cnt_out = w.counters + (launched + 1) % 3;
            t.cnt_clear = w.counters + (launched + 2) % 3;
            t.ticket = w.counters + 4 + (launched & 1);
            t.ticket_clear = w.counters + 4 + ((launched + 1) & 1);
            const hipError_t e = advance<BFS>(G, c, w, t, s);
            if (e != hipSuccess) return e;
        }
        hipError_t e = hipMemcpyAsync(host, w.counters, sizeof host, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (host[launched % 3] == 0) {
            *converged = true;
            break;
        }
        if (launched >= max_iter) break;
        batch = batch * 2 < 32 ? batch * 2 : 32;
    }
    if (iterations) *iterations = host[3];
    return hipSuccess;
}

}  // namespace

bool traversal_group_supported(int g) {
#define LB_G(G) if (g == G) return true;
    LB_TRAVERSAL_GROUPS(LB_G)
#undef LB_G
    return false;
}

hipError_t sssp(const csr_dev &G, int32_t source, float *dist, const trav_cfg &c, int32_t max_iter,
                int32_t *iterations, bool *converged, void *ws, hipStream_t s) {
    return run_traversal<false>(G, source, dist, nullptr, c, max_iter, iterations, converged, ws, s);
}

hipError_t bfs(const csr_dev &G, int32_t source, int32_t *depth, const trav_cfg &c, int32_t max_iter,
               int32_t *iterations, bool *converged, void *ws, hipStream_t s) {
    return run_traversal<true>(G, source, nullptr, depth, c, max_iter, iterations, converged, ws, s);
}

}  // namespace lbk
