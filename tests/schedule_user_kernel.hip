// A user's kernels written only against the public schedule header: SpMV
// over CSR and COO tile sets under each schedule, and a persistent variant
// on the work queue.  Compiled (not run) by the CPU test suite to show the
// header stands alone.
#include "lb_schedule.hpp"

template <class Sched>
__device__ void spmv_tiles(const Sched &sch, const int32_t *ci, const float *val, const float *x, float *y) {
    for (int64_t p : sch.tiles()) {
        const lb::tile_ref t = sch.ts.tile(p);
        float acc = 0.f;
        for (int64_t e : sch.atoms(t)) acc += val[e] * x[ci[e]];
        y[t.id] = acc;  // thread-mapped: one thread per tile
    }
}

__global__ void csr_thread(lb::csr_tile_set ts, const int32_t *ci, const float *val, const float *x, float *y) {
    spmv_tiles(lb::thread_mapped<lb::csr_tile_set>{ts}, ci, val, x, y);
}

__global__ void coo_thread(lb::coo_tile_set ts, const int32_t *ci, const float *val, const float *x, float *y) {
    spmv_tiles(lb::thread_mapped<lb::coo_tile_set>{ts}, ci, val, x, y);
}

template <int G>
__global__ __launch_bounds__(lb::group_block<G>::BLOCK) void csr_group(lb::csr_tile_set ts, const int32_t *ci,
                                                                       const float *val, const float *x, float *y) {
    const lb::group_mapped<G, lb::csr_tile_set> sch{ts};
    for (int64_t p : sch.tiles()) {
        const lb::tile_ref t = sch.ts.tile(p);
        float acc = 0.f;
        for (int64_t e : sch.atoms(t)) acc += val[e] * x[ci[e]];
        for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
        if (sch.lane() == 0) y[t.id] = acc;
    }
}
template __global__ void csr_group<32>(lb::csr_tile_set, const int32_t *, const float *, const float *, float *);

// G tiles per group, rounds from a grid stride or from a work queue: each
// atom's tile comes from get_tile; per-tile sums go through LDS atomics.
template <int G, bool QUEUE>
__global__ __launch_bounds__(lb::group_block<G>::BLOCK) void csr_scan(lb::csr_tile_set ts, const int32_t *ci,
                                                                      const float *val, const float *x, float *y,
                                                                      int32_t *ticket) {
    using sched = lb::group_mapped_scan<G, lb::csr_tile_set>;
    __shared__ typename sched::storage st[sched::GPB];
    __shared__ float acc[sched::GPB][G];
    __shared__ int32_t slot;
    sched sch(ts, st);
    auto body = [&](int64_t round) {
        acc[threadIdx.x / G][sch.lane()] = 0.f;
        const int32_t total = sch.load(round);  // ends with a block barrier
        for (int64_t a : sch.atoms(total)) {
            const int32_t q = sch.get_tile(static_cast<int32_t>(a));
            const int32_t e = sch.atom(static_cast<int32_t>(a), q);
            atomicAdd(&acc[threadIdx.x / G][q], val[e] * x[ci[e]]);
        }
        __syncthreads();
        const int64_t t = (round + threadIdx.x / G) * G + sch.lane();
        if (t < ts.num_tiles) y[t] = acc[threadIdx.x / G][sch.lane()];
        sch.done();
    };
    if constexpr (QUEUE) {
        for (int64_t r : sch.queued_rounds(ticket, &slot)) body(r);
    } else {
        for (int64_t r : sch.rounds()) body(r);
    }
}
template __global__ void csr_scan<64, false>(lb::csr_tile_set, const int32_t *, const float *, const float *,
                                             float *, int32_t *);
template __global__ void csr_scan<256, true>(lb::csr_tile_set, const int32_t *, const float *, const float *,
                                             float *, int32_t *);

// A frontier (indexed tile set) walked until a caller-given bound, in
// persistent form with infinite_range.
__global__ void frontier_sizes(lb::indexed_tile_set ts, int64_t *sizes, int64_t bound) {
    for (int64_t i : lb::infinite_range{static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x,
                                        static_cast<int64_t>(gridDim.x) * blockDim.x}) {
        if (i >= bound || i >= ts.num_tiles) break;
        const lb::tile_ref t = ts.tile(i);
        sizes[i] = t.end - t.begin;
    }
}
