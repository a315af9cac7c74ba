// Device-side schedules of the load-balancing programming model (Osama,
// Porumbescu, Owens, "A Programming Model for GPU Load Balancing", PPoPP'23)
// for HIP kernels on gfx950 (wave64).  Header-only: a kernel includes it,
// builds a tile set over its data and lets a schedule hand tiles and atoms
// to its threads, so the computation is written once and the schedule is a
// template argument.
//
// Tile sets (Sec. 3.1 and 4.1): tiles own contiguous ranges of atoms.
//   csr_tile_set      tile p is row p; its atoms are [offsets[p], offsets[p+1]).
//   coo_tile_set      tile p is row p of a row-sorted COO; its atoms are
//                     found by binary search of the row indices.
//   indexed_tile_set  tile position p names row ids[p] (a graph frontier,
//                     a list of selected rows); its atoms are that row's.
//   Each gives tile(p) -> {id, begin, end} (one read of ids[p] for the
//   indexed set).
//
// Ranges (Sec. 5.1): step_range, grid_stride_range, infinite_range, and
// queue_rounds, a work queue that hands rounds to persistent blocks.
//
// Schedules (Sec. 4.2, 5.1, 5.2.3):
//   thread_mapped<TS>          each thread takes whole tiles (grid stride) and
//                              walks their atoms one by one.
//   group_mapped<G, TS>        a group of G lanes takes one tile and strides
//                              its atoms by G (K = 1 tile per group).
//   group_mapped_scan<G, TS>   a group of G lanes takes G tiles, prefix-sums
//                              their atom counts in LDS and strides the
//                              flattened atoms; get_tile(a) is the last tile
//                              whose prefix sum is <= a (upper_bound - 1), so
//                              empty tiles own no atom (K = G); its rounds
//                              come from a grid stride (rounds()) or from a
//                              work queue (queued_rounds()).
//
// Group shape: groups of up to one wavefront are packed 256 lanes to a
// block; a group of more than 64 lanes is one block.  Launch group
// schedules with group_block<G>::BLOCK threads per block.
//
// Example, the SSSP relaxation of Sec. 5.3 over a frontier:
//
//   using sched = lb::group_mapped_scan<64, lb::indexed_tile_set>;
//   __shared__ sched::storage st[sched::GPB];
//   sched s(lb::indexed_tile_set{frontier, offsets, frontier_size}, st);
//   for (int64_t round : s.rounds()) {          // uniform across the block
//       const int32_t total = s.load(round);    // every thread of the block
//       for (int64_t a : s.atoms(total)) {
//           const int32_t q = s.get_tile(a);
//           const int32_t u = s.tile(q), e = s.atom(a, q);
//           ... relax edge e of vertex u ...
//       }
//       s.done();                                // every thread of the block
//   }
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lb {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

// ---------------------------------------------------------------- ranges (Sec. 5.1)

// [begin, end) in steps of `step`; 64-bit so a grid stride never wraps.
struct step_range {
    int64_t b, e, s;
    struct iterator {
        int64_t v, s;
        __device__ int64_t operator*() const { return v; }
        __device__ iterator &operator++() {
            v += s;
            return *this;
        }
        __device__ bool operator!=(const iterator &o) const { return v < o.v; }
    };
    __device__ iterator begin() const { return {b, s}; }
    __device__ iterator end() const { return {e, s}; }
};

__device__ __forceinline__ step_range grid_stride_range(int64_t begin, int64_t end) {
    return {static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x + begin, end,
            static_cast<int64_t>(gridDim.x) * blockDim.x};
}

// begin, begin + step, ... with no end (Sec. 5.1, persistent kernels): the
// loop body decides when to stop.
struct infinite_range {
    int64_t b, s;
    struct iterator {
        int64_t v, s;
        __device__ int64_t operator*() const { return v; }
        __device__ iterator &operator++() {
            v += s;
            return *this;
        }
        __device__ bool operator!=(const iterator &) const { return true; }
    };
    __device__ iterator begin() const { return {b, s}; }
    __device__ iterator end() const { return {b, s}; }
};

// A work queue for persistent blocks: rounds [0, count) are handed out at run
// time by atomicAdd on a device counter (thread 0 claims, LDS broadcasts),
// so a block that finishes early takes more work.  The iterator yields round
// starts `step` apart; one claim takes `batch` of them (batch > 1 trades
// balance for fewer atomics on the one counter, which serialise when
// thousands of blocks claim small rounds).  Uniform across the block: every
// thread of the block iterates it.  The counter must hold 0 when the launch
// starts; s_slot is one int of LDS.
struct queue_rounds {
    int32_t *ticket;
    int32_t *s_slot;
    int64_t step, count;  // rounds per yielded start; rounds in all
    int64_t batch = 1;    // yielded starts per claim
    __device__ int64_t claim() const {
        __syncthreads();  // every thread has read the previous claim
        if (threadIdx.x == 0) *s_slot = atomicAdd(ticket, static_cast<int32_t>(step * batch));
        __syncthreads();
        return *s_slot;
    }
    struct iterator {
        const queue_rounds *q;
        int64_t v;
        int64_t left;  // starts of the current claim after v
        __device__ int64_t operator*() const { return v; }
        __device__ iterator &operator++() {
            if (left > 0) {
                v += q->step;
                --left;
            } else {
                v = q->claim();
                left = q->batch - 1;
            }
            return *this;
        }
        __device__ bool operator!=(const iterator &o) const { return v < o.v; }
    };
    __device__ iterator begin() const { return {this, claim(), batch - 1}; }
    __device__ iterator end() const { return {this, count, 0}; }
};

// ---------------------------------------------------------------- collectives used by the schedules

// Inclusive prefix sum over aligned groups of G lanes (G a power of two <= 64).
template <int G>
__device__ __forceinline__ int32_t group_scan_incl(int32_t v) {
    const int gl = threadIdx.x & (G - 1);
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
        const int32_t o = __shfl_up(v, off, G);
        if (gl >= off) v += o;
    }
    return v;
}

// Block-wide inclusive prefix sum (all threads call); s_wave holds BLOCK/64 ints.
template <int BLOCK>
__device__ __forceinline__ int32_t block_scan_incl(int32_t v, int32_t *s_wave) {
    constexpr int NW = BLOCK / kWave;
    const int w = wave_id();
    v = group_scan_incl<kWave>(v);
    if (lane_id() == kWave - 1) s_wave[w] = v;
    __syncthreads();
    int32_t pre = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k)
        if (k < w) pre += s_wave[k];
    __syncthreads();
    return v + pre;
}

// Index of the tile owning atom a given the K + 1 exclusive prefix sums of
// K tiles' atom counts: the last q with scan[q] <= a (upper_bound - 1).
template <int K>
__device__ __forceinline__ int32_t get_tile(const int32_t *scan, int32_t a) {
    int32_t lo = 0, hi = K + 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (scan[mid] <= a)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo - 1;
}

// ---------------------------------------------------------------- tile sets (Sec. 3.1, 4.1)

struct tile_ref {
    int32_t id, begin, end;  // tile id and its atoms [begin, end)
};

// Rows of a CSR offsets array as tiles.
struct csr_tile_set {
    const int32_t *row_offsets;
    int64_t num_tiles;
    int64_t num_atoms;
    __device__ int32_t atoms_begin(int64_t p) const { return row_offsets[p]; }
    __device__ int32_t atoms_end(int64_t p) const { return row_offsets[p + 1]; }
    __device__ int32_t atom_count(int64_t p) const { return row_offsets[p + 1] - row_offsets[p]; }
    __device__ tile_ref tile(int64_t p) const {
        return {static_cast<int32_t>(p), row_offsets[p], row_offsets[p + 1]};
    }
};

// A row-sorted COO as tiles: tile p is row p and its atoms are the entries
// with row_idx == p.  With no offsets array, the atoms-per-tile iterator is
// a binary search of row_idx for the first entry of row p and of row p + 1.
struct coo_tile_set {
    const int32_t *row_idx;
    int64_t num_tiles;
    int64_t num_atoms;
    __device__ int32_t first_entry(int64_t r) const {  // lower_bound(row_idx, r)
        int64_t lo = 0, hi = num_atoms;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (row_idx[mid] < r)
                lo = mid + 1;
            else
                hi = mid;
        }
        return static_cast<int32_t>(lo);
    }
    __device__ tile_ref tile(int64_t p) const {
        return {static_cast<int32_t>(p), first_entry(p), first_entry(p + 1)};
    }
};

// Selected rows as tiles: position p is row ids[p].
struct indexed_tile_set {
    const int32_t *ids;
    const int32_t *row_offsets;
    int64_t num_tiles;
    __device__ tile_ref tile(int64_t p) const {
        const int32_t t = ids[p];
        return {t, row_offsets[t], row_offsets[t + 1]};
    }
};

// ---------------------------------------------------------------- schedules (Sec. 4.2)

// Thread-mapped (Sec. 4.2 listing): tile position p goes to global thread p and the
// threads stride by the grid; a thread walks its tile's atoms in order.
template <class TS>
struct thread_mapped {
    TS ts;
    __device__ step_range tiles() const { return grid_stride_range(0, ts.num_tiles); }
    __device__ step_range atoms(const tile_ref &t) const { return {t.begin, t.end, 1}; }
    __device__ step_range atoms(int64_t p) const { return atoms(ts.tile(p)); }
};
using thread_mapped_schedule = thread_mapped<csr_tile_set>;

template <int G>
struct group_block {
    static_assert(G >= 1 && G <= 1024 && (G & (G - 1)) == 0, "group size: a power of two in [1, 1024]");
    static constexpr int BLOCK = G > kWave ? G : 256;
    static constexpr int GPB = BLOCK / G;  // groups per block
};

// Group-mapped with one tile per group (Sec. 5.2.2, warp- and block-level;
// K = 1): groups take
// tiles in a grid stride; lane l of a group takes atoms begin + l,
// begin + l + G, ...
template <int G, class TS>
struct group_mapped {
    static constexpr int BLOCK = group_block<G>::BLOCK;
    static constexpr int GPB = group_block<G>::GPB;
    TS ts;
    __device__ int lane() const { return threadIdx.x & (G - 1); }
    __device__ step_range tiles() const {
        return {static_cast<int64_t>(blockIdx.x) * GPB + threadIdx.x / G, ts.num_tiles,
                static_cast<int64_t>(gridDim.x) * GPB};
    }
    __device__ step_range atoms(const tile_ref &t) const { return {t.begin + lane(), t.end, G}; }
};

// Group-mapped with G tiles per group (Sec. 5.2.3, K = G).  Rounds are
// uniform across the block: in round r the g-th group of block b takes the
// chunk of G consecutive tile positions r + g (chunks past the end are
// empty).  load() and done() contain block barriers, so every thread of the
// block calls them, in every round.
template <int G, class TS>
struct group_mapped_scan {
    static constexpr int BLOCK = group_block<G>::BLOCK;
    static constexpr int GPB = group_block<G>::GPB;
    struct storage {
        int32_t scan[G + 1];  // exclusive prefix sums of the chunk's atom counts
        int32_t first[G];     // first atom of each tile of the chunk
        int32_t id[G];        // tile ids of the chunk
        int32_t wave[G > kWave ? G / kWave : 1];
    };
    TS ts;
    storage *st;  // this group's storage

    __device__ group_mapped_scan(const TS &tiles, storage *block_storage)
        : ts(tiles), st(block_storage + threadIdx.x / G) {}

    __device__ int lane() const { return threadIdx.x & (G - 1); }

    __device__ step_range rounds() const {
        const int64_t chunks = (ts.num_tiles + G - 1) / G;
        return {static_cast<int64_t>(blockIdx.x) * GPB, chunks, static_cast<int64_t>(gridDim.x) * GPB};
    }

    // The same rounds handed out by a work queue (a persistent grid claims
    // them at run time; `ticket` must be 0 at launch, s_slot one int of LDS).
    // batch: rounds of GPB chunks per claim.
    __device__ queue_rounds queued_rounds(int32_t *ticket, int32_t *s_slot, int64_t batch = 1) const {
        return {ticket, s_slot, GPB, (ts.num_tiles + G - 1) / G, batch < 1 ? 1 : batch};
    }

    // Loads the group's chunk for this round and returns its atom count.
    __device__ int32_t load(int64_t round) {
        const int64_t p = (round + threadIdx.x / G) * G + lane();
        tile_ref t{0, 0, 0};
        if (p < ts.num_tiles) t = ts.tile(p);
        int32_t inc;
        if constexpr (G <= kWave)
            inc = group_scan_incl<G>(t.end - t.begin);
        else
            inc = block_scan_incl<G>(t.end - t.begin, st->wave);
        st->scan[lane() + 1] = inc;
        if (lane() == 0) st->scan[0] = 0;
        st->first[lane()] = t.begin;
        st->id[lane()] = t.id;
        __syncthreads();
        return st->scan[G];
    }

    // Flattened atom positions [0, total) of the chunk, strided by G.
    __device__ step_range atoms(int32_t total) const { return {lane(), total, G}; }
    // Chunk slot of the tile owning flattened atom a.
    __device__ int32_t get_tile(int32_t a) const { return lb::get_tile<G>(st->scan, a); }
    __device__ int32_t tile(int32_t q) const { return st->id[q]; }
    // Atom id of flattened atom a, which slot q owns.
    __device__ int32_t atom(int32_t a, int32_t q) const { return st->first[q] + (a - st->scan[q]); }
    // Ends the round: storage may be overwritten by the next load.
    __device__ void done() const { __syncthreads(); }
};

}  // namespace lb
