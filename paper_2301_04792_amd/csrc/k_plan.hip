// Planned SpMV: short rows on the merge path, long rows on LDS panels of x.
//
// The merge path (Sec. 5.2.1) balances rows and nonzeros, but every nonzero
// still gathers x[col] through the cache hierarchy.  With scattered columns
// over a large x that gather, not HBM, bounds the kernel.  A plan built once
// per pattern moves the long rows (at least long_min nonzeros) to a second
// schedule in which x is read from LDS:
//
//  * x is cut into panels of P columns.  With sorted columns, the nonzeros
//    of long row q that fall in panel p are one contiguous segment
//    [sb[q][p], sb[q][p+1]) of the row.
//  * The long rows are grouped into chunks (consecutive long rows, about
//    16K nonzeros per panel on average).  Block (chunk c, panel p) stages
//    panel p of x in LDS and consumes the chunk's segments in panel p.
//  * Each segment is cut into tasks of at most kPanelTask nonzeros (the
//    plan's table tb holds each (row, panel) pair's first task, row-major,
//    so a row's tasks are consecutive).  The block prefix-sums its segments'
//    task counts in LDS; wavefront w takes tasks w, w + NW, ... and finds a
//    task's segment by binary search in that prefix sum: the group-mapped
//    schedule with get_tile (Sec. 5.2.3) over (row, panel) tiles whose
//    atoms are tasks.  A task's lanes load its nonzeros coalesced, read x
//    from LDS, and one wave sum (fixed order) is stored as the task's sum.
//  * Blocks are dealt to the 8 XCDs round robin; panel p goes to XCD p mod 8
//    (blocks of one chunk are consecutive), so an XCD's L2 only ever holds
//    its eighth of x while it stages panels.
//  * plan_finish adds, for every long row, its task sums in (panel, task)
//    order, and completes the short rows cut by unit boundaries (the carries
//    of the merge path and the second column band's sums).
// No atomics anywhere: the result is bit-reproducible for a fixed plan.
#include <mutex>

#include "lb_device.h"
#include "lb_internal.h"

namespace lbk {
using namespace lb;

// ------------------------------------------------------------------ panel consume

template <typename VT, typename XT>
__global__ __launch_bounds__(kPanelBlock) void panel_spmv(int32_t NP, int32_t NC, int32_t P, int32_t cols,
                                                          const int32_t *__restrict__ chunk_q,
                                                          const int32_t *__restrict__ sb,
                                                          const int32_t *__restrict__ tb,
                                                          const int32_t *__restrict__ ci,
                                                          const VT *__restrict__ val, const XT *__restrict__ x,
                                                          float *__restrict__ part) {
    constexpr int PMAX = kPanelBytes / static_cast<int>(sizeof(XT));
    constexpr int NW = kPanelBlock / kWave;
    constexpr int U = kPanelTask / kWave;  // loads per lane and task
    constexpr int S = kPanelBatch;         // tasks per wavefront and iteration
    static_assert(kPanelRows == kPanelBlock, "one chunk row per thread in the setup");
    static_assert(S <= kWave, "one search lane per task of a batch");
    __shared__ XT xs[PMAX];
    __shared__ int32_t s_scan[kPanelRows + 1];  // exclusive prefix of the rows' task counts
    __shared__ int32_t s_beg[kPanelRows];       // segment of each chunk row in this panel
    __shared__ int32_t s_end[kPanelRows];
    __shared__ int32_t s_out[kPanelRows];       // first task (output slot) of each row in this panel
    __shared__ int32_t s_wave[NW];

    const int PG = (NP + kXcds - 1) / kXcds;  // panel groups: one panel per XCD each
    const int xcd = static_cast<int>(blockIdx.x % kXcds);
    const int sq = static_cast<int>(blockIdx.x / kXcds);
    const int c = sq / PG;
    const int p = kXcds * (sq % PG) + xcd;
    if (c >= NC || p >= NP) return;  // uniform across the block, before any barrier
    const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
    const int32_t col0 = p * P;
    const int32_t ncol = P < cols - col0 ? P : cols - col0;

    // The chunk's rows in this panel: segment, task count, first task.
    const int32_t q0 = chunk_q[c];
    const int32_t nq = chunk_q[c + 1] - q0;  // in [1, kPanelRows] (the plan's chunks)
    const int64_t stride = static_cast<int64_t>(NP) + 1;
    int32_t cnt = 0;
    if (tid < nq) {
        const int64_t e = (q0 + tid) * stride + p;
        const int32_t b = sb[e], en = sb[e + 1], t0 = tb[e], t1 = tb[e + 1];
        s_beg[tid] = b;
        s_end[tid] = en;
        s_out[tid] = t0;
        cnt = t1 - t0;
    }

    // Stage the panel: 16-byte loads when the slice is 16-byte aligned, all
    // of a thread's loads issued before its LDS stores.
    {
        const char *src = reinterpret_cast<const char *>(x + col0);
        char *dst = reinterpret_cast<char *>(xs);
        const int32_t nbytes = ncol * static_cast<int32_t>(sizeof(XT));
        int32_t done = 0;
        if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            constexpr int R = kPanelBytes / 16 / kPanelBlock;
            const int32_t n16 = nbytes >> 4;
            u32x4 r[R];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int32_t i = tid + k * kPanelBlock;
                r[k] = reinterpret_cast<const u32x4 *>(src)[i < n16 ? i : 0];
            }
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int32_t i = tid + k * kPanelBlock;
                if (i < n16) reinterpret_cast<u32x4 *>(dst)[i] = r[k];
            }
            done = (n16 * 16) / static_cast<int32_t>(sizeof(XT));
        }
        for (int32_t i = done + tid; i < ncol; i += kPanelBlock) xs[i] = x[col0 + i];
    }
    const int32_t inc = block_scan_incl<kPanelBlock>(cnt, s_wave);
    if (tid < nq) s_scan[tid] = inc - cnt;
    if (tid == kPanelBlock - 1) s_scan[nq] = inc;  // the last thread's inclusive sum is the total
    __syncthreads();
    const int32_t NT = s_scan[nq];

    // Wavefront w takes tasks w, w + NW, ...; S of them per iteration, with
    // every load of the S tasks issued before the first wait.
    for (int32_t base = w; base < NT; base += NW * S) {
        // lane s < S finds the row of task base + s * NW (the last k < nq with
        // s_scan[k] <= t: exact for a live task, as s_scan[nq] = NT > t, and
        // in range for a dead one); the S searches run side by side
        int32_t my_k = 0;
        {
            const int32_t t = base + (lane < S ? lane : 0) * NW;
            int32_t lo = 0, hi = nq;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (s_scan[mid] <= t)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            my_k = lo - 1;
        }
        int32_t a0[S], len[S], out[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int32_t t = base + s * NW;
            const int32_t k = __shfl(my_k, s);
            const int32_t sub = t - s_scan[k];
            a0[s] = s_beg[k] + sub * kPanelTask;
            const int32_t rest = s_end[k] - a0[s];
            len[s] = t < NT ? (rest < kPanelTask ? rest : kPanelTask) : 0;  // >= 1 for a live task
            out[s] = s_out[k] + sub;
            if (t >= NT) a0[s] = a0[0];  // a dead slot reloads the first task's first nonzero
        }
        int32_t cc[S][U];
        VT vv[S][U];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int32_t last = len[s] > 0 ? len[s] - 1 : 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t a = lane + u * kWave;
                const int32_t j = a0[s] + (a < last ? a : last);
                cc[s][u] = ld_stream(ci + j);
                vv[s][u] = ld_stream(val + j);
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            float acc = 0.f;
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (lane + u * kWave < len[s]) acc += to_f32(vv[s][u]) * to_f32(xs[cc[s][u] - col0]);
            acc = group_sum<kWave>(acc);
            if (lane == 0 && len[s] > 0) part[out[s]] = acc;
        }
    }
}

// ------------------------------------------------------------------ finish

// One wavefront per item: items [0, NA) are the active merge-path units,
// items [NA, NA + NL) the long rows.
//  * Unit v (active): the rows that close in it, [i0, i1), are short except
//    possibly i0.  A short i0 gets the carries of the units before v that
//    ended inside it (the run of units u < v with part_i[u + 1] == i0, every
//    one of them active, read backwards 64 carries at a time); with two
//    bands every closing short row also gets the second band's sum.
//  * Long row q: y[LR[q]] = sum of its task sums, in order (lanes stride,
//    then a fixed butterfly).
// Each row has exactly one writer.
template <int BANDS>
__global__ __launch_bounds__(256) void plan_finish(int32_t NA, int32_t NL, const int32_t *__restrict__ active,
                                                   const int32_t *__restrict__ part_i,
                                                   const int32_t *__restrict__ ro, int32_t long_min,
                                                   const float *__restrict__ carry_val, float *__restrict__ y,
                                                   const float *__restrict__ y_hi, const int32_t *__restrict__ LR,
                                                   const int32_t *__restrict__ tb, int32_t NP,
                                                   const float *__restrict__ part) {
    const int lane = lane_id();
    const int64_t item = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
    if (item >= static_cast<int64_t>(NA) + NL) return;  // uniform across the wavefront
    if (item >= NA) {
        const int64_t q = item - NA;
        const int64_t stride = static_cast<int64_t>(NP) + 1;
        const int32_t t0 = tb[q * stride], t1 = tb[q * stride + NP];
        float s = 0.f;
        for (int32_t t = t0 + lane; t < t1; t += kWave) s += part[t];
        s = group_sum<kWave>(s);
        if (lane == 0) y[LR[q]] = s;
        return;
    }
    const int32_t v = active[item];
    const int32_t i0 = part_i[v], i1 = part_i[v + 1];
    if (i0 >= i1) return;  // no row closes in this unit
    const bool long0 = ro[i0 + 1] - ro[i0] >= long_min;
    const int32_t r0 = i0 + lane;
    float first = 0.f;
    if (r0 < i1) first = BANDS == 2 ? y[r0] + y_hi[r0] : y[r0];
    float carried = 0.f;
    if (!long0) {
        for (int64_t hi = static_cast<int64_t>(v) * BANDS;; hi -= kWave) {  // carries [0, BANDS v) precede v
            const int64_t q = hi - 1 - lane;
            const bool match = q >= 0 && part_i[q / BANDS + 1] == i0;
            carried += group_sum<kWave>(match ? carry_val[q] : 0.f);
            if (__popcll(__ballot(match)) < kWave) break;  // the run started inside this chunk
        }
    }
    if (r0 < i1 && !(lane == 0 && long0)) {
        if (lane == 0)
            y[r0] = first + carried;
        else if (BANDS == 2)
            y[r0] = first;
    }
    if (BANDS == 2)
        for (int32_t r = r0 + kWave; r < i1; r += kWave) y[r] = y[r] + y_hi[r];
}

// ------------------------------------------------------------------ plan building

// sb[q][p] for p in [0, NP): the first nonzero of long row LR[q] whose column
// is at least p * P (lower bound in the row's sorted columns); sb[q][NP] =
// the row's end.  Also flags (bit 0) a long row whose columns do not
// strictly increase.  One thread per (row, panel) pair; thread (q, NP) checks
// the order.
__global__ __launch_bounds__(256) void plan_segments(int32_t NL, int32_t NP, int32_t P,
                                                     const int32_t *__restrict__ LR, const int32_t *__restrict__ ro,
                                                     const int32_t *__restrict__ ci, int32_t *__restrict__ sb,
                                                     int32_t *__restrict__ flags) {
    const int64_t stride = static_cast<int64_t>(NP) + 1;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < NL * stride;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t q = e / stride;
        const int32_t p = static_cast<int32_t>(e - q * stride);
        const int32_t r = LR[q];
        const int32_t b = ro[r], en = ro[r + 1];
        if (p == NP) {
            sb[e] = en;
            bool bad = false;
            for (int32_t j = b + 1; j < en && !bad; ++j) bad = ci[j] <= ci[j - 1];
            if (bad) atomicOr(flags, 1);
            continue;
        }
        const int32_t key = p * P;
        int32_t lo = b, hi = en;
        while (lo < hi) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            if (ci[mid] < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        sb[e] = lo;
    }
}

// ------------------------------------------------------------------ launchers

bool panel_cols_ok(int64_t P, lb_dtype_t xt) {
    const int64_t pmax = kPanelBytes / (xt == LB_BF16 ? 2 : 4);
    return P >= kWave && P <= pmax && P % kWave == 0;
}

hipError_t plan_segments_launch(int32_t NL, int32_t NP, int32_t P, const int32_t *LR, const int32_t *ro,
                                const int32_t *ci, int32_t *sb, int32_t *flags, hipStream_t s) {
    const int64_t n = static_cast<int64_t>(NL) * (NP + 1);
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(plan_segments, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, NL, NP, P, LR, ro, ci,
                       sb, flags);
    return hipGetLastError();
}

// The library's second stream on the device that runs `s`, with the two
// events that fork work onto it and join it back; created on first use.
struct side_stream {
    std::mutex mu;
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int kMaxSideDevices = 64;
static std::mutex g_side_mu;
static side_stream g_side[kMaxSideDevices];

static hipError_t side_for(hipStream_t s, side_stream **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (s) {
        hipDevice_t sd = 0;
        if ((e = hipStreamGetDevice(s, &sd)) != hipSuccess) return e;
        dev = static_cast<int>(sd);
    }
    if (dev < 0 || dev >= kMaxSideDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_side_mu);
    side_stream &ss = g_side[dev];
    if (!ss.s) {
        int cur = 0;
        if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        hipStream_t st = nullptr;
        hipEvent_t f = nullptr, j = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&f, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
        const hipError_t back = cur != dev ? hipSetDevice(cur) : hipSuccess;
        if (e != hipSuccess) return e;
        if (back != hipSuccess) return back;
        ss.s = st;
        ss.fork = f;
        ss.join = j;
    }
    *out = &ss;
    return hipSuccess;
}

static hipError_t launch_panel(const csr_dev &A, const plan_dev &pl, const void *x, float *part, hipStream_t s) {
    prof_scope pr(s, "panel_consume");
    const int64_t PG = (pl.NP + kXcds - 1) / kXcds;
    const int64_t grid = static_cast<int64_t>(kXcds) * PG * pl.NC;
    if (A.dt == LB_BF16)
        hipLaunchKernelGGL((panel_spmv<bf16_bits, bf16_bits>), dim3(static_cast<uint32_t>(grid)), dim3(kPanelBlock), 0,
                           s, pl.NP, pl.NC, pl.P, A.cols, pl.chunk_q, pl.sb, pl.tb, A.ci,
                           static_cast<const bf16_bits *>(A.val), static_cast<const bf16_bits *>(x), part);
    else
        hipLaunchKernelGGL((panel_spmv<float, float>), dim3(static_cast<uint32_t>(grid)), dim3(kPanelBlock), 0, s,
                           pl.NP, pl.NC, pl.P, A.cols, pl.chunk_q, pl.sb, pl.tb, A.ci,
                           static_cast<const float *>(A.val), static_cast<const float *>(x), part);
    return hipGetLastError();
}

hipError_t planned_spmv(const csr_dev &A, const plan_dev &pl, const void *x, float *y, void *ws, hipStream_t s) {
    const plan_ws w = plan_ws_carve(ws, pl);
    hipError_t e = hipSuccess;
    if (pl.NL > 0 && pl.NA > 0 && pl.streams == 2) {
        // long rows on the second stream, after the work already on s; short
        // rows on s meanwhile; s then waits for the long rows
        side_stream *ss = nullptr;
        if ((e = side_for(s, &ss)) != hipSuccess) return e;
        std::lock_guard<std::mutex> g(ss->mu);
        if ((e = hipEventRecord(ss->fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(ss->s, ss->fork, 0)) != hipSuccess) return e;
        if ((e = launch_panel(A, pl, x, w.part, ss->s)) != hipSuccess) return e;
        if ((e = hipEventRecord(ss->join, ss->s)) != hipSuccess) return e;
        if ((e = merge_spmv_planned_consume(A, pl, x, y, w.carry_val, w.y_hi, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, ss->join, 0)) != hipSuccess) return e;
    } else {
        if (pl.NL > 0 && (e = launch_panel(A, pl, x, w.part, s)) != hipSuccess) return e;
        if (pl.NA > 0 && (e = merge_spmv_planned_consume(A, pl, x, y, w.carry_val, w.y_hi, s)) != hipSuccess)
            return e;
    }
    const int64_t items = static_cast<int64_t>(pl.NA) + pl.NL;
    if (items == 0) return hipSuccess;
    prof_scope pr(s, "plan_finish");
    const int64_t blocks = (items + 3) / 4;  // a wavefront per item
    if (pl.bands == 2)
        hipLaunchKernelGGL(plan_finish<2>, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, pl.NA, pl.NL,
                           pl.active, pl.part_i, A.ro, pl.long_min, w.carry_val, y, w.y_hi, pl.LR, pl.tb, pl.NP,
                           w.part);
    else
        hipLaunchKernelGGL(plan_finish<1>, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, pl.NA, pl.NL,
                           pl.active, pl.part_i, A.ro, pl.long_min, w.carry_val, y, w.y_hi, pl.LR, pl.tb, pl.NP,
                           w.part);
    return hipGetLastError();
}

}  // namespace lbk
