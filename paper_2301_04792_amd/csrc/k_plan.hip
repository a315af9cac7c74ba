// Planned SpMV: short rows on the merge path, long rows on LDS panels of x.
//
// The merge path (Sec. 5.2.1) balances rows and nonzeros, but every nonzero
// still gathers x[col] through the cache hierarchy.  With scattered columns
// over a large x that gather, not HBM, bounds the kernel.  A plan built once
// per pattern moves the long rows (at least long_min nonzeros) to a second
// schedule in which x is read from LDS:
//
//  * x is cut into panels of P columns.  With sorted columns, the nonzeros
//    of long row q that fall in panel p are one contiguous segment of the
//    row.
//  * R blocks serve each panel: a block stages its panel of x in LDS once
//    and consumes an equal share of the panel's segments.
//  * The plan cuts each segment into tasks of at most kPanelTask nonzeros
//    and lists each panel's tasks by class: a task spanning at most G
//    aligned groups of four nonzeros (G = 64, 32, 16 or 8) is served by a
//    group of G lanes, one group of four per lane (the group-mapped
//    schedule, Sec. 5.2.2, with the group size matched to the tile), so a
//    wavefront step serves 64 / G tasks and a task's sum is a log2(G)-step
//    reduction.  A lane loads its four nonzeros with one 16-byte column load
//    and one value load, reads x from LDS, and the group's last lane stores
//    the task's sum (a DPP reduction).
//  * The short rows' merge-path blocks own whole rows (a block adds the head
//    of its first row and leaves its open row to the unit where it closes),
//    so they leave no carries.
//  * plan_combine sums, for every long row, its task sums in (panel, task)
//    order, and with two column bands adds each short row's second band.
//    With one band and no long rows the consume is the whole call.
// No atomics anywhere: the result is bit-reproducible for a fixed plan.
#include <algorithm>
#include <mutex>

#include "lb_device.h"
#include "lb_internal.h"

namespace lbk {
using namespace lb;

// ------------------------------------------------------------------ panel consume

// The tasks [T0, T1) of class G: wavefront w serves tasks w * TPW + i * NW *
// TPW + lane / G (TPW = 64 / G tasks per step; w rotated by `rot`, so the
// wavefronts that get a last partial round differ from class to class),
// kPanelBatch steps at a time with every load of them issued before the first
// wait.
// VEC = 4: lane l of a group loads the aligned group of four nonzeros
// a0 / 4 + l; lanes past the task's last group reload it (no extra cache
// lines).  Needs nnz >= 4 and col_idx / values aligned to their vectors; the
// array's last nnz mod 4 nonzeros, outside every full group, are loaded one
// by one by the task that holds them.  VEC = 1: lane l of a group loads
// nonzeros l, l + G, l + 2G, l + 3G of the task.
template <int G, int VEC, typename VT, typename XT>
__device__ __forceinline__ void panel_class_tasks(int32_t T0, int32_t T1, int rot, const panel_task *__restrict__ tasks,
                                                  int32_t nnz, int32_t col0, const int32_t *__restrict__ ci,
                                                  const VT *__restrict__ val, const XT *xs, float *__restrict__ part) {
    constexpr int NW = kPanelBlock / kWave;
    constexpr int TPW = kWave / G;
    constexpr int S = kPanelBatch;
    const int lane = lane_id(), w = (wave_id() + rot) % NW;
    const int gl = lane & (G - 1);
    const int32_t last_full = (nnz >> 2) - 1;  // VEC 4: the last group of four inside the array
    int32_t base = T0 + w * TPW + lane / G;
    if (base - lane / G >= T1) return;
    // descriptors of the current batch; the next batch's are loaded while
    // this one's nonzeros are in flight
    int32_t a0[S], len[S], out[S];
    auto load_desc = [&](int32_t b, int32_t *da0, int32_t *dlen, int32_t *dout) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int32_t t = b + s * NW * TPW;
            const panel_task d = tasks[t < T1 ? t : T0];  // a dead slot reads the first task and stores nothing
            da0[s] = d.a0;
            dlen[s] = t < T1 ? d.len : 0;
            dout[s] = d.out;
        }
    };
    load_desc(base, a0, len, out);
    for (;;) {
        int32_t cc[S][4];
        VT vv[S][4];
        if constexpr (VEC == 4) {
            using vec_t = typename vec4_of<VT>::type;
            typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
            bool tail = false;  // some task reaches the nonzeros past the last full group
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int32_t glast = (a0[s] + (len[s] > 0 ? len[s] : 1) - 1) >> 2;
                int32_t g = (a0[s] >> 2) + gl;
                g = g < glast ? g : glast;
                g = g < last_full ? g : last_full;
                const i32x4 c4 = ld_stream(reinterpret_cast<const i32x4 *>(ci) + g);
                const vec_t v4 = ld_stream(reinterpret_cast<const vec_t *>(val) + g);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    cc[s][e] = c4[e];
                    vv[s][e] = v4[e];
                }
                tail = tail || (len[s] > 0 && glast > last_full);
            }
            if (__builtin_expect(__ballot(tail) != 0, 0)) {  // at most one task per launch
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const int32_t g = (a0[s] >> 2) + gl;
                    if (len[s] > 0 && g > last_full) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int32_t j = 4 * g + e < nnz ? 4 * g + e : nnz - 1;
                            cc[s][e] = ci[j];
                            vv[s][e] = val[j];
                        }
                    }
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int32_t last = len[s] > 0 ? len[s] - 1 : 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int32_t a = gl + u * G;
                    const int32_t j = a0[s] + (a < last ? a : last);
                    cc[s][u] = ld_stream(ci + j);
                    vv[s][u] = ld_stream(val + j);
                }
            }
        }
        const int32_t nbase = base + NW * TPW * S;
        const bool more = nbase - lane / G < T1;  // uniform over the wavefront
        int32_t na0[S], nlen[S], nout[S];
        if (more) load_desc(nbase, na0, nlen, nout);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            // the task-relative index of this lane's u-th nonzero
            const int32_t a_base = VEC == 4 ? 4 * ((a0[s] >> 2) + gl) - a0[s] : gl;
            float acc = 0.f;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t a = a_base + (VEC == 4 ? u : u * G);
                const bool live = a >= 0 && a < len[s];
                const int32_t xi = live ? cc[s][u] - col0 : 0;
                const float xv = to_f32(xs[xi]);
                acc += live ? to_f32(vv[s][u]) * xv : 0.f;
            }
            acc = group_sum_dpp<G>(acc);
            if (gl == G - 1 && len[s] > 0) part[out[s]] = acc;
        }
        if (!more) break;
        base = nbase;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            a0[s] = na0[s];
            len[s] = nlen[s];
            out[s] = nout[s];
        }
    }
}

// Block b serves panel p = b mod NP, share r = b / NP of R: the r-th of R
// equal slices of each of the panel's class lists.
template <typename VT, typename XT, int VEC>
__global__ __launch_bounds__(kPanelBlock) void panel_spmv(int32_t NP, int32_t R, int32_t P, int32_t cols, int32_t nnz,
                                                          const int32_t *__restrict__ pcls_off,
                                                          const panel_task *__restrict__ tasks,
                                                          const int32_t *__restrict__ ci,
                                                          const VT *__restrict__ val, const XT *__restrict__ x,
                                                          float *__restrict__ part) {
    constexpr int PMAX = kPanelBytes / static_cast<int>(sizeof(XT));
    static_assert(kPanelClasses == 4 && kPanelTask <= 4 * kWave - 3, "a task spans at most 64 groups of 4");
    __shared__ XT xs[PMAX];

    const int p = static_cast<int>(blockIdx.x % NP);
    const int r = static_cast<int>(blockIdx.x / NP);  // < R: the grid is NP * R blocks
    const int tid = threadIdx.x;
    const int32_t col0 = p * P;
    const int32_t ncol = P < cols - col0 ? P : cols - col0;
    const int32_t *off = pcls_off + static_cast<int64_t>(p) * kPanelClasses;  // classes 0..3 and the next panel's start
    int32_t lo[kPanelClasses + 1];
#pragma unroll
    for (int k = 0; k < kPanelClasses; ++k) {
        const int64_t n = off[k + 1] - off[k];
        lo[k] = off[k] + static_cast<int32_t>(n * r / R);
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
    __syncthreads();
    auto hi = [&](int k) { return off[k] + static_cast<int32_t>((static_cast<int64_t>(off[k + 1]) - off[k]) * (r + 1) / R); };
    panel_class_tasks<64, VEC>(lo[0], hi(0), 0, tasks, nnz, col0, ci, val, xs, part);
    panel_class_tasks<32, VEC>(lo[1], hi(1), 2, tasks, nnz, col0, ci, val, xs, part);
    panel_class_tasks<16, VEC>(lo[2], hi(2), 4, tasks, nnz, col0, ci, val, xs, part);
    panel_class_tasks<8, VEC>(lo[3], hi(3), 6, tasks, nnz, col0, ci, val, xs, part);
}

// ------------------------------------------------------------------ combine

// After the consume and the panel launch.  Two bands: every short row adds
// its second band's sum (y += y_hi; long rows, flagged in long_bits, are
// skipped), blocks [0, EB), four rows per thread with 16-byte accesses when
// y and y_hi are 16-byte aligned.  Every long row gets the sum
// of its task sums in (panel, task) order (lanes stride, then a fixed
// butterfly), one wavefront per long row in the blocks after EB.  Each row
// has one writer.
__global__ __launch_bounds__(256) void plan_combine(int32_t rows, int32_t EB, int32_t NL,
                                                    const uint32_t *__restrict__ long_bits, float *__restrict__ y,
                                                    const float *__restrict__ y_hi, const int32_t *__restrict__ LR,
                                                    const int32_t *__restrict__ row_task,
                                                    const float *__restrict__ part) {
    if (static_cast<int32_t>(blockIdx.x) < EB) {
        typedef float f32x4 __attribute__((ext_vector_type(4)));
        const bool vec = ((reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(y_hi)) & 15) == 0;
        const int64_t quads = vec ? rows / 4 : 0;  // rows [0, 4 * quads) four at a time
        for (int64_t g = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; g < quads;
             g += static_cast<int64_t>(EB) * 256) {
            const f32x4 a = reinterpret_cast<const f32x4 *>(y)[g];
            const f32x4 h = reinterpret_cast<const f32x4 *>(y_hi)[g];
            const uint32_t lb = (long_bits[g >> 3] >> ((g & 7) * 4)) & 15u;  // rows 4g .. 4g + 3
            if (lb == 0) {
                reinterpret_cast<f32x4 *>(y)[g] = a + h;
            } else {  // a long row's y is the long-row pass's: store the short ones only
                for (int e = 0; e < 4; ++e)
                    if (((lb >> e) & 1u) == 0) y[4 * g + e] = a[e] + h[e];
            }
        }
        for (int64_t r = 4 * quads + static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; r < rows;
             r += static_cast<int64_t>(EB) * 256) {
            const float a = y[r], h = y_hi[r];  // loaded whatever the flag: no dependent wait
            if (((long_bits[r >> 5] >> (r & 31)) & 1u) == 0) y[r] = a + h;
        }
        return;
    }
    const int64_t q = static_cast<int64_t>(blockIdx.x - EB) * 4 + wave_id();
    if (q >= NL) return;  // uniform across the wavefront
    const int lane = lane_id();
    const int32_t t0 = row_task[q], t1 = row_task[q + 1];
    constexpr int U = 8;  // loads in flight per lane
    float s = 0.f;
    for (int32_t t = t0 + lane; t < t1; t += U * kWave) {
        float v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = t + k * kWave < t1 ? part[t + k * kWave] : 0.f;
#pragma unroll
        for (int k = 0; k < U; ++k) s += v[k];  // the lane's sums in task order
    }
    s = group_sum<kWave>(s);
    if (lane == 0) y[LR[q]] = s;
}

// ------------------------------------------------------------------ plan building

// sb[q][p] for p in [0, NP): the first nonzero of long row LR[q] whose column
// is at least p * P (lower bound in the row's sorted columns); sb[q][NP] =
// the row's end.  One thread per (row, panel) pair.
__global__ __launch_bounds__(256) void plan_segments(int32_t NL, int32_t NP, int32_t P,
                                                     const int32_t *__restrict__ LR, const int32_t *__restrict__ ro,
                                                     const int32_t *__restrict__ ci, int32_t *__restrict__ sb) {
    const int64_t stride = static_cast<int64_t>(NP) + 1;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < NL * stride;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t q = e / stride;
        const int32_t p = static_cast<int32_t>(e - q * stride);
        const int32_t r = LR[q];
        const int32_t b = ro[r], en = ro[r + 1];
        if (p == NP) {
            sb[e] = en;
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

// Flags (bit 0) a long row whose columns do not strictly increase: block q
// (grid stride) checks the consecutive pairs of row LR[q], strided by its
// threads.
__global__ __launch_bounds__(256) void plan_order_check(int32_t NL, const int32_t *__restrict__ LR,
                                                        const int32_t *__restrict__ ro,
                                                        const int32_t *__restrict__ ci, int32_t *__restrict__ flags) {
    for (int32_t q = blockIdx.x; q < NL; q += gridDim.x) {
        const int32_t r = LR[q];
        const int32_t b = ro[r], en = ro[r + 1];
        bool bad = false;
        for (int32_t j = b + 1 + static_cast<int32_t>(threadIdx.x); j < en; j += blockDim.x)
            bad = bad || ci[j] <= ci[j - 1];
        if (bad) atomicOr(flags, 1);
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
                       sb);
    hipLaunchKernelGGL(plan_order_check, dim3(static_cast<uint32_t>(NL < 65536 ? NL : 65536)), dim3(256), 0, s, NL, LR,
                       ro, ci, flags);
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

// Four nonzeros per lane and load need nnz >= 4 and col_idx / values aligned
// to their vectors (16 bytes; BF16 values 8).
static bool panel_vec4_ok(const csr_dev &A) {
    const uintptr_t va = A.dt == LB_BF16 ? 8 : 16;
    return A.nnz >= 4 && reinterpret_cast<uintptr_t>(A.ci) % 16 == 0 && reinterpret_cast<uintptr_t>(A.val) % va == 0;
}

template <typename T>
static hipError_t launch_panel_t(const csr_dev &A, const plan_dev &pl, const void *x, float *part, hipStream_t s) {
    const dim3 grid(static_cast<uint32_t>(static_cast<int64_t>(pl.NP) * pl.R));
    const T *val = static_cast<const T *>(A.val);
    const T *xx = static_cast<const T *>(x);
    if (panel_vec4_ok(A))
        hipLaunchKernelGGL((panel_spmv<T, T, 4>), grid, dim3(kPanelBlock), 0, s, pl.NP, pl.R, pl.P, A.cols, A.nnz,
                           pl.pcls_off, pl.tasks, A.ci, val, xx, part);
    else
        hipLaunchKernelGGL((panel_spmv<T, T, 1>), grid, dim3(kPanelBlock), 0, s, pl.NP, pl.R, pl.P, A.cols, A.nnz,
                           pl.pcls_off, pl.tasks, A.ci, val, xx, part);
    return hipGetLastError();
}

static hipError_t launch_panel(const csr_dev &A, const plan_dev &pl, const void *x, float *part, hipStream_t s) {
    prof_scope pr(s, "panel_consume");
    if (A.dt == LB_BF16) return launch_panel_t<bf16_bits>(A, pl, x, part, s);
    return launch_panel_t<float>(A, pl, x, part, s);
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
        if ((e = merge_spmv_planned_consume(A, pl, x, y, w.y_hi, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, ss->join, 0)) != hipSuccess) return e;
    } else {
        if (pl.NL > 0 && (e = launch_panel(A, pl, x, w.part, s)) != hipSuccess) return e;
        if (pl.NA > 0 && (e = merge_spmv_planned_consume(A, pl, x, y, w.y_hi, s)) != hipSuccess)
            return e;
    }
    prof_scope pr(s, "plan_finish");
    const int64_t eb = pl.bands == 2 ? std::min<int64_t>((static_cast<int64_t>(pl.rows) / 4 + 255) / 256 + 1, 4096) : 0;
    const int64_t blocks = eb + (static_cast<int64_t>(pl.NL) + 3) / 4;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(plan_combine, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, pl.rows,
                       static_cast<int32_t>(eb), pl.NL, pl.long_bits, y, w.y_hi, pl.LR, pl.row_task, w.part);
    return hipGetLastError();
}

}  // namespace lbk
