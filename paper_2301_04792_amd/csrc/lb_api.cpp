// C ABI of the load-balanced sparse library: argument checks, schedule
// resolution (Sec. 6.2 heuristic, tuned picks), workspace sizing, dispatch
// to the kernel launchers, kernel timing and the autotuner.
//
// Every check that can be made on the host runs before the first HIP call,
// so invalid arguments never reach the device (and can be tested without a
// GPU).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "lb.h"
#include "lb_internal.h"

namespace {

constexpr int64_t kMaxCoord = 0x7ffffffe;  // rows + nnz must stay below this (int32 merge coordinates)
constexpr int kDefaultBlock = 256;
constexpr int kDefaultItems = 8;
constexpr int kLocalItems = 12;    // planned SpMV with local columns (four nonzeros per lane)
constexpr int kScatteredBlock = 128;  // planned SpMV with scattered columns
constexpr int kDefaultGroup = 64;
constexpr int kMaxK = 64;

thread_local std::string g_last_hip;

lb_status_t hip_status(hipError_t e) {
    if (e == hipSuccess) return LB_OK;
    g_last_hip = hipGetErrorString(e);
    return LB_ERR_HIP;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

bool dtype_built(lb_dtype_t d) { return d == LB_F32 || d == LB_BF16; }

lb_status_t check_csr(const lb_csr_t *A) {
    if (!A) return LB_ERR_INVALID_ARG;
    if (A->rows < 0 || A->cols < 0 || A->nnz < 0) return LB_ERR_INVALID_ARG;
    if (A->rows > 0 && !A->row_offsets) return LB_ERR_INVALID_ARG;
    if (A->nnz > 0 && (!A->col_idx || !A->values)) return LB_ERR_INVALID_ARG;
    if (A->nnz > 0 && A->cols == 0) return LB_ERR_INVALID_ARG;
    // offsets[0] = 0 and offsets[rows] = nnz: no rows means no nonzeros (this
    // also covers a COO without rows and a CSC without columns)
    if (A->nnz > 0 && A->rows == 0) return LB_ERR_INVALID_ARG;
    if (A->value_dtype != LB_F32 && A->value_dtype != LB_BF16 && A->value_dtype != LB_F64)
        return LB_ERR_INVALID_ARG;
    if (!dtype_built(A->value_dtype)) return LB_ERR_UNSUPPORTED;
    if (A->rows + A->nnz > kMaxCoord || A->cols > kMaxCoord) return LB_ERR_OVERFLOW;
    return LB_OK;
}

lbk::csr_dev to_dev(const lb_csr_t *A) {
    lbk::csr_dev d;
    d.rows = static_cast<int32_t>(A->rows);
    d.cols = static_cast<int32_t>(A->cols);
    d.nnz = static_cast<int32_t>(A->nnz);
    d.ro = A->row_offsets;
    d.ci = A->col_idx;
    d.val = A->values;
    d.dt = A->value_dtype;
    return d;
}

// ------------------------------------------------------------------ autotune cache

// A tuned pick is kept for a matrix shape, k, dtype, batched flag and a
// fingerprint of the sparsity pattern, on the device it was timed on (arch
// and CU count) and for this ABI version.  The fingerprint cannot be taken
// inside an asynchronous call (it reads the pattern), so LB_AUTO finds it
// through a binding: lb_autotune and lb_autotune_lookup bind the matrix's
// device arrays (pointers and shape) to its fingerprint.  A matrix without
// a binding gets the Sec. 6.2 rule.
struct tune_key {
    int64_t rows, cols, nnz;
    int32_t k;
    int32_t dtype;
    int32_t batched;
    uint64_t fp;
    bool operator<(const tune_key &o) const {
        return std::tie(rows, cols, nnz, k, dtype, batched, fp) <
               std::tie(o.rows, o.cols, o.nnz, o.k, o.dtype, o.batched, o.fp);
    }
};

struct bind_key {
    const void *ro, *ci;
    int64_t rows, cols, nnz;
    int32_t batched;
    bool operator<(const bind_key &o) const {
        return std::tie(ro, ci, rows, cols, nnz, batched) < std::tie(o.ro, o.ci, o.rows, o.cols, o.nnz, o.batched);
    }
};

std::mutex g_tune_mu;
std::map<tune_key, lb_schedule_t> g_tune;
std::map<bind_key, uint64_t> g_bind;
std::vector<std::string> g_tune_foreign;  // file lines of other devices or ABI versions, kept verbatim
bool g_tune_loaded = false;
std::string g_device_tag;

const char *tune_path() { return std::getenv("LB_AUTOTUNE_CACHE"); }

// "<arch>:<compute units>" of the current device, "none:0" without one.
std::string device_tag_now() {
    int dev = 0, n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0 || hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return "none:0";
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "none:0";
    }
    std::string arch(prop.gcnArchName);
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return arch + ":" + std::to_string(prop.multiProcessorCount);
}

const std::string &device_tag_locked() {
    if (g_device_tag.empty()) g_device_tag = device_tag_now();
    return g_device_tag;
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *p = tune_path();
    if (!p || !*p) return;
    std::ifstream f(p);
    std::string line;
    const std::string &tag = device_tag_locked();
    // one entry per line: lbtune abi device rows cols nnz k dtype batched fingerprint(hex)
    //                     kind group tiles items block grid x_bands vector_width
    while (std::getline(f, line)) {
        std::istringstream ss(line);
        std::string magic, dev;
        int abi = 0;
        if (!(ss >> magic >> abi >> dev) || magic != "lbtune") continue;  // not an entry: dropped
        if (abi != LB_ABI_VERSION || dev != tag) {
            g_tune_foreign.push_back(line);
            continue;
        }
        tune_key key{};
        lb_schedule_t s{};
        int kind = 0;
        if (ss >> key.rows >> key.cols >> key.nnz >> key.k >> key.dtype >> key.batched >> std::hex >> key.fp >>
            std::dec >> kind >> s.group_size >> s.tiles_per_group >> s.items_per_thread >> s.block_size >>
            s.grid_size >> s.x_bands >> s.vector_width) {
            s.kind = static_cast<lb_sched_kind_t>(kind);
            g_tune[key] = s;
        }
    }
}

void tune_save_locked() {
    const char *p = tune_path();
    if (!p || !*p) return;
    std::ofstream f(p, std::ios::trunc);
    for (const std::string &l : g_tune_foreign) f << l << '\n';
    const std::string &tag = device_tag_locked();
    for (const auto &kv : g_tune) {
        const tune_key &k = kv.first;
        const lb_schedule_t &s = kv.second;
        f << "lbtune " << LB_ABI_VERSION << ' ' << tag << ' ' << k.rows << ' ' << k.cols << ' ' << k.nnz << ' '
          << k.k << ' ' << k.dtype << ' ' << k.batched << ' ' << std::hex << k.fp << std::dec << ' '
          << static_cast<int>(s.kind) << ' ' << s.group_size << ' ' << s.tiles_per_group << ' '
          << s.items_per_thread << ' ' << s.block_size << ' ' << s.grid_size << ' ' << s.x_bands << ' '
          << s.vector_width << '\n';
    }
}

bool tune_lookup(const tune_key &key, lb_schedule_t *out) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const tune_key &key, const lb_schedule_t &s) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load_locked();
    g_tune[key] = s;
    tune_save_locked();
}

void tune_bind(const bind_key &b, uint64_t fp) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_bind[b] = fp;
}

// The tuned pick for a bound matrix (false when unbound or untuned).
bool tune_lookup_bound(const bind_key &b, const tune_key &shape, lb_schedule_t *out) {
    uint64_t fp = 0;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_bind.find(b);
        if (it == g_bind.end()) return false;
        fp = it->second;
    }
    tune_key key = shape;
    key.fp = fp;
    return tune_lookup(key, out);
}

// FNV-1a, 64 bit.
struct fnv64 {
    uint64_t h = 0xcbf29ce484222325ull;
    void add(const void *p, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 0x100000001b3ull;
        }
    }
    template <typename T>
    void add(const T &v) {
        add(&v, sizeof v);
    }
};

constexpr int32_t kFingerprintSamples = 4096;

// ------------------------------------------------------------------ schedule checks

lb_status_t fill_defaults(const lb_schedule_t *in, lb_schedule_t *out) {
    lb_schedule_t s = *in;
    if (s.group_size < 0 || s.tiles_per_group < 0 || s.items_per_thread < 0 || s.block_size < 0 || s.grid_size < 0)
        return LB_ERR_INVALID_ARG;
    if (s.x_bands < 0 || s.x_bands > 2) return LB_ERR_INVALID_ARG;
    if (s.x_bands == 0) s.x_bands = 1;
    if (s.x_bands == 2 && s.kind != LB_MERGE_PATH) return LB_ERR_UNSUPPORTED;
    if (s.vector_width == 0) s.vector_width = 1;
    if (s.vector_width != 1 && s.vector_width != 4) return LB_ERR_INVALID_ARG;
    if (s.vector_width == 4 && (s.kind != LB_MERGE_PATH || s.x_bands != 1)) return LB_ERR_UNSUPPORTED;
    switch (s.kind) {
        case LB_THREAD_MAPPED:
            if (s.block_size == 0) s.block_size = kDefaultBlock;
            if (s.block_size % 64 != 0 || s.block_size > 1024) return LB_ERR_INVALID_ARG;
            break;
        case LB_GROUP_MAPPED:
            if (s.group_size == 0) s.group_size = kDefaultGroup;
            if (!is_pow2(s.group_size) || s.group_size > 1024) return LB_ERR_INVALID_ARG;
            if (s.tiles_per_group == 0) s.tiles_per_group = 1;
            if (s.tiles_per_group != 1 && s.tiles_per_group != s.group_size) return LB_ERR_UNSUPPORTED;
            s.block_size = s.group_size > 64 ? s.group_size : 256;
            break;
        case LB_MERGE_PATH:
            if (s.block_size == 0) s.block_size = kDefaultBlock;
            if (s.items_per_thread == 0) s.items_per_thread = kDefaultItems;
            if (!lbk::merge_config_supported(s.block_size, s.items_per_thread)) return LB_ERR_UNSUPPORTED;
            if (s.vector_width == 4 && s.items_per_thread % 4 != 0) return LB_ERR_UNSUPPORTED;
            break;
        case LB_WORK_QUEUE:
            if (s.group_size == 0) s.group_size = kDefaultGroup;
            if (!is_pow2(s.group_size) || s.group_size > 1024) return LB_ERR_INVALID_ARG;
            if (s.tiles_per_group == 0) s.tiles_per_group = s.group_size;
            if (s.tiles_per_group != s.group_size) return LB_ERR_UNSUPPORTED;
            s.block_size = s.group_size > 64 ? s.group_size : 256;
            break;
        default:
            return LB_ERR_INVALID_ARG;
    }
    *out = s;
    return LB_OK;
}

// Sec. 6.2: merge-path unless (rows < alpha or cols < alpha) and nnz < beta.
lb_schedule_t heuristic(const lb_csr_t *A) {
    constexpr int64_t alpha = 500, beta = 10000;
    lb_schedule_t s{};
    if ((A->rows < alpha || A->cols < alpha) && A->nnz < beta) {
        const double mean = A->rows ? static_cast<double>(A->nnz) / static_cast<double>(A->rows) : 0.0;
        if (mean < 8.0) {
            s.kind = LB_THREAD_MAPPED;
        } else {
            int g = 1;
            while (g < mean && g < 64) g <<= 1;
            s.kind = LB_GROUP_MAPPED;
            s.group_size = g;
            s.tiles_per_group = 1;
        }
    } else {
        s.kind = LB_MERGE_PATH;
    }
    return s;
}

lb_status_t resolve(const lb_csr_t *A, int32_t k, const lb_schedule_t *in, lb_schedule_t *out) {
    if (!in || !out) return LB_ERR_INVALID_ARG;
    lb_schedule_t s = *in;
    if (s.kind == LB_AUTO) {
        lb_schedule_t tuned;
        const tune_key key{A->rows, A->cols, A->nnz, k, static_cast<int32_t>(A->value_dtype), 0, 0};
        const bind_key b{A->row_offsets, A->col_idx, A->rows, A->cols, A->nnz, 0};
        if (tune_lookup_bound(b, key, &tuned))
            s = tuned;
        else
            s = heuristic(A);
    }
    const lb_status_t st = fill_defaults(&s, out);
    if (st != LB_OK) return st;
    // column bands and vector loads: lb_spmv only
    if ((out->x_bands != 1 || out->vector_width != 1) && k != 1) return LB_ERR_UNSUPPORTED;
    if (out->kind == LB_MERGE_PATH && k == 1 && s.block_size == 0 && s.items_per_thread == 0 && out->x_bands == 1 &&
        out->vector_width == 1) {
        // Default units on a small matrix: the shortest unit (128 x 4, 256 x 4
        // or 256 x 8 items) that keeps the one-launch form (at most
        // kSelfSplitUnits units) spreads the matrix over the most CUs, each
        // block with less to load, sum and search before its first write.
        for (const auto &bi : {std::pair<int, int>{128, 4}, {256, 4}, {256, 8}}) {
            if (lbk::merge_units(A->rows, A->nnz, static_cast<int64_t>(bi.first) * bi.second) <= lbk::kSelfSplitUnits) {
                out->block_size = bi.first;
                out->items_per_thread = bi.second;
                break;
            }
        }
    }
    return LB_OK;
}

// Entry points other than lb_spmv take the plain merge-path consume only
// (one column band, one nonzero per lane and load).
lb_status_t one_band(const lb_schedule_t &s) {
    return s.x_bands == 1 && s.vector_width == 1 ? LB_OK : LB_ERR_UNSUPPORTED;
}

int spmm_pass_cols(int32_t k) { return k >= 8 ? 8 : (k >= 4 ? 4 : (k >= 2 ? 2 : 1)); }

size_t ws_bytes_for(const lb_csr_t *A, const lb_schedule_t &s, int32_t k) {
    if (s.kind == LB_WORK_QUEUE) return 256;  // the queue's counter
    if (s.kind != LB_MERGE_PATH) return 0;
    const int64_t W = static_cast<int64_t>(s.block_size) * s.items_per_thread;
    const int64_t T = lbk::merge_units(A->rows, A->nnz, W);
    if (s.x_bands == 2) return lbk::merge_banded_ws_bytes(T, A->rows);
    return lbk::merge_ws_bytes(T, k <= 0 ? 1 : spmm_pass_cols(k));
}

// ------------------------------------------------------------------ COO and CSC

lb_status_t check_coo(const lb_coo_t *A) {
    if (!A) return LB_ERR_INVALID_ARG;
    if (A->nnz > 0 && !A->row_idx) return LB_ERR_INVALID_ARG;
    // the CSR checks on the sizes, dtype and entry arrays; a COO has no offsets array
    static const int32_t no_offsets = 0;
    const lb_csr_t c{A->rows, A->cols, A->nnz, &no_offsets, A->col_idx, A->values, A->value_dtype};
    return check_csr(&c);
}

// The CSC checked as the CSR of its transpose (tiles are columns).
lb_status_t check_csc(const lb_csc_t *A, lb_csr_t *as_csr) {
    if (!A) return LB_ERR_INVALID_ARG;
    const lb_csr_t c{A->cols, A->rows, A->nnz, A->col_offsets, A->row_idx, A->values, A->value_dtype};
    lb_status_t st = check_csr(&c);
    if (st != LB_OK) return st;
    *as_csr = c;
    return LB_OK;
}

// Schedule of a COO product: LB_AUTO takes the Sec. 6.2 rule (groups of at least 8 lanes).
lb_status_t coo_schedule(const lb_coo_t *A, const lb_schedule_t *in, lb_schedule_t *out) {
    if (!in || !out) return LB_ERR_INVALID_ARG;
    lb_schedule_t s = *in;
    if (s.kind == LB_AUTO) {
        const lb_csr_t c{A->rows, A->cols, A->nnz, nullptr, nullptr, nullptr, A->value_dtype};
        s = heuristic(&c);
        if (s.kind == LB_GROUP_MAPPED && s.group_size < 8) s.group_size = 8;
    }
    lb_status_t st = fill_defaults(&s, out);
    if (st != LB_OK) return st;
    if (out->kind == LB_WORK_QUEUE || one_band(*out) != LB_OK) return LB_ERR_UNSUPPORTED;
    if (out->kind == LB_GROUP_MAPPED) {
        if (out->tiles_per_group != 1) return LB_ERR_UNSUPPORTED;
        if (!lbk::traversal_group_supported(out->group_size)) return LB_ERR_UNSUPPORTED;
    }
    return LB_OK;
}

lb_status_t csc_schedule(const lb_schedule_t *in, lb_schedule_t *out) {
    lb_schedule_t s = in ? *in : lb_schedule_t{LB_MERGE_PATH, 0, 0, 0, 0, 0};
    if (s.kind == LB_AUTO) s.kind = LB_MERGE_PATH;
    if (s.block_size == 0 && s.items_per_thread == 0) {  // larger units combine more rows per block
        s.block_size = 512;
        s.items_per_thread = 8;
    }
    if (s.kind != LB_MERGE_PATH) return LB_ERR_UNSUPPORTED;
    const lb_status_t st = fill_defaults(&s, out);
    return st != LB_OK ? st : one_band(*out);
}

// ------------------------------------------------------------------ graph traversal checks

// A graph is a square CSR; BFS reads no values, so they may be absent.
lb_status_t check_graph(const lb_csr_t *G, bool need_values) {
    if (!G) return LB_ERR_INVALID_ARG;
    lb_csr_t c = *G;
    if (!need_values && !c.values) {
        c.values = c.col_idx;  // placeholder so the CSR checks pass; never read
        c.value_dtype = LB_F32;
    }
    lb_status_t st = check_csr(&c);
    if (st != LB_OK) return st;
    if (G->rows != G->cols || G->rows == 0) return LB_ERR_INVALID_ARG;
    if (need_values && G->value_dtype != LB_F32) return LB_ERR_UNSUPPORTED;
    return LB_OK;
}

lb_status_t traversal_cfg(const lb_csr_t *G, const lb_schedule_t *in, lbk::trav_cfg *out) {
    lb_schedule_t s = in ? *in : lb_schedule_t{LB_AUTO, 0, 0, 0, 0, 0};
    if (s.group_size < 0 || s.tiles_per_group < 0 || s.items_per_thread < 0 || s.block_size < 0 || s.grid_size < 0)
        return LB_ERR_INVALID_ARG;
    if (s.x_bands < 0 || s.x_bands > 2) return LB_ERR_INVALID_ARG;
    if (s.vector_width != 0 && s.vector_width != 1 && s.vector_width != 4) return LB_ERR_INVALID_ARG;
    if (s.x_bands > 1 || s.vector_width > 1) return LB_ERR_UNSUPPORTED;
    if (s.kind == LB_AUTO) {  // the Sec. 6.2 rule, as for SpMV; groups of at least 8 lanes
        const lb_schedule_t h = heuristic(G);
        s.kind = h.kind;
        s.group_size = h.group_size < 8 ? 8 : h.group_size;
        s.tiles_per_group = 1;
    }
    lbk::trav_cfg c{};
    c.kind = s.kind;
    c.grid = s.grid_size;
    switch (s.kind) {
        case LB_THREAD_MAPPED:
            c.block = s.block_size ? s.block_size : kDefaultBlock;
            if (c.block % 64 != 0 || c.block > 1024) return LB_ERR_INVALID_ARG;
            break;
        case LB_GROUP_MAPPED:
        case LB_WORK_QUEUE:
            c.group = s.group_size ? s.group_size : kDefaultGroup;
            if (!is_pow2(c.group) || c.group > 1024) return LB_ERR_INVALID_ARG;
            if (!lbk::traversal_group_supported(c.group)) return LB_ERR_UNSUPPORTED;
            c.tiles_per_group = s.tiles_per_group ? s.tiles_per_group : (s.kind == LB_WORK_QUEUE ? c.group : 1);
            if (c.tiles_per_group != 1 && c.tiles_per_group != c.group) return LB_ERR_UNSUPPORTED;
            if (s.kind == LB_WORK_QUEUE && c.tiles_per_group != c.group) return LB_ERR_UNSUPPORTED;
            break;
        case LB_MERGE_PATH:  // one configuration: 256 threads x 8 merge items per unit
            if ((s.block_size && s.block_size != 256) || (s.items_per_thread && s.items_per_thread != 8))
                return LB_ERR_UNSUPPORTED;
            break;
        default: return LB_ERR_INVALID_ARG;
    }
    *out = c;
    return LB_OK;
}

template <bool BFS>
lb_status_t traversal(const lb_csr_t *G, int64_t source, void *out, const lb_schedule_t *s, int32_t max_iterations,
                      int32_t *iterations, void *workspace, size_t workspace_bytes, void *stream) {
    lb_status_t st = check_graph(G, !BFS);
    if (st != LB_OK) return st;
    if (!out || source < 0 || source >= G->rows || max_iterations < 0) return LB_ERR_INVALID_ARG;
    lbk::trav_cfg c;
    st = traversal_cfg(G, s, &c);
    if (st != LB_OK) return st;
    if (!workspace || workspace_bytes < lbk::trav_ws_bytes(G->rows, G->nnz)) return LB_ERR_WORKSPACE_TOO_SMALL;
    const int64_t cap = G->rows + 1;
    const int32_t max_iter = static_cast<int32_t>(max_iterations == 0 || max_iterations > cap ? cap : max_iterations);
    lbk::csr_dev d = to_dev(G);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    bool converged = false;
    hipError_t e;
    if constexpr (BFS)
        e = lbk::bfs(d, static_cast<int32_t>(source), static_cast<int32_t *>(out), c, max_iter, iterations,
                     &converged, workspace, hs);
    else
        e = lbk::sssp(d, static_cast<int32_t>(source), static_cast<float *>(out), c, max_iter, iterations,
                      &converged, workspace, hs);
    if (e != hipSuccess) return hip_status(e);
    return converged ? LB_OK : LB_ERR_NOT_CONVERGED;
}


// ------------------------------------------------------------------ profiling

struct prof_rec {
    std::string name;
    hipEvent_t start, stop;
    bool closed;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<prof_rec> g_prof;

}  // namespace

namespace lbk {

bool profiling_enabled() { return g_prof_on; }

void profile_mark(hipStream_t s, const char *name, bool begin) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    if (begin) {
        g_prof.push_back({name, e, nullptr, false});
        return;
    }
    for (auto it = g_prof.rbegin(); it != g_prof.rend(); ++it) {
        if (!it->closed && it->name == name) {
            it->stop = e;
            it->closed = true;
            return;
        }
    }
    (void)hipEventDestroy(e);
}

}  // namespace lbk

namespace {

std::vector<lb_schedule_t> candidates(const lb_csr_t *A, int32_t k) {
    std::vector<lb_schedule_t> c;
    for (int b : {128, 256, 512})
        for (int it : {4, 8, 12, 16})
            c.push_back({LB_MERGE_PATH, 0, 0, it, b, 0});
    c.push_back({LB_THREAD_MAPPED, 0, 0, 0, 256, 0});
    if (k == 1) {
        for (int g : {8, 16, 32, 64, 256, 1024}) {
            c.push_back({LB_GROUP_MAPPED, g, 1, 0, 0, 0});
            c.push_back({LB_GROUP_MAPPED, g, g, 0, 0, 0});
        }
        for (int g : {64, 256}) c.push_back({LB_WORK_QUEUE, g, g, 0, 0, 0});
        // two column bands of x: only when x is larger than one XCD's L2
        const int64_t x_bytes = A->cols * (A->value_dtype == LB_BF16 ? 2 : 4);
        if (x_bytes >= (int64_t(4) << 20))
            for (const auto &bi : {std::pair<int, int>{256, 8}, {256, 12}, {512, 8}, {128, 16}})
                c.push_back({LB_MERGE_PATH, 0, 0, bi.second, bi.first, 0, 2, 1});
        // four nonzeros per lane and load (pays where columns are local)
        for (const auto &bi : {std::pair<int, int>{256, 8}, {256, 12}, {128, 16}, {512, 8}})
            c.push_back({LB_MERGE_PATH, 0, 0, bi.second, bi.first, 0, 1, 4});
    }
    return c;
}

template <typename F>
lb_status_t time_call(F &&f, hipStream_t hs, float *ms_out) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return LB_ERR_HIP;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return LB_ERR_HIP;
    }
    lb_status_t st = f();  // warm-up
    std::vector<float> t;
    for (int rep = 0; rep < 5 && st == LB_OK; ++rep) {
        (void)hipEventRecord(a, hs);
        st = f();
        (void)hipEventRecord(b, hs);
        if (hipEventSynchronize(b) != hipSuccess) st = LB_ERR_HIP;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != LB_OK) return st;
    std::sort(t.begin(), t.end());
    *ms_out = t[t.size() / 2];
    return LB_OK;
}

// ------------------------------------------------------------------ lb_spmv

// Host checks and schedule resolution shared by lb_spmv and lb_spmv_noalloc;
// *need receives the workspace bytes of the resolved schedule.
lb_status_t spmv_prepare(const lb_csr_t *A, const void *x, lb_dtype_t x_dtype, float *y, const lb_schedule_t *s,
                         lb_schedule_t *r, size_t *need) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (A->rows > 0 && !y) return LB_ERR_INVALID_ARG;
    if (A->nnz > 0 && !x) return LB_ERR_INVALID_ARG;
    if (x_dtype != A->value_dtype) return LB_ERR_UNSUPPORTED;
    st = resolve(A, 1, s, r);
    if (st != LB_OK) return st;
    *need = ws_bytes_for(A, *r, 1);
    return LB_OK;
}

// The launches of y = A x under the resolved schedule r; workspace holds at
// least ws_bytes_for(A, r, 1) bytes.
lb_status_t spmv_launch(const lb_csr_t *A, const void *x, float *y, const lb_schedule_t &r, void *workspace,
                        hipStream_t hs) {
    if (A->rows == 0) return LB_OK;
    if (A->nnz == 0) return hip_status(lbk::fill_f32(y, A->rows, 0.f, hs));
    const lbk::csr_dev d = to_dev(A);
    switch (r.kind) {
        case LB_THREAD_MAPPED: return hip_status(lbk::thread_mapped_spmv(d, x, y, r.block_size, r.grid_size, hs));
        case LB_GROUP_MAPPED:
            return hip_status(
                lbk::group_mapped_spmv(d, x, y, r.group_size, r.tiles_per_group, r.grid_size, nullptr, hs));
        case LB_WORK_QUEUE:
            return hip_status(lbk::group_mapped_spmv(d, x, y, r.group_size, r.group_size, r.grid_size,
                                                     static_cast<int32_t *>(workspace), hs));
        case LB_MERGE_PATH:
            return hip_status(lbk::merge_spmv(d, x, y, r.block_size, r.items_per_thread, r.x_bands, workspace, hs,
                                              nullptr, r.vector_width));
        default: return LB_ERR_INVALID_ARG;
    }
}

// ------------------------------------------------------------------ planned SpMV


// Resolves the plan's inputs for A (defaults, checks) into *out; host only.
lb_status_t plan_params(const lb_csr_t *A, const lb_spmv_plan_t *in, lb_spmv_plan_t *out) {
    lb_spmv_plan_t p{};
    p.block_size = in->block_size ? in->block_size : kDefaultBlock;
    p.items_per_thread = in->items_per_thread ? in->items_per_thread : kDefaultItems;
    if (p.block_size < 0 || p.items_per_thread < 0) return LB_ERR_INVALID_ARG;
    if (!lbk::merge_config_supported(p.block_size, p.items_per_thread)) return LB_ERR_UNSUPPORTED;
    const int64_t W = static_cast<int64_t>(p.block_size) * p.items_per_thread;
    const int64_t sx = A->value_dtype == LB_BF16 ? 2 : 4;
    p.x_bands = in->x_bands;  // 0: decided by the build (size of x, locality of the columns)
    if (p.x_bands != 0 && p.x_bands != 1 && p.x_bands != 2) return LB_ERR_INVALID_ARG;
    (void)sx;
    p.panel_cols = in->panel_cols ? in->panel_cols : static_cast<int32_t>(lbk::kPanelBytes / sx);
    p.streams = in->streams ? in->streams : 1;
    p.vector_width = in->vector_width;  // 0: decided by the build (locality of the columns)
    if (p.vector_width != 0 && p.vector_width != 1 && p.vector_width != 4) return LB_ERR_INVALID_ARG;
    if (p.vector_width == 4 && p.x_bands == 2) return LB_ERR_UNSUPPORTED;
    if (p.vector_width == 4) p.x_bands = 1;
    p.panel_blocks = in->panel_blocks;  // 0: resolved by the build from the device's CUs
    if (p.panel_blocks < 0) return LB_ERR_INVALID_ARG;
    if (p.streams != 1 && p.streams != 2) return LB_ERR_INVALID_ARG;
    if (!lbk::panel_cols_ok(p.panel_cols, A->value_dtype)) return LB_ERR_INVALID_ARG;
    const int64_t NP = (A->cols + p.panel_cols - 1) / p.panel_cols;
    if (in->long_min == -1) {
        p.long_min = 0x7fffffff;  // no row is long
    } else if (in->long_min == 0) {
        p.long_min = static_cast<int32_t>(std::max<int64_t>(W, 16 * NP));
    } else {
        if (in->long_min < W) return LB_ERR_INVALID_ARG;
        p.long_min = in->long_min;
    }
    p.value_dtype = A->value_dtype;
    p.rows = A->rows;
    p.cols = A->cols;
    p.nnz = A->nnz;
    p.panels = static_cast<int32_t>(NP);
    p.units = static_cast<int32_t>(lbk::merge_units(A->rows, A->nnz, W));
    *out = p;
    return LB_OK;
}

lbk::plan_dev plan_dev_of(const lb_spmv_plan_t &p) {
    lbk::plan_dev d{};
    d.rows = static_cast<int32_t>(p.rows);
    d.T = p.units;
    d.NA = p.active_units;
    d.NL = p.long_rows;
    d.NP = p.panels;
    d.R = p.panel_blocks;
    d.P = p.panel_cols;
    d.long_min = p.long_min;
    d.bands = p.x_bands;
    d.streams = p.streams;
    d.block = p.block_size;
    d.items = p.items_per_thread;
    d.vec = p.vector_width;
    d.ntasks = p.tasks;
    const lbk::plan_layout L = lbk::plan_layout_of(p.units, p.units, p.long_rows, p.panels, p.tasks, p.rows);
    const char *b = static_cast<const char *>(p.buffer);
    d.part_i = reinterpret_cast<const int32_t *>(b + L.part_i);
    d.part_j = reinterpret_cast<const int32_t *>(b + L.part_j);
    d.units = reinterpret_cast<const lbk::plan_unit *>(b + L.units);
    d.LR = reinterpret_cast<const int32_t *>(b + L.LR);
    d.long_bits = reinterpret_cast<const uint32_t *>(b + L.long_bits);
    d.row_task = reinterpret_cast<const int32_t *>(b + L.row_task);
    d.pcls_off = reinterpret_cast<const int32_t *>(b + L.pcls_off);
    d.tasks = reinterpret_cast<const lbk::panel_task *>(b + L.tasks);
    return d;
}

}  // namespace

// ------------------------------------------------------------------ static scratch

// lb_spmv_noalloc's workspace: one copy per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in, not device
// memory; host code uses only the per-device address that
// hipGetSymbolAddress returns for it.  Nothing in it has to start at zero:
// the merge-path launches write the split, carries and band sums before
// reading them, and the work queue clears its counter with a fill kernel.
static constexpr size_t kScratchBytes = LB_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// The device address of `scratch` on the device that runs `hs` (the current
// device for the null stream), looked up once per device with that device
// current.
lb_status_t scratch_address(hipStream_t hs, void **out) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_status(e);
    int dev = cur;
    if (hs) {
        hipDevice_t sd = 0;
        e = hipStreamGetDevice(hs, &sd);
        if (e != hipSuccess) return hip_status(e);
        dev = static_cast<int>(sd);
    }
    if (dev < 0 || dev >= kMaxDevices) return LB_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return hip_status(e);
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t back = dev != cur ? hipSetDevice(cur) : hipSuccess;
        if (e != hipSuccess) return hip_status(e);
        if (back != hipSuccess) return hip_status(back);
        if (!p) return LB_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LB_OK;
}

}  // namespace

// Samples of col_idx for pattern fingerprints (host code uses only the
// address hipGetSymbolAddress returns; calls are serialised by g_fp_mu).
static __device__ int32_t g_fp_samples[kFingerprintSamples];

namespace {

std::mutex g_fp_mu;

// Fingerprint of a pattern: FNV-1a over the sizes, every row offset, the
// column indices at kFingerprintSamples evenly spaced positions and (a
// batch) the matrices' base tables.  Synchronizes hs.
lb_status_t fingerprint(int64_t rows, int64_t cols, int64_t nnz, const int32_t *ro, const int32_t *ci,
                        const int64_t *const *bases, int64_t count, hipStream_t hs, uint64_t *out) {
    std::lock_guard<std::mutex> g(g_fp_mu);
    std::vector<int32_t> h_ro(static_cast<size_t>(rows) + 1, 0), h_smp(kFingerprintSamples, 0);
    std::vector<int64_t> h_base(bases ? 3 * static_cast<size_t>(count + 1) : 0);
    int32_t *d_smp = nullptr;
    hipError_t e = hipGetSymbolAddress(reinterpret_cast<void **>(&d_smp), HIP_SYMBOL(g_fp_samples));
    if (e == hipSuccess && rows > 0)
        e = hipMemcpyAsync(h_ro.data(), ro, h_ro.size() * 4, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess && nnz > 0) e = lbk::gather_samples(ci, nnz, kFingerprintSamples, d_smp, hs);
    if (e == hipSuccess && nnz > 0) e = hipMemcpyAsync(h_smp.data(), d_smp, h_smp.size() * 4, hipMemcpyDeviceToHost, hs);
    for (int t = 0; bases && t < 3 && e == hipSuccess; ++t)
        e = hipMemcpyAsync(h_base.data() + t * (count + 1), bases[t], static_cast<size_t>(count + 1) * 8,
                           hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return hip_status(e);
    fnv64 h;
    h.add(rows);
    h.add(cols);
    h.add(nnz);
    h.add(h_ro.data(), h_ro.size() * 4);
    h.add(h_smp.data(), h_smp.size() * 4);
    h.add(h_base.data(), h_base.size() * 8);
    *out = h.h;
    return LB_OK;
}

// out[i] = a[pos[i]] for a few thousand positions (at most
// kFingerprintSamples), through the fingerprint sample buffer; synchronizes hs.
lb_status_t device_gather(const int32_t *a, const std::vector<int32_t> &pos, std::vector<int32_t> &out,
                          hipStream_t hs) {
    const int32_t n = static_cast<int32_t>(std::min<size_t>(pos.size(), kFingerprintSamples / 2));
    if (n == 0) return LB_OK;
    std::lock_guard<std::mutex> g(g_fp_mu);
    int32_t *d = nullptr;
    hipError_t e = hipGetSymbolAddress(reinterpret_cast<void **>(&d), HIP_SYMBOL(g_fp_samples));
    // the positions go in the buffer's upper half, the values in its lower half
    if (e == hipSuccess)
        e = hipMemcpyAsync(d + kFingerprintSamples / 2, pos.data(), static_cast<size_t>(n) * 4, hipMemcpyHostToDevice,
                           hs);
    if (e == hipSuccess) e = lbk::gather_at(a, d + kFingerprintSamples / 2, n, d, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(out.data(), d, static_cast<size_t>(n) * 4, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    return hip_status(e);
}

}  // namespace

// ================================================================== C ABI

extern "C" {

LB_API int lb_abi_version(void) { return LB_ABI_VERSION; }

LB_API const char *lb_status_string(lb_status_t st) {
    switch (st) {
        case LB_OK: return "ok";
        case LB_ERR_INVALID_ARG: return "invalid argument";
        case LB_ERR_UNSUPPORTED: return "unsupported dtype, schedule or parameter";
        case LB_ERR_OVERFLOW: return "size exceeds int32 merge coordinates";
        case LB_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case LB_ERR_HIP: return "HIP error";
        case LB_ERR_INVALID_CSR: return "CSR arrays violate a device-side precondition";
        case LB_ERR_NOT_CONVERGED: return "traversal frontier not empty after max_iterations";
        case LB_ERR_SCRATCH_LIMIT: return "input needs more scratch than lb_spmv_noalloc's static buffer";
    }
    return "unknown status";
}

LB_API const char *lb_last_hip_error(void) { return g_last_hip.c_str(); }

LB_API lb_status_t lb_resolve_schedule(const lb_csr_t *A, int32_t k, const lb_schedule_t *in, lb_schedule_t *out) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    return resolve(A, k, in, out);
}

LB_API lb_status_t lb_workspace_size(const lb_csr_t *A, const lb_schedule_t *s, int32_t k, size_t *bytes) {
    if (!bytes || k < 0 || k > kMaxK) return LB_ERR_INVALID_ARG;
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    lb_schedule_t r;
    st = resolve(A, k, s, &r);
    if (st != LB_OK) return st;
    if (k == 0) {  // backward always runs on the merge-path split
        if (r.kind != LB_MERGE_PATH) {
            lb_schedule_t m{};
            m.kind = LB_MERGE_PATH;
            fill_defaults(&m, &r);
        }
    }
    *bytes = ws_bytes_for(A, r, k);
    return LB_OK;
}

LB_API lb_status_t lb_spmv(const lb_csr_t *A, const void *x, lb_dtype_t x_dtype, float *y, const lb_schedule_t *s,
                           void *workspace, size_t workspace_bytes, void *stream) {
    lb_schedule_t r;
    size_t need = 0;
    lb_status_t st = spmv_prepare(A, x, x_dtype, y, s, &r, &need);
    if (st != LB_OK) return st;
    if (need > 0 && (workspace_bytes < need || !workspace)) return LB_ERR_WORKSPACE_TOO_SMALL;
    return spmv_launch(A, x, y, r, workspace, static_cast<hipStream_t>(stream));
}

LB_API lb_status_t lb_spmv_noalloc(const lb_csr_t *A, const void *x, lb_dtype_t x_dtype, float *y,
                                   const lb_schedule_t *s, void *stream) {
    lb_schedule_t r;
    size_t need = 0;
    lb_status_t st = spmv_prepare(A, x, x_dtype, y, s, &r, &need);
    if (st != LB_OK) return st;
    if (need > kScratchBytes) return LB_ERR_SCRATCH_LIMIT;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (A->rows == 0) return LB_OK;
    void *ws = nullptr;
    if (need > 0) {
        st = scratch_address(hs, &ws);
        if (st != LB_OK) return st;
    }
    return spmv_launch(A, x, y, r, ws, hs);
}

LB_API lb_status_t lb_spmv_plan_build(const lb_csr_t *A, lb_spmv_plan_t *plan, void *buffer, size_t buffer_bytes,
                                      void *stream) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (!plan) return LB_ERR_INVALID_ARG;
    lb_spmv_plan_t p;
    st = plan_params(A, plan, &p);
    if (st != LB_OK) return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const int64_t rows = A->rows, NP = p.panels;
    // row lengths on the host: the long rows and a bound on the tasks
    std::vector<int32_t> ro(static_cast<size_t>(rows) + 1, 0);
    if (rows > 0) {
        hipError_t e = hipMemcpyAsync(ro.data(), A->row_offsets, ro.size() * 4, hipMemcpyDeviceToHost, hs);
        if (e == hipSuccess) e = hipStreamSynchronize(hs);
        if (e != hipSuccess) return hip_status(e);
    }
    if (p.x_bands == 0 || p.vector_width == 0) {
        // Column locality: the columns are scattered when the median column
        // span (last - first) of up to 1024 sampled rows with two or more
        // nonzeros exceeds cols / 16 (a stencil's rows span a few grid rows).
        // Two column bands pay when x is larger than an XCD's L2 (4 MiB) and
        // the columns are scattered; four nonzeros per lane and load pay when
        // they are local (one band).
        bool scattered = false;
        std::vector<int32_t> pos;
        const int64_t step = std::max<int64_t>(1, rows / 1024);
        for (int64_t r = 0; r < rows && pos.size() < 2048; r += step)
            if (ro[r + 1] - ro[r] >= 2) {
                pos.push_back(ro[r]);
                pos.push_back(ro[r + 1] - 1);
            }
        std::vector<int32_t> cols(pos.size());
        lb_status_t sst = device_gather(A->col_idx, pos, cols, hs);
        if (sst != LB_OK) return sst;
        std::vector<int64_t> span;
        for (size_t i = 0; i + 1 < cols.size(); i += 2) span.push_back(static_cast<int64_t>(cols[i + 1]) - cols[i]);
        if (!span.empty()) {
            std::nth_element(span.begin(), span.begin() + span.size() / 2, span.end());
            scattered = span[span.size() / 2] > A->cols / 16;
        }
        const int64_t sx = A->value_dtype == LB_BF16 ? 2 : 4;
        if (p.x_bands == 0) p.x_bands = scattered && A->cols * sx >= (int64_t(4) << 20) ? 2 : 1;
        if (p.vector_width == 0) p.vector_width = !scattered && p.x_bands == 1 ? 4 : 1;
        lb_spmv_plan_t in2 = *plan;
        in2.x_bands = p.x_bands;
        in2.vector_width = p.vector_width;
        bool again = false;
        if (plan->items_per_thread == 0 && p.vector_width == 4) {
            // local columns: longer units (12 items per thread) amortize each
            // block's fixed latency (split, search, scan) over more nonzeros
            in2.items_per_thread = kLocalItems;
            again = true;
        } else if (plan->items_per_thread == 0 && plan->block_size == 0 && p.vector_width == 1) {
            // scattered columns: shorter units (128 threads; 8 items with two
            // bands, 4 with one) spread the gather-bound short rows over more
            // blocks and lower the default long_min, moving rows of W to 2047
            // nonzeros to the panels
            in2.block_size = kScatteredBlock;
            in2.items_per_thread = p.x_bands == 2 ? 8 : 4;
            again = true;
        }
        if (again) {
            st = plan_params(A, &in2, &p);
            if (st != LB_OK) return st;
        }
    }
    std::vector<int32_t> LR;
    int64_t long_nnz = 0, task_bound = 0;
    for (int64_t r = 0; r < rows; ++r) {
        const int64_t len = static_cast<int64_t>(ro[r + 1]) - ro[r];
        if (len < p.long_min) continue;
        LR.push_back(static_cast<int32_t>(r));
        long_nnz += len;
        task_bound += (len + lbk::kPanelTask - 1) / lbk::kPanelTask + NP;
    }
    if (task_bound > kMaxCoord) return LB_ERR_OVERFLOW;
    p.long_rows = static_cast<int32_t>(LR.size());
    p.long_nnz = long_nnz;
    if (p.panel_blocks == 0) {
        // one round of one resident block per CU (a panel fills the CU's
        // LDS), rounded down to whole panels: a second round that only some
        // blocks run would idle the rest and restage panels
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        (void)hipGetLastError();
        p.panel_blocks = static_cast<int32_t>(std::max<int64_t>(1, static_cast<int64_t>(cus) / std::max<int64_t>(NP, 1)));
    }
    if (static_cast<int64_t>(p.panel_blocks) * NP >= kMaxCoord) return LB_ERR_OVERFLOW;
    const int64_t T = p.units;
    p.tasks = static_cast<int32_t>(task_bound);  // a bound until the build
    p.active_units = static_cast<int32_t>(T);    // a bound until the build
    const lbk::plan_layout L = lbk::plan_layout_of(T, T, p.long_rows, NP, task_bound, rows);
    p.plan_bytes = L.total;
    p.workspace_bytes = lbk::plan_ws_bytes(p.x_bands, rows, task_bound);
    p.buffer = nullptr;
    if (!buffer || buffer_bytes < p.plan_bytes) {
        *plan = p;
        return LB_ERR_WORKSPACE_TOO_SMALL;
    }
    char *b = static_cast<char *>(buffer);
    int32_t *flags = reinterpret_cast<int32_t *>(b + L.flags);
    int32_t *part_i = reinterpret_cast<int32_t *>(b + L.part_i);
    int32_t *part_j = reinterpret_cast<int32_t *>(b + L.part_j);
    int32_t *d_LR = reinterpret_cast<int32_t *>(b + L.LR);
    int32_t *sb = reinterpret_cast<int32_t *>(b + L.sb);
    const int64_t nsb = static_cast<int64_t>(p.long_rows) * (NP + 1);
    std::vector<int32_t> h_sb(static_cast<size_t>(nsb)), h_part(static_cast<size_t>(T + 1)),
        h_partj(static_cast<size_t>(T + 1));
    int32_t h_flags = 0;
    hipError_t e = hipMemsetAsync(flags, 0, 4, hs);
    if (e == hipSuccess && rows > 0)
        e = lbk::merge_partition(A->row_offsets, static_cast<int32_t>(rows), static_cast<int32_t>(A->nnz),
                                 p.block_size * p.items_per_thread, static_cast<int32_t>(T), part_i, part_j, hs);
    if (e == hipSuccess && !LR.empty()) e = hipMemcpyAsync(d_LR, LR.data(), LR.size() * 4, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && nsb > 0)
        e = lbk::plan_segments_launch(p.long_rows, static_cast<int32_t>(NP), p.panel_cols, d_LR, A->row_offsets,
                                      A->col_idx, sb, flags, hs);
    if (e == hipSuccess && nsb > 0) e = hipMemcpyAsync(h_sb.data(), sb, h_sb.size() * 4, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess && rows > 0)
        e = hipMemcpyAsync(h_part.data(), part_i, h_part.size() * 4, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess && rows > 0)
        e = hipMemcpyAsync(h_partj.data(), part_j, h_partj.size() * 4, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(&h_flags, flags, 4, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return hip_status(e);
    if (h_flags & 1) return LB_ERR_INVALID_CSR;
    // Tasks: each (row, panel) segment cut into pieces of at most kPanelTask
    // nonzeros; a piece's sum goes to slot row_task[q] + (pieces of row q in
    // earlier panels) + its index, so a row's sums are consecutive.  Each
    // panel lists its pieces by class (the aligned groups of four they span),
    // in row order inside a class.
    std::vector<int32_t> row_task(static_cast<size_t>(p.long_rows) + 1, 0);
    std::vector<int32_t> slot(static_cast<size_t>(nsb));  // first slot of (row q, panel p)
    for (int64_t q = 0; q < p.long_rows; ++q) {
        const int32_t *sq = h_sb.data() + q * (NP + 1);
        int64_t o = row_task[q];
        for (int64_t pp = 0; pp <= NP; ++pp) {
            slot[q * (NP + 1) + pp] = static_cast<int32_t>(o);
            if (pp < NP) o += (static_cast<int64_t>(sq[pp + 1]) - sq[pp] + lbk::kPanelTask - 1) / lbk::kPanelTask;
        }
        row_task[q + 1] = static_cast<int32_t>(o);
    }
    const int64_t ntasks = p.long_rows > 0 ? row_task.back() : 0;
    std::vector<int32_t> pcls_off(static_cast<size_t>(NP) * lbk::kPanelClasses + 1, 0);
    std::vector<lbk::panel_task> tasks;
    tasks.reserve(static_cast<size_t>(ntasks));
    {
        std::vector<lbk::panel_task> cls[lbk::kPanelClasses];
        for (int64_t pp = 0; pp < NP; ++pp) {
            for (auto &v : cls) v.clear();
            for (int64_t q = 0; q < p.long_rows; ++q) {
                const int64_t e2 = q * (NP + 1) + pp;
                const int32_t sbeg = h_sb[e2], send = h_sb[e2 + 1];
                int32_t out = slot[e2];
                for (int32_t a0 = sbeg; a0 < send; a0 += lbk::kPanelTask, ++out) {
                    const int32_t len = std::min<int32_t>(lbk::kPanelTask, send - a0);
                    const int64_t ng = ((static_cast<int64_t>(a0) + len - 1) >> 2) - (a0 >> 2) + 1;
                    cls[lbk::panel_class(ng)].push_back(lbk::panel_task{a0, len, out, 0});
                }
            }
            for (int k = 0; k < lbk::kPanelClasses; ++k) {
                pcls_off[pp * lbk::kPanelClasses + k] = static_cast<int32_t>(tasks.size());
                tasks.insert(tasks.end(), cls[k].begin(), cls[k].end());
            }
        }
        pcls_off.back() = static_cast<int32_t>(tasks.size());
    }
    // units with short-row work: a short row closes in it (only its first
    // closing row can be long); a short row is owned, whole, by the unit
    // where it closes
    auto is_short = [&](int64_t r) { return static_cast<int64_t>(ro[r + 1]) - ro[r] < p.long_min; };
    std::vector<lbk::plan_unit> h_units;
    h_units.reserve(static_cast<size_t>(T));
    for (int64_t u = 0; u < T; ++u) {
        const int32_t i0 = h_part[u], i1 = h_part[u + 1];
        if (!(i1 > i0 + 1 || (i0 < i1 && is_short(i0)))) continue;
        // the record its block reads: products of [ja, jb) (a long first row
        // and the open row left out), the head of row i0 (ro[i0] <= j0)
        lbk::plan_unit r{i0, i1, h_partj[u], h_partj[u + 1], h_partj[u], h_partj[u + 1], ro[i0], 0};
        if (!is_short(i0)) {
            r.flags = 1;
            r.ja = ro[i0 + 1];
            r.h0 = r.j0;
        }
        if (i1 < rows) r.jb = std::min(ro[i1], r.j1);
        if (r.jb < r.ja) r.jb = r.ja;
        if (!r.flags) {  // a long row i0 keeps the merge walk (its nonzeros are skipped there)
            int64_t most = 0;
            for (int32_t q = i0; q < i1 && most <= lbk::kRowPerThreadMax; ++q)
                most = std::max<int64_t>(most, static_cast<int64_t>(ro[q + 1]) - std::max(ro[q], r.j0));
            if (most <= lbk::kRowPerThreadMax) r.flags |= 2;
        }
        h_units.push_back(r);
    }
    std::vector<uint32_t> long_bits(static_cast<size_t>((rows + 31) / 32), 0u);
    for (int32_t r : LR) long_bits[static_cast<size_t>(r) >> 5] |= 1u << (r & 31);
    e = hipSuccess;
    auto up = [&](size_t off, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes > 0) e = hipMemcpyAsync(b + off, src, bytes, hipMemcpyHostToDevice, hs);
    };
    up(L.row_task, row_task.data(), row_task.size() * 4);
    up(L.pcls_off, pcls_off.data(), pcls_off.size() * 4);
    up(L.tasks, tasks.data(), tasks.size() * sizeof(lbk::panel_task));
    up(L.units, h_units.data(), h_units.size() * sizeof(lbk::plan_unit));
    up(L.long_bits, long_bits.data(), long_bits.size() * 4);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return hip_status(e);
    p.active_units = static_cast<int32_t>(h_units.size());
    p.tasks = static_cast<int32_t>(ntasks);
    p.workspace_bytes = lbk::plan_ws_bytes(p.x_bands, rows, ntasks);
    p.buffer = buffer;
    *plan = p;
    return LB_OK;
}

LB_API lb_status_t lb_spmv_planned(const lb_csr_t *A, const lb_spmv_plan_t *plan, const void *x, lb_dtype_t x_dtype,
                                   float *y, void *workspace, size_t workspace_bytes, void *stream) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (!plan) return LB_ERR_INVALID_ARG;
    if (plan->rows != A->rows || plan->cols != A->cols || plan->nnz != A->nnz ||
        plan->value_dtype != A->value_dtype)
        return LB_ERR_INVALID_ARG;
    if (A->rows > 0 && (!y || !plan->buffer)) return LB_ERR_INVALID_ARG;
    if (A->nnz > 0 && !x) return LB_ERR_INVALID_ARG;
    if (x_dtype != A->value_dtype) return LB_ERR_UNSUPPORTED;
    if (plan->workspace_bytes > 0 && (workspace_bytes < plan->workspace_bytes || !workspace))
        return LB_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (A->rows == 0) return LB_OK;
    if (A->nnz == 0) return hip_status(lbk::fill_f32(y, A->rows, 0.f, hs));
    return hip_status(lbk::planned_spmv(to_dev(A), plan_dev_of(*plan), x, y, workspace, hs));
}

LB_API lb_status_t lb_transpose_workspace_size(const lb_csr_t *A, size_t *bytes) {
    if (!bytes) return LB_ERR_INVALID_ARG;
    const lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (A->cols + A->nnz > kMaxCoord) return LB_ERR_OVERFLOW;
    *bytes = lbk::transpose_ws_bytes(A->cols, A->nnz);
    return LB_OK;
}

LB_API lb_status_t lb_transpose_pattern(const lb_csr_t *A, int32_t *at_row_offsets, int32_t *at_col_idx,
                                        int32_t *perm, void *workspace, size_t workspace_bytes, void *stream) {
    size_t need = 0;
    const lb_status_t st = lb_transpose_workspace_size(A, &need);
    if (st != LB_OK) return st;
    if (!at_row_offsets || (A->nnz > 0 && (!at_col_idx || !perm))) return LB_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < need) return LB_ERR_WORKSPACE_TOO_SMALL;
    return hip_status(lbk::transpose_pattern(to_dev(A), at_row_offsets, at_col_idx, perm, workspace,
                                             static_cast<hipStream_t>(stream)));
}

lb_status_t backward_transposed_schedule(const lb_schedule_t *s, lb_schedule_t *out) {
    lb_schedule_t in = s ? *s : lb_schedule_t{LB_MERGE_PATH, 0, 0, 0, 0, 0};
    if (in.kind == LB_AUTO) in.kind = LB_MERGE_PATH;
    if (in.kind != LB_MERGE_PATH) return LB_ERR_UNSUPPORTED;
    const lb_status_t st = fill_defaults(&in, out);
    return st != LB_OK ? st : one_band(*out);
}

LB_API lb_status_t lb_backward_transposed_workspace_size(const lb_csr_t *A, const lb_schedule_t *s, size_t *bytes) {
    if (!bytes) return LB_ERR_INVALID_ARG;
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (A->cols + A->nnz > kMaxCoord) return LB_ERR_OVERFLOW;
    lb_schedule_t r;
    st = backward_transposed_schedule(s, &r);
    if (st != LB_OK) return st;
    *bytes = lbk::backward_transposed_ws_bytes(A->rows, A->cols, A->nnz, r.block_size, r.items_per_thread);
    return LB_OK;
}

LB_API lb_status_t lb_spmv_backward_transposed(const lb_csr_t *A, const int32_t *at_row_offsets,
                                               const int32_t *at_col_idx, const int32_t *perm, const void *x,
                                               lb_dtype_t x_dtype, const float *dy, float *dx, float *dvalues,
                                               const lb_schedule_t *s, void *workspace, size_t workspace_bytes,
                                               void *stream) {
    size_t need = 0;
    lb_status_t st = lb_backward_transposed_workspace_size(A, s, &need);
    if (st != LB_OK) return st;
    if (x_dtype != A->value_dtype) return LB_ERR_UNSUPPORTED;
    if (A->rows > 0 && A->nnz > 0 && !dy && (dx || dvalues)) return LB_ERR_INVALID_ARG;
    if (dvalues && A->nnz > 0 && !x) return LB_ERR_INVALID_ARG;
    if (dx && (!at_row_offsets || (A->nnz > 0 && (!at_col_idx || !perm)))) return LB_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < need) return LB_ERR_WORKSPACE_TOO_SMALL;
    lb_schedule_t r;
    (void)backward_transposed_schedule(s, &r);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (A->nnz == 0 || A->rows == 0) {  // no entries: dx = 0, no dvalues
        if (dx && A->cols > 0) return hip_status(lbk::fill_f32(dx, A->cols, 0.f, hs));
        return LB_OK;
    }
    return hip_status(lbk::backward_transposed(to_dev(A), at_row_offsets, at_col_idx, perm, x, dy, dx, dvalues,
                                               r.block_size, r.items_per_thread, workspace, hs));
}

lb_status_t check_spgemm(const lb_csr_t *A, const lb_csr_t *B) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    st = check_csr(B);
    if (st != LB_OK) return st;
    if (B->rows != A->cols) return LB_ERR_INVALID_ARG;
    if (A->value_dtype != LB_F32 || B->value_dtype != LB_F32) return LB_ERR_UNSUPPORTED;
    return LB_OK;
}

lbk::spgemm_dev to_spgemm(const lb_csr_t *A, const lb_csr_t *B) {
    return {static_cast<int32_t>(A->rows), static_cast<int32_t>(A->cols), static_cast<int32_t>(B->cols),
            static_cast<int32_t>(A->nnz), A->row_offsets, A->col_idx, static_cast<const float *>(A->values), B->row_offsets, B->col_idx,
            static_cast<const float *>(B->values)};
}

LB_API lb_status_t lb_spgemm_workspace_size(const lb_csr_t *A, const lb_csr_t *B, size_t *bytes) {
    if (!bytes) return LB_ERR_INVALID_ARG;
    const lb_status_t st = check_spgemm(A, B);
    if (st != LB_OK) return st;
    *bytes = lbk::spgemm_ws_bytes(A->rows, B->cols);
    return LB_OK;
}

LB_API lb_status_t lb_spgemm_count(const lb_csr_t *A, const lb_csr_t *B, int32_t *c_row_offsets, int64_t *c_nnz,
                                   void *workspace, size_t workspace_bytes, void *stream) {
    size_t need = 0;
    lb_status_t st = lb_spgemm_workspace_size(A, B, &need);
    if (st != LB_OK) return st;
    if (!c_row_offsets || !c_nnz) return LB_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < need) return LB_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    int64_t total = 0;
    const hipError_t e = lbk::spgemm_count(to_spgemm(A, B), c_row_offsets, &total, workspace, hs);
    if (e != hipSuccess) return hip_status(e);
    if (total > kMaxCoord) return LB_ERR_OVERFLOW;
    *c_nnz = total;
    return LB_OK;
}

LB_API lb_status_t lb_spgemm_compute(const lb_csr_t *A, const lb_csr_t *B, const int32_t *c_row_offsets,
                                     int32_t *c_col_idx, float *c_values, void *workspace, size_t workspace_bytes,
                                     void *stream) {
    size_t need = 0;
    lb_status_t st = lb_spgemm_workspace_size(A, B, &need);
    if (st != LB_OK) return st;
    if (!c_row_offsets || !c_col_idx || !c_values) return LB_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < need) return LB_ERR_WORKSPACE_TOO_SMALL;
    return hip_status(lbk::spgemm_compute(to_spgemm(A, B), c_row_offsets, c_col_idx, c_values, workspace,
                                          static_cast<hipStream_t>(stream)));
}

LB_API lb_status_t lb_coo_workspace_size(const lb_coo_t *A, const lb_schedule_t *s, size_t *bytes) {
    if (!bytes) return LB_ERR_INVALID_ARG;
    lb_status_t st = check_coo(A);
    if (st != LB_OK) return st;
    lb_schedule_t r;
    st = coo_schedule(A, s, &r);
    if (st != LB_OK) return st;
    *bytes = 0;
    if (r.kind == LB_MERGE_PATH) {
        const int64_t W = static_cast<int64_t>(r.block_size) * r.items_per_thread;
        *bytes = lbk::merge_ws_bytes(lbk::merge_units(A->rows, A->nnz, W), 1);
    }
    return LB_OK;
}

LB_API lb_status_t lb_spmv_coo(const lb_coo_t *A, const void *x, lb_dtype_t x_dtype, float *y, const lb_schedule_t *s,
                               void *workspace, size_t workspace_bytes, void *stream) {
    lb_status_t st = check_coo(A);
    if (st != LB_OK) return st;
    if (A->rows > 0 && !y) return LB_ERR_INVALID_ARG;
    if (A->nnz > 0 && !x) return LB_ERR_INVALID_ARG;
    if (x_dtype != A->value_dtype) return LB_ERR_UNSUPPORTED;
    lb_schedule_t r;
    st = coo_schedule(A, s, &r);
    if (st != LB_OK) return st;
    size_t need = 0;
    (void)lb_coo_workspace_size(A, &r, &need);
    if (need > 0 && (workspace_bytes < need || !workspace)) return LB_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (A->rows == 0) return LB_OK;
    if (A->nnz == 0) return hip_status(lbk::fill_f32(y, A->rows, 0.f, hs));
    const lbk::coo_dev d{static_cast<int32_t>(A->rows), static_cast<int32_t>(A->cols), static_cast<int32_t>(A->nnz),
                         A->row_idx, A->col_idx, A->values, A->value_dtype};
    return hip_status(lbk::coo_spmv(d, x, y, r.kind, r.group_size, r.block_size, r.items_per_thread, r.grid_size,
                                    workspace, hs));
}

LB_API lb_status_t lb_coo_merge_path_partition(const int32_t *row_idx, int64_t rows, int64_t nnz,
                                               int64_t items_per_unit, int64_t num_units, int32_t *out_row,
                                               int32_t *out_nz, void *stream) {
    if (rows < 0 || nnz < 0 || items_per_unit <= 0 || num_units < 0) return LB_ERR_INVALID_ARG;
    if (rows + nnz > kMaxCoord || items_per_unit > kMaxCoord || num_units > kMaxCoord) return LB_ERR_OVERFLOW;
    if (!out_row || !out_nz || (nnz > 0 && !row_idx)) return LB_ERR_INVALID_ARG;
    return hip_status(lbk::coo_partition(row_idx, static_cast<int32_t>(rows), static_cast<int32_t>(nnz),
                                         static_cast<int32_t>(items_per_unit), static_cast<int32_t>(num_units),
                                         out_row, out_nz, static_cast<hipStream_t>(stream)));
}

LB_API lb_status_t lb_csc_workspace_size(const lb_csc_t *A, const lb_schedule_t *s, size_t *bytes) {
    if (!bytes) return LB_ERR_INVALID_ARG;
    lb_csr_t c;
    lb_status_t st = check_csc(A, &c);
    if (st != LB_OK) return st;
    lb_schedule_t r;
    st = csc_schedule(s, &r);
    if (st != LB_OK) return st;
    *bytes = ws_bytes_for(&c, r, 0);
    return LB_OK;
}

LB_API lb_status_t lb_spmv_csc(const lb_csc_t *A, const void *x, lb_dtype_t x_dtype, float *y, const lb_schedule_t *s,
                               void *workspace, size_t workspace_bytes, void *stream) {
    lb_csr_t c;
    lb_status_t st = check_csc(A, &c);
    if (st != LB_OK) return st;
    if (A->rows > 0 && !y) return LB_ERR_INVALID_ARG;
    if (A->nnz > 0 && !x) return LB_ERR_INVALID_ARG;
    if (x_dtype != LB_F32) return LB_ERR_UNSUPPORTED;
    lb_schedule_t r;
    st = csc_schedule(s, &r);
    if (st != LB_OK) return st;
    const size_t need = ws_bytes_for(&c, r, 0);
    if (workspace_bytes < need || !workspace) return LB_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (A->rows == 0) return LB_OK;
    hipError_t e = lbk::fill_f32(y, A->rows, 0.f, hs);
    if (e != hipSuccess || A->nnz == 0) return hip_status(e);
    // the scatter of the backward pass: columns are its tiles, x its per-tile
    // value; a long row of A is hit from many columns, so each block first
    // sums its products per row in LDS
    return hip_status(lbk::merge_backward(to_dev(&c), nullptr, static_cast<const float *>(x), y, nullptr,
                                          r.block_size, r.items_per_thread, workspace, hs, true));
}

LB_API lb_status_t lb_traversal_workspace_size(const lb_csr_t *G, size_t *bytes) {
    if (!bytes) return LB_ERR_INVALID_ARG;
    const lb_status_t st = check_graph(G, false);
    if (st != LB_OK) return st;
    *bytes = lbk::trav_ws_bytes(G->rows, G->nnz);
    return LB_OK;
}

LB_API lb_status_t lb_sssp(const lb_csr_t *G, int64_t source, float *dist, const lb_schedule_t *s,
                           int32_t max_iterations, int32_t *iterations, void *workspace, size_t workspace_bytes,
                           void *stream) {
    return traversal<false>(G, source, dist, s, max_iterations, iterations, workspace, workspace_bytes, stream);
}

LB_API lb_status_t lb_bfs(const lb_csr_t *G, int64_t source, int32_t *depth, const lb_schedule_t *s,
                          int32_t max_iterations, int32_t *iterations, void *workspace, size_t workspace_bytes,
                          void *stream) {
    return traversal<true>(G, source, depth, s, max_iterations, iterations, workspace, workspace_bytes, stream);
}

LB_API lb_status_t lb_spmm(const lb_csr_t *A, const void *X, lb_dtype_t x_dtype, int32_t k, int64_t ldx, float *Y,
                           int64_t ldy, const lb_schedule_t *s, void *workspace, size_t workspace_bytes,
                           void *stream) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (k < 1 || k > kMaxK || ldx < k || ldy < k) return LB_ERR_INVALID_ARG;
    if (A->rows > 0 && !Y) return LB_ERR_INVALID_ARG;
    if (A->nnz > 0 && !X) return LB_ERR_INVALID_ARG;
    if (x_dtype != A->value_dtype) return LB_ERR_UNSUPPORTED;
    if (A->cols * ldx > (int64_t(1) << 40) || A->rows * ldy > (int64_t(1) << 40)) return LB_ERR_OVERFLOW;
    lb_schedule_t r;
    st = resolve(A, k, s, &r);
    if (st != LB_OK) return st;
    if (r.kind == LB_GROUP_MAPPED || r.kind == LB_WORK_QUEUE || one_band(r) != LB_OK) return LB_ERR_UNSUPPORTED;
    const size_t need = ws_bytes_for(A, r, k);
    if (need > 0 && (workspace_bytes < need || !workspace)) return LB_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (A->rows == 0) return LB_OK;
    const lbk::csr_dev d = to_dev(A);
    if (A->nnz == 0) {
        if (ldy == k) return hip_status(lbk::fill_f32(Y, A->rows * k, 0.f, hs));
        // strided Y: use the thread-mapped kernel, which writes every (row, col) (rows are empty)
        return hip_status(lbk::thread_mapped_spmm(d, X, k, ldx, Y, ldy, kDefaultBlock, 0, hs));
    }
    if (r.kind == LB_THREAD_MAPPED)
        return hip_status(lbk::thread_mapped_spmm(d, X, k, ldx, Y, ldy, r.block_size, r.grid_size, hs));
    return hip_status(lbk::merge_spmm(d, X, k, ldx, Y, ldy, r.block_size, r.items_per_thread, workspace, hs));
}

LB_API lb_status_t lb_spmv_backward(const lb_csr_t *A, const void *x, lb_dtype_t x_dtype, const float *dy, float *dx,
                                    float *dvalues, const lb_schedule_t *s, void *workspace, size_t workspace_bytes,
                                    void *stream) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (A->rows > 0 && A->nnz > 0 && !dy && (dx || dvalues)) return LB_ERR_INVALID_ARG;
    if (dvalues && A->nnz > 0 && !x) return LB_ERR_INVALID_ARG;
    if (x_dtype != A->value_dtype) return LB_ERR_UNSUPPORTED;
    lb_schedule_t in = s ? *s : lb_schedule_t{LB_MERGE_PATH, 0, 0, 0, 0, 0};
    if (in.kind == LB_AUTO) in.kind = LB_MERGE_PATH;
    if (in.kind != LB_MERGE_PATH) return LB_ERR_UNSUPPORTED;
    lb_schedule_t r;
    st = fill_defaults(&in, &r);
    if (st != LB_OK) return st;
    if (one_band(r) != LB_OK) return LB_ERR_UNSUPPORTED;
    const size_t need = ws_bytes_for(A, r, 0);
    if (workspace_bytes < need || !workspace) return LB_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (dx) {
        hipError_t e = lbk::fill_f32(dx, A->cols, 0.f, hs);
        if (e != hipSuccess) return hip_status(e);
    }
    if (A->nnz == 0 || (!dx && !dvalues)) return LB_OK;
    const lbk::csr_dev d = to_dev(A);
    return hip_status(lbk::merge_backward(d, x, dy, dx, dvalues, r.block_size, r.items_per_thread, workspace, hs));
}

// ------------------------------------------------------------------ batched

static lb_status_t check_batch(const lb_batch_t *B) {
    if (!B) return LB_ERR_INVALID_ARG;
    if (B->count < 0 || B->total_rows < 0 || B->total_cols < 0 || B->total_nnz < 0) return LB_ERR_INVALID_ARG;
    if (B->count > 0 && (!B->mat_row_base || !B->mat_nnz_base || !B->mat_col_base)) return LB_ERR_INVALID_ARG;
    if (B->total_rows > 0 && !B->row_offsets) return LB_ERR_INVALID_ARG;
    if (B->total_nnz > 0 && (!B->col_idx || !B->values)) return LB_ERR_INVALID_ARG;
    if (B->total_nnz > 0 && (B->total_rows == 0 || B->total_cols == 0)) return LB_ERR_INVALID_ARG;
    if (B->value_dtype != LB_F32 && B->value_dtype != LB_BF16 && B->value_dtype != LB_F64) return LB_ERR_INVALID_ARG;
    if (!dtype_built(B->value_dtype)) return LB_ERR_UNSUPPORTED;
    if (B->total_rows + B->total_nnz > kMaxCoord || B->total_cols > kMaxCoord || B->count > kMaxCoord)
        return LB_ERR_OVERFLOW;
    return LB_OK;
}

static lbk::batch_dev to_dev(const lb_batch_t *B) {
    lbk::batch_dev d;
    d.count = static_cast<int32_t>(B->count);
    d.total_rows = static_cast<int32_t>(B->total_rows);
    d.total_cols = static_cast<int32_t>(B->total_cols);
    d.total_nnz = static_cast<int32_t>(B->total_nnz);
    d.ro = B->row_offsets;
    d.ci = B->col_idx;
    d.val = B->values;
    d.dt = B->value_dtype;
    d.row_base = B->mat_row_base;
    d.nnz_base = B->mat_nnz_base;
    d.col_base = B->mat_col_base;
    return d;
}

static lb_status_t resolve_batched(const lb_batch_t *B, int32_t k, const lb_schedule_t *s, lb_schedule_t *out) {
    lb_schedule_t in = s ? *s : lb_schedule_t{LB_AUTO, 0, 0, 0, 0, 0};
    if (in.kind == LB_AUTO) {
        lb_schedule_t tuned;
        const tune_key key{B->total_rows, B->total_cols, B->total_nnz, k, static_cast<int32_t>(B->value_dtype), 1, 0};
        const bind_key b{B->row_offsets, B->col_idx, B->total_rows, B->total_cols, B->total_nnz, 1};
        if (tune_lookup_bound(b, key, &tuned))
            in = tuned;
        else
            in = lb_schedule_t{LB_MERGE_PATH, 0, 0, 0, 0, 0};
    }
    if (in.kind != LB_MERGE_PATH) return LB_ERR_UNSUPPORTED;
    const lb_status_t st = fill_defaults(&in, out);
    return st != LB_OK ? st : one_band(*out);
}

LB_API lb_status_t lb_batched_workspace_size(const lb_batch_t *B, const lb_schedule_t *s, int32_t k, size_t *bytes) {
    if (!bytes || k < 1 || k > kMaxK) return LB_ERR_INVALID_ARG;
    lb_status_t st = check_batch(B);
    if (st != LB_OK) return st;
    lb_schedule_t r;
    st = resolve_batched(B, k, s, &r);
    if (st != LB_OK) return st;
    *bytes = lbk::batched_ws_bytes(to_dev(B), r.block_size, r.items_per_thread, k);
    return LB_OK;
}

LB_API lb_status_t lb_batched_spmm(const lb_batch_t *B, const void *X, lb_dtype_t x_dtype, int32_t k, float *Y,
                                   const lb_schedule_t *s, void *workspace, size_t workspace_bytes, void *stream) {
    lb_status_t st = check_batch(B);
    if (st != LB_OK) return st;
    if (k < 1 || k > kMaxK) return LB_ERR_INVALID_ARG;
    if (B->total_rows > 0 && !Y) return LB_ERR_INVALID_ARG;
    if (B->total_nnz > 0 && !X) return LB_ERR_INVALID_ARG;
    if (x_dtype != B->value_dtype) return LB_ERR_UNSUPPORTED;
    lb_schedule_t r;
    st = resolve_batched(B, k, s, &r);
    if (st != LB_OK) return st;
    const lbk::batch_dev d = to_dev(B);
    const size_t need = lbk::batched_ws_bytes(d, r.block_size, r.items_per_thread, k);
    if (need > 0 && (workspace_bytes < need || !workspace)) return LB_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (B->total_rows == 0) return LB_OK;
    if (B->total_nnz == 0) return hip_status(lbk::fill_f32(Y, B->total_rows * k, 0.f, hs));
    return hip_status(lbk::batched_spmm(d, X, k, Y, r.block_size, r.items_per_thread, workspace, hs));
}

// ------------------------------------------------------------------ test hooks

LB_API lb_status_t lb_merge_path_partition(const int32_t *row_offsets, int64_t rows, int64_t nnz,
                                           int64_t items_per_unit, int64_t num_units, int32_t *out_row,
                                           int32_t *out_nz, void *stream) {
    if (rows < 0 || nnz < 0 || items_per_unit < 1 || num_units < 0) return LB_ERR_INVALID_ARG;
    if (!row_offsets || !out_row || !out_nz) return LB_ERR_INVALID_ARG;
    if (rows + nnz > kMaxCoord || items_per_unit > kMaxCoord || num_units > kMaxCoord) return LB_ERR_OVERFLOW;
    return hip_status(lbk::merge_partition(row_offsets, static_cast<int32_t>(rows), static_cast<int32_t>(nnz),
                                           static_cast<int32_t>(items_per_unit), static_cast<int32_t>(num_units),
                                           out_row, out_nz, static_cast<hipStream_t>(stream)));
}

LB_API lb_status_t lb_group_tile_owner(const lb_csr_t *A, int32_t tiles_per_group, int32_t *owner, void *stream) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (!is_pow2(tiles_per_group) || tiles_per_group < 2 || tiles_per_group > 1024) return LB_ERR_INVALID_ARG;
    if (A->nnz > 0 && !owner) return LB_ERR_INVALID_ARG;
    if (A->rows == 0 || A->nnz == 0) return LB_OK;
    return hip_status(lbk::group_tile_owner(to_dev(A), tiles_per_group, owner, static_cast<hipStream_t>(stream)));
}

static __device__ int32_t g_validate_flags;

LB_API lb_status_t lb_validate_csr(const lb_csr_t *A, void *stream) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (!A->row_offsets) return LB_ERR_INVALID_ARG;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    int32_t *flags = nullptr;
    hipError_t e = hipGetSymbolAddress(reinterpret_cast<void **>(&flags), HIP_SYMBOL(g_validate_flags));
    if (e != hipSuccess) return hip_status(e);
    int32_t zero = 0, host = 0;
    e = hipMemcpyAsync(flags, &zero, sizeof zero, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = lbk::validate_csr(to_dev(A), flags, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(&host, flags, sizeof host, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return hip_status(e);
    return host ? LB_ERR_INVALID_CSR : LB_OK;
}

// ------------------------------------------------------------------ autotune

LB_API lb_status_t lb_autotune_workspace_size(const lb_csr_t *A, int32_t k, size_t *bytes) {
    if (!bytes || k < 1 || k > kMaxK) return LB_ERR_INVALID_ARG;
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    // the largest candidate workspace: the smallest merge-path unit, or the
    // two-band candidates' (units of at least 2048 items, plus a rows buffer)
    const int64_t T = lbk::merge_units(A->rows, A->nnz, 128 * 4);
    const size_t one = lbk::merge_ws_bytes(T, spmm_pass_cols(k));
    const size_t two = k == 1 ? lbk::merge_banded_ws_bytes(lbk::merge_units(A->rows, A->nnz, 2048), A->rows) : 0;
    *bytes = one > two ? one : two;
    return LB_OK;
}


LB_API lb_status_t lb_autotune(const lb_csr_t *A, const void *X, lb_dtype_t x_dtype, int32_t k, float *Y,
                               void *workspace, size_t workspace_bytes, lb_schedule_t *best, void *stream) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (!best || k < 1 || k > kMaxK) return LB_ERR_INVALID_ARG;
    size_t need = 0;
    lb_autotune_workspace_size(A, k, &need);
    if (workspace_bytes < need || !workspace) return LB_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    uint64_t fp = 0;
    st = fingerprint(A->rows, A->cols, A->nnz, A->row_offsets, A->col_idx, nullptr, 0, hs, &fp);
    if (st != LB_OK) return st;
    // The Sec. 6.2 pick with default parameters is the incumbent; a candidate
    // replaces it only if it is more than 2 % faster, so timing noise does
    // not flip the choice between equivalent configurations.
    lb_schedule_t best_s = heuristic(A);
    fill_defaults(&best_s, &best_s);
    float best_ms = 1e30f;
    {
        auto run0 = [&]() -> lb_status_t {
            if (k == 1) return lb_spmv(A, X, x_dtype, Y, &best_s, workspace, workspace_bytes, stream);
            return lb_spmm(A, X, x_dtype, k, k, Y, k, &best_s, workspace, workspace_bytes, stream);
        };
        st = time_call(run0, hs, &best_ms);
        if (st == LB_ERR_HIP) return st;
        if (st != LB_OK) best_ms = 1e30f;
        else best_ms *= 0.98f;
    }
    for (const lb_schedule_t &c : candidates(A, k)) {
        float ms = 0.f;
        auto run = [&]() -> lb_status_t {
            if (k == 1) return lb_spmv(A, X, x_dtype, Y, &c, workspace, workspace_bytes, stream);
            return lb_spmm(A, X, x_dtype, k, k, Y, k, &c, workspace, workspace_bytes, stream);
        };
        st = time_call(run, hs, &ms);
        if (st == LB_ERR_HIP) return st;
        if (st != LB_OK) continue;
        if (ms < best_ms) {
            best_ms = ms;
            fill_defaults(&c, &best_s);
        }
    }
    tune_store(tune_key{A->rows, A->cols, A->nnz, k, static_cast<int32_t>(A->value_dtype), 0, fp}, best_s);
    tune_bind(bind_key{A->row_offsets, A->col_idx, A->rows, A->cols, A->nnz, 0}, fp);
    *best = best_s;
    return LB_OK;
}

LB_API lb_status_t lb_batched_autotune(const lb_batch_t *B, const void *X, lb_dtype_t x_dtype, int32_t k, float *Y,
                                       void *workspace, size_t workspace_bytes, lb_schedule_t *best, void *stream) {
    lb_status_t st = check_batch(B);
    if (st != LB_OK) return st;
    if (!best || k < 1 || k > kMaxK) return LB_ERR_INVALID_ARG;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    uint64_t fp = 0;
    const int64_t *bases[3] = {B->mat_row_base, B->mat_nnz_base, B->mat_col_base};
    st = fingerprint(B->total_rows, B->total_cols, B->total_nnz, B->row_offsets, B->col_idx, bases, B->count, hs,
                     &fp);
    if (st != LB_OK) return st;
    float best_ms = 1e30f;
    lb_schedule_t best_s{};
    bool any = false;
    for (int b : {128, 256, 512}) {
        for (int it : {4, 8, 12, 16}) {
            const lb_schedule_t c{LB_MERGE_PATH, 0, 0, it, b, 0};
            size_t need = 0;
            if (lb_batched_workspace_size(B, &c, k, &need) != LB_OK || need > workspace_bytes) continue;
            float ms = 0.f;
            auto run = [&]() -> lb_status_t {
                return lb_batched_spmm(B, X, x_dtype, k, Y, &c, workspace, workspace_bytes, stream);
            };
            st = time_call(run, hs, &ms);
            if (st == LB_ERR_HIP) return st;
            if (st != LB_OK) continue;
            if (ms < best_ms) {
                best_ms = ms;
                fill_defaults(&c, &best_s);
                any = true;
            }
        }
    }
    if (!any) return LB_ERR_WORKSPACE_TOO_SMALL;
    tune_store(tune_key{B->total_rows, B->total_cols, B->total_nnz, k, static_cast<int32_t>(B->value_dtype), 1, fp},
               best_s);
    tune_bind(bind_key{B->row_offsets, B->col_idx, B->total_rows, B->total_cols, B->total_nnz, 1}, fp);
    *best = best_s;
    return LB_OK;
}

LB_API void lb_autotune_clear(void) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune.clear();
    g_bind.clear();
    g_tune_loaded = true;  // do not reload the file after an explicit clear
}

LB_API lb_status_t lb_pattern_fingerprint(const lb_csr_t *A, uint64_t *fp, void *stream) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (!fp) return LB_ERR_INVALID_ARG;
    return fingerprint(A->rows, A->cols, A->nnz, A->row_offsets, A->col_idx, nullptr, 0,
                       static_cast<hipStream_t>(stream), fp);
}

LB_API lb_status_t lb_autotune_lookup(const lb_csr_t *A, int32_t k, uint64_t fp, int32_t *found, lb_schedule_t *out) {
    lb_status_t st = check_csr(A);
    if (st != LB_OK) return st;
    if (!found || !out || k < 1 || k > kMaxK) return LB_ERR_INVALID_ARG;
    tune_bind(bind_key{A->row_offsets, A->col_idx, A->rows, A->cols, A->nnz, 0}, fp);
    lb_schedule_t s{};
    *found = tune_lookup(tune_key{A->rows, A->cols, A->nnz, k, static_cast<int32_t>(A->value_dtype), 0, fp}, &s);
    if (*found) *out = s;
    return LB_OK;
}

LB_API const char *lb_autotune_device_tag(void) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    return device_tag_locked().c_str();
}

// ------------------------------------------------------------------ measurement probes

LB_API int32_t lb_probe_default_grid(void) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus * 8;
}

LB_API lb_status_t lb_probe_stream_read(const void *buf, size_t bytes, float *out, int32_t grid, void *stream) {
    if (!buf || !out || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(buf) % 16 != 0 || grid < 0)
        return LB_ERR_INVALID_ARG;
    if (bytes == 0) return LB_OK;
    if (grid == 0) grid = lb_probe_default_grid();
    return hip_status(lbk::probe_stream_read(buf, bytes, out, grid, static_cast<hipStream_t>(stream)));
}

LB_API lb_status_t lb_probe_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0 ||
        reinterpret_cast<uintptr_t>(dst) % 16 != 0)
        return LB_ERR_INVALID_ARG;
    const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
    if (bytes > 0 && a < b + bytes && b < a + bytes) return LB_ERR_INVALID_ARG;  // overlapping
    if (bytes == 0) return LB_OK;
    return hip_status(lbk::probe_copy(src, dst, bytes, static_cast<hipStream_t>(stream)));
}

LB_API lb_status_t lb_probe_gather(const int32_t *idx, int64_t n, const float *x, int64_t cols, float *out,
                                   int32_t grid, int32_t bands, void *stream) {
    if (n < 0 || cols < 0 || grid < 0 || !out || (n > 0 && (!idx || !x || cols == 0))) return LB_ERR_INVALID_ARG;
    if (bands != 1 && bands != 2 && bands != 4 && bands != 8) return LB_ERR_INVALID_ARG;
    if (cols > kMaxCoord) return LB_ERR_OVERFLOW;
    if (n == 0) return LB_OK;
    if (grid == 0) grid = lb_probe_default_grid();
    if (bands > 1) grid = grid < 8 ? 8 : grid / 8 * 8;
    return hip_status(lbk::probe_gather(idx, n, x, static_cast<int32_t>((cols + bands - 1) / bands), out, grid, bands,
                                        static_cast<hipStream_t>(stream)));
}

// ------------------------------------------------------------------ profiling

LB_API void lb_profile_enable(int on) { g_prof_on = on != 0; }

LB_API void lb_profile_reset(void) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (auto &r : g_prof) {
        (void)hipEventSynchronize(r.closed ? r.stop : r.start);
        (void)hipEventDestroy(r.start);
        if (r.closed) (void)hipEventDestroy(r.stop);
    }
    g_prof.clear();
}

LB_API lb_status_t lb_profile_read(const char *name, double *total_ms, int64_t *launches) {
    if (!name || !total_ms || !launches) return LB_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(g_prof_mu);
    double t = 0.0;
    int64_t n = 0;
    for (auto &r : g_prof) {
        if (!r.closed || r.name != name) continue;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e != hipSuccess) return hip_status(e);
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (e != hipSuccess) return hip_status(e);
        t += ms;
        ++n;
    }
    *total_ms = t;
    *launches = n;
    return LB_OK;
}

}  // extern "C"
