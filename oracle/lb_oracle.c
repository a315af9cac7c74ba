/*
 * CPU oracle for the load-balanced sparse kernels -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the bench's CPU-baseline leg may
 * load this library.  It shares no code, header or constant with the GPU
 * library; it is written from the paper's definitions (Osama, Porumbescu,
 * Owens, "A Programming Model for GPU Load Balancing", PPoPP'23):
 *
 *   - SpMV (Sec. 1 problem statement; Sec. 4.3 SpMV listing): for each row
 *     (tile) r, y[r] is the sum over its nonzeros (atoms) j in
 *     [row_offsets[r], row_offsets[r+1]) of values[j] * x[col_idx[j]]; an
 *     empty row yields 0 and y is overwritten, not accumulated.
 *   - SpMM (Sec. 5.3 SpMM listing): the same sum for every column of a dense
 *     right-hand side.  The printed listing indexes B with the nonzero's
 *     position; the only meaningful reading is B(col_idx[nz], col).
 *   - Merge-path split (Sec. 5.2.1): row ends and nonzeros are equal units
 *     of work; the walk consumes row end r when row_offsets[r+1] <= j (the
 *     nonzero at index row_offsets[r+1] belongs to the next row), else
 *     nonzero j.  Recorded at diagonals d_t = min(t*W, m + nnz).
 *   - Backward of y = A x (not in the paper): dx = A^T dy,
 *     dvalues[j] = dy[row(j)] * x[col_idx[j]].
 *   - COO and CSC SpMV (Sec. 3.1 names both among the library's formats):
 *     the same y = A x, the matrix given per entry (COO) or per column (CSC).
 *   - SpGEMM C = A B (Gustavson; Sec. 5.3 names it as an extension):
 *     structural union of each row's products, columns ascending, values in
 *     double.
 *   - SSSP (Sec. 5.3, the graph example) and BFS (named in Sec. 6) on the
 *     same tile sets: vertices are tiles, out-edges are atoms.  Distances
 *     are float32 as in the paper's example; see orc_sssp.
 *
 * All SpMV-family sums are plain sequential loops in ascending nonzero
 * order, in double.
 * Inputs are read in the same storage type the GPU reads (float32, or BF16
 * bit patterns) and widened exactly to double.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define ORC_F32 0
#define ORC_BF16 1
#define ORC_F64 2

/* Exact widening of one stored element to double. */
static double orc_load(const void *p, int dtype, int64_t i)
{
    if (dtype == ORC_F32)
        return (double)((const float *)p)[i];
    if (dtype == ORC_BF16) {
        /* a BF16 value is the upper 16 bits of an IEEE binary32 */
        uint32_t bits = (uint32_t)((const uint16_t *)p)[i] << 16;
        float f;
        memcpy(&f, &bits, sizeof f);
        return (double)f;
    }
    return ((const double *)p)[i];
}

static int orc_dtype_ok(int dt) { return dt == ORC_F32 || dt == ORC_BF16 || dt == ORC_F64; }

int orc_abi_version(void) { return 1; }

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the parallel loops below use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the thread count of the parallel loops (timing only: every result is
 * the same for any count, each row being summed by one thread in order). */
int orc_set_num_threads(int n)
{
    if (n < 1) return 1;
#ifdef _OPENMP
    omp_set_num_threads(n);
#endif
    return 0;
}

/* y[r] = sum_j values[j] * x[col_idx[j]] over row r; optionally with |.| of
 * every term (abs_terms != 0), which gives the per-row tolerance scale. */
int orc_spmv(int64_t m, const int32_t *row_offsets, const int32_t *col_idx,
             const void *values, int vdt, const void *x, int xdt, int abs_terms,
             double *y)
{
    if (m < 0 || !orc_dtype_ok(vdt) || !orc_dtype_ok(xdt)) return 1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r) {
        double sum = 0.0;
        for (int64_t j = row_offsets[r]; j < row_offsets[r + 1]; ++j) {
            double t = orc_load(values, vdt, j) * orc_load(x, xdt, col_idx[j]);
            sum += abs_terms ? (t < 0 ? -t : t) : t;
        }
        y[r] = sum;
    }
    return 0;
}

/* Y[r, c] = sum_j values[j] * X[col_idx[j], c] for c in [0, k); X is
 * row-major with leading dimension ldx, Y with ldy. */
int orc_spmm(int64_t m, const int32_t *row_offsets, const int32_t *col_idx,
             const void *values, int vdt, const void *X, int xdt, int64_t k,
             int64_t ldx, int abs_terms, double *Y, int64_t ldy)
{
    if (m < 0 || k < 0 || !orc_dtype_ok(vdt) || !orc_dtype_ok(xdt)) return 1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < m; ++r) {
        for (int64_t c = 0; c < k; ++c) {
            double sum = 0.0;
            for (int64_t j = row_offsets[r]; j < row_offsets[r + 1]; ++j) {
                double t = orc_load(values, vdt, j) * orc_load(X, xdt, (int64_t)col_idx[j] * ldx + c);
                sum += abs_terms ? (t < 0 ? -t : t) : t;
            }
            Y[r * ldy + c] = sum;
        }
    }
    return 0;
}

/* dx[c] = sum over nonzeros j with col_idx[j] == c of values[j] * dy[row(j)]
 * (the transpose product), visiting rows in ascending order.  dy is double. */
int orc_spmv_transpose(int64_t m, int64_t n, const int32_t *row_offsets,
                       const int32_t *col_idx, const void *values, int vdt,
                       const double *dy, int abs_terms, double *dx)
{
    if (m < 0 || n < 0 || !orc_dtype_ok(vdt)) return 1;
    for (int64_t c = 0; c < n; ++c) dx[c] = 0.0;
    for (int64_t r = 0; r < m; ++r) {
        for (int64_t j = row_offsets[r]; j < row_offsets[r + 1]; ++j) {
            double t = orc_load(values, vdt, j) * dy[r];
            dx[col_idx[j]] += abs_terms ? (t < 0 ? -t : t) : t;
        }
    }
    return 0;
}

/* dvalues[j] = dy[row(j)] * x[col_idx[j]], one product per nonzero. */
int orc_dvalues(int64_t m, const int32_t *row_offsets, const int32_t *col_idx,
                const double *dy, const void *x, int xdt, double *dvalues)
{
    if (m < 0 || !orc_dtype_ok(xdt)) return 1;
    for (int64_t r = 0; r < m; ++r)
        for (int64_t j = row_offsets[r]; j < row_offsets[r + 1]; ++j)
            dvalues[j] = dy[r] * orc_load(x, xdt, col_idx[j]);
    return 0;
}

/* Walk the merge of the row-end list (row_offsets[1..m]) with the nonzero
 * index list (0..nnz-1) one step at a time and record, at every diagonal
 * d_t = min(t * W, m + nnz) for t in [0, T], how many row ends (out_i) and
 * nonzeros (out_j) precede it. */
int orc_merge_walk(int64_t m, int64_t nnz, const int32_t *row_offsets, int64_t W,
                   int64_t T, int32_t *out_i, int32_t *out_j)
{
    if (m < 0 || nnz < 0 || W <= 0 || T < 0) return 1;
    int64_t total = m + nnz;
    int64_t i = 0, j = 0, d = 0;
    for (int64_t t = 0; t <= T; ++t) {
        int64_t target = t * W < total ? t * W : total;
        while (d < target) {
            if (i < m && row_offsets[i + 1] <= j)
                ++i;          /* row end i comes first (ties included) */
            else
                ++j;          /* nonzero j */
            ++d;
        }
        out_i[t] = (int32_t)i;
        out_j[t] = (int32_t)j;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Graph traversal on the same CSR tile sets (Sec. 5.3, the SSSP example;
 * Sec. 6 names BFS as another application built on the schedules).
 * Vertices are tiles (rows) and a vertex's out-edges are its atoms: edge j
 * of vertex u goes to col_idx[j] with weight w[j].
 * ------------------------------------------------------------------------ */

/* Single-source shortest paths.  The paper's SSSP offers, along every edge
 * (u, v, w), the distance dist[u] + w to v and keeps the smaller value,
 * repeating until nothing changes.  Distances are float32 (the example
 * declares them float), so every offer is one float32 addition and the
 * result is the least solution of
 *     dist[source] = 0,  dist[v] = min over edges (u, v, w) of fl(dist[u] + w)
 * (+inf where no path exists).  With w >= 0 an offer is never below
 * dist[u] and fl(a + w) does not decrease as a grows, so settling vertices
 * in increasing distance (Dijkstra) reaches exactly that solution.  Binary
 * heap with lazy deletion: a vertex may be pushed once per improvement and
 * stale heap entries are skipped when popped.
 * Returns 1 for bad sizes, 2 for a negative or NaN weight. */
typedef struct {
    float d;
    int32_t v;
} orc_heap_item;

static void orc_heap_push(orc_heap_item *h, int64_t *size, float d, int32_t v)
{
    int64_t i = (*size)++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= d) break;
        h[i] = h[p];
        i = p;
    }
    h[i].d = d;
    h[i].v = v;
}

static orc_heap_item orc_heap_pop(orc_heap_item *h, int64_t *size)
{
    orc_heap_item top = h[0];
    int64_t n = --(*size);
    if (n > 0) {
        orc_heap_item last = h[n];
        int64_t i = 0;
        for (;;) {
            int64_t c = 2 * i + 1;
            if (c >= n) break;
            if (c + 1 < n && h[c + 1].d < h[c].d) ++c;
            if (h[c].d >= last.d) break;
            h[i] = h[c];
            i = c;
        }
        h[i] = last;
    }
    return top;
}

int orc_sssp(int64_t n, const int32_t *row_offsets, const int32_t *col_idx,
             const float *w, int64_t source, float *dist)
{
    if (n <= 0 || source < 0 || source >= n) return 1;
    int64_t E = row_offsets[n];
    for (int64_t j = 0; j < E; ++j)
        if (!(w[j] >= 0.0f)) return 2;
    for (int64_t v = 0; v < n; ++v) dist[v] = INFINITY;
    orc_heap_item *heap = (orc_heap_item *)malloc((size_t)(E + 1) * sizeof *heap);
    unsigned char *settled = (unsigned char *)calloc((size_t)n, 1);
    if (!heap || !settled) {
        free(heap);
        free(settled);
        return 3;
    }
    int64_t size = 0;
    dist[source] = 0.0f;
    orc_heap_push(heap, &size, 0.0f, (int32_t)source);
    while (size > 0) {
        orc_heap_item top = orc_heap_pop(heap, &size);
        int32_t u = top.v;
        if (settled[u]) continue; /* a stale entry */
        settled[u] = 1;
        for (int64_t j = row_offsets[u]; j < row_offsets[u + 1]; ++j) {
            int32_t v = col_idx[j];
            float offer = dist[u] + w[j]; /* one float32 addition */
            if (offer < dist[v]) {
                dist[v] = offer;
                orc_heap_push(heap, &size, offer, v);
            }
        }
    }
    free(heap);
    free(settled);
    return 0;
}

/* Breadth-first search: depth[v] is the least number of edges on a path
 * from source to v, -1 if there is none.  FIFO queue, one visit per vertex. */
int orc_bfs(int64_t n, const int32_t *row_offsets, const int32_t *col_idx,
            int64_t source, int32_t *depth)
{
    if (n <= 0 || source < 0 || source >= n) return 1;
    int32_t *queue = (int32_t *)malloc((size_t)n * sizeof *queue);
    if (!queue) return 3;
    for (int64_t v = 0; v < n; ++v) depth[v] = -1;
    int64_t head = 0, tail = 0;
    depth[source] = 0;
    queue[tail++] = (int32_t)source;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t j = row_offsets[u]; j < row_offsets[u + 1]; ++j) {
            int32_t v = col_idx[j];
            if (depth[v] < 0) {
                depth[v] = depth[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    return 0;
}

/* ------------------------------------------------------------------------
 * Other tile sets (Sec. 3.1 lists COO and CSC among the library's formats;
 * Sec. 5.2.1: merge-path needs only an iterator counting atoms per tile).
 * ------------------------------------------------------------------------ */

/* COO sorted by row: nonzero j is (row_idx[j], col_idx[j], values[j]).
 * y[r] = sum over j with row_idx[j] == r of values[j] * x[col_idx[j]], in
 * ascending j (the CSR sum of the same matrix); rows without entries are 0. */
int orc_spmv_coo(int64_t m, int64_t nnz, const int32_t *row_idx, const int32_t *col_idx,
                 const void *values, int vdt, const void *x, int xdt, int abs_terms, double *y)
{
    if (m < 0 || nnz < 0 || !orc_dtype_ok(vdt) || !orc_dtype_ok(xdt)) return 1;
    for (int64_t r = 0; r < m; ++r) y[r] = 0.0;
    for (int64_t j = 0; j < nnz; ++j) {
        double t = orc_load(values, vdt, j) * orc_load(x, xdt, col_idx[j]);
        y[row_idx[j]] += abs_terms ? (t < 0 ? -t : t) : t;
    }
    return 0;
}

/* CSC: column c's nonzeros are [col_offsets[c], col_offsets[c+1]), with rows
 * row_idx[j].  y[r] = sum over the nonzeros of row r of values[j] * x[c],
 * visiting columns in ascending order. */
int orc_spmv_csc(int64_t m, int64_t n, const int32_t *col_offsets, const int32_t *row_idx,
                 const void *values, int vdt, const void *x, int xdt, int abs_terms, double *y)
{
    if (m < 0 || n < 0 || !orc_dtype_ok(vdt) || !orc_dtype_ok(xdt)) return 1;
    for (int64_t r = 0; r < m; ++r) y[r] = 0.0;
    for (int64_t c = 0; c < n; ++c) {
        double xc = orc_load(x, xdt, c);
        for (int64_t j = col_offsets[c]; j < col_offsets[c + 1]; ++j) {
            double t = orc_load(values, vdt, j) * xc;
            y[row_idx[j]] += abs_terms ? (t < 0 ? -t : t) : t;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Sparse matrix-matrix product C = A B (Gustavson; Sec. 5.3 names it as an
 * extension: size each output row, allocate, multiply).  A is m x k, B is
 * k x n, both CSR.  Row i of C holds every column c reached by a product
 * A[i, j] * B[j, c] (structurally, even when the sum is 0), in ascending
 * order, with value sum over j of A[i, j] * B[j, c] in double (products in
 * ascending A entry, then ascending B entry).  Dense accumulator per row.
 * ------------------------------------------------------------------------ */

static int orc_cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Pass 1: c_row_offsets[m + 1] (entries per row, prefix-summed). */
int orc_spgemm_count(int64_t m, int64_t n, const int32_t *a_ro, const int32_t *a_ci,
                     const int32_t *b_ro, const int32_t *b_ci, int64_t *c_ro)
{
    if (m < 0 || n < 0) return 1;
    unsigned char *seen = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t *list = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof *list);
    if (!seen || !list) {
        free(seen);
        free(list);
        return 3;
    }
    c_ro[0] = 0;
    for (int64_t i = 0; i < m; ++i) {
        int64_t cnt = 0;
        for (int64_t e = a_ro[i]; e < a_ro[i + 1]; ++e) {
            int32_t j = a_ci[e];
            for (int64_t f = b_ro[j]; f < b_ro[j + 1]; ++f) {
                int32_t c = b_ci[f];
                if (!seen[c]) {
                    seen[c] = 1;
                    list[cnt++] = c;
                }
            }
        }
        for (int64_t t = 0; t < cnt; ++t) seen[list[t]] = 0;
        c_ro[i + 1] = c_ro[i] + cnt;
    }
    free(seen);
    free(list);
    return 0;
}

/* Pass 2: columns (ascending) and values of every row; c_ro from pass 1.
 * With abs_terms, the values are sums of |A[i, j] * B[j, c]| (the scale of
 * the tolerance). */
int orc_spgemm_compute(int64_t m, int64_t n, const int32_t *a_ro, const int32_t *a_ci,
                       const void *a_val, int adt, const int32_t *b_ro, const int32_t *b_ci,
                       const void *b_val, int bdt, const int64_t *c_ro, int abs_terms,
                       int32_t *c_ci, double *c_val)
{
    if (m < 0 || n < 0 || !orc_dtype_ok(adt) || !orc_dtype_ok(bdt)) return 1;
    double *acc = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof *acc);
    unsigned char *seen = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!acc || !seen) {
        free(acc);
        free(seen);
        return 3;
    }
    for (int64_t i = 0; i < m; ++i) {
        int64_t cnt = 0;
        int32_t *cols = c_ci + c_ro[i];
        for (int64_t e = a_ro[i]; e < a_ro[i + 1]; ++e) {
            int32_t j = a_ci[e];
            double a = orc_load(a_val, adt, e);
            for (int64_t f = b_ro[j]; f < b_ro[j + 1]; ++f) {
                int32_t c = b_ci[f];
                double t = a * orc_load(b_val, bdt, f);
                acc[c] += abs_terms ? (t < 0 ? -t : t) : t;
                if (!seen[c]) {
                    seen[c] = 1;
                    if (c_ro[i] + cnt >= c_ro[i + 1]) {
                        free(acc);
                        free(seen);
                        return 4; /* c_ro does not match the product */
                    }
                    cols[cnt++] = c;
                }
            }
        }
        if (c_ro[i] + cnt != c_ro[i + 1]) {
            free(acc);
            free(seen);
            return 4;
        }
        qsort(cols, (size_t)cnt, sizeof *cols, orc_cmp_i32);
        for (int64_t t = 0; t < cnt; ++t) {
            c_val[c_ro[i] + t] = acc[cols[t]];
            acc[cols[t]] = 0.0;
            seen[cols[t]] = 0;
        }
    }
    free(acc);
    free(seen);
    return 0;
}
