/*
 * FP64 CPU oracle for load-balanced CSR SpMV -- TEST INFRASTRUCTURE ONLY.
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
 *
 * All sums are plain sequential loops in ascending nonzero order, in double.
 * Inputs are read in the same storage type the GPU reads (float32, or BF16
 * bit patterns) and widened exactly to double.
 */
#include <stdint.h>
#include <stddef.h>
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
