/*
 * Oracle Laplacian product in plain C with OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU FP64 oracle.  It is loaded by
 * oracle/laplacian.py; the product library never links or calls it, and it
 * includes nothing from the product's sources.
 *
 * Paper: Sec. 3.2, Eq. 2 with weights: L_C = D - A, so for a block X
 *   (L_C X)_{i,c} = sum_j w_ij (x_{i,c} - x_{j,c}),
 * summed in difference form (a constant column maps to exactly zero).  The
 * entries of row i are taken in CSR order, one row per loop iteration, so the
 * result does not depend on the number of threads.
 */
#include <stdint.h>

/* Y = L_C X.  X and Y are n x m row-major FP64; w may be NULL (unit weights).
 * rowptr has n+1 int64 entries, col nnz int32 entries. */
void oracle_lap_apply(int64_t n, const int64_t *rowptr, const int32_t *col,
                      const double *w, const double *X, int64_t m, double *Y,
                      int threads)
{
    #pragma omp parallel for schedule(dynamic, 1024) num_threads(threads)
    for (int64_t i = 0; i < n; ++i) {
        const double *xi = X + i * m;
        double *yi = Y + i * m;
        for (int64_t c = 0; c < m; ++c)
            yi[c] = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const double *xj = X + (int64_t)col[k] * m;
            const double wk = w ? w[k] : 1.0;
            for (int64_t c = 0; c < m; ++c)
                yi[c] += wk * (xi[c] - xj[c]);
        }
    }
}

/* STREAM-style triad a = b + s c over n doubles (host bandwidth reference for
 * the oracle's product rate).  Returns nothing; the caller times it. */
void oracle_triad(int64_t n, double *a, const double *b, const double *c,
                  double s, int threads)
{
    #pragma omp parallel for schedule(static) num_threads(threads)
    for (int64_t i = 0; i < n; ++i)
        a[i] = b[i] + s * c[i];
}
