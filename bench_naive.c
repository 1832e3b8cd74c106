/*
 * bench_naive.c -- the CPU comparison point of the benchmark: the step's
 * operations written as plain double-precision loops (scaled vector addition,
 * inner product, norm, matrix-vector product in both storage layouts),
 * parallelised over the host's cores with OpenMP and left for the compiler to
 * vectorise.  It is neither the parity reference nor part of the library:
 * its reductions are ordinary float64 sums in whatever order the threads and
 * vector lanes take, so their results differ from the oracle's by rounding.
 * bench.py loads it through ctypes and times it on the same inputs as the
 * GPU step.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>

int naive_max_threads(void) { return omp_get_max_threads(); }

void naive_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }

/* x = a y + b z */
void naive_axpby(int64_t n, double a, const double *y, double b, const double *z, double *x)
{
#pragma omp parallel for simd schedule(static)
    for (int64_t i = 0; i < n; ++i)
        x[i] = a * y[i] + b * z[i];
}

/* sum x_i y_i */
double naive_dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
#pragma omp parallel for simd reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; ++i)
        s += x[i] * y[i];
    return s;
}

/* sqrt(sum x_i^2) */
double naive_nrm2(int64_t n, const double *x)
{
    double s = 0.0;
#pragma omp parallel for simd reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; ++i)
        s += x[i] * x[i];
    return sqrt(s);
}

/* y = A x, A m x n row-major with leading dimension lda: one row per
 * iteration, rows shared out among the threads. */
void naive_gemv_row(int64_t m, int64_t n, const double *A, int64_t lda, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        const double *a = A + i * lda;
        double s = 0.0;
#pragma omp simd reduction(+ : s)
        for (int64_t j = 0; j < n; ++j)
            s += a[j] * x[j];
        y[i] = s;
    }
}

/* y = A x, A m x n column-major with leading dimension lda: y is built as
 * the sum of x_j times column j, each thread owning a block of rows of y and
 * walking every column over that block. */
void naive_gemv_col(int64_t m, int64_t n, const double *A, int64_t lda, const double *x, double *y)
{
#pragma omp parallel
    {
        const int64_t t = omp_get_thread_num(), nt = omp_get_num_threads();
        const int64_t i0 = m * t / nt, i1 = m * (t + 1) / nt;
        for (int64_t i = i0; i < i1; ++i)
            y[i] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double xj = x[j];
            const double *a = A + j * lda;
#pragma omp simd
            for (int64_t i = i0; i < i1; ++i)
                y[i] += xj * a[i];
        }
    }
}
