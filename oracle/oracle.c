/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the
 * bandwidth-limited linear algebra operations of Rupp, Tillet, Rudolf,
 * Weinbub, Grasser, Juengel, "Performance Portability Study of Linear Algebra
 * Kernels in OpenCL" (IWOCL 2014, arXiv:1409.0669).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity reference for the GPU
 * library.  It shares no code, header, table or helper with the GPU path and
 * is never linked into it.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.
 *
 * Conventions
 *  - Every array is double precision and holds the exact value of the stored
 *    element: f32 and bf16 inputs are widened exactly before they arrive here.
 *  - `prec` selects the precision in which a single-rounding operation is
 *    carried out: O_F64, O_F32, or O_BF16 (bf16 storage, f32 arithmetic, one
 *    final round-to-nearest-even to bf16).  f32 arithmetic is ordinary C float
 *    arithmetic (SSE, FLT_EVAL_METHOD == 0) and fmaf(); the file is compiled
 *    with -ffp-contract=off so no multiply-add is fused behind our back.
 *  - Reductions (inner product, norm, matrix-vector product) return the sum
 *    of exact products in double precision, evaluated with the compensated
 *    Dot2 algorithm of Ogita, Rump and Oishi ("Accurate sum and dot product",
 *    SIAM J. Sci. Comput. 26(6), 2005, Algorithm 5.3), whose result is as
 *    accurate as if it had been computed in twice the working precision and
 *    then rounded.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define O_F64 0
#define O_F32 1
#define O_BF16 2

#define O_ROW_MAJOR 0
#define O_COL_MAJOR 1

/* ---- rounding to bf16 ---------------------------------------------------
 * bf16 keeps the sign, the 8 exponent bits and the top 7 fraction bits of an
 * IEEE binary32 value.  Round to nearest, ties to even: add half an ulp of the
 * bf16 result (0x7fff) plus the lowest kept bit (which turns an exact tie into
 * a round-up only when that bit is odd), then truncate the low 16 bits.  A NaN
 * stays a quiet NaN. */
static float o_f32_to_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    if ((u & 0x7fffffffu) > 0x7f800000u) {
        u = (u | 0x00400000u) & 0xffff0000u;
    } else {
        uint32_t keep_lsb = (u >> 16) & 1u;
        u = (u + 0x7fffu + keep_lsb) & 0xffff0000u;
    }
    float r;
    memcpy(&r, &u, sizeof r);
    return r;
}

double o_round_bf16(double v) /* v must already be an f32 value */
{
    return (double)o_f32_to_bf16((float)v);
}

/* Round an f32 arithmetic result to the storage precision. */
static double o_store32(int prec, float r)
{
    return prec == O_BF16 ? (double)o_f32_to_bf16(r) : (double)r;
}

/* ---- scalars ------------------------------------------------------------
 * A scaling factor is held in the compute precision of the operation (double
 * for f64 storage, float for f32 and bf16 storage).  When a device-resident
 * factor is supplied as well, the effective factor is the product of the two,
 * rounded once in the compute precision. */
double o_scalar(int prec, double host, int has_dev, double dev)
{
    if (prec == O_F64)
        return has_dev ? host * dev : host;
    float h = (float)host;
    if (!has_dev)
        return (double)h;
    return (double)(h * (float)dev);
}

/* ---- vector copy x <- y (Section 2, the first kernel body) --------------- */
void o_copy(int64_t n, const double *y, double *x)
{
    for (int64_t i = 0; i < n; ++i)
        x[i] = y[i];
}

/* ---- scaled vector addition x <- alpha*y + beta*z (Section 2) -------------
 * The paper states the operation only as a real-number assignment.  The
 * rounding sequence used here (and required of the GPU path) is
 *     x_i = RN( alpha*y_i + RN(beta*z_i) ),
 * i.e. beta*z_i is rounded first and then a fused multiply-add forms the
 * result.  alpha and beta are the effective compute-precision factors. */
void o_axpby(int prec, int64_t n, double alpha, const double *y,
             double beta, const double *z, double *x)
{
    if (prec == O_F64) {
        for (int64_t i = 0; i < n; ++i) {
            double bz = beta * z[i];
            x[i] = fma(alpha, y[i], bz);
        }
        return;
    }
    float a = (float)alpha, b = (float)beta;
    for (int64_t i = 0; i < n; ++i) {
        float bz = b * (float)z[i];
        x[i] = o_store32(prec, fmaf(a, (float)y[i], bz));
    }
}

/* ---- scaling x <- alpha*y (the BLAS scal operation) ------------------------
 * One product per element, rounded once to the storage precision.  Unlike
 * alpha*y + 0*z there is no 0*y_i term, so infinite and NaN entries scale as
 * IEEE products do. */
void o_scal(int prec, int64_t n, double alpha, const double *y, double *x)
{
    if (prec == O_F64) {
        for (int64_t i = 0; i < n; ++i)
            x[i] = alpha * y[i];
        return;
    }
    float a = (float)alpha;
    for (int64_t i = 0; i < n; ++i)
        x[i] = o_store32(prec, a * (float)y[i]);
}

/* ---- error-free transformations ----------------------------------------- */
/* Knuth's TwoSum: s + e == a + b exactly, s = RN(a + b). */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/* TwoProduct with a fused multiply-add: p + e == a * b exactly. */
static void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* ---- inner product alpha <- <x, y> (Section 2) ---------------------------
 * Sum of x_i * y_i over n entries with strides incx, incy, evaluated with
 * Dot2 (Ogita, Rump, Oishi 2005): the running sum p is carried with its
 * exact error, the product errors and sum errors are gathered in s, and p + s
 * is the result.  The error terms are meaningless once the running sum is
 * infinite or NaN (they become inf - inf); the IEEE value of the sum is then
 * the running sum itself, which is returned. */
double o_dot(int64_t n, const double *x, int64_t incx, const double *y,
             int64_t incy)
{
    if (n <= 0)
        return 0.0;
    double p, s;
    two_prod(x[0], y[0], &p, &s);
    for (int64_t i = 1; i < n; ++i) {
        double h, r, q;
        two_prod(x[i * incx], y[i * incy], &h, &r);
        two_sum(p, h, &p, &q);
        s = s + (q + r);
    }
    return isfinite(p) ? p + s : p;
}

/* ---- sum of magnitudes sum |x_i| (the BLAS asum operation) ----------------
 * Evaluated with Sum2 (Ogita, Rump, Oishi 2005, Algorithm 4.4): the running
 * sum carries its exact TwoSum errors, which are added at the end; the
 * result is as accurate as if summed in twice the working precision.  A
 * non-finite running sum is returned as it is (as for the inner product). */
double o_asum(int64_t n, const double *x, int64_t incx)
{
    if (n <= 0)
        return 0.0;
    double p = fabs(x[0]), s = 0.0;
    for (int64_t i = 1; i < n; ++i) {
        double q;
        two_sum(p, fabs(x[i * incx]), &p, &q);
        s = s + q;
    }
    return isfinite(p) ? p + s : p;
}

/* ---- Euclidean norm: square root of <x, x>, without scaling -------------- */
double o_nrm2(int64_t n, const double *x)
{
    return sqrt(o_dot(n, x, 1, x, 1));
}

/* ---- dense matrix-vector product (Section 2) ------------------------------
 * A is m-by-n.  Row-major: A_ij at A[i*lda + j].  Column-major: A_ij at
 * A[i + j*lda].  trans == 0 computes y = A x (y has m entries, x has n);
 * trans == 1 computes y = A^T x (y has n entries, x has m).  Each output entry
 * is the inner product of one row of op(A) with x, as in the paper's
 * one-work-group-per-row kernel. */
void o_gemv(int layout, int trans, int64_t m, int64_t n, const double *A,
            int64_t lda, const double *x, double *y)
{
    int64_t rs = layout == O_ROW_MAJOR ? lda : 1; /* step between rows */
    int64_t cs = layout == O_ROW_MAJOR ? 1 : lda; /* step between columns */
    if (!trans) {
        for (int64_t i = 0; i < m; ++i)
            y[i] = o_dot(n, A + i * rs, cs, x, 1);
    } else {
        for (int64_t j = 0; j < n; ++j)
            y[j] = o_dot(m, A + j * cs, rs, x, 1);
    }
}

/* ---- rank-1 overwrite A <- u v^T ------------------------------------------
 * The gradient of y = A x with respect to A.  Each entry is one product,
 * rounded once to the storage precision. */
void o_ger(int prec, int layout, int64_t m, int64_t n, const double *u,
           const double *v, double *A, int64_t lda)
{
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            int64_t at = layout == O_ROW_MAJOR ? i * lda + j : i + j * lda;
            if (prec == O_F64)
                A[at] = u[i] * v[j];
            else
                A[at] = o_store32(prec, (float)u[i] * (float)v[j]);
        }
    }
}
