// A C-style caller of libbwla with no Python and no torch: device buffers from
// hipMalloc, a stream of its own, workspaces sized by the library, and inputs
// of small integers, so that every result has an exact value the host
// computes with integer arithmetic and every comparison is for equality.
// Prints one line per check and "abi check ok" when all pass; exits non-zero
// otherwise.
#include <hip/hip_runtime_api.h>

#include "bwla.h"

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static int failures = 0;

static void expect(int ok, const char *what)
{
    printf("%s %s\n", ok ? "ok  " : "FAIL", what);
    if (!ok)
        failures++;
}

#define HIP(call)                                                                                            \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess) {                                                                              \
            printf("FAIL %s: %s\n", #call, hipGetErrorString(e_));                                           \
            exit(2);                                                                                         \
        }                                                                                                    \
    } while (0)

#define BW(call)                                                                                             \
    do {                                                                                                     \
        bwla_status s_ = (call);                                                                             \
        if (s_ != BWLA_OK) {                                                                                 \
            printf("FAIL %s: %s (%s)\n", #call, bwla_status_string(s_), bwla_last_error());                 \
            exit(3);                                                                                         \
        }                                                                                                    \
    } while (0)

static void *dev_copy(const void *h, size_t bytes)
{
    void *d = NULL;
    HIP(hipMalloc(&d, bytes ? bytes : 1));
    if (bytes)
        HIP(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice));
    return d;
}

static void *workspace(bwla_op op, bwla_dtype t, bwla_layout layout, int trans, int64_t m, int64_t n,
                       size_t *bytes)
{
    BW(bwla_workspace_size(op, t, BWLA_ACC_PLAIN, layout, trans, m, n, bytes));
    void *ws = NULL;
    HIP(hipMalloc(&ws, *bytes ? *bytes : 1));
    return ws;
}

int main(void)
{
    expect(bwla_abi_version() == BWLA_ABI_VERSION, "ABI version of the loaded library matches the header");
    hipStream_t s;
    HIP(hipStreamCreate(&s));

    // vectors: x_i in -3..3, y_i in -2..2
    const int64_t n = (1 << 20) + 3;
    double *hx = (double *)malloc(n * sizeof(double)), *hy = (double *)malloc(n * sizeof(double));
    float *fx = (float *)malloc(n * sizeof(float));
    int64_t dot_exact = 0, sq_exact = 0;
    for (int64_t i = 0; i < n; ++i) {
        hx[i] = (double)(i % 7 - 3);
        hy[i] = (double)(i % 5 - 2);
        fx[i] = (float)hx[i];
        dot_exact += (int64_t)(i % 7 - 3) * (int64_t)(i % 5 - 2);
        sq_exact += (int64_t)(i % 7 - 3) * (int64_t)(i % 7 - 3);
    }
    double *dx = (double *)dev_copy(hx, n * sizeof(double)), *dy = (double *)dev_copy(hy, n * sizeof(double));
    float *dfx = (float *)dev_copy(fx, n * sizeof(float));
    double *dz = NULL, *dout = NULL;
    HIP(hipMalloc((void **)&dz, n * sizeof(double)));
    HIP(hipMalloc((void **)&dout, sizeof(double)));
    size_t wsb = 0;
    void *ws = workspace(BWLA_OP_DOT, BWLA_F64, BWLA_ROW_MAJOR, 0, 0, n, &wsb);

    BW(bwla_copy(BWLA_F64, n, dx, dz, s));
    double *hz = (double *)malloc(n * sizeof(double));
    HIP(hipMemcpyAsync(hz, dz, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP(hipStreamSynchronize(s));
    expect(memcmp(hz, hx, n * sizeof(double)) == 0, "copy f64, 2^20 + 3 elements");

    BW(bwla_axpby(BWLA_F64, n, 2.0, NULL, dx, 3.0, NULL, dy, dz, s));
    HIP(hipMemcpyAsync(hz, dz, n * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP(hipStreamSynchronize(s));
    int ok = 1;
    for (int64_t i = 0; i < n; ++i)
        ok &= hz[i] == 2.0 * hx[i] + 3.0 * hy[i];
    expect(ok, "axpby f64 z = 2 x + 3 y, every element exact");

    double got = 0;
    BW(bwla_dot(BWLA_F64, BWLA_ACC_PLAIN, n, dx, dy, BWLA_F64, dout, ws, wsb, s));
    HIP(hipMemcpyAsync(&got, dout, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP(hipStreamSynchronize(s));
    expect(got == (double)dot_exact, "dot f64 equals the integer sum");
    BW(bwla_dot(BWLA_F64, BWLA_ACC_COMPENSATED, n, dx, dy, BWLA_F64, dout, ws, wsb, s));
    HIP(hipMemcpyAsync(&got, dout, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP(hipStreamSynchronize(s));
    expect(got == (double)dot_exact, "compensated dot f64 equals the integer sum");
    BW(bwla_nrm2(BWLA_F64, BWLA_ACC_PLAIN, n, dx, BWLA_F64, dout, ws, wsb, s));
    HIP(hipMemcpyAsync(&got, dout, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP(hipStreamSynchronize(s));
    expect(fabs(got - sqrt((double)sq_exact)) <= 0x1p-52 * sqrt((double)sq_exact),
           "nrm2 f64 is the square root of the integer sum of squares (within one rounding)");
    size_t wsf = 0;
    void *wf = workspace(BWLA_OP_DOT, BWLA_F32, BWLA_ROW_MAJOR, 0, 0, n, &wsf);
    BW(bwla_dot(BWLA_F32, BWLA_ACC_PLAIN, n, dfx, dfx, BWLA_F64, dout, wf, wsf, s));
    HIP(hipMemcpyAsync(&got, dout, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP(hipStreamSynchronize(s));
    expect(got == (double)sq_exact, "dot f32 with a float64 output equals the integer sum");

    // matrix-vector: A (m x k) entries in -3..3, both layouts, both transposes
    const int64_t m = 1000, k = 777;
    double *hA = (double *)malloc(m * k * sizeof(double)), *hAc = (double *)malloc(m * k * sizeof(double));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < k; ++j) {
            const double a = (double)((i * 3 + j * 5) % 7 - 3);
            hA[i * k + j] = a;  // row-major, lda = k
            hAc[i + j * m] = a; // column-major, lda = m
        }
    double *dA = (double *)dev_copy(hA, m * k * sizeof(double)), *dAc = (double *)dev_copy(hAc, m * k * sizeof(double));
    double *dyv = NULL, *hyv = (double *)malloc((m > k ? m : k) * sizeof(double));
    HIP(hipMalloc((void **)&dyv, (m > k ? m : k) * sizeof(double)));
    for (int layout = 0; layout < 2; ++layout)
        for (int trans = 0; trans < 2; ++trans) {
            const int64_t in = trans ? m : k, out = trans ? k : m;
            size_t gb = 0;
            void *gw = workspace(BWLA_OP_GEMV_ROWS, BWLA_F64, (bwla_layout)layout, trans, m, k, &gb);
            BW(bwla_gemv(BWLA_F64, BWLA_ACC_PLAIN, (bwla_layout)layout, trans, m, k, layout ? (void *)dAc : (void *)dA,
                         layout ? m : k, dx, BWLA_F64, dyv, gw, gb, s));
            HIP(hipMemcpyAsync(hyv, dyv, out * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP(hipStreamSynchronize(s));
            ok = 1;
            for (int64_t o = 0; o < out; ++o) {
                int64_t e = 0;
                for (int64_t q = 0; q < in; ++q) {
                    const int64_t i = trans ? q : o, j = trans ? o : q;
                    e += (int64_t)hA[i * k + j] * (int64_t)hx[q];
                }
                ok &= hyv[o] == (double)e;
            }
            char what[96];
            snprintf(what, sizeof what, "gemv f64 %s-major trans=%d, every output exact", layout ? "column" : "row",
                     trans);
            expect(ok, what);
            HIP(hipFree(gw));
        }

    // rank-1 overwrite A <- u v^T
    BW(bwla_ger(BWLA_F64, BWLA_ROW_MAJOR, m, k, dx, dy, dA, k, s));
    HIP(hipMemcpyAsync(hA, dA, m * k * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP(hipStreamSynchronize(s));
    ok = 1;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < k; ++j)
            ok &= hA[i * k + j] == hx[i] * hy[j];
    expect(ok, "ger f64 row-major, every entry exact");

    // a batch plan: two GEMVs over slices of A (now u v^T) and two dots
    bwla_gemv_desc g[2] = {{dA, 10, k, k, dx, dyv}, {dA + 10 * k, 300, 200, k, dy, dyv + 10}};
    bwla_dot_desc d[2] = {{dx, dy, n, dout}, {dx, dx, 5, dz}};
    bwla_batch_plan *plan = NULL;
    BW(bwla_batch_plan_create(BWLA_F64, BWLA_ACC_PLAIN, BWLA_F64, g, 2, d, 2, NULL, &plan));
    BW(bwla_batch_run(plan, s));
    double r[310], d0 = 0, d1 = 0;
    HIP(hipMemcpyAsync(r, dyv, 310 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP(hipMemcpyAsync(&d0, dout, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP(hipMemcpyAsync(&d1, dz, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP(hipStreamSynchronize(s));
    ok = d0 == (double)dot_exact && d1 == 9.0 + 4.0 + 1.0 + 0.0 + 1.0;
    for (int64_t i = 0; i < 10; ++i) {
        int64_t e = 0;
        for (int64_t j = 0; j < k; ++j)
            e += (int64_t)(hx[i] * hy[j]) * (int64_t)hx[j];
        ok &= r[i] == (double)e;
    }
    for (int64_t i = 0; i < 300; ++i) {
        int64_t e = 0;
        for (int64_t j = 0; j < 200; ++j)
            e += (int64_t)(hx[10 + i] * hy[j]) * (int64_t)hy[j];
        ok &= r[10 + i] == (double)e;
    }
    expect(ok, "batch plan of two GEMVs and two dots, every output exact");
    bwla_batch_plan_destroy(plan);

    // validation: nothing enqueued, a status and a message
    expect(bwla_dot(BWLA_F64, BWLA_ACC_PLAIN, -1, dx, dy, BWLA_F64, dout, ws, wsb, s) == BWLA_ERR_INVALID_ARG &&
               strlen(bwla_last_error()) > 0,
           "negative length rejected with a message");
    expect(bwla_dot(BWLA_F64, BWLA_ACC_PLAIN, n, dx, dy, BWLA_F64, dout, ws, 8, s) == BWLA_ERR_WORKSPACE,
           "short workspace rejected");

    HIP(hipStreamSynchronize(s));
    HIP(hipFree(dx));
    HIP(hipFree(dy));
    HIP(hipFree(dfx));
    HIP(hipFree(dz));
    HIP(hipFree(dout));
    HIP(hipFree(ws));
    HIP(hipFree(wf));
    HIP(hipFree(dA));
    HIP(hipFree(dAc));
    HIP(hipFree(dyv));
    HIP(hipStreamDestroy(s));
    free(hx);
    free(hy);
    free(fx);
    free(hz);
    free(hA);
    free(hAc);
    free(hyv);
    if (failures) {
        printf("%d checks failed\n", failures);
        return 1;
    }
    printf("abi check ok\n");
    return 0;
}
