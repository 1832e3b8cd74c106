// ger.hip -- rank-1 overwrite A <- u v^T, the gradient of y = A x with
// respect to A.  Write-bandwidth bound: every entry is one product rounded
// once to the storage type.
//
// With A viewed as L lines of K contiguous elements (rows of a row-major A,
// columns of a column-major A), entry (l, k) is a[l] * b[k] where a is the
// per-line factor and b runs along the line.  A work-group owns R lines and
// blockDim*V consecutive elements of them: each thread loads its pack of b
// once and writes R packs.
#include "device.hpp"
#include "kernels.hpp"

namespace bwla {

template <typename T, int V, int R>
__global__ __launch_bounds__(1024) void k_ger(int64_t L, int64_t K, const T *a, const T *b, T *A,
                                              int64_t ld, int64_t kblocks)
{
    using C = compute_t<T>;
    const int64_t lblk = xcd_block();
    const int64_t lg = lblk / kblocks;
    const int64_t kb = lblk - lg * kblocks;
    const int64_t k0 = (kb * blockDim.x + threadIdx.x) * V;
    if (k0 >= K)
        return;
    const int64_t l0 = lg * R;
    const bool full = k0 + V <= K;
    C bv[V];
    if (full) {
        Pack<T, V> p = load_pack<T, V>(b + k0);
#pragma unroll
        for (int e = 0; e < V; ++e)
            bv[e] = widen(p.v[e]);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e)
            bv[e] = k0 + e < K ? widen(b[k0 + e]) : C(0);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t l = l0 + r;
        if (l >= L)
            break;
        const C al = widen(a[l]);
        T *dst = A + l * ld + k0;
        if (full) {
            Pack<T, V> o;
#pragma unroll
            for (int e = 0; e < V; ++e)
                o.v[e] = narrow<T>(al * bv[e]);
            store_pack_nt<T, V>(dst, o);
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (k0 + e < K)
                    dst[e] = narrow<T>(al * bv[e]);
        }
    }
}

template <typename T>
hipError_t launch_ger(int64_t L, int64_t K, const void *a, const void *b, void *A, int64_t ld,
                      const Cfg &c, hipStream_t s)
{
    return with_vec(c.vec, [&](auto V) {
        return with_rows(c.rows, [&](auto R) {
            const int64_t kblocks = (K + (int64_t)c.block * V.value - 1) / ((int64_t)c.block * V.value);
            const int64_t lgroups = (L + R.value - 1) / R.value;
            hipLaunchKernelGGL((k_ger<T, V.value, R.value>), dim3((unsigned)(kblocks * lgroups)),
                               dim3(c.block), 0, s, L, K, (const T *)a, (const T *)b, (T *)A, ld,
                               kblocks);
            return hipGetLastError();
        });
    });
}

template hipError_t launch_ger<BWLA_T>(int64_t, int64_t, const void *, const void *, void *, int64_t,
                                       const Cfg &, hipStream_t);

} // namespace bwla
