// reduce.hip -- inner product <x, y>, Euclidean norm sqrt(<x, x>) and sum of
// magnitudes sum |x_i| (paper Section 2: inner product with a work-group
// reduction in local memory; the other two read one vector).
//
// Stage 1: every thread accumulates its packs (same pack walk, increment
// schemes and nontemporal 16-byte loads as the streaming kernels) into U independent accumulators in the
// compute precision, plain or compensated.  The accumulators leave the thread
// as float64 (pairs when compensated), are summed across the wave with DPP and
// cross-row exchanges, across the work-group through LDS, and the work-group
// partial is written to the workspace.  Stage 2 (a one-work-group kernel)
// sums all partials in a fixed order and writes the scalar.  No atomics are
// used, so the result is deterministic for a given configuration.
#include "device.hpp"
#include "kernels.hpp"

namespace bwla {

// One term of the reduction: x_i y_i, x_i^2, or |x_i| (an exact product by 1).
template <int MODE, bool EXACT, typename C, bool COMP>
__device__ __forceinline__ void reduce_term(Acc<C, COMP> &acc, C a, C b)
{
    if constexpr (MODE == kRedAbs)
        acc.template add_prod<true>(abs_c(a), C(1));
    else
        acc.template add_prod<EXACT>(a, MODE == kRedSq ? a : b);
}

template <typename T, int V, int U, bool COMP, int MODE>
__global__ __launch_bounds__(1024) void k_dot(int64_t n, const T *x, const T *y, DD *partials,
                                              void *out, int out_f64, int inc)
{
    using C = compute_t<T>;
    constexpr bool EXACT = std::is_same<T, bf16_t>::value;
    Acc<C, COMP> acc[U];
    const int64_t npack = n / V;
    int64_t begin, stride, end;
    const int64_t lb = xcd_block();
    if (inc == 0) {
        begin = lb * blockDim.x + threadIdx.x;
        stride = (int64_t)gridDim.x * blockDim.x;
        end = npack;
    } else {
        int64_t per = (npack + gridDim.x - 1) / gridDim.x;
        per = (per + blockDim.x - 1) / blockDim.x * blockDim.x;
        int64_t b = lb * per;
        begin = b + threadIdx.x;
        stride = blockDim.x;
        end = b + per < npack ? b + per : npack;
    }
    int64_t p = begin;
    for (; p + (U - 1) * stride < end; p += U * stride) {
        Pack<T, V> vx[U], vy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vx[u] = load_pack_nt<T, V>(x + (p + u * stride) * V);
            if constexpr (MODE == kRedDot)
                vy[u] = load_pack_nt<T, V>(y + (p + u * stride) * V);
        }
        end_of_loads();
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e)
                reduce_term<MODE, EXACT>(acc[u], widen(vx[u].v[e]),
                                         MODE == kRedDot ? widen(vy[u].v[e]) : C(0));
    }
    for (; p < end; p += stride) {
        Pack<T, V> vx = load_pack_nt<T, V>(x + p * V), vy;
        if constexpr (MODE == kRedDot)
            vy = load_pack_nt<T, V>(y + p * V);
#pragma unroll
        for (int e = 0; e < V; ++e)
            reduce_term<MODE, EXACT>(acc[0], widen(vx.v[e]), MODE == kRedDot ? widen(vy.v[e]) : C(0));
    }
    const int64_t tail = n - npack * V;
    if (blockIdx.x == 0 && threadIdx.x < tail) {
        const int64_t i = npack * V + threadIdx.x;
        reduce_term<MODE, EXACT>(acc[0], widen(x[i]), MODE == kRedDot ? widen(y[i]) : C(0));
    }
    DD v = acc[0].to_dd();
#pragma unroll
    for (int u = 1; u < U; ++u)
        v = combine<COMP>(v, acc[u].to_dd());

    __shared__ DD lds[16];
    DD bs = block_sum<COMP>(v, lds);
    if (threadIdx.x == 0) {
        if (gridDim.x == 1) {
            double r = bs.hi + bs.lo;
            store_out(out, 0, out_f64, MODE == kRedSq ? __builtin_sqrt(r) : r);
        } else {
            partials[blockIdx.x] = bs;
        }
    }
}

#if BWLA_T_IS_F64 // type-independent kernels live in the f64 object only
__global__ void k_fill_zero(void *out, int64_t count, int out_f64)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < count; i += (int64_t)gridDim.x * blockDim.x)
        store_out(out, i, out_f64, 0.0);
}

// Stage 2 of the scalar reductions: one work-group sums the partials, each
// thread a fixed strided subset in index order with kScalarBatch loads in
// flight, then the work-group tree.  Many partials (grids of one work-group
// per few KiB) get 1024 threads instead of 256.
constexpr int kScalarBatch = 8;

template <bool COMP>
__global__ __launch_bounds__(1024) void k_combine_scalar(const DD *partials, int64_t count, void *out,
                                                         int out_f64, int do_sqrt)
{
    __shared__ DD lds[16];
    DD t = {0.0, 0.0};
    const int64_t step = blockDim.x;
    int64_t i = threadIdx.x;
    for (; i + (kScalarBatch - 1) * step < count; i += kScalarBatch * step) {
        DD v[kScalarBatch];
#pragma unroll
        for (int b = 0; b < kScalarBatch; ++b)
            v[b] = partials[i + b * step];
        end_of_loads();
#pragma unroll
        for (int b = 0; b < kScalarBatch; ++b)
            t = combine<COMP>(t, v[b]);
    }
    for (; i < count; i += step)
        t = combine<COMP>(t, partials[i]);
    t = block_sum<COMP>(t, lds);
    if (threadIdx.x == 0) {
        double r = t.hi + t.lo;
        store_out(out, 0, out_f64, do_sqrt ? __builtin_sqrt(r) : r);
    }
}
#endif

template <typename T>
hipError_t launch_dot(int64_t n, bool comp, int mode, const void *x, const void *y, int out_f64,
                      void *out, void *ws, const Cfg &c, hipStream_t s)
{
    DD *partials = (DD *)ws;
    // packs in flight per thread: 1, 2, 4, or 8 (a single stream -- nrm2,
    // asum -- needs more bytes in flight per thread than two)
    auto with_unroll_red = [](int u, auto &&f) -> hipError_t {
        if (u == 8)
            return f(std::integral_constant<int, 8>{});
        return with_unroll(u, f);
    };
    hipError_t e = with_vec(c.vec, [&](auto V) {
        return with_unroll_red(c.unroll, [&](auto U) {
            return with_bool(comp, [&](auto CP) {
                auto go = [&](auto M) {
                    hipLaunchKernelGGL((k_dot<T, V.value, U.value, CP.value, M.value>), dim3(c.grid),
                                       dim3(c.block), 0, s, n, (const T *)x, (const T *)y, partials,
                                       out, out_f64, c.inc);
                    return hipGetLastError();
                };
                switch (mode) {
                case kRedDot: return go(std::integral_constant<int, kRedDot>{});
                case kRedSq: return go(std::integral_constant<int, kRedSq>{});
                case kRedAbs: return go(std::integral_constant<int, kRedAbs>{});
                default: return hipErrorInvalidValue;
                }
            });
        });
    });
    if (e != hipSuccess || c.grid == 1)
        return e;
    return launch_combine_scalar(partials, c.grid, comp, mode == kRedSq, out_f64, out, s);
}

template hipError_t launch_dot<BWLA_T>(int64_t, bool, int, const void *, const void *, int, void *,
                                       void *, const Cfg &, hipStream_t);

#if BWLA_T_IS_F64
hipError_t launch_fill_zero(void *out, int64_t count, int out_f64, hipStream_t s)
{
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, out, count, out_f64);
    return hipGetLastError();
}

hipError_t launch_combine_scalar(const void *partials, int64_t count, bool comp, bool do_sqrt,
                                 int out_f64, void *out, hipStream_t s)
{
    return with_bool(comp, [&](auto CP) {
        const int threads = count > 8 * 256 ? 1024 : 256;
        hipLaunchKernelGGL((k_combine_scalar<CP.value>), dim3(1), dim3(threads), 0, s, (const DD *)partials,
                           count, out, out_f64, (int)do_sqrt);
        return hipGetLastError();
    });
}
#endif

} // namespace bwla
