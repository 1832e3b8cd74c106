// strided.hip -- vectors with an increment, in the reference-BLAS convention:
// logical element i of (p, inc) sits at p[i*inc] for inc >= 0 and at
// p[(n-1-i)*|inc|] for inc < 0; inc == 0 (inputs only) repeats p[0].
//
// The paper's Section 2 notes that the vector data types suit strided access
// poorly, and on gfx950 a 16-byte pack cannot span a stride either, so these
// kernels move one element per lane per access.  Consecutive lanes take
// consecutive logical elements (a wave touches 64 elements |inc| apart), each
// thread keeps U elements in flight per trip, and work-groups are numbered
// XCD-contiguously.  Unit-increment calls never come here: they use the
// packed kernels.
//
// Elementwise modes: copy x = y; axpby x = RN(fma(a, y, RN(b z))) exactly as
// the packed axpby; scal x = RN(a y).  Reduction modes: <x, y>, sum x_i^2
// (the norm takes the square root at the end) and sum |x_i|; partials and the
// second stage as in the packed reductions.
#include "device.hpp"
#include "kernels.hpp"

namespace bwla {

__device__ __forceinline__ int64_t elem_off(int64_t i, int64_t inc, int64_t n)
{
    return inc >= 0 ? i * inc : (i - (n - 1)) * inc;
}

template <typename T, int MODE>
__device__ __forceinline__ T strided_elem(compute_t<T> a, T y, compute_t<T> b, T z)
{
    if constexpr (MODE == kElemCopy) {
        return y;
    } else if constexpr (MODE == kElemScal) {
        return narrow<T>(a * widen(y));
    } else {
        compute_t<T> bz = b * widen(z);
        return narrow<T>(fma_c(a, widen(y), bz));
    }
}

template <typename T, int MODE, int U>
__global__ __launch_bounds__(256) void k_strided_elem(int64_t n, compute_t<T> a, const compute_t<T> *adev,
                                                      compute_t<T> b, const compute_t<T> *bdev, const T *y,
                                                      int64_t incy, const T *z, int64_t incz, T *x,
                                                      int64_t incx)
{
    if (MODE != kElemCopy && adev)
        a = a * *adev;
    if (MODE == kElemAxpby && bdev)
        b = b * *bdev;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        T vy[U], vz[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vy[u] = y[elem_off(i + u * stride, incy, n)];
            if constexpr (MODE == kElemAxpby)
                vz[u] = z[elem_off(i + u * stride, incz, n)];
        }
        end_of_loads();
#pragma unroll
        for (int u = 0; u < U; ++u)
            x[elem_off(i + u * stride, incx, n)] = strided_elem<T, MODE>(a, vy[u], b, vz[u]);
    }
    for (; i < n; i += stride) {
        const T vy = y[elem_off(i, incy, n)];
        T vz = vy;
        if constexpr (MODE == kElemAxpby)
            vz = z[elem_off(i, incz, n)];
        x[elem_off(i, incx, n)] = strided_elem<T, MODE>(a, vy, b, vz);
    }
}

template <typename T, int MODE, bool COMP>
__device__ __forceinline__ void strided_term(Acc<compute_t<T>, COMP> &acc, T xv, T yv)
{
    constexpr bool EXACT = std::is_same<T, bf16_t>::value;
    const compute_t<T> a = widen(xv);
    if constexpr (MODE == kRedDot)
        acc.template add_prod<EXACT>(a, widen(yv));
    else if constexpr (MODE == kRedSq)
        acc.template add_prod<EXACT>(a, a);
    else
        acc.template add_prod<true>(abs_c(a), compute_t<T>(1)); // exact product
}

template <typename T, int MODE, int U, bool COMP>
__global__ __launch_bounds__(256) void k_strided_reduce(int64_t n, const T *x, int64_t incx, const T *y,
                                                        int64_t incy, DD *partials, void *out, int out_f64)
{
    Acc<compute_t<T>, COMP> acc[U];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        T vx[U], vy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vx[u] = x[elem_off(i + u * stride, incx, n)];
            if constexpr (MODE == kRedDot)
                vy[u] = y[elem_off(i + u * stride, incy, n)];
        }
        end_of_loads();
#pragma unroll
        for (int u = 0; u < U; ++u)
            strided_term<T, MODE, COMP>(acc[u], vx[u], MODE == kRedDot ? vy[u] : vx[u]);
    }
    for (; i < n; i += stride) {
        const T vx = x[elem_off(i, incx, n)];
        strided_term<T, MODE, COMP>(acc[0], vx, MODE == kRedDot ? y[elem_off(i, incy, n)] : vx);
    }
    DD v = acc[0].to_dd();
#pragma unroll
    for (int u = 1; u < U; ++u)
        v = combine<COMP>(v, acc[u].to_dd());
    __shared__ DD lds[16];
    DD bs = block_sum<COMP>(v, lds);
    if (threadIdx.x == 0) {
        if (gridDim.x == 1) {
            const double r = bs.hi + bs.lo;
            store_out(out, 0, out_f64, MODE == kRedSq ? __builtin_sqrt(r) : r);
        } else {
            partials[blockIdx.x] = bs;
        }
    }
}

template <typename T>
hipError_t launch_strided_elem(int mode, int64_t n, double alpha, const void *adev, double beta,
                               const void *bdev, const void *y, int64_t incy, const void *z, int64_t incz,
                               void *x, int64_t incx, int grid, hipStream_t s)
{
    using C = compute_t<T>;
    constexpr int U = kStridedUnroll;
    auto go = [&](auto M) {
        hipLaunchKernelGGL((k_strided_elem<T, M.value, U>), dim3(grid), dim3(kStridedBlock), 0, s, n, (C)alpha,
                           (const C *)adev, (C)beta, (const C *)bdev, (const T *)y, incy, (const T *)z, incz,
                           (T *)x, incx);
        return hipGetLastError();
    };
    switch (mode) {
    case kElemCopy: return go(std::integral_constant<int, kElemCopy>{});
    case kElemAxpby: return go(std::integral_constant<int, kElemAxpby>{});
    case kElemScal: return go(std::integral_constant<int, kElemScal>{});
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_strided_reduce(int mode, int64_t n, bool comp, const void *x, int64_t incx, const void *y,
                                 int64_t incy, int out_f64, void *out, void *ws, int grid, hipStream_t s)
{
    constexpr int U = kStridedUnroll;
    DD *partials = (DD *)ws;
    hipError_t e = with_bool(comp, [&](auto CP) {
        auto go = [&](auto M) {
            hipLaunchKernelGGL((k_strided_reduce<T, M.value, U, CP.value>), dim3(grid), dim3(kStridedBlock), 0,
                               s, n, (const T *)x, incx, (const T *)y, incy, partials, out, out_f64);
            return hipGetLastError();
        };
        switch (mode) {
        case kRedDot: return go(std::integral_constant<int, kRedDot>{});
        case kRedSq: return go(std::integral_constant<int, kRedSq>{});
        case kRedAbs: return go(std::integral_constant<int, kRedAbs>{});
        default: return hipErrorInvalidValue;
        }
    });
    if (e != hipSuccess || grid == 1)
        return e;
    return launch_combine_scalar(partials, grid, comp, mode == kRedSq, out_f64, out, s);
}

template hipError_t launch_strided_elem<BWLA_T>(int, int64_t, double, const void *, double, const void *,
                                                const void *, int64_t, const void *, int64_t, void *, int64_t,
                                                int, hipStream_t);
template hipError_t launch_strided_reduce<BWLA_T>(int, int64_t, bool, const void *, int64_t, const void *,
                                                  int64_t, int, void *, void *, int, hipStream_t);

} // namespace bwla
