// stream.hip -- streaming kernels: vector copy x <- y and scaled vector
// addition x <- alpha y + beta z (paper Section 2), scaling x <- alpha y (the
// BLAS scal), and the fused update of a conjugate-gradient-style step
// (x += a p, r -= a q, <r, r> in one pass).
//
// Work decomposition.  The vector is cut into packs of V consecutive elements
// (the paper's vector data types).  Each thread handles U packs per loop trip,
// all loads issued before any arithmetic, so U*V*sizeof(T) bytes per thread
// are in flight; every access is a 16-byte nontemporal one (the data is
// touched once).  The loop increment is either the whole grid (GLOBAL, the
// paper's first skeleton) or the work-group inside one contiguous chunk per
// work-group (LOCAL, the paper's second skeleton; chunks are multiples of the
// work-group size so accesses stay aligned).  The n % V tail elements are
// handled element-wise by the first threads of work-group 0.
#include "device.hpp"
#include "kernels.hpp"

namespace bwla {

struct Range {
    int64_t begin, stride, end;
};

// Pack indices visited by this thread under the chosen increment scheme.
// Work-groups are numbered XCD-contiguously (xcd_block).
__device__ __forceinline__ Range pack_range(int64_t npack, int inc)
{
    Range r;
    const int64_t lb = xcd_block();
    if (inc == 0) {
        r.begin = lb * blockDim.x + threadIdx.x;
        r.stride = (int64_t)gridDim.x * blockDim.x;
        r.end = npack;
    } else {
        int64_t per = (npack + gridDim.x - 1) / gridDim.x;
        per = (per + blockDim.x - 1) / blockDim.x * blockDim.x;
        int64_t b = lb * per;
        r.begin = b + threadIdx.x;
        r.stride = blockDim.x;
        r.end = b + per < npack ? b + per : npack;
    }
    return r;
}

// ---------------------------------------------------------------------------
// copy
// ---------------------------------------------------------------------------
template <typename T, int V, int U>
__global__ __launch_bounds__(1024) void k_copy(int64_t n, const T *y, T *x, int inc)
{
    const int64_t npack = n / V;
    Range rg = pack_range(npack, inc);
    int64_t p = rg.begin;
    for (; p + (U - 1) * rg.stride < rg.end; p += U * rg.stride) {
        Pack<T, V> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = load_pack_nt<T, V>(y + (p + u * rg.stride) * V);
        end_of_loads();
#pragma unroll
        for (int u = 0; u < U; ++u)
            store_pack_nt<T, V>(x + (p + u * rg.stride) * V, v[u]);
    }
    for (; p < rg.end; p += rg.stride)
        store_pack_nt<T, V>(x + p * V, load_pack_nt<T, V>(y + p * V));
    const int64_t tail = n - npack * V;
    if (blockIdx.x == 0 && threadIdx.x < tail)
        x[npack * V + threadIdx.x] = y[npack * V + threadIdx.x];
}

// ---------------------------------------------------------------------------
// scal: x_i = RN_T(a * y_i) (x may be y: the in-place BLAS scal)
// ---------------------------------------------------------------------------
template <typename T, int V, int U>
__global__ __launch_bounds__(1024) void k_scal(int64_t n, compute_t<T> a, const compute_t<T> *adev,
                                               const T *y, T *x, int inc)
{
    if (adev)
        a = a * *adev;
    const int64_t npack = n / V;
    Range rg = pack_range(npack, inc);
    int64_t p = rg.begin;
    for (; p + (U - 1) * rg.stride < rg.end; p += U * rg.stride) {
        Pack<T, V> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = load_pack_nt<T, V>(y + (p + u * rg.stride) * V);
        end_of_loads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int e = 0; e < V; ++e)
                v[u].v[e] = narrow<T>(a * widen(v[u].v[e]));
            store_pack_nt<T, V>(x + (p + u * rg.stride) * V, v[u]);
        }
    }
    for (; p < rg.end; p += rg.stride) {
        Pack<T, V> v = load_pack_nt<T, V>(y + p * V);
#pragma unroll
        for (int e = 0; e < V; ++e)
            v.v[e] = narrow<T>(a * widen(v.v[e]));
        store_pack_nt<T, V>(x + p * V, v);
    }
    const int64_t tail = n - npack * V;
    if (blockIdx.x == 0 && threadIdx.x < tail) {
        const int64_t i = npack * V + threadIdx.x;
        x[i] = narrow<T>(a * widen(y[i]));
    }
}

// ---------------------------------------------------------------------------
// axpby: x_i = RN_T( fma(a, y_i, RN_C(b * z_i)) ) in compute precision C
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T axpby_elem(compute_t<T> a, T y, compute_t<T> b, T z)
{
    compute_t<T> bz = b * widen(z);
    return narrow<T>(fma_c(a, widen(y), bz));
}

template <typename T, int V, int U>
__global__ __launch_bounds__(1024) void k_axpby(int64_t n, compute_t<T> a, const compute_t<T> *adev,
                                                compute_t<T> b, const compute_t<T> *bdev, const T *y,
                                                const T *z, T *x, int inc)
{
    if (adev)
        a = a * *adev;
    if (bdev)
        b = b * *bdev;
    const int64_t npack = n / V;
    Range rg = pack_range(npack, inc);
    int64_t p = rg.begin;
    for (; p + (U - 1) * rg.stride < rg.end; p += U * rg.stride) {
        Pack<T, V> vy[U], vz[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vy[u] = load_pack_nt<T, V>(y + (p + u * rg.stride) * V);
            vz[u] = load_pack_nt<T, V>(z + (p + u * rg.stride) * V);
        }
        end_of_loads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            Pack<T, V> o;
#pragma unroll
            for (int e = 0; e < V; ++e)
                o.v[e] = axpby_elem<T>(a, vy[u].v[e], b, vz[u].v[e]);
            store_pack_nt<T, V>(x + (p + u * rg.stride) * V, o);
        }
    }
    for (; p < rg.end; p += rg.stride) {
        Pack<T, V> vy = load_pack_nt<T, V>(y + p * V), vz = load_pack_nt<T, V>(z + p * V), o;
#pragma unroll
        for (int e = 0; e < V; ++e)
            o.v[e] = axpby_elem<T>(a, vy.v[e], b, vz.v[e]);
        store_pack_nt<T, V>(x + p * V, o);
    }
    const int64_t tail = n - npack * V;
    if (blockIdx.x == 0 && threadIdx.x < tail) {
        int64_t i = npack * V + threadIdx.x;
        x[i] = axpby_elem<T>(a, y[i], b, z[i]);
    }
}

// ---------------------------------------------------------------------------
// fused CG-style update: x += a p ; r -= a q ; <r_new, r_new>
// Elementwise results equal axpby(x; a, p, 1, x) and axpby(r; -a, q, 1, r).
// ---------------------------------------------------------------------------
template <typename T, int V, int U, bool COMP>
__global__ __launch_bounds__(1024) void k_cg(int64_t n, compute_t<T> a, const compute_t<T> *adev, T *x,
                                             const T *p, T *r, const T *q, DD *partials, void *out,
                                             int out_f64, int inc)
{
    using C = compute_t<T>;
    constexpr bool EXACT = std::is_same<T, bf16_t>::value;
    if (adev)
        a = a * *adev;
    const C one = 1, na = -a;
    Acc<C, COMP> acc[U];
    const int64_t npack = n / V;
    Range rg = pack_range(npack, inc);
    int64_t i = rg.begin;
    for (; i + (U - 1) * rg.stride < rg.end; i += U * rg.stride) {
        Pack<T, V> vx[U], vp[U], vr[U], vq[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t o = (i + u * rg.stride) * V;
            vx[u] = load_pack_nt<T, V>(x + o);
            vp[u] = load_pack_nt<T, V>(p + o);
            vr[u] = load_pack_nt<T, V>(r + o);
            vq[u] = load_pack_nt<T, V>(q + o);
        }
        end_of_loads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t o = (i + u * rg.stride) * V;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                vx[u].v[e] = axpby_elem<T>(a, vp[u].v[e], one, vx[u].v[e]);
                vr[u].v[e] = axpby_elem<T>(na, vq[u].v[e], one, vr[u].v[e]);
                C rn = widen(vr[u].v[e]);
                acc[u].template add_prod<EXACT>(rn, rn);
            }
            store_pack_nt<T, V>(x + o, vx[u]);
            store_pack_nt<T, V>(r + o, vr[u]);
        }
    }
    for (; i < rg.end; i += rg.stride) {
        const int64_t o = i * V;
        Pack<T, V> vx = load_pack_nt<T, V>(x + o), vp = load_pack_nt<T, V>(p + o);
        Pack<T, V> vr = load_pack_nt<T, V>(r + o), vq = load_pack_nt<T, V>(q + o);
#pragma unroll
        for (int e = 0; e < V; ++e) {
            vx.v[e] = axpby_elem<T>(a, vp.v[e], one, vx.v[e]);
            vr.v[e] = axpby_elem<T>(na, vq.v[e], one, vr.v[e]);
            C rn = widen(vr.v[e]);
            acc[0].template add_prod<EXACT>(rn, rn);
        }
        store_pack_nt<T, V>(x + o, vx);
        store_pack_nt<T, V>(r + o, vr);
    }
    const int64_t tail = n - npack * V;
    if (blockIdx.x == 0 && threadIdx.x < tail) {
        const int64_t o = npack * V + threadIdx.x;
        x[o] = axpby_elem<T>(a, p[o], one, x[o]);
        T rv = axpby_elem<T>(na, q[o], one, r[o]);
        r[o] = rv;
        C rn = widen(rv);
        acc[0].template add_prod<EXACT>(rn, rn);
    }
    DD v = acc[0].to_dd();
#pragma unroll
    for (int u = 1; u < U; ++u)
        v = combine<COMP>(v, acc[u].to_dd());
    __shared__ DD lds[16];
    DD bs = block_sum<COMP>(v, lds);
    if (threadIdx.x == 0) {
        if (gridDim.x == 1)
            store_out(out, 0, out_f64, bs.hi + bs.lo);
        else
            partials[blockIdx.x] = bs;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_copy(int64_t n, const void *y, void *x, const Cfg &c, hipStream_t s)
{
    return with_vec(c.vec, [&](auto V) {
        return with_unroll(c.unroll, [&](auto U) {
            hipLaunchKernelGGL((k_copy<T, V.value, U.value>), dim3(c.grid), dim3(c.block), 0, s, n,
                               (const T *)y, (T *)x, c.inc);
            return hipGetLastError();
        });
    });
}

template <typename T>
hipError_t launch_scal(int64_t n, double alpha, const void *adev, const void *y, void *x, const Cfg &c,
                       hipStream_t s)
{
    using C = compute_t<T>;
    return with_vec(c.vec, [&](auto V) {
        return with_unroll(c.unroll, [&](auto U) {
            hipLaunchKernelGGL((k_scal<T, V.value, U.value>), dim3(c.grid), dim3(c.block), 0, s, n, (C)alpha,
                               (const C *)adev, (const T *)y, (T *)x, c.inc);
            return hipGetLastError();
        });
    });
}

template <typename T>
hipError_t launch_axpby(int64_t n, double alpha, const void *adev, const void *y, double beta,
                        const void *bdev, const void *z, void *x, const Cfg &c, hipStream_t s)
{
    using C = compute_t<T>;
    return with_vec(c.vec, [&](auto V) {
        return with_unroll(c.unroll, [&](auto U) {
            hipLaunchKernelGGL((k_axpby<T, V.value, U.value>), dim3(c.grid), dim3(c.block), 0, s, n,
                               (C)alpha, (const C *)adev, (C)beta, (const C *)bdev, (const T *)y,
                               (const T *)z, (T *)x, c.inc);
            return hipGetLastError();
        });
    });
}

template <typename T>
hipError_t launch_cg(int64_t n, bool comp, double alpha, const void *adev, void *x, const void *p,
                     void *r, const void *q, int out_f64, void *out, void *ws, const Cfg &c,
                     hipStream_t s)
{
    using C = compute_t<T>;
    DD *partials = (DD *)ws;
    hipError_t e = with_vec(c.vec, [&](auto V) {
        return with_unroll(c.unroll, [&](auto U) {
            return with_bool(comp, [&](auto CP) {
                hipLaunchKernelGGL((k_cg<T, V.value, U.value, CP.value>), dim3(c.grid), dim3(c.block),
                                   0, s, n, (C)alpha, (const C *)adev, (T *)x, (const T *)p, (T *)r,
                                   (const T *)q, partials, out, out_f64, c.inc);
                return hipGetLastError();
            });
        });
    });
    if (e != hipSuccess || c.grid == 1)
        return e;
    return launch_combine_scalar(partials, c.grid, comp, false, out_f64, out, s);
}

template hipError_t launch_copy<BWLA_T>(int64_t, const void *, void *, const Cfg &, hipStream_t);
template hipError_t launch_scal<BWLA_T>(int64_t, double, const void *, const void *, void *, const Cfg &,
                                        hipStream_t);
template hipError_t launch_axpby<BWLA_T>(int64_t, double, const void *, const void *, double,
                                         const void *, const void *, void *, const Cfg &, hipStream_t);
template hipError_t launch_cg<BWLA_T>(int64_t, bool, double, const void *, void *, const void *,
                                      void *, const void *, int, void *, void *, const Cfg &,
                                      hipStream_t);

} // namespace bwla
