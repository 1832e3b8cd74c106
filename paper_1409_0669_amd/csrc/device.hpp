// device.hpp -- gfx950 device building blocks shared by the library's kernels:
// storage/compute type traits, 16-byte packed global loads and stores,
// error-free transformations, and wave64 and work-group float64 reductions.
//
// Cross-work-group combines are done by a second, small kernel rather than by
// a "last work-group" ticket inside the first: on gfx950 every agent-scope
// fence that such a ticket needs writes back and invalidates the XCD's L2,
// which serialises badly across thousands of work-groups.  The kernel
// boundary gives the visibility for free and keeps the combine order fixed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bwla {

using bf16_t = __bf16;

// Compute precision of a storage type: double for f64, float for f32/bf16.
template <typename T> struct Compute;
template <> struct Compute<double> { using type = double; };
template <> struct Compute<float> { using type = float; };
template <> struct Compute<bf16_t> { using type = float; };
template <typename T> using compute_t = typename Compute<T>::type;

template <typename T> __device__ __forceinline__ compute_t<T> widen(T v) { return (compute_t<T>)v; }
// float -> bf16 conversion is an LLVM fptrunc, round to nearest even (a single
// v_cvt_pk_bf16_f32 on gfx950).
template <typename T> __device__ __forceinline__ T narrow(compute_t<T> v) { return (T)v; }

__device__ __forceinline__ double fma_c(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_c(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ---------------------------------------------------------------------------
// Packed global memory access: V consecutive elements per thread.  Packs of
// 16 bytes or more are moved as 16-byte (dwordx4) accesses; smaller packs as
// one 8/4/2-byte access.  Callers guarantee alignment to V*sizeof(T).
// ---------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <typename T, int V> struct Pack {
    T v[V];
};

template <typename T, int V>
__device__ __forceinline__ Pack<T, V> load_pack(const T *p)
{
    constexpr int B = V * (int)sizeof(T);
    Pack<T, V> r;
    if constexpr (B >= 16) {
        const u32x4 *s = reinterpret_cast<const u32x4 *>(p);
        u32x4 tmp[B / 16];
#pragma unroll
        for (int i = 0; i < B / 16; ++i)
            tmp[i] = s[i];
        __builtin_memcpy(&r, tmp, B);
    } else if constexpr (B == 8) {
        u32x2 tmp = *reinterpret_cast<const u32x2 *>(p);
        __builtin_memcpy(&r, &tmp, B);
    } else if constexpr (B == 4) {
        uint32_t tmp = *reinterpret_cast<const uint32_t *>(p);
        __builtin_memcpy(&r, &tmp, B);
    } else {
        uint16_t tmp = *reinterpret_cast<const uint16_t *>(p);
        __builtin_memcpy(&r, &tmp, B);
    }
    return r;
}

template <typename T, int V>
__device__ __forceinline__ void store_pack(T *p, const Pack<T, V> &r)
{
    constexpr int B = V * (int)sizeof(T);
    if constexpr (B >= 16) {
        u32x4 tmp[B / 16];
        __builtin_memcpy(tmp, &r, B);
        u32x4 *d = reinterpret_cast<u32x4 *>(p);
#pragma unroll
        for (int i = 0; i < B / 16; ++i)
            d[i] = tmp[i];
    } else if constexpr (B == 8) {
        u32x2 tmp;
        __builtin_memcpy(&tmp, &r, B);
        *reinterpret_cast<u32x2 *>(p) = tmp;
    } else if constexpr (B == 4) {
        uint32_t tmp;
        __builtin_memcpy(&tmp, &r, B);
        *reinterpret_cast<uint32_t *>(p) = tmp;
    } else {
        uint16_t tmp;
        __builtin_memcpy(&tmp, &r, B);
        *reinterpret_cast<uint16_t *>(p) = tmp;
    }
}

// Streaming (nontemporal) variants for data touched exactly once -- vector
// operands, the matrix of a GEMV, outputs.  On gfx950 they set the
// nontemporal hint on the 16-byte accesses, which keeps once-read streams
// from displacing reusable lines in the caches; measured on MI355X, copy goes
// from ~6.0 to ~6.6 TB/s and a read-only stream from ~6.3 to ~7.0 TB/s.
template <typename T, int V>
__device__ __forceinline__ Pack<T, V> load_pack_nt(const T *p)
{
    constexpr int B = V * (int)sizeof(T);
    Pack<T, V> r;
    if constexpr (B >= 16) {
        const u32x4 *s = reinterpret_cast<const u32x4 *>(p);
        u32x4 tmp[B / 16];
#pragma unroll
        for (int i = 0; i < B / 16; ++i)
            tmp[i] = __builtin_nontemporal_load(s + i);
        __builtin_memcpy(&r, tmp, B);
    } else if constexpr (B == 8) {
        u32x2 tmp = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
        __builtin_memcpy(&r, &tmp, B);
    } else if constexpr (B == 4) {
        uint32_t tmp = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(p));
        __builtin_memcpy(&r, &tmp, B);
    } else {
        uint16_t tmp = __builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(p));
        __builtin_memcpy(&r, &tmp, B);
    }
    return r;
}

// Ends the load phase of an unrolled trip: no instruction moves across it,
// so every load issued above is in flight before the arithmetic below starts.
// Without it the machine scheduler sinks part of a trip's loads into the
// arithmetic (to shorten register live ranges) and waits on each at once,
// which cuts the bytes a wave keeps in flight -- on gfx950 down to one or two
// packs for some compensated instantiations, halving their bandwidth.
__device__ __forceinline__ void end_of_loads() { __builtin_amdgcn_sched_barrier(0); }

template <typename T, int V>
__device__ __forceinline__ void store_pack_nt(T *p, const Pack<T, V> &r)
{
    constexpr int B = V * (int)sizeof(T);
    if constexpr (B >= 16) {
        u32x4 tmp[B / 16];
        __builtin_memcpy(tmp, &r, B);
        u32x4 *d = reinterpret_cast<u32x4 *>(p);
#pragma unroll
        for (int i = 0; i < B / 16; ++i)
            __builtin_nontemporal_store(tmp[i], d + i);
    } else if constexpr (B == 8) {
        u32x2 tmp;
        __builtin_memcpy(&tmp, &r, B);
        __builtin_nontemporal_store(tmp, reinterpret_cast<u32x2 *>(p));
    } else if constexpr (B == 4) {
        uint32_t tmp;
        __builtin_memcpy(&tmp, &r, B);
        __builtin_nontemporal_store(tmp, reinterpret_cast<uint32_t *>(p));
    } else {
        uint16_t tmp;
        __builtin_memcpy(&tmp, &r, B);
        __builtin_nontemporal_store(tmp, reinterpret_cast<uint16_t *>(p));
    }
}

// ---------------------------------------------------------------------------
// XCD-aware work-group numbering.  The hardware hands consecutive work-group
// ids to the 8 XCDs in turn; renumbering so that each XCD's work-groups
// cover one contiguous range of the logical index space keeps each XCD on
// its own stretch of memory.  A bijection on [0, gridDim.x) for any grid size.
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block()
{
    const int64_t g = gridDim.x, b = blockIdx.x;
    const int64_t xcd = b % kXcds, idx = b / kXcds;
    const int64_t q = g / kXcds, r = g % kXcds;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// ---------------------------------------------------------------------------
// Error-free transformations (exact for finite values without overflow).
// ---------------------------------------------------------------------------
// s + e == a + b, s = RN(a + b)   (Knuth)
template <typename C> __device__ __forceinline__ void two_sum(C a, C b, C &s, C &e)
{
    s = a + b;
    C bv = s - a;
    e = (a - (s - bv)) + (b - bv);
}
// s + e == a + b given |a| >= |b| or a == 0   (Dekker)
template <typename C> __device__ __forceinline__ void fast_two_sum(C a, C b, C &s, C &e)
{
    s = a + b;
    e = b - (s - a);
}

// |a| in the compute precision (clears the sign bit: |-0| = +0).
__device__ __forceinline__ float abs_c(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double abs_c(double a) { return __builtin_fabs(a); }

// A float64 value carried with its rounding error (hi + lo, |lo| <= ulp(hi)/2).
struct DD {
    double hi, lo;
};

// Once the sum is infinite or NaN the error terms are meaningless (inf - inf)
// and the IEEE value of the sum is the plain sum, which is kept with lo = 0.
__device__ __forceinline__ DD dd_add(DD a, DD b)
{
    double s, e;
    two_sum(a.hi, b.hi, s, e);
    DD r;
    if (!__builtin_isfinite(s)) {
        r.hi = s;
        r.lo = 0.0;
        return r;
    }
    e += a.lo + b.lo;
    fast_two_sum(s, e, r.hi, r.lo);
    return r;
}

// Accumulator of a reduction.  PLAIN keeps one running sum; COMPENSATED keeps
// the running sum and the gathered rounding errors of products and sums.
template <typename C, bool COMP> struct Acc {
    C s = 0, e = 0;
    // s += a*b.  EXACT_PROD: a*b is exact in C (bf16 operands in float), so
    // no product error is gathered.
    template <bool EXACT_PROD>
    __device__ __forceinline__ void add_prod(C a, C b)
    {
        if constexpr (!COMP) {
            s = fma_c(a, b, s);
        } else {
            C h = a * b;
            C q, t;
            two_sum(s, h, t, q);
            s = t;
            if constexpr (EXACT_PROD) {
                e += q;
            } else {
                C r = fma_c(a, b, -h);
                e += q + r;
            }
        }
    }
    __device__ __forceinline__ void merge(const Acc &o)
    {
        if constexpr (!COMP) {
            s += o.s;
        } else {
            C t, q;
            two_sum(s, o.s, t, q);
            s = t;
            e += q + o.e;
        }
    }
    // Leave the thread as a float64 pair.
    __device__ __forceinline__ DD to_dd() const
    {
        DD r;
        if constexpr (!COMP) {
            r.hi = (double)s;
            r.lo = 0.0;
        } else if (!__builtin_isfinite(s)) { // see dd_add
            r.hi = (double)s;
            r.lo = 0.0;
        } else {
            fast_two_sum((double)s, (double)e, r.hi, r.lo);
        }
        return r;
    }
};

template <bool COMP> __device__ __forceinline__ DD combine(DD a, DD b)
{
    if constexpr (COMP) {
        return dd_add(a, b);
    } else {
        DD r;
        r.hi = a.hi + b.hi;
        r.lo = 0.0;
        return r;
    }
}

// ---------------------------------------------------------------------------
// Wave64 reduction.  Butterfly exchanges: DPP quad permutations and row
// mirrors inside each 16-lane row, then cross-row exchanges.  Partners
// compute a+b and b+a, which round identically, so every lane ends with the
// bitwise same total and the pattern is fixed (deterministic).
// ---------------------------------------------------------------------------
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v)
{
    int2 b = __builtin_bit_cast(int2, v);
    int lo = __builtin_amdgcn_update_dpp(0, b.x, CTRL, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, b.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, make_int2(lo, hi));
}
constexpr int kDppXor1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7-i within 8 lanes
constexpr int kDppMirror = 0x140;     // lane i <-> 15-i within 16 lanes

template <int CTRL> __device__ __forceinline__ DD dpp_dd(DD v)
{
    DD r;
    r.hi = dpp_f64<CTRL>(v.hi);
    r.lo = dpp_f64<CTRL>(v.lo);
    return r;
}
__device__ __forceinline__ DD shfl_xor_dd(DD v, int m)
{
    DD r;
    r.hi = __shfl_xor(v.hi, m);
    r.lo = __shfl_xor(v.lo, m);
    return r;
}

template <bool COMP> __device__ __forceinline__ DD wave_sum(DD v)
{
    v = combine<COMP>(v, dpp_dd<kDppXor1>(v));
    v = combine<COMP>(v, dpp_dd<kDppXor2>(v));
    v = combine<COMP>(v, dpp_dd<kDppHalfMirror>(v));
    v = combine<COMP>(v, dpp_dd<kDppMirror>(v));
    v = combine<COMP>(v, shfl_xor_dd(v, 16));
    v = combine<COMP>(v, shfl_xor_dd(v, 32));
    return v;
}

// Sum over one work-group (blockDim.x a multiple of 64, at most 1024).  `lds`
// holds at least 16 DD.  The result is valid in every thread.  Contains
// barriers: every thread of the block must call it.
template <bool COMP> __device__ __forceinline__ DD block_sum(DD v, DD *lds)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    v = wave_sum<COMP>(v);
    if (lane == 0)
        lds[wave] = v;
    __syncthreads();
    DD t = {0.0, 0.0};
    if (lane < nw)
        t = lds[lane];
    t = wave_sum<COMP>(t);
    __syncthreads(); // lds may be reused by the caller afterwards
    return t;
}

// Rounds a float64 result to the output element type.
__device__ __forceinline__ void store_out(void *out, int64_t i, int out_f64, double v)
{
    if (out_f64)
        reinterpret_cast<double *>(out)[i] = v;
    else
        reinterpret_cast<float *>(out)[i] = (float)v;
}

} // namespace bwla
