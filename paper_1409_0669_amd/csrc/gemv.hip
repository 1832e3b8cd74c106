// gemv.hip -- dense matrix-vector products (paper Section 2: each output
// entry is the inner product of one row with the right-hand side; the paper
// notes other blockings are possible, and these kernels use two).
//
// A matrix is viewed as L "lines" of K contiguous elements, ld elements apart.
// A row-major A has its rows as lines, a column-major A its columns, so:
//   row-major  y = A x    and column-major y = A^T x  -> rows kernel
//   row-major  y = A^T x  and column-major y = A x    -> cols kernel
//
// rows kernel: out[l] = sum_k A[l*ld + k] v[k].  A work-group owns R lines
//   (and, with split > 1, one of `split` slices of their length).  Each
//   thread loads a pack of v once into registers and reuses it for the R
//   lines, so v is read from cache once per R lines of A; A itself is read
//   with nontemporal loads (touched once), U packs per line in flight.  The R sums are
//   reduced across the wave (DPP) and across waves through LDS.  With split >
//   1 each slice writes float64 partials and a second kernel combines them in
//   slice order.
//
// cols kernel: out[k] = sum_l A[l*ld + k] v[l].  A work-group owns a tile of
//   64*V consecutive outputs (V per lane, so each wave access is 64*V
//   contiguous elements) and one of `split` slices of the lines; its waves
//   take interleaved lines of the slice, U lines in flight (up to 32).  Each
//   v[l] is one scalar load per wave, issued with the loads of its line, so
//   the first loads of A start without a staging pass or a barrier.  Per-wave
//   partial sums are combined through LDS in wave order; with split > 1 the
//   slices' partials are combined in slice order by a second kernel.
//
// Dot epilogue (w != NULL): the caller also wants s = <w, y> over the
// outputs, with y as stored (the storage type equals the compute type
// here).  Whichever kernel stores an output also forms w_o * y_o and reduces
// those products over its outputs to one float64 pair per work-group:
// the rows or cols kernel when split == 1, the line combine otherwise.  The
// scalar second stage then sums the pairs in work-group order.  This saves
// re-reading y and w and one launch of the separate inner product.
#include "device.hpp"
#include "kernels.hpp"

namespace bwla {

// One product of the dot epilogue, left as a float64 pair.
template <typename C, bool COMP> __device__ __forceinline__ DD epilogue_term(C w, C y)
{
    Acc<C, COMP> a;
    a.template add_prod<false>(w, y);
    return a.to_dd();
}

template <typename T, int V, int R, int U, bool COMP>
__global__ __launch_bounds__(1024) void k_gemv_rows(int64_t L, int64_t K, const T *A, int64_t ld,
                                                    const T *v, DD *partials, void *out, int out_f64,
                                                    int split, const T *w, DD *dparts)
{
    using C = compute_t<T>;
    constexpr bool EXACT = std::is_same<T, bf16_t>::value;
    const int64_t lb = xcd_block();
    const int64_t group = lb / split;
    const int s = (int)(lb - group * split);
    const int64_t l0 = group * R;
    const int nr = (int)(L - l0 < R ? L - l0 : R);
    const T *row[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        row[r] = A + (l0 + (r < nr ? r : nr - 1)) * ld; // rows past L re-read the last one

    const int64_t kpack = K / V;
    const int64_t per = (kpack + split - 1) / split;
    const int64_t pb = (int64_t)s * per;
    const int64_t pe = pb + per < kpack ? pb + per : kpack;
    // the dot epilogue's weight of this thread's line, fetched before the
    // main loop: read at the end it would be one more memory latency in
    // every work-group's tail
    C wl = C(0);
    if (w != nullptr && split == 1 && (int)threadIdx.x < nr)
        wl = widen(w[l0 + threadIdx.x]);

    // U trips of the pack loop per iteration, all loads first: R * U packs of
    // A in flight per thread.  Each row's sum still takes the packs in the
    // order p, p + blockDim, ..., so U does not change any result.
    Acc<C, COMP> acc[R];
    int64_t p = pb + threadIdx.x;
    for (; p + (int64_t)(U - 1) * blockDim.x < pe; p += (int64_t)U * blockDim.x) {
        Pack<T, V> xv[U], av[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xv[u] = load_pack<T, V>(v + (p + (int64_t)u * blockDim.x) * V);
#pragma unroll
            for (int r = 0; r < R; ++r)
                av[u][r] = load_pack_nt<T, V>(row[r] + (p + (int64_t)u * blockDim.x) * V);
        }
        end_of_loads();
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int e = 0; e < V; ++e)
                    acc[r].template add_prod<EXACT>(widen(av[u][r].v[e]), widen(xv[u].v[e]));
    }
    for (; p < pe; p += blockDim.x) {
        Pack<T, V> xv = load_pack<T, V>(v + p * V);
        Pack<T, V> av[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            av[r] = load_pack_nt<T, V>(row[r] + p * V);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int e = 0; e < V; ++e)
                acc[r].template add_prod<EXACT>(widen(av[r].v[e]), widen(xv.v[e]));
    }
    const int64_t tail = K - kpack * V; // < V elements, taken by the last slice
    if (s == split - 1 && threadIdx.x < tail) {
        const int64_t k = kpack * V + threadIdx.x;
        C xk = widen(v[k]);
#pragma unroll
        for (int r = 0; r < R; ++r)
            acc[r].template add_prod<EXACT>(widen(row[r][k]), xk);
    }

    __shared__ DD lds[16 * R];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        DD d = wave_sum<COMP>(acc[r].to_dd());
        if (lane == 0)
            lds[wave * R + r] = d;
    }
    __syncthreads();
    DD t = {0.0, 0.0};
    if (threadIdx.x < R) {
        t = lds[threadIdx.x];
        for (int wv = 1; wv < nw; ++wv)
            t = combine<COMP>(t, lds[wv * R + threadIdx.x]);
        if (split == 1) {
            if ((int)threadIdx.x < nr)
                store_out(out, l0 + threadIdx.x, out_f64, t.hi + t.lo);
        } else {
            partials[(group * split + s) * R + threadIdx.x] = t;
        }
    }
    if (w != nullptr && split == 1 && wave == 0) { // the whole first wave
        DD d = {0.0, 0.0};
        if ((int)threadIdx.x < nr)
            d = epilogue_term<C, COMP>(wl, (C)(t.hi + t.lo));
        d = wave_sum<COMP>(d);
        if (lane == 0)
            dparts[group] = d;
    }
}

template <typename T, int V, int U, bool COMP>
__global__ __launch_bounds__(1024) void k_gemv_cols(int64_t L, int64_t K, const T *A, int64_t ld,
                                                    const T *__restrict__ v, DD *partials, void *out,
                                                    int out_f64, int split, const T *w, DD *dparts, int xchg)
{
    using C = compute_t<T>;
    constexpr bool EXACT = std::is_same<T, bf16_t>::value;
    constexpr int TK = 64 * V;
    const int64_t blk = xcd_block();
    const int64_t tile = blk / split;
    const int s = (int)(blk - tile * split);
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    // the wave index as a wave-uniform (scalar) value, so that every v[l]
    // below is one scalar load shared by the wave
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t k0 = tile * TK + (int64_t)lane * V;
    const bool full = k0 + V <= K;
    const int64_t per = (L + split - 1) / split;
    const int64_t lb = (int64_t)s * per;
    const int64_t le = lb + per < L ? lb + per : L;

    // LDS for the cross-wave combine (the hand-over path).
    __shared__ __attribute__((aligned(16))) DD red[TK];
    Acc<C, COMP> acc[V];

    // v[l] is read with the U lines' loads (no staging pass and no barrier
    // before the first loads of A).
    const T *vt = v + lb;
    const T *base = A + lb * ld + k0;
    const int64_t tn = le - lb;
    int64_t j = wave;
    if (full) {
        for (; j + (int64_t)(U - 1) * nw < tn; j += (int64_t)U * nw) {
            Pack<T, V> a[U];
            C xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                a[u] = load_pack_nt<T, V>(base + (j + (int64_t)u * nw) * ld);
                xv[u] = widen(vt[j + (int64_t)u * nw]);
            }
            end_of_loads();
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < V; ++e)
                    acc[e].template add_prod<EXACT>(widen(a[u].v[e]), xv[u]);
        }
        for (; j < tn; j += nw) {
            Pack<T, V> a = load_pack_nt<T, V>(base + j * ld);
            const C xl = widen(vt[j]);
#pragma unroll
            for (int e = 0; e < V; ++e)
                acc[e].template add_prod<EXACT>(widen(a.v[e]), xl);
        }
    } else if (k0 < K) {
        for (; j < tn; j += nw) {
            const C xl = widen(vt[j]);
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (k0 + e < K)
                    acc[e].template add_prod<EXACT>(widen(base[j * ld + e]), xl);
        }
    }

    // Combine the waves' partial sums in wave order through LDS.  With xchg
    // the launch gave every wave but the first (nw - 1) * TK pairs of dynamic
    // LDS: all waves write at once and wave 0 adds them in wave order after
    // one barrier.  Otherwise the waves hand over one at a time through a
    // buffer of one tile of pairs.  Both orders of addition are the same.
    DD d[V];
#pragma unroll
    for (int e = 0; e < V; ++e)
        d[e] = acc[e].to_dd();
    if (xchg) {
        extern __shared__ DD xs[];
        if (wave > 0)
#pragma unroll
            for (int e = 0; e < V; ++e)
                xs[(wave - 1) * TK + lane * V + e] = d[e];
        __syncthreads();
        if (wave == 0)
            for (int wv = 1; wv < nw; ++wv)
#pragma unroll
                for (int e = 0; e < V; ++e)
                    d[e] = combine<COMP>(d[e], xs[(wv - 1) * TK + lane * V + e]);
    } else {
        for (int wv = 1; wv < nw; ++wv) {
            if (wave == wv)
#pragma unroll
                for (int e = 0; e < V; ++e)
                    red[lane * V + e] = d[e];
            __syncthreads();
            if (wave == 0)
#pragma unroll
                for (int e = 0; e < V; ++e)
                    d[e] = combine<COMP>(d[e], red[lane * V + e]);
            __syncthreads();
        }
    }
    if (wave == 0) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            if (split == 1) {
                if (k0 + e < K)
                    store_out(out, k0 + e, out_f64, d[e].hi + d[e].lo);
            } else {
                partials[(tile * split + s) * TK + lane * V + e] = d[e];
            }
        }
        if (w != nullptr && split == 1) {
            DD t = {0.0, 0.0};
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (k0 + e < K)
                    t = combine<COMP>(t, epilogue_term<C, COMP>(widen(w[k0 + e]), (C)(d[e].hi + d[e].lo)));
            t = wave_sum<COMP>(t);
            if (lane == 0)
                dparts[tile] = t;
        }
    }
}

#if BWLA_T_IS_F64 // type-independent kernels live in the f64 object only
// Second stage of a split GEMV: one thread per output sums its slices' float64
// partials in slice order.  Consecutive outputs read consecutive partials.
// With w (same element type as out), the work-group also reduces w_o * y_o
// over its outputs into dparts[blockIdx.x].
// B partials in flight per round trip: the smallest power of two (2 to 16)
// that holds the split, so a split of up to 16 is one round trip.
template <bool COMP, int B>
__global__ __launch_bounds__(256) void k_combine_lines(const DD *partials, int64_t outputs, int64_t G,
                                                       int64_t split, void *out, int out_f64,
                                                       const void *w, DD *dparts)
{
    __shared__ DD lds[16];
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = o < outputs;
    double y = 0.0;
    if (live) {
        const int64_t g = o / G, r = o - g * G;
        const DD *p = partials + g * split * G + r;
        // slice order as written, B partials in flight at a time: a split of
        // s costs ceil(s / B) load round trips (one at a time, a split of 128
        // cost 32 us of load latency).  The last batch re-reads the last
        // partial in its unused places (no branch between the loads) and
        // adds only the first nb.
        DD t = {0.0, 0.0};
        for (int64_t q = 0; q < split; q += B) {
            const int64_t nb = split - q < B ? split - q : B;
            DD v[B];
#pragma unroll
            for (int b = 0; b < B; ++b)
                v[b] = p[(q + (b < nb ? b : nb - 1)) * G];
            end_of_loads();
#pragma unroll
            for (int b = 0; b < B; ++b)
                if (b < nb)
                    t = q + b == 0 ? v[0] : combine<COMP>(t, v[b]);
        }
        y = t.hi + t.lo;
        store_out(out, o, out_f64, y);
    }
    if (w == nullptr)
        return;
    DD d = {0.0, 0.0};
    if (live) {
        if (out_f64)
            d = epilogue_term<double, COMP>(reinterpret_cast<const double *>(w)[o], y);
        else
            d = epilogue_term<float, COMP>(reinterpret_cast<const float *>(w)[o], (float)y);
    }
    d = block_sum<COMP>(d, lds);
    if (threadIdx.x == 0)
        dparts[blockIdx.x] = d;
}

hipError_t launch_combine_lines(const void *partials, int64_t outputs, int64_t G, int64_t split,
                                bool comp, int out_f64, void *out, const void *w, void *dparts,
                                hipStream_t s)
{
    const int64_t blocks = (outputs + 255) / 256;
    return with_bool(comp, [&](auto CP) {
        auto go = [&](auto B) {
            hipLaunchKernelGGL((k_combine_lines<CP.value, B.value>), dim3((unsigned)blocks), dim3(256), 0, s,
                               (const DD *)partials, outputs, G, split, out, out_f64, w, (DD *)dparts);
            return hipGetLastError();
        };
        if (split <= 2)
            return go(std::integral_constant<int, 2>{});
        if (split <= 4)
            return go(std::integral_constant<int, 4>{});
        if (split <= 8)
            return go(std::integral_constant<int, 8>{});
        return go(std::integral_constant<int, 16>{});
    });
}
#endif


// Workspace: [split partials of the GEMV][dot-epilogue pairs].  With w the
// epilogue pairs are then summed into *dot by the scalar combine.
template <typename T>
hipError_t launch_gemv_rows(int64_t L, int64_t K, bool comp, const void *A, int64_t ld,
                            const void *v, int out_f64, void *out, void *ws, const Cfg &c,
                            hipStream_t s, const void *w, size_t dparts_offset, int dot_f64,
                            void *dot)
{
    DD *partials = (DD *)ws;
    DD *dparts = w ? (DD *)((char *)ws + dparts_offset) : nullptr;
    hipError_t e = with_vec(c.vec, [&](auto V) {
        return with_rows(c.rows, [&](auto R) {
            return with_bool(comp, [&](auto CP) {
                auto go = [&](auto U) {
                    const int64_t groups = (L + R.value - 1) / R.value;
                    hipLaunchKernelGGL((k_gemv_rows<T, V.value, R.value, U.value, CP.value>),
                                       dim3((unsigned)(groups * c.split)), dim3(c.block), 0, s, L, K,
                                       (const T *)A, ld, (const T *)v, partials, out, out_f64, c.split,
                                       (const T *)w, dparts);
                    return hipGetLastError();
                };
                if (c.unroll == 2)
                    return go(std::integral_constant<int, 2>{});
                return go(std::integral_constant<int, 1>{});
            });
        });
    });
    if (e == hipSuccess && c.split > 1)
        e = launch_combine_lines(partials, L, c.rows, c.split, comp, out_f64, out, w, dparts, s);
    if (e != hipSuccess || !w)
        return e;
    return launch_combine_scalar(dparts, gemv_dot_parts(true, L, K, c), comp, false, dot_f64, dot, s);
}

template <typename T>
hipError_t launch_gemv_cols(int64_t L, int64_t K, bool comp, const void *A, int64_t ld,
                            const void *v, int out_f64, void *out, void *ws, const Cfg &c,
                            hipStream_t s, const void *w, size_t dparts_offset, int dot_f64,
                            void *dot)
{
    DD *partials = (DD *)ws;
    DD *dparts = w ? (DD *)((char *)ws + dparts_offset) : nullptr;
    // lines in flight per wave: 1, 2, 4, 8, 16 or 32 (16 and 32 only within
    // kColsLoadBytes per lane; the configuration resolution keeps to that)
    auto with_unroll_cols = [](int u, auto &&f) -> hipError_t {
        switch (u) {
        case 32: return f(std::integral_constant<int, 32>{});
        case 16: return f(std::integral_constant<int, 16>{});
        case 8: return f(std::integral_constant<int, 8>{});
        }
        return with_unroll(u, f);
    };
    hipError_t e = with_vec(c.vec, [&](auto V) {
        return with_unroll_cols(c.unroll, [&](auto U) -> hipError_t {
            if constexpr (U.value > 8 && (size_t)U.value * V.value * sizeof(T) > kColsLoadBytes) {
                return hipErrorInvalidValue;
            } else {
                return with_bool(comp, [&](auto CP) {
                    const int64_t tiles = (K + 64 * V.value - 1) / (64 * V.value);
                    // the one-barrier wave combine when its exchange area is
                    // small enough not to limit how many work-groups share a CU
                    const size_t xbytes = (size_t)(c.block / 64 - 1) * 64 * V.value * sizeof(DD);
                    const int xchg = xbytes > 0 && xbytes <= kColsXchgBytes;
                    hipLaunchKernelGGL((k_gemv_cols<T, V.value, U.value, CP.value>),
                                       dim3((unsigned)(tiles * c.split)), dim3(c.block),
                                       (unsigned)(xchg ? xbytes : 0), s, L, K, (const T *)A, ld,
                                       (const T *)v, partials, out, out_f64, c.split, (const T *)w,
                                       dparts, xchg);
                    return hipGetLastError();
                });
            }
        });
    });
    if (e == hipSuccess && c.split > 1)
        e = launch_combine_lines(partials, K, 64 * (int64_t)c.vec, c.split, comp, out_f64, out, w,
                                 dparts, s);
    if (e != hipSuccess || !w)
        return e;
    return launch_combine_scalar(dparts, gemv_dot_parts(false, L, K, c), comp, false, dot_f64, dot, s);
}

template hipError_t launch_gemv_rows<BWLA_T>(int64_t, int64_t, bool, const void *, int64_t,
                                             const void *, int, void *, void *, const Cfg &,
                                             hipStream_t, const void *, size_t, int, void *);
template hipError_t launch_gemv_cols<BWLA_T>(int64_t, int64_t, bool, const void *, int64_t,
                                             const void *, int, void *, void *, const Cfg &,
                                             hipStream_t, const void *, size_t, int, void *);

} // namespace bwla
