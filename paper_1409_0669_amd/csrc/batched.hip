// batched.hip -- many uneven row-major GEMVs and dots, batched.
//
// Two designs share the work-item list.  The grouped launch (k_grouped_gemv
// and k_grouped_dot, below the persistent kernel) runs one work-group per
// item; it is the one plans use.  The persistent kernel (k_batched) keeps a
// grid sized to the machine busy from an atomic work queue; it has not been
// validated on hardware and plan creation refuses it (see api.cpp).
//
// The host flattens every problem into work items -- row tiles of a GEMV
// (full row length) and fixed-size chunks of a dot -- ordered by decreasing
// cost.  The persistent kernel would launch a grid sized to the machine and
// be wave-persistent: each wave64 repeatedly takes the next item from an atomic
// counter (lane 0 draws, readfirstlane broadcasts) until the list is
// exhausted, and reduces its item within the wave, so the kernel has no LDS
// traffic and no work-group barriers -- waves never wait for each other and
// every wave reaches the exit.  GEMV rows are handled by groups of G lanes (G
// a power of two sized to the row length), reduced by butterfly exchanges
// inside the group.  A dot chunk is reduced across the wave; a single-chunk
// dot writes its result directly, otherwise the chunk's float64 partial goes
// to a slot of the dot and a small finalize kernel combines each dot's slots
// in chunk order.  Every result depends only on its own problem's sizes, never
// on the batch order or on which wave ran which item.
#include "device.hpp"
#include "kernels.hpp"

namespace bwla {

template <typename T, int V, bool COMP>
__device__ __forceinline__ void gemv_tile(const BatchGemv &g, int64_t rb, int64_t re, int out_f64)
{
    using C = compute_t<T>;
    constexpr bool EXACT = std::is_same<T, bf16_t>::value;
    const int lane = threadIdx.x & 63;
    const int G = g.lanes;
    const int rpw = 64 / G;
    const int sub = lane / G, gl = lane - sub * G;
    const T *A = (const T *)g.A;
    const T *x = (const T *)g.x;
    const int64_t K = g.n, kpack = K / V;
    for (int64_t base = rb; base < re; base += rpw) {
        const int64_t r = base + sub;
        const int64_t rr = r < re ? r : re - 1;
        const T *row = A + rr * g.lda;
        Acc<C, COMP> acc;
        for (int64_t p = gl; p < kpack; p += G) {
            Pack<T, V> av = load_pack<T, V>(row + p * V), xv = load_pack<T, V>(x + p * V);
#pragma unroll
            for (int e = 0; e < V; ++e)
                acc.template add_prod<EXACT>(widen(av.v[e]), widen(xv.v[e]));
        }
        for (int64_t k = kpack * V + gl; k < K; k += G)
            acc.template add_prod<EXACT>(widen(row[k]), widen(x[k]));
        DD d = acc.to_dd();
        for (int m = G >> 1; m >= 1; m >>= 1)
            d = combine<COMP>(d, shfl_xor_dd(d, m));
        if (gl == 0 && r < re)
            store_out(g.y, r, out_f64, d.hi + d.lo);
    }
}

template <typename T, int V, bool COMP>
__device__ __forceinline__ void dot_chunk(const BatchArgs &a, const BatchItem &w)
{
    using C = compute_t<T>;
    constexpr bool EXACT = std::is_same<T, bf16_t>::value;
    const int lane = threadIdx.x & 63;
    const BatchDot &d = a.dots[w.prob];
    const T *x = (const T *)d.x, *y = (const T *)d.y;
    Acc<C, COMP> acc[2];
    const int64_t pb = w.begin / V, pe = w.end / V; // chunk starts are pack-aligned
    int64_t p = pb + lane;
    for (; p + 64 < pe; p += 128) {
        Pack<T, V> x0 = load_pack<T, V>(x + p * V), y0 = load_pack<T, V>(y + p * V);
        Pack<T, V> x1 = load_pack<T, V>(x + (p + 64) * V), y1 = load_pack<T, V>(y + (p + 64) * V);
#pragma unroll
        for (int e = 0; e < V; ++e) {
            acc[0].template add_prod<EXACT>(widen(x0.v[e]), widen(y0.v[e]));
            acc[1].template add_prod<EXACT>(widen(x1.v[e]), widen(y1.v[e]));
        }
    }
    for (; p < pe; p += 64) {
        Pack<T, V> x0 = load_pack<T, V>(x + p * V), y0 = load_pack<T, V>(y + p * V);
#pragma unroll
        for (int e = 0; e < V; ++e)
            acc[0].template add_prod<EXACT>(widen(x0.v[e]), widen(y0.v[e]));
    }
    const int64_t tail = w.end - pe * V; // < V, only in a dot's last chunk
    if (lane < tail)
        acc[0].template add_prod<EXACT>(widen(x[pe * V + lane]), widen(y[pe * V + lane]));
    DD v = wave_sum<COMP>(combine<COMP>(acc[0].to_dd(), acc[1].to_dd()));
    if (lane == 0) {
        if (d.chunks == 1)
            store_out(d.out, 0, a.out_f64, v.hi + v.lo);
        else
            reinterpret_cast<DD *>(a.partials)[d.slot0 + w.chunk] = v;
    }
}

template <typename T, int V, bool COMP>
__global__ __launch_bounds__(1024) void k_batched(BatchArgs a)
{
    const int lane = threadIdx.x & 63;
    // Each trip takes a distinct item from the counter, so no wave can make
    // more than n_items trips; the bound ends the loop even if a draw went
    // wrong.
    for (int64_t trip = 0; trip <= a.n_items; ++trip) {
        // Every lane takes part in the draw (lane 0 adds 1, the others 0) and
        // readfirstlane then returns lane 0's value.  No branch here depends on
        // the lane: with the draw under `if (lane == 0)` the compiler may split
        // the loop on that condition, so that lanes 1..63 re-enter it without
        // lane 0 and readfirstlane returns their stale value instead.
        const unsigned got = atomicAdd(a.work_counter, lane == 0 ? 1u : 0u);
        const int64_t it = (int64_t)__builtin_amdgcn_readfirstlane(got);
        if (it >= a.n_items)
            break;
        const BatchItem w = a.items[it];
        if (w.kind == 0)
            gemv_tile<T, V, COMP>(a.gemv[w.prob], w.begin, w.end, a.out_f64);
        else
            dot_chunk<T, V, COMP>(a, w);
    }
}

// ---------------------------------------------------------------------------
// Grouped launch: one work-group per work item, no work queue.  Items are
// ordered largest first and the hardware dispatcher hands work-groups to CUs
// in index order as they free up, which schedules the items the way a
// largest-first queue would -- without a software loop over items, without
// atomics, and with barriers only in straight-line code.
// ---------------------------------------------------------------------------
// Rows of one GEMV tile, one G-lane group per row as in gemv_tile, but each
// group carries kTileRowsInFlight rows at once and each lane kTilePacksInFlight
// packs of each row, so that one trip issues all their loads (and the shared
// packs of x) before any arithmetic.  Loop control is wave-uniform; rows past
// the tile re-read its last row and are not stored.  No barriers.
constexpr int kTileRowsInFlight = 4;
constexpr int kTilePacksInFlight = 2;

template <typename T, int V, bool COMP>
__device__ __forceinline__ void gemv_tile_block(const BatchGemv &g, int64_t rb, int64_t re, int out_f64)
{
    using C = compute_t<T>;
    constexpr bool EXACT = std::is_same<T, bf16_t>::value;
    constexpr int RB = kTileRowsInFlight, U = kTilePacksInFlight;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int G = g.lanes;
    const int rpw = 64 / G;
    const int sub = lane / G, gl = lane - sub * G;
    const T *A = (const T *)g.A;
    const T *x = (const T *)g.x;
    const int64_t K = g.n, kpack = K / V;
    const int64_t slots = (int64_t)nw * rpw; // rows the work-group holds per row batch
    for (int64_t base = rb + (int64_t)wave * rpw; base < re; base += RB * slots) {
        const T *row[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            const int64_t r = base + j * slots + sub;
            row[j] = A + (r < re ? r : re - 1) * g.lda;
        }
        Acc<C, COMP> acc[RB];
        int64_t p = gl;
        for (; p + (int64_t)(U - 1) * G < kpack; p += (int64_t)U * G) {
            Pack<T, V> xv[U], av[RB][U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                xv[u] = load_pack<T, V>(x + (p + (int64_t)u * G) * V);
#pragma unroll
            for (int j = 0; j < RB; ++j)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    av[j][u] = load_pack_nt<T, V>(row[j] + (p + (int64_t)u * G) * V);
#pragma unroll
            for (int j = 0; j < RB; ++j)
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        acc[j].template add_prod<EXACT>(widen(av[j][u].v[e]), widen(xv[u].v[e]));
        }
        for (; p < kpack; p += G) {
            const Pack<T, V> xv = load_pack<T, V>(x + p * V);
            Pack<T, V> av[RB];
#pragma unroll
            for (int j = 0; j < RB; ++j)
                av[j] = load_pack_nt<T, V>(row[j] + p * V);
#pragma unroll
            for (int j = 0; j < RB; ++j)
#pragma unroll
                for (int e = 0; e < V; ++e)
                    acc[j].template add_prod<EXACT>(widen(av[j].v[e]), widen(xv.v[e]));
        }
        for (int64_t k = kpack * V + gl; k < K; k += G) {
            const C xk = widen(x[k]);
#pragma unroll
            for (int j = 0; j < RB; ++j)
                acc[j].template add_prod<EXACT>(widen(row[j][k]), xk);
        }
#pragma unroll
        for (int j = 0; j < RB; ++j) {
            DD d = acc[j].to_dd();
            for (int m = G >> 1; m >= 1; m >>= 1)
                d = combine<COMP>(d, shfl_xor_dd(d, m));
            const int64_t r = base + j * slots + sub;
            if (gl == 0 && r < re)
                store_out(g.y, r, out_f64, d.hi + d.lo);
        }
    }
}

// GEMV tile with x staged in LDS, for rows of at most tile_stage_elems()
// entries.  Rows may start anywhere (lda need not keep them 16-byte
// aligned): each row is read as a head of h < V elements up to its first
// 16-byte boundary, then whole 16-byte packs, then a tail of fewer than V
// elements, and the x entry of every A entry comes from LDS.  x is held
// interleaved by column residue, xs[(c % V) * P + c / V], so the lanes of a
// group -- which take consecutive packs -- read consecutive LDS words for each
// element position of a pack, whatever the row's head.  The residue stride P
// is congruent to G modulo 64, so groups of one wave whose rows start at
// different residues read disjoint banks.
//
// A row belongs to a group of G lanes (a compile-time constant here, so every
// LDS and global offset within a trip is an immediate), G sized on the host
// so that each lane owns about the plan's packs per lane (the batch table
// entry's unroll, kStagedPacks by default) of it.  One trip issues the
// U packs of A and their U*V x entries before any arithmetic; two
// accumulators per lane split the dependency chain.  Loop control is
// wave-uniform; rows past the tile re-read its last row and are not stored.
template <typename T, int V, bool COMP, int G>
__device__ __forceinline__ void staged_rows(const BatchGemv &g, int64_t rb, int64_t re, int out_f64,
                                            const compute_t<T> *xs, int P)
{
    using C = compute_t<T>;
    constexpr bool EXACT = std::is_same<T, bf16_t>::value;
    // packs in flight per trip: 8 for 2-element packs, 4 for 4- and
    // 8-element packs (whose x values per trip would not fit the registers)
    constexpr int U = V >= 4 ? 4 : 8;
    constexpr int RPW = 64 / G;
    const int n = (int)g.n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int sub = lane / G, gl = lane % G;
    const T *A = (const T *)g.A;
    const int64_t slots = (int64_t)nw * RPW;
    for (int64_t base = rb + (int64_t)wave * RPW; base < re; base += slots) {
        const int64_t r = base + sub;
        const T *row = A + (r < re ? r : re - 1) * g.lda;
        const int mis = (int)(((uintptr_t)row & 15) / sizeof(T)); // elements past a 16-byte boundary
        const int h = mis ? (V - mis < n ? V - mis : n) : 0;
        const int np = (n - h) / V;
        const int t0 = h + np * V;
        // head (h < V elements before the first 16-byte boundary) and tail
        // (< V elements after the last whole pack): lane gl takes element gl
        // of each; rows with G < V lanes finish them after the packs
        const T hv = gl < h ? row[gl] : T(0);
        const T tv = t0 + gl < n ? row[t0 + gl] : T(0);
        // x entry of element e of this lane's k-th pack (column
        // h + (gl + k G) V + e): xs[xo[e] + k G].  Word offsets from the LDS
        // array itself (not pointers advanced in the loop), so that the
        // reads stay LDS reads with immediate offsets.
        int xo[V];
#pragma unroll
        for (int e = 0; e < V; ++e)
            xo[e] = ((h + e) % V) * P + (h + e) / V + gl;
        const T *ap = row + h + (int64_t)gl * V;
        Acc<C, COMP> acc[2];
        int p = gl;
        for (; p + (U - 1) * G < np; p += U * G) {
            Pack<T, V> av[U];
            C xv[U][V];
#pragma unroll
            for (int u = 0; u < U; ++u)
                av[u] = load_pack_nt<T, V>(ap + u * G * V);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < V; ++e)
                    xv[u][e] = xs[xo[e] + u * G];
            end_of_loads();
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < V; ++e)
                    acc[u & 1].template add_prod<EXACT>(widen(av[u].v[e]), xv[u][e]);
            ap += U * G * V;
#pragma unroll
            for (int e = 0; e < V; ++e)
                xo[e] += U * G;
        }
        for (; p < np; p += G) {
            const Pack<T, V> a = load_pack_nt<T, V>(ap);
            C xv[V];
#pragma unroll
            for (int e = 0; e < V; ++e)
                xv[e] = xs[xo[e]];
#pragma unroll
            for (int e = 0; e < V; ++e)
                acc[0].template add_prod<EXACT>(widen(a.v[e]), xv[e]);
            ap += G * V;
#pragma unroll
            for (int e = 0; e < V; ++e)
                xo[e] += G;
        }
        if (gl < h)
            acc[1].template add_prod<EXACT>(widen(hv), xs[(gl % V) * P + gl / V]);
        if (t0 + gl < n)
            acc[1].template add_prod<EXACT>(widen(tv), xs[((t0 + gl) % V) * P + (t0 + gl) / V]);
        for (int k = gl + G; k < h; k += G) // only when G < V
            acc[1].template add_prod<EXACT>(widen(row[k]), xs[(k % V) * P + k / V]);
        for (int k = t0 + gl + G; k < n; k += G)
            acc[1].template add_prod<EXACT>(widen(row[k]), xs[(k % V) * P + k / V]);
        DD d = combine<COMP>(acc[0].to_dd(), acc[1].to_dd());
#pragma unroll
        for (int m = G >> 1; m >= 1; m >>= 1)
            d = combine<COMP>(d, shfl_xor_dd(d, m));
        if (gl == 0 && r < re)
            store_out(g.y, r, out_f64, d.hi + d.lo);
    }
}

// Stages x (widened to the compute type) in LDS, then runs the rows of the
// tile with the row-group size the host chose.  Contains a barrier: every
// thread of the work-group calls it.
template <typename T, int V, bool COMP>
__device__ __forceinline__ void gemv_tile_staged(const BatchGemv &g, int64_t rb, int64_t re, int out_f64,
                                                 compute_t<T> *xs)
{
    using C = compute_t<T>;
    // Each thread stages whole pack columns q (x entries qV .. qV + V - 1 to
    // words e * P + q), SQ columns per round so that 8 entries are in flight:
    // consecutive threads then write consecutive words of each residue row,
    // free of bank conflicts whatever P is.
    constexpr int SQ = V >= 8 ? 1 : 8 / V;
    const int n = (int)g.n;
    const int G = __builtin_amdgcn_readfirstlane(g.lanes);
    const int P = staged_stride(n, V, G);
    const int nq = (n + V - 1) / V;
    const T *x = (const T *)g.x;
    for (int q0 = threadIdx.x; q0 < nq; q0 += SQ * blockDim.x) {
        C v[SQ][V];
#pragma unroll
        for (int k = 0; k < SQ; ++k)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int c = (q0 + k * (int)blockDim.x) * V + e;
                v[k][e] = c < n ? widen(x[c]) : C(0);
            }
#pragma unroll
        for (int k = 0; k < SQ; ++k) {
            const int q = q0 + k * (int)blockDim.x;
            if (q < nq)
#pragma unroll
                for (int e = 0; e < V; ++e)
                    xs[e * P + q] = v[k][e];
        }
    }
    __syncthreads();
    switch (G) {
    case 1: staged_rows<T, V, COMP, 1>(g, rb, re, out_f64, xs, P); break;
    case 2: staged_rows<T, V, COMP, 2>(g, rb, re, out_f64, xs, P); break;
    case 4: staged_rows<T, V, COMP, 4>(g, rb, re, out_f64, xs, P); break;
    case 8: staged_rows<T, V, COMP, 8>(g, rb, re, out_f64, xs, P); break;
    case 16: staged_rows<T, V, COMP, 16>(g, rb, re, out_f64, xs, P); break;
    case 32: staged_rows<T, V, COMP, 32>(g, rb, re, out_f64, xs, P); break;
    default: staged_rows<T, V, COMP, 64>(g, rb, re, out_f64, xs, P); break;
    }
}

// One dot chunk reduced by a whole work-group: each thread keeps
// kChunkPacksInFlight packs of both operands in flight per trip, two
// accumulators, then the work-group tree (block_sum, barriers in
// straight-line code).
constexpr int kChunkPacksInFlight = 8;

template <typename T, int V, bool COMP>
__device__ __forceinline__ void dot_chunk_block(const BatchArgs &a, const BatchItem &w, DD *lds)
{
    using C = compute_t<T>;
    constexpr bool EXACT = std::is_same<T, bf16_t>::value;
    constexpr int U = kChunkPacksInFlight;
    const BatchDot &d = a.dots[w.prob];
    const T *x = (const T *)d.x, *y = (const T *)d.y;
    Acc<C, COMP> acc[2];
    const int64_t pb = w.begin / V, pe = w.end / V; // chunk starts are pack-aligned
    const int64_t step = blockDim.x;
    int64_t p = pb + threadIdx.x;
    for (; p + (U - 1) * step < pe; p += U * step) {
        Pack<T, V> xs[U], ys[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xs[u] = load_pack_nt<T, V>(x + (p + u * step) * V);
            ys[u] = load_pack_nt<T, V>(y + (p + u * step) * V);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e)
                acc[u & 1].template add_prod<EXACT>(widen(xs[u].v[e]), widen(ys[u].v[e]));
    }
    for (; p < pe; p += step) {
        const Pack<T, V> x0 = load_pack_nt<T, V>(x + p * V), y0 = load_pack_nt<T, V>(y + p * V);
#pragma unroll
        for (int e = 0; e < V; ++e)
            acc[0].template add_prod<EXACT>(widen(x0.v[e]), widen(y0.v[e]));
    }
    const int64_t tail = w.end - pe * V; // < V, only in a dot's last chunk
    if (threadIdx.x < tail)
        acc[0].template add_prod<EXACT>(widen(x[pe * V + threadIdx.x]), widen(y[pe * V + threadIdx.x]));
    DD v = block_sum<COMP>(combine<COMP>(acc[0].to_dd(), acc[1].to_dd()), lds);
    if (threadIdx.x == 0) {
        if (d.chunks == 1)
            store_out(d.out, 0, a.out_f64, v.hi + v.lo);
        else
            reinterpret_cast<DD *>(a.partials)[d.slot0 + w.chunk] = v;
    }
}

// Three kernels: staged GEMV items (a.items[0, a.n_staged_items)), the
// other GEMV items (up to a.n_gemv_items) and dot items (the rest), so that
// each gets the registers (and the staged tiles the LDS) of its own code
// paths.  The staged kernel's x stage is dynamic LDS, sized by the plan for
// its longest staged x.  Its waits on memory and LDS are hidden by other
// waves, so it asks for 6 waves per SIMD where that costs no spills (f32:
// 79 VGPRs); the bf16 and f64 forms are left to the compiler (98-130
// VGPRs; asked for more waves, they spill).
template <typename T, bool COMP>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(std::is_same<T, float>::value ? 6 : 1, 8)))
void k_grouped_gemv_staged(BatchArgs a)
{
    using C = compute_t<T>;
    constexpr int NATIVE = 16 / (int)sizeof(T);
    extern __shared__ __attribute__((aligned(16))) char stage[];
    const BatchItem w = a.items[blockIdx.x];
    gemv_tile_staged<T, NATIVE, COMP>(a.gemv[w.prob], w.begin, w.end, a.out_f64, reinterpret_cast<C *>(stage));
}

template <typename T, bool COMP>
__global__ __launch_bounds__(512) void k_grouped_gemv(BatchArgs a)
{
    constexpr int NATIVE = 16 / (int)sizeof(T);
    const BatchItem w = a.items[a.n_staged_items + blockIdx.x];
    const BatchGemv &g = a.gemv[w.prob];
    // the item is the same for every thread of the work-group
    const int mode = __builtin_amdgcn_readfirstlane(g.mode);
    if (mode == kModePacked)
        gemv_tile_block<T, NATIVE, COMP>(g, w.begin, w.end, a.out_f64);
    else
        gemv_tile_block<T, 1, COMP>(g, w.begin, w.end, a.out_f64);
}

template <typename T, bool COMP>
__global__ __launch_bounds__(512) void k_grouped_dot(BatchArgs a)
{
    constexpr int NATIVE = 16 / (int)sizeof(T);
    __shared__ DD lds[16];
    const BatchItem w = a.items[a.n_gemv_items + blockIdx.x];
    const int mode = __builtin_amdgcn_readfirstlane(a.dots[w.prob].mode); // block_sum holds barriers
    if (mode == kModePacked)
        dot_chunk_block<T, NATIVE, COMP>(a, w, lds);
    else
        dot_chunk_block<T, 1, COMP>(a, w, lds);
}

#if BWLA_T_IS_F64 // type-independent kernels live in the f64 object only
__global__ void k_zero_counters(unsigned *c, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        c[i] = 0u;
}

// One thread per dot: combine the chunk partials of multi-chunk dots in
// chunk order (single-chunk dots were written by the batched kernel).
template <bool COMP>
__global__ __launch_bounds__(256) void k_batch_finalize(const BatchDot *dots, int64_t nd, const DD *partials,
                                                        int out_f64)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd)
        return;
    const BatchDot d = dots[i];
    if (d.chunks <= 1)
        return;
    const DD *p = partials + d.slot0;
    DD t = p[0];
    for (int c = 1; c < d.chunks; ++c)
        t = combine<COMP>(t, p[c]);
    store_out(d.out, 0, out_f64, t.hi + t.lo);
}
#endif

template <typename T>
hipError_t launch_batched(const BatchArgs &a, bool comp, int grid, int block, hipStream_t s)
{
    constexpr int NATIVE = 16 / (int)sizeof(T);
    auto go = [&](auto V) {
        return with_bool(comp, [&](auto CP) {
            hipLaunchKernelGGL((k_batched<T, V.value, CP.value>), dim3(grid), dim3(block), 0, s, a);
            return hipGetLastError();
        });
    };
    if (a.vec == 1)
        return go(std::integral_constant<int, 1>{});
    return go(std::integral_constant<int, NATIVE>{});
}

template hipError_t launch_batched<BWLA_T>(const BatchArgs &, bool, int, int, hipStream_t);

template <typename T>
hipError_t launch_grouped(const BatchArgs &a, bool comp, int block, size_t stage_bytes, hipStream_t s)
{
    return with_bool(comp, [&](auto CP) {
        const int64_t ng = a.n_gemv_items - a.n_staged_items, nd = a.n_items - a.n_gemv_items;
        if (a.n_staged_items > 0)
            hipLaunchKernelGGL((k_grouped_gemv_staged<T, CP.value>), dim3((unsigned)a.n_staged_items), dim3(block),
                               (unsigned)stage_bytes, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        if (ng > 0)
            hipLaunchKernelGGL((k_grouped_gemv<T, CP.value>), dim3((unsigned)ng), dim3(block), 0, s, a);
        e = hipGetLastError();
        if (e != hipSuccess || nd <= 0)
            return e;
        hipLaunchKernelGGL((k_grouped_dot<T, CP.value>), dim3((unsigned)nd), dim3(block), 0, s, a);
        return hipGetLastError();
    });
}

template hipError_t launch_grouped<BWLA_T>(const BatchArgs &, bool, int, size_t, hipStream_t);

#if BWLA_T_IS_F64
hipError_t launch_batch_reset(unsigned *counters, int64_t count, hipStream_t s)
{
    int64_t blocks = (count + 255) / 256;
    if (blocks > 1024)
        blocks = 1024;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(k_zero_counters, dim3((unsigned)blocks), dim3(256), 0, s, counters, count);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchDot *dots, int64_t nd, const double *partials, bool comp,
                                 int out_f64, hipStream_t s)
{
    if (nd <= 0)
        return hipSuccess;
    const int64_t blocks = (nd + 255) / 256;
    return with_bool(comp, [&](auto CP) {
        hipLaunchKernelGGL((k_batch_finalize<CP.value>), dim3((unsigned)blocks), dim3(256), 0, s, dots, nd,
                           (const DD *)partials, out_f64);
        return hipGetLastError();
    });
}
#endif

} // namespace bwla
