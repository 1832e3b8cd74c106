// kernels.hpp -- host-side launchers of the gfx950 kernels (internal).  Each
// kernel source is compiled once per storage type; the API layer validates
// arguments and resolves the configuration before calling these.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace bwla {

// Resolved kernel configuration (no zero fields left).
struct Cfg {
    int block, vec, unroll, grid, inc, rows, split;
};

// The workspace of a reduction holds its float64 partials (DD pairs).
constexpr size_t kColsXchgBytes = 32768; // largest dynamic LDS of the cols kernel's wave combine
// The cols kernel keeps 16 or 32 lines in flight per wave only while the
// bytes of A each lane holds in flight stay within this (32 VGPRs): beyond
// it the loads would spill.  Up to 8 lines are always allowed.
constexpr size_t kColsLoadBytes = 128;

// Map a runtime value onto a compile-time constant for template dispatch.
template <typename F> hipError_t with_vec(int v, F &&f)
{
    switch (v) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    }
    return hipErrorInvalidValue;
}
template <typename F> hipError_t with_unroll(int u, F &&f)
{
    switch (u) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    }
    return hipErrorInvalidValue;
}
template <typename F> hipError_t with_rows(int r, F &&f)
{
    switch (r) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    }
    return hipErrorInvalidValue;
}
template <typename F> hipError_t with_bool(bool b, F &&f)
{
    if (b)
        return f(std::integral_constant<bool, true>{});
    return f(std::integral_constant<bool, false>{});
}

// --- streaming: copy, axpby, fused CG update --------------------------------
template <typename T>
hipError_t launch_copy(int64_t n, const void *y, void *x, const Cfg &c, hipStream_t s);
template <typename T>
hipError_t launch_scal(int64_t n, double alpha, const void *adev, const void *y, void *x, const Cfg &c,
                       hipStream_t s);
template <typename T>
hipError_t launch_axpby(int64_t n, double alpha, const void *adev, const void *y, double beta,
                        const void *bdev, const void *z, void *x, const Cfg &c, hipStream_t s);
template <typename T>
hipError_t launch_cg(int64_t n, bool comp, double alpha, const void *adev, void *x, const void *p,
                     void *r, const void *q, int out_f64, void *out, void *ws, const Cfg &c,
                     hipStream_t s);

// --- reductions: dot, nrm2, asum (mode kRedDot, kRedSq, kRedAbs) -----------
// Partials needed: c.grid DD pairs.
template <typename T>
hipError_t launch_dot(int64_t n, bool comp, int mode, const void *x, const void *y, int out_f64,
                      void *out, void *ws, const Cfg &c, hipStream_t s);

// --- vectors with an increment (BLAS convention; see strided.hip) ----------
enum { kElemCopy = 0, kElemAxpby = 1, kElemScal = 2 };
enum { kRedDot = 0, kRedSq = 1, kRedAbs = 2 };
constexpr int kStridedBlock = 256; // threads per work-group
constexpr int kStridedUnroll = 4;  // elements in flight per thread
// x = copy(y) / RN(fma(a, y, RN(b z))) / RN(a y) with a, b the effective
// factors (host value times *adev / *bdev when given).
template <typename T>
hipError_t launch_strided_elem(int mode, int64_t n, double alpha, const void *adev, double beta,
                               const void *bdev, const void *y, int64_t incy, const void *z, int64_t incz,
                               void *x, int64_t incx, int grid, hipStream_t s);
// <x, y>, sqrt(sum x_i^2) or sum |x_i|; `grid` DD partials in ws when grid > 1.
template <typename T>
hipError_t launch_strided_reduce(int mode, int64_t n, bool comp, const void *x, int64_t incx, const void *y,
                                 int64_t incy, int out_f64, void *out, void *ws, int grid, hipStream_t s);

// --- matrix-vector ---------------------------------------------------------
// A line is a contiguous run of K elements; lines are ld apart.
//   rows kernel:  out[l] = sum_k A[l*ld + k] * v[k]     (l < L)
//   cols kernel:  out[k] = sum_l A[l*ld + k] * v[l]     (k < K)
// ws holds the split partials from offset 0.  With w != NULL (same element
// type as out, one entry per output) the launch also writes
// *dot = sum_o w[o] * out[o], using gemv_dot_parts() float64 pairs at byte
// offset dparts_offset of ws.
template <typename T>
hipError_t launch_gemv_rows(int64_t L, int64_t K, bool comp, const void *A, int64_t ld,
                            const void *v, int out_f64, void *out, void *ws, const Cfg &c,
                            hipStream_t s, const void *w = nullptr, size_t dparts_offset = 0,
                            int dot_f64 = 1, void *dot = nullptr);
template <typename T>
hipError_t launch_gemv_cols(int64_t L, int64_t K, bool comp, const void *A, int64_t ld,
                            const void *v, int out_f64, void *out, void *ws, const Cfg &c,
                            hipStream_t s, const void *w = nullptr, size_t dparts_offset = 0,
                            int dot_f64 = 1, void *dot = nullptr);
// Number of float64 pairs the dot epilogue writes: one per work-group of the
// kernel that stores y (the rows or cols kernel, or the line combine when
// split > 1).
inline int64_t gemv_dot_parts(bool rows, int64_t L, int64_t K, const Cfg &c)
{
    const int64_t outputs = rows ? L : K;
    if (c.split > 1)
        return (outputs + 255) / 256;
    return rows ? (L + c.rows - 1) / c.rows : (K + 64 * (int64_t)c.vec - 1) / (64 * (int64_t)c.vec);
}
// --- rank-1 overwrite: A[l*ld + k] = a[l] * b[k] ---------------------------
template <typename T>
hipError_t launch_ger(int64_t L, int64_t K, const void *a, const void *b, void *A, int64_t ld,
                      const Cfg &c, hipStream_t s);

// --- zero fill of `count` outputs of float64 or float32 ---------------------
hipError_t launch_fill_zero(void *out, int64_t count, int out_f64, hipStream_t s);

// --- second stage of the reductions (type independent) ----------------------
// out = sum of `count` DD partials in index order (sqrt applied if asked).
hipError_t launch_combine_scalar(const void *partials, int64_t count, bool comp, bool do_sqrt,
                                 int out_f64, void *out, hipStream_t s);
// out[o] = sum over q < split of partials[((o / G) * split + q) * G + o % G],
// for o < outputs: the slices of a split GEMV combined in slice order.  With
// w != NULL, work-group b also writes dparts[b] = sum of w[o] * out[o] over
// its 256 outputs.
hipError_t launch_combine_lines(const void *partials, int64_t outputs, int64_t G, int64_t split,
                                bool comp, int out_f64, void *out, const void *w, void *dparts,
                                hipStream_t s);

// --- batched persistent kernel ----------------------------------------------
struct BatchItem {
    int32_t kind;   // 0 = GEMV row tile, 1 = dot chunk
    int32_t prob;   // problem index within its kind
    int64_t begin;  // first row (GEMV) or first element (dot)
    int64_t end;    // one past the last row / element
    int32_t chunk;  // chunk index within the dot
    int32_t pad;
};
// How the grouped launch reads one problem (the persistent kernel uses the
// plan-wide BatchArgs::vec instead).
enum {
    kModeStaged = 0, // GEMV with n <= tile_stage_elems(): x staged in LDS, 16-byte packs of A
    kModePacked = 1, // 16-byte packs of every operand (all of them 16-byte aligned)
    kModeScalar = 2  // one element per access
};
constexpr int kTileStageBytes = 32768; // most LDS a staged GEMV tile's x may take
constexpr int kStagedPacks = 16;       // default packs of a row each lane of a staged tile owns (sets its row-group size)
// Longest x a staged tile takes, for storage elements of `es` bytes: x is
// held in the compute precision (8 bytes for f64, 4 otherwise) in V = 16/es
// residue rows whose stride is at most ceil(n / V) + 64 words.
constexpr int tile_stage_elems(int es) { return kTileStageBytes / (es == 8 ? 8 : 4) - 64 * (16 / es); }
// Residue stride (words) of a staged x of n entries held in V residue rows
// (column c at word (c % V) * stride + c / V), read by G-lane row groups: at
// least ceil(n / V), and congruent to G modulo 64, so that row groups of one
// wave whose rows start at different residues read disjoint LDS banks.
__host__ __device__ constexpr int staged_stride(int64_t n, int V, int G)
{
    const int64_t p0 = (n + V - 1) / V;
    return (int)(p0 + ((G - p0) % 64 + 64) % 64);
}
// LDS bytes of that staged x for storage elements of `es` bytes.
constexpr size_t tile_stage_bytes(int es, int64_t n, int G)
{
    return (size_t)(16 / es) * (size_t)staged_stride(n, 16 / es, G) * (es == 8 ? 8 : 4);
}
struct BatchGemv {
    const void *A;
    int64_t m, n, lda;
    const void *x;
    void *y;
    int32_t lanes; // lanes per row (power of two, <= 64)
    int32_t mode;  // kMode*
};
struct BatchDot {
    const void *x, *y;
    int64_t n;
    void *out;
    int64_t slot0;  // first partial slot of this dot
    int32_t chunks; // number of chunks
    int32_t mode;   // kModePacked or kModeScalar
};
struct BatchArgs {
    const BatchItem *items;
    int64_t n_items;
    int64_t n_gemv_items;   // grouped launch: items[0, n_gemv_items) are GEMV tiles, the rest dot chunks
    int64_t n_staged_items; // grouped launch: of those, items[0, n_staged_items) are staged tiles
    const BatchGemv *gemv;
    const BatchDot *dots;
    double *partials;       // 2 doubles per dot chunk
    unsigned *work_counter; // next item to take
    int out_f64;
    int vec;                // elements per pack: 1 or 16 bytes' worth
};
template <typename T>
hipError_t launch_batched(const BatchArgs &a, bool comp, int grid, int block, hipStream_t s);
hipError_t launch_batch_reset(unsigned *counters, int64_t count, hipStream_t s);
// One work-group per item (a.n_items work-groups of `block` threads);
// staged tiles get `stage_bytes` of dynamic LDS.
template <typename T>
hipError_t launch_grouped(const BatchArgs &a, bool comp, int block, size_t stage_bytes, hipStream_t s);
// Combines the chunk partials of every multi-chunk dot, in chunk order.
hipError_t launch_batch_finalize(const BatchDot *dots, int64_t nd, const double *partials, bool comp,
                                 int out_f64, hipStream_t s);

} // namespace bwla
