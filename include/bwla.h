/*
 * bwla.h -- C ABI of the bandwidth-limited linear algebra library for AMD
 * Instinct MI355X (gfx950).
 *
 * The operations are those whose performance portability is studied in
 * Rupp, Tillet, Rudolf, Weinbub, Grasser, Juengel, "Performance Portability
 * Study of Linear Algebra Kernels in OpenCL", IWOCL 2014 (arXiv:1409.0669),
 * Section 2: vector copy x <- y, scaled vector addition x <- alpha y + beta z,
 * the inner product <x, y>, and the dense matrix-vector product; plus the
 * Euclidean norm, the transposed product and the rank-1 overwrite needed for
 * gradients, a batched launch for many uneven problems, and a fused
 * conjugate-gradient-style update.
 *
 * Conventions shared by every entry point
 *  - All data pointers are DEVICE pointers owned by the caller.  The library
 *    never frees them and keeps no reference after the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is only enqueued; no call synchronises the host with the device.
 *  - Sizes and leading dimensions are int64_t element counts.
 *  - Arguments are validated before anything is enqueued; on any error code
 *    nothing was enqueued, and bwla_last_error() holds a message for the
 *    calling thread.  Device faults surface at the caller's next
 *    synchronisation, as with any HIP kernel.
 *  - Storage types: BWLA_F64 (double), BWLA_F32 (float), BWLA_BF16 (bfloat16).
 *    Arithmetic is carried out in the "compute precision": double for f64
 *    storage, float for f32 and bf16 storage.  Every conversion to a narrower
 *    format rounds to nearest, ties to even.
 *  - Reductions (dot, nrm2, gemv, cg_update) take a workspace `ws` of at
 *    least bwla_workspace_size() bytes for the float64 partial sums of their
 *    first stage; a second small kernel combines them in a fixed order.  Its
 *    contents on entry do not matter.  One workspace serves any sequence of
 *    calls on ONE stream; calls that may run concurrently (other streams)
 *    need separate workspaces.  ws may be NULL when the size is 0.  No entry
 *    point allocates device memory except bwla_batch_plan_create.
 */
#ifndef BWLA_H
#define BWLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BWLA_ABI_VERSION 4

/* In C++ the enumerations below have int as their fixed underlying type, so
 * every int a caller passes is a value of the parameter's type and the library
 * can reject the ones it does not know (without it, an out-of-range value is
 * undefined behaviour in C++).  In C an enumeration argument is an int. */
#ifdef __cplusplus
#define BWLA_ENUM_INT : int
#else
#define BWLA_ENUM_INT
#endif

typedef enum BWLA_ENUM_INT {
    BWLA_OK = 0,
    BWLA_ERR_INVALID_ARG = 1,   /* negative size, NULL pointer, bad lda, overlap */
    BWLA_ERR_UNSUPPORTED = 2,   /* dtype / accumulation / output-type combination */
    BWLA_ERR_WORKSPACE = 3,     /* ws missing or smaller than bwla_workspace_size() */
    BWLA_ERR_HIP = 4,           /* a HIP runtime call or kernel launch failed */
    BWLA_ERR_NOT_CAPTURABLE = 5 /* the call would allocate while the stream is capturing */
} bwla_status;

typedef enum BWLA_ENUM_INT { BWLA_F64 = 0, BWLA_F32 = 1, BWLA_BF16 = 2 } bwla_dtype;
typedef enum BWLA_ENUM_INT { BWLA_ROW_MAJOR = 0, BWLA_COL_MAJOR = 1 } bwla_layout;

/* Accumulation of reductions.  PLAIN: one running sum per thread in the
 * compute precision.  COMPENSATED: the running sum carries its rounding error
 * (TwoSum) and, for f64/f32, the product error (TwoProduct by fma) -- the
 * Dot2 scheme of Ogita, Rump and Oishi; for bf16 the products are exact in
 * f32 and only the sum is compensated (Kahan-style).  In both modes, partial
 * sums leave the thread as float64 and every combine across threads and
 * work-groups is done in float64 (double-float64 pairs when COMPENSATED). */
typedef enum BWLA_ENUM_INT { BWLA_ACC_PLAIN = 0, BWLA_ACC_COMPENSATED = 1 } bwla_acc;

/* Loop increment of the streaming kernels, the paper's two kernel skeletons
 * (Section 2): GLOBAL advances each thread by the whole grid; LOCAL gives each
 * work-group one contiguous chunk, advanced by the work-group size. */
typedef enum BWLA_ENUM_INT { BWLA_INC_GLOBAL = 0, BWLA_INC_LOCAL = 1 } bwla_increment;

typedef enum BWLA_ENUM_INT {
    BWLA_OP_COPY = 0,
    BWLA_OP_AXPBY = 1,
    BWLA_OP_DOT = 2,
    BWLA_OP_GEMV_ROWS = 3, /* each output is a reduction along a contiguous line of A */
    BWLA_OP_GEMV_COLS = 4, /* each output runs along a contiguous line; reduction across lines */
    BWLA_OP_GER = 5,
    BWLA_OP_NRM2 = 6,
    BWLA_OP_CG = 7,        /* the fused CG-style update */
    BWLA_OP_BATCH = 8,     /* the batch plans (bwla_batch_plan_create) */
    BWLA_OP_COUNT = 9
} bwla_op;

/* Kernel configuration: the paper's triple (kernel source, local work size,
 * global work size; Section 1 and Section 2) with the source variant spelled
 * out.  A zero field means "library default".  Which fields an op uses:
 *   COPY, AXPBY, DOT, NRM2, CG: block, vec, unroll, grid, increment
 *   GEMV_ROWS:        block, vec, rows (lines per block), unroll (packs of each
 *                     line in flight: 1 or 2), split (blocks along a line), grid
 *   GEMV_COLS:        block, vec, unroll (lines in flight), split (blocks across
 *                     lines), grid
 *   GER:              block, vec, rows
 *   BATCH:            block (work-group size, at most 512), unroll (packs of a
 *                     GEMV row each lane of a staged tile owns: sets how many
 *                     lanes share a row); its size class is that of the plan's
 *                     algorithmic bytes
 * block:  threads per work-group, a multiple of 64 in [64, 1024]
 * vec:    consecutive elements per thread per access: 1, 2, 4, 8 or 16 (the
 *         paper's vector data types); widths above 16 bytes are issued as
 *         several 16-byte loads
 * unroll: independent accesses in flight per thread per iteration: 1, 2, 4,
 *         8, 16 or 32 (the streaming operations take up to 4, DOT and NRM2 up
 *         to 8; GEMV_COLS takes 16 and 32 while those lines hold at most 128
 *         bytes of A per thread, and halves larger values until they do)
 * GEMV_ROWS work-groups are never larger than the packs of one slice of a
 * line (rounded up to 64 threads), whatever the table says.
 * grid:   number of work-groups (streaming and reductions).  For GEMV_ROWS
 *         and GEMV_COLS with split 0, a nonzero grid is the number of
 *         work-groups the split aims for on every shape: split =
 *         ceil(grid / output tiles), so an entry tuned on one shape of a
 *         size class keeps its work-group count on other aspect ratios.
 *         bwla_get_config reports in grid the work-groups a GEMV launches.
 * rows:   1, 2, 4 or 8
 * split:  >= 1; values above 1 make several work-groups share one output
 *         tile, combining their float64 partials in a fixed order.  0: from
 *         grid, or (grid 0) a library heuristic that follows the shape. */
typedef struct {
    int32_t block, vec, unroll, grid, increment, rows, split;
} bwla_config;

/* ---- vector copy: x <- y (paper Section 2, first kernel) ----------------
 * n >= 0 elements of type t.  x may equal y (no-op); partial overlap is an
 * error.  Nothing is enqueued for n == 0. */
bwla_status bwla_copy(bwla_dtype t, int64_t n, const void *y, void *x, void *stream);

/* ---- scaled vector addition: x <- alpha y + beta z (paper Section 2) ------
 * Effective factors (compute precision c): a = RN_c(alpha) if alpha_dev is
 * NULL, else RN_c(RN_c(alpha) * (*alpha_dev)); likewise b.  alpha_dev and
 * beta_dev, when given, point to ONE device element of the compute type
 * (double for f64 storage, float otherwise).  Each element is computed as
 *     x_i = RN_t( fma_c(a, y_i, RN_c(b * z_i)) )
 * so the result is bitwise reproducible.  z is read even when b == 0 (IEEE
 * semantics).  x may equal y or z exactly (in-place updates); partial overlap
 * is an error. */
bwla_status bwla_axpby(bwla_dtype t, int64_t n, double alpha, const void *alpha_dev,
                       const void *y, double beta, const void *beta_dev, const void *z,
                       void *x, void *stream);

/* ---- inner product: out <- <x, y> (paper Section 2, inner product) --------
 * Two-stage reduction: each work-group writes a float64 partial, and a
 * second one-work-group kernel combines all partials in a fixed order, so
 * the result is deterministic for a given configuration.  out is
 * ONE device element of out_t: BWLA_F64 for f64 input; BWLA_F32 or BWLA_F64
 * for f32/bf16 input.  n == 0 writes 0. */
bwla_status bwla_dot(bwla_dtype t, bwla_acc acc, int64_t n, const void *x, const void *y,
                     bwla_dtype out_t, void *out, void *ws, size_t ws_bytes, void *stream);

/* ---- inner product without a workspace -----------------------------------
 * For callers that cannot allocate or pass device memory for partials (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Computes exactly what bwla_dot computes -- same kernels, same
 * configuration, bitwise the same result -- but keeps the first stage's
 * float64 partials in a static device array of the library (1 MiB per GPU,
 * 65536 pairs, held from the first call on that GPU until the process
 * ends) instead of a caller workspace.  It calls no allocating routine.  A
 * configuration needing more partials than the array holds is refused with
 * BWLA_ERR_WORKSPACE (the default and tuned configurations never do: the
 * grid of a reduction is capped at 65536 work-groups).  Every call on one
 * GPU shares that GPU's array: calls that may overlap on one GPU (several
 * streams, several host threads) race and must be serialised by the caller.
 * Arguments, errors and the n == 0 case are as for bwla_dot. */
bwla_status bwla_dot_noalloc(bwla_dtype t, bwla_acc acc, int64_t n, const void *x, const void *y,
                             bwla_dtype out_t, void *out, void *stream);

/* ---- Euclidean norm: out <- sqrt(<x, x>) (no overflow scaling) -------------
 * Same reduction as bwla_dot on (x, x), reading x once. */
bwla_status bwla_nrm2(bwla_dtype t, bwla_acc acc, int64_t n, const void *x,
                      bwla_dtype out_t, void *out, void *ws, size_t ws_bytes, void *stream);

/* ---- vectors with an increment ----------------------------------------------
 * The paper's Section 2 builds the level-1 and level-2 BLAS from these
 * operations and notes that its vector data types suit strided vectors
 * poorly; these entry points complete the BLAS-style interface.  A vector is
 * (p, n, inc) in the reference-BLAS convention: logical element i is at
 * p[i*inc] for inc >= 0 and at p[(n-1-i)*|inc|] for inc < 0 (a negative
 * increment walks the buffer backwards from its far end).  inc == 0 repeats
 * p[0] and is allowed for inputs only.  Arithmetic and rounding are exactly
 * those of the unit-increment operation; with every increment 1 the call is
 * the unit-increment one (packed kernels).  Otherwise each element is moved
 * on its own (no 16-byte packs across a stride).  An output may alias an
 * input exactly (same pointer and increment); any other shared byte is an
 * error (interleaved vectors with equal |inc| that share no element are
 * fine).  (n - 1) * |inc| * element size must stay below 2^60. */
bwla_status bwla_copy_strided(bwla_dtype t, int64_t n, const void *y, int64_t incy, void *x,
                              int64_t incx, void *stream);
bwla_status bwla_axpby_strided(bwla_dtype t, int64_t n, double alpha, const void *alpha_dev,
                               const void *y, int64_t incy, double beta, const void *beta_dev,
                               const void *z, int64_t incz, void *x, int64_t incx, void *stream);
/* x <- alpha x in place (the BLAS scal): x_i = RN_t(a * x_i) with a the
 * effective factor as in bwla_axpby.  One product per element, so infinite
 * and NaN entries scale as IEEE products do (unlike axpby with beta = 0,
 * which forms 0 * z). */
bwla_status bwla_scal(bwla_dtype t, int64_t n, double alpha, const void *alpha_dev, void *x,
                      int64_t incx, void *stream);
/* ---- out-of-place scaling: x <- alpha y, unit increments ------------------
 * x_i = RN_t(a * y_i), a the effective factor as in bwla_axpby (alpha_dev,
 * when given, is ONE device element of the compute type): one product and
 * one rounding per element, one read of y and one write of x.  This is the
 * gradient of the inner product z = <x, y>: dz/dx_i = y_i, so for an
 * incoming gradient zbar (left on the device as alpha_dev) dx = zbar * y and
 * dy = zbar * x, each one call.  x may equal y exactly (then this is
 * bwla_scal in place); partial overlap is an error, and so is alpha_dev
 * inside x.  Nothing is enqueued for n == 0. */
bwla_status bwla_scal_to(bwla_dtype t, int64_t n, double alpha, const void *alpha_dev, const void *y,
                         void *x, void *stream);
/* Reductions with increments; workspace as for bwla_dot (bwla_workspace_size
 * with BWLA_OP_DOT, BWLA_OP_NRM2 or BWLA_OP_CG serves every increment). */
bwla_status bwla_dot_strided(bwla_dtype t, bwla_acc acc, int64_t n, const void *x, int64_t incx,
                             const void *y, int64_t incy, bwla_dtype out_t, void *out, void *ws,
                             size_t ws_bytes, void *stream);
bwla_status bwla_nrm2_strided(bwla_dtype t, bwla_acc acc, int64_t n, const void *x, int64_t incx,
                              bwla_dtype out_t, void *out, void *ws, size_t ws_bytes, void *stream);
/* out <- sum |x_i| (the BLAS asum), reduced as bwla_nrm2 reduces x_i^2. */
bwla_status bwla_asum(bwla_dtype t, bwla_acc acc, int64_t n, const void *x, int64_t incx,
                      bwla_dtype out_t, void *out, void *ws, size_t ws_bytes, void *stream);

/* ---- dense matrix-vector product: y <- op(A) x (paper Section 2) ----------
 * A is m x n.  Row-major: A_ij at A[i*lda + j], lda >= max(1, n).
 * Column-major: A_ij at A[i + j*lda], lda >= max(1, m).
 * trans == 0: op(A) = A, x has n entries, y has m.  trans == 1: op(A) = A^T,
 * x has m entries, y has n.  y is overwritten (never read) in out_t (F64 for
 * f64 storage; F32 or F64 otherwise).  A zero-length reduction writes y = 0.
 * y must not overlap A or x. */
bwla_status bwla_gemv(bwla_dtype t, bwla_acc acc, bwla_layout layout, int trans, int64_t m,
                      int64_t n, const void *A, int64_t lda, const void *x, bwla_dtype out_t,
                      void *y, void *ws, size_t ws_bytes, void *stream);

/* ---- matrix-vector product with an inner-product epilogue -----------------
 * y <- op(A) x exactly as bwla_gemv with out_t = t, and in the same launch
 * sequence dot <- <w, y> = sum_i w_i y_i over the out_len entries of y, taken
 * with y as stored.  This is the GEMV-then-inner-product pair of one
 * conjugate-gradient iteration (q = A p followed by <p, q>), one of the
 * composite operations that the paper's abstract expects to inherit the
 * tuned kernels' performance; it is fused so that y and w are not read back
 * after the GEMV: each work-group that
 * stores outputs also reduces w_i y_i over them to a float64 partial, and
 * the partials are summed in a fixed order as in bwla_dot.
 * t is BWLA_F64 or BWLA_F32 (BWLA_ERR_UNSUPPORTED for BWLA_BF16, whose GEMV
 * output is never bf16).  w has out_len entries of type t (out_len = m for
 * trans == 0, n for trans == 1) and may alias x; dot is ONE device element of
 * dot_t (BWLA_F64 for f64; BWLA_F32 or BWLA_F64 for f32).  y must not
 * overlap A, x or w; dot must not overlap A, x, y or w.  out_len == 0 writes
 * dot = 0 only; a zero-length reduction writes y = 0 and dot = 0.
 * Workspace: at least bwla_gemv_dot_workspace_size() bytes. */
bwla_status bwla_gemv_dot(bwla_dtype t, bwla_acc acc, bwla_layout layout, int trans, int64_t m,
                          int64_t n, const void *A, int64_t lda, const void *x, void *y,
                          const void *w, bwla_dtype dot_t, void *dot, void *ws, size_t ws_bytes,
                          void *stream);

/* Bytes of workspace bwla_gemv_dot needs for these arguments under the
 * current configuration table (at least what bwla_gemv needs). */
bwla_status bwla_gemv_dot_workspace_size(bwla_dtype t, bwla_layout layout, int trans, int64_t m,
                                         int64_t n, size_t *bytes);

/* ---- y <- alpha op(A) x + beta y with increments (the BLAS gemv) -----------
 * Defined as the composite: s = op(A) x exactly as bwla_gemv stores it in
 * out_t, then y_i <- RN(fma(a, s_i, RN(b y_i))) in out_t's precision (as
 * bwla_axpby), or y_i <- RN(a s_i) when beta == 0, in which case y is not
 * read.  a, b: alpha, beta rounded to out_t.  x is (x, in_len, incx) and y
 * is (y, out_len, incy) in the increment convention above (incy != 0).
 * alpha == 1, beta == 0 with unit increments is bwla_gemv itself; otherwise
 * s goes through the workspace (and a strided x is gathered there first),
 * at least bwla_gemv_ex_workspace_size() bytes.  y must not overlap A or x. */
bwla_status bwla_gemv_ex(bwla_dtype t, bwla_acc acc, bwla_layout layout, int trans, int64_t m,
                         int64_t n, double alpha, const void *A, int64_t lda, const void *x,
                         int64_t incx, double beta, bwla_dtype out_t, void *y, int64_t incy,
                         void *ws, size_t ws_bytes, void *stream);
bwla_status bwla_gemv_ex_workspace_size(bwla_dtype t, bwla_dtype out_t, bwla_layout layout, int trans,
                                        int64_t m, int64_t n, size_t *bytes);

/* ---- rank-1 overwrite: A <- u v^T ------------------------------------------
 * The gradient of y = A x with respect to A for an incoming gradient u = ybar
 * and v = x.  A is m x n in the given layout and leading dimension; every
 * entry is RN_t(u_i * v_j) computed in the compute precision, so the result
 * is bitwise reproducible.  Entries between the row (column) length and lda
 * are not touched.  A must not overlap u or v. */
bwla_status bwla_ger(bwla_dtype t, bwla_layout layout, int64_t m, int64_t n, const void *u,
                     const void *v, void *A, int64_t lda, void *stream);

/* ---- fused update of a conjugate-gradient-style step ----------------------
 * In one pass over the vectors: x <- x + a p, r <- r - a q, out <- <r, r>,
 * with a = RN_c(alpha) (or RN_c(RN_c(alpha) * (*alpha_dev))).  Elementwise
 * results are bitwise those of bwla_axpby(x; alpha=a, y=p, beta=1, z=x) and
 * bwla_axpby(r; alpha=-a, y=q, beta=1, z=r); the reduction uses the new r.
 * Workspace as for bwla_dot. */
bwla_status bwla_cg_update(bwla_dtype t, bwla_acc acc, int64_t n, double alpha,
                           const void *alpha_dev, void *x, const void *p, void *r,
                           const void *q, bwla_dtype out_t, void *out, void *ws,
                           size_t ws_bytes, void *stream);

/* Bytes of workspace that the call with these arguments needs under the
 * current configuration table.  `op` is the public operation: BWLA_OP_DOT,
 * BWLA_OP_NRM2 or BWLA_OP_CG (m ignored, n = length; any of the three gives
 * a size that serves all three, bwla_asum and every increment),
 * BWLA_OP_GEMV_ROWS or BWLA_OP_GEMV_COLS for
 * bwla_gemv (either is accepted: the kernel is chosen from layout and
 * trans). */
bwla_status bwla_workspace_size(bwla_op op, bwla_dtype t, bwla_acc acc, bwla_layout layout,
                                int trans, int64_t m, int64_t n, size_t *bytes);

/* ---- batched uneven problems ---------------------------------------------
 * A plan holds many row-major GEMVs (y = A x, out_t output) and many dots
 * (out = <x, y>, out_t output) of one storage type.  Work is flattened into
 * items (row tiles of a GEMV, chunks of a dot) ordered largest first and run
 * with one work-group per item, one launch per kind of item (GEMV tiles with
 * x staged in LDS, the other GEMV tiles, dot chunks; the hardware dispatcher
 * hands out each launch's items in order).  Each dot's chunk partials are
 * combined in chunk order by a finalize kernel, so results do not depend on
 * the batch order or on scheduling.
 * create: copies the descriptors to the device and allocates the plan's own
 *         counters and partial slots (the only allocating call; not allowed
 *         while `stream` capture is active).
 * run:    enqueues the batched kernels and the dot finalize kernel.
 * capture: records the same kernels into a HIP graph owned by the plan.
 * replay: launches the captured graph.
 * Descriptor pointers must stay valid while the plan is used.
 * cfg (may be NULL) sets the work-group size (cfg->block, a multiple of 64
 * up to 512) and the packs of a GEMV row each lane of a staged tile owns
 * (cfg->unroll, a power of two up to 32); other fields are ignored.  A zero
 * (or NULL) field takes the configuration table's BWLA_OP_BATCH entry for
 * (t, acc, size class of the plan's algorithmic bytes), else the defaults
 * (256 threads, 16 packs per lane).
 * (The library also holds a persistent work-queue form of this launch, a
 * machine-sized grid drawing items from an atomic counter.  It has not been
 * validated on hardware and is switched off: with
 * BWLA_ENABLE_UNVALIDATED_BATCH=1 in the environment, plan creation returns
 * BWLA_ERR_UNSUPPORTED instead of building a plan for it.) */
typedef struct bwla_batch_plan bwla_batch_plan;
typedef struct {
    const void *A;
    int64_t m, n, lda;
    const void *x;
    void *y;
} bwla_gemv_desc;
typedef struct {
    const void *x;
    const void *y;
    int64_t n;
    void *out;
} bwla_dot_desc;

bwla_status bwla_batch_plan_create(bwla_dtype t, bwla_acc acc, bwla_dtype out_t,
                                   const bwla_gemv_desc *g, int32_t ng, const bwla_dot_desc *d,
                                   int32_t nd, const bwla_config *cfg, bwla_batch_plan **out);
bwla_status bwla_batch_run(bwla_batch_plan *p, void *stream);
bwla_status bwla_batch_capture(bwla_batch_plan *p, void *stream);
bwla_status bwla_batch_replay(bwla_batch_plan *p, void *stream);
/* Number of work items, persistent grid size and algorithmic bytes moved. */
bwla_status bwla_batch_info(const bwla_batch_plan *p, int64_t *items, int32_t *grid,
                            double *bytes);
void bwla_batch_plan_destroy(bwla_batch_plan *p);

/* ---- configuration table ---------------------------------------------------
 * One entry per (op, storage type, accumulation mode, size class).  The
 * accumulation mode matters for the operations that reduce (DOT, NRM2, CG,
 * GEMV_ROWS, GEMV_COLS): compensated arithmetic adds vector-ALU work per
 * element, and on gfx950 it runs best with more waves in flight than the
 * plain form.  COPY, AXPBY and GER always use their plain entry.  Size class
 * by the bytes the call streams: 0 < 1 MiB, 1 < 16 MiB, 2 < 256 MiB,
 * 3 < 1 GiB, 4 otherwise.  acc is BWLA_ACC_PLAIN, BWLA_ACC_COMPENSATED or -1
 * (both); size_class -1 sets every class.  cfg == NULL restores the defaults.
 * The table is shared by all threads (mutex-guarded).  If the environment
 * variable BWLA_TUNING names a tuning table, it is loaded before the first
 * call resolves a configuration.  Workspace sizes (bwla_workspace_size and
 * the other *_workspace_size calls) cover both accumulation modes under the
 * current table. */
bwla_status bwla_set_config(bwla_op op, bwla_dtype t, int acc, int size_class, const bwla_config *cfg);
/* The configuration a call with this op, type, accumulation mode and shape
 * would use after defaults are resolved (m = lines, n = line length for
 * GEMV/GER; m ignored for vectors; for BATCH, n = the plan's algorithmic
 * bytes and m ignored). */
bwla_status bwla_get_config(bwla_op op, bwla_dtype t, bwla_acc acc, int64_t m, int64_t n, bwla_config *cfg);
/* Load a tuning table written by the autotuner: text, one entry per line,
 * "op dtype acc size_class block vec unroll grid increment rows split" (acc
 * and size_class as for bwla_set_config), '#' starts a comment.  Either every
 * entry is valid and the whole table is installed, or nothing changes. */
bwla_status bwla_load_tuning(const char *path);

const char *bwla_status_string(bwla_status st);
const char *bwla_last_error(void); /* message of the last failed call on this thread */
int bwla_abi_version(void);
/* Number of compute units of the current device (used for default grids). */
int bwla_device_cus(void);

#ifdef __cplusplus
}
#endif
#endif /* BWLA_H */
