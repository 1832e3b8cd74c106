// api.cpp -- the C ABI declared in include/bwla.h: argument validation,
// configuration table and defaults, workspace sizing, kernel dispatch and
// batch plans.  Every check runs before anything is enqueued.
#include "bwla.h"
#include "device.hpp"
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace bwla;

namespace {

thread_local std::string g_last_error;

bwla_status fail(bwla_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

bwla_status hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return BWLA_OK;
    return fail(BWLA_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// BWLA_LOG set to anything but "" or "0": every call that launches kernels
// writes one line to stderr with the entry point, storage type, accumulation
// mode, shape and the configuration it resolved (bwla_config's fields; grid
// is the number of work-groups launched).
bool log_enabled()
{
    static const bool on = [] {
        const char *v = getenv("BWLA_LOG");
        return v && v[0] && strcmp(v, "0") != 0;
    }();
    return on;
}

void log_call(const char *what, int t, int acc, int64_t m, int64_t n, const Cfg &c)
{
    if (!log_enabled())
        return;
    static const char *const tname[3] = {"f64", "f32", "bf16"};
    fprintf(stderr,
            "bwla: %s %s %s m=%lld n=%lld block=%d vec=%d unroll=%d grid=%d increment=%d rows=%d split=%d\n",
            what, tname[t], acc < 0 ? "-" : acc == BWLA_ACC_COMPENSATED ? "compensated" : "plain", (long long)m,
            (long long)n, c.block, c.vec, c.unroll, c.grid, c.inc, c.rows, c.split);
}

bool valid_dtype(int t) { return t == BWLA_F64 || t == BWLA_F32 || t == BWLA_BF16; }
size_t dsize(int t) { return t == BWLA_F64 ? 8 : (t == BWLA_F32 ? 4 : 2); }
int native_vec(int t) { return (int)(16 / dsize(t)); }

// ---------------------------------------------------------------------------
// device properties
// ---------------------------------------------------------------------------
int device_cus()
{
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (!cached[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

// ---------------------------------------------------------------------------
// configuration table
// ---------------------------------------------------------------------------
constexpr int kClasses = 5;
constexpr int kAccs = 2; // plain, compensated: the reductions tune the two apart
std::mutex g_cfg_mu;
bwla_config g_table[BWLA_OP_COUNT][3][kAccs][kClasses]; // zero-initialised: all defaults

int size_class(double bytes)
{
    if (bytes < 1048576.0)
        return 0;
    if (bytes < 16777216.0)
        return 1;
    if (bytes < 268435456.0)
        return 2;
    if (bytes < 1073741824.0)
        return 3;
    return 4;
}

bool load_table_file(const char *path, std::string *err);

// A table named by BWLA_TUNING is loaded once, before the first lookup.
void load_env_table_once()
{
    static std::once_flag once;
    std::call_once(once, [] {
        const char *p = getenv("BWLA_TUNING");
        std::string err;
        if (p && p[0] && !load_table_file(p, &err))
            fprintf(stderr, "bwla: ignoring BWLA_TUNING=%s: %s\n", p, err.c_str());
    });
}

bwla_config lookup(int op, int t, int acc, double bytes)
{
    load_env_table_once();
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    return g_table[op][t][acc == BWLA_ACC_COMPENSATED][size_class(bytes)];
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Largest pack width (elements, power of two, <= want) such that every address
// in `ptrs` and every line stride `ld` keeps packs aligned.
int fit_vec(int want, size_t esize, std::initializer_list<const void *> ptrs, int64_t ld = 0)
{
    int v = want;
    while (v > 1) {
        bool ok = true;
        for (const void *p : ptrs)
            if (p && ((uintptr_t)p % (v * esize)) != 0)
                ok = false;
        if (ld && (ld % v) != 0)
            ok = false;
        if (ok)
            break;
        v >>= 1;
    }
    return v;
}

bwla_status check_cfg(const bwla_config &c)
{
    if (c.block && (c.block < 64 || c.block > 1024 || c.block % 64))
        return fail(BWLA_ERR_INVALID_ARG, "config: block %d is not a multiple of 64 in [64, 1024]", c.block);
    if (c.vec && !(is_pow2(c.vec) && c.vec <= 16))
        return fail(BWLA_ERR_INVALID_ARG, "config: vec %d not in {1,2,4,8,16}", c.vec);
    if (c.unroll && !(is_pow2(c.unroll) && c.unroll <= 32))
        return fail(BWLA_ERR_INVALID_ARG, "config: unroll %d not in {1,2,4,8,16,32}", c.unroll);
    if (c.rows && !(is_pow2(c.rows) && c.rows <= 8))
        return fail(BWLA_ERR_INVALID_ARG, "config: rows %d not in {1,2,4,8}", c.rows);
    if (c.grid < 0 || c.split < 0)
        return fail(BWLA_ERR_INVALID_ARG, "config: negative grid or split");
    if (c.increment != BWLA_INC_GLOBAL && c.increment != BWLA_INC_LOCAL)
        return fail(BWLA_ERR_INVALID_ARG, "config: increment %d", c.increment);
    return BWLA_OK;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// --- resolved configurations ---------------------------------------------
// Defaults below come from sweeps of the configuration space on MI355X
// (256 CUs): streaming kernels run best with one pack per thread and a grid
// covering the vector once; reductions with one 256-thread work-group per CU
// holding four packs in flight per thread (fewer, longer-lived waves stream
// better and keep the second stage small).
constexpr int kOpCg = BWLA_OP_CG;

Cfg resolve_vector(int op, int t, int acc, int64_t n, std::initializer_list<const void *> ptrs, int nstreams)
{
    const bool reduction = op == BWLA_OP_DOT || op == BWLA_OP_NRM2 || op == BWLA_OP_CG;
    bwla_config u = lookup(op, t, reduction ? acc : BWLA_ACC_PLAIN, (double)n * dsize(t) * nstreams);
    Cfg c;
    c.block = u.block ? u.block : 256;
    c.vec = fit_vec(u.vec ? u.vec : native_vec(t), dsize(t), ptrs);
    c.unroll = u.unroll ? u.unroll : (op == BWLA_OP_DOT || op == BWLA_OP_NRM2 ? 4 : 1);
    if (c.unroll > 4 && op != BWLA_OP_DOT && op != BWLA_OP_NRM2)
        c.unroll = 4; // eight packs in flight exist for the reductions (and the cols GEMV) only
    if (c.unroll > 8)
        c.unroll = 8; // sixteen and more: the cols GEMV only
    c.inc = u.increment;
    c.rows = 1;
    c.split = 1;
    const int64_t npack = std::max<int64_t>(1, n / c.vec);
    const int64_t one_pass = std::max<int64_t>(1, ceil_div(npack, (int64_t)c.block * c.unroll));
    int64_t grid = u.grid;
    if (!grid) {
        if (op == BWLA_OP_DOT)
            grid = std::min<int64_t>(one_pass, device_cus());
        else if (op == BWLA_OP_NRM2) // one stream: twice the work-groups for the bytes in flight
            grid = std::min<int64_t>(one_pass, 2 * (int64_t)device_cus());
        else
            grid = one_pass;
    }
    grid = std::min<int64_t>(grid, 1 << 30);
    if (reduction) // partial slots and the second stage stay small
        grid = std::min<int64_t>(grid, 65536);
    c.grid = (int)std::max<int64_t>(grid, 1);
    return c;
}

Cfg resolve_rows(int t, int acc, int64_t L, int64_t K, const void *A, int64_t ld, const void *v)
{
    bwla_config u = lookup(BWLA_OP_GEMV_ROWS, t, acc, (double)L * K * dsize(t));
    Cfg c;
    c.block = u.block ? u.block : 1024;
    c.vec = fit_vec(u.vec ? u.vec : native_vec(t), dsize(t), {A, v}, ld);
    c.unroll = u.unroll == 2 ? 2 : 1; // packs of each line in flight per thread: 1 or 2
    c.inc = 0;
    c.rows = u.rows ? u.rows : 2;
    const int64_t groups = std::max<int64_t>(1, ceil_div(L, c.rows));
    int64_t split = u.split;
    if (!split && u.grid) {
        // a work-group count tuned on one shape of the size class: keep that
        // count on every aspect ratio of the class
        split = ceil_div(u.grid, groups);
    } else if (!split) {
        // enough work-groups for every CU to hold two, each slice at least
        // two block-widths of packs long
        const int64_t target = (int64_t)device_cus() * 2;
        const int64_t kpack = std::max<int64_t>(1, K / c.vec);
        split = groups >= target ? 1 : ceil_div(target, groups);
        split = std::min<int64_t>(split, std::max<int64_t>(1, kpack / (2 * c.block)));
    }
    split = std::max<int64_t>(1, std::min<int64_t>(split, std::max<int64_t>(1, K)));
    split = std::min<int64_t>(split, (int64_t)(0x7fffffff / std::max<int64_t>(1, groups)));
    c.split = (int)split;
    c.grid = (int)std::min<int64_t>(groups * split, 0x7fffffff); // reported only: work-groups launched
    // No more threads than the packs of a slice: a table entry tuned on long
    // lines would leave most of a work-group idle on short ones.
    const int64_t per_slice = ceil_div(std::max<int64_t>(1, K / c.vec), split);
    const int64_t need = std::max<int64_t>(64, ceil_div(per_slice, 64) * 64);
    c.block = (int)std::min<int64_t>(c.block, need);
    return c;
}

Cfg resolve_cols(int t, int acc, int64_t L, int64_t K, const void *A, int64_t ld, const void *v)
{
    (void)v; // x is staged element by element: its alignment does not constrain the pack width
    bwla_config u = lookup(BWLA_OP_GEMV_COLS, t, acc, (double)L * K * dsize(t));
    Cfg c;
    c.block = u.block ? u.block : 512;
    c.vec = fit_vec(u.vec ? u.vec : native_vec(t), dsize(t), {A}, ld);
    c.unroll = u.unroll ? u.unroll : 4; // lines in flight per wave: 1 to 32
    while (c.unroll > 8 && (size_t)c.unroll * c.vec * dsize(t) > kColsLoadBytes)
        c.unroll /= 2; // more would spill: at most kColsLoadBytes of A in flight per lane
    c.inc = 0;
    c.rows = 1;
    const int64_t tiles = std::max<int64_t>(1, ceil_div(K, 64 * (int64_t)c.vec));
    const int64_t waves = c.block / 64;
    int64_t split = u.split;
    if (!split && u.grid) {
        // a work-group count tuned on one shape of the size class (see the rows kernel)
        split = ceil_div(u.grid, tiles);
        split = std::min<int64_t>(split, std::max<int64_t>(1, L / waves)); // every wave keeps a line
    } else if (!split) {
        // about one work-group per CU, each wave with at least 16 lines
        const int64_t target = (int64_t)device_cus();
        split = tiles >= target ? 1 : ceil_div(target, tiles);
        split = std::min<int64_t>(split, std::max<int64_t>(1, L / (waves * 16)));
    }
    split = std::max<int64_t>(1, std::min<int64_t>(split, std::max<int64_t>(1, L)));
    split = std::min<int64_t>(split, (int64_t)(0x7fffffff / std::max<int64_t>(1, tiles)));
    c.split = (int)split;
    c.grid = (int)std::min<int64_t>(tiles * split, 0x7fffffff); // reported only: work-groups launched
    return c;
}

Cfg resolve_ger(int t, int64_t L, int64_t K, const void *a, const void *b, const void *A, int64_t ld)
{
    bwla_config u = lookup(BWLA_OP_GER, t, BWLA_ACC_PLAIN, (double)L * K * dsize(t));
    Cfg c;
    c.block = u.block ? u.block : 256;
    c.vec = fit_vec(u.vec ? u.vec : native_vec(t), dsize(t), {b, A}, ld);
    c.unroll = 1;
    c.grid = 0;
    c.inc = 0;
    c.rows = u.rows ? u.rows : 4;
    c.split = 1;
    (void)a;
    return c;
}

// Batch plans: the work-group size and the packs of a GEMV row each lane of a
// staged tile owns (in unroll), from the table entry of the plan's size class.
Cfg resolve_batch(int t, int acc, double bytes)
{
    bwla_config u = lookup(BWLA_OP_BATCH, t, acc, bytes);
    Cfg c{};
    c.block = std::min(u.block ? u.block : 256, 512);
    c.vec = native_vec(t);
    c.unroll = u.unroll ? u.unroll : kStagedPacks;
    c.grid = 0;
    c.inc = 0;
    c.rows = 1;
    c.split = 1;
    return c;
}

// Workspace = the float64 (DD) partials of the first stage.
size_t ws_dot(const Cfg &c) { return c.grid > 1 ? (size_t)c.grid * sizeof(DD) : 0; }
size_t ws_rows(const Cfg &c, int64_t L)
{
    if (c.split <= 1)
        return 0;
    return (size_t)ceil_div(L, c.rows) * c.split * c.rows * sizeof(DD);
}
size_t ws_cols(const Cfg &c, int64_t K)
{
    if (c.split <= 1)
        return 0;
    return (size_t)ceil_div(K, 64 * (int64_t)c.vec) * c.split * 64 * c.vec * sizeof(DD);
}

// Parses a tuning table ("op dtype acc size_class block vec unroll grid
// increment rows split" per line, '#' comments; acc and size_class -1 mean
// every mode / class) and installs it atomically: either every entry is valid
// and applied, or nothing changes.
bool load_table_file(const char *path, std::string *err)
{
    FILE *f = fopen(path, "r");
    if (!f) {
        *err = std::string("cannot open ") + path;
        return false;
    }
    char line[512];
    int lineno = 0;
    struct Entry {
        int op, t, a, k;
        bwla_config c;
    };
    std::vector<Entry> entries;
    while (fgets(line, sizeof line, f)) {
        ++lineno;
        char *hash = strchr(line, '#');
        if (hash)
            *hash = 0;
        Entry e{};
        int got = sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d", &e.op, &e.t, &e.a, &e.k, &e.c.block,
                         &e.c.vec, &e.c.unroll, &e.c.grid, &e.c.increment, &e.c.rows, &e.c.split);
        if (got <= 0)
            continue; // blank or comment line
        if (got != 11 || e.op < 0 || e.op >= BWLA_OP_COUNT || !valid_dtype(e.t) || e.a < -1 ||
            e.a >= kAccs || e.k < -1 || e.k >= kClasses || check_cfg(e.c) != BWLA_OK) {
            fclose(f);
            char buf[600];
            snprintf(buf, sizeof buf, "%s:%d: malformed tuning entry", path, lineno);
            *err = buf;
            return false;
        }
        entries.push_back(e);
    }
    fclose(f);
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    for (const Entry &e : entries)
        for (int a = 0; a < kAccs; ++a)
            for (int k = 0; k < kClasses; ++k)
                if ((e.a < 0 || e.a == a) && (e.k < 0 || e.k == k))
                    g_table[e.op][e.t][a][k] = e.c;
    return true;
}

// --- overlap checks ----------------------------------------------------------
struct Span {
    uintptr_t lo, hi; // [lo, hi)
};
Span span(const void *p, size_t bytes) { return Span{(uintptr_t)p, (uintptr_t)p + bytes}; }
bool overlaps(Span a, Span b) { return a.lo < b.hi && b.lo < a.hi && a.hi > a.lo && b.hi > b.lo; }
bool same(Span a, Span b) { return a.lo == b.lo && a.hi == b.hi; }
size_t matrix_bytes(int64_t lines, int64_t K, int64_t ld, size_t es)
{
    if (lines <= 0 || K <= 0)
        return 0;
    return (size_t)((lines - 1) * ld + K) * es;
}

bwla_status out_type_ok(int t, int out_t)
{
    if (!valid_dtype(out_t) || out_t == BWLA_BF16)
        return fail(BWLA_ERR_UNSUPPORTED, "output type %d: results are float64 or float32", out_t);
    if (t == BWLA_F64 && out_t != BWLA_F64)
        return fail(BWLA_ERR_UNSUPPORTED, "f64 input requires an f64 output");
    return BWLA_OK;
}

template <typename F> hipError_t by_type(int t, F &&f)
{
    switch (t) {
    case BWLA_F64: return f((double *)nullptr);
    case BWLA_F32: return f((float *)nullptr);
    default: return f((bf16_t *)nullptr);
    }
}

// Common front half of dot/nrm2/cg: validation of the reduction arguments.
bwla_status check_reduction(int t, int acc, int64_t n, int out_t, void *out, void *ws, size_t ws_bytes,
                            size_t need)
{
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (acc != BWLA_ACC_PLAIN && acc != BWLA_ACC_COMPENSATED)
        return fail(BWLA_ERR_UNSUPPORTED, "accumulation mode %d", acc);
    if (n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
    bwla_status st = out_type_ok(t, out_t);
    if (st)
        return st;
    if (!out)
        return fail(BWLA_ERR_INVALID_ARG, "out is NULL");
    if (need && (!ws || ws_bytes < need))
        return fail(BWLA_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given%s", need, ws_bytes,
                    ws ? "" : " (NULL)");
    return BWLA_OK;
}

// --- vectors with an increment ------------------------------------------------
uint64_t uabs(int64_t v) { return v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v; }

// Bytes from the lowest to the highest element of (p, n, inc), one element
// included.
Span sspan(const void *p, int64_t n, int64_t inc, size_t es)
{
    if (n <= 0)
        return Span{(uintptr_t)p, (uintptr_t)p};
    return span(p, (size_t)((uint64_t)(n - 1) * uabs(inc) + 1) * es);
}

// True when no byte is shared.  Overlapping spans with the same nonzero |inc|
// can still interleave: their elements are then at least one element apart
// modulo the stride.
bool sdisjoint(const void *a, int64_t inca, const void *b, int64_t incb, int64_t n, size_t es)
{
    if (!overlaps(sspan(a, n, inca, es), sspan(b, n, incb, es)))
        return true;
    if (uabs(inca) != uabs(incb) || inca == 0)
        return false;
    const uint64_t S = uabs(inca) * es;
    const uint64_t d = (uintptr_t)a > (uintptr_t)b ? (uintptr_t)a - (uintptr_t)b : (uintptr_t)b - (uintptr_t)a;
    const uint64_t r = d % S;
    return r >= es && S - r >= es;
}

// (n - 1) * |inc| * es stays far inside the address space.
bool sfits(int64_t n, int64_t inc, size_t es)
{
    return n <= 1 || uabs(inc) <= ((uint64_t)1 << 60) / es / (uint64_t)(n - 1);
}

int strided_grid(int64_t n, bool reduction)
{
    const int64_t per = (int64_t)kStridedBlock * kStridedUnroll;
    const int64_t cap = (int64_t)(reduction ? 2 : 8) * device_cus(); // reductions: few partials
    return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(std::max<int64_t>(n, 1), per), cap));
}
// The fixed shape of the increment kernels, for the log.
Cfg strided_cfg(int64_t n, bool reduction)
{
    return Cfg{kStridedBlock, 1, kStridedUnroll, strided_grid(n, reduction), 0, 1, 1};
}
size_t ws_strided(int64_t n)
{
    const int g = strided_grid(n, true);
    return g > 1 ? (size_t)g * sizeof(DD) : 0;
}

} // namespace

// ===========================================================================
// entry points
// ===========================================================================
extern "C" {

int bwla_abi_version(void) { return BWLA_ABI_VERSION; }
int bwla_device_cus(void) { return device_cus(); }
const char *bwla_last_error(void) { return g_last_error.c_str(); }

const char *bwla_status_string(bwla_status st)
{
    switch (st) {
    case BWLA_OK: return "ok";
    case BWLA_ERR_INVALID_ARG: return "invalid argument";
    case BWLA_ERR_UNSUPPORTED: return "unsupported";
    case BWLA_ERR_WORKSPACE: return "workspace too small";
    case BWLA_ERR_HIP: return "HIP error";
    case BWLA_ERR_NOT_CAPTURABLE: return "not capturable";
    }
    return "unknown status";
}

bwla_status bwla_copy(bwla_dtype t, int64_t n, const void *y, void *x, void *stream)
{
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
    if (n == 0)
        return BWLA_OK;
    if (!x || !y)
        return fail(BWLA_ERR_INVALID_ARG, "NULL vector with n > 0");
    Span sx = span(x, n * dsize(t)), sy = span(y, n * dsize(t));
    if (same(sx, sy))
        return BWLA_OK;
    if (overlaps(sx, sy))
        return fail(BWLA_ERR_INVALID_ARG, "x partially overlaps y");
    Cfg c = resolve_vector(BWLA_OP_COPY, t, BWLA_ACC_PLAIN, n, {x, y}, 2);
    log_call("copy", t, -1, 1, n, c);
    hipError_t e = by_type(t, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        return launch_copy<T>(n, y, x, c, (hipStream_t)stream);
    });
    return hip_check(e, "copy launch");
}

bwla_status bwla_axpby(bwla_dtype t, int64_t n, double alpha, const void *alpha_dev, const void *y,
                       double beta, const void *beta_dev, const void *z, void *x, void *stream)
{
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
    if (n == 0)
        return BWLA_OK;
    if (!x || !y || !z)
        return fail(BWLA_ERR_INVALID_ARG, "NULL vector with n > 0");
    const size_t b = n * dsize(t);
    Span sx = span(x, b), sy = span(y, b), sz = span(z, b);
    if ((overlaps(sx, sy) && !same(sx, sy)) || (overlaps(sx, sz) && !same(sx, sz)))
        return fail(BWLA_ERR_INVALID_ARG, "x partially overlaps y or z (only exact aliasing is allowed)");
    const size_t cs = t == BWLA_F64 ? 8 : 4;
    Span sxa = span(x, b);
    if ((alpha_dev && overlaps(sxa, span(alpha_dev, cs))) || (beta_dev && overlaps(sxa, span(beta_dev, cs))))
        return fail(BWLA_ERR_INVALID_ARG, "a device scalar lies inside the output x");
    Cfg c = resolve_vector(BWLA_OP_AXPBY, t, BWLA_ACC_PLAIN, n, {x, y, z}, 3);
    log_call("axpby", t, -1, 1, n, c);
    hipError_t e = by_type(t, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        return launch_axpby<T>(n, alpha, alpha_dev, y, beta, beta_dev, z, x, c, (hipStream_t)stream);
    });
    return hip_check(e, "axpby launch");
}

// Bytes of bwla_dot_noalloc's static scratch (defined with it below).
constexpr size_t kScratchBytes = (size_t)65536 * sizeof(DD);

// dot (kRedDot), nrm2 (kRedSq) and asum (kRedAbs), any increments: the
// validation (everything but the workspace) and the resolved launch.
struct RedPlan {
    bool packed; // unit increments: the packed kernels
    Cfg c;       // their configuration (packed only)
    size_t need; // workspace bytes the launch uses
};

// Workspace: the caller's (ws, ws_bytes), or with `scratch` the static
// array of bwla_dot_noalloc (kScratchBytes).
static bwla_status reduce_check(bwla_dtype t, bwla_acc acc, int mode, int64_t n, const void *x, int64_t incx,
                                const void *y, int64_t incy, bwla_dtype out_t, void *out, void *ws,
                                size_t ws_bytes, bool scratch, RedPlan *plan)
{
    const bool two = mode == kRedDot;
    plan->packed = incx == 1 && (!two || incy == 1);
    plan->c = Cfg{};
    plan->need = 0;
    // dtype, mode, n and the output
    bwla_status st = check_reduction(t, acc, n, out_t, out, nullptr, 0, 0);
    if (st)
        return st;
    const size_t es = dsize(t);
    if (plan->packed) {
        plan->c = resolve_vector(two ? BWLA_OP_DOT : BWLA_OP_NRM2, t, acc, n, {x, y}, two ? 2 : 1);
        plan->need = n > 0 ? ws_dot(plan->c) : 0;
    } else {
        plan->need = n > 0 ? ws_strided(n) : 0;
    }
    if (scratch && plan->need > kScratchBytes)
        return fail(BWLA_ERR_WORKSPACE, "this configuration needs %zu bytes of partials; the static scratch of "
                                        "bwla_dot_noalloc holds %zu", plan->need, kScratchBytes);
    if (!scratch && plan->need && (!ws || ws_bytes < plan->need))
        return fail(BWLA_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given%s", plan->need, ws_bytes,
                    ws ? "" : " (NULL)");
    if (!sfits(n, incx, es) || (two && !sfits(n, incy, es)))
        return fail(BWLA_ERR_INVALID_ARG, "increment too large for n = %lld", (long long)n);
    if (n > 0 && (!x || (two && !y)))
        return fail(BWLA_ERR_INVALID_ARG, "NULL vector with n > 0");
    const size_t os = out_t == BWLA_F64 ? 8 : 4;
    Span so = span(out, os);
    if (n > 0 && (overlaps(so, sspan(x, n, incx, es)) || (two && overlaps(so, sspan(y, n, incy, es)))))
        return fail(BWLA_ERR_INVALID_ARG, "out overlaps an input");
    return BWLA_OK;
}

static bwla_status reduce_launch(const RedPlan &plan, bwla_dtype t, bwla_acc acc, int mode, int64_t n, const void *x,
                                 int64_t incx, const void *y, int64_t incy, bwla_dtype out_t, void *out, void *ws,
                                 void *stream)
{
    const bool two = mode == kRedDot;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0)
        return hip_check(launch_fill_zero(out, 1, out_t == BWLA_F64, s), "fill launch");
    const bool comp = acc == BWLA_ACC_COMPENSATED;
    const int of64 = out_t == BWLA_F64;
    if (log_enabled()) {
        const char *what = mode == kRedDot ? (plan.packed ? "dot" : "dot strided")
                           : mode == kRedSq ? (plan.packed ? "nrm2" : "nrm2 strided") : "asum";
        log_call(what, t, acc, 1, n, plan.packed ? plan.c : strided_cfg(n, true));
    }
    hipError_t e = by_type(t, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        if (plan.packed)
            return launch_dot<T>(n, comp, mode, x, two ? y : x, of64, out, ws, plan.c, s);
        return launch_strided_reduce<T>(mode, n, comp, x, incx, two ? y : x, two ? incy : incx, of64, out, ws,
                                        strided_grid(n, true), s);
    });
    return hip_check(e, mode == kRedDot ? "dot launch" : mode == kRedSq ? "nrm2 launch" : "asum launch");
}

static bwla_status reduce_common(bwla_dtype t, bwla_acc acc, int mode, int64_t n, const void *x, int64_t incx,
                                 const void *y, int64_t incy, bwla_dtype out_t, void *out, void *ws,
                                 size_t ws_bytes, void *stream)
{
    RedPlan plan;
    bwla_status st = reduce_check(t, acc, mode, n, x, incx, y, incy, out_t, out, ws, ws_bytes, false, &plan);
    if (st)
        return st;
    return reduce_launch(plan, t, acc, mode, n, x, incx, y, incy, out_t, out, ws, stream);
}

bwla_status bwla_dot(bwla_dtype t, bwla_acc acc, int64_t n, const void *x, const void *y,
                     bwla_dtype out_t, void *out, void *ws, size_t ws_bytes, void *stream)
{
    return reduce_common(t, acc, kRedDot, n, x, 1, y, 1, out_t, out, ws, ws_bytes, stream);
}

// --- the inner product for callers that cannot allocate ----------------------
// Its first-stage partials go to a file-scope device array instead of a
// caller workspace.  kScratchBytes (above) covers every configuration of the packed
// inner product: the grid of a reduction is capped at 65536 work-groups, one
// float64 pair each.  Host code never passes `scratch` itself (its name is a
// host-side stand-in): each device's address of it is looked up once, with
// that device current, and kept in g_scratch_ptr.
static __device__ __align__(256) DD scratch[kScratchBytes / sizeof(DD)];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {};

static bwla_status scratch_ptr(void **ptr)
{
    int dev = 0;
    bwla_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st)
        return st;
    if (dev < 0 || dev >= 64)
        return fail(BWLA_ERR_UNSUPPORTED, "device %d: the static scratch table holds devices 0..63", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (st)
            return st;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return BWLA_OK;
}

bwla_status bwla_dot_noalloc(bwla_dtype t, bwla_acc acc, int64_t n, const void *x, const void *y,
                             bwla_dtype out_t, void *out, void *stream)
{
    RedPlan plan;
    bwla_status st = reduce_check(t, acc, kRedDot, n, x, 1, y, 1, out_t, out, nullptr, 0, true, &plan);
    if (st)
        return st;
    void *ws = nullptr;
    if (plan.need && (st = scratch_ptr(&ws)) != BWLA_OK)
        return st;
    // every partial slot the second stage reads is written by this call's
    // first stage: nothing in the scratch has to start at zero
    return reduce_launch(plan, t, acc, kRedDot, n, x, 1, y, 1, out_t, out, ws, stream);
}

bwla_status bwla_nrm2(bwla_dtype t, bwla_acc acc, int64_t n, const void *x, bwla_dtype out_t,
                      void *out, void *ws, size_t ws_bytes, void *stream)
{
    return reduce_common(t, acc, kRedSq, n, x, 1, nullptr, 1, out_t, out, ws, ws_bytes, stream);
}

bwla_status bwla_dot_strided(bwla_dtype t, bwla_acc acc, int64_t n, const void *x, int64_t incx, const void *y,
                             int64_t incy, bwla_dtype out_t, void *out, void *ws, size_t ws_bytes, void *stream)
{
    return reduce_common(t, acc, kRedDot, n, x, incx, y, incy, out_t, out, ws, ws_bytes, stream);
}

bwla_status bwla_nrm2_strided(bwla_dtype t, bwla_acc acc, int64_t n, const void *x, int64_t incx,
                              bwla_dtype out_t, void *out, void *ws, size_t ws_bytes, void *stream)
{
    return reduce_common(t, acc, kRedSq, n, x, incx, nullptr, 1, out_t, out, ws, ws_bytes, stream);
}

bwla_status bwla_asum(bwla_dtype t, bwla_acc acc, int64_t n, const void *x, int64_t incx, bwla_dtype out_t,
                      void *out, void *ws, size_t ws_bytes, void *stream)
{
    return reduce_common(t, acc, kRedAbs, n, x, incx, nullptr, 1, out_t, out, ws, ws_bytes, stream);
}

// --- strided elementwise operations ---------------------------------------------
bwla_status bwla_copy_strided(bwla_dtype t, int64_t n, const void *y, int64_t incy, void *x, int64_t incx,
                              void *stream)
{
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
    if (n == 0)
        return BWLA_OK;
    const size_t es = dsize(t);
    if (incx == 0)
        return fail(BWLA_ERR_INVALID_ARG, "the output increment is 0");
    if (!sfits(n, incx, es) || !sfits(n, incy, es))
        return fail(BWLA_ERR_INVALID_ARG, "increment too large for n = %lld", (long long)n);
    if (incx == 1 && incy == 1)
        return bwla_copy(t, n, y, x, stream);
    if (!x || !y)
        return fail(BWLA_ERR_INVALID_ARG, "NULL vector with n > 0");
    if (x == y && incx == incy)
        return BWLA_OK;
    if (!sdisjoint(x, incx, y, incy, n, es))
        return fail(BWLA_ERR_INVALID_ARG, "x overlaps y");
    log_call("copy strided", t, -1, 1, n, strided_cfg(n, false));
    hipError_t e = by_type(t, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        return launch_strided_elem<T>(kElemCopy, n, 0.0, nullptr, 0.0, nullptr, y, incy, nullptr, 0, x, incx,
                                      strided_grid(n, false), (hipStream_t)stream);
    });
    return hip_check(e, "strided copy launch");
}

bwla_status bwla_axpby_strided(bwla_dtype t, int64_t n, double alpha, const void *alpha_dev, const void *y,
                               int64_t incy, double beta, const void *beta_dev, const void *z, int64_t incz,
                               void *x, int64_t incx, void *stream)
{
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
    if (n == 0)
        return BWLA_OK;
    const size_t es = dsize(t);
    if (incx == 0)
        return fail(BWLA_ERR_INVALID_ARG, "the output increment is 0");
    if (!sfits(n, incx, es) || !sfits(n, incy, es) || !sfits(n, incz, es))
        return fail(BWLA_ERR_INVALID_ARG, "increment too large for n = %lld", (long long)n);
    if (incx == 1 && incy == 1 && incz == 1)
        return bwla_axpby(t, n, alpha, alpha_dev, y, beta, beta_dev, z, x, stream);
    if (!x || !y || !z)
        return fail(BWLA_ERR_INVALID_ARG, "NULL vector with n > 0");
    if (!(x == y && incx == incy) && !sdisjoint(x, incx, y, incy, n, es))
        return fail(BWLA_ERR_INVALID_ARG, "x overlaps y (only exact aliasing is allowed)");
    if (!(x == z && incx == incz) && !sdisjoint(x, incx, z, incz, n, es))
        return fail(BWLA_ERR_INVALID_ARG, "x overlaps z (only exact aliasing is allowed)");
    const size_t cs = t == BWLA_F64 ? 8 : 4;
    Span sx = sspan(x, n, incx, es);
    if ((alpha_dev && overlaps(sx, span(alpha_dev, cs))) || (beta_dev && overlaps(sx, span(beta_dev, cs))))
        return fail(BWLA_ERR_INVALID_ARG, "a device scalar lies inside the output x");
    log_call("axpby strided", t, -1, 1, n, strided_cfg(n, false));
    hipError_t e = by_type(t, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        return launch_strided_elem<T>(kElemAxpby, n, alpha, alpha_dev, beta, beta_dev, y, incy, z, incz, x, incx,
                                      strided_grid(n, false), (hipStream_t)stream);
    });
    return hip_check(e, "strided axpby launch");
}

bwla_status bwla_scal(bwla_dtype t, int64_t n, double alpha, const void *alpha_dev, void *x, int64_t incx,
                      void *stream)
{
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
    if (n == 0)
        return BWLA_OK;
    const size_t es = dsize(t);
    if (incx == 0)
        return fail(BWLA_ERR_INVALID_ARG, "the increment is 0");
    if (!sfits(n, incx, es))
        return fail(BWLA_ERR_INVALID_ARG, "increment too large for n = %lld", (long long)n);
    if (!x)
        return fail(BWLA_ERR_INVALID_ARG, "NULL vector with n > 0");
    if (alpha_dev && overlaps(sspan(x, n, incx, es), span(alpha_dev, t == BWLA_F64 ? 8 : 4)))
        return fail(BWLA_ERR_INVALID_ARG, "the device scalar lies inside x");
    hipStream_t s = (hipStream_t)stream;
    // unit increment: one read and one write stream, as the copy (its table entry)
    const Cfg c = incx == 1 ? resolve_vector(BWLA_OP_COPY, t, BWLA_ACC_PLAIN, n, {x}, 2) : strided_cfg(n, false);
    log_call(incx == 1 ? "scal" : "scal strided", t, -1, 1, n, c);
    hipError_t e = by_type(t, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        if (incx == 1)
            return launch_scal<T>(n, alpha, alpha_dev, x, x, c, s);
        return launch_strided_elem<T>(kElemScal, n, alpha, alpha_dev, 0.0, nullptr, x, incx, nullptr, 0, x, incx,
                                      strided_grid(n, false), s);
    });
    return hip_check(e, "scal launch");
}

bwla_status bwla_scal_to(bwla_dtype t, int64_t n, double alpha, const void *alpha_dev, const void *y, void *x,
                         void *stream)
{
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "n = %lld < 0", (long long)n);
    if (n == 0)
        return BWLA_OK;
    if (!x || !y)
        return fail(BWLA_ERR_INVALID_ARG, "NULL vector with n > 0");
    const size_t b = n * dsize(t);
    Span sx = span(x, b), sy = span(y, b);
    if (overlaps(sx, sy) && !same(sx, sy))
        return fail(BWLA_ERR_INVALID_ARG, "x partially overlaps y (only exact aliasing is allowed)");
    if (alpha_dev && overlaps(sx, span(alpha_dev, t == BWLA_F64 ? 8 : 4)))
        return fail(BWLA_ERR_INVALID_ARG, "the device scalar lies inside x");
    // one read stream and one write stream, as the copy: its table entry
    Cfg c = resolve_vector(BWLA_OP_COPY, t, BWLA_ACC_PLAIN, n, {x, y}, 2);
    log_call("scal_to", t, -1, 1, n, c);
    hipError_t e = by_type(t, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        return launch_scal<T>(n, alpha, alpha_dev, y, x, c, (hipStream_t)stream);
    });
    return hip_check(e, "scal_to launch");
}

// Which kernel serves (layout, trans), and the line view of A.
struct GemvPlan {
    bool rows;       // rows kernel (reduction along lines) or cols kernel
    int64_t L, K;    // lines, elements per line
    int64_t out_len; // entries of y
    int64_t in_len;  // entries of x
};

static GemvPlan gemv_plan(int layout, int trans, int64_t m, int64_t n)
{
    GemvPlan g;
    const bool row_major = layout == BWLA_ROW_MAJOR;
    g.L = row_major ? m : n;
    g.K = row_major ? n : m;
    g.rows = row_major ? !trans : trans;
    g.out_len = trans ? n : m;
    g.in_len = trans ? m : n;
    return g;
}

// Workspace of a GEMV, and of a GEMV with the dot epilogue: the split
// partials, then (with the epilogue) one float64 pair per work-group that
// stores y.
static size_t gemv_ws(const GemvPlan &g, const Cfg &c, bool with_dot, size_t *dparts_offset)
{
    const size_t base = g.rows ? ws_rows(c, g.L) : ws_cols(c, g.K);
    if (dparts_offset)
        *dparts_offset = base;
    if (!with_dot)
        return base;
    return base + (size_t)gemv_dot_parts(g.rows, g.L, g.K, c) * sizeof(DD);
}

static Cfg gemv_cfg(bwla_dtype t, int acc, const GemvPlan &g, const void *A, int64_t lda, const void *x)
{
    return g.rows ? resolve_rows(t, acc, g.L, g.K, A, lda, x) : resolve_cols(t, acc, g.L, g.K, A, lda, x);
}

// Shared body of bwla_gemv and bwla_gemv_dot (w == NULL: no epilogue).
static bwla_status gemv_common(bwla_dtype t, bwla_acc acc, bwla_layout layout, int trans, int64_t m,
                               int64_t n, const void *A, int64_t lda, const void *x, bwla_dtype out_t,
                               void *y, const void *w, bwla_dtype dot_t, void *dot, void *ws,
                               size_t ws_bytes, void *stream)
{
    const bool fused = dot != nullptr;
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (acc != BWLA_ACC_PLAIN && acc != BWLA_ACC_COMPENSATED)
        return fail(BWLA_ERR_UNSUPPORTED, "accumulation mode %d", acc);
    if (layout != BWLA_ROW_MAJOR && layout != BWLA_COL_MAJOR)
        return fail(BWLA_ERR_INVALID_ARG, "layout %d", layout);
    if (trans != 0 && trans != 1)
        return fail(BWLA_ERR_INVALID_ARG, "trans %d", trans);
    if (m < 0 || n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "negative size m=%lld n=%lld", (long long)m, (long long)n);
    bwla_status st = out_type_ok(t, out_t);
    if (st)
        return st;
    if (fused) {
        if (t == BWLA_BF16)
            return fail(BWLA_ERR_UNSUPPORTED, "gemv_dot needs y in the storage type; bf16 has no bf16 GEMV output");
        if ((st = out_type_ok(t, dot_t)))
            return st;
    }
    GemvPlan g = gemv_plan(layout, trans, m, n);
    if (lda < std::max<int64_t>(1, g.K))
        return fail(BWLA_ERR_INVALID_ARG, "lda %lld < %lld", (long long)lda, (long long)std::max<int64_t>(1, g.K));
    const size_t es = dsize(t), os = out_t == BWLA_F64 ? 8 : 4;
    hipStream_t s = (hipStream_t)stream;
    if (fused) {
        Span sd = span(dot, dot_t == BWLA_F64 ? 8 : 4);
        if (g.out_len > 0 && (!y || !w))
            return fail(BWLA_ERR_INVALID_ARG, "y or w is NULL");
        if (g.out_len > 0 && (overlaps(sd, span(y, g.out_len * os)) || overlaps(sd, span(w, g.out_len * es))))
            return fail(BWLA_ERR_INVALID_ARG, "dot overlaps y or w");
        if (g.in_len > 0 && g.out_len > 0 &&
            (overlaps(sd, span(A, matrix_bytes(g.L, g.K, lda, es))) || overlaps(sd, span(x, g.in_len * es))))
            return fail(BWLA_ERR_INVALID_ARG, "dot overlaps A or x");
        if (g.out_len > 0 && overlaps(span(y, g.out_len * os), span(w, g.out_len * es)))
            return fail(BWLA_ERR_INVALID_ARG, "y overlaps w");
    }
    if (g.out_len == 0)
        return fused ? hip_check(launch_fill_zero(dot, 1, dot_t == BWLA_F64, s), "fill launch") : BWLA_OK;
    if (!y)
        return fail(BWLA_ERR_INVALID_ARG, "y is NULL");
    if (g.in_len > 0 && (!A || !x))
        return fail(BWLA_ERR_INVALID_ARG, "NULL A or x with a nonzero reduction length");
    Span sy = span(y, g.out_len * os);
    if (g.in_len > 0 && (overlaps(sy, span(A, matrix_bytes(g.L, g.K, lda, es))) ||
                         overlaps(sy, span(x, g.in_len * es))))
        return fail(BWLA_ERR_INVALID_ARG, "y overlaps A or x");
    if (g.in_len == 0) {
        bwla_status r = hip_check(launch_fill_zero(y, g.out_len, out_t == BWLA_F64, s), "fill launch");
        if (r || !fused)
            return r;
        return hip_check(launch_fill_zero(dot, 1, dot_t == BWLA_F64, s), "fill launch");
    }
    const bool comp = acc == BWLA_ACC_COMPENSATED;
    const int of64 = out_t == BWLA_F64, df64 = dot_t == BWLA_F64;
    Cfg c = gemv_cfg(t, acc, g, A, lda, x);
    size_t off = 0;
    const size_t need = gemv_ws(g, c, fused, &off);
    if (need && (!ws || ws_bytes < need))
        return fail(BWLA_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    // the shape logged is the kernel's: g.L lines of g.K contiguous elements
    log_call(fused ? (g.rows ? "gemv_dot rows" : "gemv_dot cols") : (g.rows ? "gemv rows" : "gemv cols"), t, acc,
             g.L, g.K, c);
    const void *wv = fused ? w : nullptr;
    hipError_t e = by_type(t, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        if (g.rows)
            return launch_gemv_rows<T>(g.L, g.K, comp, A, lda, x, of64, y, ws, c, s, wv, off, df64, dot);
        return launch_gemv_cols<T>(g.L, g.K, comp, A, lda, x, of64, y, ws, c, s, wv, off, df64, dot);
    });
    return hip_check(e, g.rows ? "gemv (rows) launch" : "gemv (cols) launch");
}

bwla_status bwla_gemv(bwla_dtype t, bwla_acc acc, bwla_layout layout, int trans, int64_t m, int64_t n,
                      const void *A, int64_t lda, const void *x, bwla_dtype out_t, void *y, void *ws,
                      size_t ws_bytes, void *stream)
{
    return gemv_common(t, acc, layout, trans, m, n, A, lda, x, out_t, y, nullptr, out_t, nullptr, ws,
                       ws_bytes, stream);
}

bwla_status bwla_gemv_dot(bwla_dtype t, bwla_acc acc, bwla_layout layout, int trans, int64_t m, int64_t n,
                          const void *A, int64_t lda, const void *x, void *y, const void *w,
                          bwla_dtype dot_t, void *dot, void *ws, size_t ws_bytes, void *stream)
{
    if (!dot)
        return fail(BWLA_ERR_INVALID_ARG, "dot is NULL");
    return gemv_common(t, acc, layout, trans, m, n, A, lda, x, t, y, w, dot_t, dot, ws, ws_bytes, stream);
}

bwla_status bwla_gemv_dot_workspace_size(bwla_dtype t, bwla_layout layout, int trans, int64_t m, int64_t n,
                                         size_t *bytes)
{
    if (!bytes)
        return fail(BWLA_ERR_INVALID_ARG, "bytes is NULL");
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (layout != BWLA_ROW_MAJOR && layout != BWLA_COL_MAJOR)
        return fail(BWLA_ERR_INVALID_ARG, "layout %d", layout);
    if (trans != 0 && trans != 1)
        return fail(BWLA_ERR_INVALID_ARG, "trans %d", trans);
    if (m < 0 || n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "negative size");
    *bytes = 0;
    GemvPlan g = gemv_plan(layout, trans, m, n);
    if (g.out_len == 0 || g.in_len == 0)
        return BWLA_OK; // only fills run
    size_t best = 0; // largest over the pack widths and accumulation modes the call could use
    for (int acc = 0; acc < kAccs; ++acc)
        for (int v = 1; v <= 16; v <<= 1) {
            const void *fake = (const void *)(uintptr_t)(v * dsize(t));
            best = std::max(best, gemv_ws(g, gemv_cfg(t, acc, g, fake, v, fake), true, nullptr));
        }
    *bytes = best;
    return BWLA_OK;
}

// y <- alpha op(A) x + beta y with increments: the GEMV into a contiguous
// temporary of the workspace, then a strided scal (beta == 0: y is not read)
// or axpby into y.  A strided x is first gathered into the workspace.
// Workspace: [x gathered | temporary y | GEMV partials], 256-byte aligned parts.
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bwla_status bwla_gemv_ex(bwla_dtype t, bwla_acc acc, bwla_layout layout, int trans, int64_t m, int64_t n,
                         double alpha, const void *A, int64_t lda, const void *x, int64_t incx, double beta,
                         bwla_dtype out_t, void *y, int64_t incy, void *ws, size_t ws_bytes, void *stream)
{
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (acc != BWLA_ACC_PLAIN && acc != BWLA_ACC_COMPENSATED)
        return fail(BWLA_ERR_UNSUPPORTED, "accumulation mode %d", acc);
    if (layout != BWLA_ROW_MAJOR && layout != BWLA_COL_MAJOR)
        return fail(BWLA_ERR_INVALID_ARG, "layout %d", layout);
    if (trans != 0 && trans != 1)
        return fail(BWLA_ERR_INVALID_ARG, "trans %d", trans);
    if (m < 0 || n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "negative size m=%lld n=%lld", (long long)m, (long long)n);
    bwla_status st = out_type_ok(t, out_t);
    if (st)
        return st;
    GemvPlan g = gemv_plan(layout, trans, m, n);
    if (lda < std::max<int64_t>(1, g.K))
        return fail(BWLA_ERR_INVALID_ARG, "lda %lld < %lld", (long long)lda, (long long)std::max<int64_t>(1, g.K));
    const size_t es = dsize(t), os = out_t == BWLA_F64 ? 8 : 4;
    if (incy == 0)
        return fail(BWLA_ERR_INVALID_ARG, "the output increment is 0");
    if (!sfits(g.out_len, incy, os) || !sfits(g.in_len, incx, es))
        return fail(BWLA_ERR_INVALID_ARG, "increment too large");
    if (g.out_len == 0)
        return BWLA_OK;
    if (!y)
        return fail(BWLA_ERR_INVALID_ARG, "y is NULL");
    if (g.in_len > 0 && (!A || !x))
        return fail(BWLA_ERR_INVALID_ARG, "NULL A or x with a nonzero reduction length");
    Span sy = sspan(y, g.out_len, incy, os);
    if (g.in_len > 0 && (overlaps(sy, span(A, matrix_bytes(g.L, g.K, lda, es))) ||
                         overlaps(sy, sspan(x, g.in_len, incx, es))))
        return fail(BWLA_ERR_INVALID_ARG, "y overlaps A or x");
    if (alpha == 1.0 && beta == 0.0 && incx == 1 && incy == 1)
        return gemv_common(t, acc, layout, trans, m, n, A, lda, x, out_t, y, nullptr, out_t, nullptr, ws,
                           ws_bytes, stream);
    // workspace parts
    const bool gather = incx != 1 && g.in_len > 0;
    const size_t off_tmp = align256(gather ? (size_t)g.in_len * es : 0);
    const size_t off_g = align256(off_tmp + (size_t)g.out_len * os);
    const void *xs = gather ? ws : x;
    Cfg c{};
    size_t need = off_g;
    if (g.in_len > 0) {
        c = gemv_cfg(t, acc, g, A, lda, xs);
        need += gemv_ws(g, c, false, nullptr);
    }
    if (!ws || ws_bytes < need)
        return fail(BWLA_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (g.in_len > 0)
        log_call(g.rows ? "gemv_ex rows" : "gemv_ex cols", t, acc, g.L, g.K, c);
    hipStream_t s = (hipStream_t)stream;
    void *tmp = (char *)ws + off_tmp;
    void *gws = (char *)ws + off_g;
    const bool comp = acc == BWLA_ACC_COMPENSATED;
    const int of64 = out_t == BWLA_F64;
    hipError_t e = hipSuccess;
    if (g.in_len == 0) {
        e = launch_fill_zero(tmp, g.out_len, of64, s);
    } else {
        e = by_type(t, [&](auto *tag) {
            using T = std::remove_pointer_t<decltype(tag)>;
            hipError_t r = hipSuccess;
            if (gather)
                r = launch_strided_elem<T>(kElemCopy, g.in_len, 0.0, nullptr, 0.0, nullptr, x, incx, nullptr, 0,
                                           ws, 1, strided_grid(g.in_len, false), s);
            if (r != hipSuccess)
                return r;
            if (g.rows)
                return launch_gemv_rows<T>(g.L, g.K, comp, A, lda, xs, of64, tmp, gws, c, s);
            return launch_gemv_cols<T>(g.L, g.K, comp, A, lda, xs, of64, tmp, gws, c, s);
        });
    }
    if (e != hipSuccess)
        return hip_check(e, "gemv_ex launch");
    e = by_type(out_t, [&](auto *tag) {
        using O = std::remove_pointer_t<decltype(tag)>;
        if (beta == 0.0)
            return launch_strided_elem<O>(kElemScal, g.out_len, alpha, nullptr, 0.0, nullptr, tmp, 1, nullptr, 0,
                                          y, incy, strided_grid(g.out_len, false), s);
        return launch_strided_elem<O>(kElemAxpby, g.out_len, alpha, nullptr, beta, nullptr, tmp, 1, y, incy, y,
                                      incy, strided_grid(g.out_len, false), s);
    });
    return hip_check(e, "gemv_ex update launch");
}

bwla_status bwla_gemv_ex_workspace_size(bwla_dtype t, bwla_dtype out_t, bwla_layout layout, int trans,
                                        int64_t m, int64_t n, size_t *bytes)
{
    if (!bytes)
        return fail(BWLA_ERR_INVALID_ARG, "bytes is NULL");
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    bwla_status st = out_type_ok(t, out_t);
    if (st)
        return st;
    if (layout != BWLA_ROW_MAJOR && layout != BWLA_COL_MAJOR)
        return fail(BWLA_ERR_INVALID_ARG, "layout %d", layout);
    if (trans != 0 && trans != 1)
        return fail(BWLA_ERR_INVALID_ARG, "trans %d", trans);
    if (m < 0 || n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "negative size");
    *bytes = 0;
    GemvPlan g = gemv_plan(layout, trans, m, n);
    if (g.out_len == 0)
        return BWLA_OK;
    const size_t os = out_t == BWLA_F64 ? 8 : 4;
    size_t best = align256(align256((size_t)g.in_len * dsize(t)) + (size_t)g.out_len * os);
    size_t gw = 0;
    if (g.in_len > 0)
        for (int acc = 0; acc < kAccs; ++acc)
            for (int v = 1; v <= 16; v <<= 1) {
                const void *fake = (const void *)(uintptr_t)(v * dsize(t));
                gw = std::max(gw, gemv_ws(g, gemv_cfg(t, acc, g, fake, v, fake), false, nullptr));
            }
    *bytes = best + gw;
    return BWLA_OK;
}

bwla_status bwla_ger(bwla_dtype t, bwla_layout layout, int64_t m, int64_t n, const void *u, const void *v,
                     void *A, int64_t lda, void *stream)
{
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (layout != BWLA_ROW_MAJOR && layout != BWLA_COL_MAJOR)
        return fail(BWLA_ERR_INVALID_ARG, "layout %d", layout);
    if (m < 0 || n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "negative size m=%lld n=%lld", (long long)m, (long long)n);
    const bool row_major = layout == BWLA_ROW_MAJOR;
    const int64_t L = row_major ? m : n, K = row_major ? n : m;
    if (lda < std::max<int64_t>(1, K))
        return fail(BWLA_ERR_INVALID_ARG, "lda %lld < %lld", (long long)lda, (long long)std::max<int64_t>(1, K));
    if (m == 0 || n == 0)
        return BWLA_OK;
    if (!u || !v || !A)
        return fail(BWLA_ERR_INVALID_ARG, "NULL pointer");
    const size_t es = dsize(t);
    Span sa = span(A, matrix_bytes(L, K, lda, es));
    if (overlaps(sa, span(u, m * es)) || overlaps(sa, span(v, n * es)))
        return fail(BWLA_ERR_INVALID_ARG, "A overlaps u or v");
    const void *a = row_major ? u : v; // per-line factor
    const void *b = row_major ? v : u; // factor along the line
    Cfg c = resolve_ger(t, L, K, a, b, A, lda);
    hipError_t e = by_type(t, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        return launch_ger<T>(L, K, a, b, A, lda, c, (hipStream_t)stream);
    });
    return hip_check(e, "ger launch");
}

bwla_status bwla_cg_update(bwla_dtype t, bwla_acc acc, int64_t n, double alpha, const void *alpha_dev,
                           void *x, const void *p, void *r, const void *q, bwla_dtype out_t, void *out,
                           void *ws, size_t ws_bytes, void *stream)
{
    // dtype, mode, n and the output first: the configuration lookup indexes
    // its table by dtype
    bwla_status st = check_reduction(t, acc, n, out_t, out, nullptr, 0, 0);
    if (st)
        return st;
    Cfg c = resolve_vector(kOpCg, t, acc, n, {x, p, r, q}, 6);
    const size_t need = n > 0 ? ws_dot(c) : 0;
    if ((st = check_reduction(t, acc, n, out_t, out, ws, ws_bytes, need)))
        return st;
    if (n == 0)
        return hip_check(launch_fill_zero(out, 1, out_t == BWLA_F64, (hipStream_t)stream), "fill launch");
    if (!x || !p || !r || !q)
        return fail(BWLA_ERR_INVALID_ARG, "NULL vector with n > 0");
    const size_t b = n * dsize(t);
    Span sx = span(x, b), sp = span(p, b), sr = span(r, b), sq = span(q, b);
    Span so = span(out, out_t == BWLA_F64 ? 8 : 4);
    if (overlaps(sx, sr) || overlaps(sx, sp) || overlaps(sx, sq) || overlaps(sr, sp) || overlaps(sr, sq))
        return fail(BWLA_ERR_INVALID_ARG, "the updated vectors x, r must not overlap each other or p, q");
    if (overlaps(so, sx) || overlaps(so, sr) || overlaps(so, sp) || overlaps(so, sq))
        return fail(BWLA_ERR_INVALID_ARG, "out overlaps a vector");
    hipError_t e = by_type(t, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        return launch_cg<T>(n, acc == BWLA_ACC_COMPENSATED, alpha, alpha_dev, x, p, r, q,
                            out_t == BWLA_F64, out, ws, c, (hipStream_t)stream);
    });
    return hip_check(e, "cg update launch");
}

bwla_status bwla_workspace_size(bwla_op op, bwla_dtype t, bwla_acc acc, bwla_layout layout, int trans,
                                int64_t m, int64_t n, size_t *bytes)
{
    if (acc != BWLA_ACC_PLAIN && acc != BWLA_ACC_COMPENSATED)
        return fail(BWLA_ERR_UNSUPPORTED, "accumulation mode %d", acc);
    if (!bytes)
        return fail(BWLA_ERR_INVALID_ARG, "bytes is NULL");
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (m < 0 || n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "negative size");
    *bytes = 0;
    // The pack width a call ends up with depends on pointer alignment, and the
    // default grid and split depend on the pack width, so size for the largest
    // requirement over every width the call could use.  A fake address
    // v*sizeof(T) (and line stride v) is aligned to exactly v elements.  The
    // size also serves the other accumulation mode, whose table entry may
    // differ, so a buffer sized once serves both.
    size_t best = 0;
    for (int a = 0; a < kAccs; ++a) {
        for (int v = 1; v <= 16; v <<= 1) {
            const void *fake = (const void *)(uintptr_t)(v * dsize(t));
            switch (op) {
            case BWLA_OP_DOT: // dot, nrm2, asum (any increments) and the CG update share one sizing
            case BWLA_OP_NRM2:
            case BWLA_OP_CG:
                best = std::max(best, ws_strided(n));
                best = std::max(best, ws_dot(resolve_vector(BWLA_OP_DOT, t, a, n, {fake}, 2)));
                best = std::max(best, ws_dot(resolve_vector(BWLA_OP_NRM2, t, a, n, {fake}, 1)));
                best = std::max(best, ws_dot(resolve_vector(kOpCg, t, a, n, {fake}, 6)));
                break;
            case BWLA_OP_GEMV_ROWS:
            case BWLA_OP_GEMV_COLS: {
                if (layout != BWLA_ROW_MAJOR && layout != BWLA_COL_MAJOR)
                    return fail(BWLA_ERR_INVALID_ARG, "layout %d", layout);
                GemvPlan g = gemv_plan(layout, trans, m, n);
                if (g.out_len == 0 || g.in_len == 0)
                    break; // no kernel runs
                if (g.rows)
                    best = std::max(best, ws_rows(resolve_rows(t, a, g.L, g.K, fake, v, fake), g.L));
                else
                    best = std::max(best, ws_cols(resolve_cols(t, a, g.L, g.K, fake, v, fake), g.K));
                break;
            }
            default:
                break;
            }
        }
    }
    *bytes = best;
    return BWLA_OK;
}

// ---------------------------------------------------------------------------
// configuration entry points
// ---------------------------------------------------------------------------
bwla_status bwla_set_config(bwla_op op, bwla_dtype t, int acc, int size_class, const bwla_config *cfg)
{
    if (op < 0 || op >= BWLA_OP_COUNT)
        return fail(BWLA_ERR_INVALID_ARG, "op %d", op);
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (acc < -1 || acc >= kAccs)
        return fail(BWLA_ERR_INVALID_ARG, "accumulation mode %d", acc);
    if (size_class < -1 || size_class >= kClasses)
        return fail(BWLA_ERR_INVALID_ARG, "size class %d", size_class);
    bwla_config c{};
    if (cfg) {
        bwla_status st = check_cfg(*cfg);
        if (st)
            return st;
        c = *cfg;
    }
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    for (int a = 0; a < kAccs; ++a)
        for (int k = 0; k < kClasses; ++k)
            if ((acc < 0 || acc == a) && (size_class < 0 || size_class == k))
                g_table[op][t][a][k] = c;
    return BWLA_OK;
}

bwla_status bwla_get_config(bwla_op op, bwla_dtype t, bwla_acc acc, int64_t m, int64_t n, bwla_config *cfg)
{
    if (!cfg)
        return fail(BWLA_ERR_INVALID_ARG, "cfg is NULL");
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (acc != BWLA_ACC_PLAIN && acc != BWLA_ACC_COMPENSATED)
        return fail(BWLA_ERR_UNSUPPORTED, "accumulation mode %d", acc);
    if (m < 0 || n < 0)
        return fail(BWLA_ERR_INVALID_ARG, "negative size");
    Cfg c;
    switch (op) {
    case BWLA_OP_COPY: c = resolve_vector(op, t, acc, n, {}, 2); break;
    case BWLA_OP_AXPBY: c = resolve_vector(op, t, acc, n, {}, 3); break;
    case BWLA_OP_DOT: c = resolve_vector(op, t, acc, n, {}, 2); break;
    case BWLA_OP_NRM2: c = resolve_vector(op, t, acc, n, {}, 1); break;
    case BWLA_OP_CG: c = resolve_vector(op, t, acc, n, {}, 6); break;
    case BWLA_OP_GEMV_ROWS: c = resolve_rows(t, acc, m, n, nullptr, 0, nullptr); break;
    case BWLA_OP_GEMV_COLS: c = resolve_cols(t, acc, m, n, nullptr, 0, nullptr); break;
    case BWLA_OP_GER: c = resolve_ger(t, m, n, nullptr, nullptr, nullptr, 0); break;
    case BWLA_OP_BATCH: c = resolve_batch(t, acc, (double)n); break;
    default: return fail(BWLA_ERR_INVALID_ARG, "op %d", op);
    }
    cfg->block = c.block;
    cfg->vec = c.vec;
    cfg->unroll = c.unroll;
    cfg->grid = c.grid;
    cfg->increment = c.inc;
    cfg->rows = c.rows;
    cfg->split = c.split;
    return BWLA_OK;
}

bwla_status bwla_load_tuning(const char *path)
{
    if (!path)
        return fail(BWLA_ERR_INVALID_ARG, "path is NULL");
    load_env_table_once(); // so a later first lookup cannot overwrite this table
    std::string err;
    if (!load_table_file(path, &err))
        return fail(BWLA_ERR_INVALID_ARG, "%s", err.c_str());
    return BWLA_OK;
}

} // extern "C"

// ===========================================================================
// batch plans
// ===========================================================================
struct bwla_batch_plan {
    int t = 0, acc = 0, out_t = 0;
    bool persistent = false; // persistent work-queue kernel (opt-in) or grouped launch
    int device = 0;
    int grid = 0, block = 256, vec = 1;
    int64_t n_items = 0, n_dots = 0;
    int64_t n_gemv_items = 0; // grouped launch: GEMV items come first
    int64_t n_staged_items = 0; // of those, the staged tiles come first
    size_t stage_bytes = 0;     // dynamic LDS of the staged-tile kernel
    double bytes = 0;
    BatchItem *d_items = nullptr;
    BatchGemv *d_gemv = nullptr;
    BatchDot *d_dots = nullptr;
    double *d_partials = nullptr;
    unsigned *d_counters = nullptr; // the work counter
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {
void plan_free(bwla_batch_plan *p)
{
    if (!p)
        return;
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    (void)hipFree(p->d_items);
    (void)hipFree(p->d_gemv);
    (void)hipFree(p->d_dots);
    (void)hipFree(p->d_partials);
    (void)hipFree(p->d_counters);
    delete p;
}

// Plans use the grouped launch (one work-group per item).  The persistent
// work-queue kernel hung on hardware twice (a compiler-divergent loop around
// its work draw; see batched.hip) and its corrected form has not been run on
// a GPU, so it stays switched off: a plan asked for it with
// BWLA_ENABLE_UNVALIDATED_BATCH=1 is refused with BWLA_ERR_UNSUPPORTED.
bool persistent_requested()
{
    const char *v = getenv("BWLA_ENABLE_UNVALIDATED_BATCH");
    return v && v[0] == '1';
}

hipError_t enqueue_batch(bwla_batch_plan *p, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (p->n_items == 0)
        return e; // nothing to compute
    if (p->persistent) {
        e = launch_batch_reset(p->d_counters, 1, s);
        if (e != hipSuccess)
            return e;
    }
    BatchArgs a;
    a.items = p->d_items;
    a.n_items = p->n_items;
    a.n_gemv_items = p->n_gemv_items;
    a.n_staged_items = p->n_staged_items;
    a.gemv = p->d_gemv;
    a.dots = p->d_dots;
    a.partials = p->d_partials;
    a.work_counter = p->d_counters;
    a.out_f64 = p->out_t == BWLA_F64;
    a.vec = p->vec;
    e = by_type(p->t, [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        if (p->persistent)
            return launch_batched<T>(a, p->acc == BWLA_ACC_COMPENSATED, p->grid, p->block, s);
        return launch_grouped<T>(a, p->acc == BWLA_ACC_COMPENSATED, p->block, p->stage_bytes, s);
    });
    if (e != hipSuccess)
        return e;
    return launch_batch_finalize(p->d_dots, p->n_dots, p->d_partials, p->acc == BWLA_ACC_COMPENSATED,
                                 p->out_t == BWLA_F64, s);
}
} // namespace

extern "C" {

bwla_status bwla_batch_plan_create(bwla_dtype t, bwla_acc acc, bwla_dtype out_t, const bwla_gemv_desc *g,
                                   int32_t ng, const bwla_dot_desc *d, int32_t nd, const bwla_config *cfg,
                                   bwla_batch_plan **out)
{
    if (!out)
        return fail(BWLA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!valid_dtype(t))
        return fail(BWLA_ERR_UNSUPPORTED, "dtype %d", t);
    if (acc != BWLA_ACC_PLAIN && acc != BWLA_ACC_COMPENSATED)
        return fail(BWLA_ERR_UNSUPPORTED, "accumulation mode %d", acc);
    bwla_status st = out_type_ok(t, out_t);
    if (st)
        return st;
    if (ng < 0 || nd < 0 || (ng > 0 && !g) || (nd > 0 && !d))
        return fail(BWLA_ERR_INVALID_ARG, "bad descriptor arrays");
    if (cfg && (st = check_cfg(*cfg)) != BWLA_OK)
        return st;
    if (cfg && cfg->block > 512)
        return fail(BWLA_ERR_INVALID_ARG, "batch work-groups hold at most 512 threads (block %d)", cfg->block);
    if (persistent_requested())
        return fail(BWLA_ERR_UNSUPPORTED, "the persistent batched kernel is switched off (not validated on "
                                          "hardware); unset BWLA_ENABLE_UNVALIDATED_BATCH to use the grouped launch");
    const size_t es = dsize(t), os = out_t == BWLA_F64 ? 8 : 4;
    bool aligned = true;
    const int nv = native_vec(t);
    for (int i = 0; i < ng; ++i) {
        const bwla_gemv_desc &q = g[i];
        if (q.m < 0 || q.n < 0 || q.lda < std::max<int64_t>(1, q.n))
            return fail(BWLA_ERR_INVALID_ARG, "gemv %d: bad sizes or lda", i);
        if (q.m > 0 && !q.y)
            return fail(BWLA_ERR_INVALID_ARG, "gemv %d: y is NULL", i);
        if (q.m > 0 && q.n > 0 && (!q.A || !q.x))
            return fail(BWLA_ERR_INVALID_ARG, "gemv %d: NULL A or x", i);
        if (q.m > 0 && q.n > 0) {
            Span sy = span(q.y, q.m * os);
            if (overlaps(sy, span(q.A, matrix_bytes(q.m, q.n, q.lda, es))) || overlaps(sy, span(q.x, q.n * es)))
                return fail(BWLA_ERR_INVALID_ARG, "gemv %d: y overlaps A or x", i);
            if (fit_vec(nv, es, {q.A, q.x}, q.lda) != nv)
                aligned = false;
        }
    }
    for (int i = 0; i < nd; ++i) {
        const bwla_dot_desc &q = d[i];
        if (q.n < 0 || !q.out || (q.n > 0 && (!q.x || !q.y)))
            return fail(BWLA_ERR_INVALID_ARG, "dot %d: bad size or NULL pointer", i);
        if (q.n > 0) {
            Span so = span(q.out, os);
            if (overlaps(so, span(q.x, q.n * es)) || overlaps(so, span(q.y, q.n * es)))
                return fail(BWLA_ERR_INVALID_ARG, "dot %d: out overlaps an input", i);
            if (fit_vec(nv, es, {q.x, q.y}) != nv)
                aligned = false;
        }
    }
    // the plan's algorithmic bytes select its table entry (a cfg field that
    // is set overrides it)
    double total = 0;
    for (int i = 0; i < ng; ++i)
        total += (double)g[i].m * g[i].n * es + (double)g[i].n * es + (double)g[i].m * os;
    for (int i = 0; i < nd; ++i)
        total += 2.0 * d[i].n * es + os;
    const Cfg bc = resolve_batch(t, acc, total);
    const int packs_per_lane = cfg && cfg->unroll ? cfg->unroll : bc.unroll;
    bwla_batch_plan *p = new bwla_batch_plan();
    p->t = t;
    p->acc = acc;
    p->out_t = out_t;
    p->vec = aligned ? nv : 1;
    p->block = cfg && cfg->block ? cfg->block : bc.block;
    p->persistent = false;
    (void)hipGetDevice(&p->device);

    // work items, with their cost in bytes for the largest-first order
    struct Work {
        BatchItem it;
        double cost;
    };
    std::vector<Work> work;
    std::vector<BatchGemv> hg(ng);
    std::vector<BatchDot> hd(nd);
    // Work items: sized for one wave64 each in the persistent kernel, for one
    // work-group each in the grouped launch.  Chunk starts stay multiples of
    // 64 * 16 elements, so every chunk begins on a pack boundary.
    const int64_t kTileElems = p->persistent ? (1 << 15) : (1 << 16); // elements of A per GEMV row tile
    const int64_t kChunk = p->persistent ? (1 << 14) : (1 << 16);     // elements per dot chunk
    for (int i = 0; i < ng; ++i) {
        const bwla_gemv_desc &q = g[i];
        BatchGemv &b = hg[i];
        b.A = q.A;
        b.m = q.m;
        b.n = q.n;
        b.lda = q.lda;
        b.x = q.x;
        b.y = q.y;
        // grouped launch: x staged in LDS when it fits (rows at any
        // alignment; measured as fast as, or faster than, x in registers on
        // aligned rows), else 16-byte packs of every operand when A's rows
        // and x are 16-byte aligned, else one element per access
        int v_item = p->vec;
        if (!p->persistent) {
            if (q.n <= tile_stage_elems((int)es))
                b.mode = kModeStaged, v_item = nv;
            else if (q.m > 0 && q.n > 0 && fit_vec(nv, es, {q.A, q.x}, q.lda) == nv)
                b.mode = kModePacked, v_item = nv;
            else
                b.mode = kModeScalar, v_item = 1;
        } else {
            b.mode = p->vec == 1 ? kModeScalar : kModePacked;
        }
        int64_t packs = std::max<int64_t>(1, ceil_div(q.n, v_item));
        if (b.mode == kModeStaged && !p->persistent) // each lane owns up to packs_per_lane packs of its row
            packs = ceil_div(packs, packs_per_lane);
        int lanes = 1;
        while (lanes < 64 && lanes < packs)
            lanes <<= 1;
        b.lanes = lanes;
        if (q.m == 0)
            continue;
        int64_t rpi = std::max<int64_t>(1, std::min<int64_t>(q.m, kTileElems / std::max<int64_t>(1, q.n)));
        if (b.mode == kModeStaged && !p->persistent) {
            // whole row batches per tile: a staged work-group holds block / lanes
            // rows at a time, so a tile of a multiple of that leaves no slot idle
            const int64_t slots = std::max<int64_t>(1, p->block / lanes);
            if (rpi > slots)
                rpi = rpi / slots * slots;
            p->stage_bytes = std::max(p->stage_bytes, tile_stage_bytes((int)es, q.n, lanes));
        }
        for (int64_t r0 = 0; r0 < q.m; r0 += rpi) {
            Work w{};
            w.it.kind = 0;
            w.it.pad = b.mode == kModeStaged ? 0 : 1; // sort key: staged tiles first
            w.it.prob = i;
            w.it.begin = r0;
            w.it.end = std::min(q.m, r0 + rpi);
            w.cost = (double)(w.it.end - w.it.begin) * std::max<int64_t>(q.n, 1) * es;
            work.push_back(w);
        }
        p->bytes += (double)q.m * q.n * es + (double)q.n * es + (double)q.m * os;
    }
    int64_t slots = 0;
    for (int i = 0; i < nd; ++i) {
        const bwla_dot_desc &q = d[i];
        BatchDot &b = hd[i];
        b.x = q.x;
        b.y = q.y;
        b.n = q.n;
        b.out = q.out;
        b.slot0 = slots;
        b.chunks = (int32_t)std::max<int64_t>(1, ceil_div(q.n, kChunk));
        if (p->persistent)
            b.mode = p->vec == 1 ? kModeScalar : kModePacked;
        else
            b.mode = q.n > 0 && fit_vec(nv, es, {q.x, q.y}) == nv ? kModePacked : kModeScalar;
        for (int c = 0; c < b.chunks; ++c) {
            Work w{};
            w.it.kind = 1;
            w.it.prob = i;
            w.it.begin = (int64_t)c * kChunk;
            w.it.end = std::min<int64_t>(q.n, (int64_t)(c + 1) * kChunk);
            w.it.chunk = c;
            w.cost = (double)std::max<int64_t>(1, w.it.end - w.it.begin) * 2 * es;
            work.push_back(w);
        }
        slots += b.chunks;
        p->bytes += 2.0 * q.n * es + os;
    }
    // Largest first.  The grouped launch runs GEMV tiles and dot chunks as two
    // kernels, so it orders by kind first.
    if (p->persistent)
        std::stable_sort(work.begin(), work.end(), [](const Work &a, const Work &b) { return a.cost > b.cost; });
    else
        std::stable_sort(work.begin(), work.end(), [](const Work &a, const Work &b) {
            if (a.it.kind != b.it.kind)
                return a.it.kind < b.it.kind;
            if (a.it.pad != b.it.pad)
                return a.it.pad < b.it.pad;
            return a.cost > b.cost;
        });
    for (const Work &w : work) {
        p->n_gemv_items += w.it.kind == 0;
        p->n_staged_items += w.it.kind == 0 && w.it.pad == 0;
    }
    for (Work &w : work)
        w.it.pad = 0;
    std::vector<BatchItem> items(work.size());
    for (size_t i = 0; i < work.size(); ++i)
        items[i] = work[i].it;
    p->n_items = (int64_t)items.size();
    p->n_dots = nd;
    if (p->n_items > 0x7fffffff) {
        delete p;
        return fail(BWLA_ERR_INVALID_ARG, "batch has more than 2^31 - 1 work items");
    }
    if (p->persistent) {
        // One wave per item at a time: enough work-groups to fill every CU's
        // wave slots, but no more waves than items.
        const int64_t per_cu = std::max(1, 2048 / p->block);
        const int64_t waves_per_block = p->block / 64;
        int64_t grid = cfg && cfg->grid ? cfg->grid : (int64_t)device_cus() * per_cu;
        grid = std::min<int64_t>(grid, ceil_div(std::max<int64_t>(1, p->n_items), waves_per_block));
        p->grid = (int)std::max<int64_t>(1, grid);
    } else {
        p->grid = (int)std::max<int64_t>(1, p->n_items); // one work-group per item
    }
    // the shape logged: work items and the plan's algorithmic bytes; unroll
    // is the packs per lane of the staged GEMV tiles
    log_call("batch plan", t, acc, p->n_items, (int64_t)total,
             Cfg{p->block, p->vec, packs_per_lane, p->grid, 0, 1, 1});

    auto alloc_copy = [&](void **dst, const void *src, size_t bytes) -> hipError_t {
        if (bytes == 0)
            bytes = 16;
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess)
            return e;
        if (src)
            return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        return hipSuccess;
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess)
        e = alloc_copy((void **)&p->d_items, items.data(), items.size() * sizeof(BatchItem));
    if (e == hipSuccess)
        e = alloc_copy((void **)&p->d_gemv, hg.data(), hg.size() * sizeof(BatchGemv));
    if (e == hipSuccess)
        e = alloc_copy((void **)&p->d_dots, hd.data(), hd.size() * sizeof(BatchDot));
    if (e == hipSuccess)
        e = alloc_copy((void **)&p->d_partials, nullptr, (size_t)std::max<int64_t>(1, slots) * 2 * sizeof(double));
    if (e == hipSuccess) {
        std::vector<unsigned> zeros(1, 0u);
        e = alloc_copy((void **)&p->d_counters, zeros.data(), zeros.size() * sizeof(unsigned));
    }
    if (e != hipSuccess) {
        plan_free(p);
        return hip_check(e, "batch plan allocation");
    }
    *out = p;
    return BWLA_OK;
}

bwla_status bwla_batch_run(bwla_batch_plan *p, void *stream)
{
    if (!p)
        return fail(BWLA_ERR_INVALID_ARG, "plan is NULL");
    if (p->n_items == 0)
        return BWLA_OK;
    return hip_check(enqueue_batch(p, (hipStream_t)stream), "batched launch");
}

bwla_status bwla_batch_capture(bwla_batch_plan *p, void *stream)
{
    if (!p)
        return fail(BWLA_ERR_INVALID_ARG, "plan is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (!s)
        return fail(BWLA_ERR_NOT_CAPTURABLE, "the default stream cannot be captured; pass a created stream");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    bwla_status st = hip_check(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
    if (st)
        return st;
    if (cs != hipStreamCaptureStatusNone)
        return fail(BWLA_ERR_NOT_CAPTURABLE, "stream is already capturing");
    if (p->exec) {
        (void)hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    st = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (st)
        return st;
    hipError_t e = enqueue_batch(p, s);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return hip_check(e != hipSuccess ? e : e2, "batch capture");
    }
    p->graph = graph;
    st = hip_check(hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    return st;
}

bwla_status bwla_batch_replay(bwla_batch_plan *p, void *stream)
{
    if (!p)
        return fail(BWLA_ERR_INVALID_ARG, "plan is NULL");
    if (!p->exec)
        return fail(BWLA_ERR_INVALID_ARG, "plan has no captured graph");
    return hip_check(hipGraphLaunch(p->exec, (hipStream_t)stream), "hipGraphLaunch");
}

bwla_status bwla_batch_info(const bwla_batch_plan *p, int64_t *items, int32_t *grid, double *bytes)
{
    if (!p)
        return fail(BWLA_ERR_INVALID_ARG, "plan is NULL");
    if (items)
        *items = p->n_items;
    if (grid)
        *grid = p->grid;
    if (bytes)
        *bytes = p->bytes;
    return BWLA_OK;
}

void bwla_batch_plan_destroy(bwla_batch_plan *p) { plan_free(p); }

} // extern "C"
