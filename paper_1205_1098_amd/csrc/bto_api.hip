// C entry points of libbto: argument checks, workspace layout, and the
// fused / unfused kernel sequences for the seven Table I kernels.

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "bto.h"
#include "bto_batch.hpp"
#include "bto_internal.hpp"
#include "bto_tuned.hpp"

using namespace bto;

namespace {

thread_local std::string t_error;

bto_status fail(bto_status s, const std::string &msg)
{
    t_error = msg;
    return s;
}

// ---- tile configurations ---------------------------------------------------
//
// Each matrix sweep has a slot whose tile shape can be changed at run time
// (the autotuner does).  Workspace sizes are computed for the most demanding
// shape any slot may take (kv >= 2 for the row-dot sweeps, whose partials
// are per wave tile; rb >= 32 for the column sums), so they depend on the
// arguments alone.

std::mutex g_cfg_mu;
TileCfg g_cfg[SLOT_COUNT][kSizeBuckets] = BTO_TUNED_DEFAULTS;

constexpr int kMinKv = kMinTileKv;
constexpr int kMinRb = 32;

TileCfg cfg_of(Slot s, int64_t m, int64_t n)
{
    std::lock_guard<std::mutex> g(g_cfg_mu);
    return g_cfg[s][size_bucket(m, n)];
}

int64_t max_ncols(int64_t n) { return ceil_div(n, 128 * kMinKv); }
int64_t max_nbands(int64_t m) { return ceil_div(m, kMinRb); }

// ---- workspace carving -------------------------------------------------------

struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *p) : base(static_cast<char *>(p)) {}
    double *take(int64_t ndoubles)
    {
        double *p = base ? reinterpret_cast<double *>(base + off) : nullptr;
        off += round256((size_t)(ndoubles > 0 ? ndoubles : 0) * sizeof(double));
        return p;
    }
};

size_t bytes_rowparts(int64_t m, int64_t n) { return round256((size_t)(max_ncols(n) * m) * 8); }
size_t bytes_colparts(int64_t m, int64_t n) { return round256((size_t)(max_nbands(m) * n) * 8); }
size_t bytes_vec(int64_t n) { return round256((size_t)n * 8); }

size_t ws_bytes(bto_kernel k, int64_t m, int64_t n, bto_form f)
{
    switch (k) {
    case BTO_K_BICGK: {
        const size_t tiles = bytes_rowparts(m, n) + bytes_colparts(m, n);
        if (f == BTO_UNFUSED)
            return tiles;
        // either fused kernel may be selected by tuning: room for both
        const size_t rowres = round256((size_t)(rowres_max_parts(m, n, true) * n) * 8);
        return tiles > rowres ? tiles : rowres;
    }
    case BTO_K_GEMVER:
    case BTO_K_DGEMVT:
        return bytes_rowparts(m, n) + bytes_colparts(m, n);
    case BTO_K_GEMVER_CONTRACTED:
        // the tile partials, then the two passes' auxiliary dot parts
        return bytes_rowparts(m, n) + bytes_colparts(m, n) + bytes_vec(2 * max_nbands(m)) +
               bytes_vec(2 * max_ncols(n));
    case BTO_K_BATAX:
    case BTO_K_ATAX: {
        size_t split = bytes_vec(m) + bytes_rowparts(m, n) + bytes_colparts(m, n);
        if (f == BTO_UNFUSED)
            return split;
        // sized for the largest grid any tunable workgroup size can give
        int64_t g = atax_rowres_max_parts(m, n);
        size_t rowres = round256((size_t)(g * n) * 8);
        return g > 0 ? rowres : split;
    }
    case BTO_K_DGEMV:
        return bytes_rowparts(m, n);
    case BTO_K_GESUMMV:
        // fused: both matrices' row-dot partials; unfused: one set, reused,
        // and the temporary alpha A x
        return f == BTO_FUSED ? 2 * bytes_rowparts(m, n) : bytes_rowparts(m, n) + bytes_vec(m);
    case BTO_K_AXPYDOT:
        return round256((size_t)dot_parts(n) * 8);
    case BTO_K_WAXPBY:
    case BTO_K_VADD:
        return f == BTO_UNFUSED ? bytes_vec(n) : 0;
    default:
        break;
    }
    return 0;
}

// ---- argument checks ---------------------------------------------------------

struct Span {
    const char *name;
    uintptr_t lo, hi;  // [lo, hi), empty when lo == hi
    bool out;
};

Span vspan(const char *name, const void *p, int64_t n, bool out)
{
    uintptr_t lo = reinterpret_cast<uintptr_t>(p);
    return {name, lo, n > 0 ? lo + (uintptr_t)n * 8 : lo, out};
}

Span mspan(const char *name, const void *p, int64_t m, int64_t n, int64_t ld, bool out)
{
    uintptr_t lo = reinterpret_cast<uintptr_t>(p);
    if (m <= 0 || n <= 0)
        return {name, lo, lo, out};
    return {name, lo, lo + (uintptr_t)((m - 1) * ld + n) * 8, out};
}

Span wspan(const void *p, size_t bytes)
{
    uintptr_t lo = reinterpret_cast<uintptr_t>(p);
    return {"ws", lo, lo + bytes, true};
}

struct AllowedAlias {
    const char *a, *b;
};

bool name_is(const char *x, const char *y) { return std::string(x) == y; }

// An output may not overlap any other operand, except in an exact alias the
// entry point allows (same start and same extent).
bto_status check_aliases(const std::vector<Span> &sp, const std::vector<AllowedAlias> &ok)
{
    for (size_t i = 0; i < sp.size(); ++i) {
        for (size_t j = i + 1; j < sp.size(); ++j) {
            const Span &a = sp[i], &b = sp[j];
            if (!a.out && !b.out)
                continue;
            if (a.lo == a.hi || b.lo == b.hi)
                continue;
            if (a.lo >= b.hi || b.lo >= a.hi)
                continue;
            bool exact = a.lo == b.lo && a.hi == b.hi;
            bool allowed = false;
            for (const AllowedAlias &al : ok)
                if ((name_is(al.a, a.name) && name_is(al.b, b.name)) ||
                    (name_is(al.a, b.name) && name_is(al.b, a.name)))
                    allowed = true;
            if (!(exact && allowed))
                return fail(BTO_ERR_ALIAS, std::string("operand ") + a.name + " overlaps " + b.name);
        }
    }
    return BTO_SUCCESS;
}

bto_status need(bool cond, const char *what)
{
    return cond ? BTO_SUCCESS : fail(BTO_ERR_INVALID_ARG, what);
}

#define BTO_TRY(expr)                         \
    do {                                      \
        bto_status _s = (expr);               \
        if (_s != BTO_SUCCESS)                \
            return _s;                        \
    } while (0)

bto_status check_form(bto_form f)
{
    return need(f == BTO_FUSED || f == BTO_UNFUSED, "form must be BTO_FUSED or BTO_UNFUSED");
}

bto_status check_matrix(int64_t m, int64_t n, const void *A, int64_t lda, const char *name)
{
    BTO_TRY(need(m >= 0 && n >= 0, "negative size"));
    BTO_TRY(need(lda >= (n > 1 ? n : 1), "leading dimension smaller than max(1, n)"));
    if (m > 0 && n > 0 && A == nullptr)
        return fail(BTO_ERR_INVALID_ARG, std::string(name) + " is NULL");
    if (m > (int64_t)65535 * kMinRb)
        return fail(BTO_ERR_UNSUPPORTED, "more rows than the tile grid can address");
    return BTO_SUCCESS;
}

bto_status check_vec(const void *p, int64_t n, const char *name)
{
    if (n > 0 && p == nullptr)
        return fail(BTO_ERR_INVALID_ARG, std::string(name) + " is NULL");
    return BTO_SUCCESS;
}

bto_status check_ws(void *ws, size_t have, size_t needed)
{
    if (have < needed)
        return fail(BTO_ERR_WORKSPACE, "workspace too small: need " + std::to_string(needed) +
                                           " bytes, got " + std::to_string(have));
    if (needed > 0 && ws == nullptr)
        return fail(BTO_ERR_INVALID_ARG, "ws is NULL");
    if (needed > 0 && (reinterpret_cast<uintptr_t>(ws) & 255u))
        return fail(BTO_ERR_INVALID_ARG, "ws is not 256-byte aligned");
    return BTO_SUCCESS;
}

// Host containers throw std::bad_alloc when memory runs out; no exception
// may cross the C boundary, so the plan builders report it as a status.
template <typename F>
bto_status host_guard(F &&body)
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(BTO_ERR_UNSUPPORTED, "out of host memory while building the plan");
    } catch (...) {
        return fail(BTO_ERR_UNSUPPORTED, "host error while building the plan");
    }
}

bto_status check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(BTO_ERR_HIP, std::string("HIP: ") + hipGetErrorString(e));
    return BTO_SUCCESS;
}

TileArgs targs(int64_t m, int64_t n, const double *A, int64_t lda)
{
    TileArgs a{};
    a.m = m;
    a.n = n;
    a.A = A;
    a.lda = lda;
    a.ldb = lda;
    return a;
}

FinishJob fjob(const double *P, int64_t nparts, int64_t len, double scale, const double *add,
               double *out)
{
    return FinishJob{P, nparts, len, scale, add, out};
}

const FinishJob kNoJob{nullptr, 0, 0, 0.0, nullptr, nullptr};

// out_rows = scale * A xr : tile sweep of A with row dots + finish
bto_status unsupported(Slot s)
{
    return fail(BTO_ERR_UNSUPPORTED, std::string("tile configuration of ") + kSlotNames[s] +
                                         " is not supported");
}

bto_status gemv_n(Slot s, int64_t m, int64_t n, const double *A, int64_t lda, const double *xr,
                  double scale, double *out, double *Prow, hipStream_t st)
{
    TileCfg c = cfg_of(s, m, n);
    TileArgs a = targs(m, n, A, lda);
    a.xr = xr;
    a.Prow = Prow;
    if (!launch_tile(kSlotNames[s], OP_ROWDOT, c, a, st))
        return unsupported(s);
    int64_t np = n > 0 ? tile_ncols(c, n) : 0;
    launch_finish("finish", fjob(Prow, np, m, scale, nullptr, out), kNoJob, st);
    return BTO_SUCCESS;
}

// out_cols = scale * A^T yc + add
bto_status gemv_t(Slot s, int64_t m, int64_t n, const double *A, int64_t lda, const double *yc,
                  double scale, const double *add, double *out, double *Pcol, hipStream_t st)
{
    TileCfg c = cfg_of(s, m, n);
    TileArgs a = targs(m, n, A, lda);
    a.yc = yc;
    a.Pcol = Pcol;
    if (!launch_tile(kSlotNames[s], OP_COLSUM, c, a, st))
        return unsupported(s);
    int64_t np = m > 0 ? tile_nbands(c, m) : 0;
    launch_finish("finish", fjob(Pcol, np, n, scale, add, out), kNoJob, st);
    return BTO_SUCCESS;
}

}  // namespace

// ---- timing ------------------------------------------------------------------

namespace {

struct TimingRec {
    int name;
    hipEvent_t a, b;
};

std::mutex g_tmu;
bool g_tenabled = false;
std::string g_tonly;   // when set, only launches of this name are timed
std::vector<TimingRec> g_recs;
std::vector<std::string> g_tnames;
std::vector<double> g_tms;
std::vector<int64_t> g_tcount;
std::vector<hipEvent_t> g_pool;
thread_local hipEvent_t t_start = nullptr;
thread_local int t_name = -1;
thread_local bool t_capturing = false;   // no timing events inside a graph capture

hipEvent_t take_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence (cache writeback and invalidate)
    // at each record, which would slow the kernels being timed
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
        return nullptr;
    return e;
}

int name_index(const char *name)
{
    for (size_t i = 0; i < g_tnames.size(); ++i)
        if (g_tnames[i] == name)
            return (int)i;
    g_tnames.emplace_back(name);
    g_tms.push_back(0.0);
    g_tcount.push_back(0);
    return (int)g_tnames.size() - 1;
}

}  // namespace

namespace bto {

void timing_begin(hipStream_t st, const char *name)
{
    std::lock_guard<std::mutex> g(g_tmu);
    t_start = nullptr;
    if (!g_tenabled || t_capturing)
        return;
    if (!g_tonly.empty() && g_tonly != name)
        return;
    hipEvent_t e = take_event();
    if (!e)
        return;
    (void)hipEventRecord(e, st);
    t_start = e;
    t_name = name_index(name);
}

void timing_end(hipStream_t st)
{
    std::lock_guard<std::mutex> g(g_tmu);
    if (!t_start)
        return;
    hipEvent_t e = take_event();
    if (!e) {
        g_pool.push_back(t_start);
        t_start = nullptr;
        return;
    }
    (void)hipEventRecord(e, st);
    g_recs.push_back({t_name, t_start, e});
    t_start = nullptr;
}

}  // namespace bto

extern "C" {

int bto_version(void) { return 100; }

size_t bto_workspace_bytes(bto_kernel k, int64_t m, int64_t n, bto_form f)
{
    if (m < 0 || n < 0 || (f != BTO_FUSED && f != BTO_UNFUSED))
        return 0;
    return ws_bytes(k, m, n, f);
}

const char *bto_status_string(bto_status s)
{
    switch (s) {
    case BTO_SUCCESS: return "success";
    case BTO_ERR_INVALID_ARG: return "invalid argument";
    case BTO_ERR_ALIAS: return "illegal operand overlap";
    case BTO_ERR_WORKSPACE: return "workspace too small";
    case BTO_ERR_HIP: return "HIP error";
    case BTO_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *bto_last_error(void) { return t_error.c_str(); }

// ---- BICGK -------------------------------------------------------------------

bto_status bto_bicgk(int64_t m, int64_t n, const double *A, int64_t lda, const double *p,
                     const double *r, double *q, double *s, void *ws, size_t ws_bytes_,
                     bto_form form, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(check_form(form));
    BTO_TRY(check_matrix(m, n, A, lda, "A"));
    BTO_TRY(check_vec(p, n, "p"));
    BTO_TRY(check_vec(r, m, "r"));
    BTO_TRY(check_vec(q, m, "q"));
    BTO_TRY(check_vec(s, n, "s"));
    const size_t need_ws = ws_bytes(BTO_K_BICGK, m, n, form);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({mspan("A", A, m, n, lda, false), vspan("p", p, n, false),
                           vspan("r", r, m, false), vspan("q", q, m, true),
                           vspan("s", s, n, true), wspan(ws, need_ws)},
                          {}));

    const int bt = form == BTO_FUSED ? get_bicgk_rowres_threads(size_bucket(m, n)) : 0;
    const int64_t G = bt ? rowres_parts(m, n, bt, true) : 0;
    if (G > 0) {
        // row-resident sweep: q rows directly, s from G partial vectors
        Carve cw(ws);
        double *P = cw.take(G * n);
        launch_bicgk_rowres(m, n, A, lda, p, r, q, P, bt, st);
        launch_finish("finish", fjob(P, G, n, 1.0, nullptr, s), kNoJob, st);
        return check_launch();
    }
    Carve cv(ws);
    double *Prow = cv.take(max_ncols(n) * m);
    double *Pcol = cv.take(max_nbands(m) * n);
    if (form == BTO_FUSED && m > 0 && n > 0) {
        TileCfg c = cfg_of(SLOT_BICGK_FUSED, m, n);
        TileArgs a = targs(m, n, A, lda);
        a.xr = p;
        a.yc = r;
        a.Prow = Prow;
        a.Pcol = Pcol;
        if (!launch_tile(kSlotNames[SLOT_BICGK_FUSED], OP_ROWDOT | OP_COLSUM, c, a, st))
            return unsupported(SLOT_BICGK_FUSED);
        launch_finish("finish", fjob(Prow, tile_ncols(c, n), m, 1.0, nullptr, q),
                      fjob(Pcol, tile_nbands(c, m), n, 1.0, nullptr, s), st);
    } else {
        BTO_TRY(gemv_n(SLOT_GEMV_N, m, n, A, lda, p, 1.0, q, Prow, st));
        BTO_TRY(gemv_t(SLOT_GEMV_T, m, n, A, lda, r, 1.0, nullptr, s, Pcol, st));
    }
    return check_launch();
}

// ---- GEMVER ------------------------------------------------------------------

}  // extern "C"

namespace {

// GEMVER's checks and launches on a given workspace (the caller's, or the
// library's own scratch for bto_gemver_noalloc).
bto_status gemver_run(int64_t m, int64_t n, double alpha, double beta, const double *A,
                      int64_t lda, const double *u1, const double *v1, const double *u2,
                      const double *v2, const double *y, const double *z, double *B,
                      int64_t ldb, double *x, double *w, void *ws, size_t ws_bytes_,
                      bto_form form, hipStream_t st)
{
    BTO_TRY(check_form(form));
    BTO_TRY(check_matrix(m, n, A, lda, "A"));
    BTO_TRY(check_matrix(m, n, B, ldb, "B"));
    BTO_TRY(check_vec(u1, m, "u1"));
    BTO_TRY(check_vec(u2, m, "u2"));
    BTO_TRY(check_vec(y, m, "y"));
    BTO_TRY(check_vec(w, m, "w"));
    BTO_TRY(check_vec(v1, n, "v1"));
    BTO_TRY(check_vec(v2, n, "v2"));
    BTO_TRY(check_vec(z, n, "z"));
    BTO_TRY(check_vec(x, n, "x"));
    if (B == A && ldb != lda && m > 1 && n > 0)
        return fail(BTO_ERR_ALIAS, "B == A requires ldb == lda");
    const size_t need_ws = ws_bytes(BTO_K_GEMVER, m, n, form);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({mspan("A", A, m, n, lda, false), vspan("u1", u1, m, false),
                           vspan("v1", v1, n, false), vspan("u2", u2, m, false),
                           vspan("v2", v2, n, false), vspan("y", y, m, false),
                           vspan("z", z, n, false), mspan("B", B, m, n, ldb, true),
                           vspan("x", x, n, true), vspan("w", w, m, true), wspan(ws, need_ws)},
                          {{"A", "B"}}));

    Carve cv(ws);
    double *Prow = cv.take(max_ncols(n) * m);
    double *Pcol = cv.take(max_nbands(m) * n);
    if (form == BTO_FUSED) {
        // pass 1: B = A + u1 v1^T + u2 v2^T and the partial sums of B^T y
        TileCfg c = cfg_of(SLOT_GEMVER_P1, m, n);
        TileArgs a = targs(m, n, A, lda);
        a.B = B;
        a.ldb = ldb;
        a.u1 = u1;
        a.v1 = v1;
        a.u2 = u2;
        a.v2 = v2;
        a.yc = y;
        a.Pcol = Pcol;
        if (!launch_tile(kSlotNames[SLOT_GEMVER_P1], OP_UPD1 | OP_UPD2 | OP_COLSUM, c, a, st))
            return unsupported(SLOT_GEMVER_P1);
        const int64_t np = (m > 0 && n > 0) ? tile_nbands(c, m) : 0;
        launch_finish("finish", fjob(Pcol, np, n, beta, z, x), kNoJob, st);
        // pass 2: w = alpha B x
        BTO_TRY(gemv_n(SLOT_GEMVER_P2, m, n, B, ldb, x, alpha, w, Prow, st));
    } else {
        TileCfg c = cfg_of(SLOT_GER, m, n);
        TileArgs a = targs(m, n, A, lda);
        a.B = B;
        a.ldb = ldb;
        a.u1 = u1;
        a.v1 = v1;
        if (!launch_tile("ger", OP_UPD1, c, a, st))     // B = A + u1 v1^T
            return unsupported(SLOT_GER);
        a = targs(m, n, B, ldb);
        a.B = B;
        a.ldb = ldb;
        a.u1 = u2;
        a.v1 = v2;
        launch_tile("ger", OP_UPD1, c, a, st);          // B = B + u2 v2^T
        BTO_TRY(gemv_t(SLOT_GEMV_T, m, n, B, ldb, y, beta, z, x, Pcol, st));
        BTO_TRY(gemv_n(SLOT_GEMV_N, m, n, B, ldb, x, alpha, w, Prow, st));
    }
    return check_launch();
}

// ---- GEMVER on library-owned scratch -----------------------------------------
//
// The column-sum and row-dot partials of bto_gemver_noalloc live in this
// file-scope device array.  Each device that runs the entry point holds its
// own copy, at its own address, from the first call on that device until
// the process ends.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in); it passes the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
// Every partial is written before it is read, so nothing needs clearing.

constexpr size_t kNoAllocScratchBytes = size_t(80) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

bto_status noalloc_scratch(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(BTO_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(BTO_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(BTO_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BTO_SUCCESS;
}

}  // namespace

extern "C" {

bto_status bto_gemver(int64_t m, int64_t n, double alpha, double beta, const double *A,
                      int64_t lda, const double *u1, const double *v1, const double *u2,
                      const double *v2, const double *y, const double *z, double *B,
                      int64_t ldb, double *x, double *w, void *ws, size_t ws_bytes_,
                      bto_form form, hipStream_t st)
{
    t_error.clear();
    return gemver_run(m, n, alpha, beta, A, lda, u1, v1, u2, v2, y, z, B, ldb, x, w, ws,
                      ws_bytes_, form, st);
}

size_t bto_gemver_noalloc_max_scratch_bytes(void) { return kNoAllocScratchBytes; }

bto_status bto_gemver_noalloc(int64_t m, int64_t n, double alpha, double beta, const double *A,
                              int64_t lda, const double *u1, const double *v1, const double *u2,
                              const double *v2, const double *y, const double *z, double *B,
                              int64_t ldb, double *x, double *w, bto_form form, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(check_form(form));
    BTO_TRY(need(m >= 0 && n >= 0, "negative size"));
    const size_t need_ws = ws_bytes(BTO_K_GEMVER, m, n, form);
    if (need_ws > kNoAllocScratchBytes)
        return fail(BTO_ERR_WORKSPACE, "bto_gemver_noalloc: " + std::to_string(m) + " x " +
                                           std::to_string(n) + " needs " +
                                           std::to_string(need_ws) + " bytes of scratch, above "
                                           "the library's " +
                                           std::to_string(kNoAllocScratchBytes));
    void *ws = nullptr;
    if (need_ws > 0)
        BTO_TRY(noalloc_scratch(&ws));
    return gemver_run(m, n, alpha, beta, A, lda, u1, v1, u2, v2, y, z, B, ldb, x, w, ws,
                      need_ws, form, st);
}

// ---- ATAX --------------------------------------------------------------------

namespace {

// y = scale * A^T (A x): ATAX (scale 1) and BATAX
bto_status atax_scaled(bto_kernel kind, int64_t m, int64_t n, double scale, const double *A,
                       int64_t lda, const double *x, double *y, void *ws, size_t ws_bytes_,
                       bto_form form, hipStream_t st)
{
    BTO_TRY(check_form(form));
    BTO_TRY(check_matrix(m, n, A, lda, "A"));
    BTO_TRY(check_vec(x, n, "x"));
    BTO_TRY(check_vec(y, n, "y"));
    const size_t need_ws = ws_bytes(kind, m, n, form);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({mspan("A", A, m, n, lda, false), vspan("x", x, n, false),
                           vspan("y", y, n, true), wspan(ws, need_ws)},
                          {}));

    const int threads = get_rowres_threads(size_bucket(m, n));
    const int64_t G = form == BTO_FUSED ? atax_rowres_parts(m, n, threads) : 0;
    Carve cv(ws);
    if (G > 0) {
        double *P = cv.take(G * n);
        launch_atax_rowres(m, n, A, lda, x, P, threads, st);
        launch_finish("finish", fjob(P, G, n, scale, nullptr, y), kNoJob, st);
    } else {
        double *t = cv.take(m);
        double *Prow = cv.take(max_ncols(n) * m);
        double *Pcol = cv.take(max_nbands(m) * n);
        BTO_TRY(gemv_n(SLOT_GEMV_N, m, n, A, lda, x, 1.0, t, Prow, st));
        BTO_TRY(gemv_t(SLOT_GEMV_T, m, n, A, lda, t, scale, nullptr, y, Pcol, st));
    }
    return check_launch();
}

}  // namespace

bto_status bto_atax(int64_t m, int64_t n, const double *A, int64_t lda, const double *x,
                    double *y, void *ws, size_t ws_bytes_, bto_form form, hipStream_t st)
{
    t_error.clear();
    return atax_scaled(BTO_K_ATAX, m, n, 1.0, A, lda, x, y, ws, ws_bytes_, form, st);
}

bto_status bto_batax(int64_t m, int64_t n, double beta, const double *A, int64_t lda,
                     const double *x, double *y, void *ws, size_t ws_bytes_, bto_form form,
                     hipStream_t st)
{
    t_error.clear();
    return atax_scaled(BTO_K_BATAX, m, n, beta, A, lda, x, y, ws, ws_bytes_, form, st);
}

// ---- GEMVER with B contracted ---------------------------------------------------

bto_status bto_gemver_contracted(int64_t m, int64_t n, double alpha, double beta,
                                 const double *A, int64_t lda, const double *u1,
                                 const double *v1, const double *u2, const double *v2,
                                 const double *y, const double *z, double *x, double *w,
                                 void *ws, size_t ws_bytes_, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(check_matrix(m, n, A, lda, "A"));
    BTO_TRY(check_vec(u1, m, "u1"));
    BTO_TRY(check_vec(v1, n, "v1"));
    BTO_TRY(check_vec(u2, m, "u2"));
    BTO_TRY(check_vec(v2, n, "v2"));
    BTO_TRY(check_vec(y, m, "y"));
    BTO_TRY(check_vec(z, n, "z"));
    BTO_TRY(check_vec(x, n, "x"));
    BTO_TRY(check_vec(w, m, "w"));
    const size_t need_ws = ws_bytes(BTO_K_GEMVER_CONTRACTED, m, n, BTO_FUSED);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({mspan("A", A, m, n, lda, false), vspan("u1", u1, m, false),
                           vspan("v1", v1, n, false), vspan("u2", u2, m, false),
                           vspan("v2", v2, n, false), vspan("y", y, m, false),
                           vspan("z", z, n, false), vspan("x", x, n, true),
                           vspan("w", w, m, true), wspan(ws, need_ws)},
                          {}));

    Carve cv(ws);
    double *Prow = cv.take(max_ncols(n) * m);
    double *Pcol = cv.take(max_nbands(m) * n);
    double *aux1 = cv.take(2 * max_nbands(m));   // u1.y, u2.y per row band
    double *aux2 = cv.take(2 * max_ncols(n));    // v1.x, v2.x per wave tile

    // pass 1: A^T y per band, and the band's u1.y and u2.y
    const TileCfg c1 = cfg_of(SLOT_DGEMVT_P1, m, n);
    TileArgs a1 = targs(m, n, A, lda);
    a1.yc = y;
    a1.u1 = u1;
    a1.u2 = u2;
    a1.Pcol = Pcol;
    a1.Prow = aux1;
    if (!launch_tile(kSlotNames[SLOT_DGEMVT_P1], OP_COLSUM | OP_AUX, c1, a1, st))
        return unsupported(SLOT_DGEMVT_P1);
    const int64_t nb = m > 0 ? tile_nbands(c1, m) : 0;
    launch_finish_aux("finish", {fjob(Pcol, nb, n, beta, z, x), aux1, n > 0 ? nb : 0, v1, v2},
                      st);

    // pass 2: A x per wave tile, and the tile's v1.x and v2.x
    const TileCfg c2 = cfg_of(SLOT_DGEMVT_P2, m, n);
    TileArgs a2 = targs(m, n, A, lda);
    a2.xr = x;
    a2.v1 = v1;
    a2.v2 = v2;
    a2.Prow = Prow;
    a2.Pcol = aux2;
    if (!launch_tile(kSlotNames[SLOT_DGEMVT_P2], OP_ROWDOT | OP_AUX, c2, a2, st))
        return unsupported(SLOT_DGEMVT_P2);
    const int64_t nt = n > 0 ? tile_ncols(c2, n) : 0;
    launch_finish_aux("finish", {fjob(Prow, nt, m, alpha, nullptr, w), aux2, m > 0 ? nt : 0, u1, u2},
                      st);
    return check_launch();
}

// ---- DGEMVT ------------------------------------------------------------------

bto_status bto_dgemvt(int64_t m, int64_t n, double alpha, double beta, const double *A,
                      int64_t lda, const double *y, const double *z, double *x, double *w,
                      void *ws, size_t ws_bytes_, bto_form form, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(check_form(form));
    BTO_TRY(check_matrix(m, n, A, lda, "A"));
    BTO_TRY(check_vec(y, m, "y"));
    BTO_TRY(check_vec(w, m, "w"));
    BTO_TRY(check_vec(z, n, "z"));
    BTO_TRY(check_vec(x, n, "x"));
    const size_t need_ws = ws_bytes(BTO_K_DGEMVT, m, n, form);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({mspan("A", A, m, n, lda, false), vspan("y", y, m, false),
                           vspan("z", z, n, false), vspan("x", x, n, true),
                           vspan("w", w, m, true), wspan(ws, need_ws)},
                          {}));

    Carve cv(ws);
    double *Prow = cv.take(max_ncols(n) * m);
    double *Pcol = cv.take(max_nbands(m) * n);
    if (form == BTO_FUSED) {
        BTO_TRY(gemv_t(SLOT_DGEMVT_P1, m, n, A, lda, y, beta, z, x, Pcol, st));
        BTO_TRY(gemv_n(SLOT_DGEMVT_P2, m, n, A, lda, x, alpha, w, Prow, st));
    } else {
        BTO_TRY(gemv_t(SLOT_GEMV_T, m, n, A, lda, y, beta, z, x, Pcol, st));
        BTO_TRY(gemv_n(SLOT_GEMV_N, m, n, A, lda, x, alpha, w, Prow, st));
    }
    return check_launch();
}

// ---- DGEMV and GESUMMV -------------------------------------------------------

namespace {

FinishLin flin(const double *P, int64_t np, int64_t len, double scale, const double *P2,
               int64_t np2, double scale2, const double *add, double add_scale, double *out)
{
    return FinishLin{fjob(P, np, len, scale, add, out), P2, np2, scale2, add_scale};
}

}  // namespace

bto_status bto_dgemv(int64_t m, int64_t n, double alpha, double beta, const double *A,
                     int64_t lda, const double *x, const double *y, double *z, void *ws,
                     size_t ws_bytes_, bto_form form, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(check_form(form));
    BTO_TRY(check_matrix(m, n, A, lda, "A"));
    BTO_TRY(check_vec(x, n, "x"));
    BTO_TRY(check_vec(y, m, "y"));
    BTO_TRY(check_vec(z, m, "z"));
    const size_t need_ws = ws_bytes(BTO_K_DGEMV, m, n, form);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({mspan("A", A, m, n, lda, false), vspan("x", x, n, false),
                           vspan("y", y, m, false), vspan("z", z, m, true),
                           wspan(ws, need_ws)},
                          {{"z", "y"}}));

    // one BLAS operation: both forms are the same sweep and reduction
    double *Prow = Carve(ws).take(max_ncols(n) * m);
    const TileCfg c = cfg_of(SLOT_GEMV_N, m, n);
    TileArgs a = targs(m, n, A, lda);
    a.xr = x;
    a.Prow = Prow;
    if (!launch_tile(kSlotNames[SLOT_GEMV_N], OP_ROWDOT, c, a, st))
        return unsupported(SLOT_GEMV_N);
    const int64_t np = n > 0 ? tile_ncols(c, n) : 0;
    launch_finish_lin("finish", flin(Prow, np, m, alpha, nullptr, 0, 0.0, y, beta, z), st);
    return check_launch();
}

bto_status bto_gesummv(int64_t m, int64_t n, double alpha, double beta, const double *A,
                       int64_t lda, const double *B, int64_t ldb, const double *x, double *y,
                       void *ws, size_t ws_bytes_, bto_form form, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(check_form(form));
    BTO_TRY(check_matrix(m, n, A, lda, "A"));
    BTO_TRY(check_matrix(m, n, B, ldb, "B"));
    BTO_TRY(check_vec(x, n, "x"));
    BTO_TRY(check_vec(y, m, "y"));
    const size_t need_ws = ws_bytes(BTO_K_GESUMMV, m, n, form);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({mspan("A", A, m, n, lda, false), mspan("B", B, m, n, ldb, false),
                           vspan("x", x, n, false), vspan("y", y, m, true),
                           wspan(ws, need_ws)},
                          {}));

    Carve cv(ws);
    const TileCfg c = cfg_of(SLOT_GEMV_N, m, n);
    const int64_t np = n > 0 ? tile_ncols(c, n) : 0;
    TileArgs a = targs(m, n, A, lda);
    a.xr = x;
    a.Prow = cv.take(max_ncols(n) * m);
    if (form == BTO_FUSED) {
        // both matrices' row dots, then one reduction that forms y
        TileArgs b = targs(m, n, B, ldb);
        b.xr = x;
        b.Prow = cv.take(max_ncols(n) * m);
        if (!launch_tile(kSlotNames[SLOT_GEMV_N], OP_ROWDOT, c, a, st) ||
            !launch_tile(kSlotNames[SLOT_GEMV_N], OP_ROWDOT, c, b, st))
            return unsupported(SLOT_GEMV_N);
        launch_finish_lin("finish", flin(a.Prow, np, m, alpha, b.Prow, np, beta, nullptr, 0.0, y),
                          st);
    } else {
        double *t = cv.take(m);
        // t = alpha A x, then y = beta B x + t
        if (!launch_tile(kSlotNames[SLOT_GEMV_N], OP_ROWDOT, c, a, st))
            return unsupported(SLOT_GEMV_N);
        launch_finish_lin("finish", flin(a.Prow, np, m, alpha, nullptr, 0, 0.0, nullptr, 0.0, t),
                          st);
        TileArgs b = targs(m, n, B, ldb);
        b.xr = x;
        b.Prow = a.Prow;
        if (!launch_tile(kSlotNames[SLOT_GEMV_N], OP_ROWDOT, c, b, st))
            return unsupported(SLOT_GEMV_N);
        launch_finish_lin("finish", flin(a.Prow, np, m, beta, nullptr, 0, 0.0, t, 1.0, y), st);
    }
    return check_launch();
}

// ---- one fused pass -----------------------------------------------------------

size_t bto_pass_workspace_bytes(int ops, int64_t m, int64_t n)
{
    if (m < 0 || n < 0 || (ops & ~31) != 0)
        return 0;
    if (ops & BTO_PASS_CHAIN)
        return ws_bytes(BTO_K_ATAX, m, n, BTO_FUSED);
    // the tile partials and the auxiliary dots of a contracted pass, or the
    // row-resident sweep's partials (row dots and column sums of A alone)
    const size_t tiles = ws_bytes(BTO_K_GEMVER_CONTRACTED, m, n, BTO_FUSED);
    const size_t both = ws_bytes(BTO_K_BICGK, m, n, BTO_FUSED);
    return tiles > both ? tiles : both;
}

bto_status bto_pass(const bto_pass_desc *d, void *ws, size_t ws_bytes_, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(need(d != nullptr, "pass descriptor is NULL"));
    const int ops = d->ops;
    const bool R = ops & BTO_PASS_ROWDOT, C = ops & BTO_PASS_COLSUM;
    const bool S = ops & BTO_PASS_STORE, K = ops & BTO_PASS_CONTRACT, H = ops & BTO_PASS_CHAIN;
    const int64_t m = d->m, n = d->n;
    BTO_TRY(need((ops & ~31) == 0, "unknown pass operation"));
    BTO_TRY(need(R || C || S, "the pass computes nothing"));
    BTO_TRY(need(!(S && K), "STORE and CONTRACT exclude each other"));
    BTO_TRY(need(!K || R || C, "CONTRACT needs ROWDOT or COLSUM"));
    BTO_TRY(need(!H || (R && C && !S && !K), "CHAIN takes ROWDOT | COLSUM over A alone"));
    BTO_TRY(check_matrix(m, n, d->A, d->lda, "A"));
    if (H) {
        BTO_TRY(need(!d->row_out && !d->y && !d->col_add && !d->row_add,
                     "CHAIN takes no row output, column weights or adds"));
        return atax_scaled(BTO_K_ATAX, m, n, d->col_scale, d->A, d->lda, d->x, d->col_out, ws,
                           ws_bytes_, BTO_FUSED, st);
    }
    if (K && R && C)
        return fail(BTO_ERR_UNSUPPORTED, "a contracted pass takes row dots or column sums, not both");
    if (K && ((R && d->row_add && d->row_add_scale != 1.0) ||
              (C && d->col_add && d->col_add_scale != 1.0)))
        return fail(BTO_ERR_UNSUPPORTED, "a contracted pass adds its vector with scale 1");
    if (S)
        BTO_TRY(check_matrix(m, n, d->B, d->ldb, "B"));
    if (S || K) {
        BTO_TRY(check_vec(d->u1, m, "u1"));
        BTO_TRY(check_vec(d->v1, n, "v1"));
        BTO_TRY(check_vec(d->u2, m, "u2"));
        BTO_TRY(check_vec(d->v2, n, "v2"));
    }
    if (R) {
        BTO_TRY(check_vec(d->x, n, "x"));
        BTO_TRY(check_vec(d->row_out, m, "row_out"));
    }
    if (C) {
        BTO_TRY(check_vec(d->y, m, "y"));
        BTO_TRY(check_vec(d->col_out, n, "col_out"));
    }
    const size_t need_ws = bto_pass_workspace_bytes(ops, m, n);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    const bool UV = S || K;
    // operands the pass does not use (or leaves NULL) take part as empty spans
    auto vs = [](const char *nm, const void *p, int64_t k, bool out, bool used) {
        return vspan(nm, p, used && p ? k : 0, out);
    };
    BTO_TRY(check_aliases(
        {mspan("A", d->A, m, n, d->lda, false), mspan("B", d->B, S ? m : 0, n, d->ldb, true),
         vs("u1", d->u1, m, false, UV), vs("v1", d->v1, n, false, UV),
         vs("u2", d->u2, m, false, UV), vs("v2", d->v2, n, false, UV),
         vs("x", d->x, n, false, R), vs("y", d->y, m, false, C),
         vs("row_out", d->row_out, m, true, R), vs("row_add", d->row_add, m, false, R),
         vs("col_out", d->col_out, n, true, C), vs("col_add", d->col_add, n, false, C),
         wspan(ws, need_ws)},
        {{"B", "A"}, {"row_out", "row_add"}, {"col_out", "col_add"}}));

    if (R && C && !S && !K && d->row_scale == 1.0 && !d->row_add) {
        // BiCGK's pass: the row-resident sweep when tuning selects it, as in
        // bto_bicgk (it writes the row dots whole, unscaled)
        const int bt = get_bicgk_rowres_threads(size_bucket(m, n));
        const int64_t G = bt ? rowres_parts(m, n, bt, true) : 0;
        if (G > 0) {
            double *P = Carve(ws).take(G * n);
            launch_bicgk_rowres(m, n, d->A, d->lda, d->x, d->y, d->row_out, P, bt, st);
            launch_finish_lin("finish", flin(P, G, n, d->col_scale, nullptr, 0, 0.0, d->col_add,
                                             d->col_add_scale, d->col_out),
                              st);
            return check_launch();
        }
    }
    Carve cv(ws);
    double *Prow = cv.take(max_ncols(n) * m);
    double *Pcol = cv.take(max_nbands(m) * n);
    double *aux1 = cv.take(2 * max_nbands(m));   // u1.y, u2.y per row band
    double *aux2 = cv.take(2 * max_ncols(n));    // v1.x, v2.x per wave tile
    TileArgs a = targs(m, n, d->A, d->lda);
    int tops = 0;
    if (UV) {
        a.u1 = d->u1;
        a.v1 = d->v1;
        a.u2 = d->u2;
        a.v2 = d->v2;
    }
    if (S) {
        a.B = d->B;
        a.ldb = d->ldb;
        tops |= OP_UPD1 | OP_UPD2;
    }
    if (R) {
        a.xr = d->x;
        a.Prow = Prow;
        tops |= OP_ROWDOT;
    }
    if (C) {
        a.yc = d->y;
        a.Pcol = Pcol;
        tops |= OP_COLSUM;
    }
    if (K) {
        tops |= OP_AUX;
        if (C)
            a.Prow = aux1;
        else
            a.Pcol = aux2;
    }
    // the slot whose tuned configuration serves this operation mix
    Slot slot;
    if (S)
        slot = SLOT_GEMVER_P1;
    else if (K)
        slot = C ? SLOT_DGEMVT_P1 : SLOT_DGEMVT_P2;
    else if (R && C)
        slot = SLOT_BICGK_FUSED;
    else
        slot = R ? SLOT_GEMV_N : SLOT_GEMV_T;
    const TileCfg c = cfg_of(slot, m, n);
    if (!launch_tile(kSlotNames[slot], tops, c, a, st))
        return unsupported(slot);
    if (R) {
        const int64_t np = n > 0 ? tile_ncols(c, n) : 0;
        if (K)
            launch_finish_aux("finish",
                              {fjob(Prow, np, m, d->row_scale, d->row_add, d->row_out), aux2,
                               m > 0 ? np : 0, d->u1, d->u2},
                              st);
        else
            launch_finish_lin("finish", flin(Prow, np, m, d->row_scale, nullptr, 0, 0.0, d->row_add,
                                             d->row_add_scale, d->row_out),
                              st);
    }
    if (C) {
        const int64_t nb = m > 0 ? tile_nbands(c, m) : 0;
        if (K)
            launch_finish_aux("finish",
                              {fjob(Pcol, nb, n, d->col_scale, d->col_add, d->col_out), aux1,
                               n > 0 ? nb : 0, d->v1, d->v2},
                              st);
        else
            launch_finish_lin("finish", flin(Pcol, nb, n, d->col_scale, nullptr, 0, 0.0, d->col_add,
                                             d->col_add_scale, d->col_out),
                              st);
    }
    return check_launch();
}

// ---- AXPYDOT -----------------------------------------------------------------

bto_status bto_axpydot(int64_t n, double alpha, const double *w, const double *v,
                       const double *u, double *z, double *r, void *ws, size_t ws_bytes_,
                       bto_form form, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(check_form(form));
    BTO_TRY(need(n >= 0, "negative size"));
    BTO_TRY(check_vec(w, n, "w"));
    BTO_TRY(check_vec(v, n, "v"));
    BTO_TRY(check_vec(u, n, "u"));
    BTO_TRY(check_vec(z, n, "z"));
    BTO_TRY(check_vec(r, 1, "r"));
    const size_t need_ws = ws_bytes(BTO_K_AXPYDOT, 0, n, form);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({vspan("w", w, n, false), vspan("v", v, n, false),
                           vspan("u", u, n, false), vspan("z", z, n, true),
                           vspan("r", r, 1, true), wspan(ws, need_ws)},
                          {{"z", "w"}}));

    double *parts = Carve(ws).take(dot_parts(n));
    if (form == BTO_FUSED) {
        launch_dot(true, n, alpha, w, v, u, z, parts, r, st);
    } else {
        launch_ew(EW_AXMY, n, w, v, nullptr, alpha, 0.0, z, st);  // z = w - alpha v
        launch_dot(false, n, 0.0, z, nullptr, u, nullptr, parts, r, st);
    }
    return check_launch();
}

// ---- WAXPBY ------------------------------------------------------------------

bto_status bto_waxpby(int64_t n, double alpha, const double *x, double beta, const double *y,
                      double *w, void *ws, size_t ws_bytes_, bto_form form, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(check_form(form));
    BTO_TRY(need(n >= 0, "negative size"));
    BTO_TRY(check_vec(x, n, "x"));
    BTO_TRY(check_vec(y, n, "y"));
    BTO_TRY(check_vec(w, n, "w"));
    const size_t need_ws = ws_bytes(BTO_K_WAXPBY, 0, n, form);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({vspan("x", x, n, false), vspan("y", y, n, false),
                           vspan("w", w, n, true), wspan(ws, need_ws)},
                          {{"w", "x"}, {"w", "y"}}));
    if (form == BTO_FUSED) {
        launch_ew(EW_WAXPBY, n, x, y, nullptr, alpha, beta, w, st);
    } else {
        double *t = Carve(ws).take(n);
        launch_ew(EW_SCAL, n, x, nullptr, nullptr, alpha, 0.0, t, st);  // t = alpha x
        launch_ew(EW_AXPY, n, t, y, nullptr, beta, 0.0, w, st);         // w = t + beta y
    }
    return check_launch();
}

// ---- DOT -----------------------------------------------------------------------

size_t bto_dot_workspace_bytes(int64_t n) { return n < 0 ? 0 : round256((size_t)dot_parts(n) * 8); }

bto_status bto_dot(int64_t n, const double *x, const double *y, double *r, void *ws,
                   size_t ws_bytes_, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(need(n >= 0, "negative size"));
    BTO_TRY(check_vec(x, n, "x"));
    BTO_TRY(check_vec(y, n, "y"));
    BTO_TRY(check_vec(r, 1, "r"));
    const size_t need_ws = bto_dot_workspace_bytes(n);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({vspan("x", x, n, false), vspan("y", y, n, false),
                           vspan("r", r, 1, true), wspan(ws, need_ws)},
                          {}));
    double *parts = Carve(ws).take(dot_parts(n));
    launch_dot(false, n, 0.0, x, nullptr, y, nullptr, parts, r, st);
    return check_launch();
}

// ---- linear combination --------------------------------------------------------

bto_status bto_lincomb(int64_t n, int count, const double *const *x, const double *coef,
                       double *out, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(need(n >= 0, "negative size"));
    BTO_TRY(need(count >= 1 && count <= kMaxLin, "count must be 1 to 8"));
    BTO_TRY(need(x != nullptr && coef != nullptr, "x and coef are host arrays of count entries"));
    static const char *names[kMaxLin] = {"x0", "x1", "x2", "x3", "x4", "x5", "x6", "x7"};
    LinArgs a{};
    std::vector<Span> spans;
    std::vector<AllowedAlias> ok;
    for (int k = 0; k < count; ++k) {
        BTO_TRY(check_vec(x[k], n, names[k]));
        a.x[k] = x[k];
        a.c[k] = coef[k];
        spans.push_back(vspan(names[k], x[k], n, false));
        ok.push_back({"out", names[k]});
    }
    BTO_TRY(check_vec(out, n, "out"));
    a.out = out;
    spans.push_back(vspan("out", out, n, true));
    BTO_TRY(check_aliases(spans, ok));
    launch_lincomb(n, count, a, st);
    return check_launch();
}

// ---- VADD --------------------------------------------------------------------

bto_status bto_vadd(int64_t n, const double *w, const double *y, const double *z, double *x,
                    void *ws, size_t ws_bytes_, bto_form form, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(check_form(form));
    BTO_TRY(need(n >= 0, "negative size"));
    BTO_TRY(check_vec(w, n, "w"));
    BTO_TRY(check_vec(y, n, "y"));
    BTO_TRY(check_vec(z, n, "z"));
    BTO_TRY(check_vec(x, n, "x"));
    const size_t need_ws = ws_bytes(BTO_K_VADD, 0, n, form);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({vspan("w", w, n, false), vspan("y", y, n, false),
                           vspan("z", z, n, false), vspan("x", x, n, true), wspan(ws, need_ws)},
                          {{"x", "w"}, {"x", "y"}, {"x", "z"}}));
    if (form == BTO_FUSED) {
        launch_ew(EW_VADD3, n, w, y, z, 0.0, 0.0, x, st);
    } else {
        double *t = Carve(ws).take(n);
        launch_ew(EW_ADD2, n, w, y, nullptr, 0.0, 0.0, t, st);  // t = w + y
        launch_ew(EW_ADD2, n, t, z, nullptr, 0.0, 0.0, x, st);  // x = t + z
    }
    return check_launch();
}

// ---- timing ------------------------------------------------------------------

bto_status bto_timing_enable(int enable)
{
    std::lock_guard<std::mutex> g(g_tmu);
    g_tenabled = enable != 0;
    return BTO_SUCCESS;
}

bto_status bto_timing_only(const char *name)
{
    std::lock_guard<std::mutex> g(g_tmu);
    g_tonly = name ? name : "";
    return BTO_SUCCESS;
}

bto_status bto_timing_collect(void)
{
    std::lock_guard<std::mutex> g(g_tmu);
    bto_status st = BTO_SUCCESS;
    for (const TimingRec &r : g_recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            st = fail(BTO_ERR_HIP, "event timing failed");
        } else {
            g_tms[r.name] += ms;
            g_tcount[r.name] += 1;
        }
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    return st;
}

int bto_timing_count(void)
{
    std::lock_guard<std::mutex> g(g_tmu);
    return (int)g_tnames.size();
}

bto_status bto_timing_get(int idx, const char **name, int64_t *launches, double *total_ms)
{
    std::lock_guard<std::mutex> g(g_tmu);
    if (idx < 0 || idx >= (int)g_tnames.size())
        return fail(BTO_ERR_INVALID_ARG, "timing index out of range");
    if (name) *name = g_tnames[idx].c_str();
    if (launches) *launches = g_tcount[idx];
    if (total_ms) *total_ms = g_tms[idx];
    return BTO_SUCCESS;
}

void bto_timing_reset(void)
{
    std::lock_guard<std::mutex> g(g_tmu);
    for (const TimingRec &r : g_recs) {
        g_pool.push_back(r.a);
        g_pool.push_back(r.b);
    }
    g_recs.clear();
    g_tnames.clear();
    g_tms.clear();
    g_tcount.clear();
}

// ---- tuning --------------------------------------------------------------------

// Slot SLOT_COUNT is the row-resident ATAX sweep: its "shape" is the
// workgroup size (256, 512 or 1024 threads); rb and rev are 0.  Slot
// SLOT_COUNT + 1 is the row-resident BiCGK sweep, the same with shape 0
// meaning "use the tile kernel of slot bicgk_fused instead".
constexpr int kRowresSlot = SLOT_COUNT;
constexpr int kBicgkRowresSlot = SLOT_COUNT + 1;

int bto_tune_slot_count(void) { return SLOT_COUNT + 2; }

const char *bto_tune_slot_name(int slot)
{
    if (slot == kRowresSlot)
        return "atax_rowres";
    if (slot == kBicgkRowresSlot)
        return "bicgk_rowres";
    return (slot >= 0 && slot < SLOT_COUNT) ? kSlotNames[slot] : "";
}

int bto_tune_slot_ops(int slot)
{
    return (slot >= 0 && slot < SLOT_COUNT) ? kSlotOps[slot] : 0;
}

// The size bucket a tuning call addresses: that of a problem of max(m, n)
// = size, or every bucket for size 0 (get: the 16384 bucket).
static bool tune_buckets(int64_t size, int &lo, int &hi)
{
    if (size < 0)
        return false;
    if (size == 0) {
        lo = 0;
        hi = kSizeBuckets - 1;
    } else {
        lo = hi = size_bucket(size, size);
    }
    return true;
}

bto_status bto_tune_get_for(int slot, int64_t size, int *shape, int *rb, int *rev)
{
    t_error.clear();
    int lo, hi;
    if (!tune_buckets(size, lo, hi))
        return fail(BTO_ERR_INVALID_ARG, "negative size");
    const int b = size == 0 ? size_bucket(16384, 16384) : lo;
    if (slot == kRowresSlot || slot == kBicgkRowresSlot) {
        std::lock_guard<std::mutex> g(g_cfg_mu);
        if (shape)
            *shape = slot == kRowresSlot ? get_rowres_threads(b) : get_bicgk_rowres_threads(b);
        if (rb) *rb = 0;
        if (rev) *rev = 0;
        return BTO_SUCCESS;
    }
    if (slot < 0 || slot >= SLOT_COUNT)
        return fail(BTO_ERR_INVALID_ARG, "slot out of range");
    std::lock_guard<std::mutex> g(g_cfg_mu);
    const TileCfg c = g_cfg[slot][b];
    if (shape) *shape = c.shape;
    if (rb) *rb = c.rb;
    if (rev) *rev = c.rev;
    return BTO_SUCCESS;
}

bto_status bto_tune_set_for(int slot, int64_t size, int shape, int rb, int rev)
{
    t_error.clear();
    int lo, hi;
    if (!tune_buckets(size, lo, hi))
        return fail(BTO_ERR_INVALID_ARG, "negative size");
    if (slot == kRowresSlot || slot == kBicgkRowresSlot) {
        const bool atax = slot == kRowresSlot;
        const bool ok_threads = shape == 256 || shape == 512 || shape == 1024 ||
                                (!atax && shape == 0);
        if (rb != 0 || rev != 0 || !ok_threads)
            return fail(BTO_ERR_INVALID_ARG, atax ? "atax_rowres takes (256|512|1024, 0, 0)"
                                                  : "bicgk_rowres takes (0|256|512|1024, 0, 0)");
        std::lock_guard<std::mutex> g(g_cfg_mu);
        for (int b = lo; b <= hi; ++b) {
            if (atax) set_rowres_threads(b, shape);
            else set_bicgk_rowres_threads(b, shape);
        }
        return BTO_SUCCESS;
    }
    if (slot < 0 || slot >= SLOT_COUNT)
        return fail(BTO_ERR_INVALID_ARG, "slot out of range");
    TileCfg c{shape, rb, rev};
    if (!tile_cfg_supported(kSlotOps[slot], c))
        return fail(BTO_ERR_INVALID_ARG, "tile configuration not supported for this slot");
    std::lock_guard<std::mutex> g(g_cfg_mu);
    for (int b = lo; b <= hi; ++b)
        g_cfg[slot][b] = c;
    return BTO_SUCCESS;
}

bto_status bto_tune_get(int slot, int *shape, int *rb, int *rev)
{
    return bto_tune_get_for(slot, 0, shape, rb, rev);
}

bto_status bto_tune_set(int slot, int shape, int rb, int rev)
{
    return bto_tune_set_for(slot, 0, shape, rb, rev);
}

int bto_tune_bucket_count(void) { return kSizeBuckets; }

int bto_tune_bucket(int64_t size) { return size < 0 ? -1 : size_bucket(size, size); }

bto_status bto_tune_shape(int shape, int *kv, int *depth, int *waves_across, int *waves_down)
{
    t_error.clear();
    if (shape < 0 || shape >= kTileShapes)
        return fail(BTO_ERR_INVALID_ARG, "shape out of range");
    int info[4];
    tile_shape_info(shape, info);
    if (kv) *kv = info[0];
    if (depth) *depth = info[1];
    if (waves_across) *waves_across = info[2];
    if (waves_down) *waves_down = info[3];
    return BTO_SUCCESS;
}

// ---- probes --------------------------------------------------------------------

bto_status bto_probe_copy(const double *src, double *dst, int64_t n, hipStream_t st)
{
    t_error.clear();
    BTO_TRY(need(n >= 0, "negative size"));
    BTO_TRY(check_vec(src, n, "src"));
    BTO_TRY(check_vec(dst, n, "dst"));
    BTO_TRY(check_aliases({vspan("src", src, n, false), vspan("dst", dst, n, true)}, {}));
    launch_copy(n, src, dst, st);
    return check_launch();
}

size_t bto_probe_read_workspace_bytes(int64_t n)
{
    return n < 0 ? 0 : round256((size_t)read_parts(n) * 8);
}

bto_status bto_probe_read(const double *src, int64_t n, double *out, void *ws, size_t ws_bytes_,
                          hipStream_t st)
{
    t_error.clear();
    BTO_TRY(need(n >= 0, "negative size"));
    BTO_TRY(check_vec(src, n, "src"));
    BTO_TRY(check_vec(out, 1, "out"));
    const size_t need_ws = bto_probe_read_workspace_bytes(n);
    BTO_TRY(check_ws(ws, ws_bytes_, need_ws));
    BTO_TRY(check_aliases({vspan("src", src, n, false), vspan("out", out, 1, true),
                           wspan(ws, need_ws)},
                          {}));
    if (n == 0) {
        // an empty sum is 0: the finish alone writes it
        launch_read(0, src, static_cast<double *>(ws), out, st);
        return check_launch();
    }
    launch_read(n, src, static_cast<double *>(ws), out, st);
    return check_launch();
}

bto_status bto_probe_triad(double *a, const double *b, const double *c, double s, int64_t n,
                           hipStream_t st)
{
    t_error.clear();
    BTO_TRY(need(n >= 0, "negative size"));
    BTO_TRY(check_vec(a, n, "a"));
    BTO_TRY(check_vec(b, n, "b"));
    BTO_TRY(check_vec(c, n, "c"));
    BTO_TRY(check_aliases({vspan("a", a, n, true), vspan("b", b, n, false), vspan("c", c, n, false)}, {}));
    launch_triad(n, a, b, c, s, st);
    return check_launch();
}

}  // extern "C"

// ---- batched execution ---------------------------------------------------------

struct bto_batch_plan {
    int capacity = 0;               // instances per refill
    int unit_capacity = 0;
    int count = 0;
    BatchItem *d_items = nullptr;
    BatchUnit *d_units = nullptr;
    int *d_meta = nullptr;          // kMetaInts control ints
    int *d_sync = nullptr;          // two per instance: tiles done, x ready
    double *d_scratch = nullptr;
    int64_t scratch_cap = 0;        // doubles
    int64_t split_bytes = kBatchSplitBytes;   // <= 0: never split
    // pinned staging of {items, units, meta} for asynchronous refills, and
    // the event that marks when the last refill has been read
    char *h_stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t staged = nullptr;
    int threads = 256;
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
};

namespace {

struct BSpan {
    uintptr_t lo, hi;
    int inst;
    bool out;
    bool a_or_b;   // the instance's A or B (exact B == A alias allowed)
};

// Rows per tile of an instance, or 0 when it runs whole: fused instances
// whose matrix exceeds split_bytes are cut into row tiles of about that
// size (at least 8 rows, at most kBatchMaxTiles tiles).
int64_t tile_rows_for(int kind, int form, int64_t m, int64_t n, int64_t split_bytes)
{
    (void)kind;
    if (form != BTO_FUSED || split_bytes <= 0 || m < 16 || n <= 0)
        return 0;
    if ((double)m * (double)n * 8.0 <= (double)split_bytes)
        return 0;
    int64_t r = ceil_div(split_bytes, 8 * n);
    r = r < 8 ? 8 : r;
    const int64_t rmin = ceil_div(m, (int64_t)kBatchMaxTiles);
    r = r < rmin ? rmin : r;
    r = ceil_div(r, (int64_t)8) * 8;
    return ceil_div(m, r) > 1 ? r : 0;
}

int64_t part_stride(int64_t n) { return ceil_div(n, (int64_t)32) * 32; }

bto_status batch_check_one(const bto_batch_desc &d, int idx, std::vector<BSpan> &spans,
                           BatchItem &it, int64_t &scratch, int64_t split_bytes)
{
    const std::string where = "instance " + std::to_string(idx) + ": ";
    auto bad = [&](bto_status st, const std::string &msg) { return fail(st, where + msg); };
    if (d.kind != BTO_K_GEMVER && d.kind != BTO_K_BICGK && d.kind != BTO_K_ATAX)
        return bad(BTO_ERR_UNSUPPORTED, "kind must be GEMVER, BICGK or ATAX");
    if (d.form != BTO_FUSED && d.form != BTO_UNFUSED)
        return bad(BTO_ERR_INVALID_ARG, "unknown form");
    const int64_t m = d.m, n = d.n;
    if (m < 0 || n < 0)
        return bad(BTO_ERR_INVALID_ARG, "negative size");
    if (n > batch_max_n())
        return bad(BTO_ERR_UNSUPPORTED, "more columns than a batched instance may have");
    // rows start 16-byte aligned: an even leading dimension (unused with one row)
    if (d.lda < (n > 1 ? n : 1) || ((d.lda & 1) && m > 1))
        return bad(BTO_ERR_INVALID_ARG, "lda must be even and at least max(1, n)");
    const bool empty = m == 0 || n == 0;
    if (!empty && (d.A == nullptr || !aligned16(d.A)))
        return bad(BTO_ERR_INVALID_ARG, "A must be a 16-byte aligned device pointer");
    int nin = 0, nout = 0;
    int64_t in_len[6] = {0}, out_len[2] = {0};
    if (d.kind == BTO_K_GEMVER) {
        nin = 6; nout = 2;
        const int64_t il[6] = {m, n, m, n, m, n};
        std::copy(il, il + 6, in_len);
        out_len[0] = n; out_len[1] = m;
        if (d.ldb < (n > 1 ? n : 1) || ((d.ldb & 1) && m > 1))
            return bad(BTO_ERR_INVALID_ARG, "ldb must be even and at least max(1, n)");
        if (!empty && (d.B == nullptr || !aligned16(d.B)))
            return bad(BTO_ERR_INVALID_ARG, "B must be a 16-byte aligned device pointer");
        if (d.B == d.A && d.ldb != d.lda && !empty)
            return bad(BTO_ERR_ALIAS, "B == A requires ldb == lda");
    } else if (d.kind == BTO_K_BICGK) {
        nin = 2; nout = 2;
        in_len[0] = n; in_len[1] = m;
        out_len[0] = m; out_len[1] = n;
    } else {
        nin = 1; nout = 1;
        in_len[0] = n;
        out_len[0] = n;
    }
    for (int k = 0; k < nin; ++k) {
        if (in_len[k] > 0 && d.in[k] == nullptr)
            return bad(BTO_ERR_INVALID_ARG, "input vector " + std::to_string(k) + " is NULL");
        if (in_len[k] > 1 && !aligned16(d.in[k]))
            return bad(BTO_ERR_INVALID_ARG, "input vector " + std::to_string(k) +
                                                " must be 16-byte aligned");
    }
    for (int k = 0; k < nout; ++k) {
        if (out_len[k] > 0 && d.out[k] == nullptr)
            return bad(BTO_ERR_INVALID_ARG, "output vector " + std::to_string(k) + " is NULL");
        if (out_len[k] > 1 && !aligned16(d.out[k]))
            return bad(BTO_ERR_INVALID_ARG, "output vector " + std::to_string(k) +
                                                " must be 16-byte aligned");
    }

    auto add = [&](const void *p, int64_t bytes, bool out, bool ab) {
        if (bytes > 0) {
            uintptr_t lo = reinterpret_cast<uintptr_t>(p);
            spans.push_back({lo, lo + (uintptr_t)bytes, idx, out, ab});
        }
    };
    if (!empty) {
        add(d.A, ((m - 1) * d.lda + n) * 8, false, true);
        if (d.kind == BTO_K_GEMVER)
            add(d.B, ((m - 1) * d.ldb + n) * 8, true, true);
    }
    for (int k = 0; k < nin; ++k)
        add(d.in[k], in_len[k] * 8, false, false);
    for (int k = 0; k < nout; ++k)
        add(d.out[k], out_len[k] * 8, true, false);

    it = BatchItem{};
    it.kind = d.kind;
    it.form = d.form;
    it.m = m;
    it.n = n;
    it.lda = d.lda;
    it.ldb = d.kind == BTO_K_GEMVER ? d.ldb : d.lda;
    it.alpha = d.alpha;
    it.beta = d.beta;
    it.A = d.A;
    it.B = d.B;
    for (int k = 0; k < 6; ++k) it.vec[k] = k < nin ? d.in[k] : nullptr;
    for (int k = 0; k < 2; ++k) it.out[k] = k < nout ? d.out[k] : nullptr;
    it.scratch_off = 0;
    it.part_off = 0;
    it.ntiles = 1;
    it.tile_rows = m;
    if (d.kind == BTO_K_ATAX && d.form == BTO_UNFUSED) {
        it.scratch_off = scratch;
        scratch += ceil_div(m, (int64_t)32) * 32;   // 256-byte steps
    }
    const int64_t r = tile_rows_for(d.kind, d.form, m, n, split_bytes);
    if (r > 0) {
        it.tile_rows = r;
        it.ntiles = (int32_t)ceil_div(m, r);
        it.part_off = scratch;
        scratch += it.ntiles * part_stride(n);
    }
    return BTO_SUCCESS;
}

// No output of any instance may overlap another operand, except an
// instance's B exactly equal to its own A.
bto_status batch_check_overlaps(std::vector<BSpan> &spans)
{
    std::vector<BSpan> outs;
    for (const BSpan &s : spans)
        if (s.out) outs.push_back(s);
    std::sort(outs.begin(), outs.end(), [](const BSpan &a, const BSpan &b) { return a.lo < b.lo; });
    for (size_t i = 1; i < outs.size(); ++i)
        if (outs[i].lo < outs[i - 1].hi)
            return fail(BTO_ERR_ALIAS, "outputs of instances " + std::to_string(outs[i - 1].inst) +
                                           " and " + std::to_string(outs[i].inst) + " overlap");
    for (const BSpan &s : spans) {
        if (s.out)
            continue;
        // the output with the largest start below s.hi is the only candidate
        auto it = std::lower_bound(outs.begin(), outs.end(), s.hi,
                                   [](const BSpan &o, uintptr_t v) { return o.lo < v; });
        if (it == outs.begin())
            continue;
        const BSpan &o = *(it - 1);
        if (o.hi <= s.lo)
            continue;
        const bool exact_ab = o.inst == s.inst && o.a_or_b && s.a_or_b && o.lo == s.lo &&
                              o.hi == s.hi;
        if (!exact_ab)
            return fail(BTO_ERR_ALIAS, "an output of instance " + std::to_string(o.inst) +
                                           " overlaps an input of instance " +
                                           std::to_string(s.inst));
    }
    return BTO_SUCCESS;
}

// Matrix passes of a unit times its rows and columns: the work used to
// order the queue (largest first).
double unit_cost(const BatchItem &it, const BatchUnit &u)
{
    const double rows = (double)(u.r1 - u.r0), cols = (double)it.n;
    double passes;
    if (it.kind == BTO_K_GEMVER)
        passes = u.phase == 0 ? (it.form == BTO_FUSED ? 3.0 : 6.0) : (u.phase == 1 ? 2.0 : 1.0);
    else
        passes = u.phase == 0 && it.form == BTO_UNFUSED ? 2.0 : 1.0;
    return passes * rows * cols + rows + cols;
}

void plan_free(bto_batch_plan *p)
{
    if (!p) return;
    if (p->staged) (void)hipEventSynchronize(p->staged);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->d_items) (void)hipFree(p->d_items);
    if (p->d_units) (void)hipFree(p->d_units);
    if (p->d_meta) (void)hipFree(p->d_meta);
    if (p->d_sync) (void)hipFree(p->d_sync);
    if (p->d_scratch) (void)hipFree(p->d_scratch);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    if (p->staged) (void)hipEventDestroy(p->staged);
    delete p;
}

// Validate `descs` and build the device table image: the items and the
// queue of units.  Whole instances and first-sweep tiles come first,
// largest first; GEMVER's second-sweep tiles follow all of them, so a
// workgroup that takes one only waits for tiles other running workgroups
// already hold.
bto_status plan_image(const bto_batch_desc *descs, int count, int64_t split_bytes,
                      std::vector<BatchItem> &items, std::vector<BatchUnit> &units,
                      int64_t &scratch)
{
    if (count < 0 || (count > 0 && !descs))
        return fail(BTO_ERR_INVALID_ARG, "bad instance list");
    std::vector<BSpan> spans;
    items.assign((size_t)count, BatchItem{});
    scratch = 0;
    for (int i = 0; i < count; ++i)
        BTO_TRY(batch_check_one(descs[i], i, spans, items[i], scratch, split_bytes));
    BTO_TRY(batch_check_overlaps(spans));
    std::vector<BatchUnit> first, second;
    for (int i = 0; i < count; ++i) {
        const BatchItem &it = items[i];
        if (it.ntiles <= 1) {
            first.push_back({i, 0, 0, it.m});
            continue;
        }
        for (int t = 0; t < it.ntiles; ++t) {
            const int64_t r0 = t * it.tile_rows;
            const int64_t r1 = std::min(it.m, r0 + it.tile_rows);
            first.push_back({i, 1, r0, r1});
            if (it.kind == BTO_K_GEMVER)
                second.push_back({i, 2, r0, r1});
        }
    }
    auto by_cost = [&](std::vector<BatchUnit> &v) {
        std::vector<double> cost(v.size());
        std::vector<size_t> idx(v.size());
        for (size_t k = 0; k < v.size(); ++k) {
            cost[k] = unit_cost(items[v[k].item], v[k]);
            idx[k] = k;
        }
        std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
        std::vector<BatchUnit> out(v.size());
        for (size_t k = 0; k < v.size(); ++k) out[k] = v[idx[k]];
        v.swap(out);
    };
    by_cost(first);
    by_cost(second);
    units = first;
    units.insert(units.end(), second.begin(), second.end());
    return BTO_SUCCESS;
}

// the most units one instance can make
constexpr int kUnitsPerItem = 2 * kBatchMaxTiles;

size_t stage_size(int capacity, int unit_capacity)
{
    return round256(sizeof(BatchItem) * (size_t)capacity) +
           round256(sizeof(BatchUnit) * (size_t)unit_capacity) + 256;
}

}  // namespace

static bto_status plan_alloc(int capacity, int unit_capacity, int64_t scratch_doubles,
                             const bto_batch_config *config, bto_batch_plan **out)
{
    bto_batch_config cfg{kBatchDefaultThreads, 0, 0, 0};
    if (config) {
        cfg = *config;
        if (cfg.threads == 0) cfg.threads = kBatchDefaultThreads;
    }
    if (!batch_threads_supported(cfg.threads))
        return fail(BTO_ERR_INVALID_ARG, "threads must be 256 or 512");
    if (cfg.wgs_per_cu < 0 || cfg.wgs_per_cu > 8)
        return fail(BTO_ERR_INVALID_ARG, "wgs_per_cu must be 0 (the default) to 8");
    if (capacity < 0 || unit_capacity < 0 || scratch_doubles < 0)
        return fail(BTO_ERR_INVALID_ARG, "negative capacity");
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(BTO_ERR_HIP, "no device");

    bto_batch_plan *p = new bto_batch_plan();
    p->capacity = capacity;
    p->unit_capacity = unit_capacity;
    p->threads = cfg.threads;
    p->split_bytes = cfg.split_bytes == 0 ? kBatchSplitBytes : cfg.split_bytes;
    // 0: as many workgroups as can be resident at once
    const int per_cu = cfg.wgs_per_cu ? cfg.wgs_per_cu : kBatchDefaultWgsPerCu;
    p->grid = cus * per_cu;
    p->scratch_cap = scratch_doubles;
    p->stage_bytes = stage_size(capacity, unit_capacity);
    auto hip_fail = [&](const char *what) {
        plan_free(p);
        return fail(BTO_ERR_HIP, std::string(what) + ": " + hipGetErrorString(hipGetLastError()));
    };
    if (hipMalloc(&p->d_meta, 256) != hipSuccess || hipMemset(p->d_meta, 0, 256) != hipSuccess)
        return hip_fail("hipMalloc");
    const size_t cap1 = capacity > 0 ? (size_t)capacity : 1;
    const size_t ucap1 = unit_capacity > 0 ? (size_t)unit_capacity : 1;
    if (hipMalloc(&p->d_items, sizeof(BatchItem) * cap1) != hipSuccess ||
        hipMalloc(&p->d_units, sizeof(BatchUnit) * ucap1) != hipSuccess ||
        hipMalloc(&p->d_sync, 2 * sizeof(int) * cap1) != hipSuccess ||
        hipMemset(p->d_sync, 0, 2 * sizeof(int) * cap1) != hipSuccess)
        return hip_fail("hipMalloc");
    if (scratch_doubles > 0 &&
        hipMalloc(&p->d_scratch, sizeof(double) * (size_t)scratch_doubles) != hipSuccess)
        return hip_fail("hipMalloc");
    if (hipHostMalloc((void **)&p->h_stage, p->stage_bytes, hipHostMallocDefault) != hipSuccess)
        return hip_fail("hipHostMalloc");
    if (hipEventCreateWithFlags(&p->staged, hipEventDisableTiming) != hipSuccess)
        return hip_fail("hipEventCreate");
    if (cfg.use_graph) {
        if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
            return hip_fail("hipStreamCreate");
        if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return hip_fail("hipStreamBeginCapture");
        t_capturing = true;
        launch_batch(p->d_items, p->d_units, p->d_meta, p->d_sync, p->d_scratch, p->threads,
                     p->grid, p->cap);
        t_capturing = false;
        if (hipStreamEndCapture(p->cap, &p->graph) != hipSuccess)
            return hip_fail("hipStreamEndCapture");
        if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
            return hip_fail("hipGraphInstantiate");
    }
    *out = p;
    return BTO_SUCCESS;
}

// Copy a validated table image into the plan on `stream` (asynchronously,
// through the plan's pinned staging, after the previous refill was read).
static bto_status plan_store(bto_batch_plan *p, const std::vector<BatchItem> &items,
                             const std::vector<BatchUnit> &units, hipStream_t stream)
{
    const int count = (int)items.size();
    const int nunits = (int)units.size();
    if (hipEventSynchronize(p->staged) != hipSuccess)
        return fail(BTO_ERR_HIP, "hipEventSynchronize");
    const size_t bi = round256(sizeof(BatchItem) * (size_t)p->capacity);
    const size_t bu = round256(sizeof(BatchUnit) * (size_t)p->unit_capacity);
    char *st = p->h_stage;
    if (count > 0)
        std::memcpy(st, items.data(), sizeof(BatchItem) * (size_t)count);
    if (nunits > 0)
        std::memcpy(st + bi, units.data(), sizeof(BatchUnit) * (size_t)nunits);
    int meta[kMetaInts] = {0, nunits, 0, count};
    std::memcpy(st + bi + bu, meta, sizeof(meta));
    if ((count > 0 &&
         hipMemcpyAsync(p->d_items, st, sizeof(BatchItem) * (size_t)count, hipMemcpyHostToDevice,
                        stream) != hipSuccess) ||
        (nunits > 0 &&
         hipMemcpyAsync(p->d_units, st + bi, sizeof(BatchUnit) * (size_t)nunits,
                        hipMemcpyHostToDevice, stream) != hipSuccess) ||
        hipMemcpyAsync(p->d_meta, st + bi + bu, sizeof(meta), hipMemcpyHostToDevice, stream) !=
            hipSuccess ||
        hipEventRecord(p->staged, stream) != hipSuccess)
        return fail(BTO_ERR_HIP, std::string("refill: ") + hipGetErrorString(hipGetLastError()));
    p->count = count;
    return BTO_SUCCESS;
}

static int64_t split_of(const bto_batch_config *config)
{
    if (!config || config->split_bytes == 0)
        return kBatchSplitBytes;
    return config->split_bytes;
}

extern "C" {

int64_t bto_batch_max_n(void) { return batch_max_n(); }

int64_t bto_batch_scratch_doubles(const bto_batch_desc *descs, int count,
                                  const bto_batch_config *config)
{
    if (count < 0 || (count > 0 && !descs))
        return -1;
    const int64_t split = split_of(config);
    int64_t need = 0;
    for (int i = 0; i < count; ++i) {
        const bto_batch_desc &d = descs[i];
        if (d.m < 0 || d.n < 0)
            return -1;
        if (d.kind == BTO_K_ATAX && d.form == BTO_UNFUSED)
            need += ceil_div(d.m, (int64_t)32) * 32;
        const int64_t r = tile_rows_for(d.kind, d.form, d.m, d.n, split);
        if (r > 0)
            need += ceil_div(d.m, r) * part_stride(d.n);
    }
    return need;
}

bto_status bto_batch_plan_create(const bto_batch_desc *descs, int count,
                                 const bto_batch_config *config, bto_batch_plan **plan)
{
    return host_guard([&]() -> bto_status {
        t_error.clear();
        if (!plan)
            return fail(BTO_ERR_INVALID_ARG, "plan is NULL");
        *plan = nullptr;
        std::vector<BatchItem> items;
        std::vector<BatchUnit> units;
        int64_t scratch = 0;
        BTO_TRY(plan_image(descs, count, split_of(config), items, units, scratch));
        bto_batch_plan *p = nullptr;
        BTO_TRY(plan_alloc(count, (int)units.size(), scratch, config, &p));
        bto_status s = plan_store(p, items, units, p->cap ? p->cap : nullptr);
        if (s == BTO_SUCCESS && hipEventSynchronize(p->staged) != hipSuccess)
            s = fail(BTO_ERR_HIP, "hipEventSynchronize");
        if (s != BTO_SUCCESS) {
            plan_free(p);
            return s;
        }
        *plan = p;
        return BTO_SUCCESS;
    });
}

bto_status bto_batch_plan_create_empty(int capacity, int64_t scratch_doubles,
                                       const bto_batch_config *config, bto_batch_plan **plan)
{
    return host_guard([&]() -> bto_status {
        t_error.clear();
        if (!plan)
            return fail(BTO_ERR_INVALID_ARG, "plan is NULL");
        *plan = nullptr;
        // the unit queue holds up to kUnitsPerItem units per instance (an int)
        if (capacity < 0 || capacity > INT_MAX / kUnitsPerItem)
            return fail(BTO_ERR_INVALID_ARG, "capacity out of range");
        return plan_alloc(capacity, capacity * kUnitsPerItem, scratch_doubles, config, plan);
    });
}

bto_status bto_batch_plan_reset(bto_batch_plan *plan, const bto_batch_desc *descs, int count,
                                hipStream_t stream)
{
    return host_guard([&]() -> bto_status {
        t_error.clear();
        if (!plan)
            return fail(BTO_ERR_INVALID_ARG, "plan is NULL");
        if (count > plan->capacity)
            return fail(BTO_ERR_INVALID_ARG, "more instances than the plan's capacity");
        std::vector<BatchItem> items;
        std::vector<BatchUnit> units;
        int64_t scratch = 0;
        BTO_TRY(plan_image(descs, count, plan->split_bytes, items, units, scratch));
        if (scratch > plan->scratch_cap)
            return fail(BTO_ERR_WORKSPACE, "the instances need " + std::to_string(scratch) +
                                               " doubles of scratch, the plan has " +
                                               std::to_string(plan->scratch_cap));
        if ((int64_t)units.size() > plan->unit_capacity)
            return fail(BTO_ERR_INVALID_ARG, "more work units than the plan can queue");
        return plan_store(plan, items, units, stream);
    });
}

bto_status bto_batch_plan_launch(bto_batch_plan *plan, hipStream_t stream)
{
    t_error.clear();
    if (!plan)
        return fail(BTO_ERR_INVALID_ARG, "plan is NULL");
    if (plan->exec) {
        timing_begin(stream, "batch_graph");
        const hipError_t e = hipGraphLaunch(plan->exec, stream);
        timing_end(stream);
        if (e != hipSuccess)
            return fail(BTO_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    } else {
        launch_batch(plan->d_items, plan->d_units, plan->d_meta, plan->d_sync, plan->d_scratch,
                     plan->threads, plan->grid, stream);
    }
    return check_launch();
}

bto_status bto_batch_plan_check(bto_batch_plan *plan, hipStream_t stream)
{
    t_error.clear();
    if (!plan)
        return fail(BTO_ERR_INVALID_ARG, "plan is NULL");
    int meta[kMetaInts] = {0, 0, 0, 0};
    if (hipStreamSynchronize(stream) != hipSuccess ||
        hipMemcpy(meta, plan->d_meta, sizeof(meta), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(BTO_ERR_HIP, std::string("check: ") + hipGetErrorString(hipGetLastError()));
    if (meta[kMetaError] != 0)
        return fail(BTO_ERR_HIP, "a tile of the last launch gave up waiting for its instance's "
                                 "first sweep; its results are not valid");
    return BTO_SUCCESS;
}

bto_status bto_batch_plan_error_async(bto_batch_plan *plan, int *dst, hipStream_t stream)
{
    t_error.clear();
    if (!plan || !dst)
        return fail(BTO_ERR_INVALID_ARG, "plan or dst is NULL");
    const hipError_t e = hipMemcpyAsync(dst, plan->d_meta + kMetaError, sizeof(int),
                                        hipMemcpyDefault, stream);
    if (e != hipSuccess)
        return fail(BTO_ERR_HIP, std::string("error copy: ") + hipGetErrorString(e));
    return BTO_SUCCESS;
}

bto_status bto_batch_plan_destroy(bto_batch_plan *plan)
{
    t_error.clear();
    plan_free(plan);
    return BTO_SUCCESS;
}

}  // extern "C"

// ---- tiled batches ---------------------------------------------------------------
//
// Fused GEMVER and BiCGK instances cut into workgroup tiles, grouped by kind
// (GEMVER's first sweeps, which store B; the read-only sweeps of narrow and
// of wide matrices) and launched group by group, with launches of finish
// units between the sweeps: first sweeps, their sums, GEMVER's second
// sweeps, their sums.  Kernel boundaries order the phases, so no tile waits
// for another and no device-scope fence is issued.  The device header
// gives each group's first tile and tile count, so a refillable plan keeps
// its launches (and its captured graph) and only its tables change.

struct bto_tiled_batch {
    bto_tiled_config cfg{};
    bool refillable = false;
    int capacity = 0;                   // instances per refill
    int64_t cap_entries = 0, cap_units = 0, cap_jobs = 0, cap_funits = 0, cap_scratch = 0;
    char *d_tables = nullptr;           // one allocation holding the tables below
    BTileEntry *d_entries = nullptr;
    BTileUnit *d_units = nullptr;       // tile groups, in group order
    FinishJob *d_jobs = nullptr;        // jobs after the first sweeps, then after the second
    BFinishUnit *d_funits = nullptr;
    int *d_hdr = nullptr;               // kBtHdrInts: first tile and count per group
    double *d_scratch = nullptr;        // partial sums
    int grid[BG_COUNT] = {};            // workgroups per launch (0: nothing to launch)
    int cus = 0;                        // compute units of the plan's device
    int count = 0;
    // pinned staging of the tables for asynchronous refills, and the event
    // that marks when the last refill has been read
    char *h_stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t staged = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
};

namespace {

// Defaults from the tiled-batch search (tune.py --batch: 4096 mixed
// GEMVER/BiCGK instances, n log-uniform on [64, 2048], MI355X): the first
// sweeps in tiles of 256 columns (8 waves down, two 16-byte pairs per lane,
// two rows in flight per wave), of 32 rows for GEMVER and 256 rows for
// BiCGK; GEMVER's second sweeps in 64-row tiles of 256 columns for matrices
// up to 512 columns wide and of 512 columns (2 waves, each sweeping the
// whole band) above; one workgroup per tile.  The best dozen configurations
// were within 1.5% of each other.
constexpr bto_tiled_config kTiledDefaults = {
    /*store_shape*/ 2, /*narrow_shape*/ 2, /*wide_shape*/ 7, /*narrow_n*/ 512,
    /*store_rb*/ 16, /*bicgk_rb*/ 64, /*read_rb*/ 64, /*wgs_per_cu*/ 0, /*use_graph*/ 1};
constexpr int kTiledFinishWgsPerCu = 8;
constexpr int kTiledRefillWgsPerCu = 2;   // refillable plans made with the defaults


bto_status tiled_check_config(const bto_tiled_config &c)
{
    if (!btile_shape_ok(c.store_shape, kBtFirstOps, c.store_rb))
        return fail(BTO_ERR_INVALID_ARG, "store_shape / store_rb: not an instantiated tile shape "
                                         "for the first sweeps with that band height");
    if (!btile_shape_ok(c.store_shape, kBtFirstOps, c.bicgk_rb))
        return fail(BTO_ERR_INVALID_ARG, "store_shape / bicgk_rb: not an instantiated tile shape "
                                         "for BiCGK's sweeps with that band height");
    for (int sh : {c.narrow_shape, c.wide_shape})
        if (!btile_shape_ok(sh, OP_ROWDOT, c.read_rb))
            return fail(BTO_ERR_INVALID_ARG, "narrow_shape / wide_shape / read_rb: not an "
                                             "instantiated tile shape for GEMVER's second sweeps "
                                             "with that band height");
    if (c.narrow_n < 0)
        return fail(BTO_ERR_INVALID_ARG, "narrow_n must not be negative");
    if (c.wgs_per_cu < 0 || c.wgs_per_cu > 16)
        return fail(BTO_ERR_INVALID_ARG, "wgs_per_cu must be 0 (a workgroup per tile) to 16");
    if (c.use_graph != 0 && c.use_graph != 1)
        return fail(BTO_ERR_INVALID_ARG, "use_graph must be 0 or 1");
    return BTO_SUCCESS;
}

// What one instance adds to each table.
struct TiledNeeds {
    int64_t entries = 0, units = 0, jobs = 0, funits = 0, scratch = 0;
};

int64_t round32(int64_t d) { return ceil_div(d > 0 ? d : 1, (int64_t)32) * 32; }

int read_shape_of(const bto_tiled_config &c, int64_t n)
{
    return n <= c.narrow_n ? c.narrow_shape : c.wide_shape;
}

TiledNeeds tiled_needs(const bto_tiled_config &c, int kind, int64_t m, int64_t n)
{
    TiledNeeds t;
    const bool some = m > 0 && n > 0;
    // the first sweeps (GEMVER's and BiCGK's) in store_shape tiles, of store_rb
    // rows for GEMVER and bicgk_rb rows for BiCGK
    const int64_t frb = kind == BTO_K_BICGK ? c.bicgk_rb : c.store_rb;
    const int64_t fbands = some ? ceil_div(m, frb) : 0;
    const int64_t ftiles = fbands * (some ? ceil_div(n, btile_cols(c.store_shape)) : 0);
    t.jobs = 2;
    t.funits = ceil_div(m, (int64_t)64) + ceil_div(n, (int64_t)64);
    if (kind == BTO_K_GEMVER) {
        const int rs = read_shape_of(c, n);
        const int64_t rbands = some ? ceil_div(m, (int64_t)c.read_rb) : 0;
        const int64_t nwt = some ? ceil_div(n, btile_wave_cols(rs)) : 0;
        t.entries = some ? 2 : 0;
        t.units = ftiles + rbands * (some ? ceil_div(n, btile_cols(rs)) : 0);
        t.scratch = round32(fbands * n) + round32(nwt * m);
    } else {
        const int64_t nwt = some ? ceil_div(n, btile_wave_cols(c.store_shape)) : 0;
        t.entries = some ? 1 : 0;
        t.units = ftiles;
        t.scratch = round32(nwt * m) + round32(fbands * n);
    }
    return t;
}

struct TiledImage {
    std::vector<BTileEntry> entries;
    std::vector<BTileUnit> units[BG_COUNT];   // tile groups
    std::vector<FinishJob> jobs[BG_COUNT];    // finish groups

    int64_t njobs() const
    {
        int64_t k = 0;
        for (const auto &j : jobs) k += (int64_t)j.size();
        return k;
    }
    int64_t nunits() const
    {
        int64_t k = 0;
        for (const auto &u : units) k += (int64_t)u.size();
        return k;
    }
    int64_t nfinish_units() const
    {
        int64_t k = 0;
        for (const auto &js : jobs)
            for (const FinishJob &j : js) k += ceil_div(j.len, (int64_t)64);
        return k;
    }
    int64_t scratch = 32;   // doubles; offset 0 is left unused, so no area is at "null"
};

// Validate the instances and lay out entries, tiles, finish jobs and the
// partial-sum areas (offsets into a scratch area starting at 0, kept as
// fake pointers until they are rebased onto the plan's scratch).
bto_status tiled_image(const bto_tiled_config &c, const bto_batch_desc *descs, int count,
                       TiledImage &img)
{
    if (count < 0 || (count > 0 && !descs))
        return fail(BTO_ERR_INVALID_ARG, "bad instance list");
    std::vector<BSpan> spans;
    std::vector<BatchItem> items((size_t)count);
    int64_t unused = 0;
    for (int i = 0; i < count; ++i) {
        BTO_TRY(batch_check_one(descs[i], i, spans, items[i], unused, -1));
        if (descs[i].kind == BTO_K_ATAX || descs[i].form != BTO_FUSED)
            return fail(BTO_ERR_UNSUPPORTED, "instance " + std::to_string(i) +
                                                 ": tiled batches run fused GEMVER and BiCGK");
    }
    BTO_TRY(batch_check_overlaps(spans));
    // largest instances first, so that the small ones fill the end
    std::vector<int> order((size_t)count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (double)items[a].m * (double)items[a].n > (double)items[b].m * (double)items[b].n;
    });
    auto take = [&](int64_t doubles) {   // an offset, as a fake pointer until rebased
        const int64_t off = img.scratch;
        img.scratch += round32(doubles);
        return reinterpret_cast<double *>((uintptr_t)(off * 8));
    };
    // the bands of the instance one after another, each band's column blocks
    // side by side, so that neighbouring tiles read neighbouring memory
    auto tiles = [&](int group, int entry, int64_t nb, int64_t nc) {
        if ((int64_t)img.units[group].size() + nb * nc > INT_MAX)
            return false;
        for (int64_t b = 0; b < nb; ++b)
            for (int64_t k = 0; k < nc; ++k)
                img.units[group].push_back({entry, (int32_t)b, (int32_t)k, 0});
        return true;
    };
    const auto too_many = [] { return fail(BTO_ERR_UNSUPPORTED, "too many tiles for one launch"); };
    int64_t fin_blocks = 0;
    for (int i : order) {
        const BatchItem &it = items[i];
        const int64_t m = it.m, n = it.n;
        const bool some = m > 0 && n > 0;
        // the first sweeps: store_shape tiles, of store_rb rows (GEMVER) or
        // bicgk_rb rows (BiCGK)
        const int frb = it.kind == BTO_K_BICGK ? c.bicgk_rb : c.store_rb;
        const int64_t fbands = some ? ceil_div(m, (int64_t)frb) : 0;
        const int64_t fcols = some ? ceil_div(n, btile_cols(c.store_shape)) : 0;
        const bool rows16 = it.lda % 2 == 0 || m <= 1;
        BTileEntry e{};
        e.rb = frb;
        e.a.m = m;
        e.a.n = n;
        e.a.lda = it.lda;
        e.a.ldb = it.ldb;
        e.a.A = it.A;
        if (it.kind == BTO_K_BICGK) {
            // q = A p, s = A^T r: row dots per wave tile, column sums per band
            const int64_t nwt = some ? ceil_div(n, btile_wave_cols(c.store_shape)) : 0;
            double *prow = take(nwt * m), *pcol = take(fbands * n);
            e.a.xr = it.vec[0];
            e.a.yc = it.vec[1];
            e.a.Prow = prow;
            e.a.Pcol = pcol;
            e.vec = aligned16(it.A) && rows16;
            e.ops = OP_ROWDOT | OP_COLSUM;
            if (some) {
                img.entries.push_back(e);
                if (!tiles(BG_FIRST, (int)img.entries.size() - 1, fbands, fcols))
                    return too_many();
            }
            img.jobs[BG_FIN1].push_back({prow, nwt, m, 1.0, nullptr, it.out[0]});
            img.jobs[BG_FIN1].push_back({pcol, fbands, n, 1.0, nullptr, it.out[1]});
        } else {
            // B = A + u1 v1^T + u2 v2^T and x = beta B^T y + z, then w = alpha B x
            const int rs = read_shape_of(c, n);
            const int64_t rbands = some ? ceil_div(m, (int64_t)c.read_rb) : 0;
            const int64_t rcols = some ? ceil_div(n, btile_cols(rs)) : 0;
            const int64_t nwt = some ? ceil_div(n, btile_wave_cols(rs)) : 0;
            double *pcol = take(fbands * n), *prow = take(nwt * m);
            e.a.B = it.B;
            e.a.u1 = it.vec[0];
            e.a.v1 = it.vec[1];
            e.a.u2 = it.vec[2];
            e.a.v2 = it.vec[3];
            e.a.yc = it.vec[4];
            e.a.Pcol = pcol;
            e.vec = aligned16(it.A) && aligned16(it.B) && rows16 && (it.ldb % 2 == 0 || m <= 1);
            e.ops = OP_UPD1 | OP_UPD2 | OP_COLSUM;
            BTileEntry e2{};
            e2.rb = c.read_rb;
            e2.a.m = m;
            e2.a.n = n;
            e2.a.lda = it.ldb;
            e2.a.ldb = it.ldb;
            e2.a.A = it.B;
            e2.a.xr = it.out[0];
            e2.a.Prow = prow;
            e2.vec = aligned16(it.B) && (it.ldb % 2 == 0 || m <= 1);
            e2.ops = OP_ROWDOT;
            if (some) {
                img.entries.push_back(e);
                if (!tiles(BG_FIRST, (int)img.entries.size() - 1, fbands, fcols))
                    return too_many();
                img.entries.push_back(e2);
                if (!tiles(n <= c.narrow_n ? BG_ROW_NARROW : BG_ROW_WIDE,
                           (int)img.entries.size() - 1, rbands, rcols))
                    return too_many();
            }
            img.jobs[BG_FIN1].push_back({pcol, fbands, n, it.beta, it.vec[5], it.out[0]});
            img.jobs[BG_FIN_W].push_back({prow, nwt, m, it.alpha, nullptr, it.out[1]});
        }
        if ((int64_t)img.entries.size() > INT_MAX)
            return fail(BTO_ERR_UNSUPPORTED, "too many instances for one launch");
        // every finish indexes its 64-output blocks with an int
        fin_blocks += ceil_div(m, (int64_t)64) + ceil_div(n, (int64_t)64);
        if (fin_blocks > INT_MAX)
            return fail(BTO_ERR_UNSUPPORTED, "too many outputs for one launch");
    }
    return BTO_SUCCESS;
}

void finish_units(const std::vector<FinishJob> &jobs, int first_job, std::vector<BFinishUnit> &u)
{
    for (size_t j = 0; j < jobs.size(); ++j)
        for (int64_t b = 0; b < ceil_div(jobs[j].len, (int64_t)64); ++b)
            u.push_back({first_job + (int32_t)j, (int32_t)b});
}

// The flat tables of an image, with its partial-sum offsets rebased onto
// `base` (the plan's scratch).
struct TiledTables {
    std::vector<BTileEntry> entries;
    std::vector<BTileUnit> units;
    std::vector<FinishJob> jobs;
    std::vector<BFinishUnit> funits;
    int hdr[kBtHdrInts] = {};
};

void tiled_tables(TiledImage &img, uintptr_t base, TiledTables &t)
{
    auto rebase = [&](double *&q) {
        if (q) q = reinterpret_cast<double *>(base + reinterpret_cast<uintptr_t>(q));
    };
    for (BTileEntry &e : img.entries) {
        rebase(e.a.Prow);
        rebase(e.a.Pcol);
    }
    for (auto &jobs : img.jobs)
        for (FinishJob &j : jobs)
            j.P = reinterpret_cast<const double *>(base + reinterpret_cast<uintptr_t>(j.P));
    t.entries.swap(img.entries);
    for (int g = 0; g < BG_COUNT; ++g) {
        if (bt_is_finish(g)) {
            t.hdr[2 * g] = (int)t.funits.size();
            finish_units(img.jobs[g], (int)t.jobs.size(), t.funits);
            t.hdr[2 * g + 1] = (int)t.funits.size() - t.hdr[2 * g];
            t.jobs.insert(t.jobs.end(), img.jobs[g].begin(), img.jobs[g].end());
        } else {
            t.hdr[2 * g] = (int)t.units.size();
            t.hdr[2 * g + 1] = (int)img.units[g].size();
            t.units.insert(t.units.end(), img.units[g].begin(), img.units[g].end());
        }
    }
}

void tiled_free(bto_tiled_batch *p)
{
    if (!p) return;
    if (p->staged) (void)hipEventSynchronize(p->staged);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->d_tables) (void)hipFree(p->d_tables);
    if (p->d_scratch) (void)hipFree(p->d_scratch);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    if (p->staged) (void)hipEventDestroy(p->staged);
    delete p;
}

void tiled_group(const bto_tiled_batch *p, int g, hipStream_t st)
{
    const bto_tiled_config &c = p->cfg;
    switch (g) {
    case BG_FIRST:
        launch_btile(c.store_shape, kBtFirstOps, p->d_entries, p->d_units, p->d_hdr, g,
                     p->grid[g], st);
        break;
    case BG_ROW_NARROW:
    case BG_ROW_WIDE:
        launch_btile(g == BG_ROW_NARROW ? c.narrow_shape : c.wide_shape, OP_ROWDOT, p->d_entries,
                     p->d_units, p->d_hdr, g, p->grid[g], st);
        break;
    default:
        launch_btile_finish(p->d_jobs, p->d_funits, p->d_hdr, g, p->grid[g], st);
        break;
    }
}

void tiled_enqueue(const bto_tiled_batch *p, hipStream_t st)
{
    for (int g = 0; g < BG_COUNT; ++g)
        tiled_group(p, g, st);
}

size_t tiled_stage_layout(const bto_tiled_batch *p, size_t off[5])
{
    size_t o = 0;
    off[0] = o; o += round256(sizeof(BTileEntry) * (size_t)p->cap_entries);
    off[1] = o; o += round256(sizeof(BTileUnit) * (size_t)p->cap_units);
    off[2] = o; o += round256(sizeof(FinishJob) * (size_t)p->cap_jobs);
    off[3] = o; o += round256(sizeof(BFinishUnit) * (size_t)p->cap_funits);
    off[4] = o; o += round256(sizeof(int) * kBtHdrInts);
    return o;
}

// Point the plan's tables at their offsets in its one allocation.
void tiled_point(bto_tiled_batch *p, const size_t off[5])
{
    p->d_entries = reinterpret_cast<BTileEntry *>(p->d_tables + off[0]);
    p->d_units = reinterpret_cast<BTileUnit *>(p->d_tables + off[1]);
    p->d_jobs = reinterpret_cast<FinishJob *>(p->d_tables + off[2]);
    p->d_funits = reinterpret_cast<BFinishUnit *>(p->d_tables + off[3]);
    p->d_hdr = reinterpret_cast<int *>(p->d_tables + off[4]);
}

// Allocate a plan's device tables (capacities set), its staging and event.
bto_status tiled_alloc(bto_tiled_batch *p)
{
    auto bytes = [](size_t each, int64_t n) { return each * (size_t)(n > 0 ? n : 1); };
    size_t off[5];
    p->stage_bytes = tiled_stage_layout(p, off);
    if (hipMalloc(&p->d_tables, p->stage_bytes) != hipSuccess ||
        hipMalloc(&p->d_scratch, bytes(sizeof(double), p->cap_scratch)) != hipSuccess)
        return fail(BTO_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(hipGetLastError()));
    tiled_point(p, off);
    if (hipMemset(p->d_hdr, 0, sizeof(int) * kBtHdrInts) != hipSuccess)
        return fail(BTO_ERR_HIP, "hipMemset");
    if (hipHostMalloc((void **)&p->h_stage, p->stage_bytes, hipHostMallocDefault) != hipSuccess)
        return fail(BTO_ERR_HIP, "hipHostMalloc");
    if (hipEventCreateWithFlags(&p->staged, hipEventDisableTiming) != hipSuccess)
        return fail(BTO_ERR_HIP, "hipEventCreate");
    return BTO_SUCCESS;
}

// Copy validated tables into the plan on `stream` (asynchronously, through
// the pinned staging, after the previous refill has been read).  A plan
// launched without a graph gives its kernels the tables' addresses at each
// launch, so its tables are packed one after another and sent in one copy;
// a captured graph keeps the fixed layout its launches were recorded with,
// and each table is sent on its own.
bto_status tiled_store(bto_tiled_batch *p, const TiledTables &t, hipStream_t stream)
{
    if (hipEventSynchronize(p->staged) != hipSuccess)
        return fail(BTO_ERR_HIP, "hipEventSynchronize");
    const size_t bytes[5] = {sizeof(BTileEntry) * t.entries.size(),
                             sizeof(BTileUnit) * t.units.size(), sizeof(FinishJob) * t.jobs.size(),
                             sizeof(BFinishUnit) * t.funits.size(), sizeof(int) * kBtHdrInts};
    const void *src[5] = {t.entries.data(), t.units.data(), t.jobs.data(), t.funits.data(), t.hdr};
    const bool packed = !p->cfg.use_graph;
    size_t off[5];
    size_t end = 0;
    if (packed) {
        for (int k = 0; k < 5; ++k) {
            off[k] = end;
            end += round256(bytes[k]);
        }
    } else {
        tiled_stage_layout(p, off);
    }
    char *st = p->h_stage;
    for (int k = 0; k < 5; ++k)
        if (bytes[k])
            std::memcpy(st + off[k], src[k], bytes[k]);
    if (packed) {
        tiled_point(p, off);
        if (hipMemcpyAsync(p->d_tables, st, end, hipMemcpyHostToDevice, stream) != hipSuccess)
            return fail(BTO_ERR_HIP, std::string("refill: ") + hipGetErrorString(hipGetLastError()));
    } else {
        for (int k = 0; k < 5; ++k) {
            if (bytes[k] == 0)
                continue;
            if (hipMemcpyAsync(p->d_tables + off[k], st + off[k], bytes[k],
                               hipMemcpyHostToDevice, stream) != hipSuccess)
                return fail(BTO_ERR_HIP,
                            std::string("refill: ") + hipGetErrorString(hipGetLastError()));
        }
    }
    if (hipEventRecord(p->staged, stream) != hipSuccess)
        return fail(BTO_ERR_HIP, "hipEventRecord");
    return BTO_SUCCESS;
}

bto_status tiled_capture(bto_tiled_batch *p)
{
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
        return fail(BTO_ERR_HIP, "hipStreamCreate");
    if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(BTO_ERR_HIP, "hipStreamBeginCapture");
    t_capturing = true;
    tiled_enqueue(p, p->cap);
    t_capturing = false;
    if (hipStreamEndCapture(p->cap, &p->graph) != hipSuccess)
        return fail(BTO_ERR_HIP, "hipStreamEndCapture");
    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        return fail(BTO_ERR_HIP, "hipGraphInstantiate");
    return BTO_SUCCESS;
}

bto_status device_cus(int &cus)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return fail(BTO_ERR_HIP, "no device");
    return BTO_SUCCESS;
}

bto_status resolve_config(const bto_tiled_config *config, bto_tiled_config &c)
{
    c = config ? *config : kTiledDefaults;
    return tiled_check_config(c);
}

// Workgroups per launch for a set of tiles: one per tile, or persistent
// workgroups (never more than tiles); none for an empty group.
void set_grids(bto_tiled_batch *p, const int *hdr)
{
    for (int g = 0; g < BG_COUNT; ++g) {
        const int64_t n = hdr[2 * g + 1];
        const int64_t per = bt_is_finish(g) ? kTiledFinishWgsPerCu : p->cfg.wgs_per_cu;
        const int64_t cap = per > 0 ? (int64_t)p->cus * per : n;
        p->grid[g] = (int)(n < cap ? n : cap);
    }
}

bto_status tiled_create(const bto_batch_desc *descs, int count, const bto_tiled_config &c,
                        bto_tiled_batch **plan)
{
    TiledImage img;
    BTO_TRY(tiled_image(c, descs, count, img));
    int cus = 0;
    BTO_TRY(device_cus(cus));
    bto_tiled_batch *p = new bto_tiled_batch();
    p->cfg = c;
    p->count = count;
    p->capacity = count;
    p->cap_entries = (int64_t)img.entries.size();
    p->cap_units = img.nunits();
    p->cap_jobs = img.njobs();
    p->cap_scratch = img.scratch;
    p->cap_funits = img.nfinish_units();
    bto_status s = tiled_alloc(p);
    TiledTables t;
    if (s == BTO_SUCCESS) {
        tiled_tables(img, reinterpret_cast<uintptr_t>(p->d_scratch), t);
        s = tiled_store(p, t, nullptr);
    }
    if (s == BTO_SUCCESS && hipEventSynchronize(p->staged) != hipSuccess)
        s = fail(BTO_ERR_HIP, "hipEventSynchronize");
    if (s != BTO_SUCCESS) {
        tiled_free(p);
        return s;
    }
    p->cus = cus;
    set_grids(p, t.hdr);
    if (c.use_graph) {
        s = tiled_capture(p);
        if (s != BTO_SUCCESS) {
            tiled_free(p);
            return s;
        }
    }
    *plan = p;
    return BTO_SUCCESS;
}

}  // namespace

extern "C" {

void bto_tiled_config_default(bto_tiled_config *config)
{
    if (config)
        *config = kTiledDefaults;
}

int bto_tiled_shape_count(void) { return kBtShapeCount; }

bto_status bto_tiled_shape(int shape, int *kv, int *depth, int *waves_across, int *waves_down)
{
    t_error.clear();
    if (shape < 0 || shape >= kBtShapeCount)
        return fail(BTO_ERR_INVALID_ARG, "no such tile shape");
    int v[4];
    btile_shape_info(shape, v);
    if (kv) *kv = v[0];
    if (depth) *depth = v[1];
    if (waves_across) *waves_across = v[2];
    if (waves_down) *waves_down = v[3];
    return BTO_SUCCESS;
}

bto_status bto_tiled_batch_create(const bto_batch_desc *descs, int count, int use_graph,
                                  bto_tiled_batch **plan)
{
    return host_guard([&]() -> bto_status {
        t_error.clear();
        if (!plan)
            return fail(BTO_ERR_INVALID_ARG, "plan is NULL");
        *plan = nullptr;
        bto_tiled_config c = kTiledDefaults;
        c.use_graph = use_graph ? 1 : 0;
        return tiled_create(descs, count, c, plan);
    });
}

bto_status bto_tiled_batch_create_config(const bto_batch_desc *descs, int count,
                                         const bto_tiled_config *config, bto_tiled_batch **plan)
{
    return host_guard([&]() -> bto_status {
        t_error.clear();
        if (!plan)
            return fail(BTO_ERR_INVALID_ARG, "plan is NULL");
        *plan = nullptr;
        bto_tiled_config c;
        BTO_TRY(resolve_config(config, c));
        return tiled_create(descs, count, c, plan);
    });
}

bto_status bto_tiled_batch_create_empty(int capacity, int64_t max_m, int64_t max_n,
                                        const bto_tiled_config *config, bto_tiled_batch **plan)
{
    return host_guard([&]() -> bto_status {
        t_error.clear();
        if (!plan)
            return fail(BTO_ERR_INVALID_ARG, "plan is NULL");
        *plan = nullptr;
        bto_tiled_config c;
        BTO_TRY(resolve_config(config, c));
        if (!config && c.wgs_per_cu == 0)
            c.wgs_per_cu = kTiledRefillWgsPerCu;
        if (c.wgs_per_cu == 0 && c.use_graph)
            return fail(BTO_ERR_INVALID_ARG, "a refillable plan in a graph needs persistent "
                                             "workgroups (wgs_per_cu 1 to 16)");
        if (capacity < 0 || max_m < 0 || max_n < 0)
            return fail(BTO_ERR_INVALID_ARG, "negative capacity or size");
        if (max_n > batch_max_n())
            return fail(BTO_ERR_UNSUPPORTED, "more columns than a batched instance may have");
        // the most any one instance within the bounds can need, per table:
        // each count grows with m and n within one read shape
        TiledNeeds worst;
        for (int kind : {BTO_K_GEMVER, BTO_K_BICGK})
            for (int64_t n : {max_n, max_n < c.narrow_n ? max_n : (int64_t)c.narrow_n}) {
                const TiledNeeds t = tiled_needs(c, kind, max_m, n);
                worst.entries = std::max(worst.entries, t.entries);
                worst.units = std::max(worst.units, t.units);
                worst.jobs = std::max(worst.jobs, t.jobs);
                worst.funits = std::max(worst.funits, t.funits);
                worst.scratch = std::max(worst.scratch, t.scratch);
            }
        const double cap = capacity;
        if (cap * (double)worst.units > INT_MAX || cap * (double)worst.funits > INT_MAX)
            return fail(BTO_ERR_UNSUPPORTED, "too many tiles for one launch");
        int cus = 0;
        BTO_TRY(device_cus(cus));
        bto_tiled_batch *p = new bto_tiled_batch();
        p->cfg = c;
        p->refillable = true;
        p->capacity = capacity;
        p->cap_entries = capacity * worst.entries;
        p->cap_units = capacity * worst.units;
        p->cap_jobs = capacity * worst.jobs;
        p->cap_funits = capacity * worst.funits;
        p->cap_scratch = 32 + capacity * worst.scratch;
        p->cus = cus;
        // a graph replays fixed launches that read their tile counts from the
        // device header; without one, each refill sizes the launches itself
        for (int g = 0; g < BG_COUNT && c.use_graph; ++g)
            p->grid[g] = cus * (bt_is_finish(g) ? kTiledFinishWgsPerCu : c.wgs_per_cu);
        bto_status s = tiled_alloc(p);
        if (s == BTO_SUCCESS && c.use_graph)
            s = tiled_capture(p);
        if (s != BTO_SUCCESS) {
            tiled_free(p);
            return s;
        }
        *plan = p;
        return BTO_SUCCESS;
    });
}

bto_status bto_tiled_batch_reset(bto_tiled_batch *plan, const bto_batch_desc *descs, int count,
                                 hipStream_t stream)
{
    return host_guard([&]() -> bto_status {
        t_error.clear();
        if (!plan)
            return fail(BTO_ERR_INVALID_ARG, "plan is NULL");
        if (!plan->refillable)
            return fail(BTO_ERR_INVALID_ARG, "the plan was not made by bto_tiled_batch_create_empty");
        if (count > plan->capacity)
            return fail(BTO_ERR_INVALID_ARG, "more instances than the plan's capacity");
        TiledImage img;
        BTO_TRY(tiled_image(plan->cfg, descs, count, img));
        if ((int64_t)img.entries.size() > plan->cap_entries || img.nunits() > plan->cap_units ||
            img.njobs() > plan->cap_jobs || img.nfinish_units() > plan->cap_funits ||
            img.scratch > plan->cap_scratch)
            return fail(BTO_ERR_WORKSPACE, "the instances need more tiles or scratch than the "
                                           "plan was made for");
        TiledTables t;
        tiled_tables(img, reinterpret_cast<uintptr_t>(plan->d_scratch), t);
        BTO_TRY(tiled_store(plan, t, stream));
        if (!plan->exec)
            set_grids(plan, t.hdr);
        plan->count = count;
        return BTO_SUCCESS;
    });
}

bto_status bto_tiled_batch_launch(bto_tiled_batch *plan, hipStream_t stream)
{
    t_error.clear();
    if (!plan)
        return fail(BTO_ERR_INVALID_ARG, "plan is NULL");
    if (plan->exec) {
        timing_begin(stream, "tiled_batch_graph");
        const hipError_t e = hipGraphLaunch(plan->exec, stream);
        timing_end(stream);
        if (e != hipSuccess)
            return fail(BTO_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    } else {
        tiled_enqueue(plan, stream);
    }
    return check_launch();
}

bto_status bto_tiled_batch_destroy(bto_tiled_batch *plan)
{
    t_error.clear();
    tiled_free(plan);
    return BTO_SUCCESS;
}

}  // extern "C"
