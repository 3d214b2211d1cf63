// Host-side declarations shared by the translation units of libbto.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bto {

// Per-kernel event timing (enabled through bto_timing_enable).
void timing_begin(hipStream_t st, const char *name);
void timing_end(hipStream_t st);

// Launch `kernel` unless the grid is empty, bracketed by timing events.
template <typename... KArgs, typename... Args>
inline void launch(const char *name, void (*kernel)(KArgs...), dim3 grid, dim3 block,
                   hipStream_t st, Args... args)
{
    if (grid.x == 0 || grid.y == 0 || grid.z == 0)
        return;
    timing_begin(st, name);
    kernel<<<grid, block, 0, st>>>(static_cast<KArgs>(args)...);
    timing_end(st);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Round a byte count up to the 256-byte granule used to carve workspaces.
inline size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

// ---- vector kernels (bto_vec.hip) ---------------------------------------

enum EwOp {
    EW_VADD3,    // out = (a + b) + c
    EW_ADD2,     // out = a + b
    EW_WAXPBY,   // out = s0*a + s1*b
    EW_SCAL,     // out = s0*a
    EW_AXPY,     // out = a + s0*b
    EW_AXMY,     // out = a - s0*b
};

// out = sum_k c[k] x[k], k = 0..count-1 added left to right, in one pass
constexpr int kMaxLin = 8;
struct LinArgs {
    const double *x[kMaxLin];
    double c[kMaxLin];
    double *out;
};
void launch_lincomb(int64_t n, int count, const LinArgs &a, hipStream_t st);

void launch_ew(EwOp op, int64_t n, const double *a, const double *b, const double *c,
               double s0, double s1, double *out, hipStream_t st);

// Number of partial sums the deterministic dot product of length n uses.
int64_t dot_parts(int64_t n);

// Dot partials: fused (z = w - alpha*v stored, partials of z.u) or plain
// (partials of w.u; v, z unused), then the fixed-order finish into *r.
void launch_dot(bool fused_axpy, int64_t n, double alpha, const double *w, const double *v,
                const double *u, double *z, double *parts, double *r, hipStream_t st);

// Read probe: *out = sum of src[0..n) (fixed order), partials in `parts`
// (read_parts(n) doubles).
int64_t read_parts(int64_t n);
void launch_read(int64_t n, const double *src, double *parts, double *out, hipStream_t st);

void launch_copy(int64_t n, const double *src, double *dst, hipStream_t st);
void launch_triad(int64_t n, double *a, const double *b, const double *c, double s,
                  hipStream_t st);

// ---- matrix kernels (bto_mat.hip) ---------------------------------------

enum TileOps {
    OP_ROWDOT = 1,  // partial row dots with xr, per column tile
    OP_COLSUM = 2,  // partial column sums weighted by yc, per row band
    OP_UPD1 = 4,    // B = A + u1 v1^T  (stored)
    OP_UPD2 = 8,    // ... + u2 v2^T    (with OP_UPD1)
    // the two dots of a rank-2 correction, for sweeps that leave B = A +
    // u1 v1^T + u2 v2^T unformed: with OP_COLSUM the band's u1.yc and u2.yc
    // into Prow[2 band], Prow[2 band + 1]; with OP_ROWDOT the wave tile's
    // v1.xr and v2.xr into Pcol[2 t], Pcol[2 t + 1]
    OP_AUX = 16,
};

struct TileCfg {
    int shape;  // index into the instantiated tile shapes (KV, D, WC, WR)
    int rb;     // rows per workgroup band
    int rev;    // walk row bands in reverse order
};

struct TileArgs {
    int64_t m, n, lda, ldb;
    const double *A;
    double *B;
    const double *xr;  // length n, row-dot weights
    const double *yc;  // length m, column-sum weights
    const double *u1, *v1, *u2, *v2;
    double *Prow;      // [wave tiles][m]
    double *Pcol;      // [row bands][n]
};

// Shapes 0..5 serve read-only sweeps, 6..14 sweeps that store B.
constexpr int kTileShapes = 15;
// The narrowest wave tile of any shape, in 16-byte pairs per lane: row-dot
// partials ([wave tiles][m]) are sized for it.
constexpr int kMinTileKv = 1;
bool tile_cfg_supported(int ops, const TileCfg &c);
int tile_kv(const TileCfg &c);
void tile_shape_info(int shape, int out[4]);   // kv, depth, waves across, waves down
int64_t tile_ncols(const TileCfg &c, int64_t n);     // number of wave tiles across n
inline int64_t tile_nbands(const TileCfg &c, int64_t m) { return ceil_div(m, c.rb); }
// Returns false (launching nothing) when the configuration is not supported.
bool launch_tile(const char *name, int ops, const TileCfg &c, const TileArgs &a, hipStream_t st);

// out[i] = scale * sum_k P[k*len + i] (+ add[i]) for two independent jobs in
// one launch (the second may have len 0).
struct FinishJob {
    const double *P;
    int64_t nparts, len;
    double scale;
    const double *add;
    double *out;
};
void launch_finish(const char *name, const FinishJob &j0, const FinishJob &j1, hipStream_t st);
// out[i] = scale * sum_k P[k*len + i] + scale2 * sum_k P2[k*len + i]
//          + add_scale * add[i]   (the P2 term when P2 is set, the last when add is)
struct FinishLin {
    FinishJob j;
    const double *P2;
    int64_t nparts2;
    double scale2, add_scale;
};
void launch_finish_lin(const char *name, const FinishLin &f, hipStream_t st);
// out[i] = scale * (sum_k P[k*len + i] + c1[i] S1 + c2[i] S2) + add[i], where
// S1 = sum_k aux[2k] and S2 = sum_k aux[2k + 1] (k < naux), in fixed orders
struct FinishAux {
    FinishJob j;
    const double *aux;
    int64_t naux;
    const double *c1, *c2;
};
void launch_finish_aux(const char *name, const FinishAux &f, hipStream_t st);

// Tiled batches (bto_btile.hip): the sweeps of many instances cut into
// workgroup tiles (one sweep of one instance, a band of rows, a block of
// columns), launched per group of tiles of one kind with a kernel
// specialised for the group's tile shape and operations, then their
// partial sums reduced by finish launches.
struct BTileEntry {     // one sweep of one instance
    TileArgs a;
    int32_t vec;        // A (and B) 16-byte aligned with even leading dimensions
    int32_t ops;        // the sweep's operations (OP_* flags)
    int32_t rb;         // rows per band of its tiles
    int32_t pad;
};
struct BTileUnit {      // one tile
    int32_t entry, band, cblk, pad;
};
struct BFinishUnit {    // 64 outputs of one finish job
    int32_t job, block;
};
// The groups of a tiled batch, in launch order.  The first launch runs
// GEMVER's first sweeps and BiCGK's sweeps together (a tile of either kind
// per workgroup, the entry's ops telling which), so that tiles that read and
// write interleave with tiles that only read.  The device header holds, for
// group g, the index of its first tile (or finish unit) at [2g] and their
// count at [2g + 1].
enum BtGroup {
    BG_FIRST = 0,       // GEMVER: B = A + u1 v1^T + u2 v2^T and column sums; BiCGK sweeps
    BG_FIN1,            // sums of GEMVER's x and BiCGK's q and s
    BG_ROW_NARROW,      // GEMVER second sweeps (w = alpha B x), matrices at most narrow_n wide
    BG_ROW_WIDE,        // ... wider ones
    BG_FIN_W,           // sums of GEMVER's w
    BG_COUNT
};
inline bool bt_is_finish(int g) { return g == BG_FIN1 || g == BG_FIN_W; }
constexpr int kBtHdrInts = 2 * BG_COUNT;
constexpr int kBtShapeCount = 12;
// a tile shape that is instantiated for `ops` and can take bands of rb rows
bool btile_shape_ok(int shape, int ops, int rb);
int64_t btile_cols(int shape);        // columns per workgroup block
int64_t btile_wave_cols(int shape);   // columns per wave tile (one row-dot partial each)
int btile_threads(int shape);
void btile_shape_info(int shape, int out[4]);   // kv, depth, waves across, waves down
// `grid` workgroups; with fewer than the group's tiles they step through them.
// ops is OP_ROWDOT for GEMVER's second sweeps, or kBtFirstOps for the first
// launch, whose tiles take their operations from their entries.
constexpr int kBtFirstOps = -1;
void launch_btile(int shape, int ops, const BTileEntry *entries, const BTileUnit *units,
                  const int *hdr, int group, int grid, hipStream_t st);
void launch_btile_finish(const FinishJob *jobs, const BFinishUnit *units, const int *hdr,
                         int group, int grid, hipStream_t st);

// Row-resident ATAX: each workgroup keeps one row of A on chip at a time.
// Row-resident sweeps: the number of workgroups (partial column-sum
// vectors) for a workgroup size, 0 when n is too wide or threads is 0.
int64_t rowres_parts(int64_t m, int64_t n, int threads, bool bicgk);
int64_t rowres_max_parts(int64_t m, int64_t n, bool bicgk);   // over every workgroup size
inline int64_t atax_rowres_parts(int64_t m, int64_t n, int threads)
{
    return rowres_parts(m, n, threads, false);
}
inline int64_t atax_rowres_max_parts(int64_t m, int64_t n) { return rowres_max_parts(m, n, false); }
// workgroup sizes of the row-resident sweeps, per size bucket
bool set_rowres_threads(int bucket, int t);            // 256, 512 or 1024
int get_rowres_threads(int bucket);
bool set_bicgk_rowres_threads(int bucket, int t);      // 0 (tile kernel), 256, 512 or 1024
int get_bicgk_rowres_threads(int bucket);
void launch_bicgk_rowres(int64_t m, int64_t n, const double *A, int64_t lda, const double *p,
                         const double *r, double *q, double *P, int threads, hipStream_t st);
void launch_atax_rowres(int64_t m, int64_t n, const double *A, int64_t lda, const double *x,
                        double *P, int threads, hipStream_t st);

}  // namespace bto
