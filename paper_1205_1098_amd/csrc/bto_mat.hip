// Matrix (BLAS-2) kernels over a row-major A.
//
// k_tile is one sweep of A in 2-D tiles (a column tile of 128*KV columns by
// a band of rb rows per 4-wave workgroup).  Each lane owns KV 16-byte column
// pairs of the tile for the whole band, so the per-column vectors it needs
// (the row-dot weights, v1, v2, the column-sum accumulators) live in
// registers and A streams through once.  Depending on OPS one sweep
//   - forms B = A + u1 v1^T (+ u2 v2^T) and stores it          (OP_UPD1/2)
//   - accumulates the row dots  sum_j B_ij xr_j  per column tile (OP_ROWDOT)
//   - accumulates the column sums sum_i B_ij yc_i per row band   (OP_COLSUM)
// where B is A when no update is asked for.  This is the fused loop nest
// {p(i){i{j ...}}} of Section III-C with the row-band partition p(i) across
// workgroups and the column tile across lanes.  Row-dot partials land in
// Prow[column tile][row], column-sum partials in Pcol[row band][column];
// k_finish reduces them in a fixed order.

#include "bto_dev.hpp"
#include "bto_internal.hpp"

namespace bto {

namespace {

constexpr int kTileThreads = 256;

// Load the 16-byte pair of row `row` at column j (masked past n).
template <bool VEC, bool FULL>
__device__ __forceinline__ d2 load_pair(const double *row, int64_t j, int64_t n)
{
    if constexpr (FULL && VEC) {
        return ld2_nt(row + j);
    } else if constexpr (FULL) {
        return d2{ld1_nt(row + j), ld1_nt(row + j + 1)};
    } else {
        d2 r{0.0, 0.0};
        if (j < n) r.x = ld1_nt(row + j);
        if (j + 1 < n) r.y = ld1_nt(row + j + 1);
        return r;
    }
}

template <bool VEC, bool FULL>
__device__ __forceinline__ void store_pair(double *row, int64_t j, int64_t n, d2 v)
{
    if constexpr (FULL && VEC) {
        st2_nt(row + j, v);
    } else if constexpr (FULL) {
        st1_nt(row + j, v.x);
        st1_nt(row + j + 1, v.y);
    } else {
        if (j < n) st1_nt(row + j, v.x);
        if (j + 1 < n) st1_nt(row + j + 1, v.y);
    }
}

__device__ __forceinline__ d2 load_vec_pair(const double *v, int64_t j, int64_t n)
{
    d2 r{0.0, 0.0};
    if (j < n) r.x = v[j];
    if (j + 1 < n) r.y = v[j + 1];
    return r;
}

template <int KV, int RU, int OPS, bool VEC, bool FULL>
__device__ __forceinline__ void tile_body(const TileArgs &a, int64_t ct, int64_t rb, int rbrows,
                                          double *lds)
{
    constexpr bool ROWDOT = OPS & OP_ROWDOT;
    constexpr bool COLSUM = OPS & OP_COLSUM;
    constexpr bool UPD1 = OPS & OP_UPD1;
    constexpr bool UPD2 = OPS & OP_UPD2;
    constexpr int CT = 128 * KV;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t c0 = ct * CT;
    const int64_t n = a.n;

    d2 xr[KV], v1[KV], v2[KV], acc[KV];
#pragma unroll
    for (int k = 0; k < KV; ++k) {
        const int64_t j = c0 + 2 * (lane + kWave * k);
        acc[k] = d2{0.0, 0.0};
        if (ROWDOT) xr[k] = load_vec_pair(a.xr, j, n);
        if (UPD1) v1[k] = load_vec_pair(a.v1, j, n);
        if (UPD2) v2[k] = load_vec_pair(a.v2, j, n);
    }

    const int rpw = rbrows >> 2;  // rows per wave
    const int64_t r0 = rb * rbrows + (int64_t)wave * rpw;
    const int64_t r1 = r0 + rpw < a.m ? r0 + rpw : a.m;
    double mine = 0.0;

    for (int64_t i0 = r0; i0 < r1; i0 += RU) {
        d2 v[RU][KV];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t i = i0 + u;
            const double *row = a.A + i * a.lda;
#pragma unroll
            for (int k = 0; k < KV; ++k) {
                const int64_t j = c0 + 2 * (lane + kWave * k);
                v[u][k] = (i < r1) ? load_pair<VEC, FULL>(row, j, n) : d2{0.0, 0.0};
            }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int64_t i = i0 + u;
            if (i >= r1)
                break;
            if (UPD1) {
                const double s1 = a.u1[i];
                const double s2 = UPD2 ? a.u2[i] : 0.0;
                double *brow = a.B + i * a.ldb;
#pragma unroll
                for (int k = 0; k < KV; ++k) {
                    d2 b = v[u][k] + s1 * v1[k];
                    if (UPD2) b = b + s2 * v2[k];
                    v[u][k] = b;
                    store_pair<VEC, FULL>(brow, c0 + 2 * (lane + kWave * k), n, b);
                }
            }
            if (COLSUM) {
                const double yi = a.yc[i];
#pragma unroll
                for (int k = 0; k < KV; ++k)
                    acc[k] += v[u][k] * yi;
            }
            if (ROWDOT) {
                double p = 0.0;
#pragma unroll
                for (int k = 0; k < KV; ++k) {
                    p += v[u][k].x * xr[k].x;
                    p += v[u][k].y * xr[k].y;
                }
                p = wave_sum(p);
                if (lane == (int)(i - r0))
                    mine = p;
            }
        }
    }

    if (ROWDOT) {
        if (lane < r1 - r0)
            a.Prow[ct * a.m + r0 + lane] = mine;
    }
    if (COLSUM) {
        // combine the four waves' column sums in wave order
#pragma unroll
        for (int k = 0; k < KV; ++k) {
            const int c = 2 * (lane + kWave * k);
            lds[wave * CT + c] = acc[k].x;
            lds[wave * CT + c + 1] = acc[k].y;
        }
        lds_barrier();
        for (int c = threadIdx.x; c < CT; c += kTileThreads) {
            const int64_t j = c0 + c;
            if (j < n) {
                double s = ((lds[c] + lds[CT + c]) + lds[2 * CT + c]) + lds[3 * CT + c];
                a.Pcol[rb * n + j] = s;
            }
        }
    }
}

template <int KV, int RU, int OPS, bool VEC>
__global__ __launch_bounds__(kTileThreads) void k_tile(TileArgs a, int rbrows, int rev)
{
    __shared__ double lds[(OPS & OP_COLSUM) ? 4 * 128 * KV : 1];
    const int64_t ct = blockIdx.x;
    const int64_t rb = rev ? (int64_t)gridDim.y - 1 - blockIdx.y : (int64_t)blockIdx.y;
    const bool full = (ct + 1) * (128 * KV) <= a.n;
    if (full)
        tile_body<KV, RU, OPS, VEC, true>(a, ct, rb, rbrows, lds);
    else
        tile_body<KV, RU, OPS, VEC, false>(a, ct, rb, rbrows, lds);
}

template <int KV, int RU, int OPS>
void launch_tile_t(const char *name, const TileCfg &c, const TileArgs &a, hipStream_t st)
{
    dim3 grid((unsigned)tile_ncols(c, a.n), (unsigned)tile_nbands(c, a.m));
    bool vec = aligned16(a.A) && (a.lda % 2 == 0);
    if (OPS & OP_UPD1)
        vec = vec && aligned16(a.B) && (a.ldb % 2 == 0);
    if (vec)
        launch(name, k_tile<KV, RU, OPS, true>, grid, dim3(kTileThreads), st, a, c.rb, c.rev);
    else
        launch(name, k_tile<KV, RU, OPS, false>, grid, dim3(kTileThreads), st, a, c.rb, c.rev);
}

template <int OPS>
bool launch_tile_ops(const char *name, const TileCfg &c, const TileArgs &a, hipStream_t st)
{
#define BTO_TILE_CASE(KV_, RU_)                                       \
    if (c.kv == KV_ && c.ru == RU_) {                                 \
        if (st != (hipStream_t)-1)                                    \
            launch_tile_t<KV_, RU_, OPS>(name, c, a, st);             \
        return true;                                                  \
    }
    BTO_TILE_CASE(2, 2)
    BTO_TILE_CASE(2, 4)
    BTO_TILE_CASE(4, 2)
    BTO_TILE_CASE(4, 4)
    BTO_TILE_CASE(8, 1)
    BTO_TILE_CASE(8, 2)
#undef BTO_TILE_CASE
    return false;
}

bool dispatch_tile(const char *name, int ops, const TileCfg &c, const TileArgs &a, hipStream_t st)
{
    switch (ops) {
    case OP_ROWDOT: return launch_tile_ops<OP_ROWDOT>(name, c, a, st);
    case OP_COLSUM: return launch_tile_ops<OP_COLSUM>(name, c, a, st);
    case OP_ROWDOT | OP_COLSUM: return launch_tile_ops<OP_ROWDOT | OP_COLSUM>(name, c, a, st);
    case OP_UPD1: return launch_tile_ops<OP_UPD1>(name, c, a, st);
    case OP_UPD1 | OP_UPD2 | OP_COLSUM:
        return launch_tile_ops<OP_UPD1 | OP_UPD2 | OP_COLSUM>(name, c, a, st);
    default: return false;
    }
}

// ---- fixed-order reduction of partials -----------------------------------
//
// One workgroup per 64 outputs: wave w sums parts [w*q, (w+1)*q) of each of
// its lane's outputs sequentially (q = ceil(nparts/4)), then wave 0 adds
// the four wave sums in order and applies the epilogue.

__global__ __launch_bounds__(256) void k_finish(FinishJob j0, FinishJob j1, int64_t nb0)
{
    __shared__ double lds[4][64];
    const bool first = blockIdx.x < nb0;
    const FinishJob &j = first ? j0 : j1;
    const int64_t b = first ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - nb0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t idx = b * 64 + lane;
    const int64_t q = (j.nparts + 3) / 4;
    const int64_t k0 = wave * q;
    const int64_t k1 = k0 + q < j.nparts ? k0 + q : j.nparts;
    double s = 0.0;
    if (idx < j.len) {
        const double *p = j.P + idx;
        int64_t k = k0;
        for (; k + 8 <= k1; k += 8) {
            double t[8];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                t[e] = p[(k + e) * j.len];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                s += t[e];
        }
        for (; k < k1; ++k)
            s += p[k * j.len];
    }
    lds[wave][lane] = s;
    lds_barrier();
    if (wave == 0 && idx < j.len) {
        double t = ((lds[0][lane] + lds[1][lane]) + lds[2][lane]) + lds[3][lane];
        j.out[idx] = j.add ? j.scale * t + j.add[idx] : j.scale * t;
    }
}

// ---- row-resident ATAX ----------------------------------------------------
//
// y = A^T (A x) in one sweep of A: workgroup g owns rows [g*m/G, (g+1)*m/G).
// For each row it loads the whole row into registers (NPT doubles per
// thread), reduces t_i = A_i . x across the workgroup, and updates its
// register copy of y with A_i^T t_i while the next row is already in
// flight.  x sits in LDS.  This is the max-fuse organism of Section IV-A,
// {p(i){i{j 1}{j 2}}}: the t_i reduction must finish before the update
// (Section III-D), so the row stays on chip in between.

template <int T, int NPT, bool VEC>
__global__ __launch_bounds__(T) void k_atax_rowres(int64_t m, int64_t n, const double *A,
                                                   int64_t lda, const double *x, double *P)
{
    constexpr int NP = NPT / 2;     // pairs per thread
    constexpr int NW = T / kWave;   // waves per workgroup
    __shared__ d2 xs[T * NP];
    __shared__ double red[2][NW];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int p = tid; p < T * NP; p += T)
        xs[p] = load_vec_pair(x, 2 * (int64_t)p, n);
    lds_barrier();

    const int64_t G = gridDim.x, g = blockIdx.x;
    const int64_t r0 = g * m / G, r1 = (g + 1) * m / G;

    d2 yacc[NP], cur[NP], nxt[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        yacc[k] = d2{0.0, 0.0};
        cur[k] = d2{0.0, 0.0};
        nxt[k] = d2{0.0, 0.0};
    }
    auto load_row = [&](int64_t i, d2 *dst) {
        const double *row = A + i * lda;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int64_t j = 2 * (int64_t)(tid + T * k);
            if (VEC && j + 1 < n)
                dst[k] = ld2_nt(row + j);
            else
                dst[k] = load_pair<false, false>(row, j, n);
        }
    };
    if (r0 < r1)
        load_row(r0, cur);
    for (int64_t i = r0; i < r1; ++i) {
        if (i + 1 < r1)
            load_row(i + 1, nxt);
        double part = 0.0;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const d2 xv = xs[tid + T * k];
            part += cur[k].x * xv.x;
            part += cur[k].y * xv.y;
        }
        part = wave_sum(part);
        const int buf = (int)(i & 1);
        if (lane == 0)
            red[buf][wave] = part;
        lds_barrier();
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w)
            t += red[buf][w];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            yacc[k] += cur[k] * t;
            cur[k] = nxt[k];
        }
    }
    double *out = P + g * n;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int64_t j = 2 * (int64_t)(tid + T * k);
        if (j < n) out[j] = yacc[k].x;
        if (j + 1 < n) out[j + 1] = yacc[k].y;
    }
}

struct RowresShape {
    int T, NPT;
};

// The narrowest (threads, doubles per thread) pair that covers n; T*NPT >= n.
RowresShape rowres_shape(int64_t n)
{
    static const RowresShape shapes[] = {{256, 2}, {256, 4}, {256, 8}, {512, 8}, {1024, 8}, {1024, 16}};
    for (const RowresShape &s : shapes)
        if ((int64_t)s.T * s.NPT >= n)
            return s;
    return {0, 0};
}

int rowres_blocks_per_cu(const RowresShape &s)
{
    // LDS holds x (T*NPT doubles); at most 160 KiB per CU.
    int by_lds = (int)(160 * 1024 / ((int64_t)s.T * s.NPT * 8 + 64));
    int by_threads = 2048 / s.T;
    int b = by_lds < by_threads ? by_lds : by_threads;
    return b < 1 ? 1 : b;
}

constexpr int kCUs = 256;

}  // namespace

bool tile_cfg_supported(int ops, const TileCfg &c)
{
    // rb >= 32 keeps the column-sum partials within the workspace the C
    // entry points size for (at most ceil(m / 32) row bands)
    if (c.rb < 32 || c.rb > 256 || c.rb % 4 != 0 || (c.rev != 0 && c.rev != 1))
        return false;
    return dispatch_tile("", ops, c, TileArgs{}, (hipStream_t)-1);
}

void launch_tile(const char *name, int ops, const TileCfg &c, const TileArgs &a, hipStream_t st)
{
    if (a.m <= 0 || a.n <= 0)
        return;
    dispatch_tile(name, ops, c, a, st);
}

void launch_finish(const char *name, const FinishJob &j0, const FinishJob &j1, hipStream_t st)
{
    const int64_t nb0 = ceil_div(j0.len, 64), nb1 = ceil_div(j1.len, 64);
    launch(name, k_finish, dim3((unsigned)(nb0 + nb1)), dim3(256), st, j0, j1, nb0);
}

int64_t atax_rowres_parts(int64_t m, int64_t n)
{
    RowresShape s = rowres_shape(n);
    if (s.T == 0 || m <= 0 || n <= 0)
        return 0;
    int64_t g = (int64_t)kCUs * rowres_blocks_per_cu(s);
    return g < m ? g : m;
}

void launch_atax_rowres(int64_t m, int64_t n, const double *A, int64_t lda, const double *x,
                        double *P, hipStream_t st)
{
    RowresShape s = rowres_shape(n);
    const int64_t G = atax_rowres_parts(m, n);
    if (G == 0)
        return;
    const bool vec = aligned16(A) && lda % 2 == 0;
#define BTO_ROWRES_CASE(T_, NPT_)                                                             \
    if (s.T == T_ && s.NPT == NPT_) {                                                         \
        if (vec)                                                                              \
            launch("atax_rowres", k_atax_rowres<T_, NPT_, true>, dim3((unsigned)G), dim3(T_), \
                   st, m, n, A, lda, x, P);                                                   \
        else                                                                                  \
            launch("atax_rowres", k_atax_rowres<T_, NPT_, false>, dim3((unsigned)G),          \
                   dim3(T_), st, m, n, A, lda, x, P);                                         \
        return;                                                                               \
    }
    BTO_ROWRES_CASE(256, 2)
    BTO_ROWRES_CASE(256, 4)
    BTO_ROWRES_CASE(256, 8)
    BTO_ROWRES_CASE(512, 8)
    BTO_ROWRES_CASE(1024, 8)
    BTO_ROWRES_CASE(1024, 16)
#undef BTO_ROWRES_CASE
}

}  // namespace bto
