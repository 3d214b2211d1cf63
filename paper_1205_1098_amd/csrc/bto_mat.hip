// Matrix (BLAS-2) kernels over a row-major A: the single-sweep tile
// kernel k_tile (its device templates are in bto_tile.hpp), the fixed-order
// finishes of the partial sums, and the row-resident ATAX and BiCGK sweeps.
//
// Read-only sweeps stream best with wide contiguous workgroup rows (WC*KV*2
// KiB per row); sweeps that also write B stream best with narrow wave rows
// and short bands.  Both families are instantiated below and the shape is a
// run-time choice.

#include <atomic>
#include <mutex>

#include "bto_dev.hpp"
#include "bto_internal.hpp"
#include "bto_tile.hpp"
#include "bto_tuned.hpp"

namespace bto {

namespace {

template <int KV, int D, int WC, int WR, int OPS, bool VEC>
__global__ __launch_bounds__(kWave *WC *WR) void k_tile(TileArgs a, int rb, int rev)
{
    __shared__ double lds[(OPS & (OP_COLSUM | OP_AUX)) ? tile_lds_doubles<KV, WC, WR>() : 1];
    const int64_t band = rev ? (int64_t)gridDim.y - 1 - blockIdx.y : (int64_t)blockIdx.y;
    tile_block<KV, D, WC, WR, OPS, VEC>(a, band, (int64_t)blockIdx.x, rb, lds);
}


bool shape_allowed(int ops, int shape)
{
    if (shape < 0 || shape >= kNumShapes)
        return false;
    // 16 waves of 8-pair lanes cannot hold both row-dot weights and column
    // accumulators in the 128 registers a 1024-thread workgroup allows
    if (shape == 1 && (ops & OP_ROWDOT) && (ops & OP_COLSUM))
        return false;
    const bool writes = ops & OP_UPD1;
    return writes ? shape >= kFirstWriteShape : shape < kFirstWriteShape;
}

template <int KV, int D, int WC, int WR, int OPS>
void launch_tile_t(const char *name, const TileCfg &c, const TileArgs &a, hipStream_t st)
{
    dim3 grid((unsigned)ceil_div(a.n, WC * 128 * KV), (unsigned)ceil_div(a.m, c.rb));
    bool vec = aligned16(a.A) && (a.lda % 2 == 0);
    if (OPS & OP_UPD1)
        vec = vec && aligned16(a.B) && (a.ldb % 2 == 0);
    dim3 block(kWave * WC * WR);
    if (vec)
        launch(name, k_tile<KV, D, WC, WR, OPS, true>, grid, block, st, a, c.rb, c.rev);
    else
        launch(name, k_tile<KV, D, WC, WR, OPS, false>, grid, block, st, a, c.rb, c.rev);
}

template <int OPS>
void launch_tile_ops(const char *name, const TileCfg &c, const TileArgs &a, hipStream_t st)
{
    constexpr bool W = OPS & OP_UPD1;
#define BTO_SHAPE(IDX, KV_, D_, WC_, WR_)                           \
    case IDX:                                                       \
        launch_tile_t<KV_, D_, WC_, WR_, OPS>(name, c, a, st);      \
        return;
    if constexpr (!W) {
        switch (c.shape) {
            BTO_SHAPE(0, 8, 2, 4, 1)
        case 1:
            if constexpr (!((OPS & OP_ROWDOT) && (OPS & OP_COLSUM)))
                launch_tile_t<8, 1, 4, 4, OPS>(name, c, a, st);
            return;
            BTO_SHAPE(2, 4, 2, 8, 2)
            BTO_SHAPE(3, 4, 2, 4, 4)
            BTO_SHAPE(4, 4, 4, 4, 1)
            BTO_SHAPE(5, 8, 2, 4, 2)
        default: return;
        }
    } else {
        switch (c.shape) {
            BTO_SHAPE(6, 2, 2, 1, 4)
            BTO_SHAPE(7, 2, 4, 1, 4)
            BTO_SHAPE(8, 4, 2, 1, 4)
            BTO_SHAPE(9, 4, 4, 1, 4)
            BTO_SHAPE(10, 2, 3, 1, 16)
            BTO_SHAPE(11, 1, 2, 1, 16)
            BTO_SHAPE(12, 1, 4, 1, 8)
            BTO_SHAPE(13, 2, 2, 1, 8)
            BTO_SHAPE(14, 1, 2, 2, 8)
        default: return;
        }
    }
#undef BTO_SHAPE
}

void dispatch_tile(const char *name, int ops, const TileCfg &c, const TileArgs &a, hipStream_t st)
{
    switch (ops) {
    case OP_ROWDOT: launch_tile_ops<OP_ROWDOT>(name, c, a, st); break;
    case OP_COLSUM: launch_tile_ops<OP_COLSUM>(name, c, a, st); break;
    case OP_ROWDOT | OP_COLSUM: launch_tile_ops<OP_ROWDOT | OP_COLSUM>(name, c, a, st); break;
    case OP_UPD1: launch_tile_ops<OP_UPD1>(name, c, a, st); break;
    case OP_UPD1 | OP_UPD2 | OP_COLSUM:
        launch_tile_ops<OP_UPD1 | OP_UPD2 | OP_COLSUM>(name, c, a, st);
        break;
    case OP_UPD1 | OP_UPD2: launch_tile_ops<OP_UPD1 | OP_UPD2>(name, c, a, st); break;
    case OP_UPD1 | OP_UPD2 | OP_ROWDOT:
        launch_tile_ops<OP_UPD1 | OP_UPD2 | OP_ROWDOT>(name, c, a, st);
        break;
    case OP_UPD1 | OP_UPD2 | OP_ROWDOT | OP_COLSUM:
        launch_tile_ops<OP_UPD1 | OP_UPD2 | OP_ROWDOT | OP_COLSUM>(name, c, a, st);
        break;
    case OP_COLSUM | OP_AUX: launch_tile_ops<OP_COLSUM | OP_AUX>(name, c, a, st); break;
    case OP_ROWDOT | OP_AUX: launch_tile_ops<OP_ROWDOT | OP_AUX>(name, c, a, st); break;
    default: break;
    }
}

// The finish of a sweep with a rank-2 correction: every workgroup first adds
// the auxiliary parts (wave 0, lanes in order, then the wave sum), then its
// 64 outputs as in finish_block, then applies the correction.
__global__ __launch_bounds__(256) void k_finish_aux(FinishAux f)
{
    __shared__ double lds[4][64];
    __shared__ double S[2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave == 0) {
        double s1 = 0.0, s2 = 0.0;
        for (int64_t k = lane; k < f.naux; k += kWave) {
            s1 += f.aux[2 * k];
            s2 += f.aux[2 * k + 1];
        }
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        if (lane == 0) {
            S[0] = s1;
            S[1] = s2;
        }
    }
    const FinishJob &j = f.j;
    const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
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
        t = (t + f.c1[idx] * S[0]) + f.c2[idx] * S[1];
        j.out[idx] = j.add ? j.scale * t + j.add[idx] : j.scale * t;
    }
}

__global__ __launch_bounds__(256) void k_finish(FinishJob j0, FinishJob j1, int64_t nb0)
{
    __shared__ double lds[4][64];
    const bool first = blockIdx.x < nb0;
    const int64_t b = first ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - nb0;
    finish_block(first ? j0 : j1, b, lds);
}

// Wave `wave`'s share of sum_k P[k*len + idx], parts [wave*q, (wave+1)*q),
// in increasing k (the split and order of finish_block).
__device__ __forceinline__ double part_share(const double *P, int64_t nparts, int64_t len,
                                             int64_t idx, int wave)
{
    const int64_t q = (nparts + 3) / 4;
    const int64_t k0 = wave * q;
    const int64_t k1 = k0 + q < nparts ? k0 + q : nparts;
    double s = 0.0;
    const double *p = P + idx;
    int64_t k = k0;
    for (; k + 8 <= k1; k += 8) {
        double t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            t[e] = p[(k + e) * len];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            s += t[e];
    }
    for (; k < k1; ++k)
        s += p[k * len];
    return s;
}

// out = scale * sum P + scale2 * sum P2 + add_scale * add: each sum in the
// order of finish_block, the terms added left to right.
__global__ __launch_bounds__(256) void k_finish_lin(FinishLin f)
{
    __shared__ double lds[2][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const FinishJob &j = f.j;
    const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
    double s1 = 0.0, s2 = 0.0;
    if (idx < j.len) {
        s1 = part_share(j.P, j.nparts, j.len, idx, wave);
        if (f.P2)
            s2 = part_share(f.P2, f.nparts2, j.len, idx, wave);
    }
    lds[0][wave][lane] = s1;
    lds[1][wave][lane] = s2;
    lds_barrier();
    if (wave == 0 && idx < j.len) {
        const double t1 = ((lds[0][0][lane] + lds[0][1][lane]) + lds[0][2][lane]) + lds[0][3][lane];
        double v = j.scale * t1;
        if (f.P2) {
            const double t2 =
                ((lds[1][0][lane] + lds[1][1][lane]) + lds[1][2][lane]) + lds[1][3][lane];
            v = v + f.scale2 * t2;
        }
        if (j.add)
            v = v + f.add_scale * j.add[idx];
        j.out[idx] = v;
    }
}

// ---- row-resident sweeps (ATAX, BiCGK) ------------------------------------
//
// Workgroup g owns rows [g*m/G, (g+1)*m/G) and reads each of them once,
// whole: a thread holds NPT doubles of the row, and the same columns of the
// row-dot vector, in registers.  The column sums of its columns accumulate
// in its slice of LDS (only the owner touches a slice: no barrier), so the
// workgroup ends with one partial column-sum vector, added over the
// workgroups by the finish kernel.
//
// ATAX, y = A^T (A x): the max-fuse organism of Section IV-A,
// {p(i){i{j 1}{j 2}}}.  The dot t_i = A_i . x must be complete before the
// row's update y += A_i^T t_i (Section III-D), so it is reduced across the
// workgroup for every row while the row stays on chip.
//
// BiCGK, q = A p and s = A^T r: the column weight r_i does not depend on the
// row's dot, so the update never waits for it.  Each wave parks its partial
// dot of the row in LDS, and the partials of up to kChunk rows are added in
// wave order together (one barrier pair per chunk, not per row).
//
// Register budget: two whole rows (the one being applied and the next one)
// plus the dot vector fill most of it, hence the column sums in LDS.  Rows
// are read with buffer loads: one lane offset in a vector register and the
// pair strides as scalars.  The buffer's range (the even part of the row)
// returns zeros past the row end; an odd last column is added by a scalar
// fix-up.

typedef unsigned int u4 __attribute__((ext_vector_type(4)));
constexpr int kBufferDword3 = 0x00020000;   // raw buffer descriptor word 3 on gfx9
constexpr int kBufferNonTemporal = 2;
constexpr int kChunk = 64;                  // BiCGK rows per row-dot flush

template <int T, bool BICGK>
struct RowresLds {
    static constexpr int NW = T / kWave;
    static constexpr int kRed = BICGK ? kChunk * NW : 2 * NW;
};

template <int T, int NPT, bool VEC, bool ODD, bool BICGK>
__global__ __launch_bounds__(T) void k_rowres(int64_t m, int64_t n, const double *A, int64_t lda,
                                              const double *x, const double *r, double *q,
                                              double *P)
{
    constexpr int NP = NPT / 2;     // pairs per thread
    constexpr int NW = T / kWave;   // waves per workgroup
    constexpr bool odd = VEC && ODD;   // n is odd: one column outside whole pairs
    __shared__ d2 ys[T * NP];
    __shared__ double red[RowresLds<T, BICGK>::kRed];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    d2 xv[NP], bufa[NP], bufb[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        xv[k] = load_vec_pair(x, 2 * (int64_t)(tid + T * k), n);
        ys[tid + T * k] = d2{0.0, 0.0};
        bufa[k] = d2{0.0, 0.0};
        bufb[k] = d2{0.0, 0.0};
    }

    const int64_t G = gridDim.x, g = blockIdx.x;
    const int64_t r0 = g * m / G, r1 = (g + 1) * m / G;
    const int64_t nev = n & ~(int64_t)1;          // columns covered by whole pairs
    const double xlast = odd ? x[n - 1] : 0.0;
    // the thread and pair slot that own column n-1 when n is odd
    const int64_t plast = (n - 1) / 2;
    const bool own_last = odd && tid == (int)(plast % T);
    const int klast = (int)(plast / T);
    double lasta = 0.0, lastb = 0.0;   // A(i, n-1) when n is odd
    double wa = 0.0, wb = 0.0;         // BiCGK: the row's column weight r_i

    auto load_row = [&](int64_t i, d2 (&dst)[NP], double &last, double &wgt) {
        const double *row = A + i * lda;
        if constexpr (BICGK)
            wgt = ld_uniform(r + i);
        if constexpr (VEC) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<double *>(row), 0, (int)(nev * 8), kBufferDword3);
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, tid * 16, k * T * 16,
                                                                   kBufferNonTemporal);
                dst[k] = __builtin_bit_cast(d2, v);
            }
            if constexpr (odd)
                last = ld_uniform(row + n - 1);
        } else {
#pragma unroll
            for (int k = 0; k < NP; ++k)
                dst[k] = load_pair<false, false>(row, 2 * (int64_t)(tid + T * k), n);
        }
    };

    // BiCGK row-dot bookkeeping: rows [rbase, rbase + cnt) have parked partials
    int64_t rbase = r0;
    int cnt = 0;
    auto flush = [&]() {
        lds_barrier();
        if (tid < cnt) {
            double sum = red[tid * NW];
#pragma unroll
            for (int w = 1; w < NW; ++w)
                sum += red[tid * NW + w];
            q[rbase + tid] = sum;
        }
        lds_barrier();
        rbase += cnt;
        cnt = 0;
    };

    auto process = [&](int64_t i, const d2 (&cur)[NP], double last, double w_row) {
        double part = 0.0;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            part += cur[k].x * xv[k].x;
            part += cur[k].y * xv[k].y;
        }
        part = wave_sum(part);
        double t;
        if constexpr (BICGK) {
            if constexpr (odd) {
                if (wave == 0)
                    part += last * xlast;
            }
            if (lane == 0)
                red[cnt * NW + wave] = part;
            t = w_row;
        } else {
            const int buf = (int)(i & 1);
            if (lane == 0)
                red[buf * NW + wave] = part;
            lds_barrier();
            // lane w < NW takes wave w's sum and a butterfly adds them: every
            // wave gets the same t from the same fixed tree
            t = lane < NW ? red[buf * NW + lane] : 0.0;
            t = wave_sum(t);
            if constexpr (odd)
                t += last * xlast;
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            d2 yv = ys[tid + T * k];
            yv += cur[k] * t;
            if constexpr (odd) {
                if (own_last && k == klast)
                    yv.x += last * t;
            }
            ys[tid + T * k] = yv;
            if (k % 2 == 1)
                __builtin_amdgcn_sched_barrier(0);   // at most two y pairs in flight
        }
        if constexpr (BICGK) {
            if (++cnt == kChunk)
                flush();
        }
    };
    // two row buffers used in turn: the next row is always in flight while
    // the current one is reduced and applied (the scheduling barriers stop
    // the compiler from hoisting a buffer's reload above the update that
    // still reads it, which would need a third row of registers)
    // Inside the loop every load is unconditional, so the compiler can count
    // exactly which loads a wait must cover; the last one or two rows are
    // peeled off after it.
    int64_t i = r0;
    if (i < r1)
        load_row(i, bufa, lasta, wa);
    for (; i + 2 < r1; i += 2) {
        load_row(i + 1, bufb, lastb, wb);
        __builtin_amdgcn_sched_barrier(0);
        process(i, bufa, lasta, wa);
        __builtin_amdgcn_sched_barrier(0);
        load_row(i + 2, bufa, lasta, wa);
        __builtin_amdgcn_sched_barrier(0);
        process(i + 1, bufb, lastb, wb);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (i + 1 < r1) {
        load_row(i + 1, bufb, lastb, wb);
        __builtin_amdgcn_sched_barrier(0);
        process(i, bufa, lasta, wa);
        __builtin_amdgcn_sched_barrier(0);
        process(i + 1, bufb, lastb, wb);
    } else if (i < r1) {
        process(i, bufa, lasta, wa);
    }
    if constexpr (BICGK) {
        if (cnt > 0)
            flush();
    }

    double *out = P + g * n;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int64_t j = 2 * (int64_t)(tid + T * k);
        const d2 yv = ys[tid + T * k];
        if (j < n) out[j] = yv.x;
        if (j + 1 < n) out[j + 1] = yv.y;
    }
}

struct RowresShape {
    int T, NPT;
};

// preferred workgroup size of the row-resident sweeps per size bucket
// (tunable); for BiCGK 0 selects the tile kernel
const int kAtaxRowresDefaults[kSizeBuckets] = BTO_TUNED_ATAX_ROWRES;
const int kBicgkRowresDefaults[kSizeBuckets] = BTO_TUNED_BICGK_ROWRES;
std::atomic<int> g_rowres_threads[kSizeBuckets];
std::atomic<int> g_bicgk_rowres_threads[kSizeBuckets];
std::once_flag g_rowres_once;

void rowres_init()
{
    std::call_once(g_rowres_once, [] {
        for (int b = 0; b < kSizeBuckets; ++b) {
            g_rowres_threads[b] = kAtaxRowresDefaults[b];
            g_bicgk_rowres_threads[b] = kBicgkRowresDefaults[b];
        }
    });
}

// The workgroup size T (the preferred one first) and the fewest doubles per
// thread NPT (even) with T*NPT >= n.
RowresShape rowres_shape(int64_t n, int threads)
{
    static const int npts[] = {2, 4, 8, 16, 32};
    const int order[3][3] = {{1024, 512, 256}, {512, 1024, 256}, {256, 512, 1024}};
    const int *pref = threads == 1024 ? order[0] : (threads == 512 ? order[1] : order[2]);
    for (int o = 0; o < 3; ++o) {
        const int T = pref[o];
        for (int npt : npts) {
            if (T == 1024 && npt > 16)
                continue;   // two rows and y would not fit 128 registers
            if ((int64_t)T * npt >= n)
                return {T, npt};
        }
    }
    return {0, 0};
}

int rowres_blocks_per_cu(const RowresShape &s, bool bicgk)
{
    // LDS holds the workgroup's column sums (T*NPT doubles) and the row-dot
    // exchange; at most 160 KiB per CU.
    const int64_t red = 8 * (int64_t)(s.T / kWave) * (bicgk ? kChunk : 2);
    int by_lds = (int)(160 * 1024 / ((int64_t)s.T * s.NPT * 8 + red + 16));
    int by_threads = 2048 / s.T;
    int b = by_lds < by_threads ? by_lds : by_threads;
    return b < 1 ? 1 : b;
}

constexpr int kCUs = 256;


}  // namespace

bool tile_cfg_supported(int ops, const TileCfg &c)
{
    if (!shape_allowed(ops, c.shape) || (c.rev != 0 && c.rev != 1))
        return false;
    const Shape &s = kShapes[c.shape];
    if (c.rb < s.wr || c.rb % s.wr != 0 || c.rb > 4096)
        return false;
    // row-dot results are gathered one row per lane: at most 64 rows per wave
    if ((ops & OP_ROWDOT) && c.rb / s.wr > kWave)
        return false;
    // rb >= 32 keeps the column-sum partials within the workspace the C
    // entry points size for (at most ceil(m / 32) row bands)
    if ((ops & OP_COLSUM) && c.rb < 32)
        return false;
    return true;
}

int tile_kv(const TileCfg &c) { return kShapes[c.shape].kv; }

void tile_shape_info(int shape, int out[4])
{
    const Shape &s = kShapes[shape];
    out[0] = s.kv;
    out[1] = s.d;
    out[2] = s.wc;
    out[3] = s.wr;
}

int64_t tile_ncols(const TileCfg &c, int64_t n) { return ceil_div(n, 128 * kShapes[c.shape].kv); }

// The grid's y extent holds at most 65535 row bands.  A configuration whose
// bands are too short for m gets taller ones (a multiple of its row groups):
// a row's dot partials and the column sums' band count as seen by the caller
// do not change, since column-sum sweeps already use bands of 32 rows or more
// and the entry points refuse more than 65535 * 32 rows.
TileCfg fit_grid(TileCfg c, int64_t m)
{
    const int64_t need = ceil_div(m, 65535);
    if (c.rb < need) {
        const int wr = kShapes[c.shape].wr;
        c.rb = (int)(ceil_div(need, wr) * wr);
    }
    return c;
}

bool launch_tile(const char *name, int ops, const TileCfg &c, const TileArgs &a, hipStream_t st)
{
    if (!tile_cfg_supported(ops, c))
        return false;
    if (a.m <= 0 || a.n <= 0)
        return true;
    dispatch_tile(name, ops, fit_grid(c, a.m), a, st);
    return true;
}

void launch_finish_lin(const char *name, const FinishLin &f, hipStream_t st)
{
    const int64_t nb = ceil_div(f.j.len, 64);
    if (nb > 0)
        launch(name, k_finish_lin, dim3((unsigned)nb), dim3(256), st, f);
}

void launch_finish_aux(const char *name, const FinishAux &f, hipStream_t st)
{
    const int64_t nb = ceil_div(f.j.len, 64);
    if (nb > 0)
        launch(name, k_finish_aux, dim3((unsigned)nb), dim3(256), st, f);
}

void launch_finish(const char *name, const FinishJob &j0, const FinishJob &j1, hipStream_t st)
{
    const int64_t nb0 = ceil_div(j0.len, 64), nb1 = ceil_div(j1.len, 64);
    launch(name, k_finish, dim3((unsigned)(nb0 + nb1)), dim3(256), st, j0, j1, nb0);
}

bool set_rowres_threads(int bucket, int t)
{
    if (t != 256 && t != 512 && t != 1024)
        return false;
    rowres_init();
    g_rowres_threads[bucket] = t;
    return true;
}

int get_rowres_threads(int bucket)
{
    rowres_init();
    return g_rowres_threads[bucket].load();
}

bool set_bicgk_rowres_threads(int bucket, int t)
{
    if (t != 0 && t != 256 && t != 512 && t != 1024)
        return false;
    rowres_init();
    g_bicgk_rowres_threads[bucket] = t;
    return true;
}

int get_bicgk_rowres_threads(int bucket)
{
    rowres_init();
    return g_bicgk_rowres_threads[bucket].load();
}

// Workgroups of a row-resident sweep: as many as fit at once, but no more
// than give each at least kMinRowsPerGroup rows (each writes an n-long
// partial that the finish reads back: with one row apiece the partials
// would weigh as much as the matrix) unless that leaves a compute unit
// idle, and never more than m.
constexpr int64_t kMinRowsPerGroup = 16;

static int64_t rowres_parts_for(int64_t m, const RowresShape &s, bool bicgk)
{
    if (s.T == 0 || m <= 0)
        return 0;
    int64_t g = (int64_t)kCUs * rowres_blocks_per_cu(s, bicgk);
    int64_t want = ceil_div(m, kMinRowsPerGroup);
    want = want < kCUs ? kCUs : want;
    g = g < want ? g : want;
    return g < m ? g : m;
}

int64_t rowres_parts(int64_t m, int64_t n, int threads, bool bicgk)
{
    if (n <= 0 || threads == 0)
        return 0;
    return rowres_parts_for(m, rowres_shape(n, threads), bicgk);
}

int64_t rowres_max_parts(int64_t m, int64_t n, bool bicgk)
{
    if (n <= 0)
        return 0;
    int64_t best = 0;
    for (int t : {256, 512, 1024}) {
        const int64_t p = rowres_parts_for(m, rowres_shape(n, t), bicgk);
        best = p > best ? p : best;
    }
    return best;
}

template <int T_, int NPT_, bool BICGK>
static void launch_rowres_shape(int64_t G, int64_t m, int64_t n, const double *A, int64_t lda,
                                const double *x, const double *r, double *q, double *P,
                                hipStream_t st)
{
    const char *name = BICGK ? "bicgk_rowres" : "atax_rowres";
    const dim3 g((unsigned)G), b(T_);
    const bool vec = aligned16(A) && lda % 2 == 0;
    if (vec && (n & 1))
        launch(name, k_rowres<T_, NPT_, true, true, BICGK>, g, b, st, m, n, A, lda, x, r, q, P);
    else if (vec)
        launch(name, k_rowres<T_, NPT_, true, false, BICGK>, g, b, st, m, n, A, lda, x, r, q, P);
    else
        launch(name, k_rowres<T_, NPT_, false, false, BICGK>, g, b, st, m, n, A, lda, x, r, q,
               P);
}

template <bool BICGK>
static void launch_rowres(int64_t m, int64_t n, const double *A, int64_t lda, const double *x,
                          const double *r, double *q, double *P, int threads, hipStream_t st)
{
    const RowresShape s = rowres_shape(n, threads);
    const int64_t G = rowres_parts(m, n, threads, BICGK);
    if (G == 0)
        return;
#define BTO_ROWRES_CASE(T_, NPT_)                                                   \
    if (s.T == T_ && s.NPT == NPT_)                                                 \
        return launch_rowres_shape<T_, NPT_, BICGK>(G, m, n, A, lda, x, r, q, P, st);
    BTO_ROWRES_CASE(256, 2)
    BTO_ROWRES_CASE(256, 4)
    BTO_ROWRES_CASE(256, 8)
    BTO_ROWRES_CASE(256, 16)
    BTO_ROWRES_CASE(256, 32)
    BTO_ROWRES_CASE(512, 2)
    BTO_ROWRES_CASE(512, 4)
    BTO_ROWRES_CASE(512, 8)
    BTO_ROWRES_CASE(512, 16)
    BTO_ROWRES_CASE(512, 32)
    BTO_ROWRES_CASE(1024, 2)
    BTO_ROWRES_CASE(1024, 4)
    BTO_ROWRES_CASE(1024, 8)
    BTO_ROWRES_CASE(1024, 16)
#undef BTO_ROWRES_CASE
}

void launch_atax_rowres(int64_t m, int64_t n, const double *A, int64_t lda, const double *x,
                        double *P, int threads, hipStream_t st)
{
    launch_rowres<false>(m, n, A, lda, x, nullptr, nullptr, P, threads, st);
}

void launch_bicgk_rowres(int64_t m, int64_t n, const double *A, int64_t lda, const double *p,
                         const double *r, double *q, double *P, int threads, hipStream_t st)
{
    launch_rowres<true>(m, n, A, lda, p, r, q, P, threads, st);
}

}  // namespace bto
