// Device templates of the matrix tile sweeps, shared by the single-sweep
// kernels (bto_mat.hip) and the tiled batches (bto_btile.hip).
//
// A tile sweep reads a row-major A in 2-D tiles.  A workgroup is WC x WR
// waves: the WC waves of a row group sit side by side across the columns
// (each owns a wave tile of 128*KV columns, i.e. KV 16-byte pairs per lane),
// the WR row groups split the workgroup's band of rb rows.  Each lane keeps
// the per-column vectors of its columns in registers for the whole band
// (the row-dot weights, v1, v2, the column-sum accumulators), so A streams
// through exactly once, with D rows of loads kept in flight per wave.
// Depending on OPS one sweep
//   - forms B = A + u1 v1^T (+ u2 v2^T) and stores it          (OP_UPD1/2)
//   - accumulates the row dots  sum_j B_ij xr_j  per wave tile  (OP_ROWDOT)
//   - accumulates the column sums sum_i B_ij yc_i per row band  (OP_COLSUM)
// where B is A when no update is asked for.  This is the fused loop nest
// {p(i){i{j ...}}} of Section III-C: the row-band partition p(i) runs across
// workgroups, the columns across lanes.  Row-dot partials land in
// Prow[wave tile][row], column-sum partials in Pcol[row band][column]; a
// finish reduces them in a fixed order.
#pragma once

#include "bto_dev.hpp"
#include "bto_internal.hpp"

namespace bto {

namespace {

// Load the 16-byte pair of row `row` at column j (masked past n).
template <bool VEC, bool FULL>
__device__ __forceinline__ d2 load_pair(const double *row, int64_t j, int64_t n)
{
    if constexpr (FULL && VEC) {
        return ld2_nt(row + j);
    } else if constexpr (FULL) {
        return d2{ld1_nt(row + j), ld1_nt(row + j + 1)};
    } else if constexpr (VEC) {
        // rows start 16-byte aligned and j is even: a pair inside the row is
        // one 16-byte access, only an odd last column is read alone
        if (j + 1 < n)
            return ld2_nt(row + j);
        d2 r{0.0, 0.0};
        if (j < n) r.x = ld1_nt(row + j);
        return r;
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
    } else if constexpr (VEC) {
        if (j + 1 < n)
            st2_nt(row + j, v);
        else if (j < n)
            st1_nt(row + j, v.x);
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

// One wave's sweep over rows [r0, r1) of its wave tile starting at column c0.
template <int KV, int D, int OPS, bool VEC, bool FULL>
__device__ __forceinline__ void tile_rows(const TileArgs &a, int64_t c0, int64_t r0, int64_t r1,
                                          int lane, d2 (&acc)[KV], double &mine)
{
    constexpr bool ROWDOT = OPS & OP_ROWDOT;
    constexpr bool COLSUM = OPS & OP_COLSUM;
    constexpr bool UPD1 = OPS & OP_UPD1;
    constexpr bool UPD2 = OPS & OP_UPD2;
    const int64_t n = a.n;

    d2 xr[KV], v1[KV], v2[KV];
#pragma unroll
    for (int k = 0; k < KV; ++k) {
        const int64_t j = c0 + 2 * (lane + kWave * k);
        if (ROWDOT) xr[k] = load_vec_pair(a.xr, j, n);
        if (UPD1) v1[k] = load_vec_pair(a.v1, j, n);
        if (UPD2) v2[k] = load_vec_pair(a.v2, j, n);
    }

    auto load_row = [&](int64_t i, d2 (&dst)[KV]) {
        const double *row = a.A + i * a.lda;
#pragma unroll
        for (int k = 0; k < KV; ++k)
            dst[k] = load_pair<VEC, FULL>(row, c0 + 2 * (lane + kWave * k), n);
    };

    d2 ring[D][KV];
#pragma unroll
    for (int q = 0; q < D; ++q) {
        if (r0 + q < r1) {
            load_row(r0 + q, ring[q]);
        } else {
#pragma unroll
            for (int k = 0; k < KV; ++k)
                ring[q][k] = d2{0.0, 0.0};
        }
    }

    for (int64_t i0 = r0; i0 < r1; i0 += D) {
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const int64_t i = i0 + q;
            if (i >= r1)
                break;
            d2 v[KV];
#pragma unroll
            for (int k = 0; k < KV; ++k)
                v[k] = ring[q][k];
            if (i + D < r1)
                load_row(i + D, ring[q]);
            if (UPD1) {
                const double s1 = ld_uniform(a.u1 + i);
                const double s2 = UPD2 ? ld_uniform(a.u2 + i) : 0.0;
                double *brow = a.B + i * a.ldb;
#pragma unroll
                for (int k = 0; k < KV; ++k) {
                    d2 b = v[k] + s1 * v1[k];
                    if (UPD2) b = b + s2 * v2[k];
                    v[k] = b;
                    store_pair<VEC, FULL>(brow, c0 + 2 * (lane + kWave * k), n, b);
                }
            }
            if (COLSUM) {
                const double yi = ld_uniform(a.yc + i);
#pragma unroll
                for (int k = 0; k < KV; ++k)
                    acc[k] += v[k] * yi;
            }
            if (ROWDOT) {
                double p = 0.0;
#pragma unroll
                for (int k = 0; k < KV; ++k) {
                    p += v[k].x * xr[k].x;
                    p += v[k].y * xr[k].y;
                }
                p = wave_sum(p);
                if (lane == (int)(i - r0))
                    mine = p;
            }
        }
    }
}

// LDS of one workgroup tile: the WR row groups' column sums, then two
// doubles per row group for the auxiliary dots.
template <int KV, int WC, int WR>
constexpr int tile_lds_doubles() { return WR > 1 ? WR * WC * 128 * KV + 2 * WR : 2 * WR; }

// One workgroup tile: row band `band` (rows [band*rb, band*rb + rb)) and
// column block `cblk` (WC wave tiles) of the sweep described by `a`.
template <int KV, int D, int WC, int WR, int OPS, bool VEC>
__device__ __forceinline__ void tile_block(const TileArgs &a, int64_t band, int64_t cblk, int rb,
                                           double *lds)
{
    constexpr bool ROWDOT = OPS & OP_ROWDOT;
    constexpr bool COLSUM = OPS & OP_COLSUM;
    constexpr int CTW = 128 * KV;          // wave tile width (columns)
    constexpr int CTB = WC * CTW;          // workgroup tile width
    constexpr int NT = kWave * WC * WR;    // threads

    // The wave index is uniform across the wave; saying so keeps every row
    // index scalar, so the per-row scalars (u1[i], y[i], ...) become scalar
    // loads and never make a wave wait for its own prefetched rows.
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wc = wave % WC, wr = wave / WC;
    const int64_t ctw = cblk * WC + wc;
    const int64_t c0 = ctw * CTW;
    const int rpw = rb / WR;
    const int64_t r0 = band * rb + (int64_t)wr * rpw;
    const int64_t r1 = r0 + rpw < a.m ? r0 + rpw : a.m;

    d2 acc[KV];
#pragma unroll
    for (int k = 0; k < KV; ++k)
        acc[k] = d2{0.0, 0.0};
    double mine = 0.0;
    if (c0 < a.n) {
        if (c0 + CTW <= a.n)
            tile_rows<KV, D, OPS, VEC, true>(a, c0, r0, r1, lane, acc, mine);
        else
            tile_rows<KV, D, OPS, VEC, false>(a, c0, r0, r1, lane, acc, mine);
    }

    if (ROWDOT && c0 < a.n) {
        if (lane < r1 - r0)
            a.Prow[ctw * a.m + r0 + lane] = mine;
    }
    if (COLSUM) {
        if constexpr (WR == 1) {
#pragma unroll
            for (int k = 0; k < KV; ++k) {
                const int64_t j = c0 + 2 * (lane + kWave * k);
                if (j < a.n) a.Pcol[band * a.n + j] = acc[k].x;
                if (j + 1 < a.n) a.Pcol[band * a.n + j + 1] = acc[k].y;
            }
        } else {
            // combine the WR row groups' column sums in row-group order
#pragma unroll
            for (int k = 0; k < KV; ++k) {
                const int c = wc * CTW + 2 * (lane + kWave * k);
                lds[wr * CTB + c] = acc[k].x;
                lds[wr * CTB + c + 1] = acc[k].y;
            }
            lds_barrier();
            const int64_t cb = cblk * CTB;
            for (int c = threadIdx.x; c < CTB; c += NT) {
                const int64_t j = cb + c;
                if (j < a.n) {
                    double s = lds[c];
#pragma unroll
                    for (int r = 1; r < WR; ++r)
                        s += lds[r * CTB + c];
                    a.Pcol[band * a.n + j] = s;
                }
            }
        }
    }
    if constexpr ((OPS & OP_AUX) && COLSUM) {
        // the first column block's waves add u1_i yc_i and u2_i yc_i over
        // their rows; the row groups' sums meet in LDS in row-group order
        if (cblk == 0) {
            double *aux = lds + (WR > 1 ? WR * CTB : 0);
            if (wc == 0) {
                double s1 = 0.0, s2 = 0.0;
                for (int64_t i = r0 + lane; i < r1; i += kWave) {
                    const double yi = a.yc[i];
                    s1 += a.u1[i] * yi;
                    s2 += a.u2[i] * yi;
                }
                s1 = wave_sum(s1);
                s2 = wave_sum(s2);
                if (lane == 0) {
                    aux[2 * wr] = s1;
                    aux[2 * wr + 1] = s2;
                }
            }
            lds_barrier();
            if (threadIdx.x == 0) {
                double s1 = aux[0], s2 = aux[1];
                for (int r = 1; r < WR; ++r) {
                    s1 += aux[2 * r];
                    s2 += aux[2 * r + 1];
                }
                a.Prow[2 * band] = s1;
                a.Prow[2 * band + 1] = s2;
            }
        }
    }
    if constexpr ((OPS & OP_AUX) && ROWDOT) {
        // the first band's waves add v1_j xr_j and v2_j xr_j over their
        // wave tile's columns (pairs in the sweep's lane order)
        if (band == 0 && wr == 0 && c0 < a.n) {
            double t1 = 0.0, t2 = 0.0;
#pragma unroll
            for (int k = 0; k < KV; ++k) {
                const int64_t j = c0 + 2 * (lane + kWave * k);
                const d2 x2 = load_vec_pair(a.xr, j, a.n);
                const d2 p1 = load_vec_pair(a.v1, j, a.n);
                const d2 p2 = load_vec_pair(a.v2, j, a.n);
                t1 += p1.x * x2.x;
                t1 += p1.y * x2.y;
                t2 += p2.x * x2.x;
                t2 += p2.y * x2.y;
            }
            t1 = wave_sum(t1);
            t2 = wave_sum(t2);
            if (lane == 0) {
                a.Pcol[2 * ctw] = t1;
                a.Pcol[2 * ctw + 1] = t2;
            }
        }
    }
}


// The tile shapes instantiated for each family of sweeps.
struct Shape {
    int kv, d, wc, wr;
};
constexpr Shape kShapes[] = {
    // read-only sweeps (row dots, column sums, both)
    {8, 2, 4, 1}, {8, 1, 4, 4}, {4, 2, 8, 2}, {4, 2, 4, 4}, {4, 4, 4, 1}, {8, 2, 4, 2},
    // sweeps that store B
    {2, 2, 1, 4}, {2, 4, 1, 4}, {4, 2, 1, 4}, {4, 4, 1, 4}, {2, 3, 1, 16},
    // ... narrower wave rows (1 KiB), for short-lived workgroups
    {1, 2, 1, 16}, {1, 4, 1, 8}, {2, 2, 1, 8}, {1, 2, 2, 8},
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);
static_assert(kNumShapes == kTileShapes, "the shape table and the C interface disagree");
constexpr bool kv_at_least(int i, int kv)
{
    return i == kNumShapes || (kShapes[i].kv >= kv && kv_at_least(i + 1, kv));
}
static_assert(kv_at_least(0, kMinTileKv), "a shape is narrower than the row-dot partials allow");
constexpr int kFirstWriteShape = 6;

// ---- fixed-order reduction of partials -----------------------------------
//
// One workgroup per 64 outputs: wave w sums parts [w*q, (w+1)*q) of each of
// its lane's outputs sequentially (q = ceil(nparts/4)), then wave 0 adds
// the four wave sums in order and applies the epilogue.

__device__ __forceinline__ void finish_block(const FinishJob &j, int64_t b, double (&lds)[4][64])
{
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

// Pointers read from memory (batch tables) are not known to address global
// memory; accessed as they are they would compile to flat loads and stores,
// whose completion is also counted with the scalar loads of the row
// scalars, so that every wait for u1[i] or y[i] would also wait for the
// wave's prefetched rows.  They are therefore recast to the global address
// space first.

template <typename T>
__device__ __forceinline__ T *as_global(T *p)
{
    typedef __attribute__((address_space(1))) T gT;
    return (T *)(gT *)(uintptr_t)p;
}

__device__ __forceinline__ void globalize(TileArgs &a)
{
    a.A = as_global(a.A);
    a.B = as_global(a.B);
    a.xr = as_global(a.xr);
    a.yc = as_global(a.yc);
    a.u1 = as_global(a.u1);
    a.v1 = as_global(a.v1);
    a.u2 = as_global(a.u2);
    a.v2 = as_global(a.v2);
    a.Prow = as_global(a.Prow);
    a.Pcol = as_global(a.Pcol);
}

}  // namespace

}  // namespace bto
