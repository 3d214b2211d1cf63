// Batched execution: thousands of independent GEMVER / BiCGK / ATAX
// instances of uneven size in one persistent launch.
//
// A workgroup takes one unit of work at a time: a whole instance, all of
// whose passes it runs alone, or one row tile of a large fused instance,
// which is cut into tiles so that several workgroups share it (the column
// sums then go through per-tile partials, and GEMVER's second sweep waits
// for its x; see run_tile).  Instances are limited to n <= 2048 columns.
//
// Inside the workgroup every thread owns fixed columns: a row is covered by
// a group of `tpr` threads (a power of two), thread c of the group holding
// 16-byte column pairs c, c + tpr, ... (NP of them), and the NT / tpr groups
// ("row slots") take different rows side by side, so narrow instances still
// use every lane.  A thread reads 8 pairs (4 in the sweeps that write B) per
// batch of rows with every load issued before any is used, keeps the row-dot and
// update vectors for its columns in registers and accumulates the column
// sums of its columns in registers too.  A row dot is summed inside its
// thread group with lane permutes; when a row spans several waves their
// partial sums meet in LDS.  The row slots' column sums are added in LDS in
// slot order at the end of the sweep.  The odd last column of an odd n is
// handled by the first thread of each group.
//
// The host sorts the units by decreasing work (longest first; GEMVER's
// second-sweep tiles after all others) and the persistent workgroups pull
// them from one queue counter, so the largest work starts first and the
// small units fill in at the end.  Every unit is computed the same way
// whichever workgroup takes it, so the results depend only on the instance,
// the workgroup size and the tile size, not on the schedule.

#include "bto.h"
#include "bto_batch.hpp"
#include "bto_dev.hpp"
#include "bto_internal.hpp"

namespace bto {

namespace {

constexpr int kMaxN = 2048;
constexpr int kMaxNT = 512;

// Row dots of rows wider than a wave leave one partial per wave in LDS; a
// sweep parks this many batches of them before one barrier adds them up.
constexpr int kParkBatches = 8;

enum SweepOps { SW_ROWDOT = 1, SW_COLSUM = 2, SW_UPD1 = 4, SW_UPD2 = 8, SW_ATAX = 16 };

struct Lds {
    double xs[kMaxN];            // GEMVER's x, handed from pass 1 to pass 2
    double red[2 * kMaxNT];      // column sums of the row slots (one pair per thread)
    double red_last[kMaxNT];     // the odd column's sums of the row slots
    // row-dot partials of rows wider than a wave: up to kParkBatches
    // batches of U <= 8 rows per row slot, NT / 64 waves' partials per slot
    double park[2][kParkBatches * 8 * (kMaxNT / 64)];
    int last;                    // this workgroup finished an instance's last tile
};

// A second-sweep tile waits for its instance's x at most this many sleeps
// (about a second); then it gives up, flags the launch as failed and
// carries on, so every workgroup always reaches the end of the queue.
constexpr int kSpinLimit = 1 << 22;

// The instance table is read as words through scalar loads, which hides that
// its pointers address device (global) memory.  Accessed as they are, they
// compile to flat loads and stores, whose completion is also counted with
// LDS and scalar-memory operations, so that every LDS or scalar wait would
// stall behind the wave's outstanding row loads.  Every access through a
// table pointer therefore goes through a global-address-space pointer.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> gp(T *p)
{
    return (gptr<T>)(uintptr_t)p;
}

__device__ __forceinline__ d2 gld2(gptr<const double> p)
{
    return *reinterpret_cast<gptr<const d2>>(p);
}

__device__ __forceinline__ d2 gld2_nt(gptr<const double> p)
{
    return __builtin_nontemporal_load(reinterpret_cast<gptr<const d2>>(p));
}

__device__ __forceinline__ double gld1_nt(gptr<const double> p)
{
    return __builtin_nontemporal_load(p);
}

__device__ __forceinline__ void gst2_nt(gptr<double> p, d2 v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<gptr<d2>>(p));
}

__device__ __forceinline__ void gst1_nt(gptr<double> p, double v)
{
    __builtin_nontemporal_store(v, p);
}

// 16 bytes from a vector in global memory or in LDS.
__device__ __forceinline__ d2 ld2_any(gptr<const double> p) { return gld2(p); }
__device__ __forceinline__ d2 ld2_any(const double *p) { return ld2(p); }

// Where a thread sits for one instance.
struct Geo {
    int64_t npf;   // whole column pairs, n / 2
    int odd;       // n is odd: column n-1 belongs to the first thread of each group
    int tpr;       // threads per row (a power of two)
    int rs;        // row slots, NT / tpr
    int c;         // pair column of this thread within its group
    int slot;      // row slot of this thread
};

// Pairs per thread per row: the fewest that let NT threads cover a row.
template <int NT>
__device__ __forceinline__ int pairs_per_thread(int64_t n)
{
    const int64_t npf = n >> 1;
    return npf <= NT ? 1 : (npf <= 2 * NT ? 2 : 4);
}

template <int NT, int NP>
__device__ __forceinline__ Geo geometry(int64_t n)
{
    Geo g;
    g.npf = n >> 1;
    g.odd = (int)(n & 1);
    const int64_t per = (g.npf + NP - 1) / NP;
    int t = 1;
    while (t < per)
        t <<= 1;
    g.tpr = t;
    g.rs = NT / t;
    g.c = (int)threadIdx.x & (t - 1);
    g.slot = (int)threadIdx.x / t;
    return g;
}

// Row sums of U rows at once.  Each row lies on an aligned group of `tpr`
// lanes (for tpr >= 64, on whole waves: the sum is then the wave's, as in
// wave_sum).  Each step adds a lane's value to a partner's inside the group
// (quad swaps, half-row and row mirrors, the lane 16 away, then the two
// half-waves); partners add the same two numbers, so every lane of the group
// ends with the same, order-fixed sum.  Every step runs over all U values
// before the next, so the U dependency chains overlap.
template <int U>
__device__ __forceinline__ void group_sums(double (&v)[U], int tpr)
{
    if (tpr >= 2) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] += dpp_f64<0xB1>(v[u]);    // quad_perm [1,0,3,2]
    }
    if (tpr >= 4) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] += dpp_f64<0x4E>(v[u]);    // quad_perm [2,3,0,1]
    }
    if (tpr >= 8) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] += dpp_f64<0x141>(v[u]);   // row_half_mirror
    }
    if (tpr >= 16) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] += dpp_f64<0x140>(v[u]);   // row_mirror
    }
    if (tpr >= 32) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] += swz16_f64(v[u]);
    }
    if (tpr >= 64) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = readlane_f64(v[u], 0) + readlane_f64(v[u], 32);
    }
}

// Load the thread's pairs of a length-n vector (zeros where not owned),
// from global memory (a gptr) or from LDS.
template <int NP, typename P>
__device__ __forceinline__ void load_cols(const Geo &g, P v, int64_t n, d2 (&dst)[NP],
                                          double &last)
{
    // unconditional loads (pair 0 stands in for a pair not owned), then
    // zeroed; nothing at all when there is no whole pair (n <= 1)
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int64_t p = g.c + (int64_t)g.tpr * k;
        const bool own = p < g.npf;
        const d2 val = g.npf > 0 ? ld2_any(v + (own ? 2 * p : 0)) : d2{0.0, 0.0};
        dst[k] = own ? val : d2{0.0, 0.0};
    }
    last = g.odd ? v[n - 1] : 0.0;
}

// The rows one thread holds for one batch: U rows of NP pairs, the odd
// column and the per-row scalars.
template <int U, int NP>
struct RowBatch {
    d2 a[U][NP];
    double al[U], s1[U], s2[U], yw[U];
};

// One sweep of an instance's rows.  OPS selects what each row contributes:
//   SW_UPD1 (+SW_UPD2): row <- row + s1_i v1 (+ s2_i v2), stored to dst
//   SW_ROWDOT:          rowout[i] = rscale * (row . xr)
//   SW_COLSUM:          acc += row * yc[i]
//   SW_ATAX:            acc += row * (row . xr)
// Rows i = base + u*rs + slot (u < U) form one batch (U*NP = 8 pairs per
// thread, 4 when updating or for narrow BiCGK rows); all of a batch's loads
// are issued before any is used.  Loads are never conditional: a row past
// the end re-reads the last row and a pair past the end re-reads pair 0,
// and the values are zeroed when used.
template <int NT, int NP, int OPS>
__device__ __forceinline__ void sweep(const Geo &g, int64_t m, int64_t n, const double *src,
                                      int64_t lds_, double *dst, int64_t ldd, const double *u1,
                                      const double *u2, const double *yc, double *rowout,
                                      double rscale, const d2 (&xr)[NP], double xr_last,
                                      const d2 (&v1)[NP], double v1_last, const d2 (&v2)[NP],
                                      double v2_last, d2 (&acc)[NP], double &acc_last, Lds &L)
{
    constexpr bool ROWDOT = OPS & SW_ROWDOT;
    constexpr bool COLSUM = OPS & SW_COLSUM;
    constexpr bool UPD1 = OPS & SW_UPD1;
    constexpr bool UPD2 = OPS & SW_UPD2;
    constexpr bool ATAX = OPS & SW_ATAX;
    constexpr bool DOT = ROWDOT || ATAX;
    const gptr<const double> gsrc = gp(src), gu1 = gp(u1), gu2 = gp(u2), gyc = gp(yc);
    const gptr<double> gdst = gp(dst), grow = gp(rowout);
    // pairs per thread per batch: fewer for the sweeps that update (two row
    // scalars and a store per row as well) or do two things with narrow rows
    constexpr int PIF = (UPD1 || (ROWDOT && COLSUM && NP == 1)) ? 4 : 8;
    constexpr int U = PIF / NP > 0 ? PIF / NP : 1;   // rows per slot per batch
    typedef RowBatch<U, NP> Batch;
    const int lane = threadIdx.x & 63;
    const bool lead = g.c == 0;
    const bool wide = g.tpr > kWave;        // a row spans several waves
    const int nwr = wide ? g.tpr / kWave : 1;
    const int wr = g.c / kWave;             // this wave's part of a wide row
    const int64_t batch = (int64_t)U * g.rs;
    int coff[NP];                           // column offset of each owned pair (0 if none)
    bool pv[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int p = g.c + g.tpr * k;       // below n <= 2048
        pv[k] = p < g.npf;
        coff[k] = pv[k] ? 2 * p : 0;
    }
    const bool last_here = g.odd && lead;
    int pb = 0;            // the park buffer being filled
    int fb = 0;            // batches parked in it
    int64_t gbase = 0;     // the first row parked in it

    auto load = [&](int64_t base, Batch &b) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t ri = base + (int64_t)u * g.rs + g.slot;
            const int64_t rc = ri < m ? ri : m - 1;
            const gptr<const double> row = gsrc + rc * lds_;
            // (a uniform test: with no whole pair, n <= 1, nothing is read
            // beyond column n-1, and A may be empty)
#pragma unroll
            for (int k = 0; k < NP; ++k)
                b.a[u][k] = g.npf > 0 ? gld2_nt(row + coff[k]) : d2{0.0, 0.0};
            b.al[u] = g.odd ? gld1_nt(row + n - 1) : 0.0;
            if (UPD1) b.s1[u] = gu1[rc];
            if (UPD2) b.s2[u] = gu2[rc];
            // a vector load: the weights may have been written earlier in
            // this launch (the unfused ATAX temporary)
            if (COLSUM) b.yw[u] = __builtin_nontemporal_load(gyc + rc);
        }
    };

    auto process = [&](int64_t base, Batch &b) {
        int64_t ri[U];
        bool rv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ri[u] = base + (int64_t)u * g.rs + g.slot;
            rv[u] = ri[u] < m;
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (!(rv[u] && pv[k])) b.a[u][k] = d2{0.0, 0.0};
            if (!rv[u]) b.al[u] = 0.0;
        }
        if (UPD1) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const gptr<double> brow = gdst + ri[u] * ldd;
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    d2 v = b.a[u][k] + b.s1[u] * v1[k];
                    if (UPD2) v = v + b.s2[u] * v2[k];
                    b.a[u][k] = v;
                    if (rv[u] && pv[k]) gst2_nt(brow + coff[k], v);
                }
                if (g.odd) {
                    double bl = b.al[u] + b.s1[u] * v1_last;
                    if (UPD2) bl = bl + b.s2[u] * v2_last;
                    b.al[u] = bl;
                    if (rv[u] && lead) gst1_nt(brow + n - 1, bl);
                }
                if (!rv[u]) {
                    // keep the masked row zero for the sums below
#pragma unroll
                    for (int k = 0; k < NP; ++k) b.a[u][k] = d2{0.0, 0.0};
                    b.al[u] = 0.0;
                }
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (!pv[k]) b.a[u][k] = d2{0.0, 0.0};
            }
        }
        double dot[U];
        if (DOT) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                double part = 0.0;
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    part += b.a[u][k].x * xr[k].x;
                    part += b.a[u][k].y * xr[k].y;
                }
                if (last_here) part += b.al[u] * xr_last;
                dot[u] = part;
            }
            group_sums(dot, g.tpr);
            if (wide) {
                // partials of each row's waves meet in LDS, added in wave
                // order: at once where the row's dot weights its own column
                // sums (ATAX), else once kParkBatches batches are parked
                const int at = ATAX ? 0 : fb * (int)batch;
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (lane == 0) L.park[pb][(at + u * g.rs + g.slot) * nwr + wr] = dot[u];
                if (ATAX) {
                    lds_barrier();
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const double *pp = &L.park[pb][(u * g.rs + g.slot) * nwr];
                        double t = pp[0];
                        for (int w = 1; w < nwr; ++w) t += pp[w];
                        dot[u] = t;
                    }
                    pb ^= 1;
                }
            } else if (ROWDOT) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (lead && rv[u]) grow[ri[u]] = rscale * dot[u];
            }
        }
        if (COLSUM || ATAX) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double w = ATAX ? dot[u] : (rv[u] ? b.yw[u] : 0.0);
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    acc[k] += b.a[u][k] * w;
                if (last_here) acc_last += b.al[u] * w;
            }
        }
    };

    // the parked row dots of rows gbase, gbase + 1, ... (fb batches): the
    // partials of row gbase + t sit at t * nwr, t < fb * batch <= NT / 2
    auto flush = [&]() {
        lds_barrier();
        const int64_t t = threadIdx.x;
        if (t < fb * batch && gbase + t < m) {
            const double *pp = &L.park[pb][t * nwr];
            double s = pp[0];
            for (int w = 1; w < nwr; ++w) s += pp[w];
            grow[gbase + t] = rscale * s;
        }
        pb ^= 1;
        fb = 0;
    };

    // all of a batch's loads are issued before any of its values is used;
    // the other workgroups on the compute unit cover the wait
    for (int64_t base = 0; base < m; base += batch) {
        Batch b;
        load(base, b);
        if (fb == 0) gbase = base;
        process(base, b);
        if (ROWDOT && !ATAX && wide && (++fb == kParkBatches || base + batch >= m))
            flush();
    }
}

// out[j] = scale * (column sum j) + add[j] (add may be null); optionally
// also into keep (LDS).  The row slots' sums are added in slot order.
template <int NT, int NP>
__device__ __forceinline__ void finish_cols(const Geo &g, int64_t n, const d2 (&acc)[NP],
                                            double acc_last, double scale, const double *add,
                                            double *out, double *keep, Lds &L)
{
    const gptr<const double> gadd = gp(add);
    const gptr<double> gout = gp(out);
    if (g.rs == 1) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int64_t p = g.c + (int64_t)g.tpr * k;
            if (p < g.npf) {
                d2 v = acc[k] * scale;
                if (add) v += gld2(gadd + 2 * p);
                *reinterpret_cast<gptr<d2>>(gout + 2 * p) = v;
                if (keep) *reinterpret_cast<d2 *>(keep + 2 * p) = v;
            }
        }
        if (g.odd && g.c == 0) {
            double v = acc_last * scale;
            if (add) v += gadd[n - 1];
            gout[n - 1] = v;
            if (keep) keep[n - 1] = v;
        }
    } else {
        // here NP == 1 and npf <= tpr: thread (slot, c) holds pair c of slot
        reinterpret_cast<d2 *>(L.red)[g.slot * g.tpr + g.c] = acc[0];
        if (g.c == 0) L.red_last[g.slot] = acc_last;
        __syncthreads();
        for (int64_t p = threadIdx.x; p < g.npf; p += NT) {
            const d2 *r = reinterpret_cast<const d2 *>(L.red);
            d2 v = r[p];
            for (int s = 1; s < g.rs; ++s) v += r[s * g.tpr + p];
            v = v * scale;
            if (add) v += gld2(gadd + 2 * p);
            *reinterpret_cast<gptr<d2>>(gout + 2 * p) = v;
            if (keep) *reinterpret_cast<d2 *>(keep + 2 * p) = v;
        }
        if (g.odd && threadIdx.x == 0) {
            double v = L.red_last[0];
            for (int s = 1; s < g.rs; ++s) v += L.red_last[s];
            v = v * scale;
            if (add) v += gadd[n - 1];
            gout[n - 1] = v;
            if (keep) keep[n - 1] = v;
        }
    }
    __syncthreads();
}

template <int NP>
__device__ __forceinline__ void zero(d2 (&v)[NP], double &last)
{
#pragma unroll
    for (int k = 0; k < NP; ++k) v[k] = d2{0.0, 0.0};
    last = 0.0;
}

template <int NT, int NP>
__device__ __forceinline__ void run_item(const BatchItem &it, double *tmp, Lds &L)
{
    const int64_t m = it.m, n = it.n;
    const Geo g = geometry<NT, NP>(n);
    d2 xr[NP], v1[NP], v2[NP], acc[NP];
    double xr_l, v1_l, v2_l, acc_l;
    zero(xr, xr_l);
    zero(v1, v1_l);
    zero(v2, v2_l);
    zero(acc, acc_l);
    if (it.kind == BTO_K_BICGK) {
        // q = A p ; s = A^T r
        const double *p = it.vec[0], *r = it.vec[1];
        double *q = it.out[0], *s = it.out[1];
        load_cols(g, gp(p), n, xr, xr_l);
        if (it.form == BTO_FUSED) {
            sweep<NT, NP, SW_ROWDOT | SW_COLSUM>(g, m, n, it.A, it.lda, nullptr, 0, nullptr,
                                                 nullptr, r, q, 1.0, xr, xr_l, v1, v1_l, v2,
                                                 v2_l, acc, acc_l, L);
        } else {
            sweep<NT, NP, SW_ROWDOT>(g, m, n, it.A, it.lda, nullptr, 0, nullptr, nullptr, nullptr,
                                     q, 1.0, xr, xr_l, v1, v1_l, v2, v2_l, acc, acc_l, L);
            sweep<NT, NP, SW_COLSUM>(g, m, n, it.A, it.lda, nullptr, 0, nullptr, nullptr, r,
                                     nullptr, 1.0, xr, xr_l, v1, v1_l, v2, v2_l, acc, acc_l, L);
        }
        finish_cols<NT, NP>(g, n, acc, acc_l, 1.0, nullptr, s, nullptr, L);
    } else if (it.kind == BTO_K_GEMVER) {
        // B = A + u1 v1^T + u2 v2^T ; x = beta B^T y + z ; w = alpha B x
        const double *u1 = it.vec[0], *vv1 = it.vec[1], *u2 = it.vec[2], *vv2 = it.vec[3];
        const double *y = it.vec[4], *z = it.vec[5];
        double *x = it.out[0], *w = it.out[1];
        load_cols(g, gp(vv1), n, v1, v1_l);
        if (it.form == BTO_FUSED) {
            load_cols(g, gp(vv2), n, v2, v2_l);
            sweep<NT, NP, SW_UPD1 | SW_UPD2 | SW_COLSUM>(g, m, n, it.A, it.lda, it.B, it.ldb, u1,
                                                         u2, y, nullptr, 1.0, xr, xr_l, v1, v1_l,
                                                         v2, v2_l, acc, acc_l, L);
        } else {
            sweep<NT, NP, SW_UPD1>(g, m, n, it.A, it.lda, it.B, it.ldb, u1, nullptr, nullptr,
                                   nullptr, 1.0, xr, xr_l, v1, v1_l, v2, v2_l, acc, acc_l, L);
            __syncthreads();
            load_cols(g, gp(vv2), n, v1, v1_l);
            sweep<NT, NP, SW_UPD1>(g, m, n, it.B, it.ldb, it.B, it.ldb, u2, nullptr, nullptr,
                                   nullptr, 1.0, xr, xr_l, v1, v1_l, v2, v2_l, acc, acc_l, L);
            __syncthreads();
            sweep<NT, NP, SW_COLSUM>(g, m, n, it.B, it.ldb, nullptr, 0, nullptr, nullptr, y,
                                     nullptr, 1.0, xr, xr_l, v1, v1_l, v2, v2_l, acc, acc_l, L);
        }
        finish_cols<NT, NP>(g, n, acc, acc_l, it.beta, z, x, L.xs, L);
        load_cols(g, L.xs, n, xr, xr_l);
        sweep<NT, NP, SW_ROWDOT>(g, m, n, it.B, it.ldb, nullptr, 0, nullptr, nullptr, nullptr, w,
                                 it.alpha, xr, xr_l, v1, v1_l, v2, v2_l, acc, acc_l, L);
    } else {
        // ATAX: y = A^T (A x)
        const double *xv = it.vec[0];
        double *y = it.out[0];
        load_cols(g, gp(xv), n, xr, xr_l);
        if (it.form == BTO_FUSED) {
            sweep<NT, NP, SW_ATAX>(g, m, n, it.A, it.lda, nullptr, 0, nullptr, nullptr, nullptr,
                                   nullptr, 1.0, xr, xr_l, v1, v1_l, v2, v2_l, acc, acc_l, L);
        } else {
            // t = A x into the instance's scratch, then y = A^T t
            sweep<NT, NP, SW_ROWDOT>(g, m, n, it.A, it.lda, nullptr, 0, nullptr, nullptr, nullptr,
                                     tmp, 1.0, xr, xr_l, v1, v1_l, v2, v2_l, acc, acc_l, L);
            __syncthreads();
            sweep<NT, NP, SW_COLSUM>(g, m, n, it.A, it.lda, nullptr, 0, nullptr, nullptr, tmp,
                                     nullptr, 1.0, xr, xr_l, v1, v1_l, v2, v2_l, acc, acc_l, L);
        }
        finish_cols<NT, NP>(g, n, acc, acc_l, 1.0, nullptr, y, nullptr, L);
    }
    __syncthreads();
}

// One row tile [r0, r1) of a split fused instance.
//   phase 1: the instance's first sweep over the tile's rows (row results
//            written directly), the tile's column sums into its partial
//            vector; the workgroup that completes the instance's last tile
//            adds the partials in tile order (s, y, or GEMVER's x, after
//            which it raises the instance's x-ready flag);
//   phase 2: GEMVER's w = alpha B x over the tile's rows, once x is ready.
// Partials and flags cross workgroups (and the XCDs' separate L2 caches):
// writers make their stores visible with a device-scope release before
// counting, readers acquire at device scope before reading.
template <int NT, int NP>
__device__ __forceinline__ void run_tile(const BatchItem &it, const BatchUnit &un,
                                         double *scratch, int *sync, int *err, Lds &L)
{
    const int64_t n = it.n, r0 = un.r0, mt = un.r1 - un.r0;
    const Geo g = geometry<NT, NP>(n);
    d2 xr[NP], v1[NP], v2[NP], acc[NP];
    double xr_l, v1_l, v2_l, acc_l;
    zero(xr, xr_l);
    zero(v1, v1_l);
    zero(v2, v2_l);
    zero(acc, acc_l);
    const int64_t ldp = (n + 31) / 32 * 32;
    double *part = scratch + it.part_off;
    const int T = it.ntiles;
    const double *A = it.A + r0 * it.lda;
    if (un.phase == 1) {
        const int t = (int)(r0 / it.tile_rows);
        if (it.kind == BTO_K_BICGK) {
            load_cols(g, gp(it.vec[0]), n, xr, xr_l);
            sweep<NT, NP, SW_ROWDOT | SW_COLSUM>(g, mt, n, A, it.lda, nullptr, 0, nullptr, nullptr,
                                                 it.vec[1] + r0, it.out[0] + r0, 1.0, xr, xr_l,
                                                 v1, v1_l, v2, v2_l, acc, acc_l, L);
        } else if (it.kind == BTO_K_GEMVER) {
            load_cols(g, gp(it.vec[1]), n, v1, v1_l);
            load_cols(g, gp(it.vec[3]), n, v2, v2_l);
            sweep<NT, NP, SW_UPD1 | SW_UPD2 | SW_COLSUM>(
                g, mt, n, A, it.lda, it.B + r0 * it.ldb, it.ldb, it.vec[0] + r0, it.vec[2] + r0,
                it.vec[4] + r0, nullptr, 1.0, xr, xr_l, v1, v1_l, v2, v2_l, acc, acc_l, L);
        } else {
            load_cols(g, gp(it.vec[0]), n, xr, xr_l);
            sweep<NT, NP, SW_ATAX>(g, mt, n, A, it.lda, nullptr, 0, nullptr, nullptr, nullptr,
                                   nullptr, 1.0, xr, xr_l, v1, v1_l, v2, v2_l, acc, acc_l, L);
        }
        finish_cols<NT, NP>(g, n, acc, acc_l, 1.0, nullptr, part + t * ldp, nullptr, L);
        __threadfence();   // this thread's partial (and B rows) visible device-wide
        __syncthreads();
        if (threadIdx.x == 0)
            L.last = __hip_atomic_fetch_add(sync, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
                     T - 1;
        __syncthreads();
        if (L.last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            double scale = 1.0;
            const double *add = nullptr;
            double *out = it.out[it.kind == BTO_K_BICGK ? 1 : 0];
            if (it.kind == BTO_K_GEMVER) {
                scale = it.beta;
                add = it.vec[5];
            }
            const gptr<const double> gadd = gp(add);
            const gptr<double> gout = gp(out);
            for (int64_t j = threadIdx.x; j < n; j += NT) {
                double v = part[j];
                for (int k = 1; k < T; ++k)
                    v += part[k * ldp + j];
                v = v * scale;
                if (add) v += gadd[j];
                gout[j] = v;
            }
            if (it.kind == BTO_K_GEMVER) {
                __threadfence();
                __syncthreads();
                if (threadIdx.x == 0)
                    __hip_atomic_store(sync + 1, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    } else {
        if (threadIdx.x == 0) {
            int spins = 0;
            while (__hip_atomic_load(sync + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                if (++spins > kSpinLimit) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        load_cols(g, gp(it.out[0]), n, xr, xr_l);
        sweep<NT, NP, SW_ROWDOT>(g, mt, n, it.B + r0 * it.ldb, it.ldb, nullptr, 0, nullptr, nullptr,
                                 nullptr, it.out[1] + r0, it.alpha, xr, xr_l, v1, v1_l, v2, v2_l,
                                 acc, acc_l, L);
        __syncthreads();
    }
}

template <int NT>
__device__ __forceinline__ void dispatch_tile(const BatchItem &it, const BatchUnit &un,
                                              double *scratch, int *sync, int *err, Lds &L)
{
    const int np = pairs_per_thread<NT>(it.n);
    if (np == 1) run_tile<NT, 1>(it, un, scratch, sync, err, L);
    else if (np == 2) run_tile<NT, 2>(it, un, scratch, sync, err, L);
    else if constexpr (NT < 512) run_tile<NT, 4>(it, un, scratch, sync, err, L);
}

template <int NT>
__device__ __forceinline__ void dispatch_item(const BatchItem &it, double *tmp, Lds &L)
{
    const int np = pairs_per_thread<NT>(it.n);
    if (np == 1) run_item<NT, 1>(it, tmp, L);
    else if (np == 2) run_item<NT, 2>(it, tmp, L);
    else if constexpr (NT < 512) run_item<NT, 4>(it, tmp, L);
}

// Read-only table entries at a uniform index, through scalar loads.
__device__ __forceinline__ uint32_t load_uniform_word(const void *base, int idx)
{
    typedef const uint32_t __attribute__((address_space(4))) *cw;
    return reinterpret_cast<cw>(reinterpret_cast<uintptr_t>(base))[idx];
}

template <typename R>
__device__ __forceinline__ R load_uniform_record(const R *table, int idx)
{
    static_assert(sizeof(R) % 4 == 0, "records are read as 32-bit words");
    struct Words {
        uint32_t w[sizeof(R) / 4];
    } words;
    const int first = idx * (int)(sizeof(R) / 4);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(R) / 4); ++k)
        words.w[k] = load_uniform_word(table, first + k);
    return __builtin_bit_cast(R, words);
}

// Registers (at most 128 per lane) and LDS (under 32 KiB) let four 256-thread
// workgroups, or two of 512, share a compute unit: four waves per SIMD.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
void k_batch(const BatchItem *items, const BatchUnit *units, int *meta, int *sync,
             double *scratch)
{
    // the unit count is written with the table, so a captured launch
    // serves any refill
    __shared__ Lds L;
    __shared__ int slot;
    const int count = __builtin_nontemporal_load(meta + kMetaUnits);
    for (;;) {
        if (threadIdx.x == 0)
            slot = atomicAdd(meta + kMetaNext, 1);
        __syncthreads();
        // a uniform index, so the unit and the instance come through scalar
        // loads into scalar registers (reads only: the table is written by
        // the host before the launch and never while the kernel runs)
        const int idx = __builtin_amdgcn_readfirstlane(slot);
        __syncthreads();
        if (idx >= count)
            break;   // every workgroup reaches this once the queue is drained
        const BatchUnit un = load_uniform_record(units, idx);
        const BatchItem it = load_uniform_record(items, un.item);
        if (un.phase == 0)
            dispatch_item<NT>(it, scratch + it.scratch_off, L);
        else
            dispatch_tile<NT>(it, un, scratch, sync + 2 * un.item, meta + kMetaError, L);
    }
}

// Clear the queue counter, the error flag and the instances' sync counters.
__global__ __launch_bounds__(256) void k_batch_reset(int *meta, int *sync)
{
    const int64_t nsync = 2 * (int64_t)__builtin_nontemporal_load(meta + kMetaItems);
    const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (tid == 0) {
        meta[kMetaNext] = 0;
        meta[kMetaError] = 0;
    }
    for (int64_t k = tid; k < nsync; k += (int64_t)gridDim.x * 256)
        sync[k] = 0;
}

}  // namespace

int64_t batch_max_n() { return kMaxN; }

bool batch_threads_supported(int threads) { return threads == 256 || threads == 512; }

void launch_batch(const BatchItem *items, const BatchUnit *units, int *meta, int *sync,
                  double *scratch, int threads, int grid, hipStream_t st)
{
    launch("batch_reset", k_batch_reset, dim3(16), dim3(256), st, meta, sync);
    if (threads == 512)
        launch("batch", k_batch<512>, dim3(grid), dim3(512), st, items, units, meta, sync, scratch);
    else
        launch("batch", k_batch<256>, dim3(grid), dim3(256), st, items, units, meta, sync, scratch);
}

}  // namespace bto
