// Batched execution: thousands of independent GEMVER / BiCGK / ATAX
// instances of uneven size in one persistent launch.
//
// One workgroup owns one instance at a time and runs all of its passes, so
// no instance ever depends on another workgroup: no partial-sum buffers, no
// cross-workgroup waits.  Inside the workgroup each wave takes whole rows
// (rows i = wave, wave + NW, ...), so a row dot is a single wave reduction
// and the column sums of the wave's rows accumulate in its lanes' registers;
// the waves' column sums are then added in LDS in wave order.  Column-indexed
// vectors (v1, v2, the row-dot weights) sit in LDS.  Instances are limited to
// n <= 128 * kMaxPPL columns (2048): each lane covers up to kMaxPPL 16-byte
// pairs of a row.
//
// The host sorts the instances by decreasing work (longest first) and the
// persistent workgroups pull them from one queue counter, so the largest
// instances start first and the small ones fill in at the end.  Every
// instance is computed the same way whichever workgroup takes it, so the
// results do not depend on the schedule.

#include "bto.h"
#include "bto_batch.hpp"
#include "bto_dev.hpp"
#include "bto_internal.hpp"

namespace bto {

namespace {

constexpr int kMaxPPL = 16;                   // pairs per lane: n <= 2048
constexpr int kMaxN = 128 * kMaxPPL;

enum SweepOps { SW_ROWDOT = 1, SW_COLSUM = 2, SW_UPD1 = 4, SW_UPD2 = 8, SW_ATAX = 16 };

struct Lds {
    double v1[kMaxN];     // u-update column vectors / row-dot weights
    double v2[kMaxN];
    double xr[kMaxN];     // row-dot weights (p, x) or ATAX x
    double red[kMaxN];    // column sums combined over the waves
};

__device__ __forceinline__ d2 lds_pair(const double *v, int p) { return reinterpret_cast<const d2 *>(v)[p]; }

// Load pair p (columns 2p, 2p+1) of a row; zero past n.  Rows are 16-byte
// aligned (checked when the plan is built).
__device__ __forceinline__ d2 row_pair(const double *row, int p, int64_t n)
{
    const int64_t j = 2 * (int64_t)p;
    if (j + 1 < n)
        return ld2_nt(row + j);
    d2 r{0.0, 0.0};
    if (j < n)
        r.x = row[j];
    return r;
}

// As row_pair, but a cached load: ATAX reads each row twice.
__device__ __forceinline__ d2 row_pair_cached(const double *row, int p, int64_t n)
{
    const int64_t j = 2 * (int64_t)p;
    if (j + 1 < n)
        return ld2(row + j);
    d2 r{0.0, 0.0};
    if (j < n)
        r.x = row[j];
    return r;
}

__device__ __forceinline__ void row_store(double *row, int p, int64_t n, d2 v)
{
    const int64_t j = 2 * (int64_t)p;
    if (j + 1 < n)
        st2_nt(row + j, v);
    else if (j < n)
        row[j] = v.x;
}

// One sweep of the rows of an instance matrix by the waves of the workgroup.
// OPS selects what each row contributes (see SweepOps).  Row results (dots)
// are written to rowout[i] * rscale; column sums end up in lds.red.  A row is
// handled in chunks of at most 8 pairs per lane, so a lane holds one chunk
// plus its column accumulators; ATAX, whose update needs the whole row's dot
// first, reads the row's chunks a second time (from cache) to apply it.
template <int PPL, int OPS, int NW>
__device__ __forceinline__ void sweep(int64_t m, int64_t n, const double *src, int64_t lds_,
                                      double *dst, int64_t ldd, const double *u1, const double *u2,
                                      const double *yc, double *rowout, double rscale, Lds &L)
{
    constexpr bool ROWDOT = OPS & SW_ROWDOT;
    constexpr bool COLSUM = OPS & (SW_COLSUM | SW_ATAX);
    constexpr bool UPD1 = OPS & SW_UPD1;
    constexpr bool UPD2 = OPS & SW_UPD2;
    constexpr bool ATAX = OPS & SW_ATAX;
    constexpr int CH = PPL < 8 ? PPL : 8;   // pairs per lane per chunk
    constexpr int NCH = PPL / CH;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    d2 acc[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k)
        acc[k] = d2{0.0, 0.0};

    for (int64_t i = wave; i < m; i += NW) {
        const double *row = src + i * lds_;
        // the LDS vectors do not change within a sweep; an index the
        // optimiser cannot see through keeps it from hoisting them all into
        // registers (a lane would then hold three more rows' worth)
        int lo = lane;
        asm volatile("" : "+v"(lo));
        double s1 = 0.0, s2 = 0.0, yi = 0.0;
        if (UPD1) {
            s1 = ld_uniform(u1 + i);
            if (UPD2) s2 = ld_uniform(u2 + i);
        }
        if (OPS & SW_COLSUM) {
            // a vector load: the weights may have been written earlier in this
            // launch (the unfused ATAX temporary), which the scalar cache
            // would not see
            yi = __builtin_nontemporal_load(yc + i);
        }
        double part = 0.0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            d2 a[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int p = lane + kWave * (c * CH + k);
                a[k] = ATAX ? row_pair_cached(row, p, n) : row_pair(row, p, n);
            }
            if (UPD1) {
                double *brow = dst + i * ldd;
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const int p = lane + kWave * (c * CH + k);
                    const int q = lo + kWave * (c * CH + k);
                    d2 b = a[k] + s1 * lds_pair(L.v1, q);
                    if (UPD2) b = b + s2 * lds_pair(L.v2, q);
                    a[k] = b;
                    row_store(brow, p, n, b);
                }
            }
            if (ROWDOT || ATAX) {
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const d2 w = lds_pair(L.xr, lo + kWave * (c * CH + k));
                    part += a[k].x * w.x;
                    part += a[k].y * w.y;
                }
            }
            if (OPS & SW_COLSUM) {
#pragma unroll
                for (int k = 0; k < CH; ++k)
                    acc[c * CH + k] += a[k] * yi;
            }
            if (ATAX && NCH == 1) {
                // the whole row is in registers: apply once the dot is known
                const double dot = wave_sum(part);
#pragma unroll
                for (int k = 0; k < CH; ++k)
                    acc[k] += a[k] * dot;
            }
        }
        if (ROWDOT) {
            const double dot = wave_sum(part);
            if (lane == 0)
                rowout[i] = rscale * dot;
        }
        if (ATAX && NCH > 1) {
            const double dot = wave_sum(part);
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const int p = lane + kWave * (c * CH + k);
                    acc[c * CH + k] += row_pair_cached(row, p, n) * dot;
                }
            }
        }
    }

    if (COLSUM) {
        // red = ((acc_0 + acc_1) + acc_2) + ...: the waves add in turn
        for (int w = 0; w < NW; ++w) {
            if (wave == w) {
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    const int p = lane + kWave * k;
                    if (2 * p < n) {
                        d2 *r = reinterpret_cast<d2 *>(L.red) + p;
                        *r = w == 0 ? acc[k] : *r + acc[k];
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Load a length-n vector into LDS, zero-filled up to npad (the columns the
// lanes cover), so that masked columns multiply zeros by zeros whatever an
// earlier instance left there.
__device__ __forceinline__ void stage(double *dst, const double *src, int64_t n, int64_t npad)
{
    for (int64_t j = threadIdx.x; j < npad; j += blockDim.x)
        dst[j] = j < n ? src[j] : 0.0;
}

// out[j] = scale * red[j] + add[j] (add may be null); optionally keep it in
// LDS, zero-filled up to npad.  (Columns j < n are read and written by the
// same thread, so `keep` may be the buffer `add` was staged in.)
__device__ __forceinline__ void finish_cols(const Lds &L, int64_t n, int64_t npad, double scale, const double *add,
                            double *out, double *keep)
{
    for (int64_t j = threadIdx.x; j < npad; j += blockDim.x) {
        if (j < n) {
            const double v = add ? scale * L.red[j] + add[j] : scale * L.red[j];
            out[j] = v;
            if (keep) keep[j] = v;
        } else if (keep) {
            keep[j] = 0.0;
        }
    }
}

template <int PPL, int NW>
__device__ __forceinline__ void run_item(const BatchItem &it, double *tmp, Lds &L)
{
    const int64_t m = it.m, n = it.n;
    const int64_t npad = 128 * PPL;
    if (it.kind == BTO_K_BICGK) {
        // q = A p ; s = A^T r
        const double *p = it.vec[0], *r = it.vec[1];
        double *q = it.out[0], *s = it.out[1];
        stage(L.xr, p, n, npad);
        __syncthreads();
        if (it.form == BTO_FUSED) {
            sweep<PPL, SW_ROWDOT | SW_COLSUM, NW>(m, n, it.A, it.lda, nullptr, 0, nullptr, nullptr,
                                                 r, q, 1.0, L);
        } else {
            sweep<PPL, SW_ROWDOT, NW>(m, n, it.A, it.lda, nullptr, 0, nullptr, nullptr, nullptr,
                                      q, 1.0, L);
            sweep<PPL, SW_COLSUM, NW>(m, n, it.A, it.lda, nullptr, 0, nullptr, nullptr, r,
                                      nullptr, 1.0, L);
        }
        finish_cols(L, n, npad, 1.0, nullptr, s, nullptr);
    } else if (it.kind == BTO_K_GEMVER) {
        // B = A + u1 v1^T + u2 v2^T ; x = beta B^T y + z ; w = alpha B x
        const double *u1 = it.vec[0], *v1 = it.vec[1], *u2 = it.vec[2], *v2 = it.vec[3];
        const double *y = it.vec[4], *z = it.vec[5];
        double *x = it.out[0], *w = it.out[1];
        stage(L.v1, v1, n, npad);
        stage(L.v2, v2, n, npad);
        __syncthreads();
        if (it.form == BTO_FUSED) {
            sweep<PPL, SW_UPD1 | SW_UPD2 | SW_COLSUM, NW>(m, n, it.A, it.lda, it.B, it.ldb, u1,
                                                         u2, y, nullptr, 1.0, L);
        } else {
            sweep<PPL, SW_UPD1, NW>(m, n, it.A, it.lda, it.B, it.ldb, u1, nullptr, nullptr,
                                    nullptr, 1.0, L);
            __syncthreads();
            stage(L.v1, v2, n, npad);
            __syncthreads();
            sweep<PPL, SW_UPD1, NW>(m, n, it.B, it.ldb, it.B, it.ldb, u2, nullptr, nullptr,
                                    nullptr, 1.0, L);
            __syncthreads();
            sweep<PPL, SW_COLSUM, NW>(m, n, it.B, it.ldb, nullptr, 0, nullptr, nullptr, y,
                                      nullptr, 1.0, L);
        }
        finish_cols(L, n, npad, it.beta, z, x, L.xr);
        __syncthreads();
        sweep<PPL, SW_ROWDOT, NW>(m, n, it.B, it.ldb, nullptr, 0, nullptr, nullptr, nullptr, w,
                                  it.alpha, L);
    } else {
        // ATAX: y = A^T (A x)
        const double *xv = it.vec[0];
        double *y = it.out[0];
        stage(L.xr, xv, n, npad);
        __syncthreads();
        if (it.form == BTO_FUSED) {
            sweep<PPL, SW_ATAX, NW>(m, n, it.A, it.lda, nullptr, 0, nullptr, nullptr, nullptr,
                                    nullptr, 1.0, L);
        } else {
            // t = A x into the instance's scratch, then y = A^T t
            sweep<PPL, SW_ROWDOT, NW>(m, n, it.A, it.lda, nullptr, 0, nullptr, nullptr, nullptr,
                                      tmp, 1.0, L);
            __syncthreads();
            sweep<PPL, SW_COLSUM, NW>(m, n, it.A, it.lda, nullptr, 0, nullptr, nullptr, tmp,
                                      nullptr, 1.0, L);
        }
        finish_cols(L, n, npad, 1.0, nullptr, y, nullptr);
    }
    __syncthreads();
}

template <int NW>
__device__ __forceinline__ void dispatch_item(const BatchItem &it, double *tmp, Lds &L)
{
    // the fewest 16-byte pairs per lane that cover the row
    if (it.n <= 128) run_item<1, NW>(it, tmp, L);
    else if (it.n <= 256) run_item<2, NW>(it, tmp, L);
    else if (it.n <= 512) run_item<4, NW>(it, tmp, L);
    else if (it.n <= 1024) run_item<8, NW>(it, tmp, L);
    else run_item<16, NW>(it, tmp, L);
}

// LDS (64 KiB per workgroup) allows two 4-wave workgroups per compute unit:
// two waves per SIMD, so the kernel must fit 256 registers per lane.
template <int NW>
__global__ __launch_bounds__(kWave *NW) __attribute__((amdgpu_waves_per_eu(NW == 4 ? 2 : 2)))
void k_batch(const BatchItem *items, const int *order, int *meta, double *scratch)
{
    // meta[0]: queue counter (zeroed by k_batch_reset); meta[1]: instance
    // count (written with the table, so a captured launch serves any refill)
    __shared__ Lds L;
    __shared__ int slot;
    const int count = __builtin_nontemporal_load(meta + 1);
    int *next = meta;
    for (;;) {
        if (threadIdx.x == 0)
            slot = atomicAdd(next, 1);
        __syncthreads();
        const int idx = slot;
        __syncthreads();
        if (idx >= count)
            break;   // every workgroup reaches this once the queue is drained
        const int item = order[idx];
        const BatchItem it = items[item];
        dispatch_item<NW>(it, scratch + it.scratch_off, L);
    }
}

__global__ void k_batch_reset(int *next)
{
    if (threadIdx.x == 0)
        *next = 0;
}

}  // namespace

int64_t batch_max_n() { return kMaxN; }

bool batch_threads_supported(int threads) { return threads == 256 || threads == 512; }

void launch_batch(const BatchItem *items, const int *order, int *meta, double *scratch, int threads,
                  int grid, hipStream_t st)
{
    launch("batch_reset", k_batch_reset, dim3(1), dim3(64), st, meta);
    if (threads == 512)
        launch("batch", k_batch<8>, dim3(grid), dim3(512), st, items, order, meta, scratch);
    else
        launch("batch", k_batch<4>, dim3(grid), dim3(256), st, items, order, meta, scratch);
}

}  // namespace bto
