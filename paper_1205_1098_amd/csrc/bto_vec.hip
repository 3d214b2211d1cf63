// Vector (BLAS-1) kernels: elementwise sweeps and deterministic dot products.
//
// Every kernel streams 16-byte pairs of doubles when all of its pointers are
// 16-byte aligned (the usual case for whole tensors), else single doubles.
// Loads and stores are non-temporal: each element is touched exactly once.

#include "bto_dev.hpp"
#include "bto_internal.hpp"

namespace bto {

namespace {

constexpr int kEwBlock = 128;     // threads per workgroup of the elementwise sweeps
// The dot products cover 2048 elements per workgroup: the fused AXPYDOT
// (three streams in, one out) with 1024 threads of one pair each, the plain
// dot (two streams in) with 256 threads of four pairs each; each is the
// faster arrangement for its traffic (by 4% and by 28%).
constexpr int kDotElems = 2048;
template <bool FUSED> constexpr int dot_block() { return FUSED ? 1024 : 256; }
template <bool FUSED> constexpr int dot_unroll() { return kDotElems / 2 / dot_block<FUSED>(); }

template <int OP>
__device__ __forceinline__ d2 ew_apply(d2 a, d2 b, d2 c, double s0, double s1)
{
    if constexpr (OP == EW_VADD3)
        return (a + b) + c;
    else if constexpr (OP == EW_ADD2)
        return a + b;
    else if constexpr (OP == EW_WAXPBY)
        return s0 * a + s1 * b;
    else if constexpr (OP == EW_SCAL)
        return s0 * a;
    else if constexpr (OP == EW_AXPY)
        return a + s0 * b;
    else
        return a - s0 * b;
}

template <int OP>
__device__ __forceinline__ double ew_apply1(double a, double b, double c, double s0, double s1)
{
    d2 r = ew_apply<OP>(d2{a, 0.0}, d2{b, 0.0}, d2{c, 0.0}, s0, s1);
    return r.x;
}

template <int OP>
constexpr int ew_inputs()
{
    return OP == EW_VADD3 ? 3 : (OP == EW_SCAL ? 1 : 2);
}

// out = op(a, b, c) over n elements, one 16-byte pair per thread: short-lived
// waves that load, compute, store and retire stream best when each element is
// both read and written.  No __restrict__: `out` may be exactly one of the
// inputs; each thread reads its elements before writing them.
template <int OP, bool VEC>
__global__ __launch_bounds__(kEwBlock) void k_ew(int64_t n, const double *a, const double *b,
                                                 const double *c, double s0, double s1,
                                                 double *out)
{
    constexpr int NIN = ew_inputs<OP>();
    if constexpr (VEC) {
        const int64_t p = (int64_t)blockIdx.x * kEwBlock + threadIdx.x;
        if (p < (n >> 1)) {
            d2 va = ld2_nt(a + 2 * p), vb{0.0, 0.0}, vc{0.0, 0.0};
            if (NIN > 1) vb = ld2_nt(b + 2 * p);
            if (NIN > 2) vc = ld2_nt(c + 2 * p);
            st2_nt(out + 2 * p, ew_apply<OP>(va, vb, vc, s0, s1));
        }
        if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            const int64_t k = n - 1;
            out[k] = ew_apply1<OP>(a[k], NIN > 1 ? b[k] : 0.0, NIN > 2 ? c[k] : 0.0, s0, s1);
        }
    } else {
        const int64_t base = (int64_t)blockIdx.x * (2 * kEwBlock) + threadIdx.x;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t k = base + (int64_t)u * kEwBlock;
            if (k < n)
                out[k] = ew_apply1<OP>(a[k], NIN > 1 ? b[k] : 0.0, NIN > 2 ? c[k] : 0.0, s0, s1);
        }
    }
}

// Kernel-argument pointers inside a struct are not known to address global
// memory; say so, so that the loads are global (not flat) loads.
__device__ __forceinline__ const double *glob(const double *p)
{
    return (const double *)(const __attribute__((address_space(1))) double *)(uintptr_t)p;
}

// out = c[0] x[0] + c[1] x[1] + ... (left to right), K inputs, one pass.
template <int K, bool VEC>
__global__ __launch_bounds__(kEwBlock) void k_lincomb(int64_t n, LinArgs a)
{
    if constexpr (VEC) {
        const int64_t p = (int64_t)blockIdx.x * kEwBlock + threadIdx.x;
        if (p < (n >> 1)) {
            d2 v[K];
#pragma unroll
            for (int k = 0; k < K; ++k)
                v[k] = ld2_nt(glob(a.x[k]) + 2 * p);
            d2 acc = a.c[0] * v[0];
#pragma unroll
            for (int k = 1; k < K; ++k)
                acc = acc + a.c[k] * v[k];
            st2_nt(a.out + 2 * p, acc);
        }
        if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            const int64_t i = n - 1;
            double acc = a.c[0] * glob(a.x[0])[i];
#pragma unroll
            for (int k = 1; k < K; ++k)
                acc = acc + a.c[k] * glob(a.x[k])[i];
            a.out[i] = acc;
        }
    } else {
        const int64_t base = (int64_t)blockIdx.x * (2 * kEwBlock) + threadIdx.x;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t i = base + (int64_t)u * kEwBlock;
            if (i < n) {
                double acc = a.c[0] * glob(a.x[0])[i];
#pragma unroll
                for (int k = 1; k < K; ++k)
                    acc = acc + a.c[k] * glob(a.x[k])[i];
                a.out[i] = acc;
            }
        }
    }
}

template <int K>
void launch_lincomb_t(int64_t n, const LinArgs &a, hipStream_t st)
{
    bool vec = aligned16(a.out);
    for (int k = 0; k < K; ++k)
        vec = vec && aligned16(a.x[k]);
    dim3 grid((unsigned)ceil_div(n, 2 * kEwBlock));
    if (vec)
        launch("ew_lincomb", k_lincomb<K, true>, grid, dim3(kEwBlock), st, n, a);
    else
        launch("ew_lincomb", k_lincomb<K, false>, grid, dim3(kEwBlock), st, n, a);
}

template <int OP>
void launch_ew_t(int64_t n, const double *a, const double *b, const double *c, double s0,
                 double s1, double *out, hipStream_t st)
{
    constexpr int NIN = ew_inputs<OP>();
    bool vec = aligned16(a) && aligned16(out) && (NIN < 2 || aligned16(b)) &&
               (NIN < 3 || aligned16(c));
    static const char *names[] = {"ew_vadd3", "ew_add2", "ew_waxpby", "ew_scal", "ew_axpy",
                                  "ew_axmy"};
    dim3 grid((unsigned)ceil_div(n, 2 * kEwBlock));
    if (vec)
        launch(names[OP], k_ew<OP, true>, grid, dim3(kEwBlock), st, n, a, b, c, s0, s1, out);
    else
        launch(names[OP], k_ew<OP, false>, grid, dim3(kEwBlock), st, n, a, b, c, s0, s1, out);
}

// ---- deterministic dot products ------------------------------------------
//
// Workgroup b owns elements [2048 b, 2048 (b+1)): with T threads of U pairs
// (1024 x 1 fused, 256 x 4 plain) thread t takes pairs 1024 b + t + T u,
// sums its products in u order, then the lanes and then the waves are
// added, always in the same order, and the workgroup writes one partial.  A
// single 1024-thread workgroup then sums the partials in a fixed tree.  The
// result depends on n and the form only.

constexpr int64_t kDotTile = kDotElems;   // elements per workgroup

__device__ __forceinline__ double block_sum(double v, double *lds, int nwaves)
{
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        lds[wave] = v;
    lds_barrier();
    double s = lds[0];
    for (int w = 1; w < nwaves; ++w)
        s += lds[w];
    return s;
}

// FUSED: z = w - alpha*v is stored and the partial of z.u is formed in the
// same sweep.  Otherwise the partial of w.u (v and z are not touched).
template <bool FUSED, bool VEC>
__global__ __launch_bounds__(dot_block<FUSED>()) void k_dot_part(int64_t n, double alpha,
                                                                 const double *w, const double *v,
                                                                 const double *u, double *z,
                                                                 double *parts)
{
    constexpr int kBlock = dot_block<FUSED>();
    constexpr int kUnroll = dot_unroll<FUSED>();
    __shared__ double lds[kBlock / kWave];
    d2 acc{0.0, 0.0};
    if constexpr (VEC) {
        const int64_t npair = n >> 1;
        const int64_t base = (int64_t)blockIdx.x * (kBlock * kUnroll) + threadIdx.x;
        d2 a[kUnroll], b[kUnroll], c[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const int64_t p = base + (int64_t)k * kBlock;
            a[k] = b[k] = c[k] = d2{0.0, 0.0};
            if (p < npair) {
                a[k] = ld2_nt(w + 2 * p);
                b[k] = ld2_nt(u + 2 * p);
                if (FUSED) c[k] = ld2_nt(v + 2 * p);
            }
        }
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const int64_t p = base + (int64_t)k * kBlock;
            if (p < npair) {
                d2 zz = a[k];
                if (FUSED) {
                    zz = a[k] - alpha * c[k];
                    st2_nt(z + 2 * p, zz);
                }
                acc += zz * b[k];
            }
        }
        if ((n & 1) && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
            const int64_t k = n - 1;
            double zz = w[k];
            if (FUSED) {
                zz = w[k] - alpha * v[k];
                z[k] = zz;
            }
            acc.x += zz * u[k];
        }
    } else {
        const int64_t base = (int64_t)blockIdx.x * kDotTile + threadIdx.x;
#pragma unroll
        for (int k = 0; k < 2 * kUnroll; ++k) {
            const int64_t e = base + (int64_t)k * kBlock;
            if (e < n) {
                double zz = w[e];
                if (FUSED) {
                    zz = w[e] - alpha * v[e];
                    z[e] = zz;
                }
                if (k & 1) acc.y += zz * u[e]; else acc.x += zz * u[e];
            }
        }
    }
    double s = block_sum(acc.x + acc.y, lds, kBlock / kWave);
    if (threadIdx.x == 0)
        parts[blockIdx.x] = s;
}

constexpr int kFinishBlock = 1024;

__global__ __launch_bounds__(kFinishBlock) void k_dot_finish(int64_t nparts,
                                                             const double *parts, double *r)
{
    __shared__ double lds[kFinishBlock / kWave];
    // thread t adds parts t, t + T, t + 2T, ... in that order; eight loads
    // are issued before their sums so that they are in flight together
    double s = 0.0;
    int64_t k = threadIdx.x;
    for (; k + 7 * kFinishBlock < nparts; k += 8 * kFinishBlock) {
        double t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            t[e] = parts[k + e * kFinishBlock];
#pragma unroll
        for (int e = 0; e < 8; ++e)
            s += t[e];
    }
    for (; k < nparts; k += kFinishBlock)
        s += parts[k];
    s = block_sum(s, lds, kFinishBlock / kWave);
    if (threadIdx.x == 0)
        *r = s;
}

// ---- read probe ------------------------------------------------------------
//
// out = sum of n doubles, as a pure streaming read: workgroup b owns elements
// [kReadChunk b, kReadChunk (b+1)); each of its threads keeps kReadPairs
// 16-byte loads of the next stretch in flight while it adds the current one,
// so a workgroup streams 256 KiB before it retires.  Thread t adds pairs t +
// kReadBlock k of each stretch in stretch order, then the lanes and waves are
// added in a fixed order and the finish sums the workgroup partials: the
// result depends on n only.
//
// The workgroup's LDS is sized so that at most two workgroups share a compute
// unit: with fewer reads in flight the sweep runs faster (2^28 doubles: about
// 7.2 TB/s at two workgroups per CU against 7.1 at eight), as the matrix
// sweeps, whose registers hold their occupancy to three waves per SIMD, read.
// Four loads in flight per thread read faster than two or eight.

constexpr int kReadBlock = 256;
constexpr int kReadPairs = 4;
constexpr int kReadIters = 16;
constexpr int64_t kReadChunk = (int64_t)kReadBlock * kReadPairs * 2 * kReadIters;
constexpr int kReadLdsDoubles = 80 * 1024 / 8;   // 80 KiB: two workgroups per CU

template <bool VEC>
__global__ __launch_bounds__(kReadBlock) void k_read_part(int64_t n, const double *src,
                                                          double *parts)
{
    __shared__ double lds[kReadLdsDoubles];   // the first kReadBlock / kWave hold wave sums
    const int64_t base = (int64_t)blockIdx.x * kReadChunk;
    d2 acc{0.0, 0.0};
    if (VEC && base + kReadChunk <= n) {
        const double *p = src + base + 2 * threadIdx.x;
        constexpr int64_t kStretch = 2 * kReadBlock * kReadPairs;   // doubles per stretch
        d2 cur[kReadPairs], nxt[kReadPairs];
#pragma unroll
        for (int k = 0; k < kReadPairs; ++k)
            cur[k] = ld2_nt(p + 2 * kReadBlock * k);
#pragma unroll
        for (int it = 0; it < kReadIters; ++it) {
            if (it + 1 < kReadIters) {
#pragma unroll
                for (int k = 0; k < kReadPairs; ++k)
                    nxt[k] = ld2_nt(p + (it + 1) * kStretch + 2 * kReadBlock * k);
            }
#pragma unroll
            for (int k = 0; k < kReadPairs; ++k)
                acc += cur[k];
#pragma unroll
            for (int k = 0; k < kReadPairs; ++k)
                cur[k] = nxt[k];
        }
    } else {
        const int64_t end = base + kReadChunk < n ? base + kReadChunk : n;
        for (int64_t e = base + threadIdx.x; e < end; e += kReadBlock)
            acc.x += src[e];
    }
    const double s = block_sum(acc.x + acc.y, lds, kReadBlock / kWave);
    if (threadIdx.x == 0)
        parts[blockIdx.x] = s;
}

__global__ __launch_bounds__(kEwBlock) void k_copy(int64_t npair, const double *src, double *dst)
{
    const int64_t p = (int64_t)blockIdx.x * kEwBlock + threadIdx.x;
    if (p < npair)
        st2_nt(dst + 2 * p, ld2_nt(src + 2 * p));
}

}  // namespace

void launch_lincomb(int64_t n, int count, const LinArgs &a, hipStream_t st)
{
    if (n <= 0)
        return;
    switch (count) {
    case 1: launch_lincomb_t<1>(n, a, st); break;
    case 2: launch_lincomb_t<2>(n, a, st); break;
    case 3: launch_lincomb_t<3>(n, a, st); break;
    case 4: launch_lincomb_t<4>(n, a, st); break;
    case 5: launch_lincomb_t<5>(n, a, st); break;
    case 6: launch_lincomb_t<6>(n, a, st); break;
    case 7: launch_lincomb_t<7>(n, a, st); break;
    case 8: launch_lincomb_t<8>(n, a, st); break;
    default: break;
    }
}

void launch_ew(EwOp op, int64_t n, const double *a, const double *b, const double *c,
               double s0, double s1, double *out, hipStream_t st)
{
    if (n <= 0)
        return;
    switch (op) {
    case EW_VADD3: launch_ew_t<EW_VADD3>(n, a, b, c, s0, s1, out, st); break;
    case EW_ADD2: launch_ew_t<EW_ADD2>(n, a, b, c, s0, s1, out, st); break;
    case EW_WAXPBY: launch_ew_t<EW_WAXPBY>(n, a, b, c, s0, s1, out, st); break;
    case EW_SCAL: launch_ew_t<EW_SCAL>(n, a, b, c, s0, s1, out, st); break;
    case EW_AXPY: launch_ew_t<EW_AXPY>(n, a, b, c, s0, s1, out, st); break;
    case EW_AXMY: launch_ew_t<EW_AXMY>(n, a, b, c, s0, s1, out, st); break;
    }
}

int64_t dot_parts(int64_t n)
{
    return n <= 0 ? 0 : ceil_div(n, kDotTile);
}

void launch_dot(bool fused_axpy, int64_t n, double alpha, const double *w, const double *v,
                const double *u, double *z, double *parts, double *r, hipStream_t st)
{
    const int64_t np = dot_parts(n);
    bool vec = aligned16(w) && aligned16(u) && (!fused_axpy || (aligned16(v) && aligned16(z)));
    dim3 grid((unsigned)np);
    const dim3 block(fused_axpy ? dot_block<true>() : dot_block<false>());
    if (fused_axpy) {
        if (vec)
            launch("axpydot_fused", k_dot_part<true, true>, grid, block, st, n, alpha, w, v, u, z, parts);
        else
            launch("axpydot_fused", k_dot_part<true, false>, grid, block, st, n, alpha, w, v, u, z, parts);
    } else {
        if (vec)
            launch("dot_part", k_dot_part<false, true>, grid, block, st, n, alpha, w, v, u, z, parts);
        else
            launch("dot_part", k_dot_part<false, false>, grid, block, st, n, alpha, w, v, u, z, parts);
    }
    launch("dot_finish", k_dot_finish, dim3(1), dim3(kFinishBlock), st, np, (const double *)parts,
           r);
}

int64_t read_parts(int64_t n) { return n <= 0 ? 0 : ceil_div(n, kReadChunk); }

void launch_read(int64_t n, const double *src, double *parts, double *out, hipStream_t st)
{
    const int64_t np = read_parts(n);
    if (aligned16(src))
        launch("probe_read", k_read_part<true>, dim3((unsigned)np), dim3(kReadBlock), st, n, src,
               parts);
    else
        launch("probe_read", k_read_part<false>, dim3((unsigned)np), dim3(kReadBlock), st, n, src,
               parts);
    launch("dot_finish", k_dot_finish, dim3(1), dim3(kFinishBlock), st, np, (const double *)parts,
           out);
}

void launch_copy(int64_t n, const double *src, double *dst, hipStream_t st)
{
    if (n <= 0)
        return;
    if ((n & 1) || !aligned16(src) || !aligned16(dst)) {
        launch_ew_t<EW_SCAL>(n, src, nullptr, nullptr, 1.0, 0.0, dst, st);
        return;
    }
    const int64_t npair = n / 2;
    launch("probe_copy", k_copy, dim3((unsigned)ceil_div(npair, kEwBlock)), dim3(kEwBlock), st,
           npair, src, dst);
}

void launch_triad(int64_t n, double *a, const double *b, const double *c, double s,
                  hipStream_t st)
{
    launch_ew_t<EW_AXPY>(n, b, c, nullptr, s, 0.0, a, st);
}

}  // namespace bto
