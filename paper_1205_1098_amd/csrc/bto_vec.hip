// Vector (BLAS-1) kernels: elementwise sweeps and deterministic dot products.
//
// Every kernel streams 16-byte pairs of doubles when all of its pointers are
// 16-byte aligned (the usual case for whole tensors), else single doubles.
// Loads and stores are non-temporal: each element is touched exactly once.

#include "bto_dev.hpp"
#include "bto_internal.hpp"

namespace bto {

namespace {

constexpr int kBlock = 256;
constexpr int kUnroll = 4;  // pairs per thread in the elementwise sweeps

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

// out = op(a, b, c) over n elements.  No __restrict__: `out` may be exactly
// one of the inputs; each thread reads all of its elements before writing.
template <int OP, bool VEC>
__global__ __launch_bounds__(kBlock) void k_ew(int64_t n, const double *a, const double *b,
                                               const double *c, double s0, double s1,
                                               double *out)
{
    constexpr int NIN = ew_inputs<OP>();
    if constexpr (VEC) {
        const int64_t npair = n >> 1;
        const int64_t base = (int64_t)blockIdx.x * (kBlock * kUnroll) + threadIdx.x;
        d2 va[kUnroll], vb[kUnroll], vc[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t p = base + (int64_t)u * kBlock;
            va[u] = vb[u] = vc[u] = d2{0.0, 0.0};
            if (p < npair) {
                va[u] = ld2_nt(a + 2 * p);
                if (NIN > 1) vb[u] = ld2_nt(b + 2 * p);
                if (NIN > 2) vc[u] = ld2_nt(c + 2 * p);
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t p = base + (int64_t)u * kBlock;
            if (p < npair)
                st2_nt(out + 2 * p, ew_apply<OP>(va[u], vb[u], vc[u], s0, s1));
        }
        if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            const int64_t k = n - 1;
            out[k] = ew_apply1<OP>(a[k], NIN > 1 ? b[k] : 0.0, NIN > 2 ? c[k] : 0.0, s0, s1);
        }
    } else {
        const int64_t base = (int64_t)blockIdx.x * (kBlock * kUnroll * 2) + threadIdx.x;
        double va[2 * kUnroll], vb[2 * kUnroll], vc[2 * kUnroll];
#pragma unroll
        for (int u = 0; u < 2 * kUnroll; ++u) {
            const int64_t k = base + (int64_t)u * kBlock;
            va[u] = vb[u] = vc[u] = 0.0;
            if (k < n) {
                va[u] = a[k];
                if (NIN > 1) vb[u] = b[k];
                if (NIN > 2) vc[u] = c[k];
            }
        }
#pragma unroll
        for (int u = 0; u < 2 * kUnroll; ++u) {
            const int64_t k = base + (int64_t)u * kBlock;
            if (k < n)
                out[k] = ew_apply1<OP>(va[u], vb[u], vc[u], s0, s1);
        }
    }
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
    const int64_t per_block = kBlock * kUnroll * 2;
    dim3 grid((unsigned)ceil_div(n, per_block));
    if (vec)
        launch(names[OP], k_ew<OP, true>, grid, dim3(kBlock), st, n, a, b, c, s0, s1, out);
    else
        launch(names[OP], k_ew<OP, false>, grid, dim3(kBlock), st, n, a, b, c, s0, s1, out);
}

// ---- deterministic dot products ------------------------------------------
//
// The vector is cut into dot_parts(n) contiguous chunks of dot_chunk(n)
// elements (a multiple of 512).  Each workgroup sums its chunk with four
// rotating pair accumulators per thread, then lanes, then waves, always in
// the same order, and writes one partial; a single workgroup then sums the
// partials in a fixed tree.  The result depends on n only.

int64_t dot_chunk(int64_t n)
{
    int64_t c = ceil_div(n, 2048);
    c = ceil_div(c, 512) * 512;
    return c < 4096 ? 4096 : c;
}

__device__ __forceinline__ double block_sum_256(double v, double *lds4)
{
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        lds4[wave] = v;
    lds_barrier();
    return ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
}

// FUSED: z = w - alpha*v is stored and the partial of z.u is formed in the
// same sweep.  Otherwise the partial of w.u (v and z are not touched).
template <bool FUSED, bool VEC>
__global__ __launch_bounds__(kBlock) void k_dot_part(int64_t n, int64_t chunk, double alpha,
                                                     const double *w, const double *v,
                                                     const double *u, double *z,
                                                     double *parts)
{
    __shared__ double lds4[4];
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    d2 acc[4] = {d2{0.0, 0.0}, d2{0.0, 0.0}, d2{0.0, 0.0}, d2{0.0, 0.0}};
    if constexpr (VEC) {
        // chunk is even, so lo is even; pairs [lo/2, hi/2)
        const int64_t p0 = lo / 2, p1 = hi / 2;
        int64_t p = p0 + threadIdx.x;
        for (; p + 3 * kBlock < p1; p += 4 * kBlock) {
            d2 a[4], b[4], c[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                a[k] = ld2_nt(w + 2 * (p + k * kBlock));
                b[k] = ld2_nt(u + 2 * (p + k * kBlock));
                if (FUSED) c[k] = ld2_nt(v + 2 * (p + k * kBlock));
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                d2 zz = a[k];
                if (FUSED) {
                    zz = a[k] - alpha * c[k];
                    st2_nt(z + 2 * (p + k * kBlock), zz);
                }
                acc[k] += zz * b[k];
            }
        }
        for (int k = 0; p < p1; p += kBlock, ++k) {
            d2 a = ld2_nt(w + 2 * p), b = ld2_nt(u + 2 * p);
            d2 zz = a;
            if (FUSED) {
                zz = a - alpha * ld2_nt(v + 2 * p);
                st2_nt(z + 2 * p, zz);
            }
            acc[k & 3] += zz * b;
        }
        if ((hi & 1) && hi == n && threadIdx.x == 0) {
            const int64_t k = n - 1;
            double zz = w[k];
            if (FUSED) {
                zz = w[k] - alpha * v[k];
                z[k] = zz;
            }
            acc[0].x += zz * u[k];
        }
    } else {
        int k = 0;
        for (int64_t e = lo + threadIdx.x; e < hi; e += kBlock, ++k) {
            double zz = w[e];
            if (FUSED) {
                zz = w[e] - alpha * v[e];
                z[e] = zz;
            }
            double t = zz * u[e];
            if (k & 1) acc[(k >> 1) & 3].y += t; else acc[(k >> 1) & 3].x += t;
        }
    }
    d2 s2 = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    double s = block_sum_256(s2.x + s2.y, lds4);
    if (threadIdx.x == 0)
        parts[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_dot_finish(int64_t nparts, const double *parts,
                                                       double *r)
{
    __shared__ double lds4[4];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < nparts; k += kBlock)
        s += parts[k];
    s = block_sum_256(s, lds4);
    if (threadIdx.x == 0)
        *r = s;
}

__global__ __launch_bounds__(kBlock) void k_copy(int64_t npair, const double *src, double *dst)
{
    const int64_t base = (int64_t)blockIdx.x * (kBlock * kUnroll) + threadIdx.x;
    d2 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int64_t p = base + (int64_t)u * kBlock;
        if (p < npair) v[u] = ld2_nt(src + 2 * p);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int64_t p = base + (int64_t)u * kBlock;
        if (p < npair) st2_nt(dst + 2 * p, v[u]);
    }
}

}  // namespace

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
    return n <= 0 ? 0 : ceil_div(n, dot_chunk(n));
}

void launch_dot(bool fused_axpy, int64_t n, double alpha, const double *w, const double *v,
                const double *u, double *z, double *parts, double *r, hipStream_t st)
{
    const int64_t np = dot_parts(n);
    const int64_t chunk = dot_chunk(n);
    bool vec = aligned16(w) && aligned16(u) && (!fused_axpy || (aligned16(v) && aligned16(z)));
    dim3 grid((unsigned)np), block(kBlock);
    if (fused_axpy) {
        if (vec)
            launch("axpydot_fused", k_dot_part<true, true>, grid, block, st, n, chunk, alpha, w, v, u, z, parts);
        else
            launch("axpydot_fused", k_dot_part<true, false>, grid, block, st, n, chunk, alpha, w, v, u, z, parts);
    } else {
        if (vec)
            launch("dot_part", k_dot_part<false, true>, grid, block, st, n, chunk, alpha, w, v, u, z, parts);
        else
            launch("dot_part", k_dot_part<false, false>, grid, block, st, n, chunk, alpha, w, v, u, z, parts);
    }
    launch("dot_finish", k_dot_finish, dim3(1), block, st, np, (const double *)parts, r);
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
    launch("probe_copy", k_copy, dim3((unsigned)ceil_div(npair, kBlock * kUnroll)), dim3(kBlock),
           st, npair, src, dst);
}

void launch_triad(int64_t n, double *a, const double *b, const double *c, double s,
                  hipStream_t st)
{
    launch_ew_t<EW_AXPY>(n, b, c, nullptr, s, 0.0, a, st);
}

}  // namespace bto
