// Device-side helpers shared by the gfx950 kernels of libbto.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bto {

typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kWave = 64;

// Move a double across lanes with a DPP control (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint32_t>(lo));
}

// Swap a double with the lane 16 away inside each half-wave (ds_swizzle
// bit mode: and 0x1F, or 0, xor 0x10).
__device__ __forceinline__ double swz16_f64(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_ds_swizzle(static_cast<int>(b), 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle(static_cast<int>(b >> 32), 0x401F);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint32_t>(lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(b), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// Sum over the 64 lanes of a wavefront.  Each step adds a lane's value to
// its partner's (quad swaps, half-row and row mirrors, the lane 16 away);
// partners add the same two numbers and IEEE addition commutes, so after
// the steps every lane of a half-wave holds the same half sum, and the two
// halves are added once, in lane order.  All lanes return the same value,
// which depends only on the inputs.  Needs all 64 lanes active.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    v += swz16_f64(v);
    return readlane_f64(v, 0) + readlane_f64(v, 32);
}

// The lane permutes of gfx950 that trade half-waves and rows between two
// registers (each 32-bit half of a double separately).  swap32: x keeps its
// lanes 0-31 and takes y's lanes 0-31 as its lanes 32-63; y takes x's lanes
// 32-63 as its lanes 0-31 and keeps its own lanes 32-63.  swap16: the same
// within each half-wave, with 16-lane rows.
__device__ __forceinline__ void swap32_f64(double &x, double &y)
{
    const uint64_t xb = __builtin_bit_cast(uint64_t, x), yb = __builtin_bit_cast(uint64_t, y);
    const auto lo = __builtin_amdgcn_permlane32_swap(static_cast<uint32_t>(xb),
                                                     static_cast<uint32_t>(yb), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(static_cast<uint32_t>(xb >> 32),
                                                     static_cast<uint32_t>(yb >> 32), false, false);
    x = __builtin_bit_cast(double, (static_cast<uint64_t>(hi[0]) << 32) | lo[0]);
    y = __builtin_bit_cast(double, (static_cast<uint64_t>(hi[1]) << 32) | lo[1]);
}

__device__ __forceinline__ void swap16_f64(double &x, double &y)
{
    const uint64_t xb = __builtin_bit_cast(uint64_t, x), yb = __builtin_bit_cast(uint64_t, y);
    const auto lo = __builtin_amdgcn_permlane16_swap(static_cast<uint32_t>(xb),
                                                     static_cast<uint32_t>(yb), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(static_cast<uint32_t>(xb >> 32),
                                                     static_cast<uint32_t>(yb >> 32), false, false);
    x = __builtin_bit_cast(double, (static_cast<uint64_t>(hi[0]) << 32) | lo[0]);
    y = __builtin_bit_cast(double, (static_cast<uint64_t>(hi[1]) << 32) | lo[1]);
}

// Sum over each 16-lane row: quad swaps, then the half-row and row mirrors;
// every lane of a row ends with the same row sum.
__device__ __forceinline__ double row_sum16(double v)
{
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);   // row_half_mirror
    v += dpp_f64<0x140>(v);   // row_mirror
    return v;
}

// The sums over the 64 lanes of P values at once (2 <= P <= 8), cheaper
// than P wave_sums: values are paired and each half-wave keeps one of a
// pair (lanes l and l + 32 added), then each row of a half-wave keeps one
// of a pair of those (lanes l and l + 16 added), so that one set of row
// reductions serves four values.  Row r of the k-th register then holds
// value 4k + (0, 2, 1, 3)[r]; a missing partner is a zero.  The order of
// the additions is fixed, so the results depend only on the inputs (they
// round differently from wave_sum's).  Needs all 64 lanes active.
template <int P>
__device__ __forceinline__ void wave_sums(const double (&v)[P], double (&out)[P])
{
    static_assert(P >= 2 && P <= 8, "two to eight values");
    constexpr int NW = (P + 1) / 2, NU = (NW + 1) / 2;
    double w[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        double x = v[2 * j], y = 2 * j + 1 < P ? v[2 * j + 1] : 0.0;
        swap32_f64(x, y);
        w[j] = x + y;
    }
    double u[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        double x = w[2 * k], y = 2 * k + 1 < NW ? w[2 * k + 1] : 0.0;
        swap16_f64(x, y);
        u[k] = row_sum16(x + y);
    }
    constexpr int kRowLane[4] = {0, 32, 16, 48};
#pragma unroll
    for (int q = 0; q < P; ++q)
        out[q] = readlane_f64(u[q / 4], kRowLane[q % 4]);
}

// Workgroup barrier that orders LDS accesses only.  Global loads in flight
// (prefetches) are not waited for, unlike __syncthreads().
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Streaming (non-temporal) 16-byte load and store: data touched once.
__device__ __forceinline__ d2 ld2_nt(const double *p)
{
    return __builtin_nontemporal_load(reinterpret_cast<const d2 *>(p));
}

__device__ __forceinline__ void st2_nt(double *p, d2 v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<d2 *>(p));
}

__device__ __forceinline__ double ld1_nt(const double *p)
{
    return __builtin_nontemporal_load(p);
}

__device__ __forceinline__ void st1_nt(double *p, double v)
{
    __builtin_nontemporal_store(v, p);
}

// Read a double whose address is the same in every lane through the scalar
// data cache (a scalar load, counted by lgkmcnt): waiting for it never waits
// for the wave's outstanding vector loads.  The data must not change while
// the kernel runs.  Reads only: nothing here writes through that cache.
__device__ __forceinline__ double ld_uniform(const double *p)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a >> 32));
    typedef const double __attribute__((address_space(4))) *cptr;
    return *reinterpret_cast<cptr>((static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ __forceinline__ d2 ld2(const double *p)
{
    return *reinterpret_cast<const d2 *>(p);
}

}  // namespace bto
