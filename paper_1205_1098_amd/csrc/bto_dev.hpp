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
