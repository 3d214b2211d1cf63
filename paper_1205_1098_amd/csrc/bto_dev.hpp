// Device-side helpers shared by the gfx950 kernels of libbto.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bto {

typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kWave = 64;

// Sum over the 64 lanes of a wavefront by an xor butterfly.  Every lane
// adds the same two operands at every step (IEEE addition commutes), so
// all lanes end with the identical value and the result depends only on
// the lane values, never on timing.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, kWave);
    return v;
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

__device__ __forceinline__ d2 ld2(const double *p)
{
    return *reinterpret_cast<const d2 *>(p);
}

}  // namespace bto
