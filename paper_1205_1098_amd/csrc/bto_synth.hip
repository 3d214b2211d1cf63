// Seeded synthetic data generated in device memory.
//
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a counter-based
// generator: element k of a stream whose state starts at `state` is
// mix64(state + (k+1) * 0x9E3779B97F4A7C15).  Uniform doubles on [-1, 1)
// are ((x >> 11) * 2^-53) * 2 - 1 and small integers on [lo, hi] are
// lo + (((x >> 11) * (hi - lo + 1)) >> 53), both exact, so the host
// generator of the Python package produces the same bits.  None of the
// kernels' arithmetic lives here.

#include "bto.h"
#include "bto_dev.hpp"
#include "bto_internal.hpp"

namespace bto {

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Fill a rows x cols block with leading dimension ld; element (i, j) is
// stream element offset + i*cols + j.
__global__ __launch_bounds__(256) void k_fill(double *out, int64_t rows, int64_t cols, int64_t ld,
                                              uint64_t state, int64_t offset, int kind, int lo,
                                              int hi)
{
    const int64_t total = rows * cols;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * 256) {
        const int64_t i = t / cols, j = t - i * cols;
        const uint64_t k = (uint64_t)(offset + t);
        const uint64_t x = mix64(state + (k + 1) * 0x9E3779B97F4A7C15ull) >> 11;
        double v;
        if (kind == 0)
            v = (double)x * 0x1.0p-53 * 2.0 - 1.0;
        else
            v = (double)(int64_t)lo + (double)(int64_t)((x * (uint64_t)(hi - lo + 1)) >> 53);
        out[i * ld + j] = v;
    }
}

}  // namespace

}  // namespace bto

extern "C" bto_status bto_synth_fill(double *out, int64_t rows, int64_t cols, int64_t ld,
                                     uint64_t state, int64_t offset, int kind, int lo, int hi,
                                     hipStream_t stream)
{
    using namespace bto;
    if (rows < 0 || cols < 0 || ld < cols || (rows * cols > 0 && !out) || offset < 0 ||
        (kind != 0 && kind != 1) || (kind == 1 && hi < lo))
        return BTO_ERR_INVALID_ARG;
    const int64_t total = rows * cols;
    if (total == 0)
        return BTO_SUCCESS;
    int64_t blocks = ceil_div(total, 256);
    if (blocks > 65536)
        blocks = 65536;
    launch("synth_fill", k_fill, dim3((unsigned)blocks), dim3(256), stream, out, rows, cols, ld,
           state, offset, kind, lo, hi);
    return hipGetLastError() == hipSuccess ? BTO_SUCCESS : BTO_ERR_HIP;
}
