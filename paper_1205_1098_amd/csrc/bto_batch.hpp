// Device-side description of one batched instance (shared by the batch
// kernel and the plan builder).
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace bto {

struct BatchItem {
    int32_t kind;      // BTO_K_GEMVER, BTO_K_BICGK or BTO_K_ATAX
    int32_t form;      // BTO_FUSED or BTO_UNFUSED
    int64_t m, n, lda, ldb;
    double alpha, beta;
    const double *A;
    double *B;
    const double *vec[6];
    double *out[2];
    int64_t scratch_off;   // doubles into the plan's scratch (unfused ATAX temporary)
};

int64_t batch_max_n();
bool batch_threads_supported(int threads);
// meta = {queue counter, instance count}
void launch_batch(const BatchItem *items, const int *order, int *meta, double *scratch, int threads,
                  int grid, hipStream_t st);

}  // namespace bto
