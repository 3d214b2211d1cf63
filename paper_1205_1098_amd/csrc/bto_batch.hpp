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
    int64_t part_off;      // doubles into the scratch: column-sum partials of the tiles
    int64_t tile_rows;     // rows per tile of a split instance
    int32_t ntiles;        // tiles of a split instance (1: not split)
    int32_t pad;
};

// One unit of queued work: a whole instance (phase 0), a row tile of the
// first sweep of a split fused instance (phase 1), or a row tile of GEMVER's
// second sweep (phase 2), rows [r0, r1).
struct BatchUnit {
    int32_t item;
    int32_t phase;
    int64_t r0, r1;
};

// The plan's device control block: the queue counter, the unit count, a
// flag set when a wait gave up, and the instance count (whose pairs of
// sync counters the reset kernel clears).
enum { kMetaNext = 0, kMetaUnits = 1, kMetaError = 2, kMetaItems = 3, kMetaInts = 4 };

constexpr int kBatchMaxTiles = 64;                      // tiles per split instance
// Defaults from the batch-knob search (4096 mixed GEMVER/BiCGK instances, n
// log-uniform on [64, 2048], MI355X): fused instances, 512-thread
// workgroups, two per compute unit (2, 3 or 4 tie within 0.1%), and row
// tiles only for matrices above 16 MiB (no tiles, 16 or 32 MiB tie within
// 0.6%; tiles bound the tail of a batch with one very large instance).
constexpr int kBatchDefaultThreads = 512;
constexpr int kBatchDefaultWgsPerCu = 2;
constexpr int64_t kBatchSplitBytes = 16ll << 20;        // default matrix bytes per tile

int64_t batch_max_n();
bool batch_threads_supported(int threads);
void launch_batch(const BatchItem *items, const BatchUnit *units, int *meta, int *sync,
                  double *scratch, int threads, int grid, hipStream_t st);

}  // namespace bto
