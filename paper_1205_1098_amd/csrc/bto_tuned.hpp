// The matrix sweeps' tuning slots and their default tile configurations.
//
// Each matrix sweep the entry points launch has a slot whose tile
// configuration (shape, band height, walk order) can be changed at run time
// through bto_tune_set / bto_tune_set_for, per size bucket.  The defaults are
// the best configurations the orthogonal search (fusion first, then each
// sweep's tile shape, band height and walk order, pruned by modeled
// partial-sum bytes) found on MI355X: both forms at 16384 x 16384 (which
// also serves larger problems), and the fused form for each smaller bucket,
// judged by the summed time of three square sizes across it (128/192/256,
// 300/400/512, ..., 4800/6400/8192).
#pragma once

#include "bto_internal.hpp"

namespace bto {

enum Slot {
    SLOT_BICGK_FUSED = 0,
    SLOT_GEMV_N,
    SLOT_GEMV_T,
    SLOT_GER,
    SLOT_GEMVER_P1,
    SLOT_GEMVER_P2,
    SLOT_DGEMVT_P1,
    SLOT_DGEMVT_P2,
    SLOT_COUNT
};

inline constexpr int kSlotOps[SLOT_COUNT] = {
    OP_ROWDOT | OP_COLSUM,           // BICGK_FUSED
    OP_ROWDOT,                       // GEMV_N
    OP_COLSUM,                       // GEMV_T
    OP_UPD1,                         // GER
    OP_UPD1 | OP_UPD2 | OP_COLSUM,   // GEMVER_P1
    OP_ROWDOT,                       // GEMVER_P2
    OP_COLSUM,                       // DGEMVT_P1
    OP_ROWDOT,                       // DGEMVT_P2
};

inline constexpr const char *kSlotNames[SLOT_COUNT] = {
    "bicgk_fused", "gemv_n", "gemv_t", "ger", "gemver_p1", "gemver_p2", "dgemvt_p1", "dgemvt_p2",
};

// Problems are grouped into size buckets by max(m, n): <= 256, <= 512, ...,
// <= 16384, and larger.  Each slot has a configuration per bucket.
constexpr int kSizeBuckets = 8;

inline int size_bucket(int64_t m, int64_t n)
{
    const int64_t s = m > n ? m : n;
    int b = 0;
    while (b < kSizeBuckets - 1 && (int64_t(256) << b) < s)
        ++b;
    return b;
}

// {shape, rb, rev} per slot and size bucket (written by `python -m paper_1205_1098_amd.tune --write-header`)
#define BTO_TUNED_DEFAULTS                                                                        \
    {                                                                                             \
        {{5, 128, 0}, {5, 128, 0}, {2, 32, 1}, {2, 64, 1}, {3, 128, 0}, {5, 32, 1}, {5, 128, 0}, {5, 128, 0}},  /* BICGK_FUSED */ \
        {{4, 4, 1}, {4, 4, 1}, {4, 4, 1}, {4, 4, 1}, {4, 4, 1}, {4, 4, 1}, {4, 4, 1}, {4, 4, 1}},  /* GEMV_N */ \
        {{3, 512, 0}, {3, 512, 0}, {3, 512, 0}, {3, 512, 0}, {3, 512, 0}, {3, 512, 0}, {3, 512, 0}, {3, 512, 0}},  /* GEMV_T */ \
        {{8, 4, 0}, {8, 4, 0}, {8, 4, 0}, {8, 4, 0}, {8, 4, 0}, {8, 4, 0}, {8, 4, 0}, {8, 4, 0}},  /* GER */ \
        {{6, 128, 0}, {10, 32, 1}, {11, 128, 1}, {13, 32, 0}, {12, 32, 1}, {12, 32, 0}, {11, 32, 0}, {11, 32, 0}},  /* GEMVER_P1 */ \
        {{4, 4, 1}, {4, 4, 1}, {2, 8, 1}, {3, 8, 0}, {4, 4, 0}, {3, 16, 0}, {4, 4, 1}, {4, 4, 1}},  /* GEMVER_P2 */ \
        {{3, 32, 0}, {3, 32, 0}, {3, 32, 1}, {2, 32, 1}, {3, 32, 0}, {3, 64, 0}, {3, 512, 1}, {3, 512, 1}},  /* DGEMVT_P1 */ \
        {{2, 8, 0}, {1, 4, 0}, {3, 4, 1}, {3, 8, 0}, {2, 16, 0}, {3, 64, 0}, {4, 4, 0}, {4, 4, 0}},  /* DGEMVT_P2 */ \
    }

// workgroup size of the row-resident ATAX and BiCGK sweeps per size bucket
// (BiCGK: 0 selects the tile sweep of slot bicgk_fused)
#define BTO_TUNED_ATAX_ROWRES {512, 1024, 512, 512, 1024, 512, 512, 512}
#define BTO_TUNED_BICGK_ROWRES {256, 256, 1024, 256, 512, 512, 512, 512}

}  // namespace bto
