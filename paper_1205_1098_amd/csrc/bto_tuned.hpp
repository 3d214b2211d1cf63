// The matrix sweeps' tuning slots and their default tile configurations.
//
// Each matrix sweep the entry points launch has a slot whose tile
// configuration (shape, band height, walk order) can be changed at run time
// through bto_tune_set.  The defaults are the best configurations the
// orthogonal search (fusion first, then each sweep's tile shape, band height
// and walk order) found for 16384 x 16384 on MI355X, each form searched
// separately.  The row-resident sweeps' workgroup sizes live with their
// kernels.
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

// {shape, rb, rev} per slot
#define BTO_TUNED_DEFAULTS                                                                        \
    {                                                                                             \
        {5, 128, 0},  /* BICGK_FUSED: 4 x 2 waves, 8 pairs per lane, 2 rows in flight */          \
        {4, 4, 1},    /* GEMV_N: 4 waves across 4096 columns, one row per wave */                 \
        {3, 512, 0},  /* GEMV_T: 4 x 4 waves, 512-row bands */                                    \
        {8, 4, 0},    /* GER: one row per wave, 512-column wave tiles */                          \
        {10, 32, 1},  /* GEMVER_P1: 16 waves down 256 columns, 2 rows each, 3 rows in flight */   \
        {4, 4, 1},    /* GEMVER_P2: one row per wave, bands walked backwards */                   \
        {3, 512, 1},  /* DGEMVT_P1 */                                                             \
        {4, 4, 0},    /* DGEMVT_P2 */                                                             \
    }

}  // namespace bto
