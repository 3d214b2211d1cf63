// Tiled batches: the sweeps of many fused GEMVER and BiCGK instances cut
// into workgroup tiles (a sweep of one instance, a band of rows, a block of
// columns), with the same tile_block as the single-sweep kernel k_tile.
//
// The tiles of one kind form a group, and each group is one launch of a
// kernel specialised for its tile shape and operations: the first sweeps
// (GEMVER's, which store B, together with BiCGK's, each tile taking its
// operations from its instance's entry), then GEMVER's second sweeps of
// narrow and of wide matrices.  A launch has either one workgroup per tile or a fixed number
// of persistent workgroups that step through the group's tiles (tile k,
// k + grid, k + 2 grid, ..., where the first sweeps first deal the tiles out
// in runs per XCD).  The groups' first tile and tile count are
// read from a small device header, so a plan can be refilled with other
// instances without changing the launches (a captured graph stays valid).
// A persistent workgroup fetches the record of its next tile before it
// sweeps the current one.

#include "bto_dev.hpp"
#include "bto_internal.hpp"
#include "bto_tile.hpp"

namespace bto {

namespace {

// The workgroup shapes of the tiled batches {KV, D, WC, WR}: a block is
// WC * 128 * KV columns wide and its band's rows are split over WR row
// groups, each keeping D rows of loads in flight per wave.
struct BtShapeDef {
    int kv, d, wc, wr;
};
constexpr BtShapeDef kBtShapes[] = {
    // row groups combined in LDS at the end of each tile
    {1, 2, 1, 16}, {2, 2, 4, 4}, {2, 2, 1, 8}, {2, 4, 1, 4}, {1, 8, 1, 4},
    // one row group: every wave sweeps the whole band of its columns and
    // writes its own column sums, with no barrier
    {1, 4, 4, 1}, {1, 8, 4, 1}, {2, 4, 2, 1}, {2, 4, 4, 1}, {1, 4, 2, 1}, {1, 8, 2, 1},
    {2, 8, 2, 1},
};
static_assert(sizeof(kBtShapes) / sizeof(kBtShapes[0]) == kBtShapeCount, "shape table size");

constexpr int kStoreOps = OP_UPD1 | OP_UPD2 | OP_COLSUM;
constexpr int kBicgkOps = OP_ROWDOT | OP_COLSUM;
constexpr int kRowOps = OP_ROWDOT;

// The sweep of one tile, in bands of the entry's height.  OPS = kBtFirstOps:
// the entry's ops, a store sweep (GEMVER's first) or a BiCGK sweep.
template <int KV, int D, int WC, int WR, int OPS>
__device__ __forceinline__ void bt_tile(const BTileEntry &e, const BTileUnit &u, double *lds)
{
    const int rb = e.rb;
    TileArgs a = e.a;
    globalize(a);
    if constexpr (OPS == kBtFirstOps) {
        if (e.ops == kStoreOps) {
            if (e.vec)
                tile_block<KV, D, WC, WR, kStoreOps, true>(a, u.band, u.cblk, rb, lds);
            else
                tile_block<KV, D, WC, WR, kStoreOps, false>(a, u.band, u.cblk, rb, lds);
        } else {
            if (e.vec)
                tile_block<KV, D, WC, WR, kBicgkOps, true>(a, u.band, u.cblk, rb, lds);
            else
                tile_block<KV, D, WC, WR, kBicgkOps, false>(a, u.band, u.cblk, rb, lds);
        }
    } else {
        if (e.vec)
            tile_block<KV, D, WC, WR, OPS, true>(a, u.band, u.cblk, rb, lds);
        else
            tile_block<KV, D, WC, WR, OPS, false>(a, u.band, u.cblk, rb, lds);
    }
}

// Workgroups of a launch are handed to the chip's eight XCDs in turn
// (workgroup k to XCD k mod 8), and each XCD has an L2 cache of its own.  The
// first sweeps give XCD x a contiguous run of the group's tiles rather than
// every eighth tile, so neighbouring tiles of one instance -- which share the
// cache lines at their edges when a row is not a whole number of lines --
// meet in one L2.  The runs are as even as possible (the first total mod 8
// XCDs take one tile more), so the map is a permutation of [0, total) for any
// total and any grid; persistent workgroups keep their XCD when the grid is a
// multiple of eight, as it is (a multiple of the CU count).
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_run_tile(int v, int total)
{
    const int per = total / kXcds, extra = total % kXcds;
    const int x = v % kXcds;
    return x * per + (x < extra ? x : extra) + v / kXcds;
}

template <int KV, int D, int WC, int WR, int OPS>
__global__ __launch_bounds__(kWave *WC *WR) void k_bt(const BTileEntry *__restrict__ entries,
                                                      const BTileUnit *__restrict__ units,
                                                      const int *__restrict__ hdr, int group)
{
    constexpr bool COLSUM = OPS == kBtFirstOps || (OPS & OP_COLSUM);
    __shared__ double lds[COLSUM ? tile_lds_doubles<KV, WC, WR>() : 1];
    const int first = hdr[2 * group], total = hdr[2 * group + 1];
    constexpr bool XCD_RUNS = OPS == kBtFirstOps;
    const int step = (int)gridDim.x;
    int u = (int)blockIdx.x;
    if (u >= total)
        return;
    BTileUnit cur = units[first + (XCD_RUNS ? xcd_run_tile(u, total) : u)];
    for (;;) {
        // the next tile's record is requested before this tile's rows, so it
        // is at hand when the tile ends; the instance record it points to is
        // mostly the same as this one (a large instance has many tiles, dealt
        // out in order) and then comes from the scalar cache
        const bool more = u + step < total;
        BTileUnit nxt = cur;
        if (more)
            nxt = units[first + (XCD_RUNS ? xcd_run_tile(u + step, total) : u + step)];
        bt_tile<KV, D, WC, WR, OPS>(entries[cur.entry], cur, lds);
        if (!more)
            break;
        // the column sums of this tile leave LDS before the next tile's
        // waves write theirs
        if constexpr (COLSUM && WR > 1)
            lds_barrier();
        u += step;
        cur = nxt;
    }
}

__global__ __launch_bounds__(256) void k_bt_finish(const FinishJob *__restrict__ jobs,
                                                   const BFinishUnit *__restrict__ units,
                                                   const int *__restrict__ hdr, int group)
{
    __shared__ double lds[4][64];
    const int first = hdr[2 * group], total = hdr[2 * group + 1];
    for (int u = (int)blockIdx.x; u < total; u += (int)gridDim.x) {
        const BFinishUnit fu = units[first + u];
        FinishJob j = jobs[fu.job];
        j.P = as_global(j.P);
        j.add = as_global(j.add);
        j.out = as_global(j.out);
        finish_block(j, fu.block, lds);
        // wave 0 has read every wave's sum before the next block's are written
        lds_barrier();
    }
}

const char *const kGroupNames[BG_COUNT] = {"bt_first", "bt_finish1", "bt_row_narrow",
                                            "bt_row_wide", "bt_finish_w"};

template <int S, int OPS>
void launch_shape_ops(const BTileEntry *entries, const BTileUnit *units, const int *hdr,
                      int group, int grid, hipStream_t st)
{
    constexpr BtShapeDef d = kBtShapes[S];
    launch(kGroupNames[group], k_bt<d.kv, d.d, d.wc, d.wr, OPS>, dim3((unsigned)grid),
           dim3(kWave * d.wc * d.wr), st, entries, units, hdr, group);
}

template <int S>
void launch_shape(int ops, const BTileEntry *entries, const BTileUnit *units, const int *hdr,
                  int group, int grid, hipStream_t st)
{
    switch (ops) {
    case kBtFirstOps: launch_shape_ops<S, kBtFirstOps>(entries, units, hdr, group, grid, st); break;
    case kRowOps: launch_shape_ops<S, kRowOps>(entries, units, hdr, group, grid, st); break;
    default: break;
    }
}

}  // namespace

bool btile_shape_ok(int shape, int ops, int rb)
{
    if (shape < 0 || shape >= kBtShapeCount)
        return false;
    if (ops != kBtFirstOps && ops != kRowOps)
        return false;
    const BtShapeDef &d = kBtShapes[shape];
    if (rb < d.wr || rb % d.wr != 0 || rb > 4096)
        return false;
    // row-dot results are gathered one row per lane (BiCGK's tiles run in
    // the first launch)
    if ((ops == kBtFirstOps || (ops & OP_ROWDOT)) && rb / d.wr > kWave)
        return false;
    return true;
}

int64_t btile_cols(int shape) { return (int64_t)kBtShapes[shape].wc * 128 * kBtShapes[shape].kv; }
int64_t btile_wave_cols(int shape) { return (int64_t)128 * kBtShapes[shape].kv; }
int btile_threads(int shape) { return kWave * kBtShapes[shape].wc * kBtShapes[shape].wr; }

void btile_shape_info(int shape, int out[4])
{
    const BtShapeDef &d = kBtShapes[shape];
    out[0] = d.kv;
    out[1] = d.d;
    out[2] = d.wc;
    out[3] = d.wr;
}

void launch_btile(int shape, int ops, const BTileEntry *entries, const BTileUnit *units,
                  const int *hdr, int group, int grid, hipStream_t st)
{
    if (grid <= 0)
        return;
    switch (shape) {
    case 0: launch_shape<0>(ops, entries, units, hdr, group, grid, st); break;
    case 1: launch_shape<1>(ops, entries, units, hdr, group, grid, st); break;
    case 2: launch_shape<2>(ops, entries, units, hdr, group, grid, st); break;
    case 3: launch_shape<3>(ops, entries, units, hdr, group, grid, st); break;
    case 4: launch_shape<4>(ops, entries, units, hdr, group, grid, st); break;
    case 5: launch_shape<5>(ops, entries, units, hdr, group, grid, st); break;
    case 6: launch_shape<6>(ops, entries, units, hdr, group, grid, st); break;
    case 7: launch_shape<7>(ops, entries, units, hdr, group, grid, st); break;
    case 8: launch_shape<8>(ops, entries, units, hdr, group, grid, st); break;
    case 9: launch_shape<9>(ops, entries, units, hdr, group, grid, st); break;
    case 10: launch_shape<10>(ops, entries, units, hdr, group, grid, st); break;
    case 11: launch_shape<11>(ops, entries, units, hdr, group, grid, st); break;
    default: break;
    }
}

void launch_btile_finish(const FinishJob *jobs, const BFinishUnit *units, const int *hdr,
                         int group, int grid, hipStream_t st)
{
    if (grid > 0)
        launch(kGroupNames[group], k_bt_finish, dim3((unsigned)grid), dim3(256), st, jobs, units,
               hdr, group);
}

}  // namespace bto
