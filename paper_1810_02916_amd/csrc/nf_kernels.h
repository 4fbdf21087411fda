// nf_kernels.h -- host-side launch interfaces between the translation units
// of libnf.so (not part of the public ABI).
#pragma once

#include <algorithm>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nf_internal.h"

namespace nf {

// Sizes and scratch pointers of one binning call (all boxes together).
struct BinPlan {
    int64_t N = 0;          // sum of n_b
    int64_t C = 0;          // sum of K_b^3
    int64_t max_n = 0;      // largest n_b
    int64_t max_ncell = 0;  // largest K_b^3
    int64_t nblk = 0;       // radix tiles: ceil(N / kSortTile)
    int passes = 0;         // radix passes covering keys 0..C-1 (at least 1)
    int radix_bits = 8;     // digit width: 8, or 9 when that saves a pass
    BinScratch sc{};
    uint32_t *scan_scratch = nullptr;
};

int64_t scan_scratch_words(int64_t M);
// In-place exclusive scan of M uint32 values; scratch holds scan_scratch_words(M).
hipError_t scan_exclusive(uint32_t *data, int64_t M, uint32_t *scratch, hipStream_t s);
// Fill count uint32 values (a kernel, so it can sit inside a captured graph).
hipError_t fill_u32(uint32_t *p, int64_t count, uint32_t value, hipStream_t s);
hipError_t bin_launch(const DevBox *d_boxes, int nbox, const BinPlan &p, hipStream_t s);

// Pair symmetry (nf_pair.hip).
struct F4Plan {
    int64_t C = 0, max_cells = 0;
    int32_t *P = nullptr, *nfwd = nullptr;   // [C]
    uint32_t *slotoff = nullptr;              // [C + 1] counts, then first slots
    uint32_t *itemoff = nullptr;              // [C + 1] counts, then first items
    uint32_t *scan = nullptr;                 // scan scratch
    uint32_t *tot = nullptr;                  // [4] on, items, slots
    uint64_t *blk = nullptr;                  // [2 x blocks of the count kernel] totals
    PairItem *items = nullptr;                // [cap_items]
    float4 *part = nullptr;                   // [cap_slots] (x2 compensated)
    uint32_t *counter = nullptr;              // item queue
    uint32_t cap_slots = 0, cap_items = 0;
};
int f4_queue_words();
hipError_t f4_plan_launch(const DevBox *d_boxes, int nbox, const F4Plan &fp, hipStream_t s);
hipError_t f4_ring_launch(const DevBox *d_boxes, const F4Plan &fp, bool compensated,
                          hipStream_t s);
hipError_t f4_combine_launch(const DevBox *d_boxes, int nbox, const F4Plan &fp, bool compensated,
                             hipStream_t s);

// Planner + tile kernels (nf_tile.hip).
struct TilePlan {
    int64_t TG = 0;              // cells over all boxes (planning is per cell)
    int64_t max_cells = 0;       // largest per-box cell count
    uint32_t *cellinfo = nullptr;     // [TG] item kind and cost bucket per cell
    uint32_t *bucket_cnt = nullptr;   // [plan_buckets()] items per (kind, cost bucket)
    uint32_t *bucket_off = nullptr;   // [plan_buckets()] first item of each bucket
    uint32_t *totals = nullptr;  // [3] dense, light and narrow item counts
    Item *dense = nullptr;       // dense items, heaviest first
    Item *light = nullptr;       // light items, then narrow items, each in spatial slabs
    uint32_t *counter = nullptr; // [queue_words()] queue counters
    int light_window = 1024;     // staged sources per round: 512 / 1024 / 2048 (accel numbers)
    int narrow_window = 256;     // 128 / 256 / 512
};
int plan_buckets();
int queue_words();
hipError_t plan_launch(const DevBox *d_boxes, int nbox, const TilePlan &tp, hipStream_t s);
// The planned items as (box, cell, chunk, class) int32 quadruples, dense,
// light then narrow, at most max_items of them, and the three class counts.
hipError_t plan_export_launch(const TilePlan &tp, int32_t *items, int64_t max_items,
                              int64_t *counts, hipStream_t s);
// mode 0: accelerations, 1: VJP (cot = cotangents in sorted order).
// concurrent: the light and narrow kernels run on the library's side streams
// alongside the dense kernel; otherwise all three run in turn on s.
hipError_t tile_launch(const DevBox *d_boxes, int mode, bool compensated, const TilePlan &tp,
                       const float4 *cot, bool concurrent, hipStream_t s,
                       const F4Plan *f4 = nullptr);

// Per-cell multipole moments (nf_multipole.hip).
int multipole_max_order();
int multipole_terms(int p);
// Workgroup ranges of one box (n particles, ncell cells).
int64_t multipole_ranges(int64_t n, int64_t ncell);
// Cells of more than multipole_big() particles are summed in pieces of at
// most that many particles; a box of n particles has at most
// multipole_max_pieces(n) pieces.
int multipole_big();
int64_t multipole_max_pieces(int64_t n);
struct MpPiece {
    int32_t box, cell, q0, q1, k, np;   // sorted slots [q0, q1); piece k of np
};
struct MpPlan {
    int64_t C = 0;                  // cells over all boxes
    int64_t max_ncell = 0;          // largest per-box cell count
    int64_t max_ranges = 0;         // largest per-box range count
    int64_t max_pieces = 0;         // bound on the pieces over all boxes
    const int64_t *range_base = nullptr;   // [nbox + 1] prefix of the range counts
    int32_t *first = nullptr;       // sum over boxes of (ranges + 1)
    uint32_t *npieces = nullptr;    // [C + 1] pieces per cell, then their offsets
    uint32_t *scan = nullptr;       // scan_scratch_words(C + 1)
    MpPiece *pieces = nullptr;      // [max_pieces]
    double *partial = nullptr;      // [max_pieces][terms] piece moments
};
hipError_t multipole_launch(const DevBox *d_boxes, int nbox, const MpPlan &mp, int p,
                            hipStream_t s);

// Time-step inputs and kick/drift (nf_step.hip).
struct StepIO {                 // per box, caller order
    const float *acc;           // [n][3]
    const float *vel;           // [n][3] (step statistics)
    float *vel_rw;              // [n][3] (kick)
    double *pos_rw;             // [n][3] (drift)
    float *amax, *vrms;         // [K^3] per-cell outputs
    const float *amax_in, *vrms_in;   // [K^3] per-cell inputs of the step choice
};
struct StepChoice {             // the caller's constants of the step choice
    double dlna_max, hubble, eta;
};
struct CellStat {               // per cell: max |a|, sum |v|^2, max |v|^2
    double amax, v2sum, vmax2;
};
struct PartStat {               // per particle, caller order: |a| and |v|^2
    double a, v2;
};
constexpr int kStepBlocks = 256;   // partial reductions per box (power of two)
hipError_t step_stats_launch(const DevBox *d_boxes, const StepIO *d_io, int nbox,
                             int64_t max_n, int64_t max_ncell, PartStat *part,
                             CellStat *scratch, CellStat *partial, double *glob, hipStream_t s);
hipError_t step_choose_launch(const DevBox *d_boxes, const StepIO *d_io, int nbox,
                              double *partial, const double *glob, const StepChoice &ch,
                              double *bounds, hipStream_t s);
hipError_t kick_drift_launch(const DevBox *d_boxes, const StepIO *d_io, int nbox, int64_t max_n,
                             double kick, double drift, hipStream_t s);

// Force launches.  `items` and `nitems` describe the work list built on the
// host side of the call (see nf_accel.hip).
struct ForcePlan {
    int64_t max_n = 0;
    bool compensated = false;
    bool simple = false;
    float4 *cot_sorted = nullptr;   // vjp only: [2N] source records (offset, cotangent), sorted
    int64_t N = 0;
};

hipError_t accel_launch(const DevBox *d_boxes, int nbox, const ForcePlan &p, hipStream_t s);
hipError_t vjp_launch(const DevBox *d_boxes, int nbox, const ForcePlan &p, hipStream_t s);
hipError_t gather_cot_launch(const DevBox *d_boxes, int nbox, const ForcePlan &p, hipStream_t s);

}  // namespace nf
