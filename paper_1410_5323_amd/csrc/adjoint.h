// adjoint.h -- arguments and workspace of the adjoint kernels (adjoint_fp64.hip).
#pragma once

#include "crp_internal.h"

namespace crp {

// Adjoint replay record: doubles per accepted step (pre-step state 6, step 1,
// stage states 30, stage fields 18, output direction 3, mirrored axes 1), and
// the crossing-derivative scratch per lane.
constexpr int ADJ_RECORD_DOUBLES = 59;
constexpr int ADJ_SCRATCH_DOUBLES = 36;

// Records are laid out for 64-lane wavefronts: a block of records holds one
// record per lane of a group of 64 (fields 64 doubles apart, consecutive
// records 59 x 64 apart), so a wavefront's loads and stores of one field are
// one contiguous 512-byte run.
constexpr int ADJ_GROUP = 64;
constexpr int64_t ADJ_BLOCK_DOUBLES = int64_t(ADJ_RECORD_DOUBLES) * ADJ_GROUP;
// Per parallel-replayed step: the six stages' cotangents of the vector grid's
// value (18 doubles), kept for the grid-gradient scatter after the sweep.
constexpr int ADJ_BAR_DOUBLES = 18;
constexpr int64_t ADJ_BAR_BLOCK = int64_t(ADJ_BAR_DOUBLES) * ADJ_GROUP;

// Workspace of crp_propagate_adjoint, byte offsets from the 256-byte aligned
// base.  The first part is always there:
//   [0, 256)   control: queue head (u64 at 0), parallel-replay cut in order
//              positions (i64 at 8) and in groups (i64 at 16)
//   order      int32 [n]            particles, most accepted steps first
//   buckets    8 (NBUCKET + 1)      bucket counts and cursors
//   seg        [lanes / 64][K][59][64]  each wavefront's replay records of one segment
//   scratch    [36][lanes]          crossing-derivative scratch
// The parallel-replay part holds records of the order's first groups of 64
// positions (the particles with the most steps), R records at most, each
// group padded to its most steps (R = 0: absent):
//   grp_rec    int64 [ng + 1]       first record block of group G (exclusive sums of its most steps)
//   grp_row    int64 [ng + 1]       first replay row of group G (exclusive sums of its most segments)
//   pre_ok     int32 [n]            1: the position's records are replayed
//   seg_slot   int64 [64 rows]      checkpoint record of each (row, lane), -1: none
//   prerec     [R / 64][59][64]     the record blocks
//   prebar     [R / 64][18][64]     the stages' grid-value cotangents of each record
// with ng = ceil(n / 64) groups and rows = R / (64 K) + min(ng, R / 64) + 1.
struct AdjWs {
    size_t order, buckets, seg, scratch, grp_rec, grp_row, pre_ok, seg_slot, prerec, prebar, total;
    int64_t R, rows;
};

inline AdjWs adjoint_ws_layout(int64_t n, int32_t K, int64_t lanes, int64_t R) {
    auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t nn = size_t(n > 0 ? n : 0);
    const int64_t ng = (int64_t(nn) + ADJ_GROUP - 1) / ADJ_GROUP;
    AdjWs w{};
    w.R = R >= ADJ_GROUP ? R / ADJ_GROUP * ADJ_GROUP : 0;  // whole blocks
    const int64_t blocks = w.R / ADJ_GROUP;
    w.rows = w.R > 0 ? blocks / K + (ng < blocks ? ng : blocks) + 1 : 0;
    w.order = 256;
    w.buckets = up(w.order + 4 * nn);
    w.seg = up(w.buckets + 8 * size_t(NBUCKET + 1));
    w.scratch = up(w.seg + 8 * ADJ_RECORD_DOUBLES * size_t(K) * size_t(lanes));
    size_t b = up(w.scratch + 8 * ADJ_SCRATCH_DOUBLES * size_t(lanes));
    if (w.R > 0) {
        w.grp_rec = b;
        w.grp_row = up(w.grp_rec + 8 * size_t(ng + 1));
        w.pre_ok = up(w.grp_row + 8 * size_t(ng + 1));
        w.seg_slot = up(w.pre_ok + 4 * nn);
        w.prerec = up(w.seg_slot + 8 * size_t(ADJ_GROUP) * size_t(w.rows));
        w.prebar = up(w.prerec + 8 * ADJ_RECORD_DOUBLES * size_t(w.R));
        b = up(w.prebar + 8 * ADJ_BAR_DOUBLES * size_t(w.R));
    }
    w.total = b;
    return w;
}

// Kernel arguments of the adjoint kernels.
struct AdjArgs {
    FieldDev F;
    ParamsDev P;
    const double *x0, *y0, *z0, *ux0, *uy0, *uz0, *energy;
    const int32_t *charge;
    const double *ckpt;
    const int64_t *link;
    const double *fin;
    double *fin_out;                 // the same finals: flags written back (gradient overflow)
    int64_t cap;
    int32_t K;
    int32_t grad_f32;                // grad_field holds FP32 values (else FP64)
    const double *gbar_dir, *gbar_time, *gbar_energy;
    double *grad_u0, *grad_x0, *grad_energy;
    void *grad_field;
    double *segbuf;                  // [wave][step j][59][64] replay records, then [36][lane] scratch
    int64_t lanes;                   // threads of the sweep launch
    unsigned long long *queue;       // queue head; the parallel-replay cut follows it
    const int32_t *order;            // NULL: index order
    int64_t n;
    // parallel replay (R = 0: none)
    int64_t R, rows;
    int64_t *grp_rec, *grp_row;
    int32_t *pre_ok;
    int64_t *seg_slot;
    double *prerec, *prebar;
};

// Checks done, workspace laid out: order, parallel replay, reverse sweep.
hipError_t launch_adjoint_fp64(const AdjArgs &a, int blocks, hipStream_t s);

}  // namespace crp
