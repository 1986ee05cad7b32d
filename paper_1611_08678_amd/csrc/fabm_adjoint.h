// fabm_adjoint.h -- argument block of the reverse (adjoint) pipeline
// (internal; kernels in adjoint.hip, layout in capi.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fabm_blocked.h"
#include "fabm_device.h"

namespace fabm {

// Placement per instance i: forward rows Y, YP at meta[i].f_off (packed),
// dL/dy rows G at meta[i].row_off (the caller's), reversed sources UV at
// 2 inst[i].fc_off, sums acc at inst[i].acc_off / 2, block partials at
// inst[i].acc_off / (2 D 256) * (n_params + 2 D).
struct AdjArgs {
    const InstMeta *meta;   // [batch]
    const InstMeta *cmeta;  // non-commensurate orders: [batch][D] (scalars, table offsets), or null
    const BlkInst *inst;    // [batch] (same as the forward batch)
    const int *order;       // instances by block count, descending
    const double *params;   // [batch][n_params]
    const double *y0;       // [batch][D]
    const double *Y, *YP;   // recomputed forward rows
    const double *G;        // caller's dL/dy rows
    const double *W;        // weight tables (b, a, c)
    double *UV;             // reversed sources [2D][NB*256] per instance
    double *carry;          // [batch][2][D][256]
    double *acc;            // [NB][D][4][64] per instance
    double *part;           // [NB][n_params + 2D] per instance: theta, y(0), y'(0)
    double *fbar0;          // [batch][D]
    const uint32_t *dead;   // forward non-finite flags [batch]
    double *gy0;            // [batch][D], or [batch][2][D] with `slope`
    int slope;              // initial values include y'(0): gradients [batch][2][D]
    double *gparams;        // [batch][n_params] (at meta[i].p_off)
    int64_t batch;
    // block checkpoints: Y and YP are rings of R = G + 1 forward blocks per
    // instance ([batch][R][256][D]) re-formed before each group of G reverse
    // launches; 0 when Y and YP hold every row
    int ring;
};

struct KernelTimer;
struct RecompArgs;
// With `fwd` and `rec` (block checkpoints), the forward blocks each group of
// reverse launches reads are re-formed first (A.ring = rec->G + 1).
hipError_t enqueue_adjoint(int sys, int d, const AdjArgs &A, const BatchSchedule &S,
                           const int *far_off, hipStream_t s, KernelTimer *T, const char **where,
                           const BatchArgs *fwd = nullptr, const RecompArgs *rec = nullptr);
size_t adj_smem_bytes(int d, bool pc = false);

// Rows 0..N_i of every instance from src (placed by src_meta[i].f_off) to dst
// (placed by dst_meta[i].row_off), d doubles per row.
hipError_t launch_copy_rows(const InstMeta *src_meta, const InstMeta *dst_meta, int64_t batch,
                            int64_t max_rows, int d, const double *src, double *dst,
                            hipStream_t s);

}  // namespace fabm
