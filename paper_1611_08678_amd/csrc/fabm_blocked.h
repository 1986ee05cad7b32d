// fabm_blocked.h -- argument blocks and host schedules of the BLOCKED path
// (shared by the kernels and the host dispatcher; internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "fabm_device.h"

namespace fabm {

// ---------------------------------------------------------------------------
// Event-ordered pipeline (dispatched). Rows are cut into blocks of 256.
// For a target in block J:
//   band  : sources in blocks J-1 and J, added one row at a time by the band
//           kernel of block J-1 / J (scatter after each row is formed);
//   near  : sources in block J-2, one 256x256 MFMA tile computed by the band
//           kernel of block J before its first step;
//   far   : sources in blocks [0, J-2), cut going back from J-2 into chunks of
//           2, 4, 8, ... blocks ("tasks"); a task becomes computable when the
//           band kernel of its last source block has finished ("far step" of
//           that block). Tasks longer than kItemBlocks are split into items
//           whose partials are added in order within the same far step.
// Band kernels run on the caller's stream; far steps on a second stream; the
// far step of block I waits for band block I, and band block J waits for the
// far step of block J-3, which finalises the far sum of J (all its tasks, in
// source order). Nothing waits inside a kernel.
// ---------------------------------------------------------------------------
constexpr int kItemBlocks = 16;

struct PipeArgs {
    const InstMeta *meta;
    const double *params;
    const double *y0;
    double *Y;            // caller rows [N+1][D]
    const double *W;      // b, a, c tables of length meta->wlen each
    double *Fc;           // component-major history [D][NB*256]
    double *carry;        // [2][2D][256] band accumulators handed to the next block
    double *far;          // [NB][2D][256] finalised far sums
    double *task_slot;    // [n_slots][2D][256] partial of each far task
    double *scratch;      // [max_scratch][2D][256] item partials of one far step
    const int4 *items;    // {J, I0, I1, dest}: dest >= 0 task slot, else scratch -dest-1
    const int4 *reds;     // {slot, scratch_first, n_items, 0}: multi-item task sums
    const int *tt_off;    // [NB+1] tasks of each target (CSR over tt_slot)
    const int *tt_slot;   // task slots in source order
    uint32_t *dead;       // [0]: first non-finite step (0 while finite)
    int64_t *status;
    int NB;
};

struct PipeSchedule {
    int NB = 0;
    std::vector<int4> items;         // grouped by far step
    std::vector<int> step_item_off;  // [NB+1]
    std::vector<int4> reds;          // grouped by far step
    std::vector<int> step_red_off;   // [NB+1]
    std::vector<int> tt_off;         // [NB+1]
    std::vector<int> tt_slot;
    int n_slots = 0;
    int max_scratch = 0;
};
void pipe_schedule(int NB, PipeSchedule &s);

// ---------------------------------------------------------------------------
// Single-launch persistent variant (not dispatched; see blocked_persistent.hip).
// ---------------------------------------------------------------------------
struct BlockedArgs {
    const InstMeta *meta;
    const double *params;
    const double *y0;
    double *Y;          // caller rows [N+1][D]
    int64_t *status;
    const double *W;    // b, a, c tables of length meta->wlen each
    double *Fc;         // component-major history [D][NB*L]
    double *part;       // [n_tasks][2D][L] per-task partial sums
    double *far;        // [NB][2D][L] far sums of each target block
    const int4 *tasks;  // {J, I0, I1, 0}, grouped by J in source order
    const int *queue;   // task ids in processing order
    const int *task_off;// [NB + 1]
    uint32_t *sync;     // [0] blocks complete, [1] queue head, [2] dead step, [3] abort
    uint32_t *done;     // [NB] finished tasks per target block
    uint32_t *ready;    // [NB] far sums published
    int NB;
    int n_tasks;
    uint64_t timeout_ticks;  // bound of every wait, in wall-clock ticks
};
int blocked_count_tasks(int NB);
void blocked_schedule(int NB, int4 *tasks, int *queue, int *task_off);

}  // namespace fabm
