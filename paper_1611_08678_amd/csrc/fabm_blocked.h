// fabm_blocked.h -- argument blocks and host schedules of the BLOCKED path
// (shared by the kernels and the host dispatcher; internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "fabm_device.h"

namespace fabm {

// ---------------------------------------------------------------------------
// Step pipeline (dispatched). Rows are cut into blocks of 256 and, inside a
// block, into 16 columns of 16 rows (polyphase split of the Toeplitz sums:
// row 16 kappa + tau lies in column kappa). For a target in column c of block
// J the history splits by column lag q = c - kappa:
//   band : sources in blocks J-1 and J, added one row at a time while those
//          blocks are walked (q <= 16 + rho for rho = c - 16 J);
//   near : q in [rho + 17, 47], i.e. the rest of block J-2 and the part of
//          block J-3 in columns above 16 (J-3) + rho;
//   far  : q >= 48, cut into windows q in [16 m, 16 m + 16), m = 3 .. J.
// Window m of target J reads source columns 16 (J - m) + rho - u (u < 16),
// which all lie in blocks J-m-1 and J-m, so it can be added as soon as block
// J - m is final, and every target J reads the same columns in that step.
// Launch s of the pipeline (s = -1 .. NB-2) is one kernel:
//   workgroup 0   : band of block s + 1;
//   workgroup 1   : near part of target s + 2 (sources up to block s);
//   workgroups 2..: far window m = J - s of every target J >= s + 3.
// Every launch depends on the previous one only, through ordinary stream
// order: no events, flags or waits.
// ---------------------------------------------------------------------------
constexpr int kStepThreads = 1024;  // 16 wavefronts, four per SIMD
constexpr int kNearWaves = 8;       // wavefronts sharing the near part
constexpr int kMaxFarWg = 254;      // far workgroups per launch (+ band + near <= 256 CUs)

struct StepArgs {
    const InstMeta *meta;
    const double *params;
    const double *y0;
    double *Y;          // caller rows [N+1][D]
    const double *W;    // b, a, c tables of length meta->wlen each
    double *Fc;         // component-major history [D][NB*256]
    double *carry;      // [2][2D][256] band sums handed to the next block
    double *acc;        // [NB][2D][4][64] near + far sums of each target block,
                        //   in the register order of the 16x16 MFMA result
    uint32_t *dead;     // [0]: first non-finite step (0 while finite), or kDeadWatchdog
    int64_t *status;
    int NB;
};

// Value of StepArgs::dead when a bounded wait inside the band gave up
// (reported as status -1).
constexpr uint32_t kDeadWatchdog = 0xFFFFFFFFu;

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
