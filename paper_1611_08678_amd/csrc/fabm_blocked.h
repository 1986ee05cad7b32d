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

// One trajectory as seen by the step kernels' device code.
struct InstView {
    const InstMeta *meta;
    const InstMeta *cmeta;  // non-commensurate orders: [D] entries of this instance, or null
    const double *params;
    const double *y0;
    const double *y1;   // y'(0) [D] (orders above one), or null
    double *Y;          // rows [N+1][D]
    double *YP;         // predictor rows [N+1][D] (row 0 = y0), or null
    const double *W;    // b, a, c tables of length meta->wlen each
    const float *W32;   // b, a in binary32 (FP32 far windows only)
    double *Fc;         // [D][NB*256]
    double *carry;      // [2][2D][256]
    double *acc;        // [NB][2D][4][64]
    uint32_t *dead;
    int NB;
    int64_t yrow0 = 0;  // row of the trajectory stored at Y[0] (recompute rings)
    int recompute = 0;  // band only re-forms rows: history and carry not written
};

struct StepArgs {
    const InstMeta *meta;
    InstMeta m0;        // meta[0] by value (the band reads it without a memory round trip)
    const InstMeta *cmeta;  // non-commensurate orders: [D] per-component entries, or null
    const double *params;
    const double *y0;
    const double *y1;   // y'(0) [D] (orders above one), or null
    double *Y;          // caller rows [N+1][D]
    double *YP;         // predictor rows [N+1][D] (teacher-forced sums only), or null
    const double *W;    // b, a, c tables of length meta->wlen each
    const float *W32;   // b, a in binary32 (FP32 far windows only)
    double *Fc;         // component-major history [D][NB*256]
    double *carry;      // [2][2D][256] band sums handed to the next block
    double *acc;        // [NB][2D][4][64] near + far sums of each target block,
                        //   in the register order of the 16x16 MFMA result
    uint32_t *dead;     // [0]: first non-finite step (0 while finite), or kDeadWatchdog
    int64_t *status;
    int NB;
    int far_cap;        // far workgroups per launch (host side: launch shape only)
    // sub-quadratic far history (fft_far.hip; host side): squares of level
    // >= fft_level by FFT convolution, 0 = every far window on the matrix cores
    int fft_level;
    int64_t wlen;       // length of each weight table
    double2 *fft_tw;    // twiddles exp(-2 pi i j / M) of the longest transform M
    double2 *fft_buf;   // [D][M] transform of the current square
    double2 *fft_spec;  // weight spectra of levels fft_level.., concatenated
};

// Value of StepArgs::dead when a bounded wait inside the band gave up
// (reported as status -1).
constexpr uint32_t kDeadWatchdog = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Batched step pipeline (dispatched for batch > 1): the same decomposition for
// every instance, all instances advancing one block per launch. Instances are
// sorted by block count, descending, so at launch s the instances with a band
// block s+1, a near target s+2 or far targets are prefixes of that order.
// Launch s has, in this order, one band workgroup per instance with a block
// s+1, one near workgroup per instance with a target s+2, and for every
// instance with targets >= s+3 one far workgroup per four targets (one target
// per wavefront); `far_off` (per launch, host-built) holds the prefix sums of
// far workgroups per instance in the same order.
// ---------------------------------------------------------------------------
constexpr int kBatchThreads = 256;  // four wavefronts per workgroup

// Per-instance placement in the BLOCKED workspace.
struct BlkInst {
    int64_t fc_off;   // doubles: history [D][NB*256]
    int64_t acc_off;  // doubles: near + far sums [NB][2D][4][64]
    int32_t NB;       // blocks of 256 rows
    int32_t pad;
};

struct BatchArgs {
    const InstMeta *meta;  // [batch]
    const InstMeta *cmeta; // non-commensurate orders: [batch][D], or null
    const BlkInst *inst;   // [batch]
    const int *order;      // instances by block count, descending
    const double *params;  // [batch][n_params]
    const double *y0;      // [batch][D]
    const double *y1;      // [batch][D] y'(0) (orders above one), or null
    double *Y;             // caller rows; instance i at meta[i].row_off
    double *YP;            // predictor rows placed like Y, or null
    const double *W;       // weight tables, instance i at meta[i].w_off
    const float *W32;      // binary32 b, a of instance i at 2 meta[i].w_off / 3
    double *Fc;
    double *carry;         // [batch][2][2D][256]
    double *acc;
    uint32_t *dead;        // [batch]
    int64_t *status;       // [batch]
    int64_t batch;
};

// Recomputation of forward blocks for the reverse pass of an adjoint with
// block checkpoints: the forward keeps only the history and the near + far
// sums of every block; before the reverse pass reaches the rows of forward
// block K, the band of block K is walked again (its incoming band sums
// re-formed from block K - 1's history in the forward's order, so the rows
// are bitwise the forward's) into a ring of R = G + 1 blocks per instance,
// G forward blocks per group of G reverse launches.
struct RecompArgs {
    double *ringY;   // [batch][R][256][D] trajectory rows
    double *ringYP;  // [batch][R][256][D] predictor rows
    double *rcarry;  // [batch][R][2][2D][256] band sums entering the block
    int G;           // reverse launches per group
};
constexpr int kCkptGroup = 4;

// Host schedule of one batched call. Far windows go in groups of P source
// blocks (P = 1, 2 or 4; k_step_batch): launches with (s + 1) % P == 0 take
// sources s - P + 1 .. s for every later target, the others take source s for
// the targets whose band runs before the next such launch.
struct BatchSchedule {
    std::vector<int> order;
    std::vector<int> nband, nnear, nfar, far_base;  // per launch s + 1 (s = -1 .. S-2)
    std::vector<int> far_off;         // concatenated prefix sums (groups of P source blocks)
    std::vector<int> far_off_single;  // the same with one source block per launch (reverse pass)
    int max_NB = 0;
    int P = 2;
};
constexpr int kDefaultBatchGroup = 2;
void batch_schedule(int64_t batch, const int32_t *NB, BatchSchedule &S,
                    int P = kDefaultBatchGroup);

}  // namespace fabm
