// fabm_wide.h -- the shared-grid batch path (internal).
//
// When every instance of a batch has the same alpha, h and N, the weights of
// Section 2 are one table for all of them and the history sums of all
// instances are one product: with the states of every instance side by side
// as columns (column = instance * d + component), the sums of target rows
// [t0, t0 + 64) are
//     P[r][col] = sum_{k < t0} b[t0 + r - 1 - k] F[k][col]   (and C with a),
// a Toeplitz matrix (64 x t0) times the history (t0 x columns). Each block of
// 64 rows is formed in two launches on one stream:
//   far  : the product above for block s from all earlier blocks, on the
//          matrix cores, split over source-block ranges when the columns alone
//          give too few workgroups (partials summed in a fixed order);
//   band : one wavefront per instance walks the 64 rows of block s: the sums
//          over earlier rows of the same block, the c - a correction of source
//          row 0, predictor, corrector and the two evaluations of f (a d x d
//          matrix-vector product for the linear system).
// The far product reads the history in the precision of the plan: binary64,
// binary32, or two binary16 parts per value scaled by powers of two.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fabm {

struct InstMeta;
struct KernelTimer;

constexpr int kWideBlk = 64;       // rows per block
constexpr int kWideColAlign = 128; // column padding of the history copies
constexpr int kWideMaxSplits = 64; // source-range splits of one far launch
constexpr int kWideSplitTarget = 1024;     // default far workgroups per launch
constexpr int kWideMaxSplitTarget = 4096;  // largest target the tuner tries

enum : int { WIDE_F64 = 0, WIDE_F32 = 1, WIDE_F16X2 = 2 };

struct WideArgs {
    const InstMeta *meta;   // [batch]; alpha, h, N and the scalars are shared
    const double *params;   // [batch][d*d + 2d]
    const double *y0;       // [batch][d]
    const double *y1;       // [batch][d] y'(0) (orders above one), or null
    double *Y;              // caller rows
    const double *W;        // b, a, c tables of length wlen (shared)
    const float *W32;       // binary32 b, a (FP32 far)
    double *F;              // FP64 history [NB*64][cp]
    float *F32;             // FP32 history [NB*64][cp]
    _Float16 *Fhi, *Flo;    // FP16X2 history [NB*64/8][cp][8], scaled per block and column
    int32_t *Fexp;          // [NB][cp] power-of-two scale of each block and column
    const _Float16 *T16;    // FP16X2 Toeplitz operands, [NB][2 tables][2 parts][8][128]
    const int32_t *T16exp;  // [NB][2] scale of each lag window
    double *part;           // [splits][2][64][cp] far sums (split 0 holds the total)
    uint32_t *dead;         // [batch] first non-finite row, 0 while finite
    int64_t *status;        // [batch]
    int64_t batch;
    int64_t wlen;
    int d, cp, NB, prec;
    int split_target;       // far workgroups a launch aims for (source-range splits)
};

// Enqueue the whole shared-grid solve after the weights exist.
hipError_t enqueue_wide(const WideArgs &A, hipStream_t s, KernelTimer *T, const char **where);
// Bytes of the FP16X2 Toeplitz operand table for NB blocks.
size_t wide_t16_bytes(int NB);
// Far-launch splits for a given column count (upper bound over all blocks and
// split targets up to kWideMaxSplitTarget).
int wide_max_splits(int cp, int NB);

}  // namespace fabm
