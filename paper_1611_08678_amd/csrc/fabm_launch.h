// fabm_launch.h -- host-side launchers of the library's kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

namespace fabm {

struct InstMeta;

// Raise a kernel's dynamic LDS limit to `bytes` on the current device, once
// per device: `done` is the kernel's own set of devices already configured
// (the attribute is per device, so a process driving several GPUs sets it on
// each).
inline hipError_t ensure_lds_attr(const void *fn, size_t bytes, std::atomic<uint64_t> &done)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = dev < 64 ? (uint64_t)1 << dev : 0;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_release);
    return e;
}

// Weight tables for every instance of a call (one table per instance).
// With W32, b and a are also written in binary32 (far windows in FP32).
hipError_t launch_weights(const InstMeta *meta, int64_t batch, int64_t maxN, double *W,
                          hipStream_t s, float *W32 = nullptr);
hipError_t launch_weights_one(double al, double ig1, double ig2, int64_t n, double *b, double *a,
                              double *c, hipStream_t s);

// Zero-fill of 32-bit words (a kernel, so it is safe inside captured graphs).
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);

// One instance entry written by a kernel from its argument (no staging copy).
hipError_t launch_put_meta(const InstMeta &m, InstMeta *dst, hipStream_t s);

// dst[e] = src[e] for e < n_src, 0 for n_src <= e < n_dst (a kernel).
hipError_t launch_copy_pad(const double *src, int64_t n_src, double *dst, int64_t n_dst,
                           hipStream_t s);

// Split of the initial values [batch][2][d] (y(0), then y'(0)) into y0 and
// y1, each [batch][d] (a kernel, so it is safe inside captured graphs).
hipError_t launch_split_init(const double *init, int64_t batch, int d, double *y0, double *y1,
                             hipStream_t s);

// DIRECT path, one workgroup per instance. y1 (y'(0) per instance, used for
// orders above one) may be null. cmeta, when given, holds [batch][d] entries
// with each component's own order (weights at its w_off, its step scalars).
hipError_t launch_direct_wg(int sys, int d, const InstMeta *meta, const InstMeta *cmeta,
                            int64_t batch, const double *params, const double *y0,
                            const double *y1, double *F, const double *W, double *Y,
                            int64_t *status, hipStream_t s);

// DIRECT path, one trajectory spread over the whole GPU (persistent,
// cooperative launch); `part` holds direct_grid_part_doubles(G) doubles (a
// partial slot per workgroup in each of three step buffers), every 32-bit
// word set to direct_grid_empty_word() before the launch; `sync`
// direct_grid_sync_words(G) zeroed words (the abort word). Every
// inter-workgroup wait gives up after `timeout_ticks` of the device's
// constant-rate wall clock (status -1).
size_t direct_grid_part_doubles(int G);
size_t direct_grid_sync_words(int G);
uint32_t direct_grid_empty_word();
hipError_t launch_direct_grid(int sys, int d, int G, const InstMeta *meta, const InstMeta *cmeta,
                              const double *params, const double *y0, const double *y1,
                              double *F, const double *W, double *Y, int64_t *status,
                              double *part, uint32_t *sync, uint64_t timeout_ticks,
                              hipStream_t s);

// BLOCKED path, one trajectory, as a sequence of step kernels on stream `s`
// (decomposition in fabm_blocked.h). On failure *where names the call.
struct StepArgs;
struct KernelTimer;
hipError_t enqueue_steps(int sys, int d, bool f32, const StepArgs &A, hipStream_t s,
                         KernelTimer *T, const char **where);
int step_block_len();
size_t step_smem_bytes(int d, bool pc = false);
void step_grid(int NB, int jend, int s, int *grid, int *wpw, int far_cap, int *halves);

// Sub-quadratic far history of the step pipeline (fft_far.hip). Level l of
// the dyadic squares covers 2^l source blocks; the host enqueues at most one
// square after each step launch.
int fft_far_top_level(int NB, int level);         // highest level with a square, or -1
int64_t fft_far_max_len(int NB, int level);       // longest transform (complex elements)
int64_t fft_far_spectra_len(int NB, int level);   // complex elements of one table set's spectra
int fft_far_target_end(int NB, int level, int s); // end of launch s's window targets
bool fft_far_mask_prev(int level, int s);         // launch s's windows skip block s - 1
hipError_t fft_far_prepare(int d, const StepArgs &A, hipStream_t st);  // twiddles, spectra
int fft_far_square_at(int NB, int level, int s);  // level of the square after launch s, or -1
hipError_t fft_far_square(int d, const StepArgs &A, int s, hipStream_t st);

// BLOCKED path for a batch (> 1) of trajectories: one launch per block step
// for all instances. `far_off` is S.far_off in device memory.
struct BatchArgs;
struct BatchSchedule;
hipError_t enqueue_batch(int sys, int d, bool f32, const BatchArgs &A, const BatchSchedule &S,
                         const int *far_off, hipStream_t s, KernelTimer *T, const char **where);
size_t batch_smem_bytes(int d, bool pc = false, int P = 2);

// Block checkpoints of the adjoint: re-form the forward rows of the group of
// reverse launches starting at reversed block J (one workgroup per instance
// and ring slot; `ninst` instances of the order have a reversed block J).
struct RecompArgs;
hipError_t launch_recompute(int sys, int d, const BatchArgs &A, const RecompArgs &R, int J,
                            int ninst, hipStream_t s);

// Teacher-forced history sums, direct contraction (one thread per target row
// and component group).
hipError_t launch_history_direct(const double *W, int64_t N, int d, const double *f, double *P,
                                 double *C, hipStream_t s);

}  // namespace fabm
