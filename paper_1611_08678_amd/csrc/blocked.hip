// blocked.hip -- the BLOCKED contraction path for one long trajectory as an
// event-ordered pipeline of short kernels (schedule in fabm_blocked.h).
//
// The history sums of Section 2 are Toeplitz in the lag t-1-k. Rows are cut
// into blocks of 256 steps:
//
//  * k_band_block (one workgroup, caller's stream, one launch per block J)
//    walks the 256 steps of block J. Thread i owns the accumulators of target
//    rows JL+i (this block) and (J+1)L+i (next block). Before the first step
//    it adds the far sums of J and one MFMA tile for sources in block J-2.
//    After row t is formed, f_t is broadcast through LDS and every thread adds
//    w[T-1-t] f_t to its targets T > t, so the owner of row t+1 holds complete
//    P and C sums when its turn comes: one barrier per step. The next block's
//    accumulators are handed over in `carry`.
//
//  * k_far_items / k_far_reduce (second stream, one "far step" per source
//    block I, after band block I) evaluate every far task whose last source
//    block is I (polyphase FP64 MFMA tiles, fabm_tiles.h), add multi-item
//    tasks up in order and finalise the far sum of target block I+3 by adding
//    its task partials in source order (deterministic), including the
//    (c - a) f_0 correction of source row 0.
//
// All ordering between the two streams is by HIP events; no kernel waits.
#include "fabm_blocked.h"
#include "fabm_device.h"
#include "fabm_launch.h"
#include "fabm_tiles.h"
#include "fabm_timer.h"

namespace fabm {

template <int SYS, int D>
__global__ __launch_bounds__(kBlk) void k_band_block(PipeArgs A, int J)
{
    extern __shared__ __align__(16) char smem[];
    double *sb = (double *)smem;         // b lags 0..511
    double *sa = sb + 2 * kBlk;          // a lags 0..511
    double *fs = sa + 2 * kBlk;          // [2][D] broadcast slots
    double *red = fs + 2 * D;            // [4][2D][256] near-tile combine
    int64_t *s_dead = (int64_t *)(red + 4 * 2 * D * kBlk);
    const int tid = threadIdx.x;
    const InstMeta m = A.meta[0];
    const int64_t N = m.N;
    const int64_t pitch = (int64_t)A.NB * kBlk;
    const double *wb = A.W, *wa = wb + m.wlen, *wc = wa + m.wlen;
    const double *p = A.params;
    const int64_t t0 = (int64_t)J * kBlk;
    const int64_t tend = t0 + kBlk - 1 < N ? t0 + kBlk - 1 : N;  // last row of this block

    // a non-finite state in an earlier block ends the trajectory
    if (*A.dead != 0u) {
        for (int64_t row = t0 + tid; row <= tend; row += kBlk)
#pragma unroll
            for (int i = 0; i < D; ++i) A.Y[row * D + i] = __builtin_nan("");
        return;
    }
    double y0[D];
#pragma unroll
    for (int i = 0; i < D; ++i) y0[i] = A.y0[i];
    for (int j = tid; j < 2 * kBlk; j += kBlk) {
        sb[j] = wb[j];
        sa[j] = wa[j];
    }
    if (tid == 0) *s_dead = 0;

    double pc[D], cc[D], pn[D], cn[D];
    if (J == 0) {
        if (tid == 0) {
            double f0[D];
            rhs<SYS, D>(0.0, y0, f0, p);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                fs[i] = f0[i];
                A.Fc[i * pitch] = f0[i];
                A.Y[i] = y0[i];
            }
        }
        __syncthreads();
        // source row 0 feeds targets 1 .. 511 with b_{T-1} and c_{T-1}
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double f0 = fs[i];
            pc[i] = tid >= 1 ? wb[tid - 1] * f0 : 0.0;
            cc[i] = tid >= 1 ? wc[tid - 1] * f0 : 0.0;
            pn[i] = wb[kBlk + tid - 1] * f0;
            cn[i] = wc[kBlk + tid - 1] * f0;
        }
    } else {
        const double *cin = A.carry + (int64_t)(J & 1) * 2 * D * kBlk;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            pc[i] = cin[i * kBlk + tid];
            cc[i] = cin[(D + i) * kBlk + tid];
            pn[i] = cn[i] = 0.0;
        }
        if (J >= 2) {
            double sP[D], sC[D];
            toeplitz_block_fp64<D>(wb, wa, A.Fc, pitch, J, J - 2, J - 1, red, sP, sC);
            const int64_t T = t0 + tid;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                pc[i] += sP[i];
                cc[i] += sC[i];
                // source row 0 lies in this tile only for J = 2; it takes c_{T-1}
                if (J == 2) cc[i] = fma(wc[T - 1] - wa[T - 1], A.Fc[i * pitch], cc[i]);
            }
        }
        if (J >= 3) {
            const double *fj = A.far + (int64_t)J * 2 * D * kBlk;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                pc[i] += fj[i * kBlk + tid];
                cc[i] += fj[(D + i) * kBlk + tid];
            }
        }
        __syncthreads();
    }

    for (int64_t t = (J == 0 ? 1 : t0); t <= tend; ++t) {
        const int r = (int)(t - t0);
        double *slot = fs + (t & 1) * D;
        if (tid == r) {
            double y[D], f[D];
            pece_update<SYS, D>(m, (double)t * m.h, y0, pc, cc, p, y, f);
            if (!finite_all(y) || !finite_all(f)) {
                *s_dead = t;
            } else {
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    slot[i] = f[i];
                    A.Fc[i * pitch + t] = f[i];
                    A.Y[t * D + i] = y[i];
                }
            }
        }
        __syncthreads();
        if (*s_dead) break;
        double f[D];
#pragma unroll
        for (int i = 0; i < D; ++i) f[i] = slot[i];
        if (tid > r) {
            const int lag = tid - r - 1;
            const double bw = sb[lag], aw = sa[lag];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                pc[i] = fma(bw, f[i], pc[i]);
                cc[i] = fma(aw, f[i], cc[i]);
            }
        }
        const int lag = kBlk + tid - r - 1;
        const double bw = sb[lag], aw = sa[lag];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            pn[i] = fma(bw, f[i], pn[i]);
            cn[i] = fma(aw, f[i], cn[i]);
        }
    }
    const int64_t dead = *s_dead;
    if (dead) {
        if (tid == 0) *A.dead = (uint32_t)dead;
        for (int64_t row = dead + tid; row <= tend; row += kBlk)
#pragma unroll
            for (int i = 0; i < D; ++i) A.Y[row * D + i] = __builtin_nan("");
        return;
    }
    double *cout = A.carry + (int64_t)((J + 1) & 1) * 2 * D * kBlk;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        cout[i * kBlk + tid] = pn[i];
        cout[(D + i) * kBlk + tid] = cn[i];
    }
}

// One workgroup per item {J, I0, I1, dest} of a far step.
template <int D>
__global__ __launch_bounds__(kBlk) void k_far_items(PipeArgs A, int item0)
{
    extern __shared__ __align__(16) char smem[];
    double *red = (double *)smem;
    const int4 it = A.items[item0 + blockIdx.x];
    const InstMeta m = A.meta[0];
    const int64_t pitch = (int64_t)A.NB * kBlk;
    double sP[D], sC[D];
    toeplitz_block_fp64<D>(A.W, A.W + m.wlen, A.Fc, pitch, it.x, it.y, it.z, red, sP, sC);
    double *out = it.w >= 0 ? A.task_slot + (int64_t)it.w * 2 * D * kBlk
                            : A.scratch + (int64_t)(-it.w - 1) * 2 * D * kBlk;
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        out[i * kBlk + tid] = sP[i];
        out[(D + i) * kBlk + tid] = sC[i];
    }
}

// Workgroups [0, 2D*nred): workgroup (task, cw) adds the items of a
// multi-item task in order for output column group cw. Workgroups
// [2D*nred, 2D*nred + 2D) (when Jfin >= 0): finalise column group cw of the
// far sum of target block Jfin from its task partials in source order.
template <int D>
__global__ __launch_bounds__(kBlk) void k_far_reduce(PipeArgs A, int red0, int nred, int Jfin)
{
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    if (b < 2 * D * nred) {
        const int4 rd = A.reds[red0 + b / (2 * D)];
        const int cw = b % (2 * D);
        double s = 0.0;
        for (int k = 0; k < rd.z; ++k)
            s += A.scratch[((int64_t)(rd.y + k) * 2 * D + cw) * kBlk + tid];
        A.task_slot[((int64_t)rd.x * 2 * D + cw) * kBlk + tid] = s;
        return;
    }
    const int cw = b - 2 * D * nred;
    const InstMeta m = A.meta[0];
    const int64_t pitch = (int64_t)A.NB * kBlk;
    const int k0 = A.tt_off[Jfin], k1 = A.tt_off[Jfin + 1];
    double s = 0.0;
    for (int k = k0; k < k1; ++k)
        s += A.task_slot[((int64_t)A.tt_slot[k] * 2 * D + cw) * kBlk + tid];
    if (cw >= D) {  // source row 0 takes c_{T-1}, not a_{T-1}
        const double *wa = A.W + m.wlen, *wc = wa + m.wlen;
        const int64_t T = (int64_t)Jfin * kBlk + tid;
        s = fma(wc[T - 1] - wa[T - 1], A.Fc[(cw - D) * pitch], s);
    }
    A.far[((int64_t)Jfin * 2 * D + cw) * kBlk + tid] = s;
}

__global__ void k_pipe_status(PipeArgs A)
{
    if (threadIdx.x == 0) A.status[0] = (int64_t)*A.dead;
}

// ---------------------------------------------------------------------------
// Host side: one enqueue of the whole pipeline.
// ---------------------------------------------------------------------------
// The band kernel asks for more LDS than a compute unit (160 KiB) can share
// with a far-tile workgroup (8 d KiB... 48 KiB for d = 3): far tiles then
// never land on the band's CU, whose single workgroup is latency-bound.
constexpr size_t kCuLds = 160 * 1024;
size_t pipe_far_smem(int d);
size_t pipe_band_smem(int d)
{
    const size_t need = sizeof(double) * (4 * kBlk + 2 * d + 8 * d * kBlk) + 16;
    const size_t exclusive = kCuLds - pipe_far_smem(d) + 1024;
    return need > exclusive ? need : exclusive;
}
size_t pipe_far_smem(int d) { return sizeof(double) * 8 * d * kBlk; }

template <int SYS, int D>
static hipError_t enqueue_pipe_t(const PipeArgs &A, const PipeSchedule &S, hipStream_t s,
                                 hipStream_t s2, hipEvent_t *ev_band, hipEvent_t *ev_far,
                                 int n_ev, KernelTimer *T, const char **where)
{
    // on failure *where names the call that failed
#define FABM_PIPE_TRY(what, expr)          \
    do {                                   \
        const hipError_t e_ = (expr);      \
        if (e_ != hipSuccess) {            \
            *where = what;                 \
            return e_;                     \
        }                                  \
    } while (0)
    static bool attr_done = false;
    const size_t smb = pipe_band_smem(D), smf = pipe_far_smem(D);
    if (!attr_done) {
        FABM_PIPE_TRY("hipFuncSetAttribute(band LDS)",
                      hipFuncSetAttribute((const void *)k_band_block<SYS, D>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)smb));
        FABM_PIPE_TRY("hipFuncSetAttribute(far LDS)",
                      hipFuncSetAttribute((const void *)k_far_items<D>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)smf));
        attr_done = true;
    }
    const int NB = S.NB;
    for (int J = 0; J < NB; ++J) {
        if (J >= 3)
            FABM_PIPE_TRY("hipStreamWaitEvent(band <- far)", hipStreamWaitEvent(s, ev_far[J % n_ev], 0));
        if (T) FABM_PIPE_TRY("timer begin", T->begin(KC_BAND, s));
        hipLaunchKernelGGL((k_band_block<SYS, D>), dim3(1), dim3(kBlk), smb, s, A, J);
        FABM_PIPE_TRY("launch k_band_block", hipGetLastError());
        if (T) FABM_PIPE_TRY("timer end", T->end(s));
        const int I = J;
        const int i0 = S.step_item_off[I], i1 = S.step_item_off[I + 1];
        const int r0 = S.step_red_off[I], r1 = S.step_red_off[I + 1];
        const int Jfin = I + 3 < NB ? I + 3 : -1;
        if (i1 > i0 || r1 > r0 || Jfin >= 0) {
            FABM_PIPE_TRY("hipEventRecord(band)", hipEventRecord(ev_band[I % n_ev], s));
            FABM_PIPE_TRY("hipStreamWaitEvent(far <- band)",
                          hipStreamWaitEvent(s2, ev_band[I % n_ev], 0));
            if (i1 > i0) {
                if (T) FABM_PIPE_TRY("timer begin", T->begin(KC_FAR_ITEMS, s2));
                hipLaunchKernelGGL(k_far_items<D>, dim3(i1 - i0), dim3(kBlk), smf, s2, A, i0);
                FABM_PIPE_TRY("launch k_far_items", hipGetLastError());
                if (T) FABM_PIPE_TRY("timer end", T->end(s2));
            }
            const int nb = 2 * D * ((r1 - r0) + (Jfin >= 0 ? 1 : 0));
            if (nb > 0) {
                if (T) FABM_PIPE_TRY("timer begin", T->begin(KC_FAR_REDUCE, s2));
                hipLaunchKernelGGL(k_far_reduce<D>, dim3(nb), dim3(kBlk), 0, s2, A, r0, r1 - r0,
                                   Jfin);
                FABM_PIPE_TRY("launch k_far_reduce", hipGetLastError());
                if (T) FABM_PIPE_TRY("timer end", T->end(s2));
            }
            if (Jfin >= 0)
                FABM_PIPE_TRY("hipEventRecord(far)", hipEventRecord(ev_far[Jfin % n_ev], s2));
        }
    }
    hipLaunchKernelGGL(k_pipe_status, dim3(1), dim3(64), 0, s, A);
    FABM_PIPE_TRY("launch k_pipe_status", hipGetLastError());
    return hipSuccess;
#undef FABM_PIPE_TRY
}

hipError_t enqueue_pipe(int sys, int d, const PipeArgs &A, const PipeSchedule &S, hipStream_t s,
                        hipStream_t s2, hipEvent_t *ev_band, hipEvent_t *ev_far, int n_ev,
                        KernelTimer *T, const char **where)
{
#define FABM_PIPE_CASE(SS, DD) \
    if (sys == SS && d == DD) return enqueue_pipe_t<SS, DD>(A, S, s, s2, ev_band, ev_far, n_ev, T, where);
    FABM_PIPE_CASE(SYS_LINEAR, 1)
    FABM_PIPE_CASE(SYS_LINEAR, 2)
    FABM_PIPE_CASE(SYS_LINEAR, 3)
    FABM_PIPE_CASE(SYS_LINEAR, 4)
    FABM_PIPE_CASE(SYS_CHEN, 3)
    FABM_PIPE_CASE(SYS_ROSSLER, 3)
    FABM_PIPE_CASE(SYS_VDP, 2)
    FABM_PIPE_CASE(SYS_FINANCIAL, 3)
#undef FABM_PIPE_CASE
    *where = "no BLOCKED kernel for this system/dimension";
    return hipErrorInvalidValue;
}

int pipe_block_len() { return kBlk; }

}  // namespace fabm
