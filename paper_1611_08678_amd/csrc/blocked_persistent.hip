// blocked_persistent.hip -- single-launch variant of the BLOCKED path for one
// long trajectory (band and far workers in one persistent kernel, handing work
// over through flags in global memory). NOT DISPATCHED: on MI355X the launch
// with far tasks did not complete; the flag polling compiles to plain cached
// loads that may not observe another XCD's update. Kept for reference and
// re-enablement; the dispatched BLOCKED path is the event-ordered pipeline in
// blocked.hip.
//
// The history sums of Section 2 are Toeplitz in the lag t-1-k. Rows are cut
// into blocks of L = 256 steps; for a target in block J the sources are split
//   far : k <  (J-1) L   (complete one whole block before J starts)
//   near: (J-1) L <= k < t
// One persistent cooperative launch runs two roles at once:
//
//  * the band (workgroup 0) walks the steps in order. Thread i owns the
//    accumulators of target rows JL+i (current block) and (J+1)L+i (next
//    block). After row t is formed, f_t is broadcast through LDS and every
//    thread adds its own w[T-1-t] f_t (one FMA per weight and component) to
//    its targets T > t, so at step t the owner of row t already holds
//    P_t and C_t minus nothing: one barrier per step, no global traffic on
//    the critical path except the f_t/y_t stores. At each block start it adds
//    the far sums of the new block and publishes how many blocks are done.
//
//  * far workers (all other workgroups) pop tasks (J, source blocks [I0, I1))
//    from a queue ordered by the block whose completion they wait for. A task
//    is a long Toeplitz contraction done on FP64 MFMA in polyphase form:
//    with r = 16 rho + sigma and k = 16 kappa + tau, W_q[sigma][tau] =
//    w[16 q + sigma - tau - 1] depends only on the column lag q = rho - kappa,
//    so out[:, rho] += W_q . F[:, rho - q] is a 16x16x16 product per (q, comp,
//    weight) and every column keeps its accumulator. Source chunks double in
//    length with their distance from the target (1, 2, 4, ... blocks), so a
//    chunk of s blocks has about s blocks of band time before it is needed
//    while most flops sit in long, fully dense chunks. Per-task partials are
//    summed in source order by whichever task of a target finishes last
//    (deterministic), which also adds the (c - a) f_0 correction of source 0.
#include "fabm_device.h"
#include "fabm_launch.h"
#include "fabm_blocked.h"

namespace fabm {

namespace {

constexpr int kL = 256;       // block length = band workgroup size
constexpr int kThreads = 256;
constexpr int kTile = 16;     // polyphase factor = MFMA edge

typedef double dbl4 __attribute__((ext_vector_type(4)));

}  // namespace


template <int SYS, int D>
__device__ void band_role(const BlockedArgs &A, char *smem)
{
    double *sb = (double *)smem;          // b lags 0..2L-1
    double *sa = sb + 2 * kL;             // a lags 0..2L-1
    double *fs = sa + 2 * kL;             // [2][D] broadcast slots
    int64_t *s_dead = (int64_t *)(fs + 2 * D);
    int *s_abort = (int *)(s_dead + 1);
    const int tid = threadIdx.x;
    const InstMeta m = A.meta[0];
    const int64_t N = m.N;
    const int64_t pitch = (int64_t)A.NB * kL;
    const double *wb = A.W, *wa = wb + m.wlen, *wc = wa + m.wlen;
    const double *p = A.params;
    double y0[D];
#pragma unroll
    for (int i = 0; i < D; ++i) y0[i] = A.y0[i];

    for (int j = tid; j < 2 * kL; j += kThreads) {
        sb[j] = wb[j];
        sa[j] = wa[j];
    }
    if (tid == 0) {
        double f0[D];
        rhs<SYS, D>(0.0, y0, f0, p);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            fs[i] = f0[i];
            A.Fc[i * pitch] = f0[i];
            A.Y[i] = y0[i];
        }
        *s_dead = 0;
        *s_abort = 0;
    }
    __syncthreads();

    double pc[D], cc[D], pn[D], cn[D];  // current / next block accumulators
    {
        // source k = 0 feeds targets 1 .. 2L-1 with b_{T-1} and c_{T-1}
        const int64_t Tc = tid, Tn = kL + tid;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double f0 = fs[i];
            pc[i] = Tc >= 1 ? wb[Tc - 1] * f0 : 0.0;
            cc[i] = Tc >= 1 ? wc[Tc - 1] * f0 : 0.0;
            pn[i] = wb[Tn - 1] * f0;
            cn[i] = wc[Tn - 1] * f0;
        }
    }

    int64_t t = 1;
    for (; t <= N; ++t) {
        const int r = (int)(t % kL);
        if (r == 0) {
            const int J = (int)(t / kL);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                pc[i] = pn[i];
                cc[i] = cn[i];
                pn[i] = cn[i] = 0.0;
            }
            __syncthreads();  // every f row of block J-1 is stored
            if (tid == 0) flag_publish(&A.sync[0], (uint32_t)J);
            if (J >= 2) {
                if (tid == 0) *s_abort = !wait_geq(&A.ready[J], 1u, &A.sync[3], A.timeout_ticks);
                __syncthreads();
                if (*s_abort) break;
                fence_acquire();
                const double *fj = A.far + (int64_t)J * 2 * D * kL;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    pc[i] += fj[i * kL + tid];
                    cc[i] += fj[(D + i) * kL + tid];
                }
            }
        }
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
        {
            const int lag = kL + tid - r - 1;
            const double bw = sb[lag], aw = sa[lag];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                pn[i] = fma(bw, f[i], pn[i]);
                cn[i] = fma(aw, f[i], cn[i]);
            }
        }
    }
    // a non-finite row stops the band; an expired wait aborts the launch (-1)
    const int64_t dead = *s_abort ? t : *s_dead;
    if (tid == 0) {
        A.status[0] = *s_abort ? -1 : dead;
        if (dead) {
            flag_max(&A.sync[2], (uint32_t)dead);
            flag_publish(&A.sync[0], (uint32_t)A.NB);  // let waiting far tasks drain
        }
    }
    if (dead)
        for (int64_t row = dead + tid; row <= N; row += kThreads)
#pragma unroll
            for (int i = 0; i < D; ++i) A.Y[row * D + i] = __builtin_nan("");
}

// One far task: partial sums of target block J from source blocks [I0, I1)
// for both weight tables, written to part[task] as [2D][L].
template <int D>
__device__ void far_task(const BlockedArgs &A, int task, double *red)
{
    const int4 tk = A.tasks[task];
    const int J = tk.x, I0 = tk.y, I1 = tk.z;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const InstMeta m = A.meta[0];
    const int64_t pitch = (int64_t)A.NB * kL;
    const double *wb = A.W, *wa = wb + m.wlen;

    const int rho = lane & 15, kq = lane >> 4;       // B column / K row within a 4-chunk
    const int64_t colT = (int64_t)J * (kL / kTile);  // first target column
    const int64_t k0 = (int64_t)I0 * (kL / kTile), k1 = (int64_t)I1 * (kL / kTile);
    const int64_t qlo = colT - k1 + 1, nq = (k1 - k0) + kTile - 1;
    const int64_t qa = qlo + (nq * wv) / 4, qb = qlo + (nq * (wv + 1)) / 4;

    dbl4 acc[D][2];
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i][0] = acc[i][1] = (dbl4){0.0, 0.0, 0.0, 0.0};

    for (int64_t q = qa; q < qb; ++q) {
        const int64_t col = colT + rho - q;             // source column of this lane
        const bool ok = col >= k0 && col < k1;
        const int64_t wbase = kTile * q + rho - kq - 1;  // A: row sigma = rho (lane & 15), k = kq
        double ab[4], aa[4], bf[D][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            ab[j] = wb[wbase - 4 * j];
            aa[j] = wa[wbase - 4 * j];
            // out-of-chunk columns read row 0 (always in bounds) and are zeroed
            const int64_t row = ok ? kTile * col + 4 * j + kq : 0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double v = A.Fc[i * pitch + row];
                bf[i][j] = ok ? v : 0.0;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < D; ++i) {
                acc[i][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ab[j], bf[i][j], acc[i][0], 0, 0, 0);
                acc[i][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[j], bf[i][j], acc[i][1], 0, 0, 0);
            }
    }
    // accumulator element v of lane l is D[sigma = 4 v + l/16][rho = l % 16]
    // -> target row 16 rho + sigma
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = kTile * rho + 4 * v + kq;
            red[((wv * 2 * D) + i) * kL + row] = acc[i][0][v];
            red[((wv * 2 * D) + D + i) * kL + row] = acc[i][1][v];
        }
    __syncthreads();
    double *out = A.part + (int64_t)task * 2 * D * kL;
#pragma unroll
    for (int cw = 0; cw < 2 * D; ++cw) {
        double s = red[cw * kL + tid];
#pragma unroll
        for (int w = 1; w < 4; ++w) s += red[(w * 2 * D + cw) * kL + tid];
        out[cw * kL + tid] = s;
    }
}

template <int D>
__device__ void far_role(const BlockedArgs &A, char *smem)
{
    double *red = (double *)smem;  // [4][2D][L]
    int *s_task = (int *)(red + 4 * 2 * D * kL);
    int *s_last = s_task + 1;
    const int tid = threadIdx.x;
    const InstMeta m = A.meta[0];
    const int64_t pitch = (int64_t)A.NB * kL;
    const double *wa = A.W + m.wlen, *wc = wa + m.wlen;
    for (;;) {
        if (tid == 0) {
            const uint32_t qi = __hip_atomic_fetch_add(&A.sync[1], 1u, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            *s_task = (int)qi < A.n_tasks ? A.queue[qi] : -1;
            if (*s_task >= 0 &&
                !wait_geq(&A.sync[0], (uint32_t)A.tasks[*s_task].z, &A.sync[3], A.timeout_ticks))
                *s_task = -1;
        }
        __syncthreads();
        const int task = *s_task;
        if (task < 0) break;
        fence_acquire();
        far_task<D>(A, task, red);
        __syncthreads();  // partial stored by every thread
        const int J = A.tasks[task].x;
        if (tid == 0) {
            const int K = A.task_off[J + 1] - A.task_off[J];
            const uint32_t old = __hip_atomic_fetch_add(&A.done[J], 1u, __ATOMIC_ACQ_REL,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            *s_last = (int)old == K - 1;
        }
        __syncthreads();
        if (*s_last) {
            fence_acquire();
            const int t0 = A.task_off[J], t1 = A.task_off[J + 1];
            const int64_t T = (int64_t)J * kL + tid;  // target row
            const double ca = wc[T - 1] - wa[T - 1];  // source 0 uses c, not a
            double *fj = A.far + (int64_t)J * 2 * D * kL;
#pragma unroll
            for (int cw = 0; cw < 2 * D; ++cw) {
                double s = 0.0;
                for (int k = t0; k < t1; ++k) s += A.part[((int64_t)k * 2 * D + cw) * kL + tid];
                if (cw >= D) s = fma(ca, A.Fc[(cw - D) * pitch], s);
                fj[cw * kL + tid] = s;
            }
            __syncthreads();
            if (tid == 0) flag_publish(&A.ready[J], 1u);
        }
    }
}

template <int SYS, int D>
__global__ __launch_bounds__(kThreads) void k_blocked_single(BlockedArgs A)
{
    extern __shared__ __align__(16) char smem[];
    if (blockIdx.x == 0)
        band_role<SYS, D>(A, smem);
    else
        far_role<D>(A, smem);
}

size_t blocked_smem_bytes(int d)
{
    const size_t band = sizeof(double) * (4 * kL + 2 * d) + 16;  // + s_dead, s_abort
    const size_t far = sizeof(double) * 4 * 2 * d * kL + 16;
    return band > far ? band : far;
}

hipError_t launch_blocked_single(int sys, int d, int G, const BlockedArgs &A, hipStream_t s)
{
    void *args[] = {(void *)&A};
    const size_t sm = blocked_smem_bytes(d);
#define FABM_BLK_CASE(S, DD)                                                                    \
    if (sys == S && d == DD)                                                                    \
        return hipLaunchCooperativeKernel((const void *)k_blocked_single<S, DD>, dim3(G),     \
                                          dim3(kThreads), args, (unsigned)sm, s);
    FABM_BLK_CASE(SYS_LINEAR, 1)
    FABM_BLK_CASE(SYS_LINEAR, 2)
    FABM_BLK_CASE(SYS_LINEAR, 3)
    FABM_BLK_CASE(SYS_LINEAR, 4)
    FABM_BLK_CASE(SYS_CHEN, 3)
    FABM_BLK_CASE(SYS_ROSSLER, 3)
    FABM_BLK_CASE(SYS_VDP, 2)
    FABM_BLK_CASE(SYS_FINANCIAL, 3)
    FABM_BLK_CASE(SYS_HINDMARSH_ROSE, 3)
#undef FABM_BLK_CASE
    return hipErrorInvalidValue;
}

int blocked_block_len() { return kL; }

}  // namespace fabm
