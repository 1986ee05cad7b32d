// blocked.hip -- the BLOCKED contraction path for one long trajectory as a
// sequence of step kernels (decomposition and launch contents in
// fabm_blocked.h).
//
// The history sums of Section 2 are Toeplitz in the lag t-1-k. Rows are cut
// into blocks of 256 and each block into 16 columns of 16 rows. With target
// row T = 256 J + 16 rho + sigma and source row k = 16 kappa + tau, the lag is
// 16 q + sigma - tau - 1 with the column lag q = 16 J + rho - kappa, so for a
// fixed q the sums over one source column are a 16x16 matrix W_q (entries
// w[16 q + sigma - tau - 1]) times a 16-vector of history. One window
// q = 16 m + u, u = 0..15, of a target block therefore costs, per weight
// table and state component, sixteen 16x16x16 products on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64, four K-slices each), with the 16 target
// columns rho as the N dimension: A = W_q (16 sigma x 4 tau), B = history
// (4 tau x 16 rho, column 16 (J - m) + rho - u), D = sums (16 sigma x 16 rho).
//
//  * band (workgroup 0): walks the 256 steps of block J. Thread i owns the
//    sums of target rows 256 J + i and 256 (J+1) + i. Row t is formed by its
//    owner (the predictor and corrector of Section 2), its f_t is broadcast
//    through LDS and every thread adds w[T-1-t] f_t to its targets T > t: one
//    barrier per step, no global memory traffic inside the walk. Rows are
//    written out after the walk; the next block's sums go to `carry`.
//  * near (workgroup 1, eight wavefronts): the column lags [rho+17, 47] of
//    target block J = s + 2, split over the wavefronts and added in LDS in a
//    fixed order.
//  * far (workgroups 2..): window m = J - s of each target block J >= s + 3,
//    one target per wavefront, accumulated in place in `acc`.
// Every sum is accumulated in a fixed order, so results are bit-reproducible.
#include <algorithm>

#include "fabm_blocked.h"
#include "fabm_device.h"
#include "fabm_launch.h"
#include "fabm_timer.h"

namespace fabm {

namespace {

constexpr int kBlk = 256;  // rows per block (= band threads)
constexpr int kTile = 16;  // polyphase factor = MFMA edge

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int n_params_of_sys(int sys, int d)
{
    return sys == SYS_LINEAR ? d * d + 2 * d : (sys == SYS_VDP ? 1 : 3);
}

}  // namespace

// ---------------------------------------------------------------------------
// Band: block J walked row by row by wavefronts 0..4 of workgroup 0.
//
// Wavefront 0 forms every row. Lane l holds the sums of the four target rows
// l, 64 + l, 128 + l, 192 + l of block J. At row t = 64 g + r the sums of
// lane r, group g are read out (readlane) and every lane evaluates the
// predictor and corrector with those same values, so f_t is present in all
// lanes without a broadcast; each lane then adds w[T-1-t] f_t to its targets
// T. No barrier is taken inside the walk. f_t and y_t go to LDS and a counter
// in LDS publishes how many rows are final.
// Wavefronts 1..4 hold the sums of the 256 rows of block J+1 (wavefront k,
// lane l: row 64 (k-1) + l) and add each published f_t as it appears; their
// sums are handed to the next block through `carry`.
// ---------------------------------------------------------------------------
constexpr int kBandWaves = 5;
constexpr uint32_t kSpinLimit = 1u << 26;  // polls of the row counter before giving up

__device__ __forceinline__ double readlane_f64(double x, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <int SYS, int D>
__device__ __forceinline__ void band_block(const StepArgs &A, int J, char *smem)
{
    double *sb = (double *)smem;  // b lags 0..511
    double *sa = sb + 2 * kBlk;   // a lags 0..511
    double *sF = sa + 2 * kBlk;   // [256][D] f of this block's rows
    double *sY = sF + kBlk * D;   // [256][D] y of this block's rows
    int *s_cnt = (int *)(sY + kBlk * D);  // rows of this block formed so far
    int *s_dead = s_cnt + 1;              // first non-finite row (block-relative), or -1
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
    const InstMeta m = A.meta[0];
    const int64_t N = m.N;
    const int64_t pitch = (int64_t)A.NB * kBlk;
    const double *wb = A.W, *wa = wb + m.wlen, *wc = wa + m.wlen;
    const int64_t t0 = (int64_t)J * kBlk;
    const int nrows = (int)((t0 + kBlk - 1 < N ? t0 + kBlk - 1 : N) - t0 + 1);
    constexpr int nthr = kBandWaves * kWave;

    // a non-finite state in an earlier block ends the trajectory
    if (*A.dead != 0u) {
        for (int e = tid; e < nrows * D; e += nthr) A.Y[t0 * D + e] = __builtin_nan("");
        return;
    }
    constexpr int NP = n_params_of_sys(SYS, D);
    double th[NP], y0[D];
#pragma unroll
    for (int k = 0; k < NP; ++k) th[k] = A.params[k];
#pragma unroll
    for (int i = 0; i < D; ++i) y0[i] = A.y0[i];
    for (int j = tid; j < 2 * kBlk; j += nthr) {
        sb[j] = wb[j];
        sa[j] = wa[j];
    }
    // f_0 (block 0 forms row 0 here; later blocks need it for the c - a fix)
    double f0[D];
    if (J == 0) {
        rhs<SYS, D>(0.0, y0, f0, th);
    } else {
#pragma unroll
        for (int i = 0; i < D; ++i) f0[i] = A.Fc[i * pitch];
    }
    if (tid == 0) {
        *s_cnt = J == 0 ? 1 : 0;
        *s_dead = -1;
        if (J == 0) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                sF[i] = f0[i];
                sY[i] = y0[i];
            }
        }
    }

    if (wave == 0) {
        // sums of rows 64 g + lane of block J
        double pc[4][D], cc[4][D];
        const double *cin = A.carry + (int64_t)(J & 1) * 2 * D * kBlk;
        const double *aj = A.acc + (int64_t)J * 2 * D * kBlk;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int row = 64 * g + lane;
            const int64_t T = t0 + row;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                if (J == 0) {
                    // source row 0 feeds targets 1..255 with b_{T-1} and c_{T-1}
                    pc[g][i] = T >= 1 ? wb[T - 1] * f0[i] : 0.0;
                    cc[g][i] = T >= 1 ? wc[T - 1] * f0[i] : 0.0;
                } else {
                    pc[g][i] = cin[i * kBlk + row];
                    cc[g][i] = cin[(D + i) * kBlk + row];
                }
            }
            if (J >= 2) {
                // near + far sums, stored in MFMA result order: row 16 rho + sigma
                // is element sigma/4 of lane 16 (sigma % 4) + rho
                const int rho = row >> 4, sig = row & 15;
                const int e = (sig >> 2) * kWave + 16 * (sig & 3) + rho;
                const double dca = wc[T - 1] - wa[T - 1];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    pc[g][i] += aj[i * kBlk + e];
                    // source row 0 takes c_{T-1} where the tiles used a_{T-1}
                    cc[g][i] = fma(dca, f0[i], cc[g][i] + aj[(D + i) * kBlk + e]);
                }
            }
        }
        __syncthreads();
        bool alive = true;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int r0 = (g == 0 && J == 0) ? 1 : 0;
            const int r1 = nrows - 64 * g < 64 ? nrows - 64 * g : 64;
            for (int r = r0; alive && r < r1; ++r) {
                const int row = 64 * g + r;
                const int64_t t = t0 + row;
                double P[D], Cs[D], y[D], f[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    P[i] = readlane_f64(pc[g][i], r);
                    Cs[i] = readlane_f64(cc[g][i], r);
                }
                pece_update<SYS, D>(m, (double)t * m.h, y0, P, Cs, th, y, f);
                if (!finite_all(y) || !finite_all(f)) {
                    if (lane == 0) *s_dead = row;
                    alive = false;
                    break;
                }
                if (lane == 0) {
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        sF[row * D + i] = f[i];
                        sY[row * D + i] = y[i];
                    }
                    __hip_atomic_store(s_cnt, row + 1, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                // targets 64 g2 + lane > row (lags of earlier rows are clamped
                // to 0; those sums are no longer read)
#pragma unroll
                for (int g2 = g; g2 < 4; ++g2) {
                    const int lag = 64 * g2 + lane - row - 1;
                    const int lc = lag > 0 ? lag : 0;
                    const double bw = sb[lc], aw = sa[lc];
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        pc[g2][i] = fma(bw, f[i], pc[g2][i]);
                        cc[g2][i] = fma(aw, f[i], cc[g2][i]);
                    }
                }
            }
        }
        if (!alive && lane == 0)
            __hip_atomic_store(s_cnt, kBlk + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();
    } else {
        // wavefronts 1..4: sums of row 64 (wave-1) + lane of block J+1
        const int row = 64 * (wave - 1) + lane;
        double pn[D], cn[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            // source row 0 of block 0 takes b_{T-1} and c_{T-1}
            pn[i] = J == 0 ? wb[kBlk + row - 1] * f0[i] : 0.0;
            cn[i] = J == 0 ? wc[kBlk + row - 1] * f0[i] : 0.0;
        }
        __syncthreads();
        int done = J == 0 ? 1 : 0;
        uint32_t spins = 0;
        while (done < nrows) {
            const int avail = __hip_atomic_load(s_cnt, __ATOMIC_ACQUIRE,
                                                __HIP_MEMORY_SCOPE_WORKGROUP);
            if (avail > kBlk) break;  // the walk stopped at a non-finite row
            if (avail == done) {
                if (++spins > kSpinLimit) {
                    if (lane == 0) __hip_atomic_store(s_dead, -2, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            for (; done < avail; ++done) {
                const int lag = kBlk + row - done - 1;
                const double bw = sb[lag], aw = sa[lag];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const double f = sF[done * D + i];
                    pn[i] = fma(bw, f, pn[i]);
                    cn[i] = fma(aw, f, cn[i]);
                }
            }
        }
        __syncthreads();
        if (*s_dead == -1) {
            double *cout = A.carry + (int64_t)((J + 1) & 1) * 2 * D * kBlk;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                cout[i * kBlk + row] = pn[i];
                cout[(D + i) * kBlk + row] = cn[i];
            }
        }
    }
    // rows of this block: final ones from LDS, NaN from the first non-finite on
    const int dead = *s_dead;
    const int valid = dead == -1 ? nrows : (dead < 0 ? 0 : dead);
    for (int e = tid; e < nrows * D; e += nthr)
        A.Y[t0 * D + e] = e / D < valid ? sY[e] : __builtin_nan("");
    for (int e = tid; e < valid; e += nthr) {
#pragma unroll
        for (int i = 0; i < D; ++i) A.Fc[i * pitch + t0 + e] = sF[e * D + i];
    }
    if (dead != -1 && tid == 0) *A.dead = dead == -2 ? kDeadWatchdog : (uint32_t)(t0 + dead);
}

// ---------------------------------------------------------------------------
// One column lag q = 16 m + u of a target block, for both weight tables and
// all components, added into `acc` (one wavefront). kc = 16 (J - m) is the
// source column of rho = 0 at u = 0; source columns outside [0, kmax] are
// masked to zero.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void window_lag(dbl4 (&acc)[2][D], const double *__restrict__ wb,
                                           const double *__restrict__ wa,
                                           const double *__restrict__ Fc, int64_t pitch,
                                           int64_t kc, int64_t m, int u, int64_t kmax)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int r16 = lane & 15, kq = lane >> 4;  // A row sigma / B column rho; K slot
    const int64_t kappa = kc + r16 - u;
    const bool ok = kappa >= 0 && kappa <= kmax;
    const int64_t fb = ok ? kTile * kappa + kq : 0;  // masked lanes read row 0
    const int64_t wi = kBlk * m + kTile * u + r16 - kq - 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double ab = wb[wi - 4 * j], aa = wa[wi - 4 * j];
        double bf[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double v = Fc[i * pitch + fb + 4 * j];
            bf[i] = ok ? v : 0.0;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            acc[0][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ab, bf[i], acc[0][i], 0, 0, 0);
            acc[1][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa, bf[i], acc[1][i], 0, 0, 0);
        }
    }
}

// Far windows of step s: wavefront g of G handles targets J = s + 3 + g,
// s + 3 + g + G, ... (window m = J - s, sources in blocks s - 1 and s).
template <int D>
__device__ __forceinline__ void far_windows(const StepArgs &A, int s, int g, int G)
{
    const InstMeta m = A.meta[0];
    const int64_t pitch = (int64_t)A.NB * kBlk;
    const double *wb = A.W, *wa = wb + m.wlen;
    const int lane = threadIdx.x & (kWave - 1);
    for (int J = s + 3 + g; J < A.NB; J += G) {
        double *aj = A.acc + (int64_t)J * 2 * D * kBlk + lane;
        dbl4 acc[2][D];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[t][i][v] = s == 0 ? 0.0 : aj[((t * D + i) * 4 + v) * kWave];
        const int64_t mm = J - s;
        for (int u = 0; u < kTile; ++u)
            window_lag<D>(acc, wb, wa, A.Fc, pitch, (int64_t)kTile * s, mm, u,
                          (int64_t)kTile * s + kTile - 1);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) aj[((t * D + i) * 4 + v) * kWave] = acc[t][i][v];
    }
}

// Near part of target block J = s + 2: column lags 17..47 (windows m = 2,
// all u, and m = 1, u = 1..15), masked to source columns <= 16 s + 15.
template <int D>
__device__ __forceinline__ void near_part(const StepArgs &A, int s, char *smem)
{
    double *red = (double *)smem;  // [kNearWaves][2D][4][64]
    const InstMeta m = A.meta[0];
    const int64_t pitch = (int64_t)A.NB * kBlk;
    const double *wb = A.W, *wa = wb + m.wlen;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid >> 6;
    const int J = s + 2;
    constexpr int kLags = 31;
    dbl4 acc[2][D];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < D; ++i) acc[t][i] = (dbl4){0.0, 0.0, 0.0, 0.0};
    const int p0 = kLags * w / kNearWaves, p1 = kLags * (w + 1) / kNearWaves;
    for (int p = p0; p < p1; ++p) {
        const int mm = p < kTile ? 2 : 1;
        const int u = p < kTile ? p : p - (kTile - 1);
        window_lag<D>(acc, wb, wa, A.Fc, pitch, (int64_t)kTile * (J - mm), mm, u,
                      (int64_t)kTile * s + kTile - 1);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                red[((w * 2 * D + t * D + i) * 4 + v) * kWave + lane] = acc[t][i][v];
    __syncthreads();  // the eight near wavefronts
    double *aj = A.acc + (int64_t)J * 2 * D * kBlk;
    for (int e = tid; e < 2 * D * kBlk; e += kNearWaves * kWave) {
        double v = s == 0 ? 0.0 : aj[e];
#pragma unroll
        for (int k = 0; k < kNearWaves; ++k) v += red[k * 2 * D * kBlk + e];
        aj[e] = v;
    }
}

// Launch s of the pipeline; `wpw` wavefronts of each far workgroup take part.
template <int SYS, int D>
__global__ __launch_bounds__(kStepThreads) void k_step(StepArgs A, int s, int wpw)
{
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x, wave = threadIdx.x >> 6;
    if (b == 0) {
        if (wave < kBandWaves) band_block<SYS, D>(A, s + 1, smem);
        return;
    }
    if (*A.dead != 0u) return;  // the trajectory has ended; later rows are NaN
    if (b == 1) {
        if (wave < kNearWaves) near_part<D>(A, s, smem);
        return;
    }
    if (wave < wpw) far_windows<D>(A, s, (b - 2) * wpw + wave, ((int)gridDim.x - 2) * wpw);
}

__global__ void k_step_status(StepArgs A)
{
    if (threadIdx.x == 0) {
        const uint32_t d = *A.dead;
        A.status[0] = d == kDeadWatchdog ? -1 : (int64_t)d;
    }
}

// ---------------------------------------------------------------------------
// Host side: one enqueue of the whole pipeline.
// ---------------------------------------------------------------------------
// Every workgroup asks for more than half of a compute unit's 160 KiB of
// LDS, so no two step workgroups share a compute unit: the band has one to
// itself and each far workgroup owns four SIMDs.
size_t step_smem_bytes(int d)
{
    const size_t band = sizeof(double) * (4 * kBlk + 2 * kBlk * (size_t)d) + 16;
    const size_t near = sizeof(double) * kNearWaves * 2 * (size_t)d * kBlk;
    const size_t exclusive = 81 * 1024;
    return std::max(band, std::max(near, exclusive));
}

// Grid of launch s: band, near and far workgroups, and the number of active
// wavefronts per far workgroup (one target each, four per round of SIMDs).
void step_grid(int NB, int s, int *grid, int *wpw)
{
    *grid = 1;
    *wpw = 0;
    if (s < 0 || s + 2 > NB - 1) return;
    *grid = 2;
    const int nt = NB - (s + 3);  // far targets
    if (nt <= 0) return;
    const int per_round = 4 * kMaxFarWg;
    const int rounds = std::min((nt + per_round - 1) / per_round, kStepThreads / kWave / 4);
    *wpw = 4 * rounds;
    *grid += std::min(kMaxFarWg, (nt + *wpw - 1) / *wpw);
}

template <int SYS, int D>
static hipError_t enqueue_steps_t(const StepArgs &A, hipStream_t st, KernelTimer *T,
                                  const char **where)
{
    // on failure *where names the call that failed
#define FABM_STEP_TRY(what, expr)          \
    do {                                   \
        const hipError_t e_ = (expr);      \
        if (e_ != hipSuccess) {            \
            *where = what;                 \
            return e_;                     \
        }                                  \
    } while (0)
    static bool attr_done = false;
    const size_t smem = step_smem_bytes(D);
    if (!attr_done) {
        FABM_STEP_TRY("hipFuncSetAttribute(step LDS)",
                      hipFuncSetAttribute((const void *)k_step<SYS, D>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
        attr_done = true;
    }
    for (int s = -1; s <= A.NB - 2; ++s) {
        int grid, wpw;
        step_grid(A.NB, s, &grid, &wpw);
        if (T) FABM_STEP_TRY("timer begin", T->begin(KC_BLOCKED_STEP, st));
        hipLaunchKernelGGL((k_step<SYS, D>), dim3(grid), dim3(kStepThreads), smem, st, A, s, wpw);
        FABM_STEP_TRY("launch k_step", hipGetLastError());
        if (T) FABM_STEP_TRY("timer end", T->end(st));
    }
    hipLaunchKernelGGL(k_step_status, dim3(1), dim3(kWave), 0, st, A);
    FABM_STEP_TRY("launch k_step_status", hipGetLastError());
    return hipSuccess;
#undef FABM_STEP_TRY
}

hipError_t enqueue_steps(int sys, int d, const StepArgs &A, hipStream_t s, KernelTimer *T,
                         const char **where)
{
#define FABM_STEP_CASE(SS, DD) \
    if (sys == SS && d == DD) return enqueue_steps_t<SS, DD>(A, s, T, where);
    FABM_STEP_CASE(SYS_LINEAR, 1)
    FABM_STEP_CASE(SYS_LINEAR, 2)
    FABM_STEP_CASE(SYS_LINEAR, 3)
    FABM_STEP_CASE(SYS_LINEAR, 4)
    FABM_STEP_CASE(SYS_CHEN, 3)
    FABM_STEP_CASE(SYS_ROSSLER, 3)
    FABM_STEP_CASE(SYS_VDP, 2)
    FABM_STEP_CASE(SYS_FINANCIAL, 3)
#undef FABM_STEP_CASE
    *where = "no BLOCKED kernel for this system/dimension";
    return hipErrorInvalidValue;
}

int step_block_len() { return kBlk; }

}  // namespace fabm
