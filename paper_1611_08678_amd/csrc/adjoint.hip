// adjoint.hip -- reverse-mode gradients (discrete adjoint) of the scheme of
// Section 2 with respect to y0 and theta, on the BLOCKED decomposition.
//
// For L = sum_n <g_n, y_n> the reverse pass runs n = N .. 1 with the sums
//   fbar_n = sum_{m > n} a_{m-1-n} u_m + b_{m-1-n} v_m     (n >= 1)
//   fbar_0 = sum_{m > 0} c_{m-1}   u_m + b_{m-1}   v_m
// and, at each n, with J_y, J_th the Jacobians of f:
//   ybar_n = g_n + J_y(t_n, y_n)^T fbar_n,        u_n = h^a ybar_n,
//   ypbar  = J_y(t_n, yP_n)^T (u_n / Gamma(a+2)), v_n = h^a ypbar,
//   d/dy0 collects g_0, every ybar_n and ypbar, and J_y(0, y0)^T fbar_0;
//   d/dth collects J_th^T fbar_n, J_th(yP_n)^T (u_n / Gamma(a+2)), J_th(0,y0)^T fbar_0.
// In reversed row order r = N - n the sums are causal Toeplitz sums of the
// reversed sources U_r = u_{N-r}, V_r = v_{N-r} with lag r - r' - 1, so the
// forward pipeline applies unchanged: blocks of 256 reversed rows, a band that
// walks a block row by row, and near and far windows on the FP64 matrix cores
// (two inputs, U with the a weights and V with the b weights, one output per
// component). Row r = N carries fbar_0; its c - a correction and the terms
// at y0 are added by a final per-instance kernel.
//
// The forward trajectory and its predictor values are recomputed by the
// forward pipeline into the workspace (bitwise the rows fabm_solve returns).
#include <algorithm>

#include "fabm_adjoint.h"
#include "fabm_blocked.h"
#include "fabm_device.h"
#include "fabm_launch.h"
#include "fabm_timer.h"

namespace fabm {

namespace {

constexpr int kBlk = 256;
constexpr int kTile = 16;
constexpr int kSrcCols = 31;
constexpr int kColPitch = 17;

typedef double dbl4 __attribute__((ext_vector_type(4)));


}  // namespace

// One instance as seen by the reverse kernels.
struct AdjView {
    const InstMeta *meta;
    const InstMeta *cmeta; // non-commensurate orders: [D] entries of this instance, or null
    const double *params;
    const double *Y, *YP;  // forward rows [N+1][D]
    const double *G;       // dL/dy rows [N+1][D]
    const double *W;       // b, a, c tables
    double *UV;            // reversed sources [2D][NB*256]: U then V
    double *carry;         // [2][D][256]
    double *acc;           // [NB][D][4][64]
    double *part;          // [NB][NP + 2D] per-block gradient partials
    double *fbar0;         // [D] band sums of reversed row N
    const uint32_t *dead;  // forward non-finite flag
    int NB;
    int slope;             // y'(0) partials wanted
    int ring;              // Y, YP are rings of this many 256-row blocks (0: every row)
};

template <int D>
__device__ __forceinline__ AdjView adj_view(const AdjArgs &A, int i, int np)
{
    const InstMeta *m = A.meta + i;
    const BlkInst &b = A.inst[i];
    return AdjView{m,
                   A.cmeta ? A.cmeta + (int64_t)i * D : nullptr,
                   A.params + m->p_off,
                   A.ring ? A.Y + (int64_t)i * A.ring * kBlk * D : A.Y + m->f_off * D,
                   A.ring ? A.YP + (int64_t)i * A.ring * kBlk * D : A.YP + m->f_off * D,
                   A.G + m->row_off * D,
                   A.W + m->w_off,
                   A.UV + 2 * b.fc_off,
                   A.carry + (int64_t)i * 2 * D * kBlk,
                   A.acc + b.acc_off / 2,
                   A.part + b.acc_off / (2 * D * kBlk) * (np + 2 * D),
                   A.fbar0 + (int64_t)i * D,
                   A.dead + i,
                   b.NB,
                   A.slope,
                   A.ring};
}

// ---------------------------------------------------------------------------
// Band of reversed block J: thread i owns the sums of reversed rows 256 J + i
// and 256 (J+1) + i. Row r is formed by its owner (the adjoint step), U_r and
// V_r go through LDS, every thread adds a_{T-1-r} U_r + b_{T-1-r} V_r to its
// targets T > r; one barrier per row. Each thread's gradient contributions
// (its single row) are reduced over the block in a fixed order at the end.
// ---------------------------------------------------------------------------
// PC: non-commensurate orders (component k's tables at k * 3 wlen, its
// scalars in A.cmeta[k]).
template <int SYS, int D, bool PC = false>
__device__ __forceinline__ void band_adj(const AdjView &A, int J, char *smem)
{
    constexpr int NP = n_params_of_sys(SYS, D);
    constexpr int K = PC ? D : 1;  // weight tables held
    // gradient partials: theta, y(0), then y'(0) (orders above one: every
    // row's initial part is y(0) + t_n y'(0))
    constexpr int NG = NP + 2 * D;
    double *sa = (double *)smem;      // [K] a lags 0..511
    double *sb = sa + K * 2 * kBlk;   // [K] b lags 0..511
    double *sU = sb + K * 2 * kBlk;   // [256][D]
    double *sV = sU + kBlk * D;   // [256][D]
    double *sRed = sV + kBlk * D; // [256] reduction scratch
    const int tid = threadIdx.x;
    const InstMeta m = A.meta[0];
    const int64_t N = m.N;
    const int64_t pitch = (int64_t)A.NB * kBlk;
    const double *wb = A.W, *wa = wb + m.wlen;
    const int64_t cw = 3 * m.wlen;
    const int64_t r0 = (int64_t)J * kBlk;
    const int nrows = (int)((r0 + kBlk - 1 < N ? r0 + kBlk - 1 : N) - r0 + 1);
    const int nstep = (int)((r0 + kBlk - 1 < N - 1 ? r0 + kBlk - 1 : N - 1) - r0 + 1);
    double hav[D], ig2v[D];  // h^a and 1 / Gamma(a + 2) of each component
#pragma unroll
    for (int i = 0; i < D; ++i) {
        hav[i] = PC ? A.cmeta[i].ha : m.ha;
        ig2v[i] = PC ? A.cmeta[i].ig2 : m.ig2;
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int j = tid; j < 2 * kBlk; j += kBlk) {
            sa[k * 2 * kBlk + j] = wa[k * cw + j];
            sb[k * 2 * kBlk + j] = wb[k * cw + j];
        }
    double S[D], Sn[D];
    if (J == 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) S[i] = Sn[i] = 0.0;
    } else {
        const double *cin = A.carry + (int64_t)(J & 1) * D * kBlk;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            S[i] = cin[i * kBlk + tid];
            Sn[i] = 0.0;
        }
        if (J >= 2) {
            const int rho = tid >> 4, sig = tid & 15;
            const int e = (sig >> 2) * kWave + 16 * (sig & 3) + rho;
            const double *aj = A.acc + (int64_t)J * D * kBlk;
#pragma unroll
            for (int i = 0; i < D; ++i) S[i] += aj[i * kBlk + e];
        }
    }
    // this thread's row: forward inputs at n = N - r
    double gpart[NG];
#pragma unroll
    for (int k = 0; k < NG; ++k) gpart[k] = 0.0;
    double yv[D], ypv[D], gv[D];
    const bool steps = tid < nstep;
    const int64_t n = N - (r0 + tid);
    // row n of the forward: its own row, or its place in the ring of blocks
    const int64_t nr = A.ring ? ((n >> 8) % A.ring) * kBlk + (n & (kBlk - 1)) : n;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        yv[i] = steps ? A.Y[nr * D + i] : 0.0;
        ypv[i] = steps ? A.YP[nr * D + i] : 0.0;
        gv[i] = steps ? A.G[n * D + i] : 0.0;
    }
    constexpr int NPR = NP;
    double th[NPR];
#pragma unroll
    for (int k = 0; k < NP; ++k) th[k] = A.params[k];
    __syncthreads();

    for (int r = 0; r < nstep; ++r) {
        if (tid == r) {
            const double tn = (double)n * m.h;
            double ybar[D], w2[D], ypbar[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                ybar[i] = gv[i];
                ypbar[i] = 0.0;
            }
            rhs_vjp<SYS, D>(tn, yv, S, th, ybar, gpart);
#pragma unroll
            for (int i = 0; i < D; ++i) w2[i] = hav[i] * ybar[i] * ig2v[i];
            rhs_vjp<SYS, D>(tn, ypv, w2, th, ypbar, gpart);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                gpart[NP + i] += ybar[i] + ypbar[i];
                gpart[NP + D + i] = fma(tn, ybar[i] + ypbar[i], gpart[NP + D + i]);
                sU[r * D + i] = hav[i] * ybar[i];
                sV[r * D + i] = hav[i] * ypbar[i];
            }
        }
        __syncthreads();
        double u[D], v[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            u[i] = sU[r * D + i];
            v[i] = sV[r * D + i];
        }
        if (tid > r) {
            const int lag = tid - r - 1;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int k = PC ? i : 0;
                const double aw = sa[k * 2 * kBlk + lag], bw = sb[k * 2 * kBlk + lag];
                S[i] = fma(bw, v[i], fma(aw, u[i], S[i]));
            }
        }
        const int lag = kBlk + tid - r - 1;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int k = PC ? i : 0;
            const double aw = sa[k * 2 * kBlk + lag], bw = sb[k * 2 * kBlk + lag];
            Sn[i] = fma(bw, v[i], fma(aw, u[i], Sn[i]));
        }
    }
    // reversed row N (fbar_0 without its c - a correction) lies in this block
    if (N - r0 < kBlk && tid == (int)(N - r0)) {
#pragma unroll
        for (int i = 0; i < D; ++i) A.fbar0[i] = S[i];
    }
    // sources of this block, the next block's sums
    for (int e = tid; e < nstep; e += kBlk) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            A.UV[i * pitch + r0 + e] = sU[e * D + i];
            A.UV[(D + i) * pitch + r0 + e] = sV[e * D + i];
        }
    }
    double *cout = A.carry + (int64_t)((J + 1) & 1) * D * kBlk;
#pragma unroll
    for (int i = 0; i < D; ++i) cout[i * kBlk + tid] = Sn[i];
    // gradient partials of the block: fixed-order tree over the 256 rows
    double *pj = A.part + (int64_t)J * NG;
    const int ng = A.slope ? NG : NP + D;
    for (int k = 0; k < ng; ++k) {
        __syncthreads();
        sRed[tid] = gpart[k];
        __syncthreads();
        for (int w = kBlk / 2; w >= 1; w >>= 1) {
            if (tid < w) sRed[tid] += sRed[tid + w];
            __syncthreads();
        }
        if (tid == 0) pj[k] = sRed[0];
    }
    (void)nrows;
}

// ---------------------------------------------------------------------------
// Windows: sums of reversed target block J from the staged sources of launch
// s (columns 16 s - 15 .. 16 s + 15; U then V), same decomposition as the
// forward pipeline, one sum per component: a weights on U, b weights on V.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void stage_uv(const AdjView &A, int s, double *sB)
{
    const int64_t pitch = (int64_t)A.NB * kBlk;
    const int64_t rr0 = (int64_t)kBlk * s - kTile * (kSrcCols - kTile);
    for (int e = threadIdx.x; e < 2 * D * kSrcCols * kTile; e += blockDim.x) {
        const int i = e / (kSrcCols * kTile), rem = e - i * (kSrcCols * kTile);
        const int c = rem / kTile, tau = rem - c * kTile;
        const int64_t row = rr0 + kTile * c + tau;
        sB[(i * kSrcCols + c) * kColPitch + tau] = row >= 0 ? A.UV[i * pitch + row] : 0.0;
    }
}

template <int D, bool PC = false>
__device__ __forceinline__ void window_adj(dbl4 (&acc)[D], const double *__restrict__ wa,
                                           const double *__restrict__ wb, const double *sB,
                                           int64_t m, int u, int coff, int64_t cw = 0)
{
    constexpr int K = PC ? D : 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int r16 = lane & 15, kq = lane >> 4;
    const int c = r16 - u + coff;
    const bool ok = c < kSrcCols;
    // K slot kq of slice j is source row 4 kq + j: a lane's operands of the
    // four slices are four consecutive weights and staged values
    const int sbase = (ok ? c : 0) * kColPitch + 4 * kq;
    const int64_t wi = kBlk * m + kTile * u + r16 - 4 * kq - 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double aa[K], ab[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            aa[k] = wa[k * cw + wi - j];
            ab[k] = wb[k * cw + wi - j];
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double vu = sB[i * kSrcCols * kColPitch + sbase + j];
            const double vv = sB[(D + i) * kSrcCols * kColPitch + sbase + j];
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[PC ? i : 0], ok ? vu : 0.0, acc[i],
                                                          0, 0, 0);
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ab[PC ? i : 0], ok ? vv : 0.0, acc[i],
                                                          0, 0, 0);
        }
    }
}

template <int D, bool PC = false>
__device__ __forceinline__ void far_adj(const AdjView &A, int s, int J, const double *sB)
{
    const InstMeta m = A.meta[0];
    const double *wb = A.W, *wa = wb + m.wlen;
    const int64_t cw = 3 * m.wlen;
    const int lane = threadIdx.x & (kWave - 1);
    double *aj = A.acc + (int64_t)J * D * kBlk + lane;
    dbl4 acc[D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[i][v] = s == 0 ? 0.0 : aj[(i * 4 + v) * kWave];
#pragma unroll 2
    for (int u = 0; u < kTile; ++u) window_adj<D, PC>(acc, wa, wb, sB, J - s, u, kTile - 1, cw);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) aj[(i * 4 + v) * kWave] = acc[i][v];
}

// Near part of reversed target block s + 2 (four wavefronts, partial sums
// added one wavefront after another into one LDS slot).
template <int D, bool PC = false>
__device__ __forceinline__ void near_adj(const AdjView &A, int s, const double *sB, double *red)
{
    const InstMeta m = A.meta[0];
    const double *wb = A.W, *wa = wb + m.wlen;
    const int64_t cw = 3 * m.wlen;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid >> 6;
    constexpr int NW = kBatchThreads / kWave;
    constexpr int kLags = 31;
    dbl4 acc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] = (dbl4){0.0, 0.0, 0.0, 0.0};
    const int p0 = kLags * w / NW, p1 = kLags * (w + 1) / NW;
    for (int p = p0; p < p1; ++p) {
        if (p < kTile)
            window_adj<D, PC>(acc, wa, wb, sB, 2, p, kTile - 1, cw);
        else
            window_adj<D, PC>(acc, wa, wb, sB, 1, p - (kTile - 1), 2 * kTile - 1, cw);
    }
    for (int k = 0; k < NW; ++k) {
        if (w == k) {
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double *r = red + (i * 4 + v) * kWave + lane;
                    *r = k == 0 ? acc[i][v] : *r + acc[i][v];
                }
        }
        __syncthreads();
    }
    double *aj = A.acc + (int64_t)(s + 2) * D * kBlk;
    for (int e = tid; e < D * kBlk; e += kBatchThreads) aj[e] = (s == 0 ? 0.0 : aj[e]) + red[e];
}

// Launch s of the reverse pipeline (same schedule as the forward batch).
template <int SYS, int D, bool PC = false>
__global__ __launch_bounds__(kBatchThreads) void k_adj_batch(AdjArgs A, int s, int nband, int nnear,
                                                             const int *far_off, int nfar)
{
    extern __shared__ __align__(16) char smem[];
    constexpr int NP = n_params_of_sys(SYS, D);
    int q = blockIdx.x;
    if (q < nband) {
        const AdjView V = adj_view<D>(A, A.order[q], NP);
        if (*V.dead != 0u) return;  // forward blew up: gradients are NaN
        band_adj<SYS, D, PC>(V, s + 1, smem);
        return;
    }
    q -= nband;
    int inst, first = -1;
    if (q < nnear) {
        inst = A.order[q];
    } else {
        q -= nnear;
        int lo = 0, hi = nfar;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (far_off[mid] <= q) lo = mid;
            else hi = mid;
        }
        inst = A.order[lo];
        first = s + 3 + 4 * (q - far_off[lo]);
    }
    const AdjView V = adj_view<D>(A, inst, NP);
    if (*V.dead != 0u) return;
    double *sB = (double *)smem;
    stage_uv<D>(V, s, sB);
    __syncthreads();
    if (first < 0) {
        near_adj<D, PC>(V, s, sB, sB + 2 * D * kSrcCols * kColPitch);
        return;
    }
    const int J = first + (threadIdx.x >> 6);
    if (J < V.NB) far_adj<D, PC>(V, s, J, sB);
}

// Per instance (one workgroup): fbar_0 = band sums of reversed row N plus
// sum_r (c - a)_{N-1-r} U_r; then the terms at y0 and the block partials,
// added in block order.
template <int SYS, int D, bool PC = false>
__global__ __launch_bounds__(kBatchThreads) void k_adj_final(AdjArgs A)
{
    constexpr int NP = n_params_of_sys(SYS, D);
    constexpr int NG = NP + 2 * D;
    const bool slope = A.slope != 0;
    __shared__ double red[kBatchThreads];
    __shared__ double fb0[D];
    const int i = blockIdx.x, tid = threadIdx.x;
    const AdjView V = adj_view<D>(A, i, NP);
    const InstMeta m = V.meta[0];
    const int64_t N = m.N;
    double *gy0 = A.gy0 + (int64_t)i * (slope ? 2 : 1) * D, *gth = A.gparams + m.p_off;
    const int ng = slope ? NG : NP + D;
    if (*V.dead != 0u) {
        for (int k = tid; k < ng; k += kBatchThreads) {
            if (k < NP) gth[k] = __builtin_nan("");
            else gy0[k - NP] = __builtin_nan("");
        }
        return;
    }
    const int64_t pitch = (int64_t)V.NB * kBlk;
    const double *wb = V.W, *wa = wb + m.wlen, *wc = wa + m.wlen;
    const int64_t cw = 3 * m.wlen;
    for (int c = 0; c < D; ++c) {
        const int64_t o = PC ? c * cw : 0;  // component c's tables
        double s = 0.0;
        for (int64_t r = tid; r < N; r += kBatchThreads)
            s = fma(wc[o + N - 1 - r] - wa[o + N - 1 - r], V.UV[c * pitch + r], s);
        red[tid] = s;
        __syncthreads();
        for (int w = kBatchThreads / 2; w >= 1; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0) fb0[c] = red[0] + V.fbar0[c];
        __syncthreads();
    }
    if (tid == 0) {
        double th[NP], y0[D], w[D], gy[D], gy1[D], gt[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            th[k] = V.params[k];
            gt[k] = 0.0;
        }
#pragma unroll
        for (int c = 0; c < D; ++c) {
            y0[c] = A.y0[(int64_t)i * D + c];
            w[c] = fb0[c];
            gy[c] = V.G[c];  // g_0
            gy1[c] = 0.0;
        }
        for (int J = 0; J < V.NB; ++J) {
            const double *pj = V.part + (int64_t)J * NG;
#pragma unroll
            for (int k = 0; k < NP; ++k) gt[k] += pj[k];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                gy[c] += pj[NP + c];
                gy1[c] += pj[NP + D + c];
            }
        }
        rhs_vjp<SYS, D>(0.0, y0, w, th, gy, gt);
#pragma unroll
        for (int k = 0; k < NP; ++k) gth[k] = gt[k];
#pragma unroll
        for (int c = 0; c < D; ++c) gy0[c] = gy[c];
        // y'(0) enters only for orders above one
        if (slope)
#pragma unroll
            for (int c = 0; c < D; ++c)
                gy0[D + c] = (PC ? V.cmeta[c].alpha : m.alpha) > 1.0 ? gy1[c] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
size_t adj_smem_bytes(int d, bool pc)
{
    const size_t band = sizeof(double) * (4 * kBlk * (size_t)(pc ? d : 1) + 2 * kBlk * (size_t)d +
                                          kBlk);
    const size_t win = sizeof(double) * (2 * (size_t)d * kSrcCols * kColPitch + (size_t)d * kBlk);
    return std::max(band, win);
}

template <int SYS, int D, bool PC>
static hipError_t enqueue_adjoint_t(const AdjArgs &A, const BatchSchedule &S, const int *far_off,
                                    hipStream_t st, KernelTimer *T, const char **where,
                                    const BatchArgs *fwd, const RecompArgs *rec)
{
#define FABM_ADJ_TRY(what, expr)           \
    do {                                   \
        const hipError_t e_ = (expr);      \
        if (e_ != hipSuccess) {            \
            *where = what;                 \
            return e_;                     \
        }                                  \
    } while (0)
    const size_t smem = adj_smem_bytes(D, PC);
    static std::atomic<uint64_t> attr_dev{0};
    if (PC)  // above the default limit only with per-component tables
        FABM_ADJ_TRY("hipFuncSetAttribute(adjoint LDS)",
                     ensure_lds_attr((const void *)k_adj_batch<SYS, D, PC>, smem, attr_dev));
    for (int s = -1; s <= S.max_NB - 2; ++s) {
        const size_t k = (size_t)(s + 1);
        const int nb = S.nband[k], nn = S.nnear[k], nf = S.nfar[k];
        const int nfw = S.far_off[(size_t)S.far_base[k] + (size_t)nf];
        const int grid = nb + nn + nfw;
        if (rec && (s + 1) % rec->G == 0 && nb > 0) {
            // forward rows of reverse launches s .. s + G - 1 (reversed blocks
            // s + 1 .. s + G); launch s reads none of the blocks it replaces
            if (T) FABM_ADJ_TRY("timer begin", T->begin(KC_ADJOINT, st));
            FABM_ADJ_TRY("launch k_recompute_batch",
                         launch_recompute(SYS, D, *fwd, *rec, s + 1, nb, st));
            if (T) FABM_ADJ_TRY("timer end", T->end(st));
        }
        if (grid == 0) continue;
        if (T) FABM_ADJ_TRY("timer begin", T->begin(KC_ADJOINT, st));
        hipLaunchKernelGGL((k_adj_batch<SYS, D, PC>), dim3(grid), dim3(kBatchThreads), smem, st,
                           A, s, nb, nn, far_off + S.far_base[k], nf);
        FABM_ADJ_TRY("launch k_adj_batch", hipGetLastError());
        if (T) FABM_ADJ_TRY("timer end", T->end(st));
    }
    hipLaunchKernelGGL((k_adj_final<SYS, D, PC>), dim3((unsigned)A.batch), dim3(kBatchThreads), 0,
                       st, A);
    FABM_ADJ_TRY("launch k_adj_final", hipGetLastError());
    return hipSuccess;
#undef FABM_ADJ_TRY
}

hipError_t enqueue_adjoint(int sys, int d, const AdjArgs &A, const BatchSchedule &S,
                           const int *far_off, hipStream_t s, KernelTimer *T, const char **where,
                           const BatchArgs *fwd, const RecompArgs *rec)
{
    if ((rec != nullptr) != (A.ring != 0) || (rec && (!fwd || A.ring != rec->G + 1))) {
        *where = "adjoint: block-checkpoint arguments inconsistent";
        return hipErrorInvalidValue;
    }
#define FABM_ADJ_CASE(SS, DD)                                                                \
    if (sys == SS && d == DD)                                                                \
        return A.cmeta ? enqueue_adjoint_t<SS, DD, true>(A, S, far_off, s, T, where, fwd, rec) \
                       : enqueue_adjoint_t<SS, DD, false>(A, S, far_off, s, T, where, fwd, rec);
    FABM_ADJ_CASE(SYS_LINEAR, 1)
    FABM_ADJ_CASE(SYS_LINEAR, 2)
    FABM_ADJ_CASE(SYS_LINEAR, 3)
    FABM_ADJ_CASE(SYS_LINEAR, 4)
    FABM_ADJ_CASE(SYS_CHEN, 3)
    FABM_ADJ_CASE(SYS_ROSSLER, 3)
    FABM_ADJ_CASE(SYS_VDP, 2)
    FABM_ADJ_CASE(SYS_FINANCIAL, 3)
    FABM_ADJ_CASE(SYS_HINDMARSH_ROSE, 3)
#undef FABM_ADJ_CASE
    *where = "no adjoint kernel for this system/dimension";
    return hipErrorInvalidValue;
}

__global__ __launch_bounds__(256) void k_copy_rows(const InstMeta *__restrict__ src_meta,
                                                   const InstMeta *__restrict__ dst_meta,
                                                   int64_t batch, int d,
                                                   const double *__restrict__ src,
                                                   double *__restrict__ dst)
{
    for (int64_t i = blockIdx.y; i < batch; i += gridDim.y) {
        const int64_t n = (src_meta[i].N + 1) * d;
        const double *a = src + src_meta[i].f_off * d;
        double *b = dst + dst_meta[i].row_off * d;
        for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n;
             e += (int64_t)gridDim.x * 256)
            b[e] = a[e];
    }
}

hipError_t launch_copy_rows(const InstMeta *src_meta, const InstMeta *dst_meta, int64_t batch,
                            int64_t max_rows, int d, const double *src, double *dst,
                            hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>((max_rows * d + 255) / 256, 1024);
    hipLaunchKernelGGL(k_copy_rows,
                       dim3((unsigned)std::max<int64_t>(blocks, 1),
                            (unsigned)std::min<int64_t>(batch, 65535)),
                       dim3(256), 0, s, src_meta, dst_meta, batch, d, src, dst);
    return hipGetLastError();
}

}  // namespace fabm
