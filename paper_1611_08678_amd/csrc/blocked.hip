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
#include <type_traits>

#include "fabm_blocked.h"
#include "fabm_device.h"
#include "fabm_launch.h"
#include "fabm_timer.h"

namespace fabm {

namespace {

constexpr int kBlk = 256;  // rows per block (= band threads)
constexpr int kTile = 16;  // polyphase factor = MFMA edge

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));


}  // namespace

// ---------------------------------------------------------------------------
// Band: block J walked row by row by wavefronts 0..3 of workgroup 0.
//
// Wavefront w holds, one per lane, the sums of rows 64 w + l of block J and
// of block J+1, and forms rows 64 w .. 64 w + 63 itself. At row t every lane
// adds f_{t-1} to its own sums, so lane t - 64 w holds row t's whole
// predictor and corrector sums; every lane evaluates the predictor and
// corrector on its own sums and f_t is read out of lane t - 64 w (readlane)
// for the next row. Nothing else is on that chain: rows are published in LDS
// (f_t, y_t, and a row counter every 8 rows, each group checked for
// non-finite values one group late), the other wavefronts add them to their
// sums as they appear, the contributions of a wavefront's own rows to block
// J+1 are added after its turn, and the last wavefront's next-block sums are
// finished by wavefront 0. Every target's sums are accumulated in row order.
// The sums of block J+1 go to the next launch through `carry`.
// ---------------------------------------------------------------------------
constexpr int kBandWaves = 4;
constexpr int kPublishEvery = 8;           // rows between counter updates
constexpr int kBandRows = kBlk + kWave;    // row arrays of the walk: a spare row per lane
constexpr uint32_t kSpinLimit = 1u << 26;  // polls of the row counter before giving up

__device__ __forceinline__ double readlane_f64(double x, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Wait until at least `need` rows are published. Returns the published count,
// or -1 if the walk stopped (a non-finite row) or the wait gave up (then the
// block is marked with -2).
__device__ __forceinline__ int band_wait_rows(int *s_cnt, int *s_dead, int need)
{
    uint32_t spins = 0;
    for (;;) {
        const int c = __hip_atomic_load(s_cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (c > kBlk) return -1;
        if (c >= need) return c;
        if (++spins > kSpinLimit) {
            __hip_atomic_store(s_dead, -2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_store(s_cnt, kBlk + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            return -1;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// PC: non-commensurate orders, one weight table set and one h^a, Gamma(a+2)
// per component (component k's tables at k * 3 wlen from the instance's,
// its scalars in A.cmeta[k]).
template <int SYS, int D, bool YPOUT, bool PC = false>
__device__ __forceinline__ void band_block(const InstView &A, const InstMeta &mv, int J,
                                           char *smem)
{
    constexpr int NP = n_params_of_sys(SYS, D);
    constexpr int K = PC ? D : 1;     // weight tables held
    double *sb = (double *)smem;      // [K] b lags 0..511 (next block's sums)
    double *sa = sb + K * 2 * kBlk;   // [K] a lags 0..511
    double *sbh = sa + K * 2 * kBlk;  // [K] h^a b lags 0..255 (this block's sums)
    double *sah = sbh + K * kBlk;     // [K] h^a a lags 0..255
    // row arrays: 256 rows of this block and a spare row per lane; a row of
    // sFY is f then y (one contiguous store of 2D values per formed row)
    double *sFY = sah + K * kBlk;           // [320][2D] f and y of this block's rows
    double *sYP = sFY + kBandRows * 2 * D;  // [320][D] predictor values (YPOUT)
    // the last wavefront's next-block sums, handed to wavefront 0 ([2][D][64])
    double *sH = sYP + (YPOUT ? kBandRows * D : 0);
    double *sTh = sH + 2 * D * kWave;  // theta, for systems with many parameters
    int *s_cnt = (int *)(sTh + NP);  // rows of this block published so far (> 256: stop)
    int *s_dead = s_cnt + 1;         // first non-finite row (block-relative), -1, or -2
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const InstMeta m = mv;  // the instance's entry (a kernel argument on the single path)
    const int64_t N = m.N;
    const int64_t pitch = (int64_t)A.NB * kBlk;
    const double *wb = A.W, *wa = wb + m.wlen, *wc = wa + m.wlen;
    const int64_t cw = 3 * m.wlen;  // stride between the components' tables (PC)
    const int64_t t0 = (int64_t)J * kBlk;
    const int nrows = (int)((t0 + kBlk - 1 < N ? t0 + kBlk - 1 : N) - t0 + 1);
    constexpr int nthr = kBandWaves * kWave;
    double hav[K], ig2v[K];  // h^a and 1 / Gamma(a + 2) of each table set
#pragma unroll
    for (int k = 0; k < K; ++k) {
        hav[k] = PC ? A.cmeta[k].ha : m.ha;
        ig2v[k] = PC ? A.cmeta[k].ig2 : m.ig2;
    }

    // rows go to Y and YP at row t - yrow0 (0 except in a recompute ring)
    const int64_t ro = (t0 - A.yrow0) * D;
    // a non-finite state in an earlier block ends the trajectory (tested
    // after the loads below are issued, which read only valid memory)
    const uint32_t dead_ld = *A.dead;
    // theta in registers when short; a linear system's matrix is read from LDS
    constexpr bool kThLds = NP > 12;
    double thr[kThLds || NP == 0 ? 1 : NP], y0[D];
    if constexpr (!kThLds) {
#pragma unroll
        for (int k = 0; k < NP; ++k) thr[k] = A.params[k];
    } else {
        for (int k = tid; k < NP; k += nthr) sTh[k] = A.params[k];
    }
    // teacher forcing: "theta" is the given history itself
    const double *th = SYS == SYS_TEACHER ? A.params : kThLds ? sTh : thr;
#pragma unroll
    for (int i = 0; i < D; ++i) y0[i] = A.y0[i];
    // the weight tables' entries of this thread (lags tid and tid + kBlk),
    // loaded with the rest of the prologue's reads and stored to LDS after
    // them, so the prologue waits for memory once
    static_assert(nthr == kBlk, "one thread per lag of the staged tables");
    double wst[K][4];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        wst[k][0] = wb[k * cw + tid];
        wst[k][1] = wb[k * cw + tid + kBlk];
        wst[k][2] = wa[k * cw + tid];
        wst[k][3] = wa[k * cw + tid + kBlk];
    }
    // The reads of a later block's sums, issued here for every block (each
    // address lies inside its array for any J; block 0 does not use them):
    // f_0, the carried sums, the near and far sums and the c - a weights.
    const int row = 64 * wave + lane;
    const int64_t T = t0 + row;
    double f0ld[D], cinP[D], cinC[D], accP[D], accC[D], wcT[D], waT[D];
    {
        const double *cin = A.carry + (int64_t)(J & 1) * 2 * D * kBlk;
        // near + far sums, stored in MFMA result order: row 16 rho + sigma
        // is element sigma/4 of lane 16 (sigma % 4) + rho
        const int rho = row >> 4, sig = row & 15;
        const int e = (sig >> 2) * kWave + 16 * (sig & 3) + rho;
        const double *aj = A.acc + (int64_t)J * 2 * D * kBlk;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int64_t o = PC ? i * cw : 0;
            f0ld[i] = A.Fc[i * pitch];
            cinP[i] = cin[i * kBlk + row];
            cinC[i] = cin[(D + i) * kBlk + row];
            accP[i] = aj[i * kBlk + e];
            accC[i] = aj[(D + i) * kBlk + e];
            wcT[i] = wc[o + T - 1];
            waT[i] = wa[o + T - 1];
        }
    }
    // f_0 (block 0 forms row 0 here; later blocks need it for the c - a fix)
    double f0[D];
    if (J == 0) {
        rhs<SYS, D>(0.0, y0, f0, A.params);
    } else {
#pragma unroll
        for (int i = 0; i < D; ++i) f0[i] = f0ld[i];
    }
    if (tid == 0) {
        *s_cnt = J == 0 ? 1 : 0;
        *s_dead = -1;
        if (J == 0) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                sFY[i] = f0[i];
                sFY[D + i] = y0[i];
                if constexpr (YPOUT) sYP[i] = y0[i];
            }
        }
    }
    // Sums of target row `row`: of this block in the form y0 + h^a P and
    // y0 + h^a C (what the predictor and corrector add the newest term to;
    // for orders above one y0 + t_T y'(0) in place of y0), of the next block
    // as plain P and C (handed over through `carry`).
    double base[D];
    {
        double y1[D];
        if constexpr (PC) {  // y'(0) enters the components whose own order exceeds one
#pragma unroll
            for (int i = 0; i < D; ++i)
                y1[i] = (A.y1 != nullptr && A.cmeta[i].alpha > 1.0) ? A.y1[i] : 0.0;
        } else {
            load_slope<D>(m, A.y1, y1);
        }
        taylor_base<D>((double)T * m.h, y0, y1, base);
    }
    double pc[D], cc[D], pn[D], cn[D];
    if (J == 0) {
        // source row 0 takes b_{T-1} and c_{T-1}
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int64_t o = PC ? i * cw : 0;
            pc[i] = fma(hav[PC ? i : 0], T >= 1 ? wb[o + T - 1] * f0[i] : 0.0, base[i]);
            cc[i] = fma(hav[PC ? i : 0], T >= 1 ? wc[o + T - 1] * f0[i] : 0.0, base[i]);
            pn[i] = wb[o + kBlk + row - 1] * f0[i];
            cn[i] = wc[o + kBlk + row - 1] * f0[i];
        }
    } else {
        double P[D], Cs[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            P[i] = cinP[i];
            Cs[i] = cinC[i];
            pn[i] = cn[i] = 0.0;
        }
        if (J >= 2) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double dca = wcT[i] - waT[i];
                P[i] += accP[i];
                // source row 0 takes c_{T-1} where the tiles used a_{T-1}
                Cs[i] = fma(dca, f0[i], Cs[i] + accC[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            pc[i] = fma(hav[PC ? i : 0], P[i], base[i]);
            cc[i] = fma(hav[PC ? i : 0], Cs[i], base[i]);
        }
    }
    const uint32_t dead_in = __builtin_amdgcn_readfirstlane(dead_ld);
    if (dead_in != 0u) {
        for (int e = tid; e < nrows * D; e += nthr) {
            if (A.Y) A.Y[ro + e] = __builtin_nan("");
            if constexpr (YPOUT) A.YP[ro + e] = __builtin_nan("");
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        sb[k * 2 * kBlk + tid] = wst[k][0];
        sb[k * 2 * kBlk + tid + kBlk] = wst[k][1];
        sa[k * 2 * kBlk + tid] = wst[k][2];
        sa[k * 2 * kBlk + tid + kBlk] = wst[k][3];
        sbh[k * kBlk + tid] = hav[k] * wst[k][0];
        sah[k * kBlk + tid] = hav[k] * wst[k][2];
    }
    __syncthreads();

    // rows this wavefront forms: [lo, hi)
    const int lo = 64 * wave < nrows ? 64 * wave : nrows;
    const int hi = 64 * wave + 64 < nrows ? 64 * wave + 64 : nrows;
    int done = J == 0 ? 1 : 0;  // rows already in this wavefront's sums
    bool go = true;
    // Published rows [r, r + R) into this lane's sums, in row order; the
    // weights and f values of the R rows are loaded before the first FMA.
    // Mode Both: this block's and the next block's sums (rows before the
    // lane's own); Next: the next block's only; NextH: the next block's and
    // the sums handed over by the last wavefront (target row 192 + lane).
    constexpr int kLast = kBandWaves - 1;
    double pnh[D], cnh[D];
    auto add_rows = [&](const int r, auto nrow, auto mode) __attribute__((always_inline)) {
        constexpr int R = decltype(nrow)::value;
        constexpr int M = decltype(mode)::value;
        double wbn[R][K], wan[R][K], wbh[R][K], wah[R][K], fr[R][D];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int lag = row - r - q - 1;  // >= 0 for rows before the lane's own
            const int lagh = kWave * kLast + lane - r - q - 1;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                wbn[q][k] = sb[k * 2 * kBlk + kBlk + lag];
                wan[q][k] = sa[k * 2 * kBlk + kBlk + lag];
                if constexpr (M == 0) {
                    wbh[q][k] = sbh[k * kBlk + lag];
                    wah[q][k] = sah[k * kBlk + lag];
                } else if constexpr (M == 2) {
                    wbh[q][k] = sb[k * 2 * kBlk + kBlk + lagh];
                    wah[q][k] = sa[k * 2 * kBlk + kBlk + lagh];
                }
            }
#pragma unroll
            for (int i = 0; i < D; ++i) fr[q][i] = sFY[(r + q) * 2 * D + i];
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const int k = PC ? i : 0;
                if constexpr (M == 0) {
                    pc[i] = fma(wbh[q][k], fr[q][i], pc[i]);
                    cc[i] = fma(wah[q][k], fr[q][i], cc[i]);
                } else if constexpr (M == 2) {
                    pnh[i] = fma(wbh[q][k], fr[q][i], pnh[i]);
                    cnh[i] = fma(wah[q][k], fr[q][i], cnh[i]);
                }
                pn[i] = fma(wbn[q][k], fr[q][i], pn[i]);
                cn[i] = fma(wan[q][k], fr[q][i], cn[i]);
            }
        }
    };
    // rows per batch: four with one table set and d <= 3, else fewer (registers)
    constexpr int kCatch = K > 1 ? 1 : (D <= 3 ? 4 : 2);
    using One = std::integral_constant<int, 1>;
    using Many = std::integral_constant<int, kCatch>;
    using Both = std::integral_constant<int, 0>;
    using Next = std::integral_constant<int, 1>;
    using NextH = std::integral_constant<int, 2>;
    // In a full block the last wavefront's next-block sums (over the rows
    // before its own) go to wavefront 0 when its walk starts; wavefront 0 adds
    // the last wavefront's rows to them as they are published, in row order,
    // and stores them, so the last wavefront ends with its walk.
    const bool handoff = nrows == kBlk;
    // rows in groups of kPublishEvery (aligned to the block), unrolled, so the
    // publish check runs once per group. The weights of row t (lag row - t
    // for the term f_{t-1}) come from LDS: with one table set, slot k of a
    // ring of kPublishEvery holds rows t = k mod kPublishEvery and is reloaded
    // for row t + kPublishEvery right after row t uses it, so the walk never
    // waits for them; with one set per component (more registers) each row's
    // are loaded during the row before (also for systems whose parameters
    // are read from LDS, which hold more registers).
    constexpr int kRing = K == 1 && !kThLds ? kPublishEvery : 1;
    double bwg[kRing][K], awg[kRing][K];
    auto load_row = [&](const int t, const int sl) __attribute__((always_inline)) {
        // lanes whose row is formed (row < t) read below the table, inside
        // the tables staged before it (lag >= -(kBlk + kPublishEvery)); their
        // sums are not used again
        const int lag = row - t;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            bwg[sl][q] = sbh[q * kBlk + lag];
            awg[sl][q] = sah[q * kBlk + lag];
        }
    };
    auto load_group = [&](const int g) __attribute__((always_inline)) {
        if constexpr (kRing > 1) {
#pragma unroll
            for (int k = 0; k < kRing; ++k) load_row(g + k, k);
        }
    };
    // the first group's weights load while the rows before it are added
    // (the walk starts at row lo, or at row 1 in block 0, both in group lo);
    // systems with many parameters in registers load them after (registers)
    constexpr bool kHoist = kRing > 1 && NP <= 4;
    if constexpr (kHoist) load_group(lo);
    // rows formed by earlier wavefronts: both blocks' sums
    while (go && done < lo) {
        const int c = __builtin_amdgcn_readfirstlane(band_wait_rows(s_cnt, s_dead, done + 1));
        if (c < 0) {
            go = false;
            break;
        }
        const int upto = c < lo ? c : lo;
        for (; done + kCatch <= upto; done += kCatch) add_rows(done, Many{}, Both{});
        for (; done < upto; ++done) add_rows(done, One{}, Both{});
    }
    if (handoff && go && wave == kLast) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            sH[i * kWave + lane] = pn[i];
            sH[(D + i) * kWave + lane] = cn[i];
        }
    }
    // This wavefront's rows. At row t every lane adds f_{t-1} (held in
    // scalar registers) to its own sums; lane t - lo's weights are then
    // h^a b_0 and h^a a_0, so it holds row t's whole predictor sum
    // y0 + h^a P_t and corrector sum. Every lane evaluates
    //   yP_t = y0 + h^a P_t,  y_t = (y0 + h^a C_t) + (h^a / Gamma(a+2)) f(t, yP_t)
    // on its own sums (only lane t - lo's are row t's), and f_t is read out of
    // lane t - lo (readlane) for the next row: one broadcast of d values per
    // row. Rows are checked for non-finite values when they are published.
    const int first = done;
    double hig2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        // teacher forcing returns the plain sums: y_t = C_t, yP_t = P_t
        hig2[k] = SYS == SYS_TEACHER ? 0.0 : hav[k] * ig2v[k];
    }
    double fprev[D];  // f of the row before (its terms are not in the sums yet)
#pragma unroll
    for (int i = 0; i < D; ++i) fprev[i] = 0.0;
    // lanes whose row is already formed store their (meaningless) values to
    // a spare row of their own, lanes of later rows to their row, which the
    // walk overwrites when it gets there
    const int row_off = row * D, spare_off = (kBlk + lane) * D;
    double *const fy_row = sFY + 2 * row_off, *const fy_spare = sFY + 2 * spare_off;
    int checked = first;  // check values of rows before this one are loaded
    // Rows are published in groups, each one group late: the f and y values
    // of a group are loaded from LDS after it is formed and tested after the
    // next group, so the walk never waits for them; a non-finite value stops
    // the walk there (the rows formed after it are never published).
    int pend_lo = first, pend_hi = first;  // rows of the loaded check values
    double chk = 0.0;
    auto settle = [&]() __attribute__((always_inline)) -> bool {
        if (pend_hi <= pend_lo) return true;
        const uint64_t mask = __ballot(!isfinite(chk));
        if (mask) {
            if (lane == 0) {
                *s_dead = pend_lo + __builtin_ctzll(mask) / (2 * D);
                __hip_atomic_store(s_cnt, kBlk + 1, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            return false;
        }
        // The rows' LDS stores were issued before this one and a wavefront's
        // LDS operations are performed in issue order, so a plain store of
        // the counter (kept after them by a compiler barrier) publishes them
        // without waiting for the LDS queue to drain.
        __asm__ __volatile__("" ::: "memory");
        if (lane == 0)
            __hip_atomic_store(s_cnt, pend_hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        pend_lo = pend_hi;
        return true;
    };
    // one row of the walk (k: its place in the group); full groups of
    // kPublishEvery rows run without the per-row range check
    auto step_row = [&](const int t, const int k) __attribute__((always_inline)) {
        const double tt = (double)(t0 + t) * m.h;
        double fp[D], y[D], f[D];
        const int sl = kRing > 1 ? k : 0;
        // f_{t-1} into the sums: lane t - lo then holds row t's whole
        // predictor and corrector sums (lag-0 weights h^a b_0, h^a a_0)
#pragma unroll
        for (int i = 0; i < D; ++i) {
            pc[i] = fma(bwg[sl][PC ? i : 0], fprev[i], pc[i]);
            cc[i] = fma(awg[sl][PC ? i : 0], fprev[i], cc[i]);
        }
        // the slot's weights for the row a group later (one table set), or
        // for the next row
        load_row(kRing > 1 ? t + kPublishEvery : t + 1, sl);
        rhs<SYS, D>(tt, pc, fp, th);
#pragma unroll
        for (int i = 0; i < D; ++i) y[i] = fma(hig2[PC ? i : 0], fp[i], cc[i]);
        rhs<SYS, D>(tt, y, f, th);
#pragma unroll
        for (int i = 0; i < D; ++i) fprev[i] = readlane_f64(f[i], t - lo);
        const bool own = row >= t;
        double *const fy = own ? fy_row : fy_spare;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            fy[i] = f[i];
            fy[D + i] = y[i];
            if constexpr (YPOUT) sYP[(own ? row_off : spare_off) + i] = pc[i];
        }
    };
    if constexpr (kRing == 1)
        load_row(first, 0);
    else if constexpr (!kHoist)
        load_group(lo);
    // end of a group of rows [., tl): the group before is checked (its
    // values were loaded a group ago) and published, and this group's f and
    // y values (one per lane) are loaded for the check after the next group
    auto end_group = [&](const int tl) __attribute__((always_inline)) -> bool {
        if (!settle()) return false;
        __builtin_amdgcn_wave_barrier();
        const int nv = (tl - checked) * 2 * D;
        chk = 0.0;
        if (lane < nv) {
            const int r = checked + lane / (2 * D), kk = lane % (2 * D);
            chk = sFY[r * 2 * D + kk];
        }
        pend_lo = checked;
        pend_hi = tl;
        checked = tl;
        done = tl;
        return true;
    };
    // a group with rows outside [first, hi) (block 0's first row, a ragged
    // last block): each row's range checked
    auto partial_group = [&](const int g0) __attribute__((always_inline)) -> bool {
#pragma unroll
        for (int k = 0; k < kPublishEvery; ++k) {
            const int t = g0 + k;
            if (t >= first && t < hi)
                step_row(t, k);
            else if constexpr (kRing > 1)
                load_row(t + kPublishEvery, k);  // keep the slot a group ahead
        }
        return end_group(g0 + kPublishEvery < hi ? g0 + kPublishEvery : hi);
    };
    int g0 = first & ~(kPublishEvery - 1);
    if (go && g0 < hi && (g0 < first || g0 + kPublishEvery > hi)) {
        go = partial_group(g0);
        g0 += kPublishEvery;
    }
    for (; go && g0 + kPublishEvery <= hi; g0 += kPublishEvery) {
#pragma unroll
        for (int k = 0; k < kPublishEvery; ++k) step_row(g0 + k, k);
        go = end_group(g0 + kPublishEvery);
    }
    if (go && g0 < hi) go = partial_group(g0);
    if (go && !settle()) go = false;
    if (go && !(handoff && wave == kLast)) {
        // own rows into block J+1, then rows formed by later wavefronts
        // (the next block's weights are at lag 256 + row - t - 1 >= 0)
        __builtin_amdgcn_wave_barrier();
        int t = first;
        for (; t + kCatch <= hi; t += kCatch) add_rows(t, Many{}, Next{});
        for (; t < hi; ++t) add_rows(t, One{}, Next{});
        const bool take = handoff && wave == 0;  // uniform
        bool have = false;
        while (done < nrows) {
            const int c = __builtin_amdgcn_readfirstlane(band_wait_rows(s_cnt, s_dead, done + 1));
            if (c < 0) break;
            const int cut = take && c > kWave * kLast ? kWave * kLast : c;
            for (; done + kCatch <= cut; done += kCatch) add_rows(done, Many{}, Next{});
            for (; done < cut; ++done) add_rows(done, One{}, Next{});
            if (done < c) {  // the last wavefront's rows (wavefront 0 of a full block)
                if (!have) {
                    // written before the last wavefront published any row
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        pnh[i] = sH[i * kWave + lane];
                        cnh[i] = sH[(D + i) * kWave + lane];
                    }
                    have = true;
                }
                for (; done + kCatch <= c; done += kCatch) add_rows(done, Many{}, NextH{});
                for (; done < c; ++done) add_rows(done, One{}, NextH{});
            }
        }
    }
    __syncthreads();
    // rows of this block: final ones from LDS, NaN from the first non-finite on
    const int dead = *s_dead;
    const int valid = dead == -1 ? nrows : (dead < 0 ? 0 : dead);
    if (A.Y) {
        for (int e = tid; e < nrows * D; e += nthr)
            A.Y[ro + e] = e / D < valid ? sFY[(e / D) * 2 * D + D + e % D] : __builtin_nan("");
    }
    if constexpr (YPOUT) {
        for (int e = tid; e < nrows * D; e += nthr)
            A.YP[ro + e] = e / D < valid ? sYP[e] : __builtin_nan("");
    }
    // a recomputation leaves the history and the next block's sums alone
    // (they already hold these values)
    if (A.recompute) return;
    for (int e = tid; e < valid; e += nthr) {
#pragma unroll
        for (int i = 0; i < D; ++i) A.Fc[i * pitch + t0 + e] = sFY[e * 2 * D + i];
    }
    if (dead == -1) {
        double *cout = A.carry + (int64_t)((J + 1) & 1) * 2 * D * kBlk;
        if (!(handoff && wave == kLast)) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                cout[i * kBlk + row] = pn[i];
                cout[(D + i) * kBlk + row] = cn[i];
            }
        }
        if (handoff && wave == 0) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                cout[i * kBlk + kWave * kLast + lane] = pnh[i];
                cout[(D + i) * kBlk + kWave * kLast + lane] = cnh[i];
            }
        }
    } else if (tid == 0) {
        *A.dead = dead == -2 ? kDeadWatchdog : (uint32_t)(t0 + dead);
    }
}

// ---------------------------------------------------------------------------
// MFMA windows. Launch s reads only the history of source columns
// 16 s - 15 .. 16 s + 15 (blocks s - 1 and s), for every target. Each
// workgroup stages those 31 columns in LDS (zero for negative rows), with a
// pitch of 17 doubles per column so that the 16 lanes of a K-slot read 16
// distinct even bank pairs.
// ---------------------------------------------------------------------------
constexpr int kSrcCols = 31;
// Columns staged for the windows of NP consecutive source blocks s - NP + 1 ..
// s (blocks s - NP .. s): 31 for one block, 47 for two, 79 for four.
template <int NP>
constexpr int group_cols() { return kTile * (NP + 1) - 1; }
constexpr int kColPitch = 17;
// Result layout of v_mfma_f32_16x16x4f32 (measured on gfx950 with one-hot
// operands): element v of lane l is row 4 (l / 16) + v, column l % 16 -- not
// the binary64 instruction's row 4 v + l / 16.
constexpr bool kF32RowMajorLanes = true;

template <int D, typename T = double>
constexpr size_t staged_bytes()
{
    return sizeof(T) * D * kSrcCols * kColPitch;
}

// NC = kSrcCols: columns 16 s - 15 .. 16 s + 15; NC = group_cols<NP>(): the
// 16 (NP - 1) columns before those as well (the windows of source blocks
// s - NP + 1 .. s - 1 too). Rows below
// `lo` are staged as zero.
template <int D, typename T, int NC = kSrcCols>
__device__ __forceinline__ void stage_sources(const InstView &A, int s, T *sB, int64_t lo = 0)
{
    const int64_t pitch = (int64_t)A.NB * kBlk;
    const int64_t r0 = (int64_t)kBlk * s - kTile * (NC - kTile);  // row of staged column 0
    for (int e = threadIdx.x; e < D * NC * kTile; e += blockDim.x) {
        const int i = e / (NC * kTile), rem = e - i * (NC * kTile);
        const int c = rem / kTile, tau = rem - c * kTile;
        const int64_t row = r0 + kTile * c + tau;
        sB[(i * NC + c) * kColPitch + tau] = row >= lo ? (T)A.Fc[i * pitch + row] : (T)0;
    }
}

// Far and near sums are stored through to memory (agent-scope stores): no
// workgroup of the same launch reads them again, and the launch that does
// may run on another XCD, so lines left dirty in this XCD's L2 would only be
// written back when the launch ends, lengthening it.
__device__ __forceinline__ void store_through(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One column lag q = 16 m + u of a target block, for both weight tables and
// all components, added into `acc` (one wavefront). The history column of
// lane rho is staged column rho - u + coff; columns past the staged range
// (coff > 15 only) belong to blocks not yet formed and are masked to zero.
// PC: each component has its own weight tables, cw doubles apart, so each
// takes its own A operand.
template <int D, int NC = kSrcCols, bool PC = false>
__device__ __forceinline__ void window_lag(dbl4 (&acc)[2][D], const double *__restrict__ wb,
                                           const double *__restrict__ wa, const double *sB,
                                           int64_t m, int u, int coff, int64_t cw = 0)
{
    constexpr int K = PC ? D : 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int r16 = lane & 15, kq = lane >> 4;  // A row sigma / B column rho; K slot
    const int c = r16 - u + coff;
    const bool ok = c < NC;
    // K slot kq of slice j is source row tau = 4 kq + j of the column, so a
    // lane's operands of the four slices are four consecutive weights and
    // four consecutive staged values (wide loads)
    const int sbase = (ok ? c : 0) * kColPitch + 4 * kq;
    const int64_t wi = kBlk * m + kTile * u + r16 - 4 * kq - 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double ab[K], aa[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            ab[k] = wb[k * cw + wi - j];
            aa[k] = wa[k * cw + wi - j];
        }
        double bf[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double v = sB[i * NC * kColPitch + sbase + j];
            bf[i] = ok ? v : 0.0;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            acc[0][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ab[PC ? i : 0], bf[i], acc[0][i], 0,
                                                             0, 0);
            acc[1][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[PC ? i : 0], bf[i], acc[1][i], 0,
                                                             0, 0);
        }
    }
}

// window_lag for one weight table `w` (b or a): the same products, in the
// same order, into that table's accumulators only.
template <int D, bool PC = false>
__device__ __forceinline__ void window_lag_table(dbl4 (&acc)[D], const double *__restrict__ w,
                                                 const double *sB, int64_t m, int u,
                                                 int64_t cw = 0)
{
    constexpr int K = PC ? D : 1;
    constexpr int NC = kSrcCols;
    const int lane = threadIdx.x & (kWave - 1);
    const int r16 = lane & 15, kq = lane >> 4;
    const int sbase = (r16 - u + kTile - 1) * kColPitch + 4 * kq;
    const int64_t wi = kBlk * m + kTile * u + r16 - 4 * kq - 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double a[K];
#pragma unroll
        for (int k = 0; k < K; ++k) a[k] = w[k * cw + wi - j];
        double bf[D];
#pragma unroll
        for (int i = 0; i < D; ++i) bf[i] = sB[i * NC * kColPitch + sbase + j];
#pragma unroll
        for (int i = 0; i < D; ++i)
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[PC ? i : 0], bf[i], acc[i], 0, 0, 0);
    }
}

template <int D, bool PC = false>
__device__ __forceinline__ void window_lag_table_f32(flt4 (&acc)[D], const float *__restrict__ w,
                                                     const float *sB, int64_t m, int u,
                                                     int64_t cw = 0)
{
    constexpr int K = PC ? D : 1;
    constexpr int NC = kSrcCols;
    const int lane = threadIdx.x & (kWave - 1);
    const int r16 = lane & 15, kq = lane >> 4;
    const int sbase = (r16 - u + kTile - 1) * kColPitch + 4 * kq;
    const int64_t wi = kBlk * m + kTile * u + r16 - 4 * kq - 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float a[K];
#pragma unroll
        for (int k = 0; k < K; ++k) a[k] = w[k * cw + wi - j];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float bf = sB[i * NC * kColPitch + sbase + j];
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[PC ? i : 0], bf, acc[i], 0, 0, 0);
        }
    }
}

// The same column lag on the binary32 matrix cores (v_mfma_f32_16x16x4f32):
// weights and history rounded to binary32, products summed in binary32.
template <int D, int NC = kSrcCols, bool PC = false>
__device__ __forceinline__ void window_lag_f32(flt4 (&acc)[2][D], const float *__restrict__ wb,
                                               const float *__restrict__ wa, const float *sB,
                                               int64_t m, int u, int coff = kTile - 1,
                                               int64_t cw = 0)
{
    constexpr int K = PC ? D : 1;  // one A operand per component with per-component orders
    const int lane = threadIdx.x & (kWave - 1);
    const int r16 = lane & 15, kq = lane >> 4;
    // K slot kq of slice j is source row 4 kq + j (see window_lag)
    const int sbase = (r16 - u + coff) * kColPitch + 4 * kq;
    const int64_t wi = kBlk * m + kTile * u + r16 - 4 * kq - 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float ab[K], aa[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            ab[k] = wb[k * cw + wi - j];
            aa[k] = wa[k * cw + wi - j];
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float bf = sB[i * NC * kColPitch + sbase + j];
            acc[0][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(ab[PC ? i : 0], bf, acc[0][i], 0, 0, 0);
            acc[1][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(aa[PC ? i : 0], bf, acc[1][i], 0, 0, 0);
        }
    }
}

// Row of the 16x16 result held in element v of lane l by the binary32 16x16x4
// instruction (measured on gfx950 with one-hot operands).
__device__ __forceinline__ int f32_result_row(int l, int v) { return kF32RowMajorLanes ? 4 * (l >> 4) + v : 4 * v + (l >> 4); }

// Far windows of target block J in binary32, from the NP source blocks
// s - NP + 1 .. s (source s - NP + 1 + p in staged columns from 16 p): each
// window's sums are formed in binary32 and added, in source order, to the
// binary64 sums of the target. `first`: no earlier window has written them.
template <int D, int NP = 1, bool PC = false>
__device__ __forceinline__ void far_target_f32(const InstView &A, int s, int J, const float *sB,
                                               bool first)
{
    constexpr int NC = NP == 1 ? kSrcCols : group_cols<NP>();
    const InstMeta m = A.meta[0];
    const float *wb = A.W32, *wa = wb + m.wlen;
    const int64_t cw = 2 * m.wlen;  // binary32 b, a of the next component (PC)
    const int lane = threadIdx.x & (kWave - 1);
    double *aj = A.acc + (int64_t)J * 2 * D * kBlk;
    // binary64 sums keep the binary64 result order (element sigma/4 of lane
    // 16 (sigma % 4) + rho)
    int e[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int sig = f32_result_row(lane, v), rho = lane & 15;
        e[v] = (sig >> 2) * kWave + 16 * (sig & 3) + rho;
    }
    double x[2][D][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) x[t][i][v] = first ? 0.0 : aj[(t * D + i) * kBlk + e[v]];
#pragma unroll 1
    for (int p = 0; p < NP; ++p) {
        flt4 acc[2][D];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int i = 0; i < D; ++i) acc[t][i] = (flt4){0.0f, 0.0f, 0.0f, 0.0f};
        const int64_t mm = J - (s - NP + 1 + p);
#pragma unroll 2
        for (int u = 0; u < kTile; ++u)
            window_lag_f32<D, NC, PC>(acc, wb, wa, sB, mm, u, kTile * (p + 1) - 1, cw);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) x[t][i][v] += (double)acc[t][i][v];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) store_through(&aj[(t * D + i) * kBlk + e[v]], x[t][i][v]);
}

// Far windows of target block J from the NP source blocks s - NP + 1 .. s
// (one wavefront; source s - NP + 1 + p in staged columns rho - u + 16 p + 15),
// added to the target's sums in place, in source order.
template <int D, int NP = 1, bool PC = false>
__device__ __forceinline__ void far_target(const InstView &A, int s, int J, const double *sB,
                                           bool first)
{
    constexpr int NC = NP == 1 ? kSrcCols : group_cols<NP>();
    const InstMeta m = A.meta[0];
    const double *wb = A.W, *wa = wb + m.wlen;
    const int64_t cw = 3 * m.wlen;
    const int lane = threadIdx.x & (kWave - 1);
    double *aj = A.acc + (int64_t)J * 2 * D * kBlk + lane;
    dbl4 acc[2][D];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[t][i][v] = first ? 0.0 : aj[((t * D + i) * 4 + v) * kWave];
#pragma unroll 1
    for (int p = 0; p < NP; ++p) {
        // oldest source block first: the order of the one-window launches
        const int64_t mm = J - (s - NP + 1 + p);
#pragma unroll 2
        for (int u = 0; u < kTile; ++u)
            window_lag<D, NC, PC>(acc, wb, wa, sB, mm, u, kTile * (p + 1) - 1, cw);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) store_through(&aj[((t * D + i) * 4 + v) * kWave], acc[t][i][v]);
}

// Far window of target block J from source block s for one weight table
// (tb 0: b, the predictor sums; 1: a, the corrector sums): a work unit of
// half a target, so the far work of a launch splits over the wavefronts in
// finer pieces. Each table's sums take the same products in the same order
// as in far_target.
template <int D, bool PC = false>
__device__ __forceinline__ void far_target_table(const InstView &A, int s, int J, int tb,
                                                 const double *sB, bool first)
{
    const InstMeta m = A.meta[0];
    const double *w = A.W + (tb ? m.wlen : 0);
    const int64_t cw = 3 * m.wlen;
    const int lane = threadIdx.x & (kWave - 1);
    double *aj = A.acc + (int64_t)J * 2 * D * kBlk + (int64_t)tb * D * kBlk + lane;
    dbl4 acc[D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[i][v] = first ? 0.0 : aj[(i * 4 + v) * kWave];
    const int64_t mm = J - s;
#pragma unroll 2
    for (int u = 0; u < kTile; ++u) window_lag_table<D, PC>(acc, w, sB, mm, u, cw);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) store_through(&aj[(i * 4 + v) * kWave], acc[i][v]);
}

template <int D, bool PC = false>
__device__ __forceinline__ void far_target_table_f32(const InstView &A, int s, int J, int tb,
                                                     const float *sB, bool first)
{
    const InstMeta m = A.meta[0];
    const float *w = A.W32 + (tb ? m.wlen : 0);
    const int64_t cw = 2 * m.wlen;
    const int lane = threadIdx.x & (kWave - 1);
    double *aj = A.acc + (int64_t)J * 2 * D * kBlk + (int64_t)tb * D * kBlk;
    int e[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int sig = f32_result_row(lane, v), rho = lane & 15;
        e[v] = (sig >> 2) * kWave + 16 * (sig & 3) + rho;
    }
    double x[D][4];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) x[i][v] = first ? 0.0 : aj[i * kBlk + e[v]];
    flt4 acc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i] = (flt4){0.0f, 0.0f, 0.0f, 0.0f};
    const int64_t mm = J - s;
#pragma unroll 2
    for (int u = 0; u < kTile; ++u) window_lag_table_f32<D, PC>(acc, w, sB, mm, u, cw);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) store_through(&aj[i * kBlk + e[v]], x[i][v] + (double)acc[i][v]);
}

// Near part of target block J = s + 2: column lags 17..47, i.e. window m = 2
// (all u, staged columns rho - u + 15) and window m = 1 for u = 1..15
// (staged columns rho - u + 31, masked past column 30), split over the first
// NW wavefronts. Their partial sums are added in wavefront order, either all
// at once from NW LDS slots (SEQ = false, red holds NW tiles) or one
// wavefront after another into a single slot (SEQ = true).
template <int D, int NW, bool SEQ, bool PC = false>
__device__ __forceinline__ void near_part(const InstView &A, int s, const double *sB,
                                          double *red)
{
    const InstMeta m = A.meta[0];
    const double *wb = A.W, *wa = wb + m.wlen;
    const int64_t cw = 3 * m.wlen;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid >> 6;
    const int J = s + 2;
    constexpr int kLags = 31;
    dbl4 acc[2][D];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < D; ++i) acc[t][i] = (dbl4){0.0, 0.0, 0.0, 0.0};
    const int p0 = kLags * w / NW, p1 = kLags * (w + 1) / NW;
    for (int p = p0; p < p1; ++p) {
        if (p < kTile)
            window_lag<D, kSrcCols, PC>(acc, wb, wa, sB, 2, p, kTile - 1, cw);
        else
            window_lag<D, kSrcCols, PC>(acc, wb, wa, sB, 1, p - (kTile - 1), 2 * kTile - 1, cw);
    }
    double *aj = A.acc + (int64_t)J * 2 * D * kBlk;
    if constexpr (!SEQ) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    red[((w * 2 * D + t * D + i) * 4 + v) * kWave + lane] = acc[t][i][v];
        __syncthreads();  // the near wavefronts
        for (int e = tid; e < 2 * D * kBlk; e += NW * kWave) {
            double v = s == 0 ? 0.0 : aj[e];
#pragma unroll
            for (int k = 0; k < NW; ++k) v += red[k * 2 * D * kBlk + e];
            store_through(&aj[e], v);
        }
    } else {
        for (int k = 0; k < NW; ++k) {
            if (w == k) {
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int i = 0; i < D; ++i)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            double *r = red + ((t * D + i) * 4 + v) * kWave + lane;
                            *r = k == 0 ? acc[t][i][v] : *r + acc[t][i][v];
                        }
            }
            __syncthreads();
        }
        for (int e = tid; e < 2 * D * kBlk; e += NW * kWave)
            store_through(&aj[e], (s == 0 ? 0.0 : aj[e]) + red[e]);
    }
}

__device__ __forceinline__ InstView single_view(const StepArgs &A)
{
    return InstView{A.meta, A.cmeta, A.params, A.y0, A.y1, A.Y, A.YP, A.W, A.W32, A.Fc,
                    A.carry, A.acc, A.dead, A.NB};
}

// Launch s of the single-trajectory pipeline; `wpw` wavefronts of each far
// workgroup take part (wavefront g of G handles work units g + k G: target
// s + 3 + u, or with `halves` weight table u % 2 of target s + 3 + u / 2,
// when there are more targets than far wavefronts). With
// the far history of larger distances in FFT squares, far targets end at block
// `jend` and the far windows take no source rows below `flo` (0 otherwise).
template <int SYS, int D, bool F32, bool PC = false>
__global__ __launch_bounds__(kStepThreads) void k_step(StepArgs A, int s, int wpw, int jend,
                                                       int64_t flo, int halves)
{
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x, wave = threadIdx.x >> 6;
    const InstView V = single_view(A);
    if (b == 0) {
        // teacher forcing writes the predictor sums as well
        if (wave < kBandWaves)
            band_block<SYS, D, SYS == SYS_TEACHER, PC>(V, A.m0, s + 1, smem);
        return;
    }
    if (*A.dead != 0u) return;  // the trajectory has ended; later rows are NaN
    if (b == 1 || !F32) {
        double *sB = (double *)smem;
        stage_sources<D, double>(V, s, sB, b == 1 ? 0 : flo);
        __syncthreads();
        if (b == 1) {
            if (wave < kNearWaves)
                near_part<D, kNearWaves, false, PC>(V, s, sB,
                                                    (double *)(smem + staged_bytes<D>()));
            return;
        }
        if (wave >= wpw) return;
        const int G = ((int)gridDim.x - 2) * wpw;
        if (halves) {
            const int nu = 2 * (jend - (s + 3));
            for (int k = (b - 2) * wpw + wave; k < nu; k += G)
                far_target_table<D, PC>(V, s, s + 3 + (k >> 1), k & 1, sB, s == 0);
        } else {
            for (int J = s + 3 + (b - 2) * wpw + wave; J < jend; J += G)
                far_target<D, 1, PC>(V, s, J, sB, s == 0);
        }
    } else {
        float *sB = (float *)smem;
        stage_sources<D, float>(V, s, sB, flo);
        __syncthreads();
        if (wave >= wpw) return;
        const int G = ((int)gridDim.x - 2) * wpw;
        if (halves) {
            const int nu = 2 * (jend - (s + 3));
            for (int k = (b - 2) * wpw + wave; k < nu; k += G)
                far_target_table_f32<D, PC>(V, s, s + 3 + (k >> 1), k & 1, sB, s == 0);
        } else {
            for (int J = s + 3 + (b - 2) * wpw + wave; J < jend; J += G)
                far_target_f32<D, 1, PC>(V, s, J, sB, s == 0);
        }
    }
}

// ---------------------------------------------------------------------------
// Batched pipeline (layout and schedule in fabm_blocked.h).
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ InstView batch_view(const BatchArgs &A, int i)
{
    const InstMeta *m = A.meta + i;
    const BlkInst &b = A.inst[i];
    return InstView{m,
                    A.cmeta ? A.cmeta + (int64_t)i * D : nullptr,
                    A.params + m->p_off,
                    A.y0 + (int64_t)i * D,
                    A.y1 ? A.y1 + (int64_t)i * D : nullptr,
                    A.Y ? A.Y + m->row_off * D : nullptr,
                    A.YP ? A.YP + m->row_off * D : nullptr,
                    A.W + m->w_off,
                    A.W32 ? A.W32 + m->w_off / 3 * 2 : nullptr,
                    A.Fc + b.fc_off,
                    A.carry + (int64_t)i * 2 * 2 * D * kBlk,
                    A.acc + b.acc_off,
                    A.dead + i,
                    b.NB};
}

template <int SYS, int D, bool F32, bool YPOUT, bool PC = false>
__global__ __launch_bounds__(kBatchThreads) void k_step_batch(BatchArgs A, int s, int nband,
                                                              int nnear, const int *far_off,
                                                              int nfar, int P)
{
    extern __shared__ __align__(16) char smem[];
    int q = blockIdx.x;
    if (q < nband) {
        const InstView V = batch_view<D>(A, A.order[q]);
        band_block<SYS, D, YPOUT, PC>(V, V.meta[0], s + 1, smem);
        return;
    }
    q -= nband;
    int inst, first = -1;
    if (q < nnear) {
        inst = A.order[q];
    } else {
        q -= nnear;
        // instance k of the far prefix with far_off[k] <= q < far_off[k + 1]
        int lo = 0, hi = nfar;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (far_off[mid] <= q) lo = mid;
            else hi = mid;
        }
        inst = A.order[lo];
        first = s + 3 + 4 * (q - far_off[lo]);
    }
    const InstView V = batch_view<D>(A, inst);
    if (*V.dead != 0u) return;  // this trajectory has ended; its later rows are NaN
    // Far windows in groups of P source blocks (P = 1, 2 or 4): a launch s with
    // (s + 1) % P == 0 adds the windows of sources s - P + 1 .. s to every
    // target J >= s + 3 with one read and write of its sums; the other
    // launches add source s only to the targets whose band comes before the
    // next such launch sb (J <= sb + 2). Every target gets every source block
    // in the same order as with one window per launch, so the results do not
    // depend on P.
    const bool big = P == 1 || ((s + 1) % P == 0 && s >= P - 1);
    const int sb = s + (P - 1 - s % P);
    const int J = first + (threadIdx.x >> 6);
    const bool mine = first >= 0 && J < V.NB && (big || J <= sb + 2);
    // the first write of a target's sums: launch 0, or the first group
    const bool fw = s == 0 || (big && s == P - 1);
    if (first < 0 || !F32) {
        double *sB = (double *)smem;
        if (first >= 0 && big && P == 4)
            stage_sources<D, double, group_cols<4>()>(V, s, sB);
        else if (first >= 0 && big && P == 2)
            stage_sources<D, double, group_cols<2>()>(V, s, sB);
        else
            stage_sources<D, double>(V, s, sB);
        __syncthreads();
        if (first < 0) {
            near_part<D, kBatchThreads / kWave, true, PC>(V, s, sB,
                                                          (double *)(smem + staged_bytes<D>()));
            return;
        }
        if (mine) {
            if (big && P == 4)
                far_target<D, 4, PC>(V, s, J, sB, fw);
            else if (big && P == 2)
                far_target<D, 2, PC>(V, s, J, sB, fw);
            else
                far_target<D, 1, PC>(V, s, J, sB, fw);
        }
    } else {
        float *sB = (float *)smem;
        if (big && P == 4)
            stage_sources<D, float, group_cols<4>()>(V, s, sB);
        else if (big && P == 2)
            stage_sources<D, float, group_cols<2>()>(V, s, sB);
        else
            stage_sources<D, float>(V, s, sB);
        __syncthreads();
        if (mine) {
            if (big && P == 4)
                far_target_f32<D, 4, PC>(V, s, J, sB, fw);
            else if (big && P == 2)
                far_target_f32<D, 2, PC>(V, s, J, sB, fw);
            else
                far_target_f32<D, 1, PC>(V, s, J, sB, fw);
        }
    }
}

// Forward block of the reverse pass's next group (layout in fabm_blocked.h).
// Reversed block J' covers forward rows (N - 256 J' - 256, N - 256 J'], i.e.
// forward blocks klo(J') = floor((N - 256 J' - 255) / 256) .. floor((N -
// 256 J') / 256) <= klo(J') + 1. The group of reverse launches J .. J + G - 1
// needs klo(J) - G + 1 .. klo(J) + 1; klo(J) + 1 (when needed) was formed for
// the group before, except for J = 0. Workgroup q forms block
// start - q % (G + 1) of instance order[q / (G + 1)], start = klo(J), or the
// highest block for J = 0.
__device__ __forceinline__ int64_t floor_div256(int64_t x) { return x >= 0 ? x / 256 : -((255 - x) / 256); }

template <int SYS, int D, bool PC = false>
__global__ __launch_bounds__(kBatchThreads) void k_recompute_batch(BatchArgs A, RecompArgs R,
                                                                   int J)
{
    extern __shared__ __align__(16) char smem[];
    const int G = R.G, slots = G + 1;
    const int q = blockIdx.x, inst = A.order[q / slots], j = q % slots;
    InstView V = batch_view<D>(A, inst);
    const InstMeta m = V.meta[0];
    const int64_t N = m.N;
    const int64_t klo = floor_div256(N - (int64_t)kBlk * J - (kBlk - 1));
    const int64_t khi = floor_div256(N - (int64_t)kBlk * J);
    const int64_t K = (J == 0 ? khi : klo) - j;
    if (K < 0 || K < klo - (G - 1) || K >= V.NB) return;
    if (*V.dead != 0u) return;  // the forward blew up: the gradients are NaN
    const int slot = (int)(K % slots);
    const int64_t rs = (int64_t)inst * slots + slot;
    double *cb = R.rcarry + rs * 2 * 2 * D * kBlk;
    const int row = threadIdx.x;
    if (K >= 1) {
        // band sums of block K from the rows of block K - 1, formed as the
        // forward band forms them: ascending rows, one fma per row (block 0
        // starts from its row 0 with c_{T-1} in the corrector)
        const int64_t pitch = (int64_t)V.NB * kBlk, tp = (K - 1) * kBlk;
        const double *wb = V.W, *wa = wb + m.wlen, *wc = wa + m.wlen;
        const int64_t cw = 3 * m.wlen;
        double *cin = cb + (K & 1) * 2 * D * kBlk;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int64_t o = PC ? i * cw : 0;
            const double *fi = V.Fc + i * pitch;
            double pn = 0.0, cn = 0.0;
            int t = 0;
            if (K == 1) {
                pn = wb[o + kBlk + row - 1] * fi[0];
                cn = wc[o + kBlk + row - 1] * fi[0];
                t = 1;
            }
            for (; t < kBlk; ++t) {
                const double f = fi[tp + t];
                pn = fma(wb[o + kBlk + row - t - 1], f, pn);
                cn = fma(wa[o + kBlk + row - t - 1], f, cn);
            }
            cin[i * kBlk + row] = pn;
            cin[(D + i) * kBlk + row] = cn;
        }
    }
    __syncthreads();
    V.Y = R.ringY + rs * kBlk * D;
    V.YP = R.ringYP + rs * kBlk * D;
    V.yrow0 = K * kBlk;
    V.carry = cb;
    V.recompute = 1;
    band_block<SYS, D, true, PC>(V, V.meta[0], (int)K, smem);
}

__global__ void k_batch_status(BatchArgs A)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < A.batch) {
        const uint32_t d = A.dead[i];
        A.status[i] = d == kDeadWatchdog ? -1 : (int64_t)d;
    }
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
// Band LDS: weight tables (one set, or one per component with per-component
// orders), f / y / predictor rows, theta, two counters.
static size_t band_smem_bytes(int d, bool pc)
{
    return sizeof(double) * (6 * kBlk * (size_t)(pc ? d : 1) + 3 * kBandRows * (size_t)d +
                             2 * kWave * (size_t)d + d * d + 2 * d) +
           16;
}

size_t step_smem_bytes(int d, bool pc)
{
    const size_t band = band_smem_bytes(d, pc);
    const size_t near = sizeof(double) * (kNearWaves * 2 * (size_t)d * kBlk +
                                          (size_t)d * kSrcCols * kColPitch);
    const size_t exclusive = 81 * 1024;
    return std::max(band, std::max(near, exclusive));
}

// Grid of launch s: band, near and far workgroups, the number of active
// wavefronts per far workgroup (one work unit each, four per round of
// SIMDs), and the work unit: a whole target, or (`halves`, when the targets
// outnumber the far wavefronts, so some wavefronts take several) a target's
// window for one weight table, which splits the far work more evenly.
// Launch shape of step s: band and near workgroups plus up to far_cap far
// workgroups of wpw wavefronts (the far loop strides over the targets, so any
// cap covers all of them).
void step_grid(int NB, int jend, int s, int *grid, int *wpw, int far_cap, int *halves)
{
    *grid = 1;
    *wpw = 0;
    *halves = 0;
    if (s < 0 || s + 2 > NB - 1) return;
    *grid = 2;
    int nt = std::min(jend, NB) - (s + 3);  // far targets
    if (nt <= 0) return;
    const int cap = std::max(1, std::min(far_cap > 0 ? far_cap : kMaxFarWg, kMaxFarWg));
    if (nt > cap * (kStepThreads / kWave)) {
        *halves = 1;
        nt *= 2;  // work units
    }
    const int per_round = 4 * cap;
    const int rounds = std::min((nt + per_round - 1) / per_round, kStepThreads / kWave / 4);
    *wpw = 4 * rounds;
    *grid += std::min(cap, (nt + *wpw - 1) / *wpw);
}

template <int SYS, int D, bool F32, bool PC>
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
    static std::atomic<uint64_t> attr_dev{0};
    const size_t smem = step_smem_bytes(D, PC);
    FABM_STEP_TRY("hipFuncSetAttribute(step LDS)",
                  ensure_lds_attr((const void *)k_step<SYS, D, F32, PC>, smem, attr_dev));
    const bool fft = A.fft_level > 0 && fft_far_top_level(A.NB, A.fft_level) >= 0;
    if (fft) {
        if (T) FABM_STEP_TRY("timer begin", T->begin(KC_FFT_FAR, st));
        FABM_STEP_TRY("FFT weight spectra", fft_far_prepare(D, A, st));
        if (T) FABM_STEP_TRY("timer end", T->end(st));
    }
    for (int s = -1; s <= A.NB - 2; ++s) {
        int grid, wpw;
        const int jend = fft ? fft_far_target_end(A.NB, A.fft_level, s) : A.NB;
        const int64_t flo = fft && fft_far_mask_prev(A.fft_level, s) ? (int64_t)kBlk * s : 0;
        int halves;
        step_grid(A.NB, jend, s, &grid, &wpw, A.far_cap, &halves);
        if (T) FABM_STEP_TRY("timer begin", T->begin(KC_BLOCKED_STEP, st));
        hipLaunchKernelGGL((k_step<SYS, D, F32, PC>), dim3(grid), dim3(kStepThreads), smem, st, A,
                           s, wpw, jend, flo, halves);
        FABM_STEP_TRY("launch k_step", hipGetLastError());
        if (T) FABM_STEP_TRY("timer end", T->end(st));
        if (fft && fft_far_square_at(A.NB, A.fft_level, s) >= 0) {
            // the square whose last source block this launch formed
            if (T) FABM_STEP_TRY("timer begin", T->begin(KC_FFT_FAR, st));
            FABM_STEP_TRY("FFT far square", fft_far_square(D, A, s, st));
            if (T) FABM_STEP_TRY("timer end", T->end(st));
        }
    }
    hipLaunchKernelGGL(k_step_status, dim3(1), dim3(kWave), 0, st, A);
    FABM_STEP_TRY("launch k_step_status", hipGetLastError());
    return hipSuccess;
#undef FABM_STEP_TRY
}

size_t batch_smem_bytes(int d, bool pc, int P)
{
    const size_t band = band_smem_bytes(d, pc);
    const size_t near = sizeof(double) * (2 * (size_t)d * kBlk + (size_t)d * kSrcCols * kColPitch);
    const int nc = P == 4 ? group_cols<4>() : P == 2 ? group_cols<2>() : kSrcCols;
    const size_t group = sizeof(double) * (size_t)d * nc * kColPitch;
    return std::max(std::max(band, near), group);
}

template <int SYS, int D, bool F32, bool YPOUT, bool PC>
static hipError_t enqueue_batch_t(const BatchArgs &A, const BatchSchedule &S, const int *far_off,
                                  hipStream_t st, KernelTimer *T, const char **where)
{
#define FABM_STEP_TRY(what, expr)          \
    do {                                   \
        const hipError_t e_ = (expr);      \
        if (e_ != hipSuccess) {            \
            *where = what;                 \
            return e_;                     \
        }                                  \
    } while (0)
    const size_t smem = batch_smem_bytes(D, PC, S.P);
    static std::atomic<uint64_t> attr_dev{0};
    if (smem > 64 * 1024)  // per-component tables, or wide groups of sources
        FABM_STEP_TRY("hipFuncSetAttribute(batch LDS)",
                      ensure_lds_attr((const void *)k_step_batch<SYS, D, F32, YPOUT, PC>,
                                      batch_smem_bytes(D, PC, 4), attr_dev));
    for (int s = -1; s <= S.max_NB - 2; ++s) {
        const size_t k = (size_t)(s + 1);
        const int nb = S.nband[k], nn = S.nnear[k], nf = S.nfar[k];
        const int nfw = S.far_off[(size_t)S.far_base[k] + (size_t)nf];
        const int grid = nb + nn + nfw;
        if (grid == 0) continue;
        if (T) FABM_STEP_TRY("timer begin", T->begin(KC_BLOCKED_STEP, st));
        hipLaunchKernelGGL((k_step_batch<SYS, D, F32, YPOUT, PC>), dim3(grid), dim3(kBatchThreads), smem,
                           st, A, s,
                           nb, nn, far_off + S.far_base[k], nf, S.P);
        FABM_STEP_TRY("launch k_step_batch", hipGetLastError());
        if (T) FABM_STEP_TRY("timer end", T->end(st));
    }
    hipLaunchKernelGGL(k_batch_status, dim3((unsigned)((A.batch + 255) / 256)), dim3(256), 0, st, A);
    FABM_STEP_TRY("launch k_batch_status", hipGetLastError());
    return hipSuccess;
#undef FABM_STEP_TRY
}

hipError_t enqueue_batch(int sys, int d, bool f32, const BatchArgs &A, const BatchSchedule &S,
                         const int *far_off, hipStream_t s, KernelTimer *T, const char **where)
{
    // predictor rows are written when A.YP is set (FP64 far windows only)
    // per-component orders (A.cmeta): FP64 or FP32 windows; predictor rows with FP64
#define FABM_BATCH_CASE(SS, DD)                                                                \
    if (sys == SS && d == DD)                                                                  \
        return A.cmeta ? (A.YP ? enqueue_batch_t<SS, DD, false, true, true>(A, S, far_off, s, T, where) \
                          : f32 ? enqueue_batch_t<SS, DD, true, false, true>(A, S, far_off, s, T, where) \
                               : enqueue_batch_t<SS, DD, false, false, true>(A, S, far_off, s, T, where)) \
               : A.YP  ? enqueue_batch_t<SS, DD, false, true, false>(A, S, far_off, s, T, where) \
               : f32   ? enqueue_batch_t<SS, DD, true, false, false>(A, S, far_off, s, T, where) \
                       : enqueue_batch_t<SS, DD, false, false, false>(A, S, far_off, s, T, where);
    FABM_BATCH_CASE(SYS_LINEAR, 1)
    FABM_BATCH_CASE(SYS_LINEAR, 2)
    FABM_BATCH_CASE(SYS_LINEAR, 3)
    FABM_BATCH_CASE(SYS_LINEAR, 4)
    FABM_BATCH_CASE(SYS_CHEN, 3)
    FABM_BATCH_CASE(SYS_ROSSLER, 3)
    FABM_BATCH_CASE(SYS_VDP, 2)
    FABM_BATCH_CASE(SYS_FINANCIAL, 3)
    FABM_BATCH_CASE(SYS_HINDMARSH_ROSE, 3)
#undef FABM_BATCH_CASE
    *where = "no BLOCKED kernel for this system/dimension";
    return hipErrorInvalidValue;
}

template <int SYS, int D, bool PC>
static hipError_t launch_recompute_t(const BatchArgs &A, const RecompArgs &R, int J, int ninst,
                                     hipStream_t st)
{
    const size_t smem = band_smem_bytes(D, PC);
    static std::atomic<uint64_t> attr_dev{0};
    if (smem > 64 * 1024) {
        const hipError_t e = ensure_lds_attr((const void *)k_recompute_batch<SYS, D, PC>, smem,
                                             attr_dev);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_recompute_batch<SYS, D, PC>), dim3((unsigned)(ninst * (R.G + 1))),
                       dim3(kBatchThreads), smem, st, A, R, J);
    return hipGetLastError();
}

hipError_t launch_recompute(int sys, int d, const BatchArgs &A, const RecompArgs &R, int J,
                            int ninst, hipStream_t s)
{
    if (ninst <= 0) return hipSuccess;
#define FABM_REC_CASE(SS, DD)                                                     \
    if (sys == SS && d == DD)                                                     \
        return A.cmeta ? launch_recompute_t<SS, DD, true>(A, R, J, ninst, s)      \
                       : launch_recompute_t<SS, DD, false>(A, R, J, ninst, s);
    FABM_REC_CASE(SYS_LINEAR, 1)
    FABM_REC_CASE(SYS_LINEAR, 2)
    FABM_REC_CASE(SYS_LINEAR, 3)
    FABM_REC_CASE(SYS_LINEAR, 4)
    FABM_REC_CASE(SYS_CHEN, 3)
    FABM_REC_CASE(SYS_ROSSLER, 3)
    FABM_REC_CASE(SYS_VDP, 2)
    FABM_REC_CASE(SYS_FINANCIAL, 3)
    FABM_REC_CASE(SYS_HINDMARSH_ROSE, 3)
#undef FABM_REC_CASE
    return hipErrorInvalidValue;
}

hipError_t enqueue_steps(int sys, int d, bool f32, const StepArgs &A, hipStream_t s,
                         KernelTimer *T, const char **where)
{
#define FABM_STEP_CASE(SS, DD)                                                   \
    if (sys == SS && d == DD)                                                    \
        return A.cmeta ? (f32 ? enqueue_steps_t<SS, DD, true, true>(A, s, T, where)     \
                              : enqueue_steps_t<SS, DD, false, true>(A, s, T, where))   \
               : f32   ? enqueue_steps_t<SS, DD, true, false>(A, s, T, where)    \
                       : enqueue_steps_t<SS, DD, false, false>(A, s, T, where);
    FABM_STEP_CASE(SYS_LINEAR, 1)
    FABM_STEP_CASE(SYS_LINEAR, 2)
    FABM_STEP_CASE(SYS_LINEAR, 3)
    FABM_STEP_CASE(SYS_LINEAR, 4)
    FABM_STEP_CASE(SYS_CHEN, 3)
    FABM_STEP_CASE(SYS_ROSSLER, 3)
    FABM_STEP_CASE(SYS_VDP, 2)
    FABM_STEP_CASE(SYS_FINANCIAL, 3)
    FABM_STEP_CASE(SYS_HINDMARSH_ROSE, 3)
#undef FABM_STEP_CASE
#define FABM_TEACHER_CASE(DD)                                                    \
    if (sys == SYS_TEACHER && d == DD && !A.cmeta)                               \
        return f32 ? enqueue_steps_t<SYS_TEACHER, DD, true, false>(A, s, T, where) \
                   : enqueue_steps_t<SYS_TEACHER, DD, false, false>(A, s, T, where);
    FABM_TEACHER_CASE(1)
    FABM_TEACHER_CASE(2)
    FABM_TEACHER_CASE(3)
    FABM_TEACHER_CASE(4)
#undef FABM_TEACHER_CASE
    *where = "no BLOCKED kernel for this system/dimension";
    return hipErrorInvalidValue;
}

int step_block_len() { return kBlk; }

}  // namespace fabm
