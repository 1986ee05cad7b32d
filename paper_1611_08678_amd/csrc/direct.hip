// direct.hip -- the DIRECT contraction path: at every step t the whole
// history f_0..f_{t-1} is reduced against the weight rows b_{t-1-k} and
// a_{t-1-k} (Section 2: the predictor sum of eq. (2) and the corrector sum),
// followed by the PECE update. Two shapes:
//
//  * k_direct_wg: one 256-thread workgroup per trajectory. Each step is a
//    coalesced strided pass over the history, a wavefront butterfly sum and an
//    LDS combine of the four wavefronts; lane 0 then forms y_t and f_t. Used
//    for batches of independent trajectories and for short ones.
//
//  * k_direct_grid: one long trajectory over the whole GPU (one persistent
//    workgroup per compute unit, cooperative launch so all are resident).
//    Each step every workgroup reduces a contiguous slice of [0, t), writes
//    its partial and signals an arrival counter; every workgroup then waits
//    for all arrivals, adds the partials in a fixed order (deterministic) and
//    forms row t itself: one inter-workgroup hand-off per step. Step time is
//    bound by HBM streaming of the history and weight rows at large t and by
//    that hand-off at small t.
#include "fabm_device.h"
#include "fabm_launch.h"

namespace fabm {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;

template <int D>
__device__ __forceinline__ void block_sum2(double (&sp)[D], double (&sc)[D],
                                           double (*red)[2 * D], int tid)
{
    const int lane = tid & (kWave - 1), wv = tid / kWave;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        sp[i] = wave_sum(sp[i]);
        sc[i] = wave_sum(sc[i]);
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            red[wv][i] = sp[i];
            red[wv][D + i] = sc[i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double a = red[0][i], c = red[0][D + i];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            a += red[w][i];
            c += red[w][D + i];
        }
        sp[i] = a;
        sc[i] = c;
    }
}

// Partial history sums over k in [lo, hi) for target t (strided by the block).
template <int D>
__device__ __forceinline__ void partial_sums(const double *__restrict__ Fh,
                                             const double *__restrict__ wb,
                                             const double *__restrict__ wa,
                                             const double *__restrict__ wc, int64_t t, int64_t lo,
                                             int64_t hi, int tid, double (&sp)[D], double (&sc)[D])
{
#pragma unroll
    for (int i = 0; i < D; ++i) sp[i] = sc[i] = 0.0;
    for (int64_t k = lo + tid; k < hi; k += kBlock) {
        const double bw = wb[t - 1 - k];
        const double aw = (k == 0) ? wc[t - 1] : wa[t - 1 - k];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double fk = Fh[k * D + i];
            sp[i] = fma(bw, fk, sp[i]);
            sc[i] = fma(aw, fk, sc[i]);
        }
    }
}

// Non-commensurate orders: component i has its own order, so its own weight
// rows and step scalars (cmeta[i], placed like an instance's).
template <int D>
struct CompOrders {
    const double *wb[D], *wa[D], *wc[D];
    double ha[D], ig2[D], alpha[D];
};

template <int D>
__device__ __forceinline__ CompOrders<D> comp_orders(const InstMeta *__restrict__ cm,
                                                     const double *__restrict__ W)
{
    CompOrders<D> O;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const InstMeta q = cm[i];
        O.wb[i] = W + q.w_off;
        O.wa[i] = O.wb[i] + q.wlen;
        O.wc[i] = O.wa[i] + q.wlen;
        O.ha[i] = q.ha;
        O.ig2[i] = q.ig2;
        O.alpha[i] = q.alpha;
    }
    return O;
}

// partial_sums with each component's own weight rows
template <int D>
__device__ __forceinline__ void partial_sums_orders(const double *__restrict__ Fh,
                                                    const CompOrders<D> &O, int64_t t,
                                                    int64_t lo, int64_t hi, int tid,
                                                    double (&sp)[D], double (&sc)[D])
{
#pragma unroll
    for (int i = 0; i < D; ++i) sp[i] = sc[i] = 0.0;
    for (int64_t k = lo + tid; k < hi; k += kBlock) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double bw = O.wb[i][t - 1 - k];
            const double aw = (k == 0) ? O.wc[i][t - 1] : O.wa[i][t - 1 - k];
            const double fk = Fh[k * D + i];
            sp[i] = fma(bw, fk, sp[i]);
            sc[i] = fma(aw, fk, sc[i]);
        }
    }
}

// y'(0) of the components whose order exceeds one, zeros elsewhere
template <int D>
__device__ __forceinline__ void load_slope_orders(const CompOrders<D> &O, const double *y1,
                                                  double (&v)[D])
{
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = (y1 != nullptr && O.alpha[i] > 1.0) ? y1[i] : 0.0;
}

// pece_update with each component's h^alpha and 1/Gamma(alpha+2)
template <int SYS, int D>
__device__ __forceinline__ void pece_update_orders(const CompOrders<D> &O, double tt,
                                                   const double (&base)[D], const double (&P)[D],
                                                   const double (&Cs)[D],
                                                   const double *__restrict__ p, double (&y)[D],
                                                   double (&f)[D])
{
    double yp[D], fp[D];
#pragma unroll
    for (int i = 0; i < D; ++i) yp[i] = fma(O.ha[i], P[i], base[i]);
    rhs<SYS, D>(tt, yp, fp, p);
#pragma unroll
    for (int i = 0; i < D; ++i) y[i] = fma(O.ha[i], fma(fp[i], O.ig2[i], Cs[i]), base[i]);
    rhs<SYS, D>(tt, y, f, p);
}

template <int SYS, int D, bool PC>
__global__ __launch_bounds__(kBlock) void k_direct_wg(const InstMeta *__restrict__ meta,
                                                      const InstMeta *__restrict__ cmeta,
                                                      const double *__restrict__ params,
                                                      const double *__restrict__ y0g,
                                                      const double *__restrict__ y1g,
                                                      double *__restrict__ F,
                                                      const double *__restrict__ W,
                                                      double *__restrict__ Y,
                                                      int64_t *__restrict__ status)
{
    __shared__ double red[kWaves][2 * D];
    __shared__ int64_t s_dead;
    const int inst = blockIdx.x, tid = threadIdx.x;
    const InstMeta m = meta[inst];
    const int64_t N = m.N;
    const double *wb = W + m.w_off, *wa = wb + m.wlen, *wc = wa + m.wlen;
    double *Fh = F + m.f_off * D, *Yh = Y + m.row_off * D;
    const double *p = params + m.p_off;
    double y0[D], y1[D];
#pragma unroll
    for (int i = 0; i < D; ++i) y0[i] = y0g[(int64_t)inst * D + i];
    CompOrders<D> O;
    if constexpr (PC) {
        O = comp_orders<D>(cmeta + (int64_t)inst * D, W);
        load_slope_orders<D>(O, y1g ? y1g + (int64_t)inst * D : nullptr, y1);
    } else {
        load_slope<D>(m, y1g ? y1g + (int64_t)inst * D : nullptr, y1);
    }

    if (tid == 0) {
        double f0[D];
        rhs<SYS, D>(0.0, y0, f0, p);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            Fh[i] = f0[i];
            Yh[i] = y0[i];
        }
        s_dead = 0;
    }
    __syncthreads();

    for (int64_t t = 1; t <= N; ++t) {
        if (s_dead) break;
        double sp[D], sc[D];
        if constexpr (PC) partial_sums_orders<D>(Fh, O, t, 0, t, tid, sp, sc);
        else partial_sums<D>(Fh, wb, wa, wc, t, 0, t, tid, sp, sc);
        block_sum2<D>(sp, sc, red, tid);
        if (tid == 0) {
            double y[D], f[D], base[D];
            const double tt = (double)t * m.h;
            taylor_base<D>(tt, y0, y1, base);
            if constexpr (PC) pece_update_orders<SYS, D>(O, tt, base, sp, sc, p, y, f);
            else pece_update<SYS, D>(m, tt, base, sp, sc, p, y, f);
            if (!finite_all(y) || !finite_all(f)) {
                s_dead = t;
            } else {
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    Fh[t * D + i] = f[i];
                    Yh[t * D + i] = y[i];
                }
            }
        }
        __syncthreads();
    }
    const int64_t dead = s_dead;
    if (tid == 0) status[inst] = dead;
    if (dead)
        for (int64_t r = dead + tid; r <= N; r += kBlock)
#pragma unroll
            for (int i = 0; i < D; ++i) Yh[r * D + i] = __builtin_nan("");
}

// Values shared between workgroups on different XCDs (each XCD has its own
// L2): written with agent-scope atomic stores (through to the device's
// coherence point) and read with agent-scope atomic loads (from it), so no
// L2 write-back or invalidation is needed for them.
__device__ __forceinline__ void coh_store(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double coh_load(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until this thread's earlier stores have been acknowledged (vmcnt(0));
// the compiler moves no memory operation across it.
__device__ __forceinline__ void stores_done()
{
    __asm__ __volatile__("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) expcnt(7) lgkmcnt(15)
    __asm__ __volatile__("" ::: "memory");
}

// Partial sums for target T over k in [lo, hi) (strided by the block), every
// history row read at the coherence point except row kreg, taken from `fl`
// (formed by this workgroup itself).
template <int D>
__device__ __forceinline__ void partial_sums_coh(const double *__restrict__ Fh,
                                                 const double *__restrict__ wb,
                                                 const double *__restrict__ wa,
                                                 const double *__restrict__ wc, int64_t T,
                                                 int64_t lo, int64_t hi, int tid, int64_t kreg,
                                                 const double (&fl)[D], double (&sp)[D],
                                                 double (&sc)[D])
{
#pragma unroll
    for (int i = 0; i < D; ++i) sp[i] = sc[i] = 0.0;
    for (int64_t k = lo + tid; k < hi; k += kBlock) {
        const double bw = wb[T - 1 - k];
        const double aw = (k == 0) ? wc[T - 1] : wa[T - 1 - k];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double fk = k == kreg ? fl[i] : coh_load(&Fh[k * D + i]);
            sp[i] = fma(bw, fk, sp[i]);
            sc[i] = fma(aw, fk, sc[i]);
        }
    }
}

template <int D>
__device__ __forceinline__ void partial_sums_orders_coh(const double *__restrict__ Fh,
                                                        const CompOrders<D> &O, int64_t T,
                                                        int64_t lo, int64_t hi, int tid,
                                                        int64_t kreg, const double (&fl)[D],
                                                        double (&sp)[D], double (&sc)[D])
{
#pragma unroll
    for (int i = 0; i < D; ++i) sp[i] = sc[i] = 0.0;
    for (int64_t k = lo + tid; k < hi; k += kBlock) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double bw = O.wb[i][T - 1 - k];
            const double aw = (k == 0) ? O.wc[i][T - 1] : O.wa[i][T - 1 - k];
            const double fk = k == kreg ? fl[i] : coh_load(&Fh[k * D + i]);
            sp[i] = fma(bw, fk, sp[i]);
            sc[i] = fma(aw, fk, sc[i]);
        }
    }
}

// One hand-off per step. At step t every workgroup g reduces its slice
// [t g / G, t (g + 1) / G) of the history (rows up to t - 2 from memory, the
// newest row t - 1 from its own registers) and stores its partial in its slot
// of buffer t mod 3; thread j of every workgroup waits until workgroup j's
// slot holds values (the slot's previous contents were replaced by a marker
// value no arithmetic produces), reads them, and the partials are added in
// workgroup order, so every workgroup forms row t itself, bitwise the same,
// and no row has to be published before the next step. Workgroup 0 writes
// the rows to F (through to the coherence point) and Y.
// Ordering without cache maintenance: partials, markers and history rows are
// stored and loaded at the coherence point. At the start of step t a
// workgroup marks its slot of step t + 1 (buffer (t + 1) mod 3, last read at
// step t - 2, and every workgroup has finished reading step t - 2 before it
// stored its step t - 1 partial, all of which this workgroup has read); its
// step t partial is stored only after its earlier stores are acknowledged
// (the marking, and workgroup 0's row t - 1), so a reader that sees a
// workgroup's step t values finds its step t + 1 slot marked, and a history
// row, read two steps after it was formed, is in place. Every slot starts
// marked (filled before the launch); abort word at kSyncLine * 17.
constexpr int kSyncLine = 64;   // words per line of the sync area
constexpr int kSlot = 16;       // doubles per partial slot (2d <= 8 used; 128 bytes)
constexpr int kSlotBuffers = 3;
// the marker of an empty slot: a signalling NaN (arithmetic yields quiet NaNs)
constexpr uint32_t kEmptyWord = 0xFFF4A5A5u;
constexpr uint64_t kEmptyBits = ((uint64_t)kEmptyWord << 32) | kEmptyWord;

__device__ __forceinline__ bool slot_empty(double v)
{
    return __builtin_bit_cast(uint64_t, v) == kEmptyBits;
}

// Spin until every value of slot q is present (then they are in qp, qc), or
// *abort is raised, or the wall clock passes `deadline` (then *abort is
// raised). Every wait is bounded, so a mistake ends the launch with an error
// status instead of a hung GPU.
template <int D>
__device__ __forceinline__ bool wait_slot(const double *q, double (&qp)[D], double (&qc)[D],
                                          uint32_t *abort, uint64_t deadline)
{
    for (;;) {
        bool full = true;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            qp[i] = coh_load(&q[i]);
            qc[i] = coh_load(&q[D + i]);
            full = full && !slot_empty(qp[i]) && !slot_empty(qc[i]);
        }
        if (full) return true;
        if (flag_read(abort) != 0u) return false;
        if (wall_clock64() > deadline) {
            flag_max(abort, 1u);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

template <int SYS, int D, bool PC>
__global__ __launch_bounds__(kBlock) void k_direct_grid(const InstMeta *__restrict__ meta,
                                                        const InstMeta *__restrict__ cmeta,
                                                        const double *__restrict__ params,
                                                        const double *__restrict__ y0g,
                                                        const double *__restrict__ y1g,
                                                        double *__restrict__ F,
                                                        const double *__restrict__ W,
                                                        double *__restrict__ Y,
                                                        int64_t *__restrict__ status,
                                                        double *__restrict__ part,
                                                        uint32_t *__restrict__ sync,
                                                        uint64_t timeout_ticks)
{
    __shared__ double red[kWaves][2 * D], red2[kWaves][2 * D];
    __shared__ int s_stop;
    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
    const InstMeta m = meta[0];
    const int64_t N = m.N;
    const double *wb = W + m.w_off, *wa = wb + m.wlen, *wc = wa + m.wlen;
    const double *p = params;
    uint32_t *abort = sync + kSyncLine * 17;
    double y0[D], y1[D];
#pragma unroll
    for (int i = 0; i < D; ++i) y0[i] = y0g[i];
    CompOrders<D> O;
    if constexpr (PC) {
        O = comp_orders<D>(cmeta, W);
        load_slope_orders<D>(O, y1g, y1);
    } else {
        load_slope<D>(m, y1g, y1);
    }

    double fl[D];  // the newest row's f, formed by this workgroup
    rhs<SYS, D>(0.0, y0, fl, p);
    if (g == 0 && tid == 0) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            coh_store(&F[i], fl[i]);
            Y[i] = y0[i];
        }
    }
    int64_t dead = 0;      // first non-finite row (all workgroups find the same)
    bool aborted = false;  // a wait gave up
    const uint64_t deadline_step = timeout_ticks;
    // this thread's sums for the current target over its slice without the
    // newest row, formed during the step before (none for t = 1)
    double pp[D], pq[D];
#pragma unroll
    for (int i = 0; i < D; ++i) pp[i] = pq[i] = 0.0;
    int64_t t = 1;
    for (; t <= N; ++t) {
        if (tid == 0) {
            s_stop = 0;
            // mark this workgroup's slot of step t + 1
            double *nx = part + ((int64_t)((t + 1) % kSlotBuffers) * G + g) * kSlot;
            const double empty = __builtin_bit_cast(double, kEmptyBits);
#pragma unroll
            for (int i = 0; i < 2 * D; ++i) coh_store(&nx[i], empty);
        }
        const int64_t lo = (t * g) / G, hi = (t * (g + 1)) / G;
        // the newest row t - 1 completes the sums (it is the last k of the
        // thread that holds it, as in a plain pass over the slice)
        double sp[D], sc[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            sp[i] = pp[i];
            sc[i] = pq[i];
        }
        if (t - 1 >= lo && t - 1 < hi && (int)((t - 1 - lo) % kBlock) == tid) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double bw = PC ? O.wb[i][0] : wb[0];
                const double aw = t == 1 ? (PC ? O.wc[i][0] : wc[0]) : (PC ? O.wa[i][0] : wa[0]);
                sp[i] = fma(bw, fl[i], sp[i]);
                sc[i] = fma(aw, fl[i], sc[i]);
            }
        }
        block_sum2<D>(sp, sc, red, tid);
        const int buf = (int)(t % kSlotBuffers);
        if (tid == 0) {
            // the marking above and workgroup 0's row t - 1 first
            stores_done();
            double *slot = part + ((int64_t)buf * G + g) * kSlot;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                coh_store(&slot[i], sp[i]);
                coh_store(&slot[D + i], sc[i]);
            }
        }
        // While the other partials of step t arrive: the sums for target t + 1
        // over its slice up to row t - 1 (row t - 1 from registers, earlier
        // rows from memory: row t - 2 was stored before workgroup 0's partial
        // of step t - 1)
        if (t < N) {
            const int64_t lo1 = ((t + 1) * g) / G, hi1 = ((t + 1) * (g + 1)) / G;
            const int64_t hm = hi1 < t ? hi1 : t;
            if constexpr (PC) partial_sums_orders_coh<D>(F, O, t + 1, lo1, hm, tid, t - 1, fl, pp, pq);
            else partial_sums_coh<D>(F, wb, wa, wc, t + 1, lo1, hm, tid, t - 1, fl, pp, pq);
        }
        double qp[D], qc[D];
#pragma unroll
        for (int i = 0; i < D; ++i) qp[i] = qc[i] = 0.0;
        if (tid < G) {
            const double *q = part + ((int64_t)buf * G + tid) * kSlot;
            if (!wait_slot<D>(q, qp, qc, abort, wall_clock64() + deadline_step)) {
#pragma unroll
                for (int i = 0; i < D; ++i) qp[i] = qc[i] = 0.0;
                s_stop = 1;
            }
        }
        block_sum2<D>(qp, qc, red2, tid);
        if (s_stop) {
            aborted = true;
            break;
        }
        double y[D], f[D], base[D];
        const double tt = (double)t * m.h;
        taylor_base<D>(tt, y0, y1, base);
        if constexpr (PC) pece_update_orders<SYS, D>(O, tt, base, qp, qc, p, y, f);
        else pece_update<SYS, D>(m, tt, base, qp, qc, p, y, f);
        if (!finite_all(y) || !finite_all(f)) {
            dead = t;
            break;
        }
        if (g == 0 && tid == 0) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                coh_store(&F[t * D + i], f[i]);
                Y[t * D + i] = y[i];
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) fl[i] = f[i];
        __syncthreads();  // red and red2 are reused by the next step
    }
    if (g == 0) {
        // rows from `bad` on are not final: the first non-finite step, or the
        // step whose wait gave up
        const int64_t bad = aborted ? t : dead;
        if (tid == 0) status[0] = aborted ? -1 : dead;
        if (bad)
            for (int64_t r = bad + tid; r <= N; r += kBlock)
#pragma unroll
                for (int i = 0; i < D; ++i) Y[r * D + i] = __builtin_nan("");
    }
}

// Teacher-forced sums for all targets t = 1..N: block = 256 consecutive targets;
// sources are staged through LDS 256 at a time together with the 511 weights
// the block needs for that source chunk.
template <int D>
__global__ __launch_bounds__(kBlock) void k_history_direct(const double *__restrict__ W,
                                                           int64_t N,
                                                           const double *__restrict__ f,
                                                           double *__restrict__ P,
                                                           double *__restrict__ C)
{
    __shared__ double sf[kBlock * D];
    __shared__ double sb[2 * kBlock], sa[2 * kBlock];
    const double *wb = W, *wa = W + N, *wc = W + 2 * N;
    const int tid = threadIdx.x;
    const int64_t T0 = 1 + (int64_t)blockIdx.x * kBlock;  // first target of the block
    const int64_t t = T0 + tid;
    const int64_t tmax = min(T0 + kBlock - 1, N);
    double sp[D], sc[D];
#pragma unroll
    for (int i = 0; i < D; ++i) sp[i] = sc[i] = 0.0;
    for (int64_t k0 = 0; k0 < tmax; k0 += kBlock) {
        __syncthreads();
        for (int j = tid; j < kBlock * D; j += kBlock) {
            const int64_t r = k0 + j / D;
            sf[j] = r < N ? f[k0 * D + j] : 0.0;
        }
        // lag of (target T0 + x, source k0 + j) is T0 - 1 - k0 + x - j, x - j in [-255, 255]
        for (int j = tid; j < 2 * kBlock; j += kBlock) {
            const int64_t lag = T0 - 1 - k0 + (j - (kBlock - 1));
            const bool ok = lag >= 0 && lag < N;
            sb[j] = ok ? wb[lag] : 0.0;
            sa[j] = ok ? wa[lag] : 0.0;
        }
        __syncthreads();
        if (t <= N) {
            const int jmax = (int)min((int64_t)kBlock, t - k0);
            for (int j = 0; j < jmax; ++j) {
                const int li = tid - j + (kBlock - 1);
                const double bw = sb[li];
                const double aw = (k0 + j == 0) ? wc[t - 1] : sa[li];
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    sp[i] = fma(bw, sf[j * D + i], sp[i]);
                    sc[i] = fma(aw, sf[j * D + i], sc[i]);
                }
            }
        }
    }
    if (t <= N) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            P[(t - 1) * D + i] = sp[i];
            C[(t - 1) * D + i] = sc[i];
        }
    }
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)(b < 1024 ? b : 1024)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// One instance entry written from a kernel argument (no host staging buffer).
__global__ void k_put_meta(InstMeta m, InstMeta *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = m;
}

hipError_t launch_put_meta(const InstMeta &m, InstMeta *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_put_meta, dim3(1), dim3(64), 0, s, m, dst);
    return hipGetLastError();
}

// dst[e] = e < n_src ? src[e] : 0 for e < n_dst (a kernel, safe inside graphs).
__global__ void k_copy_pad(const double *__restrict__ src, int64_t n_src, double *__restrict__ dst,
                           int64_t n_dst)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_dst;
         e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = e < n_src ? src[e] : 0.0;
}

hipError_t launch_copy_pad(const double *src, int64_t n_src, double *dst, int64_t n_dst,
                           hipStream_t s)
{
    if (n_dst <= 0) return hipSuccess;
    const int64_t b = (n_dst + 255) / 256;
    hipLaunchKernelGGL(k_copy_pad, dim3((unsigned)(b < 2048 ? b : 2048)), dim3(256), 0, s, src,
                       n_src, dst, n_dst);
    return hipGetLastError();
}

// init [batch][2][d] -> y0 [batch][d], y1 [batch][d]
__global__ void k_split_init(const double *__restrict__ init, int64_t batch, int d,
                             double *__restrict__ y0, double *__restrict__ y1)
{
    const int64_t n = batch * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / d, c = e - i * d;
        y0[e] = init[(2 * i) * d + c];
        y1[e] = init[(2 * i + 1) * d + c];
    }
}

hipError_t launch_split_init(const double *init, int64_t batch, int d, double *y0, double *y1,
                             hipStream_t s)
{
    const int64_t n = batch * d;
    if (n <= 0) return hipSuccess;
    const int64_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_split_init, dim3((unsigned)(b < 1024 ? b : 1024)), dim3(256), 0, s, init,
                       batch, d, y0, y1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dispatch over (system, dimension). LINEAR is instantiated for the small
// dimensions the direct kernels keep in registers.
// ---------------------------------------------------------------------------
template <template <int, int> class K>
struct Dispatch;

#define FABM_DIRECT_CASES(MACRO)                                   \
    MACRO(SYS_LINEAR, 1) MACRO(SYS_LINEAR, 2) MACRO(SYS_LINEAR, 3) \
    MACRO(SYS_LINEAR, 4) MACRO(SYS_CHEN, 3) MACRO(SYS_ROSSLER, 3)  \
    MACRO(SYS_VDP, 2) MACRO(SYS_FINANCIAL, 3) MACRO(SYS_HINDMARSH_ROSE, 3)

hipError_t launch_direct_wg(int sys, int d, const InstMeta *meta, const InstMeta *cmeta,
                            int64_t batch, const double *params, const double *y0,
                            const double *y1, double *F, const double *W, double *Y,
                            int64_t *status, hipStream_t s)
{
#define FABM_WG_CASE(S, DD)                                                                  \
    if (sys == S && d == DD) {                                                               \
        if (cmeta)                                                                           \
            hipLaunchKernelGGL((k_direct_wg<S, DD, true>), dim3((unsigned)batch), dim3(kBlock), \
                               0, s, meta, cmeta, params, y0, y1, F, W, Y, status);          \
        else                                                                                 \
            hipLaunchKernelGGL((k_direct_wg<S, DD, false>), dim3((unsigned)batch),          \
                               dim3(kBlock), 0, s, meta, cmeta, params, y0, y1, F, W, Y,    \
                               status);                                                      \
        return hipGetLastError();                                                            \
    }
    FABM_DIRECT_CASES(FABM_WG_CASE)
#undef FABM_WG_CASE
    return hipErrorInvalidValue;
}

size_t direct_grid_part_doubles(int G) { return (size_t)kSlotBuffers * kSlot * (size_t)G; }
size_t direct_grid_sync_words(int) { return (size_t)kSyncLine * 18; }
uint32_t direct_grid_empty_word() { return kEmptyWord; }

hipError_t launch_direct_grid(int sys, int d, int G, const InstMeta *meta, const InstMeta *cmeta,
                              const double *params, const double *y0, const double *y1,
                              double *F, const double *W, double *Y, int64_t *status,
                              double *part, uint32_t *sync, uint64_t timeout_ticks,
                              hipStream_t s)
{
    void *args[] = {(void *)&meta,   (void *)&cmeta, (void *)&params, (void *)&y0,
                    (void *)&y1,     (void *)&F,     (void *)&W,      (void *)&Y,
                    (void *)&status, (void *)&part,  (void *)&sync,   (void *)&timeout_ticks};
#define FABM_GRID_CASE(S, DD)                                                                \
    if (sys == S && d == DD)                                                                 \
        return hipLaunchCooperativeKernel(cmeta ? (const void *)k_direct_grid<S, DD, true>   \
                                                : (const void *)k_direct_grid<S, DD, false>, \
                                          dim3(G), dim3(kBlock), args, 0, s);
    FABM_DIRECT_CASES(FABM_GRID_CASE)
#undef FABM_GRID_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_history_direct(const double *W, int64_t N, int d, const double *f, double *P,
                                 double *C, hipStream_t s)
{
    const unsigned blocks = (unsigned)((N + kBlock - 1) / kBlock);
    switch (d) {
    case 1: hipLaunchKernelGGL(k_history_direct<1>, dim3(blocks), dim3(kBlock), 0, s, W, N, f, P, C); break;
    case 2: hipLaunchKernelGGL(k_history_direct<2>, dim3(blocks), dim3(kBlock), 0, s, W, N, f, P, C); break;
    case 3: hipLaunchKernelGGL(k_history_direct<3>, dim3(blocks), dim3(kBlock), 0, s, W, N, f, P, C); break;
    case 4: hipLaunchKernelGGL(k_history_direct<4>, dim3(blocks), dim3(kBlock), 0, s, W, N, f, P, C); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fabm
