// capi.hip -- the C ABI declared in include/fabm.h: argument validation,
// path choice, workspace layout, per-call instance metadata and schedules,
// kernel dispatch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "fabm.h"
#include "fabm_adjoint.h"
#include "fabm_blocked.h"
#include "fabm_device.h"
#include "fabm_launch.h"
#include "fabm_timer.h"
#include "fabm_wide.h"

using fabm::InstMeta;

struct fabm_plan_s {
    fabm_plan_desc desc;
    int32_t n_params;
    int device;
    int grid_G;          // workgroups of the persistent single-trajectory kernels
    char *h_stage;       // pinned staging of the per-call instance table
    size_t stage_cap;
    hipEvent_t stage_ev; // recorded after the staging copy; waited on before reuse
    bool stage_pending;
    uint64_t timeout_ticks;  // bound of every inter-workgroup wait (device wall clock)
    bool info_ready = false;  // device, grid_G and timeout_ticks are set
    fabm::KernelTimer timer;   // optional per-kernel timing
    // schedule of the last batched BLOCKED call, keyed by its block counts
    std::vector<int32_t> sched_nb;
    fabm::BatchSchedule sched;
    // launch shapes (defaults, or the fastest found by fabm_tune)
    int far_cap = fabm::kMaxFarWg;               // single-trajectory BLOCKED
    int split_target = fabm::kWideSplitTarget;  // shared grid
    int batch_group = fabm::kDefaultBatchGroup; // batched BLOCKED: source blocks per group
};

// A captured solve: its instance table lives in its own pinned buffer, copied
// by the graph's first node at every launch.
struct fabm_graph_s {
    char *stage = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// Last HIP failure seen by this thread (returned by fabm_last_error).
thread_local char g_last_error[256] = "";

fabm_status record_hip(const char *what, hipError_t e)
{
    if (e == hipSuccess) return FABM_OK;
    std::snprintf(g_last_error, sizeof g_last_error, "%s: %s (%d)", what, hipGetErrorString(e),
                  (int)e);
    return FABM_ERR_DEVICE;
}

#define HIP_TRY(expr)                                           \
    do {                                                        \
        const fabm_status s_ = record_hip(#expr, (expr));       \
        if (s_ != FABM_OK) return s_;                           \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxLinearDim = 64;
constexpr int64_t kGridDirectMinSteps = 8192;  // single trajectories this long use the grid kernel
constexpr int kGridMax = 256;                  // MI355X compute units
constexpr int64_t kAutoBlockedMinSteps = 1024;
constexpr uint64_t kWaitTimeoutSeconds = 10;  // no legitimate wait comes near this
constexpr int64_t kWideMaxCols = (int64_t)1 << 30;  // shared grid: instances x d
constexpr int64_t kMaxHistorySteps = (int64_t)1 << 26;  // teacher-forced sums: row index in int32 blocks

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool aligned8(const void *p) { return p && ((uintptr_t)p & 7u) == 0; }

int32_t n_params_of(int sys, int d)
{
    switch (sys) {
    case FABM_SYS_LINEAR: return (d >= 1 && d <= kMaxLinearDim) ? d * d + 2 * d : -1;
    case FABM_SYS_CHEN:
    case FABM_SYS_ROSSLER:
    case FABM_SYS_FINANCIAL: return d == 3 ? 3 : -1;
    case FABM_SYS_VDP: return d == 2 ? 1 : -1;
    case FABM_SYS_HINDMARSH_ROSE: return d == 3 ? 8 : -1;
    default: return -1;
    }
}

// Orders up to one need y(0) only; 1 < alpha <= 2 needs y'(0) as well, which
// calls pass when the plan has FABM_PLAN_INITIAL_SLOPE (`two_init`).
fabm_status check_alpha_h(double alpha, double h, bool two_init)
{
    if (!std::isfinite(alpha) || !std::isfinite(h) || h <= 0.0 || alpha <= 0.0)
        return FABM_ERR_INVALID_ARG;
    if (alpha > 2.0) return FABM_ERR_INVALID_ARG;
    if (alpha > 1.0 && !two_init) return FABM_ERR_UNSUPPORTED;
    return FABM_OK;
}

bool has_slope(const fabm_plan_s *pl) { return (pl->desc.flags & FABM_PLAN_INITIAL_SLOPE) != 0; }
bool per_component(const fabm_plan_s *pl)
{
    return (pl->desc.flags & FABM_PLAN_PER_COMPONENT_ORDER) != 0;
}
bool adjoint_checkpoint(const fabm_plan_s *pl)
{
    return (pl->desc.flags & FABM_PLAN_ADJOINT_CHECKPOINT) != 0;
}

enum class Path { Direct, Blocked, Wide, Unsupported };

// LINEAR plans that need the shared-grid form: states wider than the
// per-trajectory kernels hold in registers, split binary16 far tiles, or its
// block length asked for explicitly.
bool wide_plan(const fabm_plan_desc &d)
{
    return d.system == FABM_SYS_LINEAR &&
           (d.dim > 4 || d.far_prec == FABM_FAR_FP16X2 || d.tile_L == fabm::kWideBlk);
}

Path choose_path(const fabm_plan_s *pl, int64_t batch, const int64_t *N)
{
    if (wide_plan(pl->desc)) return Path::Wide;  // never with per-component orders
    switch (pl->desc.path) {
    case FABM_PATH_DIRECT: return Path::Direct;
    case FABM_PATH_BLOCKED: return Path::Blocked;
    default: {
        int64_t maxN = 0;
        for (int64_t i = 0; i < batch; ++i) maxN = std::max(maxN, N[i]);
        return maxN >= kAutoBlockedMinSteps ? Path::Blocked : Path::Direct;
    }
    }
}

// Device workspace of one solve call (offsets in bytes). The first
// `stage_bytes` bytes are copied from the plan's pinned staging buffer.
struct Layout {
    Path path;
    size_t meta, inst, order, far_off, far_off_rev, meta_adj, stage_bytes;
    size_t w, w32, f, part, carry, acc, sync, n_sync_words;
    // reverse pass only: forward rows, reversed sources and sums, partials
    size_t yw, ypw, uv, acc_a, carry_a, part_a, fbar0;
    size_t rcarry;  // block checkpoints: band sums entering each re-formed block
    // shared grid: low binary16 parts, their scales, Toeplitz operand table
    size_t flo, fexp, t16, t16exp;
    size_t init;   // initial values split into y0 [batch][d] and y'(0) [batch][d]
    size_t cmeta;  // per-component orders: [batch][d] entries (staged after meta)
    size_t ftw, fbuf, fspec;  // sub-quadratic far history: twiddles, transforms, spectra
    int64_t cp;    // shared grid: padded history columns
    size_t total;
    int64_t wlen;  // single-trajectory BLOCKED: weight table length
    int NB;        // single-trajectory BLOCKED: blocks
};

int blocks_of(int64_t N) { return (int)((N + 1 + fabm::step_block_len() - 1) / fabm::step_block_len()); }

// Schedule of a batched BLOCKED call (cached on the plan by block counts).
const fabm::BatchSchedule &batch_schedule_for(const fabm_plan_s *pl, int64_t batch,
                                              const int64_t *N)
{
    fabm_plan_s *mp = const_cast<fabm_plan_s *>(pl);  // host-side cache only
    std::vector<int32_t> nb((size_t)batch);
    for (int64_t i = 0; i < batch; ++i) nb[(size_t)i] = blocks_of(N[i]);
    if (nb != mp->sched_nb || mp->sched.P != mp->batch_group) {
        fabm::batch_schedule(batch, nb.data(), mp->sched, mp->batch_group);
        mp->sched_nb.swap(nb);
    }
    return mp->sched;
}

// adjoint: the reverse pass (always the batched BLOCKED layout, FP64, with the
// extra regions of the reverse pipeline).
Layout layout_for(const fabm_plan_s *pl, int64_t batch, const int64_t *N, bool adjoint = false)
{
    Layout L{};
    L.path = adjoint ? Path::Blocked : choose_path(pl, batch, N);
    const int d = pl->desc.dim;
    int64_t sumN = 0, sumRows = 0;
    for (int64_t i = 0; i < batch; ++i) {
        sumN += N[i];
        sumRows += N[i] + 1;
    }
    size_t off = 0;
    L.meta = off;
    off += sizeof(InstMeta) * (size_t)batch;
    if (L.path == Path::Blocked && (batch > 1 || adjoint)) {
        const fabm::BatchSchedule &S = batch_schedule_for(pl, batch, N);
        const int Lb = fabm::step_block_len();
        const size_t blk = sizeof(double) * 2 * d * (size_t)Lb;
        size_t nw = 0, nf = 0, na = 0;
        for (int64_t i = 0; i < batch; ++i) {
            const size_t nb = (size_t)blocks_of(N[i]);
            nw += 3 * (nb * Lb + Lb);
            nf += (size_t)d * nb * Lb;
            na += nb;
        }
        off = (off + 15) / 16 * 16;
        L.inst = off;
        off += sizeof(fabm::BlkInst) * (size_t)batch;
        L.order = off;
        off += sizeof(int) * (size_t)batch;
        L.far_off = off;
        off += sizeof(int) * S.far_off.size();
        if (adjoint) {
            // the reverse pass takes one source block per launch
            L.far_off_rev = off;
            off += sizeof(int) * S.far_off_single.size();
            off = (off + 15) / 16 * 16;
            L.meta_adj = off;
            off += sizeof(InstMeta) * (size_t)batch;
        }
        const bool pc = per_component(pl);
        if (pc) {  // one entry per (instance, component): its order's weights and scalars
            off = (off + 15) / 16 * 16;
            L.cmeta = off;
            off += sizeof(InstMeta) * (size_t)batch * d;
        }
        L.stage_bytes = off;
        off = align_up(off);
        L.w = off;
        off = align_up(off + sizeof(double) * nw * (pc ? d : 1));
        L.w32 = off;  // binary32 b, a for FP32 far windows
        if (pl->desc.far_prec == FABM_FAR_FP32 && !adjoint)
            off = align_up(off + sizeof(float) * nw / 3 * 2 * (pc ? d : 1));
        L.f = off;  // per instance: component-major history [d][NB_i*256]
        off = align_up(off + sizeof(double) * nf);
        L.carry = off;
        off = align_up(off + 2 * blk * (size_t)batch);
        L.acc = off;
        off = align_up(off + blk * na);
        L.sync = off;  // one non-finite flag per instance
        L.n_sync_words = (size_t)std::max<int64_t>(64, batch);
        off = align_up(off + sizeof(uint32_t) * L.n_sync_words);
        if (adjoint) {
            if (adjoint_checkpoint(pl)) {
                // rings of forward blocks re-formed during the reverse pass
                const size_t ring = (size_t)batch * (fabm::kCkptGroup + 1) * Lb;
                L.yw = off;
                off = align_up(off + sizeof(double) * d * ring);
                L.ypw = off;
                off = align_up(off + sizeof(double) * d * ring);
                L.rcarry = off;
                off = align_up(off + sizeof(double) * 4 * d * ring);
            } else {
                size_t rows = 0;
                for (int64_t i = 0; i < batch; ++i) rows += (size_t)N[i] + 1;
                L.yw = off;
                off = align_up(off + sizeof(double) * d * rows);
                L.ypw = off;
                off = align_up(off + sizeof(double) * d * rows);
            }
            L.uv = off;
            off = align_up(off + sizeof(double) * 2 * nf);
            L.acc_a = off;
            off = align_up(off + blk / 2 * na);
            L.carry_a = off;
            off = align_up(off + blk * (size_t)batch);
            L.part_a = off;  // per block: theta, y(0) and y'(0) partials
            off = align_up(off + sizeof(double) * ((size_t)pl->n_params + 2 * d) * na);
            L.fbar0 = off;
            off = align_up(off + sizeof(double) * d * (size_t)batch);
        }
    } else if (L.path == Path::Wide) {
        int64_t maxN = 1;
        for (int64_t i = 0; i < batch; ++i) maxN = std::max(maxN, N[i]);
        const int Lb = fabm::kWideBlk;
        L.NB = (int)((maxN + 1 + Lb - 1) / Lb);
        L.wlen = (int64_t)L.NB * Lb + Lb;
        L.cp = (batch * d + fabm::kWideColAlign - 1) / fabm::kWideColAlign * fabm::kWideColAlign;
        if (L.cp > kWideMaxCols) {  // column indices and launch shapes are 32-bit
            L.path = Path::Unsupported;
            return L;
        }
        const size_t cells = (size_t)L.NB * Lb * (size_t)L.cp;  // history rows x columns
        const fabm_far_prec fp = pl->desc.far_prec;
        L.stage_bytes = off;
        off = align_up(off);
        L.w = off;
        off = align_up(off + sizeof(double) * 3 * (size_t)L.wlen);
        L.w32 = off;
        if (fp == FABM_FAR_FP32) off = align_up(off + sizeof(float) * 2 * (size_t)L.wlen);
        L.f = off;  // the history copy the far product reads: [rows][cp]
        off = align_up(off + (fp == FABM_FAR_FP64 ? 8 : fp == FABM_FAR_FP32 ? 4 : 2) * cells);
        L.flo = L.fexp = L.t16 = L.t16exp = off;
        if (fp == FABM_FAR_FP16X2) {
            L.flo = off;
            off = align_up(off + 2 * cells);
            L.fexp = off;
            off = align_up(off + sizeof(int32_t) * (size_t)L.NB * (size_t)L.cp);
            L.t16 = off;
            off = align_up(off + fabm::wide_t16_bytes(L.NB));
            L.t16exp = off;
            off = align_up(off + sizeof(int32_t) * 2 * (size_t)L.NB);
        }
        L.part = off;  // far sums of one block, per split
        off = align_up(off + sizeof(double) * (size_t)fabm::wide_max_splits((int)L.cp, L.NB) * 2 *
                                 Lb * (size_t)L.cp);
        L.sync = off;  // first non-finite row of each instance
        L.n_sync_words = (size_t)std::max<int64_t>(64, batch);
        off = align_up(off + sizeof(uint32_t) * L.n_sync_words);
    } else if (L.path == Path::Blocked) {
        const int Lb = fabm::step_block_len();
        L.NB = blocks_of(N[0]);
        L.wlen = (int64_t)L.NB * Lb + Lb;
        const size_t blk = sizeof(double) * 2 * d * (size_t)Lb;  // one [2d][256] block of sums
        const bool pc = per_component(pl);
        if (pc) {
            off = (off + 15) / 16 * 16;
            L.cmeta = off;
            off += sizeof(InstMeta) * (size_t)d;
        }
        L.stage_bytes = off;
        off = align_up(off);
        L.w = off;
        off = align_up(off + sizeof(double) * 3 * (size_t)L.wlen * (pc ? d : 1));
        L.w32 = off;  // binary32 b, a for FP32 far windows
        if (pl->desc.far_prec == FABM_FAR_FP32)
            off = align_up(off + sizeof(float) * 2 * (size_t)L.wlen * (pc ? d : 1));
        L.f = off;  // component-major history [d][NB*256]
        off = align_up(off + sizeof(double) * (size_t)d * (size_t)L.NB * Lb);
        L.carry = off;
        off = align_up(off + 2 * blk);
        L.acc = off;  // near + far sums of every target block
        off = align_up(off + blk * (size_t)L.NB);
        L.sync = off;
        L.n_sync_words = 64;
        off = align_up(off + sizeof(uint32_t) * L.n_sync_words);
        const int64_t mfft = fabm::fft_far_max_len(L.NB, pl->desc.fft_level);
        L.ftw = L.fbuf = L.fspec = off;
        if (mfft > 0) {  // twiddles, one square's transforms, the weight spectra
            L.ftw = off;
            off = align_up(off + 16 * (size_t)mfft);
            L.fbuf = off;
            off = align_up(off + 16 * (size_t)mfft * d);
            L.fspec = off;
            off = align_up(off + 16 * (size_t)fabm::fft_far_spectra_len(L.NB, pl->desc.fft_level) *
                                     (pc ? d : 1));
        }
    } else {
        L.wlen = 0;
        const bool pc = per_component(pl);
        if (pc) {  // one entry per (instance, component): its order's weights and scalars
            off = (off + 15) / 16 * 16;
            L.cmeta = off;
            off += sizeof(InstMeta) * (size_t)batch * d;
        }
        L.stage_bytes = off;
        off = align_up(off);
        L.w = off;
        off = align_up(off + sizeof(double) * 3 * (size_t)sumN * (pc ? d : 1));
        L.f = off;
        off = align_up(off + sizeof(double) * (size_t)d * (size_t)sumRows);
        L.part = off;  // grid-kernel partial slots, by workgroup in three step buffers
        off = align_up(off + sizeof(double) * fabm::direct_grid_part_doubles(kGridMax));
        L.sync = off;  // grid-kernel abort word
        L.n_sync_words = fabm::direct_grid_sync_words(kGridMax);
        off = align_up(off + sizeof(uint32_t) * L.n_sync_words);
    }
    if (has_slope(pl)) {
        L.init = off;
        off = align_up(off + sizeof(double) * 2 * (size_t)d * (size_t)batch);
    }
    L.total = off;
    return L;
}


void host_scalars(double alpha, double h, InstMeta &m)
{
    m.alpha = alpha;
    m.h = h;
    // extended precision on the host, one rounding to binary64
    const long double al = alpha;
    m.ha = (double)std::pow((long double)h, al);
    m.ig1 = (double)(1.0L / std::tgamma(al + 1.0L));
    m.ig2 = (double)(1.0L / std::tgamma(al + 2.0L));
}

fabm_status ok_or_device(hipError_t e) { return record_hip("kernel launch", e); }

// With FABM_PLAN_INITIAL_SLOPE the caller's initial values are [batch][2][d];
// the kernels read y(0) and y'(0) as separate [batch][d] arrays in the
// workspace. Returns the arrays to pass (y1 null without the flag).
fabm_status split_init(const fabm_plan_s *pl, const Layout &L, char *base, int64_t batch,
                       const double *&y0, const double *&y1, hipStream_t s)
{
    y1 = nullptr;
    if (!has_slope(pl)) return FABM_OK;
    const int d = pl->desc.dim;
    double *a = (double *)(base + L.init), *b = a + (size_t)batch * d;
    fabm_status st = ok_or_device(fabm::launch_split_init(y0, batch, d, a, b, s));
    if (st != FABM_OK) return st;
    y0 = a;
    y1 = b;
    return FABM_OK;
}

// Launch parameters read from the device (attribute queries only, nothing
// allocated): compute units for the whole-GPU kernel, the wait bound in
// ticks of the constant clock.
fabm_status device_info(fabm_plan_s *pl)
{
    if (pl->info_ready) return FABM_OK;
    int cus = 0;
    HIP_TRY(hipGetDevice(&pl->device));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device));
    pl->grid_G = std::min(cus, kGridMax);
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, pl->device) !=
            hipSuccess ||
        rate_khz <= 0)
        rate_khz = 100000;  // gfx9 constant clock: 100 MHz
    pl->timeout_ticks = (uint64_t)rate_khz * 1000u * kWaitTimeoutSeconds;
    pl->info_ready = true;
    return FABM_OK;
}

// Device-side resources of a plan, created at its first solve so that
// fabm_plan itself touches no device.
fabm_status ensure_device(fabm_plan_s *pl)
{
    if (pl->h_stage) return FABM_OK;
    fabm_status ist = device_info(pl);
    if (ist != FABM_OK) return ist;
    pl->stage_cap = sizeof(InstMeta) * (size_t)pl->desc.max_batch;
    hipError_t e = hipHostMalloc((void **)&pl->h_stage, pl->stage_cap, hipHostMallocDefault);
    if (e != hipSuccess) {
        pl->h_stage = nullptr;
        return record_hip("hipHostMalloc(staging)", e);
    }
    e = hipEventCreateWithFlags(&pl->stage_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipHostFree(pl->h_stage);
        pl->h_stage = nullptr;
        return record_hip("hipEventCreateWithFlags(staging)", e);
    }
    return FABM_OK;
}

// Grow the pinned staging buffer (only between calls, after the last copy
// out of it has completed).
fabm_status ensure_stage(fabm_plan_s *pl, size_t bytes)
{
    if (bytes <= pl->stage_cap) return FABM_OK;
    (void)hipHostFree(pl->h_stage);
    pl->h_stage = nullptr;
    pl->stage_cap = 0;
    HIP_TRY(hipHostMalloc((void **)&pl->h_stage, bytes, hipHostMallocDefault));
    pl->stage_cap = bytes;
    return FABM_OK;
}

fabm_status wait_staging(fabm_plan_s *pl)
{
    if (pl->stage_pending) {
        HIP_TRY(hipEventSynchronize(pl->stage_ev));
        pl->stage_pending = false;
    }
    return FABM_OK;
}

fabm_status stage_copy(fabm_plan_s *pl, size_t bytes, void *dst, hipStream_t s)
{
    HIP_TRY(hipMemcpyAsync(dst, pl->h_stage, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(pl->stage_ev, s));
    pl->stage_pending = true;
    return FABM_OK;
}

// Per-instance placement, order and far-workgroup table of a batched BLOCKED
// call, written into the staging buffer.
const fabm::BatchSchedule &stage_batch(fabm_plan_s *pl, char *stage, const Layout &L,
                                       int64_t batch, const int64_t *N)
{
    const int d = pl->desc.dim;
    const fabm::BatchSchedule &BS = batch_schedule_for(pl, batch, N);
    fabm::BlkInst *hi = (fabm::BlkInst *)(stage + L.inst);
    int64_t fo = 0, ao = 0;
    for (int64_t i = 0; i < batch; ++i) {
        const int nb = blocks_of(N[i]);
        hi[i] = fabm::BlkInst{fo, ao, nb, 0};
        fo += (int64_t)d * nb * fabm::step_block_len();
        ao += (int64_t)2 * d * nb * fabm::step_block_len();
    }
    std::memcpy(stage + L.order, BS.order.data(), sizeof(int) * BS.order.size());
    std::memcpy(stage + L.far_off, BS.far_off.data(), sizeof(int) * BS.far_off.size());
    if (L.far_off_rev)
        std::memcpy(stage + L.far_off_rev, BS.far_off_single.data(),
                    sizeof(int) * BS.far_off_single.size());
    return BS;
}

// Instance entries a call without allocation may stage (on the host stack).
constexpr int kNoAllocStageEntries = 4;

// Shared body of fabm_solve, fabm_solve_batch, fabm_graph_solve_batch and
// fabm_solve_noalloc after validation. `graph_stage` (graph builds only) is a
// pinned buffer owned by the graph: the instance table is written there and
// its copy becomes a node of the graph. With `no_alloc` the table is built on
// the stack and written to the device by one small kernel per entry (no
// pinned buffer, no event, no timer). Otherwise the plan's staging buffer is
// used and guarded by an event.
fabm_status run_solve(fabm_plan_s *pl, void *ws, int64_t batch, const double *alpha,
                      const double *h, const int64_t *N, const double *y0, const double *params,
                      const int64_t *row_off, double *y_out, int64_t *status, hipStream_t s,
                      char *graph_stage = nullptr, bool no_alloc = false)
{
    const int d = pl->desc.dim;
    const Layout L = layout_for(pl, batch, N);
    if (L.path == Path::Unsupported) return FABM_ERR_UNSUPPORTED;
    if (L.path == Path::Wide)
        for (int64_t i = 1; i < batch; ++i)
            if (alpha[i] != alpha[0] || h[i] != h[0] || N[i] != N[0]) return FABM_ERR_UNSUPPORTED;
    alignas(64) char local_stage[sizeof(InstMeta) * kNoAllocStageEntries];
    if (no_alloc && (L.stage_bytes > sizeof(local_stage) || L.stage_bytes % sizeof(InstMeta)))
        return FABM_ERR_UNSUPPORTED;
    fabm_status st = no_alloc ? device_info(pl) : ensure_device(pl);
    if (st != FABM_OK) return st;
    if (!graph_stage && !no_alloc) {
        if ((st = wait_staging(pl)) != FABM_OK) return st;
        if ((st = ensure_stage(pl, L.stage_bytes)) != FABM_OK) return st;
    }
    char *stage = graph_stage ? graph_stage : no_alloc ? local_stage : pl->h_stage;

    InstMeta *hm = (InstMeta *)(stage + L.meta);
    const bool pc = per_component(pl);
    InstMeta *hc = pc ? (InstMeta *)(stage + L.cmeta) : nullptr;
    int64_t w_off = 0, f_off = 0, maxw = 0;
    for (int64_t i = 0; i < batch; ++i) {
        InstMeta &m = hm[i];
        // per-component orders: alpha is [batch][d]; the instance entry takes
        // component 0's scalars (its own weights are never read)
        host_scalars(pc ? alpha[i * d] : alpha[i], h[i], m);
        m.N = N[i];
        m.row_off = row_off ? row_off[i] : 0;
        m.wlen = L.path == Path::Wide ? L.wlen
                 : L.path != Path::Blocked
                     ? N[i]
                     : (batch == 1 ? L.wlen : (int64_t)blocks_of(N[i]) * fabm::step_block_len() +
                                                  fabm::step_block_len());
        m.w_off = w_off;
        m.p_off = (int64_t)pl->n_params * i;
        m.f_off = f_off;
        w_off += 3 * m.wlen;
        if (pc) {
            for (int c = 0; c < d; ++c) {
                InstMeta &q = hc[i * d + c];
                q = m;
                host_scalars(alpha[i * d + c], h[i], q);
                q.w_off = m.w_off + (int64_t)c * 3 * m.wlen;
            }
            w_off += (int64_t)(d - 1) * 3 * m.wlen;
        }
        f_off += N[i] + 1;
        maxw = std::max(maxw, m.wlen);
    }
    char *base = (char *)ws;
    const fabm::BatchSchedule *BS = nullptr;
    if (L.path == Path::Blocked && batch > 1) BS = &stage_batch(pl, stage, L, batch, N);
    if (graph_stage) {
        HIP_TRY(hipMemcpyAsync(base, graph_stage, L.stage_bytes, hipMemcpyHostToDevice, s));
    } else if (no_alloc) {
        // the staged bytes are whole instance entries (checked above)
        const InstMeta *e = (const InstMeta *)stage;
        for (size_t k = 0; k < L.stage_bytes / sizeof(InstMeta); ++k)
            if ((st = ok_or_device(fabm::launch_put_meta(e[k], (InstMeta *)base + k, s))) !=
                FABM_OK)
                return st;
    } else if ((st = stage_copy(pl, L.stage_bytes, base, s)) != FABM_OK) {
        return st;
    }
    const double *y1 = nullptr;
    if ((st = split_init(pl, L, base, batch, y0, y1, s)) != FABM_OK) return st;

    InstMeta *dmeta = (InstMeta *)(base + L.meta);
    double *W = (double *)(base + L.w);
    uint32_t *sync = (uint32_t *)(base + L.sync);
    fabm::KernelTimer *T = pl->timer.on && !graph_stage && !no_alloc ? &pl->timer : nullptr;
    if (T) T->reset();
    if (T) HIP_TRY(T->begin(fabm::KC_WEIGHTS, s));
    const bool f32 = (L.path == Path::Blocked || L.path == Path::Wide) &&
                     pl->desc.far_prec == FABM_FAR_FP32;
    float *W32 = f32 ? (float *)(base + L.w32) : nullptr;
    // the shared grid has one weight table, that of instance 0; per-component
    // orders have one per (instance, component)
    const InstMeta *dcmeta = pc ? (const InstMeta *)(base + L.cmeta) : nullptr;
    if ((st = ok_or_device(fabm::launch_weights(pc ? dcmeta : dmeta,
                                                L.path == Path::Wide ? 1 : pc ? batch * d : batch,
                                                maxw, W, s, W32))) != FABM_OK)
        return st;
    if (T) HIP_TRY(T->end(s));
    if ((st = ok_or_device(fabm::launch_fill_u32(sync, (int64_t)L.n_sync_words, 0u, s))) !=
        FABM_OK)
        return st;
    double *Yi = y_out + (row_off ? row_off[0] : 0) * d;  // single-trajectory kernels

    if (L.path == Path::Wide) {
        fabm::WideArgs A{};
        A.meta = dmeta;
        A.params = params;
        A.y0 = y0;
        A.y1 = y1;
        A.Y = y_out;
        A.W = W;
        A.W32 = W32;
        const fabm_far_prec fp = pl->desc.far_prec;
        A.prec = fp == FABM_FAR_FP64 ? fabm::WIDE_F64
                 : fp == FABM_FAR_FP32 ? fabm::WIDE_F32 : fabm::WIDE_F16X2;
        if (A.prec == fabm::WIDE_F64) A.F = (double *)(base + L.f);
        if (A.prec == fabm::WIDE_F32) A.F32 = (float *)(base + L.f);
        if (A.prec == fabm::WIDE_F16X2) {
            A.Fhi = (_Float16 *)(base + L.f);
            A.Flo = (_Float16 *)(base + L.flo);
            A.Fexp = (int32_t *)(base + L.fexp);
            A.T16 = (const _Float16 *)(base + L.t16);
            A.T16exp = (const int32_t *)(base + L.t16exp);
        }
        A.part = (double *)(base + L.part);
        A.dead = sync;
        A.status = status;
        A.batch = batch;
        A.wlen = L.wlen;
        A.d = d;
        A.cp = (int)L.cp;
        A.NB = L.NB;
        A.split_target = pl->split_target;
        const char *where = "";
        const hipError_t pe = fabm::enqueue_wide(A, s, T, &where);
        if (pe != hipSuccess) return record_hip(where, pe);
        return FABM_OK;
    }

    if (L.path == Path::Blocked && batch > 1) {
        fabm::BatchArgs A{};
        A.meta = dmeta;
        A.cmeta = dcmeta;
        A.inst = (const fabm::BlkInst *)(base + L.inst);
        A.order = (const int *)(base + L.order);
        A.params = params;
        A.y0 = y0;
        A.y1 = y1;
        A.Y = y_out;
        A.W = W;
        A.W32 = W32;
        A.Fc = (double *)(base + L.f);
        A.carry = (double *)(base + L.carry);
        A.acc = (double *)(base + L.acc);
        A.dead = sync;
        A.status = status;
        A.batch = batch;
        const char *where = "";
        const hipError_t pe = fabm::enqueue_batch(pl->desc.system, d, f32, A, *BS,
                                                  (const int *)(base + L.far_off), s, T, &where);
        if (pe != hipSuccess) return record_hip(where, pe);
        return FABM_OK;
    }
    if (L.path == Path::Blocked) {
        fabm::StepArgs A{};
        A.meta = dmeta;
        A.m0 = hm[0];
        A.cmeta = dcmeta;
        A.params = params;
        A.y0 = y0;
        A.y1 = y1;
        A.Y = Yi;
        A.W = W;
        A.W32 = W32;
        A.Fc = (double *)(base + L.f);
        A.carry = (double *)(base + L.carry);
        A.acc = (double *)(base + L.acc);
        A.dead = sync;
        A.status = status;
        A.NB = L.NB;
        A.far_cap = pl->far_cap;
        A.fft_level = pl->desc.fft_level;
        A.wlen = L.wlen;
        A.fft_tw = (double2 *)(base + L.ftw);
        A.fft_buf = (double2 *)(base + L.fbuf);
        A.fft_spec = (double2 *)(base + L.fspec);
        const char *where = "";
        const hipError_t pe = fabm::enqueue_steps(pl->desc.system, d, f32, A, s, T, &where);
        if (pe != hipSuccess) return record_hip(where, pe);
        return FABM_OK;
    }
    double *F = (double *)(base + L.f);
    if (batch == 1 && N[0] >= kGridDirectMinSteps) {
        double *part = (double *)(base + L.part);
        // every partial slot starts marked empty
        if ((st = ok_or_device(fabm::launch_fill_u32(
                 (uint32_t *)part, (int64_t)(2 * fabm::direct_grid_part_doubles(kGridMax)),
                 fabm::direct_grid_empty_word(), s))) != FABM_OK)
            return st;
        if (T) HIP_TRY(T->begin(fabm::KC_DIRECT_GRID, s));
        st = ok_or_device(fabm::launch_direct_grid(pl->desc.system, d, pl->grid_G, dmeta, dcmeta,
                                                   params, y0, y1, F, W, Yi, status, part, sync,
                                                   pl->timeout_ticks, s));
        if (T) HIP_TRY(T->end(s));
        return st;
    }
    if (T) HIP_TRY(T->begin(fabm::KC_DIRECT_WG, s));
    st = ok_or_device(fabm::launch_direct_wg(pl->desc.system, d, dmeta, dcmeta, batch, params, y0,
                                             y1, F, W, y_out, status, s));
    if (T) HIP_TRY(T->end(s));
    return st;
}

// Body of fabm_adjoint after validation: forward pass (batched BLOCKED, FP64)
// into the workspace with predictor rows, then the reverse pipeline.
// Phases of the adjoint: both passes, the forward pass only (trajectory also
// copied to the caller's rows), or the reverse pass on the workspace a forward
// phase left.
enum class AdjPhase { Both, Forward, Reverse };

fabm_status run_adjoint(fabm_plan_s *pl, void *ws, int64_t batch, const double *alpha,
                        const double *h, const int64_t *N, const double *y0,
                        const double *params, const int64_t *row_off, const double *gy,
                        double *gy0, double *gparams, int64_t *status, hipStream_t s,
                        AdjPhase phase = AdjPhase::Both, double *y_out = nullptr)
{
    const int d = pl->desc.dim;
    if (pl->desc.fft_level > 0) return FABM_ERR_UNSUPPORTED;  // the reverse pass has no FFT form
    const Layout L = layout_for(pl, batch, N, true);
    fabm_status st = ensure_device(pl);
    if (st != FABM_OK) return st;
    if ((st = wait_staging(pl)) != FABM_OK) return st;
    if ((st = ensure_stage(pl, L.stage_bytes)) != FABM_OK) return st;
    InstMeta *hm = (InstMeta *)(pl->h_stage + L.meta);
    InstMeta *ham = (InstMeta *)(pl->h_stage + L.meta_adj);
    const bool pc = per_component(pl);
    InstMeta *hc = pc ? (InstMeta *)(pl->h_stage + L.cmeta) : nullptr;
    int64_t w_off = 0, f_off = 0, maxw = 0;
    for (int64_t i = 0; i < batch; ++i) {
        InstMeta &m = hm[i];
        host_scalars(pc ? alpha[i * d] : alpha[i], h[i], m);
        m.N = N[i];
        m.wlen = (int64_t)blocks_of(N[i]) * fabm::step_block_len() + fabm::step_block_len();
        m.w_off = w_off;
        m.p_off = (int64_t)pl->n_params * i;
        m.f_off = f_off;
        m.row_off = f_off;  // the forward rows go to the workspace, packed
        ham[i] = m;
        ham[i].row_off = row_off[i];  // dL/dy rows are the caller's
        w_off += 3 * m.wlen;
        if (pc) {
            for (int c = 0; c < d; ++c) {
                InstMeta &q = hc[i * d + c];
                q = m;
                host_scalars(alpha[i * d + c], h[i], q);
                q.w_off = m.w_off + (int64_t)c * 3 * m.wlen;
            }
            w_off += (int64_t)(d - 1) * 3 * m.wlen;
        }
        f_off += N[i] + 1;
        maxw = std::max(maxw, m.wlen);
    }
    const fabm::BatchSchedule &BS = stage_batch(pl, pl->h_stage, L, batch, N);
    char *base = (char *)ws;
    if ((st = stage_copy(pl, L.stage_bytes, base, s)) != FABM_OK) return st;
    const double *y1 = nullptr;
    if ((st = split_init(pl, L, base, batch, y0, y1, s)) != FABM_OK) return st;
    InstMeta *dmeta = (InstMeta *)(base + L.meta);
    double *W = (double *)(base + L.w);
    uint32_t *sync = (uint32_t *)(base + L.sync);
    fabm::KernelTimer *T = pl->timer.on ? &pl->timer : nullptr;
    if (T) T->reset();
    const InstMeta *dcmeta = pc ? (const InstMeta *)(base + L.cmeta) : nullptr;
    if (phase != AdjPhase::Reverse) {
        if (T) HIP_TRY(T->begin(fabm::KC_WEIGHTS, s));
        if ((st = ok_or_device(fabm::launch_weights(pc ? dcmeta : dmeta, pc ? batch * d : batch,
                                                    maxw, W, s))) != FABM_OK)
            return st;
        if (T) HIP_TRY(T->end(s));
        if ((st = ok_or_device(fabm::launch_fill_u32(sync, (int64_t)L.n_sync_words, 0u, s))) !=
            FABM_OK)
            return st;
    }
    // block checkpoints: the forward keeps no predictor rows and its rows go
    // straight to the caller (or nowhere); the reverse pass re-forms them
    const bool ckpt = adjoint_checkpoint(pl);
    const InstMeta *dmeta_adj = (const InstMeta *)(base + L.meta_adj);
    fabm::BatchArgs A{};
    A.meta = ckpt && phase == AdjPhase::Forward ? dmeta_adj : dmeta;
    A.cmeta = dcmeta;
    A.inst = (const fabm::BlkInst *)(base + L.inst);
    A.order = (const int *)(base + L.order);
    A.params = params;
    A.y0 = y0;
    A.y1 = y1;
    A.Y = !ckpt ? (double *)(base + L.yw) : phase == AdjPhase::Forward ? y_out : nullptr;
    A.YP = ckpt ? nullptr : (double *)(base + L.ypw);
    A.W = W;
    A.Fc = (double *)(base + L.f);
    A.carry = (double *)(base + L.carry);
    A.acc = (double *)(base + L.acc);
    A.dead = sync;
    A.status = status;
    A.batch = batch;
    const int *far_off = (const int *)(base + L.far_off);
    const char *where = "";
    hipError_t pe = hipSuccess;
    if (phase != AdjPhase::Reverse) {
        pe = fabm::enqueue_batch(pl->desc.system, d, false, A, BS, far_off, s, T, &where);
        if (pe != hipSuccess) return record_hip(where, pe);
    }
    if (phase == AdjPhase::Forward && ckpt) return FABM_OK;  // rows already in y_out
    if (phase == AdjPhase::Forward) {
        int64_t maxr = 0;
        for (int64_t i = 0; i < batch; ++i) maxr = std::max(maxr, N[i] + 1);
        return ok_or_device(fabm::launch_copy_rows(dmeta, (const InstMeta *)(base + L.meta_adj),
                                                   batch, maxr, d, A.Y, y_out, s));
    }
    fabm::AdjArgs R{};
    R.meta = (const InstMeta *)(base + L.meta_adj);
    R.cmeta = dcmeta;
    R.inst = A.inst;
    R.order = A.order;
    R.params = params;
    R.y0 = y0;
    R.Y = (double *)(base + L.yw);
    R.YP = (double *)(base + L.ypw);
    R.ring = ckpt ? fabm::kCkptGroup + 1 : 0;
    R.G = gy;
    R.W = W;
    R.UV = (double *)(base + L.uv);
    R.carry = (double *)(base + L.carry_a);
    R.acc = (double *)(base + L.acc_a);
    R.part = (double *)(base + L.part_a);
    R.fbar0 = (double *)(base + L.fbar0);
    R.dead = sync;
    R.gy0 = gy0;
    R.slope = y1 != nullptr;
    R.gparams = gparams;
    R.batch = batch;
    fabm::BatchSchedule Sr = BS;  // one source block per launch
    Sr.far_off = BS.far_off_single;
    fabm::RecompArgs RC{};
    RC.ringY = (double *)(base + L.yw);
    RC.ringYP = (double *)(base + L.ypw);
    RC.rcarry = (double *)(base + L.rcarry);
    RC.G = fabm::kCkptGroup;
    A.meta = dmeta;  // the re-formed rows go to the ring, not to the caller
    pe = fabm::enqueue_adjoint(pl->desc.system, d, R, Sr, (const int *)(base + L.far_off_rev), s,
                               T, &where, ckpt ? &A : nullptr, ckpt ? &RC : nullptr);
    if (pe != hipSuccess) return record_hip(where, pe);
    return FABM_OK;
}

// Checks shared by the batched entry points.
fabm_status check_batch(const fabm_plan_s *plan, int64_t batch, const double *alpha,
                        const double *h, const int64_t *N, const int64_t *row_off)
{
    if (!plan || !alpha || !h || !N || !row_off) return FABM_ERR_INVALID_ARG;
    if (batch < 1 || batch > plan->desc.max_batch) return FABM_ERR_INVALID_ARG;
    const int64_t total_cap = plan->desc.max_total_steps
                                  ? plan->desc.max_total_steps
                                  : plan->desc.max_batch * plan->desc.max_steps;
    int64_t sumN = 0;
    std::vector<std::pair<int64_t, int64_t>> spans((size_t)batch);
    const int na = per_component(plan) ? plan->desc.dim : 1;  // orders per instance
    for (int64_t i = 0; i < batch; ++i) {
        for (int c = 0; c < na; ++c) {
            fabm_status st = check_alpha_h(alpha[i * na + c], h[i], has_slope(plan));
            if (st != FABM_OK) return st;
        }
        if (N[i] < 1 || N[i] > plan->desc.max_steps || row_off[i] < 0)
            return FABM_ERR_INVALID_ARG;
        sumN += N[i];
        spans[(size_t)i] = {row_off[i], row_off[i] + N[i] + 1};
    }
    if (sumN > total_cap) return FABM_ERR_INVALID_ARG;
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return FABM_ERR_INVALID_ARG;
    return FABM_OK;
}

}  // namespace

extern "C" {

const char *fabm_last_error(void) { return g_last_error; }

const char *fabm_status_string(fabm_status s)
{
    switch (s) {
    case FABM_OK: return "ok";
    case FABM_ERR_INVALID_ARG: return "invalid argument";
    case FABM_ERR_UNSUPPORTED: return "unsupported";
    case FABM_ERR_WORKSPACE: return "workspace too small";
    case FABM_ERR_DEVICE: return "device error";
    default: return "unknown status";
    }
}

int32_t fabm_n_params(fabm_system system, int32_t dim) { return n_params_of(system, dim); }

fabm_status fabm_plan(const fabm_plan_desc *desc, fabm_plan_t *out, size_t *workspace_bytes)
{
    if (!desc || !out) return FABM_ERR_INVALID_ARG;
    *out = nullptr;
    const int32_t np = n_params_of(desc->system, desc->dim);
    if (np < 0) return FABM_ERR_INVALID_ARG;
    if (desc->max_batch < 1 || desc->max_steps < 1 || desc->max_total_steps < 0 ||
        (desc->flags & ~(FABM_PLAN_INITIAL_SLOPE | FABM_PLAN_PER_COMPONENT_ORDER |
                         FABM_PLAN_ADJOINT_CHECKPOINT)) != 0 ||
        desc->max_steps > ((int64_t)1 << 30))
        return FABM_ERR_INVALID_ARG;
    if (desc->tile_L < 0 || desc->tile_L % 64 != 0) return FABM_ERR_INVALID_ARG;
    if (desc->path != FABM_PATH_AUTO && desc->path != FABM_PATH_DIRECT &&
        desc->path != FABM_PATH_BLOCKED)
        return FABM_ERR_INVALID_ARG;
    if (desc->far_prec != FABM_FAR_FP64 && desc->far_prec != FABM_FAR_FP32 &&
        desc->far_prec != FABM_FAR_FP16X2)
        return FABM_ERR_INVALID_ARG;
    // split binary16 far tiles and the 64-row blocks exist in the shared-grid
    // form only (LINEAR); the per-trajectory kernels keep the state in
    // registers (LINEAR up to d = 4) and use 256-row blocks
    const bool wide = wide_plan(*desc);
    if (desc->far_prec == FABM_FAR_FP16X2 && desc->system != FABM_SYS_LINEAR)
        return FABM_ERR_UNSUPPORTED;
    if (desc->tile_L != 0 && desc->tile_L != (wide ? fabm::kWideBlk : fabm::step_block_len()))
        return FABM_ERR_UNSUPPORTED;
    if (wide && desc->path == FABM_PATH_DIRECT) return FABM_ERR_UNSUPPORTED;
    // per-component orders: DIRECT, or BLOCKED per trajectory (FP64 or FP32 windows)
    if ((desc->flags & FABM_PLAN_PER_COMPONENT_ORDER) && wide) return FABM_ERR_UNSUPPORTED;
    if (wide && desc->max_batch > kWideMaxCols / desc->dim) return FABM_ERR_UNSUPPORTED;
    // sub-quadratic far history: one BLOCKED trajectory (FP64 or FP32 windows)
    if (desc->fft_level < 0 || desc->fft_level > 15) return FABM_ERR_INVALID_ARG;
    if (desc->fft_level > 0 &&
        (wide || desc->path != FABM_PATH_BLOCKED || desc->max_batch != 1 ||
         desc->max_steps > ((int64_t)1 << 24)))
        return FABM_ERR_UNSUPPORTED;

    fabm_plan_s *pl = new (std::nothrow) fabm_plan_s();
    if (!pl) return FABM_ERR_INVALID_ARG;
    pl->desc = *desc;
    pl->n_params = np;
    pl->grid_G = kGridMax;
    if (workspace_bytes) {
        const int64_t total =
            desc->max_total_steps ? desc->max_total_steps : desc->max_batch * desc->max_steps;
        std::vector<int64_t> Ns((size_t)desc->max_batch, 0);
        int64_t left = total;
        for (auto &n : Ns) {
            n = std::max<int64_t>(1, std::min(desc->max_steps, left));
            left -= n;
        }
        size_t ws = layout_for(pl, desc->max_batch, Ns.data()).total;
        int64_t one = desc->max_steps;
        ws = std::max(ws, layout_for(pl, 1, &one).total);
        *workspace_bytes = ws;
    }
    *out = pl;
    return FABM_OK;
}

void fabm_plan_destroy(fabm_plan_t plan)
{
    if (!plan) return;
    if (plan->h_stage) {
        if (plan->stage_pending) (void)hipEventSynchronize(plan->stage_ev);
        (void)hipEventDestroy(plan->stage_ev);
        (void)hipHostFree(plan->h_stage);
    }
    delete plan;
}

fabm_status fabm_workspace_size(fabm_plan_t plan, int64_t batch, const int64_t *N, size_t *bytes)
{
    if (!plan || !N || !bytes || batch < 1 || batch > plan->desc.max_batch)
        return FABM_ERR_INVALID_ARG;
    for (int64_t i = 0; i < batch; ++i)
        if (N[i] < 1 || N[i] > plan->desc.max_steps) return FABM_ERR_INVALID_ARG;
    const Layout L = layout_for(plan, batch, N);
    if (L.path == Path::Unsupported) return FABM_ERR_UNSUPPORTED;
    *bytes = L.total;
    return FABM_OK;
}

fabm_status fabm_solve(fabm_plan_t plan, void *workspace, size_t workspace_bytes, double alpha,
                       double h, int64_t N, const double *y0, const double *params,
                       double *y_out, int64_t *status, hipStream_t stream)
{
    if (!plan) return FABM_ERR_INVALID_ARG;
    // one alpha per component comes through the batched entry points
    if (per_component(plan)) return FABM_ERR_UNSUPPORTED;
    fabm_status st = check_alpha_h(alpha, h, has_slope(plan));
    if (st != FABM_OK) return st;
    if (N < 1 || N > plan->desc.max_steps) return FABM_ERR_INVALID_ARG;
    if (!aligned8(y0) || !aligned8(y_out) || !aligned8(status)) return FABM_ERR_INVALID_ARG;
    if (plan->n_params > 0 && !aligned8(params)) return FABM_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return FABM_ERR_WORKSPACE;
    if (workspace_bytes < layout_for(plan, 1, &N).total) return FABM_ERR_WORKSPACE;
    return run_solve(plan, workspace, 1, &alpha, &h, &N, y0, params, nullptr, y_out, status,
                     stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Solves without allocation (fabm_solve_noalloc): the workspace is this
// file-scope device array. Each device the library runs on holds its own copy
// (FABM_NOALLOC_SCRATCH_BYTES) until the process ends. In host code `scratch`
// names a host-side stand-in, never the device memory: the device address is
// taken once per device with hipGetSymbolAddress and only that address is
// passed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[FABM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices];  // device address of `scratch`, per device

// Device address of the current device's scratch array, looked up on the
// first call on that device (with it current).
fabm_status scratch_address(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return FABM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p % kAlign) != 0) {
            std::snprintf(g_last_error, sizeof g_last_error,
                          "hipGetSymbolAddress(scratch): unusable address %p", p);
            return FABM_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FABM_OK;
}

}  // namespace

extern "C" {

fabm_status fabm_solve_noalloc(fabm_plan_t plan, double alpha, double h, int64_t N,
                               const double *y0, const double *params, double *y_out,
                               int64_t *status, hipStream_t stream)
{
    g_last_error[0] = '\0';
    if (!plan) return FABM_ERR_INVALID_ARG;
    if (per_component(plan)) return FABM_ERR_UNSUPPORTED;
    fabm_status st = check_alpha_h(alpha, h, has_slope(plan));
    if (st != FABM_OK) return st;
    if (N < 1 || N > plan->desc.max_steps) return FABM_ERR_INVALID_ARG;
    if (!aligned8(y0) || !aligned8(y_out) || !aligned8(status)) return FABM_ERR_INVALID_ARG;
    if (plan->n_params > 0 && !aligned8(params)) return FABM_ERR_INVALID_ARG;
    // the per-trajectory paths only: the shared grid and the FFT far history
    // stage more than one instance entry or build tables with library calls
    if (plan->desc.fft_level > 0) return FABM_ERR_UNSUPPORTED;
    const Layout L = layout_for(plan, 1, &N);
    if (L.path != Path::Blocked && L.path != Path::Direct) return FABM_ERR_UNSUPPORTED;
    if (L.total > (size_t)FABM_NOALLOC_SCRATCH_BYTES) {
        std::snprintf(g_last_error, sizeof g_last_error,
                      "fabm_solve_noalloc: N = %lld needs %zu bytes of scratch, the library "
                      "holds %zu",
                      (long long)N, L.total, (size_t)FABM_NOALLOC_SCRATCH_BYTES);
        return FABM_ERR_WORKSPACE;
    }
    void *ws = nullptr;
    if ((st = scratch_address(&ws)) != FABM_OK) return st;
    return run_solve(plan, ws, 1, &alpha, &h, &N, y0, params, nullptr, y_out, status, stream,
                     nullptr, true);
}

fabm_status fabm_solve_batch(fabm_plan_t plan, void *workspace, size_t workspace_bytes,
                             int64_t batch, const double *alpha, const double *h,
                             const int64_t *N, const double *y0, const double *params,
                             const int64_t *row_off, double *y_out, int64_t *status,
                             hipStream_t stream)
{
    fabm_status cst = check_batch(plan, batch, alpha, h, N, row_off);
    if (cst != FABM_OK) return cst;
    if (!aligned8(y0) || !aligned8(y_out) || !aligned8(status)) return FABM_ERR_INVALID_ARG;
    if (plan->n_params > 0 && !aligned8(params)) return FABM_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return FABM_ERR_WORKSPACE;
    const Layout L = layout_for(plan, batch, N);
    if (L.path == Path::Unsupported) return FABM_ERR_UNSUPPORTED;
    if (workspace_bytes < L.total) return FABM_ERR_WORKSPACE;
    return run_solve(plan, workspace, batch, alpha, h, N, y0, params, row_off, y_out, status,
                     stream);
}

fabm_status fabm_graph_solve_batch(fabm_plan_t plan, void *workspace, size_t workspace_bytes,
                                   int64_t batch, const double *alpha, const double *h,
                                   const int64_t *N, const double *y0, const double *params,
                                   const int64_t *row_off, double *y_out, int64_t *status,
                                   fabm_graph_t *out)
{
    if (!out) return FABM_ERR_INVALID_ARG;
    *out = nullptr;
    fabm_status st = check_batch(plan, batch, alpha, h, N, row_off);
    if (st != FABM_OK) return st;
    if (!aligned8(y0) || !aligned8(y_out) || !aligned8(status)) return FABM_ERR_INVALID_ARG;
    if (plan->n_params > 0 && !aligned8(params)) return FABM_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return FABM_ERR_WORKSPACE;
    const Layout L = layout_for(plan, batch, N);
    if (L.path == Path::Unsupported) return FABM_ERR_UNSUPPORTED;
    if (workspace_bytes < L.total) return FABM_ERR_WORKSPACE;
    if (L.path == Path::Wide)
        for (int64_t i = 1; i < batch; ++i)
            if (alpha[i] != alpha[0] || h[i] != h[0] || N[i] != N[0]) return FABM_ERR_UNSUPPORTED;
    // the whole-GPU DIRECT kernel relies on a cooperative launch (all
    // workgroups resident at once), which is not recorded into graphs here
    if (L.path == Path::Direct && batch == 1 && N[0] >= kGridDirectMinSteps)
        return FABM_ERR_UNSUPPORTED;
    if ((st = ensure_device(plan)) != FABM_OK) return st;

    fabm_graph_s *g = new (std::nothrow) fabm_graph_s();
    if (!g) return FABM_ERR_DEVICE;
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipError_t e = hipHostMalloc((void **)&g->stage, std::max<size_t>(L.stage_bytes, 64),
                                 hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        st = record_hip("fabm_graph_solve_batch: staging or stream", e);
    } else if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed)) != hipSuccess) {
        st = record_hip("hipStreamBeginCapture", e);
    } else {
        st = run_solve(plan, workspace, batch, alpha, h, N, y0, params, row_off, y_out, status,
                       cs, g->stage);
        // the capture is ended whatever happened inside it
        e = hipStreamEndCapture(cs, &graph);
        if (st == FABM_OK && e != hipSuccess) st = record_hip("hipStreamEndCapture", e);
        if (st == FABM_OK) {
            e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) st = record_hip("hipGraphInstantiate", e);
        }
    }
    if (cs) (void)hipStreamDestroy(cs);
    g->graph = graph;
    if (st != FABM_OK) {
        fabm_graph_destroy(g);
        return st;
    }
    *out = g;
    return FABM_OK;
}

fabm_status fabm_graph_launch(fabm_graph_t graph, hipStream_t stream)
{
    if (!graph || !graph->exec) return FABM_ERR_INVALID_ARG;
    return record_hip("hipGraphLaunch", hipGraphLaunch(graph->exec, stream));
}

void fabm_graph_destroy(fabm_graph_t graph)
{
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    if (graph->stage) (void)hipHostFree(graph->stage);
    delete graph;
}

fabm_status fabm_tune(fabm_plan_t plan, void *workspace, size_t workspace_bytes, int64_t batch,
                      const double *alpha, const double *h, const int64_t *N, const double *y0,
                      const double *params, const int64_t *row_off, double *y_out,
                      int64_t *status, hipStream_t stream, fabm_tune_report *report)
{
    fabm_status st = check_batch(plan, batch, alpha, h, N, row_off);
    if (st != FABM_OK) return st;
    if (!aligned8(y0) || !aligned8(y_out) || !aligned8(status)) return FABM_ERR_INVALID_ARG;
    if (plan->n_params > 0 && !aligned8(params)) return FABM_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return FABM_ERR_WORKSPACE;
    const Layout L = layout_for(plan, batch, N);
    if (L.path == Path::Unsupported) return FABM_ERR_UNSUPPORTED;
    if (workspace_bytes < L.total) return FABM_ERR_WORKSPACE;

    fabm_tune_report rep{};
    int *knob = nullptr;
    static const int kCaps[] = {32, 64, 128, fabm::kMaxFarWg};
    static const int kTargets[] = {256, 512, 1024, 2048, fabm::kWideMaxSplitTarget};
    static const int kGroups[] = {1, 2, 4};
    const int *cand = nullptr;
    if (L.path == Path::Blocked && batch > 1) {
        rep.knob = FABM_TUNE_SOURCE_GROUP;
        knob = &plan->batch_group;
        cand = kGroups;
        rep.n = (int32_t)(sizeof kGroups / sizeof kGroups[0]);
    } else if (L.path == Path::Blocked && batch == 1) {
        rep.knob = FABM_TUNE_FAR_WORKGROUPS;
        knob = &plan->far_cap;
        cand = kCaps;
        rep.n = (int32_t)(sizeof kCaps / sizeof kCaps[0]);
    } else if (L.path == Path::Wide) {
        rep.knob = FABM_TUNE_SPLIT_TARGET;
        knob = &plan->split_target;
        cand = kTargets;
        rep.n = (int32_t)(sizeof kTargets / sizeof kTargets[0]);
    }
    if (!knob) {  // nothing to choose on this path
        rep.knob = FABM_TUNE_NONE;
        if (report) *report = rep;
        return FABM_OK;
    }
    const int keep = *knob;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return record_hip("hipEventCreate", he);
    }
    const bool prof = plan->timer.on;
    plan->timer.on = false;
    // one untimed run first (first-touch of the workspace, code objects)
    st = run_solve(plan, workspace, batch, alpha, h, N, y0, params, row_off, y_out, status, stream);
    int best = -1;
    for (int c = 0; st == FABM_OK && c < rep.n; ++c) {
        *knob = cand[c];
        rep.value[c] = cand[c];
        if ((st = record_hip("hipEventRecord", hipEventRecord(e0, stream))) != FABM_OK) break;
        st = run_solve(plan, workspace, batch, alpha, h, N, y0, params, row_off, y_out, status,
                       stream);
        if (st != FABM_OK) break;
        if ((st = record_hip("hipEventRecord", hipEventRecord(e1, stream))) != FABM_OK) break;
        if ((st = record_hip("hipEventSynchronize", hipEventSynchronize(e1))) != FABM_OK) break;
        float ms = 0.0f;
        if ((st = record_hip("hipEventElapsedTime", hipEventElapsedTime(&ms, e0, e1))) != FABM_OK)
            break;
        rep.seconds[c] = 1e-3 * (double)ms;
        if (best < 0 || rep.seconds[c] < rep.seconds[best]) best = c;
    }
    plan->timer.on = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FABM_OK || best < 0) {
        *knob = keep;
        return st != FABM_OK ? st : FABM_ERR_DEVICE;
    }
    *knob = cand[best];
    rep.chosen = best;
    if (report) *report = rep;
    return FABM_OK;
}

fabm_status fabm_adjoint_workspace_size(fabm_plan_t plan, int64_t batch, const int64_t *N,
                                        size_t *bytes)
{
    if (!plan || !N || !bytes || batch < 1 || batch > plan->desc.max_batch)
        return FABM_ERR_INVALID_ARG;
    for (int64_t i = 0; i < batch; ++i)
        if (N[i] < 1 || N[i] > plan->desc.max_steps) return FABM_ERR_INVALID_ARG;
    if (plan->desc.system == FABM_SYS_LINEAR && plan->desc.dim > 4) return FABM_ERR_UNSUPPORTED;
    if (plan->desc.fft_level > 0) return FABM_ERR_UNSUPPORTED;
    *bytes = layout_for(plan, batch, N, true).total;
    return FABM_OK;
}

fabm_status fabm_adjoint(fabm_plan_t plan, void *workspace, size_t workspace_bytes, int64_t batch,
                         const double *alpha, const double *h, const int64_t *N,
                         const double *y0, const double *params, const int64_t *row_off,
                         const double *gy, double *gy0, double *gparams, int64_t *status,
                         hipStream_t stream)
{
    fabm_status st = check_batch(plan, batch, alpha, h, N, row_off);
    if (st != FABM_OK) return st;
    if (!aligned8(y0) || !aligned8(gy) || !aligned8(gy0) || !aligned8(status))
        return FABM_ERR_INVALID_ARG;
    if (plan->n_params > 0 && (!aligned8(params) || !aligned8(gparams)))
        return FABM_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return FABM_ERR_WORKSPACE;
    size_t need = 0;
    if ((st = fabm_adjoint_workspace_size(plan, batch, N, &need)) != FABM_OK) return st;
    if (workspace_bytes < need) return FABM_ERR_WORKSPACE;
    return run_adjoint(plan, workspace, batch, alpha, h, N, y0, params, row_off, gy, gy0, gparams,
                       status, stream);
}

fabm_status fabm_adjoint_forward(fabm_plan_t plan, void *workspace, size_t workspace_bytes,
                                 int64_t batch, const double *alpha, const double *h,
                                 const int64_t *N, const double *y0, const double *params,
                                 const int64_t *row_off, double *y_out, int64_t *status,
                                 hipStream_t stream)
{
    fabm_status st = check_batch(plan, batch, alpha, h, N, row_off);
    if (st != FABM_OK) return st;
    if (!aligned8(y0) || !aligned8(y_out) || !aligned8(status)) return FABM_ERR_INVALID_ARG;
    if (plan->n_params > 0 && !aligned8(params)) return FABM_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return FABM_ERR_WORKSPACE;
    size_t need = 0;
    if ((st = fabm_adjoint_workspace_size(plan, batch, N, &need)) != FABM_OK) return st;
    if (workspace_bytes < need) return FABM_ERR_WORKSPACE;
    return run_adjoint(plan, workspace, batch, alpha, h, N, y0, params, row_off, nullptr,
                       nullptr, nullptr, status, stream, AdjPhase::Forward, y_out);
}

fabm_status fabm_adjoint_reverse(fabm_plan_t plan, void *workspace, size_t workspace_bytes,
                                 int64_t batch, const double *alpha, const double *h,
                                 const int64_t *N, const double *y0, const double *params,
                                 const int64_t *row_off, const double *gy, double *gy0,
                                 double *gparams, hipStream_t stream)
{
    fabm_status st = check_batch(plan, batch, alpha, h, N, row_off);
    if (st != FABM_OK) return st;
    if (!aligned8(y0) || !aligned8(gy) || !aligned8(gy0)) return FABM_ERR_INVALID_ARG;
    if (plan->n_params > 0 && (!aligned8(params) || !aligned8(gparams)))
        return FABM_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return FABM_ERR_WORKSPACE;
    size_t need = 0;
    if ((st = fabm_adjoint_workspace_size(plan, batch, N, &need)) != FABM_OK) return st;
    if (workspace_bytes < need) return FABM_ERR_WORKSPACE;
    return run_adjoint(plan, workspace, batch, alpha, h, N, y0, params, row_off, gy, gy0,
                       gparams, nullptr, stream, AdjPhase::Reverse);
}

fabm_status fabm_weights(double alpha, int64_t n, double *b, double *a, double *c,
                         hipStream_t stream)
{
    fabm_status st = check_alpha_h(alpha, 1.0, true);
    if (st != FABM_OK) return st;
    if (n < 1) return FABM_ERR_INVALID_ARG;
    if ((b && !aligned8(b)) || (a && !aligned8(a)) || (c && !aligned8(c)))
        return FABM_ERR_INVALID_ARG;
    InstMeta m{};
    host_scalars(alpha, 1.0, m);
    return ok_or_device(fabm::launch_weights_one(alpha, m.ig1, m.ig2, n, b, a, c, stream));
}

fabm_status fabm_plan_set_profiling(fabm_plan_t plan, int32_t enable)
{
    if (!plan) return FABM_ERR_INVALID_ARG;
    plan->timer.on = enable != 0;
    return FABM_OK;
}

fabm_status fabm_plan_kernel_times(fabm_plan_t plan, double *seconds, int64_t *launches)
{
    if (!plan || !seconds || !launches) return FABM_ERR_INVALID_ARG;
    return ok_or_device(plan->timer.totals(seconds, launches, fabm::KC_COUNT));
}

}  // extern "C"

namespace {

// Workspace of the teacher-forced BLOCKED contraction (offsets in bytes): the
// step pipeline of one trajectory run on the internal system that reads f
// from the given history, with the grid step 1 (so h^alpha = 1 and the
// returned rows are the plain sums).
struct HistLayout {
    size_t meta, w, w32, f, carry, acc, sync, st, ftf, yc, yp, y0, total;
    int64_t wlen;
    int NB;
};

HistLayout hist_layout(int64_t N, int d)
{
    HistLayout H{};
    const int Lb = fabm::step_block_len();
    H.NB = blocks_of(N);
    H.wlen = (int64_t)H.NB * Lb + Lb;
    const size_t blk = sizeof(double) * 2 * d * (size_t)Lb;
    const size_t rows = sizeof(double) * (size_t)d * (size_t)(N + 1);
    size_t off = 0;
    H.meta = off;
    off = align_up(off + sizeof(InstMeta));
    H.w = off;
    off = align_up(off + sizeof(double) * 3 * (size_t)H.wlen);
    H.w32 = off;
    off = align_up(off + sizeof(float) * 2 * (size_t)H.wlen);
    H.f = off;
    off = align_up(off + sizeof(double) * (size_t)d * (size_t)H.NB * Lb);
    H.carry = off;
    off = align_up(off + 2 * blk);
    H.acc = off;
    off = align_up(off + blk * (size_t)H.NB);
    H.sync = off;
    off = align_up(off + sizeof(uint32_t) * 64);
    H.st = off;
    off = align_up(off + sizeof(int64_t));
    H.ftf = off;  // the given history and a zero row N
    off = align_up(off + rows);
    H.yc = off;   // corrector sums, rows 0..N (row t holds target t)
    off = align_up(off + rows);
    H.yp = off;   // predictor sums
    off = align_up(off + rows);
    H.y0 = off;   // zero initial state
    off = align_up(off + sizeof(double) * (size_t)d);
    H.total = off;
    return H;
}

}  // namespace

extern "C" {

size_t fabm_history_workspace_size(int64_t N, int32_t dim)
{
    if (N < 1 || dim < 1 || dim > 4) return 0;
    const size_t direct = align_up(sizeof(double) * 3 * (size_t)N);
    return std::max(direct, hist_layout(N, dim).total);
}

fabm_status fabm_fft_far_schedule(int32_t NB, int32_t level, int32_t s, int32_t *jend,
                                  int32_t *skip_prev, int32_t *square)
{
    if (!jend || !skip_prev || !square || NB < 1 || s < -1 || s > NB - 2 || level < 0 ||
        level > 15)
        return FABM_ERR_INVALID_ARG;
    // the same decisions as the step pipeline's enqueue
    const bool fft = level > 0 && fabm::fft_far_top_level(NB, level) >= 0;
    *jend = fft ? fabm::fft_far_target_end(NB, level, s) : NB;
    *skip_prev = fft && fabm::fft_far_mask_prev(level, s) ? 1 : 0;
    *square = fft ? fabm::fft_far_square_at(NB, level, s) : -1;
    return FABM_OK;
}

fabm_status fabm_history_sums(double alpha, int64_t N, int32_t dim, const double *f, double *P,
                              double *C, fabm_path path, fabm_far_prec far_prec,
                              void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    fabm_status st = check_alpha_h(alpha, 1.0, true);
    if (st != FABM_OK) return st;
    if (N < 1 || dim < 1) return FABM_ERR_INVALID_ARG;
    if (dim > 4) return FABM_ERR_UNSUPPORTED;
    if (!aligned8(f) || !aligned8(P) || !aligned8(C)) return FABM_ERR_INVALID_ARG;
    if (far_prec != FABM_FAR_FP64 && far_prec != FABM_FAR_FP32 && far_prec != FABM_FAR_FP16X2)
        return FABM_ERR_INVALID_ARG;
    if (path != FABM_PATH_AUTO && path != FABM_PATH_DIRECT && path != FABM_PATH_BLOCKED)
        return FABM_ERR_INVALID_ARG;
    if (path != FABM_PATH_DIRECT && far_prec == FABM_FAR_FP16X2) return FABM_ERR_UNSUPPORTED;
    if (N > kMaxHistorySteps) return FABM_ERR_UNSUPPORTED;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0 ||
        workspace_bytes < fabm_history_workspace_size(N, dim))
        return FABM_ERR_WORKSPACE;
    InstMeta m{};
    host_scalars(alpha, 1.0, m);
    if (path == FABM_PATH_DIRECT) {
        double *W = (double *)workspace;
        if ((st = ok_or_device(fabm::launch_weights_one(alpha, m.ig1, m.ig2, N, W, W + N,
                                                        W + 2 * N, stream))) != FABM_OK)
            return st;
        return ok_or_device(fabm::launch_history_direct(W, N, dim, f, P, C, stream));
    }
    // BLOCKED: the step pipeline (band, near and far MFMA windows) with f read
    // from the given rows; h = 1 makes h^alpha exactly 1, so the band's
    // predictor and corrector rows are P_t and C_t themselves.
    const HistLayout H = hist_layout(N, dim);
    char *base = (char *)workspace;
    m.N = N;
    m.wlen = H.wlen;
    InstMeta *dmeta = (InstMeta *)(base + H.meta);
    double *W = (double *)(base + H.w);
    const bool f32 = far_prec == FABM_FAR_FP32;
    float *W32 = f32 ? (float *)(base + H.w32) : nullptr;
    double *ftf = (double *)(base + H.ftf);
    double *yc = (double *)(base + H.yc), *yp = (double *)(base + H.yp);
    double *y0 = (double *)(base + H.y0);
    uint32_t *sync = (uint32_t *)(base + H.sync);
    const int64_t nrow = (int64_t)dim * (N + 1);
    if ((st = ok_or_device(fabm::launch_put_meta(m, dmeta, stream))) != FABM_OK) return st;
    if ((st = ok_or_device(fabm::launch_weights(dmeta, 1, H.wlen, W, stream, W32))) != FABM_OK)
        return st;
    if ((st = ok_or_device(fabm::launch_fill_u32(sync, 64, 0u, stream))) != FABM_OK) return st;
    if ((st = ok_or_device(fabm::launch_copy_pad(f, (int64_t)dim * N, ftf, nrow, stream))) !=
        FABM_OK)
        return st;
    if ((st = ok_or_device(fabm::launch_copy_pad(nullptr, 0, y0, dim, stream))) != FABM_OK)
        return st;
    fabm::StepArgs A{};
    A.meta = dmeta;
    A.m0 = m;
    A.params = ftf;
    A.y0 = y0;
    A.Y = yc;
    A.YP = yp;
    A.W = W;
    A.W32 = W32;
    A.Fc = (double *)(base + H.f);
    A.carry = (double *)(base + H.carry);
    A.acc = (double *)(base + H.acc);
    A.dead = sync;
    A.status = (int64_t *)(base + H.st);
    A.NB = H.NB;
    A.far_cap = fabm::kMaxFarWg;
    A.wlen = H.wlen;
    const char *where = "";
    const hipError_t pe = fabm::enqueue_steps(fabm::SYS_TEACHER, dim, f32, A, stream, nullptr,
                                              &where);
    if (pe != hipSuccess) return record_hip(where, pe);
    // row t of the band's output is target t; the caller's row t - 1
    if ((st = ok_or_device(fabm::launch_copy_pad(yp + dim, (int64_t)dim * N, P, (int64_t)dim * N,
                                                 stream))) != FABM_OK)
        return st;
    return ok_or_device(
        fabm::launch_copy_pad(yc + dim, (int64_t)dim * N, C, (int64_t)dim * N, stream));
}

}  // extern "C"
