/*
 * fabm.h -- C ABI of the MI355X (gfx950) library for the fractional
 * Adams-Bashforth-Moulton predictor-corrector (Diethelm's method) as stated in
 * Section 2 of Baban, Bonchis, Fikl, Rosu, "Parallel simulations for
 * Fractional-Order Systems" (arXiv:1611.08678).
 *
 * Problem (Section 2, eq. (1)): D_*^alpha y(t) = f(t, y(t)) on [0, T] with
 * the ceil(alpha) initial values y^(k)(0): y(0) = y0 for 0 < alpha <= 1, and
 * y(0), y'(0) for 1 < alpha <= 2 (plans with FABM_PLAN_INITIAL_SLOPE). The
 * grid is t_n = n h, n = 0..N, T = N h. One step of the scheme (eq. (2)
 * predictor, then the corrector) is, for target t = n + 1:
 *
 *   P_t  = sum_{k=0}^{t-1} b_{t-1-k} f_k
 *   C_t  = c_{t-1} f_0 + sum_{k=1}^{t-1} a_{t-1-k} f_k
 *   yP_t = T_t + h^alpha P_t,            fP_t = f(t_t, yP_t)
 *   y_t  = T_t + h^alpha (C_t + fP_t / Gamma(alpha + 2)),  f_t = f(t_t, y_t)
 *
 * with T_t = y(0) for alpha <= 1 and T_t = y(0) + t_t y'(0) for
 * 1 < alpha <= 2 (the Taylor polynomial of the initial values in eq. (1)),
 *
 * with b_m = ((m+1)^a - m^a)/Gamma(a+1),
 *      a_m = ((m+2)^(a+1) - 2(m+1)^(a+1) + m^(a+1))/Gamma(a+2),
 *      c_m = (m^(a+1) - (m-a)(m+1)^a)/Gamma(a+2)          (Section 2).
 * (The paper prints b_m with a "+"; the minus sign is the one that makes the
 * rule exact for constant f and is what this library computes.)
 *
 * Conventions for every entry point:
 *   - Pointers marked (device) are device memory on the current HIP device;
 *     pointers marked (host) are host memory read before the call returns.
 *     All floating point is IEEE binary64, row-major, state index fastest.
 *   - The caller owns every buffer, including the workspace. The library never
 *     allocates device memory. fabm_plan allocates host memory only; the first
 *     solve of a plan adds a pinned staging buffer (grown as needed), released
 *     by fabm_plan_destroy.
 *   - All device work is enqueued on `stream` and the call returns without
 *     synchronising. Argument errors are detected on the host, before
 *     anything is enqueued, and reported through the return value.
 *   - Device pointers must be 8-byte aligned. Calls that share a plan must not
 *     overlap in time unless they use distinct workspaces.
 */
#ifndef FABM_H
#define FABM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FABM_OK = 0,
    FABM_ERR_INVALID_ARG = 1, /* bad alpha/h/N/dim/pointer/size */
    FABM_ERR_UNSUPPORTED = 2, /* valid request this library does not run (e.g. 1 < alpha < 2) */
    FABM_ERR_WORKSPACE = 3,   /* workspace missing or smaller than required */
    FABM_ERR_DEVICE = 4       /* a HIP call or kernel launch failed */
} fabm_status;

/* Right-hand sides f(t, y; theta) (the systems named in Section 1; the paper
 * prints no equations, these are the usual textbook forms). Parameter layout
 * of theta for each:
 *   LINEAR     f = A y + b0 + b1 t; theta = A (d*d, row-major), b0 (d), b1 (d)
 *   CHEN       (a(y-x), (c-a)x - xz + cy, xy - bz);  theta = (a, b, c), d = 3
 *   ROSSLER    (-y-z, x + a y, b + z(x-c));          theta = (a, b, c), d = 3
 *   VDP        (v, mu(1-x^2)v - x);                  theta = (mu),      d = 2
 *   FINANCIAL  (z + (y-a)x, 1 - b y - x^2, -x - cz); theta = (a, b, c), d = 3
 *   HINDMARSH_ROSE (y - a x^3 + b x^2 - z + I, c - d x^2 - y, r (s (x - xr) - z));
 *              theta = (a, b, c, d, r, s, xr, I), d = 3 (the neuron model the
 *              paper's experiments simulate) */
typedef enum {
    FABM_SYS_LINEAR = 0,
    FABM_SYS_CHEN = 1,
    FABM_SYS_ROSSLER = 2,
    FABM_SYS_VDP = 3,
    FABM_SYS_FINANCIAL = 4,
    FABM_SYS_HINDMARSH_ROSE = 5
} fabm_system;

/* How the history sums P_t, C_t are contracted.
 *   DIRECT:  every step reduces the whole history against the weight rows
 *            (an HBM/latency-bound GEMV per step).
 *   BLOCKED: history split into past-block -> future-block Toeplitz tiles
 *            contracted in bulk, plus a short sequential near-diagonal band.
 *   AUTO:    the planner's choice. */
typedef enum { FABM_PATH_AUTO = 0, FABM_PATH_DIRECT = 1, FABM_PATH_BLOCKED = 2 } fabm_path;

/* Arithmetic of the far-history tiles of the BLOCKED path. The weights, the
 * near-diagonal band and the corrector update are always binary64.
 *   FP64:   binary64 operands and sums.
 *   FP32:   binary32 operands, binary32 sums over at most one block of
 *           sources, added into binary64.
 *   FP16X2: each operand x stored as 2^e (hi + lo), hi and lo binary16 and e
 *           shared by a lag window or by one block of one history column;
 *           products hi*hi + hi*lo + lo*hi in binary32 over one block of
 *           sources, scaled and added into binary64 (shared-grid form only).
 *
 * BLOCKED comes in two forms.
 *   Per trajectory (tile_L 256): each instance's history is cut into blocks
 *     of 256 rows; every system, LINEAR up to d = 4; far tiles FP64 or FP32.
 *   Shared grid (tile_L 64): all instances of a call have the same alpha, h
 *     and N, so the weight tables are shared and the histories of all
 *     instances form one matrix with a column per (instance, component);
 *     each block of 64 rows takes its far sums from one Toeplitz-times-history
 *     product. LINEAR only, any d up to 64; far tiles FP64, FP32 or FP16X2.
 * The planner takes the shared-grid form for LINEAR plans with d > 4 or
 * FP16X2; a call to such a plan whose instances differ in alpha, h or N
 * returns UNSUPPORTED. */
typedef enum { FABM_FAR_FP64 = 0, FABM_FAR_FP32 = 1, FABM_FAR_FP16X2 = 2 } fabm_far_prec;

typedef struct {
    fabm_system system;
    int32_t dim;             /* state dimension d: LINEAR 1..64, else the system's own */
    fabm_path path;
    fabm_far_prec far_prec;
    int64_t max_batch;       /* largest batch a call will pass (>= 1) */
    int64_t max_steps;       /* largest N of any instance (>= 1) */
    int64_t max_total_steps; /* largest sum of N over a batch; 0 means max_batch*max_steps */
    int32_t tile_L;          /* BLOCKED block length: 0 (planner's choice), 256 (per
                              * trajectory) or 64 (shared grid); other multiples of 64
                              * are UNSUPPORTED */
    int32_t flags;           /* FABM_PLAN_INITIAL_SLOPE | FABM_PLAN_PER_COMPONENT_ORDER |
                              * FABM_PLAN_ADJOINT_CHECKPOINT or 0; other bits INVALID_ARG */
    int32_t fft_level;       /* 0: every far window on the matrix cores. l in 1..15:
                              * sub-quadratic far history, see below */
} fabm_plan_desc;

/* Sub-quadratic far history (fft_level = l > 0). The far sums of a BLOCKED
 * trajectory (the Section 2 history sums, blocks of 256 rows) take, for
 * target block J, every whole source block K <= J - 4 plus a triangle of
 * block J - 3. The whole-block pairs (J - 3, K), K < J - 3, whose highest
 * differing bit is l' form dyadic squares of 2^l' source by 2^l' target
 * blocks. Levels l' >= l are evaluated by FFT convolution (four-step binary64
 * transforms of length 512 * 2^l') right after the step that forms the
 * square's last source block; levels below l and the triangles stay on the
 * matrix-core windows, so the far work falls from O(N^2 d) to
 * O(N log^2 N d) plus O(N d 2^l) window work. The results differ from
 * fft_level = 0 by rounding, bounded normwise rather than per term (about
 * log2(512 * 2^l') u times the norms of the weights and of the history
 * involved). Plans: path BLOCKED with 256-row blocks, max_batch 1, far_prec
 * FP64 or FP32 (the windows' arithmetic; the transforms are binary64), one
 * order or per-component orders (one weight spectrum per component), N <=
 * 2^24; otherwise UNSUPPORTED. Calls: fabm_solve and batches of one; the
 * adjoint calls of such a plan are UNSUPPORTED. The workspace grows by
 * 16 (1 + d + 2 K) M bytes at most, M the longest transform (at most
 * 4 (N + 1) rounded up to a power of two) and K the weight table sets (d with
 * per-component orders, else 1). */

/* Schedule of the sub-quadratic far history (host only, for inspection and
 * tests): for a trajectory of NB blocks of 256 rows, fft_level `level` and
 * step launch s (-1 .. NB - 2), *jend is the end (exclusive) of the target
 * blocks launch s adds matrix-core far windows to, *skip_prev is 1 when those
 * windows leave out the columns of source block s - 1, and *square is the
 * level of the FFT square enqueued right after launch s (its sources are the
 * 2^square blocks ending at s + 1, its targets the 2^square blocks from s + 5
 * on, clipped to NB), or -1. With level 0, or no square at all for this NB,
 * every launch reads jend = NB, skip_prev = 0, square = -1. INVALID_ARG for
 * null pointers, NB < 1, s outside -1 .. NB - 2 or level outside 0..15. */
fabm_status fabm_fft_far_schedule(int32_t NB, int32_t level, int32_t s, int32_t *jend,
                                  int32_t *skip_prev, int32_t *square);

/* Plan flag: the calls of the plan pass two initial values per instance, y0
 * as [batch][2][d] (y(0), then y'(0)), which orders 1 < alpha <= 2 need
 * (eq. (1)); instances with alpha <= 1 ignore their y'(0) row. The adjoint
 * calls of such a plan return gy0 as [batch][2][d] (dL/dy(0), then
 * dL/dy'(0), zero for alpha <= 1). Without the flag, 1 < alpha <= 2 is
 * UNSUPPORTED. */
#define FABM_PLAN_INITIAL_SLOPE 1

/* Plan flag: non-commensurate orders (eq. (1) with a separate order alpha_i
 * for each state component). The batched calls of the plan take alpha as
 * [batch][d] (host); component i of an instance runs the scheme with its own
 * weights b, a, c, h^alpha_i and Gamma(alpha_i + 2), and with
 * FABM_PLAN_INITIAL_SLOPE its own Taylor term (y'(0) used where alpha_i > 1;
 * without the flag every alpha_i must be <= 1). Such plans run the DIRECT
 * kernels and the per-trajectory BLOCKED kernels with FP64 or FP32 far
 * windows (one weight table per component in the band and as the A operand
 * of the windows), and the adjoint calls (alpha [batch][d] there too); the
 * shared grid (LINEAR d > 4, FP16X2, tile_L 64) is UNSUPPORTED, and so is
 * fabm_solve (one alpha): a single trajectory is a batch of one. */
#define FABM_PLAN_PER_COMPONENT_ORDER 2

/* Plan flag: block checkpoints for the adjoint calls. The forward pass keeps
 * only what the far sums need anyway (the history f and the near + far sums
 * of every 256-row block), not every trajectory and predictor row; the reverse
 * pass re-forms the rows of each forward block shortly before it reaches them
 * (the band of that block walked again from its stored sums, its incoming band
 * sums re-formed from the previous block's history), four blocks per group of
 * reverse launches, into a ring of five blocks per instance. The re-formed
 * rows are bitwise the forward's, so the gradients are bitwise those of a plan
 * without the flag; the adjoint workspace shrinks by 16 d (N_i + 1) bytes per
 * instance (less rings of 60 KiB x d), at the cost of a second band walk per
 * block. fabm_adjoint_forward writes the rows straight to y_out. No effect on
 * the solve calls. */
#define FABM_PLAN_ADJOINT_CHECKPOINT 4

/* A plan is used by one host thread at a time: calls that share a plan share
 * its pinned staging buffer and schedule cache. Different plans are
 * independent. */
typedef struct fabm_plan_s *fabm_plan_t;

/* Description of the last HIP failure behind a FABM_ERR_DEVICE returned to
 * this thread (the failing call and the HIP error string); "" if none. The
 * string stays valid until the thread's next failing call. */
const char *fabm_last_error(void);

/* Human-readable name of a status code (static string). */
const char *fabm_status_string(fabm_status s);

/* Number of entries of theta for a system of dimension dim (-1 if invalid). */
int32_t fabm_n_params(fabm_system system, int32_t dim);

/* Build a plan for the description. On success *out receives a host-side
 * handle and *workspace_bytes (may be NULL) the device workspace size that
 * covers any call within the described maxima. Errors: INVALID_ARG for a
 * null pointer, unknown system, dim out of range, max_* < 1, bad tile_L or
 * unknown flags; UNSUPPORTED for a far precision, block length or path the
 * system does not offer (FP16X2 outside LINEAR, DIRECT for LINEAR d > 4), or
 * a shared-grid plan with max_batch * dim above 2^30 history columns. */
fabm_status fabm_plan(const fabm_plan_desc *desc, fabm_plan_t *out, size_t *workspace_bytes);

/* Release a plan (host memory only). NULL is ignored. */
void fabm_plan_destroy(fabm_plan_t plan);

/* Exact workspace bytes for one call with `batch` instances of lengths N
 * (host, [batch]). Same checks as the solve calls on N. */
fabm_status fabm_workspace_size(fabm_plan_t plan, int64_t batch, const int64_t *N,
                                size_t *bytes);

/* One trajectory (Section 2, eq. (1)-(2) and the corrector).
 *   alpha  in (0, 1]; in (1, 2] with FABM_PLAN_INITIAL_SLOPE (without it
 *          UNSUPPORTED); otherwise INVALID_ARG
 *   h      > 0, finite;   N >= 1, N <= plan max_steps
 *   y0     (device) [d]           initial state y(0); [2][d] (y(0), y'(0)) for
 *                                 plans with FABM_PLAN_INITIAL_SLOPE
 *   params (device) [n_params]    theta of the plan's system (may be NULL if n_params == 0)
 *   y_out  (device) [N+1][d]      receives y_0 .. y_N
 *   status (device) [1] int64     0, or the first step index whose state is not
 *                                 finite (that row and all later rows are NaN),
 *                                 or -1 if an inter-workgroup wait inside a
 *                                 persistent kernel exceeded its 10 s bound
 *                                 (rows not known to be final are NaN)
 *   workspace (device), workspace_bytes >= fabm_workspace_size(plan, 1, &N). */
fabm_status fabm_solve(fabm_plan_t plan, void *workspace, size_t workspace_bytes, double alpha,
                       double h, int64_t N, const double *y0, const double *params,
                       double *y_out, int64_t *status, hipStream_t stream);

/* fabm_solve without allocation, for callers that cannot allocate device
 * memory or call hipMalloc (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation). Same arguments, checks and result
 * as fabm_solve (bitwise the same rows), except that the workspace is a
 * device array inside the library of FABM_NOALLOC_SCRATCH_BYTES bytes (one
 * per device, held until the process ends), and the call allocates nothing:
 * no device memory, no pinned staging buffer, no events (the plan's kernel
 * timing does not apply). Plans: the per-trajectory paths (BLOCKED with
 * 256-row blocks, DIRECT) without fft_level and per-component orders;
 * otherwise UNSUPPORTED. A solve whose workspace (fabm_workspace_size with
 * batch 1) exceeds the scratch size returns WORKSPACE and fabm_last_error
 * states both sizes (about N <= 700000 for d = 3 on BLOCKED). Every call on a
 * device uses that device's one array, which keeps the last call's contents
 * (each call re-initialises what it reads): calls that overlap in time on one
 * device race, whatever their streams or plans. */
#define FABM_NOALLOC_SCRATCH_BYTES (64u << 20)
fabm_status fabm_solve_noalloc(fabm_plan_t plan, double alpha, double h, int64_t N,
                               const double *y0, const double *params, double *y_out,
                               int64_t *status, hipStream_t stream);

/* A batch of independent trajectories of one system, each with its own
 * alpha, h, N, y0 and theta (ragged lengths), in one enqueue.
 *   alpha (host) [batch] ([batch][d] with FABM_PLAN_PER_COMPONENT_ORDER)
 *   h, N  (host) [batch]
 *   y0      (device) [batch][d] ([batch][2][d] with FABM_PLAN_INITIAL_SLOPE);
 *   params  (device) [batch][n_params]
 *   row_off (host) [batch]  first row of instance i in y_out; the rows
 *           row_off[i] .. row_off[i] + N[i] must not overlap another instance's
 *   y_out   (device) [total rows][d];  status (device) [batch] int64 as in fabm_solve. */
fabm_status fabm_solve_batch(fabm_plan_t plan, void *workspace, size_t workspace_bytes,
                             int64_t batch, const double *alpha, const double *h,
                             const int64_t *N, const double *y0, const double *params,
                             const int64_t *row_off, double *y_out, int64_t *status,
                             hipStream_t stream);

/* Captured solves (HIP graphs) for callers that replay one solve many times
 * (serving loops, inner iterations): the launch sequence of one
 * fabm_solve_batch call (same arguments and checks) is recorded once into a
 * graph instead of running. Each fabm_graph_launch then runs the whole solve
 * on `stream`, reading the current contents of y0 and params and overwriting
 * y_out and status; alpha, h, N, row_off and every device address are fixed
 * at capture. The graph owns a pinned copy of the per-instance table; the
 * plan's other calls do not disturb it. The workspace, y0, params, y_out and
 * status must stay allocated while the graph exists, and no other call may
 * use that workspace while a launch of the graph is in flight (two launches
 * in flight on different streams race on it). Captured paths: every path
 * the plan runs eagerly except the whole-GPU DIRECT kernel of a single
 * trajectory with N >= 8192 (a cooperative launch: UNSUPPORTED). Errors: as
 * fabm_solve_batch; DEVICE if capture or instantiation fails
 * (fabm_last_error names the call). Nothing is enqueued by
 * fabm_graph_solve_batch itself. */
typedef struct fabm_graph_s *fabm_graph_t;
fabm_status fabm_graph_solve_batch(fabm_plan_t plan, void *workspace, size_t workspace_bytes,
                                   int64_t batch, const double *alpha, const double *h,
                                   const int64_t *N, const double *y0, const double *params,
                                   const int64_t *row_off, double *y_out, int64_t *status,
                                   fabm_graph_t *out);
/* Enqueue one run of a captured solve on `stream`. */
fabm_status fabm_graph_launch(fabm_graph_t graph, hipStream_t stream);
/* Release a captured solve (after its launches have completed). NULL is ignored. */
void fabm_graph_destroy(fabm_graph_t graph);

/* Autotuner. Runs the solve described by the arguments (same arguments and
 * checks as fabm_solve_batch; y_out and status receive a valid result) once
 * untimed and then once per candidate launch shape of the plan's path, times
 * each with events on `stream`, and keeps the fastest in the plan for its
 * later calls (also for its adjoint calls' forward pass). Blocks the host
 * until the runs end. A tuned plan is bitwise deterministic.
 *   single-trajectory BLOCKED: far workgroups per step launch {32, 64, 128, 254}
 *                (results bitwise independent of the choice)
 *   batched BLOCKED (batch > 1): source blocks per group of far windows
 *                {1, 2, 4}: one launch in every P adds the windows of its P
 *                latest source blocks to every later target (one read and
 *                write of the target's sums per P blocks), the others only
 *                to the targets whose band comes first (results bitwise
 *                independent of the choice; default 2)
 *   shared grid: far workgroups a launch aims for {256, 512, 1024, 2048, 4096}
 *                (the source range of a block is split until the column tiles
 *                times the splits reach it, at most 64 splits; results differ
 *                by rounding: the split changes the summation order)
 *   other paths: nothing to choose (knob NONE).
 * report (host, may be NULL) receives the candidates, their times and the
 * index chosen. */
typedef enum {
    FABM_TUNE_NONE = 0,
    FABM_TUNE_FAR_WORKGROUPS = 1,
    FABM_TUNE_SPLIT_TARGET = 2,
    FABM_TUNE_SOURCE_GROUP = 3
} fabm_tune_knob;
typedef struct {
    int32_t knob;       /* fabm_tune_knob */
    int32_t n;          /* candidates timed */
    int32_t value[8];   /* candidate values */
    double seconds[8];  /* solve time of each candidate */
    int32_t chosen;     /* index of the value kept */
} fabm_tune_report;
fabm_status fabm_tune(fabm_plan_t plan, void *workspace, size_t workspace_bytes, int64_t batch,
                      const double *alpha, const double *h, const int64_t *N, const double *y0,
                      const double *params, const int64_t *row_off, double *y_out,
                      int64_t *status, hipStream_t stream, fabm_tune_report *report);

/* Reverse-mode gradients (the discrete adjoint of the scheme above) of
 *   L = sum_i sum_{n=0}^{N_i} < gy_i[n], y_i[n] >
 * with respect to y0 (and y'(0) for orders above one) and theta of every
 * instance (batch = 1 for a single
 * trajectory), where y_i is the trajectory fabm_solve_batch returns for the
 * same inputs with far precision FP64. The forward trajectory and its
 * predictor values are recomputed in the workspace (the same rows the BLOCKED
 * path returns), then a reverse pass runs the blocked decomposition in
 * reversed time (band plus FP64 MFMA windows of the transposed Toeplitz
 * sums). The plan's path and far precision do not apply to this call.
 *   alpha, h, N, row_off (host) [batch]        as in fabm_solve_batch
 *   y0      (device) [batch][d] ([batch][2][d] with FABM_PLAN_INITIAL_SLOPE);
 *   params  (device) [batch][n_params]
 *   gy      (device) rows placed like y_out of fabm_solve_batch: dL/dy_i[n]
 *   gy0     (device) [batch][d]          receives dL/dy0_i; [batch][2][d]
 *                                        (dL/dy(0), dL/dy'(0)) with the flag
 *   gparams (device) [batch][n_params]   receives dL/dtheta_i
 *   status  (device) [batch] int64       the forward status as in fabm_solve_batch;
 *                                        an instance whose forward trajectory is not
 *                                        finite gets NaN gradients
 *   workspace_bytes >= fabm_adjoint_workspace_size(plan, batch, N). */
fabm_status fabm_adjoint(fabm_plan_t plan, void *workspace, size_t workspace_bytes, int64_t batch,
                         const double *alpha, const double *h, const int64_t *N,
                         const double *y0, const double *params, const int64_t *row_off,
                         const double *gy, double *gy0, double *gparams, int64_t *status,
                         hipStream_t stream);
fabm_status fabm_adjoint_workspace_size(fabm_plan_t plan, int64_t batch, const int64_t *N,
                                        size_t *bytes);

/* The adjoint in two calls, for callers that need the trajectory before its
 * gradient (a training step: forward, loss, backward) and would otherwise
 * solve twice. fabm_adjoint_forward runs the forward pass of fabm_adjoint
 * into the workspace (trajectory, predictor rows, history) and writes the
 * trajectory to y_out (rows placed as in fabm_solve_batch) and the status;
 * fabm_adjoint_reverse then runs only the reverse pass on what the workspace
 * holds and writes gy0 and gparams. The two calls give bitwise the gradients
 * fabm_adjoint gives for the same arguments. Between them the workspace must
 * not be used by any other call, and alpha, h, N, row_off, y0 and params must
 * be unchanged. workspace_bytes >= fabm_adjoint_workspace_size(plan, batch, N). */
fabm_status fabm_adjoint_forward(fabm_plan_t plan, void *workspace, size_t workspace_bytes,
                                 int64_t batch, const double *alpha, const double *h,
                                 const int64_t *N, const double *y0, const double *params,
                                 const int64_t *row_off, double *y_out, int64_t *status,
                                 hipStream_t stream);
fabm_status fabm_adjoint_reverse(fabm_plan_t plan, void *workspace, size_t workspace_bytes,
                                 int64_t batch, const double *alpha, const double *h,
                                 const int64_t *N, const double *y0, const double *params,
                                 const int64_t *row_off, const double *gy, double *gy0,
                                 double *gparams, hipStream_t stream);

/* Weight tables of Section 2 for one alpha, lags m = 0..n-1:
 *   b (device) [n], a (device) [n], c (device) [n]  (any may be NULL).
 * alpha in (0, 2]. Computed in binary64 with cancellation-free rearrangements
 * of the defining power differences (expm1/log1p for b, the even binomial
 * series of the second difference in a, a short series for c). */
fabm_status fabm_weights(double alpha, int64_t n, double *b, double *a, double *c,
                         hipStream_t stream);

/* Kernel classes of fabm_plan_kernel_times. */
typedef enum {
    FABM_KERNEL_WEIGHTS = 0,     /* weight tables */
    FABM_KERNEL_DIRECT_WG = 1,   /* DIRECT, one workgroup per trajectory */
    FABM_KERNEL_DIRECT_GRID = 2, /* DIRECT, one trajectory over the whole GPU */
    FABM_KERNEL_BLOCKED_STEP = 3, /* BLOCKED step: one band block plus the MFMA
                                     near and far windows of one source block */
    FABM_KERNEL_HISTORY = 4,      /* fabm_history_sums contraction */
    FABM_KERNEL_ADJOINT = 5,      /* reverse pass: band plus MFMA windows of one block */
    FABM_KERNEL_WIDE_FAR = 6,     /* shared-grid batch: far sums of one block (matrix cores) */
    FABM_KERNEL_WIDE_BAND = 7,    /* shared-grid batch: rows of one block, all instances */
    FABM_KERNEL_FFT_FAR = 8,      /* sub-quadratic far history: weight spectra, and the
                                     FFT convolution of one dyadic square */
    FABM_KERNEL_COUNT = 9
} fabm_kernel_class;

/* Instrumentation. While enabled, every solve call of the plan records a pair
 * of timing events on the launching stream around each of its kernels (this
 * adds some overhead). fabm_plan_kernel_times then synchronises on those
 * events and returns, per class, the summed kernel time of the last call in
 * seconds[FABM_KERNEL_COUNT] and the number of launches in
 * launches[FABM_KERNEL_COUNT] (host arrays). */
fabm_status fabm_plan_set_profiling(fabm_plan_t plan, int32_t enable);
fabm_status fabm_plan_kernel_times(fabm_plan_t plan, double *seconds, int64_t *launches);

/* History sums alone for a given history (teacher forcing; the Section 2
 * predictor sum of eq. (2) and the corrector sum): for t = 1..N,
 *   P[t-1] = sum_{k<t} b_{t-1-k} f[k],   C[t-1] = c_{t-1} f[0] + sum_{1<=k<t} a_{t-1-k} f[k]
 *   f (device) [N][dim], dim 1..4 (else UNSUPPORTED);  P, C (device) [N][dim].
 * `path` selects the contraction:
 *   DIRECT:  one thread per target row and component group reduces the whole
 *            history (far_prec is ignored);
 *   BLOCKED, AUTO: the step pipeline of the BLOCKED solver (band, near and
 *            far matrix-core windows of 256-row blocks, far_prec FP64 or FP32;
 *            FP16X2 is UNSUPPORTED), run with f read from the given rows in
 *            place of the right-hand side; N <= 2^26.
 * A non-finite entry of f makes that target and all later rows NaN on
 * BLOCKED. Workspace (device, 256-byte aligned): at least
 * fabm_history_workspace_size(N, dim) bytes (0 for invalid N or dim). */
fabm_status fabm_history_sums(double alpha, int64_t N, int32_t dim, const double *f, double *P,
                              double *C, fabm_path path, fabm_far_prec far_prec,
                              void *workspace, size_t workspace_bytes, hipStream_t stream);
size_t fabm_history_workspace_size(int64_t N, int32_t dim);

#ifdef __cplusplus
}
#endif

#endif /* FABM_H */
