// wide.hip -- the shared-grid batch path (decomposition in fabm_wide.h).
//
// Layout of the far product on the matrix cores. For target block s and
// source block I (lag block q = s - I >= 1) the 64 x 64 Toeplitz tile has
// entries w[q*64 + r - 1 - k], r the target row and k the source row inside
// their blocks: every entry comes from the 127-lag window
// w[(q-1)*64 .. (q+1)*64 - 2]. A workgroup owns 64 history columns and all 64
// target rows; wavefront w owns 16 of those columns and accumulates four
// 16-row tiles per weight table. The
// Toeplitz tile is the A operand (read out of the window staged in LDS), the
// history the B operand (read straight from HBM, each value once per
// workgroup).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "fabm_device.h"
#include "fabm_launch.h"
#include "fabm_timer.h"
#include "fabm_wide.h"

namespace fabm {

namespace {

constexpr int LW = kWideBlk;  // rows per block
constexpr int kWin = 2 * LW;  // lag window of one block pair (127 used)

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// Far sums are stored through to memory (agent-scope stores): the kernels
// that read them run later, on any XCD, so lines left dirty in the storing
// XCD's L2 would only be written back at the end of the launch.
__device__ __forceinline__ void store_through(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Source blocks [I0, I1) of split p out of `splits` for target block s.
__device__ __forceinline__ void split_range(int s, int p, int splits, int &I0, int &I1)
{
    I0 = (int)((int64_t)s * p / splits);
    I1 = (int)((int64_t)s * (p + 1) / splits);
}

// Writes one wavefront's 4 x 16-row tiles of both tables into split p's slot.
// FP64 results: element v of lane l is row 4 v + l/16; FP32 (and the FP16
// product): row 4 (l/16) + v; column l % 16 in both.
template <bool F32ROWS>
__device__ __forceinline__ void store_tiles(const WideArgs &A, int p, int64_t col,
                                            const dbl4 (&acc)[2][4])
{
    const int lane = threadIdx.x & 63, g = lane >> 4;
    double *out = A.part + (int64_t)p * 2 * LW * A.cp;
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * rt + (F32ROWS ? 4 * g + v : 4 * v + g);
                store_through(&out[((int64_t)tb * LW + row) * A.cp + col], acc[tb][rt][v]);
            }
}

// ---------------------------------------------------------------------------
// Far sums in binary64: v_mfma_f64_16x16x4f64, A[sigma][tau] = window[64 +
// 16 rt + sigma - 1 - 4 ks - tau] (sigma = l % 16, tau = l / 16), B[tau][n] =
// F[I*64 + 4 ks + tau][col]. The next block's history and lag window are
// loaded while the current one is multiplied.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wide_far_f64(WideArgs A, int s, int splits)
{
    __shared__ double sw[2][2][kWin];  // [buffer][table][lag window]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, sig = lane & 15;
    int I0, I1;
    split_range(s, blockIdx.y, splits, I0, I1);
    const int64_t cp = A.cp;
    const int64_t col = (int64_t)blockIdx.x * 64 + wave * 16 + sig;
    const int wj = tid & 127, wt = tid >> 7;  // lag-window entry this thread stages
    const double *wsrc = A.W + (wt ? A.wlen : 0);

    dbl4 acc[2][4];
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) acc[tb][rt] = dbl4{0.0, 0.0, 0.0, 0.0};

    double bcur[16], bnext[16];
    if (I0 < I1) {
        const double *src = A.F + ((int64_t)I0 * LW + g) * cp + col;
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) bcur[ks] = src[4 * ks * cp];
        if (wj < kWin - 1) sw[0][wt][wj] = wsrc[(int64_t)(s - I0 - 1) * LW + wj];
    }
    __syncthreads();
    for (int I = I0; I < I1; ++I) {
        const int buf = (I - I0) & 1;
        const bool more = I + 1 < I1;
        double wnext = 0.0;
        if (more) {
            const double *src = A.F + ((int64_t)(I + 1) * LW + g) * cp + col;
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) bnext[ks] = src[4 * ks * cp];
            if (wj < kWin - 1) wnext = wsrc[(int64_t)(s - I - 2) * LW + wj];
        }
        const double *wb = sw[buf][0], *wa = sw[buf][1];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                const int j = LW + 16 * rt + sig - 1 - 4 * ks - g;
                acc[0][rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(wb[j], bcur[ks], acc[0][rt], 0, 0, 0);
                acc[1][rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa[j], bcur[ks], acc[1][rt], 0, 0, 0);
            }
        }
        if (more && wj < kWin - 1) sw[buf ^ 1][wt][wj] = wnext;
        __syncthreads();
        if (more) {
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) bcur[ks] = bnext[ks];
        }
    }
    store_tiles<false>(A, blockIdx.y, col, acc);
}

// ---------------------------------------------------------------------------
// Far sums with binary32 operands: v_mfma_f32_16x16x4f32 over one source
// block (64 terms) at a time, each block's products then added into binary64
// accumulators.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wide_far_f32(WideArgs A, int s, int splits)
{
    __shared__ float sw[2][2][kWin];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, sig = lane & 15;
    int I0, I1;
    split_range(s, blockIdx.y, splits, I0, I1);
    const int64_t cp = A.cp;
    const int64_t col = (int64_t)blockIdx.x * 64 + wave * 16 + sig;
    const int wj = tid & 127, wt = tid >> 7;
    const float *wsrc = A.W32 + (wt ? A.wlen : 0);

    dbl4 acc[2][4];
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) acc[tb][rt] = dbl4{0.0, 0.0, 0.0, 0.0};

    float bcur[16], bnext[16];
    if (I0 < I1) {
        const float *src = A.F32 + ((int64_t)I0 * LW + g) * cp + col;
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) bcur[ks] = src[4 * ks * cp];
        if (wj < kWin - 1) sw[0][wt][wj] = wsrc[(int64_t)(s - I0 - 1) * LW + wj];
    }
    __syncthreads();
    for (int I = I0; I < I1; ++I) {
        const int buf = (I - I0) & 1;
        const bool more = I + 1 < I1;
        float wnext = 0.0f;
        if (more) {
            const float *src = A.F32 + ((int64_t)(I + 1) * LW + g) * cp + col;
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) bnext[ks] = src[4 * ks * cp];
            if (wj < kWin - 1) wnext = wsrc[(int64_t)(s - I - 2) * LW + wj];
        }
        const float *wb = sw[buf][0], *wa = sw[buf][1];
        flt4 c32[2][4];
#pragma unroll
        for (int tb = 0; tb < 2; ++tb)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) c32[tb][rt] = flt4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                const int j = LW + 16 * rt + sig - 1 - 4 * ks - g;
                c32[0][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wb[j], bcur[ks], c32[0][rt], 0, 0, 0);
                c32[1][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[j], bcur[ks], c32[1][rt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int tb = 0; tb < 2; ++tb)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[tb][rt][v] += (double)c32[tb][rt][v];
        if (more && wj < kWin - 1) sw[buf ^ 1][wt][wj] = wnext;
        __syncthreads();
        if (more) {
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) bcur[ks] = bnext[ks];
        }
    }
    store_tiles<true>(A, blockIdx.y, col, acc);
}

// ---------------------------------------------------------------------------
// Split binary16 operands. A value x of a lag window (or of one block of one
// history column) is stored as 2^e (hi + lo) with hi = fp16(x / 2^e) and
// lo = fp16(x / 2^e - hi), e chosen so the window's (column's) largest
// magnitude lies in [1/2, 1). Products hi*hi + hi*lo + lo*hi run on
// v_mfma_f32_16x16x32_f16 (binary32 accumulation over one source block); the
// block's sum is then scaled by 2^(e_w + e_F) and added in binary64.
//
// The A operand of lane l (row sigma = l % 16, columns 8 (l/16) .. +7) is
// eight consecutive entries of the reversed window rev[u] = w[(q+1)*64 - 2 - u]
// starting at u0 = 63 - 16 rt - sigma + 32 ks + 8 (l/16); u0 mod 8 depends on
// sigma only. The table keeps eight copies of rev shifted by 0..7 entries so
// each operand is one aligned 16-byte read: copy p holds rev[m + p].
// ---------------------------------------------------------------------------
constexpr int kT16Row = 2 * LW;                    // halves per shifted copy
constexpr int kT16Q = 2 * 2 * 8 * kT16Row;         // halves per lag block q
// In LDS each copy is padded by one 16-byte entry: the eight lanes that read
// together (sigma = 0..7 or 8..15 of one 16-lane group) take the same entry of
// eight different copies, which 256-byte copies would put in one bank.
constexpr int kT16Ent = kT16Row / 8;               // 16-byte entries per copy
constexpr int kT16Pitch = kT16Ent + 1;             // entries per copy in LDS
constexpr int kT16Copies = 2 * 2 * 8;              // (table, part, shift) copies
static_assert(kT16Q / 8 == kT16Copies * kT16Ent, "operand table layout");

__global__ __launch_bounds__(256) void k_wide_t16(WideArgs A, _Float16 *T16, int32_t *T16exp)
{
    __shared__ double sv[2][kWin];
    __shared__ double smax[2][4];
    const int q = blockIdx.x + 1;  // lag block 1 .. NB-1
    const int tid = threadIdx.x, j = tid & 127, tb = tid >> 7;
    const double *w = A.W + (tb ? A.wlen : 0);
    // rev[u] = w[(q+1)*64 - 2 - u], u = 0..126; u = 127 is padding
    const double v = j < kWin - 1 ? w[(int64_t)(q + 1) * LW - 2 - j] : 0.0;
    sv[tb][j] = v;
    double mx = fabs(v);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if ((tid & 63) == 0) smax[tb][(tid >> 6) & 1] = mx;
    __syncthreads();
    const double m2 = fmax(smax[tb][0], smax[tb][1]);
    int e = 0;
    if (m2 > 0.0 && isfinite(m2)) (void)frexp(m2, &e);
    if (j == 0) T16exp[q * 2 + tb] = e;
    _Float16 *hi = T16 + (int64_t)q * kT16Q + (int64_t)(tb * 2 + 0) * 8 * kT16Row;
    _Float16 *lo = T16 + (int64_t)q * kT16Q + (int64_t)(tb * 2 + 1) * 8 * kT16Row;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int u = j + p;
        const double x = u < kWin ? ldexp(sv[tb][u], -e) : 0.0;
        const _Float16 xh = (_Float16)x;
        hi[p * kT16Row + j] = xh;
        lo[p * kT16Row + j] = (_Float16)(x - (double)xh);
    }
}

// One wavefront: 16 columns, four 16-row tiles per table. Within a source
// block the A operand of row tile rt and k-slice ks depends on rt - 2 ks only
// (the window start moves by 16 per row tile and by 32 per k-slice), so six
// operand pairs serve the eight (rt, ks) tiles; consecutive products go to
// different accumulators. The next block's history operands are loaded while
// the current block is multiplied.
__global__ __launch_bounds__(256) void k_wide_far_f16(WideArgs A, int s, int splits)
{
    __shared__ half8 sT[2][kT16Copies * kT16Pitch];  // [buffer][table, part, copy][entry]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, sig = lane & 15;
    int I0, I1;
    split_range(s, blockIdx.y, splits, I0, I1);
    const int64_t cp = A.cp;
    const int64_t col = (int64_t)blockIdx.x * 64 + wave * 16 + sig;
    const int shift = (7 - sig) & 7;  // copy holding this lane's operands aligned

    dbl4 acc[2][4];  // [table][rt]
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) acc[tb][rt] = dbl4{0.0, 0.0, 0.0, 0.0};

    const half8 *T16 = (const half8 *)A.T16;
    const half8 *Fh = (const half8 *)A.Fhi, *Fl = (const half8 *)A.Flo;
    // History operands of a block (rows 32 ks + 8 (l/16) .. +7 of this
    // column) in a ring of three: block I's are loaded while block I - 2 is
    // multiplied, two blocks of HBM latency ahead.
    half8 bh[3][2], bl[3][2];
    int ef[3] = {0, 0, 0};
    auto load_b = [&](const int I, auto SLOT) __attribute__((always_inline)) {
        constexpr int R = decltype(SLOT)::value;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int64_t o = ((int64_t)I * (LW / 8) + 4 * ks + g) * cp + col;
            bh[R][ks] = Fh[o];
            bl[R][ks] = Fl[o];
        }
        ef[R] = A.Fexp[(int64_t)I * cp + col];
    };
    // LDS slot of table entry e (= copy * 16 + entry) of a lag block
    const int st0 = (tid / kT16Ent) * kT16Pitch + tid % kT16Ent;
    const int st1 = ((tid + 256) / kT16Ent) * kT16Pitch + (tid + 256) % kT16Ent;
    using C0 = std::integral_constant<int, 0>;
    using C1 = std::integral_constant<int, 1>;
    using C2 = std::integral_constant<int, 2>;
    if (I0 < I1) {
        const half8 *src = T16 + (int64_t)(s - I0) * (kT16Q / 8);
        sT[0][st0] = src[tid];
        sT[0][st1] = src[tid + 256];
        load_b(I0, C0{});
        if (I0 + 1 < I1) load_b(I0 + 1, C1{});
    }
    __syncthreads();
    // Block I's products go to one of two sets of binary32 sums while the
    // other set (block I - 1's) is scaled and added into binary64, so the
    // matrix cores are not drained before every conversion.
    flt4 c32[2][2][4];  // [set][table][rt]
    double psc[2] = {0.0, 0.0};  // scales of the block in the other set
    auto convert = [&](auto SET) __attribute__((always_inline)) {
        constexpr int S = decltype(SET)::value;
#pragma unroll
        for (int tb = 0; tb < 2; ++tb)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[tb][rt][v] = fma((double)c32[S][tb][rt][v], psc[tb], acc[tb][rt][v]);
    };
    // block I: sum set S = (I - I0) mod 2, history slot R = (I - I0) mod 3
    auto block = [&](const int I, auto SET, auto SLOT) __attribute__((always_inline)) {
        constexpr int S = decltype(SET)::value;
        constexpr int R = decltype(SLOT)::value;
        const int buf = (I - I0) & 1;
        const bool more = I + 1 < I1;
        const int q = s - I;
        half8 tnext[2];
        if (more) {
            const half8 *src = T16 + (int64_t)(q - 1) * (kT16Q / 8);
            tnext[0] = src[tid];
            tnext[1] = src[tid + 256];
        }
        if (I + 2 < I1) load_b(I + 2, std::integral_constant<int, (R + 2) % 3>{});
        const int ew0 = A.T16exp[q * 2 + 0], ew1 = A.T16exp[q * 2 + 1];
#pragma unroll
        for (int tb = 0; tb < 2; ++tb)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) c32[S][tb][rt] = flt4{0.0f, 0.0f, 0.0f, 0.0f};
        const half8 *tw = sT[buf];
#pragma unroll
        for (int j = -2; j <= 3; ++j) {  // j = rt - 2 ks
            const int u0 = LW - 1 - 16 * j - sig + 8 * g;
            const int m8 = (u0 - shift) >> 3;
            half8 ah[2], al[2];
#pragma unroll
            for (int tb = 0; tb < 2; ++tb) {
                ah[tb] = tw[((tb * 2 + 0) * 8 + shift) * kT16Pitch + m8];
                al[tb] = tw[((tb * 2 + 1) * 8 + shift) * kT16Pitch + m8];
            }
#pragma unroll
            for (int prod = 0; prod < 3; ++prod)
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const int rt = j + 2 * ks;
                    if (rt < 0 || rt > 3) continue;
#pragma unroll
                    for (int tb = 0; tb < 2; ++tb) {
                        const half8 a = prod == 2 ? al[tb] : ah[tb];
                        const half8 b = prod == 1 ? bl[R][ks] : bh[R][ks];
                        c32[S][tb][rt] =
                            __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c32[S][tb][rt], 0, 0, 0);
                    }
                }
        }
        // the block before (other set), while these products run
        if (I > I0) convert(std::integral_constant<int, 1 - S>{});
        psc[0] = ldexp(1.0, ew0 + ef[R]);
        psc[1] = ldexp(1.0, ew1 + ef[R]);
        if (more) {
            sT[buf ^ 1][st0] = tnext[0];
            sT[buf ^ 1][st1] = tnext[1];
        }
        __syncthreads();
    };
    // six blocks per trip (both set and slot patterns repeat), then the rest
    int I = I0;
    for (; I + 6 <= I1; I += 6) {
        block(I, C0{}, C0{});
        block(I + 1, C1{}, C1{});
        block(I + 2, C0{}, C2{});
        block(I + 3, C1{}, C0{});
        block(I + 4, C0{}, C1{});
        block(I + 5, C1{}, C2{});
    }
    if (I < I1) block(I, C0{}, C0{});
    if (I + 1 < I1) block(I + 1, C1{}, C1{});
    if (I + 2 < I1) block(I + 2, C0{}, C2{});
    if (I + 3 < I1) block(I + 3, C1{}, C0{});
    if (I + 4 < I1) block(I + 4, C0{}, C1{});
    // the last block's sums: set (I1 - 1 - I0) mod 2
    if (I1 > I0) {
        if (((I1 - 1 - I0) & 1) == 0)
            convert(C0{});
        else
            convert(C1{});
    }
    store_tiles<true>(A, blockIdx.y, col, acc);
}

// Split partials summed into split 0, in split order.
__global__ __launch_bounds__(256) void k_wide_reduce(double *part, int64_t n, int splits)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * 256) {
        double v = part[e];
        for (int p = 1; p < splits; ++p) v += part[(int64_t)p * n + e];
        store_through(&part[e], v);
    }
}

// ---------------------------------------------------------------------------
// Band: one workgroup of four wavefronts per instance. Lane c holds component
// c (d <= 64); wavefront w holds columns 16 w .. 16 w + 15 of row c of the
// system matrix. Rows of block s in order:
//   P = far P + sum_{t0 <= k < T} b[T-1-k] f_k,
//   C = far C + sum_{t0 <= k < T} a[T-1-k] f_k + (c[T-1] - a[T-1]) f_0,
//   yP = y0 + h^a P, y = y0 + h^a (C + f(yP) / Gamma(a+2)), f_T = f(y),
// with f(v) = A v + b0 + b1 t. Wavefront w forms the in-block terms of rows
// k = w, w + 4, ... and its quarter of every matrix-vector product; the four
// partials meet in LDS and every wavefront adds them in the same order, so all
// four hold identical rows. The newest row's terms are added from registers.
// The far sums of the block are read into LDS first; the slot of row r holds
// far P until row r is formed and f_r after.
// ---------------------------------------------------------------------------
constexpr int kWideBandWaves = 4;
constexpr int kWideBandCols = 64 / kWideBandWaves;  // matrix columns per wavefront

template <int PREC>
__global__ __launch_bounds__(256) void k_wide_band(WideArgs A, int s)
{
    __shared__ double sX[LW][64];  // far P of row r, then f_r
    __shared__ double sC[LW][64];  // far C of row r
    __shared__ double sWb[LW], sWa[LW], sDca[LW], sV[64];
    __shared__ double sRed[2][kWideBandWaves][64];  // matrix-vector partials (two slots)
    __shared__ double sPC[2][kWideBandWaves][64];   // in-block partials of P and C
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t i = blockIdx.x;
    const int d = A.d;
    const bool act = lane < d;
    const InstMeta m = A.meta[i];
    const int64_t N = m.N, t0 = (int64_t)s * LW, cp = A.cp;
    const int nrows = (int)((t0 + LW - 1 < N ? t0 + LW - 1 : N) - t0 + 1);
    const int64_t col = i * d + lane;
    double *Yi = A.Y + m.row_off * d;

    if (A.dead[i] != 0u) {
        if (act && w == 0)
            for (int r = 0; r < nrows; ++r) Yi[(t0 + r) * d + lane] = __builtin_nan("");
        return;
    }
    const double *p = A.params + m.p_off;
    double acol[kWideBandCols];
#pragma unroll
    for (int jj = 0; jj < kWideBandCols; ++jj) {
        const int j = kWideBandCols * w + jj;
        acol[jj] = (act && j < d) ? p[lane * d + j] : 0.0;
    }
    const double b0 = act ? p[d * d + lane] : 0.0, b1 = act ? p[d * d + d + lane] : 0.0;
    const double y0 = act ? A.y0[i * d + lane] : 0.0;
    // y'(0), used for orders above one
    const double y1 = (act && A.y1 != nullptr && m.alpha > 1.0) ? A.y1[i * d + lane] : 0.0;

    const double *wb = A.W, *wa = wb + A.wlen, *wc = wa + A.wlen;
    if (w == 0) {
        sWb[lane] = wb[lane];
        sWa[lane] = wa[lane];
        const int64_t T = t0 + lane;
        sDca[lane] = (T >= 1 && T <= N) ? wc[T - 1] - wa[T - 1] : 0.0;
    }
    const double *fp0 = A.part, *fc0 = A.part + (int64_t)LW * cp;
    for (int r = w; r < nrows; r += kWideBandWaves) {
        sX[r][lane] = (s > 0 && act) ? fp0[r * cp + col] : 0.0;
        sC[r][lane] = (s > 0 && act) ? fc0[r * cp + col] : 0.0;
    }

    // f(v) at time t for this lane's component (identical in all wavefronts)
    int slot = 0;
    auto fval = [&](double v, double t) -> double {
        if (w == 0) sV[lane] = act ? v : 0.0;
        __syncthreads();
        double c[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int jj = 0; jj < kWideBandCols; ++jj)
            c[jj & 3] = fma(acol[jj], sV[kWideBandCols * w + jj], c[jj & 3]);
        sRed[slot][w][lane] = (c[0] + c[1]) + (c[2] + c[3]);
        __syncthreads();
        const double mv = (sRed[slot][0][lane] + sRed[slot][1][lane]) +
                          (sRed[slot][2][lane] + sRed[slot][3][lane]);
        slot ^= 1;
        return fma(b1, t, b0) + mv;
    };
    const double f0 = fval(y0, 0.0);

    const double ha = m.ha, ig2 = m.ig2, h = m.h;
    const double b0w = sWb[0], a0w = sWa[0];
    double fprev = 0.0;  // f of row r - 1 (all wavefronts)
    for (int r = 0; r < nrows; ++r) {
        const int64_t T = t0 + r;
        double y, f;
        if (T == 0) {
            y = y0;
            f = f0;
        } else {
            // this wavefront's in-block terms: rows k = w, w + 4, ... <= r - 2
            double pp = 0.0, cc = 0.0;
            for (int k = w; k < r - 1; k += kWideBandWaves) {
                const double fk = sX[k][lane];
                pp = fma(sWb[r - 1 - k], fk, pp);
                cc = fma(sWa[r - 1 - k], fk, cc);
            }
            sPC[0][w][lane] = pp;
            sPC[1][w][lane] = cc;
            const double farP = sX[r][lane], farC = fma(sDca[r], f0, sC[r][lane]);
            __syncthreads();
            double P = farP + ((sPC[0][0][lane] + sPC[0][1][lane]) +
                               (sPC[0][2][lane] + sPC[0][3][lane]));
            double C = farC + ((sPC[1][0][lane] + sPC[1][1][lane]) +
                               (sPC[1][2][lane] + sPC[1][3][lane]));
            if (r > 0) {  // the newest row of the block
                P = fma(b0w, fprev, P);
                C = fma(a0w, fprev, C);
            }
            const double t = (double)T * h;
            const double base = fma(t, y1, y0);  // Taylor part of eq. (1)
            const double yp = fma(ha, P, base);
            const double fp = fval(yp, t);
            y = fma(ha, fma(fp, ig2, C), base);
            f = fval(y, t);
            if (__ballot(act && !(isfinite(y) && isfinite(f)))) {
                if (act && w == 0) {
                    for (int rr = r; rr < nrows; ++rr) Yi[(t0 + rr) * d + lane] = __builtin_nan("");
                    if (lane == 0) A.dead[i] = (uint32_t)T;
                }
                return;
            }
        }
        fprev = f;
        if (w == 0) {
            sX[r][lane] = f;
            if (act) {
                Yi[T * d + lane] = y;
                if constexpr (PREC == WIDE_F64) A.F[T * cp + col] = f;
                if constexpr (PREC == WIDE_F32) A.F32[T * cp + col] = (float)f;
            }
        }
    }
    if constexpr (PREC == WIDE_F16X2) {
        __syncthreads();  // every f_r in LDS
        if (act && s + 1 < A.NB) {
            double mx = 0.0;
            for (int r = 0; r < nrows; ++r) mx = fmax(mx, fabs(sX[r][lane]));
            int e = 0;
            if (mx > 0.0) (void)frexp(mx, &e);
            if (w == 0) A.Fexp[(int64_t)s * cp + col] = e;
            half8 *Fh = (half8 *)A.Fhi, *Fl = (half8 *)A.Flo;
            for (int r8 = w; r8 < LW / 8; r8 += kWideBandWaves) {
                half8 vh, vl;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int r = 8 * r8 + j;
                    const double x = r < nrows ? ldexp(sX[r][lane], -e) : 0.0;
                    const _Float16 xh = (_Float16)x;
                    vh[j] = xh;
                    vl[j] = (_Float16)(x - (double)xh);
                }
                const int64_t o = ((int64_t)s * (LW / 8) + r8) * cp + col;
                Fh[o] = vh;
                Fl[o] = vl;
            }
        }
    }
}

__global__ void k_wide_status(const uint32_t *dead, int64_t *status, int64_t batch)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < batch) status[i] = (int64_t)dead[i];
}

int cols_per_wg(int) { return 64; }

int splits_for(int cp, int prec, int s, int target)
{
    const int tiles = cp / cols_per_wg(prec);
    int sp = (std::max(target, 1) + tiles - 1) / tiles;
    sp = std::min(sp, kWideMaxSplits);
    return std::max(1, std::min(sp, s));
}

}  // namespace

size_t wide_t16_bytes(int NB) { return sizeof(_Float16) * (size_t)kT16Q * (size_t)NB; }

int wide_max_splits(int cp, int NB)
{
    int mx = 1;
    for (int prec = 0; prec < 3; ++prec)
        mx = std::max(mx, splits_for(cp, prec, NB, kWideMaxSplitTarget));
    return mx;
}

hipError_t enqueue_wide(const WideArgs &A, hipStream_t st, KernelTimer *T, const char **where)
{
    hipError_t e;
#define WIDE_CHECK(what)                     \
    do {                                     \
        if ((e = hipGetLastError()) != hipSuccess) { \
            *where = what;                   \
            return e;                        \
        }                                    \
    } while (0)
    if (A.prec == WIDE_F16X2 && A.NB > 1) {
        hipLaunchKernelGGL(k_wide_t16, dim3(A.NB - 1), dim3(256), 0, st, A,
                           const_cast<_Float16 *>(A.T16), const_cast<int32_t *>(A.T16exp));
        WIDE_CHECK("k_wide_t16");
    }
    const int tiles = A.cp / cols_per_wg(A.prec);
    for (int s = 0; s < A.NB; ++s) {
        if (s > 0) {
            const int sp =
                splits_for(A.cp, A.prec, s, std::min(A.split_target, kWideMaxSplitTarget));
            if (T && (e = T->begin(KC_WIDE_FAR, st)) != hipSuccess) {
                *where = "timer";
                return e;
            }
            const dim3 grid((unsigned)tiles, (unsigned)sp);
            if (A.prec == WIDE_F64)
                hipLaunchKernelGGL(k_wide_far_f64, grid, dim3(256), 0, st, A, s, sp);
            else if (A.prec == WIDE_F32)
                hipLaunchKernelGGL(k_wide_far_f32, grid, dim3(256), 0, st, A, s, sp);
            else
                hipLaunchKernelGGL(k_wide_far_f16, grid, dim3(256), 0, st, A, s, sp);
            WIDE_CHECK("k_wide_far");
            if (sp > 1) {
                const int64_t n = (int64_t)2 * LW * A.cp;
                const int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
                hipLaunchKernelGGL(k_wide_reduce, dim3((unsigned)blocks), dim3(256), 0, st, A.part,
                                   n, sp);
                WIDE_CHECK("k_wide_reduce");
            }
            if (T && (e = T->end(st)) != hipSuccess) {
                *where = "timer";
                return e;
            }
        }
        if (T && (e = T->begin(KC_WIDE_BAND, st)) != hipSuccess) {
            *where = "timer";
            return e;
        }
        const dim3 grid((unsigned)A.batch);
        if (A.prec == WIDE_F64)
            hipLaunchKernelGGL(k_wide_band<WIDE_F64>, grid, dim3(256), 0, st, A, s);
        else if (A.prec == WIDE_F32)
            hipLaunchKernelGGL(k_wide_band<WIDE_F32>, grid, dim3(256), 0, st, A, s);
        else
            hipLaunchKernelGGL(k_wide_band<WIDE_F16X2>, grid, dim3(256), 0, st, A, s);
        WIDE_CHECK("k_wide_band");
        if (T && (e = T->end(st)) != hipSuccess) {
            *where = "timer";
            return e;
        }
    }
    hipLaunchKernelGGL(k_wide_status, dim3((unsigned)((A.batch + 255) / 256)), dim3(256), 0, st,
                       A.dead, A.status, A.batch);
    WIDE_CHECK("k_wide_status");
#undef WIDE_CHECK
    return hipSuccess;
}

}  // namespace fabm
