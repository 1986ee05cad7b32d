// fft_far.hip -- sub-quadratic far history for one long trajectory: part of
// the far sums of the BLOCKED pipeline (Section 2's predictor and corrector
// sums) split into dyadic Toeplitz squares that are evaluated by FFT
// convolution once their sources exist.
//
// The far part of target column rho of block J is every source column up to
// 16 (J - 3) + rho: all of the blocks K <= J - 4 and a triangle of block J - 3.
// With J'' = J - 3, the whole-block part is the block pairs K < J''. Each pair
// has a highest bit l in which J'' and K differ (J'' has it set, K clear,
// higher bits equal), so the pairs of level l form squares
//     targets J'' in [(2j+1) 2^l, (2j+2) 2^l),  sources K in [2j 2^l, (2j+1) 2^l),
// which tile that part exactly (the relaxed scheme of fast online
// convolution: Hairer, Lubich and Schlichte, SIAM J. Sci. Stat. Comput. 6
// (1985), for Volterra convolution sums). Pairs of levels below `fft_level`
// (source and target in the same group of 2^fft_level blocks) and the
// triangles stay on the matrix-core windows of the step kernel: launch s adds
// its windows to the targets of its own group only, and the first launch of a
// group leaves out the columns of block s - 1 (a window straddles blocks
// s - 1 and s, and block s - 1 belongs to the previous group's squares). A
// square of level l >= fft_level is one Toeplitz product of L = 256 * 2^l
// target rows by L source rows, computed right after the launch that forms its
// last source block, three launches before its first target block is walked
// by the band.
//
// In rows, the square's sources start at S0 = 256 * 2j * 2^l and its targets
// at T0 = S0 + L + 768, so every lag T - 1 - k lies in [768, 2L + 766] and the
// weights it uses do not depend on j: v[m] = (b, a)[768 + m], m < 2L - 1. With
// x the L source rows of one component zero-padded to M = 2L,
//     z[L - 1 + i] = sum_k v[L - 1 + i - k] x[k]
// is the sum of target T0 + i, and the cyclic convolution of length M has no
// wrap-around on these outputs. Both tables ride in one complex transform:
// spectrum(v_b + i v_a) * spectrum(x) transforms back to z_b + i z_a for real x.
//
// Transforms of length M = M1 * M2 (M2 = min(M, 4096)) take the four-step
// route: length-M1 transforms down the columns of the M1 x M2 array, a twiddle
// w_M^(n2 k1), length-M2 transforms along the rows. The spectrum stays in that
// (transposed) order; the weight spectra are made by the same steps, so the
// pointwise product needs no reordering, and the inverse runs the steps
// backwards. Each short transform is a radix-2 transform in LDS.
//
// Rounding: the FFT product is accurate normwise (componentwise errors about
// log2(M) u max|spectrum(v)| ||x||_2 / sqrt(M)) rather than per term as in the
// direct sums; results differ from the matrix-core windows by rounding only.
#include "fabm_blocked.h"
#include "fabm_launch.h"
#include "fabm_timer.h"

namespace fabm {

namespace {

constexpr int kFftThreads = 256;
constexpr int kRowMax = 4096;  // longest transform held in LDS (64 KB of complex binary64)
constexpr int kRows = 256;     // rows per block of the step pipeline

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ int brev(int i, int logn)
{
    return logn == 0 ? 0 : (int)(__builtin_bitreverse32((uint32_t)i) >> (32 - logn));
}

// exp(-2 pi i j / Mmax), j < Mmax
__global__ void k_fft_twiddles(double2 *tw, int64_t Mmax)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < Mmax;
         j += (int64_t)gridDim.x * blockDim.x) {
        double s, c;
        sincospi(2.0 * (double)j / (double)Mmax, &s, &c);
        tw[j] = make_double2(c, -s);
    }
}

// nb transforms of length n, s[b * n + i], bit-reversed input, natural output
// (decimation in time). inv: conjugate twiddles (unscaled inverse).
__device__ void lds_dit(double2 *s, int n, int nb, const double2 *__restrict__ tw, int64_t Mmax,
                        bool inv)
{
    const int hn = n >> 1;
    for (int len = 2; len <= n; len <<= 1) {
        const int half = len >> 1;
        const int64_t ts = Mmax / len;
        for (int q = threadIdx.x; q < nb * hn; q += blockDim.x) {
            const int b = q / hn, r = q - b * hn;
            const int pos = r & (half - 1), grp = r / half;
            const int i = b * n + grp * len + pos, j = i + half;
            double2 w = tw[pos * ts];
            if (inv) w.y = -w.y;
            const double2 u = s[i], t = cmul(s[j], w);
            s[i] = make_double2(u.x + t.x, u.y + t.y);
            s[j] = make_double2(u.x - t.x, u.y - t.y);
        }
        __syncthreads();
    }
}

// One transform of length n, natural input, bit-reversed output (decimation in
// frequency).
__device__ void lds_dif(double2 *s, int n, const double2 *__restrict__ tw, int64_t Mmax, bool inv)
{
    for (int len = n; len >= 2; len >>= 1) {
        const int half = len >> 1;
        const int64_t ts = Mmax / len;
        for (int q = threadIdx.x; q < (n >> 1); q += blockDim.x) {
            const int pos = q & (half - 1), grp = q / half;
            const int i = grp * len + pos, j = i + half;
            double2 w = tw[pos * ts];
            if (inv) w.y = -w.y;
            const double2 u = s[i], v = s[j];
            s[i] = make_double2(u.x + v.x, u.y + v.y);
            s[j] = cmul(make_double2(u.x - v.x, u.y - v.y), w);
        }
        __syncthreads();
    }
}

// x_c[p] = f_c[S0 + p] for p < L, zero up to M (component c = blockIdx.y).
__global__ void k_fft_gather_hist(const double *__restrict__ Fc, int64_t pitch, int64_t S0,
                                  int64_t L, int64_t M, double2 *buf)
{
    const int c = blockIdx.y;
    double2 *x = buf + c * M;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M;
         p += (int64_t)gridDim.x * blockDim.x)
        x[p] = make_double2(p < L ? Fc[c * pitch + S0 + p] : 0.0, 0.0);
}

// v[p] = (b[off + p], a[off + p]) for p < 2L - 1 inside the tables, else zero;
// one table set per blockIdx.y (per-component orders: tables 3 wlen apart,
// spectra M apart).
__global__ void k_fft_gather_w(const double *__restrict__ W, int64_t wlen, int64_t off,
                               int64_t L, int64_t M, double2 *v)
{
    W += blockIdx.y * 3 * wlen;
    v += blockIdx.y * M;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M;
         p += (int64_t)gridDim.x * blockDim.x) {
        const bool in = p < 2 * L - 1 && off + p < wlen;
        v[p] = in ? make_double2(W[off + p], W[wlen + off + p]) : make_double2(0.0, 0.0);
    }
}

// Column step: columns n2 in [C blockIdx.x, +C) of the M1 x M2 array of
// component blockIdx.y, element (n1, n2) at M2 n1 + n2. Forward: transform
// then twiddle w_M^(n2 k1); inverse: plain inverse transform.
__global__ __launch_bounds__(kFftThreads) void k_fft_cols(double2 *buf, int64_t M, int M1,
                                                          int logM1, int M2, int C,
                                                          const double2 *__restrict__ tw,
                                                          int64_t Mmax, int inv)
{
    extern __shared__ double2 sc[];
    double2 *x = buf + blockIdx.y * M;
    const int c0 = blockIdx.x * C;
    for (int e = threadIdx.x; e < C * M1; e += blockDim.x) {
        const int n1 = e / C, cc = e - n1 * C;
        sc[cc * M1 + brev(n1, logM1)] = x[(int64_t)M2 * n1 + c0 + cc];
    }
    __syncthreads();
    lds_dit(sc, M1, C, tw, Mmax, inv != 0);
    const int64_t tstep = Mmax / M;
    for (int e = threadIdx.x; e < C * M1; e += blockDim.x) {
        const int k1 = e / C, cc = e - k1 * C;
        double2 v = sc[cc * M1 + k1];
        if (!inv) v = cmul(v, tw[(int64_t)(c0 + cc) * k1 * tstep]);
        x[(int64_t)M2 * k1 + c0 + cc] = v;
    }
}

// Row step of row k1 = blockIdx.x of component blockIdx.y. spec == nullptr:
// forward transform only (weight spectra). Otherwise forward transform,
// product with the spectrum (that of component blockIdx.y at spec_cs
// elements apart, or one shared spectrum with spec_cs = 0), inverse transform
// and the conjugate twiddle w_M^(-n2 k1).
__global__ __launch_bounds__(kFftThreads) void k_fft_rows(double2 *buf, int64_t M, int M2,
                                                          int logM2,
                                                          const double2 *__restrict__ spec,
                                                          int64_t spec_cs,
                                                          const double2 *__restrict__ tw,
                                                          int64_t Mmax)
{
    extern __shared__ double2 sr[];
    const int k1 = blockIdx.x;
    double2 *x = buf + blockIdx.y * M + (int64_t)k1 * M2;
    for (int e = threadIdx.x; e < M2; e += blockDim.x) sr[brev(e, logM2)] = x[e];
    __syncthreads();
    lds_dit(sr, M2, 1, tw, Mmax, false);
    if (!spec) {
        for (int e = threadIdx.x; e < M2; e += blockDim.x) x[e] = sr[e];
        return;
    }
    const double2 *w = spec + blockIdx.y * spec_cs + (int64_t)k1 * M2;
    for (int e = threadIdx.x; e < M2; e += blockDim.x) sr[e] = cmul(sr[e], w[e]);
    __syncthreads();
    lds_dif(sr, M2, tw, Mmax, true);
    const int64_t tstep = Mmax / M;
    for (int p = threadIdx.x; p < M2; p += blockDim.x) {
        const int n2 = brev(p, logM2);
        double2 t = tw[(int64_t)n2 * k1 * tstep];
        t.y = -t.y;
        x[n2] = cmul(sr[p], t);
    }
}

// Target rows T0 + i, i < L, inside the NB blocks: the real part (b table) is
// the predictor sum, the imaginary part (a table) the corrector sum; both go
// to the target block's sums in the MFMA result order. `first`: the square
// is the first writer of these targets (its sources start at row 0).
template <int D>
__global__ void k_fft_scatter(const double2 *__restrict__ buf, int64_t M, int logM, int64_t L,
                              int64_t T0, int NB, double *acc, int first)
{
    const double sc = ldexp(1.0, -logM);
    const int64_t rows = (int64_t)NB * kRows;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t T = T0 + i;
        if (T >= rows) break;
        const int64_t J = T / kRows;
        const int r = (int)(T - J * kRows), rho = r >> 4, sig = r & 15;
        const int e = (sig >> 2) * 64 + 16 * (sig & 3) + rho;
        double *aj = acc + J * 2 * D * kRows + e;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const double2 z = buf[c * M + L - 1 + i];
            double *p = aj + c * kRows, *q = aj + (D + c) * kRows;
            *p = first ? z.x * sc : *p + z.x * sc;
            *q = first ? z.y * sc : *q + z.y * sc;
        }
    }
}

int ilog2(int64_t x)
{
    int l = 0;
    while (((int64_t)1 << (l + 1)) <= x) ++l;
    return l;
}

struct Shape {
    int64_t M;
    int M1, M2, logM, logM1, logM2, C;
};

Shape shape_of(int level)
{
    Shape s;
    s.logM = ilog2((int64_t)2 * kRows) + level;
    s.M = (int64_t)1 << s.logM;
    s.logM2 = std::min(s.logM, ilog2(kRowMax));
    s.logM1 = s.logM - s.logM2;
    s.M1 = 1 << s.logM1;
    s.M2 = 1 << s.logM2;
    s.C = std::max(1, std::min(16, kRowMax / s.M1));
    return s;
}

int grid_of(int64_t n) { return (int)std::min<int64_t>((n + kFftThreads - 1) / kFftThreads, 8192); }

// forward transform of the ncomp arrays in buf (column step, then row step
// with spec: the product and the inverse back through the columns)
hipError_t transform(const Shape &S, double2 *buf, int ncomp, const double2 *spec,
                     int64_t spec_cs, const double2 *tw, int64_t Mmax, hipStream_t st)
{
    if (S.M1 > 1) {
        hipLaunchKernelGGL(k_fft_cols, dim3(S.M2 / S.C, ncomp), dim3(kFftThreads),
                           sizeof(double2) * S.C * S.M1, st, buf, S.M, S.M1, S.logM1, S.M2, S.C,
                           tw, Mmax, 0);
    }
    hipLaunchKernelGGL(k_fft_rows, dim3(S.M1, ncomp), dim3(kFftThreads),
                       sizeof(double2) * S.M2, st, buf, S.M, S.M2, S.logM2, spec, spec_cs, tw,
                       Mmax);
    if (spec && S.M1 > 1) {
        hipLaunchKernelGGL(k_fft_cols, dim3(S.M2 / S.C, ncomp), dim3(kFftThreads),
                           sizeof(double2) * S.C * S.M1, st, buf, S.M, S.M1, S.logM1, S.M2, S.C,
                           tw, Mmax, 1);
    }
    return hipGetLastError();
}

}  // namespace

int fft_far_top_level(int NB, int level)
{
    if (level <= 0 || NB - 4 < (1 << std::min(level, 30))) return -1;
    return ilog2(NB - 4);
}

int64_t fft_far_max_len(int NB, int level)
{
    const int top = fft_far_top_level(NB, level);
    return top < 0 ? 0 : shape_of(top).M;
}

int64_t fft_far_spectra_len(int NB, int level)
{
    const int top = fft_far_top_level(NB, level);
    int64_t n = 0;
    for (int l = level; l <= top; ++l) n += shape_of(l).M;
    return n;
}

namespace {
// weight table sets: one per component with per-component orders
int table_sets(const StepArgs &A, int d) { return A.cmeta ? d : 1; }
}  // namespace

int fft_far_target_end(int NB, int level, int s)
{
    if (level <= 0) return NB;
    const int64_t g = ((int64_t)(s >> level) + 1) << level;  // end of the source's group
    return (int)std::min<int64_t>(NB, g + 3);
}

bool fft_far_mask_prev(int level, int s)
{
    return level > 0 && s > 0 && (s & ((1 << level) - 1)) == 0;
}

hipError_t fft_far_prepare(int d, const StepArgs &A, hipStream_t st)
{
    const int K = table_sets(A, d);
    const int top = fft_far_top_level(A.NB, A.fft_level);
    if (top < 0) return hipSuccess;
    const int64_t Mmax = shape_of(top).M;
    hipLaunchKernelGGL(k_fft_twiddles, dim3(grid_of(Mmax)), dim3(kFftThreads), 0, st, A.fft_tw,
                       Mmax);
    double2 *spec = A.fft_spec;
    for (int l = A.fft_level; l <= top; ++l) {
        const Shape S = shape_of(l);
        const int64_t L = (int64_t)kRows << l;
        hipLaunchKernelGGL(k_fft_gather_w, dim3(grid_of(S.M), K), dim3(kFftThreads), 0, st, A.W,
                           A.wlen, (int64_t)3 * kRows, L, S.M, spec);
        const hipError_t e = transform(S, spec, K, nullptr, 0, A.fft_tw, Mmax, st);
        if (e != hipSuccess) return e;
        spec += S.M * K;
    }
    return hipGetLastError();
}

int fft_far_square_at(int NB, int level, int s)
{
    const int top = fft_far_top_level(NB, level);
    if (top < 0 || s < 0 || s + 5 >= NB) return -1;
    const int l = __builtin_ctz((unsigned)(s + 2));
    return l < level || l > top ? -1 : l;
}

template <int D>
hipError_t fft_far_square_t(const StepArgs &A, int s, hipStream_t st)
{
    // the square whose last source block s + 1 the launch s has just formed;
    // its first target block is s + 5
    const int l = fft_far_square_at(A.NB, A.fft_level, s);
    if (l < 0) return hipSuccess;
    const int top = fft_far_top_level(A.NB, A.fft_level);
    const int64_t j = (int64_t)((s + 2) >> l) / 2;
    const Shape S = shape_of(l);
    const int64_t Mmax = shape_of(top).M;
    const int64_t L = (int64_t)kRows << l;
    const int64_t S0 = 2 * j * L;
    const int K = table_sets(A, D);
    const double2 *spec = A.fft_spec;
    for (int q = A.fft_level; q < l; ++q) spec += shape_of(q).M * K;
    hipLaunchKernelGGL(k_fft_gather_hist, dim3(grid_of(S.M), D), dim3(kFftThreads), 0, st, A.Fc,
                       (int64_t)A.NB * kRows, S0, L, S.M, A.fft_buf);
    const hipError_t e = transform(S, A.fft_buf, D, spec, K > 1 ? S.M : 0, A.fft_tw, Mmax, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fft_scatter<D>), dim3(grid_of(L)), dim3(kFftThreads), 0, st, A.fft_buf,
                       S.M, S.logM, L, S0 + L + 3 * kRows, A.NB, A.acc, S0 == 0 ? 1 : 0);
    return hipGetLastError();
}

hipError_t fft_far_square(int d, const StepArgs &A, int s, hipStream_t st)
{
    switch (d) {
    case 1: return fft_far_square_t<1>(A, s, st);
    case 2: return fft_far_square_t<2>(A, s, st);
    case 3: return fft_far_square_t<3>(A, s, st);
    case 4: return fft_far_square_t<4>(A, s, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fabm
