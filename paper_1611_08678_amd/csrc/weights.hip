// weights.hip -- generation of the product-integration weights of Section 2
// (b_m for the predictor, a_m and c_m for the corrector) in binary64.
//
// The defining formulas are differences of powers ((m+1)^a - m^a and the
// second difference of s^(a+1)), which cancel catastrophically for large m
// (about 5 of 16 digits are lost at m = 2^20). Each weight is therefore
// evaluated from an algebraically identical form without cancellation:
//
//   b_m = m^a * expm1(a * log1p(1/m)) / Gamma(a+1)                   (m >= 1)
//   a_m = x^(a+1) * 2 * sum_{k>=1} C(a+1, 2k) x^(-2k) / Gamma(a+2),  x = m+1
//         (the even part of the binomial series of (1 +- 1/x)^(a+1); every
//          term is >= 0 for 0 < a <= 1, the terms after the first are <= 0
//          for 1 < a < 2 and vanish at a = 2), evaluated as
//         a x^a / (x Gamma(a+1)) * (1 + sum_{k>=2} C(a+1,2k)/C(a+1,2) x^(2-2k))
//   a_0 = 2 expm1(a ln 2) / Gamma(a+2)
//   c_n = (a+1) n^a sum_{j>=1} C(a, j) j/(j+1) n^(-j) / Gamma(a+2)   (n >= 2)
//       = a n^a / (2 n Gamma(a+1)) * (1 + sum_{j>=2} 2 C(a,j) j / (a (j+1)) n^(1-j))
//   c_1 = (a 2^a - expm1(a ln 2)) / Gamma(a+2),  c_0 = a / Gamma(a+2).
#include "fabm_device.h"
#include "fabm_launch.h"

namespace fabm {

__device__ __forceinline__ double weight_b(double al, double ig1, int64_t m)
{
    if (m == 0) return ig1;
    const double x = (double)m;
    return pow(x, al) * expm1(al * log1p(1.0 / x)) * ig1;
}

__device__ __forceinline__ double weight_a(double al, double ig1, double ig2, int64_t m)
{
    if (m == 0) return 2.0 * expm1(al * 0.69314718055994530942) * ig2;
    const double x = (double)(m + 1);
    const double u2 = 1.0 / (x * x);
    // sum_k C(a+1, 2k) u^(2k) = C(a+1, 2) u^2 * (1 + r_2 + r_3 + ...), with
    // C(a+1, 2) u^2 x^(a+1) / Gamma(a+2) = a x^a / (x Gamma(a+1)). The factors
    // (a + 1 - j) are formed as a + (1 - j), never as (a + 1) - j, which
    // would round a away for small a.
    double r = 1.0, s = 1.0;
    for (int k = 2; k < 200; ++k) {
        const double q = (double)(2 * k);
        r *= (al + (3.0 - q)) * (al + (2.0 - q)) / ((q - 1.0) * q) * u2;
        s += r;
        if (fabs(r) <= 1e-18 * s) break;
    }
    return al * ig1 * (pow(x, al) / x) * s;
}

__device__ __forceinline__ double weight_c(double al, double ig1, double ig2, int64_t n)
{
    if (n == 0) return al * ig2;
    if (n == 1) {
        const double e = expm1(al * 0.69314718055994530942);  // 2^a - 1
        return (al * (1.0 + e) - e) * ig2;
    }
    const double x = (double)n;
    const double v = 1.0 / x;
    // sum_j C(a, j) v^j j/(j+1) = (a v / 2) * (1 + r_2 + ...); (a+1)/Gamma(a+2) = 1/Gamma(a+1)
    double bin = 1.0, s = 1.0;  // bin = C(a, j) v^(j-1) / a
    for (int j = 2; j < 200; ++j) {
        bin *= (al - (double)(j - 1)) / (double)j * v;
        const double term = bin * (2.0 * (double)j / (double)(j + 1));
        s += term;
        if (fabs(term) <= 1e-18 * fabs(s)) break;
    }
    return 0.5 * al * ig1 * (pow(x, al) / x) * s;
}

// One thread per (instance, lag). Instance i writes b, a, c at meta[i].w_off
// (+0, +wlen, +2 wlen); lags run over 0..wlen-1. When W32 is given, b and a
// are also stored rounded to binary32 at 2 w_off / 3 (+0, +wlen).
__global__ __launch_bounds__(256) void k_weights(const InstMeta *__restrict__ meta, int64_t batch,
                                                 double *__restrict__ W, float *__restrict__ W32)
{
    // instances stride over the second grid dimension (at most 65535)
    for (int64_t i = blockIdx.y; i < batch; i += gridDim.y) {
        const InstMeta m = meta[i];
        double *b = W + m.w_off, *a = b + m.wlen, *c = a + m.wlen;
        float *b32 = W32 ? W32 + m.w_off / 3 * 2 : nullptr, *a32 = b32 ? b32 + m.wlen : nullptr;
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m.wlen;
             j += (int64_t)gridDim.x * blockDim.x) {
            const double bj = weight_b(m.alpha, m.ig1, j), aj = weight_a(m.alpha, m.ig1, m.ig2, j);
            b[j] = bj;
            a[j] = aj;
            c[j] = weight_c(m.alpha, m.ig1, m.ig2, j);
            if (b32) {
                b32[j] = (float)bj;
                a32[j] = (float)aj;
            }
        }
    }
}

// Stand-alone table for one alpha (public fabm_weights).
__global__ __launch_bounds__(256) void k_weights_one(double al, double ig1, double ig2, int64_t n,
                                                     double *__restrict__ b, double *__restrict__ a,
                                                     double *__restrict__ c)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        if (b) b[j] = weight_b(al, ig1, j);
        if (a) a[j] = weight_a(al, ig1, ig2, j);
        if (c) c[j] = weight_c(al, ig1, ig2, j);
    }
}

hipError_t launch_weights(const InstMeta *meta, int64_t batch, int64_t maxN, double *W,
                          hipStream_t s, float *W32)
{
    const int64_t blocks = (maxN + 255) / 256;
    dim3 grid((unsigned)(blocks < 4096 ? blocks : 4096), (unsigned)(batch < 65535 ? batch : 65535));
    hipLaunchKernelGGL(k_weights, grid, dim3(256), 0, s, meta, batch, W, W32);
    return hipGetLastError();
}

hipError_t launch_weights_one(double al, double ig1, double ig2, int64_t n, double *b, double *a,
                              double *c, hipStream_t s)
{
    const int64_t blocks = (n + 255) / 256;
    dim3 grid((unsigned)(blocks < 8192 ? blocks : 8192));
    hipLaunchKernelGGL(k_weights_one, grid, dim3(256), 0, s, al, ig1, ig2, n, b, a, c);
    return hipGetLastError();
}

}  // namespace fabm
