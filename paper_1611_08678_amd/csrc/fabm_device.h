// fabm_device.h -- device-side building blocks shared by the kernels of the
// library: per-instance metadata, the right-hand sides f(t, y; theta) of the
// supported systems, wavefront reductions and inter-workgroup flags.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fabm {

constexpr int kWave = 64;

// Per-instance scalars and offsets, prepared on the host for every call.
// h^alpha and the Gamma reciprocals are computed on the host (std::pow,
// std::tgamma) so no kernel evaluates Gamma.
struct InstMeta {
    double alpha;
    double h;
    double ha;   // h^alpha
    double ig1;  // 1 / Gamma(alpha + 1)
    double ig2;  // 1 / Gamma(alpha + 2)
    int64_t N;       // number of steps (targets t = 1..N)
    int64_t row_off; // first row of this instance in the caller's y_out
    int64_t w_off;   // offset (doubles) of its weight tables: b at w_off, a at +N, c at +2N
    int64_t p_off;   // offset (doubles) of its parameters
    int64_t f_off;   // first row of this instance in the (packed) history buffer
    int64_t wlen;    // length of each weight table (>= N; padded for blocked tiles)
};
static_assert(sizeof(InstMeta) == 88, "InstMeta layout");

enum : int {
    SYS_LINEAR = 0,
    SYS_CHEN = 1,
    SYS_ROSSLER = 2,
    SYS_VDP = 3,
    SYS_FINANCIAL = 4,
    SYS_HINDMARSH_ROSE = 5,
    // internal: f is read from a given history (teacher-forced history sums);
    // theta points at the rows [N + 1][D] and t is the row index
    SYS_TEACHER = 6
};

// Entries of theta of each system (LINEAR: A, b0, b1).
constexpr int n_params_of_sys(int sys, int d)
{
    return sys == SYS_LINEAR ? d * d + 2 * d
           : sys == SYS_VDP ? 1
           : sys == SYS_HINDMARSH_ROSE ? 8
           : sys == SYS_TEACHER ? 0
                                       : 3;
}

// f(t, y; theta) for the fixed set of systems (textbook forms; parameter
// layout as documented in fabm.h). D is the state dimension. Every product
// that meets a sum is written as an explicit fma, so the rounding of each
// system is fixed by this source and not by the compiler's contraction.
template <int SYS, int D>
__device__ __forceinline__ void rhs(double t, const double (&y)[D], double (&f)[D],
                                    const double *__restrict__ p)
{
    if constexpr (SYS == SYS_LINEAR) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double s = fma(p[D * D + D + i], t, p[D * D + i]);
#pragma unroll
            for (int j = 0; j < D; ++j) s = fma(p[i * D + j], y[j], s);
            f[i] = s;
        }
    } else if constexpr (SYS == SYS_CHEN) {
        const double a = p[0], b = p[1], c = p[2];
        f[0] = a * (y[1] - y[0]);
        f[1] = fma(y[0], (c - a) - y[2], c * y[1]);  // (c-a)x - xz + cy
        f[2] = fma(y[0], y[1], -b * y[2]);
    } else if constexpr (SYS == SYS_ROSSLER) {
        const double a = p[0], b = p[1], c = p[2];
        f[0] = -y[1] - y[2];
        f[1] = fma(a, y[1], y[0]);
        f[2] = fma(y[2], y[0] - c, b);
    } else if constexpr (SYS == SYS_VDP) {
        const double mu = p[0];
        f[0] = y[1];
        f[1] = fma(mu * fma(-y[0], y[0], 1.0), y[1], -y[0]);
    } else if constexpr (SYS == SYS_FINANCIAL) {
        const double a = p[0], b = p[1], c = p[2];
        f[0] = fma(y[1] - a, y[0], y[2]);
        f[1] = fma(-y[0], y[0], fma(-b, y[1], 1.0));
        f[2] = fma(-c, y[2], -y[0]);
    } else if constexpr (SYS == SYS_HINDMARSH_ROSE) {
        // theta = (a, b, c, d, r, s, xr, I)
        const double x = y[0], x2 = x * x;
        f[0] = fma(x2, fma(-p[0], x, p[1]), y[1] - y[2] + p[7]);
        f[1] = fma(-p[3], x2, p[2] - y[1]);
        f[2] = p[4] * fma(p[5], x - p[6], -y[2]);
    } else if constexpr (SYS == SYS_TEACHER) {
        // the given history row at index t (t is an integer: the grid step is 1)
        const int64_t r = (int64_t)t;
#pragma unroll
        for (int i = 0; i < D; ++i) f[i] = p[r * D + i];
    }
}

// Transposed Jacobian products of f for the reverse pass: gy += (df/dy)^T w
// and gth += (df/dtheta)^T w at (t, y). Derivatives of the forms in rhs().
template <int SYS, int D>
__device__ __forceinline__ void rhs_vjp(double t, const double (&y)[D], const double (&w)[D],
                                        const double *__restrict__ p, double (&gy)[D],
                                        double *gth)
{
    if constexpr (SYS == SYS_LINEAR) {
        // f_i = sum_j A_ij y_j + b0_i + b1_i t
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double s = gy[j];
#pragma unroll
            for (int i = 0; i < D; ++i) s = fma(p[i * D + j], w[i], s);
            gy[j] = s;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
#pragma unroll
            for (int j = 0; j < D; ++j) gth[i * D + j] = fma(w[i], y[j], gth[i * D + j]);
            gth[D * D + i] += w[i];
            gth[D * D + D + i] = fma(w[i], t, gth[D * D + D + i]);
        }
    } else if constexpr (SYS == SYS_CHEN) {
        const double a = p[0], b = p[1], c = p[2];
        gy[0] += -a * w[0] + (c - a - y[2]) * w[1] + y[1] * w[2];
        gy[1] += a * w[0] + c * w[1] + y[0] * w[2];
        gy[2] += -y[0] * w[1] - b * w[2];
        gth[0] += (y[1] - y[0]) * w[0] - y[0] * w[1];
        gth[1] += -y[2] * w[2];
        gth[2] += (y[0] + y[1]) * w[1];
    } else if constexpr (SYS == SYS_ROSSLER) {
        const double a = p[0], c = p[2];
        gy[0] += w[1] + y[2] * w[2];
        gy[1] += -w[0] + a * w[1];
        gy[2] += -w[0] + (y[0] - c) * w[2];
        gth[0] += y[1] * w[1];
        gth[1] += w[2];
        gth[2] += -y[2] * w[2];
    } else if constexpr (SYS == SYS_VDP) {
        const double mu = p[0];
        gy[0] += (-2.0 * mu * y[0] * y[1] - 1.0) * w[1];
        gy[1] += w[0] + mu * (1.0 - y[0] * y[0]) * w[1];
        gth[0] += (1.0 - y[0] * y[0]) * y[1] * w[1];
    } else if constexpr (SYS == SYS_FINANCIAL) {
        const double a = p[0], b = p[1], c = p[2];
        gy[0] += (y[1] - a) * w[0] - 2.0 * y[0] * w[1] - w[2];
        gy[1] += y[0] * w[0] - b * w[1];
        gy[2] += w[0] - c * w[2];
        gth[0] += -y[0] * w[0];
        gth[1] += -y[1] * w[1];
        gth[2] += -y[2] * w[2];
    } else if constexpr (SYS == SYS_HINDMARSH_ROSE) {
        const double a = p[0], b = p[1], d = p[3], r = p[4], s = p[5], xr = p[6];
        const double x = y[0], x2 = x * x;
        gy[0] += (-3.0 * a * x2 + 2.0 * b * x) * w[0] - 2.0 * d * x * w[1] + r * s * w[2];
        gy[1] += w[0] - w[1];
        gy[2] += -w[0] - r * w[2];
        gth[0] += -x2 * x * w[0];
        gth[1] += x2 * w[0];
        gth[2] += w[1];
        gth[3] += -x2 * w[1];
        gth[4] += (s * (x - xr) - y[2]) * w[2];
        gth[5] += r * (x - xr) * w[2];
        gth[6] += -r * s * w[2];
        gth[7] += w[0];
    }
}

// Initial values (eq. (1)): an order above one needs y'(0) besides y(0), and
// every step starts from the Taylor polynomial y(0) + t y'(0). `slope` loads
// y'(0), or zeros for orders up to one or when none is given.
template <int D>
__device__ __forceinline__ void load_slope(const InstMeta &m, const double *y1, double (&v)[D])
{
    const bool on = y1 != nullptr && m.alpha > 1.0;
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = on ? y1[i] : 0.0;
}

// Initial part of the step at time tt: y(0) + tt y'(0).
template <int D>
__device__ __forceinline__ void taylor_base(double tt, const double (&y0)[D],
                                            const double (&y1)[D], double (&base)[D])
{
#pragma unroll
    for (int i = 0; i < D; ++i) base[i] = fma(tt, y1[i], y0[i]);
}

// One corrector step from the two history sums (Section 2): returns y_t and
// f_t, given P_t, C_t, the initial part of the step (y0, or its Taylor
// polynomial at t_t for orders above one) and the step scalars.
template <int SYS, int D>
__device__ __forceinline__ void pece_update(const InstMeta &m, double tt, const double (&base)[D],
                                            const double (&P)[D], const double (&Cs)[D],
                                            const double *__restrict__ p, double (&y)[D],
                                            double (&f)[D])
{
    double yp[D], fp[D];
#pragma unroll
    for (int i = 0; i < D; ++i) yp[i] = fma(m.ha, P[i], base[i]);
    rhs<SYS, D>(tt, yp, fp, p);
#pragma unroll
    for (int i = 0; i < D; ++i) y[i] = fma(m.ha, fma(fp[i], m.ig2, Cs[i]), base[i]);
    rhs<SYS, D>(tt, y, f, p);
}

template <int D>
__device__ __forceinline__ bool finite_all(const double (&v)[D])
{
    bool ok = true;
#pragma unroll
    for (int i = 0; i < D; ++i) ok = ok && isfinite(v[i]);
    return ok;
}

// Butterfly sum over a 64-lane wavefront; every lane receives the total.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Flags shared between workgroups on different XCDs (each XCD has its own
// L2): read with an agent-scope atomic load (emitted for gfx950 as
// global_load_dword with the sc1 bit, which reads at the device's coherence
// point, past the XCD's own L2) and raised with an agent-scope atomic
// read-modify-write (performed at that point).
__device__ __forceinline__ uint32_t flag_read(uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void flag_max(uint32_t *p, uint32_t v)
{
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace fabm
