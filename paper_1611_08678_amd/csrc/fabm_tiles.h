// fabm_tiles.h -- the far-history tile contraction of the BLOCKED path on
// FP64 MFMA (device code, internal).
//
// Target rows of block J (L = 256 rows) and sources in blocks [I0, I1), with
// I1 <= J - 1 so every source precedes every target. The sums
//   S_w[r] = sum_k w[JL + r - 1 - k] f_k,   w in {b, a}
// form a Toeplitz product. Polyphase split: r = 16 rho + sigma and
// k = 16 kappa + tau. The 16x16 block W_q[sigma][tau] = w[16 q + sigma - tau - 1]
// depends only on the column lag q = (JL/16 + rho) - kappa, so for each q
//   S[:, rho] += W_q . F[:, JL/16 + rho - q]      (16x16 times 16x16)
// on v_mfma_f64_16x16x4f64 (four K=4 slices per q). Each accumulator column
// stays in place while the B operand is a sliding window of history columns;
// columns outside [I0, I1) are masked to zero. The q range is split over the
// four wavefronts and the partial results are added in LDS in a fixed order.
#pragma once

#include "fabm_device.h"

namespace fabm {

constexpr int kBlk = 256;   // rows per block
constexpr int kTile = 16;   // polyphase factor = MFMA edge

typedef double dbl4 __attribute__((ext_vector_type(4)));

// All 256 threads of the workgroup call this. `red` is LDS of 4*2*D*256
// doubles. On return thread `tid` holds in sP[i], sC[i] the sums of target row
// JL + tid for component i (b weights, a weights).
template <int D>
__device__ __forceinline__ void toeplitz_block_fp64(const double *__restrict__ wb,
                                                    const double *__restrict__ wa,
                                                    const double *__restrict__ Fc, int64_t pitch,
                                                    int J, int I0, int I1, double *red,
                                                    double (&sP)[D], double (&sC)[D])
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int rho = lane & 15, kq = lane >> 4;  // A row / B column, K slot within a 4-slice
    const int64_t colT = (int64_t)J * (kBlk / kTile);
    const int64_t k0 = (int64_t)I0 * (kBlk / kTile), k1 = (int64_t)I1 * (kBlk / kTile);
    const int64_t qlo = colT - k1 + 1, nq = (k1 - k0) + kTile - 1;
    const int64_t qa = qlo + (nq * wv) / 4, qb = qlo + (nq * (wv + 1)) / 4;

    dbl4 acc[D][2];
#pragma unroll
    for (int i = 0; i < D; ++i) acc[i][0] = acc[i][1] = (dbl4){0.0, 0.0, 0.0, 0.0};

    // operands of one q: A slices of both weight tables, B slices of each component
    auto load_q = [&](int64_t q, double (&ab)[4], double (&aa)[4], double (&bf)[D][4]) {
        const int64_t col = colT + rho - q;  // history column of this lane's B entries
        const bool ok = col >= k0 && col < k1;
        const int64_t wbase = kTile * q + rho - kq - 1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            ab[j] = wb[wbase - 4 * j];
            aa[j] = wa[wbase - 4 * j];
            // masked lanes read row 0 (always in bounds) and use zero
            const int64_t row = ok ? kTile * col + 4 * j + kq : 0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double v = Fc[i * pitch + row];
                bf[i][j] = ok ? v : 0.0;
            }
        }
    };
    double ab[4], aa[4], bf[D][4];
    if (qa < qb) load_q(qa, ab, aa, bf);
    for (int64_t q = qa; q < qb; ++q) {
        // issue the next q's loads before this q's products (latency hidden
        // behind 24 MFMAs)
        double nab[4], naa[4], nbf[D][4];
        if (q + 1 < qb) load_q(q + 1, nab, naa, nbf);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < D; ++i) {
                acc[i][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ab[j], bf[i][j], acc[i][0], 0, 0, 0);
                acc[i][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[j], bf[i][j], acc[i][1], 0, 0, 0);
            }
        if (q + 1 < qb) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                ab[j] = nab[j];
                aa[j] = naa[j];
#pragma unroll
                for (int i = 0; i < D; ++i) bf[i][j] = nbf[i][j];
            }
        }
    }
    // accumulator element v of lane l is D[sigma = 4 v + l/16][rho = l % 16]
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = kTile * rho + 4 * v + kq;
            red[(wv * 2 * D + i) * kBlk + row] = acc[i][0][v];
            red[(wv * 2 * D + D + i) * kBlk + row] = acc[i][1][v];
        }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < D; ++i) {
        double p = red[i * kBlk + tid], c = red[(D + i) * kBlk + tid];
#pragma unroll
        for (int w = 1; w < 4; ++w) {
            p += red[(w * 2 * D + i) * kBlk + tid];
            c += red[(w * 2 * D + D + i) * kBlk + tid];
        }
        sP[i] = p;
        sC[i] = c;
    }
    __syncthreads();  // red may be reused by the caller
}

}  // namespace fabm
