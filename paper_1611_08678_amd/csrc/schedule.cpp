// schedule.cpp -- host-side schedule of the batched BLOCKED step pipeline:
// instance order and per-launch workgroup counts. Pure host code, no device
// calls.
#include <algorithm>
#include <tuple>
#include <vector>

#include "fabm_blocked.h"

namespace fabm {

void batch_schedule(int64_t batch, const int32_t *NB, BatchSchedule &S, int P)
{
    S.P = P;
    S.order.resize((size_t)batch);
    for (int64_t i = 0; i < batch; ++i) S.order[(size_t)i] = (int)i;
    std::stable_sort(S.order.begin(), S.order.end(), [&](int a, int b) { return NB[a] > NB[b]; });
    S.max_NB = batch > 0 ? NB[S.order[0]] : 0;
    const int L = S.max_NB;  // launches s = -1 .. L-2, index k = s + 1
    S.nband.assign((size_t)std::max(L, 1), 0);
    S.nnear.assign((size_t)std::max(L, 1), 0);
    S.nfar.assign((size_t)std::max(L, 1), 0);
    S.far_base.assign((size_t)std::max(L, 1), 0);
    S.far_off.clear();
    S.far_off_single.clear();
    // instances with NB >= x form a prefix of `order`
    auto count_at_least = [&](int x) {
        int lo = 0, hi = (int)batch;
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (NB[S.order[(size_t)mid]] >= x) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    for (int s = -1; s <= L - 2; ++s) {
        const size_t k = (size_t)(s + 1);
        S.nband[k] = count_at_least(s + 2);
        S.nnear[k] = s >= 0 ? count_at_least(s + 3) : 0;
        S.far_base[k] = (int)S.far_off.size();
        S.far_off.push_back(0);
        S.far_off_single.push_back(0);
        // far windows in groups of P source blocks: launch s with
        // (s + 1) % P == 0 takes every target J >= s + 3, the others the
        // targets J <= sb + 2 before the next such launch sb (k_step_batch)
        const int nf = s >= 0 ? count_at_least(s + 4) : 0;
        const bool big = P == 1 || (s >= P - 1 && (s + 1) % P == 0);
        const int sb = s + (P - 1 - (s >= 0 ? s % P : 0));
        for (int j = 0; j < nf; ++j) {
            const int all = NB[S.order[(size_t)j]] - (s + 3);
            const int targets = big ? all : std::min(all, sb - s);
            S.far_off.push_back(S.far_off.back() + (targets + 3) / 4);
            S.far_off_single.push_back(S.far_off_single.back() + (all + 3) / 4);
        }
        S.nfar[k] = nf;
    }
}

}  // namespace fabm
