// schedule.cpp -- host-side schedules of the BLOCKED path: the per-launch
// workgroup counts of the batched step pipeline, and the task schedule of the
// single-launch persistent variant (not dispatched; see
// blocked_persistent.hip). Pure host code, no device calls.
#include <algorithm>
#include <tuple>
#include <vector>

#include "fabm_blocked.h"

namespace fabm {

namespace {

// Chunks of the far range [0, J-1) for target block J, from the nearest
// (ending at J-1, one block) outwards, each twice as long as the previous.
template <class Fn>
void for_each_chunk(int J, Fn fn)
{
    int e = J - 1, s = 1;
    while (e > 0) {
        const int lo = std::max(0, e - s);
        fn(lo, e);
        e = lo;
        s *= 2;
    }
}

}  // namespace

int blocked_count_tasks(int NB)
{
    int n = 0;
    for (int J = 2; J < NB; ++J) for_each_chunk(J, [&](int, int) { ++n; });
    return n;
}

void blocked_schedule(int NB, int4 *tasks, int *queue, int *task_off)
{
    int n = 0;
    std::vector<int4> tmp;
    for (int J = 0; J < NB; ++J) {
        task_off[J] = n;  // blocks 0 and 1 have no far sources
        if (J < 2) continue;
        tmp.clear();
        for_each_chunk(J, [&](int lo, int hi) { tmp.push_back(int4{J, lo, hi, 0}); });
        std::reverse(tmp.begin(), tmp.end());  // source order
        for (const int4 &t : tmp) tasks[n++] = t;
    }
    task_off[NB] = n;
    // the chunk end decides when a task can start; ties go to the earlier target
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (tasks[a].z != tasks[b].z) return tasks[a].z < tasks[b].z;
        return tasks[a].x < tasks[b].x;
    });
    std::copy(order.begin(), order.end(), queue);
}

void batch_schedule(int64_t batch, const int32_t *NB, BatchSchedule &S)
{
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
        // far windows go in pairs of source blocks: odd launches take every
        // target J >= s + 3, even launches target s + 3 only (k_step_batch)
        const int nf = s >= 0 ? count_at_least(s + 4) : 0;
        const bool pair = s > 0 && (s & 1) != 0;
        for (int j = 0; j < nf; ++j) {
            const int all = NB[S.order[(size_t)j]] - (s + 3);
            const int targets = pair ? all : 1;
            S.far_off.push_back(S.far_off.back() + (targets + 3) / 4);
            S.far_off_single.push_back(S.far_off_single.back() + (all + 3) / 4);
        }
        S.nfar[k] = nf;
    }
}

}  // namespace fabm
