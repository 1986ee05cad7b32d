// schedule.cpp -- host-side task schedule of the single-launch persistent
// variant of the BLOCKED path (not dispatched; see blocked_persistent.hip).
// Pure host code, no device calls.
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

}  // namespace fabm
