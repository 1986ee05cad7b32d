// schedule.cpp -- host-side schedules of the single-trajectory BLOCKED path
// (see fabm_blocked.h). Pure host code, no device calls.
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

void pipe_schedule(int NB, PipeSchedule &s)
{
    s = PipeSchedule();
    s.NB = NB;
    // far tasks of every target, in source order, each with its own slot
    struct Task { int J, lo, hi, slot; };
    std::vector<std::vector<Task>> by_step((size_t)std::max(NB, 1));
    s.tt_off.assign((size_t)NB + 1, 0);
    std::vector<std::pair<int, int>> tmp;
    for (int J = 0; J < NB; ++J) {
        s.tt_off[(size_t)J] = (int)s.tt_slot.size();
        if (J < 3) continue;  // blocks 0..2 have no far range
        tmp.clear();
        int e = J - 2, sz = 2;  // far range [0, J-2), chunks 2, 4, 8, ... from its near end
        while (e > 0) {
            const int lo = std::max(0, e - sz);
            tmp.push_back({lo, e});
            e = lo;
            sz *= 2;
        }
        std::reverse(tmp.begin(), tmp.end());
        for (auto &c : tmp) {
            const int slot = s.n_slots++;
            s.tt_slot.push_back(slot);
            by_step[(size_t)(c.second - 1)].push_back(Task{J, c.first, c.second, slot});
        }
    }
    s.tt_off[(size_t)NB] = (int)s.tt_slot.size();
    s.step_item_off.assign((size_t)NB + 1, 0);
    s.step_red_off.assign((size_t)NB + 1, 0);
    for (int I = 0; I < NB; ++I) {
        s.step_item_off[(size_t)I] = (int)s.items.size();
        s.step_red_off[(size_t)I] = (int)s.reds.size();
        auto &v = by_step[(size_t)I];
        std::sort(v.begin(), v.end(), [](const Task &a, const Task &b) { return a.J < b.J; });
        int scratch = 0;
        for (const Task &t : v) {
            const int n = (t.hi - t.lo + kItemBlocks - 1) / kItemBlocks;
            if (n == 1) {
                s.items.push_back(int4{t.J, t.lo, t.hi, t.slot});
                continue;
            }
            const int first = scratch;
            for (int a = t.lo; a < t.hi; a += kItemBlocks)
                s.items.push_back(int4{t.J, a, std::min(a + kItemBlocks, t.hi), -(scratch++) - 1});
            s.reds.push_back(int4{t.slot, first, n, 0});
        }
        s.max_scratch = std::max(s.max_scratch, scratch);
    }
    s.step_item_off[(size_t)NB] = (int)s.items.size();
    s.step_red_off[(size_t)NB] = (int)s.reds.size();
}

}  // namespace fabm
