// timer.cpp -- optional per-kernel timing of a plan's launches: an event pair
// is recorded on the launching stream around every instrumented kernel, and
// the elapsed times are summed per kernel class when queried.
#include "fabm_timer.h"

namespace fabm {

hipError_t KernelTimer::event(hipEvent_t *out)
{
    if (next < pool.size()) {
        *out = pool[next++];
        return hipSuccess;
    }
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);  // timing enabled
    if (r != hipSuccess) return r;
    pool.push_back(e);
    ++next;
    *out = e;
    return hipSuccess;
}

void KernelTimer::reset()
{
    next = 0;
    marks.clear();
}

hipError_t KernelTimer::begin(int cls, hipStream_t s)
{
    if (!on) return hipSuccess;
    Mark m{};
    m.cls = cls;
    hipError_t r = event(&m.a);
    if (r == hipSuccess) r = hipEventRecord(m.a, s);
    if (r != hipSuccess) return r;
    marks.push_back(m);
    return hipSuccess;
}

hipError_t KernelTimer::end(hipStream_t s)
{
    if (!on || marks.empty()) return hipSuccess;
    hipError_t r = event(&marks.back().b);
    if (r == hipSuccess) r = hipEventRecord(marks.back().b, s);
    return r;
}

hipError_t KernelTimer::totals(double *seconds, int64_t *launches, int n)
{
    for (int c = 0; c < n; ++c) {
        seconds[c] = 0.0;
        launches[c] = 0;
    }
    for (const Mark &m : marks) {
        hipError_t r = hipEventSynchronize(m.b);
        if (r != hipSuccess) return r;
        float ms = 0.f;
        r = hipEventElapsedTime(&ms, m.a, m.b);
        if (r != hipSuccess) return r;
        if (m.cls >= 0 && m.cls < n) {
            seconds[m.cls] += 1e-3 * ms;
            launches[m.cls] += 1;
        }
    }
    return hipSuccess;
}

KernelTimer::~KernelTimer()
{
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

}  // namespace fabm
