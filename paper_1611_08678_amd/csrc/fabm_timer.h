// fabm_timer.h -- optional per-kernel timing of a plan (host, internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace fabm {

// Kernel classes reported by fabm_plan_kernel_times (values of fabm.h's
// FABM_KERNEL_* enumeration).
enum : int {
    KC_WEIGHTS = 0,
    KC_DIRECT_WG = 1,
    KC_DIRECT_GRID = 2,
    KC_BLOCKED_STEP = 3,
    KC_HISTORY = 4,
    KC_ADJOINT = 5,
    KC_WIDE_FAR = 6,
    KC_WIDE_BAND = 7,
    KC_FFT_FAR = 8,
    KC_COUNT = 9
};

struct KernelTimer {
    struct Mark {
        int cls;
        hipEvent_t a, b;
    };
    bool on = false;
    std::vector<hipEvent_t> pool;  // reused across calls
    size_t next = 0;
    std::vector<Mark> marks;       // launches of the last instrumented call

    void reset();
    hipError_t begin(int cls, hipStream_t s);
    hipError_t end(hipStream_t s);
    hipError_t totals(double *seconds, int64_t *launches, int n);
    ~KernelTimer();

  private:
    hipError_t event(hipEvent_t *out);
};

}  // namespace fabm
