// rfi_runtime.hpp -- host runtime internals shared by the plan and serving
// parts of librfimad.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rfi_internal.hpp"

struct rfi_plan;

namespace rfi {

// Records a HIP error for rfi_status_string and returns RFI_ERR_HIP.
int hip_fail(hipError_t e);
// Value checks shared by every batch entry point (no buffers).
int validate_values(int elem, int32_t n, const int64_t* L, const int32_t* W, const float* K,
                    const int32_t* M);
int plan_build(int elem, int32_t n, const int64_t* L, const int32_t* W, const float* K,
               const int32_t* M, uint64_t seed, rfi_plan** out);
// sched_override < 0: the plan's own schedule.
int plan_execute(rfi_plan* p, const void* x, void* y, rfi_window_stats* st, hipStream_t s,
                 int sched_override);
void plan_free(rfi_plan* p);
// Free the median-of-MAD and multi-output work tables (rfi_shutdown).
void mom_shutdown();
void multi_shutdown();
// Free the block-power work tables (rfi_shutdown).
void power_shutdown();

}  // namespace rfi
