// wcc_wide.hpp -- launch of the half-step kernel with two old cells per lane
// (128-cell wave tiles, 127 new cells each; wcc_kernels_wide.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "wcc_internal.hpp"

namespace wcc {

template <class R>
hipError_t launch_half_step_wide(const StepArgs<R>& a, int eq, int P, bool lim, int blocks, int threads,
                                 hipStream_t s);
template <class R>
hipError_t occupancy_half_step_wide(int eq, int P, bool lim, int threads, int* blocks_per_cu);

}  // namespace wcc
