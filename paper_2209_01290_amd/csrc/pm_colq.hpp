// Column pass with four words per thread (colq_kernels.hip): the column
// stages of the merged transforms for latency-bound calls, R = 2^2 .. 2^7.
#pragma once
#include "pm_internal.hpp"
#include "pm_plan.hpp"

namespace pm {

// Same arguments and batch layout as launch_col; logr in [2, 7], any
// C = N >> logr >= 1.
hipError_t launch_colq(int logr, int kind, bool inv, const ColArgs& a, hipStream_t s);
hipError_t launch_colq(int logr, int kind, bool inv, const ColArgsT<uint32_t>& a, hipStream_t s);

}  // namespace pm
