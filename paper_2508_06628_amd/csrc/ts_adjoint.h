// Shared pieces of the reverse-mode (adjoint) kernels.
#pragma once

#include "ts_internal.h"

namespace ts {

// adj_params[k] += sum over the n_slots slots of slots[q][k] (k < kAdjSlot); one small launch.
int launch_sum_slots(int64_t n_slots, const double *slots, double *adj_params, hipStream_t st);

}  // namespace ts
