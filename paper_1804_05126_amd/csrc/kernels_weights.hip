// Solver kernels of the per-cell weights stencil (one translation unit per family).
#define KIOPS_KERNEL_UNIT
#include "op_weights.h"
#include "solver_kernel.h"
#include "kernel_table.h"

namespace kiops {

const void* kernels_weights(bool mixed, int pb, bool group) { return pick_kernel<WeightsOp>(mixed, pb, group); }

}  // namespace kiops
