// Solver kernels of the Stencil2D operator (one translation unit per family).
#define KIOPS_KERNEL_UNIT
#include "op_stencil2d.h"
#include "solver_kernel.h"
#include "kernel_table.h"

namespace kiops {

const void* kernels_stencil2d(bool mixed, int pb, bool group) { return pick_kernel<Stencil2D>(mixed, pb, group); }

}  // namespace kiops
