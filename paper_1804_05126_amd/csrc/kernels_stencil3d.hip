// Solver kernels of the Stencil3D operator (one translation unit per family).
#define KIOPS_KERNEL_UNIT
#include "op_stencil3d.h"
#include "solver_kernel.h"
#include "kernel_table.h"

namespace kiops {

const void* kernels_stencil3d(bool mixed, int pb, bool group) { return pick_kernel<Stencil3D>(mixed, pb, group); }

}  // namespace kiops
