// One-solve kernels of the row-marching 5-point pass (large 2-D grids, IOP
// windows of one or two vectors).
#define KIOPS_KERNEL_UNIT
#include "op_stencil2d_march.h"
#include "solver_kernel.h"
#include "kernel_table.h"

namespace kiops {

const void* kernels_stencil2d_march(bool mixed, int pb) { return pick_solve_kernel<Stencil2DMarch>(mixed, pb); }

}  // namespace kiops
