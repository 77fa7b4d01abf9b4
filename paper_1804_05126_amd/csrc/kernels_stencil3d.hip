// Solver kernels of the Stencil3D operator (one translation unit per family),
// with the narrow-window one-solve instantiations.
#define KIOPS_KERNEL_UNIT
#include "op_stencil3d.h"
#include "solver_kernel.h"
#include "kernel_table.h"

namespace kiops {

const void* kernels_stencil3d(bool mixed, int pb, bool group, bool narrow) {
  if (narrow && !group) return pick_solve_kernel<Stencil3DNarrow>(mixed, pb);
  return pick_kernel<Stencil3D>(mixed, pb, group);
}

}  // namespace kiops
