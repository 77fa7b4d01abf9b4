// Solver kernels of the Stencil2D operator (one translation unit per family),
// with the wide-window one-solve instantiations.
#define KIOPS_KERNEL_UNIT
#include "op_stencil2d.h"
#include "solver_kernel.h"
#include "kernel_table.h"

namespace kiops {

const void* kernels_stencil2d(bool mixed, int pb, bool group, bool wide) {
  if (wide && !group) return pick_solve_kernel<Stencil2DWide>(mixed, pb);
  return pick_kernel<Stencil2D>(mixed, pb, group);
}

}  // namespace kiops
