// Solver kernels of the Stencil2D operator (one translation unit per family),
// with the wide-window one-solve instantiations and the group kernels of the
// shorter tiles the batched form's autotuner may pick.
#define KIOPS_KERNEL_UNIT
#include "op_stencil2d.h"
#include "solver_kernel.h"
#include "kernel_table.h"

namespace kiops {

const void* kernels_stencil2d(bool mixed, int pb, bool group, bool wide, int tile_rows) {
  if (wide && !group) return pick_solve_kernel<Stencil2DWide>(mixed, pb);
  if (group && tile_rows == 8) return pick_group_kernel<Stencil2DRows8>(mixed, pb);
  if (group && tile_rows == 4) return pick_group_kernel<Stencil2DRows4>(mixed, pb);
  return pick_kernel<Stencil2D>(mixed, pb, group);
}

}  // namespace kiops
