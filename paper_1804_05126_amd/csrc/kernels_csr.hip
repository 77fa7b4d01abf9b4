// Solver kernels of the CsrOp operator (one translation unit per family).
#define KIOPS_KERNEL_UNIT
#include "op_csr.h"
#include "solver_kernel.h"
#include "kernel_table.h"

namespace kiops {

const void* kernels_csr(bool mixed, int pb, bool group) { return pick_kernel<CsrOp>(mixed, pb, group); }

}  // namespace kiops
