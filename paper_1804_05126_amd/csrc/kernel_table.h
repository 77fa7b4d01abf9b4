// Entry addresses of the solver kernels: the one-solve kernel (group = false)
// and the group kernel of the batched and served forms (group = true), for a
// float (mixed) or double basis and a p-bucket pb in {0, 2, 4, 8}.  Each
// operator family lives in its own translation unit.
#pragma once

namespace kiops {

// wide: IOP windows of 3, 4 (one-solve kernel); tile_rows: 16, 8 or 4 (group kernel)
const void* kernels_stencil2d(bool mixed, int pb, bool group, bool wide, int tile_rows = 16);
const void* kernels_stencil2d_march(bool mixed, int pb);   // row-marching 5-point pass (one-solve kernel)
const void* kernels_stencil3d(bool mixed, int pb, bool group, bool narrow);   // narrow: IOP windows of 1, 2 (one-solve kernel)
const void* kernels_csr(bool mixed, int pb, bool group);
const void* kernels_weights(bool mixed, int pb, bool group);   // per-cell weights stencil
const void* kernels_serve();   // served form: 2-D and 3-D stencils, FP64 and mixed, p <= 4
// y = A x in FP64 outside a solve (kernels_apply.hip), enqueued on st
hipError_t launch_apply(const kiops_operator_desc& d, int64_t N, const double* x, double* y, hipStream_t st);

#ifdef KIOPS_KERNEL_UNIT
template <template <typename, int> class OP>
const void* pick_kernel(bool mixed, int pb, bool group) {
#define KIOPS_K(T, PB) \
  (group ? (const void*)kiops_group_kernel<OP<T, PB>, T> : (const void*)kiops_solve_kernel<OP<T, PB>, T>)
  switch (pb) {
    case 0: return mixed ? KIOPS_K(float, 0) : KIOPS_K(double, 0);
    case 2: return mixed ? KIOPS_K(float, 2) : KIOPS_K(double, 2);
    case 4: return mixed ? KIOPS_K(float, 4) : KIOPS_K(double, 4);
    default: return mixed ? KIOPS_K(float, 8) : KIOPS_K(double, 8);
  }
#undef KIOPS_K
}
// the group kernel only
template <template <typename, int> class OP>
const void* pick_group_kernel(bool mixed, int pb) {
  switch (pb) {
    case 0: return mixed ? (const void*)kiops_group_kernel<OP<float, 0>, float> : (const void*)kiops_group_kernel<OP<double, 0>, double>;
    case 2: return mixed ? (const void*)kiops_group_kernel<OP<float, 2>, float> : (const void*)kiops_group_kernel<OP<double, 2>, double>;
    case 4: return mixed ? (const void*)kiops_group_kernel<OP<float, 4>, float> : (const void*)kiops_group_kernel<OP<double, 4>, double>;
    default: return mixed ? (const void*)kiops_group_kernel<OP<float, 8>, float> : (const void*)kiops_group_kernel<OP<double, 8>, double>;
  }
}
// the one-solve kernel only
template <template <typename, int> class OP>
const void* pick_solve_kernel(bool mixed, int pb) {
  switch (pb) {
    case 0: return mixed ? (const void*)kiops_solve_kernel<OP<float, 0>, float> : (const void*)kiops_solve_kernel<OP<double, 0>, double>;
    case 2: return mixed ? (const void*)kiops_solve_kernel<OP<float, 2>, float> : (const void*)kiops_solve_kernel<OP<double, 2>, double>;
    case 4: return mixed ? (const void*)kiops_solve_kernel<OP<float, 4>, float> : (const void*)kiops_solve_kernel<OP<double, 4>, double>;
    default: return mixed ? (const void*)kiops_solve_kernel<OP<float, 8>, float> : (const void*)kiops_solve_kernel<OP<double, 8>, double>;
  }
}
#endif

}  // namespace kiops
