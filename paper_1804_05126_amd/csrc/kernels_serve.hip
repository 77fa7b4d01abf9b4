// Served form: one long-lived launch whose groups of workgroups take solves
// from their own queues as the host admits them.  A request may be a 2-D
// 5-point or a 3-D 7-point problem in FP64 or mixed precision (p <= 4); the
// parameter block says which (KParams::family) and the group runs the matching
// solver body.
#define KIOPS_KERNEL_UNIT
#include "op_stencil2d.h"
#include "op_stencil3d.h"
#include "solver_kernel.h"
#include "kernel_table.h"

namespace kiops {

namespace {
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kServeLds = cmax(cmax(Stencil3D<double, 4>::kLdsDoubles, Stencil2D<double, 4>::kLdsDoubles),
                               kLdsDoubles);
}  // namespace

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 8)))
kiops_serve_kernel(GroupQueue* __restrict__ queues, int group_size) {
  __shared__ double lds[kServeLds];
  __shared__ PassCtx<double> pd;
  __shared__ PassCtx<float> pf;
  __shared__ SmallState S;
  __shared__ int s_phase;
  __shared__ long long s_entry;
  const int g = (int)blockIdx.x / group_size;
  set_vgrid((int)blockIdx.x % group_size, group_size);
  GroupQueue& Q = queues[g];
  unsigned epoch = 0;
  for (unsigned e = 0;; ++e) {
    if (threadIdx.x < 64) {
      const long long r = wait_entry(Q, e);
      if (threadIdx.x == 0) s_entry = r;
    }
    __syncthreads();
    const long long entry = s_entry;
    __syncthreads();
    if (entry < 0) {
      if (vblock() == 0 && threadIdx.x == 0) __hip_atomic_store(&Q.exited, 1u, __ATOMIC_RELEASE, KIOPS_AGENT);
      return;
    }
    const unsigned char* blk = Q.blocks[entry % kGroupQueueLen];
    const KParams& P = *reinterpret_cast<const KParams*>(blk);
    const void* op = blk + 2048;
    switch (P.family) {
      case kFamily2D:
        solve_instance<Stencil2D<double, 4>, double>(P, *reinterpret_cast<const Stencil2D<double, 4>*>(op), S, pd,
                                                     lds, s_phase, epoch);
        break;
      case kFamily2DMixed:
        solve_instance<Stencil2D<float, 4>, float>(P, *reinterpret_cast<const Stencil2D<float, 4>*>(op), S, pf,
                                                   lds, s_phase, epoch);
        break;
      case kFamily3D:
        solve_instance<Stencil3D<double, 4>, double>(P, *reinterpret_cast<const Stencil3D<double, 4>*>(op), S, pd,
                                                     lds, s_phase, epoch);
        break;
      default:
        solve_instance<Stencil3D<float, 4>, float>(P, *reinterpret_cast<const Stencil3D<float, 4>*>(op), S, pf,
                                                   lds, s_phase, epoch);
        break;
    }
    if (vblock() == 0 && threadIdx.x == 0) {
      __threadfence();
      __hip_atomic_store(&Q.done, e + 1, __ATOMIC_RELEASE, KIOPS_AGENT);
    }
  }
}

const void* kernels_serve() { return (const void*)kiops_serve_kernel; }

}  // namespace kiops
