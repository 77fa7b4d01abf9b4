// Served form: one long-lived launch whose groups of workgroups take solves
// from their own queues as the host admits them; a large request runs on a
// gang of several groups.  A request may be a 2-D 5-point or a 3-D 7-point
// problem in FP64 or mixed precision (p <= 4); the parameter block says which
// (KParams::family) and the group runs the matching solver body.
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

__shared__ double serve_lds[kServeLds];
__shared__ PassCtx<double> serve_pd;
__shared__ PassCtx<float> serve_pf;
__shared__ SmallState serve_S;
__shared__ int serve_phase;

// The parameter block and operator struct are read-only for the whole solve
// (restrict, kept through inlining), so their fields can stay in scalar
// registers.
template <class Op, typename T>
__device__ __forceinline__ unsigned serve_body(const KParams* __restrict__ Pp, const Op* __restrict__ opp,
                                               unsigned epoch) {
  PassCtx<T>* pctx;
  if constexpr (sizeof(T) == 8) pctx = &serve_pd;
  else pctx = &serve_pf;
  const Op op = load_uniform(opp);   // operator fields in scalar registers for the passes
  solve_instance<Op, T>(*Pp, op, serve_S, *pctx, serve_lds, serve_phase, epoch);
  return epoch;
}

// Wave-uniform bounded wait until every slot of fin[0..n) holds at least val.
__device__ inline void wait_all_at_least(const unsigned* fin, int n, unsigned val, uint64_t limit) {
  const uint64_t t0 = (uint64_t)wall_clock64();
  bool all = false;
  while (!all) {
    int ok = 1;
    for (int j = (int)threadIdx.x; j < n; j += 64)
      ok &= __hip_atomic_load(&fin[j], __ATOMIC_RELAXED, KIOPS_AGENT) >= val ? 1 : 0;
    all = __all(ok) != 0;
    const bool late = __builtin_amdgcn_readfirstlane((uint64_t)wall_clock64() - t0 > limit ? 1 : 0) != 0;
    if (!all) {
      if (late) break;
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __threadfence();
}

// Workgroup blockIdx.x belongs to group blockIdx.x / group_size and takes its
// entries from that group's queue.  The queues and parameter blocks are
// fine-grained memory the host writes while this launch runs: tails are read
// with system-scope acquires and done/exited words written with system-scope
// releases (the host reads them).  A request runs on a gang: the aligned run
// of groups the host chose for it, whose workgroups [P.wg0, P.wg0 + P.nwg)
// form the virtual grid of the solve (the host pushes the same parameter
// block to every group of the gang).  Barrier slots are per workgroup
// (arrive[blockIdx.x]) and the epoch starts from P.epoch0, which the host
// sets to the largest epoch any workgroup of the gang has reached, so every
// slot is below the epochs the solve will use.  A group reports an entry
// done only after all of its workgroups have left the solve (fin), so the
// host never reuses a parameter block, control block or workspace that a
// workgroup may still read.
// Up to 256 VGPRs (two waves per SIMD): the four family bodies spill heavily
// under a 168-register cap (three waves per SIMD), and the launch holds one
// workgroup per CU either way, leaving room for another stream's work.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 8)))
kiops_serve_kernel(GroupQueue* __restrict__ queues, unsigned* __restrict__ fin, int group_size,
                   uint64_t fin_limit) {
  __shared__ long long s_entry;
  const int g = (int)blockIdx.x / group_size;
  const int local = (int)blockIdx.x % group_size;
  GroupQueue& Q = queues[g];
  for (unsigned e = 0;; ++e) {
    if (threadIdx.x < 64) {
      const long long r = wait_entry<__HIP_MEMORY_SCOPE_SYSTEM>(Q, e);
      if (threadIdx.x == 0) s_entry = r;
    }
    __syncthreads();
    const long long entry = s_entry;
    __syncthreads();
    if (entry < 0) {
      if (local == 0 && threadIdx.x == 0)
        __hip_atomic_store(&Q.exited, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      return;
    }
    // wave-uniform block pointer: the block's fields go to scalar registers
    const unsigned char* blk = uniform(Q.blocks[uniform((int)(entry % kGroupQueueLen))]);
    const KParams& P = *reinterpret_cast<const KParams*>(blk);
    const void* op = blk + 2048;
    set_vgrid((int)blockIdx.x - P.wg0, P.nwg);
    unsigned epoch = P.epoch0;
    switch (P.family) {
      case kFamily2D:
        epoch = serve_body<Stencil2D<double, 4>, double>(&P, reinterpret_cast<const Stencil2D<double, 4>*>(op), epoch);
        break;
      case kFamily2DMixed:
        epoch = serve_body<Stencil2D<float, 4>, float>(&P, reinterpret_cast<const Stencil2D<float, 4>*>(op), epoch);
        break;
      case kFamily3D:
        epoch = serve_body<Stencil3D<double, 4>, double>(&P, reinterpret_cast<const Stencil3D<double, 4>*>(op), epoch);
        break;
      default:
        epoch = serve_body<Stencil3D<float, 4>, float>(&P, reinterpret_cast<const Stencil3D<float, 4>*>(op), epoch);
        break;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (vblock() == 0) P.ctrl->epoch_end = epoch;
      __threadfence();
      __hip_atomic_store(&fin[blockIdx.x], e + 1, __ATOMIC_RELEASE, KIOPS_AGENT);
    }
    if (local == 0 && threadIdx.x < 64) {
      wait_all_at_least(fin + (size_t)g * group_size, group_size, e + 1, fin_limit);
      if (threadIdx.x == 0) __hip_atomic_store(&Q.done, e + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

const void* kernels_serve() { return (const void*)kiops_serve_kernel; }

}  // namespace kiops
