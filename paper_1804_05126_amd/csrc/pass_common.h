// Per-pass context shared by the operator passes.
//
// One pass produces the next Krylov vector without a second sweep over memory
// (Algorithm 2, with the normalisation deferred by one step):
//
//   R_kp = a * U_{kp-1} + sum_{i in [flo, kp-1]} bw[i] R_i      (orthogonalised, unnormalised)
//   U_kp = A~ R_kp = A x(R_kp) + nu B y(R_kp)                   (Theorem 1)
//
// with v_i = R_i * sinv[i] and U_{kp-1} = A~ R_{kp-1}.  Stencil operators
// recompute U_{kp-1} on the fly from R_{kp-1} (two-level stencil over a halo
// of two), so a pass reads R_{kp-1} and the older window vectors once and
// writes R_kp once.  The same pass accumulates every inner product the next
// epilogue needs:  <R_kp,R_kp>, <U_kp,U_kp>, <R_i,R_kp>, <R_i,U_kp> (i in
// [dlo, kp-1]) and <R_kp,U_kp>.
#pragma once

#include "solver_common.h"

namespace kiops {

template <typename T>
struct PassCtx {
  int kp, src, flo, dlo, ngd, first, write_out, p;
  int store_u;   // full window: also write U_kp (the inner products come from a later phase)
  int ranks;     // workgroups per CU (KParams::ranks)
  T a;
  T bw[kLdh];
  T ybp[kPM];
  T ybc[kPM];
};

// Fixed slots of the per-workgroup inner products of a windowed pass.
constexpr int kDotRR = 0, kDotUU = 1, kDotG = 2, kDotC = 2 + (kWinMax - 1), kDotCk = 2 + 2 * (kWinMax - 1);
constexpr int kDotSlots = kDotCk + 1;

struct DotAcc {
  double RR, UU, Ck;
  double G[kWinMax - 1];
  double C[kWinMax - 1];
  __device__ void zero() {
    RR = UU = Ck = 0.0;
#pragma unroll
    for (int i = 0; i < kWinMax - 1; ++i) { G[i] = 0.0; C[i] = 0.0; }
  }
};

// Basis vector pointers: R_1 may live outside the slot array (it is w in FP64).
template <typename T>
struct BasisPtrs {
  const T* R1;
  T* slots;
  int64_t N;
  __device__ const T* get(int i) const { return i == 1 ? R1 : slots + (int64_t)(i - 1) * N; }
  __device__ T* get_mut(int i) const { return i == 1 ? const_cast<T*>(R1) : slots + (int64_t)(i - 1) * N; }
};

__device__ inline int wrap_index(int v, int n) {
  if (v < 0 || v >= n) {
    v %= n;
    if (v < 0) v += n;
  }
  return v;
}

// Block-wide sum of `count` doubles held per thread in `vals`; result in out[0..count)
// of thread 0 (all threads return after the final barrier).  Fixed order.
__device__ inline void block_sum(double* vals, int count, double* lds, double* out) {
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  for (int d = 0; d < count; ++d) {
    double v = vals[d];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) lds[wv * 64 + d] = v;
  }
  __syncthreads();
  if (t < count) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += lds[w * 64 + t];
    out[t] = s;
  }
  __syncthreads();
}

}  // namespace kiops
