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

// Cross-lane moves by DPP (data-parallel primitives of the VALU, GFX9
// encodings): quad permutations, rotations within a row of 16 lanes, and the
// broadcast of a row's last lane into the next row(s).
constexpr int kDppQuadSwap1 = 0xB1;    // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadSwap2 = 0x4E;    // quad_perm [2, 3, 0, 1]
constexpr int kDppRowRor4 = 0x124;     // row_ror:4
constexpr int kDppRowRor8 = 0x128;     // row_ror:8
constexpr int kDppRowBcast15 = 0x142;  // row_bcast:15
constexpr int kDppRowBcast31 = 0x143;  // row_bcast:31

// v moved by DPP control kCtrl; lanes of rows outside kRowMask read 0.0.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, kRowMask, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, kRowMask, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Wave-wide sums of kCount doubles per lane, in place; lane 63 ends with the
// totals (other lanes hold partial sums).  A fixed tree: pairs, quads, the
// four quads of a row of 16 lanes (two rotations), then rows 0 + 1 into row 1
// and 2 + 3 into row 3, and row 1 into row 3.  VALU moves only: no LDS
// traffic.  Used where one workgroup waits on the result (the epilogue).
template <int kCount>
__device__ __forceinline__ void wave_sum(double (&v)[kCount]) {
#pragma unroll
  for (int d = 0; d < kCount; ++d) v[d] += dpp_f64<kDppQuadSwap1, 0xF>(v[d]);
#pragma unroll
  for (int d = 0; d < kCount; ++d) v[d] += dpp_f64<kDppQuadSwap2, 0xF>(v[d]);
#pragma unroll
  for (int d = 0; d < kCount; ++d) v[d] += dpp_f64<kDppRowRor4, 0xF>(v[d]);
#pragma unroll
  for (int d = 0; d < kCount; ++d) v[d] += dpp_f64<kDppRowRor8, 0xF>(v[d]);
#pragma unroll
  for (int d = 0; d < kCount; ++d) v[d] += dpp_f64<kDppRowBcast15, 0xA>(v[d]);
#pragma unroll
  for (int d = 0; d < kCount; ++d) v[d] += dpp_f64<kDppRowBcast31, 0xC>(v[d]);
}

// Block-wide sum of kCount doubles held per thread in `vals`; result in
// out[0..kCount) of thread 0 (all threads return after the final barrier).
// Fixed order.
template <int kCount>
__device__ inline void block_sum(const double (&vals)[kCount], double* lds, double* out) {
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  double v[kCount];
#pragma unroll
  for (int d = 0; d < kCount; ++d) v[d] = vals[d];
  // One slot at a time: each shuffle waits for the previous one.  This end of
  // every pass runs while the CU's other workgroups are still in theirs, and
  // the faster forms (all slots together, or wave_sum above) measured 2-3%
  // slower on the 2048^2 sweep at two workgroups per CU: the workgroups'
  // arrival spread grew.
  for (int d = 0; d < kCount; ++d) {
    double x = v[d];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) lds[wv * 64 + d] = x;
  }
  __syncthreads();
  if (t < kCount) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += lds[w * 64 + t];
    // device scope, like the pass outputs (the pass barrier relies on it)
    __hip_atomic_store(&out[t], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

}  // namespace kiops
