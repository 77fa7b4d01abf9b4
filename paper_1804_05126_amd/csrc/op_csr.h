// General sparse operator in CSR form (square, 0-based int32 indices).
//
// A stencil pass recomputes U_{k-1} = A~ R_{k-1} around its tile; for a general
// sparse matrix the neighbours of a row are arbitrary, so one Krylov step
// takes two phases separated by a grid barrier:
//
//   form:    R_k = a U_{k-1} + sum_{i in [flo, k-1]} bw_i R_i        (elementwise)
//   matvec:  U_k = A R_k + nu B y(R_k), written out for the next step,
//            with the inner products <R_k,R_k>, <U_k,U_k>, <R_k,U_k>,
//            <R_i,R_k>, <R_i,U_k> (i in the window) accumulated per row.
//
// Rows are dealt to threads in contiguous blocks per workgroup.  Every array
// is read through buffer resources whose extent is the array's size, so a
// column index or row pointer outside its range reads zero instead of
// touching other memory.
#pragma once

#include "buffer.h"
#include "pass_common.h"

namespace kiops {

template <typename T, int PB>
struct CsrOp {
  static constexpr bool kTwoPhase = true;
  static constexpr int kLdsDoubles = 0;
  static constexpr int kWavesPerEU = 4;

  int64_t N, nnz;
  const int* rowptr;
  const int* col;
  const T* val;
  const T* B[kPM];    // B[c] = b_{p-c} (Theorem 1 column order)
  int p;
  T* ubuf;            // U_k (always kept for this operator)
  const double* v_src;   // mixed precision: float copy of val made at setup
  T* v_dst;

  __device__ void setup_coefficients(const KParams& P, int64_t gt, int64_t gs) const {
    if (v_dst && v_src)
      for (int64_t e = gt; e < nnz; e += gs) v_dst[e] = (T)v_src[e];
  }

  __device__ void row_range(int64_t& r0, int64_t& r1) const {
    r0 = N * (int64_t)vblock() / vgrid();
    r1 = N * (int64_t)(vblock() + 1) / vgrid();
  }

  // R_k from U_{k-1} and the window (for k = 1: R_1 = w, copied in mixed mode)
  __device__ void form(const PassCtx<T>& c, const BasisPtrs<T>& bp, const double* w, T* Rout) const {
    int64_t r0, r1;
    row_range(r0, r1);
    if (c.first) {
      if (c.write_out)
        for (int64_t n = r0 + threadIdx.x; n < r1; n += kThreads) Rout[n] = (T)w[n];
      return;
    }
    const T* U = ubuf;
    for (int64_t n = r0 + threadIdx.x; n < r1; n += kThreads) {
      T X = c.a * U[n];
      int i = c.flo;
      for (; i + 4 <= c.src + 1; i += 4) {
        const T v0 = bp.get(i)[n], v1 = bp.get(i + 1)[n], v2 = bp.get(i + 2)[n], v3 = bp.get(i + 3)[n];
        X = fma(c.bw[i], v0, X);
        X = fma(c.bw[i + 1], v1, X);
        X = fma(c.bw[i + 2], v2, X);
        X = fma(c.bw[i + 3], v3, X);
      }
      for (; i <= c.src; ++i) X = fma(c.bw[i], bp.get(i)[n], X);
      Rout[n] = X;
    }
  }

  // U_k = A R_k + nu B y(R_k) and the inner products of the step
  __device__ void matvec(const PassCtx<T>& c, const BasisPtrs<T>& bp, const T* R, DotAcc& acc) const {
    int64_t r0, r1;
    row_range(r0, r1);
    const __amdgpu_buffer_rsrc_t rsR = make_rsrc(R, (uint64_t)N * sizeof(T));
    const __amdgpu_buffer_rsrc_t rsP = make_rsrc(rowptr, (uint64_t)(N + 1) * 4);
    const __amdgpu_buffer_rsrc_t rsC = make_rsrc(col, (uint64_t)nnz * 4);
    const __amdgpu_buffer_rsrc_t rsV = make_rsrc(val, (uint64_t)nnz * sizeof(T));
    for (int64_t n = r0 + threadIdx.x; n < r1; n += kThreads) {
      int j0 = (int)__builtin_amdgcn_raw_buffer_load_b32(rsP, (uint32_t)n * 4u, 0, 0);
      int j1 = (int)__builtin_amdgcn_raw_buffer_load_b32(rsP, (uint32_t)(n + 1) * 4u, 0, 0);
      j0 = j0 < 0 ? 0 : (j0 > (int)nnz ? (int)nnz : j0);   // a row is a sub-range of [0, nnz)
      j1 = j1 < j0 ? j0 : (j1 > (int)nnz ? (int)nnz : j1);
      T U = T(0);
      for (int j = j0; j < j1; ++j) {
        const uint32_t cj = __builtin_amdgcn_raw_buffer_load_b32(rsC, (uint32_t)j * 4u, 0, 0);
        const T a = buf_ld(rsV, (uint32_t)j * (uint32_t)sizeof(T), T(0));
        const uint32_t off = cj < (uint32_t)N ? cj * (uint32_t)sizeof(T) : kNoOffset;
        U = fma(a, buf_ld(rsR, off, T(0)), U);
      }
#pragma unroll
      for (int k = 0; k < PB; ++k)
        if (k < c.p) U = fma(B[k][n], c.ybc[k], U);
      ubuf[n] = U;
      const double Xd = (double)R[n], Ud = (double)U;
      acc.RR = fma(Xd, Xd, acc.RR);
      acc.UU = fma(Ud, Ud, acc.UU);
      acc.Ck = fma(Xd, Ud, acc.Ck);
#pragma unroll
      for (int d = 0; d < kWinMax - 1; ++d) {
        if (d < c.ngd) {
          const double Rv = (double)bp.get(c.dlo + d)[n];
          acc.G[d] = fma(Rv, Xd, acc.G[d]);
          acc.C[d] = fma(Rv, Ud, acc.C[d]);
        }
      }
    }
  }
};

}  // namespace kiops
