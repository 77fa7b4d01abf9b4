// Periodic stencil given by per-cell weights (the general form of the
// operator description):
//
//   (A u)_i = W_0[i] u_i + W_1[i] u_{i+e_x} + W_2[i] u_{i-e_x} + W_3[i] u_{i+e_y}
//             + W_4[i] u_{i-e_y} [+ W_5[i] u_{i+e_z} + W_6[i] u_{i-e_z}],
//
// 5 weights per cell in 2-D (nz = 1), 7 in 3-D, stored [s][N].  Each cell
// carries its own coefficients for every neighbour, so nothing is shared
// between the rows of a tile beyond R_k itself; one Krylov step takes the two
// phases of the general sparse operator (formation, then product and inner
// products), with the neighbour columns implicit instead of read from an
// index array.  Rows are dealt to workgroups in contiguous blocks.
#pragma once

#include "buffer.h"
#include "pass_common.h"

namespace kiops {

template <typename T, int PB>
struct WeightsOp {
  static constexpr bool kTwoPhase = true;
  static constexpr int kLdsDoubles = 0;
  static constexpr int kWavesPerEU = 4;

  int64_t N;
  int nx, ny, nz, nw;   // nw: 5 or 7 weights per cell
  const T* W;           // [nw][N]
  const T* B[kPM];      // B[c] = b_{p-c} (Theorem 1 column order)
  int p;
  T* ubuf;              // U_k (always kept for this operator)
  const double* w_src;  // mixed precision: float copy of the weights made at setup
  T* w_dst;

  __device__ void setup_coefficients(const KParams& P, int64_t gt, int64_t gs) const {
    if (w_dst && w_src)
      for (int64_t e = gt; e < (int64_t)nw * N; e += gs) w_dst[e] = (T)w_src[e];
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
      for (int i = c.flo; i <= c.src; ++i) X = fma(c.bw[i], bp.get(i)[n], X);
      Rout[n] = X;
    }
  }

  // U_k = A R_k + nu B y(R_k) and the inner products of the step
  __device__ void matvec(const PassCtx<T>& c, const BasisPtrs<T>& bp, const T* R, DotAcc& acc) const {
    int64_t r0, r1;
    row_range(r0, r1);
    const int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    for (int64_t n = r0 + threadIdx.x; n < r1; n += kThreads) {
      const int64_t ix = n % nx;
      const int64_t rest = n / nx;
      const int64_t iy = rest % ny;
      const int64_t iz = rest / ny;
      const int64_t xp = ix + 1 < nx ? n + sx : n - (nx - 1) * sx;
      const int64_t xm = ix > 0 ? n - sx : n + (nx - 1) * sx;
      const int64_t yp = iy + 1 < ny ? n + sy : n - (ny - 1) * sy;
      const int64_t ym = iy > 0 ? n - sy : n + (ny - 1) * sy;
      T U = W[n] * R[n];
      U = fma(W[N + n], R[xp], U);
      U = fma(W[2 * N + n], R[xm], U);
      U = fma(W[3 * N + n], R[yp], U);
      U = fma(W[4 * N + n], R[ym], U);
      if (nw == 7) {
        const int64_t zp = iz + 1 < nz ? n + sz : n - (nz - 1) * sz;
        const int64_t zm = iz > 0 ? n - sz : n + (nz - 1) * sz;
        U = fma(W[5 * N + n], R[zp], U);
        U = fma(W[6 * N + n], R[zm], U);
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
