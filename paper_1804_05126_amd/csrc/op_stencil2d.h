// Periodic 5-point stencil (2-D), constant diffusivity and advection,
// per-cell reaction:
//
//   (A u)_P = wE u_E + wW u_W + wN u_N + wS u_S + (wC + r_P) u_P,
//   wE = D/h^2 - ax/(2h), wW = D/h^2 + ax/(2h), wN = D/h^2 - ay/(2h),
//   wS = D/h^2 + ay/(2h), wC = -4 D/h^2   (E/W = x+-1, N/S = y+-1).
//
// Tiling: a workgroup of 256 threads owns a 64 x 16 tile of outputs.  R_{kp-1}
// is staged in LDS over the tile plus a halo of two; U_{kp-1} and then R_kp
// are formed on the tile plus a halo of one (a second LDS buffer); the
// stencil of R_kp gives U_kp on the tile.  Each thread owns one column of four
// consecutive rows of the tile, so loads and stores of a wave cover 64
// consecutive doubles of a row.
#pragma once

#include "pass_common.h"

namespace kiops {

template <typename T>
struct Stencil2D {
  static constexpr int TX = 64, TY = 16;
  static constexpr int RX = TX + 4, RY = TY + 4;   // halo-2 region (R_{kp-1})
  static constexpr int SX = TX + 2, SY = TY + 2;   // halo-1 region (R_kp)
  static constexpr int kRing = SX * SY - TX * TY;  // halo-1 positions outside the tile
  static constexpr int kLdsT = RX * RY + SX * SY;  // elements of T

  int64_t N;
  int nx, ny, tiles_x, ntiles;
  T wE, wW, wN, wS, wC;
  const T* r;
  const T* B[kPM];   // B[c] = b_{p-c} (Theorem 1 column order)
  int p;
  const double* r_src;   // mixed precision: float copy r <- r_src made at setup
  T* r_dst;

  __device__ void setup_coefficients(const KParams& P, int64_t gt, int64_t gs) const {
    if (r_dst && r_src)
      for (int64_t n = gt; n < P.N; n += gs) r_dst[n] = (T)r_src[n];
  }

  __device__ void ring_pos(int e, int& rx, int& ry) const {
    // e in [0, kRing): top row, bottom row, left column, right column of the halo-1 ring
    if (e < SX) { rx = e - 1; ry = -1; return; }
    e -= SX;
    if (e < SX) { rx = e - 1; ry = TY; return; }
    e -= SX;
    if (e < TY) { rx = -1; ry = e; return; }
    e -= TY;
    rx = TX; ry = e;
  }

  // Form R_kp at halo-1 position (rx, ry) of the tile at (x0, y0); store into sX.
  // Returns r and the B term of U_kp at that position (used on the tile).
  __device__ __forceinline__ void form(const PassCtx<T>& c, const BasisPtrs<T>& bp, const double* w,
                                       const T* sR, T* sX, int x0, int y0, int rx, int ry,
                                       T& rv, T& bcur) const {
    const int gx = wrap_index(x0 + rx, nx);
    const int gy = wrap_index(y0 + ry, ny);
    const int64_t g = (int64_t)gy * nx + gx;
    rv = r ? r[g] : T(0);
    T bprev = T(0);
    bcur = T(0);
#pragma unroll
    for (int k = 0; k < kPM; ++k) {
      if (k < c.p) {
        const T bv = B[k][g];
        bprev = fma(bv, c.ybp[k], bprev);
        bcur = fma(bv, c.ybc[k], bcur);
      }
    }
    T X;
    if (c.first) {
      X = (T)w[g];
    } else {
      const int o = (ry + 2) * RX + (rx + 2);
      const T ctr = sR[o];
      T U = wE * sR[o + 1];
      U = fma(wW, sR[o - 1], U);
      U = fma(wN, sR[o + RX], U);
      U = fma(wS, sR[o - RX], U);
      U = fma(wC + rv, ctr, U);
      U += bprev;
      X = c.a * U;
      X = fma(c.bw[c.src], ctr, X);
      for (int i = c.flo; i < c.src; ++i) X = fma(c.bw[i], bp.get(i)[g], X);
    }
    sX[(ry + 1) * SX + (rx + 1)] = X;
  }

  // One pass over the tiles owned by this workgroup (windowed inner products).
  __device__ void pass(const PassCtx<T>& c, const BasisPtrs<T>& bp, const double* w, T* Rout,
                       DotAcc& acc, T* lds) const {
    T* sR = lds;
    T* sX = lds + RX * RY;
    const int t = threadIdx.x;
    const int cx = t & (TX - 1);
    const int rg = (t >> 6) * 4;
    const T* Rsrc = c.first ? nullptr : bp.get(c.src);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
      const int x0 = (tile % tiles_x) * TX;
      const int y0 = (tile / tiles_x) * TY;
      if (!c.first) {
        for (int e = t; e < RX * RY; e += kThreads) {
          const int ry2 = e / RX, rx2 = e - ry2 * RX;
          const int gx = wrap_index(x0 - 2 + rx2, nx);
          const int gy = wrap_index(y0 - 2 + ry2, ny);
          sR[e] = Rsrc[(int64_t)gy * nx + gx];
        }
        __syncthreads();
      }
      T rv[4], bc[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) form(c, bp, w, sR, sX, x0, y0, cx, rg + i, rv[i], bc[i]);
      if (t < kRing) {
        int rx, ry;
        ring_pos(t, rx, ry);
        T dr, db;
        form(c, bp, w, sR, sX, x0, y0, rx, ry, dr, db);
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ry = rg + i;
        if (x0 + cx < nx && y0 + ry < ny) {
          const int o = (ry + 1) * SX + (cx + 1);
          const T X = sX[o];
          T U = wE * sX[o + 1];
          U = fma(wW, sX[o - 1], U);
          U = fma(wN, sX[o + SX], U);
          U = fma(wS, sX[o - SX], U);
          U = fma(wC + rv[i], X, U);
          U += bc[i];
          const int64_t g = (int64_t)(y0 + ry) * nx + (x0 + cx);
          if (c.write_out) Rout[g] = X;
          const double Xd = (double)X, Ud = (double)U;
          acc.RR = fma(Xd, Xd, acc.RR);
          acc.UU = fma(Ud, Ud, acc.UU);
          acc.Ck = fma(Xd, Ud, acc.Ck);
#pragma unroll
          for (int d = 0; d < kWinMax - 1; ++d) {
            if (d < c.ngd) {
              const int idx = c.dlo + d;
              const double Rv = (idx == c.src) ? (double)sR[(ry + 2) * RX + (cx + 2)]
                                               : (double)bp.get(idx)[g];
              acc.G[d] = fma(Rv, Xd, acc.G[d]);
              acc.C[d] = fma(Rv, Ud, acc.C[d]);
            }
          }
        }
      }
      __syncthreads();
    }
  }
};

}  // namespace kiops
